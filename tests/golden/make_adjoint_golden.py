"""Writes tests/golden/adjoint_point_mass_T2p16.json: gradients of f = sum_k <W_k, x_k> for two
problems of the differentiated workload (point mass, T = 2^16 blocks x 4 RK4 steps on [0, 10],
seeds 5000 and 5001, W seeded standard normal), entry by entry, from the oracle's exact
directional derivatives (dual numbers) along unit directions: every entry of dQ, dR, dQf (for
the symmetric unit perturbation of each pair i <= j), drf, dx0, and dr at 64 sampled samples.
Calls only oracle/ and the seeded input generators.  Run: python tests/golden/make_adjoint_golden.py
(about 600 dual-number passes; spread over the host's cores).
"""
import json
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

T, N_STEPS, SEEDS, W_SEED0, N_R = 2 ** 16, 4, (5000, 5001), 7700, 64


def problem(seed):
    from paper_2212_11744_amd import workloads as W
    return W.point_mass(seed, T, N_STEPS)


def weights(b):
    return np.random.default_rng(W_SEED0 + b).standard_normal((T + 1, 4))


def r_indices():
    ns = 2 * N_STEPS * T + 1
    rng = np.random.default_rng(99)
    inner = rng.choice(np.arange(1, ns - 1), N_R - 4, replace=False)
    return sorted(set(int(i) for i in inner) | {0, 1, 2 * N_STEPS * 1000, ns - 1})


def directions(p):
    out = []
    for name in ("Q", "Qf"):
        for i in range(4):
            for j in range(i, 4):
                out.append((name, (i, j)))
    for i in range(2):
        for j in range(i, 2):
            out.append(("R", (i, j)))
    out += [("rf", (i,)) for i in range(4)] + [("x0", (i,)) for i in range(4)]
    out += [("r", (s, c)) for s in r_indices() for c in range(4)]
    return out


def jvp(task):
    import oracle as O
    b, name, idx = task
    p = problem(SEEDS[b])
    d = np.zeros(np.shape(getattr(p, name)))
    if len(idx) == 2 and name in ("Q", "Qf", "R"):
        i, j = idx
        d[i, j] += 1.0
        d[j, i] += 1.0 if i != j else 0.0
        scale = 0.5 if i != j else 1.0
    else:
        d[idx] = 1.0
        scale = 1.0
    _, df = O.objective_jvp(p, weights(b), {name: d})
    return b, name, list(idx), df * scale


def main():
    tasks = [(b, name, idx) for b in range(len(SEEDS)) for name, idx in directions(problem(SEEDS[b]))]
    with mp.Pool(max(1, (os.cpu_count() or 2) - 1)) as pool:
        res = pool.map(jvp, tasks, chunksize=4)
    out = {"T": T, "n_steps": N_STEPS, "seeds": list(SEEDS), "w_seed0": W_SEED0,
           "r_indices": r_indices(),
           "note": "d f / d theta for f = sum_k <W_k, x_k>; W_b = default_rng(w_seed0 + b)."
                   "standard_normal((T + 1, 4)); symmetric gradients (Q, R, Qf) at pairs i <= j",
           "grads": [{} for _ in SEEDS]}
    for b, name, idx, val in res:
        out["grads"][b].setdefault(name, []).append([idx, val])
    with open(os.path.join(HERE, "adjoint_point_mass_T2p16.json"), "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", len(res), "entries")


if __name__ == "__main__":
    main()
