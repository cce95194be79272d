"""Writes tests/golden/fullsize_point_mass_T2p20.json: sampled outputs of the oracle's sequential
FP64 solve of the point-mass tracking problem at its full size (seed 2, T = 2^20 blocks x 4 RK4
steps on [0, 10]), for the full-size GPU parity test.

    python tests/golden/make_fullsize.py

Calls only the oracle and the seeded input generators.  The sampled block indices include the
ends of the horizon, tile and scan-tree boundaries (multiples of 4, 256 and 65536 and their
neighbours) and seeded random indices.  Elements are stored for sampled blocks too; each is the
oracle's element build of that single block.  Takes about a minute and a half (one host thread).
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2212_11744_amd import workloads as W  # noqa: E402

SEED, T, N_STEPS = 2, 2 ** 20, 4


def sample_indices(T):
    fixed = {0, 1, 2, 3, 4, 5, 255, 256, 257, 1023, 1024, 1025, 65535, 65536, 65537,
             262143, 262144, 524287, 524288, T - 257, T - 256, T - 5, T - 4, T - 3, T - 2, T - 1, T}
    rng = np.random.default_rng(12345)
    rand = set(int(k) for k in rng.integers(0, T + 1, size=37))
    return sorted(k for k in fixed | rand if 0 <= k <= T)


def main():
    p = W.point_mass(SEED, T, N_STEPS)
    ks = sample_indices(T)
    sol = O.solve(p)
    blocks = [k for k in ks if k < T]
    el = {}
    for k in blocks:
        sub = W.Problem(p.nx, p.nu, 1, p.n, p.t[k:k + 2].copy(), p.F, p.L, p.Q, p.R, p.Qf, p.rf,
                        p.x0, p.r[2 * p.n * k:2 * p.n * (k + 1) + 1].copy(), None, None, None)
        e = O.elements(sub)
        el[k] = {name: np.asarray(e[name][0]).tolist() for name in ("A", "b", "C", "eta", "J")}
    out = {
        "description": "Oracle (sequential FP64) outputs of the point-mass tracking problem, seed 2, "
                       "T = 2^20 blocks x 4 RK4 steps on [0, 10], at sampled boundaries k; elements of "
                       "sampled blocks (Theorem 8 by RK4, Sec. IV-B; values by Theorem 6 and Lemma 7; "
                       "trajectory and control by Sec. IV-E and Sec. II-B). Written by make_fullsize.py.",
        "seed": SEED, "T": T, "n_steps": N_STEPS, "k": ks,
        "S": [sol["S"][k].tolist() for k in ks],
        "v": [sol["v"][k].tolist() for k in ks],
        "x": [sol["x"][k].tolist() for k in ks],
        "u": [sol["u"][k].tolist() for k in ks],
        "blocks": blocks,
        "elements": [el[k] for k in blocks],
    }
    path = os.path.join(HERE, "fullsize_point_mass_T2p20.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(path, len(ks), "samples")


if __name__ == "__main__":
    main()
