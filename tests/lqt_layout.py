"""Conversions between the oracle's dense tuples and the structure-of-arrays element layout of the
C ABI (A stored as A - I, C and J as packed upper triangles).  Layout bookkeeping only."""
import numpy as np

from paper_2212_11744_amd import lqt


TILE = 512


def tile_position(k):
    """(tile, column) of item k: tiles of 512 items, column 64 (k % 8) + (k % 512) // 8."""
    k = np.asarray(k)
    return k // TILE, 64 * (k % 8) + (k % TILE) // 8


def untile(elts, T):
    """[ntile][NE][512] -> [NE][T]."""
    e = np.asarray(elts, dtype=np.float64)
    g, c = tile_position(np.arange(T))
    return e[g, :, c].T


def tile(e):
    """[NE][T] -> [ntile][NE][512] (padding zero)."""
    NE, T = e.shape
    nt = (T + TILE - 1) // TILE
    out = np.zeros((nt, NE, TILE))
    g, c = tile_position(np.arange(T))
    out[g, :, c] = np.asarray(e).T
    return out


def soa_to_dense(elts, nx, T):
    """[ntile][NE][512] array (one problem) -> dict of A, b, C, eta, J with A the full matrix."""
    e = untile(elts, T)
    sl = lqt.element_slices(nx)
    iu = np.triu_indices(nx)
    out = {"A": e[sl["A"]].T.reshape(T, nx, nx) + np.eye(nx)[None],
           "Ad": e[sl["A"]].T.reshape(T, nx, nx),
           "b": e[sl["b"]].T.copy(), "eta": e[sl["eta"]].T.copy()}
    for k in ("C", "J"):
        M = np.zeros((T, nx, nx))
        M[:, iu[0], iu[1]] = e[sl[k]].T
        M[:, iu[1], iu[0]] = e[sl[k]].T
        out[k] = M
    return out


def dense_to_soa(el, nx, Ad=None):
    """dict of A, b, C, eta, J (T leading) -> [ntile][NE][512] (A - I, packed upper triangles)."""
    T = el["A"].shape[0]
    iu = np.triu_indices(nx)
    Ad = el["A"] - np.eye(nx)[None] if Ad is None else Ad
    parts = [Ad.reshape(T, nx * nx).T, el["b"].T, el["C"][:, iu[0], iu[1]].T, el["eta"].T,
             el["J"][:, iu[0], iu[1]].T]
    return tile(np.concatenate(parts, axis=0))
