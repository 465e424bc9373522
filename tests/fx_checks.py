"""Size-independent checks shared by the oracle pins and the GPU parity tests.

These are properties of the visibility definition V_ij = sum_t x_i conj(x_j)
that hold at any size; they use numpy only (never the GPU path) and are pinned
against the oracle in the CPU tests.
"""
import numpy as np


def tri_index(i, j):
    return i * (i + 1) // 2 + j


def hermitian_from_packed(vis_f: np.ndarray, N: int):
    """[P][2] packed lower triangle -> complex [N][N] int64-valued object (re, im arrays)."""
    re = np.zeros((N, N), np.int64)
    im = np.zeros((N, N), np.int64)
    ii, jj = np.tril_indices(N)
    p = tri_index(ii, jj)
    re[ii, jj] = vis_f[p, 0]
    im[ii, jj] = vis_f[p, 1]
    re[jj, ii] = vis_f[p, 0]
    im[jj, ii] = -vis_f[p, 1]
    return re, im


def freivalds_check(vis: np.ndarray, xre: np.ndarray, xim: np.ndarray, seed: int = 0,
                    chans=None, rmax: int = 1 << 10) -> bool:
    """Exact probabilistic check of packed visibilities [F][P][2] against voltages.

    For a random integer vector r (|r| <= rmax, complex), V r must equal
    sum_t x_t (x_t^H r).  All arithmetic is int64 and exact: |V| < 2^31, N < 2^13
    and |r| <= 2^10 keep every partial sum below 2^63.
    xre/xim are [T][F][N] integer arrays.  ``chans`` restricts the channels.
    """
    T, F, N = xre.shape
    rng = np.random.default_rng(seed)
    chans = range(F) if chans is None else chans
    for f in chans:
        rr = rng.integers(-rmax, rmax + 1, N).astype(np.int64)
        ri = rng.integers(-rmax, rmax + 1, N).astype(np.int64)
        vr, vi = hermitian_from_packed(np.asarray(vis[f], np.int64), N)
        # V r
        lr = vr @ rr - vi @ ri
        li = vr @ ri + vi @ rr
        # sum_t x_t (x_t^H r):  s_t = sum_j conj(x_tj) r_j
        ar = xre[:, f, :].astype(np.int64)
        ai = xim[:, f, :].astype(np.int64)
        sr = ar @ rr + ai @ ri
        si = ar @ ri - ai @ rr
        rr2 = ar.T @ sr - ai.T @ si
        ri2 = ar.T @ si + ai.T @ sr
        if not (np.array_equal(lr, rr2) and np.array_equal(li, ri2)):
            return False
    return True
