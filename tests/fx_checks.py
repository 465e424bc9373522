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
    sum_t x_t (x_t^H r).  All arithmetic is exact: |V| < 2^31, N < 2^13 and
    |r| <= 2^10 keep every partial sum below 2^63 in int64.  When the a priori
    bound on every partial sum (2 N max|V| rmax, and the same for the voltage
    side) is below 2^53, the products run in binary64 instead, where every
    integer below 2^53 and every partial sum is exact, so the result is the
    same integer whatever the summation order.
    xre/xim are [T][F][N] integer arrays.  ``chans`` restricts the channels.
    """
    T, F, N = xre.shape
    rng = np.random.default_rng(seed)
    chans = range(F) if chans is None else chans
    ii, jj = np.tril_indices(N)
    p = tri_index(ii, jj)
    for f in chans:
        vf = np.asarray(vis[f])
        ar = xre[:, f, :]
        ai = xim[:, f, :]
        vmax = int(np.abs(vf).max()) if vf.size else 0
        xmax = max(int(np.abs(ar).max()), int(np.abs(ai).max())) if ar.size else 0
        bound = max(2 * N * vmax * rmax, 2 * N * xmax * rmax * (2 * T * xmax + 1))
        ft = np.float64 if bound < 2 ** 53 else np.int64
        rr = rng.integers(-rmax, rmax + 1, N).astype(ft)
        ri = rng.integers(-rmax, rmax + 1, N).astype(ft)
        vr = np.zeros((N, N), ft)
        vi = np.zeros((N, N), ft)
        vr[ii, jj] = vf[p, 0]
        vi[ii, jj] = vf[p, 1]
        vr[jj, ii] = vf[p, 0]
        vi[jj, ii] = -vf[p, 1]
        # V r
        lr = vr @ rr - vi @ ri
        li = vr @ ri + vi @ rr
        # sum_t x_t (x_t^H r):  s_t = sum_j conj(x_tj) r_j
        ar = ar.astype(ft)
        ai = ai.astype(ft)
        sr = ar @ rr + ai @ ri
        si = ar @ ri - ai @ rr
        rr2 = ar.T @ sr - ai.T @ si
        ri2 = ar.T @ si + ai.T @ sr
        if not (np.array_equal(lr, rr2) and np.array_equal(li, ri2)):
            return False
    return True
