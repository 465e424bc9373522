"""Pins for the oracle's beamformer on 4+4-bit voltages with 8-bit integer weights.

Paper Sec. 6 (DRX pipeline: the GPU phase-and-sum beamformer takes the 4+4
complex samples directly) and Sec. 4.1 (detect, accumulate).  Readings:
y = sum_i w_i x_i with no conjugation, exact integers; S = sum over navg
samples of |y|^2 (exact); the binary32 power is fl32(fl64(scale^2) * fl64(S)).

Each pin ties the oracle to something other than its own loops: numpy sums of
unpacked values (unit weights), a single complex product (one-hot input), the
integer X-engine oracle through the identity sum_t |w^T x_t|^2 = w^T V conj(w)
with V_ij = sum_t x_i conj(x_j), and a hand-built rounding case for the scale.
"""
import numpy as np

import oracle
import synth


def _ci4(seed, T, F, N, lo=-8, hi=7):
    rng = np.random.default_rng(seed)
    re = rng.integers(lo, hi + 1, (T, F, N))
    im = rng.integers(lo, hi + 1, (T, F, N))
    return synth.pack_ci4(re, im), re, im


def _w(seed, F, B, N, lim=127):
    rng = np.random.default_rng(seed)
    return rng.integers(-lim, lim + 1, (F, B, N, 2)).astype(np.int8)


def test_unit_weights_sum_inputs():
    T, F, N, B, navg = 12, 3, 10, 2, 4
    x, re, im = _ci4(1, T, F, N)
    w = np.zeros((F, B, N, 2), np.int8)
    w[..., 0] = 1
    P, y = oracle.beamform_ci4(x, w, np.ones(B, np.float32), navg, want_y=True)
    ys = re.sum(axis=2) + 1j * im.sum(axis=2)  # [T][F]
    for b in range(B):
        assert np.array_equal(y[b, :, :, 0], re.sum(axis=2).T)
        assert np.array_equal(y[b, :, :, 1], im.sum(axis=2).T)
    S = (np.abs(ys) ** 2).round().astype(np.int64).reshape(T // navg, navg, F).sum(axis=1).T
    assert np.array_equal(P[0], S.astype(np.float32))


def test_one_hot_input_gives_weight_times_sample_without_conjugation():
    T, F, N, B = 4, 1, 6, 3
    re = np.zeros((T, F, N), int)
    im = np.zeros((T, F, N), int)
    re[:, 0, 2] = [1, -8, 7, 0]
    im[:, 0, 2] = [0, -1, -8, 5]
    x = synth.pack_ci4(re, im)
    w = _w(2, F, B, N)
    _, y = oracle.beamform_ci4(x, w, np.ones(B, np.float32), 1, want_y=True)
    wc = w[0, :, 2, 0].astype(np.int64) + 1j * w[0, :, 2, 1]
    xc = re[:, 0, 2] + 1j * im[:, 0, 2]
    expect = wc[:, None] * xc[None, :]  # [B][T]
    assert np.array_equal(y[:, 0, :, 0], expect.real.astype(np.int64))
    assert np.array_equal(y[:, 0, :, 1], expect.imag.astype(np.int64))


def test_power_equals_quadratic_form_of_the_xengine_visibilities():
    # sum_t |sum_i w_i x_i(t)|^2 = sum_ij w_i V_ij conj(w_j), V_ij = sum_t x_i conj(x_j):
    # exact in int64, ties the beamformer to the independently pinned X-engine.
    T, F, N, B = 48, 2, 12, 4
    x, _, _ = _ci4(3, T, F, N)
    w = _w(4, F, B, N)
    P, y = oracle.beamform_ci4(x, w, np.ones(B, np.float32), T, want_y=True)
    V = oracle.xengine_int(x, "ci4", T, F, N, full=True)  # [F][N][N][2]
    for f in range(F):
        Vc = V[f, :, :, 0] + 1j * V[f, :, :, 1]
        for b in range(B):
            wc = w[f, b, :, 0].astype(np.int64) + 1j * w[f, b, :, 1]
            q = wc @ Vc @ np.conj(wc)
            assert q.imag == 0
            S = int((y[b, f, :, 0] ** 2 + y[b, f, :, 1] ** 2).sum())
            assert S == int(round(q.real))
            assert P[b, f, 0] == np.float32(float(S))


def test_extreme_values_stay_exact():
    T, F, N, B = 4, 1, 64, 1
    x = synth.pack_ci4(np.full((T, F, N), -8), np.full((T, F, N), -8))
    w = np.full((F, B, N, 2), -127, np.int8)
    _, y = oracle.beamform_ci4(x, w, np.ones(B, np.float32), 1, want_y=True)
    # (-127 - 127i)(-8 - 8i) = 1016i + ... : re = 127*8 - 127*8 = 0, im = 2*127*8 per input
    assert np.all(y[0, 0, :, 0] == 0)
    assert np.all(y[0, 0, :, 1] == 64 * 2 * 127 * 8)


def test_scale_rounding_steps():
    # one input, one sample: S = |w x|^2 = (3^2 + 4^2) * 7^2 = 1225
    x = synth.pack_ci4(np.array([[[7]]]), np.array([[[0]]]))
    w = np.array([[[[3, 4]]]], np.int8)
    s = np.float32(0.1)
    P = oracle.beamform_ci4(x, w, np.array([s]), 1)
    expect = np.float32(np.float64(s) * np.float64(s) * np.float64(1225))
    assert P[0, 0, 0] == expect
    # the binary32 square would differ in its last bits for some scales; the
    # definition squares in double
    assert P[0, 0, 0] == np.float32((float(s) ** 2) * 1225.0)
