"""Pins for the oracle beamformer (phase-and-sum + square-law detect + integrate).

Paper Sec. 6 (DRX pipeline: a phase-and-sum beamformer on the GPU) and Sec. 4.1
(detect: square-law detection; accumulate).  Reading: y = sum_i w_i x_i with no
conjugation of w; P = sum over navg consecutive samples of |y|^2.
"""
import numpy as np

import oracle
import synth


def _rand(seed, shape):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape), rng.standard_normal(shape)


def test_unit_weights_sum_inputs():
    T, F, N, B, navg = 8, 2, 5, 1, 4
    xr, xi = _rand(0, (T, F, N))
    wr, wi = np.ones((F, B, N)), np.zeros((F, B, N))
    P = oracle.beamform_detect(xr, xi, wr, wi, navg)
    y = (xr + 1j * xi).sum(axis=2)  # [T][F]
    expect = (np.abs(y) ** 2).reshape(T // navg, navg, F).sum(axis=1).T
    assert np.allclose(P[0], expect, rtol=1e-12)


def test_one_hot_input_gives_weight_times_sample():
    T, F, N, B, navg = 4, 1, 6, 3, 1
    xr = np.zeros((T, F, N))
    xi = np.zeros((T, F, N))
    xr[:, 0, 2] = [1, 2, 3, 4]
    xi[:, 0, 2] = [0, -1, 1, 0]
    wr, wi = _rand(1, (F, B, N))
    P = oracle.beamform_detect(xr, xi, wr, wi, navg)
    w = wr[0, :, 2] + 1j * wi[0, :, 2]
    x = xr[:, 0, 2] + 1j * xi[:, 0, 2]
    expect = np.abs(w[:, None] * x[None, :]) ** 2
    assert np.allclose(P[:, 0, :], expect, rtol=1e-12)


def test_no_conjugation_of_weights():
    # w = i, x = 1: y = i (not -i); |y|^2 is the same, so check via two inputs:
    # w = (1, i), x = (1, i): y = 1 + i*i = 0 without conjugation, 2 with it.
    xr = np.array([[[1.0, 0.0]]])
    xi = np.array([[[0.0, 1.0]]])
    wr = np.array([[[1.0, 0.0]]])
    wi = np.array([[[0.0, 1.0]]])
    P = oracle.beamform_detect(xr, xi, wr, wi, 1)
    assert P[0, 0, 0] == 0.0


def test_constant_magnitude_gives_navg_c2():
    T, F, N, B, navg = 32, 1, 1, 1, 16
    ph = np.linspace(0, 6, T)
    xr = (3 * np.cos(ph)).reshape(T, 1, 1)
    xi = (3 * np.sin(ph)).reshape(T, 1, 1)
    P = oracle.beamform_detect(xr, xi, np.ones((1, 1, 1)), np.zeros((1, 1, 1)), navg)
    assert np.allclose(P[0, 0], [16 * 9.0, 16 * 9.0], rtol=1e-12)


def test_beam_power_equals_w_V_wbar():
    # sum_t |w^T x_t|^2 = sum_ij w_i V_ij conj(w_j), V from the X-engine oracle
    T, F, N, B = 16, 2, 7, 3
    x = synth.cf16_voltages(5, T, F, N).astype(np.float64)
    w = synth.steering_weights(5, F, B, N).astype(np.float64)
    P = oracle.beamform_detect(x[..., 0], x[..., 1], w[..., 0], w[..., 1], T)
    V = oracle.xengine_f64(x[..., 0], x[..., 1], full=True)
    Vc = V[..., 0] + 1j * V[..., 1]
    wc = w[..., 0] + 1j * w[..., 1]
    for f in range(F):
        for b in range(B):
            q = wc[f, b] @ Vc[f] @ np.conj(wc[f, b])
            assert abs(q.imag) < 1e-9 * abs(q.real)
            assert abs(P[b, f, 0] - q.real) < 1e-10 * abs(q.real)


def test_steering_weights_unit_modulus():
    w = synth.steering_weights(1, 4, 8, 16).astype(np.float64)
    mag = np.hypot(w[..., 0], w[..., 1])
    assert np.all(np.abs(mag - 1) < 2 ** -10)
