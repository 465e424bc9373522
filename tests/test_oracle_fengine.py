"""Pins for the oracle's direct DFT and requantizer (no GPU).

Transform convention (paper Sec. 2.2 FFT module; Sec. 6: 204.8 MS/s into 4096
channels of 25 kHz, so 2N real samples give N channels): forward sign,
unnormalised, rectangular window, bins 0..N/2-1 with the Nyquist bin dropped.
"""
import numpy as np
import pytest

import oracle
import synth

NFFT = 64


def _frame(vals, ninput=1, nspec=1):
    x = np.zeros((NFFT * nspec, ninput), np.int8)
    x[:, 0] = np.resize(np.asarray(vals, np.int8), NFFT * nspec)
    return x


def test_dft_impulse_pins_sign_and_position():
    for n0 in (0, 1, 5, 33):
        v = np.zeros(NFFT, int)
        v[n0] = 3
        X = oracle.dft_real(_frame(v), NFFT)[0, :, 0]
        k = np.arange(NFFT // 2)
        expect = 3 * np.exp(-2j * np.pi * k * n0 / NFFT)
        assert np.allclose(X[:, 0], expect.real, atol=1e-12)
        assert np.allclose(X[:, 1], expect.imag, atol=1e-12)


def test_dft_dc():
    X = oracle.dft_real(_frame(np.full(NFFT, -7)), NFFT)[0, :, 0]
    assert X[0, 0] == -7 * NFFT and abs(X[0, 1]) < 1e-12
    assert np.max(np.abs(X[1:])) < 1e-10


def test_dft_quarter_rate_cosine_and_sine():
    # cos(2 pi n / 4) -> bin N/4 holds N/2; sin -> -i N/2 (forward sign)
    c = _frame([1, 0, -1, 0])
    s = _frame([0, 1, 0, -1])
    Xc = oracle.dft_real(c, NFFT)[0, :, 0]
    Xs = oracle.dft_real(s, NFFT)[0, :, 0]
    q = NFFT // 4
    assert abs(Xc[q, 0] - NFFT / 2) < 1e-10 and abs(Xc[q, 1]) < 1e-10
    assert abs(Xs[q, 0]) < 1e-10 and abs(Xs[q, 1] + NFFT / 2) < 1e-10
    mask = np.ones(NFFT // 2, bool)
    mask[q] = False
    assert np.max(np.abs(Xc[mask])) < 1e-10 and np.max(np.abs(Xs[mask])) < 1e-10


def test_dft_nyquist_is_dropped():
    # (-1)^n lives only in the Nyquist bin, which the output does not contain
    X = oracle.dft_real(_frame([5, -5]), NFFT)[0, :, 0]
    assert np.max(np.abs(X)) < 1e-10


def test_dft_parseval():
    rng = np.random.default_rng(0)
    x = rng.integers(-127, 128, (NFFT, 3)).astype(np.int8)
    X = oracle.dft_real(x, NFFT)[0]
    for i in range(3):
        v = x[:, i].astype(float)
        ny = np.sum(v * (-1.0) ** np.arange(NFFT))  # Nyquist bin, computed separately
        p = X[:, i, 0] ** 2 + X[:, i, 1] ** 2
        total = p[0] + 2 * p[1:].sum() + ny ** 2
        assert abs(total / NFFT - np.sum(v * v)) < 1e-8 * np.sum(v * v)


def test_dft_matches_numpy_rfft_multi_frame():
    rng = np.random.default_rng(1)
    nspec, ninput = 3, 5
    x = rng.integers(-128, 128, (NFFT * nspec, ninput)).astype(np.int8)
    X = oracle.dft_real(x, NFFT)
    ref = np.fft.rfft(x.astype(float).reshape(nspec, NFFT, ninput), axis=1)[:, :NFFT // 2]
    err = np.abs((X[..., 0] + 1j * X[..., 1]) - ref).max()
    assert err <= 1e-9 * np.abs(ref).max()


def test_dft_4096_tone_bin():
    # a bin-centred integer cosine at k0 of amplitude 100 (quantised) puts
    # ~N/2*100 in bin k0 with the phase of the delay
    nfft = 4096
    k0, d = 777, 13
    n = np.arange(nfft)
    v = np.rint(100 * np.cos(2 * np.pi * k0 * (n - d) / nfft))
    x = v.astype(np.int8)[:, None]
    X = oracle.dft_real(x, nfft)[0, :, 0]
    z = X[k0, 0] + 1j * X[k0, 1]
    assert abs(abs(z) - nfft / 2 * 100) < 0.01 * nfft / 2 * 100
    phase = np.angle(z)
    expect = np.angle(np.exp(-2j * np.pi * k0 * d / nfft))
    assert abs(np.angle(np.exp(1j * (phase - expect)))) < 1e-3


# ------------------------------------------------------------- requantize

def _rq(vals, scale=1.0):
    X = np.zeros((1, 1, len(vals), 2))
    X[0, 0, :, 0] = vals
    X[0, 0, :, 1] = -np.asarray(vals)
    q = oracle.requantize(X, np.array([scale], np.float32))
    return q[0, 0, :, 0].tolist(), q[0, 0, :, 1].tolist()


def test_requantize_round_half_even():
    re, im = _rq([0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 0.49, 0.51])
    assert re == [0, 2, 2, 0, -2, -2, 0, 1]
    assert im == [0, -2, -2, 0, 2, 2, 0, -1]


def test_requantize_saturates_symmetric():
    re, im = _rq([127.4, 127.5, 128.0, 1e6, -127.6, -1e9])
    assert re == [127, 127, 127, 127, -127, -127]
    assert min(im) >= -127 and max(im) <= 127


def test_requantize_applies_scale():
    re, _ = _rq([3.0, 10.0, -7.0], scale=0.5)
    assert re == [2, 5, -4]  # 1.5 -> 2, 5 -> 5, -3.5 -> -4


def test_requantize_decision_on_the_exact_product():
    # 0.5 + 1e-12 lies above the tie and 1.5 - 1e-12 below it; binary32 would
    # see both as exact ties.  The definition rounds the exact product.
    re, _ = _rq([0.5 + 1e-12, 1.5 - 1e-12, -0.5 - 1e-12])
    assert re == [1, 1, -1]
    # the scale is the binary32 value widened exactly: 0.1f * 5 = 0.50000000745
    re, _ = _rq([5.0], scale=0.1)
    assert re == [1]


def test_requantize_per_channel_scale():
    X = np.ones((2, 3, 1, 2)) * 10.0
    q = oracle.requantize(X, np.array([0.1, 0.25, 1.0], np.float32))
    assert q[:, :, 0, 0].tolist() == [[1, 2, 10], [1, 2, 10]]


def test_adc_tone_generator_shape_and_range():
    x, tau = synth.adc_tone(3, 4, 256, 2, sigma=16.0, tone_chan=20)
    assert x.shape == (512, 4) and x.dtype == np.int8
    assert x.min() >= -127 and x.max() <= 127
    assert tau.shape == (4,) and np.all((tau >= 0) & (tau <= 50))
