"""Pins for the oracle T-engine (Sec. 6: TBN pipeline and DRX T-engine --
bandwidth reduction, shift along the channel axis, inverse transform, complex
mixer, quantization to 8+8 or 4+4).

Pinned against closed forms (a single channel is a complex exponential, the
band centre is DC, the mixer rotates by a known phasor that runs on across
frames), numpy's inverse FFT of the shifted band, and hand-made rounding and
saturation cases.
"""
import numpy as np

import oracle


def _spectra(seed, S, F, N, lim=127):
    rng = np.random.default_rng(seed)
    return rng.integers(-lim, lim + 1, (S, F, N, 2)).astype(np.int8)


def test_single_channel_is_a_complex_exponential():
    S, F, N, nfft, chan0, k0 = 1, 20, 2, 8, 5, 7
    x = np.zeros((S, F, N, 2), np.int8)
    x[0, chan0 + k0, 1] = (12, -5)
    _, z = oracle.tengine(x, chan0, nfft, 0, 1, 1.0, want_z=True)
    n = np.arange(nfft)
    expect = (12 - 5j) / nfft * np.exp(2j * np.pi * (k0 - nfft // 2) * n / nfft)
    assert np.allclose(z[:, 1, 0] + 1j * z[:, 1, 1], expect, atol=1e-13)
    assert np.all(z[:, 0, :] == 0)


def test_band_centre_is_dc():
    S, F, N, nfft, chan0 = 2, 64, 1, 16, 24
    x = np.zeros((S, F, N, 2), np.int8)
    x[:, chan0 + nfft // 2, 0] = (32, 16)
    _, z = oracle.tengine(x, chan0, nfft, 0, 1, 1.0, want_z=True)
    assert np.allclose(z[:, 0, 0], 2.0, atol=1e-14) and np.allclose(z[:, 0, 1], 1.0, atol=1e-14)


def test_matches_numpy_ifft_of_the_shifted_band():
    S, F, N, nfft, chan0 = 3, 300, 4, 64, 100
    x = _spectra(1, S, F, N)
    _, z = oracle.tengine(x, chan0, nfft, 0, 1, 1.0, want_z=True)
    for s in range(S):
        X = x[s, chan0:chan0 + nfft, :, 0].astype(np.float64) + 1j * x[s, chan0:chan0 + nfft, :, 1]
        want = np.fft.ifft(np.fft.ifftshift(X, axes=0), axis=0)
        got = z[s * nfft:(s + 1) * nfft, :, 0] + 1j * z[s * nfft:(s + 1) * nfft, :, 1]
        assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_mixer_phase_runs_on_across_frames():
    S, F, N, nfft, chan0 = 3, 16, 1, 8, 4
    x = np.zeros((S, F, N, 2), np.int8)
    x[:, chan0 + nfft // 2, 0] = (80, 0)  # DC: z = 10 before mixing
    _, z = oracle.tengine(x, chan0, nfft, 3, 16, 1.0, want_z=True)  # 3/16 cycle per sample
    t = np.arange(S * nfft)
    expect = 10.0 * np.exp(2j * np.pi * ((3 * t) % 16) / 16)
    assert np.allclose(z[:, 0, 0] + 1j * z[:, 0, 1], expect, atol=1e-13)


def test_quantize_rounds_half_even_and_saturates_symmetric():
    S, F, N, nfft, chan0 = 1, 4, 1, 4, 0
    x = np.zeros((S, F, N, 2), np.int8)
    x[0, nfft // 2, 0] = (10, -6)  # DC: z = (2.5, -1.5) on every sample
    q = oracle.tengine(x, chan0, nfft, 0, 1, 1.0)
    assert q[:, 0, 0].tolist() == [2] * 4 and q[:, 0, 1].tolist() == [-2] * 4
    q8 = oracle.tengine(x, chan0, nfft, 0, 1, 1000.0, out_bits=8)
    assert q8[:, 0, 0].tolist() == [127] * 4 and q8[:, 0, 1].tolist() == [-127] * 4
    q4 = oracle.tengine(x, chan0, nfft, 0, 1, 1000.0, out_bits=4)
    assert q4[:, 0, 0].tolist() == [7] * 4 and q4[:, 0, 1].tolist() == [-7] * 4
    # the rounding decision takes the exact product (2.5 * 1.2 = 3.0000000477 in
    # double from the binary32 scale -> 3, not a tie)
    q = oracle.tengine(x, chan0, nfft, 0, 1, np.float32(1.2))
    assert q[0, 0, 0] == 3
