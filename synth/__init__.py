"""Seeded synthetic inputs shaped like the paper's arrays.

This module draws random numbers and packs them into the wire formats.  It
holds none of the correlator's arithmetic (no unpack, product, transform,
requantization or detection); the oracle and the GPU path both consume what it
produces.

Wire formats (fixed conventions):

* ci8 -- two int8 bytes per complex sample, real first.
* ci4 -- one byte per complex sample, real part in the high nibble, imaginary
  part in the low nibble, each 4-bit two's complement.
* cf16 -- two IEEE half-precision values per sample, real first.
* Voltage arrays are laid out [time][channel][input] (time slowest, inputs
  fastest), with input = 2*antenna + polarisation.
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# Basic draws


def rng_for(seed, *stream):
    """A numpy Generator keyed by a seed and an optional sub-stream index tuple."""
    return np.random.default_rng([int(seed), *[int(s) for s in stream]])


def rounded_gaussian(rng, shape, sigma: float, clip: int, chunk: int = 1 << 24):
    """int8 values clamp(rint_half_even(sigma * z), -clip, clip), z ~ N(0, 1)."""
    n = int(np.prod(shape))
    out = np.empty(n, np.int8)
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        z = rng.standard_normal(m, dtype=np.float32)
        v = np.rint(z.astype(np.float64) * sigma)
        np.clip(v, -clip, clip, out=v)
        out[s:s + m] = v.astype(np.int8)
    return out.reshape(shape)


def pack_ci4(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Pack int values in [-8, 7] into 4+4 bytes (re high nibble, im low nibble)."""
    re = np.asarray(re)
    im = np.asarray(im)
    assert re.shape == im.shape
    assert re.min(initial=0) >= -8 and re.max(initial=0) <= 7
    assert im.min(initial=0) >= -8 and im.max(initial=0) <= 7
    hi = (re.astype(np.int16) & 0xF) << 4
    lo = im.astype(np.int16) & 0xF
    return (hi | lo).astype(np.uint8)


def pack_ci8(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Stack int8 re/im into a trailing (re, im) axis."""
    return np.stack([np.asarray(re, np.int8), np.asarray(im, np.int8)], axis=-1)


# --------------------------------------------------------------------------
# X-engine voltage gulps


def voltages(seed, ntime: int, nchan: int, ninput: int, dtype: str, sigma: float,
             clip: int, gulp: int = 0):
    """One [t][f][i] gulp of i.i.d. rounded-Gaussian complex voltages.

    Returns uint8 [T][F][N] for ci4, int8 [T][F][N][2] for ci8.  ``gulp`` picks
    an independent sub-stream so that gulps of one stream differ.
    """
    rng = rng_for(seed, gulp)
    shape = (ntime, nchan, ninput)
    re = rounded_gaussian(rng, shape, sigma, clip)
    im = rounded_gaussian(rng, shape, sigma, clip)
    if dtype == "ci4":
        assert clip <= 8
        return pack_ci4(re, im)
    if dtype == "ci8":
        return pack_ci8(re, im)
    raise ValueError(dtype)


def extreme_voltages(seed, ntime: int, nchan: int, ninput: int, dtype: str):
    """Voltages drawn uniformly over the whole code range, extremes included."""
    rng = rng_for(seed, 99)
    lo, hi = (-8, 7) if dtype == "ci4" else (-128, 127)
    re = rng.integers(lo, hi + 1, size=(ntime, nchan, ninput))
    im = rng.integers(lo, hi + 1, size=(ntime, nchan, ninput))
    return pack_ci4(re, im) if dtype == "ci4" else pack_ci8(re, im)


def constant_voltages(ntime: int, nchan: int, ninput: int, dtype: str, re: int, im: int):
    """Every sample equal to (re, im)."""
    r = np.full((ntime, nchan, ninput), re)
    i = np.full((ntime, nchan, ninput), im)
    return pack_ci4(r, i) if dtype == "ci4" else pack_ci8(r, i)


# --------------------------------------------------------------------------
# F-engine input: real 8-bit ADC samples with a tone and per-input delays


def adc_tone(seed, ninput: int, nfft: int, nspec: int, sigma: float = 16.0,
             tone_chan: int = 777, amplitude: float = 1.0, delay_max: float = 50.0):
    """Real int8 samples [nspec*nfft][ninput]:

    x_i[t] = clamp(rint(sigma*n_i[t] + A*cos(2 pi tone_chan (t - tau_i) / nfft)), +-127),
    tau_i ~ U[0, delay_max] (continuous), n_i independent N(0, 1) per input.
    Returns (x, tau).
    """
    rng = rng_for(seed, 0)
    tau = rng.uniform(0.0, delay_max, size=ninput)
    ntime = nfft * nspec
    x = np.empty((ntime, ninput), np.int8)
    chunk = max(1, (1 << 24) // ninput)
    two_pi = 2.0 * np.pi
    for s in range(0, ntime, chunk):
        m = min(chunk, ntime - s)
        # phase argument reduced exactly in the integer part of t*k mod nfft
        tk = (np.arange(s, s + m, dtype=np.int64)[:, None] * tone_chan) % nfft
        ph = two_pi * (tk.astype(np.float64) - tone_chan * tau[None, :]) / nfft
        z = rng.standard_normal((m, ninput), dtype=np.float32).astype(np.float64)
        v = np.rint(sigma * z + amplitude * np.cos(ph))
        np.clip(v, -127, 127, out=v)
        x[s:s + m] = v.astype(np.int8)
    return x, tau


def fengine_scale(nchan: int, sigma: float = 16.0, nfft: int = 4096, target_rms: float = 8.0):
    """Per-channel FP32 scale mapping noise of std sigma to target_rms per component."""
    s = target_rms / np.sqrt(sigma * sigma * nfft / 2.0)
    return np.full(nchan, s, np.float32)


# --------------------------------------------------------------------------
# FP16 voltages and steering weights


def cf16_voltages(seed, ntime: int, nchan: int, ninput: int, sigma: float = 1.0,
                  chunk_t: int = 0):
    """cf16 [T][F][N][2] with re, im ~ N(0, sigma^2) rounded to half precision."""
    rng = rng_for(seed, 0)
    out = np.empty((ntime, nchan, ninput, 2), np.float16)
    step = chunk_t or max(1, (1 << 24) // (nchan * ninput * 2))
    for s in range(0, ntime, step):
        m = min(step, ntime - s)
        z = rng.standard_normal((m, nchan, ninput, 2), dtype=np.float32)
        out[s:s + m] = (z * sigma).astype(np.float16)
    return out


def steering_weights(seed, nchan: int, nbeam: int, ninput: int):
    """Unit-modulus weights cf16 [F][B][N][2]: cos(theta) + i sin(theta), theta ~ U[0, 2pi)."""
    rng = rng_for(seed, 1)
    th = rng.uniform(0.0, 2.0 * np.pi, size=(nchan, nbeam, ninput))
    return np.stack([np.cos(th), np.sin(th)], axis=-1).astype(np.float16)


def int8_steering_weights(seed, nchan: int, nbeam: int, ninput: int, amp: float = 127.0):
    """Unit-modulus weights quantized to int8: [F][B][N][2] = rint(amp cos theta),
    rint(amp sin theta), theta ~ U[0, 2pi); with the per-beam scale 1/amp
    (float32 [B]) they stand for the unit-modulus weights."""
    rng = rng_for(seed, 2)
    th = rng.uniform(0.0, 2.0 * np.pi, size=(nchan, nbeam, ninput))
    w = np.stack([np.rint(amp * np.cos(th)), np.rint(amp * np.sin(th))], axis=-1).astype(np.int8)
    return w, np.full(nbeam, 1.0 / amp, np.float32)


def extreme_int8_weights(seed, nchan: int, nbeam: int, ninput: int):
    """int8 weights [F][B][N][2] uniform over the whole code range, -128 included."""
    rng = rng_for(seed, 3)
    return rng.integers(-128, 128, size=(nchan, nbeam, ninput, 2)).astype(np.int8)


# --------------------------------------------------------------------------
# Batched mixed-size subarrays


BATCH_NINPUT = (32, 64, 96, 128, 192, 256, 384, 512)
BATCH_NCHAN = (1024, 512, 512, 256, 256, 128, 128, 64)


def batched_voltages(ntime: int = 256, ninputs=BATCH_NINPUT, nchans=BATCH_NCHAN,
                     sigma: float = 8.0, clip: int = 127, seed0: int = 40):
    """One ci8 gulp per subarray k (seed seed0 + k), each [T][F_k][N_k][2]."""
    return [voltages(seed0 + k, ntime, f, n, "ci8", sigma, clip)
            for k, (n, f) in enumerate(zip(ninputs, nchans))]
