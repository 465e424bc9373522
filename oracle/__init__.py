"""CPU oracle for the FX-correlator hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it, and it shares no code
with the GPU path: the arithmetic lives in ``oracle.c`` (plain loops in int64 /
double); this module only marshals numpy arrays into it.

Functions and the passages they follow (section numbers of the Bifrost paper):

* :func:`unpack_ci4`, :func:`unpack_ci8` -- 4+4 and 8+8 complex signed
  integers (Sec. 6, packet capture and TBN pipeline).
* :func:`xengine_int` -- V_f = sum_t x_t x_t^H per channel, lower triangle
  packed as p = i(i+1)/2 + j (Sec. 2.2 linear-algebra module; Sec. 7 plans
  correlation).  Exact in int64.
* :func:`xengine_f64` -- the same product on decoded FP16 voltages in double.
* :func:`dft_real` -- direct DFT of real frames, forward sign, unnormalised,
  Nyquist dropped (Sec. 2.2 FFT module; Sec. 6 F-engine: 2N real samples per
  N channels).
* :func:`requantize` -- per-channel scale, round half to even, saturate to
  [-127, 127] (Sec. 2.2 quantize module), decision taken in single precision.
* :func:`beamform_detect` -- phase-and-sum beam, |y|^2, integrate navg samples
  (Sec. 6 DRX pipeline; Sec. 4.1 detect and accumulate blocks).

Parity status: every function is pinned by the ``-m "not gpu"`` tests against
closed forms, brute force and independent library routines.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = ctypes.CDLL(_LIB_PATH)
        i64, i32, vp, ci = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int
        _lib.orc_unpack_ci4.argtypes = [vp, i64, vp, vp]
        _lib.orc_unpack_ci8.argtypes = [vp, i64, vp, vp]
        _lib.orc_xengine_int.argtypes = [vp, ci, i64, i32, i32, i32, i32, i64, i64, ci, vp, ci]
        _lib.orc_xengine_f64.argtypes = [vp, vp, i64, i32, i32, ci, vp, ci]
        _lib.orc_accumulate_f64.argtypes = [vp, vp, i64]
        _lib.orc_dft_real.argtypes = [vp, i32, i32, i64, vp, ci]
        _lib.orc_requantize.argtypes = [vp, vp, i64, i32, i32, vp]
        _lib.orc_beamform_detect.argtypes = [vp, vp, vp, vp, i64, i32, i32, i32, i32, vp, ci]
        _lib.orc_beamform_ci4.argtypes = [vp, vp, vp, i64, i32, i32, i32, i32, vp, vp, ci]
        _lib.orc_tengine.argtypes = [vp, i32, i32, i64, i32, i32, i64, i64, ctypes.c_float, ci, vp, vp,
                                     ci]
        for name in ("orc_unpack_ci4", "orc_unpack_ci8", "orc_xengine_int", "orc_xengine_f64",
                     "orc_accumulate_f64", "orc_dft_real", "orc_requantize",
                     "orc_beamform_detect", "orc_beamform_ci4", "orc_tengine", "orc_max_threads"):
            getattr(_lib, name).restype = ctypes.c_int
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def max_threads() -> int:
    return int(_load().orc_max_threads())


def unpack_ci4(packed: np.ndarray):
    """Return (re, im) int32 arrays for a uint8 array of 4+4 samples."""
    p = np.ascontiguousarray(packed, dtype=np.uint8)
    re = np.empty(p.shape, np.int32)
    im = np.empty(p.shape, np.int32)
    _check(_load().orc_unpack_ci4(_ptr(p), p.size, _ptr(re), _ptr(im)), "unpack_ci4")
    return re, im


def unpack_ci8(pairs: np.ndarray):
    """Return (re, im) int32 arrays for an int8 array whose last axis is (re, im)."""
    p = np.ascontiguousarray(pairs, dtype=np.int8)
    assert p.shape[-1] == 2
    re = np.empty(p.shape[:-1], np.int32)
    im = np.empty(p.shape[:-1], np.int32)
    _check(_load().orc_unpack_ci8(_ptr(p), p.size // 2, _ptr(re), _ptr(im)), "unpack_ci8")
    return re, im


def xengine_int(data: np.ndarray, dtype: str, ntime: int, nchan: int, ninput: int,
                chans=None, t0: int = 0, nt=None, full: bool = False, nthreads: int = 0):
    """Exact integer X-engine.

    ``data`` is the raw [t][f][i] voltage buffer (uint8 for ci4, int8 with a
    trailing (re, im) axis for ci8).  ``chans`` is (f0, nf); default all.
    Returns int64 [nf][N(N+1)/2][2] (or [nf][N][N][2] when ``full``).
    """
    code = {"ci4": 4, "ci8": 8}[dtype]
    buf = np.ascontiguousarray(data)
    need = ntime * nchan * ninput * (1 if code == 4 else 2)
    assert buf.nbytes == need, (buf.nbytes, need)
    f0, nf = (0, nchan) if chans is None else chans
    nt = ntime - t0 if nt is None else nt
    per = ninput * ninput if full else ninput * (ninput + 1) // 2
    out = np.zeros((nf, per, 2), np.int64)
    rc = _load().orc_xengine_int(_ptr(buf), code, ntime, nchan, ninput, f0, nf, t0, nt,
                                 int(full), _ptr(out), nthreads)
    _check(rc, "xengine_int")
    if full:
        return out.reshape(nf, ninput, ninput, 2)
    return out


def xengine_f64(re: np.ndarray, im: np.ndarray, full: bool = False, nthreads: int = 0):
    """Double-precision X-engine on decoded voltages re/im of shape [T][F][N]."""
    r = np.ascontiguousarray(re, dtype=np.float64)
    i = np.ascontiguousarray(im, dtype=np.float64)
    assert r.shape == i.shape and r.ndim == 3
    nt, nf, n = r.shape
    per = n * n if full else n * (n + 1) // 2
    out = np.zeros((nf, per, 2), np.float64)
    _check(_load().orc_xengine_f64(_ptr(r), _ptr(i), nt, nf, n, int(full), _ptr(out), nthreads),
           "xengine_f64")
    if full:
        return out.reshape(nf, n, n, 2)
    return out


def accumulate_f64(run: np.ndarray, dump: np.ndarray) -> None:
    """In-place run += dump, both float64 of equal size."""
    assert run.dtype == np.float64 and run.flags.c_contiguous
    d = np.ascontiguousarray(dump, dtype=np.float64)
    assert d.size == run.size
    _check(_load().orc_accumulate_f64(_ptr(run), _ptr(d), run.size), "accumulate_f64")


def dft_real(x: np.ndarray, nfft: int, nthreads: int = 0):
    """Direct DFT.  x is int8 [nspec*nfft][ninput]; returns [nspec][nfft/2][ninput][2] double."""
    a = np.ascontiguousarray(x, dtype=np.int8)
    assert a.ndim == 2 and a.shape[0] % nfft == 0
    nspec, ninput = a.shape[0] // nfft, a.shape[1]
    out = np.zeros((nspec, nfft // 2, ninput, 2), np.float64)
    _check(_load().orc_dft_real(_ptr(a), ninput, nfft, nspec, _ptr(out), nthreads), "dft_real")
    return out


def requantize(X: np.ndarray, scale: np.ndarray):
    """Requantize a [nspec][nchan][ninput][2] double spectrum to int8 with per-channel scales."""
    a = np.ascontiguousarray(X, dtype=np.float64)
    s = np.ascontiguousarray(scale, dtype=np.float32)
    nspec, nchan, ninput, two = a.shape
    assert two == 2 and s.shape == (nchan,)
    out = np.zeros(a.shape, np.int8)
    _check(_load().orc_requantize(_ptr(a), _ptr(s), nspec, nchan, ninput, _ptr(out)),
           "requantize")
    return out


def beamform_detect(xre, xim, wre, wim, navg: int, nthreads: int = 0):
    """Beam power [B][F][T/navg] (double) of x [T][F][N] under weights w [F][B][N]."""
    xr = np.ascontiguousarray(xre, np.float64)
    xi = np.ascontiguousarray(xim, np.float64)
    wr = np.ascontiguousarray(wre, np.float64)
    wi = np.ascontiguousarray(wim, np.float64)
    nt, nf, n = xr.shape
    nf2, nb, n2 = wr.shape
    assert nf2 == nf and n2 == n and xi.shape == xr.shape and wi.shape == wr.shape
    out = np.zeros((nb, nf, nt // navg), np.float64)
    _check(_load().orc_beamform_detect(_ptr(xr), _ptr(xi), _ptr(wr), _ptr(wi), nt, nf, n, nb,
                                       navg, _ptr(out), nthreads), "beamform_detect")
    return out


def beamform_ci4(x: np.ndarray, w: np.ndarray, scale: np.ndarray, navg: int, want_y: bool = False,
                 nthreads: int = 0):
    """Integer beamformer on ci4 voltages x (uint8 [T][F][N]) with int8 weights
    w ([F][B][N][2]) and per-beam binary32 scales: returns the binary32 beam
    power [B][F][T/navg] (and the exact int64 beams [B][F][T][2] if want_y)."""
    xa = np.ascontiguousarray(x, np.uint8)
    wa = np.ascontiguousarray(w, np.int8)
    sa = np.ascontiguousarray(scale, np.float32)
    nt, nf, n = xa.shape
    nf2, nb, n2, two = wa.shape
    assert nf2 == nf and n2 == n and two == 2 and sa.shape == (nb,)
    power = np.zeros((nb, nf, nt // navg), np.float32)
    y = np.zeros((nb, nf, nt, 2), np.int64) if want_y else None
    _check(_load().orc_beamform_ci4(_ptr(xa), _ptr(wa), _ptr(sa), nt, nf, n, nb, navg, _ptr(power),
                                    _ptr(y) if want_y else None, nthreads), "beamform_ci4")
    return (power, y) if want_y else power


def tengine(x: np.ndarray, chan0: int, nfft: int, mix_num: int, mix_den: int, scale: float,
            out_bits: int = 8, want_z: bool = False, nthreads: int = 0):
    """T-engine of ci8 spectra x (int8 [S][F][N][2]): channels chan0..chan0+nfft-1
    shifted, inverse transformed (1/nfft), mixed by exp(2 pi i (mix_num t mod
    mix_den)/mix_den) and quantized to +-127 (out_bits 8) or +-7 (out_bits 4).
    Returns int32 codes [S*nfft][N][2] (and the double z' if want_z)."""
    a = np.ascontiguousarray(x, np.int8)
    nspec, nchan, ninput, two = a.shape
    assert two == 2
    q = np.zeros((nspec * nfft, ninput, 2), np.int32)
    z = np.zeros((nspec * nfft, ninput, 2), np.float64) if want_z else None
    _check(_load().orc_tengine(_ptr(a), nchan, ninput, nspec, chan0, nfft, mix_num, mix_den,
                               float(scale), out_bits, _ptr(q), _ptr(z) if want_z else None,
                               nthreads), "tengine")
    return (q, z) if want_z else q
