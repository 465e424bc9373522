"""Python binding of libbfx (the MI355X FX-correlator hot path).

Argument marshalling only: every step of the hot path runs in the HIP kernels
of ``libbfx.so``.  The functions keep the C names of ``include/bfx.h``; device
buffers may be passed as torch tensors (their ``data_ptr()`` is used) or as
raw integer addresses, and ``stream`` defaults to torch's current HIP stream.

Importing this package loads ``libbfx.so`` and raises if it is missing: there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfx.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "bfx.h")
HEADER_PATHS = [HEADER_PATH, os.path.join(os.path.dirname(_HERE), "include", "bfx_probe.h")]

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run paper_1708_00720_amd/build.py (or __graft_entry__.build())")

# torch ships its own HIP runtime: load it before libbfx.so so that the
# library binds to that same runtime (a second copy loaded first leaves torch
# without a device).
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = ctypes.CDLL(LIB_PATH)

# status codes and dtypes (include/bfx.h)
BFX_OK, BFX_EINVAL, BFX_ERANGE, BFX_EHIP, BFX_ENOTSUP, BFX_ENOMEM = 0, -1, -2, -3, -4, -5
BFX_I8, BFX_CI4, BFX_CI8, BFX_CF16, BFX_CF32, BFX_CI32, BFX_CF64 = 1, 2, 3, 4, 5, 6, 7
BFX_ACC_OVERWRITE = 1

DTYPES = {"i8": BFX_I8, "ci4": BFX_CI4, "ci8": BFX_CI8, "cf16": BFX_CF16, "cf32": BFX_CF32,
          "ci32": BFX_CI32, "cf64": BFX_CF64}

_vp, _i32, _i64, _u32, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
_st = ctypes.c_int

_SIGS = {
    "bfx_strerror": (ctypes.c_char_p, [_st]),
    "bfx_last_error_detail": (ctypes.c_char_p, []),
    "bfx_xengine_max_ntime": (_i64, [ctypes.c_int]),
    "bfx_xengine_create": (_st, [ctypes.POINTER(_vp), _i32, _i32, ctypes.c_int]),
    "bfx_xengine_create_batched": (_st, [ctypes.POINTER(_vp), _i32, ctypes.POINTER(_i32),
                                         ctypes.POINTER(_i32), ctypes.c_int]),
    "bfx_xengine_destroy": (_st, [_vp]),
    "bfx_xengine_in_bytes": (_sz, [_vp, _i64]),
    "bfx_xengine_out_bytes": (_sz, [_vp]),
    "bfx_xengine_sub_offsets": (_st, [_vp, _i32, _i64, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "bfx_xengine_nacc": (_i64, [_vp]),
    "bfx_xengine_autotune": (_st, [_vp, _i64, ctypes.POINTER(ctypes.c_float), _vp]),
    "bfx_xengine_variant": (_i32, [_vp]),
    "bfx_xengine_num_variants": (_i32, [_vp]),
    "bfx_xengine_set_variant": (_st, [_vp, _i32]),
    "bfx_tune_cache_lookup": (_i32, [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p]),
    "bfx_xengine_accumulate": (_st, [_vp, _vp, _i64, _vp, _u32, _vp]),
    "bfx_xengine_dump": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "bfx_xengine_accumulate_run64": (_st, [_vp, _vp, _i64, _vp, _vp]),
    "bfx_fengine": (_st, [_vp, _i32, _i32, _i64, _vp, _vp, ctypes.c_int, _vp]),
    "bfx_beamform_detect": (_st, [_vp, _vp, _i32, _i32, _i32, _i64, _i32, _vp, _vp]),
    "bfx_xengine_accumulate_batched_noalloc": (_st, [_i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                                     ctypes.c_int, _vp, _i64, _vp, _u32, _vp]),
    "bfx_tengine": (_st, [_vp, _i32, _i32, _i64, _i32, _i32, _i64, _i64, ctypes.c_float, _vp, ctypes.c_int, _vp]),
    "bfx_beamform_ci4": (_st, [_vp, _vp, _vp, _i32, _i32, _i32, _i64, _i32, _vp, _vp]),
    "bfx_probe_mfma": (_st, [_i32, _i32, _i32, _vp, _vp]),
    "bfx_probe_mfma_ops": (_i64, [_i32, _i32, _i32]),
    "bfx_probe_read": (_st, [_vp, _i64, _i32, _vp, _vp]),
    "bfx_probe_lds": (_st, [_i32, _i32, _i32, _vp, _vp]),
    "bfx_probe_lds_bytes": (_i64, [_i32, _i32, _i32]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class BfxError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        self.detail = detail
        super().__init__(f"{bfx_strerror(status)} -- {detail}")


def header_symbols():
    """Names of the functions declared in include/*.h."""
    text = ""
    for path in HEADER_PATHS:
        with open(path) as fh:
            text += fh.read()
    return sorted(set(re.findall(r"\b(bfx_\w+)\s*\(", text)))


def _check(status: int):
    if status != BFX_OK:
        raise BfxError(status, _lib.bfx_last_error_detail().decode())
    return status


def _addr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dtype(d) -> int:
    return DTYPES[d] if isinstance(d, str) else int(d)


# ------------------------------------------------------------------ raw C calls

def bfx_strerror(status: int) -> str:
    return _lib.bfx_strerror(status).decode()


def bfx_last_error_detail() -> str:
    return _lib.bfx_last_error_detail().decode()


def bfx_xengine_max_ntime(dtype) -> int:
    return int(_lib.bfx_xengine_max_ntime(_dtype(dtype)))


class Plan:
    """Owns a bfx_xengine plan handle; destroyed on close() or garbage collection."""

    def __init__(self, handle: int, dtype: int, subs):
        self.handle = handle
        self.dtype = dtype
        self.subs = subs

    def close(self):
        if self.handle:
            _check(_lib.bfx_xengine_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ninput(self):
        return self.subs[0][0]

    @property
    def nchan(self):
        return self.subs[0][1]


def bfx_xengine_create(ninput: int, nchan: int, dtype) -> Plan:
    h = _vp()
    _check(_lib.bfx_xengine_create(ctypes.byref(h), ninput, nchan, _dtype(dtype)))
    return Plan(h.value, _dtype(dtype), [(ninput, nchan)])


def bfx_xengine_create_batched(ninputs, nchans, dtype) -> Plan:
    n = len(ninputs)
    a = (_i32 * n)(*ninputs)
    b = (_i32 * n)(*nchans)
    h = _vp()
    _check(_lib.bfx_xengine_create_batched(ctypes.byref(h), n, a, b, _dtype(dtype)))
    return Plan(h.value, _dtype(dtype), list(zip(ninputs, nchans)))


def bfx_xengine_destroy(plan: Plan):
    plan.close()


def bfx_xengine_in_bytes(plan: Plan, ntime: int) -> int:
    return int(_lib.bfx_xengine_in_bytes(plan.handle, ntime))


def bfx_xengine_out_bytes(plan: Plan) -> int:
    return int(_lib.bfx_xengine_out_bytes(plan.handle))


def bfx_xengine_sub_offsets(plan: Plan, k: int, ntime: int):
    io, oo = _i64(), _i64()
    _check(_lib.bfx_xengine_sub_offsets(plan.handle, k, ntime, ctypes.byref(io), ctypes.byref(oo)))
    return io.value, oo.value


def bfx_xengine_nacc(plan: Plan) -> int:
    return int(_lib.bfx_xengine_nacc(plan.handle))


BFX_XENGINE_VARIANTS = 4


def bfx_xengine_autotune(plan: Plan, ntime: int, stream=None):
    """Time every kernel variant on the plan's shape and keep the fastest;
    returns the per-variant times in microseconds."""
    times = (ctypes.c_float * BFX_XENGINE_VARIANTS)()
    _check(_lib.bfx_xengine_autotune(plan.handle, ntime, times, _stream(stream)))
    return [float(t) for t in times]


def bfx_xengine_variant(plan: Plan) -> int:
    return int(_lib.bfx_xengine_variant(plan.handle))


def bfx_xengine_num_variants(plan: Plan) -> int:
    return int(_lib.bfx_xengine_num_variants(plan.handle))


def bfx_xengine_set_variant(plan: Plan, variant: int):
    _check(_lib.bfx_xengine_set_variant(plan.handle, variant))


def bfx_tune_cache_lookup(path: str, arch: str, dtype: str, shape: str) -> int:
    return int(_lib.bfx_tune_cache_lookup(path.encode(), arch.encode(), dtype.encode(), shape.encode()))


def bfx_xengine_accumulate(plan: Plan, d_in, ntime: int, d_acc, overwrite: bool = True,
                           stream=None, flags: int | None = None):
    fl = (BFX_ACC_OVERWRITE if overwrite else 0) if flags is None else flags
    _check(_lib.bfx_xengine_accumulate(plan.handle, _addr(d_in), ntime, _addr(d_acc), fl,
                                       _stream(stream)))


def bfx_xengine_dump(plan: Plan, d_acc, d_out=None, d_run64=None, stream=None):
    _check(_lib.bfx_xengine_dump(plan.handle, _addr(d_acc), _addr(d_out), _addr(d_run64),
                                 _stream(stream)))


def bfx_xengine_accumulate_run64(plan: Plan, d_in, ntime: int, d_run64, stream=None):
    _check(_lib.bfx_xengine_accumulate_run64(plan.handle, _addr(d_in), ntime, _addr(d_run64), _stream(stream)))


def bfx_fengine(d_in, ninput: int, nfft: int, nspec: int, d_scale, d_out, out="ci8", stream=None):
    _check(_lib.bfx_fengine(_addr(d_in), ninput, nfft, nspec, _addr(d_scale), _addr(d_out),
                            _dtype(out), _stream(stream)))


def bfx_beamform_detect(d_x, d_w, ninput: int, nchan: int, nbeam: int, ntime: int, navg: int,
                        d_out, stream=None):
    _check(_lib.bfx_beamform_detect(_addr(d_x), _addr(d_w), ninput, nchan, nbeam, ntime, navg,
                                    _addr(d_out), _stream(stream)))


def bfx_xengine_accumulate_batched_noalloc(ninputs, nchans, dtype, d_in, ntime: int, d_acc,
                                           stream=None, flags: int = BFX_ACC_OVERWRITE):
    n = len(ninputs)
    a = (_i32 * n)(*ninputs)
    b = (_i32 * n)(*nchans)
    _check(_lib.bfx_xengine_accumulate_batched_noalloc(n, a, b, _dtype(dtype), _addr(d_in), ntime,
                                                       _addr(d_acc), flags, _stream(stream)))


def bfx_tengine(d_in, nchan: int, ninput: int, nspec: int, chan0: int, nfft: int, mix_num: int,
                mix_den: int, scale: float, d_out, out="ci4", stream=None):
    _check(_lib.bfx_tengine(_addr(d_in), nchan, ninput, nspec, chan0, nfft, mix_num, mix_den, scale,
                            _addr(d_out), _dtype(out), _stream(stream)))


def bfx_beamform_ci4(d_x, d_w, d_scale, ninput: int, nchan: int, nbeam: int, ntime: int, navg: int,
                     d_out, stream=None):
    _check(_lib.bfx_beamform_ci4(_addr(d_x), _addr(d_w), _addr(d_scale), ninput, nchan, nbeam, ntime,
                                 navg, _addr(d_out), _stream(stream)))


BFX_PROBE_MFMA_I8, BFX_PROBE_MFMA_F16 = 0, 1


def bfx_probe_mfma(kind: int, iters: int, nblocks: int, d_sink, stream=None):
    _check(_lib.bfx_probe_mfma(kind, iters, nblocks, _addr(d_sink), _stream(stream)))


def bfx_probe_mfma_ops(kind: int, iters: int, nblocks: int) -> int:
    return int(_lib.bfx_probe_mfma_ops(kind, iters, nblocks))


def bfx_probe_read(d_buf, nbytes: int, nblocks: int, d_sink, stream=None):
    _check(_lib.bfx_probe_read(_addr(d_buf), nbytes, nblocks, _addr(d_sink), _stream(stream)))


BFX_PROBE_LDS_TR16, BFX_PROBE_LDS_TR8, BFX_PROBE_LDS_B128 = 2, 3, 4


def bfx_probe_lds(kind: int, iters: int, nblocks: int, d_sink, stream=None):
    _check(_lib.bfx_probe_lds(kind, iters, nblocks, _addr(d_sink), _stream(stream)))


def bfx_probe_lds_bytes(kind: int, iters: int, nblocks: int) -> int:
    return int(_lib.bfx_probe_lds_bytes(kind, iters, nblocks))


# ------------------------------------------------------------------ conveniences

def visibilities_buffer(plan: Plan, device="cuda"):
    """A zeroed torch tensor sized for the plan's visibility buffer (int32 or float32 pairs)."""
    import torch
    nbytes = bfx_xengine_out_bytes(plan)
    dt = torch.float32 if plan.dtype == BFX_CF16 else torch.int32
    return torch.zeros(nbytes // 4, dtype=dt, device=device)
