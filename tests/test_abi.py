"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before any HIP call (no GPU needed for these paths)."""
import ctypes

import pytest

import paper_1708_00720_amd as bfx

FAKE = 0x100000  # aligned, non-NULL; never dereferenced: the calls below fail validation first


def test_library_exports_every_header_symbol():
    syms = bfx.header_symbols()
    assert len(syms) >= 14
    lib = ctypes.CDLL(bfx.LIB_PATH)
    for name in syms:
        assert hasattr(lib, name), name


def test_strerror_and_detail():
    for code in (0, -1, -2, -3, -4, -5):
        assert bfx.bfx_strerror(code).startswith("BFX_")
    assert "unknown" in bfx.bfx_strerror(42)
    assert isinstance(bfx.bfx_last_error_detail(), str)


def test_max_ntime_bounds():
    assert bfx.bfx_xengine_max_ntime("ci8") == 65535 == (2 ** 31 - 1) // (2 * 128 ** 2)
    assert bfx.bfx_xengine_max_ntime("ci4") == 16777215 == (2 ** 31 - 1) // (2 * 8 ** 2)
    assert bfx.bfx_xengine_max_ntime("cf16") == 2 ** 63 - 1
    assert bfx.bfx_xengine_max_ntime("cf32") == -1


@pytest.mark.parametrize("ninput,nchan,dtype", [(0, 1, "ci8"), (6, 1, "ci8"), (-4, 1, "ci4"),
                                                (8196, 1, "ci4"), (32, 0, "ci8"),
                                                (32, 70000, "ci8"), (32, 4, "cf32"),
                                                (32, 4, "i8")])
def test_create_rejects(ninput, nchan, dtype):
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_create(ninput, nchan, dtype)
    assert ei.value.status == bfx.BFX_EINVAL
    assert ei.value.detail


def test_plan_sizes_host_only():
    p = bfx.bfx_xengine_create(704, 192, "ci4")
    assert bfx.bfx_xengine_in_bytes(p, 1000) == 1000 * 192 * 704
    assert bfx.bfx_xengine_out_bytes(p) == 192 * 704 * 705 // 2 * 8
    assert bfx.bfx_xengine_sub_offsets(p, 0, 1000) == (0, 0)
    assert bfx.bfx_xengine_nacc(p) == 0
    with pytest.raises(bfx.BfxError):
        bfx.bfx_xengine_sub_offsets(p, 1, 1000)
    p.close()
    q = bfx.bfx_xengine_create(32, 64, "ci8")
    assert bfx.bfx_xengine_in_bytes(q, 512) == 512 * 64 * 32 * 2
    assert bfx.bfx_xengine_out_bytes(q) == 64 * 528 * 8
    q.close()


def test_accumulate_argument_errors_before_launch():
    p = bfx.bfx_xengine_create(32, 4, "ci8")
    cases = [
        dict(d_in=0, ntime=8, d_acc=FAKE, code=bfx.BFX_EINVAL),
        dict(d_in=FAKE, ntime=8, d_acc=0, code=bfx.BFX_EINVAL),
        dict(d_in=FAKE + 4, ntime=8, d_acc=FAKE, code=bfx.BFX_EINVAL),
        dict(d_in=FAKE, ntime=0, d_acc=FAKE, code=bfx.BFX_EINVAL),
        dict(d_in=FAKE, ntime=65536, d_acc=FAKE, code=bfx.BFX_ERANGE),
    ]
    for c in cases:
        with pytest.raises(bfx.BfxError) as ei:
            bfx.bfx_xengine_accumulate(p, c["d_in"], c["ntime"], c["d_acc"], stream=0)
        assert ei.value.status == c["code"], c
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_accumulate(p, FAKE, 8, FAKE, stream=0, flags=0x10)
    assert ei.value.status == bfx.BFX_EINVAL
    assert bfx.bfx_xengine_nacc(p) == 0  # nothing was accounted
    p.close()


def test_ci4_bound_is_cumulative_without_overwrite():
    # a rejected call changes nothing; the bound counts samples since OVERWRITE
    p = bfx.bfx_xengine_create(8, 1, "ci4")
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_accumulate(p, FAKE, 16777216, FAKE, stream=0)
    assert ei.value.status == bfx.BFX_ERANGE
    assert "16777215" in ei.value.detail
    p.close()


def test_dump_argument_errors():
    p = bfx.bfx_xengine_create(32, 4, "ci8")
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_dump(p, 0, stream=0)
    assert ei.value.status == bfx.BFX_EINVAL
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_dump(p, FAKE, FAKE + 8, stream=0)
    assert ei.value.status == bfx.BFX_EINVAL
    # d_out == d_acc and no running sum: nothing to do, succeeds without a launch
    bfx.bfx_xengine_dump(p, FAKE, FAKE, None, stream=0)
    p.close()


@pytest.mark.parametrize("kw,code", [
    (dict(nfft=100), bfx.BFX_EINVAL),
    (dict(nfft=32), bfx.BFX_EINVAL),
    (dict(ninput=3), bfx.BFX_EINVAL),
    (dict(nspec=0), bfx.BFX_EINVAL),
    (dict(out="ci4"), bfx.BFX_EINVAL),
    (dict(scale=0), bfx.BFX_EINVAL),
])
def test_fengine_argument_errors(kw, code):
    args = dict(d_in=FAKE, ninput=4, nfft=64, nspec=1, scale=FAKE, d_out=FAKE, out="ci8")
    args.update(kw)
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_fengine(args["d_in"], args["ninput"], args["nfft"], args["nspec"], args["scale"],
                        args["d_out"], out=args["out"], stream=0)
    assert ei.value.status == code


@pytest.mark.parametrize("kw", [dict(ninput=48), dict(nbeam=0), dict(nbeam=300),
                                dict(ntime=17), dict(navg=0), dict(nchan=0)])
def test_beamform_argument_errors(kw):
    args = dict(ninput=64, nchan=2, nbeam=4, ntime=32, navg=16)
    args.update(kw)
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_beamform_detect(FAKE, FAKE, args["ninput"], args["nchan"], args["nbeam"],
                                args["ntime"], args["navg"], FAKE, stream=0)
    assert ei.value.status == bfx.BFX_EINVAL


def test_beamform_rejects_grids_beyond_one_launch():
    # 65536 channels x 2^22 units of 256 samples x 8 beam groups: 2^43 workgroups
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_beamform_detect(FAKE, FAKE, 64, 65536, 256, 1 << 30, 16, FAKE, stream=0)
    assert ei.value.status == bfx.BFX_ENOTSUP
    assert "workgroups" in ei.value.detail


@pytest.mark.parametrize("navg", [3, 64, 128])
def test_beamform_unsupported_navg(navg):
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_beamform_detect(FAKE, FAKE, 64, 2, 4, 384, navg, FAKE, stream=0)
    assert ei.value.status == bfx.BFX_ENOTSUP


def test_batched_create_validation_host_side():
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_create_batched([32, 6], [4, 4], "ci8")
    assert ei.value.status == bfx.BFX_EINVAL
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_create_batched([32], [4], "cf16")
    assert ei.value.status == bfx.BFX_ENOTSUP


@pytest.mark.parametrize("kw,code", [
    (dict(ninput=96), bfx.BFX_EINVAL), (dict(ninput=0), bfx.BFX_EINVAL),
    (dict(nbeam=0), bfx.BFX_EINVAL), (dict(nbeam=257), bfx.BFX_EINVAL),
    (dict(ntime=24), bfx.BFX_EINVAL), (dict(nchan=0), bfx.BFX_EINVAL),
    (dict(navg=128, ntime=256), bfx.BFX_ENOTSUP), (dict(navg=3, ntime=48), bfx.BFX_ENOTSUP),
    (dict(nchan=65536, nbeam=256, ntime=1 << 30, navg=64), bfx.BFX_ENOTSUP),
])
def test_beamform_ci4_argument_errors(kw, code):
    args = dict(ninput=64, nchan=2, nbeam=4, ntime=32, navg=16)
    args.update(kw)
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_beamform_ci4(FAKE, FAKE, FAKE, args["ninput"], args["nchan"], args["nbeam"],
                             args["ntime"], args["navg"], FAKE, stream=0)
    assert ei.value.status == code


@pytest.mark.parametrize("kw,code", [
    (dict(nfft=100), bfx.BFX_EINVAL), (dict(nfft=32), bfx.BFX_EINVAL), (dict(ninput=3), bfx.BFX_EINVAL),
    (dict(chan0=1), bfx.BFX_EINVAL), (dict(chan0=-1), bfx.BFX_EINVAL), (dict(nspec=0), bfx.BFX_EINVAL),
    (dict(mix_den=0), bfx.BFX_EINVAL), (dict(mix_num=-1), bfx.BFX_EINVAL),
    (dict(mix_den=1 << 31), bfx.BFX_EINVAL), (dict(out="cf32"), bfx.BFX_EINVAL),
    (dict(scale=float("nan")), bfx.BFX_EINVAL), (dict(nfft=1024, nchan=1024), bfx.BFX_ENOTSUP),
    (dict(ninput=12), bfx.BFX_ENOTSUP),
])
def test_tengine_argument_errors(kw, code):
    args = dict(nchan=4096, ninput=16, nspec=2, chan0=0, nfft=4096, mix_num=1, mix_den=3, scale=1.0,
                out="ci4")
    args.update(kw)
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_tengine(FAKE, args["nchan"], args["ninput"], args["nspec"], args["chan0"], args["nfft"],
                        args["mix_num"], args["mix_den"], args["scale"], FAKE, out=args["out"], stream=0)
    assert ei.value.status == code


def test_probe_argument_errors_and_counts():
    """The peak probes validate on the host and count their work exactly."""
    for call in (lambda: bfx.bfx_probe_mfma(7, 10, 4, FAKE, stream=0),
                 lambda: bfx.bfx_probe_mfma(bfx.BFX_PROBE_MFMA_I8, 0, 4, FAKE, stream=0),
                 lambda: bfx.bfx_probe_lds(bfx.BFX_PROBE_MFMA_F16, 10, 4, FAKE, stream=0),
                 lambda: bfx.bfx_probe_lds(bfx.BFX_PROBE_LDS_TR16, 10, 0, FAKE, stream=0),
                 lambda: bfx.bfx_probe_lds(bfx.BFX_PROBE_LDS_B128, 10, 4, 0, stream=0),
                 lambda: bfx.bfx_probe_read(FAKE + 8, 1024, 4, FAKE, stream=0)):
        with pytest.raises(bfx.BfxError) as ei:
            call()
        assert ei.value.status == bfx.BFX_EINVAL
    # 8 waves x 64 lanes x 12 reads per iteration
    assert bfx.bfx_probe_lds_bytes(bfx.BFX_PROBE_LDS_TR16, 3, 5) == 8 * 512 * 12 * 3 * 5
    assert bfx.bfx_probe_lds_bytes(bfx.BFX_PROBE_LDS_B128, 3, 5) == 16 * 512 * 12 * 3 * 5
    assert bfx.bfx_probe_lds_bytes(9, 3, 5) == -1
    # 8 waves x 8 MFMAs per iteration, 2 x 32 x 32 x K ops each
    assert bfx.bfx_probe_mfma_ops(bfx.BFX_PROBE_MFMA_I8, 3, 5) == 2 * 32 * 32 * 32 * 64 * 3 * 5


def test_accumulate_run64_argument_errors():
    """The fused binary64 running sum: cf16 single-array plans, 1..65535
    samples, aligned non-NULL buffers; checked before any launch."""
    p = bfx.bfx_xengine_create(64, 2, "cf16")
    for args, code in (((FAKE, 0, FAKE), bfx.BFX_EINVAL), ((FAKE, 65536, FAKE), bfx.BFX_ERANGE),
                       ((FAKE + 8, 16, FAKE), bfx.BFX_EINVAL), ((FAKE, 16, 0), bfx.BFX_EINVAL)):
        with pytest.raises(bfx.BfxError) as ei:
            bfx.bfx_xengine_accumulate_run64(p, *args, stream=0)
        assert ei.value.status == code, args
    p.close()
    for dtype in ("ci8", "ci4"):
        p = bfx.bfx_xengine_create(64, 2, dtype)
        with pytest.raises(bfx.BfxError) as ei:
            bfx.bfx_xengine_accumulate_run64(p, FAKE, 16, FAKE, stream=0)
        assert ei.value.status == bfx.BFX_ENOTSUP
        p.close()
