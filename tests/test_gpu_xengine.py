"""GPU parity of the integer X-engine against the int64 oracle (bit-exact).

Every case calls the C ABI through the Python binding and compares with
oracle.xengine_int on the same seeded input.  Full-size cases compare sampled
channels element by element and every channel through the exact Freivalds
identity (V r = sum_t x_t (x_t^H r) in int64).
"""
import numpy as np
import pytest

import oracle
import synth
from fx_checks import freivalds_check
from gpu_util import banner, packed_vis, to_dev

pytestmark = pytest.mark.gpu


def _run(raw, dtype, T, F, N, overwrite=True, acc=None):
    import torch
    import paper_1708_00720_amd as bfx
    plan = bfx.bfx_xengine_create(N, F, dtype)
    d_in = to_dev(raw)
    if acc is None:
        acc = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, d_in, T, acc, overwrite=overwrite)
    torch.cuda.synchronize()
    plan.close()
    return acc


def _unpack(raw, dtype):
    return oracle.unpack_ci4(raw) if dtype == "ci4" else oracle.unpack_ci8(raw)


def test_small_config_ci8_bit_exact():
    # 16 antennas x 2 pol = 32 inputs, 64 channels, 512 samples, ci8 sigma=8
    T, F, N = 512, 64, 32
    banner(f"xengine ci8 T={T} F={F} N={N}")
    raw = synth.voltages(1, T, F, N, "ci8", 8.0, 127)
    got = packed_vis(_run(raw, "ci8", T, F, N), F, N)
    want = oracle.xengine_int(raw, "ci8", T, F, N)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", ["ci4", "ci8"])
@pytest.mark.parametrize("T,F,N", [
    (1, 1, 4), (5, 3, 8), (63, 9, 36), (64, 2, 64), (65, 5, 68), (130, 3, 100),
    (200, 2, 132), (77, 4, 196), (129, 3, 256), (33, 1, 324), (40, 2, 452),
])
def test_ragged_shapes_extreme_values(dtype, T, F, N):
    banner(f"xengine {dtype} extremes T={T} F={F} N={N}")
    raw = synth.extreme_voltages(1000 + T + N, T, F, N, dtype)
    got = packed_vis(_run(raw, dtype, T, F, N), F, N)
    want = oracle.xengine_int(raw, dtype, T, F, N)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dtype", ["ci4", "ci8"])
def test_accumulate_adds_across_gulps(dtype):
    import torch
    import paper_1708_00720_amd as bfx
    T, F, N = 100, 6, 72
    banner(f"xengine {dtype} two gulps RMW")
    g0 = synth.extreme_voltages(1, T, F, N, dtype)
    g1 = synth.extreme_voltages(2, T, F, N, dtype)
    plan = bfx.bfx_xengine_create(N, F, dtype)
    acc = bfx.visibilities_buffer(plan)
    acc.fill_(12345)  # overwrite must ignore old contents
    bfx.bfx_xengine_accumulate(plan, to_dev(g0), T, acc, overwrite=True)
    bfx.bfx_xengine_accumulate(plan, to_dev(g1), T, acc, overwrite=False)
    torch.cuda.synchronize()
    assert bfx.bfx_xengine_nacc(plan) == 2 * T
    got = packed_vis(acc, F, N)
    want = oracle.xengine_int(g0, dtype, T, F, N) + oracle.xengine_int(g1, dtype, T, F, N)
    assert np.array_equal(got, want)


def test_ci8_bound_exact_at_tmax_and_rejected_beyond():
    import torch
    import paper_1708_00720_amd as bfx
    N, F = 4, 1
    T = bfx.bfx_xengine_max_ntime("ci8")
    banner(f"xengine ci8 constant -128 at T_max={T}")
    raw = synth.constant_voltages(T, F, N, "ci8", -128, -128)
    plan = bfx.bfx_xengine_create(N, F, "ci8")
    acc = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, to_dev(raw), T, acc, overwrite=True)
    torch.cuda.synchronize()
    got = packed_vis(acc, F, N)
    assert np.all(got[..., 0] == T * 2 * 128 * 128) and np.all(got[..., 1] == 0)
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_accumulate(plan, to_dev(raw[:1]), 1, acc, overwrite=False)
    assert ei.value.status == bfx.BFX_ERANGE
    # worst-case imaginary part: x_i = -128-128i, x_j = 127-128i at T_max
    re = np.zeros((T, F, 2), int)
    im = np.zeros((T, F, 2), int)
    re[..., 0], im[..., 0] = -128, -128
    re[..., 1], im[..., 1] = 127, -128
    raw2 = synth.pack_ci8(re, im)
    p2 = bfx.bfx_xengine_create(4, F, "ci8")
    raw4 = np.zeros((T, F, 4, 2), np.int8)
    raw4[:, :, :2] = raw2
    acc2 = bfx.visibilities_buffer(p2)
    bfx.bfx_xengine_accumulate(p2, to_dev(raw4), T, acc2, overwrite=True)
    torch.cuda.synchronize()
    got2 = packed_vis(acc2, F, 4)
    assert tuple(got2[0, 1]) == (T * 128, T * 32640)
    plan.close()
    p2.close()


def test_bound_is_cumulative_across_add_calls():
    """Two adding calls whose sum passes T_max: the second is rejected before
    launch and leaves nacc and the visibilities as they were; a call that
    lands exactly on T_max is accepted and exact."""
    import torch
    import paper_1708_00720_amd as bfx
    N, F = 4, 1
    tmax = bfx.bfx_xengine_max_ntime("ci8")
    banner(f"xengine ci8 cumulative bound over add calls, T_max={tmax}")
    raw = synth.constant_voltages(tmax, F, N, "ci8", -128, -128)
    d = to_dev(raw)
    plan = bfx.bfx_xengine_create(N, F, "ci8")
    acc = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, d, 40000, acc, overwrite=True)
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_accumulate(plan, d, 30000, acc, overwrite=False)
    assert ei.value.status == bfx.BFX_ERANGE
    assert bfx.bfx_xengine_nacc(plan) == 40000
    bfx.bfx_xengine_accumulate(plan, d, tmax - 40000, acc, overwrite=False)
    assert bfx.bfx_xengine_nacc(plan) == tmax
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_accumulate(plan, d, 1, acc, overwrite=False)
    assert ei.value.status == bfx.BFX_ERANGE
    torch.cuda.synchronize()
    got = packed_vis(acc, F, N)
    assert np.all(got[..., 0] == tmax * 2 * 128 * 128) and np.all(got[..., 1] == 0)
    plan.close()


def test_graph_capture_needs_an_overwrite_anchor():
    """An adding accumulate captured without a preceding captured overwrite is
    rejected (replays would grow the integration unchecked); a captured
    overwrite + add sequence replays exactly, with fresh data between
    replays."""
    import torch
    import paper_1708_00720_amd as bfx
    T, F, N = 64, 3, 72
    banner("xengine ci8 graph capture: overwrite anchor")
    plan = bfx.bfx_xengine_create(N, F, "ci8")
    a = torch.zeros(bfx.bfx_xengine_in_bytes(plan, T), dtype=torch.uint8, device="cuda")
    b = torch.zeros_like(a)
    acc = bfx.visibilities_buffer(plan)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside capture (kernel attributes)
        bfx.bfx_xengine_accumulate(plan, a, T, acc, overwrite=True)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g0 = torch.cuda.CUDAGraph()
    err = None
    with torch.cuda.graph(g0):
        try:
            bfx.bfx_xengine_accumulate(plan, a, T, acc, overwrite=False)
        except bfx.BfxError as e:
            err = e
    assert err is not None and err.status == bfx.BFX_ENOTSUP
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bfx.bfx_xengine_accumulate(plan, a, T, acc, overwrite=True)
        bfx.bfx_xengine_accumulate(plan, b, T, acc, overwrite=False)
    assert bfx.bfx_xengine_nacc(plan) == 2 * T
    for rep in range(3):
        ga = synth.extreme_voltages(700 + rep, T, F, N, "ci8")
        gb = synth.extreme_voltages(710 + rep, T, F, N, "ci8")
        a.copy_(torch.from_numpy(ga.view(np.uint8).reshape(-1)))
        b.copy_(torch.from_numpy(gb.view(np.uint8).reshape(-1)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        want = oracle.xengine_int(ga, "ci8", T, F, N) + oracle.xengine_int(gb, "ci8", T, F, N)
        assert np.array_equal(packed_vis(acc, F, N), want), rep
    plan.close()


def test_ci4_long_integration_split_launches():
    # more samples than one launch sums in its int32 registers (65535)
    import torch
    import paper_1708_00720_amd as bfx
    T, F, N = 70000, 1, 8
    banner(f"xengine ci4 long integration T={T}")
    raw = synth.extreme_voltages(5, T, F, N, "ci4")
    got = packed_vis(_run(raw, "ci4", T, F, N), F, N)
    want = oracle.xengine_int(raw, "ci4", T, F, N)
    assert np.array_equal(got, want)
    torch.cuda.synchronize()


def test_repeat_runs_identical():
    T, F, N = 300, 16, 200
    banner("xengine ci4 determinism")
    raw = synth.voltages(8, T, F, N, "ci4", 2.5, 7)
    a = _run(raw, "ci4", T, F, N).cpu().numpy()
    b = _run(raw, "ci4", T, F, N).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["ci4", "ci8"])
def test_dump_copy_and_running_sum(dtype):
    import torch
    import paper_1708_00720_amd as bfx
    T, F, N = 50, 3, 40
    banner(f"xengine dump {dtype}")
    raw = synth.extreme_voltages(31, T, F, N, dtype)
    plan = bfx.bfx_xengine_create(N, F, dtype)
    acc = bfx.visibilities_buffer(plan)
    out = bfx.visibilities_buffer(plan)
    run = torch.zeros(acc.numel(), dtype=torch.float64, device="cuda")
    bfx.bfx_xengine_accumulate(plan, to_dev(raw), T, acc, overwrite=True)
    for _ in range(3):
        bfx.bfx_xengine_dump(plan, acc, out, run)
    torch.cuda.synchronize()
    want = oracle.xengine_int(raw, dtype, T, F, N)
    assert np.array_equal(packed_vis(out, F, N), want)
    assert np.array_equal(run.cpu().numpy().reshape(want.shape), 3.0 * want)


def test_streaming_704_inputs_full_size():
    """352 antennas x 2 pol, 192 channels, ci4 sigma=2.5, 1000 samples per gulp."""
    import torch
    import paper_1708_00720_amd as bfx
    T, F, N = 1000, 192, 704
    banner(f"xengine ci4 full size T={T} F={F} N={N}")
    raw = synth.voltages(2, T, F, N, "ci4", 2.5, 7, gulp=0)
    plan = bfx.bfx_xengine_create(N, F, "ci4")
    acc = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, to_dev(raw), T, acc, overwrite=True)
    torch.cuda.synchronize()
    got = packed_vis(acc, F, N)
    # element-by-element on sampled channels (first, XCD boundaries, last)
    for f in (0, 7, 8, 101, 191):
        want = oracle.xengine_int(raw, "ci4", T, F, N, chans=(f, 1))
        assert np.array_equal(got[f], want[0]), f
    # exact identity on every channel
    re, im = oracle.unpack_ci4(raw)
    assert freivalds_check(got, re, im, seed=3)


def test_bench_ring_stream_704():
    """The benchmarked step itself: 100 gulps of 704 inputs x 192 channels x
    1000 ci4 samples stream through a 4-slot input ring; gulp g is correlated
    with BFX_ACC_OVERWRITE into slot g % 4 of a 4-slot visibility ring and
    handed over by dump.  After the step every visibility slot holds the
    integration of its input slot (gulps 96..99): each is checked on all 192
    channels through the exact Freivalds identity and element by element on
    two channels against the oracle."""
    import torch
    import paper_1708_00720_amd as bfx
    T, F, N, NG, NS = 1000, 192, 704, 100, 4
    banner(f"xengine ci4 bench ring stream: {NG} gulps, {NS} slots, T={T} F={F} N={N}")
    gulps = [synth.voltages(2, T, F, N, "ci4", 2.5, 7, gulp=k) for k in range(NS)]
    plan = bfx.bfx_xengine_create(N, F, "ci4")
    ring = [to_dev(g) for g in gulps]
    vis = [bfx.visibilities_buffer(plan) for _ in range(NS)]
    for g in range(NG):
        bfx.bfx_xengine_accumulate(plan, ring[g % NS], T, vis[g % NS], overwrite=True)
        bfx.bfx_xengine_dump(plan, vis[g % NS], None, None)
    torch.cuda.synchronize()
    for k in range(NS):
        got = packed_vis(vis[k], F, N)
        for f in ((k * 37) % F, F - 1 - k):
            want = oracle.xengine_int(gulps[k], "ci4", T, F, N, chans=(f, 1))
            assert np.array_equal(got[f], want[0]), (k, f)
        re, im = oracle.unpack_ci4(gulps[k])
        assert freivalds_check(got, re, im, seed=20 + k), k
        del got, re, im
    plan.close()


@pytest.mark.parametrize("dtype,T", [("ci8", 96), ("ci8", 256), ("ci8", 320), ("ci4", 512),
                                     ("ci4", 640)])
def test_items_span_several_rounds(dtype, T):
    """512 channels of 96 inputs = 512 work items on a grid of one workgroup
    per CU, so every workgroup runs at least two items back to back, with an
    item length (stages of the LDS ring) below, equal to and above the ring
    depth: the hand-over of the next item's first stage must be exact."""
    F, N = 512, 96
    banner(f"xengine {dtype} multi-round T={T} F={F} N={N}")
    sigma, clip = (8.0, 127) if dtype == "ci8" else (2.5, 7)
    raw = synth.voltages(60 + T, T, F, N, dtype, sigma, clip)
    got = packed_vis(_run(raw, dtype, T, F, N), F, N)
    want = oracle.xengine_int(raw, dtype, T, F, N)
    bad = np.nonzero(np.any(got != want, axis=(1, 2)))[0]
    assert bad.size == 0, f"{bad.size} channels differ, first {bad[:8].tolist()}"


def test_max_ninput_ci8():
    """The largest array the API takes (8192 inputs = 128 blocks, 2080 items of
    one channel), with a ragged time count: bit-exact against the oracle."""
    T, F, N = 40, 1, 8192
    banner(f"xengine ci8 max inputs T={T} F={F} N={N}")
    raw = synth.voltages(8192, T, F, N, "ci8", 8.0, 127)
    got = packed_vis(_run(raw, "ci8", T, F, N), F, N)
    want = oracle.xengine_int(raw, "ci8", T, F, N)
    assert np.array_equal(got, want)
