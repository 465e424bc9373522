"""GPU: the X-engine kernel variants and the autotuner.  Every variant must
give the same bits (integer paths) and the same binary32 values (the FP16
path: the variants differ only in which waves issue the LDS copies and how
far ahead the LDS stages are read, not in the arithmetic); the tuner keeps
the plan's accumulation count, picks a valid variant and records it in the
tune cache."""
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner, packed_vis, to_dev

pytestmark = pytest.mark.gpu


def _acc_variants(plan, d_in, T, nvar, twice=False):
    """Each variant's visibilities after one overwrite launch (and, with
    twice, a second, accumulating launch on the same input)."""
    import torch
    import paper_1708_00720_amd as bfx
    outs = []
    for v in range(nvar):
        bfx.bfx_xengine_set_variant(plan, v)
        acc = bfx.visibilities_buffer(plan)
        bfx.bfx_xengine_accumulate(plan, d_in, T, acc, overwrite=True)
        if twice:
            bfx.bfx_xengine_accumulate(plan, d_in, T, acc, overwrite=False)
        torch.cuda.synchronize()
        outs.append(acc.cpu().numpy().copy())
    return outs


@pytest.mark.parametrize("dtype", ["ci4", "ci8"])
def test_int_variants_bit_exact(dtype):
    import torch
    import paper_1708_00720_amd as bfx
    T, F, N = 200, 40, 132
    banner(f"variants {dtype} T={T} F={F} N={N}")
    raw = synth.extreme_voltages(77, T, F, N, dtype)
    plan = bfx.bfx_xengine_create(N, F, dtype)
    want = oracle.xengine_int(raw, dtype, T, F, N)
    nv = bfx.bfx_xengine_num_variants(plan)
    assert nv == (4 if dtype == "ci4" else 2)
    outs = _acc_variants(plan, to_dev(raw), T, nv)
    for v, o in enumerate(outs):
        assert np.array_equal(packed_vis(torch.from_numpy(o), F, N), want), f"variant {v}"
    # overwrite, then accumulate onto it
    outs = _acc_variants(plan, to_dev(raw), T, nv, twice=True)
    for v, o in enumerate(outs):
        assert np.array_equal(packed_vis(torch.from_numpy(o), F, N), 2 * want), f"variant {v} twice"
    plan.close()


def test_f16_variants_identical():
    import paper_1708_00720_amd as bfx
    T, F, N = 96, 24, 100
    banner(f"variants cf16 T={T} F={F} N={N}")
    x = synth.cf16_voltages(5, T, F, N)
    plan = bfx.bfx_xengine_create(N, F, "cf16")
    outs = _acc_variants(plan, to_dev(x), T, bfx.bfx_xengine_num_variants(plan))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    plan.close()


@pytest.mark.parametrize("T", [16, 17, 32, 48, 100])
def test_f16_read_ahead_many_items(T):
    """The FP16 variants that read two stages ahead hand each workgroup's
    read cursor over from item to item about seven times here (600 channels
    x 3 items of a 200-input array on at most 256 workgroups), with items of
    2 (T = 17, 32), 3 and 7 stages, and T = 16 (one stage) runs variants 0
    and 1 in their place: every variant gives the same values as variant 0,
    and variant 0 equals the oracle on two channels within the binary32
    summation bound."""
    import paper_1708_00720_amd as bfx
    F, N = 600, 200
    banner(f"variants cf16 read-ahead T={T} F={F} N={N}")
    x = synth.cf16_voltages(60 + T, T, F, N)
    plan = bfx.bfx_xengine_create(N, F, "cf16")
    nv = bfx.bfx_xengine_num_variants(plan)
    assert nv == 4
    outs = _acc_variants(plan, to_dev(x), T, nv)
    for v, o in enumerate(outs[1:], 1):
        assert np.array_equal(o, outs[0]), f"variant {v}"
    plan.close()
    chans = [0, F - 1]
    xs = x[:, chans]
    want = oracle.xengine_f64(xs[..., 0].astype(np.float64), xs[..., 1].astype(np.float64))
    got = outs[0].astype(np.float64).reshape(F, N * (N + 1) // 2, 2)[chans]
    # |dV_ij| <= gamma_{T+1} sqrt(V_ii V_jj) (binary16 products exact in binary32)
    il, jl = np.tril_indices(N)
    diag = want[:, il * (il + 1) // 2 + il, 0]                      # V_ii at each packed (i, j)
    diagj = want[:, jl * (jl + 1) // 2 + jl, 0]
    gamma = (T + 1) * 2.0 ** -24 / (1 - (T + 1) * 2.0 ** -24)
    err = np.hypot(got[..., 0] - want[..., 0], got[..., 1] - want[..., 1])
    assert np.all(err <= gamma * np.sqrt(diag * diagj))


def test_batched_variants_bit_exact():
    import paper_1708_00720_amd as bfx
    T = 77
    Ns, Fs = (36, 100, 68), (6, 20, 12)
    banner(f"variants batched ci8 T={T}")
    plan = bfx.bfx_xengine_create_batched(Ns, Fs, "ci8")
    arena = np.zeros(bfx.bfx_xengine_in_bytes(plan, T), dtype=np.uint8)
    for k, (N, F) in enumerate(zip(Ns, Fs)):
        g = synth.extreme_voltages(300 + k, T, F, N, "ci8").view(np.uint8).reshape(-1)
        io, _ = bfx.bfx_xengine_sub_offsets(plan, k, T)
        arena[io:io + g.size] = g
    outs = _acc_variants(plan, to_dev(arena), T, bfx.bfx_xengine_num_variants(plan))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    plan.close()


def test_autotune_picks_and_caches(tmp_path, monkeypatch):
    import torch
    import paper_1708_00720_amd as bfx
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("BFX_TUNE_CACHE", str(cache))
    T, F, N = 256, 16, 192
    banner(f"autotune ci4 T={T} F={F} N={N}")
    plan = bfx.bfx_xengine_create(N, F, "ci4")
    raw = synth.voltages(3, 64, F, N, "ci4", 2.5, 7)
    acc = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, to_dev(raw), 64, acc, overwrite=True)
    torch.cuda.synchronize()
    assert bfx.bfx_xengine_nacc(plan) == 64
    times = bfx.bfx_xengine_autotune(plan, T)
    print("variant times (us):", times)
    assert len(times) == 4 and all(t > 0 for t in times)  # int8 and FP8, four or eight DMA waves
    best = bfx.bfx_xengine_variant(plan)
    assert best == int(np.argmin(times))
    assert bfx.bfx_xengine_nacc(plan) == 64  # the tuning runs leave the count alone
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and f'"shape": "{N}x{F}"' in lines[0] and f'"variant": {best}' in lines[0]
    # a new plan of the same shape starts with the cached choice
    p2 = bfx.bfx_xengine_create(N, F, "ci4")
    assert bfx.bfx_xengine_variant(p2) == best
    # and the tuned plan still computes the exact result
    got = packed_vis(acc, F, N)
    assert np.array_equal(got, oracle.xengine_int(raw, "ci4", 64, F, N))
    p2.close()
    plan.close()
