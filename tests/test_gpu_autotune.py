"""GPU: the X-engine kernel variants and the autotuner.  Every variant must
give the same bits (integer paths) and the same binary32 values (the FP16
path: the variants differ only in which waves issue the LDS copies, not in
the arithmetic); the tuner keeps the plan's accumulation count, picks a
valid variant and records it in the tune cache."""
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
