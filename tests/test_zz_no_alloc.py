"""The allocation-free batched X-engine (bfx_xengine_accumulate_batched_noalloc)
against the batched plan's accumulate (the entry point it is a variant of):
bit-identical visibility arenas on two calls in a row, the second with a
smaller input, both through the C ABI."""
import numpy as np
import pytest

import synth
from gpu_util import banner

pytestmark = pytest.mark.gpu


def _arena(plan, gulps, T, bfx):
    import torch
    arena = torch.zeros(bfx.bfx_xengine_in_bytes(plan, T), dtype=torch.uint8)
    for k, g in enumerate(gulps):
        io, _ = bfx.bfx_xengine_sub_offsets(plan, k, T)
        b = g.view(np.uint8).reshape(-1)
        arena[io:io + b.size] = torch.from_numpy(b)
    return arena.cuda()


@pytest.mark.parametrize("dtype", ["ci8", "ci4"])
def test_noalloc_matches_batched_plan_twice(dtype):
    import torch
    import paper_1708_00720_amd as bfx
    sigma, clip = (8.0, 127) if dtype == "ci8" else (2.5, 7)
    cases = [
        (256, synth.BATCH_NINPUT, synth.BATCH_NCHAN),
        (100, (40, 200, 8, 96), (33, 5, 70, 2)),  # smaller: fewer subarrays, ragged sizes
    ]
    for call, (T, Ns, Fs) in enumerate(cases):
        banner(f"noalloc batched {dtype} call {call}: T={T} N={Ns} F={Fs}")
        gulps = [synth.voltages(800 + 10 * call + k, T, f, n, dtype, sigma, clip)
                 for k, (n, f) in enumerate(zip(Ns, Fs))]
        plan = bfx.bfx_xengine_create_batched(Ns, Fs, dtype)
        arena = _arena(plan, gulps, T, bfx)
        want = bfx.visibilities_buffer(plan)
        bfx.bfx_xengine_accumulate(plan, arena, T, want, overwrite=True)
        got = torch.full_like(want, -7)
        bfx.bfx_xengine_accumulate_batched_noalloc(Ns, Fs, dtype, arena, T, got)
        torch.cuda.synchronize()
        # compare every subarray's block (the padding between blocks is not written)
        for k, (n, f) in enumerate(zip(Ns, Fs)):
            _, oo = bfx.bfx_xengine_sub_offsets(plan, k, T)
            m = f * n * (n + 1) // 2 * 2
            a = got[oo // 4:oo // 4 + m].cpu().numpy()
            b = want[oo // 4:oo // 4 + m].cpu().numpy()
            assert np.array_equal(a, b), (call, k)
        plan.close()


def test_noalloc_rejects_before_launch():
    import paper_1708_00720_amd as bfx
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_accumulate_batched_noalloc([32] * 17, [4] * 17, "ci8", 0x100000, 8, 0x100000)
    assert ei.value.status == bfx.BFX_EINVAL
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_accumulate_batched_noalloc([32], [4], "ci8", 0x100000, 8, 0x100000, flags=0)
    assert ei.value.status == bfx.BFX_ENOTSUP
    # 8192 inputs x 40 channels = 83,200 items, beyond the scratch work list
    with pytest.raises(bfx.BfxError) as ei:
        bfx.bfx_xengine_accumulate_batched_noalloc([8192], [40], "ci8", 0x100000, 8, 0x100000)
    assert ei.value.status == bfx.BFX_ENOTSUP
