"""GPU parity of the ci4 X-engine on FP8 MFMA (kernel variants 2 and 3 of a
ci4 plan) against the int64 oracle: bit-exact int32 visibilities.

Every 4-bit value is exact in e4m3 and every partial sum is an integer below
2^23, so binary32 accumulation gives the exact integers.  Cases: the whole
code range (-8 included) over ragged shapes, the most negative codes at the
largest per-launch sample count (the largest partial sums) and beyond it
(split launches), and the 704-input workload (sampled channels plus
Freivalds on all 192)."""
import numpy as np
import pytest

import oracle
import synth
from fx_checks import freivalds_check
from gpu_util import banner, packed_vis, to_dev

pytestmark = pytest.mark.gpu


def _run(raw, T, F, N, variant, overwrite=True):
    import torch
    import paper_1708_00720_amd as bfx
    plan = bfx.bfx_xengine_create(N, F, "ci4")
    bfx.bfx_xengine_set_variant(plan, variant)
    acc = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, to_dev(raw), T, acc, overwrite=overwrite)
    torch.cuda.synchronize()
    plan.close()
    return packed_vis(acc, F, N)


@pytest.mark.parametrize("variant", [2, 3])
@pytest.mark.parametrize("T,F,N", [(1, 1, 4), (63, 9, 36), (64, 2, 64), (65, 5, 68), (130, 3, 100),
                                   (77, 4, 196), (129, 3, 256), (40, 2, 452)])
def test_fp8_extremes_ragged(variant, T, F, N):
    banner(f"xengine ci4 fp8 v{variant} extremes T={T} F={F} N={N}")
    raw = synth.extreme_voltages(2000 + T + N, T, F, N, "ci4")
    assert np.array_equal(_run(raw, T, F, N, variant), oracle.xengine_int(raw, "ci4", T, F, N))


@pytest.mark.parametrize("T", [65535, 70000])
def test_fp8_largest_sums(T):
    """-8-8i everywhere: Re V = T * 128 per pair, the largest partial sums a
    launch can hold (65535 samples: 8,388,480 < 2^23); 70000 samples take two
    launches."""
    F, N = 1, 8
    banner(f"xengine ci4 fp8 -8-8i T={T}")
    raw = synth.constant_voltages(T, F, N, "ci4", -8, -8)
    got = _run(raw, T, F, N, 2)
    assert np.all(got[..., 0] == T * 128) and np.all(got[..., 1] == 0)
    # and a mixed-sign pair: x_i = -8-8i, x_j = 7-8i -> Re = T(-56+64), Im = T(-8*7 - (-8)(-8))
    re = np.full((T, F, N), -8, int)
    im = np.full((T, F, N), -8, int)
    re[:, :, 1::2] = 7
    raw2 = synth.pack_ci4(re, im)
    assert np.array_equal(_run(raw2, T, F, N, 3), oracle.xengine_int(raw2, "ci4", T, F, N))


def test_fp8_workload_704():
    T, F, N = 1000, 192, 704
    banner(f"xengine ci4 fp8 workload T={T} F={F} N={N}")
    raw = synth.voltages(2, T, F, N, "ci4", 2.5, 7, gulp=1)
    got = _run(raw, T, F, N, 2)
    for f in (0, 9, 191):
        assert np.array_equal(got[f], oracle.xengine_int(raw, "ci4", T, F, N, chans=(f, 1))[0]), f
    re, im = oracle.unpack_ci4(raw)
    assert freivalds_check(got, re, im, seed=5)
