"""GPU parity of the integer beamformer on 4+4-bit voltages (bfx_beamform_ci4)
against the oracle: bit-exact binary32 beam power.

The beams y and the detected sums S are exact integers on both sides and the
one conversion P = fl32(fl64(scale^2) * fl64(S)) takes the same rounding
steps, so every output word must be equal.  Cases: extreme codes (-8 voltages,
-128 weights) over ragged shapes and every navg, a sum S above 2^53 (where the
conversion to double rounds), and the full workload (512 inputs, 2048
channels, 1024 samples, 32 beams, navg 16) on sampled channels.  Up to 512
inputs the library runs a persistent kernel whose workgroups walk many
(channel, beam group, 1024-sample) items in turn; beyond that, one workgroup
per (channel, 256 samples, beam group).  Both are covered, and a ragged case
with thousands of items checks the item-to-item hand-over.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner, to_dev

pytestmark = pytest.mark.gpu


def _run(x, w, scale, N, F, B, T, navg, out_offset=0):
    """Run the library; the output starts out_offset floats into its buffer."""
    import torch
    import paper_1708_00720_amd as bfx
    n = B * F * (T // navg)
    buf = torch.full((n + out_offset,), float("nan"), dtype=torch.float32, device="cuda")
    out = buf[out_offset:]
    bfx.bfx_beamform_ci4(to_dev(x), to_dev(w), torch.from_numpy(np.asarray(scale, np.float32)).cuda(),
                         N, F, B, T, navg, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(B, F, T // navg)


@pytest.mark.parametrize("N,F,B,T,navg", [
    (64, 1, 1, 16, 16), (64, 3, 5, 48, 1), (128, 2, 32, 256, 2), (192, 5, 33, 320, 4),
    (320, 3, 40, 512, 8), (512, 9, 64, 272, 16), (256, 4, 7, 640, 32), (448, 2, 16, 768, 64),
    (576, 3, 17, 272, 16), (1024, 2, 33, 512, 64),
    # a stage that ends inside the data (ntime not a multiple of 16)
    (64, 2, 3, 37, 1), (256, 3, 9, 1000, 8),
    # above 512 inputs at navg 16 and 32: a full 256-sample unit and a partial one, 37 beams
    (704, 3, 37, 400, 16), (576, 2, 9, 320, 32),
])
def test_extreme_codes_ragged(N, F, B, T, navg):
    banner(f"beamform_ci4 extremes N={N} F={F} B={B} T={T} navg={navg}")
    x = synth.extreme_voltages(300 + N + B, T, F, N, "ci4")
    w = synth.extreme_int8_weights(400 + T, F, B, N)
    scale = np.random.default_rng(N * B).uniform(0.001, 3.0, B).astype(np.float32)
    got = _run(x, w, scale, N, F, B, T, navg)
    want = oracle.beamform_ci4(x, w, scale, navg)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_most_negative_codes_large_sums():
    """Every voltage -8-8i and every weight -128-128i at the largest input
    count: y = -128 * 8 * 8192 * 2i per sample, and the window sum over 64
    samples (1.8e16) lies above 2^53, where the conversion to double rounds."""
    N, F, B, T, navg = 8192, 1, 3, 128, 64
    banner(f"beamform_ci4 most negative codes N={N} navg={navg}")
    x = synth.constant_voltages(T, F, N, "ci4", -8, -8)
    w = np.full((F, B, N, 2), -128, np.int8)
    scale = np.array([1.0, 0.1, 3.0e-5], np.float32)
    got = _run(x, w, scale, N, F, B, T, navg)
    want = oracle.beamform_ci4(x, w, scale, navg)
    S = navg * (2 * 128 * 8 * N) ** 2
    assert S > 2 ** 53
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_full_size_sampled_channels():
    """512 inputs, 2048 channels, 1024 samples, 32 quantized unit-modulus
    beams, navg 16: sampled channels bit-exact against the oracle."""
    N, F, B, T, navg = 512, 2048, 32, 1024, 16
    banner(f"beamform_ci4 full size N={N} F={F} B={B} T={T} navg={navg}")
    x = synth.voltages(9, T, F, N, "ci4", 2.5, 7)
    w, scale = synth.int8_steering_weights(10, F, B, N)
    got = _run(x, w, scale, N, F, B, T, navg)
    for f in (0, 1, 7, 8, 1000, 2047):
        want = oracle.beamform_ci4(np.ascontiguousarray(x[:, f:f + 1]), w[f:f + 1], scale, navg)
        assert np.array_equal(got[:, f:f + 1].view(np.uint32), want.view(np.uint32)), f


def test_many_items_ragged():
    """128 inputs, 520 channels, 40 beams (two beam groups, the second
    partial), 2304 samples (two whole 1024-sample items and a partial one),
    navg 32: about 3000 items, so every workgroup hands over between items of
    different channels, beam groups and time blocks.  Sampled channels are
    checked bit-exact."""
    N, F, B, T, navg = 128, 520, 40, 2304, 32
    banner(f"beamform_ci4 many items N={N} F={F} B={B} T={T} navg={navg}")
    x = synth.extreme_voltages(31, T, F, N, "ci4")
    w = synth.extreme_int8_weights(32, F, B, N)
    scale = np.random.default_rng(33).uniform(0.001, 3.0, B).astype(np.float32)
    got = _run(x, w, scale, N, F, B, T, navg)
    for f in (0, 1, 7, 8, 255, 256, 263, 511, 512, 519):
        want = oracle.beamform_ci4(np.ascontiguousarray(x[:, f:f + 1]), w[f:f + 1], scale, navg)
        assert np.array_equal(got[:, f:f + 1].view(np.uint32), want.view(np.uint32)), f


@pytest.mark.parametrize("navg", [16, 32, 64])
@pytest.mark.parametrize("out_offset", [0, 1])
def test_window_rows(navg, out_offset):
    """navg 16 to 64, where a lane gathers 4, 2 or 1 consecutive windows of its
    beam and stores them once per 1024-sample item: 1088 samples (a second
    item of 64 samples, so only the first windows of its first time quarter
    exist), 68, 34 or 17 windows per row, 40 beams (a partial beam group).
    With the output 16- or 8-byte aligned a lane's windows leave at once; one
    float further on, window by window.  Every channel bit-exact."""
    N, F, B, T = 256, 5, 40, 1088
    banner(f"beamform_ci4 window rows N={N} F={F} B={B} T={T} navg={navg} out_offset={out_offset}")
    x = synth.extreme_voltages(41, T, F, N, "ci4")
    w = synth.extreme_int8_weights(42, F, B, N)
    scale = np.random.default_rng(43).uniform(0.001, 3.0, B).astype(np.float32)
    got = _run(x, w, scale, N, F, B, T, navg, out_offset)
    want = oracle.beamform_ci4(x, w, scale, navg)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
