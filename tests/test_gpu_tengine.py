"""GPU parity of the T-engine (bfx_tengine: band selection, channel shift,
inverse transform, complex mixer, 8+8 / 4+4 quantization) against the oracle.

The GPU computes in binary32 and the oracle in double, so a code may round the
other way only where scale * z' lies within the binary32 error of a
half-integer.  The window is set a priori: the inverse transform's normwise
error 8 log2(N) u ||X||_2 / sqrt(N) (X the band of that frame and input), the
mixer's phase and product rounding 25 u |z'|, and the scale product's own
rounding u |scale z'|, all times scale.  Every other code must be equal, and
flagged codes may differ by one at most.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner, to_dev

pytestmark = pytest.mark.gpu

NFFT = 4096
U32 = 2.0 ** -24


def _run(x, nchan, ninput, nspec, chan0, mix_num, mix_den, scale, out):
    import torch
    import paper_1708_00720_amd as bfx
    per = 2 if out == "ci8" else 1
    d_out = torch.full((nspec * NFFT * ninput * per,), 0x55, dtype=torch.uint8, device="cuda")
    bfx.bfx_tengine(to_dev(x), nchan, ninput, nspec, chan0, NFFT, mix_num, mix_den, scale, d_out, out=out)
    torch.cuda.synchronize()
    h = d_out.cpu().numpy()
    if out == "ci8":
        q = h.view(np.int8).reshape(nspec * NFFT, ninput, 2).astype(np.int32)
        return q[..., 0], q[..., 1]
    re, im = oracle.unpack_ci4(h.reshape(nspec * NFFT, ninput))
    return re, im


def _check(x, gre, gim, chan0, mix_num, mix_den, scale, out, frames, inputs, run_frames=None):
    """Compare the GPU codes of (frames x inputs) with the oracle's.  The
    oracle runs on each listed frame alone, which gives its mixer the time
    index n instead of s * nfft + n: the caller lists frames s with
    mix_num * s * nfft = 0 (mod mix_den), where the two phases agree.  When
    x and the codes hold only some frames of the run, run_frames gives each
    listed frame's index in the run (for that condition)."""
    nflag = ndiff = total = 0
    for k, s in enumerate(frames):
        rs = s if run_frames is None else run_frames[k]
        assert (mix_num * rs * NFFT) % mix_den == 0
        sub = np.ascontiguousarray(x[s:s + 1][:, :, inputs])
        q, z = oracle.tengine(sub, chan0, NFFT, mix_num, mix_den, scale,
                              out_bits=8 if out == "ci8" else 4, want_z=True)
        band = sub[0, chan0:chan0 + NFFT].astype(np.float64)        # [nfft][n][2]
        xn = np.sqrt((band ** 2).sum(axis=(0, 2)))                   # ||X||_2 per input
        fft_err = 8 * 12 * U32 * xn / np.sqrt(NFFT)                  # [n]
        zs = scale * z                                               # [nfft][n][2]
        win = scale * (fft_err[None, :, None] + 25 * U32 * np.hypot(z[..., 0], z[..., 1])[..., None]) \
            + 2 * U32 * np.abs(zs)
        near = np.abs(np.abs(zs - np.floor(zs)) - 0.5) < win
        g = np.stack([gre[s * NFFT:(s + 1) * NFFT][:, inputs], gim[s * NFFT:(s + 1) * NFFT][:, inputs]], -1)
        d = g - q
        bad = (d != 0) & ~near
        assert not bad.any(), (s, np.argwhere(bad)[:5])
        assert np.all(np.abs(d) <= 1)
        nflag += int(near.sum())
        ndiff += int((d != 0).sum())
        total += d.size
    return total, nflag, ndiff


@pytest.mark.parametrize("out,scale", [("ci8", 100.0), ("ci4", 6.0), ("ci8", 3.0), ("ci4", 0.7)])
def test_extreme_codes_small(out, scale):
    """Uniform codes over the whole int8 range (-128 included), a band inside
    a wider channel axis, a mixer of 5/4 channel (period 4 frames), five
    frames checked at frames 0 and 4; the large scales saturate many
    outputs."""
    nspec, nchan, ninput, chan0 = 5, NFFT + 40, 16, 40
    mix_num, mix_den = 5, 4 * NFFT
    banner(f"tengine {out} extremes scale={scale}")
    x = synth.extreme_voltages(77, nspec, nchan, ninput, "ci8")
    gre, gim = _run(x, nchan, ninput, nspec, chan0, mix_num, mix_den, scale, out)
    total, nflag, ndiff = _check(x, gre, gim, chan0, mix_num, mix_den, scale, out, (0, 4),
                                 list(range(ninput)))
    lim = 127 if out == "ci8" else 7
    assert gre.min() >= -lim and gim.min() >= -lim
    assert gre.max() <= lim and gim.max() <= lim
    print(f"{total} codes, {nflag} in the tie window, {ndiff} differ by one; "
          f"{int((np.abs(gre) == lim).sum())} saturated real parts")


def test_workload_sampled():
    """The benchmarked shape: 256 inputs, 128 frames of 4096-channel ci8
    spectra (rounded Gaussian sigma 8), the whole 4096-channel band, mixer 1/3
    channel (period 3 frames), 4+4 output; frames 0, 3 and 126 on 16 inputs
    each."""
    nspec, nchan, ninput, chan0 = 128, NFFT, 256, 0
    mix_num, mix_den, scale = 1, 3 * NFFT, 16.0
    banner("tengine ci4 bench shape: 256 inputs, 128 frames")
    x = synth.voltages(12, nspec, nchan, ninput, "ci8", 8.0, 127)
    gre, gim = _run(x, nchan, ninput, nspec, chan0, mix_num, mix_den, scale, "ci4")
    inputs = [0, 1, 7, 8, 100, 128, 200, 255, 31, 32, 63, 64, 65, 129, 190, 254]
    total, nflag, ndiff = _check(x, gre, gim, chan0, mix_num, mix_den, scale, "ci4", (0, 3, 126), inputs)
    print(f"{total} codes, {nflag} in the tie window, {ndiff} differ by one")


@pytest.mark.parametrize("out", ["ci8", "ci4"])
def test_fewest_inputs_odd_frames_no_mixer(out):
    """One group of 8 inputs (the smallest), 9 frames (the last frame group
    of the grid is partly empty), no mixer (mix_num 0): every frame's codes
    against the oracle."""
    nspec, nchan, ninput, chan0 = 9, NFFT, 8, 0
    banner(f"tengine {out} 8 inputs, 9 frames, no mixer")
    x = synth.voltages(13, nspec, nchan, ninput, "ci8", 8.0, 127)
    scale = 16.0 if out == "ci8" else 4.0
    gre, gim = _run(x, nchan, ninput, nspec, chan0, 0, 1, scale, out)
    total, nflag, ndiff = _check(x, gre, gim, chan0, 0, 1, scale, out, tuple(range(nspec)), list(range(ninput)))
    print(f"{total} codes, {nflag} in the tie window, {ndiff} differ by one")


def test_largest_mixer_denominator():
    """mix_den = 2^31 - 1 (the largest accepted; prime, so the phase index
    never repeats within the run) with mix_num = 7: frame 0 against the
    oracle, whose exact integer phase index the kernel must reproduce."""
    nspec, nchan, ninput, chan0 = 2, NFFT, 16, 0
    mix_num, mix_den, scale = 7, 2 ** 31 - 1, 16.0
    banner("tengine ci8 mix_den 2^31-1")
    x = synth.voltages(14, nspec, nchan, ninput, "ci8", 8.0, 127)
    gre, gim = _run(x, nchan, ninput, nspec, chan0, mix_num, mix_den, scale, "ci8")
    total, nflag, ndiff = _check(x, gre, gim, chan0, mix_num, mix_den, scale, "ci8", (0,), list(range(ninput)))
    print(f"{total} codes, {nflag} in the tie window, {ndiff} differ by one")


def test_most_inputs_sampled():
    """65536 inputs (the largest accepted), 9 frames of 4096 channels: the
    input passes 2^32 bytes (frame 8 starts at 4.3 GB) and a frame's band
    spans 2^29 bytes, so the kernel's 32-bit lane and row offsets reach their
    largest values.  Uniform codes over the whole int8 range, 4+4 output,
    mixer 1/4 channel (period 4 frames); 12 sampled inputs of frames 0 and 8
    against the oracle."""
    import torch
    import paper_1708_00720_amd as bfx
    nspec, nchan, ninput, chan0 = 9, NFFT, 65536, 0
    mix_num, mix_den, scale = 1, 4 * NFFT, 2.0
    frames = (0, 8)
    inputs = [0, 1, 7, 8, 4095, 4096, 32767, 32768, 65527, 65528, 65534, 65535]
    banner(f"tengine ci4 ninput={ninput} nspec={nspec}")
    gen = torch.Generator(device="cuda").manual_seed(15)
    d_in = torch.randint(-128, 128, (nspec * nchan * ninput * 2,), dtype=torch.int8, device="cuda", generator=gen)
    idx = torch.tensor(inputs, device="cuda")
    fidx = torch.tensor(frames, device="cuda")
    x = d_in.view(nspec, nchan, ninput, 2).index_select(0, fidx).index_select(2, idx).cpu().numpy()
    d_out = torch.full((nspec * NFFT * ninput,), 0x55, dtype=torch.uint8, device="cuda")
    bfx.bfx_tengine(d_in, nchan, ninput, nspec, chan0, NFFT, mix_num, mix_den, scale, d_out, out="ci4")
    torch.cuda.synchronize()
    h = d_out.view(nspec, NFFT, ninput).index_select(0, fidx).index_select(2, idx).cpu().numpy()
    del d_in, d_out
    gre, gim = oracle.unpack_ci4(h.reshape(len(frames) * NFFT, len(inputs)))
    # compact frame c is frame frames[c] of the run
    total, nflag, ndiff = _check(x, gre, gim, chan0, mix_num, mix_den, scale, "ci4", range(len(frames)),
                                 list(range(len(inputs))), run_frames=frames)
    print(f"{total} codes, {nflag} in the tie window, {ndiff} differ by one")
