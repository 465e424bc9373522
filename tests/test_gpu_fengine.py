"""GPU parity of the F-engine (4096-point real FFT + requantize) against the oracle.

* binary32 spectrum vs the double direct DFT: normwise relative error per
  (frame, input) <= 1e-6;
* ci8 codes vs the oracle's requantizer applied to the double spectrum: equal,
  except at near-ties where the binary32 transform may round the other way,
  which must differ by exactly one code.  The tie window comes from an a priori
  error bound of the binary32 FFT, not from the GPU's output;
* the F+X workload (256 inputs, 512 frames) in stages: binary32 spectra on
  sampled frames and inputs; every ci8 code of two whole frames; the integer
  X-engine on the GPU's own ci8 spectra, bit-exact against the oracle on the
  same bytes; and the closed-form visibility magnitude and phase slope of a
  bin-centred tone with per-input delays.
"""
import numpy as np
import pytest

import oracle
import synth
from fx_checks import freivalds_check
from gpu_util import banner, packed_vis, to_dev

pytestmark = pytest.mark.gpu

NFFT, NCHAN = 4096, 2048
U32 = 2.0 ** -24  # unit roundoff of binary32


def _run_f(x, ninput, nspec, scale, out_kind):
    import torch
    import paper_1708_00720_amd as bfx
    d_in = to_dev(x)
    d_scale = torch.from_numpy(np.asarray(scale, np.float32)).cuda()
    if out_kind == "cf32":
        out = torch.zeros(nspec * NCHAN * ninput * 2, dtype=torch.float32, device="cuda")
    else:
        out = torch.zeros(nspec * NCHAN * ninput * 2, dtype=torch.int8, device="cuda")
    bfx.bfx_fengine(d_in, ninput, NFFT, nspec, d_scale, out, out=out_kind)
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(nspec, NCHAN, ninput, 2)


def _oracle_spectrum(x, ninput, frames, inputs):
    """Double DFT of the selected (frame, input) sequences; returns {(s, i): complex array}."""
    res = {}
    for s in frames:
        sub = np.ascontiguousarray(x[s * NFFT:(s + 1) * NFFT][:, inputs])
        X = oracle.dft_real(sub, NFFT)[0]  # [2048][len(inputs)][2]
        for col, i in enumerate(inputs):
            res[(s, i)] = X[:, col, 0] + 1j * X[:, col, 1]
    return res


def _normwise(got, want):
    return np.linalg.norm(got - want) / np.linalg.norm(want)


@pytest.mark.parametrize("kind", ["tone", "fullrange"])
def test_spectrum_binary32_normwise(kind):
    ninput, nspec = 32, 3
    banner(f"fengine cf32 {kind} ninput={ninput} nspec={nspec}")
    if kind == "tone":
        x, _ = synth.adc_tone(30, ninput, NFFT, nspec)
    else:
        x = np.random.default_rng(31).integers(-128, 128, (NFFT * nspec, ninput)).astype(np.int8)
    got = _run_f(x, ninput, nspec, np.ones(NCHAN), "cf32")
    want = _oracle_spectrum(x, ninput, range(nspec), list(range(ninput)))
    worst = 0.0
    for (s, i), w in want.items():
        g = got[s, :, i, 0].astype(np.float64) + 1j * got[s, :, i, 1]
        worst = max(worst, _normwise(g, w))
    print(f"worst normwise relative error {worst:.3e}")
    assert worst <= 1e-6


def _tie_window(x_block):
    """A priori bound on |X32 - X64| per element for a 4096-point binary32 FFT.

    Each radix-16 pass adds a relative error of at most a few units of
    roundoff to every element it touches; a conservative per-element bound is
    c * log2(N) * u * ||x||_2 with c = 8 (summation + twiddle rounding).
    """
    return 8 * 12 * U32 * np.linalg.norm(x_block.astype(np.float64))


def _check_ci8_codes(x, got, scale, frames, inputs):
    """ci8 codes of the GPU against the oracle's requantizer on the double
    spectrum.  A code may differ only where s*v lies within the a priori
    binary32 error of a half-integer: the FFT bound scaled by s, plus the
    rounding of the binary32 product s*v itself (u |s v|).  Such codes must
    differ by exactly one.  Returns (codes, flagged, differing)."""
    nflag = nmiss = total = 0
    for s in frames:
        blk = np.ascontiguousarray(x[s * NFFT:(s + 1) * NFFT][:, inputs])
        X = oracle.dft_real(blk, NFFT)                      # [1][2048][n][2]
        q = oracle.requantize(X, scale)[0]                  # [2048][n][2]
        for col, i in enumerate(inputs):
            prod = X[0, :, col, :] * scale[:, None].astype(np.float64)
            win = _tie_window(blk[:, col]) * float(scale[0]) + U32 * np.abs(prod)
            near = np.abs(np.abs(prod - np.floor(prod)) - 0.5) < win
            diff = got[s, :, i, :].astype(int) - q[:, col, :].astype(int)
            total += diff.size
            nflag += int(near.sum())
            bad = (diff != 0) & ~near
            assert not bad.any(), (s, i, np.argwhere(bad)[:5])
            assert np.all(np.abs(diff[near]) <= 1)
            nmiss += int((diff != 0).sum())
    return total, nflag, nmiss


def test_ci8_equal_except_flagged_near_ties():
    ninput, nspec = 32, 4
    banner(f"fengine ci8 ninput={ninput} nspec={nspec}")
    x, _ = synth.adc_tone(32, ninput, NFFT, nspec)
    scale = synth.fengine_scale(NCHAN)
    got = _run_f(x, ninput, nspec, scale, "ci8")
    total, nflag, nmiss = _check_ci8_codes(x, got, scale, range(nspec), list(range(ninput)))
    print(f"{total} codes, {nflag} inside the tie window, {nmiss} differ by one")
    assert got.min() >= -127  # saturation never emits -128


@pytest.fixture(scope="module")
def fx_full():
    """The F+X workload run once on the GPU: 256 real inputs x 512 frames of
    4096 (noise sigma 16 plus a unit tone at channel 777 with per-input
    delays), F-engine to ci8, then the integer X-engine over the 512 spectra
    of every channel.  Returns the input, the delays, the GPU's ci8 spectra
    and its visibilities (host copies)."""
    import torch
    import paper_1708_00720_amd as bfx
    ninput, nspec = 256, 512
    banner("F+X full size: fengine ci8 -> xengine ci8 (256 inputs, 2048 ch, 512 spectra)")
    x, tau = synth.adc_tone(3, ninput, NFFT, nspec)
    scale = synth.fengine_scale(NCHAN)
    d_in = to_dev(x)
    d_scale = torch.from_numpy(scale).cuda()
    spec = torch.zeros(nspec * NCHAN * ninput * 2, dtype=torch.int8, device="cuda")
    bfx.bfx_fengine(d_in, ninput, NFFT, nspec, d_scale, spec, out="ci8")
    plan = bfx.bfx_xengine_create(ninput, NCHAN, "ci8")
    vis = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, spec, nspec, vis, overwrite=True)
    torch.cuda.synchronize()
    plan.close()
    spec_h = spec.cpu().numpy().reshape(nspec, NCHAN, ninput, 2)
    vis_h = packed_vis(vis, NCHAN, ninput)
    del d_in, spec, vis
    return dict(x=x, tau=tau, scale=scale, spec=spec_h, vis=vis_h, ninput=ninput, nspec=nspec)


def test_full_size_sampled_spectra(fx_full):
    """256 inputs, 512 frames (the F+X configuration), binary32 spectrum sampled."""
    ninput, nspec = 256, 512
    banner(f"fengine cf32 full size ninput={ninput} nspec={nspec}")
    x = fx_full["x"]
    got = _run_f(x, ninput, nspec, np.ones(NCHAN), "cf32")
    frames = (0, 7, 8, 255, 511)
    inputs = [0, 1, 15, 16, 17, 128, 254, 255]
    want = _oracle_spectrum(x, ninput, frames, inputs)
    worst = 0.0
    for (s, i), w in want.items():
        g = got[s, :, i, 0].astype(np.float64) + 1j * got[s, :, i, 1]
        worst = max(worst, _normwise(g, w))
    print(f"worst normwise relative error {worst:.3e}")
    assert worst <= 1e-6


def test_fx_ci8_full_size_near_ties(fx_full):
    """Stage (ii) at the F+X size: every code of frames 0 and 511 (all 256
    inputs) equals the oracle's, except flagged near-ties (off by one)."""
    d = fx_full
    banner("F+X stage ii: ci8 codes, frames 0 and 511, 256 inputs")
    total, nflag, nmiss = _check_ci8_codes(d["x"], d["spec"], d["scale"], (0, d["nspec"] - 1),
                                           list(range(d["ninput"])))
    print(f"{total} codes, {nflag} inside the tie window, {nmiss} differ by one")
    assert d["spec"].min() >= -127


def test_fx_xengine_on_gpu_ci8_bit_exact(fx_full):
    """Stage (iii): the X-engine on the GPU's own ci8 spectra equals the integer
    oracle on those same bytes -- element by element on sampled channels
    (including the tone channel), and through the exact Freivalds identity on
    all 2048 channels."""
    d = fx_full
    spec, vis, N, S = d["spec"], d["vis"], d["ninput"], d["nspec"]
    banner("F+X stage iii: X-engine on the GPU's ci8 vs the oracle")
    raw = np.ascontiguousarray(spec)  # [S][F][N][2] int8 = the X-engine's [t][f][i] ci8
    for f in (0, 1, 776, 777, 1024, 2047):
        want = oracle.xengine_int(raw, "ci8", S, NCHAN, N, chans=(f, 1))
        assert np.array_equal(vis[f], want[0]), f
    re, im = spec[..., 0], spec[..., 1]
    assert freivalds_check(vis, re, im, seed=11)


def test_fx_chain_tone_closed_form(fx_full):
    """Stage (iv): a unit tone at channel 777 with per-input delays.

    After scaling the tone has amplitude 2048 * s per component pair; the
    visibility at 777 is E[V_ij] = T (2048 s)^2 exp(-2 pi i 777 (tau_i - tau_j) / 4096).
    """
    d = fx_full
    ninput, nspec, k0, tau = d["ninput"], d["nspec"], 777, d["tau"]
    banner("F+X stage iv: tone closed form")
    V = d["vis"][k0].astype(np.float64)
    a = 2048.0 * float(d["scale"][0])
    expect_mag = nspec * a * a
    # noise std of a cross visibility: sqrt(T (sigma_q^4 + 2 sigma_q^2 a^2)), sigma_q^2 = 64*2
    sq2 = 2 * 64.0
    sd = np.sqrt(nspec * (sq2 * sq2 / 2 + 2 * (sq2 / 2) * a * a))
    slope = -2 * np.pi * k0 / NFFT
    ii, jj = np.tril_indices(ninput, -1)
    z = V[ii * (ii + 1) // 2 + jj, 0] + 1j * V[ii * (ii + 1) // 2 + jj, 1]
    rot = np.exp(1j * slope * (tau[ii] - tau[jj]))
    res = np.abs(z - expect_mag * rot) / sd
    phs = np.angle(z / rot)
    print(f"{res.size} pairs, max |V - E[V]| / sd = {res.max():.2f}, median {np.median(res):.2f}")
    assert res.max() < 6.5
    assert abs(np.median(phs)) < 0.01  # phase residual after removing the slope
    # fitted phase slope over all cross pairs: the model slope plus the
    # least-squares slope of the residual phase against the delay difference
    # (no wrapping while the model is within pi / 50 rad per sample)
    dt = tau[ii] - tau[jj]
    resid = np.angle(z / rot)
    est = slope + np.sum(resid * dt) / np.sum(dt * dt)
    print(f"fitted phase slope {est:.5f} rad/sample (model {slope:.5f})")
    assert abs(est / slope - 1) < 0.01


def test_most_inputs_sampled():
    """65536 inputs (the largest accepted) and 17 frames: the input passes 2^32
    bytes (frame 16 starts at 4.3 GB) and a frame spans 2^28 bytes, so the
    kernel's 32-bit lane, row and channel offsets reach their largest values.
    Uniform codes over the whole int8 range (-128 included).  Binary32
    spectra of 12 sampled inputs (both ends of the range, group edges) in
    frames 0 and 16 against the double DFT, then their ci8 codes against the
    oracle's requantizer (near-ties flagged a priori)."""
    import torch
    import paper_1708_00720_amd as bfx
    ninput, nspec = 65536, 17
    frames = (0, 16)
    inputs = [0, 1, 7, 8, 4095, 4096, 32767, 32768, 65527, 65528, 65534, 65535]
    banner(f"fengine cf32 + ci8 ninput={ninput} nspec={nspec}")
    gen = torch.Generator(device="cuda").manual_seed(43)
    d_in = torch.randint(-128, 128, (nspec * NFFT * ninput,), dtype=torch.int8, device="cuda", generator=gen)
    rows = d_in.view(nspec * NFFT, ninput)
    idx = torch.tensor(inputs, device="cuda")
    # the sampled columns of the sampled frames, as a compact 2-frame array
    xc = np.concatenate([rows[s * NFFT:(s + 1) * NFFT].index_select(1, idx).cpu().numpy() for s in frames])
    fidx = torch.tensor(frames, device="cuda")

    out = torch.zeros(nspec * NCHAN * ninput * 2, dtype=torch.float32, device="cuda")
    bfx.bfx_fengine(d_in, ninput, NFFT, nspec, torch.ones(NCHAN, device="cuda"), out, out="cf32")
    torch.cuda.synchronize()
    got = out.view(nspec, NCHAN, ninput, 2).index_select(0, fidx).index_select(2, idx).cpu().numpy()
    del out
    want = _oracle_spectrum(xc, len(inputs), range(len(frames)), list(range(len(inputs))))
    worst = 0.0
    for (s, i), w in want.items():
        g = got[s, :, i, 0].astype(np.float64) + 1j * got[s, :, i, 1]
        worst = max(worst, _normwise(g, w))
    print(f"worst normwise relative error {worst:.3e}")
    assert worst <= 1e-6

    scale = synth.fengine_scale(NCHAN)
    out = torch.zeros(nspec * NCHAN * ninput * 2, dtype=torch.int8, device="cuda")
    bfx.bfx_fengine(d_in, ninput, NFFT, nspec, torch.from_numpy(np.asarray(scale, np.float32)).cuda(), out,
                    out="ci8")
    torch.cuda.synchronize()
    gotq = out.view(nspec, NCHAN, ninput, 2).index_select(0, fidx).index_select(2, idx).cpu().numpy()
    del out, d_in
    total, nflag, nmiss = _check_ci8_codes(xc, gotq, scale, range(len(frames)), list(range(len(inputs))))
    print(f"{total} codes, {nflag} inside the tie window, {nmiss} differ by one")
    assert gotq.min() >= -127
