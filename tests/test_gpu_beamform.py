"""GPU parity of the phase-and-sum beamformer with square-law detection and
integration (binary16 products, binary32 accumulation) against the FP64 oracle
on the same binary16 voltages and weights.

Error bound per output P[b][f][u] = sum_{t in u} |y_t|^2.  With
S_t = sum_i |w_i||x_i| (so |y_t| <= S_t), the binary32 beam sum has
|dy_t| <= gamma_{2N} S_t (products exact), hence
|dP| <= (2 gamma_{2N} + gamma_navg + O(u^2)) sum_{t in u} S_t^2.
The tests assert 1.5x that bound (covering one extra rounding per MFMA) and
print the observed normalised and relative errors.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner, to_dev

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _gamma(n):
    return n * U32 / (1 - n * U32)


def _run(x16, w16, N, F, B, T, navg):
    import torch
    import paper_1708_00720_amd as bfx
    out = torch.full((B * F * (T // navg),), float("nan"), dtype=torch.float32, device="cuda")
    bfx.bfx_beamform_detect(to_dev(x16), to_dev(w16), N, F, B, T, navg, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64).reshape(B, F, T // navg)


def _expect(x16, w16, navg):
    x = x16.astype(np.float64)
    w = w16.astype(np.float64)
    P = oracle.beamform_detect(x[..., 0], x[..., 1], w[..., 0], w[..., 1], navg)
    # S[b][f][t] = sum_i |w_fbi| |x_tfi|
    ax = np.hypot(x[..., 0], x[..., 1])  # [T][F][N]
    aw = np.hypot(w[..., 0], w[..., 1])  # [F][B][N]
    S = np.einsum("fbi,tfi->bft", aw, ax)
    T = x.shape[0]
    S2 = (S ** 2).reshape(S.shape[0], S.shape[1], T // navg, navg).sum(axis=3)
    return P, S2


def _check(got, x16, w16, navg, label):
    N = x16.shape[2]
    want, S2 = _expect(x16, w16, navg)
    assert np.all(np.isfinite(got)), "an output was not written"
    err = np.abs(got - want)
    norm = err / S2
    rel = err / want
    bound = 1.5 * (2 * _gamma(2 * N) + _gamma(navg))
    print(f"{label}: max |dP|/sum S^2 {norm.max():.3e} (bound {bound:.3e}); "
          f"relative error max {rel.max():.3e} median {np.median(rel):.3e}")
    assert norm.max() <= bound


def test_beamform_basic():
    N, F, B, T, navg = 64, 8, 8, 64, 16
    banner(f"beamform N={N} F={F} B={B} T={T} navg={navg}")
    x = synth.cf16_voltages(11, T, F, N)
    w = synth.steering_weights(12, F, B, N)
    _check(_run(x, w, N, F, B, T, navg), x, w, navg, "basic")


@pytest.mark.parametrize("navg", [1, 2, 4, 8, 32])
def test_beamform_navg(navg):
    N, F, B, T = 96, 3, 5, 96
    banner(f"beamform navg={navg} N={N} F={F} B={B} T={T}")
    x = synth.cf16_voltages(20 + navg, T, F, N)
    w = synth.steering_weights(40 + navg, F, B, N)
    _check(_run(x, w, N, F, B, T, navg), x, w, navg, f"navg={navg}")


@pytest.mark.parametrize("N,F,B,T,navg", [
    (32, 1, 1, 16, 16),      # smallest unit: one beam, one window
    (96, 3, 8, 64, 4),       # one partial K chunk of 24 16-byte chunks per row (not 16k)
    (544, 2, 40, 48, 16),    # three K chunks (256 + 256 + 32 inputs), two beam groups, ragged time
    (1056, 1, 70, 272, 8),   # five K chunks, three beam groups, a 256-sample unit + a 16-sample tail
    (512, 9, 32, 512, 16),   # channel count not a multiple of 8
    (256, 2, 16, 600, 8),    # two full 256-sample units + an 88-sample tail
    (128, 3, 7, 336, 16),    # a full unit + 5 windows of the next; an odd beam count
])
def test_beamform_ragged(N, F, B, T, navg):
    banner(f"beamform ragged N={N} F={F} B={B} T={T} navg={navg}")
    x = synth.cf16_voltages(300 + N + B, T, F, N)
    w = synth.steering_weights(400 + N + B, F, B, N)
    _check(_run(x, w, N, F, B, T, navg), x, w, navg, f"ragged {N}x{F}x{B}x{T}")


def test_beamform_unit_weights_match_xengine():
    """Closed-form cross-check between the two GPU products: with w = 1 on all
    inputs, sum over a window of |sum_i x_i|^2 = 1^T V 1 summed over the same
    samples, where V is the X-engine's visibility matrix (computed here by the
    oracle in FP64 and compared within the binary32 bound)."""
    N, F, B, T, navg = 64, 4, 1, 32, 32
    banner("beamform unit weights vs 1^T V 1")
    x = synth.cf16_voltages(90, T, F, N)
    w = np.zeros((F, B, N, 2), np.float16)
    w[..., 0] = 1.0
    got = _run(x, w, N, F, B, T, navg)[0, :, 0]  # [F]
    V = oracle.xengine_f64(x[..., 0].astype(np.float64), x[..., 1].astype(np.float64), full=True)
    ones = np.sum(V[..., 0], axis=(1, 2))  # 1^T V 1 is real: sum of Re V_ij over i, j
    S2 = (np.abs(x.astype(np.float64)[..., 0] + 1j * x.astype(np.float64)[..., 1]).sum(axis=2) ** 2).sum(axis=0)
    assert np.all(np.abs(got - ones) <= 1.5 * (2 * _gamma(2 * N) + _gamma(navg)) * S2)


def test_beamform_full_size_sampled(cf16_full):
    """512 inputs, 2048 channels, 32 beams, 1024 samples, 16-sample integration;
    sampled channels against the oracle, every output finite and positive."""
    N, F, B, T, navg = 512, 2048, 32, 1024, 16
    banner(f"beamform full size N={N} F={F} B={B} T={T} navg={navg}")
    x = cf16_full
    w = synth.steering_weights(5, F, B, N)
    got = _run(x, w, N, F, B, T, navg)
    assert np.all(np.isfinite(got)) and np.all(got > 0)
    chans = [0, 7, 8, 1023, 2047]
    _check(got[:, chans], np.ascontiguousarray(x[:, chans]), np.ascontiguousarray(w[chans]), navg,
           "full size, 5 channels")


def test_beamform_max_inputs_and_beams():
    """ninput = 8192 (32 K chunks) and nbeam = 256 (8 beam groups), the API
    maxima, with navg = 32."""
    N, F, B, T, navg = 8192, 2, 256, 64, 32
    banner(f"beamform max N={N} F={F} B={B} T={T} navg={navg}")
    x = synth.cf16_voltages(81, T, F, N)
    w = synth.steering_weights(82, F, B, N)
    _check(_run(x, w, N, F, B, T, navg), x, w, navg, "max sizes")
