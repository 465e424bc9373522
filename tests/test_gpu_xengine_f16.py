"""GPU parity of the binary16 X-engine (FP16 MFMA, FP32 accumulation) and of the
FP64 running sum of its dumps, against the FP64 oracle on the same cf16 values.

Error metric per product: |V_gpu - V_64| / sqrt(V_ii V_jj) (complex modulus;
the Cauchy-Schwarz normalisation).  binary16 products are exact in binary32,
so the only error is the binary32 summation: a sum of T products plus the
final Re/Im combination is within gamma_{T+1} = (T+1)u/(1-(T+1)u) of
sum |x_i||x_j| <= sqrt(V_ii V_jj), u = 2^-24.  The tests assert that bound
and print the observed max and rms.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner, to_dev

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _bound(T):
    n = T + 1
    return n * U32 / (1 - n * U32)


def _tri_ij(N):
    i = np.repeat(np.arange(N), np.arange(1, N + 1))
    j = np.concatenate([np.arange(k + 1) for k in range(N)])
    return i, j


def _normalised_error(got, want, N):
    """got, want: [F][P][2]; returns the per-product error array [F][P]."""
    i, j = _tri_ij(N)
    diag = want[:, i * (i + 1) // 2 + i, 0], want[:, j * (j + 1) // 2 + j, 0]
    norm = np.sqrt(diag[0] * diag[1])
    d = np.hypot(got[..., 0] - want[..., 0], got[..., 1] - want[..., 1])
    return d / norm


def _oracle(x16, chans=None):
    x = x16 if chans is None else x16[:, chans]
    return oracle.xengine_f64(x[..., 0].astype(np.float64), x[..., 1].astype(np.float64))


def _run(x16, T, F, N, overwrite=True, acc=None, plan=None):
    import torch
    import paper_1708_00720_amd as bfx
    own = plan is None
    if own:
        plan = bfx.bfx_xengine_create(N, F, "cf16")
    if acc is None:
        acc = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, to_dev(x16), T, acc, overwrite=overwrite)
    torch.cuda.synchronize()
    if own:
        plan.close()
    return acc


def _host(acc, F, N):
    return acc.cpu().numpy().astype(np.float64).reshape(F, N * (N + 1) // 2, 2)


def _check(got, want, N, T, label):
    err = _normalised_error(got, want, N)
    print(f"{label}: max {err.max():.3e} rms {np.sqrt(np.mean(err ** 2)):.3e} "
          f"bound {_bound(T):.3e}")
    assert np.all(np.isfinite(got))
    assert err.max() <= _bound(T), err.max()
    return err


def test_fp16_small_config():
    T, F, N = 512, 64, 32
    banner(f"xengine cf16 T={T} F={F} N={N}")
    x = synth.cf16_voltages(5, T, F, N)
    _check(_host(_run(x, T, F, N), F, N), _oracle(x), N, T, "cf16 32x64x512")


@pytest.mark.parametrize("T,F,N", [
    (1, 1, 4), (17, 3, 36), (16, 2, 64), (100, 2, 100), (33, 2, 196), (40, 1, 260), (70, 1, 452),
])
def test_fp16_ragged_shapes(T, F, N):
    banner(f"xengine cf16 ragged T={T} F={F} N={N}")
    x = synth.cf16_voltages(500 + T + N, T, F, N)
    _check(_host(_run(x, T, F, N), F, N), _oracle(x), N, T, f"cf16 ragged {T}x{F}x{N}")


def test_fp16_exact_on_small_integers():
    """Small-integer voltages make every partial sum an exact binary32 integer,
    so the FP path must reproduce the integer oracle exactly."""
    T, F, N = 96, 3, 68
    banner(f"xengine cf16 integer-valued T={T} F={F} N={N}")
    raw = synth.voltages(77, T, F, N, "ci8", 8.0, 127)
    x = raw.astype(np.float16)  # [T][F][N][2], exact
    got = _host(_run(x, T, F, N), F, N)
    want = oracle.xengine_int(raw, "ci8", T, F, N).astype(np.float64)
    assert np.array_equal(got, want)


def test_fp16_accumulate_across_gulps():
    import paper_1708_00720_amd as bfx
    T1, T2, F, N = 48, 80, 4, 100
    banner(f"xengine cf16 RMW T={T1}+{T2} F={F} N={N}")
    x1 = synth.cf16_voltages(61, T1, F, N)
    x2 = synth.cf16_voltages(62, T2, F, N)
    plan = bfx.bfx_xengine_create(N, F, "cf16")
    acc = bfx.visibilities_buffer(plan)
    _run(x1, T1, F, N, overwrite=True, acc=acc, plan=plan)
    _run(x2, T2, F, N, overwrite=False, acc=acc, plan=plan)
    assert bfx.bfx_xengine_nacc(plan) == T1 + T2
    plan.close()
    want = _oracle(np.concatenate([x1, x2]))
    _check(_host(acc, F, N), want, N, T1 + T2 + 1, "cf16 RMW")


def test_fp64_running_sum_of_dumps():
    """run64 += dump over three gulps: equal to the FP64 oracle of the whole
    integration within the binary32 bound of each dump, and the running sum of
    k identical dumps is exactly k * dump in FP64."""
    import torch
    import paper_1708_00720_amd as bfx
    T, F, N, K = 64, 5, 36, 3
    banner(f"xengine cf16 dump running sum T={T} F={F} N={N} K={K}")
    plan = bfx.bfx_xengine_create(N, F, "cf16")
    acc = bfx.visibilities_buffer(plan)
    out = torch.zeros_like(acc)
    P = N * (N + 1) // 2
    run64 = torch.zeros(F * P * 2, dtype=torch.float64, device="cuda")
    xs = [synth.cf16_voltages(70 + k, T, F, N) for k in range(K)]
    for x in xs:
        bfx.bfx_xengine_accumulate(plan, to_dev(x), T, acc, overwrite=True)
        bfx.bfx_xengine_dump(plan, acc, out, run64)
    torch.cuda.synchronize()
    assert torch.equal(out, acc)  # the copy is exact
    want = _oracle(np.concatenate(xs))
    got = run64.cpu().numpy().reshape(F, P, 2)
    _check(got, want, N, T + 1, "running sum of 3 dumps")

    # identical dumps: the last dump handed over k more times
    run_k = torch.zeros_like(run64)
    for _ in range(5):
        bfx.bfx_xengine_dump(plan, acc, None, run_k)
    torch.cuda.synchronize()
    assert torch.equal(run_k, 5.0 * acc.double())
    plan.close()


def test_fp16_full_size_sampled_channels(cf16_full):
    """512 inputs, 2048 channels, 1024 samples (4.3 GB of cf16): sampled
    channels against the FP64 oracle; every channel's autocorrelations are
    real and positive and match T * mean |x|^2 statistically."""
    T, F, N = 1024, 2048, 512
    banner(f"xengine cf16 full size T={T} F={F} N={N}")
    x = cf16_full
    acc = _run(x, T, F, N)
    chans = [0, 7, 8, 1023, 2047]
    P = N * (N + 1) // 2
    vis = acc.view(F, P, 2)
    got = vis[chans].cpu().numpy().astype(np.float64)
    want = _oracle(x, chans)
    _check(got, want, N, T, "cf16 full size, 5 channels")
    i = np.arange(N)
    auto = vis[:, i * (i + 1) // 2 + i].cpu().numpy()
    assert np.all(auto[..., 0] > 0)
    # Im V_ii = C[im][re] - C[re][im]: two binary32 sums of the same exact
    # products, so at most the summation bound
    assert np.all(np.abs(auto[..., 1]) <= _bound(T) * auto[..., 0])
    print(f"Im V_ii exactly zero in {np.mean(auto[..., 1] == 0):.4f} of autocorrelations")
    # E[V_ii] = T * 2 sigma^2 (sigma = 1), sd = sqrt(T * 2 * 2) per entry
    z = (auto[..., 0] - 2.0 * T) / np.sqrt(4.0 * T)
    assert abs(z.mean()) < 0.05 and 0.8 < z.std() < 1.2


@pytest.mark.parametrize("T", [48, 128, 160])
def test_fp16_items_span_several_rounds(T):
    """512 work items (512 channels of 96 inputs) on one workgroup per CU:
    consecutive items per workgroup, item lengths below, equal to and above
    the LDS ring depth."""
    F, N = 512, 96
    banner(f"xengine cf16 multi-round T={T} F={F} N={N}")
    x = synth.cf16_voltages(80 + T, T, F, N)
    _check(_host(_run(x, T, F, N), F, N), _oracle(x), N, T, f"cf16 multi-round T={T}")


def test_dump_full_size_running_sum():
    """The dump at the FP16 workload's size (2048 channels x 131,328
    baselines, 537 M binary32 values, one thread per four values): the copy is
    exact and two dumps add exactly 2 * value in binary64 everywhere."""
    import torch
    import paper_1708_00720_amd as bfx
    F, N = 2048, 512
    banner(f"dump full size F={F} N={N}")
    plan = bfx.bfx_xengine_create(N, F, "cf16")
    acc = bfx.visibilities_buffer(plan)
    g = torch.Generator(device="cuda").manual_seed(11)
    acc.copy_(torch.randn(acc.numel(), device="cuda", generator=g).view(acc.shape))
    out = torch.zeros_like(acc)
    run64 = torch.zeros(acc.numel(), dtype=torch.float64, device="cuda")
    bfx.bfx_xengine_dump(plan, acc, out, run64)
    bfx.bfx_xengine_dump(plan, acc, None, run64)
    torch.cuda.synchronize()
    assert torch.equal(out, acc)
    assert torch.equal(run64, 2.0 * acc.reshape(-1).double())
    plan.close()


@pytest.mark.parametrize("T,F,N", [(64, 5, 36), (96, 3, 100), (128, 2, 200), (40, 9, 64)])
def test_fused_running_sum_equals_accumulate_then_dump(T, F, N):
    """bfx_xengine_accumulate_run64 over three gulps gives the same bits as
    accumulate (overwrite) followed by dump into a running sum, for both
    kernel variants, on packed one-block arrays and ragged multi-block ones."""
    import torch
    import paper_1708_00720_amd as bfx
    banner(f"xengine cf16 fused running sum T={T} F={F} N={N}")
    plan = bfx.bfx_xengine_create(N, F, "cf16")
    P = N * (N + 1) // 2
    xs = [to_dev(synth.cf16_voltages(90 + k + N, T, F, N)) for k in range(3)]
    for v in range(bfx.bfx_xengine_num_variants(plan)):
        bfx.bfx_xengine_set_variant(plan, v)
        acc = bfx.visibilities_buffer(plan)
        two_step = torch.zeros(F * P * 2, dtype=torch.float64, device="cuda")
        fused = torch.full((F * P * 2,), 0.0, dtype=torch.float64, device="cuda")
        for x in xs:
            bfx.bfx_xengine_accumulate(plan, x, T, acc, overwrite=True)
            bfx.bfx_xengine_dump(plan, acc, None, two_step)
            bfx.bfx_xengine_accumulate_run64(plan, x, T, fused)
        torch.cuda.synchronize()
        assert torch.equal(fused, two_step), f"variant {v}"
        assert bool(torch.isfinite(fused).all())
    plan.close()
