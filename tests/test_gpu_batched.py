"""GPU parity of the batched X-engine: several subarrays of uneven input and
channel counts correlated by one persistent launch, bit-exact against the
oracle per subarray and against one plain plan per subarray; captured in a
HIP graph and replayed with fresh data between replays."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import banner

pytestmark = pytest.mark.gpu


def _arena(plan, gulps, T, dtype):
    """Host gulps (one per subarray) -> device input arena of the plan."""
    import torch
    import paper_1708_00720_amd as bfx
    arena = torch.zeros(bfx.bfx_xengine_in_bytes(plan, T), dtype=torch.uint8)
    for k, g in enumerate(gulps):
        io, _ = bfx.bfx_xengine_sub_offsets(plan, k, T)
        b = np.ascontiguousarray(g).view(np.uint8).reshape(-1)
        arena[io:io + b.size] = torch.from_numpy(b)
    return arena.cuda()


def _sub_vis(plan, acc, k, N, F):
    import paper_1708_00720_amd as bfx
    _, oo = bfx.bfx_xengine_sub_offsets(plan, k, 0)
    P = N * (N + 1) // 2
    n = F * P * 2
    return acc[oo // 4:oo // 4 + n].cpu().numpy().astype(np.int64).reshape(F, P, 2)


def _check_all(plan, acc, gulps, T, dtype, Ns, Fs, t0=0, nt=None):
    for k, (N, F) in enumerate(zip(Ns, Fs)):
        got = _sub_vis(plan, acc, k, N, F)
        want = oracle.xengine_int(gulps[k], dtype, T, F, N, t0=t0, nt=nt)
        assert np.array_equal(got, want), f"subarray {k} (N={N}, F={F}) differs"


def test_batched_mixed_sizes_bit_exact():
    """8 subarrays, inputs {32..512}, channels {1024..64}, ci8 sigma=8, 256
    samples: one launch, every subarray bit-exact vs the oracle."""
    import torch
    import paper_1708_00720_amd as bfx
    T = 256
    Ns, Fs = synth.BATCH_NINPUT, synth.BATCH_NCHAN
    banner(f"batched ci8 8 subarrays T={T}")
    gulps = synth.batched_voltages(T)
    plan = bfx.bfx_xengine_create_batched(Ns, Fs, "ci8")
    arena = _arena(plan, gulps, T, "ci8")
    acc = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, arena, T, acc, overwrite=True)
    torch.cuda.synchronize()
    _check_all(plan, acc, gulps, T, "ci8", Ns, Fs)
    plan.close()


@pytest.mark.parametrize("dtype", ["ci4", "ci8"])
def test_batched_equals_plain_plans_ragged(dtype):
    """Ragged sizes (inputs not multiples of 64, odd channel counts, time not a
    multiple of the stage): batched result == one plain plan per subarray."""
    import torch
    import paper_1708_00720_amd as bfx
    from gpu_util import to_dev
    T = 77
    Ns, Fs = (4, 36, 100, 260, 68), (3, 2, 5, 1, 9)
    banner(f"batched {dtype} ragged T={T}")
    gulps = [synth.extreme_voltages(900 + k, T, F, N, dtype) for k, (N, F) in enumerate(zip(Ns, Fs))]
    plan = bfx.bfx_xengine_create_batched(Ns, Fs, dtype)
    arena = _arena(plan, gulps, T, dtype)
    acc = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, arena, T, acc, overwrite=True)
    torch.cuda.synchronize()
    _check_all(plan, acc, gulps, T, dtype, Ns, Fs)
    for k, (N, F) in enumerate(zip(Ns, Fs)):
        p1 = bfx.bfx_xengine_create(N, F, dtype)
        a1 = bfx.visibilities_buffer(p1)
        bfx.bfx_xengine_accumulate(p1, to_dev(gulps[k]), T, a1, overwrite=True)
        torch.cuda.synchronize()
        assert np.array_equal(a1.cpu().numpy().astype(np.int64).reshape(F, -1, 2),
                              _sub_vis(plan, acc, k, N, F))
        p1.close()
    plan.close()


def test_batched_accumulate_and_long_ci4_split():
    """RMW across two gulps, and a ci4 gulp longer than one launch's sample
    bound (the host cuts it into launches with a time offset into every
    subarray of the arena)."""
    import torch
    import paper_1708_00720_amd as bfx
    Ns, Fs = (8, 40), (2, 3)
    banner("batched RMW + ci4 70000-sample split")
    T1 = 50
    g1 = [synth.voltages(950 + k, T1, F, N, "ci8", 8.0, 127) for k, (N, F) in enumerate(zip(Ns, Fs))]
    g2 = [synth.voltages(960 + k, T1, F, N, "ci8", 8.0, 127) for k, (N, F) in enumerate(zip(Ns, Fs))]
    plan = bfx.bfx_xengine_create_batched(Ns, Fs, "ci8")
    acc = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, _arena(plan, g1, T1, "ci8"), T1, acc, overwrite=True)
    bfx.bfx_xengine_accumulate(plan, _arena(plan, g2, T1, "ci8"), T1, acc, overwrite=False)
    torch.cuda.synchronize()
    for k, (N, F) in enumerate(zip(Ns, Fs)):
        want = (oracle.xengine_int(g1[k], "ci8", T1, F, N) + oracle.xengine_int(g2[k], "ci8", T1, F, N))
        assert np.array_equal(_sub_vis(plan, acc, k, N, F), want)
    plan.close()

    T = 70000
    g = [synth.voltages(970 + k, T, F, N, "ci4", 2.5, 7) for k, (N, F) in enumerate(zip(Ns, Fs))]
    plan = bfx.bfx_xengine_create_batched(Ns, Fs, "ci4")
    acc = bfx.visibilities_buffer(plan)
    bfx.bfx_xengine_accumulate(plan, _arena(plan, g, T, "ci4"), T, acc, overwrite=True)
    torch.cuda.synchronize()
    _check_all(plan, acc, g, T, "ci4", Ns, Fs)
    plan.close()


def test_batched_hip_graph_replays():
    """One captured gulp step (accumulate with overwrite, then dump to a
    separate buffer) replayed 4 times; between replays the arena is refilled
    eagerly with a new gulp and every replay is checked bit-exactly."""
    import torch
    import paper_1708_00720_amd as bfx
    T = 256
    Ns, Fs = synth.BATCH_NINPUT[:5], synth.BATCH_NCHAN[:5]
    banner("batched hipGraph replays")
    plan = bfx.bfx_xengine_create_batched(Ns, Fs, "ci8")
    gulps0 = synth.batched_voltages(T, Ns, Fs, seed0=500)
    arena = _arena(plan, gulps0, T, "ci8")
    acc = bfx.visibilities_buffer(plan)
    out = torch.zeros_like(acc)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside capture (kernel attributes, lazy init)
        bfx.bfx_xengine_accumulate(plan, arena, T, acc, overwrite=True)
        bfx.bfx_xengine_dump(plan, acc, out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bfx.bfx_xengine_accumulate(plan, arena, T, acc, overwrite=True)
        bfx.bfx_xengine_dump(plan, acc, out)
    for rep in range(4):
        gulps = synth.batched_voltages(T, Ns, Fs, seed0=600 + 10 * rep)
        arena.copy_(_arena(plan, gulps, T, "ci8"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _check_all(plan, out, gulps, T, "ci8", Ns, Fs)
    plan.close()
