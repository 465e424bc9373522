#!/usr/bin/env python3
"""Throughput of the FX-correlator X-engine on one MI355X.

Workload (the streaming configuration the headline metric is quoted on):
352 antennas x 2 polarisations = 704 inputs, 192 channels, ci4 voltages
(rounded Gaussian sigma=2.5 clipped to +-7), 1000 samples per integration.
A step streams 100 gulps through a 4-slot device ring of input gulps (the
paper's default ring = 4 gulps): gulp g is one integration, correlated with
BFX_ACC_OVERWRITE into slot g % 4 of a 4-slot ring of visibility buffers and
handed over there by dump (no copy: the consumer reads the slot).  All
inputs are resident in HBM before timing starts.

Prints one JSON line.  Extra fields: input GB/s, the dominant kernel's
roofline (HIP-event-timed launches on the launch stream), graph-replay
timing of one ring cycle (median, p10, p90), the CPU oracle's rate on a
bounded sample, and the parity of the benchmarked ring's visibilities with
the oracle on the channels the CPU sample computed.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "X-engine TeraCMAC/s + input GB/s at 704 inputs; int8 exact vs FP16/FP32 path"
N_INPUT, N_CHAN, N_TIME, N_GULP, N_SLOT = 704, 192, 1000, 100, 4
PEAK_INT8_TOPS = 5000.0  # MI355X dense int8 MFMA, 5.0 POP/s
KERNEL_SRCS = [os.path.join(ROOT, "paper_1708_00720_amd", "csrc", f)
               for f in ("xengine_int.hip", "xe_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "xengine_int_ci4_704_traffic.json")


def cmac_per_gulp():
    return N_CHAN * N_TIME * N_INPUT * (N_INPUT + 1) // 2


def kernel_hash():
    """Hash of the sources the integer X-engine kernel is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(per_launch_cmac):
    """HBM bytes per launch from committed counter runs, if taken on this kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    if rec.get("kernel_sha256_16") != kernel_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(raw_gulp, budget_s=15.0):
    """Oracle X-engine on whole channels of one gulp until ~budget_s elapses
    (all OpenMP threads), plus one channel on a single thread.  Returns the
    record and the oracle's visibilities of the channels it computed."""
    import numpy as np
    import oracle
    threads = oracle.max_threads()
    done_ch = 0
    t0 = time.perf_counter()
    f = 0
    parts = []
    while time.perf_counter() - t0 < budget_s and done_ch < N_CHAN:
        nf = min(threads, N_CHAN - f)
        parts.append(oracle.xengine_int(raw_gulp, "ci4", N_TIME, N_CHAN, N_INPUT, chans=(f, nf),
                                        nthreads=threads))
        f += nf
        done_ch += nf
    dt = time.perf_counter() - t0
    cmac_ch = N_TIME * N_INPUT * (N_INPUT + 1) // 2
    t1 = time.perf_counter()
    oracle.xengine_int(raw_gulp, "ci4", N_TIME, N_CHAN, N_INPUT, chans=(N_CHAN - 1, 1), nthreads=1)
    dt1 = time.perf_counter() - t1
    rec = {"value": done_ch * cmac_ch / dt / 1e12, "unit": "TeraCMAC/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{done_ch} of {N_CHAN} channels of one 704-input ci4 gulp "
                     f"({N_TIME} samples), int64 triple loop, {dt:.1f} s",
           "single_thread_value": cmac_ch / dt1 / 1e12,
           "single_thread_sample": f"channel {N_CHAN - 1} of the same gulp on one thread, {dt1:.1f} s",
           "cpu_model": cpu_model()}
    return rec, np.concatenate(parts, axis=0)


PEAK_FP16_TFLOPS = 2500.0  # MI355X dense FP16 MFMA
PEAK_FP32_TFLOPS = 157.3   # FP32 vector, counting packed (two-per-lane) FMA
# FP32 vector without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# (FMA) x 2.4 GHz.  The kernels are built with packed FP32 disabled.
PEAK_FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_HBM_GBPS = 8000.0


def time_launches(fn, reps, warm=2):
    """Average / median / min duration (ms) of fn() over reps calls, each
    bracketed by HIP events on torch's current stream (the launch stream)."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warm):
        fn()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    d = sorted(a.elapsed_time(b) for a, b in evs)
    return sum(d) / len(d), d[len(d) // 2], d[0]


def measured_peaks():
    """Sustainable rates of this device from the library's peak probes: dense
    MFMA (int8 and binary16, back-to-back MFMAs on 8 independent accumulators
    per wave, no memory traffic), LDS reads per CU (transposing 8-byte reads
    and plain 16-byte reads) and HBM reads (a 2 GiB buffer streamed once with
    16-byte loads).  Best of 5 event-timed launches each."""
    import torch
    import paper_1708_00720_amd as bfx
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
    out = {}
    for name, kind in (("int8_mfma_TOPs", bfx.BFX_PROBE_MFMA_I8), ("fp16_mfma_TFLOPs", bfx.BFX_PROBE_MFMA_F16)):
        iters, nb = 2000, 4 * ncu
        _, _, best = time_launches(lambda: bfx.bfx_probe_mfma(kind, iters, nb, sink), 5)
        out[name] = round(bfx.bfx_probe_mfma_ops(kind, iters, nb) / (best * 1e-3) / 1e12, 1)
    # LDS read bandwidth per CU (bytes per ns; bytes per clock at the 2.4 GHz
    # peak clock): transposing 8-byte reads, as the X-engines' fragment
    # reads, and plain 16-byte reads
    for name, kind in (("lds_tr16", bfx.BFX_PROBE_LDS_TR16), ("lds_tr8", bfx.BFX_PROBE_LDS_TR8),
                       ("lds_b128", bfx.BFX_PROBE_LDS_B128)):
        iters, nb = 20000, ncu
        _, _, best = time_launches(lambda: bfx.bfx_probe_lds(kind, iters, nb, sink), 5)
        per_cu_ns = bfx.bfx_probe_lds_bytes(kind, iters, nb) / ncu / (best * 1e6)
        out[f"{name}_bytes_per_ns_per_cu"] = round(per_cu_ns, 1)
        out[f"{name}_bytes_per_clk_per_cu_at_2p4GHz"] = round(per_cu_ns / 2.4, 1)
    buf = torch.ones(1 << 29, dtype=torch.int32, device="cuda")  # 2 GiB
    nbytes = buf.numel() * 4
    _, _, best = time_launches(lambda: bfx.bfx_probe_read(buf, nbytes, 32 * ncu, sink), 5)
    out["hbm_read_GBps"] = round(nbytes / (best * 1e-3) / 1e9, 1)
    out["int8_frac_of_published"] = round(out["int8_mfma_TOPs"] / PEAK_INT8_TOPS, 3)
    out["fp16_frac_of_published"] = round(out["fp16_mfma_TFLOPs"] / PEAK_FP16_TFLOPS, 3)
    out["hbm_frac_of_published"] = round(out["hbm_read_GBps"] / PEAK_HBM_GBPS, 3)
    out["compute_units"] = ncu
    del buf
    return out


def graph_replay_timing(gulp, replays, warm=5):
    """One ring cycle (4 gulps: accumulate with overwrite + dump each)
    captured in a HIP graph, replayed `replays` times after `warm` warm-up
    replays, each replay bracketed by HIP events on the replay stream.
    Returns per-gulp median, p10 and p90 (microseconds)."""
    import numpy as np
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for k in range(N_SLOT):
            gulp(k, s.cuda_stream)
    torch.cuda.synchronize()
    for _ in range(warm):
        g.replay()
    torch.cuda.synchronize()
    cur = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(replays)]
    for a, b in evs:
        a.record(cur)
        g.replay()
        b.record(cur)
    torch.cuda.synchronize()
    per_gulp = np.array([a.elapsed_time(b) for a, b in evs]) * 1e3 / N_SLOT
    med = float(np.median(per_gulp))
    return {"replays": replays, "gulps_per_replay": N_SLOT,
            "us_per_gulp_median": round(med, 2),
            "us_per_gulp_p10": round(float(np.percentile(per_gulp, 10)), 2),
            "us_per_gulp_p90": round(float(np.percentile(per_gulp, 90)), 2),
            "tcmac_per_s_median": round(cmac_per_gulp() / (med * 1e-6) / 1e12, 2)}


def _row(kernel, workload, avg_ms, med_ms, work, work_unit, peak, peak_unit, bound, nbytes,
         extra=None):
    """One measured row: `work` per launch in units of `work_unit` (ops or
    bytes), achieved rate against `peak` of the bound resource."""
    if bound == "hbm":
        achieved = nbytes / (avg_ms * 1e-3) / 1e9
    else:
        achieved = work / (avg_ms * 1e-3) / 1e12
    r = {"kernel": kernel, "workload": workload, "bound": bound,
         "avg_launch_us": round(avg_ms * 1e3, 2), "median_launch_us": round(med_ms * 1e3, 2),
         "achieved": round(achieved, 2), "peak": peak, "unit": peak_unit,
         "frac": round(achieved / peak, 4),
         "algorithmic_" + work_unit + "_per_launch": work,
         "algorithmic_hbm_bytes_per_launch": nbytes,
         "hbm_GBps_algorithmic": round(nbytes / (avg_ms * 1e-3) / 1e9, 1)}
    if extra:
        r.update(extra)
    return r


def row_fengine(reps):
    """F-engine: 256 real int8 inputs x 512 frames of 4096 (ADC noise sigma 16
    plus a unit tone at channel 777 with per-input delays), ci8 out."""
    import torch
    import paper_1708_00720_amd as bfx
    N, S, NFFT = 256, 512, 4096
    g = torch.Generator(device="cuda").manual_seed(3)
    t = torch.arange(S * NFFT, device="cuda", dtype=torch.float64)[:, None]
    tau = torch.rand(1, N, device="cuda", dtype=torch.float64, generator=g) * 50.0
    tone = torch.cos(2 * torch.pi * 777.0 * (t - tau) / NFFT)
    x = torch.randn(S * NFFT, N, device="cuda", dtype=torch.float64, generator=g) * 16.0 + tone
    x = torch.clamp(torch.round(x), -127, 127).to(torch.int8)
    del t, tone
    scale = torch.full((NFFT // 2,), 8.0 / (16.0 * (NFFT / 2) ** 0.5), device="cuda",
                       dtype=torch.float32)
    out = torch.empty(S * (NFFT // 2) * N * 2, dtype=torch.int8, device="cuda")
    avg, med, _ = time_launches(lambda: bfx.bfx_fengine(x, N, NFFT, S, scale, out, out="ci8"), reps)
    nbytes = S * NFFT * N + S * (NFFT // 2) * N * 2
    flops = int(2.5 * NFFT * 12) * S * N
    r = _row("fengine_kernel<ci8>", "256 inputs x 512 frames x 4096-point real FFT -> ci8",
             avg, med, flops, "flops", round(PEAK_FP32_UNPACKED_TFLOPS, 1), "TFLOP/s", "alu",
             nbytes,
             {"hbm_frac_algorithmic": round(nbytes / (avg * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
              "fp32_frac_of_packed_peak": round(flops / (avg * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
              "msamples_per_s": round(S * NFFT * N / (avg * 1e-3) / 1e6, 1)})
    del x, out
    return r


def _cf16_block(T, F, N, seed):
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    return torch.randn(T * F * N * 2, device="cuda", dtype=torch.float32, generator=g).to(torch.float16)


def row_xengine_f16(reps, x=None):
    """FP16 X-engine: 512 inputs, 2048 channels, 1024 samples cf16 N(0,1)."""
    import torch
    import paper_1708_00720_amd as bfx
    T, F, N = 1024, 2048, 512
    x = _cf16_block(T, F, N, 5) if x is None else x
    plan = bfx.bfx_xengine_create(N, F, "cf16")
    tune_us = bfx.bfx_xengine_autotune(plan, T)
    acc = bfx.visibilities_buffer(plan)
    avg, med, _ = time_launches(lambda: bfx.bfx_xengine_accumulate(plan, x, T, acc, overwrite=True), reps)
    cmac = F * T * N * (N + 1) // 2
    nbytes = T * F * N * 4 + F * N * (N + 1) // 2 * 8
    r = _row("xengine_f16_kernel", "512 inputs x 2048 channels x 1024 samples, cf16 -> cf32",
             avg, med, 8 * cmac, "flops", PEAK_FP16_TFLOPS, "TFLOP/s", "mfma", nbytes,
             {"tcmac_per_s": round(cmac / (avg * 1e-3) / 1e12, 2),
              "hbm_frac_algorithmic": round(nbytes / (avg * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
              "kernel_variant": bfx.bfx_xengine_variant(plan),
              "autotune_us": [round(t, 1) for t in tune_us]})
    # FP64 running sum of the binary32 dump (row a5, floating-point path)
    run64 = torch.zeros(acc.numel(), dtype=torch.float64, device="cuda")
    davg, dmed, _ = time_launches(lambda: bfx.bfx_xengine_dump(plan, acc, None, run64), max(3, reps // 2))
    dbytes = acc.numel() * 4 + run64.numel() * 16
    # the same gulp folded straight into the running sum (fused epilogue):
    # no binary32 buffer written and read back
    favg, fmed, _ = time_launches(lambda: bfx.bfx_xengine_accumulate_run64(plan, x, T, run64), max(3, reps // 2))
    fbytes = T * F * N * 4 + run64.numel() * 16
    d = _row("dump_kernel<float> (FP64 running sum)", "2048 x 131328 cf32 visibilities",
             davg, dmed, dbytes, "bytes", PEAK_HBM_GBPS, "GB/s", "hbm", dbytes,
             {"fused_accumulate_run64": {
                 "avg_launch_us": round(favg * 1e3, 2),
                 "separate_accumulate_plus_dump_us": round((avg + davg) * 1e3, 2),
                 "algorithmic_hbm_bytes_per_launch": fbytes,
                 "hbm_GBps_algorithmic": round(fbytes / (favg * 1e-3) / 1e9, 1),
                 "fp16_mfma_frac": round(8 * cmac / (favg * 1e-3) / 1e12 / PEAK_FP16_TFLOPS, 4)}})
    plan.close()
    del acc, run64
    return r, d, x


def row_beamform(reps, x=None):
    """Beamformer: 512 inputs, 2048 channels, 32 beams, 1024 samples, navg 16."""
    import torch
    import paper_1708_00720_amd as bfx
    T, F, N, B, NAVG = 1024, 2048, 512, 32, 16
    x = _cf16_block(T, F, N, 5) if x is None else x
    g = torch.Generator(device="cuda").manual_seed(6)
    th = torch.rand(F * B * N, device="cuda", dtype=torch.float64, generator=g) * (2 * torch.pi)
    w = torch.stack([torch.cos(th), torch.sin(th)], dim=-1).to(torch.float16).reshape(-1)
    del th
    out = torch.empty(B * F * (T // NAVG), dtype=torch.float32, device="cuda")
    avg, med, _ = time_launches(lambda: bfx.bfx_beamform_detect(x, w, N, F, B, T, NAVG, out), reps)
    cmac = B * F * T * N
    nbytes = T * F * N * 4 + F * B * N * 4 + out.numel() * 4
    r = _row("beamform_kernel<4>", "512 inputs x 2048 channels x 1024 samples, 32 beams, navg 16",
             avg, med, nbytes, "bytes", PEAK_HBM_GBPS, "GB/s", "hbm", nbytes,
             {"tcmac_per_s": round(cmac / (avg * 1e-3) / 1e12, 2),
              "fp16_mfma_frac": round(8 * cmac / (avg * 1e-3) / 1e12 / PEAK_FP16_TFLOPS, 4)})
    del w, out
    return r


def row_tengine(reps):
    """T-engine: 256 inputs, 128 frames of 4096-channel ci8 spectra (rounded
    Gaussian sigma 8), the whole band back to 4096 samples per frame, mixer
    1/3 channel, 4+4 output."""
    import torch
    import paper_1708_00720_amd as bfx
    S, F, N, NFFT = 128, 4096, 256, 4096
    g = torch.Generator(device="cuda").manual_seed(12)
    x = torch.clamp(torch.round(8.0 * torch.randn(S * F * N * 2, device="cuda", generator=g)),
                    -127, 127).to(torch.int8)
    out = torch.empty(S * NFFT * N, dtype=torch.uint8, device="cuda")
    avg, med, _ = time_launches(lambda: bfx.bfx_tengine(x, F, N, S, 0, NFFT, 1, 3 * NFFT, 16.0, out, out="ci4"),
                                reps)
    nbytes = S * NFFT * N * 2 + S * NFFT * N
    flops = int(5 * NFFT * 12) * S * N  # 5 N log2 N per complex transform
    r = _row("tengine_kernel<ci4>", "256 inputs x 128 frames x 4096-channel band -> 4+4 time series",
             avg, med, flops, "flops", round(PEAK_FP32_UNPACKED_TFLOPS, 1), "TFLOP/s", "alu", nbytes,
             {"hbm_frac_algorithmic": round(nbytes / (avg * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
              "msamples_per_s": round(S * NFFT * N / (avg * 1e-3) / 1e6, 1)})
    del x, out
    return r


def row_beamform_ci4(reps):
    """Integer beamformer on ci4: 512 inputs, 2048 channels, 1024 samples,
    32 beams of int8 quantized unit-modulus weights, navg 16."""
    import torch
    import paper_1708_00720_amd as bfx
    T, F, N, B, NAVG = 1024, 2048, 512, 32, 16
    g = torch.Generator(device="cuda").manual_seed(9)
    z = torch.randn(2, T * F * N, device="cuda", generator=g)
    re = torch.clamp(torch.round(2.5 * z[0]), -7, 7).to(torch.int32)
    im = torch.clamp(torch.round(2.5 * z[1]), -7, 7).to(torch.int32)
    x = (((re & 15) << 4) | (im & 15)).to(torch.uint8)
    del z, re, im
    th = torch.rand(F * B * N, device="cuda", dtype=torch.float64, generator=g) * (2 * torch.pi)
    w = torch.stack([torch.round(127 * torch.cos(th)), torch.round(127 * torch.sin(th))],
                    dim=-1).to(torch.int8).reshape(-1)
    del th
    scale = torch.full((B,), 1.0 / 127, dtype=torch.float32, device="cuda")
    out = torch.empty(B * F * (T // NAVG), dtype=torch.float32, device="cuda")
    avg, med, _ = time_launches(lambda: bfx.bfx_beamform_ci4(x, w, scale, N, F, B, T, NAVG, out), reps)
    cmac = B * F * T * N
    nbytes = T * F * N + F * B * N * 2 + out.numel() * 4
    r = _row("beamform_ci4_persistent_kernel<4>", "512 inputs x 2048 channels x 1024 samples ci4, 32 int8 beams, navg 16",
             avg, med, nbytes, "bytes", PEAK_HBM_GBPS, "GB/s", "hbm", nbytes,
             {"tcmac_per_s": round(cmac / (avg * 1e-3) / 1e12, 2),
              "int8_mfma_frac": round(8 * cmac / (avg * 1e-3) / 1e12 / PEAK_INT8_TOPS, 4)})
    del x, w, out
    return r


def row_batched(reps):
    """Batched: 8 subarrays (32..512 inputs, 1024..64 channels), ci8, 256
    samples, one persistent launch; also each subarray alone for comparison."""
    import torch
    import paper_1708_00720_amd as bfx
    T = 256
    Ns = (32, 64, 96, 128, 192, 256, 384, 512)
    Fs = (1024, 512, 512, 256, 256, 128, 128, 64)
    plan = bfx.bfx_xengine_create_batched(Ns, Fs, "ci8")
    tune_us = bfx.bfx_xengine_autotune(plan, T)
    g = torch.Generator(device="cuda").manual_seed(40)
    nin = bfx.bfx_xengine_in_bytes(plan, T)
    arena = torch.clamp(torch.round(torch.randn(nin, device="cuda", generator=g) * 8.0),
                        -127, 127).to(torch.int8)
    acc = bfx.visibilities_buffer(plan)
    avg, med, _ = time_launches(lambda: bfx.bfx_xengine_accumulate(plan, arena, T, acc, overwrite=True), reps)
    cmac = sum(F * T * N * (N + 1) // 2 for N, F in zip(Ns, Fs))
    nbytes = sum(T * F * N * 2 + F * N * (N + 1) // 2 * 8 for N, F in zip(Ns, Fs))
    # each subarray alone: standalone HBM-roofline fractions
    alone = []
    for N, F in zip(Ns, Fs):
        p1 = bfx.bfx_xengine_create(N, F, "ci8")
        bfx.bfx_xengine_autotune(p1, T)
        a1 = bfx.visibilities_buffer(p1)
        x1 = arena[:T * F * N * 2]
        a_avg, _, _ = time_launches(lambda: bfx.bfx_xengine_accumulate(p1, x1, T, a1, overwrite=True), reps)
        b1 = T * F * N * 2 + F * N * (N + 1) // 2 * 8
        alone.append({"ninput": N, "nchan": F, "avg_launch_us": round(a_avg * 1e3, 2),
                      "hbm_frac": round(b1 / (a_avg * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
                      "tcmac_per_s": round(F * T * N * (N + 1) // 2 / (a_avg * 1e-3) / 1e12, 2)})
        p1.close()
    best = max(a["hbm_frac"] for a in alone)
    frac = nbytes / (avg * 1e-3) / 1e9 / PEAK_HBM_GBPS
    r = _row("xengine_batched_kernel<ci8>", "8 subarrays (32..512 inputs), ci8, 256 samples",
             avg, med, nbytes, "bytes", PEAK_HBM_GBPS, "GB/s", "hbm", nbytes,
             {"tcmac_per_s": round(cmac / (avg * 1e-3) / 1e12, 2),
              "sum_standalone_us": round(sum(a["avg_launch_us"] for a in alone), 2),
              "best_standalone_hbm_frac": best,
              "batched_over_best_standalone": round(frac / best, 4),
              "kernel_variant": bfx.bfx_xengine_variant(plan),
              "autotune_us": [round(t, 1) for t in tune_us],
              "standalone": alone})
    plan.close()
    return r


def row_fx_xengine(reps):
    """The X half of the F+X chain: the integer X-engine on the F-engine's ci8
    output shape, 256 inputs x 2048 channels x 512 spectra (rounded Gaussian
    sigma 8 codes stand in for the channelized data)."""
    import torch
    import paper_1708_00720_amd as bfx
    N, F, T = 256, 2048, 512
    g = torch.Generator(device="cuda").manual_seed(3)
    x = torch.clamp(torch.round(8.0 * torch.randn(T * F * N * 2, device="cuda", generator=g)),
                    -127, 127).to(torch.int8)
    plan = bfx.bfx_xengine_create(N, F, "ci8")
    tune_us = bfx.bfx_xengine_autotune(plan, T)
    acc = bfx.visibilities_buffer(plan)
    avg, med, _ = time_launches(lambda: bfx.bfx_xengine_accumulate(plan, x, T, acc, overwrite=True), reps)
    cmac = F * T * N * (N + 1) // 2
    nbytes = T * F * N * 2 + F * N * (N + 1) // 2 * 8
    r = _row("xengine_int_kernel<ci8>", "256 inputs x 2048 channels x 512 spectra ci8 (the X half of F+X)",
             avg, med, nbytes, "bytes", PEAK_HBM_GBPS, "GB/s", "hbm", nbytes,
             {"tcmac_per_s": round(cmac / (avg * 1e-3) / 1e12, 2),
              "int8_mfma_frac": round(8 * cmac / (avg * 1e-3) / 1e12 / PEAK_INT8_TOPS, 4),
              "kernel_variant": bfx.bfx_xengine_variant(plan),
              "autotune_us": [round(t, 1) for t in tune_us]})
    plan.close()
    del x, acc
    return r


def row_share_g8(reps):
    """One GPU's share of the headline gulp when a node of 8 GPUs shards it
    by channel: 704 inputs x 24 channels x 1000 samples, ci4 (the corner
    turn that would deliver it is not run)."""
    import torch
    import paper_1708_00720_amd as bfx
    import synth
    F = N_CHAN // 8
    raw = synth.voltages(2, N_TIME, F, N_INPUT, "ci4", 2.5, 7, gulp=0)
    x = torch.from_numpy(raw.reshape(-1)).cuda()
    plan = bfx.bfx_xengine_create(N_INPUT, F, "ci4")
    tune_us = bfx.bfx_xengine_autotune(plan, N_TIME)
    acc = bfx.visibilities_buffer(plan)
    avg, med, _ = time_launches(lambda: bfx.bfx_xengine_accumulate(plan, x, N_TIME, acc, overwrite=True), reps)
    cmac = F * N_TIME * N_INPUT * (N_INPUT + 1) // 2
    nbytes = N_TIME * F * N_INPUT + F * N_INPUT * (N_INPUT + 1) // 2 * 8
    variant = bfx.bfx_xengine_variant(plan)
    plan.close()
    # The same share for 4 consecutive gulps in one batched launch (4
    # subarrays of 704 x 24): 4x the work items, so the grid's last round of
    # items is no longer mostly empty.
    bplan = bfx.bfx_xengine_create_batched([N_INPUT] * 4, [F] * 4, "ci4")
    btune = bfx.bfx_xengine_autotune(bplan, N_TIME)
    arena = torch.empty(bfx.bfx_xengine_in_bytes(bplan, N_TIME), dtype=torch.uint8, device="cuda")
    for k in range(4):
        io, _ = bfx.bfx_xengine_sub_offsets(bplan, k, N_TIME)
        arena[io:io + x.numel()].copy_(x)
    bacc = bfx.visibilities_buffer(bplan)
    bavg, _, _ = time_launches(lambda: bfx.bfx_xengine_accumulate(bplan, arena, N_TIME, bacc, overwrite=True),
                               reps)
    bplan.close()
    r = _row("xengine_int_kernel<ci4>", f"704 inputs x {F} channels x 1000 samples ci4 (one GPU's share "
             "of the headline gulp at 8 GPUs)", avg, med, 8 * cmac, "ops", PEAK_INT8_TOPS, "TOP/s", "mfma",
             nbytes, {"tcmac_per_s": round(cmac / (avg * 1e-3) / 1e12, 2),
                      "kernel_variant": variant,
                      "autotune_us": [round(t, 1) for t in tune_us],
                      "batched_4_gulps": {"avg_launch_us": round(bavg * 1e3, 2),
                                          "us_per_gulp": round(bavg * 1e3 / 4, 2),
                                          "frac": round(8 * 4 * cmac / (bavg * 1e-3) / 1e12 / PEAK_INT8_TOPS, 4),
                                          "autotune_us": [round(t, 1) for t in btune]}})
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch-timing-reps", type=int, default=50)
    ap.add_argument("--profile-launches", type=int, default=0,
                    help="only run this many X-engine launches on one gulp (for counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration)")
    ap.add_argument("--no-rows", action="store_true",
                    help="skip the other hot-path rows (F-engine, FP16 X, beamformer, batched)")
    ap.add_argument("--peak-probes", action="store_true",
                    help="only run the library's MFMA and HBM peak probes")
    ap.add_argument("--row-reps", type=int, default=20)
    ap.add_argument("--graph-replays", type=int, default=60,
                    help="replays of the captured 4-gulp ring cycle (timed one by one)")
    ap.add_argument("--only-row", choices=["fengine", "xf16", "beamform", "beamform_ci4", "tengine",
                                           "batched", "share_g8", "fx_xengine"],
                    help="only time one row (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the X-engine "
              "shards by channel across GPUs with no exchange beyond the F->X corner turn, "
              "which this single-GPU build does not run.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1708_00720_amd as bfx
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    if args.copy_calibration:
        # known traffic: reads 1 GiB, writes 1 GiB
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 1 << 30}), flush=True)
        return
    if args.peak_probes:
        print(json.dumps(measured_peaks()), flush=True)
        return
    if args.only_row:
        fn = {"fengine": row_fengine, "xf16": lambda r: dict(zip(("xengine_f16", "dump_run64"), row_xengine_f16(r)[:2])),
              "beamform": row_beamform, "beamform_ci4": row_beamform_ci4, "tengine": row_tengine,
              "batched": row_batched, "share_g8": row_share_g8, "fx_xengine": row_fx_xengine}[args.only_row]
        print(json.dumps(fn(args.row_reps)), flush=True)
        return
    if args.profile_launches:
        raw = synth.voltages(2, N_TIME, N_CHAN, N_INPUT, "ci4", 2.5, 7, gulp=0)
        d_in = torch.from_numpy(raw.reshape(-1)).to(dev)
        plan = bfx.bfx_xengine_create(N_INPUT, N_CHAN, "ci4")
        bfx.bfx_xengine_autotune(plan, N_TIME)  # the variant the bench line times
        vis = bfx.visibilities_buffer(plan, device=dev)
        for _ in range(args.profile_launches):
            bfx.bfx_xengine_accumulate(plan, d_in, N_TIME, vis, overwrite=True)
        torch.cuda.synchronize()
        print(json.dumps({"profile_launches": args.profile_launches}), flush=True)
        plan.close()
        return

    # ---- inputs: 4 distinct gulps, one per ring slot, resident in HBM
    gulp_bytes = N_TIME * N_CHAN * N_INPUT
    ring = torch.empty((N_SLOT, gulp_bytes), dtype=torch.uint8, device=dev)
    first_gulp = None
    for k in range(N_SLOT):
        raw = synth.voltages(2, N_TIME, N_CHAN, N_INPUT, "ci4", 2.5, 7, gulp=k)
        ring[k].copy_(torch.from_numpy(raw.reshape(-1)))
        if k == 0:
            first_gulp = raw
        print(f"[bench] gulp {k} staged", file=sys.stderr, flush=True)

    plan = bfx.bfx_xengine_create(N_INPUT, N_CHAN, "ci4")
    # plan setup, before any timing: pick the kernel variant for this shape
    tune_us = bfx.bfx_xengine_autotune(plan, N_TIME)
    variant = bfx.bfx_xengine_variant(plan)
    print(f"[bench] autotune: variant {variant}, times {tune_us} us", file=sys.stderr, flush=True)
    # ring of visibility buffers: gulp g's integration lands in slot g % 4
    vis = [bfx.visibilities_buffer(plan, device=dev) for _ in range(N_SLOT)]
    handle = plan.handle
    lib = bfx._lib
    s_ptr = stream.cuda_stream
    acc_ptrs = [v.data_ptr() for v in vis]
    slot_ptrs = [ring[k].data_ptr() for k in range(N_SLOT)]

    def gulp(g, sp):
        st = lib.bfx_xengine_accumulate(handle, slot_ptrs[g % N_SLOT], N_TIME, acc_ptrs[g % N_SLOT],
                                        bfx.BFX_ACC_OVERWRITE, sp)
        if st != 0:
            raise bfx.BfxError(st, bfx.bfx_last_error_detail())
        # hand-over in place: the consumer reads the slot (no copy, no running sum)
        st = lib.bfx_xengine_dump(handle, acc_ptrs[g % N_SLOT], None, None, sp)
        if st != 0:
            raise bfx.BfxError(st, bfx.bfx_last_error_detail())

    def step():
        for g in range(N_GULP):
            gulp(g, s_ptr)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print("[bench] timed steps done", file=sys.stderr, flush=True)

    ms_per_step = dt / args.steps * 1e3
    cmac_step = cmac_per_gulp() * N_GULP
    tcmac = cmac_step / (ms_per_step * 1e-3) / 1e12
    in_gbs = gulp_bytes * N_GULP / (ms_per_step * 1e-3) / 1e9
    out_bytes = bfx.bfx_xengine_out_bytes(plan)

    # ---- dominant kernel: average launch duration from HIP events on the
    # launch stream, one event pair per launch
    reps = args.launch_timing_reps
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for r in range(reps):
        evs[r][0].record(stream)
        lib.bfx_xengine_accumulate(handle, slot_ptrs[r % N_SLOT], N_TIME, acc_ptrs[r % N_SLOT],
                                   bfx.BFX_ACC_OVERWRITE, s_ptr)
        evs[r][1].record(stream)
    torch.cuda.synchronize()
    durs = sorted(a.elapsed_time(b) for a, b in evs)
    avg_ms = sum(durs) / len(durs)
    achieved = 8.0 * cmac_per_gulp() / (avg_ms * 1e-3) / 1e12  # TOP/s (1 CMAC = 8 int8 ops)
    roofline = {
        "kernel_variant": variant,
        "autotune_us": [round(t, 1) for t in tune_us],
        "kernel": "xengine_int_kernel<ci4>",
        "bound": "mfma",
        "achieved": round(achieved, 2),
        "peak": PEAK_INT8_TOPS,
        "unit": "TOP/s",
        "frac": round(achieved / PEAK_INT8_TOPS, 4),
        "traffic": measured_traffic(cmac_per_gulp()),
        "avg_launch_us": round(avg_ms * 1e3, 2),
        "median_launch_us": round(durs[len(durs) // 2] * 1e3, 2),
        "algorithmic_ops_per_launch": 8 * cmac_per_gulp(),
        "algorithmic_hbm_bytes_per_launch": gulp_bytes + out_bytes,
        "hbm_GBps_algorithmic": round((gulp_bytes + out_bytes) / (avg_ms * 1e-3) / 1e9, 1),
    }

    # the exact FP8-MFMA variants of the same plan, timed the same way
    fp8 = None
    if bfx.bfx_xengine_num_variants(plan) > 2:
        fp8 = {}
        for v in (2, 3):
            bfx.bfx_xengine_set_variant(plan, v)
            fevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                    for _ in range(reps)]
            for r in range(reps):
                fevs[r][0].record(stream)
                lib.bfx_xengine_accumulate(handle, slot_ptrs[r % N_SLOT], N_TIME, acc_ptrs[r % N_SLOT],
                                           bfx.BFX_ACC_OVERWRITE, s_ptr)
                fevs[r][1].record(stream)
            torch.cuda.synchronize()
            fd = sorted(a.elapsed_time(b) for a, b in fevs)
            favg = sum(fd) / len(fd)
            fp8[f"variant_{v}"] = {"avg_launch_us": round(favg * 1e3, 2),
                                   "tcmac_per_s": round(cmac_per_gulp() / (favg * 1e-3) / 1e12, 2),
                                   "fp8_frac": round(8.0 * cmac_per_gulp() / (favg * 1e-3) / 1e12 / PEAK_INT8_TOPS, 4)}
        bfx.bfx_xengine_set_variant(plan, variant)
        roofline["fp8_mfma_variants"] = fp8

    graph = graph_replay_timing(gulp, args.graph_replays)
    print("[bench] peak probes", file=sys.stderr, flush=True)
    peaks = measured_peaks()
    roofline["frac_of_measured_int8_peak"] = round(achieved / peaks["int8_mfma_TOPs"], 4)

    rows = None
    if not args.no_rows:
        rows = {}
        print("[bench] row: F-engine", file=sys.stderr, flush=True)
        rows["fengine"] = row_fengine(args.row_reps)
        print("[bench] row: FP16 X-engine + FP64 running sum", file=sys.stderr, flush=True)
        rows["xengine_f16"], rows["dump_run64"], x16 = row_xengine_f16(max(5, args.row_reps // 2))
        print("[bench] row: beamformer", file=sys.stderr, flush=True)
        rows["beamform"] = row_beamform(args.row_reps, x16)
        del x16
        print("[bench] row: T-engine", file=sys.stderr, flush=True)
        rows["tengine"] = row_tengine(args.row_reps)
        print("[bench] row: ci4 beamformer", file=sys.stderr, flush=True)
        rows["beamform_ci4"] = row_beamform_ci4(args.row_reps)
        print("[bench] row: batched", file=sys.stderr, flush=True)
        rows["batched"] = row_batched(args.row_reps)
        print("[bench] row: X half of F+X", file=sys.stderr, flush=True)
        rows["fx_xengine"] = row_fx_xengine(args.row_reps)
        print("[bench] row: one GPU's share at 8 GPUs", file=sys.stderr, flush=True)
        rows["share_g8"] = row_share_g8(args.row_reps)
        torch.cuda.empty_cache()

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu, want = cpu_baseline(first_gulp)
        # the benchmarked ring's slot 0 holds gulp 0's integration
        P = N_INPUT * (N_INPUT + 1) // 2
        nch = want.shape[0]
        got = vis[0][:nch * P * 2].cpu().numpy().astype(np.int64).reshape(nch, P, 2)
        parity = {"visibility_slot": 0, "channels_checked": int(nch),
                  "bit_exact_vs_oracle": bool(np.array_equal(got, want))}
        print(f"[bench] parity of ring slot 0 on {nch} channels: "
              f"{parity['bit_exact_vs_oracle']}", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC,
        "value": round(tcmac, 3),
        "unit": "TeraCMAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {
            "workload": "X-engine streaming: 704 inputs (352 antennas x 2 pol), 192 channels, "
                        "ci4, 1000 samples per integration, 100 gulps per step through a "
                        "4-slot device ring",
            "ninput": N_INPUT, "nchan": N_CHAN, "ntime": N_TIME, "gulps_per_step": N_GULP,
            "ring_slots": N_SLOT, "input": "ci4", "output": "ci32 lower triangle",
        },
        "input_GBps": round(in_gbs, 2),
        "roofline": roofline,
        "graph_replay": graph,
        "measured_peaks": peaks,
        "cpu_baseline": cpu,
        "parity": parity,
        "rows": rows,
    }
    print(json.dumps(line), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
