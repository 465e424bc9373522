#!/usr/bin/env python3
"""Throughput of the FX-correlator X-engine on one MI355X.

Workload (the streaming configuration the headline metric is quoted on):
352 antennas x 2 polarisations = 704 inputs, 192 channels, ci4 voltages
(rounded Gaussian sigma=2.5 clipped to +-7), 1000 samples per integration.
A step streams 100 gulps through a 4-slot device ring (the paper's default
ring = 4 gulps): each gulp is one integration, correlated with
BFX_ACC_OVERWRITE into the visibility buffer and handed over by dump.  All
inputs are resident in HBM before timing starts.

Prints one JSON line.  Extra fields: input GB/s, the dominant kernel's
roofline (HIP-event-timed launches on the launch stream) and the CPU oracle's
rate on a bounded sample.
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
KERNEL_SRC = os.path.join(ROOT, "paper_1708_00720_amd", "csrc", "xengine_int.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "xengine_int_ci4_704_traffic.json")


def cmac_per_gulp():
    return N_CHAN * N_TIME * N_INPUT * (N_INPUT + 1) // 2


def kernel_hash():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(per_launch_cmac):
    """HBM bytes per launch from committed counter runs, if taken on this kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    if rec.get("kernel_sha256_16") != kernel_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(raw_gulp, budget_s=15.0):
    """Oracle X-engine on whole channels of one gulp until ~budget_s elapses."""
    import oracle
    threads = oracle.max_threads()
    done_ch = 0
    t0 = time.perf_counter()
    f = 0
    while time.perf_counter() - t0 < budget_s and done_ch < N_CHAN:
        nf = min(threads, N_CHAN - f)
        oracle.xengine_int(raw_gulp, "ci4", N_TIME, N_CHAN, N_INPUT, chans=(f, nf),
                           nthreads=threads)
        f += nf
        done_ch += nf
    dt = time.perf_counter() - t0
    cmac = done_ch * N_TIME * N_INPUT * (N_INPUT + 1) // 2
    return {"value": cmac / dt / 1e12, "unit": "TeraCMAC/s", "cores": threads, "kind": "oracle",
            "sample": f"{done_ch} of {N_CHAN} channels of one 704-input ci4 gulp "
                      f"({N_TIME} samples), int64 triple loop, {dt:.1f} s"}


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
    if args.profile_launches:
        raw = synth.voltages(2, N_TIME, N_CHAN, N_INPUT, "ci4", 2.5, 7, gulp=0)
        d_in = torch.from_numpy(raw.reshape(-1)).to(dev)
        plan = bfx.bfx_xengine_create(N_INPUT, N_CHAN, "ci4")
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
    vis = bfx.visibilities_buffer(plan, device=dev)
    handle = plan.handle
    lib = bfx._lib
    s_ptr = stream.cuda_stream
    acc_ptr = vis.data_ptr()
    slot_ptrs = [ring[k].data_ptr() for k in range(N_SLOT)]

    def step():
        for g in range(N_GULP):
            st = lib.bfx_xengine_accumulate(handle, slot_ptrs[g % N_SLOT], N_TIME, acc_ptr,
                                            bfx.BFX_ACC_OVERWRITE, s_ptr)
            if st != 0:
                raise bfx.BfxError(st, bfx.bfx_last_error_detail())
            st = lib.bfx_xengine_dump(handle, acc_ptr, acc_ptr, None, s_ptr)
            if st != 0:
                raise bfx.BfxError(st, bfx.bfx_last_error_detail())

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
        lib.bfx_xengine_accumulate(handle, slot_ptrs[r % N_SLOT], N_TIME, acc_ptr,
                                   bfx.BFX_ACC_OVERWRITE, s_ptr)
        evs[r][1].record(stream)
    torch.cuda.synchronize()
    durs = sorted(a.elapsed_time(b) for a, b in evs)
    avg_ms = sum(durs) / len(durs)
    achieved = 8.0 * cmac_per_gulp() / (avg_ms * 1e-3) / 1e12  # TOP/s (1 CMAC = 8 int8 ops)
    roofline = {
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

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(first_gulp)

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
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
