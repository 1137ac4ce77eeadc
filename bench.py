#!/usr/bin/env python3
"""Throughput of the QTAM forward + inverse transform on one MI355X.

Workload (the batched form): 256 segments x 131072 samples (32 s at 4096 Hz) of
seeded coloured Gaussian noise with an injected chirp and two sine-Gaussian
glitches each; 256 log-spaced rows from 10 to 2048 Hz; Q in {4, 8, 16}, each
its own plan; FP32. One step = forward + inverse of the whole batch under each
of the three plans (the forward as one sweep that computes each segment's
spectrum once for the three). Inputs are resident in HBM before timing starts.

`--workload one|precision|diff` times the other workloads instead (one
segment; 32 x 256 s at 8192 Hz; the differentiable denoiser's training step),
with their error against the oracle on a sample; `--serving` the serving loop.

Prints one JSON line (rank 0). Extra fields: latency percentiles of a step,
per-kernel times measured with HIP events on the launch stream, the roofline of
the dominant kernel and of the whole path, and the FP64 CPU oracle timed on a
bounded sample of the same workload (with the error of the GPU results on that
sample against it).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s

WORKLOAD = dict(fs=4096.0, n=131072, batch=256, rows=256, f_min=10.0, f_max=2048.0, qs=(4.0, 8.0, 16.0))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=WORKLOAD["batch"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg (profiling runs)")
    ap.add_argument("--cpu-cores", type=int, default=16,
                    help="host processes of the all-cores oracle timing (1: skip it)")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--serving", action="store_true",
                    help="run the continuous-batching serving workload instead")
    ap.add_argument("--rate", type=float, default=200.0, help="serving: Poisson arrival rate (1/s)")
    ap.add_argument("--duration", type=float, default=30.0, help="serving: seconds of arrivals")
    ap.add_argument("--hbm-budget-gb", type=float, default=96.0, help="serving: device memory budget")
    ap.add_argument("--sweep", default="1000,5000,20000", help="serving: extra arrival rates for the saturation sweep")
    ap.add_argument("--no-composite", action="store_true", help="skip the composite-bank leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the bounded serving leg")
    ap.add_argument("--separate-plans", action="store_true",
                    help="time each plan's own forward (its own spectrum) instead of the forward sweep")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the short timing of the other forward form (profiling runs)")
    ap.add_argument("--workload", default="batched", choices=["batched", "one", "precision", "diff"],
                    help="which workload to time (batched: the default benchmark)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run only a plain device copy of 1 GiB (calibrates the HBM byte counters)")
    return ap.parse_args()


COPY_PROBE_BYTES = 1 << 30
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic_256x131072_fp32.txt")


def copy_probe():
    """A plain device-to-device copy of COPY_PROBE_BYTES (reads and writes that
    many bytes once): what FETCH_SIZE / WRITE_SIZE read for it scales the
    counters to bytes."""
    import torch
    src = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": COPY_PROBE_BYTES, "launches": 3}), flush=True)
    return 0


def source_digest() -> str:
    """Digest of the kernel sources: counters taken on other sources are stale."""
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2603_29785_amd", "csrc")
    for name in sorted(os.listdir(base)):
        if name.endswith((".hip", ".hpp", ".cpp")):
            with open(os.path.join(base, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, batch: int):
    """Calibrated HBM bytes per launch of `kernel` from the committed counter
    summary, or None when it is absent, for another batch, or stale."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_digest") != source_digest() or int(kv.get("batch", -1)) != batch or kernel not in kv:
        return None
    return float(kv[kernel])


def long_rows(plan) -> bool:
    """Envelope rows longer than one workgroup's transform go through two
    passes (the first forward pass and the second inverse pass then move only
    the intermediate)."""
    return plan.N_out > (8192 if plan.fp64 else 32768)


def kernel_bytes(kind: str, plan, batch: int, b: int):
    """Algorithmic bytes of one launch (b = bytes per real): the kernel's share
    of what forward + inverse must move per segment, 2 b N + 4 b R N_out (read
    the signal, write the envelopes, read them, write the reconstruction).
    Kernels that only pass intermediates between those (spectrum, packed kept
    slots, half spectrum) have a share of 0."""
    N, R, no = plan.N, plan.R, plan.N_out
    x, y = N * b, R * no * 2 * b
    two = long_rows(plan)
    # N/2 = 3 2^k or 5 2^k: a permutation kernel reads the signal and another
    # writes the reconstruction; the power-of-two transforms between move
    # intermediates only
    dec = (N // 2) & (N // 2 - 1) != 0
    xt = 0 if dec else x
    per_seg = {
        "spectrum_fft": xt, "spectrum_fft_pass1": xt, "spectrum_permute": x,    # read the signal
        "spectrum_fft_pass2": 0, "spectrum_twist": 0, "spectrum_radix": 0,
        "fwd_rows": 0 if two else y, "fwd_rows_pass2": y if two else 0,        # write the envelopes
        "inv_rows": y, "inv_rows_pass2": 0,                                     # read the envelopes
        "overlap_add": 0, "synthesis_radix": 0, "synthesis_fft_pass1": 0,
        "synthesis_fft": xt, "synthesis_fft_pass2": xt, "synthesis_permute": x,  # write the reconstruction
    }.get(kind)
    return None if per_seg is None else float(per_seg) * batch


def design_bytes(kind: str, plan, batch: int, b: int):
    """Bytes one launch reads and writes once by this design (its input and
    output buffers, intermediates included): signal [N], half spectrum [N/2]
    complex, envelopes [R, N_out] complex, kept slots [sum of row supports]
    complex, per segment."""
    N, R, no, sl = plan.N, plan.R, plan.N_out, plan.info.sum_len
    c = 2 * b
    per_seg = {
        "fwd_rows": R * no * c + (N // 2) * c,           # write envelopes, read the spectrum once
        "inv_rows": R * no * c + sl * c,                 # read envelopes, write the kept slots
        "overlap_add": sl * c + (N // 2) * c,            # read kept slots, write the half spectrum
        "spectrum_fft": N * b + (N // 2) * c,            # read signal, write spectrum
        "spectrum_twist": 2 * (N // 2) * c,              # read and write the half spectrum in place
        "spectrum_fft_pass1": N * b + (N // 2) * c,
        "spectrum_fft_pass2": 2 * (N // 2) * c,
        "synthesis_fft": (N // 2) * c + N * b,
        "synthesis_fft_pass1": 2 * (N // 2) * c,
        "synthesis_fft_pass2": (N // 2) * c + N * b,
    }.get(kind)
    return None if per_seg is None else float(per_seg) * batch


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), else the platform's."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py times one GPU only: segments shard across GPUs with no exchange, so each "
              "GPU's share is this same single-GPU run; multi-GPU runs are not supported, use --gpus 1",
              file=sys.stderr)
        return 2
    if args.serving:
        return serving_main(args)
    if args.copy_probe:
        return copy_probe()
    if args.workload != "batched":
        return other_workload(args)

    import torch
    import paper_2603_29785_amd as qt
    import synthetic

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    W = WORKLOAD
    B = args.batch
    b = 8 if args.precision == "fp64" else 4
    rdt = torch.float64 if args.precision == "fp64" else torch.float32

    t0 = time.time()
    x_host = synthetic.batched_segments(B, W["n"], W["fs"], dtype=np.float64)
    x = torch.from_numpy(x_host).to(device=dev, dtype=rdt)
    print("inputs ready in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)
    plans = [qt.Plan(W["fs"], W["n"], q, W["f_min"], W["f_max"], W["rows"], precision=args.precision)
             for q in W["qs"]]
    n_out = plans[0].N_out
    assert all(p.N_out == n_out for p in plans)
    ws_bytes = max(p.workspace_bytes(B) for p in plans)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    cdt = torch.complex128 if b == 8 else torch.complex64
    ys = [torch.empty((B, W["rows"], n_out), dtype=cdt, device=dev) for _ in plans]
    xr = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)

    def step_sweep():
        # the Q set as one sweep: each segment's spectrum once, every plan's rows from it
        qt.forward_sweep(plans, x, outs=ys, ws=ws, stream=stream)
        for p, y in zip(plans, ys):
            p.inverse(y, out=xr, ws=ws, stream=stream)

    def step_separate():
        for p, y in zip(plans, ys):
            p.forward(x, out=y, ws=ws, stream=stream)
            p.inverse(y, out=xr, ws=ws, stream=stream)

    step, other = (step_separate, step_sweep) if args.separate_plans else (step_sweep, step_separate)
    form = "separate plans" if args.separate_plans else "forward sweep"

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    lat = np.array([a.elapsed_time(c) for a, c in ev])
    samples_per_step = len(plans) * B * W["n"]
    value = samples_per_step * args.steps / wall
    ms_per_step = 1e3 * wall / args.steps
    print("timed %d steps: %.3f ms/step" % (args.steps, ms_per_step), file=sys.stderr, flush=True)

    # whole-path roofline, algorithmic bytes per segment: each plan writes and
    # reads its envelopes (4 b R N_out) and writes a reconstruction (b N); the
    # signal is read once by the sweep, once per plan by separate plans
    reads_x = len(plans) if args.separate_plans else 1
    alg_path = B * (reads_x * b * W["n"] + len(plans) * (b * W["n"] + 4 * b * W["rows"] * n_out))
    path_gbs = alg_path / (ms_per_step * 1e-3) / 1e9

    # the other forward form, briefly, for comparison
    compare = None
    if not args.no_compare:
        for _ in range(3):
            other()
        torch.cuda.synchronize()
        reps = max(5, min(10, args.steps))
        t0 = time.perf_counter()
        for _ in range(reps):
            other()
        torch.cuda.synchronize()
        compare = {"form": "forward sweep" if args.separate_plans else "separate plans",
                   "ms_per_step": 1e3 * (time.perf_counter() - t0) / reps, "steps": reps}

    # per-kernel durations with HIP events on the launch stream
    kernels = {}
    roofline = None
    path_counters = None
    if not args.no_kernel_timing:
        for p in plans:
            p.timing(True)
        reps = max(3, min(10, args.steps))
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        for p in plans:
            for name, (ms, cnt) in p.timing_collect().items():
                k = kernels.setdefault(name, dict(total_ms=0.0, launches=0, bytes=0.0, design_bytes=0.0))
                k["total_ms"] += ms
                k["launches"] += cnt
                # one call per plan and step covers the batch (in chunks)
                k["bytes"] += (kernel_bytes(name, p, B, b) or 0.0) * reps
                k["design_bytes"] += (design_bytes(name, p, B, b) or 0.0) * reps
            p.timing(False)
        for name, k in kernels.items():
            k["avg_ms"] = k["total_ms"] / max(k["launches"], 1)
            k["achieved_GBs"] = k["bytes"] / (k["total_ms"] * 1e-3) / 1e9 if k["total_ms"] > 0 else None
            k["design_GBs"] = k["design_bytes"] / (k["total_ms"] * 1e-3) / 1e9 if k["total_ms"] > 0 else None
        # whole path by the calibrated HBM counters of the committed profile
        # (when it was taken on these kernel sources): bytes moved per step
        # over the step time
        if args.precision == "fp32":
            moved = [measured_traffic(n, B) for n in kernels]
            if all(m is not None for m in moved) and moved:
                per_step = sum(m * kernels[n]["launches"] for m, n in zip(moved, kernels)) / reps
                path_hbm = per_step / (ms_per_step * 1e-3) / 1e9
                path_counters = {"achieved": round(path_hbm, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(path_hbm / HBM_PEAK_GBS, 4), "bytes_per_step": per_step,
                                 "what": "HBM bytes of every kernel (FETCH_SIZE x2 + WRITE_SIZE, committed "
                                         "counters) over the step time"}
        dom = max(kernels, key=lambda n: kernels[n]["total_ms"])
        k = kernels[dom]
        ach = k["achieved_GBs"]
        nl = max(k["launches"], 1)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(dom, B) if args.precision == "fp32" else None,
                    "avg_launch_ms": round(k["avg_ms"], 4),
                    "bytes_per_launch": k["bytes"] / nl,
                    "bytes_what": "the kernel's share of the algorithmic bytes 2bN + 4bR N_out per segment "
                                  "and plan (read x, write Y, read Y, write x-hat), x segments per launch",
                    "design_bytes_per_launch": k["design_bytes"] / nl,
                    "design_frac": round(k["design_GBs"] / HBM_PEAK_GBS, 4),
                    "design_what": "every buffer the kernel reads or writes once, intermediates included"}

    out = {
        "metric": "fwd+inv QTAM samples/s @1 GPU; p50/p99 latency; recon rel-err vs FP64",
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if b == 8 else "f32",
        "data": "synthetic",
        "config": {"workload": "batched QTAM fwd+inv: %d segments x %d samples @ %g Hz, coloured noise + "
                               "chirp + 2 sine-Gaussians; Q in %s (one plan each, %s), %d rows %g-%g Hz, N_out %d"
                               % (B, W["n"], W["fs"], list(W["qs"]),
                                  "each with its own spectrum" if args.separate_plans
                                  else "forward as one sweep over a shared spectrum",
                                  W["rows"], W["f_min"], W["f_max"], n_out),
                   "form": form,
                   "batch": B, "n_samples": W["n"], "fs": W["fs"], "q": list(W["qs"]), "rows": W["rows"],
                   "f_min": W["f_min"], "f_max": W["f_max"], "n_out": n_out, "precision": args.precision},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "what": "one step (3 plans x fwd+inv of the batch), HIP events"},
        "path_roofline": {"achieved": round(path_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(path_gbs / HBM_PEAK_GBS, 4),
                          "bytes_per_step": alg_path, "counters": path_counters},
        "kernels": {n: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in k.items()}
                    for n, k in kernels.items()},
        "roofline": roofline,
        "other_form": compare,
    }

    if not args.no_composite:
        out["composite"] = composite_leg(args, x, B, W, ms_per_step)
    if not args.no_serving:
        del ys, xr, ws
        torch.cuda.empty_cache()
        out["serving"] = serving_leg(200.0, 10.0, sweep_rates=(5000.0,), sweep_duration=5.0)
    served = out["serving"].pop("served_sample") if "serving" in out else []
    if not args.no_cpu:
        out.update(cpu_leg(args, plans, x_host, x, B, W))
        if "serving" in out:
            out["serving"]["serving"]["checked"] = oracle_check_served(served)
    print(json.dumps(out), flush=True)
    return 0


OTHER_WORKLOADS = {
    "one": dict(fs=4096.0, n=16384, batch=1, rows=64, q=8.0, f_min=20.0, f_max=1000.0,
                what="one segment: 4 s at 4096 Hz, white noise + sine-Gaussian (100 Hz, Q 8, SNR 20); Q 8, "
                     "64 rows 20-1000 Hz"),
    "precision": dict(fs=8192.0, n=2097152, batch=32, rows=512, q=12.0, f_min=5.0, f_max=4096.0,
                      what="long segments: 32 x 256 s at 8192 Hz, coloured noise + chirp + 2 sine-Gaussians; "
                           "Q 12, 512 rows 5-4096 Hz"),
    "diff": dict(fs=4096.0, n=32768, batch=64, rows=128, q=8.0, f_min=20.0, f_max=2000.0,
                 what="differentiable denoiser: 64 x 8 s at 4096 Hz; forward, per-row gain x soft threshold, "
                      "inverse, MSE against the clean signal, backward through the adjoint kernels; Q 8, "
                      "128 rows 20-2000 Hz"),
}


def other_workload(args):
    """One of the other workloads: steps timed with HIP events, samples/s,
    latency; the CPU leg adds the oracle on one segment (its time and the
    GPU's error against it)."""
    import torch
    import paper_2603_29785_amd as qt
    import synthetic

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    W = OTHER_WORKLOADS[args.workload]
    B, n, fs = W["batch"], W["n"], W["fs"]
    fp64 = args.precision == "fp64"
    rdt = torch.float64 if fp64 else torch.float32
    plan = qt.Plan(fs, n, W["q"], W["f_min"], W["f_max"], W["rows"], precision=args.precision)
    stream = torch.cuda.current_stream()
    if args.workload == "one":
        x_host = synthetic.single_segment()[None, :]
    elif args.workload == "precision":
        x_host = synthetic.batched_segments(B, n, fs, workload=4, dtype=np.float64)
    else:
        x_host, clean_host = synthetic.differentiable_pairs(B, n, fs, dtype=np.float64)
    x = torch.from_numpy(x_host).to(device="cuda", dtype=rdt)
    if args.workload == "diff":
        from paper_2603_29785_amd.autograd import GainThresholdDenoiser
        clean = torch.from_numpy(clean_host).to(device="cuda", dtype=rdt)
        noise = torch.from_numpy(synthetic.coloured(n, fs, synthetic.rng_for(5, 10_000))).to(device="cuda",
                                                                                          dtype=rdt)
        model = GainThresholdDenoiser(plan, 3.0 * plan.forward(noise).abs().median(dim=-1).values)
        xin = x.clone().requires_grad_(True)

        def step():
            model.zero_grad(set_to_none=True)
            xin.grad = None
            loss = torch.mean((model(xin) - clean) ** 2)
            loss.backward()
    else:
        ws = torch.empty(plan.workspace_bytes(B), dtype=torch.uint8, device="cuda")
        y = torch.empty((B, plan.R, plan.N_out), dtype=torch.complex128 if fp64 else torch.complex64, device="cuda")
        xr = torch.empty_like(x)

        def step():
            plan.forward(x, out=y, ws=ws, stream=stream)
            plan.inverse(y, out=xr, ws=ws, stream=stream)
    steps = args.steps if args.workload != "one" else max(args.steps, 200)
    for _ in range(max(args.warmup, 2)):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    ms = 1e3 * wall / steps
    out = {"metric": "fwd+inv QTAM samples/s @1 GPU; p50/p99 latency; recon rel-err vs FP64",
           "value": B * n / (ms * 1e-3), "unit": "samples/s", "n_gpus": 1, "steps": steps,
           "warmup": max(args.warmup, 2), "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if fp64 else "f32", "data": "synthetic",
           "config": {"workload": W["what"], "batch": B, "n_samples": n, "fs": fs, "q": W["q"],
                      "rows": W["rows"], "f_min": W["f_min"], "f_max": W["f_max"], "n_out": plan.N_out,
                      "precision": args.precision},
           "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                          "what": "one step, HIP events"}}
    if not args.no_cpu:
        out.update(cpu_leg_one_segment(args, plan, W, x, fp64))
    print(json.dumps(out), flush=True)
    return 0


def composite_leg(args, x, B, W, ms_main):
    """The same Q set as one composite bank (one spectrum, one launch per
    kernel, the frame summed over all 3 R rows): forward with row statistics,
    per-segment best plane by energy, inverse from the whole bank."""
    import torch
    import paper_2603_29785_amd as qt
    planes = [(q, "bisquare", 0.0) for q in W["qs"]]
    p = qt.Plan(W["fs"], W["n"], 1.0, W["f_min"], W["f_max"], W["rows"], precision=args.precision, planes=planes)
    ws = torch.empty(p.workspace_bytes(B), dtype=torch.uint8, device=x.device)
    y = torch.empty((B, p.R, p.N_out), dtype=torch.complex128 if p.fp64 else torch.complex64, device=x.device)
    m = torch.empty((B, p.R), dtype=y.dtype, device=x.device)
    xr = torch.empty_like(x)
    stream = torch.cuda.current_stream(x.device)

    def step():
        p.forward_metric(x, out=y, metric=m, ws=ws, stream=stream)
        sel = p.select_planes(y, m, "energy", stream=stream)
        p.inverse(y, out=xr, ws=ws, stream=stream)
        return sel

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    reps = max(3, min(10, args.steps))
    t0 = time.perf_counter()
    for _ in range(reps):
        _, best, _ = step()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    counts = np.bincount(best.cpu().numpy(), minlength=p.planes).tolist()
    del y, m, ws
    return {"rows": p.R, "planes": p.planes, "ms_per_step": ms,
            "samples_per_s": len(W["qs"]) * B * W["n"] / (ms * 1e-3),
            "speed_vs_main_step": ms_main / ms, "best_plane_counts": counts,
            "what": "forward with row statistics + energy selection + inverse of one %d-row bank "
                    "(Q %s), samples counted once per plane" % (p.R, list(W["qs"]))}


# ---------------------------------------------------------------------------
# The CPU leg: the only part of the benchmark that runs the FP64 oracle. It
# times the oracle on the host (cpu_baseline) and measures the GPU results'
# error against it on the same input bits.
# ---------------------------------------------------------------------------
def cpu_leg_one_segment(args, plan, W, x_dev, fp64):
    """The other workloads' CPU leg: the oracle's forward and inverse of
    segment 0 on one host core, and the GPU's coefficients (same input bits)
    and inverse (of the oracle's coefficients rounded to the device
    precision) against it."""
    import torch
    from oracle import oracle as o
    n = W["n"]
    op = o.OraclePlan(fs=W["fs"], n=n, q=W["q"], f_min=W["f_min"], f_max=W["f_max"], rows=W["rows"])
    x0 = x_dev[0].double().cpu().numpy()
    t0 = time.perf_counter()
    Yo = op.forward(x0)
    Yc = Yo.astype(np.complex128 if fp64 else np.complex64)   # the oracle's coefficients in device precision
    xo = op.inverse(Yc.astype(np.complex128))
    t = time.perf_counter() - t0
    Yg = plan.forward(x_dev[0:1].contiguous())[0].cpu().numpy()
    xg = plan.inverse(torch.from_numpy(Yc[None]).to("cuda"))[0].cpu().numpy()
    return {"recon_rel_err": {"coef": float(np.linalg.norm(Yg - Yo) / np.linalg.norm(Yo)),
                              "recon": float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)),
                              "segments": 1, "vs": "FP64 CPU oracle", "precision": args.precision},
            "cpu_baseline": {"value": n / t, "unit": "samples/s", "cores": 1, "kind": "oracle",
                             "sample": "segment 0: one FP64 forward + inverse, %.1f ms, single thread" % (1e3 * t),
                             "host": cpu_model()}}


def oracle_check_served(served):
    """Served reconstructions (a sample spread over the serving stream)
    against the oracle's reconstruction x_M of the same input bits."""
    from oracle import oracle as o
    errs = []
    for k, x, result in served:
        op = o.OraclePlan(fs=k.fs, n=k.n, q=k.q, f_min=k.f_min, f_max=k.f_max, rows=k.rows)
        xm = op.project(x)
        errs.append(float(np.linalg.norm(result - xm) / np.linalg.norm(xm)))
    return {"requests": len(errs), "max_rel_err": max(errs) if errs else None,
            "what": "served reconstruction vs the FP64 oracle's x_M, rel-L2, on requests spread over the stream"}


def _oracle_worker(job):
    """One host process of the all-cores oracle timing: forward + inverse of
    its own segments of the batched workload (FP64) until its time is up.
    Imports numpy and the oracle only (no GPU)."""
    import synthetic
    from oracle import oracle as o
    W, first, count, seconds, fp32_inputs = job
    ops = [o.OraclePlan(fs=W["fs"], n=W["n"], q=q, f_min=W["f_min"], f_max=W["f_max"], rows=W["rows"])
           for q in W["qs"]]
    xs = synthetic.batched_segments(count, W["n"], W["fs"], first=first, dtype=np.float64)
    if fp32_inputs:
        xs = xs.astype(np.float32).astype(np.float64)
    done, t_oracle = 0, 0.0
    while t_oracle < seconds:
        ta = time.perf_counter()
        ops[done % 3].inverse(ops[done % 3].forward(xs[done % count]))
        t_oracle += time.perf_counter() - ta
        done += 1
    return done, t_oracle


def cpu_all_cores_leg(W, prec, cores, seconds):
    """The same oracle in `cores` host processes at once (one per core, own
    segments each): samples/s of the whole host."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    # fresh interpreters (spawn): nothing of this GPU process is inherited; a
    # worker that dies fails the pool instead of being replaced
    jobs = [(dict(W), 16 * k, 4, seconds, prec == "fp32") for k in range(cores)]
    with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as pool:
        futs = [pool.submit(_oracle_worker, j) for j in jobs]
        out = [f.result(timeout=4 * seconds + 120) for f in futs]
    done = sum(d for d, _ in out)
    rate = sum(d * W["n"] / t for d, t in out)   # processes ran concurrently: rates add
    return {"value": rate, "unit": "samples/s", "cores": cores, "kind": "oracle", "host": cpu_model(),
            "sample": "%d segments of %d samples over %d processes (one per core, plans cycling Q=4/8/16), "
                      "FP64 forward+inverse, %.0f s each" % (done, W["n"], cores, seconds)}


def cpu_leg(args, plans, x_host, x_dev, B, W):
    """FP64 oracle on a bounded sample of the workload (single thread), and
    the GPU's error against it on the same segments."""
    import torch
    from oracle import oracle as o

    ops = [o.OraclePlan(fs=W["fs"], n=W["n"], q=q, f_min=W["f_min"], f_max=W["f_max"], rows=W["rows"])
           for q in W["qs"]]
    prec = plans[0].params["precision"]
    t0 = time.perf_counter()
    done = 0
    errs_y, errs_x = [], []
    seg = 0
    t_oracle = 0.0
    while True:
        i = (seg * 37) % B
        p, op = plans[seg % 3], ops[seg % 3]
        xi = x_host[i]
        if prec == "fp32":
            xi = xi.astype(np.float32).astype(np.float64)
        ta = time.perf_counter()
        Yo = op.forward(xi)
        xo = op.inverse(Yo)
        done += 1
        t_oracle += time.perf_counter() - ta
        # the GPU's results on the same segment
        Yg = p.forward(x_dev[i:i + 1].contiguous())
        xg = p.inverse(Yg)
        Yg = Yg[0].cpu().numpy()
        xg = xg[0].cpu().numpy()
        errs_y.append(float(np.linalg.norm(Yg - Yo) / np.linalg.norm(Yo)))
        errs_x.append(float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)))
        seg += 1
        elapsed = time.perf_counter() - t0
        if elapsed >= args.cpu_seconds or seg >= 3 * B:
            break
    # the oracle's own time only (the GPU calls on the same segments are not counted)
    cpu_value = done * W["n"] / t_oracle
    cpu = {"value": cpu_value, "unit": "samples/s", "cores": 1, "kind": "oracle",
           "sample": "%d segments of %d samples (plans cycling Q=4/8/16), FP64 forward+inverse, "
                     "single thread, %.1f s of oracle time" % (done, W["n"], t_oracle),
           "host": cpu_model(), "host_cpus": os.cpu_count()}
    res = {"cpu_baseline": cpu,
           "recon_rel_err": {"coef_max": max(errs_y), "recon_max": max(errs_x), "segments": done,
                             "vs": "FP64 CPU oracle", "precision": prec}}
    cores = min(os.cpu_count() or 1, args.cpu_cores)
    if cores > 1:
        try:
            res["cpu_baseline_all_cores"] = cpu_all_cores_leg(W, prec, cores, min(args.cpu_seconds, 8.0))
        except Exception as e:   # the single-thread baseline above stands on its own
            res["cpu_baseline_all_cores"] = {"error": repr(e)}
    return res


def serving_leg(rate, duration, sweep_rates=(), sweep_duration=10.0, burst_n=400, hbm_budget_gb=96.0,
                check_n=8):
    """Poisson arrivals of segments of 1, 4, 16 or 64 s at 4096 or 16384 Hz,
    Q in {4, 8, 16, 32}, 64-512 rows over 10-2048 Hz, FP32, through the
    continuous-batching server (payloads in pinned host memory, as a client
    hands them over); then a saturation sweep, and a burst against the plain
    one-segment-per-launch form on the same requests. A sample of the served
    results (check_n requests spread over the stream) is kept, with its
    inputs, for the CPU leg to compare with the oracle (oracle_check_served)."""
    import torch
    import synthetic
    from paper_2603_29785_amd.serving import BucketKey, GpuExecutor, Request, Server, plain_run

    torch.cuda.set_device(0)
    pool = {}
    t0 = time.time()
    for sec in (1, 4, 16, 64):
        for fs in (4096.0, 16384.0):
            n = int(sec * fs)
            pool[(fs, n)] = [torch.from_numpy(synthetic.injected_segment(n, fs, synthetic.rng_for(3, 100 * sec + j))[0]
                                              .astype(np.float32)).pin_memory() for j in range(2)]
    print("signal pool ready in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)

    def key_of(a):
        return BucketKey(a.fs, a.n, a.q, a.rows, 10.0, 2048.0)

    def make(a, rid=[0], keep=False):
        rid[0] += 1
        return Request(rid[0], key_of(a), pool[(a.fs, a.n)][a.seed % 2], keep_result=keep)

    budget = int(hbm_budget_gb * (1 << 30))
    ex = GpuExecutor(streams=4)
    srv = Server(ex, hbm_budget=budget, streams=4)
    arrivals = synthetic.serving_stream(rate=rate, duration=duration, seed=3000)
    # warm-up: one request per bucket so plans, buffers and graphs exist
    keys = sorted({key_of(a) for a in arrivals}, key=lambda k: (k.n, k.q, k.rows, k.fs))
    t0 = time.time()
    for k in keys:
        srv.submit(Request(-1, k, pool[(k.fs, k.n)][0], keep_result=False))
    srv.drain(timeout=600)
    for res in list(srv.resources.values()):
        ex.warm(res)
    warm_rejected = sum(r.status == "rejected" for r in srv.done)
    srv.done.clear()
    srv.launches = 0
    print("warm-up: %d buckets in %.1f s (%d shapes not on the device path)"
          % (len(keys), time.time() - t0, warm_rejected), file=sys.stderr, flush=True)

    checked = set(range(0, len(arrivals), max(1, len(arrivals) // max(check_n, 1)))) if check_n else set()
    made = []

    def make_stream(a, ctr=[0]):
        r = make(a, keep=ctr[0] in checked)
        ctr[0] += 1
        if r.keep_result:
            made.append((r, a))
        return r

    srv.run_stream(arrivals, make_stream, timeout=120)
    st = srv.stats()
    st["offered_rate"] = rate
    st["offered_samples_per_s"] = sum(a.n for a in arrivals) / duration
    print("serving at %g/s: %s" % (rate, st), file=sys.stderr, flush=True)

    # a sample of served results with their input bits, for the oracle check of the CPU leg
    served = [(r.key, r.data.numpy().astype(np.float64), r.result) for r, a in made if r.status == "done"]

    sweep = []
    for sr in sweep_rates:
        srv.done.clear()
        srv.launches = 0
        arr = synthetic.serving_stream(rate=sr, duration=sweep_duration, seed=4000)
        srv.run_stream(arr, make, timeout=60)
        s2 = srv.stats()
        s2["offered_rate"] = sr
        s2["offered_samples_per_s"] = sum(a.n for a in arr) / sweep_duration
        sweep.append({k: s2.get(k) for k in ("offered_rate", "offered_samples_per_s", "completed", "p50_ms",
                                             "p99_ms", "samples_per_s", "launches")})
        print("sweep %g/s: %s" % (sr, sweep[-1]), file=sys.stderr, flush=True)
        if s2.get("p99_ms", 0) > 1000.0:
            break

    # saturation burst vs the plain form on the same requests
    burst = [make(a, keep=True) for a in synthetic.serving_stream(rate=1e6, duration=4e-4 * burst_n,
                                                                  seed=5000)[:burst_n]]
    burst = [r for r in burst if r.key in srv.resources or r.key in ex.plans]
    srv.done.clear()
    srv.launches = 0
    t0 = time.perf_counter()
    for r in burst:
        r.arrival = time.perf_counter()
        srv.submit(r)
    srv.drain(timeout=300)
    t_srv = time.perf_counter() - t0
    samples = sum(r.key.n for r in burst)
    alone = [Request(r.rid, r.key, r.data.numpy()) for r in burst]
    t_plain = plain_run(alone, plans=ex.plans)
    same = sum(np.array_equal(a.result, b.result) for a, b in zip(burst, alone))
    srv.shutdown()
    return {
        "config": "Poisson %g req/s for %g s, 1/4/16/64 s at 4096/16384 Hz, Q in 4/8/16/32, 64-512 rows "
                  "10-2048 Hz, FP32, HBM budget %g GB, 4 streams, 2 slot sets per bucket"
                  % (rate, duration, hbm_budget_gb),
        "latency_ms": {"p50": st.get("p50_ms"), "p99": st.get("p99_ms"), "max": st.get("max_ms"),
                       "what": "arrival (payload in pinned host memory) to the reconstruction back in pinned "
                               "host memory: H2D, forward+inverse, D2H"},
        "serving": st, "sweep": sweep, "served_sample": served,
        "burst": {"requests": len(burst), "seconds": t_srv, "serving_samples_per_s": samples / t_srv,
                  "plain_samples_per_s": samples / t_plain, "speedup": t_plain / t_srv,
                  "identical_results": same, "what": "burst at saturation: continuous batching vs one "
                                                     "segment per launch on the same requests"},
    }


def serving_main(args):
    """The serving workload alone, as its own bench line."""
    sweep = [float(r) for r in args.sweep.split(",") if r]
    leg = serving_leg(args.rate, args.duration, sweep, min(args.duration, 10.0), 400, args.hbm_budget_gb)
    served = leg.pop("served_sample")
    if not args.no_cpu:
        leg["serving"]["checked"] = oracle_check_served(served)
    b = leg["burst"]
    out = {
        "metric": "fwd+inv QTAM samples/s @1 GPU; p50/p99 latency; recon rel-err vs FP64",
        "value": b["serving_samples_per_s"], "unit": "samples/s", "n_gpus": 1, "steps": b["requests"],
        "warmup": 0, "ms_per_step": 1e3 * b["seconds"] / max(b["requests"], 1), "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving: " + leg["config"]},
    }
    out.update(leg)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
