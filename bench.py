"""Throughput of the PCA holography hot path on one MI355X.

Workload: independent stacks of 32 consecutive 1024 x 1024 uint16
interferograms (the paper-scale configuration), lambda 785 nm, pitch 20 um,
z 0.3 m, principal components 2..31 kept, FP32 arithmetic.  A step is one
hh_pipeline_batch call on B stacks (default 16; --batch 1 uses hh_pipeline on
one stack): Fresnel FFT of every frame, covariance, Jacobi eigendecomposition
(one launch for the whole batch), projection + |.|^2 image.  Inputs are seeded
synthetic stacks, already resident in HBM; four distinct stacks are rotated so
that consecutive stacks never read an input that the previous one left in the
256 MB last-level cache.  Per-stack latency is measured separately on single
stacks (hh_pipeline): back to back with each waited for, and paced at the
paper's rate of 20 stacks/s (a 500 frames/s camera, a 32-frame window every 25
frames).  The roofline figure is the whole path's: the stack's algorithmic HBM
bytes (input once, the hologram written once and read twice, the image once)
over the time per stack, against the 8 TB/s HBM peak.

Prints ONE JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "interferograms/s through Fresnel+PCA (1024^2, 32-frame); % HBM roofline; p99 latency"
NT, NY, NX, K_LO, K_HI = 32, 1024, 1024, 2, 31
LAM, PITCH, Z = 785e-9, 20e-6, 0.3
HBM_PEAK_GBS = 8000.0
PCIE_PEAK_GBS = 64.0   # host link, one direction (PCIe 5.0 x16)
PAPER_INTERFEROGRAMS_PER_S = 20 * 32  # PCA of 32-frame stacks "up to 20 times per second" (Titan RTX)
PACED_STACKS_PER_S = 20.0  # 500 frames/s, a 32-frame window every 25 frames


# Algorithmic HBM bytes of each kernel, as (bytes per pixel-frame, bytes per pixel)
# of the stack it works on.  They split the stack's algorithmic bytes (input once,
# the hologram written once and read by the covariance and by the projection, the
# image once) among the kernels that move them; the FFT's row-to-column
# intermediate is not algorithmic and is not counted (it is reported from the
# counters instead).  Row pass: reads the uint16 frame (2); column pass: writes
# the hologram (8, or the 4-byte FP16 residual, plus the mean's transform);
# covariance: reads the hologram (8; 4 + the complex64 mean per pixel for the FP16
# residual; the 2-byte frames for the exact form); projection: reads the hologram
# and writes the image (4 per pixel); frame_mean: reads the frames and writes the
# float mean.
KERNEL_BYTES = {
    "fresnel_rows": (2.0, 0.0),
    "fresnel_cols": (8.0, 0.0),
    "fresnel_cols_r16": (4.0, 0.0),
    "frame_mean": (2.0, 4.0),
    "gram_partial": (8.0, 0.0),
    "gram_partial_lp": (8.0, 0.0),
    "gram_partial_r16": (4.0, 8.0),
    "gram_partial_u16": (2.0, 0.0),
    "project_complement": (8.0, 4.0),
    "project_direct": (8.0, 4.0),
    "project_r16_complement": (4.0, 12.0),
    "project_r16_direct": (4.0, 12.0),
}


K_KEPT = K_HI - K_LO + 1
# Partial images of the projection-first column pass at 1024^2 on 256 compute units
# (64 strips of 16 columns, about two groups per unit: 8 chunks of the kept list).
ENERGY_CHUNKS = 8
# Projection first (HH_PROJ_FIRST): the row pass reads the frames and writes the K
# row-transformed combined frames (8 B per pixel each); the column pass reads them
# and writes one partial image per chunk; the final sum reads the partials and
# writes the image.
KERNEL_BYTES.update({
    "proj_rows": (2.0, 8.0 * K_KEPT),
    "cols_energy": (0.0, 8.0 * K_KEPT + 4.0 * ENERGY_CHUNKS),
    "energy_sum": (0.0, 4.0 * ENERGY_CHUNKS + 4.0),
})


def algorithmic_bytes(kernel: str, launches_per_step: int) -> float:
    """Compulsory HBM bytes of one launch of `kernel` for the 1024^2 x 32 stack;
    launches that split a stack (frame groups) share its bytes evenly."""
    c = KERNEL_BYTES.get(kernel)
    if c is None:
        return float("nan")
    per_stack = c[0] * NT * NY * NX + c[1] * NY * NX
    return per_stack / max(1, launches_per_step)


# Launch choices for the 1024^2 x 32 workload, picked by the autotuner (hh_autotune)
# or by timing the candidate shapes with --tuning, and pinned so that runs are
# reproducible and comparable with the counter runs below; --autotune reruns the
# tuner instead.
PINNED_TUNING = {"fp32": "8,7,512,32,1,0", "fp32fused": "8,7,512,32,1,1", "fp16store": "8,7,256,16,0",
                 "exact": "8,7,1024,16,0",
                 "bf16": "8,7,256,32,0", "bf16x3": "8,7,256,32,0", "fp16": "8,7,256,32,0", "fp16x3": "8,7,256,32,0",
                 "fp8e4m3": "8,7,256,32,0"}

# HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE (fetch
# counter scaled by 2.000 and write by 1.000, the factors a plain 256 MiB copy gives),
# valid only for the kernel sources they were taken on (fingerprint of those files) and
# the pinned launch choices; anything else reports null.
MEASURED_TRAFFIC = {
    "fingerprint": "726137a800e68eeb",
    "fp32": {"tuning": "8,7,512,32,1,0", "bytes": {
        "fresnel_cols": (259.8 + 268.0) * 2 ** 20, "fresnel_rows": (64.4 + 256.0) * 2 ** 20,
        "gram_partial": (257.1 + 8.3) * 2 ** 20, "project_complement": (256.0 + 4.0) * 2 ** 20}},
    "fp16store": {"tuning": "8,7,256,16,0,0", "bytes": {
        "fresnel_cols_r16": (64.3 + 35.0) * 2 ** 20, "fresnel_rows": (20.3 + 64.0) * 2 ** 20,
        "gram_partial_r16": (143.0 + 16.5) * 2 ** 20, "project_r16_complement": (136.0 + 4.0) * 2 ** 20,
        "frame_mean": (64.0 + 4.0) * 2 ** 20}},
    "exact+first": {"tuning": "8,7,1024,16,0,0", "bytes": {
        "proj_rows": (64.8 + 240.0) * 2 ** 20, "cols_energy": (240.5 + 32.0) * 2 ** 20,
        "gram_partial_u16": (64.1 + 4.1) * 2 ** 20, "energy_sum": (32.0 + 4.0) * 2 ** 20}},
}


# sources of the kernels whose traffic is tabulated (the eigensolver and the host
# API are not among them: launch choices are checked through the tuning string)
TRAFFIC_SOURCES = ("fft_common.h", "hh_internal.h", "fresnel.hip", "fresnel_pca.hip", "gram.hip", "project.hip",
                   "projfirst.hip")


def source_fingerprint() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(name.encode())
        h.update(open(os.path.join(ROOT, "paper_2004_00923_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(precision: str, tuning: str, kernel: str):
    t = MEASURED_TRAFFIC.get(precision)
    if not t or t["tuning"] != tuning or MEASURED_TRAFFIC["fingerprint"] != source_fingerprint():
        return None
    return t["bytes"].get(kernel)


def stack_bytes(precision: str, proj: str = "auto") -> int:
    """Compulsory HBM bytes of one stack through the whole path: input once, the
    hologram written once and read by the covariance and by the projection, the
    image once (the row-to-column FFT intermediate is not counted).  The FP16
    storage form reads the input twice (mean, then transform), stores the residual
    in 4 bytes and the complex64 mean once (written, read twice).  Projection
    first forms no hologram: the input is read twice (covariance, row pass) and
    the K row-transformed combined frames are written and read once (counted
    here, as they are the only hologram-sized traffic of that form), plus the
    partial images."""
    npf, npx = NT * NY * NX, NY * NX
    if proj == "first":
        return npf * (2 + 2) + npx * (2 * 8 * K_KEPT + 2 * 4 * ENERGY_CHUNKS + 4)
    if precision == "fp16store":
        return npf * (2 + 2 + 3 * 4) + npx * (4 + 4 + 3 * 8 + 4)
    if precision == "exact":   # covariance from the frames: input read twice, hologram written and read once
        return npf * (2 + 2 + 2 * 8) + 4 * npx
    return npf * (2 + 3 * 8) + 4 * npx


def _host_info() -> dict:
    import platform

    import numpy as np
    import scipy
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info
        libs = [f"{d.get('internal_api')} {d.get('version')}" for d in threadpool_info() if d.get("user_api") == "blas"]
        blas = ", ".join(libs) or blas
    except Exception:  # pragma: no cover
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "numpy": np.__version__, "scipy": scipy.__version__,
            "blas": blas}


# Host cores the all-core oracle leg uses at most: a single-GPU host's share of the CPUs
# (16 per GPU), whatever os.cpu_count() reports.
HOST_CORE_SHARE = 16


def cpu_baseline(frames_list, budget_s: float = 12.0, min_runs: int = 5):
    """The FP64 oracle as it stands (numpy FFT, matmul, LAPACK eigh) on whole
    32 x 1024 x 1024 stacks, generation excluded, timed twice: BLAS on one
    thread, and BLAS on every core of the host share.  numpy's FFT has no thread
    option and runs on one thread in both legs (the oracle is not tuned for
    this).  Each leg takes the median of at least `min_runs` stacks, or of as
    many as fit in `budget_s` seconds when a stack takes longer."""
    import numpy as np
    import oracle
    from threadpoolctl import threadpool_limits
    cores = max(1, min(os.cpu_count() or 1, HOST_CORE_SHARE))
    legs = {}
    for name, threads in (("1_thread", 1), ("all_cores", cores)):
        times = []
        t_start = time.perf_counter()
        with threadpool_limits(threads):
            i = 0
            while len(times) < min_runs:
                f = frames_list[i % len(frames_list)]
                t0 = time.perf_counter()
                oracle.pipeline_ref(f, LAM, Z, PITCH, K_LO, K_HI)
                times.append(time.perf_counter() - t0)
                i += 1
                if time.perf_counter() - t_start > budget_s and len(times) >= 2:
                    break
        sec = float(np.median(times))
        legs[name] = {"threads": threads, "stacks": len(times), "median_s_per_stack": sec,
                      "interferograms_per_s": NT / sec}
    best = max(legs.values(), key=lambda leg: leg["interferograms_per_s"])
    info = _host_info()
    return {"value": best["interferograms_per_s"], "unit": "interferograms/s", "cores": best["threads"],
            "kind": "oracle",
            "sample": (f"median over {best['stacks']} whole 32x1024x1024 stacks through the FP64 numpy oracle "
                       f"(generation excluded), BLAS on {best['threads']} thread(s), numpy FFT single-threaded; "
                       f"host {info['cpu_model']}, {info['os_cpu_count']} logical CPUs, numpy {info['numpy']}, "
                       f"scipy {info['scipy']}, BLAS {info['blas']}"),
            "legs": legs, "host": info}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--paced", type=int, default=45,
                    help="stacks of the paced latency leg (one every 50 ms; the first 5 are not counted)")
    ap.add_argument("--batch", type=int, default=16,
                    help="stacks per step, processed by one hh_pipeline_batch call (1 = hh_pipeline)")
    ap.add_argument("--precision", default="fp32",
                    help="arithmetic of the covariance contraction: fp32, bf16, fp16, bf16x3, fp16x3, fp8e4m3")
    ap.add_argument("--proj", default="auto", choices=["auto", "direct", "complement", "first"],
                    help="evaluation of the image: first = projection first from the frames (needs --precision "
                         "exact)")
    ap.add_argument("--streams", type=int, default=4,
                    help="consecutive batches alternate over this many streams, each with its own workspace "
                         "and images (one batch's latency-bound eigensolver overlaps the next batch's FFTs)")
    ap.add_argument("--autotune", action="store_true",
                    help="run the autotuner first (untimed) instead of the pinned launch choices")
    ap.add_argument("--tuning", default=None,
                    help="launch choices 'rows,cols,pxw,group[,gram_ref[,fused]]', e.g. 2,0,512,0 (default: the pinned "
                         "ones)")
    ap.add_argument("--workload", default="stack", choices=["stack", "batched8", "serve", "eigh"],
                    help="stack: the 1024^2 x 32 headline; batched8: 8 uneven stacks replayed as one HIP graph; "
                         "serve: two simulated cameras through the streaming server; eigh: the eigensolver alone "
                         "at 16, 32 and 64 frames")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (each stack is "
              "independent: more GPUs would each run this same per-GPU workload).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2004_00923_amd.hh as hh
    from paper_2004_00923_amd.synth import gen_stack

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev).fill_(1)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": a.numel(), "copies": 5}))
        return
    if args.workload == "batched8":
        return bench_batched8(args, hh, torch, dev)
    if args.workload == "serve":
        return bench_serve(args, hh, torch, dev)
    if args.workload == "eigh":
        return bench_eigh(args, hh, torch, dev)
    print("bench: generating 4 synthetic 32x1024x1024 stacks", file=sys.stderr, flush=True)
    host = [gen_stack(s, NT, NY, NX) for s in range(4)]
    frames = [torch.from_numpy(f).to(dev) for f in host]
    if args.precision not in hh.PRECISIONS:
        print(f"bench.py: unknown --precision {args.precision}; one of {sorted(hh.PRECISIONS)}", file=sys.stderr)
        sys.exit(2)
    p = hh.Params(nx=NX, ny=NY, nt=NT, k_lo=K_LO, k_hi=K_HI, precision=hh.PRECISIONS[args.precision],
                  proj_mode=hh.PROJ_MODES[args.proj])
    form = args.precision + ("+first" if args.proj == "first" else "")
    B = max(1, args.batch)
    ws1 = hh.alloc_workspace(hh.workspace_bytes(p), dev)
    if args.autotune:
        print("bench: autotuning launch choices (untimed)", file=sys.stderr, flush=True)
        hh.autotune(p, frames[0], ws1, reps=5)
    else:
        vals = [int(v) for v in (args.tuning or PINNED_TUNING.get(args.precision, "0,0,256,0")).split(",")]
        hh.tuning_set(p, *vals)
    tuning = hh.tuning_get(p)
    tuning_str = ",".join(str(tuning[k]) for k in ("fft_rows", "fft_cols", "gram_pxw", "group", "gram_ref", "fused"))
    img1 = torch.empty((NY, NX), dtype=torch.float32, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    S = max(1, args.streams) if B > 1 else 1
    streams = [torch.cuda.current_stream(dev)] + [torch.cuda.Stream(device=dev) for _ in range(S - 1)]
    if B > 1:
        ps = [p] * B
        # one workspace, image set and stream per lane of the double buffering
        lanes = []
        for _ in range(S):
            imgs_l = [torch.empty((NY, NX), dtype=torch.float32, device=dev) for _ in range(B)]
            info_l = [torch.empty(1, dtype=torch.int32, device=dev) for _ in range(B)]
            lanes.append((imgs_l, info_l, hh.alloc_workspace(hh.batch_workspace_bytes(ps), dev)))
        binfo = lanes[0][1]
        # stack j of step i reads input (i + j) % 4: consecutive stacks never share an input
        batches = [[hh.Batch(ps, [frames[(r + j) % 4] for j in range(B)], imgs_l, ws_l, infos=info_l)
                    for r in range(4)] for imgs_l, info_l, ws_l in lanes]
        if S > 1:
            main = streams[0]
            for st in streams[1:]:
                st.wait_stream(main)

    def step(i, single=False, one_stream=False):
        if single or B == 1:
            hh.hh_pipeline(p, frames[i % 4], img1, ws1, info=info)
        elif one_stream:
            batches[0][i % 4].run(streams[0])
        else:
            batches[i % S][i % 4].run(streams[i % S])

    print(f"bench: warmup {args.warmup}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    sweeps = int((binfo[0] if B > 1 else info).cpu()[0])

    # timed region: exactly K steps, synchronised on both sides
    print(f"bench: timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = NT * B * args.steps / elapsed

    # per-kernel durations from HIP events recorded around each launch, over a
    # second timed pass of the same K steps on one stream (kernels in isolation)
    hh.profile_reset()
    hh.profile_enable(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        step(i, one_stream=True)
    torch.cuda.synchronize()
    prof_elapsed = time.perf_counter() - t1
    hh.profile_enable(False)
    prof = hh.profile_read()
    hh.profile_reset()
    kernels = {}
    for name, (n, total_ms) in prof.items():
        per_step = n / (args.steps * B)
        avg_us = 1e3 * total_ms / n
        b = algorithmic_bytes(name, max(1, round(per_step)))
        kernels[name] = {"launches_per_step": per_step, "avg_us": avg_us,
                         "share": total_ms / (1e3 * prof_elapsed) if prof_elapsed > 0 else None,
                         "gbs": (b / (avg_us * 1e-6) / 1e9) if b == b else None}
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches_per_step"])
    d = kernels[dom]
    sb = stack_bytes(args.precision, args.proj)
    ms_per_stack = ms_per_step / B
    stack_gbs = sb / (ms_per_stack * 1e-3) / 1e9
    # measured HBM bytes per stack: every kernel's counter bytes times its launches per stack
    per_kernel_traffic = {k: measured_traffic(form, tuning_str, k) for k in kernels}
    stack_traffic = None
    if all(v is not None for k, v in per_kernel_traffic.items() if kernels[k]["gbs"] is not None):
        stack_traffic = sum(v * kernels[k]["launches_per_step"] for k, v in per_kernel_traffic.items()
                            if v is not None)
    # the whole path against HBM: the stack's algorithmic bytes over the time per stack
    roofline = {"bound": "hbm", "scope": "whole stack (every kernel of the path, throughput run)",
                "achieved": stack_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": stack_gbs / HBM_PEAK_GBS,
                "traffic": stack_traffic,
                "traffic_unit": "HBM bytes per stack, rocprofv3 FETCH_SIZE x2 + WRITE_SIZE summed over the kernels",
                "algorithmic_bytes": sb, "us_per_stack": 1e3 * ms_per_stack}
    # the dominant kernel alone, on its share of the algorithmic bytes
    kernel_roofline = {"bound": "hbm", "kernel": dom, "achieved": d["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": (d["gbs"] / HBM_PEAK_GBS) if d["gbs"] else None,
                       "traffic": per_kernel_traffic.get(dom),
                       "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE)",
                       "algorithmic_bytes": algorithmic_bytes(dom, max(1, round(d["launches_per_step"]))),
                       "avg_us": d["avg_us"]}

    # isolated per-stack latency (each stack waited for)
    lat = []
    for i in range(60):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        step(i, single=True)
        e1.record()
        torch.cuda.synchronize()
        lat.append(e0.elapsed_time(e1))
    lat = np.array(lat[10:])

    # paced: one stack every 1/20 s (a 500 frames/s camera, 32-frame windows every 25
    # frames); latency from the launch of the stack to its image
    paced = []
    period = 1.0 / PACED_STACKS_PER_S
    t_next = time.perf_counter()
    for i in range(args.paced):
        while time.perf_counter() < t_next:
            time.sleep(max(0.0, min(0.002, t_next - time.perf_counter())))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        step(i, single=True)
        e1.record()
        e1.synchronize()
        paced.append(e0.elapsed_time(e1))
        t_next += period
    paced = np.array(paced[5:]) if len(paced) > 10 else np.array(paced)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "interferograms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": value / PAPER_INTERFEROGRAMS_PER_S,
        "dtype": "f32" if args.precision == "fp32" else f"f32 ({args.precision} covariance operands)",
        "data": "synthetic",
        "config": {"workload": f"{B} stacks of 32x1024x1024 uint16 per step (one hh_pipeline_batch call; 4 seeded "
                               f"stacks rotated), lambda 785 nm, pitch 20 um, z 0.3 m, PCs 2..31, {form}",
                   "stacks_per_s": value / NT, "precision": args.precision, "proj": args.proj,
                   "jacobi_sweeps": sweeps,
                   "stacks_per_step": B, "ms_per_stack": ms_per_stack, "tuning": tuning,
                   "streams": S},
        "roofline": roofline,
        "kernel_roofline": kernel_roofline,
        "latency_ms": {"isolated_p50": float(np.percentile(lat, 50)), "isolated_p99": float(np.percentile(lat, 99)),
                       "paced_stacks_per_s": PACED_STACKS_PER_S, "paced_stacks": int(len(paced)),
                       "p50": float(np.percentile(paced, 50)) if len(paced) else None,
                       "p99": float(np.percentile(paced, 99)) if len(paced) else None},
        "kernels": kernels,
    }
    if not args.no_cpu:
        print("bench: timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(host)
    print(json.dumps(out), flush=True)

def bench_eigh(args, hh, torch, dev):
    """The FP64 eigensolver alone (Eq. (5)): the covariance of one seeded 128^2 stack of
    16, 32 and 64 frames, formed on the GPU (hh_fresnel, hh_covariance), solved one
    problem per launch by the Jacobi solver and by the Householder + QL solver; HIP
    events on the launch stream, median and minimum over the timed launches."""
    import numpy as np
    from paper_2004_00923_amd.synth import gen_stack
    reps = max(5, min(args.steps, 200))
    out = {}
    for n in (16, 32, 64):
        p = hh.Params(nx=128, ny=128, nt=n, k_lo=0, k_hi=n - 1)
        frames = torch.from_numpy(gen_stack(3, n, 128, 128)).to(dev)
        holo = torch.empty((n, 128, 128), dtype=torch.complex64, device=dev)
        hh.hh_fresnel(p, frames, holo)
        ws = hh.alloc_workspace(hh.covariance_workspace_bytes(p), dev)
        cov = torch.empty((n, n), dtype=torch.complex128, device=dev)
        hh.hh_covariance(p, holo, cov, ws)
        ev = torch.empty(n, dtype=torch.float64, device=dev)
        V = torch.empty((n, n), dtype=torch.complex128, device=dev)
        info = torch.empty(1, dtype=torch.int32, device=dev)
        solvers = (("jacobi", lambda: hh.hh_eigh(n, cov, ev, V, info)),
                   ("tridiag", lambda: hh.hh_eigh_tridiag(n, cov, ev, V, info)))
        for name, fn in solvers:
            for _ in range(max(1, args.warmup // 10)):
                fn()
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                fn()
                b.record()
                b.synchronize()
                ts.append(a.elapsed_time(b) * 1e3)
            out[f"{name}_{n}"] = {"median_us": float(np.median(ts)), "min_us": float(min(ts)),
                                  "info": int(info.item())}
    print(json.dumps({"metric": "FP64 eigensolver time per problem (one workgroup per problem)", "unit": "us",
                      "higher_is_better": False, "data": "synthetic", "steps": reps,
                      "config": {"workload": "eigh of the covariance of one seeded 128x128 stack of 16, 32 and 64 "
                                             "frames, one problem per launch"},
                      "results": out}), flush=True)


def bench_batched8(args, hh, torch, dev):
    """8 uneven stacks (frames 512^2, 1024^2, 2048x1024; 16, 32, 64 frames; seeds
    0..7) captured once as a HIP graph; a step is one graph replay."""
    import numpy as np
    from paper_2004_00923_amd.synth import gen_stack
    shapes, nts = [(512, 512), (1024, 1024), (1024, 2048)], [16, 32, 64]
    specs = [(nts[(i + i // 3) % 3],) + shapes[i % 3] for i in range(8)]
    print("bench: generating the 8 uneven stacks", file=sys.stderr, flush=True)
    frames = [torch.from_numpy(gen_stack(i, nt, ny, nx)).to(dev) for i, (nt, ny, nx) in enumerate(specs)]
    tunings = {}
    forms = {}
    for form in ("fp32", args.precision if args.precision != "fp32" else "bf16x3"):
        prec = hh.PRECISIONS[form]
        ps = [hh.Params(nx=nx, ny=ny, nt=nt, k_lo=2, k_hi=nt - 1, precision=prec if nt <= 32 else hh.HH_FP32)
              for nt, ny, nx in specs]
        imgs = [torch.empty((ny, nx), dtype=torch.float32, device=dev) for _, ny, nx in specs]
        # the autotuner picks the launch choices of every distinct shape (untimed), then the graph is captured
        for i, p in enumerate(ps):
            key = (form, p.nx, p.ny, p.nt)
            if key not in tunings:
                print(f"bench: autotuning {p.nt}x{p.ny}x{p.nx} {form}", file=sys.stderr, flush=True)
                tws = hh.alloc_workspace(hh.workspace_bytes(p), dev)
                tunings[key] = hh.autotune(p, frames[i], tws, reps=3)
                del tws
        ws = hh.alloc_workspace(hh.batch_workspace_bytes(ps), dev)
        g = hh.Graph(ps, frames, imgs, ws)
        stream = torch.cuda.current_stream()
        for _ in range(args.warmup):
            g.launch(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.launch(stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # each launch alone, bracketed by HIP events on the stream it is launched on
        durs = []
        for _ in range(min(args.steps, 20)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            g.launch(stream)
            b.record(stream)
            b.synchronize()
            durs.append(a.elapsed_time(b) * 1e-3)
        g.close()
        nfr = sum(nt for nt, _, _ in specs)
        npf = sum(nt * ny * nx for nt, ny, nx in specs)
        # algorithmic bytes per launch: per px-frame 2 (frames) + 8 x 3 (H written once,
        # read by the covariance and by the projection); per pixel 4 (image)
        byt = sum(nt * ny * nx * 26 + 4 * ny * nx for nt, ny, nx in specs)
        launch_s = float(np.mean(durs))
        gbs = byt / launch_s / 1e9
        forms[form] = {"interferograms_per_s": nfr * args.steps / el, "ms_per_launch": 1e3 * el / args.steps,
                       "px_frames_per_s": npf * args.steps / el,
                       "hbm_frac": byt * args.steps / el / 1e9 / HBM_PEAK_GBS,
                       "roofline": {"bound": "hbm", "scope": "one graph launch (every kernel of the 8 stacks)",
                                    "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                                    "traffic": None, "algorithmic_bytes": byt, "us_per_launch": 1e6 * launch_s}}
    f32 = forms["fp32"]
    out = {"metric": "interferograms/s through Fresnel+PCA, 8 uneven stacks per graph launch",
           "value": f32["interferograms_per_s"], "unit": "interferograms/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": f32["ms_per_launch"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "8 uneven stacks (512^2x16, 1024^2x32, 2048x1024x64, 512^2x32, 1024^2x64, "
                                  "2048x1024x16, 512^2x64, 1024^2x16), seeds 0..7, PCs 2..nt-1, one HIP graph",
                      "interferograms_per_launch": sum(nt for nt, _, _ in specs)},
           "roofline": f32["roofline"],
           "forms": forms,
           "tuning": {f"{k[0]} {k[3]}x{k[2]}x{k[1]}": v for k, v in tunings.items()}}
    print(json.dumps(out), flush=True)


def bench_serve(args, hh, torch, dev):
    """Two simulated cameras (1024^2 at 500 frames/s, 2048x1024 at 250 frames/s),
    32-frame windows every 25 frames, through the streaming server: paced at the
    camera rates for latency, then unthrottled for the sustained rate."""
    from paper_2004_00923_amd.serve import CameraSpec, Server, summarize
    from paper_2004_00923_amd.synth import gen_stack
    n_src = 57
    print("bench: generating camera frames", file=sys.stderr, flush=True)
    src = {}
    for name, ny, nx, seed in (("A", 1024, 1024, 100), ("B", 1024, 2048, 101)):
        f = gen_stack(seed, n_src, ny, nx)
        t = torch.empty(f.shape, dtype=torch.uint16, pin_memory=True)
        t.copy_(torch.from_numpy(f))
        src[name] = t
    res = {}
    # the server analyses FP32 holograms held in its rings: the forms that read them
    mixed = args.precision if args.precision not in ("fp32", "fp16store", "exact") else "fp16"
    forms = ["fp32", mixed]
    for form in forms:
        cams = [CameraSpec("A", 1024, 1024, 500.0, 100, precision=form),
                CameraSpec("B", 1024, 2048, 250.0, 101, precision=form)]
        for paced, wa, wb in ((True, 40, 20), (False, 120, 60)):
            srv = Server(hbm_budget_bytes=64 << 30, device=dev)
            for c in cams:
                srv.admit(c, src[c.name])
            print(f"bench: serve {form} {'paced' if paced else 'unthrottled'}", file=sys.stderr, flush=True)
            srv.run({"A": 4, "B": 2}, paced=False)   # warm-up
            r = srv.run({"A": wa, "B": wb}, paced=paced)
            res[f"{form}_{'paced' if paced else 'unthrottled'}"] = summarize(r, cams)
    a = res["fp32_paced"]["A"]
    # algorithmic HBM bytes of one window with the resident ring (hop new frames read
    # as uint16 and written as holograms, the window's holograms read twice, the image)
    hop, win = 25, 32
    win_bytes = {"A": 1024 * 1024 * (hop * (2 + 8) + win * 8 * 2 + 4),
                 "B": 2048 * 1024 * (hop * (2 + 8) + win * 8 * 2 + 4)}
    # frames enter over the host link: each window brings `hop` new uint16 frames
    in_bytes = {"A": 1024 * 1024 * 2 * hop, "B": 2048 * 1024 * 2 * hop}
    for k, v in res.items():
        if k.endswith("unthrottled"):
            gbs = sum(v[n]["windows_per_s"] * win_bytes[n] for n in ("A", "B")) / 1e9
            v["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": gbs / HBM_PEAK_GBS, "bytes_per_window": win_bytes}
            ing = sum(v[n]["windows_per_s"] * in_bytes[n] for n in ("A", "B")) / 1e9
            v["ingest"] = {"bound": "host link (PCIe 5.0 x16)", "achieved": ing, "peak": PCIE_PEAK_GBS,
                           "unit": "GB/s", "frac": ing / PCIE_PEAK_GBS, "bytes_per_window": in_bytes}
    # the FFT row of Table 1: one 32-frame window per frame (hop 1) of a 1024^2 camera
    # at 500 frames/s, demodulated by the temporal DFT (Eqs. (8)-(9), band 8..24 of the
    # paper = 0-based 7..23): paced for latency, then unthrottled for the sustained rate
    fspec = CameraSpec("F", 1024, 1024, 500.0, 100, hop=1, k_lo=7, k_hi=23, demod="fourier", ring_hops=96)
    fourier = {}
    for paced, wf in ((True, 250), (False, 1000)):
        srv = Server(hbm_budget_bytes=64 << 30, device=dev)
        srv.admit(fspec, src["A"])
        print(f"bench: serve fourier hop 1 {'paced' if paced else 'unthrottled'}", file=sys.stderr, flush=True)
        srv.run({"F": 8}, paced=False)   # warm-up
        r = srv.run({"F": wf}, paced=paced)
        sm = summarize(r, [fspec])["F"]
        # output voxels: the window's 32 holograms demodulated per output image
        sm["output_gvoxel_per_s"] = sm["windows_per_s"] * 32 * 1024 * 1024 / 1e9
        # algorithmic bytes per output: one new frame read as uint16 and written as a
        # hologram, the window's 32 holograms read once, the image
        # algorithmic bytes per window: the new frame in, its hologram written and read once,
        # the image out; a window that reads its 32 holograms itself moves 270 B per pixel
        # (runs of consecutive windows rendered in one launch share 31 of them through the cache)
        fb = 1024 * 1024 * (2 + 8 + 8 + 4)
        fr = 1024 * 1024 * (2 + 8 + 32 * 8 + 4)
        gbs = sm["windows_per_s"] * fb / 1e9
        sm["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": gbs / HBM_PEAK_GBS, "bytes_per_window": fb,
                          "window_reads_gbs": sm["windows_per_s"] * fr / 1e9,
                          "window_reads_frac": sm["windows_per_s"] * fr / 1e9 / HBM_PEAK_GBS,
                          "window_reads_bytes_per_window": fr}
        fourier["paced" if paced else "unthrottled"] = sm
    out = {"metric": "frame-to-image latency p99 (ms), camera A 1024^2 at 500 frames/s, with camera B",
           "value": a["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": 40, "warmup": 4,
           "ms_per_step": a["p50_ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "camera A 1024^2 @500 fps + camera B 2048x1024 @250 fps, window 32, hop 25, "
                                  "hologram rings resident in HBM, continuous batching"},
           "sustained_windows_per_s": {k: v["A"]["windows_per_s"] + v["B"]["windows_per_s"]
                                       for k, v in res.items() if k.endswith("unthrottled")},
           "roofline": res["fp32_unthrottled"]["roofline"],
           "ingest": res["fp32_unthrottled"]["ingest"],
           "serve": res,
           "fourier_hop1": fourier}
    print(json.dumps(out), flush=True)



if __name__ == "__main__":
    main()
