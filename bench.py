#!/usr/bin/env python3
"""Benchmark of the fused LBM step on one MI355X.

Workload: D3Q19 square duct 256x128x128, periodic x, halfway bounce-back
walls on y and z, tau0 = 0.52 with Smagorinsky closure (C_s = 0.1), Guo
forcing a_x = 1e-5, seeded +-1e-3 initial velocity, FP32 storage and
arithmetic.  A step is one call-level pass of the whole hot path: the
fused relax-propagate kernel (moments, equilibrium, force term, LES,
relaxation, in-place A-A streaming with bounce-back) every step, plus the
wall-force and balance reductions of the last step of the call.

Prints ONE JSON line (rank 0).  ``value`` = MLUPS (lattice updates per
second / 1e6) with the state resident in HBM.  ``roofline`` relates the
algorithmic bytes of the step kernel (2 Q s bytes per node: each of Q
distributions read and written once, s = bytes per stored value) to its
average launch time measured with HIP events on the stream the kernel runs
on.  ``cpu_baseline`` times the FP64 CPU oracle on a bounded sample of the
same workload on this host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the other storage precisions")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def timed_steps(lat, torch, steps):
    """Run `steps` steps in one lbm_step call bracketed by HIP events on the
    library's stream (torch's current stream); returns seconds."""
    stream = torch.cuda.current_stream()
    lat.set_stream(stream.cuda_stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def run_variant(W, lbm, torch, storage, steps, warmup):
    w = W.duct_les(storage=storage)
    lat = lbm.from_workload(w)
    lat.set_stream(torch.cuda.current_stream().cuda_stream)
    if warmup:
        lat.step(warmup)
    t = timed_steps(lat, torch, steps)
    bal = lat.force_balance()
    fw = lat.wall_force()
    lat.close()
    bytes_per_node = 2 * w.Q * {W.F64: 8, W.F32: 4, W.F16: 2, W.BF16: 2}[storage]
    mlups = w.N * steps / t / 1e6
    return {
        "mlups": mlups,
        "ms_per_step": t * 1e3 / steps,
        "gbs": bytes_per_node * w.N * steps / t / 1e9,
        "frac": bytes_per_node * w.N * steps / t / 1e9 / HBM_PEAK_GBS,
        "balance_residual_rel": float(np.abs(bal[9:12]).max() / max(abs(bal[3]), 1e-300)),
        "wall_drag_x": float(fw[:, 0, 0].sum()),
    }


def cpu_baseline(W, budget_s):
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import make_oracle
    w = W.duct_les()
    threads = oracle.threads(0)
    o = make_oracle(w)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    n = max(1, int(budget_s / max(t1, 1e-3)) - 1)
    t0 = time.perf_counter()
    o.step(n)
    t = time.perf_counter() - t0
    return {
        "value": w.N * n / t / 1e6,
        "unit": "MLUPS",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d steps of the full %dx%dx%d duct (FP64, LES, walls) after 1 untimed step, %.1f s"
                  % (n, w.nx, w.ny, w.nz, t),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the distributed slab decomposition is design-only); "
              "got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2512_12213_amd import lbm
    from paper_2512_12213_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    lbm.lib()

    # headline: FP32 storage
    w = W.duct_les()
    lat = lbm.from_workload(w)
    lat.set_stream(torch.cuda.current_stream().cuda_stream)
    print("bench: warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    if args.warmup:
        lat.step(args.warmup)
    torch.cuda.synchronize()
    print("bench: timing %d steps" % args.steps, file=sys.stderr, flush=True)
    t = timed_steps(lat, torch, args.steps)
    bal = lat.force_balance()
    lat.close()
    N = w.N
    mlups = N * args.steps / t / 1e6
    bytes_per_launch = 2 * w.Q * 4 * N  # 152 B per node for FP32 D3Q19
    launch_s = t / args.steps
    achieved = bytes_per_launch / launch_s / 1e9

    out = {
        "metric": "MLUPS + % HBM roofline (FP32/16-bit vs FP64 at stated err); adjoint MLUPS",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "duct_les_d3q19_256x128x128",
            "lattice": "D3Q19", "nx": w.nx, "ny": w.ny, "nz": w.nz,
            "storage": "f32", "force_model": "guo", "tau0": w.tau, "les_cs": w.les_cs,
            "a_x": w.body_force[0], "u0": "uniform +-1e-3, seed 2512",
            "streaming": "in-place A-A", "diagnostics": "wall force + balance on the last step of the call",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "kernel": "k_step<D3Q19, F32> (even/odd A-A parities alternate; average over both)",
            "bytes_per_launch": bytes_per_launch,
        },
        "balance_residual_rel": float(np.abs(bal[9:12]).max() / max(abs(bal[3]), 1e-300)),
    }
    if not args.no_variants:
        variants = {}
        for name, st in (("f16", W.F16), ("bf16", W.BF16), ("f64", W.F64)):
            print("bench: variant %s" % name, file=sys.stderr, flush=True)
            variants[name] = run_variant(W, lbm, torch, st, max(args.steps // 2, 10), min(args.warmup, 10))
        out["variants"] = variants
    if not args.no_cpu:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
