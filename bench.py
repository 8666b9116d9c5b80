#!/usr/bin/env python3
"""Benchmark of the fused LBM step on one MI355X.

Headline workload: D3Q19 square duct 256x128x128, periodic x, halfway
bounce-back walls on y and z, tau0 = 0.52 with Smagorinsky closure
(C_s = 0.1), Guo forcing a_x = 1e-5, seeded +-1e-3 initial velocity, FP32
storage and arithmetic.  A step is one call-level pass of the whole hot path:
the fused relax-propagate kernel (moments, equilibrium, force term, LES
relaxation, in-place A-A streaming with bounce-back) every step, plus the
wall-force and balance reductions of the last step of the call.

Prints ONE JSON line.  ``value`` = MLUPS of whole lbm_step calls (lattice
updates per second / 1e6, state resident in HBM, HIP events around the call
on the library's stream).  ``roofline.achieved`` = algorithmic bytes of one
step launch (2 Q s bytes per node: each of Q distributions read and written
once, s bytes per stored value) / the step kernel's mean launch duration,
measured with HIP events recorded between consecutive launches on that
stream.  ``cpu_baseline`` times the FP64 CPU reference on a bounded sample
of the same workload on this host.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES = {0: 8, 1: 4, 2: 2, 3: 2}  # storage -> bytes per value
KERNEL_SOURCES = ("paper_2512_12213_amd/csrc/kernels.hip", "paper_2512_12213_amd/csrc/kernels.hpp",
                  "paper_2512_12213_amd/csrc/device.hpp", "paper_2512_12213_amd/csrc/lattice.hpp",
                  "paper_2512_12213_amd/build.py")
TRAFFIC_RECORD = "profiles/k_step_d3q19_f32_duct_les_256x128x128.md"


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per step launch from the committed hardware-counter record,
    or None when the kernel sources changed since the counters were taken."""
    try:
        rec = {}
        with open(os.path.join(ROOT, TRAFFIC_RECORD)) as f:
            for line in f:
                k, _, v = line.strip().partition(": ")
                rec[k] = v
        if rec.get("kernel_source_sha256") != kernel_source_hash():
            return None
        return int(rec["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the other precisions and workloads")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--only", choices=["adjoint", "hartmann", "halfstep", "sphere", "formats", "stress", "history",
                                       "large"],
                    default=None,
                    help="run only this measurement (for profiling its kernels) and print its record")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run one 1 GiB device-to-device copy (a plain copy kernel of known size, "
                         "used to scale hardware byte counters)")
    return ap.parse_args()


def W_obstacle_mask(w):
    from paper_2512_12213_amd import workloads as W
    return W.obstacle_mask(w)


def copy_ceiling(torch, nbytes, repeats=20):
    """torch's device-to-device copy of nbytes / 2 bytes (nbytes moved: read +
    write), for context: it is not a tuned copy (a plain float4 copy kernel
    reaches about 6.2 TB/s on MI355X)."""
    n = nbytes // 2 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(repeats):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / repeats
    del src, dst
    return 2 * n * 4 / t / 1e9


def timed_run(lbm, torch, w, steps, warmup, storage=None, stress_every_step=False, wall_history=False):
    """Warm up, then time one lbm_step(steps) call; returns a result dict.
    stress_every_step: every step also stores the stress and strain rate of
    the state it starts from (lbm_set_step_stress, FP32, 2 x 4 x ncomp bytes
    per node more).  wall_history: every step also records its wall force
    (lbm_set_wall_force_history)."""
    lat = lbm.from_workload(w, storage=storage)
    if wall_history:
        lat.set_wall_force_history(True)
    stream = torch.cuda.current_stream()
    lat.set_stream(stream.cuda_stream)
    nc = 3 if w.D == 2 else 6
    if stress_every_step:
        sig = torch.empty((nc, w.nz, w.ny, w.nx), dtype=torch.float32, device="cuda")
        strain = torch.empty_like(sig)
        lat.set_step_stress(sig.data_ptr(), strain.data_ptr(), 1)
    if warmup:
        lat.step(warmup)
    lat.set_timing(True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3
    tim = lat.step_timings()
    if wall_history:
        assert lat.wall_force_history().shape[0] == steps
    bal = lat.force_balance()
    fw = lat.wall_force()
    lat.close()
    st = w.storage if storage is None else storage
    mask = W_obstacle_mask(w)
    nfluid = w.N if mask is None else int((mask == 0).sum())
    ind_planes = 21 if w.Q == 19 else 10  # induction directions x field components
    bpn = 2 * w.Q * BYTES[st] + (2 * ind_planes * BYTES[st] if w.mhd is not None else 0)
    if stress_every_step:
        bpn += 2 * nc * 4
    n_even = (steps - 1 + 1) // 2
    launch = (tim["even"] * n_even + tim["odd"] * (steps - 1 - n_even)) / max(steps - 1, 1)
    return {
        "mlups": w.N * steps / t / 1e6,
        "fluid_mlups": nfluid * steps / t / 1e6,
        "ms_per_step": t * 1e3 / steps,
        "launch_us": {"even": tim["even"] * 1e6, "odd": tim["odd"] * 1e6, "mean": launch * 1e6,
                      "diagnostic_last_step": tim["diag"] * 1e6, "reduce_and_copy": tim["tail"] * 1e6},
        "bytes_per_launch": bpn * w.N,
        "achieved_gbs": bpn * w.N / launch / 1e9,
        "frac": bpn * w.N / launch / 1e9 / HBM_PEAK_GBS,
        "balance_residual_rel": float(np.abs(bal[9:12]).max() / max(abs(bal[3]), 1e-300)),
        "wall_force_x_total": float(fw[:, 0, 0].sum()),
    }


def halfstep_run(lbm, torch, W, calls=5):
    """The half-step distribution of the last step (one read-only kernel over
    the state, FP64 outputs, then the device-to-host copies) on the FP32 duct
    after 20 steps: whole-call time with density, velocity and stress
    requested (the kernel's own time is in the rocprofv3 trace)."""
    w = W.duct_les()
    lat = lbm.from_workload(w)
    stream = torch.cuda.current_stream()
    lat.set_stream(stream.cuda_stream)
    lat.step(20)
    lat.halfstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        lat.halfstep()
    t = (time.perf_counter() - t0) / calls
    # the same outputs into device buffers (lbm_halfstep_device), timed
    # with events around the calls on the library's stream
    nc = 3 if w.D == 2 else 6
    dev = dict(dtype=torch.float64, device="cuda")
    bufs = [torch.empty((w.Q, w.nz, w.ny, w.nx), **dev), torch.empty((w.nz, w.ny, w.nx), **dev),
            torch.empty((w.D, w.nz, w.ny, w.nx), **dev), torch.empty((nc, w.nz, w.ny, w.nx), **dev)]
    ptrs = [b.data_ptr() for b in bufs]
    lat.halfstep_device(*ptrs)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(calls):
        lat.halfstep_device(*ptrs)
    e1.record(stream)
    torch.cuda.synchronize()
    td = e0.elapsed_time(e1) * 1e-3 / calls
    lat.close()
    nbytes = w.N * (2 * w.Q * 4 + 8 * (w.Q + 1 + w.D + nc))
    return {"call_ms": t * 1e3, "nodes": w.N,
            "outputs": "f_bar, rho_bar, u_bar, sigma_bar to host (FP64)",
            "device_call_ms": round(td * 1e3, 4), "device_bytes": nbytes,
            "device_frac": round(nbytes / td / 1e9 / HBM_PEAK_GBS, 4)}


def adjoint_run(lbm, torch, W, adj_prec, K=40, repeats=3, curved=False):
    """Differentiable duct with a sphere (128x64x64, r = 8, tau 0.55, per-node
    Guo force field, 400 steps, checkpoints every 40, FP32): recorded forward
    and full checkpointed backward (segment recompute + adjoint steps),
    timed with events around the calls; best of `repeats`.  curved: the
    sphere's links at their exact wall distance (interpolated bounce-back,
    its pass and the pass's transpose in every step)."""
    w = W.duct_sphere()
    w.curved = curved
    T = w.steps
    a0 = W.force_field(w.nx, w.ny, w.nz, base=w.body_force, amp=0.3, seed=16)
    af = torch.from_numpy(a0.astype(np.float32)).cuda()
    ga = torch.empty_like(af)
    lat = lbm.from_workload(w)
    lat.set_adjoint_precision(adj_prec)
    stream = torch.cuda.current_stream()
    lat.set_stream(stream.cuda_stream)
    lat.set_body_force_field(af.data_ptr())
    u0 = W.initial_velocity(w)
    best_f = best_b = None
    for _ in range(repeats):
        lat.init_equilibrium(u0)
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        J = lat.adjoint_forward(T, K, 4, 0)
        e1.record(stream)
        gu = lat.adjoint_backward(1.0, ga.data_ptr(), False)
        e2.record(stream)
        torch.cuda.synchronize()
        tf = e0.elapsed_time(e1) * 1e-3
        tb = e1.elapsed_time(e2) * 1e-3
        best_f = tf if best_f is None else min(best_f, tf)
        best_b = tb if best_b is None else min(best_b, tb)
    lat.close()
    lu = w.N * T
    # reverse bytes per node and step: recompute (2 Q 4 + 4 x 4 rho/U written + 12 field)
    # + adjoint (2 Q s_adj + 4 x 4 read + 12 field + 2 x 12 gradient read-modify-write)
    s_adj = 8 if adj_prec == W.F64 else 4
    rbytes = (2 * 19 * 4 + 16 + 12 if K else 0) + (2 * 19 * s_adj + 16 + 12 + 24)
    return {
        "workload": "duct_sphere_d3q19_128x64x64_r8%s_T400_%s_f32" % ("_curved" if curved else "",
                                                                       "ckpt%d" % K if K else "tape"),
        "adjoint_state": "f64" if adj_prec == W.F64 else "f32",
        "J": J,
        "dJ_duw_x": float(gu[1, 0]),
        "forward_ms": round(best_f * 1e3, 3),
        "backward_ms": round(best_b * 1e3, 3),
        "forward_mlups": round(lu / best_f / 1e6, 1),
        "adjoint_mlups": round(lu / best_b / 1e6, 1),
        "backward_bytes_per_node_step": rbytes,
        "backward_achieved_gbs": round(rbytes * lu / best_b / 1e9, 1),
    }


def cpu_baseline(W, budget_s):
    """The CPU oracle as it stands on this host: all threads on the full duct
    (about budget_s of work), one thread on a few steps of the same, and the
    oracle's reverse pass on two steps of the differentiable duct."""
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
    oracle.threads(1)
    t0 = time.perf_counter()
    o.step(2)
    t_one = time.perf_counter() - t0
    oracle.threads(threads)
    o.close()
    wa = W.duct_sphere()
    oracle.threads(threads, complex_step=True)
    a0 = W.force_field(wa.nx, wa.ny, wa.nz, base=wa.body_force, amp=0.3, seed=16)
    oa = make_oracle(wa, complex_step=True)
    oa.set_body_force_field(a0)
    t0 = time.perf_counter()
    oa.adjoint(2, 4, 0)
    t_adj = time.perf_counter() - t0
    # the other configurations: the channel in full, the Hartmann duct 20
    # steps after 2 untimed ones
    wp = W.poiseuille()
    op = make_oracle(wp)
    t0 = time.perf_counter()
    op.step(wp.steps)
    t_chan = time.perf_counter() - t0
    op.close()
    wh = W.hartmann_duct()
    oh = make_oracle(wh)
    oh.step(2)
    t0 = time.perf_counter()
    oh.step(20)
    t_mhd = time.perf_counter() - t0
    oh.close()
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": w.N * n / t / 1e6,
        "unit": "MLUPS",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model,
        "nproc": os.cpu_count(),
        "channel_64x32_f64_mlups": wp.N * wp.steps / t_chan / 1e6,
        "hartmann_duct_192x96x96_mlups": wh.N * 20 / t_mhd / 1e6,
        "sample": "%d steps of the full %dx%dx%d duct (FP64, LES, walls) after 1 untimed step, %.1f s"
                  % (n, w.nx, w.ny, w.nz, t),
        "single_thread_mlups": w.N * 2 / t_one / 1e6,
        "adjoint_mlups": wa.N * 2 / t_adj / 1e6,
        "adjoint_sample": "forward and reverse pass (complex-step node Jacobians) of 2 steps of the "
                          "128x64x64 duct with a sphere, %d threads, %.1f s" % (threads, t_adj),
    }


# Stated accuracy targets against the FP64 oracle per storage format:
# (fields rho, v, sigma, S; wall force)
TARGETS = {"f64": (1e-12, 1e-12), "f32": (1e-5, 1e-4), "f16": (2e-3, 2e-3), "bf16": (2e-3, 2e-3)}


def errors_vs_oracle(lbm, W):
    """Each storage format's error against the FP64 oracle on the duct with
    LES at 64x32x32, 300 steps (same workload recipe as the timed duct):
    density (absolute, rho0 = 1), velocity, stress and strain rate (max-norm
    relative), wall force (2-norm relative over the four walls), and whether
    each meets the stated target of its format."""
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import make_oracle
    w = W.duct_les(nx=64, ny=32, nz=32, steps=300)
    o = make_oracle(w)
    o.step(w.steps)
    ro, vo = o.get_macro()
    so, So = o.stress()
    fo = o.wall_force(4)
    o.close()

    def rel(x, ref):
        return float(np.abs(x - ref).max() / np.abs(ref).max())

    out = {"workload": "duct_les_d3q19_64x32x32, 300 steps, FP64 oracle; max-norm relative errors"}
    for st, name in ((W.F64, "f64"), (W.F32, "f32"), (W.F16, "f16"), (W.BF16, "bf16")):
        g = lbm.from_workload(w, storage=st)
        g.step(w.steps)
        rg, vg = g.get_macro()
        sg, Sg = g.stress()
        fg = g.wall_force()[:4]
        g.close()
        e = {"rho": float(np.abs(rg - ro).max()), "v": rel(vg, vo), "sigma": rel(sg, so), "S": rel(Sg, So),
             "wall_force": float(np.linalg.norm(fg[:, 0] - fo[:, 0]) / np.linalg.norm(fo[:, 0]))}
        tf, tw = TARGETS[name]
        e["meets_target"] = {k: bool(e[k] <= (tw if k == "wall_force" else tf)) for k in list(e)}
        out[name] = e
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (the decomposition over several GPUs is not implemented); "
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
    if args.calibrate:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.only == "adjoint":
        print(json.dumps({"adjoint": adjoint_run(lbm, torch, W, W.F64, repeats=1),
                          "adjoint_tape": adjoint_run(lbm, torch, W, W.F64, K=0, repeats=1),
                          "adjoint_curved": adjoint_run(lbm, torch, W, W.F64, repeats=1, curved=True)}),
              flush=True)
        return
    if args.only == "hartmann":
        rh = timed_run(lbm, torch, W.hartmann_duct(), args.steps, args.warmup)
        print(json.dumps({"hartmann_duct_f32_192x96x96": rh}), flush=True)
        return
    if args.only == "halfstep":
        print(json.dumps({"halfstep_duct_les_f32_256x128x128": halfstep_run(lbm, torch, W)}), flush=True)
        return
    if args.only == "formats":
        # the duct in the other storage formats (FP16, BF16, FP64)
        rs = {}
        for name, st in (("duct_f16", W.F16), ("duct_bf16", W.BF16), ("duct_f64", W.F64)):
            rs[name] = timed_run(lbm, torch, W.duct_les(), args.steps, args.warmup, storage=st)
        print(json.dumps(rs), flush=True)
        return
    if args.only == "stress":
        rs = {"duct_les_f32_stress_every_step": timed_run(lbm, torch, W.duct_les(), args.steps, args.warmup,
                                                           stress_every_step=True),
              "duct_les_f32": timed_run(lbm, torch, W.duct_les(), args.steps, args.warmup)}
        print(json.dumps(rs), flush=True)
        return
    if args.only == "history":
        rs = {"duct_les_f32_wall_force_every_step": timed_run(lbm, torch, W.duct_les(), args.steps, args.warmup,
                                                               wall_history=True),
              "duct_les_f32": timed_run(lbm, torch, W.duct_les(), args.steps, args.warmup)}
        print(json.dumps(rs), flush=True)
        return
    if args.only == "large":
        # the duct beyond the last-level cache, next to the headline size
        rs = {"duct_les_f32_512x256x256": timed_run(lbm, torch, W.duct_les(nx=512, ny=256, nz=256), args.steps,
                                                    args.warmup),
              "duct_les_f32": timed_run(lbm, torch, W.duct_les(), args.steps, args.warmup)}
        print(json.dumps(rs), flush=True)
        return
    if args.only == "sphere":
        # the duct with a sphere, halfway and interpolated walls
        rs = {}
        for curved in (False, True):
            ws = W.duct_sphere()
            ws.curved = curved
            rs["duct_sphere_%sf32_128x64x64" % ("curved_" if curved else "")] = timed_run(
                lbm, torch, ws, args.steps, args.warmup)
        print(json.dumps(rs), flush=True)
        return

    w = W.duct_les()
    print("bench: headline FP32 duct, warmup %d, timed %d steps" % (args.warmup, args.steps),
          file=sys.stderr, flush=True)
    r = timed_run(lbm, torch, w, args.steps, args.warmup)
    copy_gbs = copy_ceiling(torch, r["bytes_per_launch"])
    out = {
        "metric": "MLUPS + % HBM roofline (FP32/16-bit vs FP64 at stated err); adjoint MLUPS",
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 5),
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
            "streaming": "in-place A-A, row-blocked layout",
            "diagnostics": "wall force + balance on the last step of each call",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(r["achieved_gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(r["frac"], 4),
            "traffic": measured_traffic(),
            "kernel": "lbm::k_step<D3Q19, F32, no MHD, parity, no diagnostics, row-uniform>",
            "bytes_per_launch": r["bytes_per_launch"],
            "launch_us": {k: round(v, 2) for k, v in r["launch_us"].items()},
            "torch_copy_gbs": round(copy_gbs, 1),
        },
        "balance_residual_rel": r["balance_residual_rel"],
    }
    if not args.no_variants:
        variants = {}
        # at least 200 timed steps after 40 untimed ones: with fewer the GPU
        # is still raising its clocks during the timed steps of the faster
        # variants (16-bit duct: 59.2 us per launch after 10 untimed steps,
        # 56.8 us after 40, on one box)
        half = max(args.steps, 200)
        vwarm = max(args.warmup, 40)
        for name, st in (("duct_f16", W.F16), ("duct_bf16", W.BF16), ("duct_f64", W.F64)):
            print("bench: variant %s" % name, file=sys.stderr, flush=True)
            variants[name] = timed_run(lbm, torch, w, half, vwarm, storage=st)
        print("bench: variant duct storing the stress and strain rate every step", file=sys.stderr, flush=True)
        variants["duct_les_f32_stress_every_step"] = timed_run(lbm, torch, w, half, vwarm,
                                                               stress_every_step=True)
        print("bench: variant duct recording the wall force of every step", file=sys.stderr, flush=True)
        variants["duct_les_f32_wall_force_every_step"] = timed_run(lbm, torch, w, half, vwarm,
                                                                   wall_history=True)
        print("bench: variant duct without LES", file=sys.stderr, flush=True)
        wn = W.duct_les()
        wn.les_cs = 0.0
        variants["duct_no_les_f32"] = timed_run(lbm, torch, wn, half, vwarm)
        print("bench: variant large duct (beyond the last-level cache)", file=sys.stderr, flush=True)
        variants["duct_les_f32_512x256x256"] = timed_run(lbm, torch, W.duct_les(nx=512, ny=256, nz=256), 60, 5)
        print("bench: variant duct with the Stokes equilibrium and porous resistance", file=sys.stderr, flush=True)
        wsd = W.duct_les()
        wsd.stokes, wsd.darcy = True, 1e-4
        variants["duct_stokes_darcy_f32"] = timed_run(lbm, torch, wsd, half, vwarm)
        print("bench: variant hartmann duct", file=sys.stderr, flush=True)
        variants["hartmann_duct_f32_192x96x96"] = timed_run(lbm, torch, W.hartmann_duct(), half, vwarm)
        print("bench: variant hartmann duct, Lorentz-force coupling", file=sys.stderr, flush=True)
        hl = W.hartmann_duct()
        hl.lorentz = True
        variants["hartmann_duct_lorentz_f32_192x96x96"] = timed_run(lbm, torch, hl, half, vwarm)
        print("bench: variant 2D hartmann channel", file=sys.stderr, flush=True)
        variants["hartmann_channel_d2q9_f32_4096x2048"] = timed_run(
            lbm, torch, W.hartmann_channel(nx=4096, ny=2048, storage=W.F32), half, vwarm)
        for curved in (False, True):
            print("bench: variant duct with sphere, curved %d" % curved, file=sys.stderr, flush=True)
            ws = W.duct_sphere()
            ws.curved = curved
            variants["duct_sphere_%sf32_128x64x64" % ("curved_" if curved else "")] = timed_run(lbm, torch, ws, half, vwarm)
        print("bench: variant couette cylinder", file=sys.stderr, flush=True)
        variants["couette_cylinder_f32_512x128"] = timed_run(lbm, torch, W.couette_cylinder(), 2000, 100)
        print("bench: variant poiseuille", file=sys.stderr, flush=True)
        variants["poiseuille_f64_64x32"] = timed_run(lbm, torch, W.poiseuille(), 5000, 100)
        for v in variants.values():
            for k in ("mlups", "fluid_mlups", "achieved_gbs"):
                v[k] = round(v[k], 2)
            v["frac"] = round(v["frac"], 4)
            v["ms_per_step"] = float("%.5g" % v["ms_per_step"])
            v["launch_us"] = {k: round(x, 2) for k, x in v["launch_us"].items()}
        out["variants"] = variants
    if not args.no_variants:
        print("bench: adjoint (differentiable duct with sphere)", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_run(lbm, torch, W, W.F64)
        out["adjoint_f32_state"] = adjoint_run(lbm, torch, W, W.F32)
        out["adjoint_tape"] = adjoint_run(lbm, torch, W, W.F64, K=0)
        out["adjoint_curved"] = adjoint_run(lbm, torch, W, W.F64, curved=True)
    if not args.no_cpu:
        print("bench: CPU reference baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(W, args.cpu_seconds)
        print("bench: storage formats against the oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"]["errors_vs_oracle"] = errors_vs_oracle(lbm, W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
