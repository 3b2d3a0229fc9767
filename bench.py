#!/usr/bin/env python3
"""Throughput of the D3Q19 MRT permeability step on one MI355X.

A step is one pass of the whole hot path over the fluid nodes: pull gather
with halfway bounce-back, MRT + Guo collision, store, and the FP64
mean-velocity reduction that feeds k and the convergence test (one kernel
launch per step).  Inputs are resident in HBM before timing starts.

Default workload: the 512^3 Gaussian-random-field rock of porosity 0.20
(correlation length 6 voxels, x-spanning cluster only), tau = 1, Set E
Lambda = 3/16, g = 1e-6.  `value` is MFLUPS with FP32 deviation storage; the
FP16, BF16 and reference-density FP16 storage paths, the link-wise TRT
collision and the discrete adjoint are timed on the same image and reported
beside it.  The library replays its captured step graphs; an untimed run of
the same call pattern captures them before the timed region.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MFLUPS & %HBM peak, D3Q19-MRT 512^3 pack: fp32 vs fp16-store vs adjoint"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per fluid-lattice update: 19 populations read + 19 written.
ALG_BYTES = {"f32": 19 * 4 * 2, "f16": 19 * 2 * 2, "bf16": 19 * 2 * 2, "f16r": 20 * 2 * 2}
# Index bytes per node the design adds: the int32 [18] table; or, for the bitmap,
# one packed coordinate per node plus the 16-byte entries read once per step
# (one per 18 voxels of a row: 16 * ny * nz * words), the 16-byte count slots
# (one per row, read at the x wrap) and the 16-byte wrap slots (two per plane
# and word, read at the y wrap), all counted as read once.


def index_bytes(index: str, shape, nf: int) -> float:
    if index == "table":
        return 18 * 4
    nz, ny, nx = shape
    words = (nx + 17) // 18
    return 4 + (16 * ny * nz * words + 16 * ny * nz + 32 * nz * words) / nf
# Adjoint reverse step per node: read lambda^{n+1} and fh^{n-1}, write lambda^n
# (228 B), and update the node's running FP32 sum of dk/dg(x) (read 12 B,
# write 12 B; the first step of a checkpoint segment writes it only).
ADJ_POP_BYTES = 3 * 19 * 4
ADJ_ACC_BYTES = 2 * 3 * 4
ADJ_ALG_BYTES = ADJ_POP_BYTES + ADJ_ACC_BYTES
# The reverse sweep also recomputes the states inside each checkpoint segment:
# K - 1 forward steps per segment of K reverse steps, 152 B per node each.


def kernel_source_hash() -> str:
    """sha256[:16] of the sources that set a step's memory traffic: the
    kernels and the host code that orders the nodes."""
    h = hashlib.sha256()
    for f in ("lbm_kernels.hip", "lbm_host.cpp", "lbm_host.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1902_11193_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(workload: str, storage: str, index: str):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE/WRITE_SIZE counts,
    if they were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    e = d.get(f"{workload}/{storage}/{index}")
    if not e or e.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def time_steps(solver, steps, warmup):
    import torch

    solver.step(warmup)
    solver.mean_velocity()          # flush and sync
    # The same call pattern as the timed region, started at the same step
    # parity and buffer, so the library captures its replay graphs here and
    # not inside the timed region.
    solver.step(steps + steps % 2)
    solver.mean_velocity()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    solver.step(steps)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def run_forward(P, mask, args, storage, collision="mrt"):
    import torch

    s = P.Solver(mask, args.tau, args.Lambda, "E", (args.g, 0.0, 0.0), storage, args.index)
    s.set_collision(collision)
    ms, wall = time_steps(s, args.steps, args.warmup)
    k = float(s.permeability()[0])
    nf = s.n_fluid
    s.close()
    del s
    torch.cuda.empty_cache()
    mflups = nf / (ms * 1e-3) / 1e6
    alg_gbs = ALG_BYTES[storage] * nf / (ms * 1e-3) / 1e9
    des_gbs = (ALG_BYTES[storage] + index_bytes(args.index, mask.shape, nf)) * nf / (ms * 1e-3) / 1e9
    voxel_mlups = mask.size / (ms * 1e-3) / 1e6   # per voxel of the image, as dense codes count
    return dict(ms_per_step=ms, MFLUPS=mflups, MLUPS_per_voxel=voxel_mlups, GBps_algorithmic=alg_gbs,
                GBps_designed=des_gbs,
                frac_hbm_algorithmic=alg_gbs / HBM_PEAK_GBS, k_after_timed=k,
                steps_total=args.warmup + args.steps + args.steps % 2 + args.steps, wall_s=wall)


def run_adjoint(P, mask, args, N=None, K=None, g=None, label="grf_512"):
    """The discrete adjoint: whole-job node-steps per second, and from the
    library's event timing of its phases the reverse step's HBM roofline
    (252 algorithmic bytes per node, 240 on the first step of a segment; the
    fraction over the 228 population bytes alone beside it) and that of the
    reverse sweep with its recompute (a 152-byte forward step per node for all
    but one of a segment's reverse steps)."""
    import torch

    N = N or args.adj_steps
    K = K or args.adj_checkpoint
    g = args.g if g is None else g
    s = P.Solver(mask, args.tau, args.Lambda, "E", (g, 0.0, 0.0), "f32", args.index)
    s.adjoint(min(N, 2 * K), K)        # untimed: first-launch costs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = s.adjoint(N, K)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ph = s.adjoint_timing()
    nf = s.n_fluid
    out = dict(workload=label, n_fluid=nf, n_steps=N, checkpoint_every=K, seconds=t,
               node_steps_per_s=nf * N / t, MFLUPS_equivalent=nf * N / t / 1e6,
               k=r["k"], dk_dtau=r["dk_dtau"], dk_dLambda=r["dk_dLambda"], **ph)
    s.close()
    del s, r
    torch.cuda.empty_cache()
    nrev = N - 1
    if nrev > 0 and ph["reverse_ms"] > 0:
        rev_s = ph["reverse_ms"] * 1e-3 / nrev
        segments = -(-nrev // K)
        per_node = ADJ_ALG_BYTES - (ADJ_ACC_BYTES / 2) * segments / nrev   # mean over the launches
        ach = per_node * nf / rev_s / 1e9
        out["reverse_step_us"] = rev_s * 1e6
        out["roofline"] = dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                               traffic=traffic_for(label, "adjoint", args.index),
                               kernel="k_adjoint<BitmapIdx, false>",
                               algorithmic_bytes_per_launch=per_node * nf,
                               frac_population_bytes=ADJ_POP_BYTES * nf / rev_s / 1e9 / HBM_PEAK_GBS)
        both = (ph["reverse_ms"] + ph["recompute_ms"]) * 1e-3
        sweep = per_node * nrev + 2 * 19 * 4 * (nrev - segments)   # bytes per node: reverse steps + recompute steps
        ach2 = sweep * nf / both / 1e9
        out["roofline_with_recompute"] = dict(bound="hbm", achieved=ach2, peak=HBM_PEAK_GBS, unit="GB/s",
                                              frac=ach2 / HBM_PEAK_GBS, bytes_per_node_step=sweep / nrev)
    return out


def run_steady(P, mask, args, storage):
    """Run to the paper's steady-state criterion (per-step relative change of
    k below eps) in segments, printing progress; reports steps, k and rate."""
    import torch

    s = P.Solver(mask, args.tau, args.Lambda, "E", (args.g, 0.0, 0.0), storage, args.index)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, conv, k = 0, False, float("nan")
    trajectory = []
    while done < args.max_steps and not conv:
        r = s.run_to_steady(eps=args.eps, check_every=100, max_steps=min(2000, args.max_steps - done))
        done += r["steps"]
        conv, k = r["converged"], float(r["k"][0])
        trajectory.append((done, k))
        print(f"[bench] steady {storage}: {done} steps, k = {k:.9g}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    # The per-step test can also be met where k turns (an acoustic overshoot);
    # stepping on shows how far k still moves after the criterion first holds.
    s.step(args.steady_extra)
    k_extra = float(s.permeability()[0])
    print(f"[bench] steady {storage}: +{args.steady_extra} steps, k = {k_extra:.9g}", file=sys.stderr, flush=True)
    nf = s.n_fluid
    s.close()
    del s
    torch.cuda.empty_cache()
    return dict(storage=storage, steps=done, converged=conv, k=k, seconds=t, MFLUPS=nf * done / t / 1e6,
                eps=args.eps, trajectory=trajectory, extra_steps=args.steady_extra, k_after_extra=k_extra,
                k_drift_after_extra=k_extra / k - 1)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(mask_full, crop_n: int, steps: int):
    import torch

    import oracle as O
    from lbm_inputs import crop

    m = crop(mask_full, crop_n)
    p = O.Problem(m, 1.0, 3 / 16, "E", (1e-6, 0.0, 0.0))
    t = O.time_steps(p, steps)
    return dict(value=p.nf * steps / t / 1e6, unit="MFLUPS", cores=torch.get_num_threads(), kind="oracle",
                host_cpus=os.cpu_count(), cpu_model=cpu_model(),
                sample=f"{steps} steps of the FP64 oracle on the {crop_n}^3 corner crop of the workload "
                       f"({p.nf} fluid nodes), {t:.1f} s, on {torch.get_num_threads()} threads")


def cpu_configs(steps: int):
    """The FP64 oracle on each parity case (32^3 sphere array in full, 64^3
    crop of the 256^3 pack, 128^3 crop of the 512^3 rock, 32^3 crop of the
    128^3 pack), single-threaded and with all host threads."""
    import torch

    import oracle as O
    from lbm_inputs import crop, workload

    cases = [("sc_sphere_32", lambda: workload("sc_sphere_32")),
             ("pack_256 crop 64", lambda: crop(workload("pack_256"), 64)),
             ("grf_512 crop 128", lambda: crop(workload("grf_512"), 128)),
             ("pack_128 crop 32", lambda: crop(workload("pack_128"), 32))]
    nthreads = torch.get_num_threads()
    out = []
    for name, make in cases:
        m = make()
        p = O.Problem(m, 1.0, 3 / 16, "E", (1e-6, 0.0, 0.0))
        row = dict(case=name, n_fluid=p.nf, steps=steps)
        for th in (1, nthreads):
            torch.set_num_threads(th)
            t = O.time_steps(p, steps)
            row[f"MFLUPS_{th}_threads"] = p.nf * steps / t / 1e6
        torch.set_num_threads(nthreads)
        print(f"[bench] oracle {name}: {row}", file=sys.stderr, flush=True)
        out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="grf_512")
    ap.add_argument("--index", default="bitmap", choices=["bitmap", "table"])
    ap.add_argument("--variants", default="f16,bf16,f16r,trt,f16_trt,adjoint,adjoint_c4")
    ap.add_argument("--tau", type=float, default=1.0)
    ap.add_argument("--Lambda", type=float, default=3 / 16)
    ap.add_argument("--g", type=float, default=None)
    ap.add_argument("--adj-steps", type=int, default=400)
    ap.add_argument("--adj-checkpoint", type=int, default=20)
    ap.add_argument("--cpu-crop", type=int, default=128)
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-configs", type=int, default=0, metavar="STEPS",
                    help="also time the oracle on every parity case for STEPS steps (1 thread and all)")
    ap.add_argument("--steady", action="store_true",
                    help="also run FP32 and FP16 storage to steady state and compare k")
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--max-steps", type=int, default=30000)
    ap.add_argument("--steady-extra", type=int, default=3000)
    ap.add_argument("--steady-storages", default="f32,f16,f16r")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (a kernel of known traffic for counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path "
              "(the domain would split into x-slabs with halo exchange; not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1902_11193_amd as P
    from lbm_inputs import WORKLOADS, workload, porosity

    w = WORKLOADS[args.workload]
    if args.g is None:
        args.g = w["g"]
    t0 = time.time()
    mask = workload(args.workload, verbose=True)
    gen_s = time.time() - t0
    print(f"[bench] {args.workload}: generated in {gen_s:.1f}s, porosity {porosity(mask):.4f}", file=sys.stderr,
          flush=True)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()

    main_r = run_forward(P, mask, args, "f32")
    print(f"[bench] f32 {main_r['MFLUPS']:.0f} MFLUPS {main_r['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    variants = {}
    for v in [x for x in args.variants.split(",") if x]:
        if v in ("f16", "bf16", "f16r"):
            variants[f"{v}_store"] = run_forward(P, mask, args, v)
            variants[f"{v}_store"]["k_rel_vs_f32"] = variants[f"{v}_store"]["k_after_timed"] / main_r["k_after_timed"] - 1
        elif v in ("trt", "f16_trt"):
            st = "f16" if v == "f16_trt" else "f32"
            variants[f"{v}_collision"] = run_forward(P, mask, args, st, "trt")
            base = main_r if st == "f32" else variants.get("f16_store")
            if base:
                variants[f"{v}_collision"]["k_rel_vs_mrt"] = variants[f"{v}_collision"]["k_after_timed"] / base["k_after_timed"] - 1
        elif v == "adjoint":
            variants["adjoint"] = run_adjoint(P, mask, args)
        elif v == "adjoint_c4":
            # the 128^3 sphere pack, 4000 steps, checkpoint every 200
            variants["adjoint_c4"] = run_adjoint(P, workload("pack_128"), args, N=4000, K=200, g=1e-6,
                                                 label="pack_128")
        print(f"[bench] {v} done", file=sys.stderr, flush=True)

    steady = None
    if args.steady:
        steady = {st: run_steady(P, mask, args, st) for st in args.steady_storages.split(",")}
        for st in [x for x in steady if x != "f32"]:
            if "f32" in steady:
                steady[f"k_rel_{st}_vs_f32"] = steady[st]["k"] / steady["f32"]["k"] - 1
                steady[f"k_rel_{st}_vs_f32_after_extra"] = (steady[st]["k_after_extra"] /
                                                           steady["f32"]["k_after_extra"] - 1)

    nf = int((mask == 0).sum())
    alg_per_launch = ALG_BYTES["f32"] * nf
    achieved = alg_per_launch / (main_r["ms_per_step"] * 1e-3) / 1e9
    traffic = traffic_for(args.workload, "f32", args.index)
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=traffic, kernel="k_step<CodecF32, BitmapIdx>" if args.index == "bitmap"
                    else "k_step<CodecF32, TableIdx>", algorithmic_bytes_per_launch=alg_per_launch)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(mask, args.cpu_crop, args.cpu_steps)
    out = {
        "metric": METRIC,
        "value": main_r["MFLUPS"],
        "unit": "MFLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": w["n"], "porosity": porosity(mask), "n_fluid": nf,
                   "tau": args.tau, "Lambda": args.Lambda, "relaxation_set": "E", "g": args.g,
                   "storage": "f32", "index": args.index, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "f32": main_r,
        "variants": variants,
    }
    if steady is not None:
        out["steady"] = steady
    if args.cpu_configs:
        out["cpu_configs"] = cpu_configs(args.cpu_configs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
