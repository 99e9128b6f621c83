"""Benchmark of the fused PF-LB step on one MI355X.

Workload: 3-D droplet in a Taylor-Green vortex, D3Q19 + D3Q7, 256^3 periodic,
conservative Allen-Cahn, u0 = 0.05, Re = 1000, R = 40, rho ratio 10, W = 4,
M = 0.05, We = 10; g stored as fp16 of 4096 g_i / w_i, h in fp32, fp32
arithmetic (the headline form), with the fp32 and fp64 forms timed beside it
and the mixed and fp32 errors against the fp64 run stated.

Prints ONE JSON line (see the repository's benchmark contract).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0   # MI355X HBM3E, GB/s


def bytes_per_update(d, precision):
    """Algorithmic HBM bytes of one lattice update: every stored population
    read once and written once (AC on D3Q7 stores 6 phase-field populations)."""
    d3 = d["lattice"] == "D3Q19_D3Q7"
    qg = 19 if d3 else 9
    qh = (6 if d["model"] == "AC" else 7) if d3 else 5
    sg = {"fp64": 8, "fp32": 4, "mixed_fp16": 2, "mixed_bf16": 2}[precision]
    sh = 8 if precision == "fp64" else 4
    extra = 2 * 3 * (8 if precision == "fp64" else 4) if d["model"] == "CH" else 0
    return 2 * (qg * sg + qh * sh) + extra


def time_form(d, phi, u, precision, steps, warmup, zblock=0):
    import torch
    from paper_2511_11360_amd.solver import Solver
    s = Solver(d, precision=precision, zblock=zblock)
    s.init(phi, u)
    s.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    t0 = time.perf_counter()
    s.step(steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    return s, ms / steps, wall


def rel_l2(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def cpu_baseline(seconds=12.0):
    """Oracle (plain numpy, float64) on a bounded sample of the same workload:
    the 64^3 instance of the droplet-in-vortex case, single BLAS thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import model as om
    from paper_2511_11360_amd import workloads as wl
    d, phi, u = wl.taylor_green_droplet_3d(n=64)
    with threadpool_limits(limits=1):
        p = om.Params(**d)
        st = om.init(p, phi, u)
        st = om.step(p, st)
        n = 0
        t0 = time.perf_counter()
        while True:
            st = om.step(p, st)
            n += 1
            el = time.perf_counter() - t0
            if el > seconds or n >= 200:
                break
    nodes = 64 ** 3
    return {"value": round(nodes * n / el / 1e6, 4), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": "64^3 instance of the same workload, %d steps, %.1f s, numpy float64, "
                      "1 thread" % (n, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--We", type=float, default=10.0)
    ap.add_argument("--precision", default="mixed_fp16")
    ap.add_argument("--zblock", type=int, default=0)
    ap.add_argument("--err-steps", type=int, default=500)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_11360_amd import workloads as wl

    torch.cuda.set_device(0)
    d, phi, u = wl.taylor_green_droplet_3d(n=args.n, We=args.We)
    nodes = args.n ** 3

    print("bench: headline %s %d^3, %d warmup + %d timed steps" % (args.precision, args.n, args.warmup,
                                                                  args.steps), file=sys.stderr, flush=True)
    s, ms, wall = time_form(d, phi, u, args.precision, args.steps, args.warmup, args.zblock)
    mlups = nodes / (ms * 1e-3) / 1e6
    bpu = bytes_per_update(d, args.precision)
    achieved = bpu * nodes / (ms * 1e-3) / 1e9
    del s
    torch.cuda.empty_cache()

    forms = {}
    if not args.no_forms:
        ref = None
        for prec in ("fp64", "fp32", args.precision):
            print("bench: form %s" % prec, file=sys.stderr, flush=True)
            sf, msf, _ = time_form(d, phi, u, prec, max(50, args.steps // 3), 10, args.zblock)
            b = bytes_per_update(d, prec)
            ent = {"MLUPS": round(nodes / (msf * 1e-3) / 1e6, 1),
                   "ms_per_step": round(msf, 4), "bytes_per_update": b,
                   "hbm_frac": round(b * nodes / (msf * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
            # error after err_steps steps from the same initial state, against fp64
            sf.init(phi, u)
            sf.step(args.err_steps)
            phi_f, u_f, _, _ = sf.fields()
            if prec == "fp64":
                ref = (phi_f, u_f)
            else:
                ent["rel_l2_phi_vs_fp64"] = rel_l2(phi_f, ref[0])
                ent["rel_l2_u_vs_fp64"] = rel_l2(u_f, ref[1])
                ent["err_steps"] = args.err_steps
            forms[prec] = ent
            del sf
            torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        print("bench: oracle cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline()

    out = {
        "metric": "coupled PF-LB MLUPS + % HBM roofline; mixed-prec vs FP64/FP32 at stated error",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "3-D droplet in Taylor-Green vortex, D3Q19+D3Q7, %d^3 periodic, "
                               "conservative AC, We=%g, rho ratio 10, R=40, W=4, M=0.05" % (args.n, args.We),
                   "storage": args.precision, "nodes": nodes, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "bytes_per_update": bpu},
        "cpu_baseline": cpu,
        "forms": forms,
        "wall_s_timed": round(wall, 3),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
