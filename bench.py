"""Benchmark of the fused PF-LB step on one MI355X.

Workload: 3-D droplet in a Taylor-Green vortex, D3Q19 + D3Q7, 256^3 periodic,
conservative Allen-Cahn, u0 = 0.05, Re = 1000, R = 40, rho ratio 10, W = 4,
M = 0.05, We = 10. Headline form: g stored as fp16 of 4096 g_i / w_i, h in
fp32, fp32 arithmetic; the fp64, fp32 and bf16-stored forms are timed beside
it, and the per-field error of every reduced form against the fp64 form (whose
parity with the oracle the test-suite establishes) is stated, on this workload
and on a laminar one (a sheared droplet between moving walls).

Prints ONE JSON line.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_tgv256.json")


def bytes_per_update(d, precision):
    """Algorithmic HBM bytes of one lattice update: every stored population
    read once and written once (AC, the nonlocal model and Liang2018 on D3Q7
    store 6 phase-field populations; CH and Liang2018 also carry the 3
    components of (phi u); the nonlocal model reads the phase-field
    populations once more for the global sums of its multiplier; Liang2014
    also carries (phi u), its mu_phi is formed in the step kernel)."""
    d3 = d["lattice"] != "D2Q9_D2Q5"
    qg = {"D2Q9_D2Q5": 9, "D3Q19_D3Q7": 19, "D3Q27_D3Q7": 27}[d["lattice"]]
    qh = (7 if d["model"] in ("CH", "L14") else 6) if d3 else 5
    sg = {"fp64": 8, "fp32": 4, "mixed_fp16": 2, "mixed_bf16": 2}[precision]
    sh = 8 if precision == "fp64" else 4
    st = 8 if precision == "fp64" else 4
    extra = 2 * 3 * st if d["model"] in ("CH", "L18", "L14") else 0
    if d["model"] == "NL":
        extra += qh * sh
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
    return s, ev0.elapsed_time(ev1) / steps, wall


ADJ_BYTES = 2 * (19 + 7) * 8 + 26 * 8 + 2 * 6 * 8   # lambda in + out, forward g, h, workspace


def time_adjoint(steps):
    """The discrete adjoint step (float64, canonical layout) on the 128^3
    sheared droplet between moving walls, at the forward state after 20 steps,
    chaining lambda through two buffers. Algorithmic bytes per node: lambda
    read and written (2 x 26 x 8), the forward state read (26 x 8), six
    workspace values written and read (2 x 6 x 8)."""
    import torch
    from paper_2511_11360_amd import workloads as wl
    from paper_2511_11360_amd.solver import Solver
    d, phi, u, _ = wl.sheared_droplet_3d()
    s = Solver(d, precision="fp64")
    s.init(phi, u)
    s.step(20)
    fg, fh = s.get_distributions()
    gen = torch.Generator(device=fg.device).manual_seed(5)
    lam = [(torch.randn(fg.shape, dtype=torch.float64, device=fg.device, generator=gen),
            torch.randn(fh.shape, dtype=torch.float64, device=fg.device, generator=gen)),
           (torch.empty_like(fg), torch.empty_like(fh))]
    dparams = torch.zeros(3, dtype=torch.float64, device=fg.device)
    work = s.adjoint_workspace()

    def run(k, first):
        for i in range(k):
            a, b = lam[(first + i) % 2], lam[(first + i + 1) % 2]
            s.adjoint_step(fg, fh, a[0], a[1], b[0], b[1], dparams, work)
    run(4, 0)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)
    run(steps, 0)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    nodes = d["nx"] * d["ny"] * d["nz"]
    return {"workload": "3-D sheared droplet, D3Q19+D3Q7, 128^3, walls moving at -+0.02 (adjoint "
                        "of the AC step, float64)",
            "ms_per_step": round(ms, 4), "MLUPS": round(nodes / (ms * 1e-3) / 1e6, 1),
            "bytes_per_update": ADJ_BYTES,
            "hbm_frac": round(ADJ_BYTES * nodes / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}


def field_errors(d, phi, u, steps, forms):
    """Relative L2 error per field (phi, |u| vector, p) of each form against
    the fp64 form after `steps` steps from the same initial state."""
    import torch
    from paper_2511_11360_amd.solver import Solver
    out = {}
    ref = None
    for prec in ["fp64"] + list(forms):
        s = Solver(d, precision=prec)
        s.init(phi, u)
        s.step(steps)
        f = s.fields()
        if prec == "fp64":
            ref = f
        else:
            e = {}
            for name, a, b in (("phi", f[0], ref[0]), ("u", f[1], ref[1]), ("p", f[2], ref[2])):
                e[name] = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
            out[prec] = e
        del s
        torch.cuda.empty_cache()
    return out


def cpu_baseline(seconds=12.0):
    """Oracle (plain numpy, float64) on a bounded sample of the same workload:
    the 64^3 instance of the droplet-in-vortex case, single BLAS thread."""
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
            "sample": "64^3 instance of the same droplet-in-vortex workload (R scaled to 10), "
                      "%d steps in %.1f s, numpy float64, one thread" % (n, el)}


def measured_traffic(precision):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    from paper_2511_11360_amd import profiling
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != profiling.kernel_source_hash():
        return None
    code = {"fp64": 0, "fp32": 1, "mixed_fp16": 2, "mixed_bf16": 3}[precision]
    vals = [v["fetch"] + v["write"] for k, v in t["per_dispatch_bytes"].items()
            if "Pair3D, 0, %d," % code in k and v["fetch"] is not None and v["write"] is not None]
    if not vals:
        return None
    return sum(vals) / len(vals)


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
    ap.add_argument("--no-models", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2511_11360_amd import workloads as wl

    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
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
    errors = {}
    if not args.no_forms:
        for prec in ("fp64", "fp32", "mixed_fp16", "mixed_bf16"):
            print("bench: form %s" % prec, file=sys.stderr, flush=True)
            sf, msf, _ = time_form(d, phi, u, prec, max(60, args.steps // 3), 10, args.zblock)
            b = bytes_per_update(d, prec)
            forms[prec] = {"MLUPS": round(nodes / (msf * 1e-3) / 1e6, 1), "ms_per_step": round(msf, 4),
                           "bytes_per_update": b,
                           "hbm_frac": round(b * nodes / (msf * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
            del sf
            torch.cuda.empty_cache()
        for k in ("fp32", "mixed_fp16", "mixed_bf16"):
            forms[k]["speedup_vs_fp64"] = round(forms[k]["MLUPS"] / forms["fp64"]["MLUPS"], 3)
            forms[k]["speedup_vs_fp32"] = round(forms[k]["MLUPS"] / forms["fp32"]["MLUPS"], 3)
        print("bench: errors against fp64", file=sys.stderr, flush=True)
        errors["this_workload"] = {"steps": args.err_steps,
                                   "rel_l2": field_errors(d, phi, u, args.err_steps,
                                                          ("fp32", "mixed_fp16", "mixed_bf16"))}
        dl, phl, ul, _ = wl.sheared_droplet_3d(n=64, R=16.0, W=4.0)
        errors["laminar_sheared_droplet_64"] = {
            "steps": 1000, "rel_l2": field_errors(dl, phl, ul, 1000, ("fp32", "mixed_fp16", "mixed_bf16"))}

    # the other phase-field models and the D3Q27 lattice, same workload and storage form
    models = {}
    if not args.no_models:
        for key, extra in (("CH", {"model": "CH"}), ("NL_lam0", {"model": "NL", "lam": 0.0}),
                           ("NL_lam0.9", {"model": "NL", "lam": 0.9}), ("L18", {"model": "L18"}),
                           ("L14", {"model": "L14"}),
                           ("AC_D3Q27", {"lattice": "D3Q27_D3Q7"})):
            dm = dict(d, **extra)
            print("bench: model %s" % key, file=sys.stderr, flush=True)
            sm, msm, _ = time_form(dm, phi, u, args.precision, max(60, args.steps // 3), 10, args.zblock)
            b = bytes_per_update(dm, args.precision)
            models[key] = {"MLUPS": round(nodes / (msm * 1e-3) / 1e6, 1), "ms_per_step": round(msm, 4),
                           "bytes_per_update": b,
                           "hbm_frac": round(b * nodes / (msm * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
            del sm
            torch.cuda.empty_cache()

    adjoint = None
    if not args.no_adjoint:
        print("bench: adjoint", file=sys.stderr, flush=True)
        adjoint = time_adjoint(100)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        print("bench: oracle cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline()

    traffic = measured_traffic(args.precision)
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
                               "conservative AC, u0=0.05, Re=1000, R=40, rho ratio 10, W=4, M=0.05, "
                               "We=%g" % (args.n, args.We),
                   "storage": {"mixed_fp16": "g fp16 (4096 g/w), h fp32",
                               "mixed_bf16": "g bf16 (g/w), h fp32",
                               "fp32": "g, h fp32", "fp64": "g, h fp64"}[args.precision],
                   "nodes": nodes, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "traffic_unit": "bytes per launch",
                     "algorithmic_bytes_per_launch": bpu * nodes,
                     "bytes_per_update": bpu},
        "cpu_baseline": cpu,
        "forms": forms,
        "models": models,
        "adjoint": adjoint,
        "errors_vs_fp64": errors,
        "wall_s_timed": round(wall, 3),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
