"""Summaries of rocprofv3 output for the step kernel.

    python -m paper_2511_11360_amd.profiling stats <dir>/<prefix>_kernel_stats.csv
    python -m paper_2511_11360_amd.profiling traffic <fetch_dir> <write_dir> <out.json> [--note TEXT]
        [--kernels k_step,k_adj]
    python -m paper_2511_11360_amd.profiling trace <dir>/<prefix>_kernel_trace.csv [--split-us T]

`trace` lists calls and average / min / max duration per kernel from a
kernel-trace CSV; with --split-us, the dispatches of each kernel shorter and
longer than T microseconds separately (one kernel launched on two box sizes).

`traffic` reads two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` kernel-trace runs of
`bench.py --copy-calibration ...`, takes the plain 1 GiB device copy of that
run as the calibration (bytes the copy truly moves divided by what each
counter reports for it) and writes the per-dispatch HBM bytes of every step
kernel, with the sha256 of the kernel source they were taken on.
"""
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in
                  ("step.h", "step_inst.hip", "kernels.hip", "lattice.h", "internal.h")]
COPY_BYTES = 1 << 30


def kernel_source_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stats(path):
    rows = list(csv.reader(open(path)))
    out = []
    for r in rows[1:]:
        out.append((r[0], int(r[1]), float(r[3]) / 1e3))
    return out


def trace(path, split_us=None):
    groups = {}
    for r in csv.DictReader(open(path)):
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        key = r["Kernel_Name"]
        if split_us is not None:
            key = (key, "< %g us" % split_us if us < split_us else ">= %g us" % split_us)
        groups.setdefault(key, []).append(us)
    out = []
    for k, v in groups.items():
        out.append((k, len(v), sum(v) / len(v), min(v), max(v)))
    return sorted(out, key=lambda t: -t[1] * t[2])


def _counter_rows(d):
    path = [os.path.join(d, f) for f in os.listdir(d) if f.endswith("counter_collection.csv")][0]
    return list(csv.DictReader(open(path)))


def traffic(fetch_dir, write_dir, kernels=("k_step",)):
    res = {}
    for tag, d in (("fetch", fetch_dir), ("write", write_dir)):
        rows = _counter_rows(d)
        copy = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]
                or "copy_kernel" in r["Kernel_Name"].lower()]
        if not copy:
            raise SystemExit("no copy kernel in %s (run bench.py with --copy-calibration)" % d)
        # the calibration copy is the run's first copy (bench.py runs it twice
        # before anything else); it reads COPY_BYTES and writes COPY_BYTES,
        # the counters report KiB
        factor = COPY_BYTES / (copy[0] * 1024.0)
        per = {}
        for r in rows:
            n = r["Kernel_Name"]
            if not any(k in n for k in kernels):
                continue
            per.setdefault(n, []).append(float(r["Counter_Value"]) * 1024.0 * factor)
        res[tag] = {"copy_factor": factor, "kernels": {k: sum(v) / len(v) for k, v in per.items()}}
    return res


def main(argv):
    if argv[0] == "stats":
        for name, calls, avg_us in stats(argv[1]):
            print("%-80s %6d %12.1f us" % (name[:80], calls, avg_us))
        return 0
    if argv[0] == "trace":
        split = float(argv[argv.index("--split-us") + 1]) if "--split-us" in argv else None
        for name, calls, avg, lo, hi in trace(argv[1], split):
            label = name if isinstance(name, str) else "%s [%s]" % name
            print("%-96s %6d %11.1f %11.1f %11.1f us" % (label[:96], calls, avg, lo, hi))
        return 0
    if argv[0] == "traffic":
        note = ""
        if "--note" in argv:
            note = argv[argv.index("--note") + 1]
        kern = argv[argv.index("--kernels") + 1].split(",") if "--kernels" in argv else ["k_step"]
        t = traffic(argv[1], argv[2], kern)
        out = {"kernel_source_sha256": kernel_source_hash(), "note": note,
               "fetch_copy_factor": t["fetch"]["copy_factor"],
               "write_copy_factor": t["write"]["copy_factor"],
               "per_dispatch_bytes": {k: {"fetch": t["fetch"]["kernels"].get(k),
                                          "write": t["write"]["kernels"].get(k)}
                                      for k in t["fetch"]["kernels"]}}
        with open(argv[3], "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
        print(json.dumps(out, indent=1, sort_keys=True))
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
