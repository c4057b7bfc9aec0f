#!/usr/bin/env python3
"""rocprofv3 passes over bench.py and their summary (run on an MI355X).

  python profile.py run WORKLOAD OUTDIR      kernel trace + counter passes
        (WORKLOAD: sweep8192, structured16384, or fill_sweep8192 for the
        hole-filling / features-only leg)
  python profile.py copy OUTDIR              FETCH_SIZE / WRITE_SIZE of a 1 GiB copy
  python profile.py summary WORKLOAD OUTDIR COPYDIR MD
        writes MD (per-kernel durations and counters, markdown) and updates
        profiles/traffic.json (measured HBM bytes per launch of every kernel,
        with the digest of the kernel sources they were taken from)

Each pass is its own rocprofv3 run (one counter set per run; no trace
domains next to counters), the program under the profiler is `python3
bench.py ...` directly after `--`, started as a child process of this
script, which itself never touches the GPU.  FETCH_SIZE and WRITE_SIZE are
scaled by what they read for a plain device-to-device copy of known size.
"""
from __future__ import annotations

import collections
import json
import os
import re
import sqlite3
import subprocess
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
KERNELS = ["k_tile_export", "k_seam_local", "k_border_merge", "k_reduce_roots", "k_leaders", "k_scan_reduce",
           "k_scan_apply", "k_border_canon", "k_tile_emit", "k_fill_top", "k_fill_scan", "k_fill_ids",
           "k_fill_merge", "k_fill_labels"]
PASSES = {
    "pmc1": ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
             "SQ_INSTS_BRANCH", "SQ_INSTS_SMEM"],
    "pmc2": ["SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU",
             "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_LDS"],
    "pmc3": ["SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_INSTS_LDS_ATOMIC", "FETCH_SIZE"],
    "pmc4": ["WRITE_SIZE", "TCC_ATOMIC_sum", "SQ_INST_LEVEL_VMEM"],
}
COPY_MIB = 1024


def _bench_cmd(workload: str):
    if workload == "fill_sweep8192":  # label, fill holes, features only: once per sweep image after a warm call
        return ["python3", os.path.join(ROOT, "bench.py"), "--fill-only"]
    return ["python3", os.path.join(ROOT, "bench.py"), "--workload", workload, "--steps", "1", "--warmup", "1",
            "--no-cpu-baseline", "--no-also"]


def _rocprof(args, out, log):
    env = dict(os.environ, TMPDIR="/tmp")
    with open(log, "w") as f:
        p = subprocess.run(["timeout", "-s", "KILL", "300", "rocprofv3", *args], cwd="/tmp", env=env, stdout=f,
                           stderr=subprocess.STDOUT)
    print(f"  {out}: exit {p.returncode}", flush=True)
    if p.returncode != 0:
        sys.exit(p.returncode)


def run(workload: str, outdir: str):
    outdir = os.path.abspath(outdir)  # the profiler runs from /tmp
    os.makedirs(outdir, exist_ok=True)
    print(f"== trace {workload}", flush=True)
    _rocprof(["--kernel-trace", "--stats", "-d", f"{outdir}/trace", "-o", "run", "--", *_bench_cmd(workload)],
             "trace", f"{outdir}/trace.log")
    for name, counters in PASSES.items():
        print(f"== {name}", flush=True)
        _rocprof(["--pmc", *counters, "-d", f"{outdir}/{name}", "-o", "run", "--", *_bench_cmd(workload)],
                 name, f"{outdir}/{name}.log")


def copy(outdir: str):
    outdir = os.path.abspath(outdir)
    os.makedirs(outdir, exist_ok=True)
    for name, c in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        print(f"== copy {c}", flush=True)
        _rocprof(["--pmc", c, "-d", f"{outdir}/{name}", "-o", "run", "--", "python3", os.path.join(ROOT, "bench.py"),
                  "--copy-calibration", str(COPY_MIB)], name, f"{outdir}/{name}.log")


def _short(name: str) -> str:
    m = re.search(r"ccl::(?:fill::)?(k_\w+)", name)
    return m.group(1) if m else name[:40]


def _db(path: str):
    for dirpath, _, files in os.walk(path):
        for f in files:
            if f.endswith("_results.db"):
                return sqlite3.connect(os.path.join(dirpath, f))
    raise FileNotFoundError(path)


def _counters(path: str):
    """kernel -> counter -> list of per-dispatch values"""
    out = collections.defaultdict(lambda: collections.defaultdict(list))
    db = _db(path)
    q = "select kernel_name, dispatch_id, counter_name, sum(value) from counters_collection group by dispatch_id, counter_name"
    for name, _, cn, val in db.execute(q):
        out[_short(name)][cn].append(float(val))
    return out


def source_digest() -> str:
    import hashlib
    hsh = hashlib.sha256()
    for f in ("ccl_pipeline.h", "ccl.hip"):
        with open(os.path.join(ROOT, "paper_2006_09299_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()[:16]


def summary(workload: str, outdir: str, copydir: str, md: str):
    db = _db(f"{outdir}/trace")
    dur = collections.defaultdict(list)
    for name, d in db.execute("select name, duration from kernels"):
        dur[_short(name)].append(d / 1e3)
    cnt = collections.defaultdict(lambda: collections.defaultdict(list))
    for p in PASSES:
        for k, cs in _counters(f"{outdir}/{p}").items():
            for c, v in cs.items():
                cnt[k][c] += v
    copy_bytes = COPY_MIB << 20
    cf = _counters(f"{copydir}/fetch")
    cw = _counters(f"{copydir}/write")
    fetch_kib = max(max(v["FETCH_SIZE"]) for v in cf.values() if "FETCH_SIZE" in v)
    write_kib = max(max(v["WRITE_SIZE"]) for v in cw.values() if "WRITE_SIZE" in v)
    f_scale = copy_bytes / (fetch_kib * 1024)
    w_scale = copy_bytes / (write_kib * 1024)

    def avg(k, c):
        v = cnt[k].get(c)
        return sum(v) / len(v) if v else float("nan")

    lines = [f"# rocprofv3 summary: {workload}", "",
             f"Kernel sources digest `{source_digest()}` (bench.py reports `traffic` only for this digest).", "",
             "Commands (from the repository root, on an MI355X):", "",
             f"    python profile.py run {workload} {outdir}",
             f"    python profile.py copy {copydir}",
             f"    python profile.py summary {workload} {outdir} {copydir} {md}", "",
             "which run, from /tmp with TMPDIR=/tmp, for the trace and for each counter pass:", "",
             f"    rocprofv3 --kernel-trace --stats -d {outdir}/trace -o run -- {' '.join(_bench_cmd(workload))}"]
    for p, cs in PASSES.items():
        lines.append(f"    rocprofv3 --pmc {' '.join(cs)} -d {outdir}/{p} -o run -- {' '.join(_bench_cmd(workload))}")
    lines += ["(OUTDIR is made absolute before the runs.)", "", f"Copy calibration ({COPY_MIB} MiB device-to-device): FETCH_SIZE reads {fetch_kib:.0f} KiB "
              f"(scale {f_scale:.3f}), WRITE_SIZE reads {write_kib:.0f} KiB (scale {w_scale:.3f}).", "",
              "Per dispatch averages (every dispatch of the profiled run: warm-up and timed steps):", "",
              "VALU issue % = VALU instructions x 4 cycles (a wave64 instruction on a 16-lane SIMD) / "
              "(1024 SIMDs x kernel duration x 2.4 GHz): how busy the vector units are on average.", "",
              "| kernel | dispatches | avg us | HBM read MB | HBM write MB | VALU/wave | SALU/wave | LDS/wave | VALU issue % | wait % | LDS bank-conflict % | LDS atomics/wave | L2 atomics/launch |",
              "|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    traffic = {}
    for k in KERNELS:
        if k not in dur and k not in cnt:
            continue
        d = dur.get(k, [float("nan")])
        waves = avg(k, "SQ_WAVES")
        rd = avg(k, "FETCH_SIZE") * 1024 * f_scale
        wr = avg(k, "WRITE_SIZE") * 1024 * w_scale
        traffic[k] = {"read_bytes": int(rd), "write_bytes": int(wr), "bytes_per_launch": int(rd + wr),
                      "avg_us": round(sum(d) / len(d), 2)}
        us = sum(d) / len(d)
        valu_util = 100 * avg(k, "SQ_INSTS_VALU") * 4 / (1024 * us * 1e-6 * 2.4e9)
        lines.append(f"| {k} | {len(d)} | {us:.1f} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | "
                     f"{avg(k, 'SQ_INSTS_VALU') / waves:.0f} | {avg(k, 'SQ_INSTS_SALU') / waves:.0f} | "
                     f"{avg(k, 'SQ_INSTS_LDS') / waves:.0f} | {valu_util:.0f} | "
                     f"{100 * avg(k, 'SQ_WAIT_ANY') / avg(k, 'SQ_WAVE_CYCLES'):.0f} | "
                     f"{100 * avg(k, 'SQ_LDS_BANK_CONFLICT') / max(avg(k, 'SQ_LDS_IDX_ACTIVE'), 1):.0f} | "
                     f"{avg(k, 'SQ_INSTS_LDS_ATOMIC') / waves:.1f} | {avg(k, 'TCC_ATOMIC_sum'):.0f} |")
    with open(md, "w") as f:
        f.write("\n".join(lines) + "\n")
    tj = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(tj) as f:
            t = json.load(f)
    except (OSError, ValueError):
        t = {}
    if t.get("source_digest") != source_digest():
        t = {"source_digest": source_digest(), "workloads": {}}
    t["workloads"][workload] = traffic
    with open(tj, "w") as f:
        json.dump(t, f, indent=1, sort_keys=True)
    print(f"wrote {md} and {tj}")


if __name__ == "__main__":
    a = sys.argv[1:]
    if a[:1] == ["run"] and len(a) == 3:
        run(a[1], a[2])
    elif a[:1] == ["copy"] and len(a) == 2:
        copy(a[1])
    elif a[:1] == ["summary"] and len(a) == 5:
        summary(a[1], a[2], a[3], a[4])
    else:
        sys.exit(__doc__)
