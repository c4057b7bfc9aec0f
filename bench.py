#!/usr/bin/env python3
"""Throughput of the B&W labeling + features + tree + Euler path on one MI355X.

One step = one pass of the whole path over the workload, inputs resident in
HBM before the timed region:
  structured16384  three 16384 x 16384 images of nested disks + 5% salt
                   (seeds 0, 1, 2; default: the single-image size the HBM
                   target is stated on)
  sweep8192        25 images 8192 x 8192, Bernoulli(p) on g x g blocks,
                   p in {.1,.3,.5,.7,.9} x g in {1,2,4,8,16}
Prints one JSON line (stdout); progress goes to stderr.

`value` and `ms_per_step` time the steps as a user runs them (plain
ccl_label calls back to back on one stream, events around the whole step
loop).  Per-kernel durations come from a second, equally long pass over the
same images with HIP events recorded around every kernel (ccl_label_traced,
on the stream the kernels run on); the events add a few microseconds between
kernels, so that pass's total is reported apart (`traced_ms_per_image`).  Algorithmic bytes per image (what the method must move):
B = w*h*(1 + 4) + 45 * n_labels + 16 (read the image, write the label image
and one 45-byte row of the feature / parent / colour tables per label).
`roofline` is the dominant kernel (largest average duration): B per image
(one image per launch) / its average duration, against 8 TB/s; beside it,
`kernel_own` credits the kernel only with the bytes it moves itself
(k_tile_export reads the image, k_tile_emit writes the rest).  `path_hbm` is
B over the whole path's time per image.  `traffic` is the kernel's measured
HBM bytes per launch from the committed rocprofv3 counter summary
(profiles/traffic.json, FETCH_SIZE and WRITE_SIZE scaled by a plain copy's
readings) when that summary was taken from the current kernel sources, else
null.  `hbm_copy_ceiling` is the best rate of a plain 1 GiB device-to-device
copy on the same GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(w: int, h: int, n_labels: int) -> int:
    return w * h * 5 + 45 * n_labels + 16


def kernel_algorithmic_bytes(name: str, w: int, h: int, n_labels: int) -> int:
    if name == "k_tile_export":
        return w * h
    if name == "k_tile_emit":
        return w * h * 4 + 45 * n_labels + 16
    return 0


def source_digest() -> str:
    """Digest of the kernel sources (the counter summary is valid for these only)."""
    import hashlib
    hsh = hashlib.sha256()
    for f in ("ccl_pipeline.h", "ccl.hip"):
        with open(os.path.join(ROOT, "paper_2006_09299_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from profiles/traffic.json, or None."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_digest") != source_digest():
        return None
    k = t.get("workloads", {}).get(workload, {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


class HipEvents:
    """hipEvent_t handles through the HIP runtime torch already loaded."""

    def __init__(self):
        self.rt = ctypes.CDLL("libamdhip64.so")
        self.rt.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.rt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.rt.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self, n):
        arr = (ctypes.c_void_p * n)()
        for i in range(n):
            ev = ctypes.c_void_p()
            rc = self.rt.hipEventCreate(ctypes.byref(ev))
            if rc != 0:
                raise RuntimeError(f"hipEventCreate failed ({rc})")
            arr[i] = ev.value
        return arr

    def ms(self, a, b) -> float:
        f = ctypes.c_float()
        rc = self.rt.hipEventElapsedTime(ctypes.byref(f), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(f.value)

    def destroy(self, arr):
        for ev in arr:
            self.rt.hipEventDestroy(ev)


def make_workload(name: str):
    import synth
    if name == "sweep8192":
        imgs = []
        for p, g, seed, img in synth.sweep_8192():
            imgs.append(((p, g, seed), img))
            say(f"  generated 8192^2 p={p} g={g} seed={seed}")
        return imgs
    if name == "structured16384":
        imgs = []
        for seed in STRUCTURED_SEEDS:
            imgs.append((("structured", seed), synth.structured(16384, 16384, seed=seed)))
            say(f"  generated 16384^2 structured seed={seed}")
        return imgs
    raise SystemExit(f"unknown workload {name}")


STRUCTURED_SEEDS = (0, 1, 2)
WORKLOAD_TEXT = {
    "structured16384": "16384x16384 uint8 nested disks/annuli (radii 4..2000 px, depth 1..8) + 5% salt, "
                       "seeds 0-2, one image per launch",
    "sweep8192": "8192x8192 uint8 Bernoulli(p) on g x g blocks, p in {.1,.3,.5,.7,.9} x g in {1,2,4,8,16}, "
                 "one image per launch",
}


def host_cpu():
    """Model name and usable cores of the host that runs the oracle."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "usable_cores": usable, "logical_cpus": os.cpu_count()}


def _variant_config(shape):
    """The compiled variant a single-image call takes for this shape."""
    from paper_2006_09299_amd import _capi
    h, w = shape
    v = _capi.variant_for(w, h)
    th, tw, _, threads, sup, _ = _capi.variant_info(v)
    return {"variant": v, "tile": [th, tw], "threads": threads, "super_tile": sup}


def run_gpu(work, steps: int, warmup: int):
    import torch
    import paper_2006_09299_amd as ccl
    from paper_2006_09299_amd import _capi

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    gpu_imgs = [torch.from_numpy(img).to(dev) for _, img in work]
    torch.cuda.synchronize()
    h, w = work[0][1].shape
    # table capacity: true label counts from one untimed pass
    probe = ccl.Buffers(w, h, w * h // 4 + 1024, dev)
    counts = []
    for t in gpu_imgs:
        ccl.launch(t, probe)
        torch.cuda.synchronize()
        counts.append(int(probe.counts[0].item()))
    del probe
    buf = ccl.Buffers(w, h, max(counts) + 16, dev)
    lib = _capi.lib()
    pitch = w
    say(f"  labels per image: min {min(counts)} max {max(counts)}")

    def call(t, events=None):
        if events is None:
            rc = lib.ccl_label(t.data_ptr(), w, h, pitch, ctypes.byref(buf.out), buf.ws.data_ptr(), buf.ws_bytes,
                               ctypes.c_void_p(stream.cuda_stream))
        else:
            rc = lib.ccl_label_traced(t.data_ptr(), w, h, pitch, ctypes.byref(buf.out), buf.ws.data_ptr(),
                                      buf.ws_bytes, ctypes.c_void_p(stream.cuda_stream), events)
        _capi.check(rc, "ccl_label")

    for _ in range(warmup):
        for t in gpu_imgs:
            call(t)
    torch.cuda.synchronize()

    # the step as a user runs it: plain calls, one after another on the stream
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for s in range(steps):
        for t in gpu_imgs:
            call(t)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(stop)
    # the same steps again with a HIP event before every kernel (per-kernel
    # durations; the events add a few microseconds between kernels, so this
    # pass is timed on its own)
    hip = HipEvents()
    ev = [[hip.create(_capi.TRACE_EVENTS) for _ in gpu_imgs] for _ in range(steps)]
    start.record(stream)
    for s in range(steps):
        for i, t in enumerate(gpu_imgs):
            call(t, ev[s][i])
    stop.record(stream)
    torch.cuda.synchronize()
    traced_ms = start.elapsed_time(stop)

    names = _capi.kernel_names()
    per_kernel = {n: 0.0 for n in names}
    for s in range(steps):
        for i in range(len(gpu_imgs)):
            e = ev[s][i]
            for k, n in enumerate(names):
                d = hip.ms(e[k], e[k + 1])
                per_kernel[n] += d
    for row in ev:
        for e in row:
            hip.destroy(e)
    launches = steps * len(gpu_imgs)
    avg = {n: v / launches for n, v in per_kernel.items()}
    alg = sum(algorithmic_bytes(w, h, c) for c in counts)
    kalg = {n: sum(kernel_algorithmic_bytes(n, w, h, c) for c in counts) / len(gpu_imgs) for n in names}
    return dict(total_ms=total_ms, traced_ms=traced_ms, wall_s=wall, steps=steps, pixels_per_step=w * h * len(gpu_imgs),
                alg_bytes_per_step=alg, kernel_avg_ms=avg, kernel_alg_bytes=kalg, counts=counts)


def roofline(r, workload: str):
    """Roofline entry of the dominant kernel of a run_gpu result: the path's
    algorithmic bytes per image (one image per launch) over the kernel's
    average duration; `kernel_own` counts only the bytes the kernel itself
    moves."""
    k = max(r["kernel_avg_ms"], key=r["kernel_avg_ms"].get)
    ms = r["kernel_avg_ms"][k]
    b_launch = r["alg_bytes_per_step"] / len(r["counts"])
    gbs = b_launch / (ms / 1e3) / 1e9
    own = r["kernel_alg_bytes"][k] / (ms / 1e3) / 1e9
    traffic = measured_traffic(workload, k)
    out = {"bound": "hbm", "kernel": k, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
           "alg_bytes_per_launch": int(b_launch), "avg_ms": round(ms, 5),
           "kernel_own": {"alg_bytes_per_launch": int(r["kernel_alg_bytes"][k]), "GBs": round(own, 1),
                          "frac": round(own / HBM_PEAK_GBS, 4)}}
    if traffic is not None:  # measured HBM bytes over the same duration
        out["traffic_frac"] = round(traffic / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def summarize(r, workload: str):
    ms = r["total_ms"] / r["steps"] / len(r["counts"])
    px = r["pixels_per_step"] / len(r["counts"])
    b = r["alg_bytes_per_step"] / len(r["counts"])
    return {"Gpixel_s": round(px / (ms / 1e3) / 1e9, 3), "ms_per_image": round(ms, 4),
            "path_hbm": {"alg_GBs": round(b / (ms / 1e3) / 1e9, 1), "frac": round(b / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
            "traced_ms_per_image": round(r["traced_ms"] / r["steps"] / len(r["counts"]), 4),
            "roofline": roofline(r, workload), "launches_per_image": len(r["kernel_avg_ms"]),
            "kernel_avg_ms": {k: round(v, 5) for k, v in r["kernel_avg_ms"].items()}}


def cold_warm(work, reps: int = 1):
    """Whole-path time per image with the caches cold (1 GiB written between
    images, so neither L2 nor the 256 MB Infinity Cache holds the image or
    the workspace) and warm (the same image again right after)."""
    import torch
    import paper_2006_09299_amd as ccl
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    h, w = work[0][1].shape
    buf = ccl.Buffers(w, h, w * h // 4 + 1024, dev)
    flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    cold, warm = [], []
    for _, img in work:
        t = torch.from_numpy(img).to(dev)
        ccl.launch(t, buf)  # module load, first touch of the buffers
        for _ in range(reps):
            flush.fill_(1)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record(stream)
            ccl.launch(t, buf)
            e[1].record(stream)
            e[2].record(stream)
            ccl.launch(t, buf)
            e[3].record(stream)
            torch.cuda.synchronize()
            cold.append(e[0].elapsed_time(e[1]))
            warm.append(e[2].elapsed_time(e[3]))
        del t
    del flush, buf
    cold.sort()
    warm.sort()
    med = lambda v: v[len(v) // 2]
    gps = lambda ms: round(w * h / (ms / 1e3) / 1e9, 2)
    return {"images": len(work), "flush_bytes": 1 << 30,
            "cold": {"median_ms": round(med(cold), 4), "Gpixel_s_median": gps(med(cold)),
                     "Gpixel_s_total": round(w * h * len(cold) / (sum(cold) / 1e3) / 1e9, 2)},
            "warm": {"median_ms": round(med(warm), 4), "Gpixel_s_median": gps(med(warm)),
                     "Gpixel_s_total": round(w * h * len(warm) / (sum(warm) / 1e3) / 1e9, 2)}}


def run_c1(reps: int = 400):
    """512 x 512, p = 0.5, seed 0: one image per launch sequence, eager and
    replayed from a captured HIP graph."""
    import torch
    import synth
    import paper_2006_09299_amd as ccl
    dev = torch.device("cuda:0")
    img = synth.bernoulli_blocks(512, 512, 0.5, 1, 0)
    t = torch.from_numpy(img).to(dev)
    buf = ccl.Buffers(512, 512, 512 * 512 // 4 + 1024, dev)
    for _ in range(5):
        ccl.launch(t, buf)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        ccl.launch(t, buf)
    b.record()
    torch.cuda.synchronize()
    eager_ms = a.elapsed_time(b) / reps
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ccl.launch(t, buf)
    torch.cuda.synchronize()
    for _ in range(5):
        g.replay()
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    graph_ms = a.elapsed_time(b) / reps
    n = int(buf.counts[0].item())
    px = 512 * 512
    return {"shape": [512, 512], "p": 0.5, "seed": 0, "n_labels": n,
            "eager_us_per_image": round(eager_ms * 1e3, 2), "eager_Gpixel_s": round(px / (eager_ms / 1e3) / 1e9, 2),
            "graph_us_per_image": round(graph_ms * 1e3, 2), "graph_Gpixel_s": round(px / (graph_ms / 1e3) / 1e9, 2),
            "path_hbm_frac_graph": round(algorithmic_bytes(512, 512, n) / (graph_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def copy_ceiling(mib: int = 1024, reps: int = 5):
    """Best device-to-device copy rate (read + write bytes / time) on this GPU."""
    import torch
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    best = float("inf")
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    gbs = 2 * n / (best / 1e3) / 1e9
    return {"GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes_copied": n}


def run_batch(n_images: int, steps: int, warmup: int, host_out=None):
    """The uneven batch: one captured launch sequence per step (graph
    replay), autotuned variant; then the same images one launch per image.
    host_out (a list), if given, receives the host images."""
    import numpy as np
    import torch
    import synth
    import paper_2006_09299_amd as ccl
    from paper_2006_09299_amd import tune

    dev = torch.device("cuda:0")
    specs = synth.batch_specs(n_images)
    imgs = []
    for i, sp in enumerate(specs):
        im = sp.make()
        if host_out is not None:
            host_out.append(im)
        imgs.append(torch.from_numpy(im).to(dev))
        if (i + 1) % 1024 == 0:
            say(f"  generated {i + 1}/{n_images} batch images")
    px = sum(sp.pixels for sp in specs)
    sample = imgs[:: max(1, n_images // 256)]
    variant = tune.autotune(sample)
    say(f"  autotuned variant {variant} {ccl.variant_info(variant)} on {len(sample)} sampled images")
    # capacities from one pass
    rs = ccl.label_batch(imgs, variant=variant)
    caps = [r.n_labels + 16 for r in rs]
    del rs
    plan = ccl.BatchPlan(imgs, variant=variant, caps=caps)
    plan.capture()
    for _ in range(warmup):
        plan.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lat = []
    a.record()
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.replay()
        e1.record()
        lat.append((e0, e1))
    b.record()
    torch.cuda.synchronize()
    batch_ms = a.elapsed_time(b) / steps
    lat_ms = sorted(x.elapsed_time(y) for x, y in lat)
    # one launch per image (same variant, preallocated buffers per image)
    bufs = [ccl.Buffers(int(t.shape[1]), int(t.shape[0]), c, dev, variant=variant) for t, c in zip(imgs, caps)]
    for t, bf in zip(imgs, bufs):
        ccl.launch(t, bf)
    torch.cuda.synchronize()
    a.record()
    for _ in range(steps):
        for t, bf in zip(imgs, bufs):
            ccl.launch(t, bf)
    b.record()
    torch.cuda.synchronize()
    loop_ms = a.elapsed_time(b) / steps
    out = {"images": n_images, "Gpixel": round(px / 1e9, 4), "variant": variant,
           "tile": list(ccl.variant_info(variant)[:2]), "hash_reduce": ccl.variant_info(variant)[2],
           "threads": ccl.variant_info(variant)[3], "super_tile": ccl.variant_info(variant)[4],
           "reduce_group": ccl.variant_info(variant)[5],
           "graph_ms_per_batch": round(batch_ms, 3), "Gpixel_s": round(px / (batch_ms / 1e3) / 1e9, 2),
           "batch_latency_ms_p50": round(lat_ms[len(lat_ms) // 2], 3),
           "batch_latency_ms_p99": round(lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))], 3),
           "batch_latency_ms_max": round(lat_ms[-1], 3),
           "per_image_loop_ms": round(loop_ms, 3),
           "per_image_loop_Gpixel_s": round(px / (loop_ms / 1e3) / 1e9, 2),
           "speedup_vs_loop": round(loop_ms / batch_ms, 2)}
    say(f"  batch: {json.dumps(out)}")
    return out


SERVE_POOL = 512  # distinct request images (contiguous, pinned)


def serve_sources(n_stream: int, n_pool: int = SERVE_POOL):
    """Pinned host images for the serving stream: the stream's requests
    (sides log-uniform in [256, 8192], p ~ U(0.1, 0.9), g in {1, 4}) ranked
    by area, and n_pool of them at evenly spaced area quantiles generated at
    their own size and parameters with contiguous rows (one plain copy
    uploads each).  Returns (areas, images), both in increasing area."""
    import numpy as np
    import torch
    import synth
    specs = [rq.spec for rq in synth.serve_stream(n_stream)]
    order = sorted(range(len(specs)), key=lambda k: specs[k].w * specs[k].h)
    pick = [order[round(k * (len(order) - 1) / (n_pool - 1))] for k in range(n_pool)]
    pool = []
    for k, j in enumerate(pick):
        pool.append(torch.from_numpy(specs[j].make()).pin_memory())
        if (k + 1) % 64 == 0:
            say(f"  serve pool: {k + 1}/{n_pool} images")
    areas = np.array([t.numel() for t in pool])
    say(f"  serve pool: mean {areas.mean() / 1e6:.2f} Mpx per image; stream mean "
        f"{np.mean([s.w * s.h for s in specs]) / 1e6:.2f} Mpx")
    return areas, pool


def run_serve(n_requests: int, sources, rate_hz: float = 2000.0, warmup_s: float = 1.0, budget_gib: int = 48,
              batched: bool = True):
    """Open-loop Poisson request stream through the serving loop: arrivals as
    the stream draws them; every request carries the pool image nearest its
    own drawn area (the pool holds the stream's area quantiles).
    Latency = completion observed - scheduled arrival."""
    import numpy as np
    import synth
    from paper_2006_09299_amd.serve import Server

    areas, pool = sources
    warm = int(warmup_s * rate_hz)
    stream = synth.serve_stream(n_requests + warm, rate_hz=rate_hz)
    host = []
    for rq in stream:
        a = rq.spec.w * rq.spec.h
        k = int(np.searchsorted(areas, a))
        if k == len(areas) or (k > 0 and a - areas[k - 1] < areas[k] - a):
            k -= 1
        host.append(pool[k])
    say(f"  serve: {len(host)} requests at {rate_hz:.0f}/s, mean {np.mean([t.numel() for t in host]) / 1e6:.2f} Mpx "
        f"(drawn: {np.mean([rq.spec.w * rq.spec.h for rq in stream]) / 1e6:.2f})")
    srv = Server(budget_gib << 30, max_slots=512 if batched else 1, streams=4 if batched else 1,
                 max_batch=64 if batched else 1)
    lat, px_done, t_first, t_last, qmax = [], 0, None, None, 0
    i = 0
    start = srv.now()
    next_note = 2.0
    while i < len(stream) or not srv.idle():
        now = srv.now() - start
        while i < len(stream) and stream[i].arrival_s <= now:
            srv.submit(i, host[i], arrival=start + stream[i].arrival_s)
            i += 1
        for r in srv.step():
            if r.rid >= warm:
                lat.append(r.done - r.arrival)
                px_done += r.img.numel()
                t_first = r.arrival if t_first is None else min(t_first, r.arrival)
                t_last = r.done if t_last is None else max(t_last, r.done)
            srv.release(r.rid)
        qmax = max(qmax, srv.queued())
        if now >= next_note:
            say(f"  serve: {now:.0f} s, {i} submitted, {len(lat)} measured done, queue {srv.queued()}")
            next_note += 2.0
    st = srv.stats()
    srv.close()
    lat.sort()
    q = lambda f: round(1e3 * lat[min(len(lat) - 1, int(f * len(lat)))], 3)
    span = t_last - t_first
    return {"requests": len(lat), "rate_hz": rate_hz, "distinct_images": len(pool),
            "mean_Mpx": round(px_done / len(lat) / 1e6, 3),
            "offered_Gpixel_s": round(px_done / (len(lat) / rate_hz) / 1e9, 2),
            "Gpixel_s": round(px_done / span / 1e9, 2), "p50_ms": q(0.50), "p99_ms": q(0.99), "max_ms": round(1e3 * lat[-1], 3),
            "max_queue": qmax, "rejected": srv.rejected, "streams": srv.streams, "max_batch": srv.max_batch,
            "micro_batches": st.launches, "relaunched": st.relaunched}


def run_widened(work, reps: int = 3):
    """Widened rows of the path, on the same images: hole filling after a
    labeling (ccl_fill_holes, filled label image and tables), the
    features-only mode (ccl_label with no label image) and the complementary
    connectivity pair (ccl_label_conn, 4-adjacent foreground).  Per image: label
    once, then `reps` timed calls (events on the stream the kernels run on)."""
    import torch
    import paper_2006_09299_amd as ccl
    from paper_2006_09299_amd import _capi

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    lib = _capi.lib()
    h, w = work[0][1].shape
    buf = ccl.Buffers(w, h, w * h // 4 + 1024, dev)
    fo = ccl.Buffers(w, h, w * h // 4 + 1024, dev, labels=False)
    c4 = ccl.Buffers(w, h, w * h // 4 + 1024, dev, variant=0)
    olab = torch.empty((h, w), dtype=torch.int32, device=dev)
    ofeat = torch.empty((buf.cap, 5), dtype=torch.int64, device=dev)
    opar = torch.empty(buf.cap, dtype=torch.int32, device=dev)
    ocol = torch.empty(buf.cap, dtype=torch.uint8, device=dev)
    oc = torch.zeros(2, dtype=torch.int64, device=dev)
    out = _capi.ccl_outputs_t(olab.data_ptr(), ofeat.data_ptr(), opar.data_ptr(), ocol.data_ptr(), buf.cap,
                              oc.data_ptr())
    wsb = int(lib.ccl_fill_workspace_bytes(buf.cap))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    fill_ms, fo_ms, c4_ms, label_ms, px, fill_bytes = 0.0, 0.0, 0.0, 0.0, 0, 0
    for _, img in work:
        t = torch.from_numpy(img).to(dev)
        ccl.launch(t, buf)  # warm
        ccl.launch(t, fo)
        ccl.launch(t, c4, fg_adjacency=4)
        torch.cuda.synchronize()
        n_lab = int(buf.counts[0].item())
        if int(c4.counts[0].item()) > c4.cap:
            raise RuntimeError("table capacity too small for the complementary pair")
        for _ in range(reps + 1):  # the first of each is a warm-up
            e = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
            e[0].record(stream)
            ccl.launch(t, buf)
            e[1].record(stream)
            e[2].record(stream)
            rc = lib.ccl_fill_holes(ctypes.byref(buf.out), w, h, ctypes.byref(out), None, ctypes.c_void_p(ws.data_ptr()),
                                    wsb, ctypes.c_void_p(stream.cuda_stream))
            _capi.check(rc, "ccl_fill_holes")
            e[3].record(stream)
            e[4].record(stream)
            ccl.launch(t, fo)
            e[5].record(stream)
            e[6].record(stream)
            ccl.launch(t, c4, fg_adjacency=4)
            e[7].record(stream)
            torch.cuda.synchronize()
            if _ > 0:
                label_ms += e[0].elapsed_time(e[1])
                fill_ms += e[2].elapsed_time(e[3])
                fo_ms += e[4].elapsed_time(e[5])
                c4_ms += e[6].elapsed_time(e[7])
        n_fill = int(oc[0].item())
        px += w * h * reps
        # read the label image and the labeling's tables, write the filled ones
        fill_bytes += reps * (8 * w * h + 45 * n_lab + 45 * n_fill)
    gps = lambda ms: round(px / (ms / 1e3) / 1e9, 2)
    fill_gbs = fill_bytes / (fill_ms / 1e3) / 1e9
    return {"images": len(work), "label_Gpixel_s": gps(label_ms),
            "fill_holes": {"Gpixel_s": gps(fill_ms), "ms_per_image": round(fill_ms / (px / (w * h)), 4),
                           "label_plus_fill_Gpixel_s": gps(label_ms + fill_ms),
                           "alg_GBs": round(fill_gbs, 1), "hbm_frac": round(fill_gbs / HBM_PEAK_GBS, 4)},
            "features_only": {"Gpixel_s": gps(fo_ms), "ms_per_image": round(fo_ms / (px / (w * h)), 4)},
            "fg4_bg8": {"Gpixel_s": gps(c4_ms), "ms_per_image": round(c4_ms / (px / (w * h)), 4)}}


def cpu_baseline(work, budget_s: float = 40.0):
    """The oracle as it stands, one thread, on the headline workload's images
    (one pass each, until the time budget is spent)."""
    import oracle
    oracle.build(force=False)
    px, secs, used = 0, 0.0, []
    for tag, img in work:
        t0 = time.perf_counter()
        oracle.label(img)
        secs += time.perf_counter() - t0
        px += img.size
        used.append(tag)
        say(f"  oracle {tag}: {secs:.1f} s so far")
        if secs >= budget_s:
            break
    return dict(value=px / secs / 1e9, unit="Gpixel/s", cores=1, kind="oracle",
                sample=f"{len(used)} of {len(work)} workload images {used}, one pass each, one thread, "
                       f"{secs:.1f} s",
                host=host_cpu())


def oracle_timings(sweep, batch_host):
    """The oracle on the other configurations: 512 x 512 (p = 0.5, seed 0;
    median of 5, in ms), every image of the 8192^2 sweep once (one thread),
    and the 4096-image uneven batch over all usable host cores (threads; the
    oracle's C call runs without the interpreter lock)."""
    import concurrent.futures as cf
    import oracle
    import synth
    oracle.build(force=False)
    out = {"host": host_cpu()}
    img = synth.bernoulli_blocks(512, 512, 0.5, 1, 0)
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        oracle.label(img)
        ts.append(time.perf_counter() - t0)
    ts.sort()
    out["c1_512"] = {"median_ms": round(ts[2] * 1e3, 3), "Mpixel_s": round(img.size / ts[2] / 1e6, 2), "cores": 1}
    per, secs, px = {}, 0.0, 0
    for tag, im in sweep:
        t0 = time.perf_counter()
        oracle.label(im)
        dt = time.perf_counter() - t0
        per[f"p{tag[0]}_g{tag[1]}"] = round(dt * 1e3, 1)
        secs += dt
        px += im.size
    say(f"  oracle sweep: {secs:.1f} s for {len(sweep)} images")
    out["sweep8192"] = {"images": len(sweep), "total_s": round(secs, 2), "Mpixel_s": round(px / secs / 1e6, 2),
                        "cores": 1, "ms_per_image": per}
    if batch_host:
        cores = out["host"]["usable_cores"]
        px = sum(im.size for im in batch_host)
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(cores) as ex:
            for _ in ex.map(oracle.label, batch_host):
                pass
        dt = time.perf_counter() - t0
        say(f"  oracle batch: {dt:.1f} s on {cores} threads")
        out["batch4096"] = {"images": len(batch_host), "total_s": round(dt, 2), "Mpixel_s": round(px / dt / 1e6, 2),
                            "cores": cores}
    return out


# The paper's CPU timings (Sec. 4: 2048 x 2048 random images by density and
# granularity, one thread of a Skylake Gold 6126 @ 2.60 GHz), cycles per pixel
PAPER_TABLE1_CPP = {"BWA": [2.80, 15.3], "+Euler": [0.0, 0.66], "+hole filling": [0.0, 0.74],
                    "+features": [0.0, 10.3], "+relabeling": [0.59, 13.2]}
PAPER_TABLE2_CPP = {"BWAR": [3.41, 28.9], "BWAER": [3.41, 29.0], "BWAE": [2.80, 15.9], "BWAF": [2.80, 24.8]}


def host_lsl_bw(side: int = 2048, reps: int = 5):
    """The paper's own algorithm on the host (liblslbw.so, one thread), in
    cycles per pixel on side x side Bernoulli images of the sweep's densities
    and granularities, per configuration of Tables 1 and 2; the best of `reps`
    calls per image, then min / max over the images (the paper's protocol).
    Cycles are time-stamp-counter ticks, i.e. at the host's nominal clock."""
    import synth
    from paper_2006_09299_amd import lslbw
    ctx = lslbw.Context(side, side)
    per = {name: [] for name in lslbw.CONFIGS}
    t0 = time.perf_counter()
    ticks = ns = 0
    for gi, g in enumerate(synth.SWEEP_G):
        for pi, p in enumerate(synth.SWEEP_P):
            img = synth.bernoulli_blocks(side, side, p, g, 100 + 5 * gi + pi)
            for name, fl in lslbw.CONFIGS.items():
                rs = [ctx.label(img, fl) for _ in range(reps)]
                per[name].append(min(r.tsc for r in rs) / img.size)
                ticks += sum(r.tsc for r in rs)
                ns += sum(r.ns for r in rs)
    ctx.close()
    cpp = {k: [round(min(v), 2), round(max(v), 2)] for k, v in per.items()}
    extra = {"+Euler": "BWAE", "+hole filling": "BWA+fill", "+features": "BWAF", "+relabeling": "BWAR"}
    table1 = {"BWA": cpp["BWA"]}
    for k, cfg in extra.items():  # extra time over the base, image by image
        d = [a - b for a, b in zip(per[cfg], per["BWA"])]
        table1[k] = [round(min(d), 2), round(max(d), 2)]
    say(f"  host LSL-BW: {time.perf_counter() - t0:.1f} s")
    return {"images": f"{side}x{side}, p in {list(synth.SWEEP_P)} x g in {list(synth.SWEEP_G)}",
            "unit": "cycles/pixel (min, max over images)", "threads": 1, "host": host_cpu(),
            "tsc_GHz": round(ticks / ns, 3),
            "table1": {"ours": table1, "paper": PAPER_TABLE1_CPP},
            "table2": {"ours": {k: cpp[k] for k in PAPER_TABLE2_CPP}, "paper": PAPER_TABLE2_CPP},
            "all_configs": cpp,
            "paper_host": "Skylake Gold 6126 @ 2.60 GHz, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="structured16384", choices=["structured16384", "sweep8192"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-also", action="store_true", help="only the headline workload")
    ap.add_argument("--serve-requests", type=int, default=20000, help="measured requests of the serving leg")
    ap.add_argument("--fill-only", action="store_true",
                    help="only the hole-filling / features-only leg on the sweep images (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one plain device-to-device copy of MIB MiB (scales the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        say(f"copied {n} bytes")
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build labels each image on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.fill_only:
        fx = run_widened(make_workload("sweep8192"), reps=1)
        print(json.dumps({"widened_sweep8192": fx}), flush=True)
        return
    say(f"bench: workload {args.workload}, steps {args.steps}, warmup {args.warmup}")
    work = make_workload(args.workload)
    r = run_gpu(work, args.steps, args.warmup)
    head = summarize(r, args.workload)
    ms_step = r["total_ms"] / r["steps"]
    say(f"  {head['Gpixel_s']} Gpixel/s, {ms_step:.3f} ms/step, kernels {json.dumps(head['kernel_avg_ms'])}")
    import paper_2006_09299_amd as ccl
    out = {
        "metric": "Gpixel/s labeling+features+tree+Euler (1 GPU)",
        "value": head["Gpixel_s"],
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "name": args.workload, "images_per_step": len(work),
                   "shape": list(work[0][1].shape), **_variant_config(work[0][1].shape)},
        "roofline": head["roofline"],
        "path_hbm": head["path_hbm"],
        "ms_per_image": head["ms_per_image"],
        "traced_ms_per_image": head["traced_ms_per_image"],
        "launches_per_image": head["launches_per_image"],
        "hbm_copy_ceiling": copy_ceiling(),
        "kernel_avg_ms": head["kernel_avg_ms"],
    }
    also = {}
    sweep, batch_host = None, []
    if not args.no_also:
        if args.workload == "sweep8192":
            sweep = work
            say("bench: secondary workload structured16384")
            w2 = make_workload("structured16384")
            also["structured16384"] = summarize(run_gpu(w2, max(2, args.steps), 1), "structured16384")
            del w2
        else:
            say("bench: secondary workload sweep8192")
            sweep = make_workload("sweep8192")
            also["sweep8192"] = summarize(run_gpu(sweep, max(2, min(args.steps, 5)), 1), "sweep8192")
        say("bench: 8192^2 sweep, caches cold and warm")
        also["sweep8192_cold_warm"] = cold_warm(sweep)
        say(f"  {json.dumps(also['sweep8192_cold_warm'])}")
        say("bench: 512^2, eager and graph-replayed")
        also["c1_512"] = run_c1()
        say(f"  {json.dumps(also['c1_512'])}")
        say("bench: hole filling, features-only mode and the 4/8 connectivity pair on the sweep images")
        fx = run_widened(sweep)
        say(f"  {json.dumps(fx)}")
        also["widened_sweep8192"] = fx
        say("bench: batch4096")
        also["batch4096"] = run_batch(4096, max(3, args.steps), 1, host_out=batch_host)
        say("bench: serving (continuous batching), then one request per launch")
        src = serve_sources(args.serve_requests + 2000)
        sv = run_serve(args.serve_requests, src)
        say(f"  serve: {json.dumps(sv)}")
        sv1 = run_serve(min(args.serve_requests, 4000), src, batched=False)
        say(f"  serve, one request per launch: {json.dumps(sv1)}")
        # offered load far above what one GPU can take: the server's capacity
        sv2 = run_serve(args.serve_requests, src, rate_hz=40000.0, warmup_s=0.05)
        say(f"  serve, overloaded: {json.dumps(sv2)}")
        also["serve"] = {"continuous_batching": sv, "one_request_per_launch": sv1, "overloaded_40k_req_s": sv2}
        del src
    if not args.no_cpu_baseline:
        say("bench: cpu baseline (oracle) on the headline workload")
        out["cpu_baseline"] = cpu_baseline(work)
        if sweep is not None:
            say("bench: oracle on 512^2, the sweep and the batch")
            also["oracle"] = oracle_timings(sweep, batch_host)
        say("bench: the paper's algorithm on the host (single-thread LSL-BW), cycles per pixel")
        also["host_lsl_bw"] = host_lsl_bw()
        say(f"  {json.dumps(also['host_lsl_bw'])}")
    if also:
        out["also"] = also
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
