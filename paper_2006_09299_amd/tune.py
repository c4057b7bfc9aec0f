"""Autotuner: picks the variant (tile shape, root-reduction scheme) of the
batched path for a workload by timing every compiled variant on a sample of
it, and remembers the choice in a JSON cache keyed by GPU architecture,
image-size bucket and run-density bucket.  All variants give identical
results; only their speed differs."""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Optional, Sequence

import torch

from . import _capi
from .batch import BatchPlan

CACHE_ENV = "CCL_TUNE_CACHE"


def cache_path() -> str:
    p = os.environ.get(CACHE_ENV)
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "paper_2006_09299_amd", "tune.json")


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: Dict[str, dict]) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def variants_digest() -> str:
    """Digest of the variant table of the loaded library (shape, reduction,
    workgroup size, merge schedule of every index): a cache entry written for
    another table is never used."""
    import hashlib
    h = hashlib.sha256()
    for v in range(_capi.num_variants()):
        h.update(repr(tuple(_capi.variant_info(v))).encode())
    return h.hexdigest()[:12]


def workload_key(imgs: Sequence[torch.Tensor]) -> str:
    """arch / variant table digest / log2(mean pixels per image) /
    run-density bucket (horizontal colour changes per pixel, in steps of
    0.05)."""
    arch = torch.cuda.get_device_properties(imgs[0].device).gcnArchName.split(":")[0]
    px = sum(int(t.numel()) for t in imgs) / len(imgs)
    sample = imgs[: min(len(imgs), 16)]
    changes = sum(int((t[:, 1:] != t[:, :-1]).sum()) for t in sample)
    total = sum(int(t.numel()) for t in sample)
    dens = changes / max(total, 1)
    return f"{arch}/v{variants_digest()}/px2^{round(math.log2(max(px, 1)))}/runs{round(dens / 0.05) * 0.05:.2f}"


def time_variant(imgs: Sequence[torch.Tensor], variant: int, reps: int = 3) -> float:
    """Median milliseconds of one graph replay of the batch."""
    plan = BatchPlan(imgs, variant=variant)
    plan.capture()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        plan.replay()
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def autotune(imgs: Sequence[torch.Tensor], variants: Optional[Sequence[int]] = None, reps: int = 3,
             force: bool = False, path: Optional[str] = None) -> int:
    """Best variant for batches like `imgs` (cached); a variant forced from
    the environment (CCL_VARIANT / CCL_TILE) is returned untimed."""
    forced = _capi.env_variant()
    if forced is not None:
        return forced
    path = path or cache_path()
    key = workload_key(imgs)
    data = _load(path)
    if not force and key in data:
        try:
            v = int(data[key]["variant"])
        except (KeyError, TypeError, ValueError):
            v = -1
        if 0 <= v < _capi.num_variants():
            return v  # else: a damaged entry, timed again
    if variants is None:
        variants = range(_capi.num_variants())
    timings = {int(v): time_variant(imgs, int(v), reps) for v in variants}
    best = min(timings, key=timings.get)
    data[key] = {"variant": best, "ms": {str(k): round(t, 4) for k, t in timings.items()},
                 "tiles": {str(k): list(_capi.variant_info(k)) for k in timings}}
    _store(path, data)
    return best
