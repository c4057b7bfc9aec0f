"""Seeded synthetic binary images shared by the tests, the smoke check and the
benchmark.  This module holds no labeling arithmetic: it only draws pixels.

The paper (Lemaitre & Lacassagne 2020, Sec. 4) measures on random images of
varying foreground density p and granularity g in the style of Grana et al.
2018: Bernoulli(p) cells of g x g pixels.  Those image sets are not available
here, so every workload is drawn from numpy's PCG64 with a fixed seed:

* ``bernoulli_blocks``: iid Bernoulli(p) on g x g blocks, cropped to h x w;
* ``structured``: nested disks/annuli with radii log-uniform in [4, 2000],
  depth 1..8 and alternating colour, then 5% salt (pixels set to foreground);
* ``batch_specs``: the uneven batch (sides log-uniform in [64, 2048]);
* ``serve_stream``: a Poisson request stream (sides log-uniform in [256, 8192]).

All images are uint8 with values {0, 1} (nonzero = foreground).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Iterator, List

import numpy as np

# 8192 x 8192 density x granularity sweep
SWEEP_P = (0.1, 0.3, 0.5, 0.7, 0.9)
SWEEP_G = (1, 2, 4, 8, 16)


def bernoulli_blocks(h: int, w: int, p: float, g: int = 1, seed: int = 0) -> np.ndarray:
    """iid Bernoulli(p) on g x g blocks: kron(B(p, ceil(h/g) x ceil(w/g)), ones(g, g))[:h, :w]."""
    rng = np.random.default_rng(seed)
    bh, bw = -(-h // g), -(-w // g)
    cells = (rng.random((bh, bw), dtype=np.float32) < np.float32(p)).astype(np.uint8)
    if g == 1:
        return np.ascontiguousarray(cells[:h, :w])
    img = np.repeat(np.repeat(cells, g, axis=0), g, axis=1)
    return np.ascontiguousarray(img[:h, :w])


def sweep_8192(side: int = 8192):
    """The 25-image density x granularity sweep: yields (p, g, seed, image).
    seed = 100 + 5 * gi + pi."""
    for gi, g in enumerate(SWEEP_G):
        for pi, p in enumerate(SWEEP_P):
            seed = 100 + 5 * gi + pi
            yield p, g, seed, bernoulli_blocks(side, side, p, g, seed)


def _paint_disk(img: np.ndarray, cy: float, cx: float, r: float, val: int) -> None:
    h, w = img.shape
    y0, y1 = max(0, int(math.floor(cy - r))), min(h, int(math.ceil(cy + r)) + 1)
    x0, x1 = max(0, int(math.floor(cx - r))), min(w, int(math.ceil(cx + r)) + 1)
    if y0 >= y1 or x0 >= x1:
        return
    yy = (np.arange(y0, y1, dtype=np.float32) - np.float32(cy))[:, None]
    xx = (np.arange(x0, x1, dtype=np.float32) - np.float32(cx))[None, :]
    inside = yy * yy + xx * xx <= np.float32(r * r)
    img[y0:y1, x0:x1][inside] = val


def structured(h: int = 16384, w: int = 16384, seed: int = 0, groups: int = 256,
               rmin: float = 4.0, rmax: float = 2000.0, max_depth: int = 8,
               salt: float = 0.05) -> np.ndarray:
    """Nested disks on a background canvas, then salt.

    For each of ``groups`` groups, placed one after another (later groups paint
    over earlier ones):
      * centre uniform over the image (disks may be clipped by the border);
      * depth d uniform in 1..max_depth;
      * d radii log-uniform in [rmin, rmax], sorted descending and forced at
        least 2 px apart so every ring is >= 2 px thick;
      * disks painted largest first with colours foreground, background,
        foreground, ...; each inner centre is jittered inside its parent disk
        so that it stays inside it.
    Finally ``salt`` of the pixels, drawn iid, are set to foreground.
    """
    rng = np.random.default_rng(seed)
    img = np.zeros((h, w), dtype=np.uint8)
    for _ in range(groups):
        cy, cx = rng.uniform(0, h), rng.uniform(0, w)
        d = int(rng.integers(1, max_depth + 1))
        radii = np.sort(np.exp(rng.uniform(math.log(rmin), math.log(rmax), size=d)))[::-1]
        for k in range(1, d):
            radii[k] = min(radii[k], radii[k - 1] - 2.0)
        for k in range(d):
            r = float(radii[k])
            if r < 1.0:
                break
            if k > 0:
                slack = float(radii[k - 1]) - r - 1.0
                if slack > 0:
                    ang = rng.uniform(0, 2 * math.pi)
                    rad = rng.uniform(0, slack)
                    cy, cx = cy + rad * math.sin(ang), cx + rad * math.cos(ang)
            _paint_disk(img, cy, cx, r, 1 if k % 2 == 0 else 0)
    if salt > 0:
        img |= (rng.random((h, w), dtype=np.float32) < np.float32(salt)).astype(np.uint8)
    return img


@dataclass(frozen=True)
class ImageSpec:
    w: int
    h: int
    p: float
    g: int
    seed: int

    def make(self) -> np.ndarray:
        return bernoulli_blocks(self.h, self.w, self.p, self.g, self.seed)

    @property
    def pixels(self) -> int:
        return self.w * self.h


def _log_uniform_side(rng: np.random.Generator, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_specs(n: int = 4096, seed: int = 7, lo: int = 64, hi: int = 2048) -> List[ImageSpec]:
    """The uneven batch: w, h independent log-uniform in [lo, hi]; p ~ U(0.3, 0.7);
    g in {1, 4} with probability 1/2 each.  Image i draws from seed (seed, i)."""
    specs = []
    for i in range(n):
        rng = np.random.default_rng([seed, i])
        w = _log_uniform_side(rng, lo, hi)
        h = _log_uniform_side(rng, lo, hi)
        p = float(rng.uniform(0.3, 0.7))
        g = 1 if rng.random() < 0.5 else 4
        specs.append(ImageSpec(w, h, p, g, seed * 1_000_003 + i))
    return specs


@dataclass(frozen=True)
class Request:
    arrival_s: float
    spec: ImageSpec


def serve_stream(n: int = 20000, rate_hz: float = 2000.0, seed: int = 11,
                 lo: int = 256, hi: int = 8192) -> List[Request]:
    """Open-loop Poisson arrivals (exponential gaps, mean 1/rate); sides
    log-uniform in [lo, hi]; p ~ U(0.1, 0.9); g in {1, 4}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate_hz))
        w = _log_uniform_side(rng, lo, hi)
        h = _log_uniform_side(rng, lo, hi)
        p = float(rng.uniform(0.1, 0.9))
        g = 1 if rng.random() < 0.5 else 4
        out.append(Request(t, ImageSpec(w, h, p, g, seed * 1_000_003 + i)))
    return out


def iter_images(specs) -> Iterator[np.ndarray]:
    for s in specs:
        yield s.make()
