"""CPU oracle for black-and-white connected-component labeling and analysis.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product path (the HIP
library and its Python binding) never imports this package.

``label(img)`` runs the plain C definition in ``ccl_oracle.c`` (pixel-level
two-pass union-find for both polarities, direct feature sums, breadth-first
search over the region adjacency graph for the inclusion tree, Euler number
as #foreground components - #holes).  See that file's header for the readings
taken where the paper (Lemaitre & Lacassagne 2020) is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ccl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ERRORS = {-1: "invalid argument", -2: "out of memory", -3: "capacity", -4: "adjacency graph is not a tree"}

_lib = None


def build(force: bool = True) -> str:
    """Compile ``ccl_oracle.c`` into ``liboracle.so`` with plain gcc -O2."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


_ARGS = [
    ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
    ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
    ctypes.c_void_p, ctypes.c_void_p,
]


def _bind(lib):
    f = lib.oracle_label
    f.restype = ctypes.c_int64
    f.argtypes = list(_ARGS)
    if hasattr(lib, "oracle_label_conn"):
        g = lib.oracle_label_conn
        g.restype = ctypes.c_int64
        g.argtypes = list(_ARGS) + [ctypes.c_int32]
    return lib


def load_variant(path: str):
    """Load another build of the oracle source (used by tests that plant a
    mistake in a copy of the source and check that the pins catch it)."""
    return _bind(ctypes.CDLL(path))


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


@dataclass
class Result:
    """Outputs of one labeling, indexed by canonical id (exterior = 0)."""

    labels: np.ndarray    # int32 [h, w]
    bbox: np.ndarray      # int64 [n, 4]: xmin, xmax, ymin, ymax
    S: np.ndarray         # int64 [n]
    Sx: np.ndarray        # int64 [n]
    Sy: np.ndarray        # int64 [n]
    parent: np.ndarray    # int32 [n]; parent[0] = -1
    color: np.ndarray     # uint8 [n]; 1 = foreground
    euler: int

    @property
    def n_labels(self) -> int:
        return int(self.parent.shape[0])


def label(img: np.ndarray, lib=None, fg8: bool = True) -> Result:
    """Label a 2-D uint8 image (nonzero = foreground); rows may be strided.
    fg8=False takes the complementary connectivity pair (4-adjacent
    foreground, 8-adjacent background)."""
    img = np.asarray(img)
    if img.dtype != np.uint8 or img.ndim != 2:
        raise ValueError("oracle.label expects a 2-D uint8 array")
    if img.strides[1] != 1:
        img = np.ascontiguousarray(img)
    h, w = img.shape
    pitch = img.strides[0] if h > 1 else w
    lib = lib if lib is not None else _load()
    labels = np.empty((h, w), dtype=np.int32)
    euler = np.zeros(1, dtype=np.int64)
    # first table capacity: a quarter of the pixels covers every image of the
    # workloads but checkerboard-like ones; a larger count is reported and
    # the call is repeated with the exact size
    cap = h * w // 4 + 16
    while True:
        feat = np.empty((cap, 7), dtype=np.int64)
        parent = np.empty(cap, dtype=np.int32)
        color = np.empty(cap, dtype=np.uint8)
        args = (img.ctypes.data, w, h, pitch, labels.ctypes.data, cap, feat.ctypes.data,
                parent.ctypes.data, color.ctypes.data, euler.ctypes.data)
        n = lib.oracle_label(*args) if fg8 else lib.oracle_label_conn(*args, 0)
        if n == -3:
            cap = int(labels.max()) + 1 if labels.size else cap * 2
            continue
        if n < 0:
            raise RuntimeError(f"oracle_label failed: {ERRORS.get(int(n), n)}")
        break
    n = int(n)
    feat = feat[:n]
    return Result(
        labels=labels,
        bbox=feat[:, 0:4].copy(),
        S=feat[:, 4].copy(),
        Sx=feat[:, 5].copy(),
        Sy=feat[:, 6].copy(),
        parent=parent[:n].copy(),
        color=color[:n].copy(),
        euler=int(euler[0]),
    )


def fill_holes(img: np.ndarray, lib=None):
    """Hole filling, the optional step of the transitive closure (Sec. 3.2,
    Algorithm 3; Fig. 2, "hole filled"): a component whose surrounding is
    not the exterior is merged into it, so every hole, with everything
    nested inside it, joins the top-level foreground component around it.

    Written as the plain definition it reaches: the filled image is the
    complement of the exterior (the background connected to the image
    frame), labeled like any image.  Returns (filled Result, map) where
    map[c] is the filled id of the original component c (the filled label at
    c's first pixel; the exterior keeps 0)."""
    r = label(img, lib)
    f = label((r.labels != 0).astype(np.uint8), lib)
    mp = np.zeros(r.n_labels, dtype=np.int32)
    ids, first = np.unique(r.labels.ravel(), return_index=True)  # first pixel of each id in raster order
    mp[ids] = f.labels.ravel()[first]
    return f, mp
