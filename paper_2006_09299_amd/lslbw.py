"""Binding of liblslbw.so: the paper's own algorithm, LSL-BW, single-thread on
the host (segment detection, B&W unification with initial adjacency,
transitive closure with the adjacency tree and optional hole filling,
relabeling; Lemaitre & Lacassagne 2020, Sec. 2 and Sec. 3.2, Algorithms
1-4).  It is the like-for-like CPU comparison of the GPU path, timed in
cycles per pixel as the paper's Tables 1 and 2 are; interface and readings in
include/lslbw.h.  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(_HERE, "host", "liblslbw.so")

FEATURES, RELABEL, EULER, FILL, FG4 = 1, 2, 4, 8, 16
# the paper's configurations (Table 2's "Our" column; A = adjacency tree,
# B / W = background / foreground labels, E Euler, F features, R relabel)
CONFIGS = {
    "BWA": 0,
    "BWAE": EULER,
    "BWAF": FEATURES,
    "BWAR": RELABEL,
    "BWAER": EULER | RELABEL,
    "BWA+fill": FILL,
    "BWAEFR": EULER | FEATURES | RELABEL,
}


# lslbw_feature_t (40 bytes)
FEATURE_DTYPE = np.dtype([("xmin", "<i4"), ("xmax", "<i4"), ("ymin", "<i4"), ("ymax", "<i4"),
                          ("S", "<i8"), ("Sx", "<i8"), ("Sy", "<i8")])


class _Time(ctypes.Structure):
    _fields_ = [("tsc", ctypes.c_uint64), ("ns", ctypes.c_uint64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is not built (python -m paper_2006_09299_amd.build)")
        lib = ctypes.CDLL(LIB)
        lib.lslbw_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]
        lib.lslbw_create.restype = ctypes.c_int
        lib.lslbw_destroy.argtypes = [ctypes.c_void_p]
        lib.lslbw_destroy.restype = None
        lib.lslbw_label.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(_Time)]
        lib.lslbw_label.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class HostResult:
    labels: np.ndarray | None  # int32 [h, w] (RELABEL)
    features: np.ndarray | None  # int64 [n, 7]: xmin, xmax, ymin, ymax, S, Sx, Sy (FEATURES)
    parent: np.ndarray       # int32 [n]
    color: np.ndarray        # uint8 [n]
    n_labels: int
    euler: int
    tsc: int                 # time-stamp-counter ticks of the call
    ns: int


class Context:
    """Working tables for w x h images (reused across calls)."""

    def __init__(self, w: int, h: int):
        self.lib = _load()
        self.w, self.h = int(w), int(h)
        p = ctypes.c_void_p()
        rc = self.lib.lslbw_create(self.w, self.h, ctypes.byref(p))
        if rc != 0:
            raise RuntimeError(f"lslbw_create failed ({rc})")
        self.ptr = p

    def close(self):
        if self.ptr:
            self.lib.lslbw_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        self.close()

    def label(self, img: np.ndarray, flags: int = FEATURES | RELABEL | EULER, cap: int | None = None) -> HostResult:
        img = np.asarray(img)
        if img.dtype != np.uint8 or img.ndim != 2 or img.shape != (self.h, self.w):
            raise ValueError(f"expected a {self.h}x{self.w} uint8 image")
        if img.strides[1] != 1:
            img = np.ascontiguousarray(img)
        pitch = img.strides[0] if self.h > 1 else self.w
        cap = self.w * self.h + 1 if cap is None else int(cap)
        labels = np.empty((self.h, self.w), np.int32) if flags & RELABEL else None
        feat = np.empty(cap, FEATURE_DTYPE) if flags & FEATURES else None
        parent = np.empty(cap, np.int32)
        color = np.empty(cap, np.uint8)
        counts = np.zeros(2, np.int64)
        t = _Time()
        rc = self.lib.lslbw_label(self.ptr, img.ctypes.data, pitch, int(flags),
                                  None if labels is None else labels.ctypes.data,
                                  None if feat is None else feat.ctypes.data,
                                  parent.ctypes.data, color.ctypes.data, cap, counts.ctypes.data, ctypes.byref(t))
        if rc != 0:
            raise RuntimeError(f"lslbw_label failed ({rc})")
        n = int(counts[0])
        k = min(n, cap)
        fk = None
        if feat is not None:
            fk = np.stack([feat[f][:k].astype(np.int64) for f in FEATURE_DTYPE.names], axis=1)
        return HostResult(labels=labels, features=fk,
                          parent=parent[:k].copy(), color=color[:k].copy(), n_labels=n, euler=int(counts[1]),
                          tsc=int(t.tsc), ns=int(t.ns))


def label(img: np.ndarray, flags: int = FEATURES | RELABEL | EULER) -> HostResult:
    img = np.asarray(img)
    ctx = Context(img.shape[1], img.shape[0])
    try:
        return ctx.label(img, flags)
    finally:
        ctx.close()
