"""ctypes view of libccl.so (include/ccl.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccl.so")

CCL_OK = 0
CCL_EINVAL = -1
CCL_ENOSPC = -2
CCL_EHIP = -3
CCL_ECAPACITY = -4
CCL_ETOOBIG = -5


class ccl_outputs_t(ctypes.Structure):
    _fields_ = [
        ("labels", ctypes.c_void_p),
        ("features", ctypes.c_void_p),
        ("parent", ctypes.c_void_p),
        ("color", ctypes.c_void_p),
        ("cap", ctypes.c_int64),
        ("counts", ctypes.c_void_p),
    ]


class ccl_image_t(ctypes.Structure):
    _fields_ = [
        ("img", ctypes.c_void_p),
        ("w", ctypes.c_int32),
        ("h", ctypes.c_int32),
        ("pitch", ctypes.c_int64),
        ("out", ccl_outputs_t),
    ]


class ccl_server_config_t(ctypes.Structure):
    _fields_ = [
        ("max_slots", ctypes.c_int32),
        ("streams", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("cap_divisor", ctypes.c_int32),
    ]


class ccl_done_t(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("w", ctypes.c_int32),
        ("h", ctypes.c_int32),
        ("launches", ctypes.c_int32),
        ("n_labels", ctypes.c_int64),
        ("euler", ctypes.c_int64),
        ("out", ccl_outputs_t),
    ]


class ccl_server_stats_t(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "queued", "live", "in_flight", "ready", "pool_used", "pool_bytes", "admitted", "completed", "launches",
        "relaunched")]


EXPORTS = (
    "ccl_workspace_bytes", "ccl_label", "ccl_label_traced", "ccl_kernel_name", "ccl_num_variants",
    "ccl_variant_info", "ccl_workspace_bytes_v", "ccl_label_v", "ccl_batch_sizes", "ccl_batch_prepare",
    "ccl_label_batch", "ccl_strerror", "ccl_tile_shape", "ccl_server_create", "ccl_server_footprint",
    "ccl_server_submit", "ccl_server_poll", "ccl_server_release", "ccl_server_stats", "ccl_server_destroy",
    "ccl_fill_workspace_bytes", "ccl_fill_holes", "ccl_label_conn", "ccl_label_noalloc", "ccl_variant_for",
)
NOALLOC_SCRATCH_BYTES = 96 << 20  # CCL_NOALLOC_SCRATCH_BYTES
TRACE_EVENTS = 10

_lib = None


class CclError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


def lib():
    """Load libccl.so; raises when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first (python -m paper_2006_09299_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        L.ccl_workspace_bytes.restype = ctypes.c_size_t
        L.ccl_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.ccl_variant_for.restype = ctypes.c_int32
        L.ccl_variant_for.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.ccl_label.restype = ctypes.c_int
        L.ccl_label.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                ctypes.POINTER(ccl_outputs_t), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.ccl_label_traced.restype = ctypes.c_int
        L.ccl_label_traced.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.POINTER(ccl_outputs_t), ctypes.c_void_p, ctypes.c_size_t,
                                       ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
        L.ccl_kernel_name.restype = ctypes.c_char_p
        L.ccl_kernel_name.argtypes = [ctypes.c_int]
        L.ccl_num_variants.restype = ctypes.c_int32
        L.ccl_num_variants.argtypes = []
        L.ccl_variant_info.restype = ctypes.c_int
        L.ccl_variant_info.argtypes = [ctypes.c_int32] + [ctypes.POINTER(ctypes.c_int32)] * 6
        L.ccl_workspace_bytes_v.restype = ctypes.c_size_t
        L.ccl_workspace_bytes_v.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.ccl_label_v.restype = ctypes.c_int
        L.ccl_label_v.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.POINTER(ccl_outputs_t), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                  ctypes.c_int32]
        L.ccl_batch_sizes.restype = ctypes.c_int
        L.ccl_batch_sizes.argtypes = [ctypes.POINTER(ccl_image_t), ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
        L.ccl_batch_prepare.restype = ctypes.c_int
        L.ccl_batch_prepare.argtypes = [ctypes.POINTER(ccl_image_t), ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_size_t]
        L.ccl_label_batch.restype = ctypes.c_int
        L.ccl_label_batch.argtypes = [ctypes.POINTER(ccl_image_t), ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.ccl_strerror.restype = ctypes.c_char_p
        L.ccl_strerror.argtypes = [ctypes.c_int]
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.ccl_server_create.restype = ctypes.c_int
        L.ccl_server_create.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(ccl_server_config_t),
                                        ctypes.POINTER(ctypes.c_void_p)]
        L.ccl_server_footprint.restype = ctypes.c_int
        L.ccl_server_footprint.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
        L.ccl_server_submit.restype = ctypes.c_int
        L.ccl_server_submit.argtypes = [vp, vp, i32, i32, i64, i64]
        L.ccl_server_poll.restype = ctypes.c_int
        L.ccl_server_poll.argtypes = [vp, ctypes.POINTER(ccl_done_t), i32, ctypes.POINTER(i32)]
        L.ccl_server_release.restype = ctypes.c_int
        L.ccl_server_release.argtypes = [vp, i64]
        L.ccl_server_stats.restype = ctypes.c_int
        L.ccl_server_stats.argtypes = [vp, ctypes.POINTER(ccl_server_stats_t)]
        L.ccl_server_destroy.restype = ctypes.c_int
        L.ccl_server_destroy.argtypes = [vp]
        L.ccl_fill_workspace_bytes.restype = ctypes.c_size_t
        L.ccl_fill_workspace_bytes.argtypes = [i64]
        L.ccl_fill_holes.restype = ctypes.c_int
        L.ccl_fill_holes.argtypes = [ctypes.POINTER(ccl_outputs_t), i32, i32, ctypes.POINTER(ccl_outputs_t), vp, vp,
                                     ctypes.c_size_t, vp]
        L.ccl_label_conn.restype = ctypes.c_int
        L.ccl_label_conn.argtypes = [vp, i32, i32, i64, ctypes.POINTER(ccl_outputs_t), vp, ctypes.c_size_t, vp, i32]
        L.ccl_label_noalloc.restype = ctypes.c_int
        L.ccl_label_noalloc.argtypes = [vp, i32, i32, i64, ctypes.POINTER(ccl_outputs_t), vp]
        L.ccl_tile_shape.restype = None
        L.ccl_tile_shape.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().ccl_strerror(int(code)).decode()


def check(code: int, where: str) -> None:
    if code != CCL_OK:
        raise CclError(code, where)


def workspace_bytes(w: int, h: int, variant=None) -> int:
    """Workspace of `variant`, or (None) of what ccl_label runs for the size."""
    if variant is None:
        return int(lib().ccl_workspace_bytes(int(w), int(h)))
    return int(lib().ccl_workspace_bytes_v(int(w), int(h), int(variant)))


def variant_for(w: int, h: int) -> int:
    """The variant ccl_label runs for a w x h image."""
    v = int(lib().ccl_variant_for(int(w), int(h)))
    check(v if v < 0 else 0, "ccl_variant_for")
    return v


VARIANT_ENV, TILE_ENV = "CCL_VARIANT", "CCL_TILE"


def env_variant() -> Optional[int]:
    """Variant forced from the environment, for experiments: CCL_VARIANT=<index>
    or CCL_TILE=<rows>x<cols> (the lowest-numbered variant of that tile shape);
    None when neither is set.  Calls that are given a variant ignore it."""
    n = num_variants()
    s = os.environ.get(VARIANT_ENV, "").strip()
    if s:
        try:
            v = int(s)
        except ValueError:
            v = -1
        if not 0 <= v < n:
            raise ValueError(f"{VARIANT_ENV}={s!r}: expected a variant index in [0, {n})")
        return v
    s = os.environ.get(TILE_ENV, "").strip().lower()
    if s:
        for v in range(n):
            th, tw = variant_info(v)[:2]
            if s == f"{th}x{tw}":
                return v
        shapes = sorted({"%dx%d" % tuple(variant_info(v)[:2]) for v in range(n)})
        raise ValueError(f"{TILE_ENV}={s!r}: no compiled variant has that tile shape ({', '.join(shapes)})")
    return None


def num_variants() -> int:
    return int(lib().ccl_num_variants())


def variant_info(v: int):
    """(tile rows, tile columns, uses the LDS hash reduction, threads per tile,
    super-tile side, tiles per root-reduction workgroup)"""
    vals = [ctypes.c_int32() for _ in range(6)]
    check(lib().ccl_variant_info(int(v), *[ctypes.byref(x) for x in vals]), "ccl_variant_info")
    th, tw, hs, nt, sup, rg = (x.value for x in vals)
    return th, tw, bool(hs), nt, sup, rg


def kernel_names():
    return [lib().ccl_kernel_name(k).decode() for k in range(TRACE_EVENTS - 1)]


def tile_shape():
    th, tw = ctypes.c_int32(), ctypes.c_int32()
    lib().ccl_tile_shape(ctypes.byref(th), ctypes.byref(tw))
    return th.value, tw.value
