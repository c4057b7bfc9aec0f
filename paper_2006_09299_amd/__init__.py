"""MI355X-native black-and-white connected-component labeling and analysis.

Run-based labeling after Lemaitre & Lacassagne (2020): foreground components
(8-adjacency) and background components (4-adjacency) of a binary image,
their bounding boxes and raw moments S, Sx, Sy, the Euler number and the
inclusion tree, all computed by the HIP kernels of libccl.so on gfx950.
This module only marshals arguments: PyTorch provides device memory and the
stream; every step of the computation runs in the library's kernels.

    from paper_2006_09299_amd import label
    r = label(img)          # img: 2-D uint8 tensor on the GPU, nonzero = foreground
    r.labels, r.bbox, r.S, r.Sx, r.Sy, r.parent, r.color, r.euler
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import torch

from . import _capi
from ._capi import CclError, num_variants, strerror, tile_shape, variant_info, workspace_bytes  # noqa: F401

FEATURE_BYTES = 40  # ccl_feature_t: int32 xmin, xmax, ymin, ymax; int64 S, Sx, Sy


@dataclass
class Result:
    """Outputs indexed by canonical id (exterior = 0); device tensors."""

    labels: Optional[torch.Tensor]  # int32 [h, w] (None in features-only mode)
    features: torch.Tensor          # int64 [n, 5] raw records (see bbox / S / Sx / Sy)
    parent: torch.Tensor            # int32 [n]; parent[0] = -1
    color: torch.Tensor             # uint8 [n]; 1 = foreground
    n_labels: int
    euler: int

    @property
    def bbox(self) -> torch.Tensor:  # int32 [n, 4]: xmin, xmax, ymin, ymax
        return self.features.view(torch.int32)[:, 0:4]

    @property
    def S(self) -> torch.Tensor:
        return self.features[:, 2]

    @property
    def Sx(self) -> torch.Tensor:
        return self.features[:, 3]

    @property
    def Sy(self) -> torch.Tensor:
        return self.features[:, 4]


class Buffers:
    """Preallocated outputs + workspace for repeated calls on one image shape."""

    def __init__(self, w: int, h: int, cap: int, device, labels: bool = True, variant: Optional[int] = None):
        self.w, self.h, self.cap = int(w), int(h), int(cap)
        # None: the environment's override (CCL_VARIANT / CCL_TILE), else the
        # variant ccl_label itself runs for this size
        if variant is None:
            variant = _capi.env_variant()
        self.variant = _capi.variant_for(w, h) if variant is None else int(variant)
        self.labels = torch.empty((h, w), dtype=torch.int32, device=device) if labels else None
        self.features = torch.empty((cap, 5), dtype=torch.int64, device=device)
        self.parent = torch.empty(cap, dtype=torch.int32, device=device)
        self.color = torch.empty(cap, dtype=torch.uint8, device=device)
        self.counts = torch.zeros(2, dtype=torch.int64, device=device)
        self.ws_bytes = workspace_bytes(w, h, self.variant)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        self.out = _capi.ccl_outputs_t(
            self.labels.data_ptr() if labels else None, self.features.data_ptr(), self.parent.data_ptr(),
            self.color.data_ptr(), self.cap, self.counts.data_ptr())


def _check_image(img: torch.Tensor):
    if not isinstance(img, torch.Tensor) or img.dtype != torch.uint8 or img.dim() != 2:
        raise ValueError("expected a 2-D uint8 tensor")
    if not img.is_cuda:
        raise ValueError("expected a GPU tensor (the library computes on the GPU only)")
    if img.shape[0] < 1 or img.shape[1] < 1:
        raise ValueError("empty image")
    if img.stride(1) != 1:
        raise ValueError("rows must be contiguous (stride(1) == 1)")
    h, w = img.shape
    pitch = img.stride(0) if h > 1 else w
    return int(w), int(h), int(pitch)


def launch(img: torch.Tensor, buf: Buffers, stream: Optional[int] = None, fg_adjacency: int = 8) -> None:
    """Enqueue one labeling into preallocated buffers (no synchronisation).
    fg_adjacency=4 takes the complementary connectivity pair (buffers made
    for variant 0 only)."""
    w, h, pitch = _check_image(img)
    if (w, h) != (buf.w, buf.h):
        raise ValueError("buffers were made for another shape")
    if stream is None:
        stream = torch.cuda.current_stream(img.device).cuda_stream
    if fg_adjacency == 8:
        rc = _capi.lib().ccl_label_v(img.data_ptr(), w, h, pitch, ctypes.byref(buf.out), buf.ws.data_ptr(),
                                     buf.ws_bytes, ctypes.c_void_p(stream), buf.variant)
    else:
        if buf.variant != 0:
            raise ValueError("the complementary connectivity pair is compiled for variant 0 only "
                             "(Buffers(..., variant=0))")
        rc = _capi.lib().ccl_label_conn(img.data_ptr(), w, h, pitch, ctypes.byref(buf.out), buf.ws.data_ptr(),
                                        buf.ws_bytes, ctypes.c_void_p(stream), int(fg_adjacency))
    _capi.check(rc, "ccl_label")


def label(img: torch.Tensor, cap: Optional[int] = None, labels: bool = True, variant: Optional[int] = None,
          fg_adjacency: int = 8) -> Result:
    """Label one image; synchronises to read the number of labels.

    cap: table capacity; by default a quarter of the pixels, grown and rerun
    when the image has more components (w*h + 1 always suffices).
    fg_adjacency: 8 (8-adjacent foreground, 4-adjacent background) or 4 (the
    complementary pair)."""
    w, h, pitch = _check_image(img)
    if variant is None and fg_adjacency != 8:
        variant = 0  # the complementary pair is compiled in variant 0's shape
    full = w * h + 1
    if cap is None:
        cap = min(full, max(1024, full // 4))
    while True:
        buf = Buffers(w, h, cap, img.device, labels=labels, variant=variant)
        launch(img, buf, fg_adjacency=fg_adjacency)
        counts = buf.counts.cpu()
        n, euler = int(counts[0]), int(counts[1])
        if n <= cap:
            break
        cap = n
    return Result(buf.labels, buf.features[:n], buf.parent[:n], buf.color[:n], n, euler)


def fill_holes(res: Result, shape=None, labels: bool = True, return_map: bool = False, stream: Optional[int] = None):
    """Hole filling on a finished labeling (ccl_fill_holes): every hole, with
    everything nested in it, joins the top-level foreground component around
    it.  `res` is a Result of label() / label_batch(); `shape` (h, w) is
    needed only when res has no label image.  Returns the filled image's
    Result (and, with return_map, the filled id of every original id);
    synchronises to read the number of filled labels."""
    if res.labels is not None:
        h, w = res.labels.shape
    elif shape is None:
        raise ValueError("fill_holes needs shape=(h, w) for a result without a label image")
    else:
        h, w = shape
    dev = res.parent.device
    n = int(res.n_labels)
    for t in (res.features, res.parent, res.color) + ((res.labels,) if res.labels is not None else ()):
        if not t.is_contiguous():
            raise ValueError("fill_holes expects the contiguous tables of a labeling")
    want_labels = labels and res.labels is not None
    counts_in = torch.tensor([n, int(res.euler)], dtype=torch.int64, device=dev)
    inp = _capi.ccl_outputs_t(res.labels.data_ptr() if res.labels is not None else None, res.features.data_ptr(),
                              res.parent.data_ptr(), res.color.data_ptr(), n, counts_in.data_ptr())
    olabels = torch.empty((h, w), dtype=torch.int32, device=dev) if want_labels else None
    ofeat = torch.empty((n, 5), dtype=torch.int64, device=dev)
    oparent = torch.empty(n, dtype=torch.int32, device=dev)
    ocolor = torch.empty(n, dtype=torch.uint8, device=dev)
    ocounts = torch.zeros(2, dtype=torch.int64, device=dev)
    out = _capi.ccl_outputs_t(olabels.data_ptr() if want_labels else None, ofeat.data_ptr(), oparent.data_ptr(),
                              ocolor.data_ptr(), n, ocounts.data_ptr())
    mp = torch.empty(n, dtype=torch.int32, device=dev) if return_map else None
    wsb = int(_capi.lib().ccl_fill_workspace_bytes(n))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    rc = _capi.lib().ccl_fill_holes(ctypes.byref(inp), int(w), int(h), ctypes.byref(out),
                                    ctypes.c_void_p(mp.data_ptr()) if mp is not None else None,
                                    ctypes.c_void_p(ws.data_ptr()), wsb, ctypes.c_void_p(stream))
    _capi.check(rc, "ccl_fill_holes")
    c = ocounts.cpu()
    nf, eu = int(c[0]), int(c[1])
    if nf < 0:
        raise _capi.CclError(_capi.CCL_ECAPACITY, "ccl_fill_holes (the labeling's tables were truncated)")
    filled = Result(olabels, ofeat[:nf], oparent[:nf], ocolor[:nf], nf, eu)
    return (filled, mp) if return_map else filled


from .batch import BatchPlan, label_batch  # noqa: E402,F401
