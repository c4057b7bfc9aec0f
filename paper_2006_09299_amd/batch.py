"""Batched labeling: many images of uneven sizes in one launch sequence.

Every kernel of the path covers every tile of every image of the batch
(ccl_label_batch); the per-image descriptors live in device memory, so the
whole sequence can be captured once into a HIP graph and replayed.  PyTorch
only provides the memory, the stream and the graph object.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import torch

from . import _capi
from . import Result, _check_image

DEFAULT_CAP_FRACTION = 4  # tables hold w*h/4 + 1024 entries unless told otherwise


def default_cap(w: int, h: int) -> int:
    full = w * h + 1
    return min(full, max(1024, full // DEFAULT_CAP_FRACTION))


class BatchPlan:
    """Outputs, descriptors and workspace for a fixed list of device images.

    launch() enqueues the batch on the current stream; capture() records that
    launch into a HIP graph that replay() runs again (inputs may be rewritten
    in place between replays; shapes and buffers stay fixed)."""

    def __init__(self, imgs: Sequence[torch.Tensor], variant: int = 0, caps: Optional[Sequence[int]] = None,
                 labels: bool = True):
        if len(imgs) == 0:
            raise ValueError("empty batch")
        self.imgs = list(imgs)
        self.variant = int(variant)
        dev = self.imgs[0].device
        n = len(self.imgs)
        self.n = n
        self.shapes = []
        self.labels: List[Optional[torch.Tensor]] = []
        self.features: List[torch.Tensor] = []
        self.parent: List[torch.Tensor] = []
        self.color: List[torch.Tensor] = []
        self.caps = []
        self.counts = torch.zeros((n, 2), dtype=torch.int64, device=dev)
        self.descs = (_capi.ccl_image_t * n)()
        for i, img in enumerate(self.imgs):
            w, h, pitch = _check_image(img)
            if img.device != dev:
                raise ValueError("all images of a batch must be on one device")
            cap = int(caps[i]) if caps is not None else default_cap(w, h)
            lab = torch.empty((h, w), dtype=torch.int32, device=dev) if labels else None
            feat = torch.empty((cap, 5), dtype=torch.int64, device=dev)
            par = torch.empty(cap, dtype=torch.int32, device=dev)
            col = torch.empty(cap, dtype=torch.uint8, device=dev)
            self.shapes.append((h, w))
            self.labels.append(lab)
            self.features.append(feat)
            self.parent.append(par)
            self.color.append(col)
            self.caps.append(cap)
            out = _capi.ccl_outputs_t(lab.data_ptr() if labels else None, feat.data_ptr(), par.data_ptr(),
                                      col.data_ptr(), cap, self.counts[i].data_ptr())
            self.descs[i] = _capi.ccl_image_t(img.data_ptr(), w, h, pitch, out)
        L = _capi.lib()
        db, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _capi.check(L.ccl_batch_sizes(self.descs, n, self.variant, ctypes.byref(db), ctypes.byref(wb)),
                    "ccl_batch_sizes")
        host = torch.empty(db.value, dtype=torch.uint8).pin_memory()
        _capi.check(L.ccl_batch_prepare(self.descs, n, self.variant, ctypes.c_void_p(host.data_ptr()), db.value),
                    "ccl_batch_prepare")
        self.dev_desc = host.to(dev, non_blocking=False)
        self.ws_bytes = wb.value
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)
        self.graph = None

    @property
    def pixels(self) -> int:
        return sum(h * w for h, w in self.shapes)

    def launch(self, stream: Optional[int] = None) -> None:
        if stream is None:
            stream = torch.cuda.current_stream(self.ws.device).cuda_stream
        rc = _capi.lib().ccl_label_batch(self.descs, self.n, self.variant, ctypes.c_void_p(self.dev_desc.data_ptr()),
                                         ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes, ctypes.c_void_p(stream))
        _capi.check(rc, "ccl_label_batch")

    def capture(self) -> None:
        """Record one launch of the batch into a HIP graph (no allocation,
        synchronisation or memset is recorded)."""
        self.launch()  # first launch outside the capture (module load, lazy init)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.launch()
        self.graph = g

    def replay(self) -> None:
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def results(self) -> List[Result]:
        """Synchronise and return per-image results (device tensors).
        Raises CclError(CCL_ECAPACITY) when an image had more labels than its table."""
        counts = self.counts.cpu()
        out = []
        for i in range(self.n):
            nl, eu = int(counts[i, 0]), int(counts[i, 1])
            if nl < 0:  # the kernels refused descriptors placed for another launch shape
                raise _capi.CclError(_capi.CCL_EINVAL, f"image {i}: descriptors do not match the launch")
            if nl > self.caps[i]:
                raise _capi.CclError(_capi.CCL_ECAPACITY, f"image {i}: {nl} labels > cap {self.caps[i]}")
            out.append(Result(self.labels[i], self.features[i][:nl], self.parent[i][:nl], self.color[i][:nl],
                              nl, eu))
        return out


def label_batch(imgs: Sequence[torch.Tensor], variant: Optional[int] = None) -> List[Result]:
    """Label a list of device images in one batched launch sequence; grows
    the tables and reruns the batch if an image had more components.
    variant None: the environment's override (CCL_VARIANT / CCL_TILE), else 0."""
    if variant is None:
        variant = _capi.env_variant()
        variant = 0 if variant is None else variant
    caps = None
    while True:
        plan = BatchPlan(imgs, variant=variant, caps=caps)
        plan.launch()
        counts = plan.counts.cpu()
        need = [max(int(counts[i, 0]), plan.caps[i]) for i in range(plan.n)]
        if need == plan.caps:
            return plan.results()
        caps = need
