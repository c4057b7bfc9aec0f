"""Serving loop with continuous batching: a thin binding of the library's
native server (ccl_server_* in include/ccl.h).

Requests (a host image each) are queued with submit(); every step() is one
ccl_server_poll: the server collects finished micro-batches, admits queued
requests in arrival order while a slot and device memory for their whole
footprint are free in the pool, and launches what it admitted as one
micro-batch (uploads, descriptors, ccl_label_batch) on the next idle one of
its streams.  Results stay in the pool until release().  This module only
marshals arguments and keeps the host images alive while the server needs
them; the pool is a torch allocation so that results are viewed as tensors.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass
from typing import Dict, List, Optional

import torch

from . import Result, _capi

ALIGN = 256
MAX_DONE = 256  # finished requests taken per poll call


@dataclass
class Request:
    rid: int
    img: torch.Tensor          # host uint8 [h, w] (pinned: asynchronous upload)
    arrival: float             # seconds on the server clock
    done: float = 0.0          # when step() saw it finished
    launches: int = 0
    status: int = _capi.CCL_OK
    result: Optional[Result] = None


class Server:
    def __init__(self, budget_bytes: int, max_slots: int = 256, streams: int = 4, variant: int = 0,
                 max_batch: int = 64, cap_divisor: int = 4, device="cuda:0"):
        self.dev = torch.device(device)
        self.pool = torch.empty(int(budget_bytes), dtype=torch.uint8, device=self.dev)
        self.base = self.pool.data_ptr()
        self.max_batch, self.streams = int(max_batch), int(streams)
        cfg = _capi.ccl_server_config_t(int(max_slots), int(streams), int(max_batch), int(variant),
                                        int(cap_divisor))
        h = ctypes.c_void_p()
        torch.cuda.synchronize(self.dev)  # the pool's memory is ready before other streams use it
        _capi.check(_capi.lib().ccl_server_create(ctypes.c_void_p(self.base), self.pool.numel(), ctypes.byref(cfg),
                                                  ctypes.byref(h)), "ccl_server_create")
        self._h = h
        self._done = (_capi.ccl_done_t * MAX_DONE)()
        self.pending: Dict[int, Request] = {}   # submitted, not yet returned by step()
        self.live: Dict[int, Request] = {}      # returned by step(), not yet released
        self.t0 = time.perf_counter()
        self.rejected = 0

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def close(self) -> None:
        if self._h is not None:
            _capi.check(_capi.lib().ccl_server_destroy(self._h), "ccl_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- client side -------------------------------------------------------
    def footprint(self, w: int, h: int) -> int:
        n = ctypes.c_size_t()
        _capi.check(_capi.lib().ccl_server_footprint(self._h, int(w), int(h), ctypes.byref(n)), "ccl_server_footprint")
        return n.value

    def submit(self, rid: int, img: torch.Tensor, arrival: Optional[float] = None) -> None:
        if img.dtype != torch.uint8 or img.dim() != 2 or img.is_cuda or img.stride(1) != 1:
            raise ValueError("requests carry a 2-D uint8 host image with contiguous rows")
        h, w = img.shape
        pitch = img.stride(0) if h > 1 else w
        rc = _capi.lib().ccl_server_submit(self._h, ctypes.c_void_p(img.data_ptr()), int(w), int(h), int(pitch),
                                           int(rid))
        if rc == _capi.CCL_ENOSPC:
            self.rejected += 1
            raise MemoryError(f"request {rid}: footprint above the whole device budget")
        _capi.check(rc, "ccl_server_submit")
        self.pending[rid] = Request(rid, img, self.now() if arrival is None else arrival)

    def release(self, rid: int) -> None:
        """Free the pool memory holding a finished request's results."""
        _capi.check(_capi.lib().ccl_server_release(self._h, int(rid)), "ccl_server_release")
        self.live.pop(rid)

    # -- scheduler ------------------------------------------------------------
    def _view(self, ptr: int, nbytes: int, dtype) -> torch.Tensor:
        off = ptr - self.base
        return self.pool[off:off + nbytes].view(dtype)

    def step(self) -> List[Request]:
        """One scheduling step (never blocks).  Returns the requests that
        finished since the last step, with their results."""
        L = _capi.lib()
        out: List[Request] = []
        while True:
            n = ctypes.c_int32()
            _capi.check(L.ccl_server_poll(self._h, self._done, MAX_DONE, ctypes.byref(n)), "ccl_server_poll")
            t = self.now()
            for d in self._done[:n.value]:
                r = self.pending.pop(d.tag)
                r.done, r.launches, r.status = t, d.launches, d.status
                if d.status == _capi.CCL_OK:
                    nl, h, w, o = d.n_labels, d.h, d.w, d.out
                    r.result = Result(self._view(o.labels, 4 * h * w, torch.int32).view(h, w),
                                      self._view(o.features, 40 * nl, torch.int64).view(nl, 5),
                                      self._view(o.parent, 4 * nl, torch.int32),
                                      self._view(o.color, nl, torch.uint8), nl, d.euler)
                self.live[r.rid] = r
                out.append(r)
            if n.value < MAX_DONE:
                return out

    def stats(self) -> _capi.ccl_server_stats_t:
        st = _capi.ccl_server_stats_t()
        _capi.check(_capi.lib().ccl_server_stats(self._h, ctypes.byref(st)), "ccl_server_stats")
        return st

    def queued(self) -> int:
        return self.stats().queued

    def idle(self) -> bool:
        return not self.pending

    def drain(self) -> List[Request]:
        out = []
        while not self.idle():
            out += self.step()
        return out
