"""Serving loop with continuous batching over the batched labeling path.

Requests (a host image each) arrive over time.  The scheduler admits them in
arrival order as soon as a slot and device memory for their whole footprint
(input, label image, tables, share of the workspace) are free in a fixed
device pool, groups everything admitted at one scheduling step into a
micro-batch, and enqueues that micro-batch (host-to-device copies, descriptor
upload, ccl_label_batch) on the next of several streams, so that work
admitted while earlier micro-batches still run overlaps with them on the
device.  Results (label image, features, tree) stay in device memory until
the caller releases them; completion is observed through stream events.
"""
from __future__ import annotations

import ctypes
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Deque, Dict, List, Optional, Tuple

import numpy as np
import torch

from . import Result, _capi
from .batch import default_cap

ALIGN = 256


class DevicePool:
    """First-fit sub-allocator over one device buffer (offsets, 256-byte aligned)."""

    def __init__(self, nbytes: int, device):
        self.size = int(nbytes)
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.base = self.buf.data_ptr()
        self.free: List[Tuple[int, int]] = [(0, self.size)]  # sorted (offset, size)
        self.used = 0

    def alloc(self, n: int) -> Optional[int]:
        n = (int(n) + ALIGN - 1) // ALIGN * ALIGN
        for i, (off, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, sz - n)
                self.used += n
                return off
        return None

    def release(self, off: int, n: int) -> None:
        n = (int(n) + ALIGN - 1) // ALIGN * ALIGN
        self.used -= n
        self.free.append((off, n))
        self.free.sort()
        merged: List[Tuple[int, int]] = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged

    def view(self, off: int, n: int, dtype=torch.uint8) -> torch.Tensor:
        t = self.buf[off:off + n]
        return t.view(dtype) if dtype != torch.uint8 else t


@dataclass
class Request:
    rid: int
    img: torch.Tensor          # host uint8 [h, w], pinned for asynchronous upload
    arrival: float             # seconds on the server clock
    admitted: float = 0.0
    done: float = 0.0
    cap: int = 0
    blocks: List[Tuple[int, int]] = field(default_factory=list)  # pool (offset, bytes)
    result: Optional[Result] = None


@dataclass
class _Micro:
    reqs: List[Request]
    event: torch.cuda.Event
    ws: Tuple[int, int]
    desc: Tuple[int, int]
    counts: torch.Tensor
    stream: torch.cuda.Stream
    keep: list


class Server:
    def __init__(self, budget_bytes: int, max_slots: int = 256, streams: int = 4, variant: int = 0,
                 max_batch: int = 64, device="cuda:0"):
        self.dev = torch.device(device)
        self.pool = DevicePool(budget_bytes, self.dev)
        self.max_slots = max_slots
        self.max_batch = max_batch
        self.variant = variant
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(streams)]
        self.next_stream = 0
        self.queue: Deque[Request] = deque()
        self.inflight: List[_Micro] = []
        self.live: Dict[int, Request] = {}      # admitted, not yet released
        self.t0 = time.perf_counter()
        self.rejected = 0
        self.admitted = 0
        self.completed = 0

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- client side -------------------------------------------------------
    def submit(self, rid: int, img: torch.Tensor, arrival: Optional[float] = None) -> None:
        if img.dtype != torch.uint8 or img.dim() != 2 or img.is_cuda:
            raise ValueError("requests carry a 2-D uint8 host image")
        h, w = img.shape
        if self.footprint(w, h) > self.pool.size:
            self.rejected += 1
            raise MemoryError(f"request {rid}: footprint above the whole device budget")
        self.queue.append(Request(rid, img, self.now() if arrival is None else arrival))

    def release(self, rid: int) -> None:
        """Free the device memory holding a finished request's results."""
        r = self.live.pop(rid)
        for off, n in r.blocks:
            self.pool.release(off, n)
        r.blocks = []

    # -- footprint ----------------------------------------------------------
    @staticmethod
    def _request_bytes(w: int, h: int, cap: int) -> List[int]:
        return [h * w, 4 * h * w, 40 * cap, 4 * cap, cap]  # input, labels, features, parent, colour

    def footprint(self, w: int, h: int) -> int:
        cap = default_cap(w, h)
        ws = _capi.workspace_bytes(w, h, self.variant)
        return sum((b + ALIGN - 1) // ALIGN * ALIGN for b in self._request_bytes(w, h, cap)) + ws + 4 * ALIGN

    # -- scheduler ------------------------------------------------------------
    def _admit(self, r: Request) -> bool:
        h, w = r.img.shape
        r.cap = default_cap(w, h)
        got = []
        for n in self._request_bytes(w, h, r.cap):
            off = self.pool.alloc(n)
            if off is None:
                for o, m in got:
                    self.pool.release(o, m)
                return False
            got.append((off, n))
        r.blocks = got
        return True

    def _launch(self, batch: List[Request]) -> bool:
        n = len(batch)
        descs = (_capi.ccl_image_t * n)()
        counts_blk = self.pool.alloc(16 * n)
        if counts_blk is None:
            return False
        counts = self.pool.view(counts_blk, 16 * n, torch.int64).view(n, 2)
        keep = []
        for i, r in enumerate(batch):
            h, w = r.img.shape
            (o_in, _), (o_lab, _), (o_f, _), (o_p, _), (o_c, _) = r.blocks
            b = self.pool.base
            out = _capi.ccl_outputs_t(b + o_lab, b + o_f, b + o_p, b + o_c, r.cap, counts[i].data_ptr())
            descs[i] = _capi.ccl_image_t(b + o_in, w, h, w, out)
        L = _capi.lib()
        db, wb = ctypes.c_size_t(), ctypes.c_size_t()
        _capi.check(L.ccl_batch_sizes(descs, n, self.variant, ctypes.byref(db), ctypes.byref(wb)), "ccl_batch_sizes")
        ws_off = self.pool.alloc(wb.value)
        desc_off = self.pool.alloc(db.value) if ws_off is not None else None
        if ws_off is None or desc_off is None:
            if ws_off is not None:
                self.pool.release(ws_off, wb.value)
            self.pool.release(counts_blk, 16 * n)
            return False
        host_desc = torch.empty(db.value, dtype=torch.uint8).pin_memory()
        _capi.check(L.ccl_batch_prepare(descs, n, self.variant, ctypes.c_void_p(host_desc.data_ptr()), db.value),
                    "ccl_batch_prepare")
        keep.append(host_desc)
        s = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        with torch.cuda.stream(s):
            for r in batch:
                h, w = r.img.shape
                o_in = r.blocks[0][0]
                self.pool.view(o_in, h * w).view(h, w).copy_(r.img, non_blocking=True)
            self.pool.view(desc_off, db.value).copy_(host_desc, non_blocking=True)
            rc = L.ccl_label_batch(descs, n, self.variant, ctypes.c_void_p(self.pool.base + desc_off),
                                   ctypes.c_void_p(self.pool.base + ws_off), wb.value, ctypes.c_void_p(s.cuda_stream))
            _capi.check(rc, "ccl_label_batch")
            ev = torch.cuda.Event()
            ev.record(s)
        keep.append(descs)
        self.inflight.append(_Micro(batch, ev, (ws_off, wb.value), (desc_off, db.value), counts, s, keep))
        self._counts_blocks = getattr(self, "_counts_blocks", {})
        self._counts_blocks[id(self.inflight[-1])] = (counts_blk, 16 * n)
        return True

    def step(self) -> List[Request]:
        """Admit what fits, launch it as one micro-batch, collect finished
        micro-batches.  Returns the requests completed in this step."""
        now = self.now()
        batch: List[Request] = []
        while (self.queue and self.queue[0].arrival <= now and len(batch) < self.max_batch
               and len(self.live) < self.max_slots):
            r = self.queue[0]
            if not self._admit(r):
                break
            self.queue.popleft()
            r.admitted = now
            self.live[r.rid] = r
            batch.append(r)
        if batch and not self._launch(batch):
            # no room for the micro-batch scratch: give the requests back to the queue head
            for r in reversed(batch):
                self.live.pop(r.rid)
                for off, n in r.blocks:
                    self.pool.release(off, n)
                r.blocks = []
                self.queue.appendleft(r)
            batch = []
        self.admitted += len(batch)
        done: List[Request] = []
        still = []
        for m in self.inflight:
            if not m.event.query():
                still.append(m)
                continue
            t = self.now()
            counts = m.counts.cpu()
            for i, r in enumerate(m.reqs):
                h, w = r.img.shape
                nl, eu = int(counts[i, 0]), int(counts[i, 1])
                if nl > r.cap:  # rare: more components than the table; label it alone
                    r.result = self._relabel_alone(r, nl)
                else:
                    b = r.blocks
                    lab = self.pool.view(b[1][0], 4 * h * w, torch.int32).view(h, w)
                    feat = self.pool.view(b[2][0], 40 * r.cap, torch.int64).view(r.cap, 5)[:nl]
                    par = self.pool.view(b[3][0], 4 * r.cap, torch.int32)[:nl]
                    col = self.pool.view(b[4][0], r.cap)[:nl]
                    r.result = Result(lab, feat, par, col, nl, eu)
                r.done = t
                done.append(r)
            self.pool.release(*m.ws)
            self.pool.release(*m.desc)
            self.pool.release(*self._counts_blocks.pop(id(m)))
        self.inflight = still
        self.completed += len(done)
        return done

    def _relabel_alone(self, r: Request, n_labels: int) -> Result:
        from . import label
        res = label(r.img.to(self.dev), cap=n_labels)
        torch.cuda.synchronize()
        return res

    def idle(self) -> bool:
        return not self.queue and not self.inflight

    def drain(self) -> List[Request]:
        out = []
        while not self.idle():
            out += self.step()
        return out
