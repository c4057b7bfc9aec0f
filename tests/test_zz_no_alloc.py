"""ccl_label_noalloc (the entry point for callers that cannot allocate: its
workspace is the library's static per-GPU array) against ccl_label, through
the C-ABI, bit-exact on every output: two calls in a row on one stream, the
second with a smaller image, and the size limit."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


class _Out:
    """Device outputs of one w x h image and their ccl_outputs_t."""

    def __init__(self, w, h, cap, dev):
        from paper_2006_09299_amd import _capi
        self.labels = torch.full((h, w), -7, dtype=torch.int32, device=dev)
        self.feat = torch.full((cap, 5), -7, dtype=torch.int64, device=dev)
        self.parent = torch.full((cap,), -7, dtype=torch.int32, device=dev)
        self.color = torch.full((cap,), 7, dtype=torch.uint8, device=dev)
        self.counts = torch.full((2,), -7, dtype=torch.int64, device=dev)
        self.out = _capi.ccl_outputs_t(self.labels.data_ptr(), self.feat.data_ptr(), self.parent.data_ptr(),
                                       self.color.data_ptr(), cap, self.counts.data_ptr())

    def same(self, other, n):
        assert torch.equal(self.counts, other.counts)
        assert torch.equal(self.labels, other.labels)
        assert torch.equal(self.feat[:n], other.feat[:n])
        assert torch.equal(self.parent[:n], other.parent[:n])
        assert torch.equal(self.color[:n], other.color[:n])


def _label_both(img, stream):
    from paper_2006_09299_amd import _capi
    L = _capi.lib()
    dev = _dev()
    h, w = img.shape
    t = torch.from_numpy(np.ascontiguousarray(img)).to(dev)
    cap = w * h // 2 + 16
    ref, na = _Out(w, h, cap, dev), _Out(w, h, cap, dev)
    wsb = _capi.workspace_bytes(w, h)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    sp = ctypes.c_void_p(stream.cuda_stream)
    _capi.check(L.ccl_label(t.data_ptr(), w, h, w, ctypes.byref(ref.out), ws.data_ptr(), wsb, sp), "ccl_label")
    _capi.check(L.ccl_label_noalloc(t.data_ptr(), w, h, w, ctypes.byref(na.out), sp), "ccl_label_noalloc")
    return t, ref, na


def test_noalloc_matches_ccl_label_twice_then_smaller():
    dev = _dev()
    stream = torch.cuda.current_stream(dev)
    cases = [synth.bernoulli_blocks(3000, 2900, 0.5, 1, 41), synth.bernoulli_blocks(700, 1100, 0.4, 2, 42)]
    for k, img in enumerate(cases):
        _say("noalloc call", k, img.shape)
        _, ref, na = _label_both(img, stream)
        torch.cuda.synchronize()
        n = int(ref.counts[0].item())
        na.same(ref, n)
        if k == 1:  # the smaller one also against the oracle
            o = oracle.label(img)
            assert n == o.n_labels
            assert np.array_equal(na.labels.cpu().numpy(), o.labels)
            assert np.array_equal(na.parent[:n].cpu().numpy(), o.parent)


def test_noalloc_back_to_back_on_one_stream():
    """Two calls enqueued before any synchronisation (ordered on the stream,
    sharing the array), each equal to ccl_label's result."""
    from paper_2006_09299_amd import _capi
    L = _capi.lib()
    dev = _dev()
    stream = torch.cuda.current_stream(dev)
    sp = ctypes.c_void_p(stream.cuda_stream)
    imgs = [synth.bernoulli_blocks(2048, 2048, 0.6, 1, 43), synth.bernoulli_blocks(513, 1025, 0.5, 4, 44)]
    ts = [torch.from_numpy(im).to(dev) for im in imgs]
    outs = []
    for t in ts:
        h, w = t.shape
        o = _Out(w, h, w * h // 2 + 16, dev)
        _capi.check(L.ccl_label_noalloc(t.data_ptr(), w, h, w, ctypes.byref(o.out), sp), "ccl_label_noalloc")
        outs.append(o)
    torch.cuda.synchronize()
    for img, o in zip(imgs, outs):
        _, ref, _ = _label_both(img, stream)
        torch.cuda.synchronize()
        o.same(ref, int(ref.counts[0].item()))


def test_noalloc_size_limit():
    from paper_2006_09299_amd import _capi
    L = _capi.lib()
    dev = _dev()
    # the largest square image that fits, and one row more than that fits
    side = 4096
    assert _capi.workspace_bytes(side, side) <= _capi.NOALLOC_SCRATCH_BYTES
    big_h = side
    while _capi.workspace_bytes(side, big_h) <= _capi.NOALLOC_SCRATCH_BYTES:
        big_h += 64
    t = torch.zeros((1, 1), dtype=torch.uint8, device=dev)
    o = _Out(1, 1, 4, dev)
    sp = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    # refused on the host before anything is enqueued (the pointer is never read)
    assert L.ccl_label_noalloc(t.data_ptr(), side, big_h, side, ctypes.byref(o.out), sp) == _capi.CCL_ENOSPC
    assert L.ccl_label_noalloc(None, 8, 8, 8, ctypes.byref(o.out), sp) == _capi.CCL_EINVAL
    img = synth.bernoulli_blocks(side, side, 0.5, 1, 45)
    _say("noalloc at the limit", img.shape)
    _, ref, na = _label_both(img, torch.cuda.current_stream(dev))
    torch.cuda.synchronize()
    na.same(ref, int(ref.counts[0].item()))
