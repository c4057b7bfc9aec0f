"""GPU: hole filling (ccl_fill_holes) against the oracle's hole filling,
bit-exact: filled label image, features, parent, colour, counts and the map
of original ids, on images spanning several tiles with ragged tails, the
worked example, deep nesting, degenerate images, features-only input, table
truncation and at the full 8192 x 8192 size."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import golden

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _check(img, with_labels=True):
    import paper_2006_09299_amd as ccl
    dev = _dev()
    _say("fill", img.shape, "labels" if with_labels else "features only")
    r = ccl.label(torch.from_numpy(img).to(dev), labels=with_labels)
    f, mp = ccl.fill_holes(r, shape=img.shape, return_map=True)
    torch.cuda.synchronize()
    of, omp = oracle.fill_holes(img)
    assert (f.n_labels, f.euler) == (of.n_labels, of.euler)
    if with_labels:
        assert np.array_equal(f.labels.cpu().numpy(), of.labels)
    assert np.array_equal(mp.cpu().numpy(), omp)
    assert np.array_equal(f.bbox.cpu().numpy().astype(np.int64), of.bbox)
    assert np.array_equal(f.S.cpu().numpy(), of.S)
    assert np.array_equal(f.Sx.cpu().numpy(), of.Sx)
    assert np.array_equal(f.Sy.cpu().numpy(), of.Sy)
    assert np.array_equal(f.parent.cpu().numpy(), of.parent)
    assert np.array_equal(f.color.cpu().numpy(), of.color)


def test_fig2_example():
    img, *_ = golden.fig2()
    _check(img)


@pytest.mark.parametrize("seed", range(8))
def test_random_images_span_tiles_and_tails(seed):
    rng = np.random.default_rng(700 + seed)
    h, w = int(rng.integers(1, 700)), int(rng.integers(1, 900))
    img = synth.bernoulli_blocks(h, w, float(rng.uniform(0.2, 0.8)), int(rng.choice([1, 2, 4, 8])), 800 + seed)
    _check(img)


def test_deep_nesting_and_degenerate_images():
    nested = np.zeros((301, 301), np.uint8)
    for k in range(0, 150, 2):  # 75 nested rings, one pixel apart: a chain of depth 150
        nested[k:301 - k, k:301 - k] = 1
        nested[k + 1:300 - k, k + 1:300 - k] = 0
    _check(nested)
    _check(np.zeros((130, 260), np.uint8))
    _check(np.ones((130, 260), np.uint8))
    _check(np.ones((1, 1), np.uint8))
    _check(((np.add.outer(np.arange(67), np.arange(131)) % 2) == 0).astype(np.uint8))


def test_features_only_input():
    img = synth.bernoulli_blocks(300, 500, 0.5, 2, 5)
    _check(img, with_labels=False)


def test_structured_crop():
    img = synth.structured(16384, 16384, seed=1)[4096:6144, 8192:10240].copy()
    _check(img)


def test_small_output_capacity_keeps_true_counts():
    import ctypes

    import paper_2006_09299_amd as ccl
    from paper_2006_09299_amd import _capi
    dev = _dev()
    img = synth.bernoulli_blocks(200, 300, 0.3, 1, 9)
    r = ccl.label(torch.from_numpy(img).to(dev))
    of, _ = oracle.fill_holes(img)
    assert of.n_labels > 40
    n = r.n_labels
    counts_in = torch.tensor([n, r.euler], dtype=torch.int64, device=dev)
    inp = _capi.ccl_outputs_t(r.labels.data_ptr(), r.features.data_ptr(), r.parent.data_ptr(), r.color.data_ptr(), n,
                              counts_in.data_ptr())
    cap = 40
    ofeat = torch.zeros((cap, 5), dtype=torch.int64, device=dev)
    opar = torch.zeros(cap, dtype=torch.int32, device=dev)
    ocol = torch.zeros(cap, dtype=torch.uint8, device=dev)
    oc = torch.zeros(2, dtype=torch.int64, device=dev)
    out = _capi.ccl_outputs_t(None, ofeat.data_ptr(), opar.data_ptr(), ocol.data_ptr(), cap, oc.data_ptr())
    wsb = int(_capi.lib().ccl_fill_workspace_bytes(n))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    rc = _capi.lib().ccl_fill_holes(ctypes.byref(inp), 300, 200, ctypes.byref(out), None, ctypes.c_void_p(ws.data_ptr()),
                                    wsb, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    assert oc.cpu().tolist() == [of.n_labels, of.euler]
    assert np.array_equal(ofeat.view(torch.int32)[:, 0:4].cpu().numpy().astype(np.int64), of.bbox[:cap])
    assert np.array_equal(ofeat[:, 2].cpu().numpy(), of.S[:cap])
    # a truncated labeling is refused on the device: counts[0] = -1
    counts_bad = torch.tensor([n + 5, 0], dtype=torch.int64, device=dev)
    inp_bad = _capi.ccl_outputs_t(r.labels.data_ptr(), r.features.data_ptr(), r.parent.data_ptr(), r.color.data_ptr(),
                                  n, counts_bad.data_ptr())
    rc = _capi.lib().ccl_fill_holes(ctypes.byref(inp_bad), 300, 200, ctypes.byref(out), None,
                                    ctypes.c_void_p(ws.data_ptr()), wsb,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    assert oc.cpu().tolist()[0] == -1


@pytest.mark.parametrize("p,g,seed", [(0.5, 1, 102), (0.3, 4, 111)])
def test_full_size_8192(p, g, seed):
    _check(synth.bernoulli_blocks(8192, 8192, p, g, seed))


def test_label_then_fill_captured_in_one_graph():
    """ccl_label followed by ccl_fill_holes on the same stream needs no host
    synchronisation (the fill reads the label count on the device), so both
    go into one HIP graph; replays with eager work between them, then new
    pixels in the same input buffer."""
    import ctypes

    import paper_2006_09299_amd as ccl
    from paper_2006_09299_amd import _capi
    dev = _dev()
    img = synth.bernoulli_blocks(600, 900, 0.5, 2, 17)
    h, w = img.shape
    t = torch.from_numpy(img).to(dev)
    cap = w * h // 2 + 16
    buf = ccl.Buffers(w, h, cap, dev)
    olab = torch.empty((h, w), dtype=torch.int32, device=dev)
    ofeat = torch.empty((cap, 5), dtype=torch.int64, device=dev)
    opar = torch.empty(cap, dtype=torch.int32, device=dev)
    ocol = torch.empty(cap, dtype=torch.uint8, device=dev)
    oc = torch.zeros(2, dtype=torch.int64, device=dev)
    out = _capi.ccl_outputs_t(olab.data_ptr(), ofeat.data_ptr(), opar.data_ptr(), ocol.data_ptr(), cap, oc.data_ptr())
    wsb = int(_capi.lib().ccl_fill_workspace_bytes(cap))
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)

    def seq():
        ccl.launch(t, buf)
        rc = _capi.lib().ccl_fill_holes(ctypes.byref(buf.out), w, h, ctypes.byref(out), None,
                                        ctypes.c_void_p(ws.data_ptr()), wsb,
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0

    def check(src):
        of, _ = oracle.fill_holes(src)
        n = of.n_labels
        assert oc.cpu().tolist() == [n, of.euler]
        assert np.array_equal(olab.cpu().numpy(), of.labels)
        assert np.array_equal(ofeat[:n, 2].cpu().numpy(), of.S)
        assert np.array_equal(ofeat[:n].view(torch.int32)[:, 0:4].cpu().numpy().astype(np.int64), of.bbox)

    seq()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        seq()
    for rep in range(3):
        junk = torch.randn(1 << 20, device=dev).sum()
        olab.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check(img)
        _say("fill graph replay", rep, "ok", float(junk))
    t.copy_(1 - t)
    g.replay()
    torch.cuda.synchronize()
    check(1 - img)


def test_full_size_structured_16384():
    _check(synth.structured(16384, 16384, seed=0))
