"""GPU parity: libccl.so on the MI355X against the CPU oracle, element by element.

Integer outputs, so the bar is bit-exact: labels, features, parent, colour,
number of labels and Euler number.  Sizes span many tiles (and 4 x 4-tile
super-tiles, 8 x 8 on the largest images) with ragged tails; full-size
workloads (all 25 images of the 8192^2 sweep, the 16384^2 structured images)
are compared in full and also checked by size-independent properties."""
import sys

import numpy as np
import pytest

import oracle
import refs
import synth
from golden import fig2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    import paper_2006_09299_amd as ccl
    return ccl


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _run(img, **kw):
    t = torch.from_numpy(np.ascontiguousarray(img)).to(_dev())
    r = _lib().label(t, **kw)
    torch.cuda.synchronize()
    return r


def _assert_same_tables(r, o):
    """Everything but the label image: counts, tree, colour, features."""
    assert r.n_labels == o.n_labels, (r.n_labels, o.n_labels)
    assert r.euler == o.euler
    assert np.array_equal(r.parent.cpu().numpy(), o.parent)
    assert np.array_equal(r.color.cpu().numpy(), o.color)
    assert np.array_equal(r.bbox.cpu().numpy().astype(np.int64), o.bbox)
    assert np.array_equal(r.S.cpu().numpy(), o.S)
    assert np.array_equal(r.Sx.cpu().numpy(), o.Sx)
    assert np.array_equal(r.Sy.cpu().numpy(), o.Sy)


def _assert_same(r, o):
    assert r.n_labels == o.n_labels, (r.n_labels, o.n_labels)
    assert r.euler == o.euler
    assert np.array_equal(r.labels.cpu().numpy(), o.labels)
    assert np.array_equal(r.parent.cpu().numpy(), o.parent)
    assert np.array_equal(r.color.cpu().numpy(), o.color)
    assert np.array_equal(r.bbox.cpu().numpy().astype(np.int64), o.bbox)
    assert np.array_equal(r.S.cpu().numpy(), o.S)
    assert np.array_equal(r.Sx.cpu().numpy(), o.Sx)
    assert np.array_equal(r.Sy.cpu().numpy(), o.Sy)


def _properties(img, r):
    """Checks that hold at any size, computed on the GPU with torch."""
    h, w = img.shape
    n = r.n_labels
    lab = r.labels.reshape(-1).long()
    assert int(lab.min()) >= 0 and int(lab.max()) < n
    S = r.S
    assert int(S.sum()) == h * w
    assert int(r.Sx.sum()) == h * w * (w - 1) // 2
    assert int(r.Sy.sum()) == w * h * (h - 1) // 2
    assert torch.equal(torch.bincount(lab, minlength=n), S)
    # canonical order: first pixel of id k increases with k (k >= 1)
    idx = torch.arange(h * w, device=lab.device)
    first = torch.full((n,), h * w, dtype=torch.long, device=lab.device).scatter_reduce(0, lab, idx, "amin")
    if n > 2:
        assert bool((first[2:] > first[1:-1]).all())
    xs = idx % w
    ys = idx // w
    assert torch.equal(torch.zeros(n, dtype=torch.long, device=lab.device).index_add_(0, lab, xs), r.Sx)
    assert torch.equal(torch.zeros(n, dtype=torch.long, device=lab.device).index_add_(0, lab, ys), r.Sy)
    p = r.parent.long()
    assert int(p[0]) == -1
    if n > 1:
        assert bool(((p[1:] >= 0) & (p[1:] < n)).all())
        col = r.color.long()
        assert bool((col[1:] != col[p[1:]]).all())
    assert r.euler == refs.bitquad_euler8(img)


def test_fig2_example():
    img = fig2()[0]
    _assert_same(_run(img), oracle.label(img))


@pytest.mark.parametrize("seed", range(32))
def test_512_bernoulli_half(seed):
    img = synth.bernoulli_blocks(512, 512, 0.5, 1, seed)
    _say("512x512 p=0.5 seed", seed)
    _assert_same(_run(img), oracle.label(img))


def test_random_shapes_span_tiles_and_tails():
    rng = np.random.default_rng(2024)
    for k in range(40):
        h, w = int(rng.integers(1, 400)), int(rng.integers(1, 700))
        p, g = float(rng.uniform(0.02, 0.98)), int(rng.choice([1, 2, 3, 4, 7, 16]))
        img = synth.bernoulli_blocks(h, w, p, g, 1000 + k)
        _say("random", k, h, w, p, g)
        _assert_same(_run(img), oracle.label(img))


@pytest.mark.parametrize("h,w", [(1, 1), (1, 2), (2, 1), (1, 1000), (1000, 1), (31, 127), (32, 128), (33, 129),
                                 (63, 127), (64, 128), (64, 256), (65, 257), (97, 383), (3, 130), (255, 511),
                                 (256, 512), (257, 513)])
def test_edge_shapes(h, w):
    for p in (0.0, 0.3, 0.6, 1.0):
        img = synth.bernoulli_blocks(h, w, p, 1, h * 7919 + w)
        _say("edge", h, w, p)
        _assert_same(_run(img), oracle.label(img))


def test_degenerate_images():
    cases = {
        "all_bg": np.zeros((100, 300), np.uint8),
        "all_fg": np.ones((100, 300), np.uint8),
        "checker": ((np.add.outer(np.arange(90), np.arange(333)) % 2) == 0).astype(np.uint8),
        "rows": np.tile(np.array([[0], [1]], np.uint8), (50, 257)),
        "cols": np.tile(np.array([[0, 1]], np.uint8), (70, 150)),
        "ring": np.pad(np.zeros((60, 250), np.uint8), 1, constant_values=1),
    }
    nested = np.zeros((301, 301), np.uint8)
    for j in range(30):
        a = 1 + 5 * j
        nested[a:301 - a, a:301 - a] = 1 if j % 2 == 0 else 0
    cases["nested"] = nested
    for name, img in cases.items():
        _say("degenerate", name)
        _assert_same(_run(img), oracle.label(img))


def test_pitch_alignment_and_values():
    img = synth.bernoulli_blocks(200, 301, 0.45, 2, 77)
    o = oracle.label(img)
    dev = _dev()
    for pad in (0, 1, 3, 16, 61):
        big = torch.zeros((200, 301 + pad), dtype=torch.uint8, device=dev)
        big[:, :301] = torch.from_numpy(img * 255).to(dev)
        r = _lib().label(big[:, :301])
        torch.cuda.synchronize()
        _say("pitch pad", pad)
        _assert_same(r, o)
    # offset base pointer (not 16-byte aligned) and arbitrary nonzero values
    rng = np.random.default_rng(5)
    vals = (img * rng.integers(1, 256, size=img.shape)).astype(np.uint8)
    buf = torch.zeros(200 * 301 + 7, dtype=torch.uint8, device=dev)
    buf[7:] = torch.from_numpy(vals.reshape(-1)).to(dev)
    r = _lib().label(buf[7:].view(200, 301))
    torch.cuda.synchronize()
    _assert_same(r, o)


def test_capacity_overflow_then_retry():
    img = synth.bernoulli_blocks(300, 300, 0.5, 1, 9)
    o = oracle.label(img)
    ccl = _lib()
    t = torch.from_numpy(img).to(_dev())
    buf = ccl.Buffers(300, 300, 16, t.device)
    ccl.launch(t, buf)
    torch.cuda.synchronize()
    assert int(buf.counts[0]) == o.n_labels  # true count although the tables hold 16
    assert np.array_equal(buf.labels.cpu().numpy(), o.labels)
    assert np.array_equal(buf.parent[:16].cpu().numpy(), o.parent[:16])
    _assert_same(ccl.label(t, cap=16), o)  # label() grows the tables and reruns


def _features_only(img, o):
    """labels=False: no label image is written; every table must still be
    the oracle's, and it must equal the full path's tables byte for byte."""
    t = torch.from_numpy(np.ascontiguousarray(img)).to(_dev())
    ccl = _lib()
    r = ccl.label(t, cap=o.n_labels, labels=False)
    torch.cuda.synchronize()
    assert r.labels is None
    _assert_same_tables(r, o)
    return r


def test_features_only_mode():
    img = synth.bernoulli_blocks(400, 500, 0.6, 1, 21)
    _features_only(img, oracle.label(img))
    for name, im in (("all_bg", np.zeros((130, 260), np.uint8)), ("all_fg", np.ones((130, 260), np.uint8)),
                     ("checker", ((np.add.outer(np.arange(90), np.arange(333)) % 2) == 0).astype(np.uint8))):
        _say("features-only", name)
        _features_only(im, oracle.label(im))


@pytest.mark.parametrize("p,g", [(0.5, 1), (0.7, 1), (0.5, 16)])
def test_features_only_8192(p, g):
    gi, pi = synth.SWEEP_G.index(g), synth.SWEEP_P.index(p)
    seed = 100 + 5 * gi + pi
    img = synth.bernoulli_blocks(8192, 8192, p, g, seed)
    _say("features-only 8192 p", p, "g", g, "seed", seed)
    _features_only(img, oracle.label(img))


def test_deterministic_repeats():
    img = synth.bernoulli_blocks(1000, 1500, 0.55, 1, 4)
    t = torch.from_numpy(img).to(_dev())
    ccl = _lib()
    ref = ccl.label(t)
    for _ in range(10):
        r = ccl.label(t)
        assert torch.equal(r.labels, ref.labels) and torch.equal(r.features, ref.features)
        assert torch.equal(r.parent, ref.parent) and torch.equal(r.color, ref.color)


@pytest.mark.parametrize("p,g,seed,reps", [(0.3, 4, 111, 6), (0.5, 1, 102, 4), (0.7, 2, 108, 4)])
def test_repeated_full_size_runs_agree_with_oracle(p, g, seed, reps):
    """Races in the union-find show up as run-to-run differences in the
    number of components: compare every repetition with the oracle."""
    img = synth.bernoulli_blocks(8192, 8192, p, g, seed)
    o = oracle.label(img)
    t = torch.from_numpy(img).to(_dev())
    ccl = _lib()
    first = None
    for k in range(reps):
        r = ccl.label(t, cap=o.n_labels)
        torch.cuda.synchronize()
        _say("repeat", p, g, k, r.n_labels, r.euler)
        assert (r.n_labels, r.euler) == (o.n_labels, o.euler)
        if first is None:
            first = r
            _assert_same(r, o)
        else:
            assert torch.equal(r.labels, first.labels) and torch.equal(r.features, first.features)


@pytest.mark.parametrize("p,g", [(p, g) for g in synth.SWEEP_G for p in synth.SWEEP_P])
def test_sweep_8192(p, g):
    """Every image of the benchmarked 8192^2 sweep, element by element."""
    gi, pi = synth.SWEEP_G.index(g), synth.SWEEP_P.index(p)
    seed = 100 + 5 * gi + pi
    img = synth.bernoulli_blocks(8192, 8192, p, g, seed)
    _say("8192 sweep p", p, "g", g, "seed", seed)
    r = _run(img)
    _properties(img, r)
    _assert_same(r, oracle.label(img))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_structured_16384(seed):
    img = synth.structured(16384, 16384, seed=seed)
    _say("16384 structured seed", seed)
    r = _run(img)
    _properties(img, r)
    o = oracle.label(img)
    _assert_same(r, o)
    if seed == 0:  # the benchmarked image, also without the label image
        _say("16384 structured features-only")
        _features_only(img, o)


@pytest.mark.parametrize("h,w,p,g", [(11000, 12000, 0.5, 1), (12288, 12352, 0.3, 4)])
def test_large_ragged_super_tiles(h, w, p, g):
    """Images large enough for super-tiles of 8 x 8 tiles in the single-image
    call, with ragged tiles and super-tiles at the right and bottom edges,
    element by element."""
    from paper_2006_09299_amd import _capi
    assert _capi.variant_for(w, h) == 9 and _capi.variant_info(9)[4] == 8
    img = synth.bernoulli_blocks(h, w, p, g, 31)
    _say("large ragged super-tiles", h, w, p, g)
    r = _run(img)
    _properties(img, r)
    _assert_same(r, oracle.label(img))
