"""Pins of the oracle's hole filling (oracle.fill_holes), the closure's
optional step (Lemaitre & Lacassagne 2020, Sec. 3.2, Algorithm 3; Fig. 2,
"hole filled"), against facts that do not come from the oracle itself:

* the worked example's hole-filled state (Fig. 2 and the Sec. 3.3 text);
* the paper's own closure with the hole-filling test, run literally by the
  independent Python LSL-BW in tests/refs.py, on every 3x3, 3x4 and 4x3
  image and on random small images;
* the definition through a library routine: the complement of the exterior
  (background 4-connected to a padded frame, scipy.ndimage.label) labeled
  with 8-adjacency;
* invariants tying it to the unfilled tree: the filled Euler number is the
  number of top-level foreground components, the areas add up, and closed
  forms for rings, nested rings and checkerboards.
"""
import itertools

import numpy as np
import pytest

import oracle
from tests import golden, refs

scipy_ndimage = pytest.importorskip("scipy.ndimage")


def _same_partition(a, b):
    """a and b label the same partition (bijection of ids)."""
    pairs = set(zip(a.ravel().tolist(), b.ravel().tolist()))
    return len(pairs) == len(set(a.ravel().tolist())) == len(set(b.ravel().tolist()))


def test_fig2_hole_filled_classes():
    img, prov, *_ = golden.fig2()
    f, mp = oracle.fill_holes(img)
    pos = {}
    for lab, r, c in prov:
        pos.setdefault(lab, (r, c))
    for cls in golden.fig2_filled_classes():
        ids = {int(f.labels[pos[lab]]) for lab in cls if lab in pos}
        assert len(ids) == 1, cls
    ext = {int(f.labels[pos[lab]]) for lab in golden.fig2_filled_classes()[0] if lab in pos}
    assert ext == {0}
    assert f.n_labels == 2 and f.euler == 1
    r = oracle.label(img)
    assert sorted(set(mp.tolist())) == [0, 1] and mp[0] == 0


def _lsl_filled(img):
    lab, T, I, events, F, rows = refs.lsl_bw(img, fill_holes=True)
    can, mapping = refs.canonicalize(lab)
    return can, F, T, mapping


@pytest.mark.parametrize("h,w", [(3, 3), (3, 4), (4, 3)])
def test_exhaustive_tiny_equals_the_papers_closure(h, w):
    for bits in itertools.product((0, 1), repeat=h * w):
        img = np.array(bits, dtype=np.uint8).reshape(h, w)
        f, mp = oracle.fill_holes(img)
        can, F, T, mapping = _lsl_filled(img)
        assert np.array_equal(f.labels, can), img


def test_random_small_equal_the_papers_closure_with_features():
    rng = np.random.default_rng(21)
    for _ in range(400):
        h, w = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        img = (rng.random((h, w)) < rng.uniform(0.2, 0.8)).astype(np.uint8)
        f, mp = oracle.fill_holes(img)
        can, F, T, mapping = _lsl_filled(img)
        assert np.array_equal(f.labels, can)
        for old, new in mapping.items():  # features of the closure's roots
            if F[old] is None:
                continue
            assert [f.bbox[new, 0], f.bbox[new, 1], f.bbox[new, 2], f.bbox[new, 3], f.S[new], f.Sx[new],
                    f.Sy[new]] == F[old]


def _filled_by_definition(img):
    """complement of the exterior, labeled 8-adjacent (library routines only)"""
    h, w = img.shape
    bg = np.pad(img == 0, 1, constant_values=True)
    lab4, _ = scipy_ndimage.label(bg, structure=np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]]))
    exterior = (lab4 == lab4[0, 0])[1:-1, 1:-1]
    filled = ~exterior
    lab8, n = scipy_ndimage.label(filled, structure=np.ones((3, 3), dtype=int))
    return lab8, n


@pytest.mark.parametrize("seed", range(6))
def test_definition_through_scipy(seed):
    rng = np.random.default_rng(300 + seed)
    h, w = int(rng.integers(20, 120)), int(rng.integers(20, 120))
    g = int(rng.choice([1, 2, 4]))
    small = (rng.random(((h + g - 1) // g, (w + g - 1) // g)) < rng.uniform(0.3, 0.7)).astype(np.uint8)
    img = np.kron(small, np.ones((g, g), dtype=np.uint8))[:h, :w]
    f, mp = oracle.fill_holes(img)
    lab8, n = _filled_by_definition(img)
    assert _same_partition(f.labels, lab8)
    assert f.n_labels == n + 1 if (lab8 == 0).any() else f.n_labels in (n, n + 1)


@pytest.mark.parametrize("seed", range(4))
def test_invariants_against_the_unfilled_tree(seed):
    rng = np.random.default_rng(500 + seed)
    img = (rng.random((90, 70)) < 0.45).astype(np.uint8)
    r = oracle.label(img)
    f, mp = oracle.fill_holes(img)
    top = [c for c in range(1, r.n_labels) if r.parent[c] == 0]
    assert f.euler == len(top) == f.n_labels - 1
    assert all(r.color[c] == 1 for c in top)
    assert sorted(mp[top].tolist()) == list(range(1, f.n_labels))  # top-level ids keep their order
    for c in range(1, r.n_labels):  # every component ends in its top-level ancestor
        t = c
        while r.parent[t] != 0:
            t = r.parent[t]
        assert mp[c] == mp[t]
    S = np.zeros(f.n_labels, dtype=np.int64)
    np.add.at(S, mp, r.S)
    assert np.array_equal(S, f.S)
    assert (f.parent[1:] == 0).all() and f.parent[0] == -1 and (f.color[1:] == 1).all()


def test_closed_forms():
    ring = np.ones((7, 9), np.uint8)
    ring[1:-1, 1:-1] = 0
    f, _ = oracle.fill_holes(ring)
    assert f.n_labels == 2 and f.euler == 1 and f.S[1] == 63 and f.S[0] == 0
    nested = np.zeros((21, 21), np.uint8)
    for k in range(0, 10, 4):  # three nested rings with background between them
        nested[k:21 - k, k:21 - k] = 1
        nested[k + 1:20 - k, k + 1:20 - k] = 0
    r = oracle.label(nested)
    assert r.n_labels == 7  # exterior, 3 rings, 3 holes
    f, mp = oracle.fill_holes(nested)
    assert f.n_labels == 2 and f.S[1] == 21 * 21 and (mp[1:] == 1).all()
    cb = ((np.add.outer(np.arange(5), np.arange(5)) % 2) == 0).astype(np.uint8)
    f, _ = oracle.fill_holes(cb)
    assert f.n_labels == 2 and f.euler == 1 and f.S[1] == 25 - 8  # border background stays exterior
    for img, n in ((np.zeros((4, 5), np.uint8), 1), (np.ones((4, 5), np.uint8), 2)):
        f, mp = oracle.fill_holes(img)
        assert f.n_labels == n and mp[0] == 0
