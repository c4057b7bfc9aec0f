"""Pins of the oracle under the complementary connectivity pair (4-adjacent
foreground, 8-adjacent background; the note after the unification
algorithm, Sec. 3.2), against facts that do not come from the oracle:
brute-force flood fill and the definition of surrounding on every image of
up to 12 pixels, Gray's bit-quad Euler number for 4-connected foreground,
scipy.ndimage.label partitions and sums, the paper's run-based algorithm with
the widening moved to background runs, and closed forms."""
import itertools

import numpy as np
import pytest

import oracle
from tests import refs

scipy_ndimage = pytest.importorskip("scipy.ndimage")


def _check_small(img):
    r = oracle.label(img, fg8=False)
    lab = refs.flood_label(img, fg8=False)
    assert np.array_equal(r.labels, lab), img
    assert np.array_equal(r.parent, refs.flood_tree(img, lab, fg8=False)), img
    assert r.euler == refs.bitquad_euler4(img), img


@pytest.mark.parametrize("h,w", [(3, 4), (4, 3), (2, 6), (6, 2), (3, 3), (1, 7), (7, 1)])
def test_exhaustive_small_images(h, w):
    for bits in itertools.product((0, 1), repeat=h * w):
        _check_small(np.array(bits, dtype=np.uint8).reshape(h, w))


def test_random_8x8_and_the_papers_algorithm():
    rng = np.random.default_rng(77)
    for _ in range(150):
        h, w = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        img = (rng.random((h, w)) < rng.uniform(0.2, 0.8)).astype(np.uint8)
        _check_small(img)
        lab, T, I, events, F, rows = refs.lsl_bw(img, fg8=False)
        can, mapping = refs.canonicalize(lab)
        r = oracle.label(img, fg8=False)
        assert np.array_equal(r.labels, can)
        for old, new in mapping.items():
            if F[old] is not None:
                assert [r.bbox[new, 0], r.bbox[new, 1], r.bbox[new, 2], r.bbox[new, 3], r.S[new], r.Sx[new],
                        r.Sy[new]] == F[old]


def _same_partition(a, b):
    pairs = set(zip(a.ravel().tolist(), b.ravel().tolist()))
    return len(pairs) == len(set(a.ravel().tolist())) == len(set(b.ravel().tolist()))


@pytest.mark.parametrize("seed", range(4))
def test_scipy_partition_features_and_euler(seed):
    rng = np.random.default_rng(900 + seed)
    h, w = int(rng.integers(50, 300)), int(rng.integers(50, 300))
    img = (rng.random((h, w)) < rng.uniform(0.3, 0.7)).astype(np.uint8)
    r = oracle.label(img, fg8=False)
    cross = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    fgl, nf = scipy_ndimage.label(img != 0, structure=cross)
    bgl, nb = scipy_ndimage.label(np.pad(img == 0, 1, constant_values=True), structure=np.ones((3, 3), int))
    bgl = bgl[1:-1, 1:-1]
    ref = np.where(img != 0, fgl, -bgl)  # one id space: foreground > 0, background < 0
    assert _same_partition(r.labels, ref)
    assert r.euler == refs.bitquad_euler4(img) == nf - (len(np.unique(bgl[img == 0])) - (1 if (r.labels == 0).any() else 0))
    ys, xs = np.mgrid[0:h, 0:w]
    S = np.bincount(r.labels.ravel(), minlength=r.n_labels)
    Sx = np.bincount(r.labels.ravel(), weights=xs.ravel(), minlength=r.n_labels)
    Sy = np.bincount(r.labels.ravel(), weights=ys.ravel(), minlength=r.n_labels)
    assert np.array_equal(S, r.S) and np.array_equal(Sx.astype(np.int64), r.Sx) and np.array_equal(Sy.astype(np.int64), r.Sy)


def test_closed_forms():
    cb = ((np.add.outer(np.arange(5), np.arange(5)) % 2) == 0).astype(np.uint8)
    r = oracle.label(cb, fg8=False)
    assert r.n_labels == 14 and r.euler == 13  # isolated foreground pixels, one background
    cb8 = ((np.add.outer(np.arange(8), np.arange(8)) % 2) == 0).astype(np.uint8)
    assert oracle.label(cb8, fg8=False).euler == 32
    ring = np.ones((7, 9), np.uint8)
    ring[1:-1, 1:-1] = 0
    r = oracle.label(ring, fg8=False)
    assert r.n_labels == 3 and r.euler == 0 and list(r.parent) == [-1, 0, 1]
    diamond = np.zeros((7, 7), np.uint8)  # a diagonal ring: 8-adjacent background leaks through it
    for k in range(4):
        for y, x in ((3 - k, k), (3 + k, k), (3 - k, 6 - k), (3 + k, 6 - k)):
            diamond[y, x] = 1
    r = oracle.label(diamond, fg8=False)
    assert r.euler == refs.bitquad_euler4(diamond) and (r.color == 1).sum() == r.n_labels - 1
    for img, n in ((np.zeros((4, 5), np.uint8), 1), (np.ones((4, 5), np.uint8), 2)):
        assert oracle.label(img, fg8=False).n_labels == n
