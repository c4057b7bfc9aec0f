"""The single-thread host LSL-BW (liblslbw.so: the paper's Algorithms 1-4 on
the CPU) against the oracle, bit-exact: labels, features, tree, colour,
counts, Euler number, for both connectivity pairs and with hole filling.
No GPU is involved."""
import numpy as np
import pytest

import oracle
import synth
from golden import fig2
from paper_2006_09299_amd import lslbw

ALL = lslbw.FEATURES | lslbw.RELABEL | lslbw.EULER


def _same(r, o):
    assert r.n_labels == o.n_labels, (r.n_labels, o.n_labels)
    assert r.euler == o.euler
    assert np.array_equal(r.labels, o.labels)
    assert np.array_equal(r.parent, o.parent)
    assert np.array_equal(r.color, o.color)
    assert np.array_equal(r.features[:, :4], o.bbox)
    assert np.array_equal(r.features[:, 4], o.S)
    assert np.array_equal(r.features[:, 5], o.Sx)
    assert np.array_equal(r.features[:, 6], o.Sy)


SHAPES = [(1, 1), (1, 37), (37, 1), (2, 2), (3, 5), (8, 8), (31, 64), (64, 77), (129, 257), (300, 200)]


@pytest.mark.parametrize("h,w", SHAPES)
@pytest.mark.parametrize("p,g", [(0.1, 1), (0.5, 1), (0.7, 1), (0.5, 2), (0.3, 4), (0.9, 1)])
def test_random_images_match_oracle(h, w, p, g):
    for seed in range(3):
        img = synth.bernoulli_blocks(h, w, p, g, seed)
        _same(lslbw.label(img, ALL), oracle.label(img))


@pytest.mark.parametrize("h,w", [(5, 7), (64, 77), (200, 300)])
def test_complementary_pair_matches_oracle(h, w):
    for seed in range(4):
        img = synth.bernoulli_blocks(h, w, 0.5, 1 + seed % 2, seed)
        _same(lslbw.label(img, ALL | lslbw.FG4), oracle.label(img, fg8=False))


@pytest.mark.parametrize("h,w", [(4, 4), (64, 77), (257, 129)])
def test_hole_filling_matches_oracle(h, w):
    for seed in range(4):
        img = synth.bernoulli_blocks(h, w, (0.3, 0.5, 0.7, 0.6)[seed], 1, seed)
        f, _ = oracle.fill_holes(img)
        _same(lslbw.label(img, ALL | lslbw.FILL), f)


def test_fig2_example():
    img = fig2()[0]
    _same(lslbw.label(img, ALL), oracle.label(img))
    f, _ = oracle.fill_holes(img)
    _same(lslbw.label(img, ALL | lslbw.FILL), f)


def test_degenerate_images_and_table_growth():
    # the checkerboard has a label per pixel: far beyond the initial table
    # room of w*h/4 + w + 2 labels, so the tables grow during the scan
    imgs = [np.zeros((40, 70), np.uint8), np.ones((40, 70), np.uint8),
            ((np.add.outer(np.arange(90), np.arange(133)) % 2) == 0).astype(np.uint8),
            np.tile(np.array([[1], [0]], np.uint8), (20, 33)), np.tile(np.array([[1, 0]], np.uint8), (17, 20))]
    for img in imgs:
        _same(lslbw.label(img, ALL), oracle.label(img))
        _same(lslbw.label(img, ALL | lslbw.FG4), oracle.label(img, fg8=False))


def test_nonbinary_values_and_strided_rows():
    rng = np.random.default_rng(5)
    big = rng.integers(0, 256, size=(120, 300), dtype=np.uint8)
    big[rng.random(big.shape) < 0.5] = 0
    img = big[:, 17:217]  # rows strided by 300 bytes, values 1..255 are foreground
    _same(lslbw.label(img, ALL), oracle.label(np.ascontiguousarray(img)))


def test_flags_select_outputs():
    img = synth.bernoulli_blocks(100, 150, 0.5, 1, 9)
    o = oracle.label(img)
    ctx = lslbw.Context(150, 100)
    base = ctx.label(img, 0)  # B&W labels + adjacency tree only
    assert base.labels is None and base.features is None and base.euler == 0
    assert base.n_labels == o.n_labels
    assert np.array_equal(base.parent, o.parent) and np.array_equal(base.color, o.color)
    e = ctx.label(img, lslbw.EULER)
    assert e.euler == o.euler
    r = ctx.label(img, lslbw.RELABEL)
    assert np.array_equal(r.labels, o.labels) and r.features is None
    # the same context again, and a table capacity below the label count:
    # counts stay true, tables hold the first entries
    small = ctx.label(img, ALL, cap=10)
    assert small.n_labels == o.n_labels and np.array_equal(small.parent, o.parent[:10])
    assert base.tsc > 0 and base.ns > 0
    ctx.close()


def test_argument_errors():
    lib = lslbw._load()
    import ctypes
    p = ctypes.c_void_p()
    assert lib.lslbw_create(0, 5, ctypes.byref(p)) == -1
    assert lib.lslbw_create(5, -1, ctypes.byref(p)) == -1
    ctx = lslbw.Context(8, 4)
    img = np.zeros((4, 8), np.uint8)
    counts = np.zeros(2, np.int64)
    # pitch below the width, unknown flag bits, null image
    assert lib.lslbw_label(ctx.ptr, img.ctypes.data, 7, 0, None, None, None, None, 0, counts.ctypes.data, None) == -1
    assert lib.lslbw_label(ctx.ptr, img.ctypes.data, 8, 64, None, None, None, None, 0, counts.ctypes.data, None) == -1
    assert lib.lslbw_label(ctx.ptr, None, 8, 0, None, None, None, None, 0, counts.ctypes.data, None) == -1
    with pytest.raises(ValueError):
        ctx.label(np.zeros((5, 8), np.uint8))
    ctx.close()
