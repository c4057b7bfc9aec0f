"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Every check here uses something other than the oracle itself: the Fig. 2
example printed in the paper, brute-force flood fill, the definition of
"surrounded", Gray's bit-quad Euler number, scipy's labeling routine, the
paper's own run-based algorithm, closed forms and sum invariants.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle
import refs
import synth
from golden import fig2


def _all_images(h, w):
    n = h * w
    for bits in range(1 << n):
        yield np.array([(bits >> k) & 1 for k in range(n)], dtype=np.uint8).reshape(h, w)


def _feature_sums_ok(img, r):
    h, w = img.shape
    assert r.S.sum() == h * w
    assert r.Sx.sum() == h * w * (w - 1) // 2
    assert r.Sy.sum() == w * h * (h - 1) // 2


def _tree_invariants(r):
    n = r.n_labels
    assert r.parent[0] == -1 and r.color[0] == 0
    if n > 1:
        p = r.parent[1:]
        assert np.all((p >= 0) & (p < n))
        # colours alternate along every tree edge
        assert np.all(r.color[1:] != r.color[p])
        # a component's first pixel comes after its parent's first pixel in
        # raster order, or the parent is the exterior
        assert np.all((p == 0) | (p < np.arange(1, n)))
    # depth parity equals colour: foreground at odd depth, holes at even depth
    depth = np.zeros(n, dtype=np.int64)
    for c in range(1, n):
        depth[c] = depth[r.parent[c]] + 1
    assert np.all(depth[1:] % 2 == r.color[1:])


# ---------------------------------------------------------------------------
# Fig. 2 worked example (Sec. 3.3)


def test_fig2_oracle_matches_paper_example():
    img, prov, new, equiv, final, classes = fig2()
    r = oracle.label(img)
    assert r.n_labels == 3  # the three classes of the final state
    # every printed provisional label lands in its final class
    cls_of = {}
    for ci, members in enumerate(classes):
        for lab in members:
            cls_of[lab] = ci
    canon_of_class = {}
    for lab, y, x in prov:
        c = int(r.labels[y, x])
        ci = cls_of[lab]
        assert canon_of_class.setdefault(ci, c) == c
    assert len(set(canon_of_class.values())) == 3
    ext, fgc, hole = canon_of_class[0], canon_of_class[1], canon_of_class[2]
    assert ext == 0
    assert r.color[fgc] == 1 and r.color[hole] == 0
    # the surviving surroundings of the final state: 6 in 4 (class of 1), 1 in 0
    assert r.parent[hole] == fgc and r.parent[fgc] == 0
    assert r.euler == 1 - 1  # one foreground component with one hole
    assert r.euler == refs.bitquad_euler8(img)
    _feature_sums_ok(img, r)


def test_fig2_run_based_reference_reproduces_paper_narrative():
    img, prov, new, equiv, final, classes = fig2()
    lab, T, I, events, F, rows = refs.lsl_bw(img)
    got_new = [(e[1], e[2], e[3], e[4]) for e in events if e[0] == "new"]
    assert got_new == new
    got_eq = [(e[1], e[2], e[3]) for e in events if e[0] == "equiv"]
    # same rows, same classes (the paper's text and figure differ on the
    # representative of the exterior class at row 5)
    assert [g[0] for g in got_eq] == [q[0] for q in equiv]
    cls = {m: i for i, c in enumerate(classes) for m in c}
    for g, q in zip(got_eq, equiv):
        assert {cls[g[1]], cls[g[2]]} == {cls[q[1]], cls[q[2]]}
    # provisional labels at the printed positions
    for labv, y, x in prov:
        runs, era = rows[y]
        k = next(k for k, (j0, j1) in enumerate(runs) if j0 <= x < j1)
        assert era[k] == labv
    # final surroundings on roots after the closure
    roots = [e for e in range(len(T)) if T[e] == e]
    assert roots == [0, 1, 6]
    for child, par in final:
        assert I[child] == T[par]


# ---------------------------------------------------------------------------
# Brute force on tiny images


@pytest.mark.parametrize("shape", [(1, k) for k in range(1, 9)] + [(k, 1) for k in range(2, 9)]
                         + [(2, 2), (2, 3), (3, 2), (2, 4), (4, 2), (2, 8), (8, 2), (3, 3)])
def test_exhaustive_small_labels_tree_euler(shape):
    for img in _all_images(*shape):
        r = oracle.label(img)
        exp = refs.flood_label(img)
        assert np.array_equal(r.labels, exp)
        assert np.array_equal(r.parent, refs.flood_tree(img, exp))
        assert r.euler == refs.bitquad_euler8(img)
        _feature_sums_ok(img, r)


@pytest.mark.parametrize("shape", [(3, 4), (4, 3)])
def test_exhaustive_3x4_labels_tree(shape):
    for img in _all_images(*shape):
        r = oracle.label(img)
        exp = refs.flood_label(img)
        assert np.array_equal(r.labels, exp)
        assert np.array_equal(r.parent, refs.flood_tree(img, exp))
        assert r.euler == refs.bitquad_euler8(img)


def test_exhaustive_4x4_labels_euler():
    for img in _all_images(4, 4):
        r = oracle.label(img)
        assert np.array_equal(r.labels, refs.flood_label(img))
        assert r.euler == refs.bitquad_euler8(img)


def test_random_small_tree_by_definition():
    rng = np.random.default_rng(1234)
    for _ in range(150):
        h, w = rng.integers(2, 9, size=2)
        img = (rng.random((h, w)) < rng.uniform(0.2, 0.8)).astype(np.uint8)
        r = oracle.label(img)
        exp = refs.flood_label(img)
        assert np.array_equal(r.labels, exp)
        assert np.array_equal(r.parent, refs.flood_tree(img, exp))
        _tree_invariants(r)


# ---------------------------------------------------------------------------
# The paper's own run-based algorithm (with the four-sided exterior reading)


def test_run_based_reference_agrees_on_random_images():
    rng = np.random.default_rng(99)
    for _ in range(300):
        h, w = rng.integers(1, 17, size=2)
        g = int(rng.choice([1, 2, 3]))
        img = synth.bernoulli_blocks(int(h), int(w), float(rng.uniform(0.1, 0.9)), g,
                                     int(rng.integers(1 << 30)))
        r = oracle.label(img)
        lab, T, I, events, F, rows = refs.lsl_bw(img)
        can, mapping = refs.canonicalize(lab, exterior=0)
        assert np.array_equal(can, r.labels)
        n = r.n_labels
        for root, cid in mapping.items():
            f = F[root]
            if cid == 0 and f is None:
                continue
            assert [r.bbox[cid, 0], r.bbox[cid, 1], r.bbox[cid, 2], r.bbox[cid, 3],
                    r.S[cid], r.Sx[cid], r.Sy[cid]] == f
            if cid != 0:
                assert r.parent[cid] == mapping[I[root]]
        assert len(mapping) == n


def test_literal_epilog_misses_bottom_border():
    """Reading of the exterior: with only the first/last background run of
    each row attached, a background pocket open to the bottom edge would be
    called a hole, contradicting the definition of surrounding."""
    img = np.array([[1, 1, 1], [1, 0, 1]], dtype=np.uint8)
    lab, T, I, *_ = refs.lsl_bw(img, fix_bottom=False)
    assert lab[1, 1] != 0  # the literal epilog leaves the pocket apart
    r = oracle.label(img)
    assert r.labels[1, 1] == 0  # the pocket touches the frame: exterior
    assert r.n_labels == 2 and r.euler == 1


# ---------------------------------------------------------------------------
# Library routine: scipy.ndimage.label partitions


def _same_partition(a, b):
    """True when label arrays a and b (same shape) induce the same partition."""
    a = a.ravel().astype(np.int64)
    b = b.ravel().astype(np.int64)
    pairs = np.unique(np.stack([a, b], axis=1), axis=0)
    return len(pairs) == len(np.unique(a)) == len(np.unique(b))


@pytest.mark.parametrize("h,w,p,g,seed", [(64, 64, 0.5, 1, 1), (64, 97, 0.3, 1, 2), (97, 64, 0.7, 2, 3),
                                          (256, 256, 0.45, 1, 4), (200, 300, 0.6, 4, 5),
                                          (1024, 1024, 0.5, 1, 6)])
def test_partition_matches_scipy(h, w, p, g, seed):
    img = synth.bernoulli_blocks(h, w, p, g, seed)
    r = oracle.label(img)
    fg = img != 0
    sl, nf = ndimage.label(fg, structure=np.ones((3, 3), dtype=int))
    # background: 4-connected, with a 1-px background frame joining the border
    pad = np.pad(~fg, 1, constant_values=True)
    bl, nb = ndimage.label(pad, structure=ndimage.generate_binary_structure(2, 1))
    bl = bl[1:-1, 1:-1]
    assert _same_partition(r.labels[fg], sl[fg])
    assert _same_partition(r.labels[~fg], bl[~fg])
    # component counts: the padded frame makes scipy's exterior one of its nb
    # background components, present even when no background touches the border
    assert r.n_labels == 1 + nf + (nb - 1)
    assert r.euler == nf - (nb - 1)
    # features of the library's objects
    objs = ndimage.find_objects(r.labels)  # slice k-1 is the box of id k
    for k, sl_ in enumerate(objs):
        if sl_ is None:
            continue
        cid = k + 1
        ys, xs = sl_
        assert (r.bbox[cid, 2], r.bbox[cid, 3] + 1) == (ys.start, ys.stop)
        assert (r.bbox[cid, 0], r.bbox[cid, 1] + 1) == (xs.start, xs.stop)
    idx = np.arange(r.n_labels)
    area = ndimage.sum_labels(np.ones_like(r.labels), r.labels, idx)
    assert np.array_equal(area.astype(np.int64), r.S)
    yy, xx = np.mgrid[0:h, 0:w]
    assert np.array_equal(ndimage.sum_labels(xx, r.labels, idx).astype(np.int64), r.Sx)
    assert np.array_equal(ndimage.sum_labels(yy, r.labels, idx).astype(np.int64), r.Sy)
    _feature_sums_ok(img, r)
    _tree_invariants(r)


# ---------------------------------------------------------------------------
# Closed forms


def test_all_background():
    for h, w in [(1, 1), (3, 5), (64, 64)]:
        r = oracle.label(np.zeros((h, w), np.uint8))
        assert r.n_labels == 1 and r.S[0] == h * w and r.euler == 0
        assert list(r.bbox[0]) == [0, w - 1, 0, h - 1]


def test_all_foreground_empty_exterior():
    for h, w in [(1, 1), (4, 7), (64, 64)]:
        r = oracle.label(np.ones((h, w), np.uint8))
        assert r.n_labels == 2 and r.S[0] == 0 and r.S[1] == h * w
        assert r.parent[1] == 0 and r.color[1] == 1 and r.euler == 1
        assert list(r.bbox[0]) == [2**31 - 1, -1, 2**31 - 1, -1]
        assert r.Sx[1] == h * w * (w - 1) // 2


def test_ring():
    for h, w in [(3, 3), (5, 9), (40, 33)]:
        img = np.ones((h, w), np.uint8)
        img[1:-1, 1:-1] = 0
        r = oracle.label(img)
        assert r.n_labels == 3 and r.euler == 0
        assert r.S[2] == (h - 2) * (w - 2) and r.parent[2] == 1 and r.parent[1] == 0
        assert r.S[0] == 0


@pytest.mark.parametrize("n,m,expect", [(5, 5, -3), (8, 8, -17), (2, 2, 1), (7, 4, None)])
def test_checkerboard(n, m, expect):
    img = ((np.add.outer(np.arange(n), np.arange(m)) % 2) == 0).astype(np.uint8)
    r = oracle.label(img)
    bg = img == 0
    inner = bg.copy()
    inner[0, :] = inner[-1, :] = inner[:, 0] = inner[:, -1] = False
    holes = int(inner.sum())
    assert r.euler == 1 - holes
    if expect is not None:
        assert r.euler == expect
    assert int(r.color.sum()) == 1  # one 8-connected foreground component
    assert r.n_labels == 2 + holes


def test_nested_rings_chain():
    for k in (1, 2, 3, 5):
        s = 4 * k + 3
        img = np.zeros((s, s), np.uint8)
        for j in range(k):
            a = 1 + 2 * j
            img[a:s - a, a:s - a] = 1
            img[a + 1:s - a - 1, a + 1:s - a - 1] = 0
        r = oracle.label(img)
        assert r.n_labels == 2 * k + 1
        # a chain: component c's parent is c - 1
        assert list(r.parent) == [-1] + list(range(2 * k))
        assert r.euler == 0
        _tree_invariants(r)


def test_alternating_rows():
    for h, w in [(6, 5), (9, 1), (10, 16)]:
        img = np.zeros((h, w), np.uint8)
        img[1::2] = 1
        r = oracle.label(img)
        nfg = h // 2
        assert r.euler == nfg
        assert r.n_labels == 1 + nfg
        assert np.all(r.parent[1:] == 0)


def test_pitch_and_values():
    img = synth.bernoulli_blocks(37, 53, 0.5, 1, 7)
    base = oracle.label(img)
    big = np.zeros((37, 64), np.uint8)
    big[:, :53] = img * 255
    strided = big[:, :53]
    r = oracle.label(strided)
    assert np.array_equal(r.labels, base.labels)
    rng = np.random.default_rng(3)
    vals = (img * rng.integers(1, 256, size=img.shape)).astype(np.uint8)
    r2 = oracle.label(vals)
    assert np.array_equal(r2.labels, base.labels) and np.array_equal(r2.parent, base.parent)


def test_invariants_on_sweep_sizes():
    for p in synth.SWEEP_P:
        for g in (1, 4, 16):
            img = synth.bernoulli_blocks(300, 257, p, g, 11)
            r = oracle.label(img)
            _feature_sums_ok(img, r)
            _tree_invariants(r)
            assert r.euler == refs.bitquad_euler8(img)


def test_structured_generator_small():
    img = synth.structured(512, 512, seed=1, groups=16, rmax=200.0)
    r = oracle.label(img)
    _feature_sums_ok(img, r)
    _tree_invariants(r)
    assert r.euler == refs.bitquad_euler8(img)
