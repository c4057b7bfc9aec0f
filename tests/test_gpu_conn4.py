"""GPU: the complementary connectivity pair (4-adjacent foreground,
8-adjacent background; ccl_label_conn with fg_adjacency = 4) bit-exact
against the oracle under the same pair: labels, features, tree, colour,
counts, on random images spanning tiles and super-tiles with ragged tails,
checkerboards (isolated foreground pixels, one background), diagonal rings
(leaking background), degenerate images and a full 8192 x 8192 image."""
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


def _check(img):
    import paper_2006_09299_amd as ccl
    dev = _dev()
    print("conn4", img.shape, file=sys.stderr, flush=True)
    r = ccl.label(torch.from_numpy(np.ascontiguousarray(img)).to(dev), fg_adjacency=4)
    torch.cuda.synchronize()
    o = oracle.label(img, fg8=False)
    assert (r.n_labels, r.euler) == (o.n_labels, o.euler)
    assert np.array_equal(r.labels.cpu().numpy(), o.labels)
    assert np.array_equal(r.parent.cpu().numpy(), o.parent)
    assert np.array_equal(r.color.cpu().numpy(), o.color)
    assert np.array_equal(r.bbox.cpu().numpy().astype(np.int64), o.bbox)
    assert np.array_equal(r.S.cpu().numpy(), o.S)
    assert np.array_equal(r.Sx.cpu().numpy(), o.Sx)
    assert np.array_equal(r.Sy.cpu().numpy(), o.Sy)


def test_fig2_and_degenerate():
    _check(golden.fig2()[0])
    for img in (np.zeros((70, 300), np.uint8), np.ones((70, 300), np.uint8), np.ones((1, 1), np.uint8),
                ((np.add.outer(np.arange(131), np.arange(517)) % 2) == 0).astype(np.uint8)):
        _check(img)


def test_diagonal_rings():
    img = np.zeros((300, 700), np.uint8)
    for cy, cx, rad in ((60, 80, 40), (150, 300, 90), (200, 600, 70), (64, 128, 64)):
        for k in range(rad):
            for y, x in ((cy - k, cx - rad + k), (cy + k, cx - rad + k), (cy - k, cx + rad - k), (cy + k, cx + rad - k)):
                if 0 <= y < 300 and 0 <= x < 700:
                    img[y, x] = 1
    _check(img)


@pytest.mark.parametrize("seed", range(10))
def test_random_images(seed):
    rng = np.random.default_rng(1000 + seed)
    h, w = int(rng.integers(1, 1200)), int(rng.integers(1, 1500))
    _check(synth.bernoulli_blocks(h, w, float(rng.uniform(0.1, 0.9)), int(rng.choice([1, 2, 3, 8])), 2000 + seed))


def test_full_size_8192():
    _check(synth.bernoulli_blocks(8192, 8192, 0.5, 1, 102))


def test_full_size_structured_16384():
    _check(synth.structured(16384, 16384, seed=2))
