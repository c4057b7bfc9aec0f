"""Host emulation of the HIP kernels (tests/emu/) against the oracle.

The kernel source runs on the CPU under AddressSanitizer / UBSan with small
tile shapes that put many tile seams and corners into small images, in the
single-image and the batched launch form.  This is a CPU test of the kernel
logic and of its memory accesses; the GPU parity tests check the real
library."""
import numpy as np
import pytest

import emu_runner
import oracle
import synth
from golden import fig2


def _assert_same(img, r, fg8=True):
    o = oracle.label(img, fg8=fg8)
    assert r.n_labels == o.n_labels and r.euler == o.euler
    assert np.array_equal(r.labels, o.labels)
    assert np.array_equal(r.parent, o.parent)
    assert np.array_equal(r.color, o.color)
    assert np.array_equal(r.bbox, o.bbox)
    assert np.array_equal(r.S, o.S) and np.array_equal(r.Sx, o.Sx) and np.array_equal(r.Sy, o.Sy)


def _cases(seed, n, hmax, wmax):
    rng = np.random.default_rng(seed)
    out = [fig2()[0], np.ones((9, 130), np.uint8), np.zeros((7, 65), np.uint8),
           ((np.add.outer(np.arange(11), np.arange(140)) % 2) == 0).astype(np.uint8)]
    for _ in range(n):
        h, w = int(rng.integers(1, hmax)), int(rng.integers(1, wmax))
        out.append(synth.bernoulli_blocks(h, w, float(rng.uniform(0.05, 0.95)), int(rng.choice([1, 2, 3, 5])),
                                          int(rng.integers(1 << 30))))
    return out


@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 6, 7])
def test_emulated_kernels_small_tiles(cfg):
    imgs = _cases(100 + cfg, 8, 40, 300)
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=cfg)):
        _assert_same(img, r)


def test_emulated_kernels_batched_padded_pitch():
    imgs = _cases(7, 10, 30, 200)
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=1, batch=True, pitch_pad=5)):
        _assert_same(img, r)


def test_emulated_kernels_production_tile():
    # the dense 128 x 2048 image fills the root-reduction hash of a tile group
    # more than once (flush while scanning, then at the end)
    block = np.zeros((100, 300), np.uint8)
    block[10:90, 20:280] = 1  # whole one-colour tiles inside, ragged ones around
    imgs = _cases(11, 4, 80, 400) + [synth.bernoulli_blocks(70, 300, 0.5, 1, 5),
                                     synth.bernoulli_blocks(128, 2048, 0.5, 1, 3),
                                     np.ones((64, 256), np.uint8), block]
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=0, pitch_pad=16)):
        _assert_same(img, r)


@pytest.mark.parametrize("cfg", [0, 7, 8])
def test_emulated_many_interior_components_per_tile(cfg):
    # a checkerboard puts one hole on every second pixel: more interior
    # components in a tile than one accumulator pass holds, and close to the
    # bound on their number (half the tile); 8: the complementary pair, where
    # the foreground pixels are the singletons
    img = ((np.add.outer(np.arange(70), np.arange(140)) % 2) == 0).astype(np.uint8)
    _assert_same(img, emu_runner.run([img], tile_cfg=cfg)[0], fg8=cfg != 8)


@pytest.mark.parametrize("sched", ["rev", "12345"])
def test_emulated_kernels_other_thread_orders(sched):
    # threads that pass a barrier first go on before the others have read the
    # shared state written before it: reverse and shuffled thread orders
    imgs = _cases(21, 3, 60, 300) + [synth.bernoulli_blocks(96, 768, 0.5, 1, 3)]
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=0, sched=sched)):
        _assert_same(img, r)
    imgs = _cases(22, 6, 30, 200)
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=1, batch=True, sched=sched)):
        _assert_same(img, r)


@pytest.mark.parametrize("cfg", [8, 9])
def test_emulated_kernels_complementary_connectivity(cfg):
    """4-adjacent foreground / 8-adjacent background (background diagonals
    inside tiles, across tile seams and corners)"""
    imgs = _cases(200 + cfg, 8, 40, 300)
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=cfg)):
        _assert_same(img, r, fg8=False)
    imgs = _cases(300 + cfg, 6, 30, 200)
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=cfg, batch=True, pitch_pad=3)):
        _assert_same(img, r, fg8=False)


@pytest.mark.parametrize("cfg,batch", [(0, False), (7, False), (1, True), (8, False)])
def test_emulated_features_only(cfg, batch):
    """No label image (labels = NULL): every table equal to the oracle's, and
    the label buffer left untouched."""
    imgs = _cases(400 + cfg, 3, 40, 300) + [synth.bernoulli_blocks(64 if cfg == 1 else 128, 512, 0.5, 1, 8)]
    fg8 = cfg != 8
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=cfg, batch=batch, labels=False)):
        o = oracle.label(img, fg8=fg8)
        assert r.n_labels == o.n_labels and r.euler == o.euler
        assert np.all(r.labels == -7)
        assert np.array_equal(r.parent, o.parent)
        assert np.array_equal(r.color, o.color)
        assert np.array_equal(r.bbox, o.bbox)
        assert np.array_equal(r.S, o.S) and np.array_equal(r.Sx, o.Sx) and np.array_equal(r.Sy, o.Sy)


@pytest.mark.parametrize("cfg", [10, 11, 12])
def test_emulated_merge_schedules(cfg):
    """Super-tiles of 2 x 2 and 8 x 8 tiles (the seams k_seam_local merges in
    LDS against those left to k_border_merge move) and root-reduction groups
    of 4 and 1 tiles, single and batched."""
    # 4 x 64 tiles: a 40 x 400 image spans 10 x 7 tiles, so 2 x 2 and 8 x 8
    # super-tiles and their seams both occur
    imgs = _cases(500 + cfg, 3, 48, 520)
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=cfg)):
        _assert_same(img, r)
    imgs = _cases(600 + cfg, 3, 36, 300)
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=cfg, batch=True, pitch_pad=7)):
        _assert_same(img, r)


@pytest.mark.parametrize("cfg", [13, 14])
def test_emulated_large_reduction_groups(cfg):
    """Root-reduction groups of 128 and 256 tiles, whose node-count prefix is
    taken 64 tiles at a time: images of more than 64, 128 and 256 tiles, so
    that a group's second and later chunks, and a ragged last group, occur."""
    imgs = [synth.bernoulli_blocks(48, 520, 0.5, 1, 3),  # 12 x 9 tiles of 4 x 64
            synth.bernoulli_blocks(60, 1000, 0.4, 2, 4)]  # 15 x 16 or 20 x 16 tiles
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=cfg)):
        _assert_same(img, r)
    imgs = _cases(700 + cfg, 2, 40, 600)
    for img, r in zip(imgs, emu_runner.run(imgs, tile_cfg=cfg, batch=True, pitch_pad=3)):
        _assert_same(img, r)
