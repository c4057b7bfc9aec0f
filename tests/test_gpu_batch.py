"""GPU: batched path (a9) against single-image calls and the oracle, every
variant, hipGraph capture + replay, and the autotuner."""
import json
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


def _mixed_images(n, seed, lo=1, hi=700):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        h, w = int(rng.integers(lo, hi)), int(rng.integers(lo, hi))
        out.append(synth.bernoulli_blocks(h, w, float(rng.uniform(0.2, 0.8)), int(rng.choice([1, 2, 4])),
                                          seed * 1000 + i))
    return out


def _same(r, o):
    assert r.n_labels == o.n_labels and r.euler == o.euler
    assert np.array_equal(r.labels.cpu().numpy(), o.labels)
    assert np.array_equal(r.parent.cpu().numpy(), o.parent)
    assert np.array_equal(r.color.cpu().numpy(), o.color)
    assert np.array_equal(r.bbox.cpu().numpy().astype(np.int64), o.bbox)
    assert np.array_equal(r.S.cpu().numpy(), o.S)
    assert np.array_equal(r.Sx.cpu().numpy(), o.Sx)
    assert np.array_equal(r.Sy.cpu().numpy(), o.Sy)


def test_every_variant_single_image_matches_oracle():
    import paper_2006_09299_amd as ccl
    dev = _dev()
    imgs = _mixed_images(6, 3) + [synth.bernoulli_blocks(1000, 1300, 0.5, 1, 5)]
    refs = [oracle.label(im) for im in imgs]
    for v in range(ccl.num_variants()):
        for im, o in zip(imgs, refs):
            _say("variant", v, im.shape)
            r = ccl.label(torch.from_numpy(im).to(dev), variant=v)
            torch.cuda.synchronize()
            _same(r, o)


@pytest.mark.parametrize("variant", range(13))
def test_batch_matches_oracle_per_image(variant):
    import paper_2006_09299_amd as ccl
    if variant >= ccl.num_variants():
        pytest.skip("variant not compiled")
    dev = _dev()
    imgs = _mixed_images(40, 10 + variant) + [np.ones((1, 1), np.uint8), np.zeros((3, 900), np.uint8)]
    rs = ccl.label_batch([torch.from_numpy(im).to(dev) for im in imgs], variant=variant)
    torch.cuda.synchronize()
    for k, (im, r) in enumerate(zip(imgs, rs)):
        _say("batch variant", variant, "image", k, im.shape)
        _same(r, oracle.label(im))


def test_batch_equals_single_calls_bytewise():
    import paper_2006_09299_amd as ccl
    dev = _dev()
    imgs = [torch.from_numpy(im).to(dev) for im in _mixed_images(25, 77, 30, 1500)]
    plan = ccl.BatchPlan(imgs)
    plan.launch()
    rs = plan.results()
    for k, t in enumerate(imgs):
        s = ccl.label(t, cap=plan.caps[k])
        torch.cuda.synchronize()
        assert (s.n_labels, s.euler) == (rs[k].n_labels, rs[k].euler)
        assert torch.equal(s.labels, rs[k].labels) and torch.equal(s.features, rs[k].features)
        assert torch.equal(s.parent, rs[k].parent) and torch.equal(s.color, rs[k].color)


def test_graph_capture_and_replays():
    import paper_2006_09299_amd as ccl
    dev = _dev()
    host = _mixed_images(30, 5, 50, 1200)
    imgs = [torch.from_numpy(im).to(dev) for im in host]
    plan = ccl.BatchPlan(imgs, variant=0)
    plan.capture()
    eager = ccl.label_batch(imgs)
    for rep in range(4):
        # eager work and synchronisations between replays
        junk = torch.randn(1 << 20, device=dev).sum()
        torch.cuda.synchronize()
        plan.replay()
        torch.cuda.synchronize()
        rs = plan.results()
        for r, e in zip(rs, eager):
            assert (r.n_labels, r.euler) == (e.n_labels, e.euler)
            assert torch.equal(r.labels, e.labels) and torch.equal(r.features, e.features)
            assert torch.equal(r.parent, e.parent) and torch.equal(r.color, e.color)
        _say("replay", rep, "ok", float(junk))
    # new pixels in the same buffers: the replay labels the new content
    for t in imgs:
        t.copy_(1 - t)
    plan.replay()
    torch.cuda.synchronize()
    for k, r in enumerate(plan.results()[:5]):
        _same(r, oracle.label(1 - host[k]))


def test_autotune_picks_and_caches(tmp_path):
    from paper_2006_09299_amd import tune
    import paper_2006_09299_amd as ccl
    dev = _dev()
    imgs = [torch.from_numpy(im).to(dev) for im in _mixed_images(16, 9, 64, 800)]
    path = str(tmp_path / "tune.json")
    v = tune.autotune(imgs, path=path)
    assert 0 <= v < ccl.num_variants()
    data = json.load(open(path))
    key = tune.workload_key(imgs)
    assert data[key]["variant"] == v and len(data[key]["ms"]) == ccl.num_variants()
    assert tune.autotune(imgs, path=path) == v  # cached: no timing
    rs = ccl.label_batch(imgs, variant=v)
    torch.cuda.synchronize()
    _same(rs[0], oracle.label(imgs[0].cpu().numpy()))


def test_full_uneven_batch_4096(tmp_path):
    """The benchmarked uneven batch at its full size: 4096 images with sides
    log-uniform in [64, 2048], the variant the autotuner picks on the same
    sample the benchmark tunes on, captured into a HIP graph and replayed
    twice; every image against the oracle, element by element."""
    import concurrent.futures as cf
    import os
    import paper_2006_09299_amd as ccl
    from paper_2006_09299_amd import tune
    dev = _dev()
    specs = synth.batch_specs(4096)
    host = [sp.make() for sp in specs]
    imgs = [torch.from_numpy(im).to(dev) for im in host]
    _say("batch 4096:", sum(sp.pixels for sp in specs), "pixels")
    v = tune.autotune(imgs[::16], path=str(tmp_path / "tune.json"))
    _say("batch 4096: autotuned variant", v, ccl.variant_info(v))
    first = ccl.label_batch(imgs, variant=v)  # table capacities
    caps = [r.n_labels + 16 for r in first]
    del first
    plan = ccl.BatchPlan(imgs, variant=v, caps=caps)
    plan.capture()
    for _ in range(2):
        plan.replay()
    torch.cuda.synchronize()
    rs = plan.results()
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(workers) as ex:  # the oracle's C call releases the GIL
        for k, o in enumerate(ex.map(oracle.label, host)):
            if k % 512 == 0:
                _say("batch 4096: image", k, host[k].shape)
            _same(rs[k], o)
