"""GPU: serving loop (a10).  Every result served in the mix equals the
result of labeling the same image alone (bit-exact), admission respects the
device budget, and oversize requests are refused."""
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _images(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        h, w = int(np.exp(rng.uniform(np.log(16), np.log(1500)))), int(np.exp(rng.uniform(np.log(16), np.log(1500))))
        out.append(synth.bernoulli_blocks(h, w, float(rng.uniform(0.1, 0.9)), int(rng.choice([1, 4])), seed * 100 + i))
    return out


def _check_same(a, b):
    assert (a.n_labels, a.euler) == (b.n_labels, b.euler)
    assert torch.equal(a.labels, b.labels) and torch.equal(a.features, b.features)
    assert torch.equal(a.parent, b.parent) and torch.equal(a.color, b.color)


@pytest.mark.parametrize("budget_mib,streams", [(4096, 4), (96, 2)])
def test_served_results_equal_alone(budget_mib, streams):
    import paper_2006_09299_amd as ccl
    from paper_2006_09299_amd.serve import Server
    dev = _dev()
    imgs = _images(60, budget_mib)
    srv = Server(budget_mib << 20, max_slots=32, streams=streams, max_batch=8)
    alone = {}
    for i, im in enumerate(imgs):
        alone[i] = ccl.label(torch.from_numpy(im).to(dev))
    torch.cuda.synchronize()
    # staggered arrivals: part at once, part later, all while others run
    for i, im in enumerate(imgs):
        srv.submit(i, torch.from_numpy(im).pin_memory(), arrival=0.0 if i < 30 else 0.002 * (i - 29))
    seen = 0
    max_inflight = 0
    while not srv.idle():
        done = srv.step()
        max_inflight = max(max_inflight, len(srv.inflight))
        assert srv.pool.used <= srv.pool.size
        for r in done:
            torch.cuda.synchronize()
            _check_same(r.result, alone[r.rid])
            srv.release(r.rid)
            seen += 1
    assert seen == len(imgs) and srv.pool.used == 0
    print("max micro-batches in flight", max_inflight, file=sys.stderr)


def test_oversize_request_is_refused():
    from paper_2006_09299_amd.serve import Server
    _dev()
    srv = Server(8 << 20, streams=1)
    with pytest.raises(MemoryError):
        srv.submit(0, torch.zeros((2000, 2000), dtype=torch.uint8).pin_memory())
    assert srv.rejected == 1
