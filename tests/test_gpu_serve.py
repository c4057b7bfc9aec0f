"""GPU: serving loop (a10) through the native server (ccl_server_*).  Every
result served in the mix equals the result of labeling the same image alone
(bit-exact), admission respects the device pool, requests whose first table
capacity is too small run again with the exact one, and requests that can
never fit are refused."""
import sys
import time

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


def _serve_all(srv, alone, submit_plan):
    """submit_plan: list of (rid, host tensor) batches, submitted one batch per
    scheduling step while earlier ones run; every finished result is checked
    and released."""
    seen, max_inflight = 0, 0
    plan = list(submit_plan)
    while plan or not srv.idle():
        if plan:
            for rid, t in plan.pop(0):
                srv.submit(rid, t)
        for r in srv.step():
            assert r.status == 0
            torch.cuda.synchronize()
            _check_same(r.result, alone[r.rid])
            srv.release(r.rid)
            seen += 1
        st = srv.stats()
        assert 0 <= st.pool_used <= st.pool_bytes
        max_inflight = max(max_inflight, st.in_flight)
    return seen, max_inflight


@pytest.mark.parametrize("budget_mib,streams", [(4096, 4), (96, 2)])
def test_served_results_equal_alone(budget_mib, streams):
    import paper_2006_09299_amd as ccl
    from paper_2006_09299_amd.serve import Server
    dev = _dev()
    imgs = _images(60, budget_mib)
    alone = {i: ccl.label(torch.from_numpy(im).to(dev)) for i, im in enumerate(imgs)}
    torch.cuda.synchronize()
    srv = Server(budget_mib << 20, max_slots=32, streams=streams, max_batch=8)
    host = [torch.from_numpy(im).pin_memory() for im in imgs]
    # half at once, then the rest a few at a time while the first ones run
    plan = [[(i, host[i]) for i in range(30)]] + [[(i, host[i]) for i in range(j, min(j + 3, 60))] for j in range(30, 60, 3)]
    seen, max_inflight = _serve_all(srv, alone, plan)
    st = srv.stats()
    assert seen == len(imgs) and st.pool_used == 0 and st.live == 0 and st.completed == len(imgs)
    srv.close()
    print("micro-batches", st.launches, "max in flight", max_inflight, file=sys.stderr)


def test_strided_host_images_and_relaunch_with_exact_capacity():
    import paper_2006_09299_amd as ccl
    from paper_2006_09299_amd.serve import Server
    dev = _dev()
    imgs = [synth.bernoulli_blocks(h, w, 0.5, 1, 40 + k) for k, (h, w) in enumerate([(300, 257), (64, 1000), (700, 90)])]
    alone = {i: ccl.label(torch.from_numpy(im).to(dev)) for i, im in enumerate(imgs)}
    torch.cuda.synchronize()
    assert all(a.n_labels > 1024 for a in alone.values())
    # rows padded to a wider pitch on the host; the first table holds only 1024 entries
    host = []
    for im in imgs:
        h, w = im.shape
        wide = torch.zeros((h, w + 77), dtype=torch.uint8).pin_memory()
        wide[:, :w] = torch.from_numpy(im)
        host.append(wide[:, :w])
    srv = Server(256 << 20, max_slots=8, streams=2, max_batch=4, cap_divisor=1 << 30)
    seen = 0
    for i, t in enumerate(host):
        srv.submit(i, t)
    while not srv.idle():
        for r in srv.step():
            assert r.status == 0 and r.launches == 2
            torch.cuda.synchronize()
            _check_same(r.result, alone[r.rid])
            srv.release(r.rid)
            seen += 1
    st = srv.stats()
    assert seen == 3 and st.relaunched == 3 and st.pool_used == 0
    srv.close()


def test_tables_that_can_never_fit_are_reported():
    import paper_2006_09299_amd as ccl
    from paper_2006_09299_amd.serve import Server
    dev = _dev()
    im = synth.bernoulli_blocks(256, 256, 0.5, 1, 3)
    ref = ccl.label(torch.from_numpy(im).to(dev))
    torch.cuda.synchronize()
    assert ref.n_labels > 1024
    probe = Server(64 << 20, streams=1, cap_divisor=1 << 30)
    need = probe.footprint(256, 256)  # with the first capacity, 1024 entries
    probe.close()
    srv = Server((need + 255) // 256 * 256, streams=1, cap_divisor=1 << 30)
    srv.submit(0, torch.from_numpy(im).pin_memory())
    t0 = time.time()
    done = []
    while not done:
        done = srv.step()
        assert time.time() - t0 < 60
    (r,) = done
    assert r.status == -2 and r.result is None and r.launches == 1
    srv.release(0)
    assert srv.stats().pool_used == 0
    srv.close()


def test_oversize_request_is_refused():
    from paper_2006_09299_amd.serve import Server
    _dev()
    srv = Server(8 << 20, streams=1)
    with pytest.raises(MemoryError):
        srv.submit(0, torch.zeros((2000, 2000), dtype=torch.uint8).pin_memory())
    assert srv.rejected == 1 and srv.stats().queued == 0
    srv.close()
