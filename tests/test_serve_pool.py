"""Host-side checks of the serving loop's pool sub-allocator (ccl_pool.h,
compiled with g++ and driven by an allocation trace; runs on the CPU) and of
the server entry points' argument checks."""
import ctypes
import os
import random
import subprocess

import pytest

from paper_2006_09299_amd import _capi

HERE = os.path.dirname(os.path.abspath(__file__))
ALIGN = 256


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("pool") / "pool_driver")
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    os.path.join(HERE, "native", "pool_driver.cpp"), "-o", exe], check=True)
    return exe


def _run(exe, size, ops):
    txt = f"size {size}\n" + "".join(f"a {o[1]}\n" if o[0] == "a" else f"r {o[1]} {o[2]}\n" for o in ops)
    p = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True)
    return [ln.split() for ln in p.stdout.splitlines()]


def test_pool_first_fit_and_coalescing(driver):
    r = _run(driver, 16 * ALIGN, [("a", 3 * ALIGN), ("a", 1), ("a", 5 * ALIGN - 7), ("a", 8 * ALIGN)])
    assert [int(x[0]) for x in r] == [0, 3 * ALIGN, 4 * ALIGN, -1]  # 7 units left for the last
    r = _run(driver, 16 * ALIGN, [("a", 3 * ALIGN), ("a", 1), ("a", 5 * ALIGN - 7),
                                  ("r", 3 * ALIGN, 1), ("a", 2 * ALIGN),     # the 1-unit hole is skipped
                                  ("r", 0, 3 * ALIGN), ("a", 4 * ALIGN)])    # holes [0,3) and [3,4) merged
    assert int(r[4][0]) == 9 * ALIGN and int(r[6][0]) == 0
    assert int(r[-1][1]) == (4 + 5 + 2) * ALIGN


def test_pool_zero_bytes_take_one_unit_and_size_rounds_down(driver):
    r = _run(driver, 3 * ALIGN + 100, [("a", 0), ("a", 2 * ALIGN), ("a", 1)])
    assert [int(x[0]) for x in r] == [0, ALIGN, -1]


def test_pool_random_trace_never_overlaps(driver):
    rng = random.Random(5)
    size = 1 << 20
    ops, live, model = [], {}, []
    # build the trace against a simple model of first fit over sorted holes
    free = [(0, size)]
    for step in range(3000):
        if live and rng.random() < 0.45:
            k = rng.choice(list(live))
            off, n = live.pop(k)
            ops.append(("r", off, n))
            m = (n + ALIGN - 1) // ALIGN * ALIGN
            free.append((off, m))
            free.sort()
            merged = []
            for o, s in free:
                if merged and merged[-1][0] + merged[-1][1] == o:
                    merged[-1] = (merged[-1][0], merged[-1][1] + s)
                else:
                    merged.append((o, s))
            free = merged
            model.append(None)
        else:
            n = rng.randint(1, 40000)
            m = (n + ALIGN - 1) // ALIGN * ALIGN
            got = None
            for i, (o, s) in enumerate(free):
                if s >= m:
                    got = o
                    free[i] = (o + m, s - m)
                    if s == m:
                        free.pop(i)
                    break
            ops.append(("a", n))
            model.append(got)
            if got is not None:
                live[step] = (got, n)
    out = _run(driver, size, ops)
    used = 0
    spans = {}
    for op, exp, line in zip(ops, model, out):
        if op[0] == "a":
            off = int(line[0])
            assert off == (-1 if exp is None else exp)
            if off >= 0:
                assert off % ALIGN == 0 and off + op[1] <= size
                spans[off] = off + (op[1] + ALIGN - 1) // ALIGN * ALIGN
                used += spans[off] - off
        else:
            used -= spans.pop(op[1]) - op[1]
        assert int(line[1]) == used
        s = sorted(spans.items())
        assert all(a1 <= b0 for (_, a1), (b0, _) in zip(s, s[1:]))


def test_struct_layouts_match_the_header(tmp_path):
    exe = str(tmp_path / "layouts")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", os.path.join(HERE, "native", "layouts.c"), "-o", exe],
                   check=True)
    c = dict(ln.rsplit(" ", 1) for ln in subprocess.run([exe], capture_output=True, text=True, check=True)
             .stdout.splitlines())
    for T in (_capi.ccl_outputs_t, _capi.ccl_image_t, _capi.ccl_server_config_t, _capi.ccl_done_t,
              _capi.ccl_server_stats_t):
        assert int(c[T.__name__]) == ctypes.sizeof(T), T.__name__
        for key, val in c.items():
            if key.startswith(T.__name__ + "."):
                assert int(val) == getattr(T, key.split(".")[1]).offset, key
    assert int(c["ccl_feature_t"]) == 40 and int(c["ccl_feature_t.S"]) == 16


def test_server_entry_points_reject_bad_arguments_on_host():
    L = _capi.lib()
    E = _capi.CCL_EINVAL
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every case fails validation first
    cfg = _capi.ccl_server_config_t(8, 2, 4, 0, 4)
    assert L.ccl_server_create(None, 1 << 20, ctypes.byref(cfg), ctypes.byref(h)) == E
    assert L.ccl_server_create(ctypes.c_void_p((1 << 20) + 16), 1 << 20, ctypes.byref(cfg), ctypes.byref(h)) == E
    assert L.ccl_server_create(fake, 100, ctypes.byref(cfg), ctypes.byref(h)) == E
    assert L.ccl_server_create(fake, 1 << 20, ctypes.byref(cfg), None) == E
    for bad in ((0, 2, 4, 0, 4), (8, 0, 4, 0, 4), (8, 17, 4, 0, 4), (8, 2, 0, 0, 4), (8, 2, 4, -1, 4),
                (8, 2, 4, _capi.num_variants(), 4), (8, 2, 4, 0, 0)):
        c = _capi.ccl_server_config_t(*bad)
        assert L.ccl_server_create(fake, 1 << 20, ctypes.byref(c), ctypes.byref(h)) == E, bad
    assert h.value is None
    n = ctypes.c_int32()
    st = _capi.ccl_server_stats_t()
    assert L.ccl_server_poll(None, None, 0, ctypes.byref(n)) == E
    assert L.ccl_server_submit(None, fake, 4, 4, 4, 0) == E
    assert L.ccl_server_release(None, 0) == E
    assert L.ccl_server_stats(None, ctypes.byref(st)) == E
    assert L.ccl_server_footprint(None, 4, 4, None) == E
    assert L.ccl_server_destroy(None) == E


def test_server_scheduling_on_a_mock_runtime(tmp_path):
    """ccl_server.cpp built for the host against a mock HIP runtime (copies
    run at once, events finish after a few queries) and stand-ins of the
    batch entry points; 300 random configurations (see the header of the C++
    test program for the checks).  Every path must be taken at least once: shrinking
    micro-batches, relaunch with the exact capacity, refusal at submit and
    at relaunch, and micro-batches that a batch entry point refuses (each
    request reported with the error, its memory returned)."""
    exe = str(tmp_path / "server_sched")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    "-I", os.path.join(HERE, "native", "mock"), os.path.join(HERE, "native", "server_sched.cpp"),
                    "-o", exe], check=True)
    p = subprocess.run([exe, "300"], capture_output=True, text=True)
    assert p.returncode == 0, p.stdout + p.stderr
    words = p.stdout.split()
    assert words[0] == "ok"
    stats = {k: int(v) for k, v in zip(words[3::2], words[4::2])}
    for k in ("launches", "retries", "toobig", "relaunched", "refused", "enospc_done", "failed_sizes",
              "failed_prepare", "failed_launch", "failed_reports"):
        assert stats[k] > 0, (k, p.stdout)
