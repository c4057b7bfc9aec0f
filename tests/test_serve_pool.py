"""Host-side checks of the serving pool allocator (runs on the CPU)."""
import random

import torch

from paper_2006_09299_amd.serve import ALIGN, DevicePool


def test_pool_first_fit_and_coalescing():
    p = DevicePool(16 * ALIGN, "cpu")
    a = p.alloc(3 * ALIGN)
    b = p.alloc(1)
    c = p.alloc(5 * ALIGN - 7)
    assert (a, b, c) == (0, 3 * ALIGN, 4 * ALIGN)
    assert p.alloc(8 * ALIGN) is None  # 7 blocks left
    p.release(b, 1)
    assert p.alloc(2 * ALIGN) == 9 * ALIGN  # the freed hole is too small: first fit skips it
    p.release(a, 3 * ALIGN)
    assert p.alloc(4 * ALIGN) == 0  # holes [0,3) and [3,4) coalesced
    assert p.used == 4 * ALIGN + 5 * ALIGN + 2 * ALIGN


def test_pool_random_trace_never_overlaps():
    rng = random.Random(5)
    p = DevicePool(1 << 20, "cpu")
    live = {}
    for step in range(3000):
        if live and rng.random() < 0.45:
            k = rng.choice(list(live))
            off, n = live.pop(k)
            p.release(off, n)
        else:
            n = rng.randint(1, 40000)
            off = p.alloc(n)
            if off is not None:
                live[step] = (off, n)
        spans = sorted((o, o + ((n + ALIGN - 1) // ALIGN) * ALIGN) for o, n in live.values())
        for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
            assert a1 <= b0
        assert all(o % ALIGN == 0 and o + n <= p.size for o, n in live.values())
    for off, n in live.values():
        p.release(off, n)
    assert p.free == [(0, p.size)] and p.used == 0
