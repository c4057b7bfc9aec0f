"""Host-side checks of the C-ABI library (no GPU compute): it loads, exports
every symbol include/ccl.h declares, and rejects bad arguments on the host."""
import ctypes
import os
import re

import pytest

from paper_2006_09299_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    txt = open(os.path.join(ROOT, "include", "ccl.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ccl_[a-z_]+)\s*\(", txt)))


def test_header_declares_exports():
    assert _declared_functions() == sorted(_capi.EXPORTS)


def test_library_exports_every_symbol():
    L = _capi.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_strerror_and_tile_shape():
    assert _capi.strerror(0) == "ok"
    assert "workspace" in _capi.strerror(_capi.CCL_ENOSPC)
    th, tw = _capi.tile_shape()
    assert th >= 1 and tw % 64 == 0


def test_single_image_variant_by_size():
    """ccl_label takes smaller tiles for smaller images; its workspace size is
    that variant's."""
    L = _capi.lib()
    # super-tiles of 8 x 8 tiles of 64 x 128 where the image holds 256 of them:
    # 16384 x 8192 holds 16 x 16, 16384 x 7680 16 x 15
    for (w, h), v in [((512, 512), 2), ((1024, 1024), 2), ((1300, 1300), 5), ((2048, 2048), 5),
                      ((2600, 2400), 5), ((4096, 4096), 0), ((8192, 8192), 0), ((12288, 12288), 9),
                      ((16384, 16384), 9), ((16384, 8192), 9), ((16384, 7680), 0), ((1, 1), 2)]:
        assert _capi.variant_for(w, h) == v, (w, h)
        assert L.ccl_workspace_bytes(w, h) == L.ccl_workspace_bytes_v(w, h, v) > 0
        assert _capi.workspace_bytes(w, h) == L.ccl_workspace_bytes(w, h)
    assert L.ccl_variant_for(0, 5) == _capi.CCL_EINVAL and L.ccl_variant_for(5, -1) == _capi.CCL_EINVAL


def test_workspace_bytes_pure_and_monotone():
    a = _capi.workspace_bytes(512, 512)
    assert a > 0 and a == _capi.workspace_bytes(512, 512)
    assert _capi.workspace_bytes(1024, 512) > a
    assert _capi.workspace_bytes(0, 5) == 0 and _capi.workspace_bytes(5, -1) == 0


def _call(img, w, h, pitch, out, ws, wsb):
    return _capi.lib().ccl_label(img, w, h, pitch, ctypes.byref(out) if out is not None else None, ws, wsb, None)


def test_label_rejects_bad_arguments_on_host():
    fake = 0x1000  # never dereferenced: every case fails validation first
    out = _capi.ccl_outputs_t(fake, fake, fake, fake, 10, fake)
    wsb = _capi.workspace_bytes(64, 64)
    E = _capi.CCL_EINVAL
    assert _call(None, 64, 64, 64, out, fake, wsb) == E
    assert _call(fake, 0, 64, 64, out, fake, wsb) == E
    assert _call(fake, 64, -1, 64, out, fake, wsb) == E
    assert _call(fake, 64, 64, 63, out, fake, wsb) == E
    assert _call(fake, 64, 64, 64, None, fake, wsb) == E
    assert _call(fake, 64, 64, 64, out, None, wsb) == E
    assert _call(fake, 65536, 65536, 65536, out, fake, 1 << 40) == E  # w*h >= 2^31-1
    bad_cap = _capi.ccl_outputs_t(fake, fake, fake, fake, 0, fake)
    assert _call(fake, 64, 64, 64, bad_cap, fake, wsb) == E
    no_counts = _capi.ccl_outputs_t(fake, fake, fake, fake, 10, None)
    assert _call(fake, 64, 64, 64, no_counts, fake, wsb) == E
    assert _call(fake, 64, 64, 64, out, fake, wsb - 1) == _capi.CCL_ENOSPC


def test_batch_sizes_and_prepare_on_host():
    fake = 0x1000
    imgs = (_capi.ccl_image_t * 3)()
    for i, (w, h) in enumerate([(64, 64), (100, 33), (1, 1)]):
        imgs[i] = _capi.ccl_image_t(fake, w, h, w, _capi.ccl_outputs_t(fake, fake, fake, fake, 8, fake))
    db, wb = ctypes.c_size_t(), ctypes.c_size_t()
    L = _capi.lib()
    for v in range(_capi.num_variants()):
        assert L.ccl_batch_sizes(imgs, 3, v, ctypes.byref(db), ctypes.byref(wb)) == 0
        assert db.value > 0 and wb.value >= _capi.workspace_bytes(64, 64, v)
        host = (ctypes.c_char * db.value)()
        assert L.ccl_batch_prepare(imgs, 3, v, host, db.value) == 0
        assert L.ccl_batch_prepare(imgs, 3, v, host, db.value - 1) == _capi.CCL_EINVAL
    assert L.ccl_batch_sizes(imgs, 3, _capi.num_variants(), ctypes.byref(db), ctypes.byref(wb)) == _capi.CCL_EINVAL
    imgs[1].pitch = 10  # < w
    assert L.ccl_batch_sizes(imgs, 3, 0, ctypes.byref(db), ctypes.byref(wb)) == _capi.CCL_EINVAL
    assert L.ccl_label_batch(imgs, 0, 0, host, host, 1, None) == _capi.CCL_EINVAL


def test_variants_are_described():
    n = _capi.num_variants()
    assert n >= 2
    seen = set()
    for v in range(n):
        th, tw, hs, nt, sup, rg = _capi.variant_info(v)
        assert th >= 1 and tw % 64 == 0 and nt % 64 == 0
        assert 2 <= sup <= 8 and 1 <= rg <= 128 and (hs or rg == 1)
        seen.add((th, tw, hs, nt, sup, rg))
        assert _capi.workspace_bytes(1000, 700, v) > 0
    assert len(seen) == n
    assert {x[4] for x in seen} >= {2, 4, 8}  # merge schedules on offer
    assert _capi.variant_info(0)[:2] == _capi.tile_shape()
    with pytest.raises(_capi.CclError):
        _capi.variant_info(n)


def test_fill_holes_rejects_bad_arguments_on_host():
    L = _capi.lib()
    fake = 0x1000  # never dereferenced: every case fails validation first
    E = _capi.CCL_EINVAL
    good_in = _capi.ccl_outputs_t(fake, fake, fake, fake, 100, fake)
    good_out = _capi.ccl_outputs_t(fake, fake, fake, fake, 100, fake)
    wsb = int(L.ccl_fill_workspace_bytes(100))
    assert wsb > 0 and L.ccl_fill_workspace_bytes(0) == 0

    def call(i, w, h, o, ws=fake, n=wsb):
        return L.ccl_fill_holes(ctypes.byref(i) if i is not None else None, w, h,
                                ctypes.byref(o) if o is not None else None, None, ws, n, None)

    assert call(None, 8, 8, good_out) == E
    assert call(good_in, 8, 8, None) == E
    assert call(good_in, 0, 8, good_out) == E
    assert call(good_in, 65536, 65536, good_out) == E
    assert call(_capi.ccl_outputs_t(fake, fake, None, fake, 100, fake), 8, 8, good_out) == E  # no parent
    assert call(_capi.ccl_outputs_t(fake, fake, fake, fake, 100, None), 8, 8, good_out) == E  # no counts
    assert call(_capi.ccl_outputs_t(None, fake, fake, fake, 100, fake), 8, 8, good_out) == E  # labels asked, none given
    assert call(_capi.ccl_outputs_t(fake, None, fake, fake, 100, fake), 8, 8, good_out) == E  # features likewise
    assert call(good_in, 8, 8, _capi.ccl_outputs_t(fake, fake, fake, fake, 0, fake)) == E
    assert call(good_in, 8, 8, good_out, ws=None) == E
    assert call(good_in, 8, 8, good_out, n=wsb - 1) == _capi.CCL_ENOSPC


def test_label_conn_rejects_other_adjacencies_on_host():
    L = _capi.lib()
    fake = 0x1000  # never dereferenced: every case fails validation first
    out = _capi.ccl_outputs_t(fake, fake, fake, fake, 10, fake)
    wsb = _capi.workspace_bytes(64, 64)
    for adj in (0, 1, 6, 16, -8):
        assert L.ccl_label_conn(fake, 64, 64, 64, ctypes.byref(out), fake, wsb, None, adj) == _capi.CCL_EINVAL
    assert L.ccl_label_conn(None, 64, 64, 64, ctypes.byref(out), fake, wsb, None, 4) == _capi.CCL_EINVAL


def test_noalloc_refuses_oversize_and_bad_arguments_on_host():
    """ccl_label_noalloc checks its arguments and the scratch limit before it
    touches the runtime (the pointers are never dereferenced)."""
    L = _capi.lib()
    fake = 0x1000
    out = _capi.ccl_outputs_t(fake, fake, fake, fake, 10, fake)
    h = 4096
    while _capi.workspace_bytes(4096, h) <= _capi.NOALLOC_SCRATCH_BYTES:
        h += 64
    assert L.ccl_label_noalloc(fake, 4096, h, 4096, ctypes.byref(out), None) == _capi.CCL_ENOSPC
    assert L.ccl_label_noalloc(None, 8, 8, 8, ctypes.byref(out), None) == _capi.CCL_EINVAL
    assert L.ccl_label_noalloc(fake, 64, 64, 63, ctypes.byref(out), None) == _capi.CCL_EINVAL
    assert L.ccl_label_noalloc(fake, 64, 64, 64, None, None) == _capi.CCL_EINVAL


def test_environment_variant_override(monkeypatch):
    """CCL_VARIANT / CCL_TILE force a variant for experiments (host logic)."""
    monkeypatch.delenv(_capi.VARIANT_ENV, raising=False)
    monkeypatch.delenv(_capi.TILE_ENV, raising=False)
    assert _capi.env_variant() is None
    n = _capi.num_variants()
    monkeypatch.setenv(_capi.VARIANT_ENV, str(n - 1))
    assert _capi.env_variant() == n - 1
    for bad in (str(n), "-1", "x"):
        monkeypatch.setenv(_capi.VARIANT_ENV, bad)
        with pytest.raises(ValueError):
            _capi.env_variant()
    monkeypatch.delenv(_capi.VARIANT_ENV)
    for v in range(n):
        th, tw = _capi.variant_info(v)[:2]
        monkeypatch.setenv(_capi.TILE_ENV, f"{th}x{tw}")
        f = _capi.env_variant()
        assert f <= v and _capi.variant_info(f)[:2] == (th, tw)
    monkeypatch.setenv(_capi.TILE_ENV, "7x7")
    with pytest.raises(ValueError):
        _capi.env_variant()
