"""Plant plausible mistakes in copies of the oracle source (on the CPU) and
check that the pins in this suite catch every one of them.

Each mutant runs in a child process: a planted mistake may also write out of
bounds (a renumbering that skips an id indexes past the tables), which must
not corrupt the memory of the test process itself.  A child that crashes has
not passed the pins either."""
import os
import subprocess
import sys

if __name__ == "__main__":  # child process: the repository root for the oracle package
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import numpy as np
import pytest

import oracle
import refs
from golden import fig2

SRC = os.path.join(os.path.dirname(oracle.__file__), "ccl_oracle.c")

MUTANTS = {
    "drop_NE_neighbour": ("if (diag && x + 1 < w && FG(y - 1, x + 1) == v) unite(par, me, NODE(y - 1, x + 1));", ""),
    "drop_NW_neighbour": ("if (diag && x > 0 && FG(y - 1, x - 1) == v) unite(par, me, NODE(y - 1, x - 1));", ""),
    "bg_8_connected": ("int diag = fg8 ? v : !v;", "int diag = 1;"),
    "fg_4_connected": ("int diag = fg8 ? v : !v;", "int diag = 0;"),
    "no_bottom_frame": ("x == w - 1 || y == h - 1", "x == w - 1"),
    "sx_sums_row": ("f[5] += x;", "f[5] += y;"),
    "bbox_xmax_off_by_one": ("if (x > f[1]) f[1] = x;", "if (x > f[1]) f[1] = x + 1;"),
    "euler_sign": ("*euler = nfg - (nbg - 1);", "*euler = nfg - nbg;"),
    "tree_edges_diagonal_only": ("if (x + 1 < w) {\n        int64_t q = labels[(int64_t)y * w + x + 1];",
                                 "if (x + 1 < w && y + 1 < h) {\n        int64_t q = labels[(int64_t)(y + 1) * w + x + 1];"),
    "ids_not_raster": ("id = next++;", "id = next++; if (id == 2) id = 3; else if (id == 3) id = 2;"),
}


def _pins_hold(lib) -> bool:
    try:
        img, prov, new, equiv, final, classes = fig2()
        r = oracle.label(img, lib=lib)
        if r.n_labels != 3 or r.euler != refs.bitquad_euler8(img):
            return False
        if r.S.sum() != img.size or r.Sx.sum() != 7 * 105 or r.Sy.sum() != 15 * 21:
            return False
        if int(r.bbox[1, 1]) != 13:
            return False
        for h, w in [(3, 3), (2, 4), (4, 2)]:
            for bits in range(1 << (h * w)):
                im = np.array([(bits >> k) & 1 for k in range(h * w)], np.uint8).reshape(h, w)
                r = oracle.label(im, lib=lib)
                exp = refs.flood_label(im)
                if not np.array_equal(r.labels, exp):
                    return False
                if not np.array_equal(r.parent, refs.flood_tree(im, exp)):
                    return False
                if r.euler != refs.bitquad_euler8(im):
                    return False
        return True
    except (AssertionError, RuntimeError, KeyError):
        return False


def test_unmutated_source_passes_quick_pins():
    assert _pins_hold(oracle._load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert old in src, name
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new, 1))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", str(mpath), "-o", str(so)])
    child = subprocess.run([sys.executable, os.path.abspath(__file__), str(so)], capture_output=True, text=True,
                           timeout=300)
    assert child.returncode != 0 or "PINS HOLD" not in child.stdout, f"mutant {name} survived the pins"
    if child.returncode == 0:
        assert "PINS FAIL" in child.stdout, child.stdout + child.stderr


if __name__ == "__main__":  # child: the pins on one build of the oracle source
    print("PINS HOLD" if _pins_hold(oracle.load_variant(sys.argv[1])) else "PINS FAIL", flush=True)
