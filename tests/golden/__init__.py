"""Fixtures with values fixed by the paper; see each file's header for the citation."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def read_sections(name: str) -> dict:
    """Parse a fixture: '[section]' headers, '# ' comment lines, data lines."""
    sections, cur = {}, None
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.rstrip("\n")
            if not line.strip() or line.startswith("# "):
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = line[1:-1]
                sections[cur] = []
                continue
            sections[cur].append(line)
    return sections


def fig2():
    s = read_sections("fig2_example.txt")
    img = np.array([[c == "#" for c in r] for r in s["bitmap"]], dtype=np.uint8)
    prov = [tuple(int(v) for v in r.split()) for r in s["provisional"]]
    new = [(int(a), int(b), c, int(d)) for a, b, c, d in (r.split() for r in s["new"])]
    equiv = [tuple(int(v) for v in r.split()) for r in s["equiv"]]
    final = [tuple(int(v) for v in r.split()) for r in s["final"]]
    classes = [tuple(int(v) for v in r.split()) for r in s["classes"]]
    return img, prov, new, equiv, final, classes


def fig2_filled_classes():
    s = read_sections("fig2_example.txt")
    return [tuple(int(v) for v in r.split()) for r in s["filled_classes"]]
