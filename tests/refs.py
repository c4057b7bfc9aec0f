"""Independent references used to pin the oracle (tests only).

None of these share code with ``oracle/`` or with the HIP library:

* ``flood_label``: brute-force breadth-first flood fill, one component at a
  time, numbering components in raster order of their first pixel; the
  background flood from the border pixels is the exterior (id 0).
* ``flood_tree``: the inclusion tree from the definition of "surrounded"
  (Lemaitre & Lacassagne 2020, Sec. 3.1): C1 is surrounded by C2 when every
  path from C1 to the exterior of the image meets C2; the parent of C1 is the
  unique adjacent component that surrounds it.  Checked by flooding from C1
  with C1's own adjacency while C2's pixels are forbidden.
* ``bitquad_euler8``: Gray's bit-quad Euler number for 8-connected foreground
  (Gray 1971, cited in Sec. 1): E8 = (n(Q1) - n(Q3) - 2 n(QD)) / 4 over all
  2x2 windows of the zero-padded image.
* ``lsl_bw``: the paper's run-based B&W labeling (segment detection,
  unification with initial adjacency, forward transitive closure; Sec. 2 and
  Sec. 3.2), written from the text's description with the readings the
  oracle also takes (virtual background row above row 0 that belongs to the
  exterior, background runs of the last row attached to the exterior).  It
  also records the events of the scan (new labels with their initial
  adjacency, equivalences) so the Fig. 2 narrative can be checked, and can
  take the closure's optional hole-filling step.
"""
from __future__ import annotations

from collections import deque

import numpy as np

N4 = ((-1, 0), (1, 0), (0, -1), (0, 1))
N8 = N4 + ((-1, -1), (-1, 1), (1, -1), (1, 1))


def flood_label(img: np.ndarray, fg8: bool = True) -> np.ndarray:
    """Canonical labels by flood fill (exterior = 0, others by first raster pixel).
    fg8=False: 4-adjacent foreground, 8-adjacent background."""
    fg = np.asarray(img) != 0
    h, w = fg.shape
    lab = np.full((h, w), -1, dtype=np.int64)

    def fill(seeds, k, colour):
        q = deque()
        for (y, x) in seeds:
            if lab[y, x] < 0 and fg[y, x] == colour:
                lab[y, x] = k
                q.append((y, x))
        nb = N8 if colour == fg8 else N4
        while q:
            y, x = q.popleft()
            for dy, dx in nb:
                yy, xx = y + dy, x + dx
                if 0 <= yy < h and 0 <= xx < w and lab[yy, xx] < 0 and fg[yy, xx] == colour:
                    lab[yy, xx] = k
                    q.append((yy, xx))

    border = [(y, x) for y in range(h) for x in range(w) if y in (0, h - 1) or x in (0, w - 1)]
    fill(border, 0, False)
    k = 1
    for y in range(h):
        for x in range(w):
            if lab[y, x] < 0:
                fill([(y, x)], k, bool(fg[y, x]))
                k += 1
    return lab


def adjacent_components(lab: np.ndarray) -> dict:
    """Component adjacency over 4-adjacent pixel pairs, plus the exterior frame
    for every component with a pixel on the image border."""
    h, w = lab.shape
    adj = {int(k): set() for k in np.unique(lab)}
    adj.setdefault(0, set())
    for y in range(h):
        for x in range(w):
            a = int(lab[y, x])
            for dy, dx in ((0, 1), (1, 0)):
                yy, xx = y + dy, x + dx
                if yy < h and xx < w:
                    b = int(lab[yy, xx])
                    if a != b:
                        adj[a].add(b)
                        adj[b].add(a)
            if a != 0 and (y in (0, h - 1) or x in (0, w - 1)):
                adj[a].add(0)
                adj[0].add(a)
    return adj


def surrounds(lab: np.ndarray, fg: np.ndarray, c: int, d: int, fg8: bool = True) -> bool:
    """True when every path from component c to outside the image meets d.
    Paths use c's own adjacency (8 for foreground, 4 for background, or the
    complementary pair when fg8 is False)."""
    if d == 0:
        return True  # the exterior frame lies on every path leaving the image
    h, w = lab.shape
    ys, xs = np.nonzero(lab == c)
    colour = bool(fg[ys[0], xs[0]])
    nb = N8 if colour == fg8 else N4
    seen = np.zeros((h, w), dtype=bool)
    q = deque()
    for y, x in zip(ys, xs):
        seen[y, x] = True
        q.append((int(y), int(x)))
    while q:
        y, x = q.popleft()
        if y in (0, h - 1) or x in (0, w - 1):
            return False  # reached the border without crossing d
        for dy, dx in nb:
            yy, xx = y + dy, x + dx
            if 0 <= yy < h and 0 <= xx < w and not seen[yy, xx] and lab[yy, xx] != d:
                seen[yy, xx] = True
                q.append((yy, xx))
    return True


def flood_tree(img: np.ndarray, lab: np.ndarray, fg8: bool = True) -> np.ndarray:
    """parent[c] = the unique adjacent component surrounding c; parent[0] = -1.
    Raises AssertionError when uniqueness fails."""
    fg = np.asarray(img) != 0
    n = int(lab.max()) + 1
    adj = adjacent_components(lab)
    parent = np.full(n, -2, dtype=np.int64)
    parent[0] = -1
    for c in range(1, n):
        cands = [d for d in sorted(adj[c]) if surrounds(lab, fg, c, d, fg8)]
        assert len(cands) == 1, (c, cands)
        parent[c] = cands[0]
    return parent


def bitquad_euler8(img: np.ndarray) -> int:
    """Gray's bit-quad Euler number for 8-connected foreground."""
    b = np.pad((np.asarray(img) != 0).astype(np.int64), 1)
    a, bb, c, d = b[:-1, :-1], b[:-1, 1:], b[1:, :-1], b[1:, 1:]
    s = a + bb + c + d
    q1 = int(np.sum(s == 1))
    q3 = int(np.sum(s == 3))
    qd = int(np.sum((s == 2) & (a == d)))  # the two diagonal patterns
    val = q1 - q3 - 2 * qd
    assert val % 4 == 0
    return val // 4


def bitquad_euler4(img: np.ndarray) -> int:
    """Gray's bit-quad Euler number for 4-connected foreground."""
    b = np.pad((np.asarray(img) != 0).astype(np.int64), 1)
    a, bb, c, d = b[:-1, :-1], b[:-1, 1:], b[1:, :-1], b[1:, 1:]
    s = a + bb + c + d
    val = int(np.sum(s == 1)) - int(np.sum(s == 3)) + 2 * int(np.sum((s == 2) & (a == d)))
    assert val % 4 == 0
    return val // 4


# ---------------------------------------------------------------------------
# Run-based B&W labeling with initial adjacency (the paper's method), tests only


def _segments(row: np.ndarray):
    """Alternating background/foreground runs of one row as semi-open
    intervals; the first run is background and is empty when the row starts
    with foreground."""
    w = row.shape[0]
    cuts = [0]
    colour = False
    for j in range(w):
        if bool(row[j]) != colour:
            cuts.append(j)
            colour = not colour
    cuts.append(w)
    return [(cuts[k], cuts[k + 1]) for k in range(len(cuts) - 1)]


def _run_features(i: int, j0: int, j1: int):
    """Features of one run [j0, j1) of row i in closed form:
    [xmin, xmax, ymin, ymax, S, Sx, Sy]."""
    n = j1 - j0
    return [j0, j1 - 1, i, i, n, (j0 + j1 - 1) * n // 2, i * n]


def _merge_features(f, g):
    if f is None:
        return list(g)
    return [min(f[0], g[0]), max(f[1], g[1]), min(f[2], g[2]), max(f[3], g[3]),
            f[4] + g[4], f[5] + g[5], f[6] + g[6]]


def lsl_bw(img: np.ndarray, fix_bottom: bool = True, fill_holes: bool = False, fg8: bool = True):
    """Returns (final_labels_per_pixel, T, I, events, F, rows).

    fill_holes: the closure's optional step (Algorithm 3): a root whose
    surrounding's final label is not the exterior is merged into that
    surrounding before the closure continues, so nested levels cascade into
    the top-level foreground.
    fg8=False: the complementary connectivity pair (the run widening applies
    to background runs instead of foreground ones).

    events: list of ("new", row, label, colour, surrounding) and
    ("equiv", row, kept, merged) in scan order; labels are provisional.
    F: features per label (merged into roots by the closure; None when empty).
    rows: per row, (runs, ERA) with the provisional label of every run.
    """
    fg = np.asarray(img) != 0
    h, w = fg.shape
    T = [0]      # equivalence table, label 0 = exterior
    I = [-1]     # initial adjacency
    F = [None]   # features per provisional label
    events = []
    rows_runs = []

    def root(e):
        while T[e] != e:
            e = T[e]
        return e

    prev = None  # (runs, ERA) of the row above
    for i in range(h):
        runs = _segments(fg[i])
        era = [0] * len(runs)
        for k, (j0, j1) in enumerate(runs):
            if j0 == j1:
                era[k] = 0  # empty leading background run
                continue
            colour = k % 2 == 1
            widen = 1 if colour == fg8 else 0  # the 8-adjacent colour's runs are widened
            lo, hi = max(j0 - widen, 0), min(j1 + widen, w)
            above = []
            if prev is None:
                if not colour:
                    above = [0]  # virtual background row above the image
            else:
                pruns, pera = prev
                for kk, (u0, u1) in enumerate(pruns):
                    if (kk % 2 == 1) == colour and u0 < hi and lo < u1 and u0 < u1:
                        above.append(pera[kk])
            if above:
                a = root(above[0])
                for e in above[1:]:
                    b = root(e)
                    if a < b:
                        T[b] = a
                        events.append(("equiv", i, a, b))
                    elif b < a:
                        T[a] = b
                        events.append(("equiv", i, b, a))
                        a = b
                era[k] = a
                F[a] = _merge_features(F[a], _run_features(i, j0, j1))
            else:
                ne = len(T)
                T.append(ne)
                left = era[k - 1] if k > 0 else 0
                I.append(left)
                F.append(_run_features(i, j0, j1))
                era[k] = ne
                events.append(("new", i, ne, "fg" if colour else "bg", left))
        # epilog: first run, last run when background, and (reading) every
        # background run of the last row belong to the exterior
        attach = [0]
        if len(runs) % 2 == 1:
            attach.append(len(runs) - 1)
        if fix_bottom and i == h - 1:
            attach += [k for k in range(0, len(runs), 2)]
        for k in attach:
            if runs[k][0] == runs[k][1]:
                continue
            a = root(era[k])
            if a != 0:
                T[a] = 0
                events.append(("equiv", i, 0, a))
        rows_runs.append((runs, era))
        prev = (runs, era)

    # forward transitive closure; roots point their adjacency at a root
    for e in range(1, len(T)):
        a = T[e]
        if fill_holes and a == e and T[I[e]] > 0:
            a = T[e] = I[e]
        if a < e:
            T[e] = T[a]
            if F[e] is not None:
                F[T[e]] = _merge_features(F[T[e]], F[e])
        else:
            I[e] = T[I[e]]

    lab = np.zeros((h, w), dtype=np.int64)
    for i, (runs, era) in enumerate(rows_runs):
        for k, (j0, j1) in enumerate(runs):
            lab[i, j0:j1] = T[era[k]]
    return lab, T, I, events, F, rows_runs


def canonicalize(lab: np.ndarray, exterior: int = 0):
    """Renumber a label image: `exterior` -> 0, others by first raster pixel.
    Returns (canonical image, mapping old -> new)."""
    mapping = {exterior: 0}
    out = np.empty_like(lab)
    flat = lab.ravel()
    o = out.ravel()
    nxt = 1
    for p, v in enumerate(flat):
        v = int(v)
        if v not in mapping:
            mapping[v] = nxt
            nxt += 1
        o[p] = mapping[v]
    return out, mapping
