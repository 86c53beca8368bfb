"""CPU model of the short-range cell window (no GPU).

Cells have edge h = L / nc >= 2 r_c / 3 (nc = floor(3L / (2 r_c (1 + 1e-6)))),
and a target scans the 4 x 4 x 4 cells starting at the cell of x - r_c.  This
re-derives, with the kernel's index arithmetic, that every point within r_c
of the target (minimum image) is in one of those cells, that the 64 cells
are distinct whenever nc >= 4, and that dropping the cells whose box lies
farther than r_c from the target keeps every such point.
"""
import math

import numpy as np
import pytest


def cell_of(v, L, nc):
    w = v - L * np.floor(v / L)
    return np.clip((w / L * nc).astype(int), 0, nc - 1)


@pytest.mark.parametrize("rc", [0.144, 0.2917, 0.6, 1.225, 1.5])
def test_every_point_within_rc_is_in_the_window(rc):
    L = 2 * math.pi
    nc = int(math.floor(3 * L / (2 * rc * (1 + 1e-6))))
    if nc < 4:
        pytest.skip("one cell holds every point")
    assert L / nc >= 2 * rc / 3
    rng = np.random.default_rng(int(rc * 1000))
    pts = rng.uniform(0, L, (4000, 3))
    targets = np.concatenate([rng.uniform(0, L, (200, 3)),
                              rng.choice([0.0, L - 1e-12, rc, L - rc], (60, 3))])
    pc = cell_of(pts, L, nc)
    for x in targets:
        xw = x - L * np.floor(x / L)
        s = np.floor((xw - rc) / L * nc).astype(int)
        window = {tuple((s + np.array([a, b, c])) % nc)
                  for c in range(4) for b in range(4) for a in range(4)}
        assert len(window) == 64
        d = pts - x
        d -= L * np.rint(d / L)
        near = np.nonzero((d * d).sum(1) < rc * rc)[0]
        for i in near:
            assert tuple(pc[i]) in window
        # the cull of the kernel: distance from x to the unwrapped cell box
        h = L / nc
        kept = set()
        for c in range(4):
            for b in range(4):
                for a in range(4):
                    v = s + np.array([a, b, c])
                    lo, hi = v * h - xw, xw - (v + 1) * h
                    dd = np.where(lo > 0, lo, np.where(hi > 0, hi, 0.0))
                    if (dd * dd).sum() <= rc * rc * (1 + 1e-12):
                        kept.add(tuple(v % nc))
        for i in near:
            assert tuple(pc[i]) in kept
        assert len(kept) < 64


@pytest.mark.parametrize("wpn", [1, 4])
def test_chunked_candidate_map_gives_every_lane_its_flat_order(wpn):
    """The pair kernel maps its flattened candidate range (the 64 cells' runs
    laid end to end) to point indices in chunks of 1024: each lane writes
    its cell's run within the chunk into the map, and the candidates
    q = c0 + 64 part + lane, step 64 WPN, read it.  Every candidate must be
    written exactly once before it is read, map to its own point, and every
    lane must meet its candidates in the order of one flat pass."""
    cap = 1024
    rng = np.random.default_rng(wpn)
    for trial in range(20):
        cn = rng.integers(0, 400 if trial % 2 else 30, 64)
        cn[rng.uniform(size=64) < 0.3] = 0
        cs = rng.integers(0, 10 ** 6, 64)
        excl = np.concatenate([[0], np.cumsum(cn)[:-1]])
        total = int(cn.sum())
        flat = np.concatenate([cs[c] + np.arange(cn[c]) for c in range(64)] + [np.zeros(0, int)])
        for part in range(wpn):
            order = {lane: [] for lane in range(64)}
            for c0 in range(0, total, cap):
                cend = min(total, c0 + cap)
                m = np.full(cap, -1)
                for lane in range(64):
                    lo, hi = max(excl[lane], c0), min(excl[lane] + cn[lane], cend)
                    for j in range(lo, hi):
                        assert m[j - c0] == -1
                        m[j - c0] = cs[lane] + (j - excl[lane])
                for lane in range(64):
                    for q in range(c0 + part * 64 + lane, cend, 64 * wpn):
                        assert m[q - c0] == flat[q]
                        order[lane].append(q)
            for lane in range(64):
                assert order[lane] == list(range(part * 64 + lane, total, 64 * wpn))
