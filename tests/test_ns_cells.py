"""CPU model of the near-singular pair search's cell bookkeeping (no GPU).

Segments are binned by chord midpoint into two grids, reach_j =
eta*ell_j + |B_j - A_j|/2.  Grid A has nc_A = floor(L / h) cells per axis,
h = min(max reach, 2 x mean reach) (nc_A < 3: one cell), and holds the short
segments (reach <= L / nc_A); a target scans the 27 A-cells around its own.
Grid B has nc_B = floor(L / max reach) cells (at most nc_A; below 4: one
cell) and holds the long segments; a target in A-cell c scans the 4 x 4 x 4
B-cells from the B-cell of c's lower corner minus one B edge.  This test
re-derives, on random tangles with long and short segments and targets near
the box faces, that every pair a brute-force search flags (chord distance
below eta*ell_j, minimum image) has its segment inside the window of its
grid, and that the window cells are distinct, so every pair is found once.
"""
import math

import numpy as np
import pytest


def wrap(v, L):
    return v - L * np.floor(v / L)


def cell_of(v, L, nc):
    return np.clip((wrap(v, L) / L * nc).astype(int), 0, nc - 1)


def chord_dist(A, B, x, L):
    m = 0.5 * (A + B)
    xs = x - L * np.rint((x - m) / L)
    e = B - A
    t = np.clip(((xs - A) * e).sum(-1) / (e * e).sum(-1), 0, 1)
    return np.linalg.norm(xs - A - t[..., None] * e, axis=-1)


@pytest.mark.parametrize("seed", range(6))
def test_flagged_segments_lie_in_the_27_cells(seed):
    rng = np.random.default_rng(seed)
    L = 2 * math.pi
    eta = 1.0
    nseg = 400
    A = rng.uniform(-L, 2 * L, (nseg, 3))            # unwrapped end points
    ln = np.exp(rng.uniform(np.log(0.01), np.log(0.6), nseg))
    d = rng.normal(size=(nseg, 3))
    B = A + ln[:, None] * d / np.linalg.norm(d, axis=1)[:, None]
    ell = ln * rng.uniform(1.0, 1.2, nseg)           # arc length >= chord
    reach = eta * ell + 0.5 * np.linalg.norm(B - A, axis=1)
    h = min(reach.max(), 2 * reach.mean())
    na = int(math.floor(L / (h * (1 + 1e-9))))
    na = 1 if na < 3 else na
    nb = min(int(math.floor(L / (reach.max() * (1 + 1e-9)))), na)
    nb = 1 if (nb < 4 or na == 1) else nb
    short = (na == 1) | (reach <= L / na)
    assert (~short).sum() < short.sum()          # few long segments
    acell = cell_of(0.5 * (A + B), L, na)
    bcell = cell_of(0.5 * (A + B), L, nb)
    # targets: near the segments (the interesting case) and near box faces
    x = np.concatenate([A + rng.normal(scale=0.05, size=A.shape),
                        rng.choice([0.0, L - 1e-12], size=(100, 3)) + rng.normal(scale=1e-3, size=(100, 3))])
    ha, hb = L / na, L / nb
    for xi in x:
        dist = chord_dist(A, B, xi[None], L)
        flagged = np.nonzero(dist < eta * ell)[0]
        c0 = cell_of(xi, L, na)
        if na < 3:
            continue                              # one cell: every segment is scanned
        wa = {tuple((c0 + np.array([dx, dy, dz])) % na)
              for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)}
        assert len(wa) == 27
        if nb >= 4:
            v0 = np.floor((c0 * ha - hb) / hb).astype(int)
            wb = {tuple((v0 + np.array([dx, dy, dz])) % nb)
                  for dz in range(4) for dy in range(4) for dx in range(4)}
            assert len(wb) == 64
        for j in flagged:
            if short[j]:
                assert tuple(acell[j]) in wa, (xi, j)
            elif nb >= 4:
                assert tuple(bcell[j]) in wb, (xi, j)
            # nb == 1: the single B-cell is scanned by every target


def test_cell_count_matches_the_reach_bound():
    L = 2 * math.pi
    for r in (0.1, 0.3, 1.0, 2.0, 3.0):
        nc = int(math.floor(L / (r * (1 + 1e-9))))
        nc = 1 if nc < 3 else nc
        assert nc == 1 or L / nc >= r


def pretest_f32(x, A, B, eta_ell, L, nc=34):
    """The search's sphere pre-test, in float32 as the kernel does it: the
    chord midpoint, moved into the box, is staged at its image nearest the
    centre of the target's cell (edge L/nc), and the target is tested
    against it with radius |half chord| + eta ell + 1e-5 L.  Records with a
    negative eta ell (midpoint beyond the clamped period range) pass."""
    f = np.float32
    Lf, iLf, band = f(L), f(1.0 / L), f(1e-5 * L)
    xw = wrap(x, L)
    xf = xw.astype(np.float32)
    cc = ((np.floor(xw / L * nc) + 0.5) * L / nc).astype(np.float32)
    m = wrap(0.5 * (A + B), L).astype(np.float32)
    h = (0.5 * (B - A)).astype(np.float32)
    m = m + Lf * np.rint((cc - m) * iLf).astype(np.float32)
    d = xf - m
    r2 = (d * d).sum(-1, dtype=np.float32)
    r = np.sqrt((h * h).sum(-1, dtype=np.float32)) + eta_ell.astype(np.float32) + band
    return (r2 < r * r) | (eta_ell < 0)


@pytest.mark.parametrize("seed", range(4))
def test_pretest_passes_every_flagged_pair(seed):
    # targets at and just inside eta ell of random chords (in all periodic
    # images and across the box faces): the pre-test must never drop a pair
    # the float64 chord test flags, and it should drop most of the others
    rng = np.random.default_rng(100 + seed)
    L = 2 * math.pi
    n = 20000
    A = rng.uniform(-0.2 * L, 1.2 * L, (n, 3))
    B = A + rng.normal(0, 0.01 * L, (n, 3)) * rng.uniform(0.05, 1.0, (n, 1))
    ell = np.linalg.norm(B - A, axis=1) * rng.uniform(1.0, 1.3, n)
    eta_ell = 1.0 * ell
    t = rng.uniform(0, 1, (n, 1))
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    rad = eta_ell * rng.uniform(0.0, 1.5, n)
    x = A + t * (B - A) + rad[:, None] * u + L * rng.integers(-2, 3, (n, 3))
    flagged = chord_dist(A, B, x, L) < eta_ell
    passed = pretest_f32(x, A, B, eta_ell, L)
    assert flagged.sum() > n // 4
    assert np.all(passed[flagged])
    # targets spread over a few reaches around the chord (the cells a
    # target scans), in any periodic image
    reach = eta_ell + 0.5 * np.linalg.norm(B - A, axis=1)
    xr = (0.5 * (A + B) + rng.uniform(-3, 3, (n, 3)) * reach[:, None]
          + L * rng.integers(-2, 3, (n, 3)))
    fr = chord_dist(A, B, xr, L) < eta_ell
    pr = pretest_f32(xr, A, B, eta_ell, L)
    assert np.all(pr[fr])
    # the sphere holds at most ~2x the capsule's volume (plus the margin)
    assert pr.mean() < 3.0 * fr.mean() + 0.01, (pr.mean(), fr.mean())
