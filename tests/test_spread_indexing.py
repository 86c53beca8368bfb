"""CPU model of the spread's tile/bin bookkeeping (no GPU).

The spread kernel bins points by the tile holding their stencil base and has
each T^3 tile visit the nbv^3 bins that can reach it.  This test re-derives,
for every grid size and kernel width the plan accepts, that

  * every stencil cell of every point is added by exactly one tile visit,
  * the number of bins a tile visits fits the kernel's bin table,
  * all bin and cell indices stay inside their arrays.
"""
import math

import numpy as np
import pytest


def stencil_base(u, w, n):
    i0 = math.floor(u - 0.5 * w) + 1
    return i0 % n, u - i0


def tile_edge(n):
    return 8 if n % 8 == 0 else 4


def kernel_bin_table(W, TT):
    nbmax = 1 + (W - 1 + TT - 1) // TT
    return nbmax ** 3


@pytest.mark.parametrize("n", [16, 20, 32, 36, 44, 64])
@pytest.mark.parametrize("w", [4, 5, 7, 8, 11, 13, 16])
def test_tiles_cover_each_stencil_cell_once(n, w):
    T = tile_edge(n)
    if n < w + T:
        pytest.skip("rejected by the plan (a stencil could enter a tile twice)")
    NT = n // T
    nb = 1 + -(-(w - 1) // T)
    nbv = min(nb, NT)
    assert nbv ** 3 <= kernel_bin_table(w, T) <= 256
    rng = np.random.default_rng(n * 100 + w)
    us = np.concatenate([rng.uniform(0, n, 40), [0.0, n - 1e-9, 0.5 * w, n - 0.5 * w]])
    for u in us:
        b, f = stencil_base(u, w, n)
        assert 0 <= b < n and 0.5 * w - 1 <= f < 0.5 * w + 1e-12
        tile_of_base = b // T
        assert 0 <= tile_of_base < NT
        cells = [(b + k) % n for k in range(w)]
        hits = {c: 0 for c in cells}
        for t in range(NT):
            # bins this tile visits along one axis
            visited = [(t - d) % NT for d in range(nbv)]
            if tile_of_base not in visited:
                continue
            t0 = t * T
            lx0 = (b - t0) % n
            for k in range(w):
                lx = lx0 + k
                if lx >= n:
                    lx -= n
                if lx < T:
                    hits[(t0 + lx) % n] += 1
        assert all(v == 1 for v in hits.values()), (n, w, u, hits)


def tile_weights_index(b, t0, n, W, TT):
    """The kernel's per-axis mapping: tile cell l takes stencil value k =
    (t0 + l - b) mod n when k < W, else weight 0."""
    out = []
    for l in range(TT):
        k = (t0 + l - b) % n
        out.append(k if k < W else None)
    return out


@pytest.mark.parametrize("n", [16, 20, 32, 36, 64])
def test_tile_frame_weights_cover_the_stencil_once(n):
    T = tile_edge(n)
    NT = n // T
    for W in range(4, 17):
        if n < W + T:
            continue
        nb = 1 + -(-(W - 1) // T)
        nbv = min(nb, NT)
        for b in range(n):
            covered = {}
            for t in range(NT):
                if (b // T) not in [(t - d) % NT for d in range(nbv)]:
                    continue
                t0 = t * T
                for l, k in enumerate(tile_weights_index(b, t0, n, W, T)):
                    if k is not None:
                        cell = t0 + l
                        assert (b + k) % n == cell
                        covered[k] = covered.get(k, 0) + 1
            assert sorted(covered) == list(range(W)) and all(v == 1 for v in covered.values())


def test_plan_rejects_grids_too_small_for_the_tiles():
    from paper_2406_07366_amd import binding as B
    with pytest.raises(B.BsError) as e:
        B.resolve_params(B.make_params(L=2 * math.pi, a=1e-6, tol=1e-6, grid_n=16, w=10,
                                       alpha=1.0, rcut=1.0))
    assert e.value.code == B.BS_EINVAL


def offset_weights_index(b, t0, n, W, TT):
    """The matrix-core form's per-axis mapping: one offset o per axis (the
    stencil index of the tile's first cell, taken in [1 - T, W - 1] when the
    stencil reaches the tile), tile cell l taking kernel value o + l when it
    lies in 0..W-1."""
    off = (t0 - b) % n
    o = off if off < W else off - n
    if o <= -TT:
        return None
    return [o + l if 0 <= o + l < W else None for l in range(TT)]


@pytest.mark.parametrize("n", [16, 24, 32, 40, 64])
def test_offset_form_matches_tile_frame_weights(n):
    T = 8
    for W in range(4, 17):
        if n < W + T:
            continue
        for b in range(n):
            for t in range(n // T):
                ref = tile_weights_index(b, t * T, n, W, T)
                got = offset_weights_index(b, t * T, n, W, T)
                if got is None:
                    assert all(k is None for k in ref), (n, W, b, t)
                else:
                    assert got == ref, (n, W, b, t)
                    # the packed offset o + T fits 5 bits
                    off = (t * T - b) % n
                    o = off if off < W else off - n
                    assert 1 <= o + T <= 31
