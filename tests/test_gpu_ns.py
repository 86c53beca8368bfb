"""Near-singular correction on the GPU against the oracle's adaptive
Gauss-Kronrod integrals (the correction is defined in include/bs.h: the
Q-point sum of every non-adjacent segment whose chord lies within
ns_eta * ell of a node is replaced by the exact segment integral)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2406_07366_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return math.sqrt(((a - b) ** 2).sum(1).mean() / (b ** 2).sum(1).mean())


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_07366_amd import binding
    return binding


def make_plan(B, fs, **kw):
    print(f"\n[case] {fs.name} N={fs.n_nodes} params={kw}", flush=True)
    plan = B.Plan(B.params_for(fs, **kw))
    xyz, g = B.load_workload(fs)
    plan.set_filaments(fs.offsets, xyz, g)
    plan.status()
    return plan


def small_ringpairs():
    fs = W.ringpairs(npairs=150, nbg=20, seed=77)
    fs.grid_n = 64
    fs.tol = 1e-6
    return fs


def test_ns_term_matches_oracle(B):
    fs = small_ringpairs()
    plan = make_plan(B, fs, ns_mode=B.BS_NS_ADAPTIVE)
    t = plan.velocity_terms()
    dv = t["ns"].cpu().numpy()
    ref, cnt = O.Oracle(fs).ns_correction(eta=1.0)
    assert cnt.sum() > fs.n_nodes          # ring partners are flagged
    # the flagged set: same number of pairs as the oracle's float64 test
    assert plan.ns_counts()[0] == int(cnt.sum())
    err = rel_l2(dv, ref)
    print(f"  ns term rel_l2 {err:.2e}, flagged pairs {cnt.sum()}")
    assert err < 1e-10
    # and the velocity including it equals the terms' sum
    v = plan.velocity().cpu().numpy()
    tot = sum(t[k].cpu().numpy() for k in ("local", "short", "long", "ns")) - t["self"].cpu().numpy()
    np.testing.assert_allclose(v, tot, rtol=0, atol=1e-12 * np.abs(v).max())


def test_ns_velocity_meets_reference(B):
    fs = small_ringpairs()
    plan = make_plan(B, fs, ns_mode=B.BS_NS_ADAPTIVE)
    v = plan.velocity().cpu().numpy()
    ref, _ = O.Oracle(fs).reference(psi=False, ns_eta=1.0)
    err = rel_l2(v, ref)
    plain = make_plan(B, fs)
    v0 = plain.velocity().cpu().numpy()
    err0 = rel_l2(v0, ref)
    print(f"  with NS {err:.3e}   without NS {err0:.3e}")
    assert err <= 1e-6
    assert err0 > 100 * err


def test_ns_ringpairs_full_sampled(B):
    """Full ring-pair workload (N = 2e5, grid 256^3, tol 1e-5), 128 sampled
    nodes of the ring pairs against the reference with exact near-singular
    integrals."""
    fs = W.ringpairs()
    plan = make_plan(B, fs, ns_mode=B.BS_NS_ADAPTIVE)
    v = plan.velocity().cpu().numpy()
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(160000, 128, replace=False))
    ref, _ = O.Oracle(fs).reference(targets=idx, beta=6.0, psi=False, ns_eta=1.0)
    err = rel_l2(v[idx], ref)
    print(f"  ringpairs sampled rel_l2 {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("order", [4, 6])
def test_mapped_rule_matches_oracle(B, order):
    """The fixed-cost mapped rule (sinh-mapped Gauss-Legendre split at the
    closest point, tangent-segment control variate) against the oracle's
    adaptive Gauss-Kronrod integrals on the ring pairs (gaps down to 1e-3,
    about 2/3 of the segment length at most), cubic and quintic segments:
    the near-singular term element by element."""
    fs = small_ringpairs()
    plan = make_plan(B, fs, ns_mode=B.BS_NS_MAPPED, spline_order=order)
    dv = plan.velocity_terms()["ns"].cpu().numpy()
    plan.status()
    ref, cnt = O.Oracle(fs, order=order).ns_correction(eta=1.0)
    err = rel_l2(dv, ref)
    mx = np.abs(dv - ref).max() / np.abs(ref).max()
    print(f"  order {order}: mapped ns term rel_l2 {err:.2e}, max {mx:.2e}, pairs {cnt.sum()}")
    assert err < 1e-8 and mx < 1e-7


def test_mapped_ringpairs_full_sampled(B):
    """Full ring-pair workload with the mapped rule, mixed precision at
    tolerance 1e-5: 128 sampled ring nodes against the reference."""
    fs = W.ringpairs()
    plan = make_plan(B, fs, ns_mode=B.BS_NS_MAPPED, precision=B.BS_FP32_MIXED)
    v = plan.velocity().cpu().numpy()
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(160000, 128, replace=False))
    ref, _ = O.Oracle(fs).reference(targets=idx, beta=6.0, psi=False, ns_eta=1.0)
    d = v[idx] - ref
    err = rel_l2(v[idx], ref)
    mx = np.sqrt((d ** 2).sum(1)).max() / math.sqrt((ref ** 2).sum(1).mean())
    print(f"  ringpairs mapped sampled rel_l2 {err:.3e}, max/rms {mx:.2e}")
    assert err <= 1e-5 and mx <= 5e-5


def test_far_images_take_the_float64_decision(B):
    """Every node 600 periods out along x: targets and chord midpoints lie
    beyond the packed period range, so the search's float32 tests (the
    sphere pre-test and the capsule test) pass every candidate to the
    float64 decision, which must flag the same pairs as for the unshifted
    tangle, with the same correction."""
    import copy
    fs = small_ringpairs()
    far = copy.deepcopy(fs)
    far.xyz = np.asarray(fs.xyz, dtype=np.float64) + np.array([600.0 * fs.L, 0.0, 0.0])
    far.name = fs.name + "+600L"
    p0 = make_plan(B, fs, ns_mode=B.BS_NS_ADAPTIVE)
    d0 = p0.velocity_terms()["ns"].cpu().numpy()
    n0 = p0.ns_counts()[0]
    p1 = make_plan(B, far, ns_mode=B.BS_NS_ADAPTIVE)
    d1 = p1.velocity_terms()["ns"].cpu().numpy()
    n1 = p1.ns_counts()[0]
    err = rel_l2(d1, d0)
    print(f"  shifted: flagged pairs {n1} (unshifted {n0}), ns term rel diff {err:.2e}")
    assert n1 == n0 and n0 > fs.n_nodes
    assert err < 1e-8
