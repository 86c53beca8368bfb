"""The plan's second stream: bs_set_filaments runs the near-singular pair
search there and bs_velocity the short-range and near-singular terms, beside
the long-range stages on the plan stream.  Every call sequence must give the
same numbers as the plain one (bitwise: the same kernels run in the same
order on each stream), including the calls that read the search's results
before any velocity, a second bs_set_filaments before any velocity, and the
per-stage timing mode, which keeps everything on the plan stream."""
import numpy as np
import pytest

from paper_2406_07366_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_07366_amd import binding
    return binding


def np_(t):
    return t.detach().cpu().numpy()


def sets():
    a = W.ringpairs(npairs=200, nbg=20, seed=11)
    b = W.ringpairs(npairs=200, nbg=20, seed=12)
    for fs in (a, b):
        fs.grid_n, fs.tol = 64, 1e-6
    return a, b


def plan_for(B, fs):
    print(f"\n[case] {fs.name} N={fs.n_nodes}", flush=True)
    return B.Plan(B.params_for(fs, ns_mode=B.BS_NS_ADAPTIVE))


def fresh_velocity(B, fs):
    plan = plan_for(B, fs)
    xyz, g = B.load_workload(fs)
    plan.set_filaments(fs.offsets, xyz, g)
    v = np_(plan.velocity())
    n = plan.ns_counts()
    plan.status()
    plan.close()
    return v, n


def test_second_set_before_velocity(B):
    a, b = sets()
    vb, nb = fresh_velocity(B, b)
    plan = plan_for(B, a)
    xa, ga = B.load_workload(a)
    xb, gb = B.load_workload(b)
    plan.set_filaments(a.offsets, xa, ga)     # its pair search is left pending
    plan.set_filaments(b.offsets, xb, gb)
    v = np_(plan.velocity())
    plan.status()
    assert nb[0] > 0
    assert plan.ns_counts() == nb
    assert np.array_equal(v, vb)
    plan.close()


def test_results_of_the_search_read_before_any_velocity(B):
    a, _ = sets()
    va, na = fresh_velocity(B, a)
    plan = plan_for(B, a)
    xa, ga = B.load_workload(a)
    plan.set_filaments(a.offsets, xa, ga)
    assert plan.ns_counts() == na             # joins the pending search
    plan.set_filaments(a.offsets, xa, ga)
    terms = {k: np_(t) for k, t in plan.velocity_terms().items()}
    v = np_(plan.velocity())
    assert np.array_equal(v, va)
    assert np.abs(terms["ns"]).max() > 0
    # the terms add up to the velocity (to rounding: other summation order)
    tot = terms["local"] + terms["short"] + terms["long"] - terms["self"] + terms["ns"]
    assert np.abs(tot - v).max() < 1e-12 * np.abs(v).max()
    plan.close()


def test_stage_timing_mode_gives_the_same_velocity(B):
    a, _ = sets()
    va, _ = fresh_velocity(B, a)
    plan = plan_for(B, a)
    xa, ga = B.load_workload(a)
    plan.set_profiling(True)
    plan.set_filaments(a.offsets, xa, ga)
    v1 = np_(plan.velocity())
    st = plan.stage_times(reset=True)
    plan.set_profiling(False)
    plan.set_filaments(a.offsets, xa, ga)     # search pending on the side stream
    plan.set_profiling(True)                  # the velocity then runs on the plan stream
    v2 = np_(plan.velocity())
    plan.set_profiling(False)
    assert st["pairs"][1] == 1 and st["ns_flag"][1] == 1
    assert np.array_equal(v1, va) and np.array_equal(v2, va)
    plan.close()
