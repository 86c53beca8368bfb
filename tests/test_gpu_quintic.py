"""Parity of the quintic-spline path and of the subdivided local term with
the FP64 oracle (App. B with k = 6; Sec. 5.2), through the C ABI.

The device solves the quintic spline in Hermite form (block parallel cyclic
reduction); the oracle uses the paper's B-spline form with a dense solve, so
agreement pins both.  Filaments of 6, 7, 8 and 16 nodes exercise the
periodic index wrap of the reduction (power-of-two lengths merge the two
couplings at distance n/2), 100 nodes the solve outside LDS."""
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


def np_(t):
    return t.detach().cpu().numpy()


def make_plan(B, fs, **kw):
    print(f"\n[case] {fs.name} N={fs.n_nodes} params={kw}", flush=True)
    plan = B.Plan(B.params_for(fs, **kw))
    xyz, g = B.load_workload(fs)
    plan.set_filaments(fs.offsets, xyz, g)
    plan.status()
    return plan


def ragged(counts, seed=7):
    rng = np.random.default_rng(seed)
    parts = []
    for nl in counts:
        th = 2 * np.pi * (np.arange(nl) + 0.3 * rng.uniform(size=nl)) / nl
        R = rng.uniform(0.5, 1.0)
        c = rng.uniform(0, 2 * np.pi, 3)
        rot = W.haar_rotations(rng, 1)[0]
        loc = np.stack([R * np.cos(th), 0.7 * R * np.sin(th), 0.15 * np.sin(2 * th)], 1)
        parts.append(c + loc @ rot.T)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return W.FilamentSet("ragged", 2 * np.pi, 1e-6, off, np.concatenate(parts),
                         rng.choice([-1.0, 1.0], len(counts)), 32, 1e-6)


@pytest.mark.parametrize("which", ["ellipses", "ragged"])
def test_quintic_geometry_matches_oracle(B, which):
    fs = W.ellipses() if which == "ellipses" else ragged([6, 7, 8, 16, 100, 33])
    for Q in (1, 2, 3, 4):
        plan = make_plan(B, fs, Q=Q, spline_order=6)
        g = {k: np_(v) for k, v in plan.geometry().items()}
        o = O.Oracle(fs, Q=Q, order=6)
        qp, _, qc = o.quad()
        nd = o.nodes()
        scale = np.abs(fs.xyz).max()
        e = (np.abs(g["qpos"] - qp).max() / scale, np.abs(g["qcharge"] - qc).max() / np.abs(qc).max(),
             np.abs(g["sdot"] - nd["sdot"]).max(),
             np.abs(g["sddot"] - nd["sddot"]).max() / np.abs(nd["sddot"]).max(),
             np.abs(g["ell"] - nd["ell"]).max() / nd["ell"].max())
        print(f"  Q={Q}: qpos {e[0]:.1e} qcharge {e[1]:.1e} sdot {e[2]:.1e} sddot {e[3]:.1e} "
              f"ell {e[4]:.1e}")
        assert e[0] < 1e-13 and e[1] < 1e-12 and e[2] < 1e-11 and e[3] < 1e-10 and e[4] < 1e-13
        plan.close()


@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("eps", [0.1, 0.5, 1.0])
def test_subdivided_local_term_matches_oracle(B, order, eps):
    fs = W.ellipses()
    plan = make_plan(B, fs, Q=3, spline_order=order, local_frac=eps)
    loc = np_(plan.velocity_terms()["local"])
    o = O.Oracle(fs, Q=3, order=order)
    ref, _ = o.local_sub(eps)
    err = rel_l2(loc, ref)
    print(f"  order {order} eps {eps}: local rel_l2 {err:.2e}")
    # the local term is proportional to s''; the quintic second derivatives of
    # the two solves (block cyclic reduction, dense LU) agree to ~1.3e-12
    assert err < (1e-12 if order == 4 else 1e-11)
    plan.close()


@pytest.mark.parametrize("order", [4, 6])
def test_velocity_and_energy_at_same_parameters(B, order):
    """The whole evaluation with subdivided local segments, at the oracle's
    alpha, r_c and K (sigma = 2, w = 16 make the NUFFT error ~1e-12): the
    velocity, the streamfunction and the energy line integral."""
    fs = W.leapfrog(a=1e-8)
    L = fs.L
    plan = make_plan(B, fs, alpha=7.0 / L, rcut=L / 2, Q=3, spline_order=order,
                     local_frac=0.1, sigma=2.0, w=16)
    prm = plan.params()
    v = np_(plan.velocity())
    E, psi = plan.energy()
    psi = np_(psi)
    o = O.Oracle(fs, Q=3, order=order)
    vref, pref = o.ewald(prm.alpha, prm.rcut, prm.K, local_eps=0.1)
    Eref = o.energy(pref)
    ev, ep = rel_l2(v, vref), rel_l2(psi, pref)
    print(f"  order {order}: v rel_l2 {ev:.2e} psi {ep:.2e} E {E:.15e} ref {Eref:.15e}")
    assert ev < 1e-10 and ep < 1e-10
    assert abs(E / Eref - 1) < 1e-11
    plan.close()


def test_quintic_rk4_follows_oracle(B):
    """Ten RK4 steps of the leapfrogging rings (quintic, Q = 3, local segments
    subdivided at 10 %) against the oracle's RK4 at the same parameters."""
    import torch
    fs = W.leapfrog(a=1e-8)
    L = fs.L
    plan = make_plan(B, fs, alpha=7.0 / L, rcut=L / 2, Q=3, spline_order=6,
                     local_frac=0.1, sigma=2.0, w=16)
    prm = plan.params()
    dt = 0.012
    xyz, g = B.load_workload(fs)
    x = xyz.clone()
    for _ in range(10):
        plan.rk4_step(fs.offsets, x, g, dt)
    plan.status()
    xg = np_(x)

    def vel(y):
        f2 = W.FilamentSet(fs.name, L, fs.a, fs.offsets, y, fs.gamma, fs.grid_n, fs.tol)
        return O.Oracle(f2, Q=3, order=6).ewald(prm.alpha, prm.rcut, prm.K, psi=False,
                                                  local_eps=0.1)[0]
    y = fs.xyz.copy()
    for _ in range(10):
        k1 = vel(y); k2 = vel(y + 0.5 * dt * k1); k3 = vel(y + 0.5 * dt * k2); k4 = vel(y + dt * k3)
        y = y + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    err = np.abs(xg - y).max()
    print(f"  max |x_gpu - x_oracle| after 10 steps: {err:.2e} (moved {np.abs(y - fs.xyz).max():.3f})")
    assert err < 1e-10
    plan.close()


def test_quintic_rejects_short_filaments_and_the_network(B):
    fs = ragged([5, 9])
    plan = B.Plan(B.params_for(fs, spline_order=6))
    xyz, g = B.load_workload(fs)
    with pytest.raises(B.BsError):
        plan.set_filaments(fs.offsets, xyz, g)
    plan.close()
    with pytest.raises(B.BsError):
        B.Plan(B.params_for(fs, spline_order=6, ns_mode=B.BS_NS_MLP))


def test_quintic_near_singular_term_matches_oracle(B):
    """The adaptive near-singular correction on quintic segments (the exact
    segment integral of the quintic Hermite segment minus its Q-point sum)
    against the oracle's Gauss-Kronrod integrals on its B-spline segments."""
    fs = W.ringpairs(npairs=150, nbg=20, seed=77)
    fs.grid_n, fs.tol = 64, 1e-6
    plan = make_plan(B, fs, ns_mode=B.BS_NS_ADAPTIVE, spline_order=6, Q=3)
    dv = np_(plan.velocity_terms()["ns"])
    ref, cnt = O.Oracle(fs, Q=3, order=6).ns_correction(eta=1.0)
    err = rel_l2(dv, ref)
    print(f"  quintic ns term rel_l2 {err:.2e}, flagged pairs {cnt.sum()}")
    assert cnt.sum() > fs.n_nodes and err < 1e-10
    plan.close()
