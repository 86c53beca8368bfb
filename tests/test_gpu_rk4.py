"""RK4 advance of the nodes (Sec. 5.2: dx/dt = v, spline refitted at every
stage) against the same scheme driven by the oracle's velocities, plus the
ring's Kelvin translation and energy conservation."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2406_07366_amd import workloads as W

pytestmark = pytest.mark.gpu

EULER_GAMMA = 0.5772156649015329


def kelvin_period(lam, a, delta=0.25, kappa=1.0):
    """T_kw(lambda) of Sec. 5.2 (Kelvin wave of wavelength lambda)."""
    return 2 * lam ** 2 / kappa / (math.log(lam / (math.pi * a)) + 0.5 - (delta + EULER_GAMMA))


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_07366_amd import binding
    return binding


def oracle_rk4(fs, dt, steps):
    x = fs.xyz.copy()
    for _ in range(steps):
        ks = []
        for c in (0.0, 0.5, 0.5, 1.0):
            xs = x + c * dt * ks[-1] if ks else x
            f = W.FilamentSet(**{**fs.__dict__, "xyz": xs})
            v, _ = O.Oracle(f).reference(psi=False)
            ks.append(v)
        x = x + dt / 6 * (ks[0] + 2 * ks[1] + 2 * ks[2] + ks[3])
    return x


def test_rk4_ring_matches_oracle_and_translates(B):
    import torch
    fs = W.ring()
    lmin = np.linalg.norm(np.roll(fs.xyz, -1, 0) - fs.xyz, axis=1).min()
    dt = kelvin_period(lmin, fs.a)
    steps = 10
    print(f"\n[case] ring RK4 dt={dt:.3e} steps={steps}", flush=True)
    plan = B.Plan(B.params_for(fs))
    xyz, g = B.load_workload(fs)
    plan.set_filaments(fs.offsets, xyz, g)
    v0 = plan.velocity().cpu().numpy()
    E0, _ = plan.energy()
    x = xyz.clone()
    for _ in range(steps):
        plan.rk4_step(fs.offsets, x, g, dt)
    plan.status()
    xg = x.cpu().numpy()
    plan.set_filaments(fs.offsets, x, g)
    E1, _ = plan.energy()
    xo = oracle_rk4(fs, dt, steps)
    disp = np.abs(xo - fs.xyz).max()
    err = np.abs(xg - xo).max() / disp
    fo = W.FilamentSet(**{**fs.__dict__, "xyz": xo})
    Eo0 = O.Oracle(fs).energy(O.Oracle(fs).reference()[1])
    Eo1 = O.Oracle(fo).energy(O.Oracle(fo).reference()[1])
    print(f"  max |x_gpu - x_oracle| / displacement {err:.2e}; E drift GPU {(E1 - E0) / E0:.2e}"
          f" oracle {(Eo1 - Eo0) / Eo0:.2e}")
    assert err < 1e-5
    # the ring translates along its axis at its self-induced speed
    dz = (xg[:, 2] - fs.xyz[:, 2]).mean()
    assert abs(dz - v0[:, 2].mean() * dt * steps) < 1e-6 * abs(dz)
    # the periodic images deform it only slightly (same radii as the oracle's)
    r = np.linalg.norm(xg[:, :2] - np.pi, axis=1)
    ro = np.linalg.norm(xo[:, :2] - np.pi, axis=1)
    assert np.abs(r - math.pi / 3).max() < 1e-6
    assert np.abs(r - ro).max() < 1e-9
    # energy: conserved to the time-step error, and equal to the oracle's
    assert abs(E1 - E0) < 1e-6 * abs(E0)
    assert abs(E1 - Eo1) < 1e-6 * abs(Eo1)
