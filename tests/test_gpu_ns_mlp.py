"""Learned near-singular correction: training samples against independent
quadrature, and what the trained network gains over the method without it.

The learned output has no counterpart in the paper (parity unpinned by the
paper); it is judged against the oracle's adaptive Gauss-Kronrod integrals."""
import math

import numpy as np
import pytest
import scipy.integrate

from oracle import oracle as O
from paper_2406_07366_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_07366_amd import binding
    return binding


def rel_l2(a, b):
    return math.sqrt(((a - b) ** 2).sum(1).mean() / (b ** 2).sum(1).mean())


def test_ns_samples_match_scipy_quadrature(B):
    """Each sample's exact integral (aux) is the segment integral of the cubic
    the features describe; checked with scipy.quad, and the target, its
    multiplier and error scale against the oracle's straight-chord closed form
    and quadrature along the tangent segment."""
    import torch
    print("\n[case] ns samples n=24", flush=True)
    rng = np.random.default_rng(11)
    U = torch.from_numpy(rng.random((24, 8))).cuda()
    X, T, A = B.ns_samples(U)
    X, T, A = X.cpu().numpy().astype(np.float64), T.cpu().numpy(), A.cpu().numpy()
    for i in range(24):
        x = X[i, :3]
        D0 = np.array([X[i, 3], X[i, 4], 0.0]); D1 = X[i, 5:8]
        P0, P1 = np.array([-0.5, 0, 0]), np.array([0.5, 0, 0])
        c2 = 3 * (P1 - P0) - 2 * D0 - D1
        c3 = 2 * (P0 - P1) + D0 + D1
        s = lambda u: P0 + u * (D0 + u * (c2 + u * c3))
        ds = lambda u: D0 + u * (2 * c2 + 3 * u * c3)
        ref = []
        for k in range(3):
            f = lambda u: np.cross(s(u) - x, ds(u))[k] / np.linalg.norm(s(u) - x) ** 3
            ref.append(scipy.integrate.quad(f, 0, 1, epsabs=0, epsrel=1e-12, limit=500)[0])
        ref = np.array(ref)
        # features are float32: allow their rounding
        np.testing.assert_allclose(A[i, 1:4], ref, rtol=1e-4, atol=1e-6 * np.abs(ref).max())
        # the target removes the straight tangent segment at the closest point
        us = np.linspace(0, 1, 20001)
        pts = np.array([s(u) for u in us])
        k = np.argmin(np.linalg.norm(pts - x, axis=1))
        P, tan = pts[k], ds(us[k]) / np.linalg.norm(ds(us[k]))
        d = np.linalg.norm(P - x)
        a_, b_ = np.linalg.norm(P - s(0)), np.linalg.norm(s(1) - P)
        tang = O.chord_integral(P - a_ * tan, P + b_ * tan, x) * 4 * math.pi
        mult = 1 + math.log1p(1 / d)
        # absolute integral of the tangent segment, by quadrature
        Sabs = scipy.integrate.quad(
            lambda l: 1.0 / np.linalg.norm(P + (l - a_) * tan - x) ** 2, 0, a_ + b_,
            points=[a_], epsabs=0, epsrel=1e-12, limit=500)[0]
        np.testing.assert_allclose(A[i, 0], d, rtol=1e-3)
        np.testing.assert_allclose(A[i, 4], mult, rtol=1e-3)
        np.testing.assert_allclose(A[i, 5], Sabs, rtol=2e-3)
        np.testing.assert_allclose(T[i] * mult, ref - tang, rtol=2e-2,
                                   atol=2e-3 * np.abs(ref).max())


@pytest.fixture(scope="module")
def trained(B):
    from paper_2406_07366_amd import ns_mlp
    print("\n[case] learned NS: train 5e5 samples", flush=True)
    return ns_mlp.train(n_train=500_000, n_val=100_000, epochs=40, batch=4096)


def test_error_table_matches_host_computation(B, trained):
    """bs_ns_error_table against the same statistic formed on the host from
    the network's outputs on the same samples (bins by chord distance over h)."""
    from paper_2406_07366_amd import ns_mlp
    mlp, tab, info = trained
    Xv, Tv, Av = ns_mlp.make_dataset(20_000, 5)
    rms, mx = B.ns_error_table(mlp, Xv, Tv, Av)
    Y = mlp.forward(Xv).double().cpu().numpy()
    T = Tv.double().cpu().numpy()
    A = Av.cpu().numpy()
    e = A[:, 4] * np.linalg.norm(Y - T, axis=1)
    lo, hi, nb = B.ns_error_bins()
    t = (np.log10(A[:, 6]) - math.log10(lo)) / (math.log10(hi) - math.log10(lo))
    b = np.clip((t * nb).astype(np.int64), 0, nb - 1)
    for k in range(nb):
        sel = e[b == k]
        if len(sel) == 0:
            assert np.isinf(rms[k]) and np.isinf(mx[k])
            continue
        np.testing.assert_allclose(rms[k], math.sqrt((sel ** 2).mean()), rtol=1e-5)
        np.testing.assert_allclose(mx[k], sel.max(), rtol=1e-6)
    print("  rms per bin: " + " ".join(f"{v:.1e}" for v in rms))


def test_learned_correction_gain(B, trained):
    """Ring pairs: error against the reference with exact near-singular
    integrals, for the plain Q-point rule, the graded panels, the mapped
    rule, the network on every pair in its sample box, and the network with
    its error indicator (mapped rule elsewhere), at tolerance 1e-5 and at
    1e-2, where the indicator lets the network carry pairs."""
    mlp, tab, info = trained
    fs = W.ringpairs(npairs=150, nbg=20, seed=77)
    fs.grid_n = 64
    ref, _ = O.Oracle(fs).reference(psi=False, ns_eta=1.0)
    xyz, g = B.load_workload(fs)
    errs, counts = {}, {}
    for name, mode, table, tol in (("plain", B.BS_NS_OFF, None, 1e-5),
                                   ("adaptive", B.BS_NS_ADAPTIVE, None, 1e-5),
                                   ("mapped", B.BS_NS_MAPPED, None, 1e-5),
                                   ("mlp_only", B.BS_NS_MLP, np.zeros_like(tab), 1e-5),
                                   ("mlp_1e-5", B.BS_NS_MLP, tab, 1e-5),
                                   ("mlp_1e-2", B.BS_NS_MLP, tab, 1e-2)):
        fs.tol = tol
        plan = B.Plan(B.params_for(fs, ns_mode=mode, precision=B.BS_FP32_MIXED))
        if table is not None:
            plan.set_mlp(mlp, table)
        plan.set_filaments(fs.offsets, xyz, g)
        v = plan.velocity().cpu().numpy()
        plan.status()
        counts[name] = plan.ns_counts()
        errs[name] = rel_l2(v, ref)
        npairs, nfb = counts[name]
        print(f"  {name:9s} rel_l2 {errs[name]:.3e}  pairs {npairs} by network "
              f"{npairs - nfb if mode == B.BS_NS_MLP else 0}")
        plan.close()
    assert errs["adaptive"] <= 1e-6 and errs["mapped"] <= 1e-6
    # the network alone gains over the Q-point rule (by 30x or more)
    assert errs["mlp_only"] < errs["plain"] / 30
    # with its indicator the learned path meets the tolerance it is run at
    assert errs["mlp_1e-5"] <= 1e-5
    assert errs["mlp_1e-2"] <= 1e-2
    # the network carries pairs where its error is within the budget
    assert counts["mlp_1e-2"][1] < counts["mlp_1e-2"][0]


def test_set_mlp_drops_recorded_graph(B):
    """A bs_step graph recorded with one network, then bs_set_mlp with
    another: the next step equals an eager evaluation with the second
    network bitwise (no stale network in the replayed graph)."""
    import torch
    fs = W.ringpairs(npairs=40, nbg=4, seed=5)
    fs.grid_n = 32
    lo, hi, nb = B.ns_error_bins()
    zero = np.zeros(nb, dtype=np.float32)
    netA, netB = B.MLP(B.mlp_init(0)), B.MLP(B.mlp_init(1))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        print("\n[case] graph + set_mlp", flush=True)
        xyz, g = B.load_workload(fs)
        out = torch.empty((fs.n_nodes, 3), dtype=torch.float64, device="cuda")
        ref = torch.empty_like(out)
        eager = B.Plan(B.params_for(fs, ns_mode=B.BS_NS_MLP), stream=s)
        eager.set_mlp(netB, zero)
        eager.set_filaments(fs.offsets, xyz, g)
        eager.velocity(ref)
        plan = B.Plan(B.params_for(fs, ns_mode=B.BS_NS_MLP), stream=s)
        plan.set_mlp(netA, zero)
        plan.set_graph(True)
        for _ in range(3):
            plan.step(fs.offsets, xyz, g, out)
        s.synchronize()
        vA = out.cpu().numpy()
        plan.set_mlp(netB, zero)
        assert not plan.graph_active()
        for k in range(3):
            out.fill_(float(k))
            plan.step(fs.offsets, xyz, g, out)
            s.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref.cpu().numpy()), k
        assert not np.array_equal(vA, ref.cpu().numpy())
        plan.close()
        eager.close()
