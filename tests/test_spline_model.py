"""CPU model of the device spline solves (no GPU).

Re-derives in numpy, with the kernels' own coefficients and index arithmetic,
that
  * the cyclic tridiagonal slope system of the cubic spline, solved by six
    steps of parallel cyclic reduction with periodic neighbour indices, is
    the periodic cubic interpolating spline (also for power-of-two n, where
    at distance n/2 both neighbours are the same node);
  * the quintic spline in Hermite form (node values s, slopes D and second
    derivatives S; C^3 and C^4 conditions at every node give a cyclic
    block-tridiagonal system with 2x2 blocks), solved by block parallel
    cyclic reduction (at distance n/2 of a power-of-two n the two couplings
    to the same node are merged), is the periodic quintic interpolating spline of App. B
    (scipy's, with knots at the chord-length nodes), and its quintic Hermite
    segments reproduce that spline between the nodes.
"""
import numpy as np
import pytest
import scipy.interpolate

PCR_STEPS_CUBIC = 6
PCR_STEPS_QUINTIC = 8


def _curve(n, seed, spread=0.45):
    rng = np.random.default_rng(seed)
    th = 2 * np.pi * (np.arange(n) + spread * rng.uniform(size=n)) / n
    return np.stack([1.3 * np.cos(th), 0.7 * np.sin(th), 0.2 * np.sin(3 * th)], 1)


def _tau(x):
    h = np.linalg.norm(np.roll(x, -1, 0) - x, axis=1)
    return h, np.concatenate([[0], np.cumsum(h)])


# ------------------------------------------------------------------ cubic
def cubic_pcr(h, x):
    """Slopes D of the periodic cubic spline: h_j D_{j-1} + 2(h_{j-1}+h_j) D_j
    + h_{j-1} D_{j+1} = 3(h_j d_{j-1} + h_{j-1} d_j), by the kernel's PCR."""
    n = len(h)
    hm = np.roll(h, 1)
    a, b, c = h.copy(), 2 * (hm + h), hm.copy()
    d = (np.roll(x, -1, 0) - x) / h[:, None]
    r = 3 * (h[:, None] * np.roll(d, 1, 0) + hm[:, None] * d)
    dist = 1
    for _ in range(PCR_STEPS_CUBIC):
        dm = dist % n
        a2, b2, c2, r2 = a.copy(), b.copy(), c.copy(), r.copy()
        for i in range(n):
            im, ip = (i - dm) % n, (i + dm) % n
            k1, k2 = a[i] / b[im], c[i] / b[ip]
            a2[i] = -k1 * a[im]
            c2[i] = -k2 * c[ip]
            b2[i] = b[i] - k1 * c[im] - k2 * a[ip]
            r2[i] = r[i] - k1 * r[im] - k2 * r[ip]
        a, b, c, r = a2, b2, c2, r2
        dist *= 2
    return r / b[:, None]


@pytest.mark.parametrize("n", [3, 4, 5, 7, 8, 12, 16, 31, 32, 64, 100])
def test_cubic_pcr_matches_periodic_cubic_spline(n):
    x = _curve(n, n)
    h, tau = _tau(x)
    D = cubic_pcr(h, x)
    sp = scipy.interpolate.CubicSpline(tau, np.vstack([x, x[:1]]), bc_type="periodic")
    np.testing.assert_allclose(D, sp(tau[:-1], 1), rtol=0, atol=1e-12)


def test_six_reduction_steps_suffice_for_any_spacing():
    """Every row has |a| + |c| = |b| / 2; a reduction step maps the ratio
    lambda = max (|a| + |c|) / |b| to at most lambda^2 / (1 - lambda^2), so
    six steps leave couplings below 4e-15 of the diagonal whatever n and
    the spacings.  Checked on chord lengths spread over 3000:1: the six-step
    slopes equal a dense solve of the cyclic system."""
    lam = 0.5
    for _ in range(PCR_STEPS_CUBIC):
        lam = lam * lam / (1 - lam * lam)
    assert lam < 4.1e-15
    rng = np.random.default_rng(7)
    for n in (3, 5, 16, 40, 64, 127, 128):
        for _ in range(5):
            h = np.exp(rng.uniform(-4, 4, n))
            tau = np.concatenate([[0], np.cumsum(h)])
            x = rng.normal(size=(n, 3))
            hm = np.roll(h, 1)
            A = np.zeros((n, n))
            for i in range(n):
                A[i, (i - 1) % n] += h[i]
                A[i, i] += 2 * (hm[i] + h[i])
                A[i, (i + 1) % n] += hm[i]
            d = (np.roll(x, -1, 0) - x) / h[:, None]
            r = 3 * (h[:, None] * np.roll(d, 1, 0) + hm[:, None] * d)
            ref = np.linalg.solve(A, r)
            D = cubic_pcr(h, x)
            assert np.abs(D - ref).max() <= 1e-13 * np.abs(ref).max(), (n, tau[-1])


# ----------------------------------------------------------------- quintic
def quintic_blocks(h, x):
    """Rows of node i (unknowns X = (D, S)): C^3 row scaled by 1/3 and C^4 row
    scaled by -1/12 of the quintic Hermite segments on both sides.
    Returns L, M, U [n,2,2] and R [n,2,3]."""
    n = len(h)
    hm, hp = np.roll(h, 1), h
    im2, ip2 = 1 / hm ** 2, 1 / hp ** 2
    im3, ip3 = 1 / hm ** 3, 1 / hp ** 3
    L = np.zeros((n, 2, 2)); M = np.zeros((n, 2, 2)); U = np.zeros((n, 2, 2))
    L[:, 0, 0], L[:, 0, 1] = -8 * im2, -1 / hm
    M[:, 0, 0], M[:, 0, 1] = 12 * (ip2 - im2), 3 * (1 / hm + 1 / hp)
    U[:, 0, 0], U[:, 0, 1] = 8 * ip2, -1 / hp
    L[:, 1, 0], L[:, 1, 1] = 14 * im3, 2 * im2
    M[:, 1, 0], M[:, 1, 1] = 16 * (im3 + ip3), -3 * (im2 - ip2)
    U[:, 1, 0], U[:, 1, 1] = 14 * ip3, -2 * ip2
    dm_ = (x - np.roll(x, 1, 0))          # s_i - s_{i-1}
    dp_ = (np.roll(x, -1, 0) - x)         # s_{i+1} - s_i
    R = np.zeros((n, 2, 3))
    R[:, 0] = 20 * (dp_ * ip3[:, None] - dm_ * im3[:, None])
    R[:, 1] = 30 * (dm_ / hm[:, None] ** 4 + dp_ / hp[:, None] ** 4)
    return L, M, U, R


def block_pcr(L, M, U, R):
    n = len(M)
    dist = 1
    for _ in range(PCR_STEPS_QUINTIC):
        dm = dist % n
        L2, M2, U2, R2 = L.copy(), M.copy(), U.copy(), R.copy()
        for i in range(n):
            im, ip = (i - dm) % n, (i + dm) % n
            if 2 * dm == n:
                # both neighbours are node ip: one coupling L_i + U_i
                Ci, Cj = L[i] + U[i], L[ip] + U[ip]
                K = Ci @ np.linalg.inv(M[ip])
                M2[i] = M[i] - K @ Cj
                R2[i] = R[i] - K @ R[ip]
                L2[i] = U2[i] = 0.0
            else:
                K1 = L[i] @ np.linalg.inv(M[im])
                K2 = U[i] @ np.linalg.inv(M[ip])
                L2[i] = -K1 @ L[im]
                U2[i] = -K2 @ U[ip]
                M2[i] = M[i] - K1 @ U[im] - K2 @ L[ip]
                R2[i] = R[i] - K1 @ R[im] - K2 @ R[ip]
        L, M, U, R = L2, M2, U2, R2
        dist *= 2
    X = np.linalg.solve(M, R)             # [n,2,3]
    return X[:, 0], X[:, 1]


def quintic_hermite(s0, s1, D0, D1, S0, S1, h, u, deriv):
    """Quintic on [0, h] from values, slopes and second derivatives at both
    ends, at t = u h (deriv 0, 1, 2)."""
    E0 = (s1 - s0 - D0 * h - S0 * h * h / 2) / h ** 3
    E1 = (D1 - D0 - S0 * h) / h ** 2
    E2 = (S1 - S0) / h
    c3 = 10 * E0 - 4 * E1 + E2 / 2
    c4 = (7 * E1 - 15 * E0 - E2) / h
    c5 = (E2 - 6 * E1 + 12 * E0) / (2 * h * h)
    t = u * h
    if deriv == 0:
        return s0 + t * (D0 + t * (S0 / 2 + t * (c3 + t * (c4 + t * c5))))
    if deriv == 1:
        return D0 + t * (S0 + t * (3 * c3 + t * (4 * c4 + t * 5 * c5)))
    return S0 + t * (6 * c3 + t * (12 * c4 + t * 20 * c5))


@pytest.mark.parametrize("n", [6, 7, 8, 9, 12, 16, 23, 32, 64, 100])
def test_quintic_block_pcr_matches_periodic_quintic_spline(n):
    x = _curve(n, 100 + n)
    h, tau = _tau(x)
    D, S = block_pcr(*quintic_blocks(h, x))
    sp = scipy.interpolate.make_interp_spline(tau, np.vstack([x, x[:1]]), k=5,
                                              bc_type="periodic")
    np.testing.assert_allclose(D, sp(tau[:-1], 1), rtol=0, atol=1e-11)
    np.testing.assert_allclose(S, sp(tau[:-1], 2), rtol=0, atol=1e-9)
    rng = np.random.default_rng(n)
    for j in rng.integers(0, n, 6):
        jn = (j + 1) % n
        for u in (0.13, 0.5, 0.91):
            for d in range(3):
                got = quintic_hermite(x[j], x[jn], D[j], D[jn], S[j], S[jn], h[j], u, d)
                np.testing.assert_allclose(got, sp(tau[j] + u * h[j], d), rtol=0,
                                           atol=1e-11 * 10 ** d)


def test_quintic_blocks_are_invertible_for_any_spacing():
    """det M = -12 (1/h_- + 1/h_+)^4 < 0 for the diagonal block."""
    for hm, hp in ((1.0, 1.0), (1.0, 1e-3), (0.07, 3.0)):
        _, M, _, _ = quintic_blocks(np.array([hp, 1.0, hm]), np.zeros((3, 3)))
        det = np.linalg.det(M[0])
        np.testing.assert_allclose(det, -12 * (1 / hm + 1 / hp) ** 4, rtol=1e-12)
