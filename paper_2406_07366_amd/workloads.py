"""Seeded synthetic filament sets (inputs only; no Biot-Savart arithmetic here).

This module is shared by the oracle, the tests and the benchmark.  It builds
closed vortex filaments as ordered node lists with unwrapped coordinates and
per-filament circulation (paper Sec. 2.1, "Filaments as oriented curves";
Sec. 2.2, eq:BS allows a circulation per curve).  Nothing here evaluates the
method: it only samples the parametric curves at their nodes.

Workloads (all in a cubic periodic box of side L = 2*pi, core a = 1e-6):

  ring     one circular ring, R = pi/3, centred in the box, axis z, 64 nodes
           equispaced in angle, Gamma = 1.                     (grid 32^3, tol 1e-6)
  ellipses 40 ellipses: centres U[0,L)^3, semi-axes U[pi/8, pi/3] each, Haar
           orientation, Gamma = +-1 with p = 1/2, 64 nodes each.
           Same generator as the paper's random-ellipse case (Sec. 5.1, test
           case 3) with its radii range and node count changed. (grid 64^3, tol 1e-6)
  tangle   1000 random Fourier curves x(t) = c + sum_{m=1..4} A_m cos(mt) +
           B_m sin(mt), A_m, B_m ~ N(0, (0.3/m)^2) per component, c U[0,L)^3,
           100 nodes each, Gamma = 1.                         (grid 256^3, tol 1e-5)
  ringpairs 5000 coaxial antiparallel ring pairs (R U[0.05, 0.2], axial gap d
           log-uniform in [1e-3, 1e-1], Haar orientation, 16 nodes per ring,
           Gamma = +1 / -1) plus 400 tangle-style curves of 100 nodes.
                                                              (grid 256^3, tol 1e-5)
  bigtangle tangle generator with 10000 curves (N = 1e6).      (grid 512^3, tol 1e-5)

Nodes are equispaced in each curve's own parameter (angle or t).  Draw order
within one seed: centres, shape parameters, orientations, circulation signs.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class FilamentSet:
    """Closed filaments in CSR form.

    offsets: int64 [nfil+1], filament l owns nodes offsets[l]:offsets[l+1].
    xyz:     float64 [N, 3], unwrapped node positions (consecutive nodes are
             close; the curve closes on itself, node N_l == node 0).
    gamma:   float64 [nfil], circulation of each filament.
    """

    name: str
    L: float
    a: float
    offsets: np.ndarray
    xyz: np.ndarray
    gamma: np.ndarray
    grid_n: int
    tol: float
    delta: float = 0.25
    # per filament, the lattice vector n of s(tau + T) = s(tau) + n L
    # (Sec. 2.1); None: every filament is closed
    periods: np.ndarray | None = None

    @property
    def n_nodes(self) -> int:
        return int(self.offsets[-1])

    @property
    def n_fil(self) -> int:
        return int(len(self.offsets) - 1)

    def subset(self, nfil: int) -> "FilamentSet":
        """The first nfil filaments, standalone in the same box."""
        off = self.offsets[: nfil + 1].copy()
        return dataclasses.replace(
            self,
            name=f"{self.name}[:{nfil}]",
            offsets=off,
            xyz=self.xyz[: off[-1]].copy(),
            gamma=self.gamma[:nfil].copy(),
        )


def _csr(counts):
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    return off


def haar_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotation matrices from normalised Gaussian quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def ring(n_nodes: int = 64, R: float = math.pi / 3, L: float = TWO_PI,
         centre=None, gamma: float = 1.0, a: float = 1e-6,
         grid_n: int = 32, tol: float = 1e-6) -> FilamentSet:
    """One circular ring in the plane z = const, positively oriented about +z."""
    c = np.full(3, L / 2) if centre is None else np.asarray(centre, float)
    th = TWO_PI * np.arange(n_nodes) / n_nodes
    xyz = np.stack([c[0] + R * np.cos(th), c[1] + R * np.sin(th),
                    np.full_like(th, c[2])], axis=1)
    return FilamentSet("ring", L, a, _csr([n_nodes]), xyz,
                       np.array([gamma]), grid_n, tol)


def ellipses(nfil: int = 40, n_per: int = 64, seed: int = 1002,
             L: float = TWO_PI, rmin: float = math.pi / 8, rmax: float = math.pi / 3,
             a: float = 1e-6, grid_n: int = 64, tol: float = 1e-6) -> FilamentSet:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, L, size=(nfil, 3))
    axes = rng.uniform(rmin, rmax, size=(nfil, 2))
    rot = haar_rotations(rng, nfil)
    gamma = np.where(rng.uniform(size=nfil) < 0.5, -1.0, 1.0)
    th = TWO_PI * np.arange(n_per) / n_per
    local = np.zeros((nfil, n_per, 3))
    local[:, :, 0] = axes[:, 0:1] * np.cos(th)[None, :]
    local[:, :, 1] = axes[:, 1:2] * np.sin(th)[None, :]
    xyz = centres[:, None, :] + np.einsum("fij,fnj->fni", rot, local)
    return FilamentSet("ellipses", L, a, _csr([n_per] * nfil),
                       xyz.reshape(-1, 3), gamma, grid_n, tol)


def _fourier_curves(rng, nfil, n_per, L, amp=0.3, nharm=4):
    centres = rng.uniform(0.0, L, size=(nfil, 3))
    sd = amp / np.arange(1, nharm + 1)
    A = rng.standard_normal((nfil, nharm, 3)) * sd[None, :, None]
    B = rng.standard_normal((nfil, nharm, 3)) * sd[None, :, None]
    t = TWO_PI * np.arange(n_per) / n_per
    m = np.arange(1, nharm + 1)
    cos_mt = np.cos(np.outer(m, t))  # [nharm, n_per]
    sin_mt = np.sin(np.outer(m, t))
    xyz = (centres[:, None, :]
           + np.einsum("fmc,mn->fnc", A, cos_mt)
           + np.einsum("fmc,mn->fnc", B, sin_mt))
    return xyz.reshape(-1, 3)


def tangle(nfil: int = 1000, n_per: int = 100, seed: int = 1003,
           L: float = TWO_PI, a: float = 1e-6, grid_n: int = 256,
           tol: float = 1e-5, name: str = "tangle") -> FilamentSet:
    rng = np.random.default_rng(seed)
    xyz = _fourier_curves(rng, nfil, n_per, L)
    return FilamentSet(name, L, a, _csr([n_per] * nfil), xyz,
                       np.ones(nfil), grid_n, tol)


def ringpairs(npairs: int = 5000, n_ring: int = 16, nbg: int = 400,
              n_bg: int = 100, seed: int = 1004, L: float = TWO_PI,
              a: float = 1e-6, grid_n: int = 256, tol: float = 1e-5) -> FilamentSet:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, L, size=(npairs, 3))
    radius = rng.uniform(0.05, 0.2, size=npairs)
    gap = np.exp(rng.uniform(math.log(1e-3), math.log(1e-1), size=npairs))
    rot = haar_rotations(rng, npairs)
    th = TWO_PI * np.arange(n_ring) / n_ring
    circ = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], axis=1)  # [n,3]
    rings = []
    for sgn in (-0.5, 0.5):
        local = radius[:, None, None] * circ[None]
        local[:, :, 2] += sgn * gap[:, None]
        rings.append(centres[:, None, :] + np.einsum("fij,fnj->fni", rot, local))
    # interleave: pair p -> filaments 2p (Gamma=+1, z=-d/2) and 2p+1 (Gamma=-1)
    pair_xyz = np.stack(rings, axis=1).reshape(2 * npairs * n_ring, 3)
    pair_gamma = np.tile([1.0, -1.0], npairs)
    bg = _fourier_curves(rng, nbg, n_bg, L)
    xyz = np.concatenate([pair_xyz, bg], axis=0)
    gamma = np.concatenate([pair_gamma, np.ones(nbg)])
    counts = [n_ring] * (2 * npairs) + [n_bg] * nbg
    return FilamentSet("ringpairs", L, a, _csr(counts), xyz, gamma, grid_n, tol)


def bigtangle(nfil: int = 10000, seed: int = 1005) -> FilamentSet:
    return tangle(nfil=nfil, n_per=100, seed=seed, grid_n=512, tol=1e-5,
                  name="bigtangle")


WORKLOADS = {
    "ring": ring,
    "ellipses": ellipses,
    "tangle": tangle,
    "ringpairs": ringpairs,
    "bigtangle": bigtangle,
}


def leapfrog(n_per: int = 32, L: float = TWO_PI, a: float = 1e-6, grid_n: int = 32,
             tol: float = 1e-6) -> FilamentSet:
    """Two coaxial elliptical rings of Sec. 5.2 (leapfrogging test): planes
    orthogonal to x at distance L/4, minor radius R_a = L/4 and major radius
    R_b = sqrt(2) R_a, the major axes along y and along z respectively, both
    oriented about +x (so both travel along +x), Gamma = 1."""
    Ra = L / 4
    Rb = math.sqrt(2) * Ra
    th = TWO_PI * np.arange(n_per) / n_per
    c1 = np.array([L / 4, L / 2, L / 2])
    c2 = c1 + np.array([L / 4, 0.0, 0.0])
    r1 = np.stack([np.full_like(th, c1[0]), c1[1] + Rb * np.cos(th), c1[2] + Ra * np.sin(th)], 1)
    r2 = np.stack([np.full_like(th, c2[0]), c2[1] + Ra * np.cos(th), c2[2] + Rb * np.sin(th)], 1)
    return FilamentSet("leapfrog", L, a, _csr([n_per, n_per]), np.concatenate([r1, r2]),
                       np.array([1.0, 1.0]), grid_n, tol)


WORKLOADS["leapfrog"] = leapfrog


def perf_ellipses(n_ell: int, n_per: int = 32, seed: int = 1006, L: float = TWO_PI,
                  a: float = 1e-8, tol: float = 1e-6) -> FilamentSet:
    """The random-ellipse case of the paper's performance tests (Sec. 5.3,
    after the third test case of Sec. 5.1): ellipses at uniform random
    positions with Haar orientations, minor and major radii independent and
    uniform in [L/16, L/4], Gamma = 1, n_per nodes each equispaced in angle,
    a = 1e-8.  grid_n is set per tolerance by perf_params."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, L, size=(n_ell, 3))
    axes = rng.uniform(L / 16, L / 4, size=(n_ell, 2))
    rot = haar_rotations(rng, n_ell)
    th = TWO_PI * np.arange(n_per) / n_per
    local = np.zeros((n_ell, n_per, 3))
    local[:, :, 0] = axes[:, 0:1] * np.cos(th)[None, :]
    local[:, :, 1] = axes[:, 1:2] * np.sin(th)[None, :]
    xyz = centres[:, None, :] + np.einsum("fij,fnj->fni", rot, local)
    return FilamentSet(f"perf_ellipses[{n_ell}]", L, a, _csr([n_per] * n_ell),
                       xyz.reshape(-1, 3), np.ones(n_ell), 32, tol)


def perf_params(N: int, beta: float, C_beta: float, L: float = TWO_PI, sigma: float = 1.5,
                w: int = 8):
    """Parameters of the performance tests for N nodes and one Table 1 row:
    alpha = C_beta N^(1/3) / L (eq:alpha_optimal_performance), r_c = beta /
    alpha, and a grid whose retained modes reach k_max = 2 beta alpha
    (K >= beta alpha L / pi with K = floor((floor(n / sigma) - 1) / 2)): the
    smallest multiple of 8 with no prime factor above 7 (fast transforms), or
    the next power of two if it is at most 15 % larger (pruned transforms)."""
    alpha = C_beta * N ** (1.0 / 3.0) / L

    def ok(n):
        return n >= w + 8 and (int(n / sigma + 1e-9) - 1) // 2 >= kmin

    def smooth(n):
        for f in (2, 3, 5, 7):
            while n % f == 0:
                n //= f
        return n == 1

    kmin = math.ceil(beta * alpha * L / math.pi - 1e-9)
    n = 8
    while not (ok(n) and smooth(n)):
        n += 8
    p2 = 16
    while not ok(p2):
        p2 *= 2
    if p2 <= 1.15 * n:
        n = p2
    return dict(alpha=alpha, rcut=beta / alpha, grid_n=n, beta=beta, w=w, sigma=sigma)


def six_lines(n_per: int = 128, L: float = TWO_PI, a: float = 1e-8, grid_n: int = 64,
              tol: float = 1e-6, signs=(1, 1, 1)) -> FilamentSet:
    """The infinite-lines case of Sec. 5.1: straight lines through the box,
    a pair along each Cartesian axis with opposite orientations (zero net
    vorticity), n_per nodes each.  The lines along z pass through
    (x, y) = (1/8, 3/8) L and (5/8, 7/8) L, those along x through
    (y, z) = the same, those along y through (z, x) = the same, so that no
    two lines meet (the closest pairs are L/4 apart); signs[a] orients the
    first line of the pair along axis a (+1: along +axis)."""
    u = L * np.arange(n_per) / n_per
    parts, periods, gam = [], [], []
    for ax in range(3):                       # 0: x-lines, 1: y-lines, 2: z-lines
        t1, t2 = (ax + 1) % 3, (ax + 2) % 3    # transverse axes (cyclic)
        for k, (c1, c2) in enumerate(((0.125, 0.375), (0.625, 0.875))):
            sgn = signs[ax] * (1 if k == 0 else -1)
            p = np.zeros((n_per, 3))
            p[:, ax] = u if sgn > 0 else L - u
            p[:, t1] = c1 * L
            p[:, t2] = c2 * L
            parts.append(p)
            per = [0, 0, 0]
            per[ax] = sgn
            periods.append(per)
            gam.append(1.0)
    return FilamentSet("six_lines", L, a, _csr([n_per] * 6), np.concatenate(parts),
                       np.array(gam), grid_n, tol, periods=np.array(periods, dtype=np.int64))


WORKLOADS["six_lines"] = six_lines


def helices(n_per: int = 48, amp: float = 0.4, L: float = TWO_PI, a: float = 1e-6,
            grid_n: int = 32, tol: float = 1e-6) -> FilamentSet:
    """Two wavy infinite lines (periods +e_z and -e_z, zero net vorticity)
    about the axes (x, y) = (L/4, L/3) and (3L/4, 2L/3): curved unclosed
    filaments, for the closing segment's treatment in every term."""
    tau = L * np.arange(n_per) / n_per
    parts = []
    for k, (cx, cy, sgn) in enumerate(((L / 4, L / 3, 1), (3 * L / 4, 2 * L / 3, -1))):
        z = tau if sgn > 0 else L - tau
        parts.append(np.stack([cx + amp * np.cos(2 * z + k), cy + amp * np.sin(3 * z), z], 1))
    return FilamentSet("helices", L, a, _csr([n_per] * 2), np.concatenate(parts),
                       np.array([1.0, 1.0]), grid_n, tol,
                       periods=np.array([[0, 0, 1], [0, 0, -1]], dtype=np.int64))


WORKLOADS["helices"] = helices


def trefoil(n: int = 512, L: float = TWO_PI, a: float = 1e-6, grid_n: int = 64,
            tol: float = 1e-6) -> FilamentSet:
    """The trefoil knot of Sec. 5.1: one knotted curve X(theta) =
    R (sin t + 2 sin 2t, cos t - 2 cos 2t, -sin 3t), R = L/6, n nodes
    equispaced in theta, centred in the box, Gamma = 1."""
    R = L / 6
    th = 2 * np.pi * np.arange(n) / n
    x = R * np.stack([np.sin(th) + 2 * np.sin(2 * th), np.cos(th) - 2 * np.cos(2 * th),
                      -np.sin(3 * th)], 1) + L / 2
    return FilamentSet("trefoil", L, a, _csr([n]), x, np.array([1.0]), grid_n, tol)


WORKLOADS["trefoil"] = trefoil


def make(name: str, **kw) -> FilamentSet:
    return WORKLOADS[name](**kw)
