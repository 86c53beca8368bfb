"""Write the oracle reference values that bench.py reports its accuracy against.

Calls only the FP64 CPU oracle (oracle/) and the seeded input generators;
run from the repository root:  python tests/golden/make_references.py [names]

  ref_ellipses.npz   velocities at every node of the 40-ellipse workload
  ref_tangle.npz     velocities at 256 sampled nodes of the 1e5-node tangle
  ref_ringpairs.npz  velocities (with exact near-singular segment integrals)
                     at 256 sampled nodes of the ring-pair workload
  ref_bigtangle.npz  velocities (with exact near-singular segment integrals)
                     at 512 sampled nodes of the 1e6-node tangle: 256 drawn
                     uniformly, 256 among the nodes that have a node of
                     another filament within 0.05 (where near-singular pairs
                     occur)
  ref_bigtangle_subset_energy.npz
                     energy after each of 10 RK4 steps of the first 100
                     filaments of the 1e6-node tangle (dt = Kelvin period of
                     the whole tangle's shortest chord), with exact
                     near-singular integrals in the velocities

Reference parameters: beta = 6.5 (ellipses) / 6.0 (others), r_c = L or L/2.
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O                    # noqa: E402
from paper_2406_07366_amd import workloads as W   # noqa: E402

EULER_GAMMA = 0.5772156649015329


def sample_idx(n, k=256, seed=0):
    return np.sort(np.random.default_rng(seed).choice(n, k, replace=False))


def kelvin_period(lam, a, delta=0.25, kappa=1.0):
    return 2 * lam ** 2 / kappa / (math.log(lam / (math.pi * a)) + 0.5 - (delta + EULER_GAMMA))


def min_chord(fs):
    nxt = np.arange(fs.n_nodes) + 1
    nxt[fs.offsets[1:] - 1] = fs.offsets[:-1]
    return float(np.linalg.norm(fs.xyz[nxt] - fs.xyz, axis=1).min())


def ellipses():
    fs = W.ellipses()
    v, p = O.Oracle(fs).reference()
    np.savez(os.path.join(HERE, "ref_ellipses.npz"), idx=np.arange(fs.n_nodes), v=v, psi=p)


def tangle():
    fs = W.tangle()
    idx = sample_idx(fs.n_nodes)
    v, _ = O.Oracle(fs).reference(targets=idx, beta=6.0, psi=False)
    np.savez(os.path.join(HERE, "ref_tangle.npz"), idx=idx, v=v)


def ringpairs():
    fs = W.ringpairs()
    idx = sample_idx(fs.n_nodes)
    v, _ = O.Oracle(fs).reference(targets=idx, beta=6.0, psi=False, ns_eta=1.0)
    np.savez(os.path.join(HERE, "ref_ringpairs.npz"), idx=idx, v=v)


def close_nodes(fs, radius=0.05):
    """Nodes with a node of another filament within radius (minimum image):
    input selection only, by a k-d tree over the node positions."""
    from scipy.spatial import cKDTree
    fil = np.repeat(np.arange(fs.n_fil), np.diff(fs.offsets))
    x = np.mod(fs.xyz, fs.L) % fs.L
    tree = cKDTree(x, boxsize=fs.L)
    pairs = tree.query_pairs(radius, output_type="ndarray")
    other = pairs[fil[pairs[:, 0]] != fil[pairs[:, 1]]]
    return np.unique(other.ravel())


def bigtangle():
    fs = W.bigtangle()
    uni = sample_idx(fs.n_nodes)
    close = close_nodes(fs)
    rng = np.random.default_rng(1)
    near = np.sort(rng.choice(np.setdiff1d(close, uni), 256, replace=False))
    idx = np.concatenate([uni, near])
    v, _ = O.Oracle(fs).reference(targets=idx, beta=6.0, psi=False, ns_eta=1.0)
    np.savez(os.path.join(HERE, "ref_bigtangle.npz"), idx=idx, v=v, n_uniform=len(uni))


def bigtangle_subset_energy(steps=10):
    full = W.bigtangle()
    dt = kelvin_period(min_chord(full), full.a)
    fs = full.subset(100)
    prm = O.reference_params(fs.L, 6.0, fs.L / 2)

    def make(x):
        return O.Oracle(W.FilamentSet(**{**fs.__dict__, "xyz": x}))

    def energy(x):
        o = make(x)
        _, p = o.ewald(prm["alpha"], prm["rc"], prm["K"])
        return o.energy(p)

    def vel(x):
        v, _ = make(x).ewald(prm["alpha"], prm["rc"], prm["K"], psi=False, ns_eta=1.0)
        return v

    x = fs.xyz.copy()
    E = [energy(x)]
    for k in range(steps):
        ks = []
        for c in (0.0, 0.5, 0.5, 1.0):
            ks.append(vel(x + c * dt * ks[-1] if ks else x))
        x = x + dt / 6 * (ks[0] + 2 * ks[1] + 2 * ks[2] + ks[3])
        E.append(energy(x))
        print(f"  step {k + 1}: E = {E[-1]:.15e}", flush=True)
    np.savez(os.path.join(HERE, "ref_bigtangle_subset_energy.npz"), E=np.array(E), dt=dt,
             x_final=x)


JOBS = {"ellipses": ellipses, "tangle": tangle, "ringpairs": ringpairs,
        "bigtangle": bigtangle, "bigtangle_subset_energy": bigtangle_subset_energy}

if __name__ == "__main__":
    for name in (sys.argv[1:] or list(JOBS)):
        t0 = time.time()
        JOBS[name]()
        print(f"{name}: {time.time() - t0:.1f} s", flush=True)
