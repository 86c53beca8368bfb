"""Benchmark: filament nodes per second per Biot-Savart velocity evaluation.

One step = bs_set_filaments (device-resident positions in: chord lengths,
spline fit, quadrature points, binning) + bs_velocity (local, self,
short-range pairs, spread, FFT, spectral operator, inverse FFT,
interpolation), i.e. the whole hot path from node positions to node
velocities, on one MI355X.

Default workload: 40 random ellipses x 64 nodes (N = 2560), grid 64^3,
tolerance 1e-6, FP64 path (the accuracy bar of the metric: rel. l2 error
<= 1e-6 against the converged FP64 CPU oracle).  The FP32-mixed path is timed
on the same workload and reported beside it.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
from paper_2406_07366_amd.profsum import read_traffic  # noqa: E402

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_TFLOPS = 157.3     # MI355X dense fp32 vector
FP64_VECTOR_TFLOPS = 78.6
PAIR_FLOP = 60.0               # per interacting pair (erfc, exp, sqrt, div, cross, fma)
# stages made of exactly one kernel launch, and the source file of that kernel
SINGLE_KERNEL_STAGES = {"spread": "nufft.hip", "spectral": "nufft.hip", "interp": "nufft.hip",
                        "pairs": "pairs.hip"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(a, b):
    return math.sqrt(((a - b) ** 2).sum(1).mean() / (b ** 2).sum(1).mean())


GOLDEN = os.path.join(ROOT, "tests", "golden")


def load_reference(name):
    """Oracle reference values written by tests/golden/make_references.py."""
    path = os.path.join(GOLDEN, f"ref_{name}.npz")
    if not os.path.exists(path):
        return None
    return np.load(path)


def count_pairs(plan, fs, Q, rc):
    """Interacting (node, quadrature point) pairs within r_c, minimum image,
    minus the 2Q excluded points of each node's adjacent segments (quadrature
    points from the plan's own geometry)."""
    from scipy.spatial import cKDTree
    qp = plan.geometry()["qpos"].cpu().numpy()
    L = fs.L
    tree = cKDTree(np.mod(qp, L) % L, boxsize=L)
    cnt = tree.query_ball_point(np.mod(fs.xyz, L) % L, rc, return_length=True)
    return int(cnt.sum()) - 2 * Q * fs.n_nodes


def pruned_transforms(prm):
    """Whether the resolved plan uses the pruned transforms."""
    return prm.fft_mode == 2


def stage_bytes(prm, N, Nq, fp32):
    """Algorithmic HBM bytes per launch of each stage (minimum traffic)."""
    s = 4 if fp32 else 8
    n = prm.grid_n
    n3 = n ** 3
    w = prm.w
    out = {"spread": 3 * n3 * s + Nq * (16 + (3 * w + 4) * s),
           "interp": 3 * n3 * s + N * (24 + 48)}
    if pruned_transforms(prm):
        K1, NY = prm.K + 1, 2 * prm.K + 1
        a = 3 * n * n * K1 * 2 * s          # x-transformed grid, modes 0..K
        b = 3 * NY * n * K1 * 2 * s         # after y, |my| <= K
        out.update({"fft_fwd": 3 * n3 * s + a + a + b, "spectral": 2 * b,
                    "fft_inv": b + a + a + 3 * n3 * s})
    else:
        nc = n * n * (n // 2 + 1)
        out.update({"fft_fwd": 3 * n3 * s + 3 * nc * 2 * s, "spectral": 2 * 3 * nc * 2 * s,
                    "fft_inv": 3 * nc * 2 * s + 3 * n3 * s})
    return out


def time_steps(torch, plan, fs, xyz, gamma, out, steps, warmup):
    for _ in range(warmup):
        plan.set_filaments(fs.offsets, xyz, gamma)
        plan.velocity(out)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        plan.set_filaments(fs.offsets, xyz, gamma)
        plan.velocity(out)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, ev0.elapsed_time(ev1) / steps


def stage_profile(torch, plan, fs, xyz, gamma, out, steps):
    plan.set_profiling(True)
    plan.stage_times(reset=True)
    for _ in range(steps):
        plan.set_filaments(fs.offsets, xyz, gamma)
        plan.velocity(out)
    torch.cuda.synchronize()
    st = plan.stage_times(reset=True)
    plan.set_profiling(False)
    return {k: (ms / c if c else 0.0) for k, (ms, c) in st.items()}


def cpu_baseline(fs, prm, budget_s=10.0):
    """The oracle as it stands (direct Fourier sums, brute-force pairs) at the
    plan's own alpha, r_c, K on the whole workload, repeated for ~budget_s."""
    from oracle import oracle as O
    o = O.Oracle(fs, Q=prm.Q)
    t0 = time.perf_counter()
    runs = 0
    while True:
        oo = O.Oracle(fs, Q=prm.Q)          # geometry is part of the step
        oo.ewald(prm.alpha, prm.rcut, prm.K, psi=False)
        runs += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    del o
    return {"value": fs.n_nodes * runs / dt, "unit": "nodes/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{runs} full evaluations of the {fs.name} workload (N={fs.n_nodes}) "
                      f"at the GPU plan's alpha, r_c, K with direct Fourier sums, "
                      f"{dt:.1f} s"}


EULER_GAMMA = 0.5772156649015329


def kelvin_period(lam, a, delta=0.25, kappa=1.0):
    """T_kw(lambda) of Sec. 5.2; the RK4 step is dt = T_kw(l_min)."""
    return 2 * lam ** 2 / kappa / (math.log(lam / (math.pi * a)) + 0.5 - (delta + EULER_GAMMA))


def min_chord(fs):
    x = fs.xyz
    nxt = np.arange(fs.n_nodes) + 1
    nxt[fs.offsets[1:] - 1] = fs.offsets[:-1]
    return float(np.linalg.norm(x[nxt] - x, axis=1).min())


def rk4_run(torch, B, plan, fs, steps, dt):
    """steps RK4 steps on device positions; energy after each step."""
    xyz, g = B.load_workload(fs)
    plan.set_filaments(fs.offsets, xyz, g)
    E = [plan.energy(want_psi=False)[0]]
    times = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.rk4_step(fs.offsets, xyz, g, dt)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        plan.set_filaments(fs.offsets, xyz, g)
        E.append(plan.energy(want_psi=False)[0])
    plan.status()
    return np.array(E), np.array(times), xyz.cpu().numpy()


def bigtangle(args, torch, B, W):
    """Large tangle (N = 1e6, grid 512^3, FP32-mixed + learned correction):
    velocity throughput, 10 RK4 steps with energy, and the energy drift of the
    first 100 filaments (1e4 nodes) against the FP64 oracle's energies stored
    by tests/golden/make_references.py (--drift)."""
    from paper_2406_07366_amd import ns_mlp
    fs = W.bigtangle()
    N = fs.n_nodes
    dt = kelvin_period(min_chord(fs), fs.a)
    log(f"[bench] bigtangle N={N}, dt = T_kw(l_min) = {dt:.3e}")
    mlp, table, _ = ns_mlp.train(n_train=1_000_000, n_val=100_000, epochs=40, batch=8192, log=log)
    plan = B.Plan(B.params_for(fs, precision=B.BS_FP32_MIXED, ns_mode=B.BS_NS_MLP))
    plan.set_mlp(mlp, table)
    xyz, g = B.load_workload(fs)
    out = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    ms, _ = time_steps(torch, plan, fs, xyz, g, out, args.steps, args.warmup)
    st = stage_profile(torch, plan, fs, xyz, g, out, max(5, args.steps // 2))
    npairs, nfb = plan.ns_counts()
    log(f"[bench] bigtangle: {ms:.3f} ms per velocity eval, {N / ms * 1e3:.4g} nodes/s; "
        f"ns pairs {npairs}")
    log("[bench]   stages (ms): " + ", ".join(f"{k}={v:.4f}" for k, v in st.items()))
    E, tsteps, _ = rk4_run(torch, B, plan, fs, 10, dt)
    drift = E / E[0] - 1
    log(f"[bench] RK4 10 steps: {tsteps.mean() * 1e3:.2f} ms/step, energy drift "
        + " ".join(f"{d:.2e}" for d in drift))
    res = {"ms_per_eval": ms, "nodes_per_s": N / ms * 1e3, "stages": st, "dt": dt,
           "rk4_ms_per_step": tsteps.mean() * 1e3, "energy": E.tolist(), "drift": drift.tolist(),
           "ns_pairs": npairs}
    if args.drift:
        sub = fs.subset(100)
        sub.grid_n = 128
        log(f"[bench] drift subset N={sub.n_nodes}, grid 128^3")
        ps = B.Plan(B.params_for(sub, precision=B.BS_FP32_MIXED, ns_mode=B.BS_NS_MLP))
        ps.set_mlp(mlp, table)
        Eg, _, _ = rk4_run(torch, B, ps, sub, 10, dt)
        gold = load_reference("bigtangle_subset_energy")
        assert gold is not None and abs(float(gold["dt"]) - dt) < 1e-12 * dt
        Eo = gold["E"]
        rel = np.abs(Eg - Eo) / np.abs(Eo)
        log("[bench] subset |E_gpu - E_oracle|/E_oracle per step: " + " ".join(f"{r:.2e}" for r in rel))
        log("[bench] subset drift gpu " + " ".join(f"{d:.2e}" for d in Eg / Eg[0] - 1))
        log("[bench] subset drift oracle " + " ".join(f"{d:.2e}" for d in Eo / Eo[0] - 1))
        res["subset"] = {"E_gpu": Eg.tolist(), "E_oracle": Eo.tolist(), "rel": rel.tolist()}
    return res


def table1(args, torch, B, W):
    """Sec. 5.3 performance tests on the GPU: random ellipses of 32 nodes,
    quintic splines, Q = 3, a = 1e-8, FP64; per Table 1 row alpha = C_beta
    N^(1/3)/L and the smallest grid reaching k_max = 2 beta alpha.  Errors
    are taken against the tol = 1e-14 run of the same size (as the paper
    does); the paper's single-core time C_fit N log10 N is quoted as context."""
    rows = json.load(open(os.path.join(ROOT, "tests", "golden", "table1_parameters.json")))["rows"]
    for n_ell in (int(v) for v in args.table1.split(",")):
        fs = W.perf_ellipses(n_ell)
        N = fs.n_nodes
        xyz, gamma = B.load_workload(fs)
        out = torch.empty((N, 3), dtype=torch.float64, device="cuda")
        res = {}
        for tol, beta, C_beta, sigma, w, C_fit, _ in sorted(rows, key=lambda r: r[0]):
            pp = W.perf_params(N, beta, C_beta, fs.L, sigma, w)
            plan = B.Plan(B.make_params(L=fs.L, a=fs.a, tol=tol, grid_n=pp["grid_n"],
                                        alpha=pp["alpha"], w=w, sigma=sigma, Q=3, spline_order=6))
            prm = plan.params()
            steps = max(5, min(args.steps, int(2e6 / N)))
            ms, _ = time_steps(torch, plan, fs, xyz, gamma, out, steps, max(2, args.warmup // 4))
            plan.status()
            v = out.cpu().numpy()
            res[tol] = v
            ref = res[min(res)]
            err = rel_l2(v, ref) if tol > min(res) else 0.0
            paper_us = C_fit * N * math.log10(N)
            line = {"table1": {"tol": tol, "beta": beta, "N": N, "grid_n": prm.grid_n,
                               "K": prm.K, "alpha": prm.alpha, "rcut": prm.rcut,
                               "fft_mode": prm.fft_mode, "ms_per_eval": ms,
                               "nodes_per_s": N / (ms * 1e-3), "rel_l2_vs_1e-14": err,
                               "paper_cpu_core_ms": paper_us * 1e-3}}
            print(json.dumps(line), flush=True)
            plan.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="ellipses")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--detail", default=None,
                    help="also write per-stage times, rooflines and parameters to this JSON file")
    ap.add_argument("--drift", action="store_true",
                    help="bigtangle: energy drift of a 1e4-node subset against the FP64 oracle")
    ap.add_argument("--table1", default=None, metavar="SIZES",
                    help="the paper's performance tests (Sec. 5.3, Table 1) instead of the "
                         "default line: comma-separated ellipse counts (32 nodes each); one "
                         "JSON line per tolerance and size, errors against the tol = 1e-14 run")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="end with a plain 256 MiB device copy, the size reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters of a rocprofv3 --pmc run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "only single-GPU runs are implemented: the sharded multi-GPU path does not exist; use --gpus 1"}))
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2406_07366_amd import binding as B
    from paper_2406_07366_amd import workloads as W

    if args.table1:
        table1(args, torch, B, W)
        return

    if args.workload == "bigtangle":
        res = bigtangle(args, torch, B, W)
        if args.detail:
            os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
            with open(args.detail, "w") as f:
                json.dump(res, f, indent=1, default=float)
        print(json.dumps({"workload": "bigtangle", "nodes_per_s": res["nodes_per_s"],
                          "rk4_ms_per_step": res["rk4_ms_per_step"],
                          "drift_last": res["drift"][-1]}), flush=True)
        return

    fs = W.make(args.workload)
    N = fs.n_nodes
    log(f"[bench] workload {fs.name} N={N} grid={fs.grid_n}^3 tol={fs.tol}")
    xyz, gamma = B.load_workload(fs)
    out = torch.empty((N, 3), dtype=torch.float64, device="cuda")

    # reference solution (converged oracle, stored), sampled on large workloads
    gold = load_reference(fs.name)
    if gold is None:
        raise SystemExit(f"no stored reference for {fs.name}: run tests/golden/make_references.py")
    idx, ref = gold["idx"], gold["v"]

    ns_eta = None
    mlp = table = None
    if fs.name == "ringpairs":
        # near-singular pairs dominate: plain = FP64 + adaptive integrals,
        # learned = FP32-mixed + the trained network (trained here, on the GPU)
        from paper_2406_07366_amd import ns_mlp
        log("[bench] training the near-singular network (1e6 samples) ...")
        mlp, table, info = ns_mlp.train(n_train=1_000_000, n_val=100_000, epochs=40,
                                        batch=8192, log=log)
        variants = {"fp64": (B.BS_FP64, B.BS_NS_ADAPTIVE), "mixed": (B.BS_FP32_MIXED, B.BS_NS_MLP)}
        ns_eta = 1.0
    else:
        variants = {"fp64": (B.BS_FP64, B.BS_NS_OFF), "mixed": (B.BS_FP32_MIXED, B.BS_NS_OFF)}

    results = {}
    for prec_name, (prec, ns_mode) in variants.items():
        plan = B.Plan(B.params_for(fs, precision=prec, ns_mode=ns_mode))
        if ns_mode == B.BS_NS_MLP:
            plan.set_mlp(mlp, table)
        prm = plan.params()
        plan.set_filaments(fs.offsets, xyz, gamma)
        plan.velocity(out)
        plan.status()
        err = rel_l2(out.cpu().numpy()[idx], ref)
        ms_host, ms_ev = time_steps(torch, plan, fs, xyz, gamma, out, args.steps, args.warmup)
        st = stage_profile(torch, plan, fs, xyz, gamma, out, max(20, args.steps // 4))
        npairs, nfb = plan.ns_counts() if ns_mode != B.BS_NS_OFF else (0, 0)
        log(f"[bench] {prec_name} (ns_mode {ns_mode}): {ms_host:.4f} ms/step (events {ms_ev:.4f}), "
            f"rel_l2 {err:.3e}, {N / ms_host * 1e3:.4g} nodes/s, ns pairs {npairs}")
        log("[bench]   stages (ms): " + ", ".join(f"{k}={v:.4f}" for k, v in st.items()))
        results[prec_name] = dict(ms=ms_host, ms_events=ms_ev, err=err, stages=st,
                                  prm=prm.as_dict(), plan=plan, ns_mode=ns_mode, ns_pairs=npairs)

    if args.pmc_calibrate:
        src_t = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst_t = torch.empty_like(src_t)
        for _ in range(2):
            dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t

    primary = results[args.precision]
    prm = primary["prm"]
    fp32 = args.precision == "mixed"
    Nq = N * prm["Q"]
    npairs = count_pairs(primary["plan"], fs, prm["Q"], prm["rcut"])
    sb = stage_bytes(B.resolve_params(B.params_for(fs, precision=int(fp32))), N, Nq, fp32)
    st = primary["stages"]
    roof_all = {}
    for k, b in sb.items():
        if st.get(k, 0) > 0:
            roof_all[k] = dict(bound="hbm", achieved=b / (st[k] * 1e-3) / 1e9, peak=HBM_PEAK_GBS,
                               unit="GB/s", bytes=b, ms=st[k])
    if st.get("pairs", 0) > 0:
        peak = FP32_VECTOR_TFLOPS if fp32 else FP64_VECTOR_TFLOPS
        fl = npairs * PAIR_FLOP
        roof_all["pairs"] = dict(bound="alu", achieved=fl / (st["pairs"] * 1e-3) / 1e12,
                                 peak=peak, unit="TFLOP/s", flops=fl, pairs=npairs,
                                 ms=st["pairs"])
    # dominant single-kernel stage (stage events then time exactly one kernel)
    dom = max((k for k in roof_all if k in SINGLE_KERNEL_STAGES), key=lambda k: roof_all[k]["ms"])
    d = roof_all[dom]
    srcname = SINGLE_KERNEL_STAGES[dom]
    if dom == "spectral" and pruned_transforms(B.resolve_params(B.params_for(fs))):
        srcname = "fft.hip"         # the spectral operator runs inside the z transform
    src = os.path.join(ROOT, "paper_2406_07366_amd", "csrc", srcname)
    traffic = read_traffic(os.path.join(ROOT, "profiles",
                                        f"pmc_{dom}_{fs.name}_{args.precision}.txt"), src)
    roofline = {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"],
                "peak": d["peak"], "unit": d["unit"], "frac": d["achieved"] / d["peak"],
                "traffic": traffic}
    if "bytes" in d:
        roofline["algorithmic_bytes"] = d["bytes"]

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle baseline ...")
        cpu = cpu_baseline(fs, B.resolve_params(B.params_for(fs)))
        log(f"[bench] cpu baseline {cpu['value']:.4g} nodes/s on {cpu['cores']} threads")

    value = N / (primary["ms"] * 1e-3)
    other = "mixed" if args.precision == "fp64" else "fp64"
    line = {
        "metric": "filament nodes/s per velocity eval at rel. L2 err <= 1e-6 vs FP64 oracle; "
                  "FP32+MLP vs plain",
        "value": value, "unit": "nodes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": primary["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{fs.name}: {fs.n_fil} filaments, N={N}, grid {fs.grid_n}^3, "
                               f"tol {fs.tol:g}, Q={prm['Q']}, w={prm['w']}, "
                               f"beta={prm['beta']}",
                   "rel_l2_err": primary["err"],
                   "ns_mode": primary["ns_mode"],
                   "other_precision": {"name": other, "nodes_per_s": N / (results[other]["ms"] * 1e-3),
                                       "rel_l2_err": results[other]["err"],
                                       "ns_mode": results[other]["ns_mode"]}},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if args.detail:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
        with open(args.detail, "w") as f:
            json.dump({"line": line, "roofline_all": roof_all,
                       "stages": {k: v["stages"] for k, v in results.items()},
                       "params": {k: v["prm"] for k, v in results.items()},
                       "pairs": npairs}, f, indent=1, default=float)
    for r in results.values():
        r["plan"].close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
