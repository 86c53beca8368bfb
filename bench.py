"""Benchmark: filament nodes per second per Biot-Savart velocity evaluation.

One step = bs_set_filaments (device-resident positions in: chord lengths,
spline fit, quadrature points, binning) + bs_velocity (local, self,
short-range pairs, spread, FFT, spectral operator, inverse FFT,
interpolation), i.e. the whole hot path from node positions to node
velocities, on one MI355X.

Default workload: the large random Fourier tangle (10000 curves x 100 nodes,
N = 1e6, grid 512^3), the largest single-GPU configuration.  Two legs:
  plain   every step in float64, near-singular pairs by the graded-panel
          integrator, parameters of tolerance 1e-6 (the metric's accuracy
          bar: rel. l2 error <= 1e-6 against the FP64 CPU oracle) -> "value";
  learned float32 spread, transforms, interpolation and pairs, near-singular
          pairs by the trained network (trained here, on the GPU, by the
          library's own kernels) where its error indicator allows, else the
          graded panels, tolerance 1e-5 (bar 1e-5) -> "config.other_precision".
--legs mapped,mixed adds FP64 with the fixed-cost mapped rule and FP32 with
the graded panels alone (no network).
Errors are taken at the nodes of the oracle's stored reference (sampled on
large workloads).  Other workloads: --workload ellipses | tangle | ringpairs.

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
# the single-kernel stages on the plan's stream (the pair sum runs on the second)
PLAN_STREAM_STAGES = ("spread", "spectral", "interp")


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
    cnt = tree.query_ball_point(np.mod(fs.xyz, L) % L, rc, return_length=True,
                                workers=min(16, os.cpu_count() or 1))
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




def cpu_baseline_sampled(fs, n_targets=384, seed=0):
    """The oracle as it stands on a bounded sample of a large workload.  Its
    reference evaluation (direct Fourier sums with beta = 6, r_c = L, K = 12,
    brute-force short-range sums over every periodic image within r_c, exact
    near-singular segment integrals) costs a fixed part (spline fit of every
    filament and the Fourier coefficients of all quadrature points) plus a
    part per target node; both are timed, the second on n_targets nodes, and
    nodes/s = N / (fixed + N * per_target)."""
    from oracle import oracle as O
    prm = O.reference_params(fs.L, 6.0)
    idx = np.sort(np.random.default_rng(seed).choice(fs.n_nodes, n_targets, replace=False))
    t0 = time.perf_counter()
    o = O.Oracle(fs)
    o.longrange(prm["alpha"], prm["K"], idx[:1], psi=False)
    t1 = time.perf_counter()
    o.local(idx)
    o.shortrange(prm["alpha"], prm["rc"], idx, psi=False)
    o.selfcorr(prm["alpha"], idx)
    o.ns_correction(1.0, idx)
    t2 = time.perf_counter()
    fixed, per = t1 - t0, (t2 - t1) / n_targets
    return {"value": fs.n_nodes / (fixed + fs.n_nodes * per), "unit": "nodes/s",
            "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{fs.name} (N={fs.n_nodes}): spline fit and Fourier coefficients of all "
                      f"{fs.n_nodes * 2} quadrature points ({fixed:.1f} s, K={prm['K']}, "
                      f"r_c=L, beta=6) plus local, short-range, self and exact near-singular "
                      f"terms at {n_targets} sampled nodes ({t2 - t1:.1f} s); nodes/s = "
                      f"N / (fixed + N * per-node)"}


# per workload: the legs (name, precision, near-singular mode, tolerance);
# the first two run by default, the others when named by --legs
def legs_for(name, B):
    if name in ("bigtangle", "ringpairs"):
        return [("plain", B.BS_FP64, B.BS_NS_ADAPTIVE, 1e-6),
                ("learned", B.BS_FP32_MIXED, B.BS_NS_MLP, 1e-5),
                ("mapped", B.BS_FP64, B.BS_NS_MAPPED, 1e-6),
                ("mixed", B.BS_FP32_MIXED, B.BS_NS_ADAPTIVE, 1e-5)]
    return [("plain", B.BS_FP64, B.BS_NS_OFF, 1e-6),
            ("mixed", B.BS_FP32_MIXED, B.BS_NS_OFF, 1e-5)]


NS_NAMES = ["off", "adaptive", "learned", "mapped"]


def errors(v, gold):
    """rel. l2 error over the reference nodes (eq:def_relative_errors) and the
    largest per-node error relative to the rms reference velocity."""
    idx, ref = gold["idx"], gold["v"]
    d = v[idx] - ref
    vrms = math.sqrt((ref ** 2).sum(1).mean())
    return (math.sqrt((d ** 2).sum(1).mean()) / vrms,
            float(np.sqrt((d ** 2).sum(1)).max() / vrms))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="bigtangle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--detail", default=None,
                    help="also write per-stage times, rooflines and parameters to this JSON file")
    ap.add_argument("--legs", default=None,
                    help="comma-separated subset of the legs to run (profiling runs)")
    ap.add_argument("--table1", default=None, metavar="SIZES",
                    help="the paper's performance tests (Sec. 5.3, Table 1) instead of the "
                         "default line: comma-separated ellipse counts (32 nodes each); one "
                         "JSON line per tolerance and size, errors against the tol = 1e-14 run")
    ap.add_argument("--stage-pass", action="store_true",
                    help="run only the per-stage timing pass (stages one after another, as the "
                         "roofline's kernel durations are measured) for one warm-up and --steps "
                         "evaluations of each leg and print its stage times: the command to profile when "
                         "comparing rocprofv3's kernel durations with the roofline's")
    ap.add_argument("--pmc-calibrate", action="store_true",
                    help="end with a plain 256 MiB device copy, the size reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters of a rocprofv3 --pmc run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "only single-GPU runs exist: every box here has one GPU and "
                                   "the sharded multi-GPU path is not built; use --gpus 1"}))
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2406_07366_amd import binding as B
    from paper_2406_07366_amd import workloads as W

    if args.table1:
        table1(args, torch, B, W)
        return

    fs = W.make(args.workload)
    N = fs.n_nodes
    log(f"[bench] workload {fs.name} N={N} grid={fs.grid_n}^3")
    gold = load_reference(fs.name)
    if gold is None:
        raise SystemExit(f"no stored reference for {fs.name}: run tests/golden/make_references.py")
    xyz, gamma = B.load_workload(fs)
    out = torch.empty((N, 3), dtype=torch.float64, device="cuda")

    legs = legs_for(fs.name, B)
    if args.legs:
        keep = args.legs.split(",")
        legs = [l for l in legs if l[0] in keep]
    else:
        legs = legs[:2]
    mlp = table = None
    if any(l[2] == B.BS_NS_MLP for l in legs):
        from paper_2406_07366_amd import ns_mlp
        log("[bench] training the near-singular network on the GPU (1e6 samples) ...")
        mlp, table, _ = ns_mlp.train(n_train=1_000_000, n_val=100_000, epochs=40,
                                     batch=8192, log=log)

    results = {}
    for name, prec, ns_mode, tol in legs:
        fs.tol = tol
        plan = B.Plan(B.params_for(fs, precision=prec, ns_mode=ns_mode))
        if ns_mode == B.BS_NS_MLP:
            plan.set_mlp(mlp, table)
        prm = plan.params()
        if args.stage_pass:
            stage_profile(torch, plan, fs, xyz, gamma, out, 1)   # warm-up (first launches)
            st = stage_profile(torch, plan, fs, xyz, gamma, out, max(1, args.steps))
            plan.status()
            log(f"[bench] {name} stage pass, {max(1, args.steps)} evaluations (ms): "
                + ", ".join(f"{k}={v:.4f}" for k, v in st.items()))
            plan.close()
            continue
        plan.set_filaments(fs.offsets, xyz, gamma)
        plan.velocity(out)
        plan.status()
        err, errmax = errors(out.cpu().numpy(), gold)
        ms_host, ms_ev = time_steps(torch, plan, fs, xyz, gamma, out, args.steps, args.warmup)
        plan.status()
        st = stage_profile(torch, plan, fs, xyz, gamma, out, max(3, args.steps // 4))
        npairs, nfb = plan.ns_counts() if ns_mode != B.BS_NS_OFF else (0, 0)
        log(f"[bench] {name} (prec {prec}, ns_mode {ns_mode}, tol {tol:g}): {ms_host:.4f} ms/step "
            f"(events {ms_ev:.4f}), rel_l2 {err:.3e} (max/rms {errmax:.2e}), "
            f"{N / ms_host * 1e3:.4g} nodes/s, ns pairs {npairs}"
            + (f", by network {npairs - nfb}" if ns_mode == B.BS_NS_MLP else ""))
        log("[bench]   stages (ms): " + ", ".join(f"{k}={v:.4f}" for k, v in st.items()))
        results[name] = dict(ms=ms_host, ms_events=ms_ev, err=err, errmax=errmax, stages=st,
                             prm=prm.as_dict(), plan=plan, ns_mode=ns_mode, tol=tol,
                             precision=prec, ns_pairs=npairs, ns_fallback=nfb)

    if args.stage_pass:
        return

    if args.pmc_calibrate:
        src_t = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst_t = torch.empty_like(src_t)
        for _ in range(2):
            dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t

    pname = legs[0][0]
    primary = results[pname]
    prm = primary["prm"]
    fp32 = primary["precision"] == B.BS_FP32_MIXED
    fs.tol = primary["tol"]   # the legs loop left the last leg's tolerance
    rp = B.resolve_params(B.params_for(fs, precision=primary["precision"]))
    Nq = N * prm["Q"]
    sb = stage_bytes(rp, N, Nq, fp32)
    st = primary["stages"]
    roof_all = {}
    for k, b in sb.items():
        if st.get(k, 0) > 0:
            roof_all[k] = dict(bound="hbm", achieved=b / (st[k] * 1e-3) / 1e9, peak=HBM_PEAK_GBS,
                               unit="GB/s", bytes=b, ms=st[k])
    if st.get("pairs", 0) > 0:
        npairs = count_pairs(primary["plan"], fs, prm["Q"], prm["rcut"])
        peak = FP32_VECTOR_TFLOPS if fp32 else FP64_VECTOR_TFLOPS
        fl = npairs * PAIR_FLOP
        roof_all["pairs"] = dict(bound="alu", achieved=fl / (st["pairs"] * 1e-3) / 1e12,
                                 peak=peak, unit="TFLOP/s", flops=fl, pairs=npairs,
                                 ms=st["pairs"])
    # dominant single-kernel stage of the plan's stream, the evaluation's
    # critical path (the stage events then time exactly one kernel); the pair
    # sum runs on the second stream beside it and is reported with it
    def roof_entry(k):
        d = roof_all[k]
        srcname = SINGLE_KERNEL_STAGES[k]
        if k == "spectral" and pruned_transforms(rp):
            srcname = "fft.hip"         # the spectral operator runs inside the z transform
        src = os.path.join(ROOT, "paper_2406_07366_amd", "csrc", srcname)
        traffic = read_traffic(os.path.join(
            ROOT, "profiles", f"pmc_{k}_{fs.name}_{'mixed' if fp32 else 'fp64'}.txt"), src)
        e = {"kernel": k, "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
             "unit": d["unit"], "frac": d["achieved"] / d["peak"], "traffic": traffic,
             "ms": d["ms"]}
        if "bytes" in d:
            e["algorithmic_bytes"] = d["bytes"]
        if "flops" in d:
            e["algorithmic_flops"] = d["flops"]
            e["pairs"] = d["pairs"]
        return e

    dom = max((k for k in roof_all if k in PLAN_STREAM_STAGES), key=lambda k: roof_all[k]["ms"])
    roofline = roof_entry(dom)
    if "pairs" in roof_all:
        roofline["side_stream"] = roof_entry("pairs")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle baseline ...")
        if N > 300_000:
            cpu = cpu_baseline_sampled(fs)
        else:
            cpu = cpu_baseline(fs, rp)
        log(f"[bench] cpu baseline {cpu['value']:.4g} nodes/s on {cpu['cores']} threads")

    def leg_summary(r):
        return {"nodes_per_s": N / (r["ms"] * 1e-3), "ms_per_step": r["ms"],
                "rel_l2_err": r["err"], "max_err_over_rms": r["errmax"], "tol": r["tol"],
                "meets_tol": r["err"] <= r["tol"],
                "dtype": "f32+f64" if r["precision"] == B.BS_FP32_MIXED else "f64",
                "ns_mode": NS_NAMES[r["ns_mode"]],
                "ns_pairs": r["ns_pairs"],
                "ns_by_network": (r["ns_pairs"] - r["ns_fallback"]
                                  if r["ns_mode"] == B.BS_NS_MLP else 0)}

    value = N / (primary["ms"] * 1e-3)
    cfg = {"workload": f"{fs.name}: {fs.n_fil} filaments, N={N}, grid {fs.grid_n}^3, "
                       f"Q={prm['Q']}, w={prm['w']}, beta={prm['beta']}, tol {primary['tol']:g}",
           "rel_l2_err": primary["err"], "max_err_over_rms": primary["errmax"],
           "meets_tol": primary["err"] <= primary["tol"],
           "ns_mode": NS_NAMES[primary["ns_mode"]],
           "ns_pairs": primary["ns_pairs"]}
    others = [n for n in results if n != pname]
    if others:
        cfg["other_precision"] = dict(name=others[0], **leg_summary(results[others[0]]))
    for extra in others[1:]:
        cfg[f"leg_{extra}"] = leg_summary(results[extra])
    line = {
        "metric": "filament nodes/s per velocity eval at rel. L2 err <= 1e-6 vs FP64 oracle; "
                  "FP32+MLP vs plain",
        "value": value, "unit": "nodes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": primary["ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if fp32 else "f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if args.detail:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
        with open(args.detail, "w") as f:
            json.dump({"line": line, "roofline_all": roof_all,
                       "legs": {k: leg_summary(v) for k, v in results.items()},
                       "stages": {k: v["stages"] for k, v in results.items()},
                       "params": {k: v["prm"] for k, v in results.items()}},
                      f, indent=1, default=float)
    for r in results.values():
        r["plan"].close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
