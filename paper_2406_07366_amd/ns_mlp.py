"""Training of the learned near-singular correction.

Samples come from the library's own segment integrator (bs_ns_samples, the
plain method in float64); the network is trained by the library's BF16-MFMA
forward/backward kernels with Adam (bs_mlp_adam_step).  A held-out set gives
the error table (bs_ns_error_table, computed by the library) the plan uses to
decide, per pair, between the network and the mapped rule.  This module only
drives those calls.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import binding as B


def _uniforms(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.random((n, 8))).cuda()


def make_dataset(n, seed):
    U = _uniforms(n, seed)
    X, T, A = B.ns_samples(U)
    return X, T, A


def train(n_train=1_000_000, n_val=100_000, epochs=60, batch=8192, lr=3e-3, seed=0,
          log=print):
    """Train a network on device-generated samples; returns (mlp, err_table,
    info)."""
    import torch
    t0 = time.perf_counter()
    X, T, A = make_dataset(n_train, seed)
    Xv, Tv, Av = make_dataset(n_val, seed + 1)
    torch.cuda.synchronize()
    tgen = time.perf_counter() - t0
    mlp = B.MLP(B.mlp_init(seed))
    steps = epochs * (n_train // batch)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    t1 = time.perf_counter()
    k = 0
    for ep in range(epochs):
        for i in range(n_train // batch):
            sl = slice(i * batch, (i + 1) * batch)
            lr_k = 1e-5 + 0.5 * (lr - 1e-5) * (1 + math.cos(math.pi * k / steps))
            mlp.adam_step(X[sl], T[sl], lr_k, loss=loss)
            k += 1
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log(f"[ns-mlp] epoch {ep} loss {loss.item():.3e}")
    torch.cuda.synchronize()
    ttrain = time.perf_counter() - t1
    tab, mx = B.ns_error_table(mlp, Xv, Tv, Av)
    info = dict(n_train=n_train, n_val=n_val, epochs=epochs, batch=batch, gen_s=tgen,
                train_s=ttrain, val_loss=mlp.loss_grad(Xv, Tv)[0].item(),
                err_rms=tab.tolist(), err_max=mx.tolist())
    if log:
        log(f"[ns-mlp] trained {n_train} samples x {epochs} epochs in {ttrain:.1f} s; "
            f"val loss {info['val_loss']:.3e}")
        log("[ns-mlp] rms err (h = 1) per d/h bin: " + " ".join(f"{v:.1e}" for v in tab))
        log("[ns-mlp] max err (h = 1) per d/h bin: " + " ".join(f"{v:.1e}" for v in mx))
    return mlp, tab, info


def _main(argv=None):
    """Fixed-size loops of the network kernels alone, for profiling:
         python -m paper_2406_07366_amd.ns_mlp infer [n] [reps]
         python -m paper_2406_07366_amd.ns_mlp train [batch] [steps]
    Random initial weights and uniform random features."""
    import argparse
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["infer", "train"])
    ap.add_argument("size", nargs="?", type=int, default=1_000_000)
    ap.add_argument("reps", nargs="?", type=int, default=20)
    a = ap.parse_args(argv)
    mlp = B.MLP(B.mlp_init(0))
    g = torch.Generator(device="cuda").manual_seed(0)
    X = torch.rand((a.size, 8), device="cuda", generator=g, dtype=torch.float32) * 2 - 1
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if a.what == "infer":
        Y = mlp.forward(X)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(a.reps):
            Y = mlp.forward(X)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / a.reps
        flop = 2.0 * a.size * (8 * 64 + 64 * 64 * 2 + 64 * 3)
        print(f"[mlp] forward of {a.size} samples: {ms:.4f} ms, "
              f"{flop / ms / 1e9:.1f} TFLOP/s (model flops)", flush=True)
    else:
        T = torch.rand((a.size, 3), device="cuda", generator=g, dtype=torch.float32)
        mlp.adam_step(X, T, 1e-3)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(a.reps):
            mlp.adam_step(X, T, 1e-3)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / a.reps
        print(f"[mlp] training step of batch {a.size}: {ms:.4f} ms", flush=True)


if __name__ == "__main__":
    _main()
