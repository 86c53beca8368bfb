"""MLP kernels against the FP64 oracle network: BF16 MFMA (oracle with the
same BF16-rounded weights) and the FP32 debug mode (oracle with the same FP32
weights) for forward values and the loss gradient, and a training sanity
check."""
import math

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_07366_amd import binding
    return binding


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _setup(B, n=100, seed=0):
    import torch
    P = B.mlp_init(seed)
    P[-3:] = [0.1, -0.2, 0.3]
    rng = np.random.default_rng(seed + 1)
    X = rng.standard_normal((n, 8)).astype(np.float32)
    T = rng.standard_normal((n, 3)).astype(np.float32)
    Pb = P.astype(np.float64)
    # the device rounds weights (not biases) to bf16
    wmask = np.ones(len(P), bool)
    o = 0
    for din, dout in ((8, 64), (64, 64), (64, 64), (64, 3)):
        o += din * dout
        wmask[o:o + dout] = False
        o += dout
    Pb[wmask] = B.bf16_round(P[wmask]).astype(np.float64)
    return P, Pb, X, T, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()


def test_mlp_forward_matches_oracle(B):
    P, Pb, X, T, Xd, Td = _setup(B, n=100)      # 100 = 6 tiles of 16 + ragged tail
    print("\n[case] mlp forward B=100", flush=True)
    m = B.MLP(P)
    Y = m.forward(Xd).cpu().numpy()
    Yref = O.mlp_forward(Pb, X.astype(np.float64))
    err = rel_l2(Y, Yref)
    print(f"  forward rel_l2 {err:.2e}")
    assert err < 1e-2


def test_mlp_gradient_matches_oracle(B):
    P, Pb, X, T, Xd, Td = _setup(B, n=200, seed=3)
    print("\n[case] mlp gradient B=200", flush=True)
    m = B.MLP(P)
    loss, g = m.loss_grad(Xd, Td)
    loss_ref, gref = O.mlp_loss_grad(Pb, X.astype(np.float64), T.astype(np.float64))
    g = g.cpu().numpy().astype(np.float64)
    err = rel_l2(g, gref)
    cos = float(g @ gref / (np.linalg.norm(g) * np.linalg.norm(gref)))
    print(f"  loss {loss.item():.6f} ref {loss_ref:.6f}  grad rel_l2 {err:.2e} cos {cos:.6f}")
    assert abs(loss.item() - loss_ref) < 1e-2 * loss_ref
    # BF16 activations (8-bit mantissa) into every product: 1e-2 overall
    assert err < 1e-2 and cos > 0.9999
    # every layer's block of the gradient is right, not just the total
    o = 0
    for din, dout in ((8, 64), (64, 64), (64, 64), (64, 3)):
        for n_ in (din * dout, dout):
            blk = slice(o, o + n_)
            assert rel_l2(g[blk], gref[blk]) < 6e-2, (o, n_)
            o += n_


@pytest.mark.parametrize("n", [100, 997])
def test_mlp_fp32_mode_matches_oracle(B, n):
    """Debug mode: FP32 weights and activations on FP32 MFMA.  Forward values
    and the loss gradient (every layer's block) against the FP64 oracle with
    the same FP32 weights, to 1e-6: only FP32 rounding remains."""
    P, _, X, T, Xd, Td = _setup(B, n=n, seed=5)
    print(f"\n[case] mlp fp32 mode B={n}", flush=True)
    m = B.MLP(P)
    m.set_fp32(True)
    P64, X64, T64 = P.astype(np.float64), X.astype(np.float64), T.astype(np.float64)
    Y = m.forward(Xd).cpu().numpy().astype(np.float64)
    Yref = O.mlp_forward(P64, X64)
    ferr = rel_l2(Y, Yref)
    loss, g = m.loss_grad(Xd, Td)
    loss_ref, gref = O.mlp_loss_grad(P64, X64, T64)
    g = g.cpu().numpy().astype(np.float64)
    gerr = rel_l2(g, gref)
    print(f"  forward rel_l2 {ferr:.2e}  loss {loss.item():.8f} ref {loss_ref:.8f}  "
          f"grad rel_l2 {gerr:.2e}")
    assert ferr <= 1e-6
    assert abs(loss.item() - loss_ref) <= 1e-6 * loss_ref
    assert gerr <= 1e-6
    o = 0
    for din, dout in ((8, 64), (64, 64), (64, 64), (64, 3)):
        for n_ in (din * dout, dout):
            blk = slice(o, o + n_)
            assert rel_l2(g[blk], gref[blk]) <= 1e-6, (o, n_)
            o += n_
    # back to BF16: the same network gives the BF16 results again
    m.set_fp32(False)
    Yb = m.forward(Xd).cpu().numpy().astype(np.float64)
    assert 1e-5 < rel_l2(Yb, Yref) < 1e-2


def test_mlp_training_reduces_loss(B):
    import torch
    print("\n[case] mlp training 4096 samples", flush=True)
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, (4096, 8)).astype(np.float32)
    T = np.stack([np.sin(2 * X[:, 0]) + X[:, 1] ** 2, np.cos(X[:, 2] * X[:, 3]),
                  X[:, 4] - X[:, 5] * X[:, 6]], 1).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    m = B.MLP(B.mlp_init(1))
    l0 = m.loss_grad(Xd, Td)[0].item()
    for _ in range(400):
        m.adam_step(Xd, Td, 3e-3)
    l1 = m.loss_grad(Xd, Td)[0].item()
    print(f"  loss {l0:.4e} -> {l1:.4e}")
    assert l1 < l0 / 50
