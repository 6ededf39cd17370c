"""Pins of the oracle's greedy (Alg. 1 / Alg. 4) and MLP surrogate."""
import math

import numpy as np
import pytest

from oracle import greedy, mlp
from workloads import log_uniform_mu
from oracle.operator import BlockDiffusion


def _brute_force_picks(op, thetas, n_max, kind):
    """Alg. 1 with exact dense snapshot solves, a QR basis and dense reduced solves."""
    f = op.rhs()
    dense = [op.assemble(t).toarray() for t in thetas]
    sols = [np.linalg.solve(A, f) for A in dense]
    picks = [0]
    while True:
        Wq, _ = np.linalg.qr(np.column_stack([sols[i] for i in picks]))
        vals = []
        for A in dense:
            a = np.linalg.solve(Wq.T @ A @ Wq, Wq.T @ f)
            if kind == "l1":
                vals.append(np.abs(a).sum())
            else:
                vals.append(np.linalg.norm(f - A @ (Wq @ a)) / np.linalg.norm(f))
        if len(picks) == n_max:
            return picks, vals
        v = np.array(vals)
        v[picks] = -np.inf
        picks.append(int(np.argmax(v)))


@pytest.mark.parametrize("kind", ["residual", "l1"])
def test_greedy_picks_match_brute_force(kind):
    op = BlockDiffusion((7, 7), (2, 2))
    rng = np.random.default_rng(12)
    thetas = 10 ** rng.uniform(-1, 1, (24, op.Q))
    g = greedy.adaptive_greedy(op, thetas, 5, indicator=kind, snapshot_rtol=1e-12)
    bf, vals = _brute_force_picks(op, thetas, 5, kind)
    assert g.picks == bf
    assert np.abs(g.W.T @ g.W - np.eye(5)).max() <= 1e-13


def test_residual_indicator_vanishes_on_samples():
    op = BlockDiffusion((7, 7), (2, 2))
    rng = np.random.default_rng(13)
    thetas = 10 ** rng.uniform(-1, 1, (16, op.Q))
    g = greedy.adaptive_greedy(op, thetas, 4, keep_indicators=True, snapshot_rtol=1e-12)
    last = g.indicators[-1]
    for p in g.picks:
        assert last[p] <= 1e-9


def test_masked_argmax_ties_and_exclusion():
    assert greedy.masked_argmax([1.0, 3.0, 3.0, 2.0], {0}) == 1
    assert greedy.masked_argmax([1.0, 3.0, 3.0, 2.0], {1}) == 2
    with pytest.raises(FloatingPointError):
        greedy.masked_argmax([1.0, float("nan")], set())


# --- MLP ----------------------------------------------------------------------
def test_splitmix64_published_values():
    # SplitMix64 with state 0: the first outputs of the reference generator
    # (state += golden gamma; mix) are 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4.
    assert mlp.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert mlp.splitmix64(0, 1) == 0x6E789E6AA1B965F4


def test_gelu_reference_values():
    # GELU(x) = x * Phi(x): Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707
    g = mlp.gelu(np.array([1.0, -1.0, 0.0]))
    assert g[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    assert g[1] == pytest.approx(-0.15865525393145707, rel=1e-14)
    assert g[2] == 0.0


def test_mlp_gradients_finite_differences():
    rng = np.random.default_rng(20)
    P, H = 8, 16
    params = mlp.init_params(P, H, seed=7)
    for k in ("b1", "b2", "b3"):
        params[k] = rng.standard_normal(params[k].shape) * 0.1
    X = rng.uniform(-1, 1, (12, P))
    y = rng.standard_normal(12)
    loss, g = mlp.loss_and_grads(params, X, y)
    h = 1e-6
    for name in mlp.PARAM_NAMES:
        flat = params[name].ravel()
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grads(params, X, y)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grads(params, X, y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert g[name].ravel()[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_glorot_range_and_adam_reduces_loss():
    P, H = 8, 32
    params = mlp.init_params(P, H, seed=3)
    a1 = math.sqrt(6.0 / (P + H))
    assert np.abs(params["W1"]).max() <= a1 and np.abs(params["W1"]).max() > 0.8 * a1
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (64, P))
    y = np.sin(X[:, 0]) + X[:, 1] ** 2
    opt = mlp.Adam(params, lr=1e-2)
    l0, _ = mlp.loss_and_grads(params, X, y)
    for _ in range(200):
        _, g = mlp.loss_and_grads(params, X, y)
        opt.step(params, g)
    l1, _ = mlp.loss_and_grads(params, X, y)
    assert l1 < 0.05 * l0


def test_adam_first_step_is_signed_lr():
    """With bias correction the first Adam step moves each weight by lr * sign(g)."""
    params = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    opt = mlp.Adam(params, lr=0.1, eps=0.0)
    opt.step(params, g)
    assert np.allclose(params["w"], [0.9, -1.9, 2.9], rtol=0, atol=1e-15)


# ---- multi-fidelity construction (Sec. 4.2, last paragraph) ----------------------------
def test_basis_from_greedy_picks_reproduces_greedy_basis():
    """Snapshot solves and basis updates replayed on the greedy's own picks give the greedy's basis exactly."""
    op = BlockDiffusion((15, 15), (2, 2))
    thetas = log_uniform_mu(11, 40, op.Q, 0.1, 10.0)
    g = greedy.adaptive_greedy(op, thetas, 6, indicator="residual")
    b = greedy.basis_from_parameters(op, [thetas[i] for i in g.picks])
    assert b.picks == list(range(6))
    assert np.array_equal(b.W, g.W) and np.array_equal(b.AN_q, g.AN_q)


def test_multi_fidelity_basis_spans_fine_snapshots():
    """Coarse picks, fine snapshots: W is orthonormal, every fine snapshot lies in its
    span to the snapshot tolerance, and the reduced operators are W^T A_q W."""
    from oracle import rb as orb
    coarse, fine = BlockDiffusion((15, 15), (2, 2)), BlockDiffusion((31, 31), (2, 2))
    thetas = log_uniform_mu(12, 40, coarse.Q, 0.1, 10.0)
    g, mf = greedy.multi_fidelity(coarse, fine, thetas, 5)
    W = mf.W
    assert W.shape == (fine.N, 5) and mf.picks == g.picks
    assert np.abs(W.T @ W - np.eye(5)).max() <= 1e-13
    for i in g.picks:
        x = orb.solve_cg(fine, thetas[i], rtol=1e-12).x
        assert np.linalg.norm(x - W @ (W.T @ x)) <= 1e-8 * np.linalg.norm(x)
    AN, _ = orb.reduced_operators(fine.A_q, [fine.rhs()], W)
    assert np.abs(AN - mf.AN_q).max() <= 1e-12 * np.abs(AN).max()


def test_bf16_rounding_matches_torch():
    """The oracle's BF16 rounding equals torch's float32 -> bfloat16 conversion (round to
    nearest, ties to even), ties and the largest finite values included."""
    import torch
    rng = np.random.default_rng(17)
    v = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.uniform(-30, 30, 4000),
                        # exact ties: 1 + (2k+1) 2^-8 lies halfway between BF16 neighbours
                        1.0 + (2 * np.arange(64) + 1) * 2.0 ** -8, [0.0, -0.0, 3.3e38]])
    v = v.astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(mlp.bf16_round(v), ref)


def test_bf16_mode_is_close_to_fp64():
    """With BF16 operands (relative precision 2^-8) the loss and gradients stay within a
    few 1e-3 of the FP64 network's; with operands that are already BF16 values
    the first product is exact up to FP32 rounding."""
    rng = np.random.default_rng(5)
    P, H, m = 8, 32, 64
    params = mlp.init_params(P, H, seed=3)
    X = rng.uniform(-1, 1, (m, P))
    y = np.sin(X[:, 0])
    l64, g64 = mlp.loss_and_grads(params, X, y)
    lbf, gbf = mlp.loss_and_grads(params, X, y, bf16=True)
    assert abs(lbf - l64) <= 2e-2 * l64
    for k in g64:
        assert np.linalg.norm(gbf[k] - g64[k]) <= 2e-2 * np.linalg.norm(g64[k]), k
    # BF16-representable operands: the first layer's pre-activation equals FP64's in FP32
    pb = {k: mlp.bf16_round(v) for k, v in params.items()}
    Xb = mlp.bf16_round(X)
    z64 = Xb @ pb["W1"].T
    zbf = mlp._mm(Xb, pb["W1"].T, True)
    assert np.allclose(zbf, z64, rtol=2 ** -23, atol=0)
