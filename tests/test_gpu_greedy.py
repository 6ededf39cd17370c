"""GPU adaptive greedy (Alg. 4) against the oracle's greedy: same picks, same basis
(up to the snapshot tolerance), orthonormal columns, and matching reduced operators."""
import numpy as np
import pytest

from oracle import greedy as og
from oracle import rb as orb
from oracle.operator import BlockDiffusion
from workloads import log_uniform_mu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


@pytest.mark.parametrize("indicator", ["l1", "residual"])
@pytest.mark.parametrize("dims,blocks", [((15, 15), (2, 2)), ((7, 9, 5), (2, 2, 3))])
def test_greedy_matches_oracle(lib, ctx, indicator, dims, blocks):
    op = BlockDiffusion(dims, blocks)
    mus = log_uniform_mu(80, 24, op.Q, 0.1, 10.0)
    n_max = 5
    ref = og.adaptive_greedy(op, mus, n_max, indicator=indicator, snapshot_rtol=1e-12)
    prob = lib.Problem(ctx, dims, blocks)
    basis, rep = lib.offline_build(ctx, prob, mus, mu=mus, n_max=n_max, indicator=indicator,
                                   snapshot_rtol=1e-12)
    assert rep["picks"] == ref.picks
    W, AN, fN = basis.info()
    assert np.abs(W @ W.T - np.eye(n_max)).max() <= 1e-13
    for j in range(n_max):
        assert np.linalg.norm(W[j] - ref.W[:, j]) <= 1e-7
    assert np.abs(AN - ref.AN_q).max() <= 1e-7 * np.abs(ref.AN_q).max()
    assert np.allclose(rep["max_indicator"], ref.max_indicator, rtol=1e-5, atol=1e-12)
    assert rep["true_evals"] == n_max * len(mus)


@pytest.mark.parametrize("dims,blocks", [((15, 15), (2, 2)), ((7, 9, 5), (2, 2, 3))])
def test_greedy_snapshot_sweeps(lib, ctx, dims, blocks):
    """Snapshot solves with four Gauss-Seidel sweeps per preconditioner application, on
    the GPU and in the oracle: the same picks and the basis within 1e-7 (the snapshots
    are solved to 1e-12 either way; fewer iterations than with one sweep)."""
    op = BlockDiffusion(dims, blocks)
    mus = log_uniform_mu(80, 24, op.Q, 0.1, 10.0)
    n_max = 5
    ref = og.adaptive_greedy(op, mus, n_max, indicator="residual", snapshot_rtol=1e-12,
                             snapshot_sweeps=4)
    ref1 = og.adaptive_greedy(op, mus, n_max, indicator="residual", snapshot_rtol=1e-12)
    prob = lib.Problem(ctx, dims, blocks)
    basis, rep = lib.offline_build(ctx, prob, mus, mu=mus, n_max=n_max, indicator="residual",
                                   snapshot_rtol=1e-12, snapshot_sweeps=4)
    assert rep["picks"] == ref.picks
    W, AN, fN = basis.info()
    for j in range(n_max):
        assert np.linalg.norm(W[j] - ref.W[:, j]) <= 1e-7
    assert sum(rep["snapshot_iters"]) < sum(ref1.snapshot_iters)


@pytest.mark.parametrize("dims,blocks", [((15, 15), (2, 2)), ((7, 9, 5), (2, 2, 3))])
def test_greedy_fp32_snapshots(lib, ctx, dims, blocks):
    """Snapshot solves preconditioned in FP32 (the basis's FP32 copy grows a column per
    step; CG, stopping test and Gram-Schmidt in FP64): the oracle's picks, the basis
    within 1e-7, and the grown FP32 copy serves a later FP32 solve as a fresh one does."""
    op = BlockDiffusion(dims, blocks)
    mus = log_uniform_mu(80, 24, op.Q, 0.1, 10.0)
    n_max = 5
    ref = og.adaptive_greedy(op, mus, n_max, indicator="residual", snapshot_rtol=1e-12)
    prob = lib.Problem(ctx, dims, blocks)
    basis, rep = lib.offline_build(ctx, prob, mus, mu=mus, n_max=n_max, indicator="residual",
                                   snapshot_rtol=1e-12, snapshot_prec="fp32")
    assert rep["picks"] == ref.picks
    W, AN, fN = basis.info()
    for j in range(n_max):
        assert np.linalg.norm(W[j] - ref.W[:, j]) <= 1e-7
    theta = log_uniform_mu(81, 3, op.Q, 0.1, 10.0)
    x1, _ = lib.solve_batch(ctx, prob, basis, theta, prec="fp32", fixed_iters=5)
    fresh = lib.Basis.from_host(ctx, prob, W)
    x2, _ = lib.solve_batch(ctx, prob, fresh, theta, prec="fp32", fixed_iters=5)
    x1, x2 = x1.cpu().numpy(), x2.cpu().numpy()
    assert np.abs(x1 - x2).max() <= 1e-12 * np.abs(x2).max()


def test_greedy_degenerate_candidate_is_skipped(lib, ctx):
    """A duplicated parameter gives a snapshot already in span(W): the greedy must skip
    it (RB_EDEGENERATE inside) and take the next candidate."""
    dims, blocks = (15, 15), (2, 2)
    op = BlockDiffusion(dims, blocks)
    mus = log_uniform_mu(81, 12, op.Q, 0.1, 10.0)
    mus = np.vstack([mus, mus])   # every parameter twice
    prob = lib.Problem(ctx, dims, blocks)
    basis, rep = lib.offline_build(ctx, prob, mus, mu=mus, n_max=4, indicator="residual")
    picks = rep["picks"]
    assert len(set(picks)) == 4
    assert len({p % 12 for p in picks}) == 4   # never a copy of an earlier pick
    W, AN, fN = basis.info()
    assert np.abs(W @ W.T - np.eye(4)).max() <= 1e-12


def test_basis_save_load_roundtrip(lib, ctx, tmp_path):
    dims, blocks = (15, 15), (2, 2)
    op = BlockDiffusion(dims, blocks)
    mus = log_uniform_mu(82, 10, op.Q, 0.1, 10.0)
    prob = lib.Problem(ctx, dims, blocks)
    basis, rep = lib.offline_build(ctx, prob, mus, n_max=3, indicator="l1")
    path = str(tmp_path / "basis.rb")
    basis.save(path)
    b2 = lib.Basis.load(ctx, prob, path)
    W1, A1, f1 = basis.info()
    W2, A2, f2 = b2.info()
    assert np.array_equal(W1, W2)
    assert np.abs(A1 - A2).max() <= 1e-12 * np.abs(A1).max()
    theta = log_uniform_mu(83, 3, op.Q, 0.1, 10.0)
    x1, s1 = lib.solve_batch(ctx, prob, basis, theta)
    x2, s2 = lib.solve_batch(ctx, prob, b2, theta)
    assert np.array_equal(s1.iters, s2.iters)


@pytest.mark.parametrize("coarse,fine,blocks", [((15, 15), (31, 31), (2, 2)),
                                                ((7, 7, 7), (15, 15, 15), (2, 2, 2))])
def test_multi_fidelity_matches_oracle(lib, ctx, coarse, fine, blocks):
    """Multi-fidelity build (Sec. 4.2): greedy on the coarse grid, snapshots of its picks
    on the fine grid; the fine basis matches the oracle's column by column and the
    parameters that were given twice are skipped as degenerate."""
    opc, opf = BlockDiffusion(coarse, blocks), BlockDiffusion(fine, blocks)
    mus = log_uniform_mu(83, 30, opc.Q, 0.1, 10.0)
    n_max = 5
    g_ref, f_ref = og.multi_fidelity(opc, opf, mus, n_max, snapshot_rtol=1e-12)
    pc = lib.Problem(ctx, coarse, blocks)
    _, rep = lib.offline_build(ctx, pc, mus, n_max=n_max, indicator="residual",
                               snapshot_rtol=1e-12)
    assert rep["picks"] == g_ref.picks
    pf = lib.Problem(ctx, fine, blocks)
    sel = mus[rep["picks"]]
    sel = np.vstack([sel[:2], sel[1:2], sel[2:]])     # one parameter repeated
    fb, frep = lib.basis_from_parameters(ctx, pf, sel, snapshot_rtol=1e-12)
    assert frep["n_built"] == n_max and frep["picks"] == [0, 1, 3, 4, 5]
    W, AN, fN = fb.info()
    assert np.abs(W @ W.T - np.eye(n_max)).max() <= 1e-13
    ref_sel = og.basis_from_parameters(opf, [mus[i] for i in g_ref.picks], snapshot_rtol=1e-12)
    for j in range(n_max):
        assert np.linalg.norm(W[j] - ref_sel.W[:, j]) <= 1e-7
    assert np.abs(AN - ref_sel.AN_q).max() <= 1e-7 * np.abs(ref_sel.AN_q).max()
