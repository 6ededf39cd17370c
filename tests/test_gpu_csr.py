"""GPU parity of the general sparse (CSR) path against the oracle's SparseAffine problem,
and against the stencil path on the same matrices.

Bars as in the stencil parity tests: single kernels 1e-12 relative (summation order of
the sparse sums only), k fixed RBCG iterations 1e-10, converged solves within two
iterations and 2 kappa 1e-10.  The colouring is exact integer work: bit-identical."""
import numpy as np
import pytest

from oracle import greedy as og
from oracle import rb as orb
from oracle.operator import BlockDiffusion, SparseAffine
from workloads import fem, log_uniform_mu, random_orthonormal, random_vectors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _grid_csr(op):
    """The block-diffusion terms as CSR arrays on their union pattern."""
    U = sum(abs(a) for a in op.A_q).tocsr()
    U.sort_indices()
    r = np.repeat(np.arange(op.N), np.diff(U.indptr))
    vals = np.stack([np.asarray(a.tocsr()[r, U.indices]).ravel() for a in op.A_q])
    return U.indptr.astype(np.int64), U.indices.astype(np.int32), vals


def _random(N=1500, seed=5):
    s = fem.random_system(seed, N, 6, 3)
    rp, c, v = fem.csr_arrays(s)
    return SparseAffine(rp, c, v), (rp, c, v)


def _kappa(A):
    import scipy.sparse.linalg as spla
    lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
    lmin = spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    return lmax / lmin


def test_colouring_matches_oracle(lib, ctx):
    op, arrs = _random()
    prob = lib.Problem.from_csr(ctx, *arrs)
    col, nc = prob.colors()
    ref = op.colors()
    assert np.array_equal(col, ref) and nc == ref.max() + 1 and nc >= 3
    g = BlockDiffusion((9, 7, 5), (2, 2, 2))
    pg = lib.Problem.from_csr(ctx, *_grid_csr(g))
    col, nc = pg.colors()
    assert nc == 2 and np.array_equal(col, g.colors())


@pytest.mark.parametrize("which", ["grid", "random"])
def test_apply_matches_oracle(lib, ctx, which):
    if which == "grid":
        op = BlockDiffusion((15, 15), (2, 2))
        arrs = _grid_csr(op)
        op = SparseAffine(*arrs)
    else:
        op, arrs = _random()
    prob = lib.Problem.from_csr(ctx, *arrs)
    theta = log_uniform_mu(3, 5, op.Q, 0.1, 10.0)
    u = random_vectors(4, 5, op.N)
    y = lib.apply_batch(ctx, prob, theta, _t(u)).cpu().numpy()
    for b in range(5):
        assert _rel(y[b], op.assemble(theta[b]) @ u[b]) <= 1e-13


@pytest.mark.parametrize("smoother", ["rbgs", "rbgs_sym", "jacobi", "none"])
def test_preconditioner_matches_oracle(lib, ctx, smoother):
    op, arrs = _random()
    prob = lib.Problem.from_csr(ctx, *arrs)
    W = random_orthonormal(6, op.N, 5)
    basis = lib.Basis.from_host(ctx, prob, W.T)
    theta = log_uniform_mu(7, 5, op.Q, 0.1, 10.0)
    r = random_vectors(8, 5, op.N)
    y = lib.precond_batch(ctx, prob, basis, theta, _t(r), smoother=smoother).cpu().numpy()
    AN, _ = orb.reduced_operators(op.A_q, [op.rhs()], W)
    for b in range(5):
        _, M = orb.make_preconditioner(op, theta[b], W, AN, smoother_kind=smoother)
        assert _rel(y[b], M(r[b])) <= 1e-12, (b, _rel(y[b], M(r[b])))


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 5e-2)])
@pytest.mark.parametrize("which", ["grid", "random"])
def test_preconditioner_mixed(lib, ctx, prec, tol, which):
    """FP32 / BF16 basis and FP32 smoother against the FP64 oracle preconditioner."""
    if which == "grid":
        arrs = _grid_csr(BlockDiffusion((15, 15), (2, 2)))
        op = SparseAffine(*arrs)
    else:
        op, arrs = _random()
    prob = lib.Problem.from_csr(ctx, *arrs)
    W = random_orthonormal(6, op.N, 5)
    basis = lib.Basis.from_host(ctx, prob, W.T)
    theta = log_uniform_mu(7, 20, op.Q, 0.1, 10.0)
    r = random_vectors(8, 20, op.N)
    y = lib.precond_batch(ctx, prob, basis, theta, _t(r), prec=prec).cpu().numpy()
    AN, _ = orb.reduced_operators(op.A_q, [op.rhs()], W)
    for b in range(20):
        _, M = orb.make_preconditioner(op, theta[b], W, AN)
        assert _rel(y[b], M(r[b])) <= tol, (b, _rel(y[b], M(r[b])))


@pytest.mark.parametrize("dims,blocks", [((15, 15), (2, 2)), ((7, 9, 5), (2, 2, 3))])
def test_csr_path_equals_stencil_path(lib, ctx, dims, blocks):
    """The grid operator given as CSR: same colouring, so the same iterates up to the
    order of the sparse sums."""
    op = BlockDiffusion(dims, blocks)
    ps = lib.Problem(ctx, dims, blocks)
    pc = lib.Problem.from_csr(ctx, *_grid_csr(op))
    W = random_orthonormal(9, op.N, 4)
    bs, bc = lib.Basis.from_host(ctx, ps, W.T), lib.Basis.from_host(ctx, pc, W.T)
    theta = log_uniform_mu(10, 6, op.Q, 0.1, 10.0)
    xs, ss = lib.solve_batch(ctx, ps, bs, theta, fixed_iters=7)
    xc, sc = lib.solve_batch(ctx, pc, bc, theta, fixed_iters=7)
    xs, xc = xs.cpu().numpy(), xc.cpu().numpy()
    for b in range(6):
        assert _rel(xc[b], xs[b]) <= 1e-12, (b, _rel(xc[b], xs[b]))


@pytest.mark.parametrize("flexible", [False, True])
@pytest.mark.parametrize("B", [1, 6])
def test_rbcg_fixed_iterations(lib, ctx, flexible, B):
    op, arrs = _random()
    prob = lib.Problem.from_csr(ctx, *arrs)
    W = random_orthonormal(11, op.N, 6)
    basis = lib.Basis.from_host(ctx, prob, W.T)
    AN, _ = orb.reduced_operators(op.A_q, [op.rhs()], W)
    theta = log_uniform_mu(12, B, op.Q, 0.1, 10.0)
    k = 6
    x, st = lib.solve_batch(ctx, prob, basis, theta, fixed_iters=k, flexible=flexible)
    x = x.cpu().numpy()
    for b in range(B):
        ref = orb.solve_rbcg(op, theta[b], W, AN, fixed_iters=k, flexible=flexible)
        assert _rel(x[b], ref.x) <= 1e-10, (b, _rel(x[b], ref.x))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rbcg_converged(lib, ctx, prec):
    op, arrs = _random()
    prob = lib.Problem.from_csr(ctx, *arrs)
    thetas = log_uniform_mu(13, 30, op.Q, 0.1, 10.0)
    g = og.adaptive_greedy(op, thetas, 6, indicator="residual", snapshot_rtol=1e-12)
    basis = lib.Basis.from_host(ctx, prob, g.W.T)
    theta = log_uniform_mu(14, 5, op.Q, 0.1, 10.0)
    x, st = lib.solve_batch(ctx, prob, basis, theta, prec=prec, flexible=True)
    x = x.cpu().numpy()
    for b in range(5):
        ref = orb.solve_rbcg(op, theta[b], g.W, g.AN_q, flexible=True)
        assert st.status[b] == lib.RB_OK and st.rel_res_true[b] <= 1e-10
        if prec == "fp64":
            assert abs(st.iters[b] - ref.iters) <= 2, (st.iters[b], ref.iters)
        assert _rel(x[b], ref.x) <= 2 * _kappa(op.assemble(theta[b])) * 1e-10


def test_greedy_on_sparse_problem_matches_oracle(lib, ctx):
    op, arrs = _random(N=800)
    prob = lib.Problem.from_csr(ctx, *arrs)
    mus = log_uniform_mu(15, 20, op.Q, 0.1, 10.0)
    ref = og.adaptive_greedy(op, mus, 5, indicator="residual", snapshot_rtol=1e-12)
    basis, rep = lib.offline_build(ctx, prob, mus, n_max=5, indicator="residual",
                                   snapshot_rtol=1e-12)
    assert rep["picks"] == ref.picks
    W, AN, fN = basis.info()
    for j in range(5):
        assert np.linalg.norm(W[j] - ref.W[:, j]) <= 1e-7


@pytest.mark.parametrize("case", [1, 2])
def test_fem_cases(lib, ctx, case):
    """The paper's two P1 cases (Table 1) on a 7^3 interior mesh: greedy with the L1
    indicator (R = 4 right-hand-side terms in case 2) and converged RBCG solves at random
    parameters, against the oracle."""
    s = fem.build(case, 7, 3)
    rp, c, v = fem.csr_arrays(s)
    op = SparseAffine(rp, c, v, s.b_r)
    prob = lib.Problem.from_csr(ctx, rp, c, v)
    prob.set_rhs(s.b_r)
    mus = s.draw_mu(16, 24)
    th, ph = s.theta(mus), s.phi(mus)
    ref = og.adaptive_greedy(op, th, 4, indicator="l1", snapshot_rtol=1e-12, phis=ph)
    basis, rep = lib.offline_build(ctx, prob, th, phi=ph, n_max=4, indicator="l1",
                                   snapshot_rtol=1e-12)
    assert rep["picks"] == ref.picks
    tm = s.draw_mu(17, 6)
    tt, tp = s.theta(tm), s.phi(tm)
    x, st = lib.solve_batch(ctx, prob, basis, tt, phi=tp, flexible=True)
    x = x.cpu().numpy()
    W, AN, fN = basis.info()
    for b in range(6):
        r = orb.solve_rbcg(op, tt[b], W.T.copy(), AN, flexible=True, phi=tp[b])
        assert st.status[b] == lib.RB_OK and st.rel_res_true[b] <= 1e-10
        assert abs(st.iters[b] - r.iters) <= 2
        assert _rel(x[b], r.x) <= 2 * _kappa(op.assemble(tt[b])) * 1e-10
