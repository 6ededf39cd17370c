"""Edge and degenerate cases of the HIP path (through the C ABI) against the CPU FP64
oracle and the properties the paper proves for the RB iteration (Sec. 3.2):

  * empty batches are valid calls that do nothing;
  * a complete basis (n = N): the coarse correction is A^-1 r, so RBI and RBCG stop
    after one iteration;
  * Lemma 1: a query whose solution lies in the span of W (a snapshot parameter) is
    solved in one iteration, exactly up to rounding;
  * Lemma 2: without a smoother RBI stays at the Galerkin solution W A_N^-1 W^T f;
  * the largest basis size the library takes (n = 80) and batches of several query
    tiles with a ragged last tile.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import rb as orb
from oracle.operator import BlockDiffusion
from workloads import log_uniform_mu, random_orthonormal, random_vectors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _exact(op, theta):
    return spla.spsolve(op.assemble(theta).tocsc(), op.rhs())


def test_empty_batch(lib, ctx):
    dims, blocks = (15, 15), (2, 2)
    op = BlockDiffusion(dims, blocks)
    prob = lib.Problem(ctx, dims, blocks)
    W = random_orthonormal(1, op.N, 3)
    basis = lib.Basis.from_host(ctx, prob, W.T)
    x, st = lib.solve_batch(ctx, prob, basis, np.zeros((0, op.Q)))
    assert tuple(x.shape) == (0, op.N) and len(st.iters) == 0
    st = lib.solve_multi(ctx, [prob], [basis], [])
    assert len(st.iters) == 0
    # the context still solves afterwards (flexible beta: with a random basis and the
    # one-sided smoother the literal ratio stagnates near 1e-9, in the oracle as here)
    theta = log_uniform_mu(2, 2, op.Q, 0.1, 10.0)
    x, st = lib.solve_batch(ctx, prob, basis, theta, flexible=True)
    assert (st.status == lib.RB_OK).all() and (st.rel_res_true <= 1e-10).all()
    for b in range(2):
        ref = orb.solve_rbcg(op, theta[b], W, flexible=True)
        assert abs(st.iters[b] - ref.iters) <= 1


@pytest.mark.parametrize("dims,blocks", [((61,), (2,)), ((7, 9), (2, 2)),
                                         ((3, 5, 5), (2, 2, 3))])
def test_complete_basis_one_iteration(lib, ctx, dims, blocks):
    """n = N: W A_N^-1 W^T = A^-1, and a Gauss-Seidel sweep leaves the exact solution
    where it is, so RBCG and RBI take one iteration (as the oracle does)."""
    op = BlockDiffusion(dims, blocks)
    assert op.N <= 80
    W = random_orthonormal(5, op.N, op.N)
    prob = lib.Problem(ctx, dims, blocks)
    basis = lib.Basis.from_host(ctx, prob, W.T)
    AN, _ = orb.reduced_operators(op.A_q, [op.rhs()], W)
    theta = log_uniform_mu(6, 3, op.Q, 0.1, 10.0)
    x, st = lib.solve_batch(ctx, prob, basis, theta)
    xi, sti = lib.solve_batch(ctx, prob, basis, theta, solver="rbi")
    x, xi = x.cpu().numpy(), xi.cpu().numpy()
    for b in range(3):
        ref = orb.solve_rbcg(op, theta[b], W, AN)
        _, k, _ = orb.solve_rbi(op, theta[b], W, AN, m=10, rtol=1e-10)
        assert ref.iters == 1 and k == 1
        assert st.status[b] == lib.RB_OK and st.iters[b] == 1
        assert sti.status[b] == lib.RB_OK and sti.iters[b] == 1
        xe = _exact(op, theta[b])
        assert _rel(x[b], xe) <= 1e-11 and _rel(xi[b], xe) <= 1e-11


def test_snapshot_parameter_one_iteration(lib, ctx):
    """Lemma 1: W spans the exact solutions at five parameters; queries at two of them
    are solved in one iteration by RBI and by RBCG, a third query needs more."""
    dims, blocks = (31, 31), (2, 2)
    op = BlockDiffusion(dims, blocks)
    mus = log_uniform_mu(7, 5, op.Q, 0.1, 10.0)
    W, _ = np.linalg.qr(np.column_stack([_exact(op, m) for m in mus]))
    prob = lib.Problem(ctx, dims, blocks)
    basis = lib.Basis.from_host(ctx, prob, W.T)
    theta = np.vstack([mus[1], mus[3], log_uniform_mu(8, 1, op.Q, 0.1, 10.0)[0]])
    x, st = lib.solve_batch(ctx, prob, basis, theta)
    xi, sti = lib.solve_batch(ctx, prob, basis, theta, solver="rbi", maxit=5000)
    x, xi = x.cpu().numpy(), xi.cpu().numpy()
    for b in range(2):
        assert st.iters[b] == 1 and sti.iters[b] == 1
        xe = _exact(op, theta[b])
        assert _rel(x[b], xe) <= 1e-11 and _rel(xi[b], xe) <= 1e-11
    assert st.iters[2] > 1 and sti.iters[2] > 1
    assert (st.status == lib.RB_OK).all() and (sti.status == lib.RB_OK).all()


@pytest.mark.parametrize("dims,blocks", [((31, 31), (2, 2)), ((15, 13, 11), (2, 2, 2))])
def test_rbi_without_smoother_stagnates(lib, ctx, dims, blocks):
    """Lemma 2: with no smoother every RBI iterate is the Galerkin solution."""
    op = BlockDiffusion(dims, blocks)
    W = random_orthonormal(9, op.N, 6)
    prob = lib.Problem(ctx, dims, blocks)
    basis = lib.Basis.from_host(ctx, prob, W.T)
    AN, fN = orb.reduced_operators(op.A_q, [op.rhs()], W)
    theta = log_uniform_mu(10, 3, op.Q, 0.1, 10.0)
    for m in (1, 4):
        x, _ = lib.solve_batch(ctx, prob, basis, theta, solver="rbi", smoother="none",
                               fixed_iters=m)
        x = x.cpu().numpy()
        for b in range(3):
            ANt = orb.assemble_reduced(AN, theta[b])
            xg = W @ np.linalg.solve(ANt, fN[0])
            assert _rel(x[b], xg) <= 1e-12, (m, b)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("bf16", 5e-2)])
def test_largest_basis(lib, ctx, prec, tol):
    """n = 80, the largest basis size: projection and one preconditioner application for
    70 queries (a 64-query tile and a ragged one)."""
    dims, blocks = (31, 31), (2, 2)
    op = BlockDiffusion(dims, blocks)
    n, B = 80, 70
    W = random_orthonormal(11, op.N, n)
    prob = lib.Problem(ctx, dims, blocks)
    basis = lib.Basis.from_host(ctx, prob, W.T)
    r = random_vectors(12, B, op.N)
    t = lib.project_batch(ctx, prob, basis, _t(r), prec=prec)
    scale = np.linalg.norm(r, axis=1).max()
    assert np.abs(t - r @ W).max() / scale <= (1e-13 if prec == "fp64" else tol)
    theta = log_uniform_mu(13, B, op.Q, 0.1, 10.0)
    y = lib.precond_batch(ctx, prob, basis, theta, _t(r), prec=prec).cpu().numpy()
    AN, _ = orb.reduced_operators(op.A_q, [op.rhs()], W)
    for b in (0, 37, 63, 64, 69):
        _, M = orb.make_preconditioner(op, theta[b], W, AN)
        assert _rel(y[b], M(r[b])) <= tol, b


def test_several_query_tiles(lib, ctx):
    """300 queries (four 64-query tiles and a ragged one of 44; two projection blocks
    of 256): fixed RBCG iterations against the oracle on sampled queries, then the
    converged batch (flexible beta, which does not stagnate with a random basis)."""
    dims, blocks = (15, 15), (2, 2)
    op = BlockDiffusion(dims, blocks)
    W = random_orthonormal(14, op.N, 5)
    prob = lib.Problem(ctx, dims, blocks)
    basis = lib.Basis.from_host(ctx, prob, W.T)
    AN, _ = orb.reduced_operators(op.A_q, [op.rhs()], W)
    B = 300
    theta = log_uniform_mu(15, B, op.Q, 0.1, 10.0)
    x, _ = lib.solve_batch(ctx, prob, basis, theta, fixed_iters=6)
    x = x.cpu().numpy()
    for b in (0, 63, 64, 150, 255, 256, 299):
        ref = orb.solve_rbcg(op, theta[b], W, AN, fixed_iters=6)
        assert _rel(x[b], ref.x) <= 1e-10, b
    x, st = lib.solve_batch(ctx, prob, basis, theta, prec="fp32", flexible=True)
    assert (st.status == lib.RB_OK).all() and (st.rel_res_true <= 1e-10).all()
    x = x.cpu().numpy()
    for b in (0, 299):
        ev = np.linalg.eigvalsh(op.assemble(theta[b]).toarray())
        # a relative residual <= 1e-10 bounds the relative error by cond(A) 1e-10
        assert _rel(x[b], _exact(op, theta[b])) <= 2 * (ev[-1] / ev[0]) * 1e-10
