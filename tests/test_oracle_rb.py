"""Pins of the oracle's smoother, RBI, RBCG, Cholesky and MGS against facts fixed by the
paper (Lemmas 1-3 of Sec. 3.2, Galerkin projection eq. 2b) and by linear algebra."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import rb
from oracle.operator import BlockDiffusion
from oracle.smoother import Smoother, RBGS, RBGS_SYM, JACOBI, NONE
from workloads import random_orthonormal


def _problem(dims=(7, 7), blocks=(2, 2), seed=3):
    op = BlockDiffusion(dims, blocks)
    rng = np.random.default_rng(seed)
    theta = 10 ** rng.uniform(-1, 1, op.Q)
    return op, theta, op.assemble(theta)


def _snapshot_basis(op, n, seed=5):
    """Orthonormal basis of exact solutions at n random parameters (dense solves + QR)."""
    rng = np.random.default_rng(seed)
    X = np.column_stack([np.linalg.solve(op.assemble(10 ** rng.uniform(-1, 1, op.Q)).toarray(),
                                         op.rhs()) for _ in range(n)])
    q, _ = np.linalg.qr(X)
    return q


# --- smoother -----------------------------------------------------------------
@pytest.mark.parametrize("dims,blocks", [((7, 7), (2, 2)), ((7, 5, 3), (2, 3, 2))])
def test_rbgs_is_forward_substitution_in_red_first_order(dims, blocks):
    op, theta, A = _problem(dims, blocks)
    rng = np.random.default_rng(0)
    b, y0 = rng.standard_normal(op.N), rng.standard_normal(op.N)
    col = op.colors()
    perm = np.concatenate([np.flatnonzero(col == 0), np.flatnonzero(col == 1)])
    Ad = A.toarray()[np.ix_(perm, perm)]
    # forward: y = y0 + (D + L)^-1 (b - A y0) in the permuted order
    upd = sla.solve_triangular(np.tril(Ad), (b - A @ y0)[perm], lower=True)
    expect = y0.copy()
    expect[perm] += upd
    got = Smoother(A, col, RBGS)(b, y0)
    assert np.abs(got - expect).max() <= 1e-13 * np.abs(expect).max()
    # symmetric: forward then backward substitution
    y1 = expect
    upd2 = sla.solve_triangular(np.triu(Ad), (b - A @ y1)[perm], lower=False)
    expect2 = y1.copy()
    expect2[perm] += upd2
    got2 = Smoother(A, col, RBGS_SYM)(b, y0)
    assert np.abs(got2 - expect2).max() <= 1e-13 * np.abs(expect2).max()


def test_rbgs_ignores_red_part_of_start():
    op, theta, A = _problem()
    rng = np.random.default_rng(1)
    b, y0 = rng.standard_normal(op.N), rng.standard_normal(op.N)
    col = op.colors()
    y1 = y0.copy()
    y1[col == 0] = rng.standard_normal((col == 0).sum())
    S = Smoother(A, col, RBGS)
    assert np.array_equal(S(b, y0), S(b, y1))


@pytest.mark.parametrize("kind", [RBGS, RBGS_SYM, JACOBI, NONE])
def test_smoothers_fix_the_solution(kind):
    op, theta, A = _problem()
    b = op.rhs()
    xs = np.linalg.solve(A.toarray(), b)
    y = Smoother(A, op.colors(), kind)(b, xs)
    assert np.linalg.norm(y - xs) <= 1e-12 * np.linalg.norm(xs)


def test_gs_sweeps_converge_to_solution():
    op, theta, A = _problem()
    b = op.rhs()
    xs = np.linalg.solve(A.toarray(), b)
    S = Smoother(A, op.colors(), RBGS)
    y = np.zeros(op.N)
    for _ in range(400):
        y = S(b, y)
    assert np.linalg.norm(y - xs) <= 1e-10 * np.linalg.norm(xs)


# --- reduced operators / Cholesky ---------------------------------------------
def test_affine_reduced_assembly_equals_projection():
    op, theta, A = _problem((7, 5, 3), (2, 3, 2))
    W = random_orthonormal(7, op.N, 6)
    AN_q, fN = rb.reduced_operators(op.A_q, [op.rhs()], W)
    AN, f = rb.assemble_reduced(AN_q, theta, fN)
    assert np.abs(AN - W.T @ (A @ W)).max() <= 1e-12 * np.abs(AN).max()
    assert np.abs(f - W.T @ op.rhs()).max() <= 1e-12 * np.abs(f).max()


def test_cholesky_and_solve():
    rng = np.random.default_rng(2)
    M = rng.standard_normal((12, 12))
    S = M @ M.T + 12 * np.eye(12)
    L = rb.cholesky(S)
    assert np.allclose(np.triu(L, 1), 0)
    assert np.abs(L @ L.T - S).max() <= 1e-13 * np.abs(S).max()
    assert np.abs(L - sla.cholesky(S, lower=True)).max() <= 1e-13 * np.abs(L).max()
    t = rng.standard_normal(12)
    assert np.linalg.norm(S @ rb.chol_solve(L, t) - t) <= 1e-12 * np.linalg.norm(t)
    with pytest.raises(rb.NotSPD):
        rb.cholesky(-S)


# --- RBI: Galerkin step and Lemmas 1-3 (Sec. 3.2) ------------------------------
def test_first_coarse_correction_is_galerkin():
    """After the coarse update of the first RBI iteration, W^T (f - A x_hat) = 0 (eq. 2b)."""
    op, theta, A = _problem()
    W = _snapshot_basis(op, 4)
    A_, M = rb.make_preconditioner(op, theta, W)
    f = op.rhs()
    xhat = M.coarse(f)
    assert np.linalg.norm(W.T @ (f - A @ xhat)) <= 1e-12 * np.linalg.norm(W.T @ f)


def test_lemma1_complete_basis_one_step():
    op, theta, A = _problem()
    W = random_orthonormal(11, op.N, op.N)
    x, k, hist = rb.solve_rbi(op, theta, W, m=5, rtol=1e-12)
    assert k == 1
    res = rb.solve_rbcg(op, theta, W, rtol=1e-12)
    assert res.iters == 1 and res.rel_res_true <= 1e-12


def test_lemma1_snapshot_parameter():
    """For mu in S_N the first RB iterate x_hat equals the snapshot x(mu)."""
    op = BlockDiffusion((7, 7), (2, 2))
    rng = np.random.default_rng(4)
    thetas = 10 ** rng.uniform(-1, 1, (3, op.Q))
    X = np.column_stack([np.linalg.solve(op.assemble(t).toarray(), op.rhs()) for t in thetas])
    W, _ = np.linalg.qr(X)
    for j, t in enumerate(thetas):
        A, M = rb.make_preconditioner(op, t, W)
        assert np.linalg.norm(M.coarse(op.rhs()) - X[:, j]) <= 1e-11 * np.linalg.norm(X[:, j])


def test_lemma2_stagnation_without_smoother():
    op, theta, A = _problem()
    W = _snapshot_basis(op, 3)
    A_, M = rb.make_preconditioner(op, theta, W, smoother_kind=NONE)
    f = op.rhs()
    x1, _, _ = rb.rbi(A, f, W, M.L, M.S, 1)
    x2, _, _ = rb.rbi(A, f, W, M.L, M.S, 2)
    xhat = M.coarse(f)
    assert np.linalg.norm(x1 - xhat) <= 1e-13 * np.linalg.norm(xhat)
    assert np.linalg.norm(x2 - x1) <= 1e-12 * np.linalg.norm(x1)


def test_lemma3_error_approximation():
    """The coarse correction W e_N is the Galerkin approximation of the error A^-1 r."""
    op, theta, A = _problem()
    W = _snapshot_basis(op, 4)
    Ad = A.toarray()
    xs = np.linalg.solve(Ad, op.rhs())
    rng = np.random.default_rng(8)
    x = rng.standard_normal(op.N)
    r = op.rhs() - A @ x
    A_, M = rb.make_preconditioner(op, theta, W)
    We = M.coarse(r)
    expect = W @ np.linalg.solve(W.T @ Ad @ W, W.T @ Ad @ (xs - x))
    assert np.linalg.norm(We - expect) <= 1e-11 * np.linalg.norm(expect)


def test_rbi_converges_to_dense_solution():
    op, theta, A = _problem()
    W = _snapshot_basis(op, 3)
    x, k, hist = rb.solve_rbi(op, theta, W, m=500, rtol=1e-12)
    xs = np.linalg.solve(A.toarray(), op.rhs())
    assert hist[-1] <= 1e-12 or np.linalg.norm(op.rhs() - A @ x) <= 1e-12 * np.linalg.norm(op.rhs())
    assert np.linalg.norm(x - xs) <= np.linalg.cond(A.toarray()) * 1e-12 * np.linalg.norm(xs)


# --- CG mechanics -------------------------------------------------------------
def test_plain_cg_orthogonality_and_finite_termination():
    op, theta, A = _problem()
    res = rb.solve_cg(op, theta, fixed_iters=10, keep_vectors=True)
    R = np.column_stack(res.vectors["r"][:10])
    P = np.column_stack(res.vectors["p"][:10])
    G = R.T @ R
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() <= 1e-10 * np.sqrt(np.outer(np.diag(G), np.diag(G))).max()
    H = P.T @ (A @ P)
    offh = H - np.diag(np.diag(H))
    assert np.abs(offh).max() <= 1e-10 * np.abs(np.diag(H)).max()
    # finite termination: with kappa uniform on a 7x7 grid and f = 1 only the modes with
    # odd wave numbers (1,3,5,7 per axis) are excited, so A restricted to the Krylov space
    # has at most 10 distinct eigenvalues (lambda_j + lambda_k, j <= k): CG ends in <= 10 steps
    full = rb.solve_cg(op, np.full(op.Q, 1.7), rtol=1e-10)
    assert full.converged and full.iters <= 10


def test_rbcg_residual_orthogonal_to_last_direction():
    """For the non-symmetric RB preconditioner only r_{k+1}^T p_k = 0 holds."""
    op, theta, A = _problem()
    W = _snapshot_basis(op, 2)
    A_, M = rb.make_preconditioner(op, theta, W)
    res = rb.rbcg(A, op.rhs(), M, fixed_iters=8, keep_vectors=True)
    r, p = res.vectors["r"], res.vectors["p"]
    for k in range(len(p) - 1):
        assert abs(r[k + 1] @ p[k]) <= 1e-10 * np.linalg.norm(r[k + 1]) * np.linalg.norm(p[k])


@pytest.mark.parametrize("flexible", [False, True])
@pytest.mark.parametrize("dims,blocks", [((15, 15), (2, 2)), ((7, 7, 7), (2, 2, 2))])
def test_rbcg_converged_solution_matches_dense(dims, blocks, flexible):
    op, theta, A = _problem(dims, blocks)
    W = _snapshot_basis(op, 5)
    res = rb.solve_rbcg(op, theta, W, rtol=1e-10, flexible=flexible)
    assert res.converged and res.rel_res_true <= 1e-10
    Ad = A.toarray()
    xs = np.linalg.solve(Ad, op.rhs())
    bound = np.linalg.cond(Ad) * 1e-10
    assert np.linalg.norm(res.x - xs) <= bound * np.linalg.norm(xs)


# --- MGS ----------------------------------------------------------------------
def test_mgs_orthonormal_and_span():
    op = BlockDiffusion((7, 7), (2, 2))
    rng = np.random.default_rng(9)
    X = np.column_stack([np.linalg.solve(op.assemble(10 ** rng.uniform(-1, 1, op.Q)).toarray(),
                                         op.rhs()) for _ in range(8)])
    W = np.zeros((op.N, 0))
    for j in range(X.shape[1]):
        W = np.column_stack([W, rb.mgs(W, X[:, j])])
    assert np.abs(W.T @ W - np.eye(W.shape[1])).max() <= 1e-13
    # every snapshot lies in span(W)
    for j in range(X.shape[1]):
        assert np.linalg.norm(X[:, j] - W @ (W.T @ X[:, j])) <= 1e-12 * np.linalg.norm(X[:, j])
    with pytest.raises(rb.Degenerate):
        rb.mgs(W, X[:, 3])


# ---- adaptive basis size (Sec. 4.1, last paragraph) ----------------------------------
def _adaptive_case(n_basis, dims=(15, 15), seed=3):
    op = BlockDiffusion(dims, (2, 2))
    W = random_orthonormal(seed, op.N, n_basis)
    theta = np.array([0.3, 2.0, 5.0, 0.7])
    return op, W, theta


def test_adaptive_gamma_zero_is_fixed_size():
    """gamma = 0: the size never grows, so the run equals RBCG with the leading n0
    columns, iterate for iterate."""
    op, W, theta = _adaptive_case(8)
    a = rb.solve_rbcg_adaptive(op, theta, W, 0.0, 3, flexible=True, keep_iterates=True)
    f = rb.solve_rbcg(op, theta, W[:, :3], flexible=True, keep_iterates=True)
    assert a.iters == f.iters and set(a.n_history) == {3}
    for xa, xf in zip(a.iterates, f.iterates):
        assert np.array_equal(xa, xf)


def test_adaptive_complete_basis_terminates():
    """gamma huge: the size grows by one per iteration (capped at the basis size);
    once the basis is complete (n = N) the preconditioner is A^-1 and CG stops at the
    next step, so at most N - n0 + 2 iterations on a 5 x 5 grid."""
    op = BlockDiffusion((5, 5), (2, 2))
    W = random_orthonormal(4, op.N, op.N)
    theta = np.array([0.3, 2.0, 5.0, 0.7])
    n0 = 3
    a = rb.solve_rbcg_adaptive(op, theta, W, 1e300, n0, flexible=True, rtol=1e-12)
    assert a.converged and a.iters <= op.N - n0 + 2
    assert a.n_history == [min(n0 + k, op.N) for k in range(len(a.n_history))]


def test_adaptive_two_steps_by_hand():
    """Two iterations built by hand from fixed-size preconditioners: gamma is set just
    above the first step's reduction factor, so the second direction must come from the
    preconditioner with one more vector (flexible beta)."""
    op, W, theta = _adaptive_case(8)
    A = op.assemble(theta)
    b = op.rhs()
    S = Smoother(A, op.colors(), RBGS)
    AN, _ = rb.reduced_operators(op.A_q, [b], W)
    ANt = rb.assemble_reduced(AN, theta)

    def M(n):
        return rb.RBPreconditioner(A, W[:, :n], rb.cholesky(ANt[:n, :n]), S)

    n0 = 2
    r0 = b.copy()
    y0 = M(n0)(r0)
    p0 = y0
    a0 = (r0 @ y0) / (p0 @ (A @ p0))
    x1 = a0 * p0
    r1 = r0 - a0 * (A @ p0)
    ratio = np.linalg.norm(r0) / np.linalg.norm(r1)
    gamma = 1.5 * ratio                       # ratio < gamma: grow to n0 + 1
    y1 = M(n0 + 1)(r1)
    beta = (y1 @ (r1 - r0)) / (r0 @ y0)
    p1 = y1 + beta * p0
    a1 = (r1 @ y1) / (p1 @ (A @ p1))
    x2 = x1 + a1 * p1
    ad = rb.solve_rbcg_adaptive(op, theta, W, gamma, n0, flexible=True, fixed_iters=2)
    assert ad.n_history[:2] == [n0, n0 + 1]
    assert np.linalg.norm(ad.x - x2) <= 1e-13 * np.linalg.norm(x2)
    # and with gamma below the reduction factor the size stays
    ad2 = rb.solve_rbcg_adaptive(op, theta, W, 0.5 * ratio, n0, flexible=True, fixed_iters=2)
    assert ad2.n_history[:2] == [n0, n0]


def test_several_sweeps_are_repeated_forward_substitution():
    """k forward red-black sweeps equal k steps y <- y + (D + L)^-1 (b - A y) in the
    red-first ordering, built from the dense matrix."""
    op = BlockDiffusion((9, 7), (2, 2))
    th = np.array([0.4, 3.0, 1.7, 0.9])
    A = op.assemble(th)
    c = op.colors()
    order = np.argsort(c, kind="stable")
    P = A.toarray()[np.ix_(order, order)]
    DL = np.tril(P)
    rng = np.random.default_rng(11)
    b, y0 = rng.standard_normal(op.N), rng.standard_normal(op.N)
    for k in (2, 3):
        ref = y0[order].copy()
        for _ in range(k):
            ref = ref + np.linalg.solve(DL, b[order] - P @ ref)
        y = Smoother(A, c, RBGS, sweeps=k)(b, y0)
        assert np.abs(y[order] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_residual_replacement_restarts_on_the_residual_equation():
    """R4 (stopping rule): when the recursive residual passes and the true residual
    f - A x does not, r is replaced by the true residual and CG restarts with p = M r.
    One product A p of the recursion is perturbed (a transient error), so the recursive
    residual drifts from the true one and the replacement must happen.  Pins: the solve
    still ends with a true residual <= rtol, and every iterate after the restart equals
    x_k + (the RBCG iterate of the residual equation A e = f - A x_k started from 0),
    which is what a restart is; a kept beta, a stale rho or an unpreconditioned restart
    direction each break the equality."""
    op, theta, A = _problem((15, 15), (2, 2), seed=11)
    W = _snapshot_basis(op, 3, seed=12)
    f = op.rhs()
    AN, _ = rb.reduced_operators(op.A_q, [f], W)
    Wr = W
    S = Smoother(A, op.colors(), RBGS)
    L = rb.cholesky(rb.assemble_reduced(AN, theta))
    precond = rb.RBPreconditioner(A, Wr, L, S)
    rng = np.random.default_rng(13)
    delta = rng.standard_normal(op.N)

    class Perturbed:
        """A whose third matrix-vector product (q = A p of iteration 3) is off by 1e-4."""

        def __init__(self):
            self.calls = 0

        def __matmul__(self, v):
            self.calls += 1
            out = A @ v
            if self.calls == 3:
                out = out + 1e-4 * np.linalg.norm(out) / np.linalg.norm(delta) * delta
            return out

    res = rb.rbcg(Perturbed(), f, precond, rtol=1e-10, keep_iterates=True)
    assert res.converged and res.rel_res_true <= 1e-10
    hist = np.array(res.history)
    k = int(np.flatnonzero(hist <= 1e-10)[0])          # first recursive pass = restart
    assert k < res.iters, "the true residual check must have failed once"
    # the restarted residual is the true one: the next recursive value jumps up
    assert hist[k + 1] > 1e3 * hist[k]
    xk = res.iterates[k - 1]
    rk = f - A @ xk
    for m in (1, 2, 5, res.iters - k):
        e = rb.rbcg(A, rk, precond, fixed_iters=m).x
        want = xk + e
        got = res.iterates[k - 1 + m]
        assert np.linalg.norm(got - want) <= 1e-9 * np.linalg.norm(e), m


def test_residual_floor_small_grid():
    """On a 15x15 grid the refined direct solution equals the dense solve, and its residual
    is at the level of the rounding of x (relative eps times the conditioning of the
    residual evaluation), far below any tolerance used by the solvers."""
    op = BlockDiffusion((15, 15), (2, 2))
    th = np.array([0.01, 100.0, 3.0, 0.5])
    exact, fp64, x = rb.residual_floor(op, th)
    xd = np.linalg.solve(op.assemble(th).toarray(), op.rhs())
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)
    assert exact <= 1e-13 and fp64 <= 1e-13
    # the FP64 evaluation equals the residual formed directly
    assert fp64 == np.linalg.norm(op.rhs() - op.assemble(th).tocsc() @ x) / np.linalg.norm(op.rhs())
