"""Reduced-basis iteration (RBI) and RB-preconditioned CG (RBCG), oracle side.

TEST INFRASTRUCTURE ONLY.  Follows the paper step by step, in float64:

  * reduced operators A_{N,q} = W^T A_q W, f_{N,r} = W^T f_r          (eq. 12c)
  * online assembly A_N(mu) = sum_q Theta_q A_{N,q}, f_N likewise      (eq. 12b)
  * A_N(mu) is SPD and is inverted through its Cholesky factor          (Sec. 2.1)
  * RBI(A, b, W, m): residual, projection W^T r, reduced solve, update
    x += W e, post-smoothing, repeated m times (Alg. 2; eqs. 5-8)
  * RBCG(A, b, W): CG preconditioned by one RBI step from x = 0 (Alg. 3)
  * MGS(W, x): modified Gram-Schmidt of a snapshot against W (Sec. 2.2)

Readings where the paper is silent (each also listed in the design notes):
  - stopping test is relative, ||r|| <= rtol ||b|| (eq. relerr of Sec. 5.1); when the
    recursive CG residual passes, the true residual b - A x is recomputed and must
    pass too, else r is replaced by it and CG restarts with p = y
  - the iterate is held as x + xc: the updates alpha p accumulate in the correction xc,
    which is added to x (and reset to 0) just before each true-residual check.  The
    sum is the iterate of Alg. 3; the split only keeps the rounding of later updates
    relative to the small correction instead of to x, so that a residual replacement
    is not undone by the rounding of the next cycle (group-wise updating, van der Vorst
    and Ye, SIAM J. Sci. Comput. 22, 2000).  Before the first check x = 0 and the
    iterates are exactly those of x += alpha p.
  - the RBI preconditioner skips its own exit test (the outer test just failed)
  - the reduced matrix is factored once per mu; each application is two triangular
    solves (same result as re-inverting each iteration)
  - beta is the ratio y_{k+1}^T r_{k+1} / y_k^T r_k of Alg. 3; "flexible" uses y_{k+1}^T (r_{k+1} - r_k)
  - iteration count = number of products A p
  - adaptive basis size (Sec. 4.1, last paragraph): after each iteration, if
    ||r_in|| / ||r_{k+1}|| < gamma, with r_in the residual the current search direction
    was preconditioned from (r_k, or the replaced true residual after a restart), the
    number of basis vectors used by the next preconditioner application grows by one,
    up to the size of the basis; the preconditioner with n vectors uses the leading n
    columns of W and the leading n x n block of A_N
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .smoother import Smoother, RBGS, NONE


# --- offline / online reduced operators (eqs. 12b, 12c) ------------------------
def reduced_operators(A_q, f_r, W):
    """A_{N,q} = W^T A_q W (Q x n x n) and f_{N,r} = W^T f_r (R x n)."""
    AN = np.stack([W.T @ (Aq @ W) for Aq in A_q])
    fN = np.stack([W.T @ f for f in f_r])
    return AN, fN


def assemble_reduced(AN_q, theta, fN_r=None, phi=None):
    AN = np.tensordot(np.asarray(theta, dtype=np.float64), AN_q, axes=1)
    if fN_r is None:
        return AN
    phi = np.ones(fN_r.shape[0]) if phi is None else np.asarray(phi, dtype=np.float64)
    return AN, phi @ fN_r


class NotSPD(Exception):
    pass


def cholesky(AN):
    """Lower-triangular L with L L^T = A_N (Sec. 2.1)."""
    try:
        return np.linalg.cholesky(AN)
    except np.linalg.LinAlgError as exc:
        raise NotSPD(str(exc)) from exc


def chol_solve(L, t):
    """e = A_N^{-1} t = L^-T L^-1 t."""
    u = sla.solve_triangular(L, t, lower=True)
    return sla.solve_triangular(L.T, u, lower=False)


# --- RBI (Alg. 2) -------------------------------------------------------------
class RBPreconditioner:
    """One RBI iteration from x = 0 applied to a right-hand side r (the preconditioner of Alg. 3).

    With x = 0 the residual that Alg. 2 starts from is r itself (no product with A).
    W may have zero columns (W_0 = empty): then the coarse correction is 0 and only
    the smoother acts, as in the first snapshot solve of the adaptive greedy.
    """

    def __init__(self, A, W, L, smoother: Smoother):
        self.A, self.W, self.L, self.S = A, W, L, smoother

    def coarse(self, r):
        """x = W e with A_N e = W^T r (the coarse correction of Alg. 2, eq. 5)."""
        if self.W.shape[1] == 0:
            return np.zeros_like(r)
        t = self.W.T @ r
        e = chol_solve(self.L, t)
        return self.W @ e

    def __call__(self, r):
        return self.S(r, self.coarse(r))


def rbi(A, b, W, L, smoother: Smoother, m, rtol=0.0):
    """y = RBI(A, b, W, m) (Alg. 2).  Returns (x, iterations run, residual history)."""
    x = np.zeros_like(b)
    nb = np.linalg.norm(b)
    hist = []
    k = 0
    for k in range(1, m + 1):
        r = b - A @ x                              # residual
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:                       # exit test (relative reading)
            k -= 1
            break
        if W.shape[1] > 0:
            t = W.T @ r                            # projection
            e = chol_solve(L, t)                   # reduced solve
            x = x + W @ e                          # coarse update
        x = smoother(b, x)                         # post-smoothing
    return x, k, hist


# --- RBCG (Alg. 3) ------------------------------------------------------------
@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    converged: bool
    rel_res_true: float
    rel_res_recursive: float
    status: str = "ok"
    history: list = field(default_factory=list)
    iterates: list = field(default_factory=list)


def rbcg(A, b, precond, rtol=1e-10, maxit=2000, flexible=False, fixed_iters=None,
         keep_iterates=False, keep_vectors=False, adapt=None):
    """x = RBCG(A, b, W) (Alg. 3) with the stopping rule described in the module doc.

    precond: callable r -> y (one RBI step, or identity for plain CG); with adapt,
        callable (r, n) -> y using the leading n basis vectors.
    fixed_iters: run exactly this many products A p (no stopping test) for iterate parity.
    keep_vectors: record every r_k and p_k (for orthogonality checks).
    adapt: (gamma, n0, n_max) for the adaptive basis size of Sec. 4.1; the sizes used
        by the successive preconditioner applications are returned in n_history.
    """
    nb = np.linalg.norm(b)
    n = adapt[1] if adapt is not None else None
    n_hist = []
    r_in = [0.0]

    def M(v):
        r_in[0] = np.linalg.norm(v)
        if adapt is None:
            return precond(v)
        n_hist.append(n)
        return precond(v, n)

    precond_call = M
    x = np.zeros_like(b)
    xc = np.zeros_like(b)                   # updates since the last true-residual check
    r = b.copy()                            # x0 = 0, no product needed
    y = precond_call(r)
    p = y.copy()
    rho = r @ y
    it = 0
    hist = [1.0]
    iterates = []
    status = "ok"
    rel_rec = 1.0
    vecs = {"r": [r.copy()], "p": [p.copy()]} if keep_vectors else None
    while True:
        if fixed_iters is not None and it >= fixed_iters:
            break
        if it >= maxit:
            status = "noconv"
            break
        q = A @ p
        pq = p @ q
        if not pq > 0.0 or not rho > 0.0:
            status = "breakdown"
            break
        alpha = rho / pq
        xc = xc + alpha * p
        r_old = r
        r = r - alpha * q
        it += 1
        rel_rec = np.linalg.norm(r) / nb
        hist.append(rel_rec)
        if keep_iterates:
            iterates.append(x + xc)
        if adapt is not None and r_in[0] < adapt[0] * np.linalg.norm(r):
            n = min(n + 1, adapt[2])        # residual fell by less than gamma
        if fixed_iters is None and rel_rec <= rtol:   # stopping test
            x = x + xc                      # fold the correction into x
            xc = np.zeros_like(b)
            rt = b - A @ x
            if np.linalg.norm(rt) / nb <= rtol:
                break
            r = rt                          # residual replacement and restart
            y = precond_call(r)
            p = y.copy()
            rho = r @ y
            continue
        y = precond_call(r)
        rho_new = y @ r
        if flexible:
            beta = (y @ (r - r_old)) / rho
        else:
            beta = rho_new / rho
        p = y + beta * p
        rho = rho_new
        if keep_vectors:
            vecs["r"].append(r.copy())
            vecs["p"].append(p.copy())
    x = x + xc
    rel_true = np.linalg.norm(b - A @ x) / nb
    converged = status == "ok" and rel_true <= rtol
    out = SolveResult(x, it, converged, rel_true, rel_rec, status, hist, iterates)
    out.vectors = vecs
    out.n_history = n_hist
    return out


# --- modified Gram-Schmidt (Sec. 2.2; the basis update of Alg. 1 and Alg. 4) ---
class Degenerate(Exception):
    pass


def mgs(W, x, reorth_ratio=0.5, degenerate_tol=1e-12):
    """Orthonormalise x against the orthonormal columns of W.

    One modified Gram-Schmidt pass; a second pass if the norm dropped below
    reorth_ratio of its value before the pass; Degenerate if the remainder is below
    degenerate_tol * ||x||.  Returns the new unit column.
    """
    w = np.array(x, dtype=np.float64, copy=True)
    nx = np.linalg.norm(w)
    if nx == 0.0:
        raise Degenerate("zero snapshot")
    for _ in range(2):
        before = np.linalg.norm(w)
        for j in range(W.shape[1]):
            w = w - (W[:, j] @ w) * W[:, j]
        after = np.linalg.norm(w)
        if after >= reorth_ratio * before:
            break
    if after < degenerate_tol * nx:
        raise Degenerate("snapshot lies in span(W)")
    return w / after


def make_preconditioner(op, theta, W, AN_q=None, smoother_kind=RBGS, sweeps=1):
    """Build (A(theta), RBI preconditioner) for one parameter vector."""
    A = op.assemble(theta)
    S = Smoother(A, op.colors(), smoother_kind, sweeps=sweeps)
    if W.shape[1] == 0:
        return A, RBPreconditioner(A, W, None, S)
    if AN_q is None:
        AN_q, _ = reduced_operators(op.A_q, [op.rhs()], W)
    L = cholesky(assemble_reduced(AN_q, theta))
    return A, RBPreconditioner(A, W, L, S)


def _rhs(op, phi):
    """f(mu) = sum_r Phi_r f_r (eq. 12); the problem's single right-hand side if phi is
    not given."""
    return op.rhs() if phi is None else op.rhs(phi)


def solve_rbcg(op, theta, W, AN_q=None, smoother_kind=RBGS, phi=None, sweeps=1, **kw):
    A, M = make_preconditioner(op, theta, W, AN_q, smoother_kind, sweeps)
    return rbcg(A, _rhs(op, phi), M, **kw)


class NestedRBPreconditioner:
    """RBI preconditioners of every basis size n <= W.shape[1] for one parameter: the
    leading n columns of W and the Cholesky factor of the leading n x n block of
    A_N(theta), each factored on first use."""

    def __init__(self, A, W, AN, smoother: Smoother):
        self.A, self.W, self.AN, self.S = A, W, AN, smoother
        self.cache = {}

    def __call__(self, r, n):
        if n not in self.cache:
            Wn = self.W[:, :n]
            L = cholesky(self.AN[:n, :n]) if n > 0 else None
            self.cache[n] = RBPreconditioner(self.A, Wn, L, self.S)
        return self.cache[n](r)


def solve_rbcg_adaptive(op, theta, W, gamma, n0, AN_q=None, smoother_kind=RBGS, phi=None,
                        **kw):
    """RBCG with the adaptive basis size (Sec. 4.1): starts with the leading n0 vectors
    of W and grows by one whenever the residual falls by less than gamma per step."""
    A = op.assemble(theta)
    S = Smoother(A, op.colors(), smoother_kind)
    if AN_q is None:
        AN_q, _ = reduced_operators(op.A_q, [op.rhs()], W)
    M = NestedRBPreconditioner(A, W, assemble_reduced(AN_q, theta), S)
    return rbcg(A, _rhs(op, phi), M, adapt=(gamma, n0, W.shape[1]), **kw)


def solve_cg(op, theta, phi=None, **kw):
    """Plain CG (Hestenes-Stiefel): the identity preconditioner."""
    A = op.assemble(theta)
    return rbcg(A, _rhs(op, phi), lambda r: r.copy(), **kw)


def solve_rbi(op, theta, W, AN_q=None, m=2000, rtol=1e-10, smoother_kind=RBGS, phi=None,
              sweeps=1):
    A, M = make_preconditioner(op, theta, W, AN_q, smoother_kind, sweeps)
    x, k, hist = rbi(A, _rhs(op, phi), W, M.L, M.S, m, rtol)
    return x, k, hist


def residual_floor(op, theta, phi=None, refine=4):
    """Attainable accuracy in FP64 of the solution x = A(theta)^-1 f (the definition the
    iterations converge to): a sparse direct solve refined with residuals formed in
    extended precision gives x to working precision; returned are the relative residuals
    ||f - A x|| / ||f|| of that FP64 vector evaluated exactly (long double) and in FP64.
    No FP64 iterate can be expected to pass a relative-residual test much below these."""
    import scipy.sparse.linalg as spla
    A = op.assemble(theta).tocsc()
    f = _rhs(op, phi)
    lu = spla.splu(A, permc_spec="COLAMD")
    x = lu.solve(f)
    Al = A.astype(np.longdouble)
    fl = f.astype(np.longdouble)
    for _ in range(refine):
        x = x + lu.solve(np.asarray(fl - Al @ x.astype(np.longdouble), dtype=np.float64))
    nf = np.linalg.norm(f)
    exact = float(np.linalg.norm(np.asarray(fl - Al @ x.astype(np.longdouble),
                                            dtype=np.float64))) / nf
    fp64 = float(np.linalg.norm(f - A @ x)) / nf
    return exact, fp64, x
