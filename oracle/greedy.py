"""Greedy construction of the reduced basis, oracle side (test infrastructure only).

Adaptive greedy sampling (Alg. 4, Sec. 4.2), which is the greedy of Alg. 1 (Sec. 2.2)
with each snapshot solved by RBCG with the basis built so far:

  - start: mu_1 = Xi_train[seed_index], S_1 = {mu_1}, W_0 empty;
  - for N = 1..N_max: the snapshot x(mu_N) = RBCG(A(mu_N), f, W_{N-1}) (W_0 empty:
    PCG with the smoother only); W_N = MGS(W_{N-1}, x(mu_N)), growing
    A_{N,q} = W_N^T A_q W_N and f_{N,r} = W_N^T f_r (eq. 12c); the reduced solve
    A_N(mu) a(mu) = f_N(mu) (eq. 12b) for every mu in Xi_train; the next sample
    mu_{N+1} = argmax of the indicator over Xi_train without S_N, added to S_N.

Snapshot solves use the flexible beta by default: with the post-smoothing-only
preconditioner of Alg. 3 and very small bases (W_0 empty, W_1, W_2) the literal
ratio stagnates on these problems, while the flexible form converges.

Indicators: "l1" = sum_n |a_n(mu)| (the paper's, Alg. 1); "residual" =
||f - A(mu) W a(mu)|| / ||f|| evaluated directly.  Ties go to the lowest index.
If MGS finds the snapshot degenerate, the candidate is excluded and the next best
candidate of the same sweep is taken.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .rb import (Degenerate, assemble_reduced, cholesky, chol_solve, mgs,
                 solve_rbcg)


@dataclass
class GreedyResult:
    W: np.ndarray
    picks: list
    max_indicator: list
    AN_q: np.ndarray
    fN: np.ndarray
    snapshot_iters: list = field(default_factory=list)
    indicators: list = field(default_factory=list)


def reduced_coefficients(AN_q, fN, theta):
    """a(mu) = A_N(mu)^-1 f_N for one parameter vector (eq. 12b; Alg. 1 and 4)."""
    AN = assemble_reduced(AN_q, theta)
    return chol_solve(cholesky(AN), fN)


def _rhs_terms(op):
    """The right-hand-side terms f_r (R x N) of eq. 12."""
    return op.f_r if hasattr(op, "f_r") else op.rhs()[None, :]


def indicator_values(op, W, AN_q, fN, thetas, kind, phis=None):
    """fN: R x n reduced right-hand-side terms (or a vector when R = 1); f_N(mu) =
    sum_r Phi_r(mu) f_{N,r}."""
    fN = np.atleast_2d(fN)
    f = op.rhs()
    nf = np.linalg.norm(f)
    out = np.empty(len(thetas))
    for i, th in enumerate(thetas):
        fn = fN[0] if phis is None else phis[i] @ fN
        a = reduced_coefficients(AN_q, fn, th)
        if kind == "l1":
            out[i] = np.abs(a).sum()
        elif kind == "residual":
            if phis is not None:
                f = op.rhs(phis[i])
                nf = np.linalg.norm(f)
            out[i] = np.linalg.norm(f - op.assemble(th) @ (W @ a)) / nf
        else:
            raise ValueError(kind)
    return out


def masked_argmax(values, excluded):
    v = np.array(values, dtype=np.float64, copy=True)
    if np.isnan(v).any():
        raise FloatingPointError("NaN indicator")
    v[list(excluded)] = -np.inf
    return int(np.argmax(v))  # first (lowest) index among ties


def _append(op, W, AN_q, fN, w):
    """W_N = [W_{N-1}, w] and the reduced operators grown by one row/column (eq. 12c)."""
    n = W.shape[1]
    W = np.column_stack([W, w])
    newAN = np.zeros((op.Q, n + 1, n + 1))
    newAN[:, :n, :n] = AN_q
    for q, Aq in enumerate(op.A_q):
        col = W.T @ (Aq @ w)
        newAN[q, :, n] = col
        newAN[q, n, :] = col
    fr = _rhs_terms(op)
    return W, newAN, np.column_stack([np.atleast_2d(fN).reshape(len(fr), n), fr @ w])


def adaptive_greedy(op, thetas, n_max, indicator="residual", seed_index=0,
                    snapshot_rtol=1e-10, snapshot_maxit=5000, keep_indicators=False,
                    snapshot_flexible=True, phis=None, snapshot_sweeps=1):
    """phis (M x R, optional): Phi_r of every training parameter (eq. 12)."""
    N = op.N
    W = np.zeros((N, 0))
    AN_q = np.zeros((op.Q, 0, 0))
    fN = np.zeros((len(_rhs_terms(op)), 0))
    picks = []
    excluded = set()
    maxind = []
    snap_iters = []
    all_ind = []
    mu_next = int(seed_index)
    ind = None
    while W.shape[1] < n_max:
        res = solve_rbcg(op, thetas[mu_next], W, AN_q if W.shape[1] else None,
                         rtol=snapshot_rtol, maxit=snapshot_maxit,
                         flexible=snapshot_flexible, sweeps=snapshot_sweeps,
                         phi=None if phis is None else phis[mu_next])   # snapshot
        try:
            w = mgs(W, res.x)                                            # orthonormalise
        except Degenerate:
            excluded.add(mu_next)
            if ind is None:
                raise
            mu_next = masked_argmax(ind, excluded)
            continue
        picks.append(mu_next)
        excluded.add(mu_next)
        snap_iters.append(res.iters)
        W, AN_q, fN = _append(op, W, AN_q, fN, w)
        ind = indicator_values(op, W, AN_q, fN, thetas, indicator, phis)  # indicator sweep
        if keep_indicators:
            all_ind.append(ind.copy())
        if len(excluded) >= len(thetas):
            maxind.append(float(np.max(ind)))
            break
        mu_next = masked_argmax(ind, excluded)                           # next sample
        maxind.append(float(ind[mu_next]))
    return GreedyResult(W, picks, maxind, AN_q, fN[0] if len(fN) == 1 else fN, snap_iters,
                        all_ind)


def basis_from_parameters(op, thetas, snapshot_rtol=1e-10, snapshot_maxit=5000,
                          snapshot_flexible=True, phis=None, snapshot_sweeps=1):
    """The snapshot solve and basis update of Alg. 4 for a given sequence of parameters: each snapshot is solved
    by RBCG with the basis built so far and orthonormalised into it (degenerate
    snapshots are skipped).  With the parameters picked by a greedy on a coarse grid
    this is the multi-fidelity construction of Sec. 4.2 (last paragraph).  picks lists
    the indices into thetas that entered the basis."""
    W = np.zeros((op.N, 0))
    AN_q = np.zeros((op.Q, 0, 0))
    fN = np.zeros((len(_rhs_terms(op)), 0))
    picks, snap_iters = [], []
    for i, th in enumerate(thetas):
        res = solve_rbcg(op, th, W, AN_q if W.shape[1] else None, rtol=snapshot_rtol,
                         maxit=snapshot_maxit, flexible=snapshot_flexible,
                         sweeps=snapshot_sweeps,
                         phi=None if phis is None else phis[i])           # snapshot
        try:
            w = mgs(W, res.x)                                               # orthonormalise
        except Degenerate:
            continue
        picks.append(i)
        snap_iters.append(res.iters)
        W, AN_q, fN = _append(op, W, AN_q, fN, w)
    return GreedyResult(W, picks, [], AN_q, fN[0] if len(fN) == 1 else fN, snap_iters)


def multi_fidelity(op_coarse, op_fine, thetas, n_max, indicator="residual", **kw):
    """Greedy (Alg. 4) on the coarse problem, then the snapshots of its picks solved on
    the fine problem (Sec. 4.2, last paragraph).  Both problems share the parameter
    functions Theta_q (the same kappa blocks)."""
    g = adaptive_greedy(op_coarse, thetas, n_max, indicator=indicator, **kw)
    sel = [thetas[i] for i in g.picks]
    fine = basis_from_parameters(op_fine, sel)
    fine.picks = [g.picks[i] for i in fine.picks]
    return g, fine
