"""Surrogate-ranked greedy step, oracle side (TEST INFRASTRUCTURE ONLY).

Not part of the paper.  The paper's greedy (Alg. 1, Sec. 2.2; Alg. 4, Sec. 4.2) takes
the next sample as the argmax of an indicator over the whole training set.  Here a
small network (mlp.py) ranks the candidates so that the true indicator is evaluated on
a short list only; the true indicator still decides every pick.  One greedy step k
(k = 1, 2, ... counts the basis vectors added so far):

  1. A step is a full sweep when k <= warmup_full_sweeps or k is a multiple of
     full_sweep_every: the true indicator on every candidate, pick = the argmax over the
     unpicked ones (exactly the plain greedy).
  2. Otherwise the network predicts log10(indicator) for every candidate; the short
     list is the top-K unpicked candidates by prediction (ties to the lower index, the
     list in increasing index order) followed by `explore` further unpicked candidates
     drawn uniformly at random (index floor(u M), capped at M - 1, redrawn when picked
     or already listed, at most 100 * explore draws).  The true indicator is evaluated
     on the short list.
  3. Ranking check: if at least 3 candidates were explored and the Spearman rank
     correlation of prediction and log10(true indicator) over them is below 0.5, the
     step falls back to a full sweep (1).  Otherwise the pick is the argmax of the TRUE
     indicator over the short list (ties to the lower index).
  4. Replay buffer: every evaluated unpicked candidate with a positive finite
     indicator is appended as (index, log10 indicator, k), in the order evaluated
     (short list order, or index order after a full sweep); then entries older than
     step k - 1 and entries of picked candidates are dropped.
  5. Training: targets standardised over the buffer (mean, population standard
     deviation + 1e-6), then `train_steps` Adam steps, each on a minibatch of
     min(256, buffer size) entries drawn uniformly with replacement (entry
     floor(u S), capped at S - 1).

Random numbers: one counter-based SplitMix64 sequence per surrogate (seed `seed`):
the Glorot initial weights take its first H P + H H + H values (mlp.init_params), the
exploration and minibatch draws continue from there.  Features are
u = (log10 mu - mid) / half of the log range (mlp.features).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import mlp


@dataclass
class SurrogateOptions:
    topk: int = 256
    explore: int = 64
    warmup_full_sweeps: int = 4
    full_sweep_every: int = 10
    train_steps: int = 50
    lr: float = 1e-3
    seed: int = 1234
    hidden: int = 128
    minibatch: int = 256
    bf16: bool = False      # products with BF16 operands (mlp.forward / loss_and_grads)


def init_draws(P: int, H: int) -> int:
    """How many values of the counter sequence the initial weights take."""
    return H * P + H * H + H


class SurrogateState:
    """Network parameters, Adam moments, replay buffer and the position in the counter
    sequence."""

    def __init__(self, P, opts: SurrogateOptions, params=None):
        self.P = P
        self.opts = opts
        self.params = (mlp.init_params(P, opts.hidden, opts.seed) if params is None
                       else {k: np.array(v, dtype=np.float64) for k, v in params.items()})
        self.adam = mlp.Adam(self.params, lr=opts.lr)
        self.buffer: list = []          # (index, target, step)
        self.counter = init_draws(P, opts.hidden)
        self.fallbacks = 0
        self.last_loss = 0.0

    def draw(self) -> float:
        u = mlp.uniform01(self.opts.seed, self.counter)
        self.counter += 1
        return u


def average_ranks(v):
    """Ranks 0..n-1 of v in increasing order, tied values sharing their mean rank."""
    v = np.asarray(v, dtype=np.float64)
    order = sorted(range(len(v)), key=lambda i: v[i])
    r = np.empty(len(v))
    i = 0
    while i < len(order):
        j = i
        while j + 1 < len(order) and v[order[j + 1]] == v[order[i]]:
            j += 1
        for t in range(i, j + 1):
            r[order[t]] = 0.5 * (i + j)
        i = j + 1
    return r


def spearman(a, b) -> float:
    """Pearson correlation of the average ranks; 1 for fewer than 3 pairs, 0 when either
    side is constant."""
    if len(a) < 3:
        return 1.0
    ra, rb = average_ranks(a), average_ranks(b)
    da, db = ra - ra.mean(), rb - rb.mean()
    saa, sbb = float(da @ da), float(db @ db)
    if saa <= 0 or sbb <= 0:
        return 0.0
    return float(da @ db) / math.sqrt(saa * sbb)


def top_k(pred, excluded, K):
    """The K unpicked candidates with the largest prediction (ties to the lower index),
    in increasing index order."""
    cand = [m for m in range(len(pred)) if not excluded[m]]
    cand.sort(key=lambda m: (-float(pred[m]), m))
    return sorted(cand[:K])


def argmax_lowest(values, allowed):
    """Index of the largest value among `allowed` (ties to the lower index); NaN is an
    error (a reduced matrix that is not SPD)."""
    best, arg = -math.inf, None
    for m in sorted(allowed):
        v = float(values[m])
        if math.isnan(v):
            raise FloatingPointError("NaN indicator")
        if arg is None or v > best:
            best, arg = v, m
    return arg, best


@dataclass
class StepResult:
    pick: int | None
    value: float
    full: bool
    fallback: bool
    topk: list = field(default_factory=list)
    explore: list = field(default_factory=list)
    evaluated: list = field(default_factory=list)
    rho: float | None = None
    true_evals: int = 0
    indicator: np.ndarray | None = None  # true values known after the step (-inf: not evaluated)


def surrogate_step(state: SurrogateState, k: int, U, excluded, true_indicator,
                   predict=None) -> StepResult:
    """One greedy step with the surrogate (steps 1-5 of the module docstring).

    U: M x P features; excluded: M flags of the picked candidates; true_indicator(idx)
    returns the true indicator of the listed candidates (idx None: all of them);
    predict (optional) replaces the network's predictions (a function of no argument
    returning M values), for tests of the protocol itself."""
    o = state.opts
    M = len(excluded)
    excluded = np.asarray(excluded, dtype=bool)
    full = k <= o.warmup_full_sweeps or (o.full_sweep_every > 0 and k % o.full_sweep_every == 0)
    ind = np.full(M, -math.inf)
    res = StepResult(None, 0.0, full, False)
    evaluated: list = []
    if not full:
        pred = np.asarray(predict() if predict is not None
                          else mlp.forward(state.params, U, bf16=o.bf16), dtype=np.float64)
        tk = top_k(pred, excluded, o.topk)
        listed = set(tk)
        expl = []
        tries = 0
        while len(expl) < o.explore and tries < 100 * max(o.explore, 1):
            tries += 1
            m = min(M - 1, int(state.draw() * M))
            if excluded[m] or m in listed:
                continue
            listed.add(m)
            expl.append(m)
        res.topk, res.explore = tk, expl
        evaluated = tk + expl
        if not evaluated:
            res.indicator = ind
            return res
        vals = np.asarray(true_indicator(evaluated), dtype=np.float64)
        res.true_evals += len(evaluated)
        ind[evaluated] = vals
        if len(expl) >= 3:
            te = [math.log10(max(float(ind[m]), 1e-300)) for m in expl]
            res.rho = spearman([pred[m] for m in expl], te)
        if res.rho is not None and res.rho < 0.5:
            res.fallback = True
            state.fallbacks += 1
            full = True
        else:
            res.pick, res.value = argmax_lowest(ind, evaluated)
    if full:
        ind = np.asarray(true_indicator(None), dtype=np.float64).copy()
        res.true_evals += M
        res.pick, res.value = argmax_lowest(ind, [m for m in range(M) if not excluded[m]])
        evaluated = [m for m in range(M) if not excluded[m]]
    res.full = full
    res.evaluated = evaluated
    res.indicator = ind
    # replay buffer: this step's pairs, then only the last two steps, picked ones dropped
    for m in evaluated:
        v = float(ind[m])
        if not excluded[m] and v > 0 and math.isfinite(v):
            state.buffer.append((m, math.log10(v), k))
    state.buffer = [e for e in state.buffer if e[2] >= k - 1 and not excluded[e[0]]]
    train(state, U)
    return res


def train(state: SurrogateState, U):
    """Standardised targets over the buffer, then train_steps Adam steps on minibatches
    drawn with replacement."""
    buf = state.buffer
    if not buf:
        return
    t = np.array([e[1] for e in buf])
    mean = float(t.mean())
    sd = math.sqrt(float(((t - mean) ** 2).mean())) + 1e-6
    S = len(buf)
    mb = min(state.opts.minibatch, S)
    U = np.asarray(U, dtype=np.float64)
    for _ in range(state.opts.train_steps):
        pick = [min(S - 1, int(state.draw() * S)) for _ in range(mb)]
        X = U[[buf[e][0] for e in pick]]
        y = np.array([(buf[e][1] - mean) / sd for e in pick])
        loss, g = mlp.loss_and_grads(state.params, X, y, bf16=state.opts.bf16)
        state.adam.step(state.params, g)
        state.last_loss = loss


@dataclass
class LearnedGreedyResult:
    W: np.ndarray
    picks: list
    max_indicator: list
    AN_q: np.ndarray
    fN: np.ndarray
    true_evals: int
    full_sweeps: int
    fallbacks: int
    steps: list


def learned_greedy(op, thetas, mus, n_max, mu_lo, mu_hi, opts: SurrogateOptions,
                   indicator="residual", seed_index=0, snapshot_rtol=1e-10,
                   snapshot_maxit=5000, predict=None):
    """The adaptive greedy of Alg. 4 with each sweep-and-argmax replaced by
    surrogate_step.  predict(k, W, AN_q, fN, excluded) (optional) replaces the network,
    for tests of the protocol."""
    from .greedy import _append, indicator_values
    from .rb import Degenerate, mgs, solve_rbcg

    M = len(thetas)
    U = mlp.features(np.asarray(mus, dtype=np.float64), mu_lo, mu_hi)
    state = SurrogateState(U.shape[1], opts)
    W = np.zeros((op.N, 0))
    AN_q = np.zeros((op.Q, 0, 0))
    fN = np.zeros((1, 0))
    excluded = np.zeros(M, dtype=bool)
    picks, maxind, steps = [], [], []
    true_evals = full_sweeps = 0
    last_ind = None
    mu_next = int(seed_index)
    k = 0
    while W.shape[1] < n_max:
        snap = solve_rbcg(op, thetas[mu_next], W, AN_q if W.shape[1] else None,
                          rtol=snapshot_rtol, maxit=snapshot_maxit, flexible=True)
        excluded[mu_next] = True
        try:
            w = mgs(W, snap.x)
        except Degenerate:
            if last_ind is None:
                raise
            mu_next, _ = argmax_lowest(last_ind, [m for m in range(M) if not excluded[m]])
            if mu_next is None:
                raise
            continue
        picks.append(mu_next)
        W, AN_q, fN = _append(op, W, AN_q, fN, w)
        k += 1

        def true_ind(idx, W=W, AN_q=AN_q, fN=fN):
            th = thetas if idx is None else thetas[idx]
            return indicator_values(op, W, AN_q, fN[0], th, indicator)

        pr = None
        if predict is not None:
            pr = (lambda W=W, AN_q=AN_q, fN=fN, k=k: predict(k, W, AN_q, fN, excluded.copy()))
        res = surrogate_step(state, k, U, excluded.copy(), true_ind, predict=pr)
        steps.append(res)
        true_evals += res.true_evals
        full_sweeps += int(res.full)
        last_ind = res.indicator
        maxind.append(res.value)
        if res.pick is None:
            break
        mu_next = res.pick
    return LearnedGreedyResult(W, picks, maxind, AN_q, fN[0], true_evals, full_sweeps,
                               state.fallbacks, steps)
