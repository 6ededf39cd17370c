"""Pins of the oracle's surrogate-ranked greedy step (not in the paper; its protocol is
stated in oracle/surrogate.py).  The answers here are fixed by construction: a
"network" that returns the true log-indicator must pick exactly what the plain greedy
picks, reversed predictions must trip the ranking check, and the pieces (Spearman,
top-K, exploration draws, replay buffer, standardised training) are checked against
library routines or brute force."""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import greedy, mlp
from oracle import surrogate as sg
from oracle.operator import BlockDiffusion
from workloads import log_uniform_mu


def test_spearman_matches_library_and_edge_cases():
    rng = np.random.default_rng(5)
    for n in (3, 7, 40):
        a = rng.integers(0, 5, n).astype(float)      # ties
        b = rng.standard_normal(n)
        ref = scipy.stats.spearmanr(a, b).correlation
        assert sg.spearman(a, b) == pytest.approx(ref, abs=1e-12)
    assert sg.spearman([1.0, 2.0], [2.0, 1.0]) == 1.0        # too few pairs: no check
    assert sg.spearman([1.0, 1.0, 1.0], [1.0, 2.0, 3.0]) == 0.0
    assert sg.spearman([1.0, 2.0, 3.0], [30.0, 20.0, 10.0]) == pytest.approx(-1.0)


def test_top_k_brute_force():
    rng = np.random.default_rng(6)
    v = rng.integers(0, 20, 300).astype(float)
    ex = rng.uniform(size=300) < 0.3
    cand = np.flatnonzero(~ex)
    order = cand[np.lexsort((cand, -v[cand]))]
    for K in (0, 1, 17, 500):
        got = sg.top_k(v, ex, K)
        assert got == sorted(order[:K].tolist())


def test_initial_weights_and_counter_start():
    opts = sg.SurrogateOptions(seed=99, hidden=16)
    st = sg.SurrogateState(3, opts)
    ref = mlp.init_params(3, 16, 99)
    for k in ref:
        assert np.array_equal(st.params[k], ref[k])
    assert st.counter == 16 * 3 + 16 * 16 + 16
    u = st.draw()
    assert u == mlp.uniform01(99, 16 * 3 + 16 * 16 + 16) and st.counter == 16 * 3 + 16 * 16 + 17


@pytest.fixture(scope="module")
def small():
    """A 15x15 grid, 2x2 blocks, 80 candidates, basis of 4 from the plain greedy."""
    op = BlockDiffusion((15, 15), (2, 2))
    thetas = log_uniform_mu(31, 80, op.Q, 0.1, 10.0)
    g = greedy.adaptive_greedy(op, thetas, 4, indicator="residual", snapshot_rtol=1e-12)
    eta = greedy.indicator_values(op, g.W, g.AN_q, g.fN, thetas, "residual")
    ex = np.zeros(80, dtype=bool)
    ex[g.picks] = True
    return op, thetas, g, eta, ex


def _opts(**kw):
    base = dict(topk=8, explore=6, warmup_full_sweeps=2, full_sweep_every=10, train_steps=3,
                lr=1e-3, seed=7, hidden=16)
    base.update(kw)
    return sg.SurrogateOptions(**base)


def test_perfect_network_picks_the_plain_argmax(small):
    op, thetas, g, eta, ex = small
    st = sg.SurrogateState(4, _opts())
    U = mlp.features(thetas, 0.1, 10.0)
    res = sg.surrogate_step(st, 5, U, ex, lambda idx: eta if idx is None else eta[idx],
                            predict=lambda: np.log10(eta))
    plain = greedy.masked_argmax(eta, set(np.flatnonzero(ex)))
    assert not res.full and not res.fallback
    assert res.rho == pytest.approx(1.0)
    assert res.pick == plain and res.value == eta[plain]
    assert plain in res.topk and res.true_evals == 8 + 6
    # the top-K are the K largest true values among the unpicked candidates
    cand = np.flatnonzero(~ex)
    assert set(res.topk) == set(cand[np.argsort(-eta[cand], kind="stable")[:8]].tolist())
    # exploration: distinct, unpicked, outside the top-K, drawn from the counter
    assert len(res.explore) == 6 and len(set(res.explore)) == 6
    assert not set(res.explore) & set(res.topk) and not ex[res.explore].any()


def test_reversed_network_falls_back_to_the_full_sweep(small):
    op, thetas, g, eta, ex = small
    st = sg.SurrogateState(4, _opts())
    U = mlp.features(thetas, 0.1, 10.0)
    res = sg.surrogate_step(st, 5, U, ex, lambda idx: eta if idx is None else eta[idx],
                            predict=lambda: -np.log10(eta))
    assert res.rho == pytest.approx(-1.0)
    assert res.fallback and res.full and st.fallbacks == 1
    assert res.pick == greedy.masked_argmax(eta, set(np.flatnonzero(ex)))
    assert res.true_evals == 8 + 6 + len(thetas)
    assert res.evaluated == np.flatnonzero(~ex).tolist()


@pytest.mark.parametrize("k", [1, 2, 10, 20])
def test_warmup_and_periodic_steps_are_full_sweeps(small, k):
    op, thetas, g, eta, ex = small
    st = sg.SurrogateState(4, _opts())
    U = mlp.features(thetas, 0.1, 10.0)
    res = sg.surrogate_step(st, k, U, ex, lambda idx: eta if idx is None else eta[idx],
                            predict=lambda: -np.log10(eta))  # never consulted
    assert res.full and not res.fallback and res.topk == [] and res.explore == []
    assert res.pick == greedy.masked_argmax(eta, set(np.flatnonzero(ex)))
    assert res.true_evals == len(thetas)


def test_replay_buffer_keeps_two_steps_and_drops_picks(small):
    op, thetas, g, eta, ex = small
    st = sg.SurrogateState(4, _opts(train_steps=0))
    U = mlp.features(thetas, 0.1, 10.0)
    ind = lambda idx: eta if idx is None else eta[idx]  # noqa: E731
    sg.surrogate_step(st, 1, U, ex, ind)
    n1 = len(st.buffer)
    assert n1 == int((~ex).sum()) and {e[2] for e in st.buffer} == {1}
    assert [e[0] for e in st.buffer] == np.flatnonzero(~ex).tolist()
    assert all(e[1] == pytest.approx(math.log10(eta[e[0]])) for e in st.buffer)
    ex2 = ex.copy()
    ex2[st.buffer[0][0]] = True          # picked after step 1
    sg.surrogate_step(st, 2, U, ex2, ind)
    assert {e[2] for e in st.buffer} == {1, 2}
    assert all(not ex2[e[0]] for e in st.buffer)
    sg.surrogate_step(st, 3, U, ex2, ind, predict=lambda: np.log10(eta))
    assert {e[2] for e in st.buffer} == {2, 3}


def test_training_draws_and_standardised_targets():
    """Minibatch draws continue the counter (train_steps * min(256, S) values), and
    training on standardised targets of a smooth function lowers the loss."""
    rng = np.random.default_rng(8)
    U = rng.uniform(-1, 1, (50, 3))
    opts = sg.SurrogateOptions(train_steps=40, lr=1e-2, seed=3, hidden=16)
    st = sg.SurrogateState(3, opts)
    st.buffer = [(m, 5.0 + 2.0 * math.sin(U[m, 0]) + U[m, 1], 1) for m in range(50)]
    t = np.array([e[1] for e in st.buffer])
    y = (t - t.mean()) / (t.std() + 1e-6)
    l0, _ = mlp.loss_and_grads(st.params, U, y)
    c0 = st.counter
    sg.train(st, U)
    assert st.counter == c0 + 40 * 50
    l1, _ = mlp.loss_and_grads(st.params, U, y)
    assert l1 < 0.5 * l0


def test_learned_greedy_with_a_perfect_network_is_the_plain_greedy():
    """With predictions equal to the true log-indicator every step picks the plain
    greedy's argmax, so the whole learned greedy reproduces the plain greedy's picks
    and basis; it evaluates the true indicator on far fewer candidates."""
    op = BlockDiffusion((15, 15), (2, 2))
    thetas = log_uniform_mu(33, 60, op.Q, 0.1, 10.0)
    ref = greedy.adaptive_greedy(op, thetas, 7, indicator="residual")

    def perfect(k, W, AN_q, fN, excluded):
        return np.log10(greedy.indicator_values(op, W, AN_q, fN[0], thetas, "residual"))

    opts = _opts(warmup_full_sweeps=2, full_sweep_every=5, train_steps=0)
    res = sg.learned_greedy(op, thetas, thetas, 7, 0.1, 10.0, opts, predict=perfect)
    assert res.picks == ref.picks
    assert np.abs(res.W - ref.W).max() <= 1e-12
    assert res.fallbacks == 0
    # one step per basis vector (the last one reports the final indicator): steps 1, 2
    # (warm-up) and 5 are full sweeps; steps 3, 4, 6, 7 evaluate 8 + 6 candidates
    assert res.full_sweeps == 3
    assert res.true_evals == 3 * 60 + 4 * 14
    assert res.max_indicator == pytest.approx(ref.max_indicator, rel=1e-12)
