"""Parity cases at the shapes of the other workloads (the benchmark's own 127^3 batch is
in test_gpu_fullsize.py):

  * 2D 63x63, kappa on 2x2 blocks, greedy over 256 parameters to n = 20, 16 test
    parameters solved one at a time in FP64: greedy picks and basis against the
    oracle's greedy, every solve against the oracle's RBCG with the same basis;
  * 3D 63^3, greedy over 10^4 parameters to n = 60, plain residual sweep vs the
    MLP-ranked sweep: the surrogate saves true evaluations and its basis is about as
    good on held-out parameters (indicators computed by the oracle's operator);
  * 3D 255^3 (N = 16,581,375), n = 80, 64 queries per batch, FP32 preconditioner: too
    large for the oracle's solver, so checked by properties that hold at any size.
    The basis is the 80 smoothest discrete sine modes (orthonormal on the grid), which
    the greedy would take minutes to match; every query converges, and sampled
    solutions satisfy the residual bound under the oracle's own operator;
  * the uneven batch (four grids, four basis sizes, one call), on 256 of its queries.
"""
import math

import numpy as np
import pytest

from oracle import greedy as og
from oracle import rb as orb
from oracle.operator import BlockDiffusion
from workloads import WORKLOADS, sine_basis

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _kappa_bound(dims, theta):
    # lambda_max <= max(mu) sum_a 4 / h_a^2 (Gershgorin); lambda_min >= min(mu) times the
    # smallest Dirichlet eigenvalue of the unit-coefficient Laplacian, sum_a 4 / h_a^2
    # sin^2(pi h_a / 2)
    h = [1.0 / (m + 1) for m in dims]
    lmax = max(theta) * sum(4.0 / ha**2 for ha in h)
    lmin = min(theta) * sum(4.0 / ha**2 * math.sin(math.pi * ha / 2) ** 2 for ha in h)
    return lmax / lmin


def test_plain_fp64_configuration(lib, ctx):
    """63x63, 2x2 blocks, FP64.  The GPU greedy against the oracle's greedy: the same picks,
    and columns within 1e-6 (each snapshot is an iterative solution to 1e-12, so the two
    sides' snapshots already differ by about kappa * 1e-12).  The online solves then run
    on the oracle's basis on both sides, so only summation order differs: the 16 test
    parameters one at a time and as one batch of 16, the converged solutions within 1e-10
    of the oracle's (its iterate after the GPU's iteration count if the two stopped one
    iteration apart), and the iterates after a fixed 5 iterations within 1e-10."""
    w = WORKLOADS["2d63"]
    op = BlockDiffusion(w.dims, w.blocks)
    train = w.train_mu()
    ref = og.adaptive_greedy(op, train, w.n, indicator="residual", snapshot_rtol=1e-12)
    prob = lib.Problem(ctx, w.dims, w.blocks)
    gbasis, rep = lib.offline_build(ctx, prob, train, mu=train, n_max=w.n, indicator="residual",
                                    snapshot_rtol=1e-12)
    assert rep["picks"] == ref.picks
    Wn, _, _ = gbasis.info()
    assert np.abs(Wn @ Wn.T - np.eye(w.n)).max() <= 1e-12
    for j in range(w.n):
        assert np.linalg.norm(Wn[j] - ref.W[:, j]) <= 1e-6, j
    # online: the oracle's basis on both sides
    W = ref.W
    AN, _ = orb.reduced_operators(op.A_q, [op.rhs()], W)
    basis = lib.Basis.from_host(ctx, prob, W.T)
    test = w.test_mu()
    k_fixed = 5
    xb, sb = lib.solve_batch(ctx, prob, basis, test)
    xk, sk = lib.solve_batch(ctx, prob, basis, test, fixed_iters=k_fixed)
    xb, xk = xb.cpu().numpy(), xk.cpu().numpy()
    errs = []
    for b in range(w.B):
        x, st = lib.solve_batch(ctx, prob, basis, test[b:b + 1])
        r = orb.solve_rbcg(op, test[b], W, AN)
        assert r.converged
        for xg, sg in ((x[0].cpu().numpy(), (st.status[0], st.rel_res_true[0], st.iters[0])),
                       (xb[b], (sb.status[b], sb.rel_res_true[b], sb.iters[b]))):
            status, rel, its = sg
            assert status == lib.RB_OK and rel <= 1e-10
            assert abs(int(its) - r.iters) <= 1, (b, its, r.iters)
            xo = r.x if int(its) == r.iters else orb.solve_rbcg(op, test[b], W, AN,
                                                                 fixed_iters=int(its)).x
            errs.append(_rel(xg, xo))
            assert errs[-1] <= 1e-10, (b, errs[-1])
        rk = orb.solve_rbcg(op, test[b], W, AN, fixed_iters=k_fixed)
        assert sk.iters[b] == k_fixed
        assert _rel(xk[b], rk.x) <= 1e-10, (b, _rel(xk[b], rk.x))
    print(f"63^2 FP64: largest converged-solution difference from the oracle {max(errs):.2e}")


def test_learned_greedy_configuration(lib, ctx):
    w = WORKLOADS["3d63"]
    op = BlockDiffusion(w.dims, w.blocks)
    prob = lib.Problem(ctx, w.dims, w.blocks)
    train = w.train_mu()
    held = w.test_mu(100)
    f = op.rhs()
    out = {}
    for name, kw in (("plain", {}), ("surrogate", dict(use_surrogate=1, topk=256, explore=64,
                                                      warmup_full_sweeps=4, full_sweep_every=10,
                                                      train_steps=50, lr=1e-3, mu_lo=0.1,
                                                      mu_hi=10.0, seed=1004))):
        basis, rep = lib.offline_build(ctx, prob, train, mu=train, n_max=w.n,
                                       indicator="residual", **kw)
        assert rep["n_built"] == w.n and len(set(rep["picks"])) == w.n
        Wn, AN, fN = basis.info()
        assert np.abs(Wn @ Wn.T - np.eye(w.n)).max() <= 1e-10
        worst = 0.0
        for th in held:
            a = np.linalg.solve(np.tensordot(th, AN, axes=1), fN[0])
            eta = np.linalg.norm(f - op.apply(th, Wn.T @ a)) / np.linalg.norm(f)
            worst = max(worst, eta)
        out[name] = (rep["true_evals"], worst)
    print(f"true evaluations / held-out max eta: {out}")
    assert out["plain"][0] == w.n * w.M_train
    assert out["surrogate"][0] < 0.6 * out["plain"][0]
    assert out["surrogate"][1] <= 3.0 * out["plain"][1]


def test_large_configuration_properties(lib, ctx):
    import torch
    w = WORKLOADS["3d255"]
    op = BlockDiffusion(w.dims, w.blocks)
    prob = lib.Problem(ctx, w.dims, w.blocks)
    Wn = sine_basis(w.dims, w.n)
    basis = lib.Basis.from_host(ctx, prob, Wn)
    del Wn
    test = w.test_mu()
    x, st = lib.solve_batch(ctx, prob, basis, test, prec="fp32", maxit=5000)
    assert (st.status == lib.RB_OK).all()
    assert st.rel_res_true.max() <= 1e-10
    f = op.rhs()
    for b in (0, 41):
        xb = x[b].cpu().numpy()
        assert np.linalg.norm(f - op.apply(test[b], xb)) / np.linalg.norm(f) <= 1.01e-10
    print(f"255^3, n = 80, B = 64: iterations {st.iters.min()}..{st.iters.max()}")
    del x, basis
    torch.cuda.empty_cache()


def test_large_configuration_paths_on_a_thin_grid(lib, ctx):
    """The paths the 255^3 workload takes, at a size the oracle solves: rows of 255 nodes
    (whole-row tiles of the z-marching passes, 4 x 255 nodes, and a ragged last row tile),
    a basis of n = 80 (five 16-column MFMA blocks in the projection) and 64 queries per
    batch (one 64-query projection tile).  Grid 255 x 7 x 9 with 2x2x2 blocks, mu
    log-uniform in [0.1, 10].
      * FP64 preconditioner, a fixed 30 iterations: every query's iterate within 1e-10
        of the oracle's;
      * FP32 preconditioner to 1e-10, with the snapshot basis (literal beta) and with a
        random orthonormal basis (flexible beta: with the literal one RBCG stagnates on a
        random basis, in the oracle too), a few hundred iterations each: every query
        converges, and sampled solutions differ from the oracle's FP64 solutions by at
        most 2 kappa 1e-10 (the measured difference is printed)."""
    import scipy.sparse.linalg as spla
    from workloads import log_uniform_mu, random_orthonormal
    dims, blocks = (255, 7, 9), (2, 2, 2)
    op = BlockDiffusion(dims, blocks)
    prob = lib.Problem(ctx, dims, blocks)
    # 80 exact solutions (sparse direct solves) at seeded parameters, orthonormalised
    mus = log_uniform_mu(1105, 80, op.Q, 0.1, 10.0)
    X = np.column_stack([spla.spsolve(op.assemble(m).tocsc(), op.rhs()) for m in mus])
    W_snap, _ = np.linalg.qr(X)
    W_rand = random_orthonormal(1106, op.N, 80)
    test = log_uniform_mu(2105, 64, op.Q, 0.1, 10.0)
    for name, W, flex in (("snapshots", W_snap, False), ("random", W_rand, True)):
        AN, _ = orb.reduced_operators(op.A_q, [op.rhs()], W)
        basis = lib.Basis.from_host(ctx, prob, W.T)
        if name == "snapshots":
            k = 30
            xk, sk = lib.solve_batch(ctx, prob, basis, test, fixed_iters=k, stencil="zmarch")
            xk = xk.cpu().numpy()
            worst = 0.0
            for b in range(len(test)):
                rk = orb.solve_rbcg(op, test[b], W, AN, fixed_iters=k)
                worst = max(worst, _rel(xk[b], rk.x))
                assert sk.iters[b] == k and _rel(xk[b], rk.x) <= 1e-10, (b, _rel(xk[b], rk.x))
            print(f"255x7x9 n=80 B=64 FP64, {k} iterations: largest difference {worst:.2e}")
        x, st = lib.solve_batch(ctx, prob, basis, test, prec="fp32", stencil="zmarch",
                                maxit=5000, flexible=flex)
        x = x.cpu().numpy()
        assert (st.status == lib.RB_OK).all() and st.rel_res_true.max() <= 1e-10
        errs = []
        for b in (0, 17, 63):
            ref = orb.solve_rbcg(op, test[b], W, AN, maxit=5000, flexible=flex)
            assert ref.converged
            errs.append(_rel(x[b], ref.x))
            assert errs[-1] <= 2 * _kappa_bound(dims, test[b]) * 1e-10, (b, errs[-1])
        print(f"255x7x9 n=80 B=64 FP32 ({name} basis): iterations {st.iters.min()}.."
              f"{st.iters.max()}, difference from the FP64 oracle {max(errs):.2e}")


@pytest.mark.parametrize("sweeps", [4, 8])
def test_uneven_configuration(lib, ctx, sweeps):
    """The uneven batch's four grids (63^2, 255^2, 1023^2 with 4x4 kappa blocks, 63^3 with
    2x2x2; mu log-uniform in [0.01, 100]) and basis sizes 10, 20, 40, 60 mixed in one call
    with the benchmark's options (FP32 preconditioner with four or eight Gauss-Seidel
    sweeps, flexible beta, HIP graphs, floor_factor 16, 1e-9 on 1023^2), 256 of its 1024
    queries:
    every query meets its tolerance or is accepted at the rounding level within 2x the
    residual of its exact solution rounded to doubles, and sampled queries on the 63^2 and
    63^3 grids match the oracle's RBCG with the same leading basis vectors (solutions
    within 2 kappa rtol of each other)."""
    import torch
    from workloads import UNEVEN_GRIDS, uneven_batch
    probs, bases = [], []
    for wk in UNEVEN_GRIDS:
        pr = lib.Problem(ctx, wk.dims, wk.blocks)
        tr = wk.train_mu()
        b, _ = lib.offline_build(ctx, pr, tr, mu=tr, n_max=60, indicator="l1",
                                 snapshot_maxit=100000, snapshot_rtol=wk.rtol)
        probs.append(pr)
        bases.append(b)
    qs = uneven_batch(count=256)
    xs = [torch.empty(UNEVEN_GRIDS[g].N, dtype=torch.float64, device="cuda") for g, _, _ in qs]
    queries = [(g, nu, mu, None, x, UNEVEN_GRIDS[g].rtol) for (g, nu, mu), x in zip(qs, xs)]
    opts = lib.solve_opts(prec="fp32", flexible=True, graph=True, maxit=10000, floor_factor=16.0,
                          sweeps=sweeps)
    st = lib.solve_multi(ctx, probs, bases, queries, opts=opts)
    tol = np.array([UNEVEN_GRIDS[g].rtol for g, _, _ in qs])
    assert (st.status == lib.RB_OK).all()
    assert ((st.rel_res_true <= tol) | (st.at_floor == 1)).all()
    # a query accepted above its tolerance (rounding-level test) must sit at what FP64 can
    # reach for it: within 2x the FP64-evaluated residual of its exact solution rounded to
    # doubles (the oracle's refined direct solve)
    above = np.flatnonzero(st.rel_res_true > tol)
    assert len(above) <= 4, above
    for k in above:
        g = qs[k][0]
        exact, fp64, _ = orb.residual_floor(BlockDiffusion(UNEVEN_GRIDS[g].dims,
                                                           UNEVEN_GRIDS[g].blocks), qs[k][2])
        print(f"query {k} ({UNEVEN_GRIDS[g].name}): true residual {st.rel_res_true[k]:.2e}, "
              f"tolerance {tol[k]:.0e}, FP64 floor {fp64:.2e} (exact evaluation {exact:.2e})")
        assert st.rel_res_true[k] <= 2.0 * fp64
    # sampled queries of the small grids against the oracle (same basis, same n_use)
    names = [wk.name for wk in UNEVEN_GRIDS]
    want = [("u2d63", 10), ("u2d63", 60), ("u3d63", 60)]
    picked = [next(k for k, (g, nu, _) in enumerate(qs) if (names[g], nu) == c) for c in want]
    for k in picked:
        g, nu, _ = qs[k]
        wk = UNEVEN_GRIDS[g]
        op = BlockDiffusion(wk.dims, wk.blocks)
        Wn, AN, fN = bases[g].info()
        W = np.ascontiguousarray(Wn[:nu].T)
        ref = orb.solve_rbcg(op, qs[k][2], W, AN[:, :nu, :nu], flexible=True, rtol=wk.rtol,
                             maxit=10000, sweeps=sweeps)
        assert ref.converged
        assert _rel(xs[k].cpu().numpy(), ref.x) <= 2 * _kappa_bound(wk.dims, qs[k][2]) * wk.rtol
