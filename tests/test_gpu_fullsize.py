"""Parity at the benchmark's full size and launch configuration (3D 127^3, N = 2,048,383,
n = 40, B = 256, FP32 preconditioner, literal beta): every query reaches a true relative
residual <= 1e-10 in FP64, and sampled queries are checked one by one against the
oracle's RBCG with the same basis (same iteration count within one; solutions within
2 kappa(A) 1e-10 of each other, with kappa bounded by Gershgorin and the smallest
Dirichlet eigenvalue scaled by min(mu))."""
import math

import numpy as np
import pytest

from oracle import rb as orb
from oracle.operator import BlockDiffusion
from workloads import WORKLOADS

pytestmark = pytest.mark.gpu


def _kappa_bound(w, theta):
    # lambda_max <= Gershgorin <= max(mu) * 4 d / h^2; lambda_min >= min(mu) * the
    # smallest eigenvalue of the unit-coefficient Laplacian (sum of 4/h^2 sin^2(pi h/2))
    h = 1.0 / (w.dims[0] + 1)
    d = len(w.dims)
    lmax = max(theta) * 4.0 * d / h**2
    lmin = min(theta) * d * 4.0 / h**2 * math.sin(math.pi * h / 2) ** 2
    return lmax / lmin


def test_bench_configuration_parity(lib):
    import torch
    w = WORKLOADS["3d127"]
    ctx = lib.Context(0)
    prob = lib.Problem(ctx, w.dims, w.blocks)
    train = w.train_mu()
    basis, rep = lib.offline_build(ctx, prob, train, mu=train, n_max=w.n, indicator="residual")
    assert basis.n == w.n
    test = w.test_mu(w.B)
    x, st = lib.solve_batch(ctx, prob, basis, test, prec="fp32")
    assert (st.status == lib.RB_OK).all()
    assert st.rel_res_true.max() <= 1e-10
    op = BlockDiffusion(w.dims, w.blocks)
    Wn, AN, fN = basis.info()
    W = np.ascontiguousarray(Wn.T)
    for b in (0, 137):
        ref = orb.solve_rbcg(op, test[b], W, AN, rtol=1e-10)
        xb = x[b].cpu().numpy()
        assert ref.converged
        assert abs(int(st.iters[b]) - ref.iters) <= max(2, 0.03 * ref.iters), (st.iters[b], ref.iters)
        err = np.linalg.norm(xb - ref.x) / np.linalg.norm(ref.x)
        assert err <= 2 * _kappa_bound(w, test[b]) * 1e-10, err
        # the GPU iterate satisfies the FP64 residual check independently of the library
        r = op.rhs() - op.assemble(test[b]) @ xb
        assert np.linalg.norm(r) / np.linalg.norm(op.rhs()) <= 1.01e-10
    del x
    torch.cuda.empty_cache()
