"""The allocation-free reduced factorisation (rb_reduced_factor_batch_noalloc) against
rb_reduced_factor_batch, through the C ABI: the same kernel on the same inputs, so the
factors and statuses must agree bit for bit, on two calls in a row (the second smaller,
so stale contents of the shared fixed buffer would show), and sizes beyond the buffer
are refused before any work."""
import numpy as np
import pytest

from workloads import log_uniform_mu, random_orthonormal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def _basis(lib, ctx, dims, blocks, n, seed):
    prob = lib.Problem(ctx, dims, blocks)
    W = random_orthonormal(seed, prob.N, n)
    return prob, lib.Basis.from_host(ctx, prob, W.T)


def test_noalloc_factor_equals_allocating_call(lib, ctx):
    prob1, b1 = _basis(lib, ctx, (31, 31), (2, 2), 40, 3)
    prob2, b2 = _basis(lib, ctx, (15, 15, 15), (2, 2, 2), 12, 4)
    cases = [(b1, log_uniform_mu(41, 300, 4, 0.1, 10.0)),    # first call: 300 queries, n = 40
             (b2, log_uniform_mu(42, 7, 8, 0.1, 10.0))]      # second: 7 queries, n = 12
    # one query whose reduced matrix is not SPD (a negative coefficient dominating)
    cases[1][1][3] = [-50.0, 1, 1, 1, 1, 1, 1, 1]
    for basis, theta in cases:
        L_ref, st_ref = lib.reduced_factor_batch(ctx, basis, theta)
        L, st = lib.reduced_factor_batch_noalloc(ctx, basis, theta)
        print(f"B={len(theta)} n={basis.n}: statuses {np.bincount(st).tolist()}")
        assert np.array_equal(st, st_ref)
        assert np.array_equal(L, L_ref)
    assert (cases[1][1].shape[0] == 7) and st[3] == lib.RB_ENOTSPD and (st[:3] == 0).all()


def test_noalloc_refuses_sizes_beyond_the_buffer(lib, ctx):
    _, basis = _basis(lib, ctx, (31, 31), (2, 2), 40, 5)
    # 700 queries at n = 40: 700 * 1600 * 8 bytes of factors alone exceed 8 MiB
    theta = log_uniform_mu(43, 700, 4, 0.1, 10.0)
    with pytest.raises(lib.RBError) as e:
        lib.reduced_factor_batch_noalloc(ctx, basis, theta)
    assert e.value.status == lib.RB_EINVAL and "fixed buffer" in str(e.value)
    # the buffer still serves a call that fits
    L_ref, st_ref = lib.reduced_factor_batch(ctx, basis, theta[:5])
    L, st = lib.reduced_factor_batch_noalloc(ctx, basis, theta[:5])
    assert np.array_equal(L, L_ref) and np.array_equal(st, st_ref)
