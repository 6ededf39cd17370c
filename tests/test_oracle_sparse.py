"""The oracle's general sparse affine problem (CSR input) and the finite-element
workloads of the paper's Sec. 5, pinned against independent facts."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import rb
from oracle.operator import BlockDiffusion, SparseAffine
from workloads import fem, log_uniform_mu


def _as_sparse_affine(op):
    """The block-diffusion terms written as CSR arrays on their union pattern."""
    U = sum(abs(a) for a in op.A_q).tocsr()
    U.sort_indices()
    r = np.repeat(np.arange(op.N), np.diff(U.indptr))
    vals = np.stack([np.asarray(a.tocsr()[r, U.indices]).ravel() for a in op.A_q])
    return SparseAffine(U.indptr, U.indices, vals)


@pytest.mark.parametrize("dims,blocks", [((9, 7), (2, 2)), ((5, 7, 3), (2, 2, 2))])
def test_first_fit_colouring_of_grids_is_red_black(dims, blocks):
    op = BlockDiffusion(dims, blocks)
    assert np.array_equal(_as_sparse_affine(op).colors(), op.colors())


def test_colouring_is_proper_and_first_fit():
    s = fem.random_system(5, 400, 6, 3)
    sa = SparseAffine(*fem.csr_arrays(s))
    c = sa.colors()
    S = (sum(abs(a) for a in s.A_q) + sum(abs(a) for a in s.A_q).T).tocoo()
    off = S.row != S.col
    assert (c[S.row[off]] != c[S.col[off]]).all()        # no edge inside a class
    assert c.max() + 1 >= 3
    Sc = S.tocsr()
    for i in range(0, 400, 37):                          # smallest colour free of j < i
        nb = Sc.indices[Sc.indptr[i]:Sc.indptr[i + 1]]
        used = {c[j] for j in nb if j < i}
        assert c[i] == min(set(range(c.max() + 2)) - used)


def test_sparse_affine_reproduces_block_diffusion_solves():
    """Same matrices, same colouring: RBCG through the CSR form equals the stencil form
    to rounding (only the order of the sparse sums may differ)."""
    op = BlockDiffusion((15, 15), (2, 2))
    sa = _as_sparse_affine(op)
    W = np.linalg.qr(np.random.default_rng(3).standard_normal((op.N, 5)))[0]
    th = log_uniform_mu(4, 1, op.Q, 0.1, 10.0)[0]
    a = rb.solve_rbcg(op, th, W, fixed_iters=6)
    b = rb.solve_rbcg(sa, th, W, fixed_iters=6)
    assert np.linalg.norm(a.x - b.x) <= 1e-13 * np.linalg.norm(a.x)


def test_multicolour_gauss_seidel_is_forward_substitution():
    """One sweep over the colour classes equals y0 + (D + L)^-1 (b - A y0) in the
    class-major ordering."""
    s = fem.random_system(6, 300, 6, 3)
    sa = SparseAffine(*fem.csr_arrays(s))
    th = np.array([0.5, 2.0, 1.3])
    A = sa.assemble(th).toarray()
    c = sa.colors()
    order = np.argsort(c, kind="stable")
    P = A[np.ix_(order, order)]
    rng = np.random.default_rng(7)
    b, y0 = rng.standard_normal(300), rng.standard_normal(300)
    DL = np.tril(P)
    ref = y0[order] + np.linalg.solve(DL, b[order] - P @ y0[order])
    from oracle.smoother import Smoother
    y = Smoother(sa.assemble(th), c)(b, y0)
    assert np.abs(y[order] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("d,n", [(2, 15), (3, 7)])
def test_fem_laplacian_term_is_the_scaled_grid_laplacian(d, n):
    """P1 stiffness of kappa = 1 on these meshes is h^(d-2) times the (2d+1)-point
    stencil (2d on the diagonal, -1 to the axis neighbours): a known property of the
    right-triangle and Kuhn triangulations."""
    s = fem.build(1, n, d)
    h = 1.0 / (n + 1)
    op = BlockDiffusion(tuple([n] * d), tuple([1] * d))
    ref = op.A_q[0] * h ** 2 * h ** (d - 2)
    assert abs(s.A_q[0] - ref).max() <= 1e-12


def test_fem_case1_converges_to_the_exact_solution():
    """kappa = 1 (mu = 0): the discrete solution approaches prod sin(pi x) at O(h^2)."""
    errs = []
    for n in (7, 15):
        s = fem.build(1, n, 3)
        u = spla.spsolve(s.A_q[0].tocsc(), s.b_r[0])
        g = np.stack(np.meshgrid(*([np.arange(1, n + 1)] * 3), indexing="ij"), -1)
        g = g.reshape(-1, 3)[:, ::-1] / (n + 1)
        errs.append(np.abs(u - np.prod(np.sin(np.pi * g), axis=1)).max())
    assert errs[1] < 0.35 * errs[0] and errs[1] < 0.01


def test_fem_terms_are_symmetric_and_positive():
    for case in (1, 2):
        s = fem.build(case, 7, 3)
        for A in s.A_q:
            assert abs(A - A.T).max() == 0.0
        A = s.A_q[0] + 2.0 * s.A_q[1]            # kappa = 1 + 2 g(x) > 0
        assert spla.eigsh(A, k=1, which="SA", return_eigenvectors=False)[0] > 0
    assert fem.build(2, 7, 3).R == 4
