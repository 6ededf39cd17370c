"""Pins of the oracle's affine operator (eq. 12, Sec. 2.3) against independent facts."""
import itertools
import os

import numpy as np
import pytest
import scipy.fft
import scipy.sparse as sp

from oracle.operator import BlockDiffusion

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "operator_hand.txt")


def _golden():
    cases = {}
    for line in open(GOLDEN):
        line = line.split("#")[0].strip()
        if not line:
            continue
        c, r, k, v = line.split()
        cases.setdefault(c, []).append((int(r), int(k), float(v)))
    return cases


def test_hand_examples():
    cases = _golden()
    A1 = BlockDiffusion((3,), (2,)).assemble([1.0, 3.0]).toarray()
    for r, c, v in cases["1d"]:
        assert A1[r, c] == pytest.approx(v, abs=1e-12)
    A2 = BlockDiffusion((3, 3), (2, 2)).assemble([1.0, 2.0, 3.0, 4.0]).toarray()
    for r, c, v in cases["2d"]:
        assert A2[r, c] == pytest.approx(v, abs=1e-12)


def _laplacian_kron(dims):
    """Constant-coefficient Laplacian as a Kronecker sum of 1D second differences."""
    mats = []
    for n in dims:
        h = 1.0 / (n + 1)
        mats.append(sp.diags([-1, 2, -1], [-1, 0, 1], shape=(n, n)) / h**2)
    eye = [sp.identity(n) for n in dims]
    total = None
    for a in range(len(dims)):
        # lex order has x fastest -> kron(z, y, x)
        factors = [mats[t] if t == a else eye[t] for t in range(len(dims))][::-1]
        term = factors[0]
        for f in factors[1:]:
            term = sp.kron(term, f)
        total = term if total is None else total + term
    return total.toarray()


@pytest.mark.parametrize("dims,blocks", [((7,), (2,)), ((7, 7), (2, 2)), ((7, 5, 3), (2, 3, 2)),
                                         ((11, 11), (4, 4)), ((7, 7, 7), (2, 2, 2))])
def test_sum_of_terms_is_laplacian(dims, blocks):
    op = BlockDiffusion(dims, blocks)
    A = op.assemble(np.ones(op.Q)).toarray()
    assert np.abs(A - _laplacian_kron(dims)).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("dims,blocks", [((7, 7), (2, 2)), ((7, 5, 3), (2, 3, 2))])
def test_symmetric_and_positive(dims, blocks):
    op = BlockDiffusion(dims, blocks)
    rng = np.random.default_rng(0)
    A = op.assemble(10 ** rng.uniform(-2, 2, op.Q)).toarray()
    assert np.abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("dims", [(15, 15), (7, 9, 5), (31,)])
def test_uniform_kappa_matches_dst(dims):
    """kappa == c: A = c * Laplacian, solved exactly by the DST-I eigen-decomposition."""
    blocks = tuple(2 if (n + 1) % 2 == 0 else 1 for n in dims)
    op = BlockDiffusion(dims, blocks)
    c = 2.5
    A = op.assemble(np.full(op.Q, c))
    f = op.rhs()
    x = np.linalg.solve(A.toarray(), f)
    shape = dims[::-1]
    lam = np.zeros(shape)
    for a, n in enumerate(dims):
        h = 1.0 / (n + 1)
        k = np.arange(1, n + 1)
        ev = (4.0 / h**2) * np.sin(k * np.pi * h / 2) ** 2
        sh = [1] * len(dims)
        sh[len(dims) - 1 - a] = n
        lam = lam + ev.reshape(sh)
    fhat = scipy.fft.dstn(f.reshape(shape), type=1, norm="ortho")
    xd = scipy.fft.idstn(fhat / (c * lam), type=1, norm="ortho").ravel()
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


def _brute_force(dims, blocks, theta, sub=8):
    """Dense operator built point by point, with face coefficients from a midpoint-rule
    average of kappa over each face's dual cell (sub x sub samples, never on an interface)."""
    d = len(dims)
    h = [1.0 / (n + 1) for n in dims]

    def kappa(x):
        q = 0
        stride = 1
        for a in range(d):
            q += min(int(np.floor(x[a] * blocks[a])), blocks[a] - 1) * stride
            stride *= blocks[a]
        return theta[q]

    N = int(np.prod(dims))
    A = np.zeros((N, N))
    offs = (np.arange(sub) + 0.5) / sub - 0.5

    def lex(idx):
        L, s = 0, 1
        for a in range(d):
            L += idx[a] * s
            s *= dims[a]
        return L

    for idx in itertools.product(*[range(n) for n in dims]):
        p = lex(idx)
        for a in range(d):
            for sgn in (-1, 1):
                nb = list(idx)
                nb[a] += sgn
                # face midpoint and the mean of kappa over its dual cell
                mid = [(idx[t] + 1) * h[t] for t in range(d)]
                mid[a] += 0.5 * sgn * h[a]
                tang = [t for t in range(d) if t != a]
                vals = []
                for o in itertools.product(offs, repeat=len(tang)):
                    x = list(mid)
                    for t, ot in zip(tang, o):
                        x[t] += ot * h[t]
                    vals.append(kappa(x))
                c = np.mean(vals) / h[a] ** 2
                A[p, p] += c
                if 0 <= nb[a] < dims[a]:
                    A[p, lex(nb)] -= c
    return A


@pytest.mark.parametrize("dims,blocks", [((7, 7), (2, 2)), ((5, 7, 3), (3, 2, 2)),
                                         ((11, 3), (4, 2))])
def test_brute_force_quadrature(dims, blocks):
    op = BlockDiffusion(dims, blocks)
    rng = np.random.default_rng(1)
    theta = 10 ** rng.uniform(-1, 1, op.Q)
    A = op.assemble(theta).toarray()
    Ab = _brute_force(dims, blocks, theta)
    assert np.abs(A - Ab).max() <= 1e-12 * np.abs(Ab).max()


def test_rejects_misaligned_blocks():
    with pytest.raises(ValueError):
        BlockDiffusion((6, 7), (2, 2))


@pytest.mark.parametrize("dims,blocks", [((31,), (4,)), ((15, 15), (2, 2)), ((7, 11), (4, 3)),
                                         ((7, 9, 5), (2, 2, 3)), ((5, 3, 7), (3, 2, 4))])
def test_matrix_free_apply_equals_assembly(dims, blocks):
    """The matrix-free apply (face fluxes) and the assembled sparse sum of the terms are
    two routes to the same operator; the sparse one is pinned by the hand examples, the
    Kronecker Laplacian and the DST solution above."""
    op = BlockDiffusion(dims, blocks)
    rng = np.random.default_rng(5)
    for _ in range(3):
        theta = 10.0 ** rng.uniform(-2, 2, op.Q)
        u = rng.standard_normal(op.N)
        A = op.assemble(theta)
        ref = A @ u
        scale = abs(A) @ np.abs(u)
        assert np.max(np.abs(op.apply(theta, u) - ref) / scale) <= 1e-14


SMOOTHER_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "smoother_hand.txt")


def test_smoothers_match_hand_derived_steps():
    """Jacobi (omega = 2/3), red-black Gauss-Seidel and its symmetric form on the 1D
    three-node case, against steps worked out by hand (tests/golden/smoother_hand.txt)."""
    from fractions import Fraction

    from oracle.smoother import Smoother

    op = BlockDiffusion((3,), (2,))
    A = op.assemble(np.array([1.0, 3.0]))
    b = np.ones(3)
    rows = []
    with open(SMOOTHER_GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                kind, step, *vals = line.split()
                rows.append((kind, int(step), [float(Fraction(v)) for v in vals]))
    assert {r[0] for r in rows} == {"jacobi", "rbgs", "rbgs_sym"}
    for kind, step, want in rows:
        S = Smoother(A, op.colors(), kind)
        y = np.zeros(3)
        for _ in range(step):
            y = S(b, y)
        assert np.allclose(y, want, rtol=1e-14, atol=0), (kind, step, y, want)
