"""Piecewise-linear finite-element systems of the paper's Sec. 5 (Table 1) as affine
sparse inputs: A(mu) = sum_q Theta_q(mu) A_q, b(mu) = sum_r Phi_r(mu) b_r.

This is problem generation, not the reduced-basis method: both the GPU library (through
rb_problem_create_csr) and the CPU oracle receive exactly the matrices built here.

Mesh: the unit square / cube with n interior nodes per axis (h = 1 / (n + 1)); every
square is cut into two triangles along the (+1, +1) diagonal, every cube into the six
tetrahedra of the Kuhn (Freudenthal) split around its main diagonal.  Unknowns are the
interior nodes in lexicographic order (x fastest); boundary nodes carry the Dirichlet
data, eliminated by lifting.  Element integrals use the centroid rule:
  stiffness  K_ij = sum_T w(x_T) |T| grad(phi_i) . grad(phi_j)
  load       F_i  = sum_T f(x_T) |T| / (d + 1)

Equation (R15 reading of the garbled sign): -div(kappa grad u) = f with
f = d pi^2 prod sin(pi x_a), so that u = prod sin(pi x_a) for kappa = 1.

Case 1: kappa = 1 + mu g1(x), g1 = |x - 1/2|^2, u = 0 on the boundary, mu in [0, 1]:
  Q = 2, Theta = (1, mu); R = 1.
Case 2: kappa = 1 + mu_1 g2(x), g2 = sin(20 pi (4 (x - 1/2)^2 + sum_{a>0} (x_a - 1/2)^2))^2,
  u = g_D = (1 - mu_2) c1 + mu_2 c2 on the boundary with
  c1 = cos(10 pi (4 (x - 1/2)^2 + sum_{a>0} (x_a - 1/2)^2)), c2 = cos(10 pi sum_a x_a),
  (mu_1, mu_2) in [0, 2] x [0, 1].  Lifting gives b = F - A_IB(mu_1) g_B(mu_2), which is
  affine with R = 4: Phi = (1, mu_2, mu_1, mu_1 mu_2) and
  b_r = (F - K1 c1, K1 (c1 - c2), -K2 c1, K2 (c1 - c2)) with K_q = A_q[interior, boundary].
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import permutations

import numpy as np
import scipy.sparse as sp


@dataclass
class AffineSystem:
    dims: tuple           # interior nodes per axis
    A_q: list             # Q scipy CSR matrices (N x N, interior unknowns)
    b_r: np.ndarray       # R x N
    case: int

    @property
    def N(self):
        return self.A_q[0].shape[0]

    @property
    def Q(self):
        return len(self.A_q)

    @property
    def R(self):
        return self.b_r.shape[0]

    def theta(self, mu):
        mu = np.atleast_2d(mu)
        if self.case == 0:
            return np.ascontiguousarray(mu, dtype=np.float64)
        return np.column_stack([np.ones(len(mu)), mu[:, 0]])

    def phi(self, mu):
        mu = np.atleast_2d(mu)
        if self.case in (0, 1):
            return np.ones((len(mu), 1))
        m1, m2 = mu[:, 0], mu[:, 1]
        return np.column_stack([np.ones(len(mu)), m2, m1, m1 * m2])

    def draw_mu(self, seed, M):
        rng = np.random.default_rng(seed)
        if self.case == 0:
            return 10.0 ** rng.uniform(-1.0, 1.0, size=(M, self.Q))
        if self.case == 1:
            return rng.uniform(0.0, 1.0, size=(M, 1))
        return np.column_stack([rng.uniform(0.0, 2.0, M), rng.uniform(0.0, 1.0, M)])


def _simplices(d):
    """Reference simplices of the unit square / cube as lists of corner offsets."""
    if d == 2:
        return [[(0, 0), (1, 0), (1, 1)], [(0, 0), (0, 1), (1, 1)]]
    out = []
    for perm in permutations(range(3)):
        path = [(0, 0, 0)]
        cur = [0, 0, 0]
        for a in perm:
            cur = cur.copy()
            cur[a] = 1
            path.append(tuple(cur))
        out.append(path)
    return out


def _g1(x):
    return ((x - 0.5) ** 2).sum(axis=-1)


def _radial4(x):
    return 4.0 * (x[..., 0] - 0.5) ** 2 + ((x[..., 1:] - 0.5) ** 2).sum(axis=-1)


def _g2(x):
    return np.sin(20.0 * np.pi * _radial4(x)) ** 2


def _c1(x):
    return np.cos(10.0 * np.pi * _radial4(x))


def _c2(x):
    return np.cos(10.0 * np.pi * x.sum(axis=-1))


def build(case: int, n: int, d: int = 3) -> AffineSystem:
    """P1 system of Table 1, case 1 or 2, with n interior nodes per axis in d dims."""
    m = n + 2                        # nodes per axis including the boundary
    h = 1.0 / (n + 1)
    grid = np.stack(np.meshgrid(*([np.arange(m)] * d), indexing="ij"), axis=-1)
    grid = grid.reshape(-1, d)[:, ::-1]          # rows: (i_x, i_y[, i_z]), x fastest
    strides = m ** np.arange(d)
    coords = grid * h
    interior = np.all((grid > 0) & (grid < m - 1), axis=1)
    unk = -np.ones(len(grid), dtype=np.int64)
    unk[interior] = np.arange(interior.sum())
    # all cells: lower-corner index vectors
    cells = np.stack(np.meshgrid(*([np.arange(m - 1)] * d), indexing="ij"), axis=-1)
    cells = cells.reshape(-1, d)
    rows, cols, v1, v2 = [], [], [], []
    F = np.zeros(len(grid))
    vol_fact = 1.0 / (2.0 if d == 2 else 6.0)
    for simp in _simplices(d):
        corners = [cells + np.array(off) for off in simp]          # (d+1) x ncell x d
        ids = np.stack([(c * strides).sum(axis=1) for c in corners], axis=1)
        X = coords[ids]                                             # ncell x (d+1) x d
        E = X[:, 1:, :] - X[:, :1, :]                               # edge matrix
        det = np.linalg.det(E)
        vol = np.abs(det) * vol_fact
        # gradients of the barycentric functions: G = [-1..; I] E^-T
        Einv = np.linalg.inv(E)                                     # ncell x d x d
        G = np.concatenate([-Einv.sum(axis=2, keepdims=True), Einv], axis=2)  # d x (d+1)
        G = np.transpose(G, (0, 2, 1))                              # ncell x (d+1) x d
        K = np.einsum("tia,tja->tij", G, G) * vol[:, None, None]
        xc = X.mean(axis=1)
        w2 = _g1(xc) if case == 1 else _g2(xc)
        fval = d * np.pi ** 2 * np.prod(np.sin(np.pi * xc), axis=1)
        for a in range(d + 1):
            F += np.bincount(ids[:, a], weights=fval * vol / (d + 1), minlength=len(grid))
            for b in range(d + 1):
                rows.append(ids[:, a])
                cols.append(ids[:, b])
                v1.append(K[:, a, b])
                v2.append(K[:, a, b] * w2)
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    K1 = sp.csr_matrix((np.concatenate(v1), (rows, cols)), shape=(len(grid),) * 2)
    K2 = sp.csr_matrix((np.concatenate(v2), (rows, cols)), shape=(len(grid),) * 2)
    I = np.flatnonzero(interior)
    Bn = np.flatnonzero(~interior)
    A1 = K1[I][:, I].tocsr()
    A2 = K2[I][:, I].tocsr()
    # exact symmetry (the element sums of (i, j) and (j, i) may round differently) and
    # one shared (union) pattern for both terms
    A1 = 0.5 * (A1 + A1.T)
    A2 = 0.5 * (A2 + A2.T)
    Z = (A1 + 1j * A2).tocsr()
    Z.sort_indices()
    A1 = sp.csr_matrix((Z.data.real.copy(), Z.indices.copy(), Z.indptr.copy()), shape=Z.shape)
    A2 = sp.csr_matrix((Z.data.imag.copy(), Z.indices.copy(), Z.indptr.copy()), shape=Z.shape)
    if case == 1:
        b = F[I][None, :]
    else:
        xb = coords[Bn]
        c1, c2 = _c1(xb), _c2(xb)
        K1b = K1[I][:, Bn]
        K2b = K2[I][:, Bn]
        b = np.stack([F[I] - K1b @ c1, K1b @ (c1 - c2), -(K2b @ c1), K2b @ (c1 - c2)])
    return AffineSystem(tuple([n] * d), [A1, A2], np.ascontiguousarray(b), case)


def csr_arrays(sys: AffineSystem):
    """(rowptr int64 [N+1], col int32 [nnz], vals [Q][nnz]) on the shared pattern."""
    A1 = sys.A_q[0]
    vals = []
    for A in sys.A_q:
        assert A.indptr.tolist() == A1.indptr.tolist() and np.array_equal(A.indices, A1.indices)
        vals.append(A.data)
    return (A1.indptr.astype(np.int64), A1.indices.astype(np.int32),
            np.ascontiguousarray(np.stack(vals)))


def random_system(seed: int, N: int, deg: int = 6, Q: int = 3) -> AffineSystem:
    """A random sparse SPD affine system (case 0): every term is a weighted graph
    Laplacian on a random symmetric pattern (a ring plus about deg random neighbours per
    node, each term weighting its own random subset of the edges) plus a positive diagonal
    shift, so A(theta) is SPD for theta > 0; b = 1 (R = 1).  Its colouring needs more
    than two colours."""
    rng = np.random.default_rng(seed)
    i = np.arange(N)
    src = [i]
    dst = [(i + 1) % N]
    extra = rng.integers(0, N, size=(N, deg // 2))
    src.append(np.repeat(i, deg // 2))
    dst.append(extra.ravel())
    src, dst = np.concatenate(src), np.concatenate(dst)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    edges = np.unique(lo * N + hi)
    a, b = edges // N, edges % N
    mats = []
    for q in range(Q):
        w = rng.uniform(0.1, 1.0, size=len(a)) * (rng.uniform(size=len(a)) < 0.7)
        L = sp.coo_matrix((np.concatenate([-w, -w]), (np.concatenate([a, b]),
                                                     np.concatenate([b, a]))), shape=(N, N))
        L = L.tocsr()
        L = L - sp.diags(np.asarray(L.sum(axis=1)).ravel())
        mats.append(L + sp.diags(rng.uniform(0.05, 0.2, size=N)))
    # one shared pattern: the union of the terms' patterns (zeros kept where a term
    # has no entry)
    U = sp.identity(N, format="csr")
    for A in mats:
        U = U + abs(A)
    U = U.tocsr()
    U.sort_indices()
    r = np.repeat(np.arange(N), np.diff(U.indptr))
    A_q = [sp.csr_matrix((np.asarray(A.tocsr()[r, U.indices]).ravel(), U.indices.copy(),
                          U.indptr.copy()), shape=(N, N)) for A in mats]
    return AffineSystem((N,), A_q, np.ones((1, N)), 0)
