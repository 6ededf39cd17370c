"""Affine block-diffusion operator, oracle side (test infrastructure only).

The paper's problem statement is the parametrized SPD system A(mu) x = f(mu) (eq. 1)
with affine dependence A(mu) = sum_q Theta_q(mu) A_q, f(mu) = sum_r Phi_r(mu) f_r
(eq. 12, Sec. 2.3).  The workloads are finite-difference discretisations of
-div(kappa grad u) = 1 on the unit square/cube with u = 0 on the boundary and a
conductivity kappa that is constant (= mu_q) on each of Q rectangular blocks.

Discretisation (the reading used throughout, since the paper's own cases use P1 FEM):
interior nodes i = 1..n per axis, h = 1/(n+1).  For an interior node p,

    (A u)_p = sum over the 2d faces f of p:  h_a^-2 * c_f * (u_p - u_nb)

where u_nb = 0 for a boundary neighbour and c_f is the mean of kappa over the face's
dual cell (the (d-1)-box of side h centred on the face midpoint, orthogonal to the
face normal).  Block interfaces lie on grid nodes ((n+1)/b is an integer), so the
dual cell of a face is either inside one block or split 1/2 : 1/2 (1/4 at 3D edges)
between blocks along the tangential axes.  c_f is linear in kappa, hence
A(mu) = sum_q mu_q A_q exactly with A_q the operator for kappa = indicator of block q.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class BlockDiffusion:
    def __init__(self, dims, blocks):
        self.dims = tuple(int(v) for v in dims)
        self.blocks = tuple(int(v) for v in blocks)
        if len(self.dims) != len(self.blocks) or not 1 <= len(self.dims) <= 3:
            raise ValueError("dims and blocks must have the same length 1..3")
        for n, b in zip(self.dims, self.blocks):
            if n < 1 or b < 1 or (n + 1) % b != 0:
                raise ValueError("(n+1) must be divisible by the block count on every axis")
        self.dim = len(self.dims)
        self.h = tuple(1.0 / (n + 1) for n in self.dims)
        self.N = int(np.prod(self.dims))
        self.Q = int(np.prod(self.blocks))
        self._A_q = None

    @property
    def A_q(self):
        """The sparse terms A_q, built on first use (large grids may need only apply())."""
        if self._A_q is None:
            self._A_q = [self._term(q) for q in range(self.Q)]
        return self._A_q

    # --- geometry -------------------------------------------------------------
    def block_coords(self, q):
        """Block multi-index (per axis, x first) of block number q (x fastest)."""
        out = []
        for b in self.blocks:
            out.append(q % b)
            q //= b
        return tuple(out)

    def _normal_weight(self, axis, qa):
        """Weight (0/1) of block index qa for the faces between nodes I, I+1 (I=0..n)."""
        n, b = self.dims[axis], self.blocks[axis]
        m = (n + 1) // b
        I = np.arange(n + 1)
        # the face midpoint (I + 1/2) h lies in block floor((I + 1/2) / m)
        return (np.floor((I + 0.5) / m).astype(int) == qa).astype(np.float64)

    def _tangential_weight(self, axis, qa):
        """Fraction of node J's dual interval [x_J - h/2, x_J + h/2] (J=1..n) in block qa."""
        n, b = self.dims[axis], self.blocks[axis]
        m = (n + 1) // b
        J = np.arange(1, n + 1)
        lo = (J - 0.5) / m  # interval ends in units of the block width
        hi = (J + 0.5) / m
        # length of [lo, hi] intersected with [qa, qa + 1], the interval has length 1/m
        inter = np.clip(np.minimum(hi, qa + 1) - np.maximum(lo, qa), 0.0, None)
        return inter * m

    def _term(self, q):
        """Sparse A_q: the operator with kappa = 1 on block q and 0 elsewhere."""
        qc = self.block_coords(q)
        rows, cols, vals = [], [], []
        shape_rev = self.dims[::-1]  # numpy C-order: last axis = x
        lex = np.arange(self.N).reshape(shape_rev)
        for a in range(self.dim):
            n = self.dims[a]
            # face coefficients: faces I=0..n along axis a, nodes along the other axes
            w = [None] * self.dim
            for t in range(self.dim):
                w[t] = (self._normal_weight(t, qc[t]) if t == a
                        else self._tangential_weight(t, qc[t]))
            coef = w[0]
            for t in range(1, self.dim):
                coef = np.multiply.outer(w[t], coef)  # result axes: (.., y, x) order
            coef = coef * (1.0 / self.h[a] ** 2)
            ax = self.dim - 1 - a  # numpy axis of physical axis a
            # face between interior (0-based) i-1 and i  <->  I = i  (I = 0..n)
            for I in range(n + 1):
                c = np.take(coef, I, axis=ax)
                lo_i, hi_i = I - 1, I  # 0-based interior indices of the two nodes
                if 0 <= lo_i:
                    p = np.take(lex, lo_i, axis=ax).ravel()
                    rows.append(p); cols.append(p); vals.append(c.ravel())
                if hi_i <= n - 1:
                    p = np.take(lex, hi_i, axis=ax).ravel()
                    rows.append(p); cols.append(p); vals.append(c.ravel())
                if 0 <= lo_i and hi_i <= n - 1:
                    p = np.take(lex, lo_i, axis=ax).ravel()
                    s = np.take(lex, hi_i, axis=ax).ravel()
                    rows.append(p); cols.append(s); vals.append(-c.ravel())
                    rows.append(s); cols.append(p); vals.append(-c.ravel())
        r = np.concatenate(rows); c = np.concatenate(cols); v = np.concatenate(vals)
        keep = v != 0.0
        return sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=(self.N, self.N))

    # --- affine evaluation (eq. 12) ---------------------------------------------
    def assemble(self, theta):
        """A(theta) = sum_q theta_q A_q as a sparse CSR matrix."""
        theta = np.asarray(theta, dtype=np.float64)
        A = theta[0] * self.A_q[0]
        for q in range(1, self.Q):
            A = A + theta[q] * self.A_q[q]
        return A.tocsr()

    def apply(self, theta, u):
        """A(theta) u without a matrix: the same face sum, axis by axis.  The face
        coefficients are sum_q theta_q h_a^-2 (block-q weight of the face), the flux
        through face I along axis a is c_I (u_I - u_{I-1}) with u = 0 beyond the
        boundary, and node i receives flux(i) - flux(i + 1)."""
        theta = np.asarray(theta, dtype=np.float64)
        shape = self.dims[::-1]  # numpy C-order: last axis = x
        U = np.asarray(u, dtype=np.float64).reshape(shape)
        out = np.zeros(shape)
        for a in range(self.dim):
            ax = self.dim - 1 - a
            C = 0.0
            for q in range(self.Q):
                qc = self.block_coords(q)
                w = None
                for t in range(self.dim):
                    wt = (self._normal_weight(t, qc[t]) if t == a
                          else self._tangential_weight(t, qc[t]))
                    w = wt if w is None else np.multiply.outer(wt, w)  # (.., y, x) order
                C = C + theta[q] * w
            C = C * (1.0 / self.h[a] ** 2)
            pad = [(0, 0)] * self.dim
            pad[ax] = (1, 1)
            flux = C * np.diff(np.pad(U, pad), axis=ax)  # faces I = 0..n
            out -= np.diff(flux, axis=ax)
        return out.ravel()

    def rhs(self):
        """f = 1 (R = 1, Phi_1 = 1)."""
        return np.ones(self.N)

    def colors(self):
        """Red-black colour (i + j + k) mod 2 of every node, 0-based indices, lex order."""
        idx = np.indices(self.dims[::-1]).reshape(self.dim, -1)
        return (idx.sum(axis=0) % 2).astype(np.int8)


class SparseAffine:
    """A general affine sparse problem (eq. 12, Sec. 2.3) given by its terms: the CSR
    arrays of the union pattern (rowptr [N+1], col [nnz]) and the values of every term
    on it (vals [Q][nnz]); right-hand-side terms f_r (R x N, default one term f = 1).

    Gauss-Seidel colouring (the smoother reading for sparse input): greedy first fit in
    natural row order on the symmetrised pattern without the diagonal, i.e. unknown i
    gets the smallest colour not taken by a neighbour j < i.  On the 5/7-point grids this
    is exactly the red-black colouring.
    """

    def __init__(self, rowptr, col, vals, f_r=None):
        rowptr = np.asarray(rowptr, dtype=np.int64)
        col = np.asarray(col, dtype=np.int64)
        vals = np.atleast_2d(np.asarray(vals, dtype=np.float64))
        self.N = len(rowptr) - 1
        self.Q = vals.shape[0]
        self.A_q = [sp.csr_matrix((vals[q], col, rowptr), shape=(self.N, self.N))
                    for q in range(self.Q)]
        self.f_r = (np.ones((1, self.N)) if f_r is None
                    else np.atleast_2d(np.asarray(f_r, dtype=np.float64)))
        self.R = self.f_r.shape[0]
        self._pattern = sp.csr_matrix((np.ones(len(col)), col, rowptr), shape=(self.N, self.N))

    def assemble(self, theta):
        theta = np.asarray(theta, dtype=np.float64)
        A = theta[0] * self.A_q[0]
        for q in range(1, self.Q):
            A = A + theta[q] * self.A_q[q]
        return A.tocsr()

    def rhs(self, phi=None):
        """f = sum_r phi_r f_r (phi = 1 for every term if not given)."""
        phi = np.ones(self.R) if phi is None else np.asarray(phi, dtype=np.float64)
        return phi @ self.f_r

    def colors(self):
        S = (self._pattern + self._pattern.T).tocsr()
        color = np.full(self.N, -1, dtype=np.int64)
        for i in range(self.N):
            nb = S.indices[S.indptr[i]:S.indptr[i + 1]]
            used = {int(color[j]) for j in nb if j < i}
            c = 0
            while c in used:
                c += 1
            color[i] = c
        return color
