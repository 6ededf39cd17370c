"""Seeded synthetic inputs shared by the GPU library's tests/bench and the CPU oracle.

This module holds no arithmetic of the reduced-basis method itself: it only draws
parameter vectors and random test data and names the workload shapes.  Both sides
(the HIP path and the oracle) receive exactly the arrays produced here.

Parameters follow the affine form of eq. (12) of the paper (Sec. 2.3): the caller
evaluates Theta_q(mu) on the host.  For the diffusion workloads here the block
conductivities are the parameters themselves, Theta_q(mu) = mu_q (Q = P), and the
right-hand side is f = 1 (R = 1, Phi_1 = 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np


def log_uniform_mu(seed: int, M: int, P: int, lo: float, hi: float) -> np.ndarray:
    """M parameter vectors of length P, each entry log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=(M, P))


def theta_of_mu(mu: np.ndarray) -> np.ndarray:
    """Theta_q(mu) for the block-diffusion workloads: the identity map (Q = P)."""
    return np.ascontiguousarray(mu, dtype=np.float64)


def random_vectors(seed: int, B: int, N: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal((B, N))


def random_orthonormal(seed: int, N: int, n: int) -> np.ndarray:
    """An N x n matrix with orthonormal columns (Q factor of a Gaussian matrix)."""
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((N, n)))
    return q


def sine_basis(dims, n):
    """The n discrete sine modes prod_a sqrt(2/(m_a+1)) sin(i_a pi j_a / (m_a+1)) with the
    smallest sum of squared mode numbers (ties by mode numbers), as rows of length N in
    natural order (x fastest); orthonormal on the grid.  A basis that no solver produced,
    for tests at sizes where the reference solver cannot build one."""
    import math
    d = len(dims)
    rng = range(1, 9)
    if d == 2:
        modes = sorted((i * i + j * j, i, j, 1) for i in rng for j in rng)[:n]
    else:
        modes = sorted((i * i + j * j + k * k, i, j, k) for i in rng for j in rng
                       for k in rng)[:n]

    def s(m, i):
        return math.sqrt(2.0 / (m + 1)) * np.sin(i * math.pi * np.arange(1, m + 1) / (m + 1))

    nx, ny = dims[0], dims[1]
    nz = dims[2] if d == 3 else 1
    W = np.empty((n, nx * ny * nz))
    for c, (_, i, j, k) in enumerate(modes):
        sz = s(nz, k) if d == 3 else np.ones(1)
        W[c] = np.multiply.outer(sz, np.multiply.outer(s(ny, j), s(nx, i))).ravel()
    return W


@dataclass(frozen=True)
class Workload:
    name: str
    dims: Tuple[int, ...]          # interior points per axis (x fastest)
    blocks: Tuple[int, ...]        # kappa blocks per axis; Q = prod(blocks)
    mu_range: Tuple[float, float]  # log-uniform range of every mu_q
    n: int                         # reduced-basis size used online
    M_train: int                   # training-set size for the greedy
    B: int                         # queries per launch
    seed_train: int
    seed_test: int
    note: str = ""
    rtol: float = 1e-10            # target true relative residual of the solves

    @property
    def N(self) -> int:
        return int(np.prod(self.dims))

    @property
    def Q(self) -> int:
        return int(np.prod(self.blocks))

    def train_mu(self) -> np.ndarray:
        return log_uniform_mu(self.seed_train, self.M_train, self.Q, *self.mu_range)

    def test_mu(self, count: int | None = None) -> np.ndarray:
        return log_uniform_mu(self.seed_test, self.B if count is None else count,
                              self.Q, *self.mu_range)


# The synthetic diffusion workloads (finite-difference stand-ins for the paper's
# FEM Poisson cases of Sec. 5; the paper's meshes and iFEM are not used).
WORKLOADS = {
    "2d63": Workload("2d63", (63, 63), (2, 2), (0.1, 10.0), 20, 256, 16, 1001, 2001,
                     "2D 5-point, 63x63 interior, kappa on 2x2 blocks, FP64 RB-PCG"),
    "3d127": Workload("3d127", (127, 127, 127), (2, 2, 2), (0.1, 10.0), 40, 256, 256, 1002, 2002,
                      "3D 7-point, 127^3 interior, kappa on 2x2x2 octants, mixed precision"),
    "3d63": Workload("3d63", (63, 63, 63), (2, 2, 2), (0.1, 10.0), 60, 10000, 64, 1004, 2004,
                     "3D 7-point, 63^3 interior, learned greedy over 1e4 mu"),
    "3d255": Workload("3d255", (255, 255, 255), (2, 2, 2), (0.1, 10.0), 80, 256, 64, 1005, 2005,
                      "3D 7-point, 255^3 interior, HBM-bound large case"),
}

# Uneven batch: grids mixed within one call.  On 1023^2 with a kappa contrast of 1e4
# the FP64 residual of the exact solution rounded to doubles is already 3e-11..1e-10
# (eps * || |A| |x| || / ||f||; measured by sparse direct solves on 511^2 and scaled by
# the h^-2 growth), so 1e-10 is at the rounding floor there and that grid targets 1e-9.
UNEVEN_GRIDS = (
    Workload("u2d63", (63, 63), (4, 4), (0.01, 100.0), 60, 256, 256, 1003, 2003),
    Workload("u2d255", (255, 255), (4, 4), (0.01, 100.0), 60, 256, 256, 1003, 2003),
    Workload("u2d1023", (1023, 1023), (4, 4), (0.01, 100.0), 60, 256, 256, 1003, 2003,
             rtol=1e-9),
    Workload("u3d63", (63, 63, 63), (2, 2, 2), (0.01, 100.0), 60, 256, 256, 1003, 2003),
)
UNEVEN_N_CHOICES = (10, 20, 40, 60)


def uneven_batch(seed: int = 2003, count: int = 1024):
    """(grid index, n_use, mu) for each query of the uneven batch, shuffled."""
    rng = np.random.default_rng(seed)
    grid = rng.integers(0, len(UNEVEN_GRIDS), size=count)
    nsel = rng.integers(0, len(UNEVEN_N_CHOICES), size=count)
    out = []
    for g, s in zip(grid, nsel):
        w = UNEVEN_GRIDS[int(g)]
        mu = 10.0 ** rng.uniform(np.log10(w.mu_range[0]), np.log10(w.mu_range[1]), size=w.Q)
        out.append((int(g), UNEVEN_N_CHOICES[int(s)], mu))
    return out
