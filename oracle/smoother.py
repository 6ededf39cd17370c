"""Smoothers S(A, b, y) of the RB iteration, oracle side (test infrastructure only).

The paper defines z = S(A, b, y) as a smoother (Jacobi or Gauss-Seidel) that iterates
on A x = b starting from y and returns z (Sec. 3.1, the post-smoothing step eq. 8),
and uses Gauss-Seidel for all methods (Sec. 3.3).  It fixes neither the ordering nor
the number of sweeps; the reading here is one forward red-black Gauss-Seidel sweep,
red (colour (i+j+k) mod 2 == 0) first.  Because red nodes couple only to black nodes
in the 5/7-point stencil, updating all red nodes at once is exactly Gauss-Seidel in
the red-first ordering.

Other modes: symmetric red-black GS (forward sweep then backward sweep), damped
Jacobi (omega = 2/3) and "none" (z = y, used for Lemma 2 of Sec. 3.2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

RBGS, RBGS_SYM, JACOBI, NONE = "rbgs", "rbgs_sym", "jacobi", "none"


class Smoother:
    """colors: colour class of every unknown (0 .. C-1) such that no two unknowns of one
    class are coupled; one forward sweep updates the classes in increasing order, each
    class from the latest values of all the others (Gauss-Seidel in the class-major
    ordering).  The stencil problems use the red-black colouring (C = 2); general
    sparse problems a greedy colouring."""

    def __init__(self, A, colors, kind=RBGS, omega=2.0 / 3.0, sweeps=1):
        """sweeps: how many times the sweep (forward, or forward then backward for the
        symmetric kind) is applied per smoother application."""
        self.kind = kind
        self.sweeps = int(sweeps)
        self.A = sp.csr_matrix(A)
        self.D = self.A.diagonal()
        colors = np.asarray(colors)
        ncol = int(colors.max()) + 1 if colors.size else 0
        self.sets = [np.flatnonzero(colors == c) for c in range(ncol)]
        self.rest = [np.flatnonzero(colors != c) for c in range(ncol)]
        self.blocks = [self.A[S][:, O] for S, O in zip(self.sets, self.rest)]
        self.omega = omega

    def _sweep(self, c, b, y):
        # y_c <- D_c^-1 (b_c - A_{c,rest} y_rest)
        S = self.sets[c]
        y[S] = (b[S] - self.blocks[c] @ y[self.rest[c]]) / self.D[S]

    def __call__(self, b, y0):
        y = np.array(y0, dtype=np.float64, copy=True)
        C = len(self.sets)
        if self.kind == RBGS:
            for _ in range(self.sweeps):
                for c in range(C):
                    self._sweep(c, b, y)
        elif self.kind == RBGS_SYM:
            for _ in range(self.sweeps):
                for c in list(range(C)) + list(range(C - 1, -1, -1)):
                    self._sweep(c, b, y)
        elif self.kind == JACOBI:
            y = y + self.omega * (b - self.A @ y) / self.D
        elif self.kind == NONE:
            pass
        else:
            raise ValueError(self.kind)
        return y
