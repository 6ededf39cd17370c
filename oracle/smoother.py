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
    def __init__(self, A, colors, kind=RBGS, omega=2.0 / 3.0):
        self.kind = kind
        self.A = sp.csr_matrix(A)
        self.D = self.A.diagonal()
        self.red = np.flatnonzero(colors == 0)
        self.black = np.flatnonzero(colors == 1)
        self.A_RB = self.A[self.red][:, self.black]
        self.A_BR = self.A[self.black][:, self.red]
        self.omega = omega

    def _red(self, b, y):
        # y_R <- D_R^-1 (b_R - A_RB y_B)
        y[self.red] = (b[self.red] - self.A_RB @ y[self.black]) / self.D[self.red]

    def _black(self, b, y):
        # y_B <- D_B^-1 (b_B - A_BR y_R)
        y[self.black] = (b[self.black] - self.A_BR @ y[self.red]) / self.D[self.black]

    def __call__(self, b, y0):
        y = np.array(y0, dtype=np.float64, copy=True)
        if self.kind == RBGS:
            self._red(b, y)
            self._black(b, y)
        elif self.kind == RBGS_SYM:
            self._red(b, y)
            self._black(b, y)
            self._black(b, y)
            self._red(b, y)
        elif self.kind == JACOBI:
            y = y + self.omega * (b - self.A @ y) / self.D
        elif self.kind == NONE:
            pass
        else:
            raise ValueError(self.kind)
        return y
