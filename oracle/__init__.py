"""CPU FP64 oracle for the reduced-basis iterative solvers (TEST INFRASTRUCTURE ONLY).

Plain, slow, obviously-correct NumPy/SciPy implementations of what the GPU library
computes, written from the paper (Nguyen & Chen, "Reduced-basis method for the
iterative solution of parametrized SPD linear systems"):

  operator.py  affine block-diffusion operator A(mu) = sum_q Theta_q(mu) A_q (eq. 12)
  smoother.py  S(A, b, y): Gauss-Seidel / Jacobi smoothers (eq. 8, Sec. 3.1; Sec. 3.3)
  rb.py        reduced operators (eq. 12b/12c), Cholesky (Sec. 2.1), RBI (Alg. 2),
               RBCG (Alg. 3), plain CG, modified Gram-Schmidt (Sec. 2.2)
  greedy.py    greedy sampling (Alg. 1) and adaptive greedy (Alg. 4), both indicators
  mlp.py       MLP surrogate of the greedy indicator (not in the paper)

Only tests, the smoke entry point and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library, and the library never
imports it.  Everything here works in the natural lexicographic ordering
(x fastest) and in float64.
"""
