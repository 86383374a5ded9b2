"""CPU oracle for the posterior-mean system -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct float64 implementation of what the GPU path computes, written
from the paper (Pham, Soodhalter, Wilson: fast solution of Sylvester-structured systems for
spatial source separation of the CMB):

  operator.py  the posterior precision G = Q + B^T C B (eq. (Q*), eq. (Axb)) assembled as explicit
               sparse/dense matrices with Kronecker products, the right-hand side B^T C Y
               (eq. (mu*)), and an independent sum-of-terms evaluation used to cross-check it.
  solve.py     exact solves: dense Cholesky of the assembled matrix; a Fourier solve for
               homoscedastic periodic problems; the sparse-dense Sylvester method of Alg. 3 for the
               separable equal-kappa case (Section 3.3.1).
  pcg.py       conjugate gradients (Alg. 2) with a left preconditioner inserted, plus the
               block-Jacobi preconditioner taken from the assembled matrix.
  grad.py      gradients of a loss of the solution through the adjoint method, written with
               explicitly assembled derivative matrices, and central finite differences.
  po.py        perturbation-optimisation right-hand sides (a sample of N(x*, G^-1) after a solve).
  lanczos.py   the Lanczos-Sylvester solver: block Lanczos in the N inner product (Alg. 4) inside
               the symmetric sparse Sylvester solver with its residual estimate (Alg. 5), for the
               separable equal-kappa case (Sections 3.3.2-3.3.4).

Only the test-suite, the smoke check of the package entry point and the CPU-baseline leg of the
benchmark may import anything from here.  The GPU library and its Python binding never import,
link or call this package, and this package never imports them.
"""
from . import operator, solve, pcg, grad, po, lanczos  # noqa: F401
