"""Pins of the Lanczos-Sylvester oracle (Section 3.3: Alg. 4, Alg. 5) against mathematics and
independent solvers (no GPU)."""
import os

import numpy as np
import pytest

from oracle import lanczos as olz
from oracle import operator as op
from oracle import solve as osv
from workloads import make_problem

HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) /
                 max(np.linalg.norm(np.asarray(b)), 1e-300))


def sep_problem(ny, nx, k, f, seed, kappa=0.45):
    p = make_problem(ny, nx, k, f, seed=seed, noise="separable", kappa=np.full(k, kappa))
    return p, p.meta["t"], p.meta["n"]


def test_separable_generator_factors():
    p, t, n = sep_problem(7, 9, 3, 5, 2000)
    assert np.array_equal(p.W, np.outer(t, n)) and np.all(n > 0)


def test_sylvester_form_is_the_posterior_system():
    """eq. (Axb-Sylv) multiplied back by N (left) and P (right) is G applied to M."""
    p, t, n = sep_problem(6, 5, 3, 4, 2001)
    D2, nvec, Lhat, Yhat, U, rho, P = olz.sylvester_data(p, t, n)
    M = np.random.default_rng(1).standard_normal((p.n_pix, p.k))
    lhs = (D2 @ M + nvec[:, None] * (M @ Lhat)) @ P         # N (N^-1 D2 M + M Lhat) P
    assert rel(lhs.T, op.apply_terms(p, M.T)) < 1e-13
    assert rel((nvec[:, None] * Yhat) @ P, op.rhs(p).T) < 1e-13
    # Lemma 2: Lhat = U R U^-1 with U^T P^-1 U = I, real positive eigenvalues
    assert np.allclose(Lhat @ U, U * rho[None, :], rtol=1e-12, atol=1e-12)
    assert np.allclose(U.T @ np.linalg.inv(P) @ U, np.eye(p.k), atol=1e-12)
    assert np.all(rho > 0)


def test_lanczos_blocks_are_n_orthonormal():
    """The Lanczos relation only orthogonalises against the last two blocks; the symmetry of N^-1 D2 in the N
    inner product (Lemma 1) makes every pair of blocks N-orthogonal."""
    p, t, n = sep_problem(7, 6, 3, 5, 2002)
    D2, nvec, _, Yhat, _, _, _ = olz.sylvester_data(p, t, n)
    Vs, Hs, Bs = olz.lanczos(D2, nvec, Yhat, 5)
    Vall = np.hstack(Vs)
    Gm = Vall.T @ (nvec[:, None] * Vall)
    assert np.allclose(Gm, np.eye(Gm.shape[0]), atol=1e-9)
    assert not np.allclose(Bs[2], Bs[2].T)                   # B blocks are not symmetric
    for B in Bs:
        assert np.allclose(B, np.triu(B))


def test_lanczos_tridiagonal_factorisation():
    """eq. (tridiag-factorization): V_j^T D2 V_j = T_j, by explicit product."""
    p, t, n = sep_problem(8, 7, 4, 6, 2003)
    D2, nvec, _, Yhat, _, _, _ = olz.sylvester_data(p, t, n)
    Vs, Hs, Bs = olz.lanczos(D2, nvec, Yhat, 4)
    Vj = np.hstack(Vs[:4])
    T = olz.block_tridiagonal(Hs, Bs)
    assert rel(Vj.T @ (D2 @ Vj), T) < 1e-10
    # and the Lanczos relation N^-1 D2 V_j = V_(j+1) Tbar_j
    m = p.k
    Tbar = np.zeros((5 * m, 4 * m))
    Tbar[:4 * m, :] = T
    Tbar[4 * m:, 3 * m:] = Bs[4]
    assert rel((D2 @ Vj) / nvec[:, None], np.hstack(Vs) @ Tbar) < 1e-10


@pytest.mark.parametrize("shape", [(6, 5, 3, 4), (9, 8, 4, 9), (1, 24, 2, 3), (4, 4, 1, 2)])
def test_lanczos_sylvester_equals_dense(shape):
    ny, nx, k, f = shape
    p, t, n = sep_problem(ny, nx, k, f, 2004 + ny)
    res = olz.lanczos_sylvester(p, t, n, tol=1e-11, max_iter=400)
    assert res["converged"]
    xd = osv.solve_dense(p)
    assert rel(res["x"], xd) < 1e-8
    assert rel(res["x"], osv.solve_kohler(p, t, n)) < 1e-8


def test_projected_solution_is_the_small_sylvester_solution():
    """The coefficients Z of the Galerkin approximation solve T_i Z + Z Lhat = E_1 B_0
    (eq. (Sylv-small)): the oracle's decoupled banded solves against LAPACK's Bartels-Stewart
    solver (scipy.linalg.solve_sylvester) on the explicitly assembled T_i."""
    import scipy.linalg as sla
    p, t, n = sep_problem(8, 7, 4, 6, 2008)
    D2, nvec, Lhat, Yhat, U, rho, P = olz.sylvester_data(p, t, n)
    Vs, Hs, Bs = olz.lanczos(D2, nvec, Yhat, 6)
    for i in range(1, 7):
        T = olz.block_tridiagonal(Hs[:i], Bs[:i + 1])
        C = np.zeros((i * p.k, p.k))
        C[:p.k, :] = Bs[0]
        Zref = sla.solve_sylvester(T, Lhat, C)
        Z = np.vstack(olz.galerkin_coefficients(Hs[:i], Bs[:i + 1], U, rho, P))
        assert rel(Z, Zref) < 1e-10, i


def test_gamma_is_the_residual_norm():
    """Alg. 5's gamma equals the squared N-norm of (N^-1 D2 M_i + M_i Lhat - Yhat) U for the
    explicitly assembled Galerkin approximation M_i, at every step."""
    p, t, n = sep_problem(8, 8, 3, 5, 2005)
    D2, nvec, Lhat, Yhat, U, rho, P = olz.sylvester_data(p, t, n)
    for i in range(1, 6):
        res = olz.lanczos_sylvester(p, t, n, tol=0.0, max_iter=i)
        assert res["iters"] == i
        M = res["x"].T
        R = (D2 @ M) / nvec[:, None] + M @ Lhat - Yhat
        RU = R @ U
        direct = np.sqrt(np.sum(nvec[:, None] * RU * RU))
        nb0 = np.linalg.norm(res["B"][0])
        assert res["history"][-1] == pytest.approx(direct / nb0, rel=1e-7)


def test_iterates_are_galerkin_over_an_independent_krylov_basis():
    """Step i's approximation is the Galerkin solution of eq. (Axb-Sylv) over the block Krylov
    space K_i(N^-1 D2, Yhat), built here independently (explicit powers, QR in the N inner
    product) and solved in Kronecker form."""
    p, t, n = sep_problem(7, 7, 3, 4, 2006)
    D2, nvec, Lhat, Yhat, U, rho, P = olz.sylvester_data(p, t, n)
    sq = np.sqrt(nvec)[:, None]
    for i in range(1, 5):
        blocks = [Yhat]
        for _ in range(i - 1):
            blocks.append((D2 @ blocks[-1]) / nvec[:, None])
        K = np.hstack(blocks)
        Qn, _ = np.linalg.qr(sq * K)                          # orthonormal in the plain product
        Vt = Qn / sq                                          # N-orthonormal basis of the space
        Ap = Vt.T @ (D2 @ Vt)                                 # V^T N (N^-1 D2) V
        C = Vt.T @ (nvec[:, None] * Yhat)
        dim, m = Ap.shape[0], p.k
        Kron = np.kron(np.eye(m), Ap) + np.kron(Lhat.T, np.eye(dim))
        Z = np.linalg.solve(Kron, C.reshape(-1, order="F")).reshape(dim, m, order="F")
        M_ind = Vt @ Z
        res = olz.lanczos_sylvester(p, t, n, tol=0.0, max_iter=i)
        assert rel(res["x"].T, M_ind) < 1e-8, i


def test_lanczos_sylvester_with_printed_planck_constants():
    """The paper's printed A and T (App. B) with kappa = 0 (the paper's D^2 prior, rank N - 1):
    a mixing term ~1e7 times the prior; Alg. 5 agrees with dense Cholesky."""
    A, T = [], None
    with open(os.path.join(HERE, "golden", "planck_mixing.txt")) as fh:
        for line in fh:
            if line.startswith("A "):
                A.append([float(v) for v in line.split()[1:]])
            elif line.startswith("T "):
                T = np.array([float(v) for v in line.split()[1:]])
    A = np.array(A)
    ny, nx = 6, 6
    nvec = np.random.default_rng(19).integers(1, 4, ny * nx).astype(float)
    p = make_problem(ny, nx, 4, 9, seed=19, kappa=np.zeros(4), tau=np.ones(4), A=A)
    p.W = np.outer(T, nvec)
    res = olz.lanczos_sylvester(p, T, nvec, tol=1e-12, max_iter=200)
    assert res["converged"]
    assert rel(res["x"], osv.solve_dense(p)) < 1e-7


def test_rejects_unsupported_problems():
    p, t, n = sep_problem(5, 5, 2, 3, 2007)
    p2 = make_problem(5, 5, 2, 3, seed=2007, noise="separable")   # drawn, unequal kappas
    with pytest.raises(ValueError):
        olz.lanczos_sylvester(p2, p2.meta["t"], p2.meta["n"])
    n0 = n.copy()
    n0[3] = 0.0
    p.W = np.outer(t, n0)
    with pytest.raises(ValueError):
        olz.lanczos_sylvester(p, t, n0)
