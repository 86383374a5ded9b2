"""Lanczos-Sylvester solver of Section 3.3, written from its equations.  Oracle: test
infrastructure only (tests, the smoke check and the CPU leg of the benchmark call it; the library
never does).

Case treated (Section 3.3): one prior factor shared by all components (every kappa_j equal) and
separable noise W[f, p] = t_f n_p with every n_p > 0.  The posterior-mean system is then the
Sylvester equation (eq. (Axb-Sylv))

    N^-1 D2 M + M Lhat = Yhat,
    D2 = (kappa^2 I - Lap)^2,  Lhat = A^T T A P^-1,  Yhat = Y T A P^-1,

with P = diag(tau), T = diag(t), N = diag(n) and M the N x k matrix whose column j is map j.
Its solution is the posterior mean of the Kronecker system (eq. (Axb)).

What is computed, from the equations of Section 3.3 (not from the printed listings):

  * Basis.  Yhat = V_1 B_0 with V_1^T N V_1 = I, and the block Lanczos relation for the
    operator N^-1 D2, which is symmetric in the N inner product (Lemma 1):
        N^-1 D2 [V_1 .. V_j] = [V_1 .. V_j] T_j + V_(j+1) B_(j+1) E_j^T,
    T_j block tridiagonal with diagonal blocks H_i = V_i^T D2 V_i and B_(i+1) below the
    diagonal (B_(i+1)^T above it), so that V^T D2 V = T_j (eq. (tridiag-factorization)).  Each
    new block is the part of N^-1 D2 V_j that the relation leaves, N-orthonormalised by a
    Cholesky factorisation of its N-Gram matrix (B upper triangular).
  * Galerkin approximation M_j = [V_1 .. V_j] Z_j with the projected equation
        T_j Z + Z Lhat = E_1 B_0                                     (eq. (Sylv-small)).
    By Lemma 2, Lhat = U R U^-1 with R = diag(rho), rho > 0, U = P^1/2 V_s and U^-1 = U^T P^-1
    (V_s the orthonormal eigenvectors of P^-1/2 A^T T A P^-1/2), so column l of Z U solves the
    symmetric positive definite banded system (T_j + rho_l I) (Z U) e_l = E_1 B_0 U e_l
    (eq. (soln-constr)'s decoupling, solved here by a banded Cholesky factorisation, LAPACK
    dpbtrf/dpbtrs, instead of an eigendecomposition of T_j), and Z = (Z U) U^T P^-1.
  * Residual.  Substituting both relations, the residual of eq. (Axb-Sylv) at M_j is
    N^-1 D2 M_j + M_j Lhat - Yhat = V_(j+1) B_(j+1) E_j^T Z_j, so the squared N-norm of the
    residual times U (the quantity Alg. 5 calls gamma) is ||B_(j+1) (E_j^T Z_j) U||_F^2.
  * Stopping: the first j with sqrt(gamma_j) <= tol ||B_0||_F (Alg. 5's test); a new block of
    N-norm zero ends the process (the Krylov space is invariant and M_j exact).

Readings (where the printed algorithms are garbled or inconsistent with these equations):

  * The block beside H_(i-1) in the symmetric T_j is B_i^T, so the three-term relation subtracts
    V_(i-1) B_i^T (the listing prints B_i, right only for symmetric B_i).
  * H_i = V_i^T D2 V_i is symmetric in exact arithmetic; its symmetric part is kept.
  * Alg. 5 writes Lhat = U R U^T although Lhat is not symmetric; Lemma 2's U R U^-1 with
    U^-1 = U^T P^-1 is used.
  * Alg. 5's gamma is taken as the squared N-norm of the Sylvester residual times U (its listed
    J and F readings give that value, which tests/test_oracle_lanczos.py checks against the
    explicitly formed residual).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import operator as op


def sylvester_data(prob, t: np.ndarray, nvec: np.ndarray):
    """The pieces of eq. (Axb-Sylv) for a problem with common kappa and W = t (x) n.

    Returns (D2 sparse N x N, nvec, Lhat k x k, Yhat N x k, U k x k, rho k, P k x k)."""
    kap = np.asarray(prob.kappa, dtype=np.float64)
    if not np.all(kap == kap[0]):
        raise ValueError("the Sylvester form needs one kappa for every component")
    t = np.asarray(t, dtype=np.float64).reshape(prob.f)
    nvec = np.asarray(nvec, dtype=np.float64).reshape(prob.n_pix)
    if not np.all(nvec > 0):
        raise ValueError("the Sylvester form needs n_p > 0 at every pixel (N invertible)")
    if not np.array_equal(prob.W, np.outer(t, nvec)):
        raise ValueError("the Sylvester form needs W = t (x) n")
    D2 = op.prior_block(prob.ny, prob.nx, kap[0], 1.0,      # (kappa^2 I - Lap)^T (kappa^2 I - Lap)
                        op.boundary_of(prob))
    tau = np.asarray(prob.tau, dtype=np.float64)
    P = np.diag(tau)
    Pinv = np.diag(1.0 / tau)
    T = np.diag(t)
    Lhat = prob.A.T @ T @ prob.A @ Pinv
    Yhat = prob.Y.T @ T @ prob.A @ Pinv                       # N x k
    # Lemma 2: Lhat = U R U^-1 with U^T P^-1 U = I
    Ph = np.diag(np.sqrt(tau))
    Pmh = np.diag(1.0 / np.sqrt(tau))
    rho, Vs = np.linalg.eigh(Pmh @ (prob.A.T @ T @ prob.A) @ Pmh)
    U = Ph @ Vs
    return D2, nvec, Lhat, Yhat, U, rho, P


def n_qr(W: np.ndarray, nvec: np.ndarray):
    """QR factorisation in the N inner product: W = V B with V^T N V = I, B upper triangular
    (Cholesky of the N-Gram matrix W^T N W = B^T B).  Returns (V, B); (0, 0) for a zero W."""
    Gm = W.T @ (nvec[:, None] * W)
    Gm = 0.5 * (Gm + Gm.T)
    if np.max(np.abs(np.diag(Gm))) == 0.0:
        m = W.shape[1]
        return np.zeros_like(W), np.zeros((m, m))
    B = np.linalg.cholesky(Gm).T                               # raises if not positive definite
    V = np.linalg.solve(B.T, W.T).T                            # W B^-1
    return V, B


def extend_basis(D2, nvec, Vs, Hs, Bs):
    """One more block of the Lanczos relation: with V_j the last block of Vs, append
    H_j = sym(V_j^T D2 V_j) to Hs and the N-QR factors of
    N^-1 D2 V_j - V_j H_j - V_(j-1) B_j^T  =  V_(j+1) B_(j+1)
    to Vs and Bs (Bs[0] = B_0 of the start block, Bs[i] = B_(i+1))."""
    Vj = Vs[-1]
    AV = (D2 @ Vj) / nvec[:, None]
    H = Vj.T @ (D2 @ Vj)
    H = 0.5 * (H + H.T)
    Wn = AV - Vj @ H
    if len(Vs) > 1:
        Wn = Wn - Vs[-2] @ Bs[-1].T
    Vn, Bn = n_qr(Wn, nvec)
    Hs.append(H)
    Bs.append(Bn)
    Vs.append(Vn)


def lanczos(D2, nvec, Yhat, j: int):
    """j blocks of the block Lanczos relation for N^-1 D2 in the N inner product, started from
    Yhat.  Returns (V list of j + 1 blocks, H list of j blocks, B list of j + 1 blocks with
    B[0] = B_0 from Yhat = V_1 B_0, B[i] = B_(i+1))."""
    V, B0 = n_qr(Yhat, nvec)
    Vs, Hs, Bs = [V], [], [B0]
    for _ in range(j):
        extend_basis(D2, nvec, Vs, Hs, Bs)
    return Vs, Hs, Bs


def block_tridiagonal(Hs, Bs) -> np.ndarray:
    """T_i from H_1..H_i (diagonal blocks) and B_2..B_i (below the diagonal; transposes above)."""
    i = len(Hs)
    m = Hs[0].shape[0]
    T = np.zeros((i * m, i * m))
    for a in range(i):
        T[a * m:(a + 1) * m, a * m:(a + 1) * m] = Hs[a]
        if a + 1 < i:
            Bn = Bs[a + 1]                                     # B_(a+2) in 1-based names
            T[(a + 1) * m:(a + 2) * m, a * m:(a + 1) * m] = Bn
            T[a * m:(a + 1) * m, (a + 1) * m:(a + 2) * m] = Bn.T
    return T


def _banded_lower(Hs, Bs, shift: float) -> np.ndarray:
    """T_i + shift I in LAPACK's lower banded storage (bandwidth 2m - 1), from its blocks:
    ab[d, c] = (T + shift I)[c + d, c]."""
    i = len(Hs)
    m = Hs[0].shape[0]
    n = i * m
    ab = np.zeros((2 * m, n))
    for a in range(i):
        for c in range(m):
            col = a * m + c
            for r in range(c, m):                              # the diagonal block, lower part
                ab[r - c, col] = Hs[a][r, c] + (shift if r == c else 0.0)
            if a + 1 < i:
                Bn = Bs[a + 1]                                 # block below: rows of block a + 1
                for r in range(m):
                    ab[m + r - c, col] = Bn[r, c]
    return ab


def projected_solution(Hs, Bs, U, rho):
    """Z U for the projected equation T_i Z + Z Lhat = E_1 B_0 (eq. (Sylv-small)) with
    Lhat = U diag(rho) U^-1: column l solves (T_i + rho_l I) x = E_1 B_0 U e_l by a banded
    Cholesky factorisation.  Returns Z U as an (i m) x m array."""
    i = len(Hs)
    m = Hs[0].shape[0]
    rhs = np.zeros((i * m, m))
    rhs[:m, :] = Bs[0] @ U
    ZU = np.zeros((i * m, m))
    band = min(2 * m - 1, i * m - 1)                          # sub-diagonals of T_i
    for l in range(m):
        ab = _banded_lower(Hs, Bs, rho[l])[:band + 1]
        ZU[:, l] = sla.solveh_banded(ab, rhs[:, l], lower=True)
    return ZU


def residual_gamma(Hs, Bs, U, rho) -> float:
    """gamma_i = ||B_(i+1) (E_i^T Z U)||_F^2: the squared N-norm of the Sylvester residual at the
    Galerkin approximation, times U (the residual is V_(i+1) B_(i+1) E_i^T Z)."""
    m = U.shape[0]
    ZU = projected_solution(Hs, Bs, U, rho)
    v = Bs[len(Hs)] @ ZU[-m:, :]
    return float(np.sum(v * v))


def galerkin_coefficients(Hs, Bs, U, rho, P):
    """Z = (Z U) U^T P^-1, as the list of its k x k blocks G_j (M = sum_j V_j G_j)."""
    m = U.shape[0]
    Z = projected_solution(Hs, Bs, U, rho) @ U.T @ np.linalg.inv(P)
    return [Z[j * m:(j + 1) * m, :] for j in range(len(Hs))]


def lanczos_sylvester(prob, t, nvec, tol: float = 1e-8, max_iter: int = 1000,
                      record: bool = False):
    """Galerkin approximations of eq. (Axb-Sylv) over growing block Krylov spaces until Alg. 5's
    test holds.  Returns a dict with the solution M as [k, n_pix] ('x'), the number of Lanczos
    steps ('iters'), the final estimate sqrt(gamma)/||B_0||_F ('relres_est'), its history
    ('history'), the blocks H, B and U, rho, and with record=True the basis blocks ('V')."""
    D2, nvec, Lhat, Yhat, U, rho, P = sylvester_data(prob, t, nvec)
    V1, B0 = n_qr(Yhat, nvec)
    nb0 = float(np.linalg.norm(B0))
    Vs, Hs, Bs, hist = [V1], [], [B0], []
    gamma = 0.0
    if nb0 > 0.0:
        for _ in range(max_iter):
            extend_basis(D2, nvec, Vs, Hs, Bs)
            gamma = residual_gamma(Hs, Bs, U, rho)
            hist.append(np.sqrt(gamma) / nb0)
            if np.sqrt(gamma) <= tol * nb0 or not np.any(Bs[-1]):
                break
    j = len(Hs)
    if j > 0:
        Gs = galerkin_coefficients(Hs, Bs, U, rho, P)
        M = np.hstack(Vs[:j]) @ np.vstack(Gs)
    else:
        M = np.zeros_like(Yhat)
    out = {"x": M.T.copy(), "iters": j,
           "relres_est": float(np.sqrt(gamma) / nb0) if nb0 > 0 else 0.0,
           "history": np.array(hist), "H": Hs, "B": Bs, "U": U, "rho": rho,
           "converged": bool(np.sqrt(gamma) <= tol * nb0)}
    if record:
        out["V"] = Vs
    return out
