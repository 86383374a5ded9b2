"""Lanczos-Sylvester solver: block Lanczos in the N inner product (Alg. 4) inside the symmetric
sparse Sylvester solver (Alg. 5).  Oracle: test infrastructure only (tests, the smoke check and
the CPU leg of the benchmark call it; the library never does).

Case treated (Section 3.3): one prior factor shared by all components (every kappa_j equal) and
separable noise W[f, p] = t_f n_p with every n_p > 0.  The posterior-mean system is then the
Sylvester equation (eq. (Axb-Sylv))

    N^-1 D2 M + M Lhat = Yhat,
    D2 = (kappa^2 I - Lap)^2,  Lhat = A^T T A P^-1,  Yhat = Y T A P^-1,

with P = diag(tau), T = diag(t), N = diag(n) and M the N x k matrix whose column j is map j.
Its solution is the posterior mean of the Kronecker system (eq. (Axb)).

The steps follow Alg. 4 and Alg. 5 in the paper's order and notation.  Readings where the
printed algorithms are garbled or inconsistent with the equations they implement:

  * The three-term step subtracts V_old B_i^T: the block below H_(i-1) in T_j is B_i and the
    block beside it is its transpose, so that T_j is symmetric as eq. (tridiag-factorization)
    requires (the listing prints B_i, which is only right for symmetric B_i).
  * H_i = V^T N W is symmetric in exact arithmetic; its symmetric part enters T_j.
  * Lhat is not symmetric; Lemma 2 gives Lhat = U R U^-1 with U^T P^-1 U = I.  U and R come
    from the symmetric matrix P^-1/2 A^T T A P^-1/2 = V R V^T as U = P^1/2 V.  Alg. 5 writes
    the decomposition as U R U^T; the solution formula uses U^-1 = U^T P^-1 (eq. (soln-constr)),
    and so does the final Z here.
  * In the residual estimate J is the last block row of Q_i, transposed, times B_(i+1)^T (the
    listing's Q_i E_m); with it, gamma is the squared N-norm of the Sylvester residual times U.
  * F has i*m rows (one per eigenvalue of T_i) and its numerator is (Q_i^T E_1 B_0 U)_(k,l)
    (the listing's Q_l is Q_i).
  * The loop stops when sqrt(gamma) <= eps ||B_0||_F; the first pass always runs.  A block W of
    N-norm zero ends the loop (the Krylov space is invariant; the Galerkin solution is exact).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

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


def lanczos(D2, nvec, Yhat, j: int):
    """Alg. 4: j steps of the symmetric block Lanczos process for N^-1 D2 in the N inner product,
    started from Yhat.  Returns (V list of j + 1 blocks, H list of j blocks, B list of j + 1
    blocks with B[0] = B_0 from Yhat = V_1 B_0, B[i] = B_(i+1))."""
    V, B0 = n_qr(Yhat, nvec)
    Vs, Hs, Bs = [V], [], [B0]
    for i in range(1, j + 1):
        W = (D2 @ Vs[-1]) / nvec[:, None]
        if i > 1:
            W = W - Vs[-2] @ Bs[-1].T
        H = Vs[-1].T @ (nvec[:, None] * W)
        H = 0.5 * (H + H.T)
        W = W - Vs[-1] @ H
        Vn, Bn = n_qr(W, nvec)
        Hs.append(H)
        Bs.append(Bn)
        Vs.append(Vn)
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


def residual_gamma(Hs, Bs, U, rho):
    """Alg. 5's residual estimate after i = len(Hs) steps: eigendecomposition T_i = Q Phi Q^T,
    S = (U^T B_0^T)(E_1^T Q), J = (E_i^T Q)^T B_(i+1)^T, gamma = sum_l ||e_l^T S K_l^-1 J||^2
    with K_l = rho_l I + Phi.  Returns (gamma, phi, Q)."""
    m = U.shape[0]
    T = block_tridiagonal(Hs, Bs)
    phi, Q = np.linalg.eigh(T)
    B0 = Bs[0]
    Bnext = Bs[len(Hs)]
    S = (U.T @ B0.T) @ Q[:m, :]
    J = Q[-m:, :].T @ Bnext.T
    gamma = 0.0
    for l in range(m):
        Kinv = 1.0 / (rho[l] + phi)
        v = (S[l, :] * Kinv) @ J
        gamma += float(v @ v)
    return gamma, phi, Q


def galerkin_coefficients(Hs, Bs, U, rho, P):
    """Z = Q F U^T P^-1 with F_(k,l) = (Q^T E_1 B_0 U)_(k,l) / (phi_k + rho_l) (eq. (soln-constr)).
    Returns the list of k x k blocks G_j of Z (M = sum_j V_j G_j)."""
    m = U.shape[0]
    T = block_tridiagonal(Hs, Bs)
    phi, Q = np.linalg.eigh(T)
    num = Q[:m, :].T @ (Bs[0] @ U)                             # Q^T E_1 B_0 U, (i m) x m
    F = num / (phi[:, None] + rho[None, :])
    Z = Q @ F @ U.T @ np.linalg.inv(P)
    return [Z[j * m:(j + 1) * m, :] for j in range(len(Hs))]


def lanczos_sylvester(prob, t, nvec, tol: float = 1e-8, max_iter: int = 1000,
                      record: bool = False):
    """Alg. 5.  Returns a dict with the solution M as [k, n_pix] ('x'), the number of Lanczos
    steps ('iters'), the final estimate sqrt(gamma)/||B_0||_F ('relres_est'), the history of
    that estimate ('history'), and the coefficients H, B.  With record=True also the Lanczos
    blocks of the first pass ('V')."""
    D2, nvec, Lhat, Yhat, U, rho, P = sylvester_data(prob, t, nvec)
    V, B0 = n_qr(Yhat, nvec)
    nb0 = float(np.linalg.norm(B0))
    Vold = np.zeros_like(V)
    Hs, Bs, hist, Vrec = [], [B0], [], [V]
    i = 0
    gamma = np.inf
    while np.sqrt(gamma) > tol * nb0:
        if i >= max_iter:
            break
        i += 1
        # Lanczos step
        W = (D2 @ V) / nvec[:, None]
        if i > 1:
            W = W - Vold @ Bs[-1].T
        H = V.T @ (nvec[:, None] * W)
        H = 0.5 * (H + H.T)
        W = W - V @ H
        Vold = V
        V, Bn = n_qr(W, nvec)
        Hs.append(H)
        Bs.append(Bn)
        if record:
            Vrec.append(V)
        # residual norm estimate
        gamma, _, _ = residual_gamma(Hs, Bs, U, rho)
        hist.append(np.sqrt(gamma) / nb0)
        if not np.any(Bn):
            gamma = 0.0
            break
    # coefficients of the approximation, then a second Lanczos pass assembles M block by block
    Gs = galerkin_coefficients(Hs, Bs, U, rho, P)
    M = np.zeros_like(Yhat)
    V = np.linalg.solve(B0.T, Yhat.T).T
    Vold = np.zeros_like(V)
    for j in range(1, i + 1):
        M = M + V @ Gs[j - 1]
        if j == i:
            break
        W = (D2 @ V) / nvec[:, None]
        if j > 1:
            W = W - Vold @ Bs[j - 1].T
        W = W - V @ Hs[j - 1]
        Vold = V
        V = np.linalg.solve(Bs[j].T, W.T).T
    out = {"x": M.T.copy(), "iters": i, "relres_est": float(np.sqrt(gamma) / nb0),
           "history": np.array(hist), "H": Hs, "B": Bs, "U": U, "rho": rho,
           "converged": bool(np.sqrt(gamma) <= tol * nb0)}
    if record:
        out["V"] = Vrec
    return out
