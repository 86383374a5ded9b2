"""Posterior precision operator and right-hand side as explicit matrices (oracle; tests only).

Problem (Section 2.2 and Section 3, eq. (Axb)): find mu with (Q + B^T C B) mu = B^T C Y, where
  B = A (x) I_N            (design, maps stacked by map, Section 2.1)
  C = diag(W[0,:], ..., W[f-1,:])   (noise precision; the paper's separable T (x) N is the case
                                     W[f, p] = tau_f n_p, Section 3)
  Q = bldiag(Q_1, ..., Q_k),  Q_j = tau_j L_j^T L_j,  L_j = kappa_j^2 I - Lap
The paper's prior block is phi_l D^T D = phi_l D^2 with D the graph Laplacian of the 4-neighbour
pixel graph (Section 3, definition of D; App. C).  On a periodic grid D is the 5-point Laplacian,
so the paper's case is kappa_j = 0, tau_j = phi_l.  kappa > 0 is the proper (SPDE) generalisation.

Vectors are component-major: vec(X) = [x_1; ...; x_k] for X of shape [k, n_pix], which is the
paper's column-major reshape of mu to an N x m matrix (Section 3.1).  Pixel p = iy * nx + ix.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _shift(ny: int, nx: int, dy: int, dx: int) -> sp.csr_matrix:
    """Periodic shift: (S u)[iy, ix] = u[(iy + dy) % ny, (ix + dx) % nx]."""
    n = ny * nx
    p = np.arange(n)
    iy, ix = np.divmod(p, nx)
    cols = ((iy + dy) % ny) * nx + (ix + dx) % nx
    return sp.csr_matrix((np.ones(n), (p, cols)), shape=(n, n))


def laplacian(ny: int, nx: int, boundary: str = "periodic") -> sp.csr_matrix:
    """Graph Laplacian of the 4-neighbour pixel grid (Section 3, definition of D): off-diagonal
    entries count neighbour links, the diagonal is minus the row sum of the off-diagonal part.

    periodic: Lap = Sx + Sx^T + Sy + Sy^T - 4 I.  On grids with a side below 3 two neighbour
              links land on the same pixel; the sparse sum adds them, which keeps
              Lap = (polynomial in the shift operators) for every grid size.
    face:     links only between pixels inside the grid (one HEALPix base face, whose
              neighbours are confined to the face, App. A); border pixels have fewer links and
              a correspondingly smaller diagonal.  Lap 1 = 0 and rank N - 1 (App. C).
    """
    n = ny * nx
    if boundary == "periodic":
        sx = _shift(ny, nx, 0, 1)
        sy = _shift(ny, nx, 1, 0)
        return (sx + sx.T + sy + sy.T - 4.0 * sp.identity(n, format="csr")).tocsr()
    if boundary != "face":
        raise ValueError(f"unknown boundary {boundary!r}")
    p = np.arange(n).reshape(ny, nx)
    rows = np.concatenate([p[:, :-1].ravel(), p[:-1, :].ravel()])     # right and down links
    cols = np.concatenate([p[:, 1:].ravel(), p[1:, :].ravel()])
    adj = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(n, n))
    adj = (adj + adj.T).tocsr()
    deg = np.asarray(adj.sum(axis=1)).ravel()
    return (adj - sp.diags(deg)).tocsr()


def prior_factor(ny: int, nx: int, kappa: float, boundary: str = "periodic") -> sp.csr_matrix:
    """L = kappa^2 I - Lap."""
    n = ny * nx
    return (kappa * kappa * sp.identity(n, format="csr") - laplacian(ny, nx, boundary)).tocsr()


def prior_block(ny: int, nx: int, kappa: float, tau: float,
                boundary: str = "periodic") -> sp.csr_matrix:
    """Q_j = tau L^T L, formed by an explicit sparse product (no stencil coefficients)."""
    L = prior_factor(ny, nx, kappa, boundary)
    return (tau * (L.T @ L)).tocsr()


def boundary_of(prob) -> str:
    return getattr(prob, "boundary", "periodic")


def posterior_precision(prob, dense: bool = False):
    """G = sum_j E_jj (x) Q_j + sum_f (a_f a_f^T) (x) diag(W[f, :])   (eq. (Q*) in Kronecker form).

    The first sum is Q = bldiag(Q_j); the second is B^T C B = (A^T (x) I) C (A (x) I) written per
    frequency, which in the separable case equals (A^T T A) (x) N (Section 3.1).
    """
    k, f, n_pix = prob.k, prob.f, prob.n_pix
    G = sp.csr_matrix((k * n_pix, k * n_pix))
    for j in range(k):
        E = np.zeros((k, k))
        E[j, j] = 1.0
        G = G + sp.kron(sp.csr_matrix(E), prior_block(prob.ny, prob.nx, prob.kappa[j],
                                                        prob.tau[j], boundary_of(prob)))
    for fi in range(f):
        a = prob.A[fi]
        G = G + sp.kron(sp.csr_matrix(np.outer(a, a)), sp.diags(prob.W[fi]))
    G = G.tocsr()
    return G.toarray() if dense else G


def design(prob) -> sp.csr_matrix:
    """B = A (x) I_N."""
    return sp.kron(sp.csr_matrix(prob.A), sp.identity(prob.n_pix)).tocsr()


def noise_precision(prob) -> sp.csr_matrix:
    """C = diag of W stacked by map (first N entries belong to map 1, ...)."""
    return sp.diags(prob.W.ravel()).tocsr()


def likelihood_term(prob) -> sp.csr_matrix:
    """B^T C B assembled literally as a product of the three Kronecker-structured factors."""
    B = design(prob)
    return (B.T @ noise_precision(prob) @ B).tocsr()


def rhs(prob, Y=None) -> np.ndarray:
    """b = B^T C Y (eq. (mu*)), returned as a [k, n_pix] array."""
    Yv = (prob.Y if Y is None else Y).ravel()
    b = design(prob).T @ (noise_precision(prob) @ Yv)
    return b.reshape(prob.k, prob.n_pix)


def apply(prob, X: np.ndarray, G=None) -> np.ndarray:
    """G vec(X) with the assembled sparse matrix; X is [k, n_pix] (or [..., k, n_pix])."""
    if G is None:
        G = posterior_precision(prob)
    Xm = np.asarray(X, dtype=np.float64)
    flat = Xm.reshape(-1, prob.k * prob.n_pix)
    out = (G @ flat.T).T
    return out.reshape(Xm.shape)


def apply_terms(prob, X: np.ndarray) -> np.ndarray:
    """Independent evaluation of G(X) = sum_j Q_j X E_jj + sum_f D_f X a_f a_f^T.

    Uses np.roll (periodic) or a zero-padded neighbour sum with counted links (face) for the
    Laplacian, applied twice, and an explicit per-frequency mixing sum, so a mistake in the
    Kronecker assembly does not cancel against it.
    """
    ny, nx, k = prob.ny, prob.nx, prob.k
    Xg = np.asarray(X, dtype=np.float64).reshape(k, ny, nx)
    out = np.zeros_like(Xg)
    face = boundary_of(prob) == "face"
    # face: neighbours outside the grid are absent; pad with zeros and count present links
    deg = None
    if face:
        one = np.pad(np.ones((ny, nx)), 1)
        deg = one[:-2, 1:-1] + one[2:, 1:-1] + one[1:-1, :-2] + one[1:-1, 2:]
    for j in range(k):
        u = Xg[j]

        def lap(v):
            if face:
                vp = np.pad(v, 1)
                return vp[:-2, 1:-1] + vp[2:, 1:-1] + vp[1:-1, :-2] + vp[1:-1, 2:] - deg * v
            return (np.roll(v, 1, axis=1) + np.roll(v, -1, axis=1) + np.roll(v, 1, axis=0)
                    + np.roll(v, -1, axis=0) - 4.0 * v)

        Lu = prob.kappa[j] ** 2 * u - lap(u)
        LLu = prob.kappa[j] ** 2 * Lu - lap(Lu)
        out[j] = prob.tau[j] * LLu
    Xp = Xg.reshape(k, -1)
    mix = np.zeros_like(Xp)
    for fi in range(prob.f):
        a = prob.A[fi]
        proj = a @ Xp  # a_f . x_p for every pixel
        mix += np.outer(a, prob.W[fi] * proj)
    return (out.reshape(k, -1) + mix)


def apply_at(prob, X: np.ndarray, pixels: np.ndarray) -> np.ndarray:
    """G(X) evaluated only at the given pixels (all k components): returns [k, len(pixels)].

    Builds each needed row of Q_j from the sparse product L^T L restricted to those rows, so it
    scales to full-size grids when only a sample of outputs is checked.
    """
    ny, nx, k = prob.ny, prob.nx, prob.k
    pixels = np.asarray(pixels, dtype=np.int64)
    Xp = np.asarray(X, dtype=np.float64).reshape(k, -1)
    out = np.zeros((k, len(pixels)))
    lap = laplacian(ny, nx, boundary_of(prob))
    n = ny * nx
    for j in range(k):
        L = (prob.kappa[j] ** 2 * sp.identity(n, format="csr") - lap).tocsr()
        rows = prob.tau[j] * (L.T.tocsr()[pixels] @ L)   # rows p of tau L^T L
        out[j] = rows @ Xp[j]
    for fi in range(prob.f):
        a = prob.A[fi]
        proj = a @ Xp[:, pixels]
        out += np.outer(a, prob.W[fi, pixels] * proj)
    return out
