"""Perturbation-optimisation right-hand sides (oracle; tests only).

Sampling the posterior N(x*, G^-1) of Section 2.2 by perturbing the right-hand side: with
independent standard-normal xi (one per prior component) and zeta (one per map),

  eta = H_Q xi + H_C zeta,   H_Q = bldiag(sqrt(tau_j) L_j^T),   H_C = B^T C^(1/2)

has covariance H_Q H_Q^T + H_C H_C^T = Q + B^T C B = G, so x = G^-1 (B^T C Y + eta) is an exact
posterior draw.  This is not in the paper (which computes only the mean); it is the standard way
to turn the same linear solve into a sampler.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import operator as op


def prior_root(prob) -> sp.csr_matrix:
    blocks = [np.sqrt(prob.tau[j]) * op.prior_factor(prob.ny, prob.nx, prob.kappa[j],
                                                     op.boundary_of(prob)).T
              for j in range(prob.k)]
    return sp.block_diag(blocks, format="csr")


def likelihood_root(prob) -> sp.csr_matrix:
    return (op.design(prob).T @ sp.diags(np.sqrt(prob.W.ravel()))).tocsr()


def perturbation(prob, xi, zeta) -> np.ndarray:
    """eta for one draw (xi [k, n_pix], zeta [f, n_pix]) or a batch ([s, k, n_pix], [s, f, n_pix])."""
    xi = np.asarray(xi, dtype=np.float64)
    zeta = np.asarray(zeta, dtype=np.float64)
    HQ = prior_root(prob)
    HC = likelihood_root(prob)
    if xi.ndim == 2:
        return (HQ @ xi.ravel() + HC @ zeta.ravel()).reshape(prob.k, prob.n_pix)
    s = xi.shape[0]
    eta = (HQ @ xi.reshape(s, -1).T + HC @ zeta.reshape(s, -1).T).T
    return eta.reshape(s, prob.k, prob.n_pix)
