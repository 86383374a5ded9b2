"""Gradients of a loss of the posterior mean (oracle; tests only).

x*(theta) solves G(theta) x* = b(theta) with theta = (kappa, tau, A, W, Y).  For a loss
ell(x*, theta) the adjoint method gives

  d ell / d theta = d ell / d theta |_(x* fixed) + lambda^T (db/dtheta - dG/dtheta x*),
  G lambda = d ell / d x*            (G is symmetric, so the adjoint solve uses G itself).

Here every dG/dtheta and db/dtheta is assembled as an explicit sparse matrix from the same
Kronecker factors as the forward operator (eq. (Q*), eq. (mu*)):
  dG/dtau_j   = E_jj (x) L_j^T L_j
  dG/dkappa_j = E_jj (x) tau_j (dL^T L + L^T dL),   dL = d L_j / d kappa_j = 2 kappa_j I
  dG/dA[f,j]  = (e_j a_f^T + a_f e_j^T) (x) diag(W_f),   db/dA[f,j] = e_j (x) (W_f * Y_f)
  dG/dW[f,p]  = (a_f a_f^T) (x) e_p e_p^T,                db/dW[f,p] = Y[f,p] (a_f (x) e_p)
  db/dY       = B^T C
and the contractions are taken literally.  Central finite differences of the full loss through
dense solves pin these formulas.
"""
from __future__ import annotations

import copy

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import operator as op
from . import solve as slv


def implicit_grads(prob, x, lam):
    """lambda^T (db/dtheta - dG/dtheta x) for every parameter, given x* and lambda ([k, n_pix])."""
    k, f, n_pix = prob.k, prob.f, prob.n_pix
    xv = np.asarray(x, dtype=np.float64).ravel()
    lv = np.asarray(lam, dtype=np.float64).ravel()
    out = {}
    dkap = np.zeros(k)
    dtau = np.zeros(k)
    I = sp.identity(n_pix, format="csr")
    for j in range(k):
        E = np.zeros((k, k))
        E[j, j] = 1.0
        E = sp.csr_matrix(E)
        L = op.prior_factor(prob.ny, prob.nx, prob.kappa[j], op.boundary_of(prob))
        dG_tau = sp.kron(E, (L.T @ L))
        dL = 2.0 * prob.kappa[j] * I
        dG_kap = sp.kron(E, prob.tau[j] * (dL.T @ L + L.T @ dL))
        dtau[j] = -lv @ (dG_tau @ xv)
        dkap[j] = -lv @ (dG_kap @ xv)
    out["kappa"] = dkap
    out["tau"] = dtau
    dA = np.zeros((f, k))
    for fi in range(f):
        a = prob.A[fi]
        Df = sp.diags(prob.W[fi])
        for j in range(k):
            e = np.zeros(k)
            e[j] = 1.0
            dG = sp.kron(sp.csr_matrix(np.outer(e, a) + np.outer(a, e)), Df)
            db = sp.kron(sp.csr_matrix(e[:, None]), sp.identity(n_pix)) @ (
                prob.W[fi] * prob.Y[fi])
            dA[fi, j] = lv @ db - lv @ (dG @ xv)
    out["A"] = dA
    # W: dG/dW[f,p] x = a_f (a_f . x_p) e_p ;  db/dW[f,p] = Y[f,p] a_f e_p.  The operator
    # (a_f^T (x) I_N) maps a stacked vector to the per-pixel projection onto a_f.
    dW = np.zeros((f, n_pix))
    for fi in range(f):
        proj = sp.kron(sp.csr_matrix(prob.A[fi][None, :]), sp.identity(n_pix)).tocsr()
        la = proj @ lv
        xa = proj @ xv
        dW[fi] = la * prob.Y[fi] - la * xa
    out["W"] = dW
    B = op.design(prob)
    C = op.noise_precision(prob)
    out["Y"] = (C @ (B @ lv)).reshape(f, n_pix)
    return out


def adjoint_solution_grads(prob, gbar, return_solution=False):
    """Gradient of theta -> <gbar, x*(theta)> by the adjoint method with dense Cholesky solves."""
    x, fac = slv.solve_dense(prob, return_factor=True)
    lam = sla.cho_solve(fac, np.asarray(gbar, dtype=np.float64).ravel()).reshape(prob.k, -1)
    g = implicit_grads(prob, x, lam)
    if return_solution:
        return g, x, lam
    return g


# ---- the differentiable-solve workload's loss ------------------------------------------------
# loss = ||x* - X_t||_F^2 + 1/2 sum_{f,p} W[f,p] (Y[f,p] - a_f . x*_p)^2
# (squared error to a target plus the data-misfit quadratic of the likelihood, eq. (likelihood)).

def loss_value(prob, x, x_target):
    resid = prob.Y - prob.A @ np.asarray(x).reshape(prob.k, -1)
    return float(np.sum((x - x_target) ** 2) + 0.5 * np.sum(prob.W * resid * resid))


def loss_partials(prob, x, x_target):
    """(d loss/d x*, explicit partials of the loss with x* held fixed)."""
    x = np.asarray(x).reshape(prob.k, -1)
    resid = prob.Y - prob.A @ x                     # [f, n_pix]
    gx = 2.0 * (x - x_target) - prob.A.T @ (prob.W * resid)
    part = {
        "kappa": np.zeros(prob.k),
        "tau": np.zeros(prob.k),
        "A": -(prob.W * resid) @ x.T,              # d/dA[f,j] of 1/2 sum W r^2 = -sum_p W r x_j
        "W": 0.5 * resid * resid,
        "Y": prob.W * resid,
    }
    return gx, part


def loss_grads(prob, x_target):
    """Total gradient of the loss w.r.t. (kappa, tau, A, W, Y) via adjoint + explicit terms."""
    x, fac = slv.solve_dense(prob, return_factor=True)
    gx, part = loss_partials(prob, x, x_target)
    lam = sla.cho_solve(fac, gx.ravel()).reshape(prob.k, -1)
    imp = implicit_grads(prob, x, lam)
    return {key: imp[key] + part[key] for key in imp}, x, lam


def loss_of(prob, x_target):
    return loss_value(prob, slv.solve_dense(prob), x_target)


def fd_grad(prob, x_target, name, index, h=1e-6):
    """Central difference of the loss w.r.t. one entry of parameter `name` (relative step)."""
    def with_value(delta):
        q = copy.deepcopy(prob)
        arr = getattr(q, name)
        arr[index] = arr[index] + delta
        return loss_of(q, x_target)

    base = float(np.asarray(getattr(prob, name))[index])
    step = h * max(1.0, abs(base))
    return (with_value(step) - with_value(-step)) / (2.0 * step)
