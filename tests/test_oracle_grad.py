"""Pins of the oracle's adjoint gradients: central finite differences through dense solves and the
adjoint identity (no GPU)."""
import numpy as np
import pytest

from oracle import grad as og
from oracle import operator as op
from oracle import solve as osv
from workloads import make_problem


def _target(prob, seed):
    return np.random.default_rng(seed).standard_normal((prob.k, prob.n_pix))


def test_adjoint_identity():
    """<lambda, b> == <gbar, x*> because G is symmetric."""
    prob = make_problem(6, 7, 3, 4, seed=31, noise="hetero")
    gbar = np.random.default_rng(32).standard_normal((3, prob.n_pix))
    _, x, lam = og.adjoint_solution_grads(prob, gbar, return_solution=True)
    b = op.rhs(prob)
    assert abs(np.vdot(lam, b) - np.vdot(gbar, x)) < 1e-12 * abs(np.vdot(gbar, x))


def test_all_gradients_vs_central_differences_small():
    prob = make_problem(5, 4, 2, 3, seed=33, noise="hetero", mask_frac=0.15)
    xt = _target(prob, 34)
    g, _, _ = og.loss_grads(prob, xt)
    for name in ("kappa", "tau", "A", "W", "Y"):
        arr = np.asarray(getattr(prob, name))
        for index in itertools_indices(arr.shape, limit=10, seed=35):
            fd = og.fd_grad(prob, xt, name, index, h=1e-6)
            an = g[name][index]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, index, fd, an)


def itertools_indices(shape, limit, seed):
    rng = np.random.default_rng(seed)
    total = int(np.prod(shape))
    flat = rng.choice(total, size=min(limit, total), replace=False)
    return [np.unravel_index(i, shape) if len(shape) > 1 else (int(i),) for i in flat]


@pytest.mark.slow
def test_gradients_vs_central_differences_32():
    """The differentiable workload's shape reduced to 32 x 32 (k = 4, f = 9)."""
    prob = make_problem(32, 32, 4, 9, seed=36, noise="hetero")
    xt = _target(prob, 37)
    g, _, _ = og.loss_grads(prob, xt)
    checks = [("kappa", (j,)) for j in range(4)] + [("tau", (j,)) for j in range(4)]
    checks += [("A", (0, 0)), ("A", (8, 3)), ("A", (4, 2)), ("W", (2, 100)), ("W", (7, 1023))]
    for name, index in checks:
        fd = og.fd_grad(prob, xt, name, index, h=1e-6)
        an = g[name][index]
        assert abs(fd - an) <= 2e-6 * max(1.0, abs(an)), (name, index, fd, an)


def test_homoscedastic_gradient_consistent_with_fft_solve():
    """d<gbar, x*>/dtau_j from the adjoint formula equals a finite difference of the
    independent Fourier solve (a second solver, not the dense one)."""
    prob = make_problem(8, 8, 3, 5, seed=38, noise="homo")
    gbar = np.random.default_rng(39).standard_normal((3, prob.n_pix))
    g = og.adjoint_solution_grads(prob, gbar)
    for j in range(3):
        h = 1e-6
        import copy
        pp = copy.deepcopy(prob)
        pm = copy.deepcopy(prob)
        pp.tau[j] += h
        pm.tau[j] -= h
        fd = (np.vdot(gbar, osv.solve_fft(pp)) - np.vdot(gbar, osv.solve_fft(pm))) / (2 * h)
        assert abs(fd - g["tau"][j]) < 1e-6 * max(1.0, abs(fd))
        pp = copy.deepcopy(prob)
        pm = copy.deepcopy(prob)
        pp.kappa[j] += h
        pm.kappa[j] -= h
        fd = (np.vdot(gbar, osv.solve_fft(pp)) - np.vdot(gbar, osv.solve_fft(pm))) / (2 * h)
        assert abs(fd - g["kappa"][j]) < 1e-6 * max(1.0, abs(fd))
