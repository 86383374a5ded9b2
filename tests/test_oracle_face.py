"""Pins of the oracle's face boundary (one HEALPix base face: 4-neighbour links only inside the
grid, Section 3's D with minus the row sum on the diagonal, App. A and App. C), no GPU."""
import numpy as np
import pytest

from oracle import grad as og
from oracle import lanczos as olz
from oracle import operator as op
from oracle import pcg as opcg
from oracle import po as opo
from oracle import solve as osv
from workloads import make_problem


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) /
                 max(np.linalg.norm(np.asarray(b)), 1e-300))


def paper_D_face(ny, nx):
    """The paper's D by its definition, on one face: 1 between distinct pixels that share an
    edge inside the grid, minus the row sum on the diagonal; explicit loops over pixels."""
    n = ny * nx
    D = np.zeros((n, n))
    for iy in range(ny):
        for ix in range(nx):
            p = iy * nx + ix
            for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                jy, jx = iy + dy, ix + dx
                if 0 <= jy < ny and 0 <= jx < nx:
                    D[p, jy * nx + jx] = 1.0
            D[p, p] = -(D[p].sum())
    return D


def face_problem(ny, nx, k, f, seed, **kw):
    return make_problem(ny, nx, k, f, seed=seed, boundary="face", **kw)


@pytest.mark.parametrize("ny,nx", [(5, 6), (1, 7), (2, 2), (3, 1), (4, 4), (1, 1)])
def test_face_laplacian_is_paper_D(ny, nx):
    assert np.array_equal(op.laplacian(ny, nx, "face").toarray(), paper_D_face(ny, nx))


def test_face_laplacian_null_space_and_rank():
    """D 1 = 0 and rank N - 1 on a connected face; Q = phi D^2 has rank N - 1 (App. C)."""
    D = op.laplacian(6, 5, "face").toarray()
    n = D.shape[0]
    assert np.allclose(D @ np.ones(n), 0.0)
    ev = np.linalg.eigvalsh(D)
    assert np.sum(np.abs(ev) < 1e-10) == 1 and np.all(ev < 1e-10)
    Q0 = op.prior_block(6, 5, 0.0, 1.3, "face").toarray()
    assert np.linalg.matrix_rank(Q0, tol=1e-9) == n - 1


def test_face_prior_rows_closed_form():
    """Row p of tau (kappa^2 - D)^2 on a face: diagonal tau((kappa^2 + d_p)^2 + d_p); edge
    neighbour q: -tau(2 kappa^2 + d_p + d_q); diagonal neighbours 2 tau; distance-2 neighbours
    tau (d = number of in-face neighbours).  These are the per-pixel coefficients of the fused
    13-point stencil on a face."""
    ny, nx, kap, tau = 6, 7, 0.6, 1.7
    Q = op.prior_block(ny, nx, kap, tau, "face").toarray()
    k2 = kap * kap

    def deg(iy, ix):
        return (iy > 0) + (iy < ny - 1) + (ix > 0) + (ix < nx - 1)

    def inside(iy, ix):
        return 0 <= iy < ny and 0 <= ix < nx

    for iy in range(ny):
        for ix in range(nx):
            p = iy * nx + ix
            dp = deg(iy, ix)
            expect = np.zeros(ny * nx)
            expect[p] = tau * ((k2 + dp) ** 2 + dp)
            for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                if inside(iy + dy, ix + dx):
                    expect[(iy + dy) * nx + ix + dx] = -tau * (2 * k2 + dp + deg(iy + dy, ix + dx))
            for dy, dx in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
                if inside(iy + dy, ix + dx):
                    expect[(iy + dy) * nx + ix + dx] = 2 * tau
            for dy, dx in ((0, 2), (0, -2), (2, 0), (-2, 0)):
                if inside(iy + dy, ix + dx):
                    expect[(iy + dy) * nx + ix + dx] = tau
            assert np.allclose(Q[p], expect, rtol=1e-14, atol=1e-13), (iy, ix)


@pytest.mark.parametrize("ny,nx", [(7, 9), (1, 8), (4, 3)])
def test_face_kron_assembly_equals_sum_of_terms(ny, nx):
    p = face_problem(ny, nx, 3, 5, 4000 + ny, noise="hetero")
    X = np.random.default_rng(1).standard_normal((p.k, p.n_pix))
    assert rel(op.apply(p, X), op.apply_terms(p, X)) < 1e-13
    periodic = make_problem(ny, nx, 3, 5, seed=4000 + ny, noise="hetero")
    assert rel(op.apply(p, X), op.apply(periodic, X)) > 1e-6      # the boundary matters


def test_face_apply_at_matches_full():
    p = face_problem(12, 10, 3, 4, 4010, noise="hetero", mask_frac=0.1)
    X = np.random.default_rng(2).standard_normal((p.k, p.n_pix))
    pix = np.array([0, 9, 10, 55, 110, 119, 64])
    assert rel(op.apply_at(p, X, pix), op.apply(p, X)[:, pix]) < 1e-14


@pytest.mark.parametrize("mask", [0.0, 0.2])
def test_face_dense_and_pcg(mask):
    p = face_problem(10, 9, 3, 5, 4020, noise="hetero", mask_frac=mask)
    G = op.posterior_precision(p, dense=True)
    assert np.allclose(G, G.T) and np.linalg.eigvalsh(G).min() > 0
    xd = osv.solve_dense(p)
    assert rel(op.apply_terms(p, xd), op.rhs(p)) < 1e-13
    res = opcg.pcg(p, tol=1e-13, precond="block")
    assert rel(res["x"], xd) < 1e-10


def test_face_fourier_solve_refused():
    p = face_problem(8, 8, 2, 3, 4030, noise="homo")
    with pytest.raises(ValueError):
        osv.solve_fft(p)


def test_face_gradients_vs_central_differences():
    p = face_problem(5, 4, 2, 3, 4040, noise="hetero", mask_frac=0.15)
    xt = np.random.default_rng(4041).standard_normal((p.k, p.n_pix))
    g, _, _ = og.loss_grads(p, xt)
    for name, index in (("kappa", (0,)), ("kappa", (1,)), ("tau", (1,)), ("A", (2, 1)),
                        ("W", (1, 7)), ("Y", (0, 11))):
        fd = og.fd_grad(p, xt, name, index, h=1e-6)
        an = g[name][index]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, index, fd, an)


def test_face_perturbation_covariance():
    """H H^T == G for the perturbation map on a face (exact)."""
    p = face_problem(4, 5, 2, 3, 4050, noise="hetero", mask_frac=0.2)
    k, f, n = p.k, p.f, p.n_pix
    cols = []
    for i in range(k * n):
        xi = np.zeros(k * n)
        xi[i] = 1.0
        cols.append(opo.perturbation(p, xi.reshape(k, n), np.zeros((f, n))).ravel())
    for i in range(f * n):
        zeta = np.zeros(f * n)
        zeta[i] = 1.0
        cols.append(opo.perturbation(p, np.zeros((k, n)), zeta.reshape(f, n)).ravel())
    H = np.array(cols).T
    assert rel(H @ H.T, op.posterior_precision(p, dense=True)) < 1e-13


def test_face_sylvester_solvers_equal_dense():
    """Alg. 3 and Alg. 5 on a face (equal kappa, separable noise) against dense Cholesky."""
    p = make_problem(9, 8, 3, 5, seed=4060, noise="separable", kappa=np.full(3, 0.4),
                     boundary="face")
    t, n = p.meta["t"], p.meta["n"]
    xd = osv.solve_dense(p)
    assert rel(osv.solve_kohler(p, t, n), xd) < 1e-10
    res = olz.lanczos_sylvester(p, t, n, tol=1e-11, max_iter=300)
    assert res["converged"] and rel(res["x"], xd) < 1e-8
