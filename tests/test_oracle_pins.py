"""Pins of the CPU oracle against mathematics and the paper (no GPU).

Each test checks the oracle against something other than itself: a textbook identity, a closed
form, the paper's own formulas written independently (Section 3.1 Kronecker forms, Lemma 1,
Lemma 2), brute force on tiny inputs, or an independent solver.
"""
import itertools
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import operator as op
from oracle import pcg as opcg
from oracle import po as opo
from oracle import solve as osv
from workloads import make_problem

HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def paper_D(ny, nx):
    """The paper's D by its definition (Section 3): 1 between distinct 4-neighbours, minus the
    row sum on the diagonal, built with explicit loops over pixels (needs ny, nx >= 3 so the four
    neighbours are distinct pixels)."""
    n = ny * nx
    D = np.zeros((n, n))
    for iy in range(ny):
        for ix in range(nx):
            p = iy * nx + ix
            for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                q = ((iy + dy) % ny) * nx + (ix + dx) % nx
                D[p, q] = 1.0
            D[p, p] = -(D[p].sum())
    return D


# ---------------------------------------------------------------- Kronecker conventions

def test_vec_kron_identity_brute_force():
    """vec(A X B) = (B^T (x) A) vec(X) with column-major vec, checked entry by entry."""
    rng = np.random.default_rng(0)
    for (m, n, p, q) in [(2, 3, 3, 2), (4, 1, 1, 5), (3, 3, 3, 3)]:
        A = rng.standard_normal((m, n))
        X = rng.standard_normal((n, p))
        B = rng.standard_normal((p, q))
        AXB = np.zeros((m, q))
        for i in range(m):
            for j in range(q):
                AXB[i, j] = sum(A[i, a] * X[a, b] * B[b, j] for a in range(n) for b in range(p))
        lhs = AXB.ravel(order="F")
        rhs = np.kron(B.T, A) @ X.ravel(order="F")
        assert rel(rhs, lhs) < 1e-14


@pytest.mark.parametrize("shape", [(5, 6, 3, 4), (3, 3, 2, 2), (4, 7, 1, 3)])
def test_operator_is_sum_of_matrix_terms(shape):
    """G vec(X) == vec(sum_j Q_j X E_jj + sum_f D_f X a_f a_f^T) with X an N x k matrix."""
    ny, nx, k, f = shape
    prob = make_problem(ny, nx, k, f, seed=7)
    N = prob.n_pix
    Xm = np.random.default_rng(1).standard_normal((N, k))      # columns = components
    out = np.zeros((N, k))
    for j in range(k):
        E = np.zeros((k, k))
        E[j, j] = 1.0
        Qj = op.prior_block(ny, nx, prob.kappa[j], prob.tau[j]).toarray()
        out += Qj @ Xm @ E
    for fi in range(f):
        a = prob.A[fi][:, None]
        out += np.diag(prob.W[fi]) @ Xm @ (a @ a.T)
    G = op.posterior_precision(prob, dense=True)
    assert rel(G @ Xm.ravel(order="F"), out.ravel(order="F")) < 1e-14


@pytest.mark.parametrize("ny,nx", [(1, 1), (1, 3), (2, 2), (2, 5), (3, 4), (4, 4), (5, 5),
                                   (8, 6), (7, 9)])
def test_kron_assembly_equals_sum_of_terms(ny, nx):
    prob = make_problem(ny, nx, 3, 4, seed=11)
    X = np.random.default_rng(2).standard_normal((3, prob.n_pix))
    assert rel(op.apply(prob, X), op.apply_terms(prob, X)) < 1e-13


def test_apply_at_matches_full_apply():
    prob = make_problem(9, 13, 4, 5, seed=3, noise="hetero", mask_frac=0.2)
    X = np.random.default_rng(4).standard_normal((4, prob.n_pix))
    full = op.apply(prob, X)
    pix = np.array([0, 5, 12, 13, 50, 116])
    assert rel(op.apply_at(prob, X, pix), full[:, pix]) < 1e-14


# ---------------------------------------------------------------- prior block: closed forms

@pytest.mark.parametrize("ny,nx", [(6, 8), (5, 7), (1, 4), (2, 3)])
def test_prior_fourier_eigenpairs(ny, nx):
    """Q = tau (kappa^2 - Lap)^2 has the real Fourier modes as eigenvectors with eigenvalue
    tau (kappa^2 + lam)^2, lam = 4 - 2 cos(2 pi u/nx) - 2 cos(2 pi v/ny)."""
    kappa, tau = 0.7, 1.3
    Q = op.prior_block(ny, nx, kappa, tau)
    iy, ix = np.divmod(np.arange(ny * nx), nx)
    for u in range(nx):
        for v in range(ny):
            lam = 4 - 2 * np.cos(2 * np.pi * u / nx) - 2 * np.cos(2 * np.pi * v / ny)
            ev = tau * (kappa ** 2 + lam) ** 2
            for phase in (0.0, np.pi / 2):
                mode = np.cos(2 * np.pi * (u * ix / nx + v * iy / ny) + phase)
                if np.linalg.norm(mode) < 1e-12:
                    continue
                assert rel(Q @ mode, ev * mode) < 1e-12


def test_prior_constant_vector_and_rank():
    """Q 1 = tau kappa^4 1; with kappa = 0 the prior has rank N - 1 (App. C)."""
    ny, nx = 6, 5
    one = np.ones(ny * nx)
    Q = op.prior_block(ny, nx, 0.8, 1.7)
    assert rel(Q @ one, 1.7 * 0.8 ** 4 * one) < 1e-13
    Q0 = op.prior_block(ny, nx, 0.0, 1.0).toarray()
    assert np.max(np.abs(Q0 @ one)) < 1e-12
    ev = np.linalg.eigvalsh(Q0)
    assert np.sum(ev < 1e-10) == 1
    assert np.linalg.matrix_rank(Q0) == ny * nx - 1


@pytest.mark.parametrize("ny,nx", [(3, 3), (4, 5), (6, 6)])
def test_laplacian_is_paper_D(ny, nx):
    assert np.array_equal(op.laplacian(ny, nx).toarray(), paper_D(ny, nx))


def test_thirteen_point_support():
    """On a grid of side >= 5, row p of Q has exactly 13 nonzeros: centre, 4 neighbours,
    4 diagonals and 4 at distance 2 (the (kappa^2 - Lap)^2 stencil)."""
    Q = op.prior_block(9, 11, 0.5, 1.0).tocsr()
    assert all(Q[p].nnz == 13 for p in range(0, 99, 7))


# ---------------------------------------------------------------- the paper's Kronecker forms

def test_separable_case_equals_paper_kronecker_form():
    """kappa = 0, W = T (x) N: G == P (x) D^2 + (A^T T A) (x) N (Section 3.1), with D built
    from the paper's definition and P = diag(phi)."""
    ny, nx, k, f = 4, 5, 3, 4
    rng = np.random.default_rng(5)
    t = rng.uniform(0.5, 2.0, f)
    nvec = rng.integers(1, 5, ny * nx).astype(float)       # the paper's positive integers n_i
    phi = rng.uniform(0.5, 2.0, k)
    prob = make_problem(ny, nx, k, f, seed=5, kappa=np.zeros(k), tau=phi)
    prob.W = np.outer(t, nvec)
    D = paper_D(ny, nx)
    P = np.diag(phi)
    T = np.diag(t)
    N = np.diag(nvec)
    G_paper = np.kron(P, D @ D) + np.kron(prob.A.T @ T @ prob.A, N)
    G = op.posterior_precision(prob, dense=True)
    assert rel(G, G_paper) < 1e-14
    # and B^T C B assembled literally from B = A (x) I, C = T (x) N
    B = np.kron(prob.A, np.eye(ny * nx))
    C = np.kron(T, N)
    assert rel(op.likelihood_term(prob).toarray(), B.T @ C @ B) < 1e-14


def test_block_vector_mapping():
    """Mixing part applied to M (N x k) equals N (M A^T) T A -- the block map of Section 3.1."""
    ny, nx, k, f = 5, 4, 4, 6
    rng = np.random.default_rng(6)
    t = rng.uniform(0.5, 2.0, f)
    nvec = rng.uniform(0.5, 3.0, ny * nx)
    prob = make_problem(ny, nx, k, f, seed=6)
    prob.W = np.outer(t, nvec)
    M = rng.standard_normal((ny * nx, k))
    mapped = np.diag(nvec) @ (M @ prob.A.T) @ np.diag(t) @ prob.A
    mix = op.likelihood_term(prob) @ M.ravel(order="F")
    assert rel(mix, mapped.ravel(order="F")) < 1e-14


def test_mixing_single_pixel_loops():
    """Mixing at one pixel by explicit loops: out_i = sum_f W[f,p] A[f,i] sum_j A[f,j] x_j."""
    prob = make_problem(3, 3, 3, 5, seed=8)
    X = np.random.default_rng(9).standard_normal((3, 9))
    full = op.likelihood_term(prob) @ X.ravel()
    full = full.reshape(3, 9)
    for p in (0, 4, 8):
        for i in range(3):
            s = 0.0
            for fi in range(5):
                for j in range(3):
                    s += prob.W[fi, p] * prob.A[fi, i] * prob.A[fi, j] * X[j, p]
            assert abs(full[i, p] - s) < 1e-13 * max(1.0, abs(s))


def test_rhs_loops():
    prob = make_problem(4, 3, 3, 5, seed=10, noise="hetero", mask_frac=0.3)
    b = op.rhs(prob)
    for p in range(prob.n_pix):
        for j in range(3):
            s = sum(prob.W[fi, p] * prob.Y[fi, p] * prob.A[fi, j] for fi in range(5))
            assert abs(b[j, p] - s) < 1e-13 * max(1.0, abs(s))


def test_lemma1_lemma2_symmetries():
    """Lemma 1: N^-1 D^2 symmetric in <.,.>_N.  Lemma 2: Lhat = A^T T A P^-1 symmetric in
    <.,.>_{P^-1}, hence real eigenvalues."""
    rng = np.random.default_rng(12)
    D = op.laplacian(5, 6).toarray()
    nvec = rng.uniform(0.5, 3.0, 30)
    N = np.diag(nvec)
    H = np.linalg.inv(N) @ D @ D
    x, y = rng.standard_normal(30), rng.standard_normal(30)
    assert abs(y @ N @ (H @ x) - (H @ y) @ N @ x) < 1e-10 * abs(y @ N @ (H @ x)) + 1e-12
    A = rng.uniform(0.2, 1.5, (9, 4))
    T = np.diag(rng.uniform(0.5, 2, 9))
    Pinv = np.diag(1.0 / rng.uniform(0.5, 2, 4))
    Lh = A.T @ T @ A @ Pinv
    u, v = rng.standard_normal(4), rng.standard_normal(4)
    assert abs(v @ Pinv @ (Lh @ u) - (Lh @ v) @ Pinv @ u) < 1e-12
    assert np.max(np.abs(np.linalg.eigvals(Lh).imag)) == 0.0


# ---------------------------------------------------------------- SPD and exact solves

@pytest.mark.parametrize("noise,mask", [("homo", 0.0), ("hetero", 0.0), ("hetero", 0.3)])
def test_symmetric_positive_definite(noise, mask):
    prob = make_problem(8, 7, 3, 5, seed=13, noise=noise, mask_frac=mask)
    G = op.posterior_precision(prob, dense=True)
    assert np.array_equal(G, G.T)
    assert np.linalg.eigvalsh(G).min() > 0
    sla.cho_factor(G)


def test_fully_masked_kappa_zero_is_singular():
    """Q is only semi-definite: with every weight 0 and kappa = 0, G = Q has the constants in
    its null space (App. C)."""
    prob = make_problem(4, 4, 2, 3, seed=14, kappa=np.zeros(2))
    prob.W[:] = 0.0
    G = op.posterior_precision(prob, dense=True)
    assert np.linalg.eigvalsh(G).min() < 1e-10


@pytest.mark.parametrize("shape", [(8, 8, 3, 6), (16, 12, 4, 9), (1, 1, 2, 3), (2, 7, 3, 4)])
def test_dense_solution_residual(shape):
    ny, nx, k, f = shape
    prob = make_problem(ny, nx, k, f, seed=15, noise="hetero")
    x = osv.solve_dense(prob)
    b = op.rhs(prob)
    assert rel(op.apply_terms(prob, x), b) < 1e-13


@pytest.mark.parametrize("shape", [(8, 8, 3, 6), (12, 16, 4, 9), (1, 5, 2, 3), (3, 2, 3, 4)])
def test_fft_equals_dense(shape):
    ny, nx, k, f = shape
    prob = make_problem(ny, nx, k, f, seed=16, noise="homo")
    assert rel(osv.solve_fft(prob), osv.solve_dense(prob)) < 1e-12


@pytest.mark.parametrize("shape", [(8, 8, 3, 6), (6, 10, 4, 9), (1, 5, 2, 3), (4, 3, 1, 2)])
def test_condition_number_equals_dense_spectrum(shape):
    """cond_2(G) from the per-mode Fourier blocks equals the ratio of the extreme eigenvalues of
    the explicitly assembled G (LAPACK dsyevd on the dense Kronecker matrix)."""
    ny, nx, k, f = shape
    prob = make_problem(ny, nx, k, f, seed=20 + ny, noise="homo")
    ev = np.linalg.eigvalsh(op.posterior_precision(prob, dense=True))
    assert osv.condition_number_fft(prob) == pytest.approx(ev.max() / ev.min(), rel=1e-10)


def test_fft_exact_at_1024():
    """The Fourier solve is exact at full size: its residual under the independently
    written sum-of-terms operator is at rounding level."""
    prob = make_problem(256, 256, 3, 9, seed=17, noise="homo")
    x = osv.solve_fft(prob)
    assert rel(op.apply_terms(prob, x), op.rhs(prob)) < 1e-13


def test_kohler_equals_dense():
    ny, nx, k, f = 10, 9, 3, 5
    rng = np.random.default_rng(18)
    t = rng.uniform(0.5, 2.0, f)
    nvec = rng.integers(1, 6, ny * nx).astype(float)
    prob = make_problem(ny, nx, k, f, seed=18, kappa=np.full(k, 0.4))
    prob.W = np.outer(t, nvec)
    assert rel(osv.solve_kohler(prob, t, nvec), osv.solve_dense(prob)) < 1e-11


def test_kohler_with_printed_planck_constants():
    """The paper's printed A and T (App. B): a separable, kappa = 0 problem whose mixing term is
    ~1e7 times the prior; Alg. 3 and dense Cholesky agree."""
    A, T = [], None
    with open(os.path.join(HERE, "golden", "planck_mixing.txt")) as fh:
        for line in fh:
            if line.startswith("A "):
                A.append([float(v) for v in line.split()[1:]])
            elif line.startswith("T "):
                T = np.array([float(v) for v in line.split()[1:]])
    A = np.array(A)
    assert A.shape == (9, 4) and T.shape == (9,)
    assert np.all(A[:, 0] == 1.0)                 # CMB column is all ones (App. B)
    assert np.all(A[3, 1:] == 1.006)              # reference frequency: power laws equal 1
    ny, nx = 6, 6
    nvec = np.random.default_rng(19).integers(1, 4, ny * nx).astype(float)
    prob = make_problem(ny, nx, 4, 9, seed=19, kappa=np.zeros(4), tau=np.ones(4), A=A)
    prob.W = np.outer(T, nvec)
    xd = osv.solve_dense(prob)
    xk = osv.solve_kohler(prob, T, nvec)
    assert rel(xk, xd) < 1e-8
    assert rel(op.apply(prob, xd), op.rhs(prob)) < 1e-12


# ---------------------------------------------------------------- PCG

def test_pcg_iterates_are_krylov_minimisers():
    """Iterate j of PCG minimises ||x - x*||_G over x0 + K_j(Minv G, Minv r0) (Section 3.2)."""
    prob = make_problem(4, 4, 3, 4, seed=20, noise="hetero")
    G = op.posterior_precision(prob, dense=True)
    b = op.rhs(prob).ravel()
    Minv, inv = opcg.block_jacobi(prob, kind="block")
    xs = np.linalg.solve(G, b)
    x0 = np.random.default_rng(21).standard_normal(b.size) * 0.1
    res = opcg.pcg(prob, b=b, x0=x0, tol=1e-30, max_iter=6, record=True)
    r0 = b - G @ x0

    def Mv(v):
        return Minv(v.reshape(prob.k, -1)).ravel()

    for j in range(1, 7):
        V = [Mv(r0)]
        for _ in range(j - 1):
            V.append(Mv(G @ V[-1]))
        V, _ = np.linalg.qr(np.array(V).T)
        c = np.linalg.solve(V.T @ G @ V, V.T @ (b - G @ x0))
        xj = x0 + V @ c
        assert rel(res["iterates"][j].ravel(), xj) < 1e-9
        # and it beats any other point of the affine space in the G-norm
        e_best = (xj - xs) @ G @ (xj - xs)
        other = xj + V @ np.random.default_rng(j).standard_normal(V.shape[1]) * 1e-3
        assert (other - xs) @ G @ (other - xs) > e_best


def test_pcg_finite_termination():
    prob = make_problem(3, 3, 2, 3, seed=22)
    res = opcg.pcg(prob, tol=1e-13, max_iter=200, precond="none")
    assert res["iters"] <= prob.n + 4
    assert res["relres_true"] < 1e-12


@pytest.mark.parametrize("precond", ["none", "jacobi", "block"])
def test_pcg_matches_dense(precond):
    prob = make_problem(16, 16, 3, 6, seed=23, noise="hetero", mask_frac=0.1)
    res = opcg.pcg(prob, tol=1e-13, precond=precond)
    assert rel(res["x"], osv.solve_dense(prob)) < 1e-10


def test_block_jacobi_blocks_are_inverse():
    prob = make_problem(5, 6, 4, 7, seed=24)
    G = op.posterior_precision(prob, dense=True)
    _, inv = opcg.block_jacobi(prob, kind="block")
    n = prob.n_pix
    for p in (0, 7, 29):
        blk = G[np.ix_([j * n + p for j in range(4)], [j * n + p for j in range(4)])]
        assert rel(inv[p] @ blk, np.eye(4)) < 1e-13


# ---------------------------------------------------------------- perturbation sampling

def test_po_covariance_identity():
    """H H^T == G for the perturbation map (exact, not statistical)."""
    prob = make_problem(4, 5, 3, 4, seed=25, noise="hetero", mask_frac=0.2)
    k, f, n = prob.k, prob.f, prob.n_pix
    cols = []
    for i in range(k * n):
        xi = np.zeros(k * n)
        xi[i] = 1.0
        cols.append(opo.perturbation(prob, xi.reshape(k, n), np.zeros((f, n))).ravel())
    for i in range(f * n):
        zeta = np.zeros(f * n)
        zeta[i] = 1.0
        cols.append(opo.perturbation(prob, np.zeros((k, n)), zeta.reshape(f, n)).ravel())
    H = np.array(cols).T
    G = op.posterior_precision(prob, dense=True)
    assert rel(H @ H.T, G) < 1e-13


def test_po_sample_statistics():
    prob = make_problem(3, 3, 2, 3, seed=26, noise="hetero")
    s = 20000
    rng = np.random.default_rng(27)
    xi = rng.standard_normal((s, prob.k, prob.n_pix))
    zeta = rng.standard_normal((s, prob.f, prob.n_pix))
    eta = opo.perturbation(prob, xi, zeta)
    G = op.posterior_precision(prob, dense=True)
    b = op.rhs(prob).ravel()
    X = np.linalg.solve(G, (b[None, :] + eta.reshape(s, -1)).T).T
    xs = np.linalg.solve(G, b)
    cov = np.cov(X.T)
    Ginv = np.linalg.inv(G)
    sd = np.sqrt(np.diag(Ginv))
    assert np.max(np.abs(X.mean(0) - xs) / sd) < 5.0 / np.sqrt(s) * 1.5
    assert rel(cov, Ginv) < 0.05


# ---- Fourier preconditioner (Q + I (x) Mbar)^-1 ----------------------------------------------

@pytest.mark.parametrize("shape", [(8, 8), (6, 10), (5, 3), (1, 7)])
def test_fourier_preconditioner_inverts_homoscedastic_operator(shape):
    """With W independent of the pixel, Mbar = M_p and the preconditioner is G^-1: the sparse
    assembled operator undoes it (odd, even and degenerate grid sides)."""
    p = make_problem(shape[0], shape[1], 3, 5, seed=9000 + shape[0], noise="homo")
    Minv = opcg.fourier_preconditioner(p)
    R = np.random.default_rng(9001).standard_normal((p.k, p.n_pix))
    Z = Minv(R)
    assert np.linalg.norm(op.apply(p, Z) - R) <= 1e-11 * np.linalg.norm(R)


def test_fourier_preconditioner_uses_pixel_mean_of_weights():
    """For heteroscedastic W the preconditioner is the inverse operator of the problem whose
    weights are the per-map pixel means."""
    p = make_problem(7, 9, 4, 6, seed=9010, noise="hetero", mask_frac=0.2)
    q = make_problem(7, 9, 4, 6, seed=9010, noise="hetero", mask_frac=0.2)
    q.W = np.repeat(p.W.mean(axis=1, keepdims=True), p.n_pix, axis=1)
    R = np.random.default_rng(9011).standard_normal((p.k, p.n_pix))
    Z = opcg.fourier_preconditioner(p)(R)
    assert np.linalg.norm(op.apply(q, Z) - R) <= 1e-11 * np.linalg.norm(R)
    assert np.linalg.norm(op.apply(p, Z) - R) > 1e-3 * np.linalg.norm(R)   # not G^-1 itself


def test_fourier_preconditioner_symmetric_positive_definite():
    p = make_problem(5, 4, 2, 3, seed=9020, noise="hetero", mask_frac=0.1)
    Minv = opcg.fourier_preconditioner(p)
    n = p.k * p.n_pix
    P = np.array([Minv(np.eye(n)[i].reshape(p.k, p.n_pix)).ravel() for i in range(n)]).T
    assert np.abs(P - P.T).max() <= 1e-13 * np.abs(P).max()
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0


def test_fourier_pcg_matches_dense_in_fewer_iterations():
    p = make_problem(32, 32, 3, 6, seed=9030, noise="hetero", mask_frac=0.1)
    xd = osv.solve_dense(p)
    rf = opcg.pcg(p, tol=1e-11, precond="fourier")
    rb = opcg.pcg(p, tol=1e-11, precond="block")
    assert np.linalg.norm(rf["x"] - xd) <= 1e-8 * np.linalg.norm(xd)
    assert rf["iters"] < rb["iters"] / 2, (rf["iters"], rb["iters"])


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_path_laplacian_cosine_eigenpairs(n):
    """The face grid's Laplacian along one side is a path-graph Laplacian; the cosines
    cos(pi u (i + 1/2) / n) are its eigenvectors with eigenvalue 2 - 2 cos(pi u / n) (brute
    force on a 1 x n face)."""
    L = -op.laplacian(1, n, "face").toarray()
    i = np.arange(n)
    for u in range(n):
        v = np.cos(np.pi * u * (i + 0.5) / n)
        assert np.linalg.norm(L @ v - (2 - 2 * np.cos(np.pi * u / n)) * v) <= 1e-13 * n


@pytest.mark.parametrize("shape", [(8, 8), (6, 10), (5, 3), (1, 7), (2, 2)])
def test_cosine_preconditioner_inverts_homoscedastic_face_operator(shape):
    """On a face grid the preconditioner works in the cosine basis; with W independent of the
    pixel it is G^-1 of the assembled face operator."""
    p = make_problem(shape[0], shape[1], 3, 5, seed=9040 + shape[0], noise="homo",
                     boundary="face")
    R = np.random.default_rng(9041).standard_normal((p.k, p.n_pix))
    Z = opcg.fourier_preconditioner(p)(R)
    G = op.posterior_precision(p)
    assert np.linalg.norm((G @ Z.ravel()).reshape(p.k, p.n_pix) - R) <= 1e-11 * np.linalg.norm(R)


def test_cosine_preconditioner_face_spd_and_pixel_mean():
    p = make_problem(5, 4, 2, 3, seed=9050, noise="hetero", mask_frac=0.1, boundary="face")
    Minv = opcg.fourier_preconditioner(p)
    n = p.k * p.n_pix
    P = np.array([Minv(np.eye(n)[i].reshape(p.k, p.n_pix)).ravel() for i in range(n)]).T
    assert np.abs(P - P.T).max() <= 1e-13 * np.abs(P).max()
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0
    q = make_problem(5, 4, 2, 3, seed=9050, noise="hetero", mask_frac=0.1, boundary="face")
    q.W = np.repeat(p.W.mean(axis=1, keepdims=True), p.n_pix, axis=1)
    R = np.random.default_rng(9051).standard_normal((p.k, p.n_pix))
    assert np.linalg.norm(op.apply(q, Minv(R)) - R) <= 1e-11 * np.linalg.norm(R)


def test_cosine_pcg_on_face_grid_matches_dense_in_fewer_iterations():
    p = make_problem(32, 24, 3, 6, seed=9060, noise="hetero", mask_frac=0.1, boundary="face")
    xd = osv.solve_dense(p)
    rf = opcg.pcg(p, tol=1e-11, precond="fourier")
    rb = opcg.pcg(p, tol=1e-11, precond="block")
    assert np.linalg.norm(rf["x"] - xd) <= 1e-8 * np.linalg.norm(xd)
    assert rf["iters"] < rb["iters"] / 2, (rf["iters"], rb["iters"])


# ---- diagonally scaled Fourier preconditioner S^-1 (Q + I (x) Mbar)^-1 S^-1 -------------------

def _dense_columns(Minv, k, n_pix):
    n = k * n_pix
    return np.array([Minv(np.eye(n)[i].reshape(k, n_pix)).ravel() for i in range(n)]).T


@pytest.mark.parametrize("boundary", ["periodic", "face"])
def test_prior_diagonal_closed_form(boundary):
    """diag(Q_j) at pixel p is tau_j ((kappa_j^2 + d_p)^2 + d_p), d_p the number of grid
    neighbours of p (4 on periodic grids with sides >= 3, 2 to 4 on a face): the diagonal of
    (kappa^2 I + L)^2 for the graph Laplacian L."""
    ny, nx = (6, 8) if boundary == "periodic" else (5, 7)
    p = make_problem(ny, nx, 3, 4, seed=9065, noise="hetero", boundary=boundary)
    G = op.posterior_precision(p)
    dQ = (G - op.likelihood_term(p)).diagonal().reshape(p.k, ny, nx)
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    if boundary == "periodic":
        d = np.full((ny, nx), 4.0)
    else:
        d = ((xx > 0).astype(float) + (xx < nx - 1) + (yy > 0) + (yy < ny - 1))
    for j in range(p.k):
        ref = p.tau[j] * ((p.kappa[j] ** 2 + d) ** 2 + d)
        assert np.abs(dQ[j] - ref).max() <= 1e-13 * ref.max()


@pytest.mark.parametrize("boundary", ["periodic", "face"])
def test_scaled_fourier_preconditioner_inverts_scaled_pixel_mean_operator(boundary):
    """The scaled preconditioner is the inverse of S M0 S with M0 = Q + I (x) Mbar assembled
    directly (no transforms) and s^2 = diag(G) / diag(M0): its dense matrix P is symmetric
    positive definite, P^-1 = S M0 S, and P^-1 has the diagonal of G."""
    p = make_problem(6, 8, 2, 3, seed=9070, noise="hetero", mask_frac=0.15, boundary=boundary)
    k, n = p.k, p.n_pix
    P = _dense_columns(opcg.fourier_preconditioner(p, scaled=True), k, n)
    G = op.posterior_precision(p, dense=True)
    Q = G - op.likelihood_term(p).toarray()
    mbar = (p.A.T * p.W.mean(axis=1)) @ p.A
    M0 = Q + np.kron(mbar, np.eye(n))
    s = np.sqrt(np.diag(G) / np.diag(M0))
    assert np.abs(s - 1.0).max() > 0.05   # the scaling is not trivial here
    Pinv = np.linalg.inv(0.5 * (P + P.T))
    assert np.abs(P - P.T).max() <= 1e-12 * np.abs(P).max()
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0
    assert np.abs(Pinv - s[:, None] * M0 * s[None, :]).max() <= 1e-9 * np.abs(M0).max()
    assert np.abs(np.diag(Pinv) - np.diag(G)).max() <= 1e-9 * np.abs(np.diag(G)).max()


def test_scaled_fourier_preconditioner_is_plain_for_homoscedastic_weights():
    """With W independent of the pixel, diag(G) = diag(M0), s = 1 and the scaled preconditioner
    is the plain one (and so G^-1)."""
    p = make_problem(8, 8, 3, 5, seed=9080, noise="homo")
    assert np.abs(opcg.diagonal_scale(p) - 1.0).max() <= 1e-14
    R = np.random.default_rng(9081).standard_normal((p.k, p.n_pix))
    Zs = opcg.fourier_preconditioner(p, scaled=True)(R)
    Zp = opcg.fourier_preconditioner(p)(R)
    assert np.linalg.norm(Zs - Zp) <= 1e-14 * np.linalg.norm(Zp)


@pytest.mark.parametrize("boundary", ["periodic", "face"])
def test_scaled_fourier_pcg_matches_dense_in_fewer_iterations(boundary):
    """PCG with the scaled preconditioner reaches the dense solution; on this problem (the
    gain depends on the problem: fewer iterations on most, one or two more on some small face
    grids) it needs fewer iterations than with the plain one."""
    p = make_problem(32, 32, 3, 6, seed=3, noise="hetero", mask_frac=0.1, boundary=boundary)
    xd = osv.solve_dense(p)
    rs = opcg.pcg(p, tol=1e-11, precond="fourier_diag")
    rf = opcg.pcg(p, tol=1e-11, precond="fourier")
    assert np.linalg.norm(rs["x"] - xd) <= 1e-8 * np.linalg.norm(xd)
    assert rs["iters"] < rf["iters"], (rs["iters"], rf["iters"])


# ---- block-scaled Fourier preconditioner T^T (Q + I (x) Mbar)^-1 T ----------------------------

def _block_diag_dense(T, k, n):
    """The [k n, k n] matrix of the per-pixel blocks T[p] in the component-major layout."""
    D = np.zeros((k * n, k * n))
    for p in range(n):
        idx = np.arange(k) * n + p
        D[np.ix_(idx, idx)] = T[p]
    return D


@pytest.mark.parametrize("boundary", ["periodic", "face"])
def test_block_scaled_fourier_preconditioner_matches_pixel_blocks(boundary):
    """The block-scaled preconditioner inverts T^-1 M0 T^-T with M0 = Q + I (x) Mbar assembled
    without transforms and T_p lower triangular: its dense matrix P is symmetric positive
    definite, P^-1 equals that operator, and every k x k pixel block of P^-1 equals G's."""
    p = make_problem(6, 8, 3, 4, seed=9100, noise="hetero", mask_frac=0.15, boundary=boundary)
    k, n = p.k, p.n_pix
    P = _dense_columns(opcg.fourier_preconditioner(p, scaled="block"), k, n)
    G = op.posterior_precision(p, dense=True)
    Q = G - op.likelihood_term(p).toarray()
    mbar = (p.A.T * p.W.mean(axis=1)) @ p.A
    M0 = Q + np.kron(mbar, np.eye(n))
    T = opcg.block_scale(p)
    assert np.abs(np.triu(T, 1)).max() == 0.0
    Tinv = np.linalg.inv(_block_diag_dense(T, k, n))
    Pinv = np.linalg.inv(0.5 * (P + P.T))
    assert np.abs(P - P.T).max() <= 1e-12 * np.abs(P).max()
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0
    assert np.abs(Pinv - Tinv @ M0 @ Tinv.T).max() <= 1e-9 * np.abs(M0).max()
    for pix in range(n):
        idx = np.arange(k) * n + pix
        assert np.abs(Pinv[np.ix_(idx, idx)] - G[np.ix_(idx, idx)]).max() <= 1e-9 * np.abs(G).max()


def test_block_scaled_fourier_preconditioner_special_cases():
    """Pixel-independent weights: T = I and the plain preconditioner; k = 1: T = 1 / s and the
    diagonally scaled one."""
    p = make_problem(8, 8, 3, 5, seed=9110, noise="homo")
    assert np.abs(opcg.block_scale(p) - np.eye(3)).max() <= 1e-13
    R = np.random.default_rng(9111).standard_normal((p.k, p.n_pix))
    Zb = opcg.fourier_preconditioner(p, scaled="block")(R)
    assert np.linalg.norm(Zb - opcg.fourier_preconditioner(p)(R)) <= 1e-13 * np.linalg.norm(Zb)
    q = make_problem(8, 8, 1, 3, seed=9112, noise="hetero", mask_frac=0.2)
    assert np.abs(opcg.block_scale(q)[:, 0, 0] - 1.0 / opcg.diagonal_scale(q)[0]).max() <= 1e-13
    R1 = np.random.default_rng(9113).standard_normal((1, q.n_pix))
    Zb1 = opcg.fourier_preconditioner(q, scaled="block")(R1)
    Zd1 = opcg.fourier_preconditioner(q, scaled=True)(R1)
    assert np.linalg.norm(Zb1 - Zd1) <= 1e-13 * np.linalg.norm(Zd1)


@pytest.mark.parametrize("boundary", ["periodic", "face"])
def test_block_scaled_fourier_pcg_matches_dense(boundary):
    p = make_problem(32, 32, 4, 6, seed=3, noise="hetero", mask_frac=0.1, boundary=boundary)
    xd = osv.solve_dense(p)
    rb = opcg.pcg(p, tol=1e-11, precond="fourier_block")
    rf = opcg.pcg(p, tol=1e-11, precond="fourier")
    assert np.linalg.norm(rb["x"] - xd) <= 1e-8 * np.linalg.norm(xd)
    assert rb["iters"] < rf["iters"], (rb["iters"], rf["iters"])
