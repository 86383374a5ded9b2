"""Pins of the block-CG oracle (O'Leary's block conjugate gradients) against the definition of
its iterates: column-wise G-norm minimisers over the block Krylov space (no GPU)."""
import numpy as np
import pytest

from oracle import block_pcg as obp
from oracle import operator as op
from oracle import pcg as opcg
from workloads import make_problem


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _explicit_minv(prob, G, precond):
    n = prob.k * prob.n_pix
    if precond == "none":
        return np.eye(n)
    Mb, _ = opcg.block_jacobi(prob, G, precond)
    return np.stack([Mb(e.reshape(prob.k, prob.n_pix)).ravel() for e in np.eye(n)], axis=1)


@pytest.mark.parametrize("precond", ["none", "block"])
@pytest.mark.parametrize("s", [1, 3])
def test_block_iterates_are_krylov_minimisers(precond, s):
    """Iterate j, column c: x0_c + K y with y minimising ||x - x*_c||_G over the span K of all
    columns of M^-1 R0, (M^-1 G) M^-1 R0, ..., (M^-1 G)^(j-1) M^-1 R0 (brute-force Galerkin
    solve), for every column at once."""
    prob = make_problem(4, 4, 2, 3, seed=2100 + s, noise="hetero")
    G = op.posterior_precision(prob, dense=True)
    n = prob.k * prob.n_pix
    rng = np.random.default_rng(2110 + s)
    B = rng.standard_normal((s, n))
    X0 = 0.1 * rng.standard_normal((s, n))
    its = obp.block_pcg(prob, B, X0, max_iter=4, precond=precond, G=G)
    Minv = _explicit_minv(prob, G, precond)
    R0 = (B - X0 @ G.T).T                                  # n x s
    blocks = [Minv @ R0]
    for _ in range(3):
        blocks.append(Minv @ (G @ blocks[-1]))
    for j in range(1, 5):
        K = np.hstack(blocks[:j])
        for c in range(s):
            y = np.linalg.solve(K.T @ G @ K, K.T @ R0[:, c])
            x = X0[c] + K @ y
            assert rel(its[j][c], x) < 1e-8, (j, c)


def test_single_column_equals_pcg_and_block_differs_from_independent():
    """s = 1 is plain PCG; with s = 3 the iterates differ from independent runs (the larger
    search space), which is what lets the GPU test tell block from independent CG."""
    prob = make_problem(5, 4, 2, 3, seed=2120, noise="hetero")
    G = op.posterior_precision(prob)
    rng = np.random.default_rng(2121)
    B = rng.standard_normal((3, prob.k * prob.n_pix))
    ref = opcg.pcg(prob, b=B[0], tol=0.0, max_iter=3, precond="block", G=G, record=True)
    one = obp.block_pcg(prob, B[:1], max_iter=3, precond="block", G=G)
    for j in range(1, 4):
        assert rel(one[j][0], ref["iterates"][j].ravel()) < 1e-10
    three = obp.block_pcg(prob, B, max_iter=3, precond="block", G=G)
    assert rel(three[3][0], ref["iterates"][3].ravel()) > 1e-3
