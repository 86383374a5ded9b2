"""GPU parity of the sparse-dense Sylvester solver (Alg. 3, Section 3.3.1) with conjugate-gradient
column solves on the GPU, through the C ABI, against the CPU oracle: the oracle's Alg. 3
(scipy Schur form, SuperLU column solves) and dense Cholesky of the assembled system, in the
Schur (column-by-column) and decoupled (batched eigenvector) forms, float64 and mixed precision,
periodic and face grids, masked pixels, every k, and the full 1024^2, k = 4, f = 9 workload
against the oracle's PCG."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2204_08057_amd as sy  # noqa: E402
from oracle import operator as op  # noqa: E402
from oracle import pcg as opcg  # noqa: E402
from oracle import solve as osv  # noqa: E402
from workloads import make_problem, workload  # noqa: E402


def say(*a):
    print("[kohler]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) /
                 max(np.linalg.norm(np.asarray(b)), 1e-300))


def sep(ny, nx, k, f, seed, kappa=0.45, boundary="periodic", mask=0.0):
    p = make_problem(ny, nx, k, f, seed=seed, noise="separable", kappa=np.full(k, kappa),
                     boundary=boundary)
    t, n = p.meta["t"].copy(), p.meta["n"].copy()
    if mask > 0.0:
        masked = np.random.default_rng(seed + 1).random(p.n_pix) < mask
        n[masked] = 0.0
        p.W[:, masked] = 0.0
        p.Y[:, masked] = 0.0
    return p, t, n


def run(p, t, n, tol, decouple, precision=sy.SYLV_PREC_F64):
    sp = sy.SepProblem.from_numpy(p.ny, p.nx, p.kappa[0], p.tau, p.A, t, n, boundary=p.boundary)
    Yd = torch.as_tensor(p.Y, dtype=torch.float64, device="cuda")
    X, st, rr = sy.kohler_solve(sp, Yd, sy.SolveOptions(tol=tol, precision=precision),
                                decouple=decouple)
    torch.cuda.synchronize()
    return X.cpu().numpy(), st, rr


SHAPES = [(8, 8, 3, 5), (70, 45, 4, 9), (2, 150, 2, 3), (33, 130, 1, 2), (16, 16, 8, 16),
          (4, 40, 5, 6), (24, 20, 6, 9), (9, 11, 7, 8)]


@pytest.mark.parametrize("decouple", [0, 1])
@pytest.mark.parametrize("shape", SHAPES)
def test_float64_matches_oracle_alg3_and_dense(shape, decouple):
    ny, nx, k, f = shape
    p, t, n = sep(ny, nx, k, f, 4000 + ny * 7 + nx)
    say("float64", shape, "decouple", decouple)
    X, st, rr = run(p, t, n, 1e-12, decouple)
    assert all(s["status"] == 0 for s in st), st
    ref = osv.solve_kohler(p, t, n)
    assert rel(X, ref) <= 1e-8
    if p.n_pix * k <= 4000:
        assert rel(X, osv.solve_dense(p)) <= 1e-8
    # the reported residual of eq. (Axb) is the oracle operator's residual of the GPU result
    r_or = rel(op.apply(p, X), op.rhs(p))
    assert rr == pytest.approx(r_or, rel=1e-3, abs=1e-15)


@pytest.mark.parametrize("decouple", [0, 1])
@pytest.mark.parametrize("shape", [(70, 45, 4, 9), (16, 16, 8, 16), (33, 130, 1, 2)])
def test_mixed_precision_matches_oracle(shape, decouple):
    ny, nx, k, f = shape
    p, t, n = sep(ny, nx, k, f, 4100 + ny)
    say("mixed", shape, "decouple", decouple)
    X, st, rr = run(p, t, n, 1e-11, decouple, sy.SYLV_PREC_MIXED)
    assert all(s["status"] == 0 for s in st), st
    assert rel(X, osv.solve_kohler(p, t, n)) <= 1e-7


@pytest.mark.parametrize("decouple", [0, 1])
def test_face_grid_and_masked_pixels(decouple):
    """A HEALPix-like face (links only inside the grid) with 10 % of the pixels masked (n_p = 0:
    the column matrices D2 + R_ii N stay positive definite through kappa > 0)."""
    for boundary in ("face", "periodic"):
        p, t, n = sep(30, 26, 4, 9, 4200, boundary=boundary, mask=0.1)
        say(boundary, "masked, decouple", decouple)
        X, st, rr = run(p, t, n, 1e-12, decouple)
        assert all(s["status"] == 0 for s in st), st
        assert rel(X, osv.solve_dense(p)) <= 1e-8
        assert rel(X, osv.solve_kohler(p, t, n)) <= 1e-8


def test_schur_and_decoupled_agree_and_printed_mixing():
    """The two forms give the same solution; with the paper's printed Planck mixing matrix and
    noise levels (App. B) as A and t."""
    A, T = [], None
    with open(__file__.replace("test_gpu_kohler.py", "golden/planck_mixing.txt")) as fh:
        for line in fh:
            if line.startswith("A "):
                A.append([float(v) for v in line.split()[1:]])
            elif line.startswith("T "):
                T = np.array([float(v) for v in line.split()[1:]])
    A = np.array(A)
    k, f = 4, 9
    p = make_problem(40, 36, k, f, seed=4300, noise="separable", kappa=np.full(k, 0.3), A=A)
    n = np.random.default_rng(4301).integers(1, 4, p.n_pix).astype(float)
    t = T
    p.W = np.outer(t, n)
    say("printed mixing")
    X0, st0, _ = run(p, t, n, 1e-12, 0)
    X1, st1, _ = run(p, t, n, 1e-12, 1)
    assert all(s["status"] == 0 for s in st0 + st1)
    assert rel(X0, X1) <= 1e-9
    assert rel(X0, osv.solve_dense(p)) <= 1e-8


@pytest.mark.parametrize("decouple", [0, 1])
def test_full_size_1024_matches_oracle_pcg(decouple):
    """The Lanczos-Sylvester workload (1024^2, k = 4, f = 9, separable noise, common kappa): the
    whole GPU solution (column solves to 1e-12) against the oracle's PCG to 1e-13."""
    p = workload("sylv_1024")[0]
    t, n = p.meta["t"], p.meta["n"]
    global _REF
    try:
        ref = _REF
    except NameError:
        say("oracle PCG sylv_1024 to 1e-13 (CPU)")
        ref = _REF = opcg.pcg(p, tol=1e-13, max_iter=5000, precond="block")["x"]
    say("full size, decouple", decouple)
    X, st, rr = run(p, t, n, 1e-12, decouple)
    assert all(s["status"] == 0 for s in st), st
    assert rel(X, ref) <= 1e-8
    assert rr <= 1e-10
