"""GPU parity of the Fourier preconditioner (the operator with pixel-mean weights, inverted mode
by mode through the 2-D DFT) against the CPU oracle, through the C ABI: the stand-alone
application in float64 and float32 against the oracle's numpy-FFT application, and conjugate
gradient solves preconditioned by it against dense Cholesky, the oracle's PCG with the same
preconditioner (iteration counts) and, at 1024^2, the oracle's PCG reference solution."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2204_08057_amd as sy  # noqa: E402
from oracle import pcg as opcg  # noqa: E402
from oracle import solve as osv  # noqa: E402
from workloads import make_problem, random_maps, workload  # noqa: E402

DEV = "cuda"


def say(*a):
    print("[fourier]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


# (ny, nx, k, f): odd and even powers of two (radix-2 last stage), rectangular, tiny, every k,
# and the largest tiles: k ny = 8192 column values (above 64 KB of LDS in float32, about 150 KB in
# float64) and rows of 4096
SHAPES = [(4, 4, 1, 2), (8, 16, 3, 5), (16, 8, 2, 3), (32, 64, 4, 9), (64, 64, 3, 6),
          (128, 32, 8, 16), (4, 256, 5, 4), (512, 8, 2, 3), (16, 16, 6, 7), (8, 32, 7, 8),
          (2048, 16, 4, 9), (4096, 4, 1, 2), (8, 4096, 2, 3), (1024, 8, 8, 9)]


@pytest.mark.parametrize("shape", SHAPES)
def test_preconditioner_application_matches_oracle(shape):
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=5000 + ny + nx, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(p)
    R = random_maps(p, seed=5001, nrhs=2)
    ref = np.stack([opcg.fourier_preconditioner(p)(R[i]) for i in range(2)])
    say("application", shape)
    Z64 = host(sy.precond(dp, dev(R), kind=sy.SYLV_PC_FOURIER))
    assert rel(Z64, ref) <= 1e-12
    Z32 = host(sy.precond(dp, dev(R, torch.float32), kind=sy.SYLV_PC_FOURIER))
    assert rel(Z32, ref) <= 2e-5


@pytest.mark.parametrize("precision,tol,bound", [(sy.SYLV_PREC_F64, 1e-12, 1e-8),
                                                 (sy.SYLV_PREC_MIXED, 1e-11, 1e-7)])
@pytest.mark.parametrize("shape", [(8, 16, 3, 5), (32, 64, 4, 9), (16, 16, 6, 7), (64, 32, 2, 3)])
def test_solve_matches_dense(shape, precision, tol, bound):
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=5100 + ny * nx, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(p)
    say("solve", shape, precision)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(
        tol=tol, precision=precision, precond=sy.SYLV_PC_FOURIER))
    assert st[0]["status"] == 0, st
    assert rel(host(X).reshape(p.k, p.n_pix), osv.solve_dense(p)) <= bound


@pytest.mark.parametrize("shape", [(32, 64, 4, 9), (64, 64, 3, 6), (128, 128, 3, 9)])
def test_iteration_count_matches_oracle(shape):
    """Float64 runs to 1e-8 take the oracle's iteration count with the same preconditioner to
    within 1 (same algorithm; reductions round differently)."""
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=5200 + ny, noise="hetero")
    ref = opcg.pcg(p, tol=1e-8, max_iter=2000, precond="fourier")
    say("iterations", shape, "oracle", ref["iters"])
    dp = sy.DeviceProblem.from_numpy(p)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(tol=1e-8,
                                                              precond=sy.SYLV_PC_FOURIER))
    assert st[0]["status"] == 0, st
    say("  gpu", st[0]["iters"])
    assert abs(st[0]["iters"] - ref["iters"]) <= 1


def test_homoscedastic_grid_solves_in_one_iteration():
    """With pixel-independent weights the preconditioner is G^-1 itself: one iteration."""
    p = make_problem(64, 32, 3, 6, seed=5300, noise="homo")
    dp = sy.DeviceProblem.from_numpy(p)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(tol=1e-10,
                                                              precond=sy.SYLV_PC_FOURIER))
    assert st[0]["status"] == 0 and st[0]["iters"] <= 2, st
    assert rel(host(X).reshape(p.k, p.n_pix), osv.solve_fft(p)) <= 1e-9


def test_batch_of_uneven_grids_and_right_hand_sides():
    probs = [make_problem(32, 64, 3, 5, seed=5400, noise="hetero"),
             make_problem(16, 16, 3, 5, seed=5401, noise="hetero", mask_frac=0.1)]
    nrhs = 2
    rng = np.random.default_rng(5402)
    Bx = [rng.standard_normal((nrhs, q.k, q.n_pix)) for q in probs]
    dps = [sy.DeviceProblem.from_numpy(q) for q in probs]
    say("batch")
    for precision, tol, bound in ((sy.SYLV_PREC_F64, 1e-12, 1e-8),
                                  (sy.SYLV_PREC_MIXED, 1e-11, 1e-7)):
        X, st = sy.pcg_solve(dps, Y=torch.cat([dev(q.Y.ravel()) for q in probs]),
                             Bextra=torch.cat([dev(b.ravel()) for b in Bx]), nrhs=nrhs,
                             opts=sy.SolveOptions(tol=tol, precision=precision,
                                                  precond=sy.SYLV_PC_FOURIER))
        assert all(s["status"] == 0 for s in st), st
        x = host(X)
        off = 0
        from oracle import operator as op
        for g, q in enumerate(probs):
            for r in range(nrhs):
                xs = osv.solve_dense(q, b=op.rhs(q) + Bx[g][r])
                assert rel(x[off:off + q.k * q.n_pix].reshape(q.k, q.n_pix), xs) <= bound
                off += q.k * q.n_pix


@pytest.mark.parametrize("precision,tol,bound", [(sy.SYLV_PREC_F64, 1e-12, 1e-8),
                                                 (sy.SYLV_PREC_MIXED, 1e-11, 1e-7)])
def test_het_1024_whole_solution_vs_oracle(precision, tol, bound):
    """The timing workload (1024^2, k = 3, f = 9, heteroscedastic) solved with the Fourier
    preconditioner, whole vector against the oracle's block-Jacobi PCG to 1e-13."""
    global _HET
    try:
        p, ref = _HET
    except NameError:
        p = workload("het_1024")[0]
        say("oracle PCG het_1024 to 1e-13 (CPU)")
        ref = opcg.pcg(p, tol=1e-13, max_iter=5000, precond="block")["x"]
        _HET = (p, ref)
    say("het_1024", precision)
    dp = sy.DeviceProblem.from_numpy(p)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(
        tol=tol, precision=precision, precond=sy.SYLV_PC_FOURIER))
    assert st[0]["status"] == 0, st
    say("  iterations", st[0]["iters"], "outer", st[0]["outer"])
    assert rel(host(X).reshape(p.k, p.n_pix), ref) <= bound


def test_largest_float64_column_reads_twiddles_from_global_memory():
    """2 x 4096 complex float64 column values and their twiddle table exceed 160 KB of LDS: the
    column pass then reads the twiddles from the set-up table in global memory."""
    p = make_problem(4096, 4, 2, 3, seed=5504, noise="hetero")
    dp = sy.DeviceProblem.from_numpy(p)
    R = random_maps(p, seed=5505)
    ref = opcg.fourier_preconditioner(p)(R)
    assert rel(host(sy.precond(dp, dev(R), kind=sy.SYLV_PC_FOURIER)), ref) <= 1e-12
    assert rel(host(sy.precond(dp, dev(R, torch.float32), kind=sy.SYLV_PC_FOURIER)), ref) <= 2e-5


def test_unsupported_shapes_are_refused():
    for kw in (dict(ny=24, nx=32), dict(ny=32, nx=2), dict(ny=24, nx=16, boundary="face")):
        boundary = kw.pop("boundary", "periodic")
        p = make_problem(kw["ny"], kw["nx"], 3, 4, seed=5500, noise="hetero", boundary=boundary)
        dp = sy.DeviceProblem.from_numpy(p)
        with pytest.raises(sy.SylvError):
            sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(precond=sy.SYLV_PC_FOURIER))
    # a column of k ny = 12288 complex values exceeds the column pass's tile in both precisions
    p = make_problem(4096, 4, 3, 3, seed=5502, noise="hetero")
    dp = sy.DeviceProblem.from_numpy(p)
    R = dev(random_maps(p, seed=5503))
    for dt in (torch.float64, torch.float32):
        with pytest.raises(sy.SylvError):
            sy.precond(dp, R.to(dt), kind=sy.SYLV_PC_FOURIER)
    p = make_problem(16, 16, 3, 4, seed=5501, noise="hetero")
    dp = sy.DeviceProblem.from_numpy(p)
    with pytest.raises(sy.SylvError):   # block CG takes the per-pixel preconditioners only
        sy.pcg_solve([dp], Bextra=dev(np.ones(2 * 3 * 256)), nrhs=2,
                     opts=sy.SolveOptions(precond=sy.SYLV_PC_FOURIER, block=1))


# ---- face grids (links only inside the grid): the cosine basis ---------------------------------

FACE_SHAPES = [(4, 4, 1, 2), (8, 16, 3, 5), (16, 8, 2, 3), (64, 32, 4, 9), (4, 256, 5, 4),
               (512, 8, 2, 3), (8, 32, 7, 8), (2048, 16, 4, 9), (8, 4096, 2, 3), (1024, 8, 8, 9)]


@pytest.mark.parametrize("shape", FACE_SHAPES)
def test_face_application_matches_oracle(shape):
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=5600 + ny + nx, noise="hetero", mask_frac=0.1,
                     boundary="face")
    dp = sy.DeviceProblem.from_numpy(p)
    R = random_maps(p, seed=5601, nrhs=2)
    ref = np.stack([opcg.fourier_preconditioner(p)(R[i]) for i in range(2)])
    say("face application", shape)
    assert rel(host(sy.precond(dp, dev(R), kind=sy.SYLV_PC_FOURIER)), ref) <= 1e-12
    assert rel(host(sy.precond(dp, dev(R, torch.float32), kind=sy.SYLV_PC_FOURIER)), ref) <= 2e-5


@pytest.mark.parametrize("precision,tol,bound", [(sy.SYLV_PREC_F64, 1e-12, 1e-8),
                                                 (sy.SYLV_PREC_MIXED, 1e-11, 1e-7)])
@pytest.mark.parametrize("shape", [(8, 16, 3, 5), (32, 64, 4, 9), (64, 32, 2, 3)])
def test_face_solve_matches_dense(shape, precision, tol, bound):
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=5700 + ny * nx, noise="hetero", mask_frac=0.1,
                     boundary="face")
    dp = sy.DeviceProblem.from_numpy(p)
    say("face solve", shape, precision)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(
        tol=tol, precision=precision, precond=sy.SYLV_PC_FOURIER))
    assert st[0]["status"] == 0, st
    assert rel(host(X).reshape(p.k, p.n_pix), osv.solve_dense(p)) <= bound


@pytest.mark.parametrize("shape", [(32, 64, 4, 9), (128, 128, 3, 9)])
def test_face_iteration_count_matches_oracle(shape):
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=5800 + ny, noise="hetero", boundary="face")
    ref = opcg.pcg(p, tol=1e-8, max_iter=2000, precond="fourier")
    dp = sy.DeviceProblem.from_numpy(p)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(tol=1e-8,
                                                              precond=sy.SYLV_PC_FOURIER))
    say("face iterations", shape, "oracle", ref["iters"], "gpu", st[0]["iters"])
    assert st[0]["status"] == 0, st
    assert abs(st[0]["iters"] - ref["iters"]) <= 1


def test_face_homoscedastic_grid_solves_in_one_iteration():
    p = make_problem(32, 64, 3, 6, seed=5900, noise="homo", boundary="face")
    dp = sy.DeviceProblem.from_numpy(p)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(tol=1e-10,
                                                              precond=sy.SYLV_PC_FOURIER))
    assert st[0]["status"] == 0 and st[0]["iters"] <= 2, st
    assert rel(host(X).reshape(p.k, p.n_pix), osv.solve_dense(p)) <= 1e-9


def test_face_batch_of_twelve_faces():
    """Twelve independent faces in one call (the full-sky layout, App. A), both precisions."""
    probs = [make_problem(32, 32, 4, 9, seed=6000 + g, noise="hetero", boundary="face")
             for g in range(12)]
    dps = [sy.DeviceProblem.from_numpy(q) for q in probs]
    Y = torch.cat([dev(q.Y.ravel()) for q in probs])
    say("face batch")
    for precision, tol, bound in ((sy.SYLV_PREC_F64, 1e-12, 1e-8),
                                  (sy.SYLV_PREC_MIXED, 1e-11, 1e-7)):
        X, st = sy.pcg_solve(dps, Y=Y, opts=sy.SolveOptions(tol=tol, precision=precision,
                                                            precond=sy.SYLV_PC_FOURIER))
        assert all(s["status"] == 0 for s in st), st
        x = host(X)
        off = 0
        for q in probs:
            n = q.k * q.n_pix
            assert rel(x[off:off + n].reshape(q.k, q.n_pix), osv.solve_dense(q)) <= bound
            off += n


# ---- diagonally scaled variant (SYLV_PC_FOURIER_DIAG): z = S^-1 (Q + I (x) Mbar)^-1 S^-1 r ------

DIAG_SHAPES = [("periodic", s) for s in [(8, 16, 3, 5), (32, 64, 4, 9), (128, 32, 8, 16),
                                         (2048, 16, 4, 9), (8, 4096, 2, 3), (4096, 4, 2, 3)]] + \
              [("face", s) for s in [(8, 16, 3, 5), (64, 32, 4, 9), (1024, 8, 8, 9)]]


@pytest.mark.parametrize("boundary,shape", DIAG_SHAPES)
def test_diag_application_matches_oracle(boundary, shape):
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=5700 + ny + nx, noise="hetero", mask_frac=0.1,
                     boundary=boundary)
    dp = sy.DeviceProblem.from_numpy(p)
    R = random_maps(p, seed=5701, nrhs=2)
    Minv = opcg.fourier_preconditioner(p, scaled=True)
    ref = np.stack([Minv(R[i]) for i in range(2)])
    plain = np.stack([opcg.fourier_preconditioner(p)(R[i]) for i in range(2)])
    assert rel(plain, ref) > 1e-3   # the scale is not trivial on these weights
    say("diag application", boundary, shape)
    assert rel(host(sy.precond(dp, dev(R), kind=sy.SYLV_PC_FOURIER_DIAG)), ref) <= 1e-12
    assert rel(host(sy.precond(dp, dev(R, torch.float32), kind=sy.SYLV_PC_FOURIER_DIAG)),
               ref) <= 2e-5


@pytest.mark.parametrize("precision,tol,bound", [(sy.SYLV_PREC_F64, 1e-12, 1e-8),
                                                 (sy.SYLV_PREC_MIXED, 1e-11, 1e-7)])
@pytest.mark.parametrize("boundary,shape", [("periodic", (32, 64, 4, 9)),
                                            ("periodic", (16, 16, 6, 7)),
                                            ("face", (32, 64, 4, 9)), ("face", (64, 32, 2, 3))])
def test_diag_solve_matches_dense(boundary, shape, precision, tol, bound):
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=5800 + ny * nx, noise="hetero", mask_frac=0.1,
                     boundary=boundary)
    dp = sy.DeviceProblem.from_numpy(p)
    say("diag solve", boundary, shape, precision)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(
        tol=tol, precision=precision, precond=sy.SYLV_PC_FOURIER_DIAG))
    assert st[0]["status"] == 0, st
    assert rel(host(X).reshape(p.k, p.n_pix), osv.solve_dense(p)) <= bound


@pytest.mark.parametrize("boundary,shape", [("periodic", (64, 64, 3, 6)),
                                            ("periodic", (128, 128, 3, 9)),
                                            ("face", (128, 128, 3, 9))])
def test_diag_iteration_count_matches_oracle(boundary, shape):
    """Float64 runs to 1e-8 take the oracle's iteration count with the scaled preconditioner to
    within 1."""
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=5900 + ny, noise="hetero", boundary=boundary)
    ref = opcg.pcg(p, tol=1e-8, max_iter=2000, precond="fourier_diag")
    say("diag iterations", boundary, shape, "oracle", ref["iters"])
    dp = sy.DeviceProblem.from_numpy(p)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(
        tol=1e-8, precond=sy.SYLV_PC_FOURIER_DIAG))
    assert st[0]["status"] == 0, st
    say("  gpu", st[0]["iters"])
    assert abs(st[0]["iters"] - ref["iters"]) <= 1


def test_diag_homoscedastic_grid_solves_in_one_iteration():
    """Pixel-independent weights: s = 1 and the scaled preconditioner is G^-1 as well."""
    p = make_problem(64, 32, 3, 6, seed=5950, noise="homo")
    dp = sy.DeviceProblem.from_numpy(p)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(
        tol=1e-10, precond=sy.SYLV_PC_FOURIER_DIAG))
    assert st[0]["status"] == 0 and st[0]["iters"] <= 2, st
    assert rel(host(X).reshape(p.k, p.n_pix), osv.solve_fft(p)) <= 1e-9


def test_diag_fixed_schedule_equals_adaptive():
    """The fixed schedule (no host checks) and the adaptive one run the same iterations: equal
    solutions, bitwise."""
    p = make_problem(64, 64, 3, 6, seed=5960, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(p)
    for precision in (sy.SYLV_PREC_F64, sy.SYLV_PREC_MIXED):
        o = sy.SolveOptions(tol=1e-9, precision=precision, precond=sy.SYLV_PC_FOURIER_DIAG)
        Xa, sa = sy.pcg_solve(dp, Y=dev(p.Y), opts=o)
        of = sy.SolveOptions(tol=1e-9, precision=precision, precond=sy.SYLV_PC_FOURIER_DIAG,
                             schedule=sy.SYLV_SCHED_FIXED, max_iter=sa[0]["iters"] + 5)
        Xf, sf = sy.pcg_solve(dp, Y=dev(p.Y), opts=of)
        say("diag fixed", precision, sa[0]["iters"], sf[0]["iters"])
        assert sa[0]["status"] == 0 and sf[0]["status"] == 0, (sa, sf)
        assert torch.equal(Xa, Xf)


@pytest.mark.parametrize("precision,tol,bound", [(sy.SYLV_PREC_F64, 1e-12, 1e-8),
                                                 (sy.SYLV_PREC_MIXED, 1e-11, 1e-7)])
def test_diag_het_1024_whole_solution_vs_oracle(precision, tol, bound):
    """The timing workload solved with the scaled preconditioner, whole vector against the
    oracle's block-Jacobi PCG to 1e-13."""
    global _HET
    try:
        p, ref = _HET
    except NameError:
        p = workload("het_1024")[0]
        say("oracle PCG het_1024 to 1e-13 (CPU)")
        ref = opcg.pcg(p, tol=1e-13, max_iter=5000, precond="block")["x"]
        _HET = (p, ref)
    say("diag het_1024", precision)
    dp = sy.DeviceProblem.from_numpy(p)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(
        tol=tol, precision=precision, precond=sy.SYLV_PC_FOURIER_DIAG))
    assert st[0]["status"] == 0, st
    say("  iterations", st[0]["iters"], "outer", st[0]["outer"])
    assert rel(host(X).reshape(p.k, p.n_pix), ref) <= bound


# ---- block-scaled variant (SYLV_PC_FOURIER_BLOCK): z = T^T (Q + I (x) Mbar)^-1 T r ---------------

BLOCK_SHAPES = [("periodic", s) for s in [(8, 16, 3, 5), (32, 64, 4, 9), (128, 32, 8, 16),
                                          (2048, 16, 4, 9), (16, 1024, 8, 9), (8, 4096, 1, 3),
                                          (4096, 4, 2, 3), (64, 64, 1, 3),
                                          # float64 bands whose table goes to global memory
                                          (16, 2048, 4, 9), (8, 4096, 2, 3), (16, 1024, 4, 9),
                                          (8, 2048, 2, 3)]] + \
               [("face", s) for s in [(8, 16, 3, 5), (64, 32, 4, 9), (1024, 8, 8, 9),
                                      (16, 2048, 4, 9), (16, 1024, 4, 9)]]


@pytest.mark.parametrize("boundary,shape", BLOCK_SHAPES)
def test_block_application_matches_oracle(boundary, shape):
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=6000 + ny + nx, noise="hetero", mask_frac=0.1,
                     boundary=boundary)
    dp = sy.DeviceProblem.from_numpy(p)
    R = random_maps(p, seed=6001, nrhs=2)
    Minv = opcg.fourier_preconditioner(p, scaled="block")
    ref = np.stack([Minv(R[i]) for i in range(2)])
    say("block application", boundary, shape)
    assert rel(host(sy.precond(dp, dev(R), kind=sy.SYLV_PC_FOURIER_BLOCK)), ref) <= 1e-12
    assert rel(host(sy.precond(dp, dev(R, torch.float32), kind=sy.SYLV_PC_FOURIER_BLOCK)),
               ref) <= 2e-5


def test_block_refuses_rows_wider_than_its_pass():
    p = make_problem(16, 4096, 3, 4, seed=6050, noise="hetero")
    dp = sy.DeviceProblem.from_numpy(p)
    with pytest.raises(Exception):
        sy.precond(dp, dev(random_maps(p, seed=6051)), kind=sy.SYLV_PC_FOURIER_BLOCK)
    # the plain preconditioner takes the same grid
    assert host(sy.precond(dp, dev(random_maps(p, seed=6051)), kind=sy.SYLV_PC_FOURIER)).size


@pytest.mark.parametrize("precision,tol,bound", [(sy.SYLV_PREC_F64, 1e-12, 1e-8),
                                                 (sy.SYLV_PREC_MIXED, 1e-11, 1e-7)])
@pytest.mark.parametrize("boundary,shape", [("periodic", (32, 64, 4, 9)),
                                            ("periodic", (16, 16, 6, 7)),
                                            ("face", (32, 64, 4, 9)), ("face", (64, 32, 2, 3))])
def test_block_solve_matches_dense(boundary, shape, precision, tol, bound):
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=6100 + ny * nx, noise="hetero", mask_frac=0.1,
                     boundary=boundary)
    dp = sy.DeviceProblem.from_numpy(p)
    say("block solve", boundary, shape, precision)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(
        tol=tol, precision=precision, precond=sy.SYLV_PC_FOURIER_BLOCK))
    assert st[0]["status"] == 0, st
    assert rel(host(X).reshape(p.k, p.n_pix), osv.solve_dense(p)) <= bound


@pytest.mark.parametrize("boundary,shape", [("periodic", (64, 64, 3, 6)),
                                            ("periodic", (128, 128, 3, 9)),
                                            ("face", (128, 128, 3, 9))])
def test_block_iteration_count_matches_oracle(boundary, shape):
    ny, nx, k, f = shape
    p = make_problem(ny, nx, k, f, seed=6200 + ny, noise="hetero", boundary=boundary)
    ref = opcg.pcg(p, tol=1e-8, max_iter=2000, precond="fourier_block")
    say("block iterations", boundary, shape, "oracle", ref["iters"])
    dp = sy.DeviceProblem.from_numpy(p)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(
        tol=1e-8, precond=sy.SYLV_PC_FOURIER_BLOCK))
    assert st[0]["status"] == 0, st
    say("  gpu", st[0]["iters"])
    assert abs(st[0]["iters"] - ref["iters"]) <= 1


def test_block_homoscedastic_grid_solves_in_one_iteration():
    p = make_problem(64, 32, 3, 6, seed=6300, noise="homo")
    dp = sy.DeviceProblem.from_numpy(p)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(
        tol=1e-10, precond=sy.SYLV_PC_FOURIER_BLOCK))
    assert st[0]["status"] == 0 and st[0]["iters"] <= 2, st
    assert rel(host(X).reshape(p.k, p.n_pix), osv.solve_fft(p)) <= 1e-9


def test_block_fixed_schedule_equals_adaptive_and_batch():
    """Fixed and adaptive schedules give bitwise equal solutions; a batch of two uneven grids
    with two right-hand sides each matches dense solves."""
    p = make_problem(64, 64, 3, 6, seed=6400, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(p)
    for precision in (sy.SYLV_PREC_F64, sy.SYLV_PREC_MIXED):
        o = sy.SolveOptions(tol=1e-9, precision=precision, precond=sy.SYLV_PC_FOURIER_BLOCK)
        Xa, sa = sy.pcg_solve(dp, Y=dev(p.Y), opts=o)
        of = sy.SolveOptions(tol=1e-9, precision=precision, precond=sy.SYLV_PC_FOURIER_BLOCK,
                             schedule=sy.SYLV_SCHED_FIXED, max_iter=sa[0]["iters"] + 5)
        Xf, sf = sy.pcg_solve(dp, Y=dev(p.Y), opts=of)
        say("block fixed", precision, sa[0]["iters"], sf[0]["iters"])
        assert sa[0]["status"] == 0 and sf[0]["status"] == 0, (sa, sf)
        assert torch.equal(Xa, Xf)
    probs = [make_problem(32, 64, 3, 5, seed=6401, noise="hetero"),
             make_problem(16, 16, 3, 5, seed=6402, noise="hetero", mask_frac=0.1)]
    nrhs = 2
    rng = np.random.default_rng(6403)
    Bx = [rng.standard_normal((nrhs, q.k, q.n_pix)) for q in probs]
    dps = [sy.DeviceProblem.from_numpy(q) for q in probs]
    X, st = sy.pcg_solve(dps, Y=torch.cat([dev(q.Y.ravel()) for q in probs]),
                         Bextra=torch.cat([dev(b.ravel()) for b in Bx]), nrhs=nrhs,
                         opts=sy.SolveOptions(tol=1e-11, precision=sy.SYLV_PREC_MIXED,
                                              precond=sy.SYLV_PC_FOURIER_BLOCK))
    assert all(s["status"] == 0 for s in st), st
    from oracle import operator as op
    x = host(X)
    off = 0
    for g, q in enumerate(probs):
        for r in range(nrhs):
            xs = osv.solve_dense(q, b=op.rhs(q) + Bx[g][r])
            assert rel(x[off:off + q.k * q.n_pix].reshape(q.k, q.n_pix), xs) <= 1e-7
            off += q.k * q.n_pix


@pytest.mark.parametrize("precision,tol,bound", [(sy.SYLV_PREC_F64, 1e-12, 1e-8),
                                                 (sy.SYLV_PREC_MIXED, 1e-11, 1e-7)])
def test_block_het_1024_whole_solution_vs_oracle(precision, tol, bound):
    global _HET
    try:
        p, ref = _HET
    except NameError:
        p = workload("het_1024")[0]
        say("oracle PCG het_1024 to 1e-13 (CPU)")
        ref = opcg.pcg(p, tol=1e-13, max_iter=5000, precond="block")["x"]
        _HET = (p, ref)
    say("block het_1024", precision)
    dp = sy.DeviceProblem.from_numpy(p)
    X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=sy.SolveOptions(
        tol=tol, precision=precision, precond=sy.SYLV_PC_FOURIER_BLOCK))
    assert st[0]["status"] == 0, st
    say("  iterations", st[0]["iters"], "outer", st[0]["outer"])
    assert rel(host(X).reshape(p.k, p.n_pix), ref) <= bound


def test_float64_batch_mixing_global_and_lds_twiddles():
    """A float64 batch whose grids need the stage twiddles from global memory in some length
    classes and not in others (rows of 2048 and of 1024 at k = 4 with the block-scaled row
    passes, a column of 2048 at k = 4): every instance equals its solve alone, bitwise."""
    probs = [make_problem(16, 2048, 4, 5, seed=6500, noise="hetero"),
             make_problem(16, 1024, 4, 5, seed=6501, noise="hetero"),
             make_problem(2048, 16, 4, 5, seed=6502, noise="hetero")]
    dps = [sy.DeviceProblem.from_numpy(q) for q in probs]
    for kind in (sy.SYLV_PC_FOURIER_BLOCK, sy.SYLV_PC_FOURIER):
        o = sy.SolveOptions(tol=1e-10, precision=sy.SYLV_PREC_F64, precond=kind)
        say("float64 mixed-twiddle batch", kind)
        X, st = sy.pcg_solve(dps, Y=torch.cat([dev(q.Y.ravel()) for q in probs]), opts=o)
        assert all(s["status"] == 0 for s in st), st
        off = 0
        for q, dq in zip(probs, dps):
            Xq, sq = sy.pcg_solve(dq, Y=dev(q.Y), opts=o)
            n = q.k * q.n_pix
            assert torch.equal(X[off:off + n], Xq.reshape(-1)), (kind, q.ny, q.nx)
            assert sq[0]["iters"] == [s for s in st][probs.index(q)]["iters"]
            off += n
