"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded inputs.

Tolerances (relative, float64 unless stated):
  operator apply / preconditioner / right-hand side / perturbation: 1e-13 of the output norm
    (the same sums in a different order; each output is a 13-term stencil plus a k-term mixing
    sum, so rounding differences stay at a few ulps of the largest term);
  float32 apply: 2e-6 of the output norm (float32 unit roundoff 6e-8 times the stencil's
    coefficient sum ~80 tau relative to the operator's size);
  solves: ||x - x*|| / ||x*|| <= 1e-8 (float64 PCG) and <= 1e-7 (mixed precision), run with a
    residual tolerance small enough that cond(G) * tol stays below those bounds;
  gradients: 1e-7 relative per quantity.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2204_08057_amd as sy  # noqa: E402
from oracle import grad as og  # noqa: E402
from oracle import operator as op  # noqa: E402
from oracle import pcg as opcg  # noqa: E402
from oracle import po as opo  # noqa: E402
from oracle import solve as osv  # noqa: E402
from workloads import make_problem, po_draws, random_maps, workload  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print("[gpu]", *a, flush=True)
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


SHAPES = [
    (1, 1, 1, 1), (1, 5, 2, 3), (2, 2, 3, 4), (3, 7, 3, 5), (5, 5, 4, 9), (4, 64, 2, 2),
    (17, 70, 3, 6), (64, 64, 3, 6), (33, 129, 8, 16), (130, 67, 5, 7), (16, 16, 6, 9),
    (9, 11, 7, 3),
]


@pytest.mark.parametrize("ny,nx,k,f", SHAPES)
def test_apply_f64(ny, nx, k, f):
    say("apply f64", ny, nx, k, f)
    prob = make_problem(ny, nx, k, f, seed=100 + ny * 7 + nx, noise="hetero", mask_frac=0.1)
    X = random_maps(prob, 5)
    dp = sy.DeviceProblem.from_numpy(prob)
    Y = host(sy.apply(dp, dev(X)))
    ref = op.apply(prob, X)
    assert rel(Y, ref) < 1e-13


@pytest.mark.parametrize("ny,nx,k,f", [(5, 5, 4, 9), (64, 64, 3, 6), (33, 129, 8, 16)])
def test_apply_f32(ny, nx, k, f):
    say("apply f32", ny, nx, k, f)
    prob = make_problem(ny, nx, k, f, seed=200 + ny, noise="hetero")
    X = random_maps(prob, 6)
    dp = sy.DeviceProblem.from_numpy(prob)
    Y = host(sy.apply(dp, dev(X, torch.float32)))
    ref = op.apply(prob, X.astype(np.float32).astype(np.float64))
    assert rel(Y, ref) < 2e-6


def test_apply_several_rhs_prepared():
    say("apply nrhs=3 prepared")
    prob = make_problem(40, 72, 3, 6, seed=300)
    X = random_maps(prob, 7, nrhs=3)
    dp = sy.DeviceProblem.from_numpy(prob)
    ws = sy.binding.prepare(dp, sy.SYLV_PC_NONE)
    Y1 = host(sy.apply(dp, dev(X), ws=ws, prepared=True))
    Y2 = host(sy.apply(dp, dev(X), ws=ws, prepared=True))
    assert np.array_equal(Y1, Y2)
    for r in range(3):
        assert rel(Y1[r], op.apply(prob, X[r])) < 1e-13


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_apply_launcher_matches_apply(dtype):
    """The pre-marshalled launcher runs the same entry point: bitwise the apply's output, also
    when launched repeatedly."""
    say("apply launcher", dtype)
    prob = make_problem(40, 72, 3, 6, seed=301, noise="hetero")
    X = random_maps(prob, 8, nrhs=2)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    dp = sy.DeviceProblem.from_numpy(prob)
    ws = sy.binding.prepare(dp, sy.SYLV_PC_NONE)
    Xd = dev(X, tdt)
    ref = host(sy.apply(dp, Xd, ws=ws, prepared=True))
    Y = torch.empty_like(Xd)
    launch = sy.apply_launcher(dp, Xd, Y, ws)
    for _ in range(3):
        launch()
    assert np.array_equal(host(Y), ref)
    with pytest.raises(ValueError):
        sy.apply_launcher(dp, Xd, torch.empty(3, 5, dtype=tdt, device="cuda"), ws)


@pytest.mark.parametrize("kind", [sy.SYLV_PC_BLOCK, sy.SYLV_PC_JACOBI, sy.SYLV_PC_NONE])
@pytest.mark.parametrize("ny,nx,k,f", [(1, 1, 3, 4), (2, 3, 2, 3), (24, 20, 4, 9),
                                       (13, 9, 8, 5)])
def test_precond(kind, ny, nx, k, f):
    say("precond", kind, ny, nx, k, f)
    prob = make_problem(ny, nx, k, f, seed=400 + ny, noise="hetero", mask_frac=0.2)
    R = random_maps(prob, 8)
    dp = sy.DeviceProblem.from_numpy(prob)
    Z = host(sy.precond(dp, dev(R), kind))
    name = {sy.SYLV_PC_BLOCK: "block", sy.SYLV_PC_JACOBI: "jacobi", sy.SYLV_PC_NONE: "none"}
    Minv, _ = opcg.block_jacobi(prob, kind=name[kind])
    assert rel(Z, Minv(R)) < 1e-13


@pytest.mark.parametrize("ny,nx,k,f", [(1, 3, 2, 2), (31, 45, 4, 9), (64, 64, 8, 16)])
def test_rhs(ny, nx, k, f):
    say("rhs", ny, nx, k, f)
    prob = make_problem(ny, nx, k, f, seed=500 + nx, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(prob)
    B = host(sy.rhs(dp, dev(prob.Y)))
    assert rel(B, op.rhs(prob)) < 1e-14


@pytest.mark.parametrize("ny,nx,k,f,nrhs", [(4, 5, 3, 4, 2), (37, 26, 3, 6, 3), (1, 2, 2, 2, 1)])
def test_po_perturbation(ny, nx, k, f, nrhs):
    say("po", ny, nx, k, f, nrhs)
    prob = make_problem(ny, nx, k, f, seed=600 + ny, noise="hetero", mask_frac=0.1)
    xi, zeta = po_draws(prob, nrhs, seed=601)
    dp = sy.DeviceProblem.from_numpy(prob)
    eta = host(sy.po_perturb(dp, dev(xi), dev(zeta)))
    assert rel(eta, opo.perturbation(prob, xi, zeta)) < 1e-13


# --------------------------------------------------------------------------------------- solves

def _solve(prob, precision, tol, precond=sy.SYLV_PC_BLOCK, X0=None, max_iter=5000,
           check_every=0):
    dp = sy.DeviceProblem.from_numpy(prob)
    opts = sy.SolveOptions(tol=tol, max_iter=max_iter, precision=precision, precond=precond,
                           check_every=check_every)
    X, st = sy.pcg_solve(dp, Y=dev(prob.Y), X0=None if X0 is None else dev(X0), opts=opts)
    return host(X), st[0]


@pytest.mark.parametrize("precision,bound", [(sy.SYLV_PREC_F64, 1e-8), (sy.SYLV_PREC_MIXED, 1e-7)])
@pytest.mark.parametrize("ny,nx,k,f,noise,mask", [
    (16, 16, 3, 6, "hetero", 0.0), (24, 20, 4, 9, "hetero", 0.1), (13, 29, 2, 3, "homo", 0.0),
    (1, 1, 3, 4, "hetero", 0.0), (2, 3, 3, 5, "hetero", 0.0), (8, 70, 5, 7, "separable", 0.2),
])
def test_solve_dense(precision, bound, ny, nx, k, f, noise, mask):
    say("solve dense", precision, ny, nx, k, f, noise, mask)
    prob = make_problem(ny, nx, k, f, seed=700 + ny + nx, noise=noise, mask_frac=mask)
    x, st = _solve(prob, precision, tol=1e-12 if precision == sy.SYLV_PREC_F64 else 1e-11)
    assert st["status"] == 0, st
    xs = osv.solve_dense(prob)
    assert rel(x, xs) < bound
    assert st["relres_true"] <= (1e-12 if precision == sy.SYLV_PREC_F64 else 1e-11) * 1.01
    # independent check of the reported residual (equal up to the rounding of the residual
    # itself, ~1e-16 * cond(G))
    b = op.rhs(prob)
    res = rel(op.apply(prob, x), b)
    assert res == pytest.approx(st["relres_true"], rel=1e-2, abs=1e-13)


@pytest.mark.parametrize("precision,bound", [(sy.SYLV_PREC_F64, 1e-8), (sy.SYLV_PREC_MIXED, 1e-7)])
def test_solve_tiny_workload_fft(precision, bound):
    """64 x 64, k = 3, f = 6, homoscedastic: exact Fourier solution."""
    prob = workload("tiny_64")[0]
    say("solve tiny_64", precision)
    x, st = _solve(prob, precision, tol=1e-12 if precision == sy.SYLV_PREC_F64 else 1e-11)
    assert st["status"] == 0, st
    assert rel(x, osv.solve_fft(prob)) < bound


@pytest.mark.parametrize("precision,bound,tol", [(sy.SYLV_PREC_F64, 1e-8, 1e-11),
                                                 (sy.SYLV_PREC_MIXED, 1e-7, 1e-10)])
def test_solve_full_size_homoscedastic_fft(precision, bound, tol):
    """1024 x 1024, k = 3, f = 9 with homoscedastic noise: the Fourier solve is exact at this
    size, so the whole solution is compared."""
    prob = make_problem(1024, 1024, 3, 9, seed=1001, noise="homo")
    say("solve 1024^2 homo", precision)
    x, st = _solve(prob, precision, tol=tol)
    assert st["status"] == 0, st
    assert rel(x, osv.solve_fft(prob)) < bound


@pytest.mark.parametrize("precision", [sy.SYLV_PREC_F64, sy.SYLV_PREC_MIXED])
def test_solve_full_size_heteroscedastic(precision):
    """The 1024^2 heteroscedastic workload at its timing tolerance 1e-8: the oracle recomputes
    the true residual of the GPU result with its own assembled operator, and single outputs of
    the operator at sampled pixels are compared one by one."""
    prob = workload("het_1024")[0]
    say("solve het_1024", precision)
    x, st = _solve(prob, precision, tol=1e-8)
    assert st["status"] == 0, st
    b = op.rhs(prob)
    G = op.posterior_precision(prob)
    res = rel(op.apply(prob, x, G=G), b)
    assert res <= 1e-8 * 1.001
    assert res == pytest.approx(st["relres_true"], rel=1e-3)
    pix = np.random.default_rng(9).choice(prob.n_pix, 64, replace=False)
    dp = sy.DeviceProblem.from_numpy(prob)
    Yg = host(sy.apply(dp, dev(x)))
    assert rel(Yg[:, pix], op.apply_at(prob, x, pix)) < 1e-13


@pytest.mark.parametrize("precision", [sy.SYLV_PREC_F64, sy.SYLV_PREC_MIXED])
def test_solve_full_size_masked_2048(precision):
    """The 2048^2, k = 4, f = 9 workload with 10 % masked pixels at its timing tolerance 1e-8
    (4096 partials per reduction, so the CG reductions are folded in a separate kernel): the
    residual b - G x at sampled pixels (random ones, the first row and column, masked ones),
    computed by the oracle's operator, is small, and the recursive and true residuals agree."""
    prob = workload("masked_2048")[0]
    say("solve masked_2048", precision)
    x, st = _solve(prob, precision, tol=1e-8)
    assert st["status"] == 0 and st["relres_true"] <= 1e-8, st
    rng = np.random.default_rng(2048)
    masked = np.flatnonzero(prob.W[0] == 0.0)
    edge = np.concatenate([np.arange(0, prob.nx, 5), np.arange(0, prob.n_pix, 5 * prob.nx)])
    pix = np.unique(np.concatenate([rng.choice(prob.n_pix, 1500, replace=False), edge,
                                    masked[:200]]))
    gx = op.apply_at(prob, x, pix)
    b = prob.A.T @ (prob.W[:, pix] * prob.Y[:, pix])
    assert rel(gx, b) < 3e-8


def test_backward_full_size_512():
    """The 512^2, k = 4, f = 9 differentiable-solve workload at its tolerance 1e-10: the forward
    and adjoint solutions satisfy G x = b and G lambda = gbar at sampled pixels (the oracle's
    operator, one pixel at a time), and every gradient equals the oracle's contraction
    lambda^T (db/dtheta - dG/dtheta x) formed from the GPU's own x and lambda."""
    prob = workload("grad_512")[0]
    dp = sy.DeviceProblem.from_numpy(prob)
    opts = sy.SolveOptions(tol=1e-10)
    say("backward grad_512")
    X, st = sy.pcg_solve(dp, Y=dev(prob.Y), opts=opts)
    assert st[0]["status"] == 0, st
    gbar = random_maps(prob, 5120)
    lam, g, stb = sy.pcg_backward(dp, dev(prob.Y), X.reshape(prob.k, prob.n_pix), dev(gbar), opts)
    assert stb["status"] == 0 and stb["relres_true"] <= 1e-10, stb
    x, lm = host(X).reshape(prob.k, prob.n_pix), host(lam)
    pix = np.unique(np.concatenate([np.random.default_rng(512).choice(prob.n_pix, 1500,
                                                                       replace=False),
                                    np.arange(0, prob.nx, 3)]))
    b = prob.A.T @ (prob.W[:, pix] * prob.Y[:, pix])
    assert rel(op.apply_at(prob, x, pix), b) < 1e-9
    assert rel(op.apply_at(prob, lm, pix), gbar[:, pix]) < 1e-9
    g_ref = og.implicit_grads(prob, x, lm)
    for name in ("kappa", "tau", "A", "W", "Y"):
        assert rel(host(g[name]), g_ref[name]) < 1e-10, name


@pytest.mark.parametrize("block", [0, 1])
def test_batched_full_size_8grids(block):
    """The 8 uneven grids (256^2 .. 1024^2) x 8 perturbation-optimisation right-hand sides of
    the batched workload, mixed precision to 1e-8, independent and block CG in one call: every
    one of the 64 solutions satisfies G x = b + eta at sampled pixels (oracle operator; eta from
    the GPU's perturbation map, which its own tests pin)."""
    from workloads import WORKLOADS
    probs = workload("batched_8grids")
    nrhs = WORKLOADS["batched_8grids"]["nrhs"]
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    etas = []
    for g_, (p, d) in enumerate(zip(probs, dps)):
        xi, zeta = po_draws(p, nrhs, seed=7700 + g_)
        etas.append(host(sy.po_perturb(d, dev(xi), dev(zeta))).reshape(nrhs, p.k, p.n_pix))
    Y = torch.cat([dev(p.Y.ravel()) for p in probs])
    B = torch.cat([dev(e.ravel()) for e in etas])
    say("batched full size, block", block)
    X, st = sy.pcg_solve(dps, Y=Y, Bextra=B, nrhs=nrhs,
                         opts=sy.SolveOptions(tol=1e-8, precision=sy.SYLV_PREC_MIXED, block=block))
    X = host(X)
    rng = np.random.default_rng(88)
    off = 0
    for g_, p in enumerate(probs):
        pix = rng.choice(p.n_pix, 300, replace=False)
        b = p.A.T @ (p.W[:, pix] * p.Y[:, pix])
        for r in range(nrhs):
            s_ = st[g_ * nrhs + r]
            assert s_["status"] == 0 and s_["relres_true"] <= 1e-8, (g_, r, s_)
            x = X[off:off + p.k * p.n_pix].reshape(p.k, p.n_pix)
            off += p.k * p.n_pix
            assert rel(op.apply_at(p, x, pix), b + etas[g_][r][:, pix]) < 3e-8, (g_, r)


def test_solve_warm_start_and_zero_rhs():
    prob = make_problem(20, 24, 3, 5, seed=800)
    xs = osv.solve_dense(prob)
    say("warm start")
    x, st = _solve(prob, sy.SYLV_PREC_F64, 1e-12, X0=xs + 1e-3 * random_maps(prob, 1))
    assert st["status"] == 0 and rel(x, xs) < 1e-8
    say("zero rhs")
    prob0 = make_problem(20, 24, 3, 5, seed=801)
    prob0.Y[:] = 0.0
    x0, st0 = _solve(prob0, sy.SYLV_PREC_F64, 1e-10)
    assert st0["status"] == 0 and st0["iters"] == 0 and np.all(x0 == 0)


@pytest.mark.parametrize("precision", [sy.SYLV_PREC_F64, sy.SYLV_PREC_MIXED])
def test_sweep_warm_start_saves_iterations(precision):
    """Repeated solves over a hyperparameter sweep: with the stopping test relative to ||b||, a
    solve warm-started from the previous parameter's solution meets the same tolerance in fewer
    iterations and agrees with the dense solution."""
    prob = make_problem(40, 36, 3, 6, seed=810, noise="hetero")
    dp = sy.DeviceProblem.from_numpy(prob)
    Y = dev(prob.Y)
    say("sweep warm start", precision)
    tol = 1e-10
    o = sy.SolveOptions(tol=tol, precision=precision, stop_ref=sy.SYLV_STOP_B)
    X0, st0 = sy.pcg_solve(dp, Y=Y, opts=o)
    assert st0[0]["status"] == 0
    prob.kappa = prob.kappa * 1.01
    prob.tau = prob.tau * 0.99
    dp.kappa.copy_(dev(prob.kappa))
    dp.tau.copy_(dev(prob.tau))
    Xc, stc = sy.pcg_solve(dp, Y=Y, opts=o)
    Xw, stw = sy.pcg_solve(dp, Y=Y, X0=X0, opts=o)
    assert stc[0]["status"] == 0 and stw[0]["status"] == 0
    assert stw[0]["iters"] < stc[0]["iters"], (stw, stc)
    xs = osv.solve_dense(prob)
    bound = 1e-7 if precision == sy.SYLV_PREC_F64 else 1e-6
    for X in (Xc, Xw):
        assert rel(host(X).reshape(xs.shape), xs) < bound
    assert stw[0]["relres_true"] <= tol * 1.01
    # with x0 = 0 both references give the same threshold, hence the same run
    Xr, str_ = sy.pcg_solve(dp, Y=Y, opts=sy.SolveOptions(tol=tol, precision=precision))
    assert str_[0]["iters"] == stc[0]["iters"] and np.array_equal(host(Xr), host(Xc))


def test_solve_fully_masked_uses_prior_only():
    prob = make_problem(12, 12, 2, 3, seed=802, mask_frac=0.0)
    prob.W[:] = 0.0
    say("fully masked")
    dp = sy.DeviceProblem.from_numpy(prob)
    Bx = random_maps(prob, 3)
    opts = sy.SolveOptions(tol=1e-12)
    X, st = sy.pcg_solve(dp, Bextra=dev(Bx), opts=opts)
    assert st[0]["status"] == 0
    assert rel(host(X), osv.solve_dense(prob, b=Bx)) < 1e-8


@pytest.mark.parametrize("precision", [sy.SYLV_PREC_F64, sy.SYLV_PREC_MIXED])
def test_folded_reductions_match(precision, monkeypatch):
    """Large grids fold the CG partials in a separate kernel before their consumers; forcing that
    path on small grids (threshold 0) gives the same iterations and, up to the summation order of
    the dot products, the same solution as the default path, also in a batch of uneven grids."""
    probs = [make_problem(s0, s1, 3, 5, seed=820 + i, noise="hetero")
             for i, (s0, s1) in enumerate([(20, 18), (9, 33), (24, 24)])]
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    Y = torch.cat([dev(p.Y.ravel()) for p in probs])
    opts = sy.SolveOptions(tol=1e-10, precision=precision)
    say("folded reductions", precision)
    Xa, sa = sy.pcg_solve(dps, Y=Y, opts=opts)
    monkeypatch.setenv("SYLV_PREREDUCE_MIN", "0")
    Xb, sb = sy.pcg_solve(dps, Y=Y, opts=opts)
    monkeypatch.delenv("SYLV_PREREDUCE_MIN")
    assert all(a["status"] == 0 and b["status"] == 0 for a, b in zip(sa, sb)), (sa, sb)
    for a, b in zip(sa, sb):
        assert abs(a["iters"] - b["iters"]) <= 1, (a, b)
    xa, xb = host(Xa), host(Xb)
    assert rel(xb, xa) < 1e-8
    off = 0
    for p in probs:
        n = p.k * p.n_pix
        assert rel(xb[off:off + n].reshape(p.k, p.n_pix), osv.solve_dense(p)) < 1e-7
        off += n


@pytest.mark.parametrize("precision", [sy.SYLV_PREC_F64, sy.SYLV_PREC_MIXED])
def test_iterate_complete_at_every_stop(precision):
    """Runs stopped after j = 1..7 iterations (odd and even: float64 runs advance x two steps at a
    time and flush a pending step when they stop) hold the j-th iterate: the recomputed residual
    b - G x equals the recursive residual of the run."""
    prob = make_problem(40, 36, 3, 5, seed=830, noise="hetero")
    dp = sy.DeviceProblem.from_numpy(prob)
    say("stops", precision)
    for j in range(1, 8):
        X, st = sy.pcg_solve(dp, Y=dev(prob.Y), opts=sy.SolveOptions(
            tol=1e-14, max_iter=j, precision=sy.SYLV_PREC_F64, check_every=1))
        s0 = st[0]
        assert s0["status"] == sy.binding.SYLV_NOT_CONVERGED and s0["iters"] == j, s0
        assert s0["relres_true"] == pytest.approx(s0["relres_rec"], rel=1e-9), (j, s0)
        x = host(X).reshape(prob.k, prob.n_pix)
        assert rel(op.apply(prob, x), op.rhs(prob)) == pytest.approx(s0["relres_true"], rel=1e-6)
    if precision == sy.SYLV_PREC_MIXED:
        X, st = sy.pcg_solve(dp, Y=dev(prob.Y), opts=sy.SolveOptions(tol=1e-10, precision=precision))
        assert st[0]["status"] == 0
        assert rel(host(X).reshape(prob.k, prob.n_pix), osv.solve_dense(prob)) < 1e-7


def test_solve_not_converged_reported():
    prob = make_problem(32, 32, 3, 6, seed=803)
    say("max_iter=2")
    x, st = _solve(prob, sy.SYLV_PREC_F64, 1e-12, max_iter=2, check_every=1)
    assert st["status"] == sy.binding.SYLV_NOT_CONVERGED
    assert st["iters"] == 2


def test_solve_nonfinite_reported():
    prob = make_problem(16, 16, 3, 6, seed=804)
    prob.W[2, 17] = np.nan
    say("nan weight")
    x, st = _solve(prob, sy.SYLV_PREC_F64, 1e-10)
    assert st["status"] == sy.binding.SYLV_NONFINITE


def test_solve_negative_tau_reported():
    prob = make_problem(16, 16, 3, 6, seed=805, tau=np.array([1.0, -3.0, 1.0]))
    say("negative tau")
    x, st = _solve(prob, sy.SYLV_PREC_F64, 1e-10, precond=sy.SYLV_PC_NONE)
    assert st["status"] in (sy.binding.SYLV_BREAKDOWN, sy.binding.SYLV_NONFINITE,
                            sy.binding.SYLV_NOT_CONVERGED)


def test_solve_repeatable_bitwise():
    prob = make_problem(48, 40, 3, 6, seed=806)
    say("repeatability")
    x1, s1 = _solve(prob, sy.SYLV_PREC_F64, 1e-10)
    x2, s2 = _solve(prob, sy.SYLV_PREC_F64, 1e-10)
    assert np.array_equal(x1, x2) and s1 == s2
    m1, _ = _solve(prob, sy.SYLV_PREC_MIXED, 1e-10)
    m2, _ = _solve(prob, sy.SYLV_PREC_MIXED, 1e-10)
    assert np.array_equal(m1, m2)


@pytest.mark.parametrize("precision", [sy.SYLV_PREC_F64, sy.SYLV_PREC_MIXED])
def test_batched_uneven_grids_with_po_rhs(precision):
    """Several uneven grids x several perturbed right-hand sides in one call; each equals the
    oracle's solve of its own right-hand side."""
    probs = [make_problem(s0, s1, 3, 4, seed=900 + i, noise="hetero")
             for i, (s0, s1) in enumerate([(16, 16), (24, 20), (9, 33)])]
    nrhs = 3
    say("batched", precision)
    Ycat, Bcat, etas = [], [], []
    for i, p in enumerate(probs):
        xi, zeta = po_draws(p, nrhs, seed=950 + i)
        eta = opo.perturbation(p, xi, zeta)
        etas.append(eta)
        Ycat.append(p.Y.ravel())
        Bcat.append(eta.ravel())
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    opts = sy.SolveOptions(tol=1e-12 if precision == sy.SYLV_PREC_F64 else 1e-11,
                           precision=precision)
    X, st = sy.pcg_solve(dps, Y=dev(np.concatenate(Ycat)), Bextra=dev(np.concatenate(Bcat)),
                         opts=opts, nrhs=nrhs)
    X = host(X)
    off = 0
    bound = 1e-8 if precision == sy.SYLV_PREC_F64 else 1e-7
    for i, p in enumerate(probs):
        blk = X[off:off + nrhs * p.k * p.n_pix].reshape(nrhs, p.k, p.n_pix)
        off += nrhs * p.k * p.n_pix
        b = op.rhs(p)
        for r in range(nrhs):
            assert st[i * nrhs + r]["status"] == 0, st[i * nrhs + r]
            xs = osv.solve_dense(p, b=b + etas[i][r])
            assert rel(blk[r], xs) < bound


# ------------------------------------------------------------------------------------- gradients

@pytest.mark.parametrize("ny,nx,k,f", [(12, 10, 3, 4), (7, 5, 2, 9), (16, 16, 4, 9)])
def test_backward_matches_oracle(ny, nx, k, f):
    prob = make_problem(ny, nx, k, f, seed=1100 + ny, noise="hetero", mask_frac=0.1)
    gbar = random_maps(prob, 1101)
    say("backward", ny, nx, k, f)
    g_ref, xs, lam_ref = og.adjoint_solution_grads(prob, gbar, return_solution=True)
    dp = sy.DeviceProblem.from_numpy(prob)
    lam, g, st = sy.pcg_backward(dp, dev(prob.Y), dev(xs), dev(gbar),
                                 sy.SolveOptions(tol=1e-13))
    assert st["status"] == 0, st
    assert rel(host(lam), lam_ref) < 1e-9
    for name in ("kappa", "tau", "A", "W", "Y"):
        assert rel(host(g[name]), g_ref[name]) < 1e-8, name


@pytest.mark.parametrize("kind", ["fourier", "fourier_diag", "fourier_block"])
def test_backward_with_fourier_preconditioners_matches_oracle(kind):
    """The adjoint solve and the gradients with each Fourier preconditioner (16 x 32 periodic
    grid, 10 % masked): the same oracle values as with block-Jacobi."""
    prob = make_problem(16, 32, 3, 6, seed=1150, noise="hetero", mask_frac=0.1)
    gbar = random_maps(prob, 1151)
    g_ref, xs, lam_ref = og.adjoint_solution_grads(prob, gbar, return_solution=True)
    dp = sy.DeviceProblem.from_numpy(prob)
    pc = {"fourier": sy.SYLV_PC_FOURIER, "fourier_diag": sy.SYLV_PC_FOURIER_DIAG,
          "fourier_block": sy.SYLV_PC_FOURIER_BLOCK}[kind]
    say("backward", kind)
    lam, g, st = sy.pcg_backward(dp, dev(prob.Y), dev(xs), dev(gbar),
                                 sy.SolveOptions(tol=1e-13, precond=pc))
    assert st["status"] == 0, st
    assert rel(host(lam), lam_ref) < 1e-9
    for name in ("kappa", "tau", "A", "W", "Y"):
        assert rel(host(g[name]), g_ref[name]) < 1e-8, name


def test_autograd_function_loss_gradient():
    """The differentiable-solve loss at 16 x 16 (k = 4, f = 9): torch autograd through
    SylvSolve equals the oracle's total gradient."""
    prob = make_problem(16, 16, 4, 9, seed=1200, noise="hetero")
    xt = random_maps(prob, 1201)
    say("autograd")
    g_ref, _, _ = og.loss_grads(prob, xt)
    kappa = dev(prob.kappa).requires_grad_(True)
    tau = dev(prob.tau).requires_grad_(True)
    A = dev(prob.A).requires_grad_(True)
    W = dev(prob.W).requires_grad_(True)
    Y = dev(prob.Y).requires_grad_(True)
    X = sy.SylvSolve.apply(kappa, tau, A, W, Y, prob.ny, prob.nx, sy.SolveOptions(tol=1e-13))
    resid = Y - A @ X
    loss = ((X - dev(xt)) ** 2).sum() + 0.5 * (W * resid * resid).sum()
    loss.backward()
    for name, t in (("kappa", kappa), ("tau", tau), ("A", A), ("W", W), ("Y", Y)):
        assert rel(host(t.grad), g_ref[name]) < 1e-7, name


# ------------------------------------------------------------------------------------ block CG

def _batched_inputs(probs, nrhs, seed0):
    Ycat, Bcat, etas = [], [], []
    for i, p in enumerate(probs):
        xi, zeta = po_draws(p, nrhs, seed=seed0 + i)
        eta = opo.perturbation(p, xi, zeta)
        etas.append(eta)
        Ycat.append(p.Y.ravel())
        Bcat.append(eta.ravel())
    return np.concatenate(Ycat), np.concatenate(Bcat), etas


def _check_batched(probs, X, st, nrhs, bextra_list, bound, use_y=True):
    off = 0
    for i, p in enumerate(probs):
        blk = X[off:off + nrhs * p.k * p.n_pix].reshape(nrhs, p.k, p.n_pix)
        off += nrhs * p.k * p.n_pix
        b = op.rhs(p) if use_y else 0.0
        for r in range(nrhs):
            s = st[i * nrhs + r]
            assert s["status"] == 0, (i, r, s)
            xs = osv.solve_dense(p, b=b + bextra_list[i][r])
            assert rel(blk[r], xs) < bound, (i, r, rel(blk[r], xs))


@pytest.mark.parametrize("precision,bound", [(sy.SYLV_PREC_F64, 1e-8), (sy.SYLV_PREC_MIXED, 1e-7)])
@pytest.mark.parametrize("nrhs", [2, 4, 8])
def test_block_cg_uneven_grids(precision, bound, nrhs):
    probs = [make_problem(s0, s1, 3, 5, seed=1300 + i, noise="hetero", mask_frac=0.05)
             for i, (s0, s1) in enumerate([(16, 16), (20, 28), (9, 33)])]
    say("block cg", precision, nrhs)
    Y, B, etas = _batched_inputs(probs, nrhs, 1350)
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    opts = sy.SolveOptions(tol=1e-12 if precision == sy.SYLV_PREC_F64 else 1e-11,
                           precision=precision, block=1)
    X, st = sy.pcg_solve(dps, Y=dev(Y), Bextra=dev(B), opts=opts, nrhs=nrhs)
    _check_batched(probs, host(X), st, nrhs, etas, bound)


@pytest.mark.parametrize("precision,bound", [(sy.SYLV_PREC_F64, 1e-8), (sy.SYLV_PREC_MIXED, 1e-7)])
def test_block_cg_degenerate_columns(precision, bound):
    """A zero right-hand side (converged at once, deflated) and two identical columns (singular
    Gram matrices: the group falls back to independent CG) must still solve every column."""
    p = make_problem(18, 22, 3, 4, seed=1400, noise="hetero")
    nrhs = 4
    rng = np.random.default_rng(1401)
    Bx = rng.standard_normal((nrhs, p.k, p.n_pix))
    Bx[1] = 0.0
    Bx[3] = Bx[2]
    say("block cg degenerate", precision)
    dp = sy.DeviceProblem.from_numpy(p)
    opts = sy.SolveOptions(tol=1e-12 if precision == sy.SYLV_PREC_F64 else 1e-11,
                           precision=precision, block=1)
    X, st = sy.pcg_solve([dp], Bextra=dev(Bx.ravel()), opts=opts, nrhs=nrhs)
    X = host(X).reshape(nrhs, p.k, p.n_pix)
    for r in range(nrhs):
        assert st[r]["status"] == 0, (r, st[r])
        xs = osv.solve_dense(p, b=Bx[r])
        if r == 1:
            assert np.all(X[r] == 0.0)
        else:
            assert rel(X[r], xs) < bound, (r, rel(X[r], xs))


def test_block_cg_needs_fewer_iterations():
    """Block CG over 8 right-hand sides searches an 8-times larger Krylov space per iteration:
    it must not need more iterations than independent CG on the same columns."""
    p = make_problem(48, 48, 3, 6, seed=1500, noise="hetero")
    nrhs = 8
    xi, zeta = po_draws(p, nrhs, seed=1501)
    eta = opo.perturbation(p, xi, zeta)
    dp = sy.DeviceProblem.from_numpy(p)
    say("block vs independent iterations")
    its = {}
    for block in (0, 1):
        opts = sy.SolveOptions(tol=1e-10, block=block)
        X, st = sy.pcg_solve([dp], Y=dev(p.Y), Bextra=dev(eta.ravel()), opts=opts, nrhs=nrhs)
        assert all(s["status"] == 0 for s in st)
        its[block] = max(s["iters"] for s in st)
    assert its[1] <= its[0]


@pytest.mark.parametrize("s", [2, 4, 8])
def test_block_cg_iterates_match_oracle_block_pcg(s):
    """Runs stopped after j = 1..5 block iterations hold the oracle's block-CG iterates (O'Leary's
    recurrence; float64, no preconditioner so that both sides apply the same operator): this
    shows the block recurrence is the one taken, since independent CG's iterates differ."""
    from oracle import block_pcg as obp
    p = make_problem(20, 18, 2, 3, seed=1550 + s, noise="hetero")
    rng = np.random.default_rng(1551)
    B = rng.standard_normal((s, p.k * p.n_pix))
    dp = sy.DeviceProblem.from_numpy(p)
    its = obp.block_pcg(p, B, max_iter=5, precond="none")
    say("block iterates vs oracle, s =", s)
    for j in range(1, 6):
        for block in (1, 0):
            X, st = sy.pcg_solve([dp], Bextra=dev(B.ravel()), nrhs=s, opts=sy.SolveOptions(
                tol=1e-15, max_iter=j, block=block, block_size=s if block else 0,
                precond=sy.SYLV_PC_NONE, check_every=1))
            assert all(c["status"] == sy.binding.SYLV_NOT_CONVERGED and c["iters"] == j
                       for c in st), st
            e = rel(host(X).reshape(s, -1), its[j])
            if block:
                assert e < 1e-9, (j, e)
            elif j >= 2:
                assert e > 1e-4, (j, e)       # independent CG is a different iteration


def test_block_cg_rejects_unsupported_block_size():
    p = make_problem(8, 8, 2, 3, seed=1600)
    dp = sy.DeviceProblem.from_numpy(p)
    with pytest.raises(sy.SylvError):
        sy.pcg_solve([dp], Bextra=dev(np.ones(3 * 2 * 64)), opts=sy.SolveOptions(block=1),
                     nrhs=3)


def test_float64_true_residual_meets_tolerance():
    """Residual replacement: the recomputed float64 residual of every column meets the tolerance
    even where the recursive residual drifts (batched uneven grids, independent and block CG)."""
    probs = [make_problem(s0, s0, 3, 6, seed=1700 + i, noise="hetero") for i, s0 in
             enumerate([64, 96, 128])]
    nrhs = 4
    Y, B, _ = _batched_inputs(probs, nrhs, 1750)
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    for block in (0, 1):
        say("true residual", block)
        opts = sy.SolveOptions(tol=1e-8, block=block)
        X, st = sy.pcg_solve(dps, Y=dev(Y), Bextra=dev(B), opts=opts, nrhs=nrhs)
        X = host(X)
        off = 0
        for i, p in enumerate(probs):
            blk = X[off:off + nrhs * p.k * p.n_pix].reshape(nrhs, p.k, p.n_pix)
            off += nrhs * p.k * p.n_pix
            for r in range(nrhs):
                s_ = st[i * nrhs + r]
                assert s_["status"] == 0 and s_["relres_true"] <= 1e-8, s_


def test_float64_final_update_reaches_every_tile():
    """The apply that stops a run still adds its x update on every tile: the recomputed residual
    of a 1024^2 float64 solve (4096 workgroups, far more than run at once) matches the
    recursive one and no residual-replacement restart is needed."""
    p = make_problem(1024, 1024, 3, 9, seed=1800, noise="hetero")
    dp = sy.DeviceProblem.from_numpy(p)
    say("final update 1024^2 f64")
    X, st = sy.pcg_solve([dp], Y=dev(p.Y), opts=sy.SolveOptions(tol=1e-8))
    s_ = st[0]
    assert s_["status"] == 0 and s_["outer"] == 1, s_
    assert s_["relres_true"] <= 1e-8, s_
    assert s_["relres_true"] == pytest.approx(s_["relres_rec"], rel=0.05), s_


@pytest.mark.parametrize("precision", [sy.SYLV_PREC_F64, sy.SYLV_PREC_MIXED])
def test_streaming_cache_policy_changes_no_result(precision, monkeypatch):
    """Working sets beyond the last-level cache switch the CG kernels and applies to
    non-temporal loads or stores (SYLV_STREAM forces either policy): a cache hint only, so
    solves and applies are bitwise the same under both, and match the oracle."""
    prob = make_problem(36, 40, 4, 9, seed=1580, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(prob)
    Xr = random_maps(prob, seed=1581)
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("SYLV_STREAM", mode)
        say("streaming policy", mode, "precision", precision)
        X, st = sy.pcg_solve(dp, Y=dev(prob.Y), opts=sy.SolveOptions(
            tol=1e-12 if precision == sy.SYLV_PREC_F64 else 1e-11, precision=precision))
        assert st[0]["status"] == 0, st
        dt = torch.float64 if precision == sy.SYLV_PREC_F64 else torch.float32
        Y = sy.apply(dp, dev(Xr, dt))
        out[mode] = (host(X), host(Y), st[0]["iters"])
    assert np.array_equal(out["0"][0], out["1"][0]) and out["0"][2] == out["1"][2]
    assert np.array_equal(out["0"][1], out["1"][1])
    bound = 1e-8 if precision == sy.SYLV_PREC_F64 else 1e-7
    assert rel(out["1"][0].reshape(prob.k, prob.n_pix), osv.solve_dense(prob)) <= bound
