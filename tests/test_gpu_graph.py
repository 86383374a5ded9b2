"""The fixed schedule (every iteration queued at once, no host synchronisation) and HIP graph
capture of solves and applies, through the C ABI.

Both schedules launch the same kernels in the same order and every stopping decision is taken on
the device with fixed-order reductions, so the fixed schedule must reproduce the adaptive one
bitwise.  A captured graph is replayed several times with eager work and synchronisations between
the replays; every replay must equal the eager call bitwise, and the eager results are checked
against the oracle's dense solve."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2204_08057_amd as sy  # noqa: E402
from paper_2204_08057_amd import binding as bd  # noqa: E402
from oracle import operator as op  # noqa: E402
from oracle import po as opo  # noqa: E402
from oracle import solve as osv  # noqa: E402
from workloads import make_problem, po_draws, random_maps  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print("[graph]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def opts_for(precision, schedule, **kw):
    tol = 1e-12 if precision == sy.SYLV_PREC_F64 else 1e-11
    base = dict(tol=tol, precision=precision, max_iter=400, refine_max=4, schedule=schedule)
    base.update(kw)
    return sy.SolveOptions(**base)


def buffers(probs, nrhs, opts):
    total = sum(nrhs * p.k * p.n_pix for p in probs)
    X = torch.zeros(total, dtype=torch.float64, device="cuda")
    stats = torch.zeros(len(probs) * nrhs * bd.STATS_BYTES, dtype=torch.uint8, device="cuda")
    ws = torch.empty(sy.workspace_bytes(probs, nrhs, opts), dtype=torch.uint8, device="cuda")
    return X, stats, ws


def capture(fn):
    """Capture fn() into a graph after one warm-up call on a side stream."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


PRECISIONS = [(sy.SYLV_PREC_F64, 1e-8), (sy.SYLV_PREC_MIXED, 1e-7)]


@pytest.mark.parametrize("precision,bound", PRECISIONS)
def test_fixed_schedule_equals_adaptive(precision, bound):
    p = make_problem(40, 36, 3, 6, seed=7000, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(p)
    say("fixed vs adaptive", precision)
    Xa, sa = sy.pcg_solve(dp, Y=dev(p.Y), opts=opts_for(precision, sy.SYLV_SCHED_ADAPTIVE))
    Xf, sf = sy.pcg_solve(dp, Y=dev(p.Y), opts=opts_for(precision, sy.SYLV_SCHED_FIXED))
    assert sa[0]["status"] == 0, sa
    assert sa[0]["outer"] == (1 if precision == sy.SYLV_PREC_F64 else sa[0]["outer"])
    assert sf == sa
    assert torch.equal(Xf, Xa)
    assert rel(host(Xf), osv.solve_dense(p)) < bound


def test_fixed_schedule_caps_report_not_converged():
    """Too few queued iterations: the run stops at the cap and says so."""
    p = make_problem(32, 32, 3, 6, seed=7050, noise="hetero")
    dp = sy.DeviceProblem.from_numpy(p)
    say("fixed cap")
    for precision in (sy.SYLV_PREC_F64, sy.SYLV_PREC_MIXED):
        o = opts_for(precision, sy.SYLV_SCHED_FIXED, max_iter=5, refine_max=1)
        Xf, sf = sy.pcg_solve(dp, Y=dev(p.Y), opts=o)
        oa = opts_for(precision, sy.SYLV_SCHED_ADAPTIVE, max_iter=5, refine_max=1)
        Xa, sa = sy.pcg_solve(dp, Y=dev(p.Y), opts=oa)
        assert sf[0]["status"] in (bd.SYLV_NOT_CONVERGED, bd.SYLV_STAGNATED), sf
        assert sf == sa and torch.equal(Xf, Xa)


@pytest.mark.parametrize("precision,bound", PRECISIONS)
def test_graph_replays_equal_eager(precision, bound):
    p = make_problem(48, 40, 3, 6, seed=7100, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(p)
    Yd = dev(p.Y)
    opts = opts_for(precision, sy.SYLV_SCHED_FIXED)
    X, stats, ws = buffers([dp], 1, opts)
    launch = sy.solve_launcher(dp, X, stats, ws, Y=Yd, opts=opts)

    def solve():
        X.zero_()   # x0 = 0 (a fill kernel, part of the graph)
        launch()

    say("eager", precision)
    solve()
    torch.cuda.synchronize()
    Xe, se = X.clone(), sy.stats_list(stats, 1)
    assert se[0]["status"] == 0, se
    assert rel(host(Xe).reshape(p.k, p.n_pix), osv.solve_dense(p)) < bound
    say("capture", precision)
    g = capture(solve)
    for rep in range(3):
        X.fill_(1.0e3 + rep)          # eager work between replays
        stats.zero_()
        torch.cuda.synchronize()
        say("replay", rep)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(X, Xe), rep
        assert sy.stats_list(stats, 1) == se, rep
    # new observations written in place: the same graph solves the new system
    Y2 = p.Y * 0.5 + np.random.default_rng(7101).standard_normal(p.Y.shape)
    Yd.copy_(dev(Y2))
    say("replay with new Y")
    g.replay()
    torch.cuda.synchronize()
    q = make_problem(48, 40, 3, 6, seed=7100, noise="hetero", mask_frac=0.1)
    q.Y = Y2
    Xa, sa = sy.pcg_solve(dp, Y=dev(Y2), opts=opts_for(precision, sy.SYLV_SCHED_ADAPTIVE))
    assert torch.equal(X.reshape(p.k, p.n_pix), Xa)
    assert sy.stats_list(stats, 1) == sa
    assert rel(host(X).reshape(p.k, p.n_pix), osv.solve_dense(q)) < bound


def test_graph_block_cg_uneven_grids():
    """Block CG over 4 right-hand sides on two uneven grids (mixed precision), captured once."""
    probs = [make_problem(16, 16, 3, 5, seed=7200, noise="hetero"),
             make_problem(20, 28, 3, 5, seed=7201, noise="hetero", mask_frac=0.05)]
    nrhs = 4
    etas, Ycat, Bcat = [], [], []
    for i, p in enumerate(probs):
        xi, zeta = po_draws(p, nrhs, seed=7210 + i)
        eta = opo.perturbation(p, xi, zeta)
        etas.append(eta)
        Ycat.append(p.Y.ravel())
        Bcat.append(eta.ravel())
    Yd, Bd = dev(np.concatenate(Ycat)), dev(np.concatenate(Bcat))
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    opts = opts_for(sy.SYLV_PREC_MIXED, sy.SYLV_SCHED_FIXED, block=1, max_iter=120, refine_max=3)
    X, stats, ws = buffers(dps, nrhs, opts)
    launch = sy.solve_launcher(dps, X, stats, ws, Y=Yd, Bextra=Bd, opts=opts, nrhs=nrhs)

    def solve():
        X.zero_()
        launch()

    say("block eager")
    solve()
    torch.cuda.synchronize()
    Xe, se = X.clone(), sy.stats_list(stats, len(probs) * nrhs)
    oa = opts_for(sy.SYLV_PREC_MIXED, sy.SYLV_SCHED_ADAPTIVE, block=1, max_iter=120,
                  refine_max=3)
    Xa, sa = sy.pcg_solve(dps, Y=Yd, Bextra=Bd, opts=oa, nrhs=nrhs)
    assert torch.equal(Xe, Xa) and se == sa
    off = 0
    Xh = host(Xe)
    for i, p in enumerate(probs):
        blk = Xh[off:off + nrhs * p.k * p.n_pix].reshape(nrhs, p.k, p.n_pix)
        off += nrhs * p.k * p.n_pix
        for r in range(nrhs):
            assert se[i * nrhs + r]["status"] == 0, se
            assert rel(blk[r], osv.solve_dense(p, b=op.rhs(p) + etas[i][r])) < 1e-7, (i, r)
    say("block capture")
    g = capture(solve)
    for rep in range(3):
        X.fill_(-7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(X, Xe), rep
        assert sy.stats_list(stats, len(probs) * nrhs) == se, rep


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-13), (torch.float32, 2e-6)])
def test_graph_apply_with_set_up(dtype, tol):
    """sylv_apply with prepared = 0 (operator set-up, table upload through kernel arguments and
    the apply) captured once; replays follow new X values written in place."""
    p = make_problem(37, 70, 4, 9, seed=7300, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(p)
    ws = torch.empty(sy.workspace_bytes([dp]), dtype=torch.uint8, device="cuda")
    X = dev(random_maps(p, 7301), dtype)
    Y = torch.empty_like(X)

    def run():
        sy.apply(dp, X, ws=ws, prepared=False, out=Y)

    say("apply capture", dtype)
    g = capture(run)
    for rep in range(3):
        Xn = random_maps(p, 7310 + rep)
        X.copy_(dev(Xn, dtype))
        Y.fill_(0.5)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        Yg = Y.clone()
        run()
        torch.cuda.synchronize()
        assert torch.equal(Yg, Y), rep
        ref = op.apply(p, Xn.astype(np.float32).astype(np.float64) if dtype == torch.float32 else Xn)
        assert rel(host(Yg), ref) < tol, rep


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")
def test_synchronising_calls_refused_under_capture():
    p = make_problem(16, 16, 3, 4, seed=7400, noise="hetero")
    dp = sy.DeviceProblem.from_numpy(p)
    opts = opts_for(sy.SYLV_PREC_F64, sy.SYLV_SCHED_ADAPTIVE)
    X, stats, ws = buffers([dp], 1, opts)
    launch = sy.solve_launcher(dp, X, stats, ws, Y=dev(p.Y), opts=opts)
    say("refusal")
    errors = []
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        try:
            launch()
        except sy.SylvError as e:
            errors.append(str(e))
    assert len(errors) == 1 and "captured" in errors[0], errors
    # the stream is usable afterwards
    Xa, sa = sy.pcg_solve(dp, Y=dev(p.Y), opts=opts)
    assert sa[0]["status"] == 0


def test_fixed_schedule_backward_equals_adaptive():
    """The adjoint solve and its gradient reductions under the fixed schedule (capturable) equal
    the adaptive call bitwise."""
    p = make_problem(24, 20, 3, 5, seed=7500, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(p)
    Yd = dev(p.Y)
    X, st = sy.pcg_solve(dp, Y=Yd, opts=opts_for(sy.SYLV_PREC_F64, sy.SYLV_SCHED_ADAPTIVE))
    gbar = dev(np.random.default_rng(7501).standard_normal((p.k, p.n_pix)))
    say("backward fixed vs adaptive")
    out = []
    for sched in (sy.SYLV_SCHED_ADAPTIVE, sy.SYLV_SCHED_FIXED):
        o = opts_for(sy.SYLV_PREC_F64, sched, tol=1e-12)
        out.append(sy.pcg_backward(dp, Yd, X, gbar, o))
    (la, ga, sa), (lf, gf, sf) = out
    assert sa["status"] == 0 and sa == sf
    assert torch.equal(la, lf)
    for name in ga:
        assert torch.equal(ga[name], gf[name]), name


@pytest.mark.parametrize("precision,bound", PRECISIONS)
def test_graph_face_batch(precision, bound):
    """Three face grids (HEALPix-like, links only inside a face) in one captured solve."""
    probs = [make_problem(s0, s1, 3, 4, seed=7600 + i, noise="hetero", boundary="face")
             for i, (s0, s1) in enumerate([(16, 16), (12, 20), (9, 7)])]
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    Yd = torch.cat([dev(p.Y.ravel()) for p in probs])
    opts = opts_for(precision, sy.SYLV_SCHED_FIXED)
    X, stats, ws = buffers(dps, 1, opts)
    launch = sy.solve_launcher(dps, X, stats, ws, Y=Yd, opts=opts)

    def solve():
        X.zero_()
        launch()

    say("face graph", precision)
    solve()
    torch.cuda.synchronize()
    Xe, se = X.clone(), sy.stats_list(stats, len(probs))
    g = capture(solve)
    for rep in range(2):
        X.fill_(3.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(X, Xe) and sy.stats_list(stats, len(probs)) == se, rep
    Xh, off = host(Xe), 0
    for i, p in enumerate(probs):
        assert se[i]["status"] == 0, se
        n = p.k * p.n_pix
        assert rel(Xh[off:off + n].reshape(p.k, p.n_pix), osv.solve_dense(p)) < bound, i
        off += n


@pytest.mark.parametrize("kind", [sy.SYLV_PC_FOURIER, sy.SYLV_PC_FOURIER_DIAG,
                                  sy.SYLV_PC_FOURIER_BLOCK])
@pytest.mark.parametrize("precision,bound", PRECISIONS)
def test_graph_fourier_preconditioner(precision, bound, kind):
    """Fourier-preconditioned solves (plain, diagonally and block scaled): the fixed schedule
    equals the adaptive one bitwise, and a captured solve replays bitwise equal to the eager
    call, also after new data in place."""
    p = make_problem(64, 32, 3, 6, seed=7400, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(p)
    Yd = dev(p.Y)
    fixed = opts_for(precision, sy.SYLV_SCHED_FIXED, precond=kind, max_iter=60)
    adaptive = opts_for(precision, sy.SYLV_SCHED_ADAPTIVE, precond=kind, max_iter=60)
    say("fourier fixed vs adaptive", precision, kind)
    Xa, sa = sy.pcg_solve(dp, Y=Yd, opts=adaptive)
    Xf, sf = sy.pcg_solve(dp, Y=Yd, opts=fixed)
    assert sa[0]["status"] == 0, sa
    assert sf == sa and torch.equal(Xf, Xa)
    assert rel(host(Xa).reshape(p.k, p.n_pix), osv.solve_dense(p)) < bound
    X, stats, ws = buffers([dp], 1, fixed)
    launch = sy.solve_launcher(dp, X, stats, ws, Y=Yd, opts=fixed)

    def solve():
        X.zero_()
        launch()

    solve()
    torch.cuda.synchronize()
    Xe, se = X.clone(), sy.stats_list(stats, 1)
    assert torch.equal(Xe.reshape(p.k, p.n_pix), Xa)
    g = capture(solve)
    for rep in range(3):
        X.fill_(2.0e3 + rep)
        stats.zero_()
        torch.cuda.synchronize()
        say("fourier replay", kind, rep)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(X, Xe), rep
        assert sy.stats_list(stats, 1) == se, rep
    Y2 = p.Y * 0.5 + np.random.default_rng(7401).standard_normal(p.Y.shape)
    Yd.copy_(dev(Y2))
    g.replay()
    torch.cuda.synchronize()
    X2, s2 = sy.pcg_solve(dp, Y=dev(Y2), opts=adaptive)
    assert torch.equal(X.reshape(p.k, p.n_pix), X2)
    assert sy.stats_list(stats, 1) == s2
