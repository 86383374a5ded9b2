"""The solve without allocation (sylv_pcg_solve_noalloc, the library's static per-device scratch
array as workspace) against sylv_pcg_solve with a caller workspace and the same options, through
the C ABI: two calls in a row, the second on a smaller batch, each compared with the regular
entry point and with the oracle's dense Cholesky solution; a batch beyond the scratch size and
the adaptive schedule are refused before any work is enqueued."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2204_08057_amd as sy  # noqa: E402
from oracle import operator as op  # noqa: E402
from oracle import solve as osv  # noqa: E402
from workloads import make_problem  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def _both(probs, Y, Bx, nrhs, opts):
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    Yd = torch.cat([dev(p.Y.ravel()) for p in probs])
    Bd = None if Bx is None else torch.cat([dev(b.ravel()) for b in Bx])
    say("noalloc", [(p.ny, p.nx) for p in probs], "nrhs", nrhs, "precision", opts.precision)
    Xn, sn = sy.pcg_solve_noalloc(dps if len(dps) > 1 else dps[0], Y=Yd, Bextra=Bd, opts=opts,
                                  nrhs=nrhs)
    Xn = host(Xn).reshape(-1)
    say("regular entry point")
    Xr, sr = sy.pcg_solve(dps if len(dps) > 1 else dps[0], Y=Yd, Bextra=Bd, opts=opts, nrhs=nrhs)
    Xr = host(Xr).reshape(-1)
    return Xn, sn, Xr, sr


def _check_against_oracle(probs, Bx, nrhs, X, bound):
    off = 0
    for g, p in enumerate(probs):
        for r in range(nrhs):
            b = op.rhs(p) + (0.0 if Bx is None else Bx[g][r])
            xs = osv.solve_dense(p, b=b)
            x = X[off:off + p.k * p.n_pix].reshape(p.k, p.n_pix)
            off += p.k * p.n_pix
            assert rel(x, xs) <= bound, (g, r)


def test_noalloc_two_calls_match_regular_solve():
    # first call: two problems x 2 right-hand sides (Y plus perturbations), mixed precision
    p1 = make_problem(24, 40, 3, 6, seed=71, noise="hetero", mask_frac=0.1)
    p2 = make_problem(32, 28, 3, 6, seed=72, noise="hetero")
    rng = np.random.default_rng(73)
    Bx = [rng.standard_normal((2, p.k, p.n_pix)) for p in (p1, p2)]
    opts = sy.SolveOptions(tol=1e-11, max_iter=300, precision=sy.SYLV_PREC_MIXED, refine_max=4,
                           schedule=sy.SYLV_SCHED_FIXED)
    Xn, sn, Xr, sr = _both([p1, p2], None, Bx, 2, opts)
    assert all(s["status"] == 0 for s in sn), sn
    assert [s["iters"] for s in sn] == [s["iters"] for s in sr]
    assert rel(Xn, Xr) <= 1e-13
    say("  first call: bitwise equal" if np.array_equal(Xn, Xr) else
        f"  first call: rel diff {rel(Xn, Xr):.2e}")
    _check_against_oracle([p1, p2], Bx, 2, Xn, 1e-7)

    # second call: one smaller problem, float64; the scratch still holds the first call's data
    p3 = make_problem(12, 20, 3, 5, seed=74, noise="hetero")
    opts = sy.SolveOptions(tol=1e-12, max_iter=300, schedule=sy.SYLV_SCHED_FIXED)
    Xn, sn, Xr, sr = _both([p3], None, None, 1, opts)
    assert sn[0]["status"] == 0, sn
    assert sn[0]["iters"] == sr[0]["iters"]
    assert rel(Xn, Xr) <= 1e-13
    say("  second call: bitwise equal" if np.array_equal(Xn, Xr) else
        f"  second call: rel diff {rel(Xn, Xr):.2e}")
    _check_against_oracle([p3], None, 1, Xn, 1e-8)


def test_noalloc_refuses_oversized_batch_and_adaptive_schedule():
    big = sy.DeviceProblem.from_numpy(make_problem(512, 512, 3, 2, seed=75, noise="homo"))
    Y = dev(np.zeros((2, 512 * 512)))
    fixed = sy.SolveOptions(tol=1e-8, max_iter=10, schedule=sy.SYLV_SCHED_FIXED)
    assert sy.workspace_bytes([big], 1, fixed) > sy.NOALLOC_SCRATCH_BYTES
    with pytest.raises(sy.SylvError) as e:
        sy.pcg_solve_noalloc(big, Y=Y, opts=fixed)
    assert e.value.code == -2
    small = sy.DeviceProblem.from_numpy(make_problem(8, 8, 2, 2, seed=76, noise="homo"))
    with pytest.raises(sy.SylvError) as e:
        sy.pcg_solve_noalloc(small, Y=dev(np.zeros((2, 64))), opts=sy.SolveOptions())
    assert e.value.code == -1
