"""Block sizes smaller than the number of right-hand sides, the tiling option of the applies and
the autotuner, through the C ABI, against the oracle's dense solves."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2204_08057_amd as sy  # noqa: E402
from oracle import operator as op  # noqa: E402
from oracle import po as opo  # noqa: E402
from oracle import solve as osv  # noqa: E402
from workloads import make_problem, po_draws  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print("[tune]", *a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def batch(nrhs, seed):
    probs = [make_problem(16, 16, 3, 5, seed=seed, noise="hetero"),
             make_problem(20, 28, 3, 5, seed=seed + 1, noise="hetero", mask_frac=0.05),
             make_problem(9, 33, 3, 5, seed=seed + 2, noise="hetero")]
    etas, Ycat, Bcat = [], [], []
    for i, p in enumerate(probs):
        xi, zeta = po_draws(p, nrhs, seed=seed + 10 + i)
        eta = opo.perturbation(p, xi, zeta)
        etas.append(eta)
        Ycat.append(p.Y.ravel())
        Bcat.append(eta.ravel())
    return probs, etas, dev(np.concatenate(Ycat)), dev(np.concatenate(Bcat))


def check(probs, etas, X, st, nrhs, bound):
    X = X.cpu().numpy()
    off = 0
    for i, p in enumerate(probs):
        blk = X[off:off + nrhs * p.k * p.n_pix].reshape(nrhs, p.k, p.n_pix)
        off += nrhs * p.k * p.n_pix
        b = op.rhs(p)
        for r in range(nrhs):
            assert st[i * nrhs + r]["status"] == 0, (i, r, st[i * nrhs + r])
            assert rel(blk[r], osv.solve_dense(p, b=b + etas[i][r])) < bound, (i, r)


PRECISIONS = [(sy.SYLV_PREC_F64, 1e-8, 1e-12), (sy.SYLV_PREC_MIXED, 1e-7, 1e-11)]


@pytest.mark.parametrize("precision,bound,tol", PRECISIONS)
@pytest.mark.parametrize("nrhs,bsize", [(8, 4), (8, 2), (4, 2), (16, 8)])
def test_blocks_smaller_than_nrhs(precision, bound, tol, nrhs, bsize):
    """nrhs / s independent blocks of s columns per problem."""
    probs, etas, Y, B = batch(nrhs, 8000 + nrhs + bsize)
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    say("blocks", precision, nrhs, bsize)
    o = sy.SolveOptions(tol=tol, precision=precision, block=1, block_size=bsize)
    X, st = sy.pcg_solve(dps, Y=Y, Bextra=B, opts=o, nrhs=nrhs)
    check(probs, etas, X, st, nrhs, bound)


def test_block_size_equal_to_nrhs_is_the_default():
    probs, etas, Y, B = batch(4, 8100)
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    say("block size default")
    runs = []
    for bs in (0, 4):
        o = sy.SolveOptions(tol=1e-11, precision=sy.SYLV_PREC_MIXED, block=1, block_size=bs)
        runs.append(sy.pcg_solve(dps, Y=Y, Bextra=B, opts=o, nrhs=4))
    assert torch.equal(runs[0][0], runs[1][0]) and runs[0][1] == runs[1][1]


@pytest.mark.parametrize("precision,bound,tol", PRECISIONS)
def test_apply_rows_option(precision, bound, tol):
    """Every tiling of the applies converges to the same solution; the default is 4 rows at
    k = 3 (the same iterates bitwise)."""
    p = make_problem(70, 45, 3, 6, seed=8200, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(p)
    xs = osv.solve_dense(p)
    say("apply rows", precision)
    out = {}
    for rows in (0, 2, 4, 8):
        o = sy.SolveOptions(tol=tol, precision=precision, apply_rows=rows)
        X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=o)
        assert st[0]["status"] == 0, (rows, st)
        assert rel(X.cpu().numpy(), xs) < bound, rows
        out[rows] = (X, st)
    assert torch.equal(out[0][0], out[4][0]) and out[0][1] == out[4][1]


def test_autotune_batch(tmp_path):
    probs, etas, Y, B = batch(4, 8300)
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    base = sy.SolveOptions(tol=1e-11, precision=sy.SYLV_PREC_MIXED)
    cache = str(tmp_path / "tune.json")
    say("autotune")
    tuned, res = sy.autotune(dps, Y=Y, Bextra=B, opts=base, nrhs=4, cache=cache)
    # candidates: independent CG at 2 and 4 rows (8 rows is capped to 4 at k = 3, the same
    # tiling) and block CG with blocks of 2 and 4 columns
    assert res["candidates"] == 4 and not res["cached"]
    assert res["ms"] > 0.0 and res["ms_given"] > 0.0
    if res["block"]:
        assert res["block_size"] in (2, 4) and res["apply_rows"] == 0
    else:
        assert res["apply_rows"] in (2, 4, 8) and res["block_size"] == 0
    X, st = sy.pcg_solve(dps, Y=Y, Bextra=B, opts=tuned, nrhs=4)
    check(probs, etas, X, st, 4, 1e-7)
    tuned2, res2 = sy.autotune(dps, Y=Y, Bextra=B, opts=base, nrhs=4, cache=cache)
    assert res2["cached"] and tuned2 == tuned


@pytest.mark.parametrize("precision,bound,tol", PRECISIONS)
def test_blocks_on_face_grids_and_odd_sizes(precision, bound, tol):
    """Face grids (links only inside the grid) with odd pixel counts and tails shorter than one
    wavefront: the element-wise access path of the streaming block kernels."""
    nrhs = 4
    probs = [make_problem(s0, s1, 3, 4, seed=8400 + i, noise="hetero", boundary="face")
             for i, (s0, s1) in enumerate([(5, 7), (13, 11), (3, 1), (17, 16)])]
    etas, Ycat, Bcat = [], [], []
    for i, p in enumerate(probs):
        xi, zeta = po_draws(p, nrhs, seed=8410 + i)
        eta = opo.perturbation(p, xi, zeta)
        etas.append(eta)
        Ycat.append(p.Y.ravel())
        Bcat.append(eta.ravel())
    dps = [sy.DeviceProblem.from_numpy(p) for p in probs]
    say("face blocks", precision)
    for bs in (2, 4):
        o = sy.SolveOptions(tol=tol, precision=precision, block=1, block_size=bs)
        X, st = sy.pcg_solve(dps, Y=dev(np.concatenate(Ycat)), Bextra=dev(np.concatenate(Bcat)),
                             opts=o, nrhs=nrhs)
        check(probs, etas, X, st, nrhs, bound)


@pytest.mark.parametrize("precision,bound,tol", PRECISIONS)
@pytest.mark.parametrize("k", [1, 2])
def test_apply_rows_up_to_eight_at_small_k(precision, bound, tol, k):
    """At k <= 2 the fused CG applies may take 8 output rows per lane (32 rows per tile); a grid
    with ragged tiles in both directions, every tiling against the dense solve."""
    p = make_problem(37, 70, k, 3, seed=8500 + k, noise="hetero", mask_frac=0.1)
    dp = sy.DeviceProblem.from_numpy(p)
    xs = osv.solve_dense(p)
    say("rows small k", precision, k)
    for rows in (2, 4, 8):
        o = sy.SolveOptions(tol=tol, precision=precision, apply_rows=rows)
        X, st = sy.pcg_solve(dp, Y=dev(p.Y), opts=o)
        assert st[0]["status"] == 0, (rows, st)
        assert rel(X.cpu().numpy(), xs) < bound, rows
