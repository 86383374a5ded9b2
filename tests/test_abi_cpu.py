"""C-ABI library checks that need no GPU: it loads, exports every declared entry point, and its
host-side logic (workspace sizing, argument validation, status strings) behaves."""
import ctypes
import os
import subprocess

import pytest

import paper_2204_08057_amd as sy
from paper_2204_08057_amd import binding as bd

pytestmark = pytest.mark.skipif(not os.path.exists(bd.library_path()),
                                reason="libsylv.so not built")

FAKE = 0x100000  # never dereferenced: every call below fails validation before any HIP call


def fake_problem(ny=32, nx=32, k=3, f=6, boundary=0):
    return bd._Problem(ny, nx, k, f, FAKE, FAKE, FAKE, FAKE, boundary, 0)


def test_every_declared_symbol_is_exported():
    names = sy.declared_symbols()
    assert {"sylv_apply", "sylv_precond", "sylv_pcg_solve", "sylv_pcg_backward",
            "sylv_workspace_bytes", "sylv_status_string"} <= set(names)
    L = sy.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", bd.library_path()],
                         capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(names) <= exported


def test_header_struct_sizes_match_binding():
    # int64 x2 + int32 x2 + 4 pointers + int32 x2; double, int32 x2, double, int32 x8;
    # int32 x4 + double x2 (stats and tune result)
    assert ctypes.sizeof(bd._Problem) == 64
    assert ctypes.sizeof(bd._Opts) == 56
    assert ctypes.sizeof(bd._TuneResult) == 32
    assert ctypes.sizeof(bd._Stats) == 32


def test_workspace_bytes_grows_with_problem():
    L = sy.lib()
    small = L.sylv_workspace_bytes(ctypes.byref(fake_problem(32, 32)), 1, 1, None)
    big = L.sylv_workspace_bytes(ctypes.byref(fake_problem(64, 64)), 1, 1, None)
    assert 0 < small < big
    o = bd._Opts(1e-8, 100, 0, 0.0, 0, 2, 0, 0)
    solve = L.sylv_workspace_bytes(ctypes.byref(fake_problem(64, 64)), 1, 1, ctypes.byref(o))
    assert solve > big
    two = L.sylv_workspace_bytes(ctypes.byref(fake_problem(64, 64)), 1, 2, ctypes.byref(o))
    assert two > solve
    arr = (bd._Problem * 2)(fake_problem(16, 16), fake_problem(24, 40))
    assert L.sylv_workspace_bytes(arr, 2, 3, ctypes.byref(o)) > 0
    # per pixel and component: >= 5 float64 + 5 float32 solver vectors
    assert solve >= 64 * 64 * 3 * (5 * 8 + 5 * 4)


@pytest.mark.parametrize("bad", [dict(k=0), dict(k=9), dict(f=0), dict(f=17), dict(ny=0),
                                 dict(nx=-3), dict(boundary=2), dict(boundary=-1)])
def test_invalid_problems_rejected(bad):
    L = sy.lib()
    args = dict(ny=8, nx=8, k=3, f=4)
    args.update(bad)
    p = fake_problem(**args)
    assert L.sylv_workspace_bytes(ctypes.byref(p), 1, 1, None) == 0
    rc = L.sylv_apply(ctypes.byref(p), 0, FAKE, FAKE * 2, 1, 1, FAKE, 1 << 30, None)
    assert rc == bd.SYLV_E_INVALID
    assert len(L.sylv_last_error()) > 0


def test_null_pointers_and_bad_options_rejected():
    L = sy.lib()
    p = fake_problem()
    p.W = None
    assert L.sylv_apply(ctypes.byref(p), 0, FAKE, FAKE * 2, 1, 1, FAKE, 1 << 30, None) == -1
    p = fake_problem()
    st = FAKE
    for opts in [bd._Opts(0.0, 10, 0, 0.0, 0, 2, 0, 0), bd._Opts(1e-8, 0, 0, 0.0, 0, 2, 0, 0),
                 bd._Opts(1e-8, 10, 7, 0.0, 0, 2, 0, 0), bd._Opts(1e-8, 10, 0, 0.0, 0, 9, 0, 0),
                 bd._Opts(1e-8, 10, 1, 2.0, 0, 2, 0, 0), bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0, 2),
                 bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0, 0, 2), bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0, 0, -1),
                 bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 1, 0, 1),
                 bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0, 0, 0, 3, 0),
                 bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0, 0, 0, 0, 5),
                 bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 1, 0, 0, 4, 0),
                 bd._Opts(1e-8, 70000, 0, 0.0, 0, 2, 0, 0, 0, 1),
                 bd._Opts(1e-8, 9000, 1, 0.0, 0, 2, 0, 0, 0, 1),
                 # max_iter + 1 must not overflow 32 bits and slip past the cap
                 bd._Opts(1e-8, 2**31 - 1, 0, 0.0, 0, 2, 0, 0, 0, 1),
                 bd._Opts(1e-8, 2**31 - 1, 1, 0.0, 1, 2, 0, 0, 0, 1)]:
        rc = L.sylv_pcg_solve(ctypes.byref(p), 1, 1, FAKE, None, FAKE, ctypes.byref(opts), st,
                              FAKE, 1 << 40, None)
        assert rc == bd.SYLV_E_INVALID, L.sylv_last_error()
    ok = bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0)
    # neither Y nor Bextra
    assert L.sylv_pcg_solve(ctypes.byref(p), 1, 1, None, None, FAKE, ctypes.byref(ok), st, FAKE,
                            1 << 40, None) == bd.SYLV_E_INVALID
    # mixed k across a batch
    arr = (bd._Problem * 2)(fake_problem(k=3), fake_problem(k=4))
    assert L.sylv_pcg_solve(arr, 2, 1, FAKE, None, FAKE, ctypes.byref(ok), st, FAKE, 1 << 40,
                            None) == bd.SYLV_E_INVALID


def test_autotune_arguments_rejected():
    L = sy.lib()
    p = fake_problem()
    ok = bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0)
    res = bd._TuneResult()
    # no result struct, no X, bad options, bad problem: rejected before any HIP call
    assert L.sylv_autotune(ctypes.byref(p), 1, 1, FAKE, None, FAKE, ctypes.byref(ok), FAKE, None,
                           FAKE, 1 << 40, None) == bd.SYLV_E_INVALID
    assert L.sylv_autotune(ctypes.byref(p), 1, 1, FAKE, None, None, ctypes.byref(ok), FAKE,
                           ctypes.byref(res), FAKE, 1 << 40, None) == bd.SYLV_E_INVALID
    bad = bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0, 0, 0, 0, 3)
    assert L.sylv_autotune(ctypes.byref(p), 1, 1, FAKE, None, FAKE, ctypes.byref(bad), FAKE,
                           ctypes.byref(res), FAKE, 1 << 40, None) == bd.SYLV_E_INVALID
    q = fake_problem(k=0)
    assert L.sylv_autotune(ctypes.byref(q), 1, 1, FAKE, None, FAKE, ctypes.byref(ok), FAKE,
                           ctypes.byref(res), FAKE, 1 << 40, None) == bd.SYLV_E_INVALID


def test_workspace_too_small_and_misaligned():
    L = sy.lib()
    p = fake_problem()
    need = L.sylv_workspace_bytes(ctypes.byref(p), 1, 1, None)
    rc = L.sylv_apply(ctypes.byref(p), 0, FAKE, FAKE * 2, 1, 1, FAKE, need - 1, None)
    assert rc == bd.SYLV_E_WORKSPACE
    rc = L.sylv_apply(ctypes.byref(p), 0, FAKE, FAKE * 2, 1, 1, FAKE + 8, need, None)
    assert rc == bd.SYLV_E_INVALID
    ok = bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0)
    need = L.sylv_workspace_bytes(ctypes.byref(p), 1, 1, ctypes.byref(ok))
    rc = L.sylv_pcg_solve(ctypes.byref(p), 1, 1, FAKE, None, FAKE, ctypes.byref(ok), FAKE, FAKE,
                          need - 256, None)
    assert rc == bd.SYLV_E_WORKSPACE


def test_status_strings():
    for code in (0, 1, 2, 3, 4, -1, -2, -3):
        assert sy.status_string(code) != "unknown code"
    assert sy.status_string(12345) == "unknown code"


def test_binding_refuses_host_tensors():
    torch = pytest.importorskip("torch")
    import numpy as np
    from workloads import make_problem
    prob = make_problem(4, 4, 2, 3, seed=1)
    dp = bd.DeviceProblem(4, 4, torch.tensor(prob.kappa), torch.tensor(prob.tau),
                          torch.tensor(prob.A), torch.tensor(prob.W))
    with pytest.raises(ValueError):
        dp.c_struct()
    del np


# ---- Lanczos-Sylvester entry points ---------------------------------------------------------

def fake_sep(ny=32, nx=32, k=4, f=9, kappa=0.5, boundary=0):
    return bd._SepProblem(ny, nx, k, f, kappa, FAKE, FAKE, FAKE, FAKE, boundary, 0)


def test_lanczos_struct_sizes():
    # int64 x2 + int32 x2 + double + 4 pointers + int32 x2; double + int32 x2; int32 x2 + double x2
    assert ctypes.sizeof(bd._SepProblem) == 72
    assert ctypes.sizeof(bd._LzOpts) == 24
    assert ctypes.sizeof(bd._LzStats) == 24


def test_lanczos_workspace_holds_the_basis():
    L = sy.lib()
    o = bd._LzOpts(1e-8, 100, 0)
    n1 = L.sylv_lanczos_workspace_bytes(ctypes.byref(fake_sep(64, 64)), ctypes.byref(o))
    o2 = bd._LzOpts(1e-8, 200, 0)
    n2 = L.sylv_lanczos_workspace_bytes(ctypes.byref(fake_sep(64, 64)), ctypes.byref(o2))
    blk = 64 * 64 * 4 * 8
    assert n1 >= 100 * blk + 3 * blk            # the basis plus Yhat and two running blocks
    assert n2 - n1 >= 100 * blk                 # one more block per extra step
    # the second-pass assembly keeps two blocks whatever the step count
    r1 = L.sylv_lanczos_workspace_bytes(ctypes.byref(fake_sep(64, 64)),
                                        ctypes.byref(bd._LzOpts(1e-8, 100, 0, bd.SYLV_LZ_RERUN)))
    r2 = L.sylv_lanczos_workspace_bytes(ctypes.byref(fake_sep(64, 64)),
                                        ctypes.byref(bd._LzOpts(1e-8, 200, 0, bd.SYLV_LZ_RERUN)))
    assert 5 * blk <= r1 < 6 * blk + (1 << 20)
    assert r2 - r1 <= 100 * 5 * 64 * 8     # only the small k x k blocks grow with the steps


def test_lanczos_auto_assembly_follows_the_budget():
    """Python side: SYLV_LZ_AUTO keeps the basis when it fits the budget, else reruns."""
    o = sy.LanczosOptions(max_iter=800, basis_budget=1 << 30)

    class P:
        k, n_pix = 4, 1024 * 1024
    assert o.resolved(P) == bd.SYLV_LZ_RERUN        # 800 * 4 * 2^20 * 8 B = 26.8 GB
    P.n_pix = 64 * 64
    assert o.resolved(P) == bd.SYLV_LZ_KEEP_BASIS


@pytest.mark.parametrize("bad", [dict(k=0), dict(k=9), dict(f=0), dict(f=17), dict(ny=0),
                                 dict(kappa=-1.0), dict(kappa=float("nan")), dict(boundary=3)])
def test_lanczos_invalid_problems_rejected(bad):
    L = sy.lib()
    args = dict(ny=8, nx=8, k=3, f=4, kappa=0.5)
    args.update(bad)
    p = fake_sep(**args)
    o = bd._LzOpts(1e-8, 10, 0)
    assert L.sylv_lanczos_workspace_bytes(ctypes.byref(p), ctypes.byref(o)) == 0
    st = bd._LzStats()
    rc = L.sylv_lanczos_solve(ctypes.byref(p), FAKE, FAKE, ctypes.byref(o), ctypes.byref(st),
                              FAKE, 1 << 30, None)
    assert rc == bd.SYLV_E_INVALID
    assert len(L.sylv_last_error()) > 0


def test_lanczos_bad_options_rejected():
    L = sy.lib()
    p = fake_sep()
    st = bd._LzStats()
    for o in [bd._LzOpts(0.0, 10, 0), bd._LzOpts(1.0, 10, 0), bd._LzOpts(1e-8, 0, 0),
              bd._LzOpts(1e-8, 10, -1), bd._LzOpts(1e-8, 200000, 0),
              bd._LzOpts(1e-8, 10, 0, 2), bd._LzOpts(1e-8, 10, 0, -1)]:
        assert L.sylv_lanczos_workspace_bytes(ctypes.byref(p), ctypes.byref(o)) == 0
        rc = L.sylv_lanczos_solve(ctypes.byref(p), FAKE, FAKE, ctypes.byref(o),
                                  ctypes.byref(st), FAKE, 1 << 30, None)
        assert rc == bd.SYLV_E_INVALID
    p.n = None
    o = bd._LzOpts(1e-8, 10, 0)
    assert L.sylv_lanczos_solve(ctypes.byref(p), FAKE, FAKE, ctypes.byref(o), ctypes.byref(st),
                                FAKE, 1 << 30, None) == bd.SYLV_E_INVALID
    assert L.sylv_lanczos_solve(ctypes.byref(fake_sep()), None, FAKE, ctypes.byref(o),
                                ctypes.byref(st), FAKE, 1 << 30, None) == bd.SYLV_E_INVALID


def test_bad_input_status_string():
    assert "n_p" in sy.status_string(bd.SYLV_BAD_INPUT)


def test_noalloc_solve_refusals_before_any_device_call():
    """The no-allocation solve refuses the adaptive schedule and batches whose workspace exceeds
    its static scratch array, before touching the device (FAKE pointers are never read)."""
    L = sy.lib()
    fixed = bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0, 0, bd.SYLV_SCHED_FIXED)
    adaptive = bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0, 0, bd.SYLV_SCHED_ADAPTIVE)
    small = fake_problem(16, 16)
    rc = L.sylv_pcg_solve_noalloc(ctypes.byref(small), 1, 1, FAKE, None, FAKE,
                                  ctypes.byref(adaptive), FAKE, None)
    assert rc == bd.SYLV_E_INVALID and b"fixed schedule" in L.sylv_last_error()
    big = fake_problem(1024, 1024)
    need = L.sylv_workspace_bytes(ctypes.byref(big), 1, 1, ctypes.byref(fixed))
    assert need > bd.NOALLOC_SCRATCH_BYTES
    rc = L.sylv_pcg_solve_noalloc(ctypes.byref(big), 1, 1, FAKE, None, FAKE,
                                  ctypes.byref(fixed), FAKE, None)
    assert rc == bd.SYLV_E_WORKSPACE and b"no-allocation" in L.sylv_last_error()
    assert L.sylv_pcg_solve_noalloc(None, 1, 1, FAKE, None, FAKE, ctypes.byref(fixed), FAKE,
                                    None) == bd.SYLV_E_INVALID
    bad = fake_problem(16, 16, k=9)
    assert L.sylv_pcg_solve_noalloc(ctypes.byref(bad), 1, 1, FAKE, None, FAKE,
                                    ctypes.byref(fixed), FAKE, None) == bd.SYLV_E_INVALID


def test_fourier_preconditioner_refusals_before_any_device_call():
    """The Fourier preconditioner takes periodic or face grids whose sides are powers of two in
    [4, 4096], columns that fit its LDS pass, and independent CG; anything else is refused before
    any work is enqueued (FAKE pointers are never read)."""
    L = sy.lib()
    st = FAKE
    fourier = bd._Opts(1e-8, 10, 0, 0.0, 0, bd.SYLV_PC_FOURIER, 0, 0)
    for p in (fake_problem(24, 32), fake_problem(32, 2), fake_problem(24, 16, boundary=1),
              fake_problem(8192, 8), fake_problem(4096, 64, k=8)):
        rc = L.sylv_pcg_solve(ctypes.byref(p), 1, 1, FAKE, None, FAKE, ctypes.byref(fourier),
                              st, FAKE, 1 << 40, None)
        assert rc == bd.SYLV_E_INVALID and len(L.sylv_last_error()) > 0
    block = bd._Opts(1e-8, 10, 0, 0.0, 0, bd.SYLV_PC_FOURIER, 0, 1, 0, 0, 2, 0)
    rc = L.sylv_pcg_solve(ctypes.byref(fake_problem(16, 16)), 1, 2, FAKE, None, FAKE,
                          ctypes.byref(block), st, FAKE, 1 << 40, None)
    assert rc == bd.SYLV_E_INVALID and b"block CG" in L.sylv_last_error()
    # the stand-alone application refuses the same shapes
    rc = L.sylv_precond(ctypes.byref(fake_problem(24, 32)), 0, bd.SYLV_PC_FOURIER, FAKE,
                        FAKE * 2, 1, 1, FAKE, 1 << 40, None)
    assert rc == bd.SYLV_E_INVALID
    # the solve workspace holds one half spectrum per right-hand side
    p = fake_problem(64, 64)
    plain = bd._Opts(1e-8, 10, 0, 0.0, 0, 2, 0, 0)
    n0 = L.sylv_workspace_bytes(ctypes.byref(p), 1, 2, ctypes.byref(plain))
    n1 = L.sylv_workspace_bytes(ctypes.byref(p), 1, 2, ctypes.byref(fourier))
    assert n1 - n0 >= 2 * 16 * 3 * 33 * 64


def test_block_scaled_fourier_refuses_wide_rows_before_any_device_call():
    """The block-scaled Fourier preconditioner's row passes hold every component of two grid
    rows (k nx <= 8192); wider rows are refused, by the solve and the stand-alone application,
    before any work is enqueued."""
    L = sy.lib()
    opts = bd._Opts(1e-8, 10, 0, 0.0, 0, bd.SYLV_PC_FOURIER_BLOCK, 0, 0)
    p = fake_problem(16, 4096, k=3)
    rc = L.sylv_pcg_solve(ctypes.byref(p), 1, 1, FAKE, None, FAKE, ctypes.byref(opts), FAKE,
                          FAKE, 1 << 40, None)
    assert rc == bd.SYLV_E_INVALID and b"k * nx" in L.sylv_last_error()
    rc = L.sylv_precond(ctypes.byref(p), 1, bd.SYLV_PC_FOURIER_BLOCK, FAKE, FAKE * 2, 1, 1, FAKE,
                        1 << 40, None)
    assert rc == bd.SYLV_E_INVALID and b"k * nx" in L.sylv_last_error()
    bad = bd._Opts(1e-8, 10, 0, 0.0, 0, bd.SYLV_PC_FOURIER_BLOCK + 1, 0, 0)
    rc = L.sylv_pcg_solve(ctypes.byref(fake_problem(16, 16)), 1, 1, FAKE, None, FAKE,
                          ctypes.byref(bad), FAKE, FAKE, 1 << 40, None)
    assert rc == bd.SYLV_E_INVALID
