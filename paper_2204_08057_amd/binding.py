"""ctypes binding of libsylv.so with the same entry-point names as include/sylv.h.

Only marshalling lives here: building the C structs, allocating the caller-owned workspace and
output tensors with torch on the GPU, passing the current HIP stream, and converting status codes
to exceptions.  There is no fallback path: if the library is missing or the tensors are not on
the GPU, the call raises.
"""
from __future__ import annotations

import ctypes
import os
import re
import dataclasses
from dataclasses import dataclass
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HEADER = os.path.join(ROOT, "include", "sylv.h")

SYLV_OK = 0
SYLV_NOT_CONVERGED = 1
SYLV_BREAKDOWN = 2
SYLV_NONFINITE = 3
SYLV_STAGNATED = 4
SYLV_BAD_INPUT = 5
SYLV_E_INVALID = -1
SYLV_E_WORKSPACE = -2
SYLV_E_HIP = -3
SYLV_F64 = 0
SYLV_F32 = 1
SYLV_PREC_F64 = 0
SYLV_PREC_MIXED = 1
SYLV_BC_PERIODIC = 0
SYLV_BC_FACE = 1
SYLV_STOP_R0 = 0
SYLV_STOP_B = 1
SYLV_SCHED_ADAPTIVE = 0
SYLV_SCHED_FIXED = 1
SYLV_PC_NONE = 0
SYLV_PC_JACOBI = 1
SYLV_PC_BLOCK = 2
SYLV_PC_FOURIER = 3
SYLV_PC_FOURIER_DIAG = 4
SYLV_PC_FOURIER_BLOCK = 5

STATUS_NAMES = {
    SYLV_OK: "ok", SYLV_NOT_CONVERGED: "not converged", SYLV_BREAKDOWN: "breakdown",
    SYLV_NONFINITE: "non-finite", SYLV_STAGNATED: "stagnated", SYLV_BAD_INPUT: "bad input",
}


class SylvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsylv error {code}: {msg}")
        self.code = code


class _Problem(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int64), ("nx", ctypes.c_int64), ("k", ctypes.c_int32),
                ("f", ctypes.c_int32), ("kappa", ctypes.c_void_p), ("tau", ctypes.c_void_p),
                ("A", ctypes.c_void_p), ("W", ctypes.c_void_p), ("boundary", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("refine_max", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("block", ctypes.c_int32),
                ("stop_ref", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("apply_rows", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("outer", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("relres_rec", ctypes.c_double), ("relres_true", ctypes.c_double)]


STATS_BYTES = ctypes.sizeof(_Stats)


class _TuneResult(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("apply_rows", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("ms", ctypes.c_double), ("ms_given", ctypes.c_double)]


class _SepProblem(ctypes.Structure):
    _fields_ = [("ny", ctypes.c_int64), ("nx", ctypes.c_int64), ("k", ctypes.c_int32),
                ("f", ctypes.c_int32), ("kappa", ctypes.c_double), ("tau", ctypes.c_void_p),
                ("A", ctypes.c_void_p), ("t", ctypes.c_void_p), ("n", ctypes.c_void_p),
                ("boundary", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def boundary_code(b) -> int:
    """SYLV_BC_* from 'periodic' / 'face' (or the code itself)."""
    if isinstance(b, str):
        return {"periodic": SYLV_BC_PERIODIC, "face": SYLV_BC_FACE}[b]
    return int(b)


class _LzOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("assembly", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _LzStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("relres_est", ctypes.c_double), ("relres_true", ctypes.c_double)]

_LIB = None


def library_path() -> str:
    return os.environ.get("SYLV_LIBRARY", os.path.join(HERE, "libsylv.so"))


def lib():
    """Load libsylv.so (built in-tree by build.py).  Raises if it is missing."""
    global _LIB
    if _LIB is None:
        path = library_path()
        if not os.path.exists(path):
            raise ImportError(f"libsylv.so not found at {path}; build it with "
                              "`python -m paper_2204_08057_amd.build`")
        L = ctypes.CDLL(path)
        vp, i32, sz, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_double
        P = ctypes.POINTER(_Problem)
        O = ctypes.POINTER(_Opts)
        L.sylv_workspace_bytes.argtypes = [P, i32, i32, O]
        L.sylv_workspace_bytes.restype = sz
        L.sylv_prepare.argtypes = [P, i32, vp, sz, vp]
        L.sylv_apply.argtypes = [P, i32, vp, vp, i32, i32, vp, sz, vp]
        L.sylv_precond.argtypes = [P, i32, i32, vp, vp, i32, i32, vp, sz, vp]
        L.sylv_rhs.argtypes = [P, vp, vp, vp]
        L.sylv_po_perturb.argtypes = [P, vp, vp, vp, i32, vp]
        L.sylv_pcg_solve.argtypes = [P, i32, i32, vp, vp, vp, O, vp, vp, sz, vp]
        L.sylv_pcg_solve_noalloc.argtypes = [P, i32, i32, vp, vp, vp, O, vp, vp]
        L.sylv_pcg_backward.argtypes = [P, vp, vp, vp, vp, vp, vp, vp, vp, vp, O, vp, vp, sz, vp]
        SP = ctypes.POINTER(_SepProblem)
        LO = ctypes.POINTER(_LzOpts)
        L.sylv_lanczos_workspace_bytes.argtypes = [SP, LO]
        L.sylv_lanczos_workspace_bytes.restype = sz
        L.sylv_lanczos_solve.argtypes = [SP, vp, vp, LO, ctypes.POINTER(_LzStats), vp, sz, vp]
        L.sylv_kohler_workspace_bytes.argtypes = [SP, i32, O]
        L.sylv_kohler_workspace_bytes.restype = sz
        L.sylv_kohler_solve.argtypes = [SP, vp, vp, i32, O, vp, vp, vp, sz, vp]
        L.sylv_autotune.argtypes = [P, i32, i32, vp, vp, vp, O, vp, ctypes.POINTER(_TuneResult),
                                    vp, sz, vp]
        for name in ("sylv_prepare", "sylv_apply", "sylv_precond", "sylv_rhs", "sylv_po_perturb",
                     "sylv_pcg_solve", "sylv_pcg_solve_noalloc", "sylv_pcg_backward",
                     "sylv_lanczos_solve", "sylv_kohler_solve",
                     "sylv_autotune"):
            getattr(L, name).restype = ctypes.c_int
        L.sylv_status_string.argtypes = [ctypes.c_int]
        L.sylv_status_string.restype = ctypes.c_char_p
        L.sylv_last_error.argtypes = []
        L.sylv_last_error.restype = ctypes.c_char_p
        del dbl
        _LIB = L
    return _LIB


def declared_symbols() -> List[str]:
    """Names of the functions declared in include/sylv.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sylv_[a-z_]+)\s*\(", txt)))


def status_string(code: int) -> str:
    return lib().sylv_status_string(int(code)).decode()


def _check(rc: int):
    if rc != 0:
        raise SylvError(rc, lib().sylv_last_error().decode() or status_string(rc))


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libsylv takes device tensors only")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


@dataclass
class DeviceProblem:
    """Device-resident problem: float64 CUDA tensors kappa[k], tau[k], A[f,k], W[f,n_pix]."""

    ny: int
    nx: int
    kappa: "object"
    tau: "object"
    A: "object"
    W: "object"
    boundary: int = SYLV_BC_PERIODIC

    @property
    def k(self) -> int:
        return int(self.kappa.numel())

    @property
    def f(self) -> int:
        return int(self.A.shape[0])

    @property
    def n_pix(self) -> int:
        return self.ny * self.nx

    def c_struct(self) -> _Problem:
        for name in ("kappa", "tau", "A", "W"):
            t = getattr(self, name)
            torch = _torch()
            if t.dtype != torch.float64:
                raise ValueError(f"{name} must be float64")
        return _Problem(self.ny, self.nx, self.k, self.f, _ptr(self.kappa), _ptr(self.tau),
                        _ptr(self.A), _ptr(self.W), boundary_code(self.boundary), 0)

    @staticmethod
    def from_numpy(prob, device="cuda"):
        torch = _torch()
        t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device).contiguous()  # noqa
        return DeviceProblem(prob.ny, prob.nx, t(prob.kappa), t(prob.tau), t(prob.A), t(prob.W),
                             boundary_code(getattr(prob, "boundary", "periodic")))


@dataclass
class SolveOptions:
    tol: float = 1e-8
    max_iter: int = 5000
    precision: int = SYLV_PREC_F64
    inner_tol: float = 0.0
    refine_max: int = 0
    precond: int = SYLV_PC_BLOCK
    check_every: int = 0
    block: int = 0
    stop_ref: int = SYLV_STOP_R0
    schedule: int = SYLV_SCHED_ADAPTIVE
    block_size: int = 0
    apply_rows: int = 0

    def c_struct(self) -> _Opts:
        return _Opts(self.tol, self.max_iter, self.precision, self.inner_tol, self.refine_max,
                     self.precond, self.check_every, self.block, self.stop_ref, self.schedule,
                     self.block_size, self.apply_rows)


def workspace_bytes(problems: Sequence[DeviceProblem], nrhs: int = 1,
                    opts: Optional[SolveOptions] = None) -> int:
    arr = (_Problem * len(problems))(*[p.c_struct() for p in problems])
    o = ctypes.byref(opts.c_struct()) if opts is not None else None
    return int(lib().sylv_workspace_bytes(arr, len(problems), nrhs, o))


def _workspace(nbytes: int, device):
    torch = _torch()
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def prepare(problem: DeviceProblem, precond_kind: int = SYLV_PC_BLOCK, ws=None):
    """Run the operator set-up into a workspace and return it (for prepared apply/precond)."""
    nbytes = workspace_bytes([problem])
    if ws is None:
        ws = _workspace(nbytes, problem.W.device)
    ps = problem.c_struct()
    _check(lib().sylv_prepare(ctypes.byref(ps), precond_kind, _ptr(ws), ws.numel(), _stream()))
    return ws


def apply(problem: DeviceProblem, X, ws=None, prepared: bool = False, out=None):
    """Y = G(X) for X of shape [k, n_pix] or [nrhs, k, n_pix] (float64 or float32)."""
    torch = _torch()
    dtype = SYLV_F64 if X.dtype == torch.float64 else SYLV_F32
    if X.dtype not in (torch.float64, torch.float32):
        raise ValueError("X must be float64 or float32")
    nrhs = 1 if X.dim() == 2 else X.shape[0]
    if X.shape[-2:] != (problem.k, problem.n_pix):
        raise ValueError(f"X shape {tuple(X.shape)} != (..., {problem.k}, {problem.n_pix})")
    if ws is None:
        ws = _workspace(workspace_bytes([problem]), X.device)
        prepared = False
    Y = torch.empty_like(X) if out is None else out
    ps = problem.c_struct()
    _check(lib().sylv_apply(ctypes.byref(ps), dtype, _ptr(X), _ptr(Y), nrhs, int(prepared),
                            _ptr(ws), ws.numel(), _stream()))
    return Y


def apply_launcher(problem: DeviceProblem, X, Y, ws):
    """A zero-argument callable that launches Y = G(X) on the current stream, with every
    argument marshalled once: for tight loops of applies on an operator already prepared in
    `ws` (the per-call cost is one foreign-function call).  X and Y as for `apply`."""
    torch = _torch()
    if X.dtype not in (torch.float64, torch.float32) or Y.dtype != X.dtype:
        raise ValueError("X and Y must both be float64 or both float32")
    if X.shape != Y.shape or X.shape[-2:] != (problem.k, problem.n_pix):
        raise ValueError(f"X, Y shapes {tuple(X.shape)}, {tuple(Y.shape)} != (..., {problem.k}, "
                         f"{problem.n_pix})")
    dtype = SYLV_F64 if X.dtype == torch.float64 else SYLV_F32
    nrhs = 1 if X.dim() == 2 else X.shape[0]
    ps = problem.c_struct()
    fn = lib().sylv_apply
    args = (ctypes.byref(ps), dtype, _ptr(X), _ptr(Y), nrhs, 1, _ptr(ws), ws.numel(), _stream())

    def launch():
        rc = fn(*args)
        if rc:
            _check(rc)

    launch.keep = (ps, X, Y, ws)   # the marshalled pointers stay valid while the callable lives
    return launch


def precond_launcher(problem: DeviceProblem, R, Z, kind: int, ws):
    """A zero-argument callable that launches Z = M^-1 R (preconditioner `kind`) on the current
    stream with every argument marshalled once, for an operator already prepared in `ws` with
    that preconditioner (`prepare(problem, kind)`).  R and Z as for `precond`."""
    torch = _torch()
    if R.dtype not in (torch.float64, torch.float32) or Z.dtype != R.dtype:
        raise ValueError("R and Z must both be float64 or both float32")
    if R.shape != Z.shape or R.shape[-2:] != (problem.k, problem.n_pix):
        raise ValueError(f"R, Z shapes {tuple(R.shape)}, {tuple(Z.shape)} != (..., {problem.k}, "
                         f"{problem.n_pix})")
    dtype = SYLV_F64 if R.dtype == torch.float64 else SYLV_F32
    nrhs = 1 if R.dim() == 2 else R.shape[0]
    ps = problem.c_struct()
    fn = lib().sylv_precond
    args = (ctypes.byref(ps), dtype, kind, _ptr(R), _ptr(Z), nrhs, 1, _ptr(ws), ws.numel(),
            _stream())

    def launch():
        rc = fn(*args)
        if rc:
            _check(rc)

    launch.keep = (ps, R, Z, ws)
    return launch


def precond(problem: DeviceProblem, R, kind: int = SYLV_PC_BLOCK, ws=None,
            prepared: bool = False):
    torch = _torch()
    dtype = SYLV_F64 if R.dtype == torch.float64 else SYLV_F32
    nrhs = 1 if R.dim() == 2 else R.shape[0]
    if ws is None:
        ws = _workspace(workspace_bytes([problem]), R.device)
        prepared = False
    Z = torch.empty_like(R)
    ps = problem.c_struct()
    _check(lib().sylv_precond(ctypes.byref(ps), dtype, kind, _ptr(R), _ptr(Z), nrhs,
                              int(prepared), _ptr(ws), ws.numel(), _stream()))
    return Z


def rhs(problem: DeviceProblem, Y):
    torch = _torch()
    B = torch.empty((problem.k, problem.n_pix), dtype=torch.float64, device=Y.device)
    ps = problem.c_struct()
    _check(lib().sylv_rhs(ctypes.byref(ps), _ptr(Y), _ptr(B), _stream()))
    return B


def po_perturb(problem: DeviceProblem, xi, zeta):
    torch = _torch()
    nrhs = 1 if xi.dim() == 2 else xi.shape[0]
    eta = torch.empty_like(xi)
    ps = problem.c_struct()
    _check(lib().sylv_po_perturb(ctypes.byref(ps), _ptr(xi), _ptr(zeta), _ptr(eta), nrhs,
                                 _stream()))
    return eta


def _stats_list(stats_t, n):
    raw = bytes(stats_t.cpu().numpy().tobytes())
    out = []
    for i in range(n):
        s = _Stats.from_buffer_copy(raw[i * STATS_BYTES:(i + 1) * STATS_BYTES])
        out.append(dict(status=s.status, status_name=STATUS_NAMES.get(s.status, str(s.status)),
                        iters=s.iters, outer=s.outer, relres_rec=s.relres_rec,
                        relres_true=s.relres_true))
    return out


def pcg_solve(problems, Y=None, Bextra=None, X0=None, opts: Optional[SolveOptions] = None,
              nrhs: int = 1, ws=None, return_stats: bool = True):
    """Solve G x = b for one or several problems (list) times nrhs right-hand sides.

    Y: concatenation over problems of [f, n_pix] (float64) or None; Bextra: concatenation of
    [nrhs, k, n_pix] or None; X0: initial guess with the layout of the result (zeros if None).
    Returns (X, stats) with X the concatenation of [nrhs, k, n_pix] blocks (flattened 1-D when
    several problems are given, else shaped [k, n_pix] / [nrhs, k, n_pix]).
    """
    torch = _torch()
    single = isinstance(problems, DeviceProblem)
    probs = [problems] if single else list(problems)
    opts = opts or SolveOptions()
    k = probs[0].k
    total = sum(nrhs * k * p.n_pix for p in probs)
    dev = probs[0].W.device
    if X0 is None:
        X = torch.zeros(total, dtype=torch.float64, device=dev)
    else:
        X = X0.detach().to(torch.float64).contiguous().clone().reshape(-1)
        if X.numel() != total:
            raise ValueError("X0 has the wrong size")
    nbytes = workspace_bytes(probs, nrhs, opts)
    if ws is None or ws.numel() < nbytes:
        ws = _workspace(nbytes, dev)
    stats = torch.zeros(len(probs) * nrhs * STATS_BYTES, dtype=torch.uint8, device=dev)
    arr = (_Problem * len(probs))(*[p.c_struct() for p in probs])
    o = opts.c_struct()
    _check(lib().sylv_pcg_solve(arr, len(probs), nrhs, _ptr(Y), _ptr(Bextra), _ptr(X),
                                ctypes.byref(o), _ptr(stats), _ptr(ws), ws.numel(), _stream()))
    if single:
        X = X.reshape(probs[0].k, probs[0].n_pix) if nrhs == 1 else \
            X.reshape(nrhs, probs[0].k, probs[0].n_pix)
    if return_stats:
        return X, _stats_list(stats, len(probs) * nrhs)
    return X, stats


NOALLOC_SCRATCH_BYTES = 64 << 20   # SYLV_NOALLOC_SCRATCH_BYTES


def pcg_solve_noalloc(problems, Y=None, Bextra=None, X0=None,
                      opts: Optional[SolveOptions] = None, nrhs: int = 1):
    """pcg_solve through sylv_pcg_solve_noalloc: the library's static per-device scratch array
    is the workspace (at most NOALLOC_SCRATCH_BYTES), so the call itself allocates nothing on
    the device; opts.schedule must be SYLV_SCHED_FIXED.  Returns (X, stats) like pcg_solve."""
    torch = _torch()
    single = isinstance(problems, DeviceProblem)
    probs = [problems] if single else list(problems)
    opts = opts or SolveOptions(schedule=SYLV_SCHED_FIXED)
    k = probs[0].k
    total = sum(nrhs * k * p.n_pix for p in probs)
    dev = probs[0].W.device
    if X0 is None:
        X = torch.zeros(total, dtype=torch.float64, device=dev)
    else:
        X = X0.detach().to(torch.float64).contiguous().clone().reshape(-1)
        if X.numel() != total:
            raise ValueError("X0 has the wrong size")
    stats = torch.zeros(len(probs) * nrhs * STATS_BYTES, dtype=torch.uint8, device=dev)
    arr = (_Problem * len(probs))(*[p.c_struct() for p in probs])
    o = opts.c_struct()
    _check(lib().sylv_pcg_solve_noalloc(arr, len(probs), nrhs, _ptr(Y), _ptr(Bextra), _ptr(X),
                                        ctypes.byref(o), _ptr(stats), _stream()))
    if single:
        X = X.reshape(probs[0].k, probs[0].n_pix) if nrhs == 1 else \
            X.reshape(nrhs, probs[0].k, probs[0].n_pix)
    return X, _stats_list(stats, len(probs) * nrhs)


def solve_launcher(problems, X, stats, ws, Y=None, Bextra=None,
                   opts: Optional[SolveOptions] = None, nrhs: int = 1):
    """A zero-argument callable that enqueues one sylv_pcg_solve on the stream current at call
    time, with every argument marshalled once and nothing allocated or synchronised by the
    call: with opts.schedule = SYLV_SCHED_FIXED it can be captured into a graph
    (torch.cuda.graph).  X holds the initial guess on entry and the solution on return, stats
    is a device uint8 tensor of nprob * nrhs * STATS_BYTES bytes (read with `stats_list`), ws a
    workspace of at least workspace_bytes(problems, nrhs, opts) bytes."""
    torch = _torch()
    probs = [problems] if isinstance(problems, DeviceProblem) else list(problems)
    opts = opts or SolveOptions()
    total = sum(nrhs * p.k * p.n_pix for p in probs)
    if X.dtype != torch.float64 or X.numel() != total:
        raise ValueError(f"X must be float64 with {total} elements")
    if stats.dtype != torch.uint8 or stats.numel() < len(probs) * nrhs * STATS_BYTES:
        raise ValueError("stats too small")
    nbytes = workspace_bytes(probs, nrhs, opts)
    if ws.numel() < nbytes:
        raise ValueError(f"workspace of {ws.numel()} bytes, {nbytes} needed")
    arr = (_Problem * len(probs))(*[p.c_struct() for p in probs])
    o = opts.c_struct()
    fn = lib().sylv_pcg_solve
    args = (arr, len(probs), nrhs, _ptr(Y), _ptr(Bextra), _ptr(X), ctypes.byref(o), _ptr(stats),
            _ptr(ws), ws.numel())

    def launch():
        rc = fn(*args, _stream())
        if rc:
            _check(rc)

    launch.keep = (arr, o, probs, X, stats, ws, Y, Bextra)
    return launch


def _tune_key(probs, nrhs, opts) -> str:
    grids = ",".join(f"{p.ny}x{p.nx}" for p in probs)
    return (f"k{probs[0].k} f{probs[0].f} bc{probs[0].boundary} grids[{grids}] nrhs{nrhs} "
            f"prec{opts.precision} pc{opts.precond} tol{opts.tol:g} sched{opts.schedule}")


def autotune(problems, Y=None, Bextra=None, opts: Optional[SolveOptions] = None, nrhs: int = 1,
             ws=None, cache: Optional[str] = None):
    """Time whole solves of this batch under every candidate configuration (sylv_autotune) and
    return (options with the fastest configuration filled in, result dict).  With `cache` (a
    JSON file path) a result stored for the same batch shape and options is reused, and a new
    one is stored."""
    import json
    torch = _torch()
    probs = [problems] if isinstance(problems, DeviceProblem) else list(problems)
    opts = opts or SolveOptions()
    key = _tune_key(probs, nrhs, opts)
    stored = {}
    if cache is not None and os.path.exists(cache):
        with open(cache) as fh:
            stored = json.load(fh)
        if key in stored:
            r = dict(stored[key], cached=True)
            return dataclasses.replace(opts, block=r["block"], block_size=r["block_size"],
                                       apply_rows=r["apply_rows"]), r
    dev = probs[0].W.device
    total = sum(nrhs * p.k * p.n_pix for p in probs)
    X = torch.zeros(total, dtype=torch.float64, device=dev)
    stats = torch.zeros(len(probs) * nrhs * STATS_BYTES, dtype=torch.uint8, device=dev)
    nbytes = workspace_bytes(probs, nrhs, opts)
    if ws is None or ws.numel() < nbytes:
        ws = _workspace(nbytes, dev)
    arr = (_Problem * len(probs))(*[p.c_struct() for p in probs])
    o = opts.c_struct()
    res = _TuneResult()
    rc = lib().sylv_autotune(arr, len(probs), nrhs, _ptr(Y), _ptr(Bextra), _ptr(X),
                             ctypes.byref(o), _ptr(stats), ctypes.byref(res), _ptr(ws),
                             ws.numel(), _stream())
    if rc != SYLV_OK:
        raise SylvError(rc, lib().sylv_last_error().decode())
    r = dict(block=res.block, block_size=res.block_size, apply_rows=res.apply_rows,
             candidates=res.candidates, ms=res.ms, ms_given=res.ms_given, cached=False)
    if cache is not None:
        stored[key] = {n: r[n] for n in ("block", "block_size", "apply_rows", "candidates", "ms",
                                         "ms_given")}
        with open(cache, "w") as fh:
            json.dump(stored, fh, indent=1, sort_keys=True)
    return dataclasses.replace(opts, block=r["block"], block_size=r["block_size"],
                               apply_rows=r["apply_rows"]), r


def stats_list(stats, n: int):
    """The first n sylv_pcg_stats records of a device stats tensor, as dicts (synchronises)."""
    return _stats_list(stats, n)


def pcg_backward(problem: DeviceProblem, Y, Xstar, Gbar, opts: Optional[SolveOptions] = None,
                 want=("kappa", "tau", "A", "W", "Y"), ws=None):
    """Adjoint solve G lambda = Gbar and the parameter gradients of <Gbar, x*>."""
    torch = _torch()
    opts = opts or SolveOptions(tol=1e-10)
    dev = Xstar.device
    k, f, n = problem.k, problem.f, problem.n_pix
    Lam = torch.zeros((k, n), dtype=torch.float64, device=dev)
    g = {
        "kappa": torch.zeros(k, dtype=torch.float64, device=dev) if "kappa" in want else None,
        "tau": torch.zeros(k, dtype=torch.float64, device=dev) if "tau" in want else None,
        "A": torch.zeros((f, k), dtype=torch.float64, device=dev) if "A" in want else None,
        "W": torch.zeros((f, n), dtype=torch.float64, device=dev) if "W" in want else None,
        "Y": torch.zeros((f, n), dtype=torch.float64, device=dev) if "Y" in want else None,
    }
    nbytes = workspace_bytes([problem], 1, opts)
    if ws is None or ws.numel() < nbytes:
        ws = _workspace(nbytes, dev)
    stats = torch.zeros(STATS_BYTES, dtype=torch.uint8, device=dev)
    ps = problem.c_struct()
    o = opts.c_struct()
    _check(lib().sylv_pcg_backward(ctypes.byref(ps), _ptr(Y), _ptr(Xstar),
                                   _ptr(Gbar.contiguous()), _ptr(Lam), _ptr(g["kappa"]),
                                   _ptr(g["tau"]), _ptr(g["A"]), _ptr(g["W"]), _ptr(g["Y"]),
                                   ctypes.byref(o), _ptr(stats), _ptr(ws), ws.numel(),
                                   _stream()))
    return Lam, g, _stats_list(stats, 1)[0]


class SylvSolve:
    """torch.autograd.Function: X* = G(kappa, tau, A, W)^-1 B^T C Y, differentiable in all of
    kappa, tau, A, W and Y through the adjoint solve (sylv_pcg_backward)."""

    _fn = None

    @classmethod
    def apply(cls, kappa, tau, A, W, Y, ny: int, nx: int, opts: Optional[SolveOptions] = None,
              boundary="periodic"):
        if cls._fn is None:
            cls._fn = _make_function()
        return cls._fn.apply(kappa, tau, A, W, Y, ny, nx, opts, boundary_code(boundary))


def _make_function():
    torch = _torch()

    class _SylvSolveFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, kappa, tau, A, W, Y, ny, nx, opts, bc):
            opts = opts or SolveOptions(tol=1e-10)
            prob = DeviceProblem(ny, nx, kappa.detach().contiguous(), tau.detach().contiguous(),
                                 A.detach().contiguous(), W.detach().contiguous(), bc)
            Yc = Y.detach().contiguous()
            X, stats = pcg_solve(prob, Y=Yc, opts=opts)
            if stats[0]["status"] != SYLV_OK:
                raise SylvError(stats[0]["status"], f"forward solve: {stats[0]}")
            ctx.save_for_backward(kappa, tau, A, W, Y, X)
            ctx.ny, ctx.nx, ctx.opts, ctx.bc = ny, nx, opts, bc
            return X

        @staticmethod
        def backward(ctx, gX):
            kappa, tau, A, W, Y, X = ctx.saved_tensors
            prob = DeviceProblem(ctx.ny, ctx.nx, kappa.detach().contiguous(),
                                 tau.detach().contiguous(), A.detach().contiguous(),
                                 W.detach().contiguous(), ctx.bc)
            _, g, st = pcg_backward(prob, Y.detach().contiguous(), X.detach(),
                                    gX.detach().to(torch.float64).contiguous(), ctx.opts)
            if st["status"] != SYLV_OK:
                raise SylvError(st["status"], f"adjoint solve: {st}")
            return g["kappa"], g["tau"], g["A"], g["W"], g["Y"], None, None, None, None

    return _SylvSolveFn


# ---- Lanczos-Sylvester solver (Section 3.3, Alg. 4 and Alg. 5) ----------------------------------

@dataclass
class SepProblem:
    """The separable, equal-kappa case: W[f, p] = t_f n_p, one kappa for every component.
    tau[k], A[f, k], t[f], n[n_pix] are float64 CUDA tensors; kappa is a number."""

    ny: int
    nx: int
    kappa: float
    tau: "object"
    A: "object"
    t: "object"
    n: "object"
    boundary: int = SYLV_BC_PERIODIC

    @property
    def k(self) -> int:
        return int(self.tau.numel())

    @property
    def f(self) -> int:
        return int(self.A.shape[0])

    @property
    def n_pix(self) -> int:
        return self.ny * self.nx

    def c_struct(self) -> _SepProblem:
        torch = _torch()
        for name in ("tau", "A", "t", "n"):
            if getattr(self, name).dtype != torch.float64:
                raise ValueError(f"{name} must be float64")
        return _SepProblem(self.ny, self.nx, self.k, self.f, float(self.kappa), _ptr(self.tau),
                           _ptr(self.A), _ptr(self.t), _ptr(self.n),
                           boundary_code(self.boundary), 0)

    @staticmethod
    def from_numpy(ny, nx, kappa, tau, A, t, n, device="cuda", boundary="periodic"):
        torch = _torch()
        c = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device).contiguous()  # noqa
        return SepProblem(ny, nx, float(kappa), c(tau), c(A), c(t), c(n), boundary_code(boundary))


SYLV_LZ_KEEP_BASIS = 0
SYLV_LZ_RERUN = 1
SYLV_LZ_AUTO = -1


@dataclass
class LanczosOptions:
    """assembly: SYLV_LZ_KEEP_BASIS, SYLV_LZ_RERUN, or SYLV_LZ_AUTO (keep the basis when its
    max_iter * k * n_pix doubles fit in basis_budget bytes, else the second Lanczos pass)."""
    tol: float = 1e-8
    max_iter: int = 500
    check_every: int = 0
    assembly: int = SYLV_LZ_AUTO
    basis_budget: int = 8 << 30

    def resolved(self, problem: "SepProblem") -> int:
        if self.assembly != SYLV_LZ_AUTO:
            return self.assembly
        basis = 8 * self.max_iter * problem.k * problem.n_pix
        return SYLV_LZ_KEEP_BASIS if basis <= self.basis_budget else SYLV_LZ_RERUN

    def c_struct(self, problem: "SepProblem") -> _LzOpts:
        return _LzOpts(self.tol, self.max_iter, self.check_every, self.resolved(problem), 0)


def lanczos_workspace_bytes(problem: SepProblem, opts: Optional[LanczosOptions] = None) -> int:
    opts = opts or LanczosOptions()
    ps, os_ = problem.c_struct(), opts.c_struct(problem)
    n = lib().sylv_lanczos_workspace_bytes(ctypes.byref(ps), ctypes.byref(os_))
    if n == 0:
        _check(SYLV_E_INVALID)
    return int(n)


def lanczos_solve(problem: SepProblem, Y, opts: Optional[LanczosOptions] = None, ws=None,
                  out=None):
    """X = solution of eq. (Axb-Sylv) as [k, n_pix] float64, and the statistics dict."""
    torch = _torch()
    opts = opts or LanczosOptions()
    if Y.dtype != torch.float64:
        raise ValueError("Y must be float64")
    nb = lanczos_workspace_bytes(problem, opts)
    if ws is None:
        ws = _workspace(nb, Y.device)
    X = out if out is not None else torch.empty((problem.k, problem.n_pix), dtype=torch.float64,
                                                device=Y.device)
    st = _LzStats()
    ps, os_ = problem.c_struct(), opts.c_struct(problem)
    _check(lib().sylv_lanczos_solve(ctypes.byref(ps), _ptr(Y), _ptr(X), ctypes.byref(os_),
                                    ctypes.byref(st), _ptr(ws), ws.numel(), _stream()))
    return X, {"status": st.status, "status_name": STATUS_NAMES.get(st.status, str(st.status)),
               "iters": st.iters, "relres_est": st.relres_est, "relres_true": st.relres_true,
               "assembly": "keep_basis" if os_.assembly == SYLV_LZ_KEEP_BASIS else "rerun"}


def kohler_workspace_bytes(problem: SepProblem, decouple: bool = False,
                           opts: Optional[SolveOptions] = None) -> int:
    opts = opts or SolveOptions()
    ps, o = problem.c_struct(), opts.c_struct()
    n = lib().sylv_kohler_workspace_bytes(ctypes.byref(ps), int(bool(decouple)), ctypes.byref(o))
    if n == 0:
        _check(SYLV_E_INVALID)
    return int(n)


def kohler_solve(problem: SepProblem, Y, opts: Optional[SolveOptions] = None,
                 decouple: bool = False, ws=None, out=None):
    """Solution of eq. (Axb-Sylv) by Alg. 3 with conjugate-gradient column solves on the GPU:
    (X [k, n_pix] float64, per-column statistics list, relative residual of eq. (Axb))."""
    torch = _torch()
    opts = opts or SolveOptions()
    if Y.dtype != torch.float64:
        raise ValueError("Y must be float64")
    nb = kohler_workspace_bytes(problem, decouple, opts)
    if ws is None or ws.numel() < nb:
        ws = _workspace(nb, Y.device)
    X = out if out is not None else torch.empty((problem.k, problem.n_pix), dtype=torch.float64,
                                                device=Y.device)
    stats = torch.zeros(problem.k * STATS_BYTES, dtype=torch.uint8, device=Y.device)
    rel = torch.zeros(1, dtype=torch.float64, device=Y.device)
    ps, o = problem.c_struct(), opts.c_struct()
    _check(lib().sylv_kohler_solve(ctypes.byref(ps), _ptr(Y), _ptr(X), int(bool(decouple)),
                                   ctypes.byref(o), _ptr(stats), _ptr(rel), _ptr(ws), ws.numel(),
                                   _stream()))
    return X, _stats_list(stats, problem.k), float(rel.item())
