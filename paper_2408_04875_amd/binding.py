"""ctypes binding of libpsdp.so (include/psdp.h): argument marshalling only.

Every computation runs inside the HIP library. Tensors must already live on
the GPU; this module only passes their device pointers and torch's current
HIP stream, allocates outputs with torch, and raises on any error status.
There is no CPU fallback: if the library is missing or does not load, every
call raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsdp.so")

F64, F32, BF16, I8 = 0, 1, 2, 3
PABB, PPA = 0, 1
PERTURB = {"none": 0, "full": 1, "diag": 2}
EXIT_NAMES = {0: "converged", 1: "outer_cap", 2: "stall"}


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("inner", ctypes.c_int32),
        ("qx_dtype", ctypes.c_int32),
        ("perturb", ctypes.c_int32),
        ("max_inner", ctypes.c_int32),
        ("max_outer", ctypes.c_int32),
        ("stall_outer", ctypes.c_int32),
        ("eig_maxit", ctypes.c_int32),
        ("cg_maxit", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("poll_sweeps", ctypes.c_int32),
        ("gemm_variant", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("sparse", ctypes.c_int32),
        ("lambda_reuse", ctypes.c_int32),
        ("slots", ctypes.c_int32),
        ("lanes", ctypes.c_int32),
        ("gemv_sym", ctypes.c_int32),
        ("tol_kkt", ctypes.c_double),
        ("tol_binary", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("eps_hp", ctypes.c_double),
        ("lambda_floor_rel", ctypes.c_double),
        ("alpha_min", ctypes.c_double),
        ("alpha_max", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("eig_tol", ctypes.c_double),
        ("cg_tol", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("exit_reason", ctypes.c_int32),
        ("outer_iters", ctypes.c_int32),
        ("inner_iters", ctypes.c_int64),
        ("aux_matvecs", ctypes.c_int64),
        ("final_cret_rel", ctypes.c_double),
        ("final_binary_gap", ctypes.c_double),
        ("sweeps", ctypes.c_int64),
        ("qx_seconds", ctypes.c_double),
        ("qx_flops", ctypes.c_double),
        ("qx_launches", ctypes.c_int64),
        ("aux_seconds", ctypes.c_double),
        ("aux_flops", ctypes.c_double),
        ("step_seconds", ctypes.c_double),
        ("step_launches", ctypes.c_int64),
        ("column_steps", ctypes.c_int64),
        ("sparse_sweeps", ctypes.c_int64),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ColumnPlan(ctypes.Structure):
    _fields_ = [
        ("ld", ctypes.c_int64),
        ("ncol", ctypes.c_int32),
        ("zero_col", ctypes.c_int32),
        ("list_len", ctypes.c_int32),
        ("digit_cols", ctypes.c_int32),
        ("word_cols", ctypes.c_int32),
        ("ok", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# Exported symbols of include/psdp.h with their ctypes signatures.
_P = ctypes.c_void_p
_I32, _I64, _U64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
SIGNATURES = {
    "psdp_params_default": (None, [ctypes.POINTER(Params)]),
    "psdp_status_string": (ctypes.c_char_p, [_I32]),
    "psdp_last_error": (ctypes.c_char_p, []),
    "psdp_version": (_I32, []),
    "psdp_solve_i32": (_I32, [_P, _P, _I64, _P, _P, _I32, ctypes.POINTER(Params), _P, _P, _P,
                              ctypes.POINTER(_I32), ctypes.POINTER(Stats), _P]),
    "psdp_solve_i32_ex": (_I32, [_P, _P, _I64, _P, _P, _I32, ctypes.POINTER(Params), _P, _P, _P,
                                 ctypes.POINTER(_I32), ctypes.POINTER(Stats), _P, _I32, _P, _I32, _P]),
    "psdp_solve_f64": (_I32, [_P, _P, _I64, _P, _P, _I32, ctypes.POINTER(Params), _P, _P, _P,
                              ctypes.POINTER(_I32), ctypes.POINTER(Stats), _P]),
    "psdp_solve_f64_ex": (_I32, [_P, _P, _I64, _P, _P, _I32, ctypes.POINTER(Params), _P, _P, _P,
                                 ctypes.POINTER(_I32), ctypes.POINTER(Stats), _P, _I32, _P, _I32, _P]),
    "psdp_solve_host_i32": (_I32, [_P, _P, _I64, _P, _P, _I32, ctypes.POINTER(Params), _P, _P, _P,
                                   ctypes.POINTER(_I32), ctypes.POINTER(Stats)]),
    "psdp_solve_host_f64": (_I32, [_P, _P, _I64, _P, _P, _I32, ctypes.POINTER(Params), _P, _P, _P,
                                   ctypes.POINTER(_I32), ctypes.POINTER(Stats)]),
    "psdp_solve_group_i32": (_I32, [_I32, _P, _P, _P, _P, _P, ctypes.POINTER(Params), _P, _P,
                                    ctypes.POINTER(Stats), _P]),
    "psdp_eval_penalty_grad": (_I32, [_I32, _I32, _P, _I64, _P, _P, _P, _I64, _I64, _P, _P, _P]),
    "psdp_eval_penalty_grad_noalloc": (_I32, [_I32, _I32, _P, _I64, _P, _P, _P, _I64, _I64, _P, _P, _P]),
    "psdp_penalty_adjoint": (_I32, [_I32, _I32, _P, _P, _P, _I64, _I64, _P, _P, _P, _P, _P]),
    "psdp_round_objective_i32": (_I32, [_P, _P, _I64, _P, _I64, _P, _P, _P]),
    "psdp_round_objective_f64": (_I32, [_P, _P, _I64, _P, _I64, _P, _P, _P]),
    "psdp_perturbation": (_I32, [_I64, _D, _U64, _I32, _P, _P]),
    "psdp_qx_digits": (_I32, [_P, _I64, _P, _I32, _I32, _P, _P]),
    "psdp_qx_sparse": (_I32, [_P, _I64, _P, _I32, _I32, _P, _P]),
    "psdp_qx_dense": (_I32, [_I32, _P, _I64, _P, _I32, _P, _P]),
    "psdp_release": (None, []),
    "psdp_qx_single": (_I32, [_I32, _P, _I64, _P, _I32, _P, _P]),
    "psdp_plan_columns": (_I32, [_I64, _I32, ctypes.POINTER(Params), _I32, ctypes.POINTER(ColumnPlan)]),
    "psdp_qx_digits_ex": (_I32, [_P, _I64, _P, _I32, _I32, _I32, _I32, _I32, ctypes.POINTER(_D), _P, _P]),
    "psdp_set_digit_table": (_I32, [_I64, _I32, _I32, _P, _P, _P]),
    "psdp_digit_choice": (_I32, [_I64, _I32, _I32, ctypes.POINTER(_I32)]),
}

_lib = None


def load(path: str = LIB_PATH, tuning: bool = True):
    """Loads libpsdp.so (raises if it is missing: build it with build.py).
    On the first load the product tables under tuning/ are installed
    (install_tuning) unless tuning is False."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2408_04875_amd/build.py "
                           "(or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    if tuning and os.path.isdir(TUNING_DIR):
        install_tuning()
    return lib


class PSDPError(RuntimeError):
    pass


def _check(status: int):
    if status != 0:
        lib = load()
        raise PSDPError(f"{lib.psdp_status_string(status).decode()} ({status}): "
                        f"{lib.psdp_last_error().decode()}")


def default_params(**overrides) -> Params:
    """psdp_params_default() then keyword overrides (names as in psdp.h).

    inner may be "pabb"/"ppa", qx_dtype "f64"/"f32"/"bf16"/"i8", perturb
    "none"/"full"/"diag".
    """
    p = Params()
    load().psdp_params_default(ctypes.byref(p))
    names = {f for f, _ in Params._fields_}
    for k, v in overrides.items():
        if k not in names:
            raise TypeError(f"unknown parameter {k}")
        if k == "inner" and isinstance(v, str):
            v = {"pabb": PABB, "ppa": PPA}[v]
        if k == "qx_dtype" and isinstance(v, str):
            v = {"f64": F64, "f32": F32, "bf16": BF16, "i8": I8}[v]
        if k == "perturb" and isinstance(v, str):
            v = PERTURB[v]
        setattr(p, k, v)
    return p


def plan_columns(n: int, B: int, sparse_copy: bool = False, **params) -> dict:
    """psdp_plan_columns: the column bookkeeping a solve of B starts would
    allocate (host only, no device work)."""
    out = ColumnPlan()
    prm = default_params(**params)
    _check(load().psdp_plan_columns(n, B, ctypes.byref(prm), 1 if sparse_copy else 0, ctypes.byref(out)))
    return out.as_dict()


def _torch():
    import torch
    return torch


def _dev(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise PSDPError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise PSDPError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise PSDPError(f"{name} must be contiguous")
    return t


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


@dataclasses.dataclass
class SolveResult:
    xhat: object            # uint8 tensor (B, n) (or (n,) for one start)
    obj: object             # int64 tensor (B,)
    X: object               # float64 tensor of final iterates, same shape as xhat
    best: int               # index of the smallest objective
    stats: List[dict]
    trace: Optional[object] = None   # numpy (B, trace_cap, 6) when requested


def solve(Q, b, X0=None, p0=None, trace_cap: int = 0, params: Optional[Params] = None, alpha=None,
          **kw) -> SolveResult:
    """Algorithm 3 on one instance, one or many starts.

    Q: int32 (n, n) symmetric with b int32 (n,) (psdp_solve_i32, int64
    objectives), or Q float64 with b float64 (psdp_solve_f64, FP64
    objectives); X0: float64 (B, n) starts in [0,1] (None: x^0 of eq.
    (gamma), one start); p0: float64 (n,) or None. alpha: optional host
    array (B, cap) of penalty steps replayed by the first cap updates of
    every start (psdp_solve_*_ex); trace_cap > 0 returns the per-update trace.
    """
    torch = _torch()
    lib = load()
    real = Q.dtype == torch.float64
    vt = torch.float64 if real else torch.int32
    Q = _dev(Q, vt, "Q")
    b = _dev(b, vt, "b")
    n = b.shape[0]
    single = X0 is None or X0.dim() == 1
    if X0 is not None:
        X0 = _dev(X0, torch.float64, "X0")
        X0v = X0.reshape(-1, n)
        B = X0v.shape[0]
    else:
        X0v, B = None, 1
    if p0 is not None:
        p0 = _dev(p0, torch.float64, "p0")
    prm = params if params is not None else default_params(**kw)
    xhat = torch.empty((B, n), dtype=torch.uint8, device=Q.device)
    obj = torch.empty(B, dtype=torch.float64 if real else torch.int64, device=Q.device)
    X = torch.empty((B, n), dtype=torch.float64, device=Q.device)
    best = ctypes.c_int32(0)
    stats = (Stats * B)()
    tr = None
    if trace_cap > 0 or alpha is not None:
        import numpy as np
        trp, cap = None, 0
        if trace_cap > 0:
            tr = np.full((B, trace_cap, 6), np.nan)
            trp, cap = tr.ctypes.data_as(ctypes.c_void_p), trace_cap
        ap, acap = None, 0
        if alpha is not None:
            al = np.ascontiguousarray(np.asarray(alpha, dtype=np.float64).reshape(B, -1))
            ap, acap = al.ctypes.data_as(ctypes.c_void_p), al.shape[1]
        fn = lib.psdp_solve_f64_ex if real else lib.psdp_solve_i32_ex
        st = fn(_ptr(Q), _ptr(b), n, _ptr(X0v), _ptr(p0), B, ctypes.byref(prm), _ptr(xhat), _ptr(obj), _ptr(X),
                ctypes.byref(best), stats, trp, cap, ap, acap, _stream())
    else:
        fn = lib.psdp_solve_f64 if real else lib.psdp_solve_i32
        st = fn(_ptr(Q), _ptr(b), n, _ptr(X0v), _ptr(p0), B, ctypes.byref(prm), _ptr(xhat), _ptr(obj), _ptr(X),
                ctypes.byref(best), stats, _stream())
    _check(st)
    if single:
        xhat, X = xhat[0], X[0]
    return SolveResult(xhat=xhat, obj=obj, X=X, best=best.value, stats=[s.as_dict() for s in stats],
                       trace=tr)


def solve_host(Q, b, X0=None, p0=None, params: Optional[Params] = None, **kw):
    """The host-pointer entry points (psdp_solve_host_i32 / _f64) on numpy
    arrays: returns (xhat uint8 (B, n), obj (B,), X (B, n), best, stats)."""
    import numpy as np
    lib = load()
    real = np.asarray(Q).dtype == np.float64
    vt = np.float64 if real else np.int32
    Qh = np.ascontiguousarray(Q, dtype=vt)
    bh = np.ascontiguousarray(b, dtype=vt)
    n = bh.shape[0]
    X0h = None if X0 is None else np.ascontiguousarray(np.asarray(X0, dtype=np.float64).reshape(-1, n))
    B = 1 if X0h is None else X0h.shape[0]
    p0h = None if p0 is None else np.ascontiguousarray(p0, dtype=np.float64)
    prm = params if params is not None else default_params(**kw)
    xhat = np.empty((B, n), dtype=np.uint8)
    obj = np.empty(B, dtype=np.float64 if real else np.int64)
    X = np.empty((B, n), dtype=np.float64)
    best = ctypes.c_int32(0)
    stats = (Stats * B)()
    hp = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    fn = lib.psdp_solve_host_f64 if real else lib.psdp_solve_host_i32
    _check(fn(hp(Qh), hp(bh), n, hp(X0h), hp(p0h), B, ctypes.byref(prm), hp(xhat), hp(obj), hp(X),
              ctypes.byref(best), stats))
    return xhat, obj, X, best.value, [s.as_dict() for s in stats]


def solve_group(Qs: Sequence, bs: Sequence, seeds: Optional[Sequence[int]] = None,
                sigmas: Optional[Sequence[float]] = None, params: Optional[Params] = None, **kw):
    """Algorithm 3 on several instances of different sizes, advanced together.

    seeds / sigmas: optional per-instance perturbation seeds and standard
    deviations. Returns (list of uint8 xhat tensors, int64 obj tensor, list
    of stats dicts).
    """
    torch = _torch()
    lib = load()
    count = len(Qs)
    ns = (ctypes.c_int64 * count)(*[int(q.shape[0]) for q in Qs])
    for i in range(count):
        _dev(Qs[i], torch.int32, f"Q[{i}]")
        _dev(bs[i], torch.int32, f"b[{i}]")
    qp = (ctypes.c_void_p * count)(*[q.data_ptr() for q in Qs])
    bp = (ctypes.c_void_p * count)(*[v.data_ptr() for v in bs])
    dev = Qs[0].device
    xh = [torch.empty(int(q.shape[0]), dtype=torch.uint8, device=dev) for q in Qs]
    xp = (ctypes.c_void_p * count)(*[t.data_ptr() for t in xh])
    obj = torch.empty(count, dtype=torch.int64, device=dev)
    sd = (ctypes.c_uint64 * count)(*seeds) if seeds is not None else None
    sg = (ctypes.c_double * count)(*[float(v) for v in sigmas]) if sigmas is not None else None
    prm = params if params is not None else default_params(**kw)
    stats = (Stats * count)()
    st = lib.psdp_solve_group_i32(count, ns, qp, bp, sd, sg, ctypes.byref(prm), xp, _ptr(obj), stats,
                                  _stream())
    _check(st)
    return xh, obj, [s.as_dict() for s in stats]


_DT = None


def _dtype_codes(t):
    torch = _torch()
    return {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[t.dtype]


def eval_penalty_grad(Q, b, p, X, want_grad: bool = True, noalloc: bool = False):
    """h(x_c, p) and grad h(x_c, p) for the rows x_c of X (shape (B, n)).

    Q and X share a dtype (float64, float32 or bfloat16); b and p share the
    dtype of the outputs (float64 or float32). noalloc=True runs
    psdp_eval_penalty_grad_noalloc (the library's fixed workspace; the
    outputs are still allocated here by torch).
    """
    torch = _torch()
    lib = load()
    for t, nm in ((Q, "Q"), (b, "b"), (p, "p"), (X, "X")):
        _dev(t, t.dtype, nm)
    if Q.dtype != X.dtype or b.dtype != p.dtype:
        raise PSDPError("Q/X and b/p must share dtypes")
    n = b.shape[0]
    X2 = X.reshape(-1, n)
    B = X2.shape[0]
    h = torch.empty(B, dtype=b.dtype, device=X.device)
    G = torch.empty((B, n), dtype=b.dtype, device=X.device) if want_grad else None
    fn = lib.psdp_eval_penalty_grad_noalloc if noalloc else lib.psdp_eval_penalty_grad
    st = fn(_dtype_codes(Q), _dtype_codes(b), _ptr(Q), Q.stride(0), _ptr(b), _ptr(p), _ptr(X2), n, B, _ptr(h),
            _ptr(G), _stream())
    _check(st)
    return h, G


def penalty_adjoint(X, G, w, want=("dX", "dQ", "db", "dp")):
    """dX = w o G, dQ = X^T Diag(w) X (n x n), db = X^T w, dp = (X - X o X)^T w."""
    torch = _torch()
    lib = load()
    n = X.shape[-1]
    X2 = X.reshape(-1, n)
    B = X2.shape[0]
    vdt = w.dtype
    dX = torch.empty((B, n), dtype=vdt, device=X.device) if "dX" in want else None
    dQ = torch.empty((n, n), dtype=X.dtype, device=X.device) if "dQ" in want else None
    db = torch.empty(n, dtype=vdt, device=X.device) if "db" in want else None
    dp = torch.empty(n, dtype=vdt, device=X.device) if "dp" in want else None
    st = lib.psdp_penalty_adjoint(_dtype_codes(X), _dtype_codes(w), _ptr(X2.contiguous()),
                                  _ptr(G.contiguous()) if G is not None else None, _ptr(w.contiguous()),
                                  n, B, _ptr(dX), _ptr(dQ), _ptr(db), _ptr(dp), _stream())
    _check(st)
    return dX, dQ, db, dp


def round_objective(Q, b, X):
    """x^ = [X > 1/2] and the objective of every row of X: exact int64 for
    int32 Q and b, the correctly rounded FP64 sum for float64 Q and b."""
    torch = _torch()
    lib = load()
    real = Q.dtype == torch.float64
    vt = torch.float64 if real else torch.int32
    _dev(Q, vt, "Q")
    _dev(b, vt, "b")
    _dev(X, torch.float64, "X")
    n = b.shape[0]
    X2 = X.reshape(-1, n)
    B = X2.shape[0]
    xhat = torch.empty((B, n), dtype=torch.uint8, device=X.device)
    obj = torch.empty(B, dtype=torch.float64 if real else torch.int64, device=X.device)
    fn = lib.psdp_round_objective_f64 if real else lib.psdp_round_objective_i32
    _check(fn(_ptr(Q), _ptr(b), n, _ptr(X2), B, _ptr(xhat), _ptr(obj), _stream()))
    return xhat, obj


# Layout codes of the exact integer product (psdp_qx_digits_ex).
DIGIT_LAYOUTS = {"few": 1, "mid": 2, "many": 4, "wide": 8, "tall": 16}


def qx_digits(Q, X, digits: int = 4, sparse: bool = False, layout=0, slices: int = 0, reps: int = 0):
    """Exact integer product of the I8 path: rows of X (shape (B, n) float64)
    times Q with a zero diagonal, returned as (B, n) float64. digits=4 needs
    X in [0,1] (grid 2^-27, exact result); digits=8 scales each row by a
    power of two (grid 2^(e-55), result rounded once). sparse=True computes
    the same values from a sparse copy of Q (psdp_qx_sparse). layout (a name
    of DIGIT_LAYOUTS or its code) and slices force the kernel settings
    (psdp_qx_digits_ex); reps > 0 also times that many further launches and
    returns (Y, microseconds per launch)."""
    torch = _torch()
    lib = load()
    _dev(Q, torch.int32, "Q")
    _dev(X, torch.float64, "X")
    n = Q.shape[0]
    X2 = X.reshape(-1, n)
    B = X2.shape[0]
    Y = torch.empty((B, n), dtype=torch.float64, device=X.device)
    if sparse:
        _check(lib.psdp_qx_sparse(_ptr(Q), n, _ptr(X2), B, int(digits), _ptr(Y), _stream()))
        return Y
    code = DIGIT_LAYOUTS[layout] if isinstance(layout, str) else int(layout)
    us = ctypes.c_double(0.0)
    _check(lib.psdp_qx_digits_ex(_ptr(Q), n, _ptr(X2), B, int(digits), code, int(slices), int(reps),
                                 ctypes.byref(us), _ptr(Y), _stream()))
    return (Y, us.value) if reps > 0 else Y


def set_digit_table(n: int, digits: int, entries):
    """psdp_set_digit_table: entries = [(max_cols, layout, slices), ...] with
    max_cols increasing (layout a name or code); [] removes the table."""
    import numpy as np
    mc = np.array([int(e[0]) for e in entries], dtype=np.int32)
    lay = np.array([DIGIT_LAYOUTS[e[1]] if isinstance(e[1], str) else int(e[1]) for e in entries], dtype=np.int32)
    sl = np.array([int(e[2]) for e in entries], dtype=np.int32)
    _check(load().psdp_set_digit_table(n, digits, len(entries), mc.ctypes.data, lay.ctypes.data, sl.ctypes.data))


def digit_choice(n: int, est4: int, est8: int = 0):
    """psdp_digit_choice: ((layout, slices) of the 4-digit product, (layout,
    slices) of the 8-digit product) for one launch."""
    out = (ctypes.c_int32 * 4)()
    _check(load().psdp_digit_choice(n, est4, est8, out))
    return (out[0], out[1]), (out[2], out[3])


TUNING_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")


def install_tuning(path: str = TUNING_DIR):
    """Installs every digit-product table found in the JSON files of `path`
    (written by the package's autotuner); returns the (n, digits) keys."""
    import glob
    import json
    keys = []
    for f in sorted(glob.glob(os.path.join(path, "*.json"))):
        with open(f) as fh:
            doc = json.load(fh)
        for t in doc.get("digit_tables", []):
            set_digit_table(int(t["n"]), int(t["digits"]),
                            [(e["max_cols"], e["layout"], e["slices"]) for e in t["entries"]])
            keys.append((int(t["n"]), int(t["digits"])))
    return keys


def qx_single(Q, x, dtype: str = "f32", sym: bool = False):
    """The single-instance solver's product (psdp_qx_single): Q with a zero
    diagonal stored as dtype ("f64", "f32", "bf16") times x (float64, (n,)),
    summed in FP64, by full rows (sym=False) or from the unique half of Q in
    packed upper tiles (sym=True); returns (n,) float64."""
    torch = _torch()
    lib = load()
    _dev(Q, torch.int32, "Q")
    _dev(x, torch.float64, "x")
    n = Q.shape[0]
    y = torch.empty(n, dtype=torch.float64, device=x.device)
    code = {"f64": F64, "f32": F32, "bf16": BF16}[dtype]
    _check(lib.psdp_qx_single(code, _ptr(Q), n, _ptr(x), 1 if sym else 0, _ptr(y), _stream()))
    return y


def qx_dense(Q, X, dtype: str = "f32"):
    """The batched solver's floating-point product (psdp_qx_dense): rows of
    X (shape (B, n) float64) times Q with a zero diagonal, through the kernel
    the solver picks for B columns, returned as (B, n) float64."""
    torch = _torch()
    lib = load()
    _dev(Q, torch.int32, "Q")
    _dev(X, torch.float64, "X")
    n = Q.shape[0]
    X2 = X.reshape(-1, n)
    B = X2.shape[0]
    Y = torch.empty((B, n), dtype=torch.float64, device=X.device)
    _check(lib.psdp_qx_dense({"f32": F32, "f64": F64}[dtype], _ptr(Q), n, _ptr(X2), B, _ptr(Y), _stream()))
    return Y


def perturbation(n: int, sigma: float, seed: int, mode: str = "full", device="cuda"):
    """The library's symmetric perturbation matrix (float64, (n, n))."""
    torch = _torch()
    lib = load()
    mu = torch.empty((n, n), dtype=torch.float64, device=device)
    _check(lib.psdp_perturbation(n, float(sigma), int(seed), PERTURB[mode], _ptr(mu), _stream()))
    return mu


def _make_penalty_fn():
    torch = _torch()

    class PenaltyFn(torch.autograd.Function):
        """h(x_c, p) for the rows of X, differentiable in X, Q, b and p.

        Forward runs psdp_eval_penalty_grad (h and G = grad_x h); backward runs
        psdp_penalty_adjoint: dX = w o G, dQ = X^T Diag(w) X, db = X^T w,
        dp = (X - X o X)^T w, with w the upstream gradient of h.
        """

        @staticmethod
        def forward(ctx, X, Q, b, p):
            h, G = eval_penalty_grad(Q.contiguous(), b.contiguous(), p.contiguous(), X.contiguous())
            ctx.save_for_backward(X, G)
            ctx.shape = X.shape
            return h

        @staticmethod
        def backward(ctx, w):
            X, G = ctx.saved_tensors
            need = ctx.needs_input_grad
            want = [k for k, f in zip(("dX", "dQ", "db", "dp"), need) if f]
            dX, dQ, db, dp = penalty_adjoint(X.contiguous(), G, w.contiguous().to(G.dtype), want=want)
            if dX is not None:
                dX = dX.reshape(ctx.shape).to(X.dtype)
            return dX, dQ, db, dp

    return PenaltyFn


_penalty_fn = None


def penalty_fn():
    global _penalty_fn
    if _penalty_fn is None:
        _penalty_fn = _make_penalty_fn()
    return _penalty_fn
