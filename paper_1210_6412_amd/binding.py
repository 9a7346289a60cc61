"""ctypes binding of librp (include/rp.h): argument marshalling only.

Every function here has the name of the C entry point it calls and only
converts arguments: torch CUDA tensors become device pointers, option keywords
fill an ``rp_opts`` struct, per-instance ``rp_solve_info`` records come back
as dicts.  All arithmetic runs in the HIP kernels of librp.  If the library
is missing or cannot be loaded the calls raise; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librp.so")

RP_OK = 0
RP_ERR_INVALID_ARG = 1
RP_ERR_BAD_CHAIN = 2
RP_ERR_NOT_CONVERGED = 3
RP_ERR_BREAKDOWN = 4
RP_ERR_NONFINITE = 5
RP_ERR_OOM = 6
RP_ERR_HIP = 7
RP_ERR_TOO_LARGE = 8
STATUS_NAMES = {0: "RP_OK", 1: "RP_ERR_INVALID_ARG", 2: "RP_ERR_BAD_CHAIN", 3: "RP_ERR_NOT_CONVERGED",
                4: "RP_ERR_BREAKDOWN", 5: "RP_ERR_NONFINITE", 6: "RP_ERR_OOM", 7: "RP_ERR_HIP",
                8: "RP_ERR_TOO_LARGE"}

RP_S0, RP_S1, RP_SQ = 0, 1, 2
RP_PROB0_ONLY = 1
RP_STOP_DELTA, RP_STOP_CERTIFIED, RP_STOP_RESIDUAL = 0, 1, 2
RP_FP64, RP_FP32_REFINED = 0, 1
RP_TILING_AUTO, RP_TILING_OFF = 0, 1
RP_SCHEDULE_SEGSCAN = -2
RP_UPDATE_TWO_BUFFER, RP_UPDATE_IN_PLACE = 0, 1

EXPORTED = ["rp_context_create", "rp_context_destroy", "rp_last_error", "rp_opts_default", "rp_precompute",
            "rp_system_destroy", "rp_matrix_system", "rp_classify_noalloc", "rp_system_sizes",
            "rp_system_instance_sizes",
            "rp_system_export",
            "rp_jacobi", "rp_bicgstab", "rp_solve_rhs", "rp_adjoint", "rp_scc", "rp_scc_solve", "rp_profile_enable",
            "rp_profile_read"]
PROF_KERNELS = {0: "jacobi_fp64", 1: "jacobi_fp32", 2: "spmv_fp64", 3: "spmv_fp32", 4: "vector_fp64",
                5: "vector_fp32", 6: "residual_fp64", 7: "bicgstab_fp64", 8: "bicgstab_fp32",
                9: "jacobi_tail_fp64", 10: "jacobi_tail_fp32"}


class RpChain(ctypes.Structure):
    _fields_ = [("num_instances", ctypes.c_int32), ("inst_state_offset", ctypes.POINTER(ctypes.c_int64)),
                ("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class RpOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("stop", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_iter", ctypes.c_int64), ("inner_tol", ctypes.c_double), ("max_refine", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("schedule", ctypes.c_int32), ("tiling", ctypes.c_int32),
                ("x0", ctypes.c_void_p), ("update", ctypes.c_int32), ("graph", ctypes.c_int32)]


class RpSolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("refinements", ctypes.c_int64), ("final_delta", ctypes.c_double),
                ("residual_inf", ctypes.c_double), ("error_bound", ctypes.c_double), ("status", ctypes.c_int32),
                ("lanes", ctypes.c_int32), ("panels", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class RpSccInfo(ctypes.Structure):
    _fields_ = [("components", ctypes.c_int64), ("cyclic_components", ctypes.c_int64), ("largest", ctypes.c_int64),
                ("levels", ctypes.c_int32), ("rounds", ctypes.c_int32), ("substitution_levels", ctypes.c_int32),
                ("jacobi_levels", ctypes.c_int32), ("substitution_rows", ctypes.c_int64),
                ("jacobi_rows", ctypes.c_int64), ("jacobi_sweeps", ctypes.c_int64)]


def _scc_dict(si):
    return {k: getattr(si, k) for k, _ in RpSccInfo._fields_}


class RpError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code
        self.message = message


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librp.so (torch is imported first so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"librp.so not built at {path}; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.rp_context_create.argtypes = [ctypes.POINTER(P), I, P]
    lib.rp_context_create.restype = I
    lib.rp_context_destroy.argtypes = [P]
    lib.rp_context_destroy.restype = I
    lib.rp_last_error.argtypes = [P]
    lib.rp_last_error.restype = ctypes.c_char_p
    lib.rp_opts_default.argtypes = [ctypes.POINTER(RpOpts)]
    lib.rp_opts_default.restype = None
    lib.rp_precompute.argtypes = [P, ctypes.POINTER(RpChain), P, ctypes.c_uint32, D, P, ctypes.POINTER(P)]
    lib.rp_precompute.restype = I
    lib.rp_matrix_system.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), I64, I64, P, P, P, P,
                                     ctypes.POINTER(P)]
    lib.rp_matrix_system.restype = I
    lib.rp_classify_noalloc.argtypes = [P, ctypes.POINTER(RpChain), P, ctypes.c_uint32, D, P]
    lib.rp_classify_noalloc.restype = I
    lib.rp_system_destroy.argtypes = [P]
    lib.rp_system_destroy.restype = I
    lib.rp_system_sizes.argtypes = [P] + [ctypes.POINTER(I64)] * 4
    lib.rp_system_sizes.restype = I
    lib.rp_system_instance_sizes.argtypes = [P, ctypes.POINTER(I64)]
    lib.rp_system_instance_sizes.restype = I
    lib.rp_system_export.argtypes = [P, P, P, P, P, P, P]
    lib.rp_system_export.restype = I
    for fn in (lib.rp_jacobi, lib.rp_bicgstab):
        fn.argtypes = [P, P, ctypes.POINTER(RpOpts), P, ctypes.POINTER(RpSolveInfo)]
        fn.restype = I
    lib.rp_solve_rhs.argtypes = [P, P, I, P, ctypes.POINTER(RpOpts), P, ctypes.POINTER(RpSolveInfo)]
    lib.rp_solve_rhs.restype = I
    lib.rp_adjoint.argtypes = [P, P, I, P, P, ctypes.POINTER(RpOpts), P, P, ctypes.POINTER(RpSolveInfo)]
    lib.rp_adjoint.restype = I
    lib.rp_scc.argtypes = [P, P, P, P, ctypes.POINTER(RpSccInfo)]
    lib.rp_scc.restype = I
    lib.rp_scc_solve.argtypes = [P, P, ctypes.POINTER(RpOpts), P, ctypes.POINTER(RpSolveInfo),
                                 ctypes.POINTER(RpSccInfo)]
    lib.rp_scc_solve.restype = I
    lib.rp_profile_enable.argtypes = [P, I]
    lib.rp_profile_enable.restype = I
    lib.rp_profile_read.argtypes = [P, I, ctypes.POINTER(I64), ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.rp_profile_read.restype = I
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _is_cuda(t) -> bool:
    return t.is_cuda


def _device_index(t):
    return t.device.index


def _dev(t, dtype, name, n=None, device=None):
    """Check that t is a contiguous CUDA tensor of the given dtype, element
    count and device before its pointer is handed to the library."""
    if not isinstance(t, torch.Tensor) or not _is_cuda(t):
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    if device is not None and _device_index(t) != device:
        raise ValueError(f"{name} is on {t.device}, the context is on cuda:{device}")
    return t


class Context:
    """An rp_context bound to one device and one HIP stream."""

    def __init__(self, handle, device, stream):
        self.handle = handle
        self.device = device
        self.stream = stream

    def last_error(self) -> str:
        return rp_last_error(self)

    def close(self):
        if self.handle:
            load_library().rp_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class System:
    """An rp_system (library-owned reduced system of a chain)."""
    handle: ctypes.c_void_p
    ctx: Context
    n: int
    nnz: int
    num_instances: int

    def close(self):
        if self.handle:
            load_library().rp_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check(ctx, code, ok=(RP_OK,)):
    if code not in ok:
        raise RpError(code, rp_last_error(ctx) if ctx is not None else "")
    return code


# ---------------------------------------------------------------------------
# entry points

def rp_context_create(device: int = 0, stream=None) -> Context:
    lib = load_library()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    handle = ctypes.c_void_p()
    sp = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    _check(None, lib.rp_context_create(ctypes.byref(handle), device, ctypes.c_void_p(sp)))
    return Context(handle, device, stream)


def rp_context_destroy(ctx: Context) -> None:
    ctx.close()


def rp_last_error(ctx: Context) -> str:
    return load_library().rp_last_error(ctx.handle).decode()


def rp_opts_default(**kw) -> RpOpts:
    """Default options with keyword overrides.  x0 must be a float64 CUDA
    tensor of the chain's n states (checked against the system when the
    options are used); the options keep a reference to it so that its memory
    stays valid while they do."""
    o = RpOpts()
    load_library().rp_opts_default(ctypes.byref(o))
    o._x0_tensor = None
    for k, v in kw.items():
        if k == "x0":
            if v is not None:
                _dev(v, torch.float64, "x0")
            o._x0_tensor = v
            o.x0 = v.data_ptr() if v is not None else None
        elif not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        else:
            setattr(o, k, v)
    return o


def _check_opts(opts, sys, ctx):
    """The starting point held by opts (if set through rp_opts_default) must
    match the system: n float64 elements, contiguous, on the context's device,
    and still be the tensor whose pointer the options carry."""
    t = getattr(opts, "_x0_tensor", None)
    if t is not None:
        _dev(t, torch.float64, "x0", sys.n, device=ctx.device)
        if opts.x0 != t.data_ptr():
            raise ValueError("opts.x0 no longer points at the x0 tensor the options were built with")


def rp_precompute(ctx: Context, row_ptr, col, val, goal_mask, inst_state_offset=None, flags: int = 0,
                  rowsum_tol: float = 0.0, class_out=None) -> System:
    lib = load_library()
    n = row_ptr.numel() - 1
    nnz = col.numel()
    _dev(row_ptr, torch.int32, "row_ptr", device=ctx.device)
    _dev(col, torch.int32, "col", device=ctx.device)
    _dev(val, torch.float64, "val", nnz, device=ctx.device)
    _dev(goal_mask, torch.uint8, "goal_mask", n, device=ctx.device)
    if class_out is not None:
        _dev(class_out, torch.uint8, "class_out", n, device=ctx.device)
    if inst_state_offset is None:
        inst_state_offset = [0, n]
    off = (ctypes.c_int64 * len(inst_state_offset))(*[int(v) for v in inst_state_offset])
    ch = RpChain(len(inst_state_offset) - 1, ctypes.cast(off, ctypes.POINTER(ctypes.c_int64)), n, nnz,
                 _ptr(row_ptr), _ptr(col), _ptr(val))
    handle = ctypes.c_void_p()
    _check(ctx, lib.rp_precompute(ctx.handle, ctypes.byref(ch), _ptr(goal_mask), flags, rowsum_tol,
                                  _ptr(class_out), ctypes.byref(handle)))
    return System(handle, ctx, n, nnz, len(inst_state_offset) - 1)


def rp_matrix_system(ctx: Context, row_ptr, col, val, rhs, inst_row_offset=None) -> System:
    """A x = rhs for a general square A (diagonal stored): a System for the
    same solvers."""
    n = row_ptr.numel() - 1
    nnz = col.numel()
    _dev(row_ptr, torch.int32, "row_ptr", n + 1, device=ctx.device)
    _dev(col, torch.int32, "col", device=ctx.device)
    _dev(val, torch.float64, "val", nnz, device=ctx.device)
    _dev(rhs, torch.float64, "rhs", n, device=ctx.device)
    if inst_row_offset is None:
        inst_row_offset = [0, n]
    off = (ctypes.c_int64 * len(inst_row_offset))(*[int(v) for v in inst_row_offset])
    handle = ctypes.c_void_p()
    _check(ctx, load_library().rp_matrix_system(ctx.handle, len(inst_row_offset) - 1,
                                                ctypes.cast(off, ctypes.POINTER(ctypes.c_int64)), n, nnz,
                                                _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(rhs), ctypes.byref(handle)))
    return System(handle, ctx, n, nnz, len(inst_row_offset) - 1)


def rp_classify_noalloc(ctx: Context, row_ptr, col, val, goal_mask, class_out, inst_state_offset=None,
                        flags: int = 0, rowsum_tol: float = 0.0):
    """State classes into class_out (uint8 CUDA tensor of n) with no device
    allocation in the library.  Returns class_out."""
    n = row_ptr.numel() - 1
    nnz = col.numel()
    _dev(row_ptr, torch.int32, "row_ptr", device=ctx.device)
    _dev(col, torch.int32, "col", device=ctx.device)
    _dev(val, torch.float64, "val", nnz, device=ctx.device)
    _dev(goal_mask, torch.uint8, "goal_mask", n, device=ctx.device)
    _dev(class_out, torch.uint8, "class_out", n, device=ctx.device)
    if inst_state_offset is None:
        inst_state_offset = [0, n]
    off = (ctypes.c_int64 * len(inst_state_offset))(*[int(v) for v in inst_state_offset])
    ch = RpChain(len(inst_state_offset) - 1, ctypes.cast(off, ctypes.POINTER(ctypes.c_int64)), n, nnz,
                 _ptr(row_ptr), _ptr(col), _ptr(val))
    _check(ctx, load_library().rp_classify_noalloc(ctx.handle, ctypes.byref(ch), _ptr(goal_mask), flags, rowsum_tol,
                                                   _ptr(class_out)))
    return class_out


def rp_system_destroy(sys: System) -> None:
    sys.close()


def rp_system_sizes(sys: System):
    v = [ctypes.c_int64() for _ in range(4)]
    _check(sys.ctx, load_library().rp_system_sizes(sys.handle, *[ctypes.byref(x) for x in v]))
    return tuple(int(x.value) for x in v)


def rp_system_instance_sizes(sys: System):
    arr = (ctypes.c_int64 * sys.num_instances)()
    _check(sys.ctx, load_library().rp_system_instance_sizes(sys.handle, arr))
    return [int(v) for v in arr]


def rp_system_export(ctx: Context, sys: System):
    _, _, nq, z = rp_system_sizes(sys)
    dev = torch.device("cuda", ctx.device)
    rp = torch.empty(nq + 1, dtype=torch.int32, device=dev)
    col = torch.empty(max(z, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(z, 1), dtype=torch.float64, device=dev)
    d = torch.empty(max(nq, 1), dtype=torch.float64, device=dev)
    b = torch.empty(max(nq, 1), dtype=torch.float64, device=dev)
    _check(ctx, load_library().rp_system_export(ctx.handle, sys.handle, _ptr(rp), _ptr(col), _ptr(val), _ptr(d),
                                                 _ptr(b)))
    return rp, col[:z], val[:z], d[:nq], b[:nq]


def _infos(arr):
    return [dict(iterations=int(i.iterations), refinements=int(i.refinements), final_delta=float(i.final_delta),
                 residual_inf=float(i.residual_inf), error_bound=float(i.error_bound), status=int(i.status),
                 lanes=int(i.lanes), panels=int(i.panels))
            for i in arr]


_SOLVE_OK = (RP_OK, RP_ERR_NOT_CONVERGED, RP_ERR_BREAKDOWN, RP_ERR_NONFINITE)


def _solve(fn, ctx, sys, x_out, opts):
    _check_opts(opts, sys, ctx)
    if x_out is None:
        x_out = torch.empty(sys.n, dtype=torch.float64, device=torch.device("cuda", ctx.device))
    _dev(x_out, torch.float64, "x_out", sys.n, device=ctx.device)
    info = (RpSolveInfo * sys.num_instances)()
    code = _check(ctx, fn(ctx.handle, sys.handle, ctypes.byref(opts), _ptr(x_out), info), _SOLVE_OK)
    return x_out, _infos(info), code


def rp_jacobi(ctx: Context, sys: System, x_out=None, opts: RpOpts | None = None, **kw):
    """Returns (x_out, per-instance info dicts, status code)."""
    return _solve(load_library().rp_jacobi, ctx, sys, x_out, opts or rp_opts_default(**kw))


def rp_bicgstab(ctx: Context, sys: System, x_out=None, opts: RpOpts | None = None, **kw):
    return _solve(load_library().rp_bicgstab, ctx, sys, x_out, opts or rp_opts_default(**kw))


def rp_solve_rhs(ctx: Context, sys: System, rhs, method: int = 0, y_out=None, opts: RpOpts | None = None, **kw):
    """(I - A) y = rhs on S_?.  Returns (y_out, per-instance info dicts, status code)."""
    _dev(rhs, torch.float64, "rhs", sys.n, device=ctx.device)
    if y_out is not None:
        _dev(y_out, torch.float64, "y_out", sys.n, device=ctx.device)
    o = opts or rp_opts_default(**kw)
    _check_opts(o, sys, ctx)
    if y_out is None:
        y_out = torch.empty(sys.n, dtype=torch.float64, device=torch.device("cuda", ctx.device))
    info = (RpSolveInfo * sys.num_instances)()
    code = _check(ctx, load_library().rp_solve_rhs(ctx.handle, sys.handle, method, _ptr(rhs), ctypes.byref(o),
                                                   _ptr(y_out), info), _SOLVE_OK)
    return y_out, _infos(info), code


def rp_scc(ctx: Context, sys: System, label_out=None, level_out=None):
    """Strongly connected components of S_?: (label, level, info dict); label
    and level are int32 CUDA tensors of the chain's n states (-1 outside
    S_?), allocated when not given."""
    dev = torch.device("cuda", ctx.device)
    if label_out is None:
        label_out = torch.empty(sys.n, dtype=torch.int32, device=dev)
    if level_out is None:
        level_out = torch.empty(sys.n, dtype=torch.int32, device=dev)
    _dev(label_out, torch.int32, "label_out", sys.n, device=ctx.device)
    _dev(level_out, torch.int32, "level_out", sys.n, device=ctx.device)
    si = RpSccInfo()
    _check(ctx, load_library().rp_scc(ctx.handle, sys.handle, _ptr(label_out), _ptr(level_out), ctypes.byref(si)))
    return label_out, level_out, _scc_dict(si)


def rp_scc_solve(ctx: Context, sys: System, x_out=None, opts: RpOpts | None = None, **kw):
    """Solve by components in reverse topological order, then the ordinary
    refinement.  Returns (x_out, per-instance info dicts, status code, scc info
    dict)."""
    o = opts or rp_opts_default(**kw)
    _check_opts(o, sys, ctx)
    if x_out is None:
        x_out = torch.empty(sys.n, dtype=torch.float64, device=torch.device("cuda", ctx.device))
    _dev(x_out, torch.float64, "x_out", sys.n, device=ctx.device)
    info = (RpSolveInfo * sys.num_instances)()
    si = RpSccInfo()
    code = _check(ctx, load_library().rp_scc_solve(ctx.handle, sys.handle, ctypes.byref(o), _ptr(x_out), info,
                                                   ctypes.byref(si)), _SOLVE_OK)
    return x_out, _infos(info), code, _scc_dict(si)


def rp_adjoint(ctx: Context, sys: System, x, seed, method: int = 0, lambda_out=None, grad_out=None,
               opts: RpOpts | None = None, **kw):
    """Returns (lambda_out, grad_out, per-instance info dicts, status code)."""
    dev = torch.device("cuda", ctx.device)
    _dev(x, torch.float64, "x", sys.n, device=ctx.device)
    _dev(seed, torch.float64, "seed", sys.n, device=ctx.device)
    if lambda_out is not None:
        _dev(lambda_out, torch.float64, "lambda_out", sys.n, device=ctx.device)
    if grad_out is not None:
        _dev(grad_out, torch.float64, "grad_out", sys.nnz, device=ctx.device)
    o = opts or rp_opts_default(**kw)
    _check_opts(o, sys, ctx)
    if lambda_out is None:
        lambda_out = torch.empty(sys.n, dtype=torch.float64, device=dev)
    if grad_out is None:
        grad_out = torch.empty(max(sys.nnz, 1), dtype=torch.float64, device=dev)[:sys.nnz]
    info = (RpSolveInfo * sys.num_instances)()
    code = _check(ctx, load_library().rp_adjoint(ctx.handle, sys.handle, method, _ptr(x), _ptr(seed), ctypes.byref(o),
                                                 _ptr(lambda_out), _ptr(grad_out) if sys.nnz else None, info),
                  _SOLVE_OK)
    return lambda_out, grad_out, _infos(info), code


def rp_profile_enable(ctx: Context, enable: bool = True) -> None:
    _check(ctx, load_library().rp_profile_enable(ctx.handle, 1 if enable else 0))


def rp_profile_read(ctx: Context):
    """{kernel name: (launches, total ms, algorithmic bytes)} since the last enable."""
    out = {}
    for k, name in PROF_KERNELS.items():
        n, ms, b = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(ctx, load_library().rp_profile_read(ctx.handle, k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(b)))
        out[name] = (int(n.value), float(ms.value), float(b.value))
    return out
