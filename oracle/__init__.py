"""FP64 CPU oracle for reachability probabilities (test infrastructure only).

Plain single-threaded reference used to check the GPU library.  It shares no
code with the GPU path; only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  The arithmetic lives in
``rp_oracle.c`` (plain C, FP64, one thread); this module only builds that file
with gcc, loads it with ctypes and marshals numpy arrays.

Paper: Cormie-Bowins, "A Comparison of Sequential and GPU Implementations of
Iterative Methods to Compute Reachability Probabilities" (GRAPHITE 2012).
  * partition into S_{=0}, S_{=1}, S_?  -- Section 2.2
  * reduced system (I - A) x = b        -- Section 2.3
  * Jacobi                              -- Section 3.1
  * BiCGStab                            -- Section 3.2
  * general A x = b of the experiments   -- Section 6
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rp_oracle.c")
_LIB = os.path.join(_HERE, "librp_oracle.so")

OK, BAD_CHAIN, NOT_CONVERGED, BREAKDOWN, SINGULAR, NOMEM = range(6)
S0, S1, SQ = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile rp_oracle.c with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
            "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.orc_validate.restype = I64
        lib.orc_validate.argtypes = [I64, I64, P, P, P, I64, P, D, P]
        lib.orc_partition.restype = ctypes.c_int
        lib.orc_partition.argtypes = [I64, P, P, P, P, ctypes.c_int, P]
        lib.orc_assemble.restype = ctypes.c_int
        lib.orc_assemble.argtypes = [I64, P, P, P, P, P, P, P, P, P, P, P, P]
        lib.orc_transpose.restype = ctypes.c_int
        lib.orc_transpose.argtypes = [I64, P, P, P, P, P, P]
        lib.orc_residual.restype = D
        lib.orc_residual.argtypes = [I64, P, P, P, P, P, P, P]
        lib.orc_tbound.restype = D
        lib.orc_tbound.argtypes = [I64, P, P, P, P, I64]
        lib.orc_jacobi.restype = ctypes.c_int
        lib.orc_jacobi.argtypes = [I64, P, P, P, P, P, P, D, I64, ctypes.c_int, D, P, P, P]
        lib.orc_bicgstab.restype = ctypes.c_int
        lib.orc_bicgstab.argtypes = [I64, P, P, P, P, P, P, D, I64, ctypes.c_int, D, P, P, P]
        lib.orc_dense_solve.restype = ctypes.c_int
        lib.orc_dense_solve.argtypes = [I64, P, P, P]
        lib.orc_dense_m.restype = None
        lib.orc_dense_m.argtypes = [I64, P, P, P, P, P]
        lib.orc_gradient.restype = None
        lib.orc_gradient.argtypes = [I64, P, P, P, P, P, P, P]
        lib.orc_matrix_system.restype = ctypes.c_int
        lib.orc_matrix_system.argtypes = [I64, P, P, P, P, P, P, P, P, P, P]
        lib.orc_dominance_bound.restype = D
        lib.orc_dominance_bound.argtypes = [I64, P, P, P]
        lib.orc_scc.restype = ctypes.c_int
        lib.orc_scc.argtypes = [I64, P, P, P, P, P, P]
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else ctypes.c_void_p(0 if a is None else a.ctypes.data)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


@dataclass
class Reduced:
    """Reduced system over S_? (Section 2.3): (I - A) x = b with
    d = 1 - P(i,i), A_off = off-diagonal part in CSR, b = P(i, S_{=1})."""
    nq: int
    map: np.ndarray      # int64[n]: reduced index of each state, -1 outside S_?
    arp: np.ndarray      # int64[nq+1]
    acol: np.ndarray     # int64[z]
    aval: np.ndarray     # float64[z]
    d: np.ndarray        # float64[nq]
    b: np.ndarray        # float64[nq]

    @property
    def z(self) -> int:
        return int(self.arp[-1]) if self.nq else 0


def validate(n, rp, col, val, inst_off=None, tol=1e-12):
    """Input check of Section 2 (row-stochastic P); returns (row, reason),
    row = -1 when the chain is well formed."""
    lib = _load()
    rp = _c(rp, np.int32); col = _c(col, np.int32); val = _c(val, np.float64)
    if inst_off is None:
        inst_off = np.array([0, n], dtype=np.int64)
    inst_off = _c(inst_off, np.int64)
    reason = ctypes.c_int32(0)
    row = lib.orc_validate(n, int(rp[n]) if n >= 0 else 0, _p(rp), _p(col), _p(val),
                           len(inst_off) - 1, _p(inst_off), tol, ctypes.byref(reason))
    return int(row), int(reason.value)


def partition(n, rp, col, val, goal, prob0_only=False):
    """Class array (0 = S_{=0}, 1 = S_{=1}, 2 = S_?) of Section 2.2."""
    lib = _load()
    rp = _c(rp, np.int32); col = _c(col, np.int32); val = _c(val, np.float64)
    goal = _c(goal, np.uint8)
    cls = np.zeros(max(n, 1), dtype=np.uint8)
    rc = lib.orc_partition(n, _p(rp), _p(col), _p(val), _p(goal), int(bool(prob0_only)), _p(cls))
    if rc != OK:
        raise MemoryError("oracle partition failed")
    return cls[:n]


def assemble(n, rp, col, val, cls) -> Reduced:
    """Reduced system of Section 2.3 over the S_? states of `cls`."""
    lib = _load()
    rp = _c(rp, np.int32); col = _c(col, np.int32); val = _c(val, np.float64)
    cls = _c(cls, np.uint8)
    nnz = int(rp[n])
    mp = np.zeros(max(n, 1), dtype=np.int64)
    arp = np.zeros(n + 1, dtype=np.int64)
    acol = np.zeros(max(nnz, 1), dtype=np.int64)
    aval = np.zeros(max(nnz, 1), dtype=np.float64)
    d = np.zeros(max(n, 1), dtype=np.float64)
    b = np.zeros(max(n, 1), dtype=np.float64)
    nq = ctypes.c_int64(0); z = ctypes.c_int64(0)
    lib.orc_assemble(n, _p(rp), _p(col), _p(val), _p(cls), _p(mp), ctypes.byref(nq),
                     _p(arp), _p(acol), _p(aval), _p(d), _p(b), ctypes.byref(z))
    nq = nq.value; z = z.value
    return Reduced(nq, mp[:n].copy(), arp[:nq + 1].copy(), acol[:z].copy(), aval[:z].copy(),
                   d[:nq].copy(), b[:nq].copy())


def transpose(red: Reduced) -> Reduced:
    """(I - A)^T as a Reduced system with the same diagonal (b left empty)."""
    lib = _load()
    z = red.z
    trp = np.zeros(red.nq + 1, dtype=np.int64)
    tcol = np.zeros(max(z, 1), dtype=np.int64)
    tval = np.zeros(max(z, 1), dtype=np.float64)
    lib.orc_transpose(red.nq, _p(red.arp), _p(red.acol), _p(red.aval), _p(trp), _p(tcol), _p(tval))
    return Reduced(red.nq, red.map, trp, tcol[:z].copy(), tval[:z].copy(), red.d,
                   np.zeros(red.nq))


def residual(red: Reduced, b, x):
    """r = b - (I - A) x and its max norm."""
    lib = _load()
    b = _c(b, np.float64); x = _c(x, np.float64)
    r = np.zeros(max(red.nq, 1))
    nrm = lib.orc_residual(red.nq, _p(red.arp), _p(red.acol), _p(red.aval), _p(red.d),
                           _p(b), _p(x), _p(r))
    return r[:red.nq], float(nrm)


def tbound(red: Reduced, max_iter=10_000_000):
    """Upper bound on ||(I - A)^{-1} 1||_inf (error certificate factor)."""
    lib = _load()
    return float(lib.orc_tbound(red.nq, _p(red.arp), _p(red.acol), _p(red.aval), _p(red.d), max_iter))


def jacobi(red: Reduced, b=None, x0=None, tol=1e-10, max_iter=10_000_000, stop_mode=0, tb=0.0):
    """Jacobi method of Section 3.1.  Returns (x, iters, delta, rc)."""
    lib = _load()
    b = red.b if b is None else _c(b, np.float64)
    x0 = None if x0 is None else _c(x0, np.float64)
    x = np.zeros(max(red.nq, 1))
    it = ctypes.c_int64(0); dl = ctypes.c_double(0.0)
    rc = lib.orc_jacobi(red.nq, _p(red.arp), _p(red.acol), _p(red.aval), _p(red.d), _p(b),
                        _p(x0) if x0 is not None else None, tol, max_iter, stop_mode, tb,
                        _p(x), ctypes.byref(it), ctypes.byref(dl))
    return x[:red.nq], int(it.value), float(dl.value), int(rc)


def bicgstab(red: Reduced, b=None, x0=None, tol=1e-10, max_iter=10_000_000, stop_mode=0, tb=0.0):
    """BiCGStab of Section 3.2.  Returns (x, iters, max|s|, rc)."""
    lib = _load()
    b = red.b if b is None else _c(b, np.float64)
    x0 = None if x0 is None else _c(x0, np.float64)
    x = np.zeros(max(red.nq, 1))
    it = ctypes.c_int64(0); sm = ctypes.c_double(0.0)
    rc = lib.orc_bicgstab(red.nq, _p(red.arp), _p(red.acol), _p(red.aval), _p(red.d), _p(b),
                          _p(x0) if x0 is not None else None, tol, max_iter, stop_mode, tb,
                          _p(x), ctypes.byref(it), ctypes.byref(sm))
    return x[:red.nq], int(it.value), float(sm.value), int(rc)


def dense_m(red: Reduced):
    """Dense I - A (row-major) of the reduced system."""
    lib = _load()
    m = np.zeros((red.nq, red.nq))
    lib.orc_dense_m(red.nq, _p(red.arp), _p(red.acol), _p(red.aval), _p(red.d), _p(m))
    return m


def dense_solve(m, rhs):
    """Gaussian elimination with partial pivoting (m is copied)."""
    lib = _load()
    m = np.array(m, dtype=np.float64, order="C", copy=True)
    rhs = _c(rhs, np.float64)
    nq = m.shape[0]
    x = np.zeros(max(nq, 1))
    rc = lib.orc_dense_solve(nq, _p(m), _p(rhs), _p(x))
    if rc != OK:
        raise np.linalg.LinAlgError("singular system")
    return x[:nq]


def expand(n, cls, red: Reduced, xq):
    """Full vector x over S: 0 on S_{=0}, 1 on S_{=1}, the solution on S_? (Section 2.3)."""
    x = np.where(cls == S1, 1.0, 0.0).astype(np.float64)
    idx = np.nonzero(cls == SQ)[0]
    x[idx] = xq[red.map[idx]]
    return x


def gradient(n, rp, col, cls, red: Reduced, lam, xfull):
    """dL/dP(i,j) = lam_i * xfull_j on P's stored entries of S_? rows."""
    lib = _load()
    rp = _c(rp, np.int32); col = _c(col, np.int32); cls = _c(cls, np.uint8)
    lam = _c(lam, np.float64); xfull = _c(xfull, np.float64)
    g = np.zeros(max(int(rp[n]), 1))
    lib.orc_gradient(n, _p(rp), _p(col), _p(cls), _p(red.map), _p(lam), _p(xfull), _p(g))
    return g[:int(rp[n])]


@dataclass
class Solution:
    cls: np.ndarray
    red: Reduced
    x: np.ndarray          # full vector over S
    xq: np.ndarray         # reduced solution
    iters: int
    tb: float
    rc: int


def solve(n, rp, col, val, goal, method="jacobi", prob0_only=False, tol=1e-12,
          stop_mode=1, max_iter=10_000_000) -> Solution:
    """Whole pipeline on one chain: partition, reduced system, solve.
    stop_mode 1 certifies max|x - x*| <= tol; stop_mode 0 is the paper's rule."""
    cls = partition(n, rp, col, val, goal, prob0_only)
    red = assemble(n, rp, col, val, cls)
    tb = tbound(red) if stop_mode == 1 else 0.0
    fn = jacobi if method == "jacobi" else bicgstab
    xq, it, _, rc = fn(red, tol=tol, max_iter=max_iter, stop_mode=stop_mode, tb=tb)
    return Solution(cls, red, expand(n, cls, red, xq), xq, it, tb, rc)


def adjoint(sol: Solution, seed_full, tol=1e-12, method="jacobi"):
    """Solve (I - A)^T lam = seed restricted to S_?, certified to tol."""
    red_t = transpose(sol.red)
    idx = np.nonzero(sol.cls == SQ)[0]
    rhs = np.zeros(sol.red.nq)
    rhs[sol.red.map[idx]] = np.asarray(seed_full, dtype=np.float64)[idx]
    tbt = tbound(red_t)
    fn = jacobi if method == "jacobi" else bicgstab
    lam, it, _, rc = fn(red_t, b=rhs, tol=tol, stop_mode=1, tb=tbt)
    return lam, it, tbt, rc


def matrix_system(n, rp, col, val, rhs) -> Reduced:
    """The general system A x = rhs of the experiments of Section 6 (A
    square in compressed row storage, diagonal stored) in the solvers' form:
    d = diag(A), A_off = -(off-diagonal part), b = rhs; every row is its own
    unknown (map = identity)."""
    lib = _load()
    rp = _c(rp, np.int32); col = _c(col, np.int32); val = _c(val, np.float64)
    rhs = _c(rhs, np.float64)
    nnz = int(rp[n])
    arp = np.zeros(n + 1, dtype=np.int64)
    acol = np.zeros(max(nnz, 1), dtype=np.int64)
    aval = np.zeros(max(nnz, 1), dtype=np.float64)
    d = np.zeros(max(n, 1)); b = np.zeros(max(n, 1))
    z = ctypes.c_int64(0)
    rc = lib.orc_matrix_system(n, _p(rp), _p(col), _p(val), _p(rhs), _p(arp), _p(acol), _p(aval), _p(d), _p(b),
                               ctypes.byref(z))
    if rc != OK:
        raise np.linalg.LinAlgError("a row has no nonzero diagonal entry")
    z = z.value
    return Reduced(n, np.arange(n, dtype=np.int64), arp, acol[:z].copy(), aval[:z].copy(), d[:n].copy(),
                   b[:n].copy())


def dominance_bound(red: Reduced) -> float:
    """Varah's bound on ||A^{-1}||_inf for a strictly row diagonally dominant
    A (-1 when some row is not strictly dominant)."""
    lib = _load()
    return float(lib.orc_dominance_bound(red.nq, _p(red.arp), _p(red.aval), _p(red.d)))


def solve_matrix(n, rp, col, val, rhs, method="jacobi", tol=1e-12, stop_mode=1, max_iter=10_000_000):
    """Section 6's A x = rhs: certified (stop_mode 1, by the dominance bound)
    or under the paper's rule (stop_mode 0).  Returns (x, iterations, rc)."""
    red = matrix_system(n, rp, col, val, rhs)
    tb = dominance_bound(red) if stop_mode == 1 else 0.0
    if stop_mode == 1 and tb < 0:
        raise ValueError("certified stop needs a strictly diagonally dominant A")
    fn = jacobi if method == "jacobi" else bicgstab
    x, it, _, rc = fn(red, tol=tol, max_iter=max_iter, stop_mode=stop_mode, tb=tb)
    return x, it, rc


def scc(red: Reduced):
    """Strongly connected components of A_off's graph over S_? (Tarjan):
    (label, level, ncomp) with label = smallest reduced index of the
    component and level = 0 for components no edge leaves, else 1 + the
    largest level an edge leads to (reverse topological levels)."""
    lib = _load()
    label = np.zeros(max(red.nq, 1), dtype=np.int64)
    level = np.zeros(max(red.nq, 1), dtype=np.int64)
    nc = ctypes.c_int64(0)
    rc = lib.orc_scc(red.nq, _p(red.arp), _p(red.acol), _p(red.aval), _p(label), _p(level), ctypes.byref(nc))
    if rc != OK:
        raise MemoryError("oracle scc failed")
    return label[:red.nq].copy(), level[:red.nq].copy(), int(nc.value)
