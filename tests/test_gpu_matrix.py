"""The general systems of the paper's experiments (Section 6): random
strictly diagonally dominant matrices of positive integers, A x = b, solved
by the same Jacobi and BiCGStab kernels through rp_matrix_system, against
the oracle (certified by Varah's bound on ||A^{-1}||_inf)."""
import numpy as np
import pytest
import torch

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from tests import _gpu as G

pytestmark = pytest.mark.gpu


def _dev(m):
    d = torch.device("cuda", 0)
    return (torch.from_numpy(m.rp).to(d), torch.from_numpy(m.col).to(d), torch.from_numpy(m.val).to(d),
            torch.from_numpy(m.rhs).to(d))


def _system(m):
    rp_, col, val, rhs = _dev(m)
    return rp.rp_matrix_system(G.ctx(), rp_, col, val, rhs, list(m.inst_off))


def _batch():
    ms = [cg.diag_dominant(300, density=0.10, seed=11), cg.diag_dominant(2000, density=0.01, seed=12),
          cg.diag_dominant(313, offdiag=669 - 313, seed=13), cg.diag_dominant(7647, offdiag=7647 - 1, seed=14),
          cg.diag_dominant(25_000, density=0.0004, seed=15)]
    return ms, cg.concat_matrices(ms, "dd batch")


@pytest.mark.parametrize("method", ["jacobi", "bicgstab"])
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_matrix_certified_matches_oracle(method, precision):
    ms, m = _batch()
    sys = _system(m)
    prec = rp.RP_FP64 if precision == "fp64" else rp.RP_FP32_REFINED
    G.banner(f"matrix certified {method} {precision} n={m.n}")
    x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=prec)
    assert code == rp.binding.RP_OK, info
    for k, mk in enumerate(ms):
        xo, it, rc = oracle.solve_matrix(mk.n, mk.rp, mk.col, mk.val, mk.rhs, "bicgstab", tol=1e-12)
        assert rc == oracle.OK
        lo, hi = m.inst_off[k], m.inst_off[k + 1]
        assert info[k]["error_bound"] <= 1e-10
        assert np.abs(x[lo:hi] - xo).max() <= 1e-10, (k, method, precision)


@pytest.mark.parametrize("tiling", [rp.RP_TILING_AUTO, rp.RP_TILING_OFF])
def test_matrix_paper_rule_jacobi_counts(tiling):
    ms, m = _batch()
    sys = _system(m)
    x, info, code = G.solve(sys, "jacobi", tol=1e-9, stop=rp.RP_STOP_DELTA, tiling=tiling)
    assert code == rp.binding.RP_OK, info
    for k, mk in enumerate(ms):
        red = oracle.matrix_system(mk.n, mk.rp, mk.col, mk.val, mk.rhs)
        xo, it, _, rc = oracle.jacobi(red, tol=1e-9, stop_mode=0)
        lo, hi = m.inst_off[k], m.inst_off[k + 1]
        assert abs(info[k]["iterations"] - it) <= 1, (k, info[k]["iterations"], it)
        assert np.abs(x[lo:hi] - xo).max() <= 1e-8


def test_matrix_not_dominant_and_bad_rows():
    m = cg.diag_dominant(200, density=0.05, seed=21)
    v = m.val.copy()
    rows = np.repeat(np.arange(m.n), np.diff(m.rp))
    diag = np.nonzero(rows == m.col)[0]
    v[diag[7]] *= 0.25  # row 7 no longer dominant
    bad = cg.Matrix(m.n, m.rp, m.col, v, m.rhs, m.inst_off)
    sys = _system(bad)
    with pytest.raises(rp.RpError) as e:
        G.solve(sys, "bicgstab", tol=1e-10, stop=rp.RP_STOP_CERTIFIED)
    assert e.value.code == rp.binding.RP_ERR_INVALID_ARG
    x, info, code = G.solve(sys, "bicgstab", tol=1e-12, stop=rp.RP_STOP_RESIDUAL)
    assert code == rp.binding.RP_OK
    A = np.zeros((m.n, m.n)); A[rows, m.col] = v
    assert np.abs(x - np.linalg.solve(A, m.rhs)).max() <= 1e-9
    # a row without its diagonal entry
    keep = np.ones(m.nnz, bool); keep[diag[11]] = False
    rp2 = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=m.n))]).astype(np.int32)
    nod = cg.Matrix(m.n, rp2, m.col[keep], m.val[keep], m.rhs, m.inst_off)
    with pytest.raises(rp.RpError) as e:
        _system(nod)
    assert e.value.code == rp.binding.RP_ERR_BAD_CHAIN and e.value.message.startswith("row 11:")
