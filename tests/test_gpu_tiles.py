"""Parity of the sparse kernels for every kind of on-chip window, and of the
row-chunk kernels (tiling off), with the oracle.

Instances whose padded undecided block fits a workgroup's LDS keep it whole;
larger ones get a band around each tile's rows when their entries lie near
the diagonal (model-checker-shaped chains), or no window at all when the
targets are spread uniformly.  FP64 windows hold 20,416 rows and FP32 windows
40,896, so the chains below exercise all three kinds in both precisions,
alone and mixed in one batch."""
import numpy as np
import pytest
import torch

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from tests import _gpu as G

pytestmark = pytest.mark.gpu

SEED = cg.SEED_BASE + 600


def _chain(kind):
    if kind == "band":
        return cg.program_graph(60_000, 0.01, 0.001, 64, 0.02, SEED)
    if kind == "nowindow":
        return cg.random_sparse(50_000, 1, 8, 0.01, 0.01, SEED + 1)
    return cg.concat([cg.random_sparse(3_000, 1, 8, 0.01, 0.01, SEED + 2),
                      cg.program_graph(45_000, 0.01, 0.001, 64, 0.02, SEED + 3),
                      cg.random_sparse(30_000, 1, 8, 0.01, 0.01, SEED + 4),
                      cg.random_sparse(500, 1, 4, 0.02, 0.02, SEED + 5),
                      cg.random_sparse(45_000, 1, 8, 0.01, 0.01, SEED + 6)])


_CACHE = {}


def _fixture(kind):
    """Chain, GPU system, classes and per-instance oracle references."""
    if kind not in _CACHE:
        c = _chain(kind)
        G.banner(f"tiles precompute {kind} K={c.num_instances} n={c.n}")
        sys, cls, _ = G.precompute(c)
        assert np.array_equal(cls, oracle.partition(c.n, c.rp, c.col, c.val, c.goal))
        refs = []
        for k in range(c.num_instances):
            ck = c.instance(k)
            refs.append(oracle.solve(ck.n, ck.rp, ck.col, ck.val, ck.goal, "bicgstab", tol=1e-12, stop_mode=1))
        _CACHE[kind] = (c, sys, cls, refs)
    return _CACHE[kind]


KINDS = ["band", "nowindow", "mixed"]
TILING = {"tiles": rp.RP_TILING_AUTO, "chunks": rp.RP_TILING_OFF}


def test_undecided_blocks_span_every_window_kind():
    """The chains really are larger than one LDS window where they should be."""
    sizes = {}
    for kind in KINDS:
        c, sys, cls, _ = _fixture(kind)
        sizes[kind] = [int(np.sum(cls[c.inst_off[k]:c.inst_off[k + 1]] == oracle.SQ))
                       for k in range(c.num_instances)]
    assert sizes["band"][0] > 40_896 and sizes["nowindow"][0] > 40_896
    m = sizes["mixed"]
    assert m[0] < 20_416 and 20_416 < m[2] < 40_896 and m[4] > 40_896


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("method", ["jacobi", "bicgstab"])
@pytest.mark.parametrize("tiling", list(TILING))
def test_paper_rule(kind, method, tiling):
    """Stop on the paper's rule: per-instance counts of the oracle's replay."""
    c, sys, cls, _ = _fixture(kind)
    G.banner(f"tiles delta {kind} {method} {tiling}")
    x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_DELTA, tiling=TILING[tiling])
    assert code == rp.binding.RP_OK, info
    slack = 1 if method == "jacobi" else 2
    bound = 1e-12 if method == "jacobi" else 1e-8
    for k in range(c.num_instances):
        ck = c.instance(k)
        o = oracle.solve(ck.n, ck.rp, ck.col, ck.val, ck.goal, method, tol=1e-10, stop_mode=0)
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        assert abs(info[k]["iterations"] - o.iters) <= slack, (k, info[k]["iterations"], o.iters)
        assert np.abs(x[lo:hi] - o.x).max() <= bound, k


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("method", ["jacobi", "bicgstab"])
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
@pytest.mark.parametrize("tiling", list(TILING))
def test_certified(kind, method, precision, tiling):
    c, sys, cls, refs = _fixture(kind)
    prec = rp.RP_FP64 if precision == "fp64" else rp.RP_FP32_REFINED
    G.banner(f"tiles certified {kind} {method} {precision} {tiling}")
    x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=prec,
                            tiling=TILING[tiling])
    assert code == rp.binding.RP_OK, info
    for k, ref in enumerate(refs):
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        assert np.abs(x[lo:hi] - ref.x).max() <= 1e-10, k
        assert info[k]["error_bound"] <= 1e-10 * (1 + 1e-12)


def _oracle_transposed_solve(rt, rhs):
    """Oracle solution of (I-A)^T lam = rhs to rounding level and its certified
    error bound; BiCGStab, or Jacobi where BiCGStab breaks down."""
    tbt = oracle.tbound(rt)
    lam, _, _, rc = oracle.bicgstab(rt, b=rhs, tol=1e-15, stop_mode=0, max_iter=5000)
    bound = tbt * oracle.residual(rt, rhs, lam)[1]
    if rc != 0 or bound > 1e-10:
        lam, _, _, _ = oracle.jacobi(rt, b=rhs, tol=1e-16, stop_mode=0, max_iter=200_000)
        bound = tbt * oracle.residual(rt, rhs, lam)[1]
    return lam, bound


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("method", [0, 1])
def test_adjoint(kind, method):
    """lambda of the transposed system (the tiles serve both directions).

    Both sides carry a certified bound: the library's (tol) and the oracle's
    (its ||(I-A)^{-T} 1|| bound times its FP64 residual), so they may differ
    by at most the sum.  ||(I-A)^{-T} 1|| reaches ~1.4e3 here, which puts the
    rounding floor of a certified bound near 1e-11: tol is 1e-10."""
    c, sys, cls, refs = _fixture(kind)
    G.banner(f"tiles adjoint {kind} method {method}")
    x, info, code = G.solve(sys, "bicgstab", tol=1e-12, stop=rp.RP_STOP_CERTIFIED)
    assert code == rp.binding.RP_OK
    seed = np.zeros(c.n)
    for k in range(c.num_instances):
        lo = c.inst_off[k]
        sq = np.nonzero(cls[lo:c.inst_off[k + 1]] == oracle.SQ)[0]
        seed[lo + sq[::97]] = 1.0
    tol = 1e-10
    lam, g, info, code = rp.rp_adjoint(G.ctx(), sys, torch.from_numpy(x).cuda(), torch.from_numpy(seed).cuda(),
                                       method, tol=tol, stop=rp.RP_STOP_CERTIFIED)
    assert code == rp.binding.RP_OK, info
    lam = lam.cpu().numpy()
    for k, ref in enumerate(refs):
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        sq = np.nonzero(ref.cls == oracle.SQ)[0]
        rt = oracle.transpose(ref.red)
        rhs = np.zeros(ref.red.nq)
        rhs[ref.red.map[sq]] = seed[lo:hi][sq]
        lam_o, bound_o = _oracle_transposed_solve(rt, rhs)
        assert bound_o <= 1e-10, (k, bound_o)
        want = np.zeros(hi - lo)
        want[sq] = lam_o[ref.red.map[sq]]
        assert np.abs(lam[lo:hi] - want).max() <= tol + bound_o, k
        assert info[k]["error_bound"] <= tol



@pytest.mark.parametrize("kind", KINDS)
def test_sliced_rows_paper_rule(kind):
    """Sliced rows (schedule 0) on every window kind: under the paper's rule
    the Jacobi iterates and counts are bit-identical to one lane per row (both
    sum a row in CSR order)."""
    c, sys, cls, refs = _fixture(kind)
    G.banner(f"tiles sliced delta {kind}")
    x0, i0, code0 = G.solve(sys, "jacobi", tol=1e-10, stop=rp.RP_STOP_DELTA, schedule=0)
    x1, i1, code1 = G.solve(sys, "jacobi", tol=1e-10, stop=rp.RP_STOP_DELTA, schedule=1)
    assert code0 == code1 == rp.binding.RP_OK
    assert np.array_equal(x0, x1)
    assert [i["iterations"] for i in i0] == [i["iterations"] for i in i1]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_sliced_rows_certified(kind, precision):
    """Both solvers on sliced rows within the certified tolerance of the
    oracle; in FP64 also the adjoint on the transposed slices, against the
    lane-group layout (both certified to 1e-10, so within 2e-10)."""
    c, sys, cls, refs = _fixture(kind)
    prec = rp.RP_FP64 if precision == "fp64" else rp.RP_FP32_REFINED
    G.banner(f"tiles sliced certified {kind} {precision}")
    xs = {}
    for method in ["jacobi", "bicgstab"]:
        x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=prec, schedule=0)
        assert code == rp.binding.RP_OK, (method, info)
        assert all(i["lanes"] == 0 for i in info)
        for k, ref in enumerate(refs):
            lo, hi = c.inst_off[k], c.inst_off[k + 1]
            assert np.abs(x[lo:hi] - ref.x).max() <= 1e-10, (method, k)
        xs[method] = x
    if precision == "fp64":
        seed = np.zeros(c.n)
        for k in range(c.num_instances):
            lo = c.inst_off[k]
            sq = np.nonzero(cls[lo:c.inst_off[k + 1]] == oracle.SQ)[0]
            seed[lo + sq[::89]] = 1.0
        xt = torch.from_numpy(xs["bicgstab"]).cuda()
        st = torch.from_numpy(seed).cuda()
        for method in (0, 1):
            lam0, g0, _, ca = rp.rp_adjoint(G.ctx(), sys, xt, st, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED,
                                            schedule=0)
            lam1, g1, _, cb = rp.rp_adjoint(G.ctx(), sys, xt, st, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED,
                                            schedule=4)
            assert ca == cb == rp.binding.RP_OK
            assert (lam0 - lam1).abs().max().item() <= 2e-10, method
