"""Column panels of the sliced rows: instances too large for one LDS window
whose columns have no band (uniformly random targets) stage their iterate in
LDS panel by panel, each lane keeping its rows' sums in registers.  Each lane
still adds its row's entries in column order, so the Jacobi iterates under
the paper's rule equal those of one lane per row (global gathers) bit for bit;
certified solves (both methods, both precisions; panels in FP64) and the
adjoint (panels of the transposed matrix) match the oracle."""
import numpy as np
import pytest
import torch

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from tests import _gpu as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    parts = [cg.random_sparse(60_000, 1, 8, 0.01, 0.01, seed=61), cg.random_sparse(5_000, 1, 8, 0.01, 0.01, seed=62),
             cg.random_sparse(150_000, 1, 8, 0.01, 0.01, seed=63)]
    c = cg.concat(parts, name="panels")
    G.banner(f"panels: n={c.n} nnz={c.nnz}")
    sys, cls, _ = G.precompute(c)
    refs = [oracle.solve(p.n, p.rp, p.col, p.val, p.goal, "bicgstab", tol=1e-12, stop_mode=1) for p in parts]
    return c, parts, sys, cls, refs


def test_paneled_jacobi_matches_one_lane_per_row(batch):
    c, parts, sys, cls, refs = batch
    x0, i0, code0 = G.solve(sys, "jacobi", tol=1e-10, stop=rp.RP_STOP_DELTA, schedule=0)
    x1, i1, code1 = G.solve(sys, "jacobi", tol=1e-10, stop=rp.RP_STOP_DELTA, schedule=1)
    assert code0 == code1 == rp.binding.RP_OK
    # the 150,000-state instance gets tiles of at most 4,096 rows, whose
    # panel copies would exceed the budget: it is swept without panels
    assert [i["panels"] for i in i0] == [3, 0, 0], i0
    assert all(i["lanes"] == 0 for i in i0) and all(i["lanes"] == 1 and i["panels"] == 0 for i in i1)
    assert [i["iterations"] for i in i0] == [i["iterations"] for i in i1]
    assert np.array_equal(x0, x1)


@pytest.mark.parametrize("method", ["jacobi", "bicgstab"])
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_paneled_certified_solves_match_oracle(batch, method, precision):
    c, parts, sys, cls, refs = batch
    prec = rp.RP_FP64 if precision == "fp64" else rp.RP_FP32_REFINED
    G.banner(f"panels certified {method} {precision}")
    x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=prec, schedule=0)
    assert code == rp.binding.RP_OK, info
    # FP32 tiles follow the CU share and do not fit the panel budget here
    want = [0, 0, 0] if precision == "fp32r" else [3, 0, 0]
    assert [i["panels"] for i in info] == want, info
    for k, ref in enumerate(refs):
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        assert np.array_equal(cls[lo:hi], ref.cls)
        assert np.abs(x[lo:hi] - ref.x).max() <= 1e-10, (k, method, precision)


@pytest.mark.parametrize("method", [0, 1])
def test_paneled_adjoint_matches_oracle(batch, method):
    c, parts, sys, cls, refs = batch
    seed = np.zeros(c.n)
    for k in range(c.num_instances):
        lo = c.inst_off[k]
        seed[lo + np.nonzero(refs[k].cls == oracle.SQ)[0][0]] = 1.0
    x = np.concatenate([r.x for r in refs])
    G.banner(f"panels adjoint method {method}")
    lam, g, info, code = rp.rp_adjoint(G.ctx(), sys, torch.from_numpy(x).cuda(), torch.from_numpy(seed).cuda(),
                                       method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=rp.RP_FP64,
                                       schedule=0)
    assert code == rp.binding.RP_OK, info
    assert info[0]["panels"] > 0 and info[2]["panels"] == 0, info
    lam, g = lam.cpu().numpy(), g.cpu().numpy()
    for k, ref in enumerate(refs):
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        sq = np.nonzero(ref.cls == oracle.SQ)[0]
        lam_o, _, _, rc = oracle.adjoint(ref, seed[lo:hi], tol=1e-12)
        want = np.zeros(hi - lo)
        want[sq] = lam_o[ref.red.map[sq]]
        scale = max(1.0, np.abs(lam_o).max())
        assert np.abs(lam[lo:hi] - want).max() <= 1e-10 * scale, k
        g_o = oracle.gradient(parts[k].n, parts[k].rp, parts[k].col, ref.cls, ref.red, lam_o, ref.x)
        assert np.abs(g[c.rp[lo]:c.rp[hi]] - g_o).max() <= 1.1e-10 * scale, k


def test_paneled_bicgstab_paper_rule(batch):
    """BiCGStab under the paper's rule on panels against one lane per row:
    same step counts up to the rounding order of the dot products."""
    c, parts, sys, cls, refs = batch
    x0, i0, code0 = G.solve(sys, "bicgstab", tol=1e-9, stop=rp.RP_STOP_DELTA, schedule=0)
    x1, i1, code1 = G.solve(sys, "bicgstab", tol=1e-9, stop=rp.RP_STOP_DELTA, schedule=1)
    assert code0 == code1 == rp.binding.RP_OK
    for a, b in zip(i0, i1):
        assert abs(a["iterations"] - b["iterations"]) <= 2
    assert np.abs(x0 - x1).max() <= 1e-7
