"""Tiled Jacobi batches replayed as one captured HIP graph (opts.graph = 1)
against one launch per sweep: the same iterates bit for bit and the same
iteration counts.  Each solve replays its graph many times, with the host's
status reads (and the refinement's own launches) between replays, so every
replay is checked through the final iterate of that solve."""
import numpy as np
import pytest

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from tests import _gpu as G

pytestmark = pytest.mark.gpu


def _chains():
    return [cg.concat([cg.random_sparse(3000 + 500 * i, 1, 16, 0.01, 0.01, cg.SEED_BASE + 40 + i)
                       for i in range(6)], name="batch of 6 random_sparse"),
            cg.random_sparse(60_000, 1, 8, 0.01, 0.01, seed=61),
            cg.program_graph(200_000, 0.01, 0.001, 64, 0.02, cg.SEED_BASE + 44)]


@pytest.fixture(scope="module")
def cases():
    out = []
    for c in _chains():
        refs = []
        for k in range(c.num_instances):
            ck = c.instance(k)
            refs.append(oracle.solve(ck.n, ck.rp, ck.col, ck.val, ck.goal, "bicgstab", tol=1e-12, stop_mode=1))
        out.append((c, refs))
    return out


@pytest.mark.parametrize("schedule", [0, 2])
@pytest.mark.parametrize("precision", [rp.RP_FP64, rp.RP_FP32_REFINED])
def test_graph_replays_equal_launches(cases, schedule, precision):
    for c, refs in cases:
        G.banner(f"graph jacobi schedule={schedule} prec={precision}: {c.name}")
        sys, _, _ = G.precompute(c)
        kw = dict(tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=precision, schedule=schedule)
        x0, i0, c0 = G.solve(sys, "jacobi", graph=0, **kw)
        x1, i1, c1 = G.solve(sys, "jacobi", graph=1, **kw)
        assert c0 == c1 == rp.binding.RP_OK
        assert [i["iterations"] for i in i0] == [i["iterations"] for i in i1], c.name
        assert np.array_equal(x0, x1), c.name
        for k, ref in enumerate(refs):
            lo, hi = int(c.inst_off[k]), int(c.inst_off[k + 1])
            assert np.abs(x1[lo:hi] - ref.x).max() <= 1e-10


def test_graph_with_iteration_cap_and_odd_chunk(cases):
    c, _ = cases[1]
    sys, _, _ = G.precompute(c)
    for extra in (dict(max_iter=1001), dict(chunk=31)):
        kw = dict(tol=1e-14, stop=rp.RP_STOP_RESIDUAL, precision=rp.RP_FP64, **extra)
        G.banner(f"graph jacobi with {extra}")
        x0, i0, c0 = G.solve(sys, "jacobi", graph=0, **kw)
        x1, i1, c1 = G.solve(sys, "jacobi", graph=1, **kw)
        assert c0 == c1
        assert [i["iterations"] for i in i0] == [i["iterations"] for i in i1]
        assert np.array_equal(x0, x1)
