"""The tail of a tiled Jacobi solve: once only a few instances run, each small
enough for the resident kernel, the remaining sweeps run resident (one block
per instance, many sweeps per launch) with the row sums of the tiled layout
in use.  A batch whose large chain converges fast and whose small chains mix
slowly ends in such a tail.

Bars: under the certified stop the graph replays (which never switch) are
the reference, bit for bit in the iterates and equal in the sweep counts, on
sliced rows and on two lanes per row, in FP64 and in FP32 inside FP64
refinement, and the solution is within 1e-10 of the oracle's; under the
paper's rule the sweep counts are the oracle's within one and sliced rows
equal one lane per row bit for bit.  The profile counters show that the
tail ran resident."""
import numpy as np
import pytest

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from paper_1210_6412_amd import binding as B
from tests import _gpu as G

pytestmark = pytest.mark.gpu


def _batch():
    parts = [cg.random_sparse(60_000, 1, 8, 0.05, 0.05, seed=cg.SEED_BASE + 120)]
    parts += [cg.random_sparse(n, 1, 4, 0.002, 0.002, seed=cg.SEED_BASE + 121 + i)
              for i, n in enumerate((1500, 2200, 3000, 4100))]
    return cg.concat(parts, name="fast 60,000-state chain + four slow small chains")


@pytest.fixture(scope="module")
def case():
    c = _batch()
    sys, _, _ = G.precompute(c)
    refs = []
    for k in range(c.num_instances):
        ck = c.instance(k)
        refs.append((oracle.solve(ck.n, ck.rp, ck.col, ck.val, ck.goal, "bicgstab", tol=1e-12, stop_mode=1),
                     oracle.solve(ck.n, ck.rp, ck.col, ck.val, ck.goal, "jacobi", tol=1e-10, stop_mode=0)))
    return c, sys, refs


def _profiled(sys, **kw):
    B.rp_profile_enable(G.ctx(), True)
    x, info, code = G.solve(sys, "jacobi", **kw)
    prof = B.rp_profile_read(G.ctx())
    B.rp_profile_enable(G.ctx(), False)
    return x, info, code, prof


@pytest.mark.parametrize("schedule", [0, 2])
@pytest.mark.parametrize("precision", [rp.RP_FP64, rp.RP_FP32_REFINED])
def test_tail_equals_graph_replays(case, schedule, precision):
    c, sys, refs = case
    G.banner(f"tail certified schedule={schedule} prec={precision}: {c.name}")
    kw = dict(tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=precision, schedule=schedule)
    x1, i1, c1, p1 = _profiled(sys, graph=1, **kw)
    x0, i0, c0, p0 = _profiled(sys, graph=0, **kw)
    assert c0 == c1 == rp.binding.RP_OK
    tail = "jacobi_tail_fp64" if precision == rp.RP_FP64 else "jacobi_tail_fp32"
    assert p0[tail][0] > 0 and p1[tail][0] == 0, (p0[tail], p1[tail])
    assert [i["iterations"] for i in i0] == [i["iterations"] for i in i1]
    assert np.array_equal(x0, x1)
    for k, (ref, _) in enumerate(refs):
        lo, hi = int(c.inst_off[k]), int(c.inst_off[k + 1])
        assert np.abs(x0[lo:hi] - ref.x).max() <= 1e-10, k
        assert i0[k]["error_bound"] <= 1e-10


def test_tail_paper_rule(case):
    c, sys, refs = case
    G.banner(f"tail paper rule: {c.name}")
    xs, infos = [], []
    for schedule in (0, 1):
        x, info, code, prof = _profiled(sys, tol=1e-10, stop=rp.RP_STOP_DELTA, schedule=schedule)
        assert code == rp.binding.RP_OK, info
        assert prof["jacobi_tail_fp64"][0] > 0
        xs.append(x)
        infos.append([i["iterations"] for i in info])
    assert infos[0] == infos[1] and np.array_equal(xs[0], xs[1])
    for k, (_, o) in enumerate(refs):
        lo, hi = int(c.inst_off[k]), int(c.inst_off[k + 1])
        assert abs(infos[0][k] - o.iters) <= 1, (k, infos[0][k], o.iters)
        assert np.abs(xs[0][lo:hi] - o.x).max() <= 1e-12, k
    # the small chains are the tail: they need several times the large chain's sweeps
    assert min(infos[0][1:]) > 3 * infos[0][0], infos[0]
