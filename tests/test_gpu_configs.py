"""Parity at the full sizes of the five workloads.

Class arrays and reduced systems are compared bit for bit.  Where the oracle
cannot afford a full certified solve, the GPU answer is certified
independently on the CPU: the oracle's own bound on ||(I-A)^{-1} 1|| times
the FP64 residual of the GPU's x (computed by the oracle) bounds
max|x_gpu - x*| (I - A is a nonsingular M-matrix on S_?).  Chains whose
exact answer is known (every state reaches the goal with probability one)
are checked against it directly."""
import numpy as np
import pytest

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from tests import _gpu as G

pytestmark = pytest.mark.gpu

VARIANTS = [("jacobi", rp.RP_FP64), ("bicgstab", rp.RP_FP64), ("jacobi", rp.RP_FP32_REFINED),
            ("bicgstab", rp.RP_FP32_REFINED)]


def _check_system(c, sys, cls, prob0_only=False):
    want = oracle.partition(c.n, c.rp, c.col, c.val, c.goal, prob0_only)
    assert np.array_equal(cls, want)
    red = oracle.assemble(c.n, c.rp, c.col, c.val, cls)
    arp, acol, aval, d, b = [t.cpu().numpy() for t in rp.rp_system_export(G.ctx(), sys)]
    assert np.array_equal(arp, red.arp) and np.array_equal(acol, red.acol)
    assert np.array_equal(aval, red.aval) and np.array_equal(d, red.d) and np.array_equal(b, red.b)
    return red


def _certify(c, cls, red, x, tb, tol=1e-10):
    """max|x - x*| <= tb * ||b - (I-A) x||_inf, residual by the oracle."""
    assert np.all(x[cls == 0] == 0.0) and np.all(x[cls == 1] == 1.0)
    assert np.all((x >= 0.0) & (x <= 1.0 + 1e-12))
    idx = np.nonzero(cls == oracle.SQ)[0]
    xq = np.zeros(red.nq)
    xq[red.map[idx]] = x[idx]
    _, rn = oracle.residual(red, red.b, xq)
    assert tb * rn <= tol * 1.01, (tb, rn)
    return tb * rn


def _solve_all(sys, tol=1e-10, **kw):
    out = {}
    for method, prec in VARIANTS:
        G.banner(f"solve {method} precision={prec} {kw}")
        x, info, code = G.solve(sys, method, tol=tol, stop=rp.RP_STOP_CERTIFIED, precision=prec, **kw)
        assert code == rp.binding.RP_OK, (method, prec, info[:3])
        for i in info:
            assert i["error_bound"] <= tol * (1 + 1e-12)
        out[(method, prec)] = x
    return out


def test_config1_gamblers_ruin_all_variants():
    c = cg.CONFIGS[1]()
    G.banner("config 1")
    sys, cls, _ = G.precompute(c)
    red = _check_system(c, sys, cls)
    r = 11 / 9
    i = np.arange(c.n)
    xc = np.expm1(i * np.log(r)) / np.expm1((c.n - 1) * np.log(r))
    for key, x in _solve_all(sys).items():
        assert np.abs(x - xc).max() <= 1e-10, key


def test_config3_literal_and_prob0_only():
    """Dense random chain as specified: no state is trapped away from the
    goals, so S_? is empty and x = 1; with S_{=1} := GS the iterative methods
    must find x = 1 on the 8,151 other states."""
    c = cg.CONFIGS[3]()
    G.banner("config 3 literal")
    sys, cls, _ = G.precompute(c)
    red = _check_system(c, sys, cls)
    assert red.nq == 0
    x, info, code = G.solve(sys, "jacobi", tol=1e-10)
    assert code == rp.binding.RP_OK and np.all(x == 1.0)
    G.banner("config 3 prob0-only")
    sys, cls, _ = G.precompute(c, rp.RP_PROB0_ONLY)
    red = _check_system(c, sys, cls, prob0_only=True)
    assert red.nq == c.n - int(c.goal.sum())
    for key, x in _solve_all(sys).items():
        assert np.abs(x - 1.0).max() <= 1e-10, key


def test_config3_leaky():
    c = cg.dense_random(8192, 0.10, 0.005, 0.005, cg.SEED_BASE + 3)
    G.banner("config 3 leaky")
    sys, cls, _ = G.precompute(c)
    red = _check_system(c, sys, cls)
    tb = oracle.tbound(red)
    xs = _solve_all(sys)
    for key, x in xs.items():
        _certify(c, cls, red, x, tb)
    ref = xs[("bicgstab", rp.RP_FP64)]
    for key, x in xs.items():
        assert np.abs(x - ref).max() <= 2e-10


def test_config3_leaky_sliced_rows():
    """The dense chain (~820 entries per row, beyond the last sort key) forced
    onto sliced rows: every slice is as wide as its longest row."""
    c = cg.dense_random(8192, 0.10, 0.005, 0.005, cg.SEED_BASE + 3)
    G.banner("config 3 leaky, sliced rows")
    sys, cls, _ = G.precompute(c)
    red = oracle.assemble(c.n, c.rp, c.col, c.val, cls)
    tb = oracle.tbound(red)
    xs = _solve_all(sys, schedule=0)
    for key, x in xs.items():
        _certify(c, cls, red, x, tb)


def test_config4_program_graph():
    c = cg.CONFIGS[4]()
    G.banner(f"config 4 n={c.n}")
    sys, cls, _ = G.precompute(c)
    red = _check_system(c, sys, cls)
    tb = oracle.tbound(red)
    xs = _solve_all(sys)
    for key, x in xs.items():
        _certify(c, cls, red, x, tb)


@pytest.fixture(scope="module")
def config5():
    return cg.CONFIGS[5]()


def test_config5_batched_literal(config5):
    c = config5
    G.banner(f"config 5 literal K={c.num_instances} n={c.n}")
    sys, cls, _ = G.precompute(c)
    _check_system(c, sys, cls)
    xs = _solve_all(sys)
    # instances with a non-empty S_?: certify each against the oracle's bound
    for k in range(c.num_instances):
        lo, hi = int(c.inst_off[k]), int(c.inst_off[k + 1])
        if not np.any(cls[lo:hi] == oracle.SQ):
            for x in xs.values():
                assert np.array_equal(x[lo:hi], (cls[lo:hi] == oracle.S1).astype(float))
            continue
        ck = c.instance(k)
        red = oracle.assemble(ck.n, ck.rp, ck.col, ck.val, cls[lo:hi])
        tb = oracle.tbound(red)
        for x in xs.values():
            _certify(ck, cls[lo:hi], red, x[lo:hi], tb)


def test_config5_batched_prob0_only(config5):
    c = config5
    G.banner("config 5 prob0-only")
    sys, cls, _ = G.precompute(c, rp.RP_PROB0_ONLY)
    want = oracle.partition(c.n, c.rp, c.col, c.val, c.goal, True)
    assert np.array_equal(cls, want)
    # x = 1 wherever S_{=0} is empty in the instance (every state reaches GS)
    full = oracle.partition(c.n, c.rp, c.col, c.val, c.goal, False)
    for key, x in _solve_all(sys).items():
        for k in range(c.num_instances):
            lo, hi = int(c.inst_off[k]), int(c.inst_off[k + 1])
            if not np.any(full[lo:hi] == oracle.S0):
                assert np.abs(x[lo:hi] - 1.0).max() <= 1e-10, (key, k)


def test_config5_batched_leaky_sampled():
    """Also forced onto sliced rows: its slices (411 MB FP64, 274 MB FP32)
    exceed the size above which they are read with nontemporal loads."""
    c = cg.batched(256, 1_000, 200_000, 1, 8, 0.01, 0.01, cg.SEED_BASE + 5)
    G.banner(f"config 5 leaky n={c.n}")
    sys, cls, _ = G.precompute(c)
    want = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
    assert np.array_equal(cls, want)
    xs = _solve_all(sys)
    xs.update({("sliced",) + key: x for key, x in _solve_all(sys, schedule=0).items()})
    rng = np.random.Generator(np.random.PCG64(5))
    for k in rng.choice(c.num_instances, size=12, replace=False):
        lo, hi = int(c.inst_off[k]), int(c.inst_off[k + 1])
        ck = c.instance(int(k))
        red = oracle.assemble(ck.n, ck.rp, ck.col, ck.val, cls[lo:hi])
        tb = oracle.tbound(red)
        for x in xs.values():
            _certify(ck, cls[lo:hi], red, x[lo:hi], tb)


def test_bench_workload_sampled():
    """The benchmark's workload in the configuration bench.py times (64 chains
    of 20,000 states, default options: tiles, tuned row layout): every solve of
    a bench step certified; three sampled chains against the oracle's
    certified solutions (classes bit-exact); the FP32-refined BiCGStab adjoint
    and gradient of the bench's seed (first undecided state of each chain) on
    one sampled chain against the oracle's."""
    import torch
    import bench
    c = bench.make_workload("batch", 64)
    G.banner(f"bench workload K={c.num_instances} n={c.n}")
    sys, cls, _ = G.precompute(c)
    xs = _solve_all(sys)
    seed = np.zeros(c.n)
    for k in range(c.num_instances):
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        sq = np.nonzero(cls[lo:hi] == oracle.SQ)[0]
        if sq.size:
            seed[lo + sq[0]] = 1.0
    xb = xs[("bicgstab", rp.RP_FP64)]
    lam, g, info, code = rp.rp_adjoint(G.ctx(), sys, torch.from_numpy(xb).cuda(), torch.from_numpy(seed).cuda(), 1,
                                       tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=rp.RP_FP32_REFINED)
    assert code == rp.binding.RP_OK, info[:3]
    lam, g = lam.cpu().numpy(), g.cpu().numpy()
    for k in (0, 37, 63):
        ck = c.instance(k)
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        G.banner(f"bench workload oracle chain {k}")
        ref = oracle.solve(ck.n, ck.rp, ck.col, ck.val, ck.goal, "bicgstab", tol=1e-12, stop_mode=1)
        assert np.array_equal(cls[lo:hi], ref.cls)
        for key, x in xs.items():
            assert np.abs(x[lo:hi] - ref.x).max() <= 1e-10, (key, k)
        if k == 37:
            sq = np.nonzero(ref.cls == oracle.SQ)[0]
            lam_o, _, _, _ = oracle.adjoint(ref, seed[lo:hi], tol=1e-12)
            want = np.zeros(hi - lo)
            want[sq] = lam_o[ref.red.map[sq]]
            scale = max(1.0, np.abs(lam_o).max())
            assert np.abs(lam[lo:hi] - want).max() <= 1e-10 * scale
            g_o = oracle.gradient(ck.n, ck.rp, ck.col, ref.cls, ref.red, lam_o, ref.x)
            e0, e1 = c.rp[lo], c.rp[hi]
            assert np.abs(g[e0:e1] - g_o).max() <= 1e-10 * scale
