"""Parity of the HIP library (through its C ABI) with the CPU oracle.

Bars: class arrays and the reduced system bit-exact; the paper's stopping
rules replayed with the same iteration count (+-1, rounding order differs);
certified solves within 1e-10 of the oracle's certified solution (itself
within 1e-12 of x*); gradients within 1e-10 relative."""
import numpy as np
import pytest
import torch

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from tests import _gpu as G

pytestmark = pytest.mark.gpu

SOLVERS = ["jacobi", "bicgstab"]


def _oracle_ref(c, prob0_only=False, tol=1e-12):
    return oracle.solve(c.n, c.rp, c.col, c.val, c.goal, "bicgstab", prob0_only=prob0_only, tol=tol,
                        stop_mode=1)


def _small_chains():
    out = [cg.worked_example(), cg.gamblers_ruin(60, 0.45)]
    for seed in range(10):
        rng = np.random.Generator(np.random.PCG64(7000 + seed))
        n = int(rng.integers(5, 400))
        out.append(cg.random_small(n, rng, dmax=int(rng.integers(1, 12)), goal_frac=0.05, sink_frac=0.05,
                                   zero_frac=0.1 if seed % 3 == 0 else 0.0, absorbing_goals=bool(seed % 2)))
    return out


# --------------------------------------------------------------------------
# precompute

@pytest.mark.parametrize("prob0_only", [False, True])
def test_partition_bit_exact_small(prob0_only):
    for c in _small_chains():
        G.banner(f"partition {c.name} n={c.n} prob0_only={prob0_only}")
        sys, cls, _ = G.precompute(c, rp.RP_PROB0_ONLY if prob0_only else 0)
        want = oracle.partition(c.n, c.rp, c.col, c.val, c.goal, prob0_only)
        assert np.array_equal(cls, want), c.name


def test_worked_example_system_matches_paper():
    c = cg.worked_example()
    sys, cls, _ = G.precompute(c)
    assert cls.tolist() == [2, 0, 2, 1]
    arp, acol, aval, d, b = [t.cpu().numpy() for t in rp.rp_system_export(G.ctx(), sys)]
    assert arp.tolist() == [0, 1, 2] and acol.tolist() == [1, 0] and aval.tolist() == [0.5, 0.4]
    assert d.tolist() == [1.0, 1.0] and b.tolist() == [0.5, 0.0]


@pytest.mark.parametrize("prob0_only", [False, True])
def test_reduced_system_bit_exact(prob0_only):
    chains = _small_chains() + [cg.CONFIGS[2]()]
    for c in chains:
        G.banner(f"export {c.name}")
        sys, cls, _ = G.precompute(c, rp.RP_PROB0_ONLY if prob0_only else 0)
        red = oracle.assemble(c.n, c.rp, c.col, c.val, cls)
        arp, acol, aval, d, b = [t.cpu().numpy() for t in rp.rp_system_export(G.ctx(), sys)]
        assert np.array_equal(arp, red.arp)
        assert np.array_equal(acol, red.acol)
        assert np.array_equal(aval, red.aval)
        assert np.array_equal(d, red.d)
        assert np.array_equal(b, red.b)


@pytest.mark.parametrize("cfg", [1, 2])
def test_partition_configs(cfg):
    c = cg.CONFIGS[cfg]()
    G.banner(f"partition config {cfg}")
    sys, cls, _ = G.precompute(c)
    assert np.array_equal(cls, oracle.partition(c.n, c.rp, c.col, c.val, c.goal))


# --------------------------------------------------------------------------
# the paper's stopping rules, replayed

@pytest.mark.parametrize("tiling", ["auto", "off"])
def test_jacobi_paper_rule_gamblers_ruin(tiling):
    """Stop at max|dx| < 1e-12: same sweep count as the oracle and within
    1e-10 of the closed form (resident kernel, then row chunks)."""
    c = cg.CONFIGS[1]()
    G.banner(f"jacobi delta gamblers ruin tiling={tiling}")
    sys, cls, _ = G.precompute(c)
    til = rp.RP_TILING_AUTO if tiling == "auto" else rp.RP_TILING_OFF
    x, info, code = G.solve(sys, "jacobi", tol=1e-12, stop=rp.RP_STOP_DELTA, tiling=til)
    assert code == rp.binding.RP_OK
    o = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, "jacobi", tol=1e-12, stop_mode=0)
    assert abs(info[0]["iterations"] - o.iters) <= 1
    r = 11 / 9
    i = np.arange(c.n)
    xc = np.expm1(i * np.log(r)) / np.expm1((c.n - 1) * np.log(r))
    assert np.abs(x - xc).max() <= 1e-10
    assert np.abs(x - o.x).max() <= 1e-13


@pytest.mark.parametrize("method", SOLVERS)
def test_paper_rule_config2(method):
    c = cg.CONFIGS[2]()
    G.banner(f"{method} delta config2")
    sys, cls, _ = G.precompute(c)
    x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_DELTA)
    assert code == rp.binding.RP_OK
    o = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, method, tol=1e-10, stop_mode=0)
    slack = 1 if method == "jacobi" else 2
    assert abs(info[0]["iterations"] - o.iters) <= slack
    bound = 1e-12 if method == "jacobi" else 1e-8
    assert np.abs(x - o.x).max() <= bound


# --------------------------------------------------------------------------
# certified solves: within 1e-10 of x*

@pytest.mark.parametrize("method", SOLVERS)
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
@pytest.mark.parametrize("tiling", ["auto", "off"])
def test_certified_small(method, precision, tiling):
    """Small chains: the resident Jacobi kernel and the small-tile BiCGStab
    (tiling auto), and the row-chunk kernels (tiling off)."""
    prec = rp.RP_FP64 if precision == "fp64" else rp.RP_FP32_REFINED
    til = rp.RP_TILING_AUTO if tiling == "auto" else rp.RP_TILING_OFF
    for c in _small_chains():
        G.banner(f"certified {method} {precision} {tiling} {c.name}")
        ref = _oracle_ref(c)
        sys, cls, _ = G.precompute(c)
        x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=prec, tiling=til)
        assert code == rp.binding.RP_OK, (c.name, info)
        err = np.abs(x - ref.x).max()
        assert err <= 1e-10, (c.name, err)
        assert info[0]["error_bound"] <= 1e-10 + 1e-15
        assert np.all(x[cls == 0] == 0) and np.all(x[cls == 1] == 1)


@pytest.mark.parametrize("method", SOLVERS)
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_certified_config2(method, precision):
    prec = rp.RP_FP64 if precision == "fp64" else rp.RP_FP32_REFINED
    c = cg.CONFIGS[2]()
    G.banner(f"certified {method} {precision} config2")
    ref = _oracle_ref(c)
    sys, cls, _ = G.precompute(c)
    x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=prec)
    assert code == rp.binding.RP_OK, info
    assert np.abs(x - ref.x).max() <= 1e-10
    assert info[0]["error_bound"] <= 1e-10


# --------------------------------------------------------------------------
# batched (block-diagonal) solves

@pytest.mark.parametrize("method", SOLVERS)
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_batched_matches_per_instance(method, precision):
    prec = rp.RP_FP64 if precision == "fp64" else rp.RP_FP32_REFINED
    rng = np.random.Generator(np.random.PCG64(99))
    parts = [cg.random_sparse(int(rng.integers(50, 3000)), 1, 8, 0.02, 0.02, seed=int(rng.integers(1 << 40)))
             for _ in range(7)]
    parts.insert(3, cg.random_sparse(40, 1, 3, 0.5, 0.0, seed=5, absorbing_goals=True))  # maybe empty S_?
    c = cg.concat(parts)
    G.banner(f"batched {method} {precision} K={c.num_instances}")
    sys, cls, _ = G.precompute(c)
    x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=prec)
    assert code == rp.binding.RP_OK, info
    for k in range(c.num_instances):
        ck = c.instance(k)
        ref = _oracle_ref(ck)
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        assert np.array_equal(cls[lo:hi], ref.cls)
        assert np.abs(x[lo:hi] - ref.x).max() <= 1e-10, k


@pytest.mark.parametrize("method", SOLVERS)
@pytest.mark.parametrize("tiling", ["auto", "off"])
def test_batched_paper_rule_per_instance_counts(method, tiling):
    """Small instances: the resident kernels (tiling auto) and the row chunks
    replay the paper's rule instance by instance."""
    parts = [cg.random_sparse(n, 1, 6, 0.02, 0.02, seed=100 + n) for n in (200, 900, 2500, 64)]
    c = cg.concat(parts)
    sys, cls, _ = G.precompute(c)
    til = rp.RP_TILING_AUTO if tiling == "auto" else rp.RP_TILING_OFF
    x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_DELTA, tiling=til)
    slack = 1 if method == "jacobi" else 2
    bound = 1e-12 if method == "jacobi" else 1e-8
    breakdowns = 0
    for k in range(c.num_instances):
        ck = c.instance(k)
        o = oracle.solve(ck.n, ck.rp, ck.col, ck.val, ck.goal, method, tol=1e-10, stop_mode=0)
        assert abs(info[k]["iterations"] - o.iters) <= slack, (k, info[k]["iterations"], o.iters)
        if o.rc == oracle.BREAKDOWN:  # the paper's BiCGStab breaks down here, so must the library
            assert info[k]["status"] == rp.binding.RP_ERR_BREAKDOWN, (k, info[k])
            breakdowns += 1
            continue
        assert info[k]["status"] == rp.binding.RP_OK, (k, info[k])
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        assert np.abs(x[lo:hi] - o.x).max() <= bound
    assert code == (rp.binding.RP_ERR_BREAKDOWN if breakdowns else rp.binding.RP_OK)


# --------------------------------------------------------------------------
# adjoint and gradient

@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_adjoint_gradient(method, precision):
    prec = rp.RP_FP64 if precision == "fp64" else rp.RP_FP32_REFINED
    for seed in range(4):
        rng = np.random.Generator(np.random.PCG64(8000 + seed))
        c = cg.random_small(int(rng.integers(30, 300)), rng, dmax=6, goal_frac=0.05, sink_frac=0.05)
        ref = _oracle_ref(c)
        sq = np.nonzero(ref.cls == oracle.SQ)[0]
        if sq.size == 0:
            continue
        s0 = int(sq[0])
        G.banner(f"adjoint method={method} {precision} seed={seed} n={c.n}")
        sys, cls, t = G.precompute(c)
        x, info, code = G.solve(sys, "jacobi", tol=1e-12, stop=rp.RP_STOP_CERTIFIED)
        assert code == rp.binding.RP_OK
        seed_v = np.zeros(c.n); seed_v[s0] = 1.0
        lam, g, info, code = rp.rp_adjoint(G.ctx(), sys, torch.from_numpy(x).cuda(),
                                           torch.from_numpy(seed_v).cuda(), method, tol=1e-12,
                                           stop=rp.RP_STOP_CERTIFIED, precision=prec)
        assert code == rp.binding.RP_OK, info
        lam_o, _, _, rc = oracle.adjoint(ref, seed_v, tol=1e-13)
        lam_full = np.zeros(c.n)
        lam_full[sq] = lam_o[ref.red.map[sq]]
        scale = max(1.0, np.abs(lam_o).max())
        assert np.abs(lam.cpu().numpy() - lam_full).max() <= 1e-10 * scale
        g_o = oracle.gradient(c.n, c.rp, c.col, ref.cls, ref.red, lam_o, ref.x)
        assert np.abs(g.cpu().numpy() - g_o).max() <= 1e-10 * scale


def test_autograd_function():
    c = cg.random_sparse(300, 1, 6, 0.03, 0.03, seed=77)
    t = G.dev(c)
    vals = t["val"].clone().requires_grad_(True)
    x = rp.reach_prob(vals, G.ctx(), t["row_ptr"], t["col"], t["goal"], None, 0, 0, tol=1e-12)
    ref = _oracle_ref(c)
    assert np.abs(x.detach().cpu().numpy() - ref.x).max() <= 1e-10
    sq = np.nonzero(ref.cls == oracle.SQ)[0]
    w = torch.zeros(c.n, dtype=torch.float64, device="cuda")
    w[torch.from_numpy(sq[:5]).cuda()] = 1.0
    (x * w).sum().backward()
    lam_o, _, _, _ = oracle.adjoint(ref, w.cpu().numpy(), tol=1e-13)
    g_o = oracle.gradient(c.n, c.rp, c.col, ref.cls, ref.red, lam_o, ref.x)
    assert np.abs(vals.grad.cpu().numpy() - g_o).max() <= 1e-9


# --------------------------------------------------------------------------
# error paths

@pytest.mark.parametrize("case", ["rowsum", "negative", "colrange", "unsorted", "instance"])
def test_bad_chain_reports_oracle_row(case):
    c = cg.concat([cg.random_sparse(30, 2, 4, 0.1, 0.1, seed=1), cg.random_sparse(20, 2, 4, 0.1, 0.1, seed=2)])
    rp_, col, val = c.rp.copy(), c.col.copy(), c.val.copy()
    row = 7
    k = int(rp_[row])
    if case == "rowsum":
        val[k] *= 0.9
    elif case == "negative":
        val[k] = -val[k]
    elif case == "colrange":
        col[k] = c.n + 3
    elif case == "unsorted":
        col[k], col[k + 1] = col[k + 1], col[k]
    elif case == "instance":
        col[k + 1:rp_[row + 1]] = np.arange(40, 40 + rp_[row + 1] - k - 1)
    bad = cg.Chain(c.n, rp_, col, val, c.goal, c.inst_off)
    want_row, _ = oracle.validate(c.n, rp_, col, val, c.inst_off)
    with pytest.raises(rp.RpError) as ei:
        G.precompute(bad)
    assert ei.value.code == rp.binding.RP_ERR_BAD_CHAIN
    assert ei.value.message.startswith(f"row {want_row}:")


def test_not_converged_status():
    c = cg.CONFIGS[2]()
    sys, cls, _ = G.precompute(c)
    x, info, code = G.solve(sys, "jacobi", tol=1e-10, stop=rp.RP_STOP_DELTA, max_iter=5)
    assert code == rp.binding.RP_ERR_NOT_CONVERGED
    assert info[0]["iterations"] == 5
    o = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, "jacobi", tol=1e-10, stop_mode=0, max_iter=5)
    assert np.abs(x - o.x).max() <= 1e-14


@pytest.mark.parametrize("max_iter", [1, 4, 5, 6, 13, 45])
def test_iteration_cap_at_batch_boundaries(max_iter):
    """Caps that end inside a batch, on its last iteration, and inside the
    iterations queued ahead of the next batch's check: the sweep and step
    counts equal the cap and the iterates equal the oracle's after that many
    iterations (Jacobi on tiles and on sliced rows; BiCGStab up to its
    rounding)."""
    c = cg.concat([cg.CONFIGS[2](), _random_chain(5)])
    sys, cls, _ = G.precompute(c)
    for sched in (0, 4):
        x, info, code = G.solve(sys, "jacobi", tol=0.0, stop=rp.RP_STOP_DELTA, max_iter=max_iter, schedule=sched)
        assert code == rp.binding.RP_ERR_NOT_CONVERGED
        for k in range(c.num_instances):
            lo, hi = c.inst_off[k], c.inst_off[k + 1]
            if not np.any(cls[lo:hi] == oracle.SQ):
                continue
            assert info[k]["iterations"] == max_iter, (sched, k, info[k])
            ck = c.instance(k)
            o = oracle.solve(ck.n, ck.rp, ck.col, ck.val, ck.goal, "jacobi", tol=0.0, stop_mode=0, max_iter=max_iter)
            lo, hi = c.inst_off[k], c.inst_off[k + 1]
            assert np.abs(x[lo:hi] - o.x).max() <= 1e-14, (sched, k)
    x, info, code = G.solve(sys, "bicgstab", tol=0.0, stop=rp.RP_STOP_DELTA, max_iter=max_iter)
    assert code in (rp.binding.RP_ERR_NOT_CONVERGED, rp.binding.RP_ERR_BREAKDOWN)
    for k in range(c.num_instances):
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        if info[k]["status"] == rp.binding.RP_ERR_BREAKDOWN or not np.any(cls[lo:hi] == oracle.SQ):
            continue
        assert info[k]["iterations"] == max_iter, (k, info[k])


def test_empty_undecided_set():
    """Every state decided by the searches (a chain of absorbing states):
    the solvers and the adjoint return at once with x = 1 on S_{=1}, 0 on S_{=0}."""
    ch = cg.from_dense(np.eye(5), goal=[1, 3])
    sys, cls, t = G.precompute(ch)
    assert not np.any(cls == oracle.SQ)
    want = (cls == oracle.S1).astype(float)
    for method in ("jacobi", "bicgstab"):
        for prec in (rp.RP_FP64, rp.RP_FP32_REFINED):
            for stop in (rp.RP_STOP_DELTA, rp.RP_STOP_CERTIFIED):
                if stop == rp.RP_STOP_DELTA and prec != rp.RP_FP64:
                    continue
                x, info, code = G.solve(sys, method, tol=1e-10, precision=prec, stop=stop)
                assert code == rp.binding.RP_OK
                assert np.array_equal(x, want)
    x = torch.from_numpy(want).cuda()
    lam, g, info, code = rp.rp_adjoint(G.ctx(), sys, x, torch.ones(ch.n, dtype=torch.float64, device="cuda"), 0)
    assert code == rp.binding.RP_OK
    assert np.all(lam.cpu().numpy() == 0) and np.all(g.cpu().numpy() == 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_unreachable_tolerance_stops_at_rounding_floor(precision):
    """A certified tolerance below what FP64 residuals can show ends as not
    converged after a few non-improving refinement steps, not after
    max_refine, with x still at rounding level."""
    prec = rp.RP_FP64 if precision == "fp64" else rp.RP_FP32_REFINED
    c = cg.random_sparse(3000, 1, 8, 0.02, 0.02, seed=4242)
    sys, cls, _ = G.precompute(c)
    ref = _oracle_ref(c)
    x, info, code = G.solve(sys, "bicgstab", tol=1e-18, stop=rp.RP_STOP_CERTIFIED, precision=prec, max_refine=60)
    assert code == rp.binding.RP_ERR_NOT_CONVERGED
    assert info[0]["refinements"] < 30
    assert np.abs(x - ref.x).max() <= 1e-12


@pytest.mark.parametrize("method", SOLVERS)
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_iteration_budget_across_refinements(method, precision):
    """max_iter caps the inner iterations summed over refinement steps."""
    prec = rp.RP_FP64 if precision == "fp64" else rp.RP_FP32_REFINED
    c = cg.concat([cg.random_sparse(n, 1, 8, 0.02, 0.02, seed=300 + n) for n in (700, 2500)])
    sys, cls, _ = G.precompute(c)
    cap = 7 if method == "bicgstab" else 40
    x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=prec, max_iter=cap)
    assert code == rp.binding.RP_ERR_NOT_CONVERGED
    for i in info:
        assert 0 < i["iterations"] <= cap
        assert i["status"] == rp.binding.RP_ERR_NOT_CONVERGED


def test_adjoint_bitwise_reproducible():
    """The transposed matrix is built by a stable sort by column (each column's
    entries in source-row order), so the adjoint of two independently built
    systems agrees bit for bit."""
    c = cg.concat([cg.random_sparse(n, 1, 12, 0.02, 0.02, seed=900 + n) for n in (4000, 9000)])
    lams = []
    for _ in range(2):
        sys, cls, _ = G.precompute(c)
        x, info, code = G.solve(sys, "bicgstab", tol=1e-12)
        assert code == rp.binding.RP_OK
        seed = np.zeros(c.n)
        seed[np.nonzero(cls == oracle.SQ)[0][::50]] = 1.0
        lam, g, info, code = rp.rp_adjoint(G.ctx(), sys, torch.from_numpy(x).cuda(), torch.from_numpy(seed).cuda(),
                                           0, tol=1e-10)
        assert code == rp.binding.RP_OK
        lams.append((lam.cpu().numpy(), g.cpu().numpy()))
    assert np.array_equal(lams[0][0], lams[1][0]) and np.array_equal(lams[0][1], lams[1][1])


def _random_chain(seed):
    rng = np.random.Generator(np.random.PCG64(31000 + seed))
    n = int(np.exp(rng.uniform(np.log(5), np.log(6000))))
    return cg.random_small(n, rng, dmax=int(rng.integers(1, 20)), goal_frac=float(rng.uniform(0.01, 0.2)),
                           sink_frac=float(rng.uniform(0.0, 0.1)), zero_frac=0.1 if seed % 4 == 0 else 0.0,
                           absorbing_goals=bool(seed % 3 == 0), self_loops=bool(seed % 5 != 0))


@pytest.mark.parametrize("method", SOLVERS)
@pytest.mark.parametrize("precision", ["fp64", "fp32r"])
def test_random_chains_certified_batch(method, precision):
    """Forty random chains (5..6,000 states, degrees 1..20, stored zeros,
    absorbing or live goal rows, with and without self-loops) packed in one
    batch: every instance within 1e-10 of the oracle's certified solution and
    its partition bit-exact."""
    prec = rp.RP_FP64 if precision == "fp64" else rp.RP_FP32_REFINED
    parts = [_random_chain(seed) for seed in range(40)]
    c = cg.concat(parts)
    G.banner(f"random batch {method} {precision} K={c.num_instances} n={c.n}")
    sys, cls, _ = G.precompute(c)
    x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=prec)
    assert code == rp.binding.RP_OK, [i for i in info if i["status"]][:3]
    for k, ck in enumerate(parts):
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        ref = _oracle_ref(ck)
        assert np.array_equal(cls[lo:hi], ref.cls), k
        assert np.abs(x[lo:hi] - ref.x).max() <= 1e-10, (k, ck.n)


@pytest.mark.parametrize("lanes", [1, 2, 8, 32])
def test_lanes_per_row_override(lanes):
    """opts.schedule (lanes per row) changes the summation order only."""
    for c in (cg.CONFIGS[2](), _random_chain(7)):
        G.banner(f"schedule {lanes} {c.name}")
        ref = _oracle_ref(c)
        sys, cls, _ = G.precompute(c)
        for method in SOLVERS:
            x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, schedule=lanes)
            assert code == rp.binding.RP_OK, (method, info[0])
            assert np.abs(x - ref.x).max() <= 1e-10, (method, lanes)


def test_tuned_lanes_reported_and_cached():
    """schedule -1 times the sliced rows and the lane counts once per system
    shape on the context; a second system of the same shape reuses the choice
    (0 = sliced rows)."""
    c = cg.CONFIGS[2]()
    lanes = []
    for _ in range(2):
        sys, cls, _ = G.precompute(c)
        x, info, code = G.solve(sys, "jacobi", tol=1e-10)
        assert code == rp.binding.RP_OK
        lanes.append(info[0]["lanes"])
    assert lanes[0] == lanes[1] and lanes[0] in (0, 1, 2, 4, 8, 16, 32, 64)
    x, info, code = G.solve(sys, "jacobi", tol=1e-10, schedule=16)
    assert code == rp.binding.RP_OK and info[0]["lanes"] == 16




def test_sliced_rows_match_one_lane_per_row():
    """Sliced rows (schedule 0) and one lane per row (schedule 1) both sum each
    row in CSR order, so under the paper's rule (FP64 sweeps only) the Jacobi
    iterates and counts agree bit for bit.  Certified solves on sliced rows
    (both solvers, both precisions) match the oracle; their refinement
    residuals use the lane-group kernels, so they are compared to the oracle
    only."""
    for c in (cg.CONFIGS[2](), _random_chain(11)):
        G.banner(f"sliced vs one lane {c.name}")
        ref = _oracle_ref(c)
        sys, cls, _ = G.precompute(c)
        x0, i0, code0 = G.solve(sys, "jacobi", tol=1e-10, stop=rp.RP_STOP_DELTA, schedule=0)
        x1, i1, code1 = G.solve(sys, "jacobi", tol=1e-10, stop=rp.RP_STOP_DELTA, schedule=1)
        assert code0 == code1 == rp.binding.RP_OK
        assert all(i["lanes"] == 0 for i in i0) and all(i["lanes"] == 1 for i in i1)
        assert np.array_equal(x0, x1), c.name
        assert [i["iterations"] for i in i0] == [i["iterations"] for i in i1]
        for prec in (rp.RP_FP64, rp.RP_FP32_REFINED):
            for method in SOLVERS:
                x, info, code = G.solve(sys, method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=prec,
                                        schedule=0)
                assert code == rp.binding.RP_OK, (method, prec, info[0])
                assert np.abs(x - ref.x).max() <= 1e-10, (method, prec)


# --------------------------------------------------------------------------
# stagnation of the paper's rule, and the weighted Jacobi refinement margin

@pytest.mark.parametrize("method", SOLVERS)
@pytest.mark.parametrize("where", ["resident", "tiles", "chunks"])
def test_paper_rule_unreachable_tolerance_ends_early(method, where):
    """Under the paper's rule a tolerance of 0 is never met by Jacobi (strict
    max|dx| < 0) and at most by chance by BiCGStab (every s_i exactly 0): the
    stagnation watch ends the solve once the best measure has not halved for
    max(65,536, the iterations it took to reach it) iterations, far below the
    10^7 default cap (max_iter is bounded here too).  x stays at rounding
    level."""
    n = {"resident": 2000, "tiles": 60000, "chunks": 6000}[where]
    c = cg.random_sparse(n, 1, 8, 0.02, 0.02, seed=9100 + n)
    sys, cls, _ = G.precompute(c)
    ref = _oracle_ref(c)
    kw = dict(tiling=rp.RP_TILING_OFF) if where == "chunks" else {}
    G.banner(f"stagnation {method} {where} n={n}")
    x, info, code = G.solve(sys, method, tol=0.0, stop=rp.RP_STOP_DELTA, max_iter=400_000, **kw)
    it = info[0]["iterations"]
    if method == "jacobi":
        assert code == rp.binding.RP_ERR_NOT_CONVERGED, info
        assert "stopped falling" in rp.rp_last_error(G.ctx())
        assert 65_536 < it <= 3 * 65_536, it
        assert np.abs(x - ref.x).max() <= 1e-12
    else:
        assert code in (rp.binding.RP_OK, rp.binding.RP_ERR_NOT_CONVERGED, rp.binding.RP_ERR_BREAKDOWN,
                        rp.binding.RP_ERR_NONFINITE), info
        assert it <= 3 * 65_536, it
        if code == rp.binding.RP_ERR_NOT_CONVERGED:
            assert "stopped falling" in rp.rp_last_error(G.ctx())


def _self_loop_chain(n, seed):
    """Half of the states keep most of their mass on a self-loop (P(s,s) in
    [0.9, 0.99]) and pass the rest to one or two states; the other half have
    one or two successors and no self-loop.  1% goal and 1% absorbing sink
    states.  Rows of heavy self-loops next to rows of low degree make the
    residual of a Jacobi iterate larger than the previous iterate's in the
    infinity norm, the case where handing on the last iterate instead of the
    measured one missed the refinement target."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows, cols, vals = [], [], []
    perm = rng.permutation(n)
    goals, sinks = set(perm[: n // 100]), set(perm[n // 100: n // 50])
    for s in range(n):
        if s in goals or s in sinks:
            rows.append(s); cols.append(s); vals.append(1.0)
            continue
        deg = int(rng.integers(1, 3))
        tg = rng.choice(n - 1, size=deg, replace=False)
        tg[tg >= s] += 1
        w = rng.random(deg) + 0.05
        if rng.random() < 0.5:
            loop = rng.uniform(0.9, 0.99)
            w = w / w.sum() * (1.0 - loop)
            ent = sorted([(s, loop)] + list(zip(tg.tolist(), w.tolist())))
        else:
            ent = sorted(zip(tg.tolist(), (w / w.sum()).tolist()))
        for t, v in ent:
            rows.append(s); cols.append(t); vals.append(v)
    rp_ = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp_, np.asarray(rows) + 1, 1)
    goal = np.zeros(n, dtype=np.uint8)
    goal[list(goals)] = 1
    return cg.Chain(n, np.cumsum(rp_).astype(np.int32), np.asarray(cols, dtype=np.int32),
                    np.asarray(vals, dtype=np.float64), goal, np.array([0, n], dtype=np.int64), "self-loops")


@pytest.mark.parametrize("where", ["resident", "tiles", "chunks"])
def test_fp64_jacobi_refinement_with_heavy_self_loops(where):
    n = {"resident": 3000, "tiles": 50000, "chunks": 8000}[where]
    c = _self_loop_chain(n, 4400 + n)
    sys, cls, _ = G.precompute(c)
    ref = _oracle_ref(c)
    kw = dict(tiling=rp.RP_TILING_OFF) if where == "chunks" else {}
    G.banner(f"self-loop chain {where} n={n}")
    for sched in ((-1,) if where == "chunks" else (-1, 0, 2)):
        x, info, code = G.solve(sys, "jacobi", tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=rp.RP_FP64,
                                schedule=sched, **kw)
        assert code == rp.binding.RP_OK, (sched, info)
        assert info[0]["error_bound"] <= 1e-10
        assert np.abs(x - ref.x).max() <= 1e-10


# --------------------------------------------------------------------------
# deep searches (more levels than one launch per level could afford)

def _ladder(n):
    """State i moves to i+1 w.p. 1/2 and to the sink 0 w.p. 1/2 (0 and n-1
    absorbing, goal n-1): a one-way path of depth n whose states have two
    successors, so no two of its states are merged."""
    rows, cols, vals = [0], [0], [1.0]
    for i in range(1, n - 1):
        rows += [i, i]; cols += [0, i + 1]; vals += [0.5, 0.5]
    rows.append(n - 1); cols.append(n - 1); vals.append(1.0)
    rp_ = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp_, np.asarray(rows) + 1, 1)
    goal = np.zeros(n, dtype=np.uint8)
    goal[n - 1] = 1
    return cg.Chain(n, np.cumsum(rp_).astype(np.int32), np.asarray(cols, dtype=np.int32),
                    np.asarray(vals, dtype=np.float64), goal, np.array([0, n], dtype=np.int64), "ladder")


@pytest.mark.parametrize("prob0_only", [False, True])
def test_deep_search_million_state_birth_death(prob0_only):
    """Gambler's ruin with 10^6 states: both searches walk a path of ~10^6
    levels; merging the states joined by mutual edges leaves three classes,
    so the precompute takes a few dozen launches.  Classes bit-exact."""
    import time
    c = cg.gamblers_ruin(1_000_000, 0.45)
    want = oracle.partition(c.n, c.rp, c.col, c.val, c.goal, prob0_only)
    flags = rp.RP_PROB0_ONLY if prob0_only else 0
    G.precompute(c, flags)[0].close()  # warm (module load, allocation)
    t0 = time.perf_counter()
    sys, cls, _ = G.precompute(c, flags)
    dt = time.perf_counter() - t0
    G.banner(f"1e6-state birth-death precompute: {1000 * dt:.1f} ms")
    assert np.array_equal(cls, want)
    assert dt < 1.0, dt


def test_deep_search_mixed_batch():
    """A batch of a birth-death chain, a random chain and a one-way ladder
    (no merges on the ladder: its 40,000 levels still take pull steps)."""
    c = cg.concat([cg.gamblers_ruin(50_000, 0.45), cg.random_sparse(50_000, 1, 8, 0.01, 0.01, seed=81),
                   _ladder(40_000)])
    for prob0_only in (False, True):
        want = oracle.partition(c.n, c.rp, c.col, c.val, c.goal, prob0_only)
        sys, cls, _ = G.precompute(c, rp.RP_PROB0_ONLY if prob0_only else 0)
        assert np.array_equal(cls, want), prob0_only
