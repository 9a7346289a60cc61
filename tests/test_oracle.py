"""Pins for the CPU oracle: each check ties the oracle to something other than
itself -- values printed in the paper, closed forms, brute force on tiny
chains, LAPACK, Monte Carlo and invariants of the method."""
import json
import os

import numpy as np
import pytest

import chaingen as cg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# printed examples

def test_csr_example_section4():
    g = _load("csr_example.json")
    c = cg.from_dense(g["matrix"])
    assert c.rp.tolist() == g["rstart"]
    assert c.col.tolist() == g["col"]
    assert c.val.tolist() == g["nonzero"]


def test_worked_example_partition_and_system():
    g = _load("worked_example.json")
    c = cg.from_dense(g["P"], goal=g["goal"])
    assert oracle.validate(c.n, c.rp, c.col, c.val) == (-1, 0)
    cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
    pr = g["printed"]
    assert np.nonzero(cls == oracle.S0)[0].tolist() == pr["S_eq0"]
    assert np.nonzero(cls == oracle.S1)[0].tolist() == pr["S_eq1"]
    assert np.nonzero(cls == oracle.SQ)[0].tolist() == pr["S_q"]
    red = oracle.assemble(c.n, c.rp, c.col, c.val, cls)
    # A includes the diagonal of P restricted to S_?; I - A = dense_m
    a = np.eye(red.nq) - oracle.dense_m(red)
    assert np.array_equal(a, np.array(pr["A"]))
    assert red.b.tolist() == pr["b"]
    assert red.b[0] == pr["Pr_Cyl_03"]


@pytest.mark.parametrize("method", ["jacobi", "bicgstab"])
@pytest.mark.parametrize("stop_mode", [0, 1])
def test_worked_example_solution(method, stop_mode):
    g = _load("worked_example.json")
    c = cg.from_dense(g["P"], goal=g["goal"])
    s = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, method, tol=1e-14, stop_mode=stop_mode)
    assert s.rc == oracle.OK
    np.testing.assert_allclose(s.x, g["derived"]["x"], atol=1e-13, rtol=0)
    # dense elimination of the 2x2 system
    xd = oracle.dense_solve(oracle.dense_m(s.red), s.red.b)
    np.testing.assert_allclose(xd, [0.625, 0.25], atol=1e-15, rtol=0)


# --------------------------------------------------------------------------
# gambler's ruin: closed forms for x and for the expected time in S_?

def _gr_closed(n=1000, p=0.45):
    q = 1 - p
    r = q / p
    i = np.arange(n)
    x = np.expm1(i * np.log(r)) / np.expm1((n - 1) * np.log(r))
    N = n - 1
    ii = np.arange(1, n - 1)
    t = ii / (q - p) - (N / (q - p)) * np.expm1(ii * np.log(r)) / np.expm1(N * np.log(r))
    return x, t


def test_gamblers_ruin_partition():
    c = cg.gamblers_ruin()
    cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
    assert cls[0] == oracle.S0 and cls[-1] == oracle.S1
    assert np.all(cls[1:-1] == oracle.SQ)


def test_gamblers_ruin_jacobi_paper_rule():
    """Stopping at max|dx| < 1e-12 (the paper's Jacobi rule) lands within
    1e-10 of the closed form."""
    c = cg.gamblers_ruin()
    xc, _ = _gr_closed()
    s = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, "jacobi", tol=1e-12, stop_mode=0)
    assert s.rc == oracle.OK
    assert np.abs(s.x - xc).max() <= 1e-10


@pytest.mark.parametrize("method", ["jacobi", "bicgstab"])
def test_gamblers_ruin_certified(method):
    c = cg.gamblers_ruin()
    xc, _ = _gr_closed()
    s = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, method, tol=1e-12, stop_mode=1)
    assert s.rc == oracle.OK
    assert np.abs(s.x - xc).max() <= 1e-12


def test_gamblers_ruin_dense_and_tbound():
    c = cg.gamblers_ruin()
    xc, tc = _gr_closed()
    cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
    red = oracle.assemble(c.n, c.rp, c.col, c.val, cls)
    m = oracle.dense_m(red)
    xd = oracle.dense_solve(m, red.b)
    assert np.abs(xd - xc[1:-1]).max() <= 1e-12
    td = oracle.dense_solve(m, np.ones(red.nq))
    assert np.abs(td - tc).max() <= 1e-9 * tc.max()
    tb = oracle.tbound(red)
    assert tc.max() <= tb <= tc.max() * 1.002


# --------------------------------------------------------------------------
# partition: brute-force transitive closure on tiny chains

def _closure(adj):
    n = adj.shape[0]
    r = adj.copy() | np.eye(n, dtype=bool)
    for k in range(n):
        r = r | (r[:, [k]] & r[[k], :])
    return r


def _brute_partition(c, prob0_only):
    p = c.dense()
    adj = p > 0
    goal = c.goal.astype(bool)
    reach = _closure(adj)
    s0 = ~(reach[:, goal].any(axis=1))
    if prob0_only:
        s1 = goal.copy()
    else:
        adj2 = adj.copy()
        adj2[goal, :] = False          # goal states are absorbing for "eventually GS"
        reach2 = _closure(adj2)
        s1 = ~(reach2[:, s0].any(axis=1))
    cls = np.full(c.n, 2, dtype=np.uint8)
    cls[s1] = 1
    cls[s0] = 0
    return cls


@pytest.mark.parametrize("seed", range(40))
@pytest.mark.parametrize("prob0_only", [False, True])
def test_partition_matches_transitive_closure(seed, prob0_only):
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    n = int(rng.integers(2, 40))
    c = cg.random_small(n, rng, dmax=int(rng.integers(1, 5)), goal_frac=rng.uniform(0, 0.3),
                        sink_frac=rng.uniform(0, 0.3), zero_frac=0.2 if seed % 3 == 0 else 0.0,
                        absorbing_goals=bool(seed % 2))
    cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal, prob0_only)
    assert np.array_equal(cls, _brute_partition(c, prob0_only))


@pytest.mark.parametrize("seed", range(10))
def test_partition_probability_semantics(seed):
    """S_{=0} states never reach GS; S_{=1} states reach it with probability
    one (the probability of having avoided GS for k steps decays to 0);
    S_? states reach it with a probability strictly between 0 and 1."""
    rng = np.random.Generator(np.random.PCG64(77 + seed))
    c = cg.random_small(10, rng, dmax=3, goal_frac=0.2, sink_frac=0.2)
    cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
    p = c.dense()
    goal = c.goal.astype(bool)
    # hit[s] = Pr(reach GS within k steps): value iteration from below
    hit = goal.astype(float)
    for _ in range(20000):
        hit = np.where(goal, 1.0, p @ hit)
    assert np.all(hit[cls == 0] == 0.0)
    assert np.all(hit[cls == 1] > 1 - 1e-9)
    assert np.all((hit[cls == 2] > 0) & (hit[cls == 2] < 1 - 1e-6))


# --------------------------------------------------------------------------
# solvers against LAPACK and against the defining equation on the full chain

def _chains_small():
    out = []
    for seed in range(12):
        rng = np.random.Generator(np.random.PCG64(500 + seed))
        n = int(rng.integers(20, 200))
        out.append(cg.random_small(n, rng, dmax=int(rng.integers(2, 9)), goal_frac=0.05,
                                   sink_frac=0.05, zero_frac=0.1 if seed % 4 == 0 else 0.0))
    return out


@pytest.mark.parametrize("idx", range(12))
def test_dense_elimination_matches_lapack(idx):
    c = _chains_small()[idx]
    cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
    red = oracle.assemble(c.n, c.rp, c.col, c.val, cls)
    if red.nq == 0:
        pytest.skip("empty S_?")
    m = oracle.dense_m(red)
    x = oracle.dense_solve(m, red.b)
    xl = np.linalg.solve(m, red.b)
    assert np.abs(x - xl).max() <= 1e-13


@pytest.mark.parametrize("idx", range(12))
@pytest.mark.parametrize("method", ["jacobi", "bicgstab"])
def test_certified_solution_satisfies_full_chain_equation(idx, method):
    """x solves x_s = sum_s' P(s,s') x_s' on S_? with x = 1 on S_{=1} and 0
    on S_{=0} (Section 2.3), computed from the original dense P, and agrees
    with LAPACK on the reduced system."""
    c = _chains_small()[idx]
    s = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, method, tol=1e-12, stop_mode=1)
    assert s.rc == oracle.OK
    p = c.dense()
    sq = s.cls == oracle.SQ
    res = s.x - p @ s.x
    # certified: tbound*||r|| <= 1e-12 with tbound >= 1, plus rounding
    assert np.abs(res[sq]).max(initial=0) <= 1.5e-12
    assert np.all(s.x[s.cls == oracle.S1] == 1.0) and np.all(s.x[s.cls == oracle.S0] == 0.0)
    assert np.all((s.x >= 0) & (s.x <= 1))
    if s.red.nq:
        xl = np.linalg.solve(np.eye(s.red.nq) - (p[np.ix_(sq, sq)]),
                             p[np.ix_(sq, s.cls == oracle.S1)].sum(axis=1))
        assert np.abs(s.xq - xl).max() <= 1e-12


@pytest.mark.parametrize("idx", range(12))
def test_prob0_only_gives_same_solution(idx):
    c = _chains_small()[idx]
    a = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, "bicgstab", tol=1e-12, stop_mode=1)
    b = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, "bicgstab", prob0_only=True, tol=1e-12,
                     stop_mode=1)
    assert np.abs(a.x - b.x).max() <= 2e-12


def test_jacobi_monotone_from_zero():
    """Jacobi from x = 0 increases monotonically towards x* (non-negative
    iteration matrix, b >= 0)."""
    c = cg.random_sparse(3000, 1, 16, 0.01, 0.01, seed=4242)
    cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
    red = oracle.assemble(c.n, c.rp, c.col, c.val, cls)
    xstar = oracle.dense_solve(oracle.dense_m(red), red.b) if red.nq <= 3000 else None
    prev = np.zeros(red.nq)
    for k in [1, 2, 5, 10, 50, 200]:
        x, it, _, _ = oracle.jacobi(red, max_iter=k, tol=0.0)
        assert it == k
        assert np.all(x >= prev - 4 * np.finfo(float).eps)
        assert np.all(x <= xstar + 1e-12)
        prev = x


def test_bicgstab_finite_termination():
    """In exact arithmetic BiCGStab terminates in at most n iterations
    (Section 3.2) unless it breaks down (q.r or q.v vanishing); on tiny systems
    that do not break down, n iterations leave a tiny residual.  Rounding can
    leave a near-breakdown case short of exact termination, so the check is on
    the bulk: at least 90% of the cases end at rounding level."""
    rng = np.random.Generator(np.random.PCG64(900))
    res = []
    for _ in range(400):
        c = cg.random_small(int(rng.integers(4, 14)), rng, dmax=4, goal_frac=0.2, sink_frac=0.2)
        cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
        red = oracle.assemble(c.n, c.rp, c.col, c.val, cls)
        if not 2 <= red.nq <= 8:
            continue
        x, it, _, rc = oracle.bicgstab(red, tol=0.0, max_iter=red.nq)
        if rc == oracle.BREAKDOWN:
            continue
        _, rn = oracle.residual(red, red.b, x)
        res.append(rn)
    res = np.array(res)
    assert res.size >= 50
    assert np.mean(res <= 1e-12) >= 0.9


def test_monte_carlo_path_simulation():
    """Simulated paths from s0 hit GS with the oracle's probability (5 sigma)."""
    c = cg.random_sparse(12, 1, 3, 0.17, 0.17, seed=31337, absorbing_goals=True)
    s = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, "jacobi", tol=1e-12, stop_mode=1)
    sq = np.nonzero(s.cls == oracle.SQ)[0]
    assert sq.size
    s0 = int(sq[0])
    p = c.dense()
    cum = np.cumsum(p, axis=1)
    rng = np.random.Generator(np.random.PCG64(2024))
    npath = 200_000
    state = np.full(npath, s0)
    done = np.zeros(npath, bool)
    hit = np.zeros(npath, bool)
    goal = c.goal.astype(bool)
    absorbing = np.isclose(np.diag(p), 1.0)
    for _ in range(3000):
        u = rng.random(npath)
        nxt = (u[:, None] > cum[state]).sum(axis=1)
        nxt = np.minimum(nxt, c.n - 1)
        state = np.where(done, state, nxt)
        newly = ~done & goal[state]
        hit |= newly
        done |= goal[state] | absorbing[state]
        if done.all():
            break
    est = hit.mean()
    sigma = np.sqrt(s.x[s0] * (1 - s.x[s0]) / npath)
    assert abs(est - s.x[s0]) <= 5 * sigma + 1e-4


# --------------------------------------------------------------------------
# adjoint and gradient

def _grad_case(seed, n=120):
    rng = np.random.Generator(np.random.PCG64(seed))
    c = cg.random_small(n, rng, dmax=6, goal_frac=0.05, sink_frac=0.05)
    s = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, "jacobi", tol=1e-13, stop_mode=1)
    return c, s


@pytest.mark.parametrize("seed", range(4))
def test_adjoint_duality_and_sign(seed):
    c, s = _grad_case(3000 + seed)
    if s.red.nq == 0:
        pytest.skip("empty S_?")
    sq = np.nonzero(s.cls == oracle.SQ)[0]
    s0 = int(sq[0])
    seed_v = np.zeros(c.n); seed_v[s0] = 1.0
    lam, _, _, rc = oracle.adjoint(s, seed_v, tol=1e-13)
    assert rc == oracle.OK
    # x_s0 = e^T M^-1 b = lam . b
    assert abs(s.x[s0] - lam @ s.red.b) <= 1e-12
    # lam_i = expected visits to i starting from s0: non-negative, >= 1 at s0
    assert np.all(lam >= -1e-14) and lam[s.red.map[s0]] >= 1 - 1e-12
    # against LAPACK: lam = row s0 of (I - A)^-1
    g = np.linalg.inv(oracle.dense_m(s.red))
    assert np.abs(lam - g[s.red.map[s0], :]).max() <= 1e-11 * max(1, np.abs(lam).max())


@pytest.mark.parametrize("seed", range(4))
def test_gradient_central_differences(seed):
    """dx_s0/dP(i,j) = lam_i x_j, against central differences of dense
    solves with the partition held fixed (h = 1e-6)."""
    c, s = _grad_case(4000 + seed, n=60)
    if s.red.nq == 0:
        pytest.skip("empty S_?")
    sq = np.nonzero(s.cls == oracle.SQ)[0]
    s0 = int(sq[0])
    seed_v = np.zeros(c.n); seed_v[s0] = 1.0
    lam, _, _, _ = oracle.adjoint(s, seed_v, tol=1e-14)
    g = oracle.gradient(c.n, c.rp, c.col, s.cls, s.red, lam, s.x)
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = np.repeat(np.arange(c.n), np.diff(c.rp))
    cand = np.nonzero((s.cls[rows] == oracle.SQ) & (c.val > 2e-6))[0]
    h = 1e-6
    checked = 0
    for k in rng.choice(cand, size=min(16, cand.size), replace=False):
        xs = []
        for sign in (+1, -1):
            val = c.val.copy(); val[k] += sign * h
            red = oracle.assemble(c.n, c.rp, c.col, val, s.cls)
            xs.append(np.linalg.solve(oracle.dense_m(red), red.b)[red.map[s0]])
        fd = (xs[0] - xs[1]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-8) + 1e-9
        checked += 1
    assert checked > 0
    # rows outside S_? carry no gradient
    assert np.all(g[s.cls[rows] != oracle.SQ] == 0)


@pytest.mark.parametrize("seed", range(3))
def test_gradient_sherman_morrison(seed):
    """A finite change t of one entry P(i,j) (i, j in S_?) moves x_s0 by
    exactly t lam_i x_j / (1 - t G_ji), G = (I - A)^-1."""
    c, s = _grad_case(5000 + seed, n=80)
    sq = np.nonzero(s.cls == oracle.SQ)[0]
    if sq.size < 2:
        pytest.skip("too small")
    s0 = int(sq[0])
    seed_v = np.zeros(c.n); seed_v[s0] = 1.0
    lam, _, _, _ = oracle.adjoint(s, seed_v, tol=1e-14)
    gm = np.linalg.inv(oracle.dense_m(s.red))
    rows = np.repeat(np.arange(c.n), np.diff(c.rp))
    both = np.nonzero((s.cls[rows] == oracle.SQ) & (s.cls[c.col] == oracle.SQ) & (rows != c.col))[0]
    if both.size == 0:
        pytest.skip("no S_? x S_? entry")
    k = int(both[0])
    i, j = s.red.map[rows[k]], s.red.map[c.col[k]]
    t = 0.01
    val = c.val.copy(); val[k] += t
    red = oracle.assemble(c.n, c.rp, c.col, val, s.cls)
    xnew = np.linalg.solve(oracle.dense_m(red), red.b)[red.map[s0]]
    pred = s.x[s0] + t * lam[i] * s.xq[j] / (1 - t * gm[j, i])
    assert abs(xnew - pred) <= 1e-12


# --------------------------------------------------------------------------
# iterates and input checks

def test_jacobi_iterates_worked_example():
    """On the worked example the Jacobi iteration matrix J = [[0,.5],[.4,0]]
    has J^2 = 0.2 I, so from zero x_{2m} = (1 - 0.2^m) [0.625, 0.25] and
    x_{2m+1} = x_{2m} + 0.2^m [0.5, 0] -- a true (double-buffered) Jacobi
    sweep, not an in-place one."""
    g = _load("worked_example.json")
    c = cg.from_dense(g["P"], goal=g["goal"])
    cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
    red = oracle.assemble(c.n, c.rp, c.col, c.val, cls)
    for k in range(1, 31):
        x, it, delta, _ = oracle.jacobi(red, tol=0.0, max_iter=k)
        m = k // 2
        want = (1 - 0.2 ** m) * np.array([0.625, 0.25])
        if k % 2:
            want = want + 0.2 ** m * np.array([0.5, 0.0])
        assert it == k
        np.testing.assert_allclose(x, want, rtol=0, atol=1e-15)


def test_jacobi_paper_rule_stops_on_first_small_delta():
    g = _load("worked_example.json")
    c = cg.from_dense(g["P"], goal=g["goal"])
    cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
    red = oracle.assemble(c.n, c.rp, c.col, c.val, cls)
    # deltas are 0.5, 0.2, 0.1, 0.04, 0.02, 0.008, ... ; the first below 0.03 is the 5th
    x, it, delta, rc = oracle.jacobi(red, tol=0.03, max_iter=100)
    assert rc == oracle.OK and it == 5 and abs(delta - 0.02) < 1e-15


@pytest.mark.parametrize("case", ["rowsum", "negative", "nan", "above1", "colrange",
                                  "unsorted", "duplicate", "instance", "rp"])
def test_validate_rejects_bad_chains(case):
    c = cg.concat([cg.random_sparse(30, 2, 4, 0.1, 0.1, seed=1),
                   cg.random_sparse(20, 2, 4, 0.1, 0.1, seed=2)])
    rp, col, val = c.rp.copy(), c.col.copy(), c.val.copy()
    row = 7
    k = int(rp[row])
    assert rp[row + 1] - rp[row] >= 2
    want = {"rowsum": 5, "negative": 4, "nan": 4, "above1": 4, "colrange": 2,
            "unsorted": 3, "duplicate": 3, "instance": 6, "rp": 1}[case]
    if case == "rowsum":
        val[k] *= 0.9
    elif case == "negative":
        val[k] = -val[k]
    elif case == "nan":
        val[k] = np.nan
    elif case == "above1":
        val[k] = 1.5
    elif case == "colrange":
        col[k] = c.n + 3
    elif case == "unsorted":
        col[k], col[k + 1] = col[k + 1], col[k]
    elif case == "duplicate":
        col[k + 1] = col[k]
    elif case == "instance":
        col[k + 1] = 40      # a state of the second chain
        col[k + 1:rp[row + 1]] = np.arange(40, 40 + rp[row + 1] - k - 1)
    elif case == "rp":
        rp[row + 1] = rp[row] - 1
    r, reason = oracle.validate(c.n, rp, col, val, c.inst_off)
    assert reason == want
    if case != "rp":
        assert r == row
    assert oracle.validate(c.n, c.rp, c.col, c.val, c.inst_off) == (-1, 0)


def test_bicgstab_paper_rule_worked_example_by_hand():
    """The paper-rule stop of the oracle's BiCGStab (every |s_i| <= tol,
    Section 5.2) against the two steps worked out by hand on the printed
    2x2 system of Section 2.3: the stop is on s (not on r, which crosses the
    tolerance one step earlier at tol = 0.1) and is an inclusive test (at
    tol = 0.2 exactly it stops after step 1)."""
    g = _load("bicgstab_worked_example.json")
    c = cg.from_dense(_load("worked_example.json")["P"], goal=[3])
    cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
    red = oracle.assemble(c.n, c.rp, c.col, c.val, cls)
    np.testing.assert_array_equal(oracle.dense_m(red), np.array(g["system"]["M"]))
    np.testing.assert_array_equal(red.b, g["system"]["b"])
    hand = g["derived_by_hand"]
    for case in g["cases"]:
        x, it, smax, rc = oracle.bicgstab(red, tol=case["tol"], stop_mode=0)
        assert rc == oracle.OK, case
        assert it == case["iterations"], case
        step = hand["step%d" % it]
        np.testing.assert_allclose(x, step["x"], atol=1e-15, rtol=0)
        assert abs(smax - step["max_abs_s"]) <= 1e-16, (case, smax)
    # step 1's s is exactly the double nearest 0.2
    _, it, smax, _ = oracle.bicgstab(red, tol=0.2, stop_mode=0)
    assert it == 1 and smax == 0.2
    # one step only: the residual of x after step 1 is (0.08, 0.04) by hand
    x1, _, _, _ = oracle.bicgstab(red, tol=0.0, stop_mode=0, max_iter=1)
    r, rn = oracle.residual(red, red.b, x1)
    np.testing.assert_allclose(r, hand["step1"]["r"], atol=1e-16, rtol=0)
    assert abs(rn - hand["step1"]["max_abs_r"]) <= 1e-16


# --------------------------------------------------------------------------
# general systems A x = b (the experiments of Section 6)

def _dense(m):
    a = np.zeros((m.n, m.n))
    rows = np.repeat(np.arange(m.n), np.diff(m.rp))
    a[rows, m.col] = m.val
    return a


def test_matrix_system_jacobi_splitting_by_hand():
    """A = [[4, 1], [2, 5]], b = [5, 7], x* = [1, 1]: d = diag(A), A_off = -R;
    Jacobi from 0 gives [5/4, 7/5], then [0.9, 0.9] (the iteration matrix
    J = -D^{-1} R has J^2 = I/10)."""
    c = cg.from_dense(np.array([[4.0, 1.0], [2.0, 5.0]]))
    red = oracle.matrix_system(2, c.rp, c.col, c.val, np.array([5.0, 7.0]))
    assert np.array_equal(red.d, [4.0, 5.0]) and np.array_equal(red.aval, [-1.0, -2.0])
    assert np.array_equal(red.arp, [0, 1, 2]) and np.array_equal(red.acol, [1, 0])
    x1, it, _, _ = oracle.jacobi(red, tol=0.0, max_iter=1, stop_mode=0)
    assert it == 1 and np.array_equal(x1, [1.25, 1.4])
    x2, _, _, _ = oracle.jacobi(red, tol=0.0, max_iter=2, stop_mode=0)
    assert np.abs(x2 - 0.9).max() <= 1e-15
    x, it, rc = oracle.solve_matrix(2, c.rp, c.col, c.val, np.array([5.0, 7.0]), "bicgstab", tol=1e-14)
    assert rc == oracle.OK and np.abs(x - 1.0).max() <= 1e-14


@pytest.mark.parametrize("seed", range(6))
def test_dominance_bound_bounds_the_inverse(seed):
    m = cg.diag_dominant(int(10 + 9 * seed), density=0.3, seed=500 + seed)
    a = _dense(m)
    red = oracle.matrix_system(m.n, m.rp, m.col, m.val, m.rhs)
    bound = oracle.dominance_bound(red)
    assert bound >= np.abs(np.linalg.inv(a)).sum(axis=1).max() * (1 - 1e-12)
    # a diagonal matrix: the bound is exact
    dg = cg.from_dense(np.diag(np.arange(1.0, 8.0)))
    rd = oracle.matrix_system(7, dg.rp, dg.col, dg.val, np.ones(7))
    assert oracle.dominance_bound(rd) == 1.0
    # a row that is not strictly dominant has no bound
    nd = cg.from_dense(np.array([[2.0, 2.0], [1.0, 3.0]]))
    assert oracle.dominance_bound(oracle.matrix_system(2, nd.rp, nd.col, nd.val, np.ones(2))) == -1.0


@pytest.mark.parametrize("method", ["jacobi", "bicgstab"])
@pytest.mark.parametrize("seed", range(4))
def test_solve_matrix_matches_lapack(method, seed):
    m = cg.diag_dominant(int(40 + 50 * seed), density=0.15, seed=600 + seed)
    x, it, rc = oracle.solve_matrix(m.n, m.rp, m.col, m.val, m.rhs, method, tol=1e-13)
    assert rc == oracle.OK
    assert np.abs(x - np.linalg.solve(_dense(m), m.rhs)).max() <= 1e-12


def test_matrix_without_diagonal_rejected():
    c = cg.from_dense(np.array([[0.0, 1.0], [1.0, 3.0]]))
    with pytest.raises(np.linalg.LinAlgError):
        oracle.matrix_system(2, c.rp, c.col, c.val, np.ones(2))
