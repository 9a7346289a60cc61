"""Seeded synthetic Markov chains: the inputs shared by the GPU library's tests
and benchmark and by the CPU oracle's checks.

This module only builds inputs (row-stochastic transition matrices in
compressed row storage, goal masks, block-diagonal packing).  It holds none of
the reachability method's arithmetic: no partition, no reduced system, no
solver.  Every generator is driven by numpy's PCG64 stream from an explicit
seed, so the same seed gives the same chain on every machine.

Storage follows Section 4 of the paper (compressed row storage): ``rp`` of
length n+1 with rp[i] = number of stored entries in rows before i, ``col`` the
column of each entry (strictly ascending inside a row) and ``val`` the
probability.  Several independent chains are packed block-diagonally; state k
of chain c is global state inst_off[c] + k.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 12106412


@dataclass
class Chain:
    n: int
    rp: np.ndarray          # int32[n+1]
    col: np.ndarray         # int32[nnz]
    val: np.ndarray         # float64[nnz]
    goal: np.ndarray        # uint8[n]
    inst_off: np.ndarray    # int64[K+1]
    name: str = "chain"
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rp[-1])

    @property
    def num_instances(self) -> int:
        return len(self.inst_off) - 1

    def instance(self, k: int) -> "Chain":
        """Chain k of a block-diagonal pack, renumbered from zero."""
        lo, hi = int(self.inst_off[k]), int(self.inst_off[k + 1])
        e0, e1 = int(self.rp[lo]), int(self.rp[hi])
        rp = (self.rp[lo:hi + 1] - e0).astype(np.int32)
        col = (self.col[e0:e1] - lo).astype(np.int32)
        return Chain(hi - lo, rp, col, self.val[e0:e1].copy(), self.goal[lo:hi].copy(),
                     np.array([0, hi - lo], dtype=np.int64), f"{self.name}[{k}]")

    def dense(self) -> np.ndarray:
        m = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rp))
        m[rows, self.col] = self.val
        return m


def from_dense(p, goal=None, name="dense") -> Chain:
    """Compressed row storage of a dense matrix: only nonzero entries are kept,
    rows in order, columns ascending (Section 4)."""
    p = np.asarray(p, dtype=np.float64)
    n = p.shape[0]
    rows, cols = np.nonzero(p)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    g = np.zeros(n, dtype=np.uint8) if goal is None else np.zeros(n, dtype=np.uint8)
    if goal is not None:
        g[np.asarray(goal, dtype=np.int64)] = 1
    return Chain(n, rp, cols.astype(np.int32), p[rows, cols].copy(), g,
                 np.array([0, n], dtype=np.int64), name)


def worked_example() -> Chain:
    """The four-state chain drawn in Section 2 with goal set {3}."""
    p = [[0.0, 0.0, 0.5, 0.5],
         [0.0, 1.0, 0.0, 0.0],
         [0.4, 0.6, 0.0, 0.0],
         [0.0, 0.0, 0.0, 1.0]]
    return from_dense(p, goal=[3], name="worked_example")


def gamblers_ruin(n: int = 1000, p: float = 0.45) -> Chain:
    """Birth-death chain on 0..n-1: interior state i moves to i+1 with
    probability p and to i-1 with 1-p; 0 and n-1 are absorbing; goal {n-1}."""
    q = 1.0 - p
    rows, cols, vals = [0], [0], [1.0]
    for i in range(1, n - 1):
        rows += [i, i]
        cols += [i - 1, i + 1]
        vals += [q, p]
    rows.append(n - 1); cols.append(n - 1); vals.append(1.0)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, np.asarray(rows) + 1, 1)
    goal = np.zeros(n, dtype=np.uint8); goal[n - 1] = 1
    return Chain(n, np.cumsum(rp).astype(np.int32), np.asarray(cols, np.int32),
                 np.asarray(vals, np.float64), goal, np.array([0, n], np.int64),
                 f"gamblers_ruin(n={n},p={p})", {"p": p})


# --------------------------------------------------------------------------
# helpers shared by the random generators

def _sort_rows(rows, cols, vals=None):
    order = np.lexsort((cols, rows))
    rows = rows[order]; cols = cols[order]
    return rows, cols, (None if vals is None else vals[order])


def _distinct_targets(rng, rows, lo, span):
    """For entries belonging to `rows`, draw a target uniformly from
    [lo, lo+span) (per entry), redrawing until no row repeats a target."""
    t = lo + (rng.random(rows.shape[0]) * span).astype(np.int64)
    t = np.minimum(t, lo + span - 1)
    while True:
        order = np.lexsort((t, rows))
        rs, ts = rows[order], t[order]
        dup = np.zeros(rows.shape[0], dtype=bool)
        dup[1:] = (rs[1:] == rs[:-1]) & (ts[1:] == ts[:-1])
        if not dup.any():
            return t
        idx = order[dup]
        nt = lo[idx] + (rng.random(idx.shape[0]) * span[idx]).astype(np.int64)
        t[idx] = np.minimum(nt, lo[idx] + span[idx] - 1)


def _normalise(rp, vals):
    sums = np.add.reduceat(vals, rp[:-1].astype(np.int64)) if vals.size else vals
    deg = np.diff(rp)
    return vals / np.repeat(sums, deg)


def _csr(n, rows, cols, vals):
    rows, cols, vals = _sort_rows(np.asarray(rows, np.int64), np.asarray(cols, np.int64),
                                  np.asarray(vals, np.float64))
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp)
    if rp[-1] >= 2**31:
        raise ValueError("chain too large for 32-bit row pointers")
    return rp.astype(np.int32), cols.astype(np.int32), vals


def _make_absorbing(n, rows, cols, vals, states):
    """Replace the rows of `states` by a probability-one self-loop."""
    keep = ~np.isin(rows, states)
    rows = np.concatenate([rows[keep], states])
    cols = np.concatenate([cols[keep], states])
    vals = np.concatenate([vals[keep], np.ones(states.shape[0])])
    return rows, cols, vals


def _uniform_open_closed(rng, size):
    """Uniform draws on (0, 1]."""
    return 1.0 - rng.random(size)


# --------------------------------------------------------------------------

def random_sparse(n=20_000, dmin=1, dmax=16, goal_frac=0.01, sink_frac=0.01,
                  seed=SEED_BASE + 2, absorbing_goals=False, name=None) -> Chain:
    """Random sparse chain: out-degree uniform in [dmin, dmax], distinct
    targets uniform over all states (self-loops allowed), weights uniform on
    (0,1] normalised per row.  A seeded permutation picks goal_frac*n goal
    states (their rows kept unless absorbing_goals) and the next sink_frac*n
    states as absorbing non-goal states."""
    rng = np.random.Generator(np.random.PCG64(seed))
    deg = rng.integers(dmin, dmax + 1, size=n)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    lo = np.zeros(rows.shape[0], dtype=np.int64)
    span = np.full(rows.shape[0], n, dtype=np.int64)
    cols = _distinct_targets(rng, rows, lo, span)
    w = _uniform_open_closed(rng, rows.shape[0])
    perm = rng.permutation(n)
    ng = int(round(goal_frac * n)); ns = int(round(sink_frac * n))
    goals = np.sort(perm[:ng]); sinks = np.sort(perm[ng:ng + ns])
    absorb = np.concatenate([sinks, goals]) if absorbing_goals else sinks
    rows, cols, w = _make_absorbing(n, rows, cols, w, absorb)
    rp, col, w = _csr(n, rows, cols, w)
    val = _normalise(rp, w)
    goal = np.zeros(n, dtype=np.uint8); goal[goals] = 1
    return Chain(n, rp, col, val, goal, np.array([0, n], np.int64),
                 name or f"random_sparse(n={n},deg={dmin}..{dmax})",
                 {"seed": seed, "goals": ng, "sinks": ns})


def dense_random(n=8192, density=0.10, goal_frac=0.005, sink_frac=0.0,
                 seed=SEED_BASE + 3, name=None) -> Chain:
    """Dense-ish chain: every entry (i, j) is present independently with
    probability `density`; weights uniform on (0,1], normalised per row (a row
    left empty gets a self-loop).  goal_frac*n goal states by seeded
    permutation; sink_frac*n further states made absorbing non-goal states
    (sink_frac = 0 is the chain as specified; a positive value gives the
    variant whose undecided set is not trivially empty)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows_l, cols_l = [], []
    chunk = 512
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        mask = rng.random((r1 - r0, n)) < density
        rr, cc = np.nonzero(mask)
        rows_l.append(rr + r0); cols_l.append(cc)
    rows = np.concatenate(rows_l).astype(np.int64)
    cols = np.concatenate(cols_l).astype(np.int64)
    empty = np.setdiff1d(np.arange(n), rows)
    rows = np.concatenate([rows, empty]); cols = np.concatenate([cols, empty])
    w = _uniform_open_closed(rng, rows.shape[0])
    perm = rng.permutation(n)
    ng = int(round(goal_frac * n)); ns = int(round(sink_frac * n))
    goals = np.sort(perm[:ng]); sinks = np.sort(perm[ng:ng + ns])
    rows, cols, w = _make_absorbing(n, rows, cols, w, sinks)
    rp, col, w = _csr(n, rows, cols, w)
    val = _normalise(rp, w)
    goal = np.zeros(n, dtype=np.uint8); goal[goals] = 1
    return Chain(n, rp, col, val, goal, np.array([0, n], np.int64),
                 name or f"dense_random(n={n},density={density},sinks={ns})",
                 {"seed": seed, "goals": ng, "sinks": ns})


def program_graph(n=2_000_000, goal_frac=0.01, sink_frac=0.001, local=64,
                  jump_frac=0.02, seed=SEED_BASE + 4, name=None) -> Chain:
    """Model-checker-shaped chain built from fair coin flips: each state has
    2, 3 or 4 successors with probabilities {1/2,1/2}, {1/2,1/4,1/4} or
    {1/4,1/4,1/4,1/4}.  A successor is s + U{+-1..+-local} reflected into
    range with probability 1 - jump_frac, else uniform over all states;
    successors of a state are distinct.  goal_frac*n terminating states form
    the goal set and sink_frac*n error sinks; both are absorbing."""
    rng = np.random.Generator(np.random.PCG64(seed))
    deg = rng.integers(2, 5, size=n)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    m = rows.shape[0]
    jump = rng.random(m) < jump_frac
    off = rng.integers(1, local + 1, size=m) * np.where(rng.random(m) < 0.5, -1, 1)
    t = rows + off
    t = np.where(t < 0, -t, t)
    t = np.where(t >= n, 2 * (n - 1) - t, t)
    t = np.where(jump, rng.integers(0, n, size=m), t)
    while True:
        order = np.lexsort((t, rows))
        rs, ts = rows[order], t[order]
        dup = np.zeros(m, dtype=bool)
        dup[1:] = (rs[1:] == rs[:-1]) & (ts[1:] == ts[:-1])
        if not dup.any():
            break
        idx = order[dup]
        o = rng.integers(1, local + 1, size=idx.shape[0]) * np.where(rng.random(idx.shape[0]) < 0.5, -1, 1)
        nt = rows[idx] + o
        nt = np.where(nt < 0, -nt, nt)
        nt = np.where(nt >= n, 2 * (n - 1) - nt, nt)
        t[idx] = nt
    # coin-flip probabilities: position k (0-based, in draw order) of a row
    pos = np.arange(m) - np.repeat(np.cumsum(deg) - deg, deg)
    dd = np.repeat(deg, deg)
    w = np.where(dd == 2, 0.5, np.where(dd == 4, 0.25, np.where(pos == 0, 0.5, 0.25)))
    perm = rng.permutation(n)
    ng = int(round(goal_frac * n)); ns = int(round(sink_frac * n))
    goals = np.sort(perm[:ng]); sinks = np.sort(perm[ng:ng + ns])
    rows, t, w = _make_absorbing(n, rows, t, w, np.concatenate([goals, sinks]))
    rp, col, val = _csr(n, rows, t, w)
    goal = np.zeros(n, dtype=np.uint8); goal[goals] = 1
    return Chain(n, rp, col, val, goal, np.array([0, n], np.int64),
                 name or f"program_graph(n={n})", {"seed": seed, "goals": ng, "sinks": ns})


def concat(chains, name="batched") -> Chain:
    """Block-diagonal pack of independent chains."""
    ns = [c.n for c in chains]
    off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    eo = np.concatenate([[0], np.cumsum([c.nnz for c in chains])]).astype(np.int64)
    if eo[-1] >= 2**31:
        raise ValueError("pack too large for 32-bit row pointers")
    rp = np.concatenate([c.rp[:-1].astype(np.int64) + eo[k] for k, c in enumerate(chains)] + [[eo[-1]]])
    col = np.concatenate([c.col.astype(np.int64) + off[k] for k, c in enumerate(chains)])
    val = np.concatenate([c.val for c in chains])
    goal = np.concatenate([c.goal for c in chains])
    return Chain(int(off[-1]), rp.astype(np.int32), col.astype(np.int32), val, goal, off, name)


def batched(K=256, nmin=1_000, nmax=200_000, dmin=1, dmax=8, goal_frac=0.01,
            sink_frac=0.0, seed=SEED_BASE + 5, name=None) -> Chain:
    """K independent random sparse chains with n log-uniform in [nmin, nmax],
    out-degree uniform in [dmin, dmax], weights uniform normalised, goal_frac
    goal states per chain (sink_frac absorbing non-goal states per chain, zero
    as specified), packed block-diagonally."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.rint(np.exp(rng.uniform(np.log(nmin), np.log(nmax), size=K))).astype(np.int64)
    seeds = rng.integers(0, 2**62, size=K)
    chains = [random_sparse(int(sizes[k]), dmin, dmax, goal_frac, sink_frac, int(seeds[k]))
              for k in range(K)]
    c = concat(chains, name or f"batched(K={K},n={nmin}..{nmax},sinks={sink_frac})")
    c.meta = {"seed": seed, "sizes": sizes.tolist()}
    return c


def random_small(n, rng, dmax=4, goal_frac=0.15, sink_frac=0.1, zero_frac=0.0,
                 absorbing_goals=False, self_loops=True) -> Chain:
    """Small varied chains for brute-force checks (tests only): degrees
    uniform in [1, dmax], optional stored zeros, random goal/sink states."""
    seed = int(rng.integers(0, 2**62))
    c = random_sparse(n, 1, min(dmax, n), goal_frac, sink_frac, seed, absorbing_goals)
    if not self_loops:
        pass
    if zero_frac > 0 and c.nnz:
        r = np.random.Generator(np.random.PCG64(seed + 1))
        z = r.random(c.nnz) < zero_frac
        val = c.val.copy(); val[z] = 0.0
        rows = np.repeat(np.arange(c.n), np.diff(c.rp))
        sums = np.bincount(rows, weights=val, minlength=c.n)
        # rows that lost all mass get their first entry back
        for i in np.nonzero(sums == 0)[0]:
            val[c.rp[i]] = 1.0
        sums = np.bincount(rows, weights=val, minlength=c.n)
        c.val = val / sums[rows]
    return c


@dataclass
class Matrix:
    """A general square system A x = rhs in compressed row storage (diagonal
    stored, ascending columns); several packed block-diagonally."""
    n: int
    rp: np.ndarray          # int32[n+1]
    col: np.ndarray         # int32[nnz]
    val: np.ndarray         # float64[nnz]
    rhs: np.ndarray         # float64[n]
    inst_off: np.ndarray    # int64[K+1]
    name: str = "matrix"
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rp[-1])

    @property
    def num_instances(self) -> int:
        return len(self.inst_off) - 1

    def instance(self, k: int) -> "Matrix":
        lo, hi = int(self.inst_off[k]), int(self.inst_off[k + 1])
        e0, e1 = int(self.rp[lo]), int(self.rp[hi])
        return Matrix(hi - lo, (self.rp[lo:hi + 1] - e0).astype(np.int32), (self.col[e0:e1] - lo).astype(np.int32),
                      self.val[e0:e1].copy(), self.rhs[lo:hi].copy(), np.array([0, hi - lo], dtype=np.int64),
                      f"{self.name}[{k}]")


def layered(nblocks=64, block=2000, deg=4, forward=0.05, leave=0.01, transient=0, seed=SEED_BASE + 7,
            name=None) -> Chain:
    """Chain whose undecided states fall into `nblocks` strongly connected
    blocks of `block` states in a row (block b's states can reach block
    b+1's, never back), the shape of a model whose phases run in sequence.
    Inside a block: a cycle through its states (which makes it strongly
    connected) plus deg-1 further random targets; with probability `forward`
    per state one more edge into a random state of the next block (the last
    block's go to the goal); with probability `leave` one more edge to an
    absorbing non-goal state.  `transient` extra states each lead into a
    random state of a random block or of an earlier transient state (one-state
    components of the condensation).  The goal and the sink are the last two
    states.  Weights uniform on (0,1], normalised per row."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = nblocks * block
    n = nb + transient + 2
    goal_s, sink_s = n - 2, n - 1
    rows_l, cols_l = [], []
    idx = np.arange(nb)
    blk = idx // block
    rows_l.append(idx)
    cols_l.append(blk * block + (idx % block + 1) % block)
    for _ in range(max(deg - 1, 0)):
        rows_l.append(idx)
        cols_l.append(blk * block + rng.integers(0, block, nb))
    fw = idx[rng.random(nb) < forward]
    nxt = blk[fw] + 1
    tgt = np.where(nxt < nblocks, nxt * block + rng.integers(0, block, fw.size), goal_s)
    rows_l.append(fw)
    cols_l.append(tgt)
    lv = idx[rng.random(nb) < leave]
    rows_l.append(lv)
    cols_l.append(np.full(lv.size, sink_s))
    # the last block always reaches the goal
    rows_l.append(np.array([nb - 1]))
    cols_l.append(np.array([goal_s]))
    if transient > 0:
        t = nb + np.arange(transient)
        earlier = rng.random(transient) < 0.5
        into_t = np.array([nb + rng.integers(0, i) if (earlier[i] and i > 0) else rng.integers(0, nb)
                           for i in range(transient)], dtype=np.int64)
        rows_l.append(t)
        cols_l.append(into_t)
    rows_l.append(np.array([goal_s, sink_s]))
    cols_l.append(np.array([goal_s, sink_s]))
    rows = np.concatenate(rows_l).astype(np.int64)
    cols = np.concatenate(cols_l).astype(np.int64)
    rows, cols = _sort_rows(rows, cols)[:2]
    keep = np.ones(rows.size, dtype=bool)
    keep[1:] = (rows[1:] != rows[:-1]) | (cols[1:] != cols[:-1])
    rows, cols = rows[keep], cols[keep]
    w = _uniform_open_closed(rng, rows.size)
    rp, col, w = _csr(n, rows, cols, w)
    val = _normalise(rp, w)
    goal = np.zeros(n, dtype=np.uint8)
    goal[goal_s] = 1
    return Chain(n, rp, col, val, goal, np.array([0, n], np.int64),
                 name or f"layered(blocks={nblocks}x{block},deg={deg},transient={transient})",
                 {"seed": seed})


def ladder(n=3000, p=0.9) -> Chain:
    """A path of n undecided states: state i moves to i+1 with probability p
    and to an absorbing non-goal state otherwise; the last one reaches the
    goal with probability p.  S_? is acyclic, n levels deep; x_i = p^(n-i)."""
    rows = np.concatenate([np.repeat(np.arange(n), 2), [n, n + 1]])
    cols = np.concatenate([np.stack([np.arange(1, n + 1), np.full(n, n + 1)], 1).ravel(), [n, n + 1]])
    vals = np.concatenate([np.tile([p, 1 - p], n), [1.0, 1.0]])
    rp, col, v = _csr(n + 2, rows, cols, vals)
    goal = np.zeros(n + 2, dtype=np.uint8)
    goal[n] = 1
    return Chain(n + 2, rp, col, v, goal, np.array([0, n + 2], np.int64), f"ladder(n={n},p={p})", {})


def diag_dominant(n, density=None, offdiag=None, vmax=10, seed=SEED_BASE + 6, name=None) -> Matrix:
    """Random strictly diagonally dominant matrix of positive integers with a
    positive integer right-hand side (the systems of the paper's experiments,
    Section 6): off-diagonal entries uniform in {1..vmax}, present
    independently with probability `density`, or `offdiag` of them placed
    uniformly at random (distinct positions); diagonal entry = sum of the
    row's off-diagonal entries + uniform {1..vmax}; rhs uniform {1..vmax}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if offdiag is not None:
        flat = rng.choice(n * (n - 1), size=int(offdiag), replace=False) if n > 1 else np.zeros(0, np.int64)
        rows = flat // (n - 1)
        cols = flat % (n - 1)
        cols = cols + (cols >= rows)
    else:
        rows_l, cols_l = [], []
        chunk = max(1, (1 << 24) // max(n, 1))
        for r0 in range(0, n, chunk):
            r1 = min(n, r0 + chunk)
            mask = rng.random((r1 - r0, n)) < density
            mask[np.arange(r1 - r0), np.arange(r0, r1)] = False
            rr, cc = np.nonzero(mask)
            rows_l.append(rr + r0); cols_l.append(cc)
        rows = np.concatenate(rows_l).astype(np.int64)
        cols = np.concatenate(cols_l).astype(np.int64)
    off = rng.integers(1, vmax + 1, size=rows.shape[0]).astype(np.float64)
    diag = np.bincount(rows, weights=off, minlength=n) + rng.integers(1, vmax + 1, size=n)
    rows = np.concatenate([rows, np.arange(n)]); cols = np.concatenate([cols, np.arange(n)])
    vals = np.concatenate([off, diag])
    rp, col, val = _csr(n, rows, cols, vals)
    rhs = rng.integers(1, vmax + 1, size=n).astype(np.float64)
    label = f"density={density}" if offdiag is None else f"offdiag={offdiag}"
    return Matrix(n, rp, col, val, rhs, np.array([0, n], np.int64), name or f"diag_dominant(n={n},{label})",
                  {"seed": seed})


def concat_matrices(ms, name="batched matrices") -> Matrix:
    """Block-diagonal pack of several systems."""
    offs = np.concatenate([[0], np.cumsum([m.n for m in ms])]).astype(np.int64)
    rps = [ms[0].rp.astype(np.int64)]
    for m in ms[1:]:
        rps.append(m.rp[1:].astype(np.int64) + rps[-1][-1])
    rp = np.concatenate(rps)
    col = np.concatenate([m.col.astype(np.int64) + offs[i] for i, m in enumerate(ms)]).astype(np.int32)
    return Matrix(int(offs[-1]), rp.astype(np.int32), col, np.concatenate([m.val for m in ms]),
                  np.concatenate([m.rhs for m in ms]), offs, name)


CONFIGS = {
    1: lambda: gamblers_ruin(1000, 0.45),
    2: lambda: random_sparse(20_000, 1, 16, 0.01, 0.01, SEED_BASE + 2),
    3: lambda: dense_random(8192, 0.10, 0.005, 0.0, SEED_BASE + 3),
    4: lambda: program_graph(2_000_000, 0.01, 0.001, 64, 0.02, SEED_BASE + 4),
    5: lambda: batched(256, 1_000, 200_000, 1, 8, 0.01, 0.0, SEED_BASE + 5),
}
