"""Pins of the oracle's strongly-connected-component decomposition of S_?
(the decomposition Section 8 proposes: components solved in reverse
topological order).

* hand cases: the worked example's two undecided states form one component;
  a path is all singletons with levels counting down to the sink end; a
  self-loop (kept in d) joins nothing;
* the partition equals SciPy's strong components (a library routine written
  independently), labels made canonical as the smallest index;
* the levels equal the longest path in the condensation, computed here by a
  plain fixpoint over the edges, and every edge between components goes
  strictly down in level;
* solving the components level by level (one-state components by
  substitution, the others by a dense solve with the lower levels' values
  moved to the right-hand side) gives the oracle's solution of the whole
  system."""
import numpy as np
import pytest
import scipy.sparse as sps
from scipy.sparse.csgraph import connected_components

import chaingen as cg
import oracle


def _red(c):
    cls = oracle.partition(c.n, c.rp, c.col, c.val, c.goal)
    return oracle.assemble(c.n, c.rp, c.col, c.val, cls)


def _from_edges(nq, edges, d=None):
    """Reduced system with the given positive off-diagonal entries."""
    edges = sorted(edges)
    arp = np.zeros(nq + 1, dtype=np.int64)
    for i, _, _ in edges:
        arp[i + 1] += 1
    arp = np.cumsum(arp)
    acol = np.array([j for _, j, _ in edges], dtype=np.int64)
    aval = np.array([v for _, _, v in edges], dtype=np.float64)
    d = np.ones(nq) if d is None else np.asarray(d, dtype=np.float64)
    return oracle.Reduced(nq, np.arange(nq), arp, acol, aval, d, np.zeros(nq))


def test_worked_example_is_one_component():
    red = _red(cg.worked_example())
    label, level, nc = oracle.scc(red)
    assert red.nq == 2 and label.tolist() == [0, 0] and level.tolist() == [0, 0] and nc == 1


def test_path_and_self_loop():
    red = _from_edges(4, [(0, 1, 0.5), (1, 2, 0.5), (2, 3, 0.5)], d=[1.0, 0.5, 1.0, 1.0])
    label, level, nc = oracle.scc(red)
    assert label.tolist() == [0, 1, 2, 3] and level.tolist() == [3, 2, 1, 0] and nc == 4
    # a cycle 1 -> 2 -> 1 in the middle of a path
    red = _from_edges(4, [(0, 1, 0.5), (1, 2, 0.5), (2, 1, 0.3), (2, 3, 0.2)])
    label, level, nc = oracle.scc(red)
    assert label.tolist() == [0, 1, 1, 3] and level.tolist() == [2, 1, 1, 0] and nc == 3
    # zero entries are not edges
    red = _from_edges(2, [(0, 1, 0.0), (1, 0, 0.5)])
    label, level, nc = oracle.scc(red)
    assert label.tolist() == [0, 1] and level.tolist() == [0, 1] and nc == 2


def _graphs():
    out = []
    for seed in range(12):
        rng = np.random.Generator(np.random.PCG64(5200 + seed))
        n = int(rng.integers(5, 500))
        c = cg.random_small(n, rng, dmax=int(rng.integers(1, 5)), goal_frac=0.1, sink_frac=0.1,
                            zero_frac=0.1 if seed % 3 == 0 else 0.0, absorbing_goals=bool(seed % 2))
        out.append(_red(c))
    # random graphs with many small components: a DAG with a few back edges
    for seed in range(6):
        rng = np.random.Generator(np.random.PCG64(5300 + seed))
        n = int(rng.integers(20, 800))
        edges = set()
        for i in range(n):
            for _ in range(int(rng.integers(0, 4))):
                j = int(rng.integers(0, n))
                if j != i and (j > i or rng.random() < 0.05):
                    edges.add((i, j, float(rng.random()) * 0.2 + 0.01))
        out.append(_from_edges(n, list(edges)))
    out.append(_red(cg.CONFIGS[2]()))
    return out


def _scipy_labels(red):
    keep = red.aval > 0
    rows = np.repeat(np.arange(red.nq), np.diff(red.arp))[keep]
    g = sps.csr_matrix((np.ones(rows.size), (rows, red.acol[keep])), shape=(red.nq, red.nq))
    _, lab = connected_components(g, directed=True, connection="strong")
    mn = np.full(lab.max() + 1 if lab.size else 0, red.nq, dtype=np.int64)
    np.minimum.at(mn, lab, np.arange(red.nq))
    return mn[lab]


def _fixpoint_levels(red, label):
    keep = red.aval > 0
    rows = np.repeat(np.arange(red.nq), np.diff(red.arp))[keep]
    cols = red.acol[keep]
    cross = label[rows] != label[cols]
    src, dst = label[rows][cross], label[cols][cross]
    lv = np.zeros(red.nq, dtype=np.int64)  # indexed by label
    while True:
        new = lv.copy()
        np.maximum.at(new, src, lv[dst] + 1)
        if np.array_equal(new, lv):
            break
        lv = new
    return lv[label]


def test_partition_and_levels_match_independent_computations():
    for red in _graphs():
        label, level, nc = oracle.scc(red)
        assert np.array_equal(label, _scipy_labels(red))
        assert nc == np.unique(label).size
        assert np.array_equal(level, _fixpoint_levels(red, label))
        keep = red.aval > 0
        rows = np.repeat(np.arange(red.nq), np.diff(red.arp))[keep]
        cols = red.acol[keep]
        cross = label[rows] != label[cols]
        assert (level[rows][cross] > level[cols][cross]).all()


def test_level_by_level_solve_equals_whole_solve():
    for seed in range(6):
        rng = np.random.Generator(np.random.PCG64(5400 + seed))
        c = cg.random_small(int(rng.integers(20, 300)), rng, dmax=3, goal_frac=0.15, sink_frac=0.1)
        red = _red(c)
        if red.nq == 0:
            continue
        label, level, _ = oracle.scc(red)
        m = np.diag(red.d)
        for i in range(red.nq):
            for e in range(red.arp[i], red.arp[i + 1]):
                m[i, red.acol[e]] -= red.aval[e]
        x = np.zeros(red.nq)
        for lv in range(level.max() + 1):
            for lab in np.unique(label[level == lv]):
                idx = np.nonzero(label == lab)[0]
                rest = np.nonzero(level < lv)[0]
                rhs = red.b[idx] - m[np.ix_(idx, rest)] @ x[rest]
                if idx.size == 1:
                    x[idx] = rhs / m[idx[0], idx[0]]
                else:
                    x[idx] = np.linalg.solve(m[np.ix_(idx, idx)], rhs)
        ref, _, _, rc = oracle.bicgstab(red, tol=1e-14, stop_mode=0)
        assert rc == oracle.OK
        assert np.abs(x - ref).max() <= 1e-12
