"""The seeded input generators produce valid chains with the stated shapes."""
import numpy as np
import pytest

import chaingen as cg
import oracle


def _rows(c):
    return np.repeat(np.arange(c.n), np.diff(c.rp))


@pytest.mark.parametrize("maker", [lambda: cg.CONFIGS[1](), lambda: cg.CONFIGS[2](),
                                   lambda: cg.random_sparse(5000, 1, 16, 0.01, 0.01, seed=3),
                                   lambda: cg.dense_random(512, 0.1, 0.005, 0.005, seed=3),
                                   lambda: cg.program_graph(20_000, seed=3),
                                   lambda: cg.batched(6, 1000, 5000, 1, 8, 0.01, 0.01, seed=3)])
def test_generators_emit_valid_chains(maker):
    c = maker()
    assert c.rp.dtype == np.int32 and c.col.dtype == np.int32 and c.val.dtype == np.float64
    assert c.rp[0] == 0 and c.rp[-1] == c.nnz == c.col.size == c.val.size
    assert oracle.validate(c.n, c.rp, c.col, c.val, c.inst_off) == (-1, 0)
    assert c.goal.sum() >= 1


def test_seeded_and_reproducible():
    a = cg.random_sparse(3000, 1, 16, 0.01, 0.01, seed=11)
    b = cg.random_sparse(3000, 1, 16, 0.01, 0.01, seed=11)
    c = cg.random_sparse(3000, 1, 16, 0.01, 0.01, seed=12)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    assert not np.array_equal(a.col[:100], c.col[:100])


def test_random_sparse_shape():
    c = cg.CONFIGS[2]()
    assert c.n == 20_000
    deg = np.diff(c.rp)
    sinks = np.nonzero((deg == 1) & (c.col[c.rp[:-1]] == np.arange(c.n)) & (c.val[c.rp[:-1]] == 1.0))[0]
    assert c.goal.sum() == 200
    assert len(set(sinks) - set(np.nonzero(c.goal)[0])) >= 200
    free = np.setdiff1d(np.arange(c.n), sinks)
    assert deg[free].min() >= 1 and deg[free].max() <= 16
    assert abs(deg[free].mean() - 8.5) < 0.2


def test_program_graph_coin_flips_and_locality():
    c = cg.program_graph(50_000, seed=9)
    rows = _rows(c)
    vals = np.unique(c.val)
    assert set(vals.tolist()) <= {0.25, 0.5, 1.0}
    deg = np.diff(c.rp)
    live = deg > 1
    assert set(np.unique(deg[live]).tolist()) <= {2, 3, 4}
    dist = np.abs(c.col.astype(np.int64) - rows)
    near = dist[np.repeat(live, deg)] <= 64
    assert 0.95 < near.mean() < 0.995


def test_dense_random_density():
    c = cg.dense_random(1024, 0.10, 0.005, 0.0, seed=4)
    assert abs(c.nnz / (1024 * 1024) - 0.10) < 0.005


def test_batched_packing():
    c = cg.batched(5, 1000, 4000, 1, 8, 0.01, 0.0, seed=8)
    assert c.num_instances == 5 and c.inst_off[-1] == c.n
    rows = _rows(c)
    inst = np.searchsorted(c.inst_off, rows, side="right") - 1
    tgt = np.searchsorted(c.inst_off, c.col, side="right") - 1
    assert np.array_equal(inst, tgt)
    for k in range(5):
        ck = c.instance(k)
        assert oracle.validate(ck.n, ck.rp, ck.col, ck.val) == (-1, 0)


def test_diag_dominant_matrices():
    for kw in (dict(density=0.05), dict(offdiag=300)):
        m = cg.diag_dominant(200, seed=9, **kw)
        rows = np.repeat(np.arange(m.n), np.diff(m.rp))
        assert np.all(m.val == np.round(m.val)) and np.all(m.val >= 1) and np.all(m.rhs >= 1)
        diag = rows == m.col
        assert np.array_equal(np.bincount(rows[diag], minlength=m.n), np.ones(m.n))
        off = np.bincount(rows[~diag], weights=m.val[~diag], minlength=m.n)
        assert np.all(m.val[diag] > off)
        for r in range(m.n):
            assert np.all(np.diff(m.col[m.rp[r]:m.rp[r + 1]]) > 0)
    assert cg.diag_dominant(200, offdiag=300, seed=9).nnz == 500
    b = cg.concat_matrices([cg.diag_dominant(30, density=0.2, seed=1), cg.diag_dominant(50, density=0.1, seed=2)])
    assert b.num_instances == 2 and b.instance(1).n == 50 and np.all(b.instance(1).col < 50)
