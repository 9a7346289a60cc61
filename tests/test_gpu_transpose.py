"""The transposed reduced matrix (built by a stable sort by column) at its
edges, through the adjoint solve: a system with no off-diagonal entry at all
(λ_s = seed_s / d_s in closed form), a hub column that gathers an entry from
every other row next to thousands of empty columns, and both in one batch
with an ordinary random chain.  λ is compared with the closed form or with
the oracle's transposed solve (certified bounds on both sides), and a second,
independently built system gives the same λ and gradient bit for bit."""
import numpy as np
import pytest
import torch

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from tests import _gpu as G
from tests.test_gpu_tiles import _oracle_transposed_solve

pytestmark = pytest.mark.gpu


def _chain(rows, n, goal, name):
    """CSR chain from per-row lists of (column, probability), columns sorted."""
    rp_ = np.zeros(n + 1, dtype=np.int32)
    cols, vals = [], []
    for i, r in enumerate(rows):
        r = sorted(r)
        rp_[i + 1] = rp_[i] + len(r)
        cols += [c for c, _ in r]
        vals += [v for _, v in r]
    g = np.zeros(n, dtype=np.uint8)
    g[goal] = 1
    return cg.Chain(n, rp_, np.array(cols, dtype=np.int32), np.array(vals, dtype=np.float64), g,
                    np.array([0, n], dtype=np.int64), name)


def diagonal_chain(m, seed):
    """State 0 the goal, 1 a sink, 2..m+1 each to the goal, the sink and
    itself only: S_? has no transition between two of its states."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = [[(0, 1.0)], [(1, 1.0)]]
    for s in range(2, m + 2):
        a, b = rng.uniform(0.01, 0.4), rng.uniform(0.0, 0.4)
        rows.append([(0, a), (1, b), (s, 1.0 - a - b)])
    return _chain(rows, m + 2, [0], f"diagonal({m})")


def hub_chain(m, seed):
    """State 0 the goal, 1 a sink, 2 a hub; states 3..m+2 move to the hub,
    the goal, the sink and themselves, so the hub's column holds an entry of
    every other undecided row while their own columns stay empty."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows = [[(0, 1.0)], [(1, 1.0)], [(0, 0.5), (1, 0.2), (2, 0.3)]]
    for s in range(3, m + 3):
        h, a, b = rng.uniform(0.001, 0.01), rng.uniform(0.05, 0.3), rng.uniform(0.0, 0.05)
        rows.append([(0, a), (1, b), (2, h), (s, 1.0 - a - b - h)])
    return _chain(rows, m + 3, [0], f"hub({m})")


def _seed(c, cls):
    seed = np.zeros(c.n)
    for k in range(c.num_instances):
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        sq = np.nonzero(cls[lo:hi] == oracle.SQ)[0]
        seed[lo + sq[::7]] = 1.0
        seed[lo + sq[1::7]] = 0.25
    return seed


def _adjoint(c, method):
    sys, cls, _ = G.precompute(c)
    x, _, code = G.solve(sys, "bicgstab", tol=1e-12, stop=rp.RP_STOP_CERTIFIED)
    assert code == rp.binding.RP_OK
    seed = _seed(c, cls)
    lam, g, info, code = rp.rp_adjoint(G.ctx(), sys, torch.from_numpy(x).cuda(), torch.from_numpy(seed).cuda(),
                                       method, tol=1e-10, stop=rp.RP_STOP_CERTIFIED)
    assert code == rp.binding.RP_OK, info
    return lam.cpu().numpy(), g.cpu().numpy(), seed, info


@pytest.mark.parametrize("method", [0, 1])
def test_no_off_diagonal_entries(method):
    c = diagonal_chain(5000, seed=77)
    G.banner(f"transpose: {c.name} method {method}")
    lam, _, seed, info = _adjoint(c, method)
    d = 1.0 - c.val[c.rp[2:-1] + 2]  # the self-loop is each row's last entry
    want = np.zeros(c.n)
    want[2:] = seed[2:] / d
    assert np.abs(lam - want).max() <= 1e-10
    assert info[0]["error_bound"] <= 1e-10


@pytest.mark.parametrize("method", [0, 1])
def test_hub_column_and_batch(method):
    c = cg.concat([hub_chain(6000, seed=78), diagonal_chain(700, seed=79),
                   cg.random_sparse(4000, 1, 12, 0.02, 0.02, seed=80)], name="hub + diagonal + random")
    G.banner(f"transpose: {c.name} method {method}")
    lam, g, seed, info = _adjoint(c, method)
    for k in range(c.num_instances):
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        ck = c.instance(k)
        ref = oracle.solve(ck.n, ck.rp, ck.col, ck.val, ck.goal, "bicgstab", tol=1e-12, stop_mode=1)
        sq = np.nonzero(ref.cls == oracle.SQ)[0]
        rhs = np.zeros(ref.red.nq)
        rhs[ref.red.map[sq]] = seed[lo:hi][sq]
        lam_o, bound_o = _oracle_transposed_solve(oracle.transpose(ref.red), rhs)
        want = np.zeros(hi - lo)
        want[sq] = lam_o[ref.red.map[sq]]
        assert np.abs(lam[lo:hi] - want).max() <= 1e-10 + bound_o, k
        assert info[k]["error_bound"] <= 1e-10
    lam2, g2, _, _ = _adjoint(c, method)
    assert np.array_equal(lam, lam2) and np.array_equal(g, g2)
