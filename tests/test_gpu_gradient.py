"""Gradient of the batched adjoint against central finite differences of GPU
solves (h = 1e-6, partition held fixed, rows not renormalised).

Every batched solve perturbs one entry in every chain at once (the chains are
independent), warm-starts from the unperturbed x and drives the FP64
residual down to rounding level, so the difference quotient is not swamped by
solve error.  Sampled entries are those with a gradient above 1e-2, where
rounding leaves a relative error far below the 1e-6 bar."""
import numpy as np
import pytest
import torch

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from tests import _gpu as G

pytestmark = pytest.mark.gpu

H = 1e-6


def _solve(c, val, x0, tol):
    d = torch.device("cuda", 0)
    cls = torch.empty(c.n, dtype=torch.uint8, device=d)
    sys = rp.rp_precompute(G.ctx(), torch.from_numpy(c.rp).to(d), torch.from_numpy(c.col).to(d),
                           torch.from_numpy(val).to(d), torch.from_numpy(c.goal).to(d), list(c.inst_off), 0, 1e-4,
                           cls)
    x, info, code = rp.rp_bicgstab(G.ctx(), sys, tol=tol, stop=rp.RP_STOP_RESIDUAL, max_refine=200,
                                   x0=None if x0 is None else torch.from_numpy(x0).to(d))
    assert code in (rp.binding.RP_OK, rp.binding.RP_ERR_NOT_CONVERGED), info
    return x.cpu().numpy(), cls.cpu().numpy(), sys


@pytest.mark.parametrize("adj_method", [0, 1])
def test_batched_gradient_central_differences(adj_method):
    rng = np.random.Generator(np.random.PCG64(2718))
    parts = [cg.random_sparse(int(rng.integers(1500, 3500)), 1, 8, 0.02, 0.02, seed=int(rng.integers(1 << 40)))
             for _ in range(6)]
    c = cg.concat(parts)
    G.banner(f"gradient FD K={c.num_instances} n={c.n} adjoint method {adj_method}")
    x, cls, sys = _solve(c, c.val, None, 1e-15)
    # seed: the first undecided state of every chain (x_init of each chain)
    seed = np.zeros(c.n)
    s0 = []
    for k in range(c.num_instances):
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        sq = np.nonzero(cls[lo:hi] == oracle.SQ)[0]
        assert sq.size
        s0.append(lo + sq[0])
        seed[lo + sq[0]] = 1.0
    lam, g, info, code = rp.rp_adjoint(G.ctx(), sys, torch.from_numpy(x).cuda(), torch.from_numpy(seed).cuda(),
                                       adj_method, tol=1e-10)
    assert code == rp.binding.RP_OK, info
    g = g.cpu().numpy()
    rows = np.repeat(np.arange(c.n), np.diff(c.rp))
    inst = np.searchsorted(c.inst_off, rows, side="right") - 1
    picks = []
    for k in range(c.num_instances):
        cand = np.nonzero((inst == k) & (cls[rows] == oracle.SQ) & (rows != c.col) & (c.val > 2 * H) & (c.val < 1 - 2 * H)
                          & (np.abs(g) > 1e-2))[0]
        assert cand.size >= 4
        picks.append(rng.choice(cand, size=4, replace=False))
    picks = np.array(picks)  # [K, 4]
    checked = 0
    for m in range(picks.shape[1]):
        xs = []
        for sign in (+1, -1):
            val = c.val.copy()
            val[picks[:, m]] += sign * H
            xp, cp, sp = _solve(c, val, x, 1e-15)
            assert np.array_equal(cp, cls)
            xs.append(xp)
        for k in range(c.num_instances):
            e = picks[k, m]
            fd = (xs[0][s0[k]] - xs[1][s0[k]]) / (2 * H)
            rel = abs(fd - g[e]) / abs(g[e])
            assert rel <= 1e-6, (k, e, fd, g[e], rel)
            checked += 1
    assert checked == picks.size
