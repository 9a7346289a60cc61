"""Forward solve plus gradient on the 256-chain batch (n log-uniform in
[1,000, 200,000], out-degree 1..8, 1% goal and 1% absorbing non-goal states
per chain, packed block-diagonally), FP32 sweeps inside FP64 refinement.

* The adjoint lambda and the gradient dx_init/dP(i,j) = lambda_i x_j on P's
  sparsity are compared element by element with the oracle on 12 sampled
  chains.
* Central finite differences (h = 1e-6, row not renormalised, partition
  fixed) on 64 uniformly sampled stored entries of every chain, among the
  entries (i, j) with i undecided and reachable from the chain's initial state
  inside S_? (found by a forward search, not by the adjoint) and
  2h < P_ij < 1 - 2h (P_ij + h must stay a probability).
  Each perturbed value x_init(P +- h e_ij) is obtained from the correction
  equation (I - A(+-h)) y = b(+-h) - (I - A(+-h)) x^ = r^ +- h x^_j e_i, solved
  for y itself (rp_solve_rhs), so the difference quotient
  (y+ - y-)_init / 2h is not lost to cancellation against x^.  Bar:
  |g_fd - g| / max(|g|, 1e-8) <= 1e-6.
"""
import numpy as np
import pytest
import scipy.sparse as sps
from scipy.sparse.csgraph import breadth_first_order
import torch

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from tests import _gpu as G

pytestmark = pytest.mark.gpu

H = 1e-6
PER_CHAIN = 64


@pytest.fixture(scope="module")
def base():
    c = cg.batched(256, 1_000, 200_000, 1, 8, 0.01, 0.01, cg.SEED_BASE + 5)
    G.banner(f"config 5 leaky gradient: K={c.num_instances} n={c.n} nnz={c.nnz}")
    t = G.dev(c)
    cls_d = torch.empty(c.n, dtype=torch.uint8, device="cuda")
    sys = rp.rp_precompute(G.ctx(), t["row_ptr"], t["col"], t["val"], t["goal"], t["off"], 0, 0.0, cls_d)
    cls = cls_d.cpu().numpy()
    x, info, code = rp.rp_bicgstab(G.ctx(), sys, tol=1e-12, stop=rp.RP_STOP_CERTIFIED,
                                   precision=rp.RP_FP32_REFINED)
    assert code == rp.binding.RP_OK, info[:3]
    s0 = np.zeros(c.num_instances, dtype=np.int64)
    seed = np.zeros(c.n)
    for k in range(c.num_instances):
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        sq = np.nonzero(cls[lo:hi] == oracle.SQ)[0]
        assert sq.size, k
        s0[k] = lo + sq[0]
        seed[s0[k]] = 1.0
    G.banner("config 5 leaky gradient: adjoint")
    lam, g, info, code = rp.rp_adjoint(G.ctx(), sys, x, torch.from_numpy(seed).cuda(), 1, tol=1e-10,
                                       stop=rp.RP_STOP_CERTIFIED, precision=rp.RP_FP32_REFINED)
    assert code == rp.binding.RP_OK, info[:3]
    return dict(c=c, t=t, sys=sys, cls=cls, x=x, xh=x.cpu().numpy(), s0=s0, seed=seed,
                lam=lam.cpu().numpy(), g=g.cpu().numpy())


def test_config5_adjoint_and_gradient_match_oracle(base):
    c, cls, lam, g = base["c"], base["cls"], base["lam"], base["g"]
    rng = np.random.Generator(np.random.PCG64(55))
    for k in sorted(rng.choice(c.num_instances, size=12, replace=False)):
        ck = c.instance(int(k))
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        G.banner(f"config 5 gradient vs oracle: chain {k} (n={ck.n})")
        ref = oracle.solve(ck.n, ck.rp, ck.col, ck.val, ck.goal, "bicgstab", tol=1e-12, stop_mode=1)
        assert np.array_equal(cls[lo:hi], ref.cls)
        assert np.abs(base["xh"][lo:hi] - ref.x).max() <= 1e-10
        sq = np.nonzero(ref.cls == oracle.SQ)[0]
        lam_o, _, _, rc = oracle.adjoint(ref, base["seed"][lo:hi], tol=1e-12)
        assert rc == oracle.OK
        want = np.zeros(hi - lo)
        want[sq] = lam_o[ref.red.map[sq]]
        scale = max(1.0, np.abs(lam_o).max())
        assert np.abs(lam[lo:hi] - want).max() <= 1e-10 * scale, k
        g_o = oracle.gradient(ck.n, ck.rp, ck.col, ref.cls, ref.red, lam_o, ref.x)
        e0, e1 = c.rp[lo], c.rp[hi]
        assert np.abs(g[e0:e1] - g_o).max() <= 1e-10 * scale, k


def _reachable_inside_sq(c, cls, s0):
    """States of S_? reachable from the initial states inside S_? (forward
    search over edges P > 0 between undecided states)."""
    rows = np.repeat(np.arange(c.n), np.diff(c.rp))
    keep = (c.val > 0) & (cls[rows] == oracle.SQ) & (cls[c.col] == oracle.SQ)
    src = np.concatenate([rows[keep], np.full(s0.size, c.n)])
    dst = np.concatenate([c.col[keep], s0])
    adj = sps.csr_matrix((np.ones(src.size, dtype=np.int8), (src, dst)), shape=(c.n + 1, c.n + 1))
    order = breadth_first_order(adj, c.n, directed=True, return_predecessors=False)
    reach = np.zeros(c.n + 1, dtype=bool)
    reach[order] = True
    return reach[:c.n], rows


def _base_residual(c, cls, xh):
    """r^ = b - (I - A) x^ on S_? (zero elsewhere), by the oracle, per chain."""
    r = np.zeros(c.n)
    for k in range(c.num_instances):
        ck = c.instance(k)
        lo, hi = c.inst_off[k], c.inst_off[k + 1]
        red = oracle.assemble(ck.n, ck.rp, ck.col, ck.val, cls[lo:hi])
        idx = np.nonzero(cls[lo:hi] == oracle.SQ)[0]
        xq = np.zeros(red.nq)
        xq[red.map[idx]] = xh[lo:hi][idx]
        rq, _ = oracle.residual(red, red.b, xq)
        r[lo + idx] = rq[red.map[idx]]
    return r


def test_config5_gradient_central_differences(base):
    c, cls, xh, s0, g = base["c"], base["cls"], base["xh"], base["s0"], base["g"]
    K = c.num_instances
    reach, rows = _reachable_inside_sq(c, cls, s0)
    inst = np.searchsorted(c.inst_off, rows, side="right") - 1
    rng = np.random.Generator(np.random.PCG64(64))
    picks = np.full((K, PER_CHAIN), -1, dtype=np.int64)
    ok = reach[rows] & (c.val > 2 * H) & (c.val < 1 - 2 * H)
    order = np.argsort(inst[ok], kind="stable")
    cand_all = np.nonzero(ok)[0][order]
    bounds = np.searchsorted(inst[cand_all], np.arange(K + 1))
    for k in range(K):
        cand = cand_all[bounds[k]:bounds[k + 1]]
        assert cand.size >= 8, (k, cand.size)
        m = min(PER_CHAIN, cand.size)
        picks[k, :m] = rng.choice(cand, size=m, replace=False)
    G.banner(f"config 5 FD: {int((picks >= 0).sum())} entries, base residual")
    rhat = torch.from_numpy(_base_residual(c, cls, xh)).cuda()
    xh_d = base["x"]
    t = base["t"]
    val_d = t["val"]
    base_val = val_d.clone()
    cls_d = torch.empty(c.n, dtype=torch.uint8, device="cuda")
    s0_d = torch.from_numpy(s0).cuda()
    fd = np.zeros((K, PER_CHAIN))
    for m in range(PER_CHAIN):
        live = np.nonzero(picks[:, m] >= 0)[0]
        e = torch.from_numpy(picks[live, m]).cuda()
        i = torch.from_numpy(rows[picks[live, m]]).cuda()
        j = torch.from_numpy(c.col[picks[live, m]].astype(np.int64)).cuda()
        vals = []
        for sgn in (1.0, -1.0):
            val_d.copy_(base_val)
            val_d[e] = base_val[e] + sgn * H
            sysp = rp.rp_precompute(G.ctx(), t["row_ptr"], t["col"], val_d, t["goal"], t["off"], 0, 1e-5, cls_d)
            assert torch.equal(cls_d.cpu(), torch.from_numpy(cls))
            rhs = rhat.clone()
            rhs[i] += sgn * H * xh_d[j]
            y, info, code = rp.rp_solve_rhs(G.ctx(), sysp, rhs, 1, tol=1e-24, stop=rp.RP_STOP_RESIDUAL,
                                            max_refine=200)
            assert code in (rp.binding.RP_OK, rp.binding.RP_ERR_NOT_CONVERGED), info[:3]
            vals.append(y[s0_d].cpu().numpy())
            sysp.close()
        fd[:, m] = (vals[0] - vals[1]) / (2 * H)
        if m % 8 == 7:
            G.banner(f"config 5 FD: {m + 1} of {PER_CHAIN} perturbation batches")
    val_d.copy_(base_val)
    worst = 0.0
    for k in range(K):
        for m in range(PER_CHAIN):
            ent = picks[k, m]
            if ent < 0:
                continue
            rel = abs(fd[k, m] - g[ent]) / max(abs(g[ent]), 1e-8)
            worst = max(worst, rel)
            assert rel <= 1e-6, (k, ent, fd[k, m], g[ent], rel)
    G.banner(f"config 5 FD: worst relative error {worst:.3e}")
