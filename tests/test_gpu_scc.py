"""Strongly connected components of S_? on the GPU (rp_scc) against the
oracle's Tarjan decomposition, and the solve by components in reverse
topological order (rp_scc_solve).

Bars: labels (smallest state index of the component) and levels bit-exact
per state; component counts equal; the level solve then certified within
1e-10 of the oracle's solution, with one substitution pass per level of
one-state components and Jacobi sweeps exactly on the states of the larger
components."""
import numpy as np
import pytest

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from tests import _gpu as G

pytestmark = pytest.mark.gpu


def _chains():
    out = [cg.worked_example(), cg.gamblers_ruin(100, 0.45), cg.ladder(300)]
    for seed in range(6):
        rng = np.random.Generator(np.random.PCG64(9300 + seed))
        out.append(cg.random_small(int(rng.integers(20, 800)), rng, dmax=int(rng.integers(1, 4)),
                                   goal_frac=0.1, sink_frac=0.1, zero_frac=0.1 if seed % 2 else 0.0,
                                   absorbing_goals=bool(seed % 2)))
    out.append(cg.layered(8, 50, transient=40, seed=cg.SEED_BASE + 70))
    out.append(cg.layered(20, 3000, transient=5000, seed=cg.SEED_BASE + 71))
    out.append(cg.concat([cg.layered(6, 400, transient=300, seed=cg.SEED_BASE + 80 + i) for i in range(5)]
                         + [cg.random_sparse(5000, 1, 4, 0.05, 0.05, cg.SEED_BASE + 90)], name="mixed batch"))
    out.append(cg.CONFIGS[2]())
    return out


def _expected(c):
    """Oracle labels / levels per state (per instance), in state numbering."""
    lab = np.full(c.n, -1, dtype=np.int64)
    lev = np.full(c.n, -1, dtype=np.int64)
    sizes = []
    refs = []
    for k in range(c.num_instances):
        ck = c.instance(k)
        lo = int(c.inst_off[k])
        ref = oracle.solve(ck.n, ck.rp, ck.col, ck.val, ck.goal, "bicgstab", tol=1e-12, stop_mode=1)
        refs.append(ref)
        red = ref.red
        l_red, v_red, _ = oracle.scc(red)
        full_of = np.nonzero(red.map >= 0)[0]
        sq = full_of
        lab[lo + sq] = lo + full_of[l_red[red.map[sq]]]
        lev[lo + sq] = v_red[red.map[sq]]
        sizes.append(np.bincount(l_red) if red.nq else np.zeros(0, np.int64))
    return lab, lev, sizes, refs


@pytest.fixture(scope="module")
def cases():
    return [(c,) + _expected(c) for c in _chains()]


def test_labels_and_levels_bit_exact(cases):
    for c, lab, lev, sizes, _ in cases:
        G.banner(f"scc labels: {c.name} n={c.n}")
        sys, _, _ = G.precompute(c)
        gl, gv, info = rp.rp_scc(G.ctx(), sys)
        gl, gv = gl.cpu().numpy(), gv.cpu().numpy()
        assert np.array_equal(gl, lab), c.name
        assert np.array_equal(gv, lev), c.name
        allsz = np.concatenate([s[s > 0] for s in sizes]) if sizes else np.zeros(0)
        assert info["components"] == allsz.size, (c.name, info)
        assert info["cyclic_components"] == int((allsz > 1).sum()), (c.name, info)
        assert info["largest"] == (int(allsz.max()) if allsz.size else 0), (c.name, info)
        if (lev >= 0).any():
            assert info["levels"] == int(lev.max()) + 1, (c.name, info)


@pytest.mark.parametrize("precision", [rp.RP_FP64, rp.RP_FP32_REFINED])
def test_solve_by_components_matches_oracle(cases, precision):
    for c, lab, lev, sizes, refs in cases:
        G.banner(f"scc solve prec={precision}: {c.name} n={c.n}")
        sys, _, _ = G.precompute(c)
        x, info, code, si = rp.rp_scc_solve(G.ctx(), sys, tol=1e-10, stop=rp.RP_STOP_CERTIFIED,
                                            precision=precision)
        assert code == rp.binding.RP_OK, (c.name, info[:3])
        x = x.cpu().numpy()
        for k, ref in enumerate(refs):
            lo, hi = int(c.inst_off[k]), int(c.inst_off[k + 1])
            assert np.abs(x[lo:hi] - ref.x).max() <= 1e-10, (c.name, k)
        cyc_rows = int(sum(s[s > 1].sum() for s in sizes))
        assert si["jacobi_rows"] == cyc_rows, (c.name, si)
        assert si["substitution_rows"] >= int((lab >= 0).sum()) - cyc_rows, (c.name, si)
        # levels with a component of several states take sweeps, exactly those
        sq = lab >= 0
        labs, cnt = np.unique(lab[sq], return_counts=True)
        big = np.isin(lab[sq], labs[cnt > 1])
        assert si["jacobi_levels"] == np.unique(lev[sq][big]).size, (c.name, si)
        assert si["substitution_levels"] <= si["levels"], (c.name, si)


def test_ladder_needs_no_sweep():
    """An acyclic S_?: every level is one substitution pass and the result is
    exact (x_i = p^(n-i)) before any refinement."""
    n, p = 2000, 0.9
    c = cg.ladder(n, p)
    sys, _, _ = G.precompute(c)
    x, info, code, si = rp.rp_scc_solve(G.ctx(), sys, tol=1e-10, stop=rp.RP_STOP_CERTIFIED)
    assert code == rp.binding.RP_OK
    assert si["jacobi_levels"] == 0 and si["substitution_levels"] == n and si["levels"] == n
    x = x.cpu().numpy()[:n]
    want = p ** (n - np.arange(n, dtype=np.float64))
    assert np.abs(x - want).max() <= 1e-14
    assert info[0]["iterations"] == 0


def test_matrix_systems_refused():
    m = cg.diag_dominant(50, density=0.1)
    import torch
    t = [torch.from_numpy(a).cuda() for a in (m.rp, m.col, m.val, m.rhs)]
    sys = rp.rp_matrix_system(G.ctx(), *t, list(m.inst_off))
    with pytest.raises(rp.RpError) as e:
        rp.rp_scc(G.ctx(), sys)
    assert e.value.code == rp.binding.RP_ERR_INVALID_ARG
