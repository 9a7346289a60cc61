"""Jacobi variants: the in-place (asynchronous) update of the single-vector
kernel (Section 5.1) and row sums by a backward segmented scan over the
stored entries (the entry-parallel product cited in Section 8).

Bars:
* certified solves (FP64 and FP32 inside FP64 refinement) within 1e-10 of the
  oracle's certified solution, on small chains, a batch, and a dense chain
  whose rows (~1,500 entries) span several scan windows of 1,024 entries;
* segmented scan, paper's rule: the same sweep count as the two-buffer sweep
  on row chunks (+-1: only the summation order differs) and iterates within
  1e-12 of it;
* in place, after a fixed number of sweeps from x = 0: componentwise between
  the Jacobi iterate with the same sweep count and x* (for A >= 0, b >= 0 the
  Jacobi map is monotone, so reading newer values can only move an iterate up
  towards x*, never past it);
* the variants are refused for BiCGStab and in combination."""
import numpy as np
import pytest

import chaingen as cg
import oracle
import paper_1210_6412_amd as rp
from tests import _gpu as G

pytestmark = pytest.mark.gpu

VARIANTS = {"in_place": dict(update=rp.RP_UPDATE_IN_PLACE),
            "segscan": dict(schedule=rp.RP_SCHEDULE_SEGSCAN)}


def _chains():
    out = [cg.worked_example(), cg.gamblers_ruin(200, 0.45)]
    for seed in range(4):
        rng = np.random.Generator(np.random.PCG64(9100 + seed))
        out.append(cg.random_small(int(rng.integers(50, 600)), rng, dmax=int(rng.integers(2, 14)),
                                   goal_frac=0.05, sink_frac=0.05, absorbing_goals=bool(seed % 2)))
    out.append(cg.concat([cg.random_sparse(3000 + 500 * i, 1, 16, 0.01, 0.01, cg.SEED_BASE + 40 + i)
                          for i in range(6)], name="batch of 6 random_sparse"))
    out.append(cg.dense_random(3000, 0.5, 0.01, 0.01, cg.SEED_BASE + 41))
    return out


@pytest.fixture(scope="module")
def chains():
    res = []
    for c in _chains():
        ref = oracle.solve(c.n, c.rp, c.col, c.val, c.goal, "bicgstab", tol=1e-12, stop_mode=1)
        res.append((c, ref))
    return res


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("precision", [rp.RP_FP64, rp.RP_FP32_REFINED])
def test_certified_matches_oracle(chains, variant, precision):
    for c, ref in chains:
        G.banner(f"jacobi {variant} certified prec={precision}: {c.name} n={c.n}")
        sys, cls, _ = G.precompute(c)
        assert np.array_equal(cls, ref.cls)
        x, info, code = G.solve(sys, "jacobi", tol=1e-10, stop=rp.RP_STOP_CERTIFIED, precision=precision,
                                **VARIANTS[variant])
        assert code == rp.binding.RP_OK, (c.name, info[:3])
        assert np.abs(x - ref.x).max() <= 1e-10, (c.name, np.abs(x - ref.x).max())
        assert all(i["error_bound"] <= 1e-10 for i in info if i["iterations"] > 0)


def test_segscan_paper_rule_matches_two_buffer(chains):
    for c, ref in chains:
        G.banner(f"jacobi segscan paper rule: {c.name} n={c.n}")
        sys, _, _ = G.precompute(c)
        kw = dict(tol=1e-8, stop=rp.RP_STOP_DELTA, precision=rp.RP_FP64)
        x0, i0, c0 = G.solve(sys, "jacobi", tiling=rp.RP_TILING_OFF, schedule=1, **kw)
        x1, i1, c1 = G.solve(sys, "jacobi", schedule=rp.RP_SCHEDULE_SEGSCAN, **kw)
        assert c0 == c1 == rp.binding.RP_OK
        for a, b in zip(i0, i1):
            assert abs(a["iterations"] - b["iterations"]) <= 1, (c.name, a["iterations"], b["iterations"])
        assert np.abs(x0 - x1).max() <= 1e-12, c.name


def test_in_place_between_jacobi_and_solution(chains):
    for c, ref in chains:
        sys, _, _ = G.precompute(c)
        for m in (3, 17):
            G.banner(f"jacobi in place, {m} sweeps: {c.name} n={c.n}")
            kw = dict(tol=0.0, max_iter=m, stop=rp.RP_STOP_DELTA, precision=rp.RP_FP64)
            xj, ij, cj = G.solve(sys, "jacobi", tiling=rp.RP_TILING_OFF, schedule=1, **kw)
            xi, ii, ci = G.solve(sys, "jacobi", update=rp.RP_UPDATE_IN_PLACE, **kw)
            assert cj in (rp.binding.RP_OK, rp.binding.RP_ERR_NOT_CONVERGED)
            assert ci in (rp.binding.RP_OK, rp.binding.RP_ERR_NOT_CONVERGED)
            # rounding only below; above, also the oracle's own certified
            # distance to x* (1e-12)
            assert (xi >= xj - 1e-13).all(), (c.name, m, (xj - xi).max())
            assert (xi <= ref.x + 2e-12).all(), (c.name, m, (xi - ref.x).max())


def test_variants_refused_where_undefined():
    c = cg.gamblers_ruin(50, 0.45)
    sys, _, _ = G.precompute(c)
    for kw in (dict(update=rp.RP_UPDATE_IN_PLACE), dict(schedule=rp.RP_SCHEDULE_SEGSCAN)):
        with pytest.raises(rp.RpError) as e:
            G.solve(sys, "bicgstab", **kw)
        assert e.value.code == rp.binding.RP_ERR_INVALID_ARG
    for kw in (dict(update=rp.RP_UPDATE_IN_PLACE, schedule=rp.RP_SCHEDULE_SEGSCAN), dict(update=7),
               dict(schedule=-3)):
        with pytest.raises(rp.RpError) as e:
            G.solve(sys, "jacobi", **kw)
        assert e.value.code == rp.binding.RP_ERR_INVALID_ARG
