"""rp_classify_noalloc (the state classes of rp_precompute with no device
allocation, working memory in the library's fixed per-GPU array) against
rp_precompute's class_out, bit for bit: two calls in a row, the second on a
smaller chain, so that the second call reuses the array left dirty by the
first; both search paths (one workgroup for small chains, pull steps above
32,768 states), both flag settings, a batch of instances, a bad chain and a
chain above the array's size."""
import numpy as np
import pytest
import torch

import chaingen as cg
import paper_1210_6412_amd as rp
from paper_1210_6412_amd import binding as B
from tests import _gpu as G

pytestmark = pytest.mark.gpu


def _both(c, flags):
    t = G.dev(c)
    want = torch.empty(c.n, dtype=torch.uint8, device="cuda")
    sys = rp.rp_precompute(G.ctx(), t["row_ptr"], t["col"], t["val"], t["goal"], t["off"], flags, 0.0, want)
    sys.close()
    got = torch.full((c.n,), 7, dtype=torch.uint8, device="cuda")
    B.rp_classify_noalloc(G.ctx(), t["row_ptr"], t["col"], t["val"], t["goal"], got, t["off"], flags)
    return got.cpu().numpy(), want.cpu().numpy()


@pytest.mark.parametrize("flags", [0, rp.RP_PROB0_ONLY])
def test_noalloc_classes_match_precompute_two_calls(flags):
    big = cg.concat([cg.random_sparse(60_000, 1, 8, 0.01, 0.01, seed=71), cg.gamblers_ruin(40_000, 0.45)])
    small = cg.random_sparse(3_000, 1, 8, 0.02, 0.02, seed=72)
    for c in (big, small):
        G.banner(f"no-alloc classes n={c.n} flags={flags}")
        got, want = _both(c, flags)
        assert np.array_equal(got, want), c.name
        assert set(np.unique(got)) <= {0, 1, 2}


def test_noalloc_bad_chain_matches_precompute():
    c = cg.random_sparse(2_000, 1, 8, 0.02, 0.02, seed=73)
    c.val[c.rp[1234] + 0] += 0.25  # row 1234 no longer sums to one
    t = G.dev(c)
    with pytest.raises(rp.RpError) as e1:
        rp.rp_precompute(G.ctx(), t["row_ptr"], t["col"], t["val"], t["goal"], t["off"], 0, 0.0)
    out = torch.empty(c.n, dtype=torch.uint8, device="cuda")
    with pytest.raises(rp.RpError) as e2:
        B.rp_classify_noalloc(G.ctx(), t["row_ptr"], t["col"], t["val"], t["goal"], out, t["off"])
    assert e1.value.code == e2.value.code == B.RP_ERR_BAD_CHAIN
    assert e1.value.message == e2.value.message
    # a good chain after the failure
    got, want = _both(cg.random_sparse(500, 1, 4, 0.05, 0.05, seed=74), 0)
    assert np.array_equal(got, want)


def test_noalloc_rejects_more_states_than_its_array():
    n = (1 << 23) + 64
    d = torch.device("cuda", 0)
    row_ptr = torch.arange(n + 1, dtype=torch.int32, device=d)
    col = torch.arange(n, dtype=torch.int32, device=d)
    val = torch.ones(n, dtype=torch.float64, device=d)
    goal = torch.zeros(n, dtype=torch.uint8, device=d)
    out = torch.empty(n, dtype=torch.uint8, device=d)
    with pytest.raises(rp.RpError) as e:
        B.rp_classify_noalloc(G.ctx(), row_ptr, col, val, goal, out)
    assert e.value.code == B.RP_ERR_TOO_LARGE
