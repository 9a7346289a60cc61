"""Error paths of the C ABI that need a context: a non-finite starting point
is reported as RP_ERR_NONFINITE (x is still written), and sizes beyond the
library's 32-bit indices are refused with RP_ERR_TOO_LARGE before any device
memory is touched (the raw calls below pass host arrays only; the checks
come first)."""
import ctypes

import numpy as np
import pytest
import torch

import chaingen as cg
import paper_1210_6412_amd as rp
from paper_1210_6412_amd import binding as B
from tests import _gpu as G

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("stop", [rp.RP_STOP_DELTA, rp.RP_STOP_CERTIFIED])
@pytest.mark.parametrize("method", ["jacobi", "bicgstab"])
def test_nan_start_reports_nonfinite(stop, method):
    c = cg.random_sparse(3000, 1, 8, 0.02, 0.02, seed=9400)
    sys, cls, _ = G.precompute(c)
    x0 = torch.zeros(c.n, dtype=torch.float64, device="cuda")
    sq = np.nonzero(cls == rp.RP_SQ)[0]
    x0[int(sq[len(sq) // 2])] = float("nan")
    G.banner(f"nan x0: {method} stop={stop}")
    x, info, code = G.solve(sys, method, tol=1e-10, stop=stop, x0=x0, max_iter=10_000)
    assert code == B.RP_ERR_NONFINITE, info
    assert info[0]["status"] == B.RP_ERR_NONFINITE


def test_sizes_beyond_32_bit_indices_refused():
    lib = B.load_library()
    ctx = G.ctx()
    # small real device buffers stand in for the arrays: the size check comes
    # before any of them is read
    i32 = torch.zeros(16, dtype=torch.int32, device="cuda")
    f64 = torch.zeros(16, dtype=torch.float64, device="cuda")
    u8 = torch.zeros(16, dtype=torch.uint8, device="cuda")
    p_i, p_f, p_u = i32.data_ptr(), f64.data_ptr(), u8.data_ptr()
    big = (1 << 31) + 5
    off = (ctypes.c_int64 * 2)(0, big)
    out = ctypes.c_void_p()
    for n, nnz in ((big, 10), (1000, 1 << 31)):
        ch = B.RpChain(1, ctypes.cast(off, ctypes.POINTER(ctypes.c_int64)), n, nnz, p_i, p_i, p_f)
        code = lib.rp_precompute(ctx.handle, ctypes.byref(ch), p_u, 0, 0.0, None, ctypes.byref(out))
        assert code == B.RP_ERR_TOO_LARGE, (n, nnz)
        assert "too large" in rp.rp_last_error(ctx)
    code = lib.rp_matrix_system(ctx.handle, 1, off, big, 10, p_i, p_i, p_f, p_f, ctypes.byref(out))
    assert code == B.RP_ERR_TOO_LARGE
    torch.cuda.synchronize()
