"""Host-side checks of the C ABI: librp.so loads, exports every entry point
that include/rp.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rp.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_1210_6412_amd.build as b
    if b.stale():
        b.build_library()
    from paper_1210_6412_amd import binding
    return binding.load_library()


def test_header_declares_the_four_operations():
    names = _declared()
    for fn in ["rp_precompute", "rp_jacobi", "rp_bicgstab", "rp_adjoint"]:
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1210_6412_amd import binding
    names = _declared()
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTED) == names


def test_opts_default(lib):
    from paper_1210_6412_amd import binding
    o = binding.rp_opts_default()
    assert o.tol == 1e-10 and o.stop == binding.RP_STOP_CERTIFIED and o.precision == binding.RP_FP64
    assert o.max_iter == 10_000_000 and o.inner_tol == 1e-2 and o.max_refine == 60
    assert o.chunk == 32 and o.schedule == -1 and not o.x0


def test_null_arguments_rejected(lib):
    from paper_1210_6412_amd import binding as B
    P = ctypes.c_void_p
    assert lib.rp_precompute(None, None, None, 0, 0.0, None, None) == B.RP_ERR_INVALID_ARG
    assert lib.rp_jacobi(None, None, None, None, None) == B.RP_ERR_INVALID_ARG
    assert lib.rp_bicgstab(None, None, None, None, None) == B.RP_ERR_INVALID_ARG
    assert lib.rp_adjoint(None, None, 0, None, None, None, None, None, None) == B.RP_ERR_INVALID_ARG
    assert lib.rp_context_create(None, 0, None) == B.RP_ERR_INVALID_ARG
    assert lib.rp_system_sizes(None, None, None, None, None) == B.RP_ERR_INVALID_ARG
    assert lib.rp_last_error(None) == b"null context"


def test_context_without_gpu(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1210_6412_amd import binding as B
    h = ctypes.c_void_p()
    assert lib.rp_context_create(ctypes.byref(h), 0, None) == B.RP_ERR_INVALID_ARG
