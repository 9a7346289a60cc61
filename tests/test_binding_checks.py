"""Argument checks of the Python binding, run on the CPU: a wrong x0,
lambda_out or grad_out is rejected before any pointer reaches the library
(a short or mistyped buffer would otherwise be read or written past its end
on the device).  CPU tensors stand in for device tensors by treating every
tensor as a CUDA tensor on device 0."""
from types import SimpleNamespace

import pytest
import torch


@pytest.fixture
def B(monkeypatch):
    import paper_1210_6412_amd.build as b
    if b.stale():
        b.build_library()
    from paper_1210_6412_amd import binding
    monkeypatch.setattr(binding, "_is_cuda", lambda t: True)
    monkeypatch.setattr(binding, "_device_index", lambda t: 0)

    def no_call(*a, **k):
        raise AssertionError("the library was called despite a bad argument")

    return binding, no_call


def _fakes(n=10, nnz=25):
    return SimpleNamespace(device=0, handle=None), SimpleNamespace(n=n, nnz=nnz, num_instances=1, handle=None)


def test_x0_dtype_checked_when_options_are_built(B):
    binding, _ = B
    with pytest.raises(TypeError, match="x0"):
        binding.rp_opts_default(x0=torch.zeros(10, dtype=torch.float32))


def test_x0_length_checked_against_the_system(B, monkeypatch):
    binding, no_call = B
    ctx, sys = _fakes()
    monkeypatch.setattr(binding, "load_library", lambda *a: SimpleNamespace(rp_jacobi=no_call,
                                                                           rp_opts_default=lambda o: None))
    o = binding.rp_opts_default(x0=torch.zeros(9, dtype=torch.float64))
    with pytest.raises(ValueError, match="x0 must have 10 elements"):
        binding.rp_jacobi(ctx, sys, x_out=torch.zeros(10, dtype=torch.float64), opts=o)


def test_x0_reference_kept_by_the_options(B):
    binding, _ = B
    o = binding.rp_opts_default(x0=torch.arange(10, dtype=torch.float64))
    assert o._x0_tensor is not None and o.x0 == o._x0_tensor.data_ptr()


def test_repointed_x0_rejected(B, monkeypatch):
    binding, no_call = B
    ctx, sys = _fakes()
    monkeypatch.setattr(binding, "load_library", lambda *a: SimpleNamespace(rp_bicgstab=no_call,
                                                                           rp_opts_default=lambda o: None))
    o = binding.rp_opts_default(x0=torch.zeros(10, dtype=torch.float64))
    o.x0 = o.x0 + 8
    with pytest.raises(ValueError, match="no longer points"):
        binding.rp_bicgstab(ctx, sys, x_out=torch.zeros(10, dtype=torch.float64), opts=o)


@pytest.mark.parametrize("bad, msg", [(torch.zeros(24, dtype=torch.float64), "grad_out must have 25"),
                                      (torch.zeros(25, dtype=torch.float32), "grad_out must have dtype"),
                                      (torch.zeros(50, dtype=torch.float64)[::2], "grad_out must be contiguous")])
def test_grad_out_checked(B, monkeypatch, bad, msg):
    binding, no_call = B
    ctx, sys = _fakes()
    monkeypatch.setattr(binding, "load_library", lambda *a: SimpleNamespace(rp_adjoint=no_call,
                                                                           rp_opts_default=lambda o: None))
    x = torch.zeros(10, dtype=torch.float64)
    with pytest.raises((TypeError, ValueError), match=msg):
        binding.rp_adjoint(ctx, sys, x, x.clone(), 0, grad_out=bad)


def test_lambda_out_checked(B, monkeypatch):
    binding, no_call = B
    ctx, sys = _fakes()
    monkeypatch.setattr(binding, "load_library", lambda *a: SimpleNamespace(rp_adjoint=no_call,
                                                                           rp_opts_default=lambda o: None))
    x = torch.zeros(10, dtype=torch.float64)
    with pytest.raises(ValueError, match="lambda_out must have 10"):
        binding.rp_adjoint(ctx, sys, x, x.clone(), 0, lambda_out=torch.zeros(11, dtype=torch.float64))


@pytest.mark.parametrize("bad, msg", [(torch.zeros(9, dtype=torch.int32), "label_out must have 10"),
                                      (torch.zeros(10, dtype=torch.int64), "label_out must have dtype")])
def test_scc_outputs_checked(B, monkeypatch, bad, msg):
    binding, no_call = B
    ctx, sys = _fakes()
    monkeypatch.setattr(binding, "load_library", lambda *a: SimpleNamespace(rp_scc=no_call))
    with pytest.raises((TypeError, ValueError), match=msg):
        binding.rp_scc(ctx, sys, label_out=bad, level_out=torch.zeros(10, dtype=torch.int32))


def test_scc_solve_output_checked(B, monkeypatch):
    binding, no_call = B
    ctx, sys = _fakes()
    monkeypatch.setattr(binding, "load_library", lambda *a: SimpleNamespace(rp_scc_solve=no_call,
                                                                           rp_opts_default=lambda o: None))
    with pytest.raises((TypeError, ValueError), match="x_out"):
        binding.rp_scc_solve(ctx, sys, x_out=torch.zeros(10, dtype=torch.float32))


def test_unknown_option_rejected(B, monkeypatch):
    binding, _ = B
    monkeypatch.setattr(binding, "load_library", lambda *a: SimpleNamespace(rp_opts_default=lambda o: None))
    with pytest.raises(TypeError, match="unknown option"):
        binding.rp_opts_default(graphs=1)
    o = binding.rp_opts_default(graph=1, update=binding.RP_UPDATE_IN_PLACE, schedule=binding.RP_SCHEDULE_SEGSCAN)
    assert (o.graph, o.update, o.schedule) == (1, 1, -2)
