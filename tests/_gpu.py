"""Helpers shared by the GPU tests: move a chaingen chain to the device and
run the library on it through the C ABI binding."""
import numpy as np
import torch

import paper_1210_6412_amd as rp

_CTX = {}


def ctx():
    if "c" not in _CTX:
        _CTX["c"] = rp.rp_context_create(0)
    return _CTX["c"]


def dev(chain):
    d = torch.device("cuda", 0)
    return dict(row_ptr=torch.from_numpy(chain.rp).to(d), col=torch.from_numpy(chain.col).to(d),
                val=torch.from_numpy(chain.val).to(d), goal=torch.from_numpy(chain.goal).to(d),
                off=[int(v) for v in chain.inst_off])


def precompute(chain, flags=0, rowsum_tol=0.0):
    t = dev(chain)
    cls = torch.empty(chain.n, dtype=torch.uint8, device="cuda")
    sys = rp.rp_precompute(ctx(), t["row_ptr"], t["col"], t["val"], t["goal"], t["off"], flags, rowsum_tol, cls)
    return sys, cls.cpu().numpy(), t


def solve(sys, method, **kw):
    fn = rp.rp_jacobi if method == "jacobi" else rp.rp_bicgstab
    x, info, code = fn(ctx(), sys, **kw)
    return x.cpu().numpy(), info, code


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
