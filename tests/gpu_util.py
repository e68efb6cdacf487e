"""Helpers for GPU parity tests (device transfer, relative errors)."""
import numpy as np


def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def dev(a):
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel_max(got, ref):
    """max |got - ref| / max |ref| (norm-wise relative error in the max norm)."""
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def params_of(w_or_model):
    import paper_2603_05194_amd as bec
    m = w_or_model
    if hasattr(m, "ndip"):
        return bec.make_params(m.gamma, m.beta, m.lam, m.ndip, m.omega)
    raise TypeError
