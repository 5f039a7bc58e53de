"""Shared test helpers: moving seeded synth domains onto the GPU and error
metrics.  (Not a test module.)"""
import numpy as np


def to_device(dom, precision, device="cuda"):
    """synth.Domain (FP64 numpy) -> paper_2509_00966_amd.Domain on the GPU."""
    import torch
    from paper_2509_00966_amd import Domain, complex_dtype, real_dtype

    cd, rd = complex_dtype(precision), real_dtype(precision)

    def t(x, dt):
        return torch.from_numpy(np.ascontiguousarray(x)).to(device=device, dtype=dt).contiguous()

    return Domain(tuple(dom.shape), dom.fd_order, dom.h, t(dom.psi, cd), t(dom.v_loc, rd),
                  t(dom.proj, cd), t(dom.d, rd), t(dom.occ, rd))


def oracle_inputs(dom, precision):
    """The FP64 oracle consumes the same rounded inputs the GPU path sees."""
    return dom if precision == "fp64" else dom.rounded(np.float32)


def rel_fro(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def a_tensor(a_mid, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a_mid, dtype=np.float64)).to(device)
