"""Gradient of the absorbed energy with respect to the vector-potential samples.

``AbsorbedEnergy.apply(a, domain, dt, precision, ckpt)`` propagates the
orbitals through ``len(a)`` Taylor-4 steps (``a``: float64 [n_steps] A_z
samples at the step midpoints, or [n_steps, 3]) and returns
    L = E0[psi_N] - E0[psi_0],   E0 = h^3 sum_n f_n <psi_n|H(A=0)|psi_n>,
the field-free energy gained over the pulse.  The backward pass runs the
adjoint recursion in the library,
    lambda_N = f H(0) psi_N,  lambda_k = U_k^H lambda_{k+1},
    dL/dA_k = 2 Re <lambda_{k+1}, dU_k/dA_k psi_k>,
with the forward states recomputed segment by segment from checkpoints taken
every ``ckpt`` steps.  Recomputation is bitwise reproducible, so a recomputed
segment that does not end on the next stored checkpoint means a corrupted
checkpoint, and backward raises.
"""
from __future__ import annotations

import torch

from . import api


def _full_field(a: torch.Tensor) -> torch.Tensor:
    if a.dim() == 1:
        full = torch.zeros(a.shape[0], 3, dtype=torch.float64, device=a.device)
        full[:, 2] = a
        return full.contiguous()
    return a.to(torch.float64).contiguous()


class AbsorbedEnergy(torch.autograd.Function):

    @staticmethod
    def forward(ctx, a: torch.Tensor, domain: api.Domain, dt: float, precision: str = "fp32",
                ckpt: int = 20, work: api.Workspace = None):
        if ckpt < 1:
            raise ValueError("ckpt must be >= 1")
        A = _full_field(a.detach())
        n = A.shape[0]
        dev = A.device
        work = work or api.Workspace.for_domains([domain], precision)
        psi = domain.psi.detach().clone()
        dom = domain.with_psi(psi)
        zero = torch.zeros(1, 3, dtype=torch.float64, device=dev)
        e0 = torch.zeros(1, dtype=torch.float64, device=dev)
        api.density([dom], zero, precision, work, [dict(energy=e0)])
        checkpoints = []
        for k0 in range(0, n, ckpt):
            k1 = min(n, k0 + ckpt)
            checkpoints.append(psi.clone())
            api.step([dom], A[k0:k1].contiguous(), dt, k1 - k0, precision, work)
        e1 = torch.zeros(1, dtype=torch.float64, device=dev)
        lam = torch.empty_like(psi)
        api.density([dom], zero, precision, work, [dict(energy=e1, hpsi_occ=lam)])
        ctx.save_for_backward(A, lam, psi, *checkpoints)
        ctx.meta = (domain, dt, precision, ckpt, work, a.dim())
        return (e1 - e0)[0]

    @staticmethod
    def backward(ctx, grad_out):
        A, lam_n, psi_end, *checkpoints = ctx.saved_tensors
        domain, dt, precision, ckpt, work, ndim = ctx.meta
        n = A.shape[0]
        lam = (lam_n * grad_out.to(lam_n.dtype)).contiguous()
        grad = torch.zeros(n, 3, dtype=torch.float64, device=A.device)
        for seg in range(len(checkpoints) - 1, -1, -1):
            k0 = seg * ckpt
            k1 = min(n, k0 + ckpt)
            # recompute psi_k0 .. psi_k1 from the checkpoint
            states = [checkpoints[seg].clone()]
            for k in range(k0, k1):
                nxt = states[-1].clone()
                api.step([domain.with_psi(nxt)], A[k:k + 1].contiguous(), dt, 1, precision, work)
                states.append(nxt)
            expect = checkpoints[seg + 1] if seg + 1 < len(checkpoints) else psi_end
            if not torch.equal(states[-1], expect):
                raise RuntimeError(f"recomputed segment {seg} (steps {k0}..{k1}) does not reproduce the "
                                   "stored state: corrupted checkpoint")
            for k in range(k1 - 1, k0 - 1, -1):
                api.adjoint_step([domain.with_psi(states[k - k0])], [lam], A[k:k + 1].contiguous(), dt,
                                 grad[k], precision, work)
        g = grad[:, 2] if ndim == 1 else grad
        return g, None, None, None, None, None


def absorbed_energy(a, domain, dt, precision="fp32", ckpt=20, work=None):
    return AbsorbedEnergy.apply(a, domain, dt, precision, ckpt, work)
