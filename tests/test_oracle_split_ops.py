"""The oracle's split-form nonlocal operator stays within the two-term
rounding bound of the exact FP64 operator, and reduces to it when the operands
are exactly representable."""
import numpy as np
import pytest

from oracle import hamiltonian as H
from oracle import split as S
from synth import make_domain


@pytest.mark.parametrize("mode,tol", [("bf16", 2.0 ** -13), ("fp16", 2.0 ** -18)])
def test_split_vnl_close_to_exact(mode, tol):
    dom = make_domain(3, (9, 10, 8), 5, 3, proj_per_atom=8, h=0.4, fd_order=4).rounded(np.float32)
    exact = H.apply_vnl(dom, dom.psi)
    got = S.apply_vnl_split(dom, dom.psi, mode)
    assert np.linalg.norm(got - exact) <= tol * np.linalg.norm(exact)
    assert np.linalg.norm(got - exact) > 0


def test_split_vnl_exact_on_representable_operands():
    dom = make_domain(4, (8, 8, 8), 3, 2, proj_per_atom=4, h=0.5, fd_order=2)
    # operands that bf16 holds exactly: small-integer multiples of powers of two
    rng = np.random.default_rng(0)
    dom.proj = (rng.integers(-8, 9, dom.proj.shape) + 1j * rng.integers(-8, 9, dom.proj.shape)) / 64.0
    dom.psi = (rng.integers(-8, 9, dom.psi.shape) + 1j * rng.integers(-8, 9, dom.psi.shape)) / 32.0
    dom.d = np.array([0.5, -0.25, 1.0, 0.125, -1.0, 0.75, 0.0, 0.5])
    got = S.apply_vnl_split(dom, dom.psi, "bf16")
    exact = H.apply_vnl(dom, dom.psi)
    # P = h^3 B^H psi is exact in FP64 and representable in FP32; Q = D P as well
    assert np.abs(got - exact).max() <= 1e-6 * np.abs(exact).max()
