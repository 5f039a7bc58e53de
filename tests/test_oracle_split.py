"""Pins of the hi+lo operand splitting: the BF16 and FP16 rounding agrees with
torch's own conversions, the two-term representation error stays within its
bound, and the split complex product is within the expected distance of the
exact product."""
import numpy as np
import pytest
import torch

from oracle import split as S


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    x[:4] = [0.0, -0.0, 1.0, 3.0 * 2.0 ** -130]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(S.round_bf16(x), ref)


def test_fp16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(100000) * 100).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float16).to(torch.float32).numpy()
    assert np.array_equal(S.round_fp16(x), ref)


def test_bf16_two_term_error_bound():
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(50000) * 1e-2).astype(np.float32)
    hi, lo = S.split(x, "bf16")
    # hi has 8 significant bits, lo another 8: |x - hi - lo| <= 2^-17 |x| (+ ulp of lo)
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -16 * np.abs(x))
    assert np.median(np.abs(x - hi - lo) / np.abs(x)) < 2.0 ** -17


def test_fp16_scale_exponent_and_error():
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(50000) * 3e-3).astype(np.float32)
    s = S.fp16_scale_exponent(np.abs(x).max())
    assert 2.0 ** 14 <= np.abs(x).max() * 2.0 ** s < 2.0 ** 15
    hi, lo = S.split(x, "fp16", s)
    rec = (hi + lo) * 2.0 ** -s
    big = np.abs(x) > 1e-6
    assert np.all(np.abs(x - rec)[big] <= 2.0 ** -21 * np.abs(x[big]))


@pytest.mark.parametrize("mode,tol", [("bf16", 2.0 ** -14), ("fp16", 2.0 ** -19)])
def test_split_complex_product_close_to_exact(mode, tol):
    rng = np.random.default_rng(4)
    a = (rng.standard_normal((300, 20)) + 1j * rng.standard_normal((300, 20))).astype(np.complex64) * 0.01
    b = (rng.standard_normal((300, 12)) + 1j * rng.standard_normal((300, 12))).astype(np.complex64) * 0.02
    sa = S.fp16_scale_exponent(max(np.abs(a.real).max(), np.abs(a.imag).max())) if mode == "fp16" else 0
    sb = S.fp16_scale_exponent(max(np.abs(b.real).max(), np.abs(b.imag).max())) if mode == "fp16" else 0
    exact = a.astype(np.complex128).conj().T @ b.astype(np.complex128)
    got = S.split_complex_matmul(a, b, mode, conj_a=True, sa=sa, sb=sb)
    scale = np.abs(a).T @ np.abs(b)          # sum |a||b|: the natural error scale
    assert np.all(np.abs(got - exact) <= tol * scale)
    # non-conjugated form
    exact2 = a[:20].astype(np.complex128) @ b[:20].astype(np.complex128)
    got2 = S.split_complex_matmul(a[:20], b[:20], mode, sa=sa, sb=sb)
    assert np.all(np.abs(got2 - exact2) <= tol * (np.abs(a[:20]) @ np.abs(b[:20])))
    # and the plain BF16 (one-term) product would miss that bound
    if mode == "bf16":
        ar = S.round_bf16(a.real) + 1j * S.round_bf16(a.imag)
        br = S.round_bf16(b.real) + 1j * S.round_bf16(b.imag)
        one = ar.astype(np.complex128).conj().T @ br.astype(np.complex128)
        assert np.any(np.abs(one - exact) > tol * scale)
