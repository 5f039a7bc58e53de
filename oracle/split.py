"""hi+lo split operands for the mixed-precision projector products
(oracle; test infrastructure only).

Sec. VI.C describes GEMM modes that write each FP32 operand as a sum of
BF16 terms and accumulate the term products in FP32.  The two-term form used
here keeps the products hi*hi + hi*lo + lo*hi (the lo*lo term is dropped):
    x ~ hi + lo,  hi = round(x),  lo = round(x - hi)       (round-to-nearest-even)
for BF16 directly, and for FP16 after scaling the operand by a power of two
2^s chosen from its largest magnitude so that hi and lo stay in FP16's range.
The reference product evaluates the three term products exactly in FP64, which
isolates the operand rounding from accumulation order.
"""
import numpy as np

FP16_TOP_EXP = 14      # scaled operands satisfy max|x * 2^s| < 2^15


def round_bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def round_fp16(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def fp16_scale_exponent(max_abs):
    """s with max_abs * 2^s in [2^14, 2^15): s = 15 - e where max_abs = m 2^e, m in [0.5, 1)."""
    if max_abs == 0.0:
        return 0
    _, e = np.frexp(np.float32(max_abs))
    return int(FP16_TOP_EXP + 1 - e)


def split(x, mode, scale_exp=0):
    """(hi, lo) of a float32 array; for 'fp16' the parts are of x * 2^scale_exp."""
    x = np.asarray(x, dtype=np.float32)
    if mode == "bf16":
        hi = round_bf16(x)
        lo = round_bf16(x - hi)
    elif mode == "fp16":
        xs = (x * np.float32(2.0 ** scale_exp)).astype(np.float32)
        hi = round_fp16(xs)
        lo = round_fp16(xs - hi)
    else:
        raise ValueError(mode)
    return hi.astype(np.float64), lo.astype(np.float64)


def _parts(z):
    z = np.asarray(z, dtype=np.complex64)
    return np.ascontiguousarray(z.real, np.float32), np.ascontiguousarray(z.imag, np.float32)


def split_complex_matmul(a, b, mode, conj_a=False, sa=0, sb=0):
    """op(a) @ b for complex64 a, b with each real and imaginary part split into
    hi+lo and the three term products summed exactly in FP64.
    op(a) = a^H if conj_a else a.  Returns complex128."""
    ar, ai = _parts(a)
    br, bi = _parts(b)
    (arh, arl), (aih, ail) = split(ar, mode, sa), split(ai, mode, sa)
    (brh, brl), (bih, bil) = split(br, mode, sb), split(bi, mode, sb)

    def mm(x, y):
        return (x.T if conj_a else x) @ y

    def prod(xh, xl, yh, yl):
        return mm(xh, yh) + mm(xh, yl) + mm(xl, yh)

    rr = prod(arh, arl, brh, brl)
    ii = prod(aih, ail, bih, bil)
    ri = prod(arh, arl, bih, bil)
    ir = prod(aih, ail, brh, brl)
    if conj_a:       # conj(a)^T b: (ar - i ai)^T (br + i bi)
        out = (rr + ii) + 1j * (ri - ir)
    else:            # (ar + i ai)(br + i bi)
        out = (rr - ii) + 1j * (ri + ir)
    return out * 2.0 ** (-(sa + sb))


def _max_part(z):
    z = np.asarray(z, dtype=np.complex64)
    return float(max(np.abs(z.real).max(initial=0.0), np.abs(z.imag).max(initial=0.0)))


def apply_vnl_split(dom, u, mode, coef=1.0, occ_scale=False):
    """coef * B (D o P) with both projector products in two-term split form:
    P = h^3 split(B^H u), Q = coef D P (f_n) rounded to complex64, then split(B Q).
    For 'fp16' each operand gets the power-of-two scale of its own largest
    magnitude (real and imaginary parts together)."""
    b = np.asarray(dom.proj, dtype=np.complex64)
    u32 = np.asarray(u, dtype=np.complex64)
    sb = fp16_scale_exponent(_max_part(b)) if mode == "fp16" else 0
    su = fp16_scale_exponent(_max_part(u32)) if mode == "fp16" else 0
    p = dom.h ** 3 * split_complex_matmul(b, u32, mode, conj_a=True, sa=sb, sb=su)
    q = coef * dom.d[:, None] * p
    if occ_scale:
        q = q * dom.occ[None, :]
    q32 = q.astype(np.complex64)
    sq = fp16_scale_exponent(_max_part(q32)) if mode == "fp16" else 0
    return split_complex_matmul(b, q32, mode, sa=sb, sb=sq)
