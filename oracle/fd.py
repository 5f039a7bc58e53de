"""Central finite-difference weights (oracle; test infrastructure only).

Sec. V.A.5 represents the orbitals on a finite-difference mesh; the order of
the Laplacian and gradient is a workload parameter (2, 4 or 6).  These are the
standard central-difference weights: for the second derivative
    f''(x) ~ (1/h^2) [c0 f(x) + sum_m c_m (f(x+mh) + f(x-mh))],
and for the first derivative
    f'(x)  ~ (1/h)   sum_m a_m (f(x+mh) - f(x-mh)).
The gradient is taken at the same order as the Laplacian.
"""
from fractions import Fraction as F

SECOND = {
    2: (F(-2), F(1)),
    4: (F(-5, 2), F(4, 3), F(-1, 12)),
    6: (F(-49, 18), F(3, 2), F(-3, 20), F(1, 90)),
}

FIRST = {
    2: (F(1, 2),),
    4: (F(2, 3), F(-1, 12)),
    6: (F(3, 4), F(-3, 20), F(1, 60)),
}


def radius(order: int) -> int:
    """Stencil half-width r = order / 2."""
    if order not in SECOND:
        raise ValueError(f"unsupported finite-difference order {order}")
    return order // 2


def second(order: int):
    """(c0, c1, ..., cr) as floats."""
    return tuple(float(c) for c in SECOND[order])


def first(order: int):
    """(a1, ..., ar) as floats."""
    return tuple(float(a) for a in FIRST[order])
