"""Finite differences of the detection loss, taken only where it is smooth.

The map from (lambda_k, beta, y) to the LLRs is piecewise smooth: it switches
pieces where a projection onto the box starts or stops clipping (equation
eq:projection) and where a max-log minimiser changes (equation
eq:exactinversellr).  A central difference across such a switch is not a
derivative, so every difference below is taken across a step over which the
oracle's active set (oracle.active_set: the side of the box of every projection
and the two minimisers of every bit) does not change.  The step starts at
h = 1e-6 max(1, |theta|) and is halved up to four times; a coordinate whose
active set still changes is excluded, and the caller reports how many were.
"""

import numpy as np

HALVINGS = 4


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def central(evaluate, theta0, h0=None):
    """evaluate(theta) -> (loss, active set tuple).  Returns the central difference
    at theta0, or None when the active set changes across every step tried."""
    h = 1e-6 * max(1.0, abs(theta0)) if h0 is None else h0
    for _ in range(HALVINGS + 1):
        lp, ap = evaluate(theta0 + h)
        lm, am = evaluate(theta0 - h)
        if _same(ap, am):
            return (lp - lm) / (2.0 * h)
        h /= 2.0
    return None


def one_sided(evaluate, theta0, h0=None):
    """Second-order forward difference (-3 f(0) + 4 f(h) - f(2h)) / 2h for a coordinate
    on the edge of its domain (a regulariser at 0); the active set must agree at all
    three points.  None when it never does."""
    h = 1e-6 * max(1.0, abs(theta0)) if h0 is None else h0
    l0, a0 = evaluate(theta0)
    for _ in range(HALVINGS + 1):
        l1, a1 = evaluate(theta0 + h)
        l2, a2 = evaluate(theta0 + 2.0 * h)
        if _same(a0, a1) and _same(a0, a2):
            return (-3.0 * l0 + 4.0 * l1 - l2) / (2.0 * h)
        h /= 2.0
    return None


def bce_sum(L, bits):
    """Sum over bits of softplus(L) - bit * L (P(bit = 1) = sigmoid(L)), formed as
    softplus(-L) for bit 1, which does not cancel when the bit is confidently right."""
    return float(np.sum(np.logaddexp(0.0, np.where(bits != 0, -L, L))))
