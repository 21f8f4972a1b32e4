"""Compensated summation (paper Sec. 5.1.1, Algorithms FastTwoSum, Neumaier,
SecondOrderNeumaier and DoubleDoubleSum), plus the correctly rounded inner
product the oracle uses everywhere.

Python floats are IEEE-754 binary64 and every + below is one rounded
operation, so these are exact transcriptions of the arithmetic the paper
describes.
"""
import math

import numpy as np


def fast_two_sum(a, b):
    """(s, c) with s = fl(a + b) and s + c = a + b exactly.

    The error term is computed with the larger-magnitude operand first."""
    s = a + b
    if abs(a) >= abs(b):
        c = b - (s - a)
    else:
        c = a - (s - b)
    return s, c


def neumaier_sum(values):
    """Naive running sum plus the naively summed FastTwoSum error terms."""
    s = 0.0
    c = 0.0
    for v in values:
        s, e = fast_two_sum(s, float(v))
        c = c + e
    return s + c


def second_order_neumaier_sum(values):
    """Neumaier sum whose compensation terms are themselves compensated."""
    s = 0.0
    c = 0.0
    c2 = 0.0
    for v in values:
        s, e = fast_two_sum(s, float(v))
        c, e = fast_two_sum(c, e)
        c2 = c2 + e
    return s + (c + c2)


def double_double_sum(values):
    """Running sum kept as an unevaluated pair (s, c) of doubles."""
    s = 0.0
    c = 0.0
    for v in values:
        s, e = fast_two_sum(s, float(v))
        s, c = fast_two_sum(s, c + e)
    return s


def inner(a, b):
    """<a, b> = sum conj(a) b over all components, each of Re and Im summed with
    math.fsum (correctly rounded sum of the rounded products)."""
    prod = (np.conj(np.asarray(a)) * np.asarray(b)).ravel()
    return complex(math.fsum(prod.real.tolist()), math.fsum(prod.imag.tolist()))


def norm2(a):
    """||a||^2 = <a, a>, real."""
    a = np.asarray(a).ravel()
    return math.fsum((a.real * a.real).tolist()) + math.fsum((a.imag * a.imag).tolist())


def max_norm(a):
    """||a||_inf over real and imaginary parts (Sec. 4.2.2)."""
    a = np.asarray(a)
    return float(max(np.abs(a.real).max(initial=0.0), np.abs(a.imag).max(initial=0.0)))
