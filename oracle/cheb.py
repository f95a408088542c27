"""Chebyshev points and the spectral differentiation matrix (oracle; test
infrastructure only).

Sec. 2 of the paper places a p x p tensor grid of Chebyshev points on each
leaf and enforces the PDE by spectral differentiation.  The paper does not
say which Chebyshev family; the leaf edges must carry nodes, so these are the
Chebyshev extreme (Lobatto) points, p per direction, endpoints included.

The differentiation matrix is the classical one for polynomial interpolation
at these points (Trefethen, Spectral Methods in MATLAB, ch. 6): with
c_0 = c_{p-1} = 2 and c_k = 1 otherwise,

    D[k, l] = (c_k / c_l) (-1)^(k+l) / (t_k - t_l),     k != l,
    D[k, k] = -sum_{l != k} D[k, l]       (rows of D annihilate constants).

With a mixed derivative in the operator the interior rows reach the four
leaf corners, which carry no unknown.  Each corner value is then taken from
its two edges: the degree-(p-3) polynomial through an edge's p-2 nodes
(endpoints excluded) is evaluated at the corner end (`endpoint_weights`),
and the two edges' values are averaged (a reading: the paper does not say
how corners are treated).
"""
from __future__ import annotations

import math

import numpy as np


def nodes(p: int) -> np.ndarray:
    """The p Chebyshev extreme points on [-1, 1] in increasing order,
    t_k = -cos(pi k / (p - 1)), evaluated as a sine so that the set is
    exactly symmetric about 0."""
    if p < 2:
        raise ValueError("need p >= 2")
    n = p - 1
    return np.array([math.sin(math.pi * (2 * k - n) / (2.0 * n)) for k in range(p)],
                    dtype=np.float64)


def diff_matrix(p: int) -> np.ndarray:
    """D with (D v)_k = q'(t_k), q the degree-(p-1) interpolant of v at nodes(p)."""
    t = nodes(p)
    c = np.ones(p)
    c[0] = c[-1] = 2.0
    D = np.zeros((p, p), dtype=np.float64)
    for k in range(p):
        for l in range(p):
            if k != l:
                sign = -1.0 if (k + l) % 2 else 1.0
                D[k, l] = (c[k] / c[l]) * sign / (t[k] - t[l])
    for k in range(p):
        D[k, k] = -sum(D[k, l] for l in range(p) if l != k)
    return D


def endpoint_weights(p: int):
    """Weights (lo, hi), each of length p-2: for values v_1..v_{p-2} at the
    interior nodes t_1..t_{p-2}, sum_k lo[k] v_k and sum_k hi[k] v_k are the
    degree-(p-3) interpolant evaluated at t = -1 and t = +1.  Lagrange basis
    polynomials of the interior nodes: l_k(x) = prod_{m != k} (x - t_m)/(t_k - t_m)."""
    t = nodes(p)[1:-1]
    n = t.size
    lo = np.empty(n)
    hi = np.empty(n)
    for k in range(n):
        a = b = 1.0
        for m in range(n):
            if m != k:
                a *= (-1.0 - t[m]) / (t[k] - t[m])
                b *= (1.0 - t[m]) / (t[k] - t[m])
        lo[k] = a
        hi[k] = b
    return lo, hi
