"""Pins for the oracle's Chebyshev nodes and differentiation matrix.

The differentiation matrix must be exact on polynomials of degree <= p-1
(the defining property of spectral differentiation on p points), must
annihilate constants, and must match the hand-derived p = 3 matrix.
"""
import math
import os

import numpy as np
import pytest

from oracle import cheb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("p", [2, 3, 5, 8, 16, 21, 32, 42])
def test_nodes_are_chebyshev_extrema(p):
    t = cheb.nodes(p)
    assert t[0] == -1.0 and t[-1] == 1.0
    assert np.all(np.diff(t) > 0)
    np.testing.assert_array_equal(t, -t[::-1])          # exact symmetry
    ref = np.array([-math.cos(math.pi * k / (p - 1)) for k in range(p)])
    np.testing.assert_allclose(t, ref, rtol=0, atol=5e-16)


def test_golden_p3():
    D_ref = np.loadtxt(os.path.join(GOLDEN, "cheb_D_p3.txt"))
    np.testing.assert_allclose(cheb.diff_matrix(3), D_ref, rtol=0, atol=1e-15)


def test_p2_is_secant_slope():
    # linear interpolant through (-1, v0), (1, v1): slope (v1 - v0)/2 everywhere
    np.testing.assert_allclose(cheb.diff_matrix(2), [[-0.5, 0.5], [-0.5, 0.5]], atol=1e-16)


def _poly_exactness_error(D, t, p):
    err = 0.0
    for m in range(p):
        v = t ** m
        dv = m * t ** (m - 1) if m > 0 else np.zeros_like(t)
        err = max(err, np.max(np.abs(D @ v - dv)) / max(1.0, np.max(np.abs(dv))))
    return err


@pytest.mark.parametrize("p", [4, 8, 12, 16, 20, 24, 32])
def test_exact_on_polynomials(p):
    t = cheb.nodes(p)
    D = cheb.diff_matrix(p)
    assert _poly_exactness_error(D, t, p) < 1e-13 * p * p
    # second derivative through D @ D
    D2 = D @ D
    for m in range(p):
        v = t ** m
        d2 = m * (m - 1) * t ** (m - 2) if m > 1 else np.zeros_like(t)
        assert np.max(np.abs(D2 @ v - d2)) <= 1e-12 * p ** 4 * max(1.0, np.max(np.abs(d2)))


@pytest.mark.parametrize("p", [4, 9, 16, 32])
def test_annihilates_constants(p):
    D = cheb.diff_matrix(p)
    assert np.max(np.abs(D @ np.ones(p))) < 1e-12


def test_mutation_transposed_D_is_caught():
    """A transposed D (a plausible indexing slip) fails the exactness pin."""
    p = 8
    t = cheb.nodes(p)
    assert _poly_exactness_error(cheb.diff_matrix(p).T, t, p) > 1e-2


def test_mutation_wrong_endpoint_weight_is_caught():
    """Forgetting c_0 = c_{p-1} = 2 fails the exactness pin."""
    p = 8
    t = cheb.nodes(p)
    D = np.zeros((p, p))
    for k in range(p):
        for l in range(p):
            if k != l:
                D[k, l] = (-1.0) ** (k + l) / (t[k] - t[l])
        D[k, k] = -sum(D[k, l] for l in range(p) if l != k)
    assert _poly_exactness_error(D, t, p) > 1e-2


# -- corner extrapolation weights (used when the operator has a mixed term) --

@pytest.mark.parametrize("p", [4, 5, 8, 13, 20, 32])
def test_endpoint_weights_exact_to_degree_p_minus_3(p):
    lo, hi = cheb.endpoint_weights(p)
    t = cheb.nodes(p)[1:-1]
    for d in range(p - 2):                     # degree <= p-3: exact
        assert abs(lo @ t ** d - (-1.0) ** d) <= 1e-11 * max(1.0, np.abs(lo).sum())
        assert abs(hi @ t ** d - 1.0) <= 1e-11 * max(1.0, np.abs(hi).sum())
    # degree p-2 is not reproduced: t^(p-2) minus its interpolant at the p-2
    # nodes is the node polynomial prod_m (t - t_m), so the extrapolant at
    # -1 misses (-1)^(p-2) by exactly prod_m (-1 - t_m)
    d = p - 2
    miss = np.prod(-1.0 - t)
    assert abs((-1.0) ** d - lo @ t ** d - miss) <= 1e-11 * max(1.0, abs(miss))
    assert miss != 0.0


@pytest.mark.parametrize("p", [6, 9, 16])
def test_endpoint_weights_symmetry(p):
    lo, hi = cheb.endpoint_weights(p)
    assert np.allclose(hi, lo[::-1], rtol=0, atol=1e-12 * np.abs(lo).max())
    # the nearest node dominates: extrapolation from Lobatto interior points
    assert np.argmax(np.abs(lo)) == 0 and np.argmax(np.abs(hi)) == p - 3


def test_endpoint_weights_p4_by_hand():
    # p = 4: interior nodes -1/2, 1/2; the line through them at -1 gives
    # 3/2 v_1 - 1/2 v_2
    lo, hi = cheb.endpoint_weights(4)
    assert np.allclose(lo, [1.5, -0.5], atol=1e-15)
    assert np.allclose(hi, [-0.5, 1.5], atol=1e-15)
