"""Pins for mixed orders within one problem (oracle.mixed): the edge
interpolations, the reduction to the uniform scheme, brute force against
the full system, and spectral convergence to an exact solution.

Reading (the paper allows p per leaf from a fixed set but is silent on the
edges): a shared edge carries the nodes of its lower-order leaf; the other
leaf sees the polynomial through them (P) and returns its flux through the
polynomial through its own values (R)."""
import numpy as np
import pytest

from oracle import interface as itf
from oracle import mixed as mx
from paper_2211_14969_amd import inputs


@pytest.mark.parametrize("m_from,m_to", [(2, 5), (6, 10), (10, 6), (4, 4), (18, 26)])
def test_interp_matrix_exact_on_polynomials(m_from, m_to):
    P = mx.interp_matrix(m_from, m_to)
    s, t = mx.edge_nodes(m_from), mx.edge_nodes(m_to)
    for d in range(m_from):
        assert np.allclose(P @ s ** d, t ** d, rtol=0, atol=1e-12 * max(1.0, np.abs(P).sum(1).max()))


def test_interp_identity_and_round_trip():
    assert np.array_equal(mx.interp_matrix(7, 7), np.eye(7))
    for me, m in [(6, 10), (10, 18), (3, 4)]:
        # up to the finer nodes and back is exact (a degree me-1 polynomial)
        RP = mx.interp_matrix(m, me) @ mx.interp_matrix(me, m)
        assert np.allclose(RP, np.eye(me), atol=1e-11)


def test_minimum_rule_numbering():
    prob = inputs.mixed_tiny(n=3, orders=(6, 9))
    num = mx.numbering(3, 3, prob.orders)
    for e in range(num.m_edge.size):
        assert num.m_edge[e] in (4, 7)
    # an interior edge between a p = 6 and a p = 9 leaf carries 4 nodes
    t0, t1 = 0, 1                     # orders 6 and 9 (checkerboard)
    shared = set(num.leaf_edges[t0]) & set(num.leaf_edges[t1])
    assert len(shared) == 1 and num.m_edge[shared.pop()] == 4
    assert num.nunknown == sum(int(num.m_edge[e]) for e in range(num.m_edge.size)
                               if not num.dirichlet[e])


def test_uniform_orders_reduce_to_the_uniform_scheme():
    prob = inputs.mixed_tiny(n=4, orders=(10, 10))
    sol = mx.solve(prob)
    u = inputs.tiny(p=10, n=4)
    ref = itf.solve(u)
    assert abs(mx.relerr_true(sol, prob) - itf.relerr_true(ref, u)) <= 1e-12
    assert np.allclose(np.concatenate(sol.uint), ref.uint.ravel(), rtol=0, atol=1e-12)


@pytest.mark.parametrize("orders,n", [((6, 9), 3), ((8, 12, 16), 3)])
def test_brute_force_full_system(orders, n):
    prob = inputs.mixed_tiny(n=n, orders=orders)
    prob.f = lambda x, y, xp: xp.cos(2 * x) * y       # exercise h and w too
    leaves = mx.build_leaves(prob)
    sol = mx.solve(prob, leaves)
    A, b, _ = mx.full_system(prob, leaves)
    ub = np.linalg.solve(A, b)
    assert np.linalg.norm(mx.stack_full(sol) - ub) <= 1e-10 * np.linalg.norm(ub)


@pytest.mark.parametrize("orders,tol", [((10, 14), 3e-5), ((12, 16), 1e-7),
                                        ((14, 20), 1e-9), ((16, 24), 1e-12)])
def test_mixed_orders_converge(orders, tol):
    """sin(kappa x1) on 4 x 4 leaves, orders in a checkerboard (measured
    1.4e-5, 6.3e-8, 2.5e-10, 3.8e-13)."""
    prob = inputs.mixed_tiny(n=4, orders=orders)
    assert mx.relerr_true(mx.solve(prob), prob) < tol


def _transposed_flux_transfer(num, t):
    return [(e, P, P.T) for (e, P, R) in mx._side_maps_orig(num, t)]


def _truncated_trace(num, t):
    out = []
    for (e, P, R) in mx._side_maps_orig(num, t):
        Pz = np.zeros_like(P)
        k = min(P.shape)
        Pz[:k, :k] = np.eye(k)       # nodes matched by position, not by place
        out.append((e, Pz, Pz.T))
    return out


@pytest.mark.parametrize("mutant", [_transposed_flux_transfer, _truncated_trace])
def test_planted_interface_mistakes_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(mx, "_side_maps_orig", mx.side_maps, raising=False)
    monkeypatch.setattr(mx, "side_maps", mutant)
    prob = inputs.mixed_tiny(n=4, orders=(12, 16))
    assert mx.relerr_true(mx.solve(prob), prob) > 1e-5
