"""Pins for the oracle's full pipeline: condense -> assemble -> solve -> recover.

* exact Helmholtz solutions: sin(kappa x1) (the tiny workload), the paper's
  J0(kappa |x - (-0.1, 0.5)|) (Sec. 3, eq. (constant_coeff_helm)) and the
  plane wave on the quarter annulus;
* brute force: the dense solve of the full unreduced collocation system
  equals the condensed route (static condensation is exact block
  elimination);
* the spectral convergence rate in p;
* the Dirichlet-to-Neumann property of S for plane waves;
* the paper's accuracy level at 10 points per wavelength (Sec. 3.1).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.special

from oracle import interface as itf
from oracle import leaf as lf
from paper_2211_14969_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def j0_problem(p, n, kappa, centre=(-0.1, 0.5)):
    cx, cy = centre
    sol = lambda x, y, xp: scipy.special.j0(kappa * np.sqrt((x - cx) ** 2 + (y - cy) ** 2))
    return inputs.Problem(name="j0", nx=n, ny=n, p=p, kappa=kappa,
                          coef={"k2b": lambda x, y, xp: xp.zeros_like(x) + kappa * kappa},
                          g=sol, exact=sol)


def test_tiny_workload_exact_solution():
    prob = inputs.tiny()
    assert (prob.nx, prob.ny, prob.p, prob.kappa) == (4, 4, 8, 10.0)
    sol = itf.solve(prob)
    assert sol.num.nunknown == 144
    assert itf.relerr_true(sol, prob) < 1e-3


@pytest.mark.parametrize("p,tol", [(8, 1e-3), (12, 1e-7), (16, 1e-10)])
def test_j0_exact_solution(p, tol):
    prob = j0_problem(p, 4, 10.0)
    assert itf.relerr_true(itf.solve(prob), prob) < tol


@pytest.mark.parametrize("p,tol", [(8, 2e-2), (12, 1e-4), (16, 1e-7)])
def test_annulus_plane_wave(p, tol):
    prob = inputs.annulus(p=p, ntheta=4, nr=2, kappa=10.0)
    assert itf.relerr_true(itf.solve(prob), prob) < tol


@pytest.mark.parametrize("maker", [lambda: inputs.tiny(),
                                   lambda: inputs.single_bump(p=10, n=3, kappa=20.0),
                                   lambda: inputs.annulus(p=8, ntheta=3, nr=2, kappa=12.0),
                                   lambda: inputs.multi_bump(p=9, n=2, kappa=30.0),
                                   lambda: inputs.curved(p=9, n=2, kappa=6.0)])
def test_brute_force_full_system(maker):
    prob = maker()
    leaves = itf.build_leaves(prob)
    sol = itf.solve(prob, leaves)
    A, b, num = itf.full_system(prob, leaves)
    u_brute = np.linalg.solve(A, b)
    u_cond = itf.stack_full(sol)
    assert np.linalg.norm(u_cond - u_brute) <= 1e-10 * np.linalg.norm(u_brute)
    assert itf.relerr_res(A, b, u_cond) < 1e-10


def test_brute_force_with_body_load():
    """f != 0 exercises h and w: manufactured u = sin(3x) cos(2y) + x y with
    b == 1 and kappa = 4, f = -Lap u - kappa^2 u."""
    kappa = 4.0
    u = lambda x, y, xp: xp.sin(3 * x) * xp.cos(2 * y) + x * y
    f = lambda x, y, xp: (13.0 - kappa ** 2) * xp.sin(3 * x) * xp.cos(2 * y) - kappa ** 2 * x * y
    prob = inputs.Problem(name="mf", nx=3, ny=2, p=12, kappa=kappa,
                          coef={"k2b": lambda x, y, xp: xp.zeros_like(x) + kappa ** 2},
                          g=u, exact=u, f=f)
    leaves = itf.build_leaves(prob)
    sol = itf.solve(prob, leaves)
    A, b, _ = itf.full_system(prob, leaves)
    u_brute = np.linalg.solve(A, b)
    assert np.linalg.norm(itf.stack_full(sol) - u_brute) <= 1e-10 * np.linalg.norm(u_brute)
    assert itf.relerr_true(sol, prob) < 1e-8


def test_spectral_convergence_in_p():
    errs = {}
    for p in range(6, 18, 2):
        prob = inputs.tiny(p=p)
        errs[p] = itf.relerr_true(itf.solve(prob), prob)
    for p in range(6, 14, 2):
        if errs[p] < 1e-10:
            break
        assert errs[p + 2] <= 0.1 * errs[p], errs
    assert errs[16] <= 1e-10, errs


@pytest.mark.parametrize("p", [16, 20])
def test_dtn_plane_waves(p):
    """b == 1: S maps the trace of cos(kappa x.d) to its outward normal derivative."""
    box = (0.25, 0.5, 0.5, 0.75)
    X, Y = lf.grid(box, p)
    B = lf.flat(p, lf.boundary_nodes(p))
    m = p - 2
    for kappa in (5.0, 10.0):
        c = lf.condense(lf.blocks(box, p, {"k2b": np.full(p * p, kappa ** 2)}))
        for phi in np.linspace(0.0, 2 * np.pi, 7):
            d = (math.cos(phi), math.sin(phi))
            ph = kappa * (X * d[0] + Y * d[1])
            u, ux, uy = np.cos(ph), -kappa * d[0] * np.sin(ph), -kappa * d[1] * np.sin(ph)
            dn = np.concatenate([-ux[B[:m]], ux[B[m:2 * m]], -uy[B[2 * m:3 * m]], uy[B[3 * m:]]])
            assert np.linalg.norm(c.S @ u[B] - dn) <= 1e-10 * np.linalg.norm(dn)


@pytest.mark.slow
def test_paper_accuracy_level_p22_10ppw():
    """At 10 points per wavelength and p = 22 the paper reports 6 true digits
    for problems of up to 5 million nodes; on a smaller grid (less pollution)
    the oracle must do at least as well."""
    lv = json.load(open(os.path.join(GOLDEN, "paper_levels.json")))
    digits = lv["p22_true_digits_10ppw"]["value"]
    p, n = 22, 4
    N = n * n * p * p
    kappa = 2 * math.pi * math.sqrt(N) / 10.0      # 10 points per wavelength
    prob = j0_problem(p, n, kappa, centre=tuple(lv["j0_source_point"]["value"]))
    err = itf.relerr_true(itf.solve(prob), prob)
    assert err <= 10.0 ** (-digits + 1)


def test_planted_flux_sign_breaks_brute_force_agreement(monkeypatch):
    """A sign slip in one edge's flux rows makes the reduced system wrong;
    the exact-solution pin catches it."""
    orig = lf.operator

    def bad(box, p, coef):
        L = orig(box, p, coef)
        for i in range(1, p - 1):
            L[i + p * (p - 1)] *= -1.0      # N edge
        return L

    monkeypatch.setattr(lf, "operator", bad)
    prob = inputs.tiny(p=10)
    assert itf.relerr_true(itf.solve(prob), prob) > 1e-2


# --------------------------------------------------------------------------
# the error measures of eq. (accuracy_formula), pinned by hand-computed cases
# --------------------------------------------------------------------------
def test_relerr_res_hand_computed():
    A = np.array([[2.0, 0.0], [0.0, 4.0]])
    b = np.array([2.0, 4.0])
    # A u - b = (0, 2), ||b|| = sqrt(20)
    assert itf.relerr_res(A, b, np.array([1.0, 1.5])) == pytest.approx(2.0 / math.sqrt(20.0),
                                                                       rel=1e-15)
    assert itf.relerr_res(A, b, np.array([1.0, 1.0])) == 0.0
    # u = 0 leaves the whole right-hand side: exactly 1 (not ||b|| = sqrt(61))
    A2 = np.array([[1.0, 2.0], [3.0, 4.0]])
    assert itf.relerr_res(A2, np.array([5.0, 6.0]), np.zeros(2)) == pytest.approx(1.0, rel=1e-15)


def _two_leaf_solution(uedge, uint):
    num = itf.numbering(2, 1, 4)
    return itf.Solution(uedge=np.asarray(uedge, dtype=float),
                        uint=np.asarray(uint, dtype=float).reshape(2, 4), num=num)


def test_relerr_true_counts_every_non_corner_node_once():
    """2 x 1 leaves, p = 4: 14 edge nodes (6 on the three vertical lines,
    8 on the four horizontal leaf edges; the shared edge once, no corners)
    and 2 x 4 interior nodes, 22 in all.  With u_true == 2 the denominator is
    2 sqrt(22); one edge value off by 3 and one interior value off by -2 give
    sqrt(13) / (2 sqrt(22))."""
    prob = inputs.Problem(name="const", nx=2, ny=1, p=4, kappa=0.0,
                          exact=lambda x, y, xp: xp.zeros_like(x) + 2.0)
    num = itf.numbering(2, 1, 4)
    assert num.nedge == 14
    uedge = np.full(14, 2.0)
    uedge[5] += 3.0
    uint = np.full(8, 2.0)
    uint[6] -= 2.0
    err = itf.relerr_true(_two_leaf_solution(uedge, uint), prob)
    assert err == pytest.approx(math.sqrt(13.0) / (2.0 * math.sqrt(22.0)), rel=1e-14)
    assert itf.relerr_true(_two_leaf_solution(np.full(14, 2.0), np.full(8, 2.0)), prob) == 0.0


def test_relerr_true_uses_the_node_coordinates():
    """u_true = x1 on the same grid.  Chebyshev points of p = 4 on [-1, 1] are
    -1, -1/2, 1/2, 1, so the leaf x-nodes are 0, 1/8, 3/8, 1/2 and
    1/2, 5/8, 7/8, 1.  Sum of x1^2 over the 22 nodes:
      interiors  2 (1/64 + 9/64) + 2 (25/64 + 49/64) = 168/64,
      vertical lines x = 0, 1/2, 1 (2 nodes each)    = 2 (0 + 1/4 + 1) = 160/64,
      horizontal edges (bottom and top of each leaf)  = 168/64,
    in all 496/64 = 7.75.  One interior value off by 1/2 gives
    (1/2) / sqrt(7.75)."""
    prob = inputs.Problem(name="lin", nx=2, ny=1, p=4, kappa=0.0,
                          exact=lambda x, y, xp: x + 0.0 * y)
    num = itf.numbering(2, 1, 4)
    xe, _ = itf.edge_coordinates(prob, num)
    I = lf.flat(4, lf.interior_nodes(4))
    uint = np.stack([lf.grid(box, 4)[0][I] for box in prob.boxes()])
    assert np.sum(xe ** 2) + np.sum(uint ** 2) == pytest.approx(7.75, rel=1e-15)
    uint_bad = uint.copy()
    uint_bad[1, 2] += 0.5
    err = itf.relerr_true(_two_leaf_solution(xe, uint_bad.ravel()), prob)
    assert err == pytest.approx(0.5 / math.sqrt(7.75), rel=1e-14)



@pytest.mark.parametrize("p,tol", [(8, 3e-4), (12, 1e-7), (16, 1e-11)])
def test_curved_domain_plane_wave(p, tol):
    """The paper's curved domain (eq. (parametrization), operator of
    eq. (chain_rule) with a12 != 0 and the corner reading): a plane wave in
    the physical coordinates is an exact solution; the error must fall
    spectrally with p (measured 9.9e-5, 2.6e-8, 2.5e-12 on 2 x 2 leaves,
    kappa = 8)."""
    prob = inputs.curved(p=p, n=2, kappa=8.0)
    assert itf.relerr_true(itf.solve(prob), prob) < tol
