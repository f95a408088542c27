"""Pins for one oracle leaf: operator, condensation, flux, recovery.

Spectral collocation is exact for polynomials of degree <= p-1 in each
variable, so a manufactured polynomial solution with variable coefficients
(f computed analytically) must be reproduced to rounding by condensation plus
recovery, and the condensed flux S u_b + w must equal its analytic outward
normal derivative.  This pins every term of the operator (a11, a22, c1, c2,
k2b), its sign, the per-direction scaling 2/h, the flux sign and the
boundary ordering.
"""
import numpy as np
import pytest

from oracle import leaf as lf


class Poly:
    """u(x, y) = sum_{m,n} c[m, n] s^m r^n with s = (x-xc)/hx, r = (y-yc)/hy."""

    def __init__(self, c, box):
        self.c = np.asarray(c, dtype=np.float64)
        x0, x1, y0, y1 = box
        self.xc, self.yc = 0.5 * (x0 + x1), 0.5 * (y0 + y1)
        self.hx, self.hy = x1 - x0, y1 - y0

    def _eval(self, x, y, dx, dy):
        s = (x - self.xc) / self.hx
        r = (y - self.yc) / self.hy
        out = np.zeros_like(x)
        M, N = self.c.shape
        for m in range(M):
            for n in range(N):
                if m < dx or n < dy:
                    continue
                fm = np.prod(np.arange(m - dx + 1, m + 1, dtype=np.float64)) if dx else 1.0
                fn = np.prod(np.arange(n - dy + 1, n + 1, dtype=np.float64)) if dy else 1.0
                out = out + self.c[m, n] * fm * fn * s ** (m - dx) * r ** (n - dy)
        return out / (self.hx ** dx * self.hy ** dy)

    def __call__(self, x, y):
        return self._eval(x, y, 0, 0)

    def dx(self, x, y):
        return self._eval(x, y, 1, 0)

    def dy(self, x, y):
        return self._eval(x, y, 0, 1)

    def dxx(self, x, y):
        return self._eval(x, y, 2, 0)

    def dyy(self, x, y):
        return self._eval(x, y, 0, 2)

    def dxy(self, x, y):
        return self._eval(x, y, 1, 1)


def _coef(X, Y):
    return {
        "a11": 1.0 + 0.3 * np.sin(X) * np.cos(2 * Y),
        "a22": 0.8 + 0.2 * np.cos(X + Y),
        "c1": 0.5 * X - 0.2,
        "c2": -0.7 * Y + 0.1,
        "k2b": 25.0 * (1.0 - 0.5 * np.exp(-(X ** 2 + Y ** 2))),
    }


def _coef_mixed(X, Y):
    c = _coef(X, Y)
    c["a12"] = 0.35 * np.cos(X - 2 * Y) + 0.1
    return c


def _manufactured(p, box, seed=0, coef_fn=_coef, operator=lf.operator, deg=None, fold=lf.fold):
    rng = np.random.default_rng(seed)
    deg = p - 1 if deg is None else deg
    c = rng.standard_normal((deg + 1, deg + 1))
    c /= (1.0 + np.add.outer(np.arange(deg + 1), np.arange(deg + 1))) ** 2
    u = Poly(c, box)
    X, Y = lf.grid(box, p)
    coef = coef_fn(X, Y)
    a12 = coef.get("a12", np.zeros_like(X))
    f = -(coef["a11"] * u.dxx(X, Y) + 2.0 * a12 * u.dxy(X, Y) + coef["a22"] * u.dyy(X, Y)
          + coef["c1"] * u.dx(X, Y) + coef["c2"] * u.dy(X, Y)) - coef["k2b"] * u(X, Y)
    L = operator(box, p, coef)
    I = lf.flat(p, lf.interior_nodes(p))
    B = lf.flat(p, lf.boundary_nodes(p))
    bl = fold(L, p)
    cond = lf.condense(bl, f[I])
    ub = u(X[B], Y[B])
    ui = lf.recover(cond, ub)
    # analytic outward normal derivative on W, E, S, N
    m = p - 2
    dn = np.concatenate([-u.dx(X[B[:m]], Y[B[:m]]), u.dx(X[B[m:2 * m]], Y[B[m:2 * m]]),
                         -u.dy(X[B[2 * m:3 * m]], Y[B[2 * m:3 * m]]), u.dy(X[B[3 * m:]], Y[B[3 * m:]])])
    flux = cond.S @ ub + cond.w
    err_u = np.linalg.norm(ui - u(X[I], Y[I])) / np.linalg.norm(u(X[I], Y[I]))
    err_flux = np.linalg.norm(flux - dn) / np.linalg.norm(dn)
    return err_u, err_flux


BOX = (0.3, 0.8, -0.2, 0.1)   # hx != hy, off-centre


@pytest.mark.parametrize("p", [4, 6, 8, 10, 12])
def test_manufactured_polynomial_is_exact(p):
    err_u, err_flux = _manufactured(p, BOX)
    assert err_u < 1e-11, err_u
    assert err_flux < 1e-10, err_flux


@pytest.mark.parametrize("p", [6, 10, 16])
def test_harmonic_polynomials_dtn(p):
    """kappa = 0, f = 0: u = Re/Im (z - z0)^k, k <= p-1, is reproduced and
    S maps its boundary trace to its outward normal derivative."""
    box = (-0.1, 0.4, 0.2, 0.6)
    X, Y = lf.grid(box, p)
    coef = {"k2b": np.zeros(p * p)}
    bl = lf.blocks(box, p, coef)
    cond = lf.condense(bl)
    I = lf.flat(p, lf.interior_nodes(p))
    B = lf.flat(p, lf.boundary_nodes(p))
    m = p - 2
    z = (X - 0.15) + 1j * (Y - 0.4)
    for k in range(1, p):
        for part in (np.real, np.imag):
            u = part(z ** k)
            du = k * z ** (k - 1)               # d/dx = f', d/dy = i f'
            ux, uy = part(du), part(1j * du)
            ub = u[B]
            ui = lf.recover(cond, ub)
            assert np.linalg.norm(ui - u[I]) <= 1e-11 * np.linalg.norm(u)
            dn = np.concatenate([-ux[B[:m]], ux[B[m:2 * m]], -uy[B[2 * m:3 * m]], uy[B[3 * m:]]])
            assert np.linalg.norm(cond.S @ ub - dn) <= 1e-10 * np.linalg.norm(dn)


def test_block_sizes_and_sparsity():
    p = 10
    ni, nb = (p - 2) ** 2, 4 * (p - 2)
    X, Y = lf.grid(BOX, p)
    bl = lf.blocks(BOX, p, _coef(X, Y))
    assert bl.Aii.shape == (ni, ni) and bl.Aib.shape == (ni, nb)
    assert bl.Abi.shape == (nb, ni) and bl.Abb.shape == (nb, nb)
    assert np.all(np.count_nonzero(bl.Abi, axis=1) == p - 2)
    assert np.all(np.count_nonzero(bl.Abb, axis=1) == 2)
    assert np.all(np.count_nonzero(bl.Aib, axis=1) == 4)  # one node on each edge line
    assert np.all(np.count_nonzero(bl.Aib, axis=0) == p - 2)


def test_refactor_recovery_matches_stored():
    p = 12
    X, Y = lf.grid(BOX, p)
    bl = lf.blocks(BOX, p, _coef(X, Y))
    rng = np.random.default_rng(1)
    fi = rng.standard_normal((p - 2) ** 2)
    ub = rng.standard_normal(4 * (p - 2))
    cond = lf.condense(bl, fi)
    a = lf.recover(cond, ub)
    b = lf.recover_refactor(bl, ub, fi)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)


def test_flop_count_values():
    # F(p) = 2/3 ni^3 + 2 ni^2 nb + 2 nb^2 (p-2)
    assert abs(lf.flop_count(16) / 1e6 - 9.410) < 1e-3
    assert abs(lf.flop_count(32) / 1e6 - 681.3) < 0.1
    assert abs(lf.flop_count(20) / 1e6 - 37.98) < 0.01


# -- planted mistakes: each must be caught by the manufactured-solution pin --

def _flip_east(box, p, coef):
    L = lf.operator(box, p, coef)
    for j in range(1, p - 1):
        L[(p - 1) + p * j] *= -1.0
    return L


def _drop_c1(box, p, coef):
    c = dict(coef)
    c["c1"] = np.zeros_like(coef["c1"])
    return lf.operator(box, p, c)


def _swap_h(box, p, coef):
    x0, x1, y0, y1 = box
    w = (x1 - x0, y1 - y0)
    return lf.operator((x0, x0 + w[1], y0, y0 + w[0]), p, coef)


def _k2b_sign(box, p, coef):
    c = dict(coef)
    c["k2b"] = -coef["k2b"]
    return lf.operator(box, p, c)


@pytest.mark.parametrize("mutant", [_flip_east, _drop_c1, _swap_h, _k2b_sign])
def test_planted_mistakes_are_caught(mutant):
    err_u, err_flux = _manufactured(8, BOX, operator=mutant)
    assert max(err_u, err_flux) > 1e-4



# -- the mixed term and the corners (general operator, Sec. 3.2) ------------
# With a12 != 0 the interior rows reach the corners, whose values come from
# the edges' degree-(p-3) extrapolants: exact for polynomials of degree <=
# p-3 in each variable, so such a manufactured solution is reproduced to
# rounding.

@pytest.mark.parametrize("p", [5, 6, 8, 10, 12])
def test_manufactured_polynomial_with_mixed_term(p):
    err_u, err_flux = _manufactured(p, BOX, coef_fn=_coef_mixed, deg=p - 3)
    assert err_u < 1e-10, err_u
    assert err_flux < 1e-9, err_flux


def test_mixed_term_needs_the_corners():
    # degree p-1 is beyond what the corner extrapolation reproduces: the
    # mixed term then sees the extrapolation error (the a12 == 0 operator
    # does not, which the pin above relies on)
    err_u, _ = _manufactured(8, BOX, coef_fn=_coef_mixed, deg=7)
    assert err_u > 1e-8
    err_u0, _ = _manufactured(8, BOX, coef_fn=_coef, deg=7)
    assert err_u0 < 1e-11


def _mixed_no_two(box, p, coef):
    c = dict(coef)
    c["a12"] = 0.5 * coef["a12"]
    return lf.operator(box, p, c)


def _mixed_xx(box, p, coef):
    # mixed term with the x1 derivative twice (transposed operand)
    L = lf.operator(box, p, {k: v for k, v in coef.items() if k != "a12"})
    x0, x1, y0, y1 = box
    D = lf.cheb.diff_matrix(p)
    Dx = (2.0 / (x1 - x0)) * D
    for (i, j) in lf.interior_nodes(p):
        n = i + p * j
        for l in range(p):
            for k in range(p):
                L[n, k + p * l] -= 2.0 * coef["a12"][n] * Dx[i, k] * Dx[j, l]
    return L


def _fold_swapped(L, p):
    bl = lf.fold(L, p)
    I = lf.flat(p, lf.interior_nodes(p))
    Cn = lf.flat(p, lf.corner_nodes(p))
    C = lf.corner_map(p)
    # corners taken with the weights of the opposite end
    return lf.Blocks(Aii=bl.Aii, Aib=bl.Aib - L[np.ix_(I, Cn)] @ C + L[np.ix_(I, Cn)] @ C[::-1],
                     Abi=bl.Abi, Abb=bl.Abb)


def _no_fold(L, p):
    I = lf.flat(p, lf.interior_nodes(p))
    B = lf.flat(p, lf.boundary_nodes(p))
    return lf.Blocks(Aii=L[np.ix_(I, I)], Aib=L[np.ix_(I, B)], Abi=L[np.ix_(B, I)],
                     Abb=L[np.ix_(B, B)])


@pytest.mark.parametrize("operator,fold", [(_mixed_no_two, lf.fold), (_mixed_xx, lf.fold),
                                           (lf.operator, _fold_swapped), (lf.operator, _no_fold)])
def test_planted_mixed_term_mistakes_are_caught(operator, fold):
    err_u, err_flux = _manufactured(8, BOX, coef_fn=_coef_mixed, deg=5, operator=operator,
                                    fold=fold)
    assert max(err_u, err_flux) > 1e-4
