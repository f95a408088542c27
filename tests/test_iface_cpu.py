"""Host-side planning of the nested-dissection interface solve (no device):
the bisection tree eliminates every unknown edge node exactly once, the
root has no exterior, the separators have the lengths the geometry fixes,
and the FLOP count is the sum over fronts."""
import pytest

from paper_2211_14969_amd import hps


@pytest.fixture(scope="module")
def lib():
    import os
    if not os.path.exists(hps.LIB_PATH):
        from paper_2211_14969_amd import build
        build.build()
    return hps.load()


def unknowns(nx, ny, p):
    return ((nx - 1) * ny + nx * (ny - 1)) * (p - 2)


@pytest.mark.parametrize("nx,ny,p", [(1, 1, 8), (2, 1, 6), (4, 4, 8), (5, 3, 10), (7, 1, 6),
                                     (2, 9, 12), (12, 10, 24), (32, 32, 32), (128, 16, 20),
                                     (64, 64, 16)])
def test_plan_eliminates_every_unknown_once(lib, nx, ny, p):
    plan = hps.hps_iface_plan(p, nx, ny)
    assert plan["fronts"] == nx * ny - 1
    nS, nE, lev = hps.hps_iface_plan_fronts(p, nx, ny)
    assert sum(nS) == unknowns(nx, ny, p)
    if nS:
        assert lev == sorted(lev)                  # factorisation order: by level
        assert lev.count(max(lev)) == 1 and nE[-1] == 0   # one root, nothing outside it
        assert plan["levels"] == max(lev)
        assert all(s % (p - 2) == 0 and s > 0 for s in nS)   # whole leaf edges
        assert plan["max_separator"] == max(nS)
    flop = sum((2.0 / 3.0) * s ** 3 + 2.0 * s * s * e + 2.0 * e * e * s for s, e in zip(nS, nE))
    assert plan["factor_flop"] == pytest.approx(flop, rel=1e-12)


@pytest.mark.parametrize("nx,ny,p,sep", [(32, 32, 32, 32 * 30), (64, 64, 16, 64 * 14),
                                         (128, 16, 20, 16 * 18), (4, 4, 8, 4 * 6)])
def test_root_separator_is_the_first_cut(lib, nx, ny, p, sep):
    # the longer side is cut first, so the root separator spans the shorter one
    nS, nE, lev = hps.hps_iface_plan_fronts(p, nx, ny)
    assert nS[-1] == sep
    assert hps.hps_iface_plan(p, nx, ny)["max_separator"] == sep


def test_balanced_grid_depth(lib):
    # 2^k leaves in a square: k levels, 2^(k-l) fronts on level l
    nS, nE, lev = hps.hps_iface_plan_fronts(16, 16, 16)
    assert max(lev) == 8
    for l in range(1, 9):
        assert lev.count(l) == 2 ** (8 - l)


@pytest.mark.parametrize("p,nx,ny", [(3, 4, 4), (33, 4, 4), (8, 0, 4), (8, 4, -1),
                                     (32, 64, 64)])
def test_plan_rejects(lib, p, nx, ny):
    # orders outside the build, empty grids, a separator above the limit
    # (64 leaves of p = 32 on one cut: 1920 nodes)
    with pytest.raises(hps.HpsError) as e:
        hps.hps_iface_plan(p, nx, ny)
    assert e.value.status == hps.HPS_ERR_INVALID


@pytest.mark.parametrize("nx,ny,orders", [(4, 4, (8, 12)), (5, 3, (8, 10, 16)), (32, 32, None)])
def test_plan_with_orders(lib, nx, ny, orders):
    """Per-leaf orders: one front per leaf but one, and the root separator
    carries, on every cut edge, the lower of its two leaves' orders."""
    import numpy as np
    from oracle import mixed as mx
    from paper_2211_14969_amd import inputs
    if orders is None:
        prob = inputs.mixed_bump()
        o = prob.orders
    else:
        rng = np.random.default_rng(nx * ny)
        o = rng.choice(np.asarray(orders), size=nx * ny)
    plan = hps.hps_iface_plan_orders(nx, ny, o)
    assert plan["fronts"] == nx * ny - 1
    num = mx.numbering(nx, ny, o)
    # the root cut: the longer side is halved first
    if nx >= ny:
        mid = nx // 2
        cut = [mid + (nx + 1) * iy for iy in range(ny)]
    else:
        mid = ny // 2
        cut = [(nx + 1) * ny + ix + nx * mid for ix in range(nx)]
    root = sum(int(num.m_edge[e]) for e in cut)
    assert plan["max_separator"] >= root
    # one order everywhere is the uniform plan exactly
    u = hps.hps_iface_plan_orders(nx, ny, [int(o[0])] * (nx * ny))
    assert u == hps.hps_iface_plan(int(o[0]), nx, ny)


def test_plan_orders_rejects(lib):
    with pytest.raises(hps.HpsError):
        hps.hps_iface_plan_orders(2, 2, [8, 8, 3, 8])
    with pytest.raises(hps.HpsError):
        hps.hps_iface_plan_orders(2, 2, [8, 8, 8, 40])
