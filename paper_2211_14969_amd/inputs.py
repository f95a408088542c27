"""Seeded synthetic problem definitions shared by the HIP path and the oracle.

This module holds only problem data: the leaf partition of a reference
rectangle, the PDE coefficient fields as plain functions of position, the
wavenumber and the Dirichlet data.  It contains none of the discretisation or
solver arithmetic (no Chebyshev nodes, no differentiation, no elimination):
each consumer samples the functions at its own node coordinates.

The problems follow the paper's model problem, the variable-coefficient
Helmholtz operator  A u = -Lap u - kappa^2 b(x) u  (Sec. 1, eq. (var_helm)),
written in reference coordinates as

    A u = -(a11 u_11 + 2 a12 u_12 + a22 u_22 + c1 u_1 + c2 u_2) - k2b u,

with a11 = a22 = 1, a12 = c1 = c2 = 0 and k2b = kappa^2 b on a plain square;
the quarter annulus and the paper's curved domain come from maps of the unit
square (the curved one with a mixed term, Sec. 3.2, eq. (chain_rule)).

Every function takes the array namespace ``xp`` (``numpy`` or ``torch``) so
that the same definition is evaluated on the host or on the device.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

CoefFn = Callable[..., object]

FIELDS = ("a11", "a12", "a22", "c1", "c2", "k2b")


@dataclass
class Problem:
    """One boundary value problem on a rectangle split into nx*ny equal leaves.

    Leaf ``t = ix + nx*iy`` covers
    ``[x0 + ix*hx, x0 + (ix+1)*hx] x [y0 + iy*hy, y0 + (iy+1)*hy]``.
    ``coef[name](x, y, xp)`` returns the coefficient at the given points;
    a missing entry means the default (a11 = a22 = 1, c1 = c2 = k2b = 0).
    ``g`` is the Dirichlet data; ``exact`` the exact solution when known.
    """

    name: str
    nx: int
    ny: int
    p: int
    kappa: float
    domain: tuple = (0.0, 1.0, 0.0, 1.0)
    coef: Dict[str, CoefFn] = field(default_factory=dict)
    g: Optional[CoefFn] = None
    exact: Optional[CoefFn] = None
    f: Optional[CoefFn] = None
    meta: dict = field(default_factory=dict)

    @property
    def nleaf(self) -> int:
        return self.nx * self.ny

    def boxes(self) -> np.ndarray:
        """[nleaf, 4] float64 array of (x0, x1, y0, y1), leaf order ix + nx*iy."""
        x0, x1, y0, y1 = self.domain
        hx = (x1 - x0) / self.nx
        hy = (y1 - y0) / self.ny
        ix = np.arange(self.nx, dtype=np.float64)
        iy = np.arange(self.ny, dtype=np.float64)
        IX, IY = np.meshgrid(ix, iy, indexing="xy")  # IX[iy, ix]
        IX = IX.ravel()
        IY = IY.ravel()
        out = np.empty((self.nleaf, 4), dtype=np.float64)
        out[:, 0] = x0 + IX * hx
        out[:, 1] = x0 + (IX + 1.0) * hx
        out[:, 2] = y0 + IY * hy
        out[:, 3] = y0 + (IY + 1.0) * hy
        return out

    def sample(self, name: str, x, y, xp=np):
        """Coefficient ``name`` at points (x, y); default value if not set."""
        fn = self.coef.get(name)
        if fn is None:
            base = 1.0 if name in ("a11", "a22") else 0.0
            return xp.zeros_like(x) + base
        return fn(x, y, xp)

    def has(self, name: str) -> bool:
        return name in self.coef


# ---------------------------------------------------------------------------
# coefficient fields
# ---------------------------------------------------------------------------

def _const(v):
    return lambda x, y, xp: xp.zeros_like(x) + v


def gaussian_bumps_b(centres, amp: float, width: float):
    """b(x) = 1 - amp * sum_k exp(-|x - c_k|^2 / width)."""
    cs = [(float(c[0]), float(c[1])) for c in centres]

    def b(x, y, xp):
        acc = xp.zeros_like(x)
        for cx, cy in cs:
            acc = acc + xp.exp(-((x - cx) ** 2 + (y - cy) ** 2) / width)
        return 1.0 - amp * acc

    return b


def _scaled(kappa: float, b):
    k2 = kappa * kappa
    return lambda x, y, xp: k2 * b(x, y, xp)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def tiny(p: int = 8, n: int = 4, kappa: float = 10.0) -> Problem:
    """Unit square, n x n leaves, b == 1, f = 0, g = sin(kappa x1) (exact)."""
    sol = lambda x, y, xp: xp.sin(kappa * x)
    return Problem(
        name=f"tiny_{n}x{n}_p{p}", nx=n, ny=n, p=p, kappa=kappa,
        coef={"k2b": _const(kappa * kappa)}, g=sol, exact=sol,
        meta={"b": "1"},
    )


def single_bump(p: int = 16, n: int = 64, kappa: float = 100.0) -> Problem:
    """Unit square, b = 1 - 0.5 exp(-|x - (0.5, 0.5)|^2 / 0.05), g = cos(kappa x1)."""
    b = gaussian_bumps_b([(0.5, 0.5)], 0.5, 0.05)
    return Problem(
        name=f"bump_{n}x{n}_p{p}", nx=n, ny=n, p=p, kappa=kappa,
        coef={"k2b": _scaled(kappa, b)},
        g=lambda x, y, xp: xp.cos(kappa * x),
        meta={"b": "1-0.5*exp(-|x-(.5,.5)|^2/0.05)"},
    )


def bump_centres(seed: int, count: int = 8) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(count, 2))


def multi_bump(p: int = 32, n: int = 32, kappa: float = 300.0, seed: int = 3,
               count: int = 8) -> Problem:
    """Unit square, b = 1 - 0.3 * sum of `count` Gaussian bumps of width 0.03,
    centres uniform on [0,1]^2 from `seed`; g = cos(kappa x1)."""
    cs = bump_centres(seed, count)
    b = gaussian_bumps_b(cs, 0.3, 0.03)
    return Problem(
        name=f"bumps_{n}x{n}_p{p}", nx=n, ny=n, p=p, kappa=kappa,
        coef={"k2b": _scaled(kappa, b)},
        g=lambda x, y, xp: xp.cos(kappa * x),
        meta={"b": f"1-0.3*sum_{count} exp(-|x-c|^2/0.03)", "seed": seed,
              "centres": cs.tolist()},
    )


def annulus(p: int = 20, ntheta: int = 128, nr: int = 16, kappa: float = 150.0) -> Problem:
    """Quarter annulus r in [1,2], theta in [0, pi/2], pulled back to the unit
    square by theta = (pi/2) x1, r = 1 + x2.  In those coordinates
    -Lap u - kappa^2 u = -(4/(pi^2 r^2)) u_11 - u_22 - (1/r) u_2 - kappa^2 u,
    so a11 = 4/(pi^2 r^2), a22 = 1, c2 = 1/r, k2b = kappa^2 (b == 1).
    g is the plane wave cos(kappa X) in the physical coordinate X = r cos(theta),
    an exact solution."""
    pi = math.pi
    a11 = lambda x, y, xp: 4.0 / (pi * pi * (1.0 + y) ** 2)
    c2 = lambda x, y, xp: 1.0 / (1.0 + y)
    sol = lambda x, y, xp: xp.cos(kappa * (1.0 + y) * xp.cos(0.5 * pi * x))
    return Problem(
        name=f"annulus_{ntheta}x{nr}_p{p}", nx=ntheta, ny=nr, p=p, kappa=kappa,
        coef={"a11": a11, "c2": c2, "k2b": _const(kappa * kappa)},
        g=sol, exact=sol, meta={"map": "theta=(pi/2)x1, r=1+x2"},
    )


def curved(p: int = 16, n: int = 8, kappa: float = 20.0, theta: float = 0.6,
           data: str = "wave") -> Problem:
    """The paper's curved domain (Sec. 3.2, eq. (parametrization)): the image
    of the unit square under (x1, x2) -> (x1, x2 / psi(x1)), psi(z) = 1 -
    sin(z)/4.  Pulled back to the square, -Lap u - kappa^2 u = 0 becomes
    eq. (chain_rule):
        a11 = 1, a12 = psi' x2 / psi, a22 = (psi' x2 / psi)^2 + psi^2,
        c2 = psi'' x2 / psi, k2b = kappa^2.
    data="wave": g is the plane wave cos(kappa (y1 cos(theta) + y2 sin(theta)))
    in the physical coordinates y = (x1, x2 / psi(x1)), an exact solution;
    data="one": u = 1 on the boundary, the paper's Dirichlet data."""
    psi = lambda x, xp: 1.0 - 0.25 * xp.sin(x)
    dpsi = lambda x, xp: -0.25 * xp.cos(x)
    ddpsi = lambda x, xp: 0.25 * xp.sin(x)
    a12 = lambda x, y, xp: dpsi(x, xp) * y / psi(x, xp)
    a22 = lambda x, y, xp: (dpsi(x, xp) * y / psi(x, xp)) ** 2 + psi(x, xp) ** 2
    c2 = lambda x, y, xp: ddpsi(x, xp) * y / psi(x, xp)
    ct, st = math.cos(theta), math.sin(theta)
    wave = lambda x, y, xp: xp.cos(kappa * (x * ct + y / psi(x, xp) * st))
    if data == "wave":
        g, exact = wave, wave
    elif data == "one":
        g, exact = (lambda x, y, xp: xp.zeros_like(x) + 1.0), None
    else:
        raise ValueError(data)
    return Problem(
        name=f"curved_{n}x{n}_p{p}", nx=n, ny=n, p=p, kappa=kappa,
        coef={"a12": a12, "a22": a22, "c2": c2, "k2b": _const(kappa * kappa)},
        g=g, exact=exact, meta={"map": "(x1, x2/psi(x1)), psi = 1 - sin(x1)/4", "data": data},
    )


@dataclass
class MixedProblem:
    """One boundary value problem on a rectangle of nx*ny equal leaves whose
    orders p come from a fixed set (Sec. 2: p chosen per leaf from a few
    values, as in hp-adaptivity); ``orders[t]`` is the p of leaf
    t = ix + nx*iy.  Fields as in Problem."""

    name: str
    nx: int
    ny: int
    orders: np.ndarray
    kappa: float
    domain: tuple = (0.0, 1.0, 0.0, 1.0)
    coef: Dict[str, CoefFn] = field(default_factory=dict)
    g: Optional[CoefFn] = None
    exact: Optional[CoefFn] = None
    f: Optional[CoefFn] = None
    meta: dict = field(default_factory=dict)

    @property
    def nleaf(self) -> int:
        return self.nx * self.ny

    def boxes(self) -> np.ndarray:
        return Problem.boxes(self)

    def sample(self, name: str, x, y, xp=np):
        return Problem.sample(self, name, x, y, xp)

    def has(self, name: str) -> bool:
        return name in self.coef

    def groups(self) -> List["LeafSet"]:
        """One leaf set per order, orders ascending."""
        orders = np.asarray(self.orders)
        return [LeafSet(self, int(p), np.flatnonzero(orders == p)) for p in np.unique(orders)]


@dataclass
class LeafSet:
    """The leaves of one order of a MixedProblem: a group of the leaf batch
    (it answers the questions the batch asks of a Problem)."""

    parent: MixedProblem
    p: int
    leaves: np.ndarray

    @property
    def name(self) -> str:
        return f"{self.parent.name}_p{self.p}"

    @property
    def nleaf(self) -> int:
        return int(self.leaves.size)

    @property
    def f(self):
        return self.parent.f

    @property
    def g(self):
        return self.parent.g

    @property
    def exact(self):
        return self.parent.exact

    @property
    def kappa(self) -> float:
        return self.parent.kappa

    @property
    def meta(self) -> dict:
        return self.parent.meta

    def boxes(self) -> np.ndarray:
        return self.parent.boxes()[self.leaves]

    def sample(self, name: str, x, y, xp=np):
        return self.parent.sample(name, x, y, xp)

    def has(self, name: str) -> bool:
        return self.parent.has(name)


def mixed_tiny(n: int = 4, orders=(8, 12), kappa: float = 10.0) -> MixedProblem:
    """The tiny workload's exact solution sin(kappa x1) on n x n leaves whose
    orders alternate in a checkerboard over `orders`."""
    sol = lambda x, y, xp: xp.sin(kappa * x)
    o = np.array([orders[(ix + iy) % len(orders)] for iy in range(n) for ix in range(n)])
    return MixedProblem(name=f"mixed_tiny_{n}x{n}_p{'-'.join(map(str, orders))}", nx=n, ny=n,
                        orders=o, kappa=kappa, coef={"k2b": _const(kappa * kappa)}, g=sol,
                        exact=sol, meta={"b": "1", "orders": list(orders)})


def mixed_bump(n: int = 32, orders=(12, 20, 28), kappa: float = 150.0) -> MixedProblem:
    """hp-style orders on one bump: b = 1 - 0.5 exp(-|x - (0.5, 0.5)|^2 / 0.02);
    leaves whose centre lies within 0.15 of the bump's centre take the highest
    order, within 0.3 the middle one, the rest the lowest.  g = cos(kappa x1)."""
    b = gaussian_bumps_b([(0.5, 0.5)], 0.5, 0.02)
    o = np.empty(n * n, dtype=np.int64)
    h = 1.0 / n
    for iy in range(n):
        for ix in range(n):
            r = math.hypot((ix + 0.5) * h - 0.5, (iy + 0.5) * h - 0.5)
            o[ix + n * iy] = orders[2] if r < 0.15 else (orders[1] if r < 0.3 else orders[0])
    return MixedProblem(name=f"mixed_bump_{n}x{n}", nx=n, ny=n, orders=o, kappa=kappa,
                        coef={"k2b": _scaled(kappa, b)},
                        g=lambda x, y, xp: xp.cos(kappa * x),
                        meta={"b": "1-0.5*exp(-|x-(.5,.5)|^2/0.02)", "orders": list(orders)})


UNEVEN_P = (8, 12, 16, 20, 24, 28, 30, 32)


def uneven_batch(seed: int = 5, orders=UNEVEN_P, kmin: int = 8, kmax: int = 14,
                 kappa_range=(50.0, 400.0)) -> List[Problem]:
    """Eight independent problems, one per order in `orders`.  Per problem:
    k ~ U{kmin..kmax}, 2^k leaves as 2^ceil(k/2) x 2^floor(k/2), kappa ~
    U[kappa_range], b = eight Gaussian bumps (amplitude 0.3, width 0.03)."""
    rng = np.random.default_rng(seed)
    out = []
    for idx, p in enumerate(orders):
        k = int(rng.integers(kmin, kmax + 1))
        kappa = float(rng.uniform(*kappa_range))
        cs = rng.uniform(0.0, 1.0, size=(8, 2))
        b = gaussian_bumps_b(cs, 0.3, 0.03)
        nx = 2 ** ((k + 1) // 2)
        ny = 2 ** (k // 2)
        out.append(Problem(
            name=f"uneven{idx}_p{p}_L{nx * ny}", nx=nx, ny=ny, p=p, kappa=kappa,
            coef={"k2b": _scaled(kappa, b)},
            g=lambda x, y, xp, _k=kappa: xp.cos(_k * x),
            meta={"seed": seed, "k": k, "centres": cs.tolist()},
        ))
    return out


def config(n: int) -> Problem:
    """The workloads by number: 1 tiny, 2 single bump p=16, 3 eight bumps p=32,
    4 quarter annulus p=20.  (5 is `uneven_batch`.)"""
    if n == 1:
        return tiny()
    if n == 2:
        return single_bump()
    if n == 3:
        return multi_bump()
    if n == 4:
        return annulus()
    raise ValueError(f"no single-problem workload {n}")

