"""One HPS leaf: its collocation matrix, static condensation and recovery
(oracle; test infrastructure only).

Conventions the paper leaves open (each is listed with its reason in the
design notes of the repository):

* node (i, j) of the p x p grid, i along x1 and j along x2, has flat index
  i + p*j;
* interior set I: 1 <= i, j <= p-2, ordered i fastest, so ni = (p-2)^2;
* boundary set B: the four edges without corners, in the order
  W (i = 0, j up), E (i = p-1, j up), S (j = 0, i up), N (j = p-1, i up),
  so nb = 4(p-2); corner nodes carry no unknown;
* interior rows collocate the general second-order operator of Sec. 3.2
  (eq. (chain_rule) is an instance) in reference coordinates,
      -(a11 u_11 + 2 a12 u_12 + a22 u_22 + c1 u_1 + c2 u_2) - k2b u = f;
  without the mixed term no interior row refers to a corner; with it, each
  corner value is replaced by the average of the degree-(p-3) extrapolants
  along its two edges (cheb.endpoint_weights), which folds the corner
  columns into A_ib (`fold`);
* boundary rows are the outward normal derivative (the flux whose
  continuity across leaf edges closes the system, Sec. 2), taken with the
  spectral derivative along the line of nodes normal to the edge:
      W: -u_1,  E: +u_1,  S: -u_2,  N: +u_2.

Static condensation (Sec. 2, before eq. (hps_reduced)) eliminates the
interior nodes:  X = A_ii^{-1} A_ib,  h = A_ii^{-1} f_i,
S = A_bb - A_bi X,  w = A_bi h.  For boundary values u_b the interior values
are u_i = h - X u_b and the outward flux is S u_b + w.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np
import scipy.linalg

from . import cheb

FIELDS = ("a11", "a12", "a22", "c1", "c2", "k2b")


def interior_nodes(p: int):
    """List of (i, j) for the interior set, i fastest."""
    return [(i, j) for j in range(1, p - 1) for i in range(1, p - 1)]


def boundary_nodes(p: int):
    """List of (i, j) for the boundary set in W, E, S, N order."""
    m = range(1, p - 1)
    return ([(0, j) for j in m] + [(p - 1, j) for j in m]
            + [(i, 0) for i in m] + [(i, p - 1) for i in m])


def flat(p: int, ij):
    return [i + p * j for (i, j) in ij]


def grid(box, p: int):
    """Coordinates (x, y) of the p*p nodes of leaf box (x0, x1, y0, y1),
    flat index i + p*j."""
    x0, x1, y0, y1 = (float(v) for v in box)
    t = cheb.nodes(p)
    xs = x0 + (t + 1.0) * (x1 - x0) / 2.0
    ys = y0 + (t + 1.0) * (y1 - y0) / 2.0
    X = np.empty(p * p)
    Y = np.empty(p * p)
    for j in range(p):
        for i in range(p):
            X[i + p * j] = xs[i]
            Y[i + p * j] = ys[j]
    return X, Y


def sample_coefficients(problem, box, p: int) -> Dict[str, np.ndarray]:
    """Coefficient fields of `problem` at the leaf's nodes (numpy)."""
    X, Y = grid(box, p)
    return {name: np.asarray(problem.sample(name, X, Y, np), dtype=np.float64)
            for name in FIELDS}


def operator(box, p: int, coef: Dict[str, np.ndarray]) -> np.ndarray:
    """The full p^2 x p^2 leaf matrix L over all nodes (corner rows zero;
    interior rows reach the corner columns only through the mixed term).

    `coef[name]` holds the field at every node (flat index i + p*j);
    missing fields take their default (a11 = a22 = 1, others 0)."""
    x0, x1, y0, y1 = (float(v) for v in box)
    hx, hy = x1 - x0, y1 - y0
    D = cheb.diff_matrix(p)
    Dx = (2.0 / hx) * D
    Dy = (2.0 / hy) * D
    Dxx = Dx @ Dx
    Dyy = Dy @ Dy

    def field(name, default):
        v = coef.get(name)
        return np.full(p * p, default) if v is None else np.asarray(v, dtype=np.float64)

    a11, a22 = field("a11", 1.0), field("a22", 1.0)
    a12 = field("a12", 0.0)
    c1, c2, k2b = field("c1", 0.0), field("c2", 0.0), field("k2b", 0.0)

    L = np.zeros((p * p, p * p))
    for (i, j) in interior_nodes(p):
        n = i + p * j
        for k in range(p):           # derivatives along x1: same j
            L[n, k + p * j] -= a11[n] * Dxx[i, k] + c1[n] * Dx[i, k]
        for l in range(p):           # derivatives along x2: same i
            L[n, i + p * l] -= a22[n] * Dyy[j, l] + c2[n] * Dy[j, l]
        L[n, n] -= k2b[n]
        if a12[n] != 0.0:            # mixed derivative: every node (k, l)
            for l in range(p):
                for k in range(p):
                    L[n, k + p * l] -= 2.0 * a12[n] * Dx[i, k] * Dy[j, l]
    for j in range(1, p - 1):
        for k in range(p):
            L[0 + p * j, k + p * j] = -Dx[0, k]              # W: -d/dx1
            L[(p - 1) + p * j, k + p * j] = Dx[p - 1, k]     # E: +d/dx1
    for i in range(1, p - 1):
        for l in range(p):
            L[i + p * 0, i + p * l] = -Dy[0, l]              # S: -d/dx2
            L[i + p * (p - 1), i + p * l] = Dy[p - 1, l]     # N: +d/dx2
    return L


@dataclass
class Blocks:
    Aii: np.ndarray
    Aib: np.ndarray
    Abi: np.ndarray
    Abb: np.ndarray


def corner_nodes(p: int):
    """The corners (i, j): SW, SE, NW, NE."""
    return [(0, 0), (p - 1, 0), (0, p - 1), (p - 1, p - 1)]


def corner_map(p: int) -> np.ndarray:
    """C [4, nb]: corner values (SW, SE, NW, NE) from the boundary slots,
    each the mean of the extrapolants along its two edges to that end."""
    m = p - 2
    lo, hi = cheb.endpoint_weights(p)
    W, E, S, N = 0, m, 2 * m, 3 * m        # first slot of each edge
    C = np.zeros((4, 4 * m))
    # SW: W edge to j = 0, S edge to i = 0
    C[0, W:W + m] += 0.5 * lo
    C[0, S:S + m] += 0.5 * lo
    # SE: E edge to j = 0, S edge to i = p-1
    C[1, E:E + m] += 0.5 * lo
    C[1, S:S + m] += 0.5 * hi
    # NW: W edge to j = p-1, N edge to i = 0
    C[2, W:W + m] += 0.5 * hi
    C[2, N:N + m] += 0.5 * lo
    # NE: E edge to j = p-1, N edge to i = p-1
    C[3, E:E + m] += 0.5 * hi
    C[3, N:N + m] += 0.5 * hi
    return C


def fold(L: np.ndarray, p: int) -> Blocks:
    """The four blocks of a full leaf matrix, with the interior rows' corner
    columns folded into A_ib through corner_map (the edge rows never refer to
    a corner: each takes its derivative along an interior grid line)."""
    I = flat(p, interior_nodes(p))
    B = flat(p, boundary_nodes(p))
    Cn = flat(p, corner_nodes(p))
    Aib = L[np.ix_(I, B)] + L[np.ix_(I, Cn)] @ corner_map(p)
    return Blocks(Aii=L[np.ix_(I, I)], Aib=Aib,
                  Abi=L[np.ix_(B, I)], Abb=L[np.ix_(B, B)])


def blocks(box, p: int, coef: Dict[str, np.ndarray]) -> Blocks:
    return fold(operator(box, p, coef), p)


@dataclass
class Condensed:
    X: np.ndarray      # [ni, nb]  A_ii^{-1} A_ib
    h: np.ndarray      # [ni]      A_ii^{-1} f_i
    S: np.ndarray      # [nb, nb]  A_bb - A_bi X   (Dirichlet-to-Neumann map)
    w: np.ndarray      # [nb]      A_bi h


def condense(bl: Blocks, fi: Optional[np.ndarray] = None) -> Condensed:
    """Static condensation of one leaf with LAPACK getrf/getrs (partial pivoting)."""
    lu = scipy.linalg.lu_factor(bl.Aii, check_finite=True)
    X = scipy.linalg.lu_solve(lu, bl.Aib)
    ni = bl.Aii.shape[0]
    h = np.zeros(ni) if fi is None else scipy.linalg.lu_solve(lu, np.asarray(fi, dtype=np.float64))
    S = bl.Abb - bl.Abi @ X
    w = bl.Abi @ h
    return Condensed(X=X, h=h, S=S, w=w)


def recover(c: Condensed, ub: np.ndarray) -> np.ndarray:
    """Interior values from boundary values: u_i = h - X u_b."""
    return c.h - c.X @ np.asarray(ub, dtype=np.float64)


def recover_refactor(bl: Blocks, ub: np.ndarray, fi: Optional[np.ndarray] = None) -> np.ndarray:
    """The paper's storage-free recovery (Sec. 2, remark after the batching
    paragraph): re-form and re-factor A_ii, then solve
    A_ii u_i = f_i - A_ib u_b."""
    rhs = -bl.Aib @ np.asarray(ub, dtype=np.float64)
    if fi is not None:
        rhs = rhs + fi
    lu = scipy.linalg.lu_factor(bl.Aii)
    return scipy.linalg.lu_solve(lu, rhs)


def flop_count(p: int, with_f: bool = False) -> float:
    """Useful floating-point operations of one leaf condensation: LU of A_ii,
    two triangular solves for the nb columns of A_ib, and S = A_bb - A_bi X
    with A_bi's p-2 nonzeros per row; plus one more right-hand side for f."""
    ni, nb = (p - 2) ** 2, 4 * (p - 2)
    F = (2.0 / 3.0) * ni ** 3 + 2.0 * ni * ni * nb + 2.0 * nb * nb * (p - 2)
    if with_f:
        F += 2.0 * ni * ni + 2.0 * nb * (p - 2)
    return F
