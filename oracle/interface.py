"""The reduced interface system, its solve, and the full collocation system
(oracle; test infrastructure only).

A rectangle is split into nx x ny equal leaves (leaf t = ix + nx*iy).  Each
leaf edge carries p-2 nodes (corners are never used).  An edge shared by two
leaves carries unknowns; an edge on the outer boundary carries Dirichlet
data g.

Reduced system (eq. (hps_reduced)): at every interface node the outward
fluxes of the two leaves sharing it sum to zero (Sec. 2: the flux between
adjacent leaves is continuous).  With each leaf's flux S u_b + w this gives

    A~ = sum_t P_t^T S_t[U, U] P_t,
    f~ = -sum_t P_t^T (w_t[U] + S_t[U, D] g_D),

where U are a leaf's boundary slots on interface edges and D those on the
outer boundary.  It is solved with SciPy's SuperLU and the COLAMD ordering,
the paper's own choice for its first solver (Sec. 3.1).

The full system (eq. (Au=f)) keeps every non-corner node: PDE rows at leaf
interiors, flux-sum rows at interface nodes and identity rows at Dirichlet
nodes.  Solved densely it is the brute-force reference for tiny grids.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.sparse
import scipy.sparse.linalg

from . import leaf as lf


@dataclass
class Numbering:
    """Global ids of the edge nodes.

    Edge nodes are numbered vertical edges first (line ix = 0..nx, leaf row
    iy, node j = 1..p-2), then horizontal edges (leaf column ix, line
    iy = 0..ny, node i = 1..p-2).  `slot[t]` maps leaf t's nb boundary slots
    (W, E, S, N) to edge-node ids; `dirichlet[e]` marks outer-boundary nodes;
    `unknown[e]` is the reduced-system index of an interface node (-1 for
    Dirichlet nodes)."""

    nedge: int
    slot: np.ndarray        # [nleaf, nb]
    dirichlet: np.ndarray   # [nedge] bool
    unknown: np.ndarray     # [nedge] int
    nunknown: int


def numbering(nx: int, ny: int, p: int) -> Numbering:
    m = p - 2
    nv = (nx + 1) * ny * m
    nh = nx * (ny + 1) * m

    def vid(line, iy, j):          # j = 1..p-2
        return (line + (nx + 1) * iy) * m + (j - 1)

    def hid(ix, line, i):          # i = 1..p-2
        return nv + (ix + nx * line) * m + (i - 1)

    nedge = nv + nh
    dirichlet = np.zeros(nedge, dtype=bool)
    for iy in range(ny):
        for j in range(1, p - 1):
            dirichlet[vid(0, iy, j)] = True
            dirichlet[vid(nx, iy, j)] = True
    for ix in range(nx):
        for i in range(1, p - 1):
            dirichlet[hid(ix, 0, i)] = True
            dirichlet[hid(ix, ny, i)] = True
    slot = np.empty((nx * ny, 4 * m), dtype=np.int64)
    for iy in range(ny):
        for ix in range(nx):
            t = ix + nx * iy
            s = []
            s += [vid(ix, iy, j) for j in range(1, p - 1)]        # W
            s += [vid(ix + 1, iy, j) for j in range(1, p - 1)]    # E
            s += [hid(ix, iy, i) for i in range(1, p - 1)]        # S
            s += [hid(ix, iy + 1, i) for i in range(1, p - 1)]    # N
            slot[t] = s
    unknown = -np.ones(nedge, dtype=np.int64)
    idx = np.flatnonzero(~dirichlet)
    unknown[idx] = np.arange(idx.size)
    return Numbering(nedge=nedge, slot=slot, dirichlet=dirichlet, unknown=unknown,
                     nunknown=int(idx.size))


def edge_coordinates(problem, num: Numbering):
    """(x, y) of every edge node, read off the leaf grids."""
    p = problem.p
    xe = np.full(num.nedge, np.nan)
    ye = np.full(num.nedge, np.nan)
    B = lf.flat(p, lf.boundary_nodes(p))
    for t, box in enumerate(problem.boxes()):
        X, Y = lf.grid(box, p)
        xe[num.slot[t]] = X[B]
        ye[num.slot[t]] = Y[B]
    return xe, ye


@dataclass
class LeafData:
    blocks: lf.Blocks
    cond: lf.Condensed
    fi: Optional[np.ndarray]


def build_leaves(problem, leaves: Optional[List[int]] = None) -> List[LeafData]:
    """Leaf matrices and their condensation for every leaf (or a subset)."""
    p = problem.p
    boxes = problem.boxes()
    idx = range(problem.nleaf) if leaves is None else leaves
    out = []
    I = lf.flat(p, lf.interior_nodes(p))
    for t in idx:
        coef = lf.sample_coefficients(problem, boxes[t], p)
        bl = lf.blocks(boxes[t], p, coef)
        fi = None
        if problem.f is not None:
            X, Y = lf.grid(boxes[t], p)
            fi = np.asarray(problem.f(X, Y, np), dtype=np.float64)[I]
        out.append(LeafData(blocks=bl, cond=lf.condense(bl, fi), fi=fi))
    return out


def dirichlet_values(problem, num: Numbering) -> np.ndarray:
    """g at every edge node (only Dirichlet entries are used)."""
    xe, ye = edge_coordinates(problem, num)
    return np.asarray(problem.g(xe, ye, np), dtype=np.float64)


def assemble(num: Numbering, leaves: List[LeafData], gedge: np.ndarray):
    """Reduced matrix A~ (CSC) and right-hand side f~."""
    rows, cols, vals = [], [], []
    rhs = np.zeros(num.nunknown)
    for t, ld in enumerate(leaves):
        ids = num.slot[t]
        isU = ~num.dirichlet[ids]
        U = np.flatnonzero(isU)
        Dn = np.flatnonzero(~isU)
        gU = num.unknown[ids[U]]
        S, w = ld.cond.S, ld.cond.w
        rr, cc = np.meshgrid(gU, gU, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(S[np.ix_(U, U)].ravel())
        r = w[U] + S[np.ix_(U, Dn)] @ gedge[ids[Dn]]
        np.subtract.at(rhs, gU, r)
    A = scipy.sparse.coo_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
        shape=(num.nunknown, num.nunknown)).tocsc()
    return A, rhs


def solve_reduced(A, rhs, dense_limit: int = 5000) -> np.ndarray:
    if A.shape[0] <= dense_limit:
        return np.linalg.solve(A.toarray(), rhs)
    lu = scipy.sparse.linalg.splu(A, permc_spec="COLAMD")
    return lu.solve(rhs)


@dataclass
class Solution:
    uedge: np.ndarray           # [nedge]  all edge nodes (Dirichlet ones = g)
    uint: np.ndarray            # [nleaf, ni]
    num: Numbering


def solve(problem, leaves: Optional[List[LeafData]] = None) -> Solution:
    """Condense every leaf, solve the reduced system, recover interiors."""
    num = numbering(problem.nx, problem.ny, problem.p)
    if leaves is None:
        leaves = build_leaves(problem)
    gedge = dirichlet_values(problem, num)
    A, rhs = assemble(num, leaves, gedge)
    ut = solve_reduced(A, rhs)
    uedge = gedge.copy()
    uedge[~num.dirichlet] = ut
    uint = np.stack([lf.recover(ld.cond, uedge[num.slot[t]]) for t, ld in enumerate(leaves)])
    return Solution(uedge=uedge, uint=uint, num=num)


def full_system(problem, leaves: List[LeafData]):
    """Dense full collocation system over every non-corner node.

    Unknown order: edge nodes (ids of `numbering`), then leaf interiors
    (leaf-major, interior order).  Rows: Dirichlet identity rows and
    interface flux-sum rows at edge nodes; PDE rows at interiors."""
    p = problem.p
    ni = (p - 2) ** 2
    num = numbering(problem.nx, problem.ny, p)
    n = num.nedge + problem.nleaf * ni
    A = np.zeros((n, n))
    b = np.zeros(n)
    gedge = dirichlet_values(problem, num)
    for e in np.flatnonzero(num.dirichlet):
        A[e, e] = 1.0
        b[e] = gedge[e]
    for t, ld in enumerate(leaves):
        ids = num.slot[t]
        icol = num.nedge + t * ni + np.arange(ni)
        bl = ld.blocks
        # PDE rows of this leaf's interior nodes
        A[np.ix_(icol, icol)] += bl.Aii
        A[np.ix_(icol, ids)] += bl.Aib
        if ld.fi is not None:
            b[icol] = ld.fi
        # this leaf's outward flux, added into the rows of its interface nodes
        for s, e in enumerate(ids):
            if num.dirichlet[e]:
                continue
            A[e, icol] += bl.Abi[s]
            A[e, ids] += bl.Abb[s]
    return A, b, num


def relerr_true(sol: Solution, problem) -> float:
    """eq. (accuracy_formula), right: l2 error against the exact solution over
    every non-corner node, each shared edge node counted once."""
    xe, ye = edge_coordinates(problem, sol.num)
    ue_true = np.asarray(problem.exact(xe, ye, np))
    p = problem.p
    I = lf.flat(p, lf.interior_nodes(p))
    ui_true = []
    for box in problem.boxes():
        X, Y = lf.grid(box, p)
        ui_true.append(np.asarray(problem.exact(X[I], Y[I], np)))
    ui_true = np.stack(ui_true)
    num = np.sqrt(np.sum((sol.uedge - ue_true) ** 2) + np.sum((sol.uint - ui_true) ** 2))
    den = np.sqrt(np.sum(ue_true ** 2) + np.sum(ui_true ** 2))
    return float(num / den)


def stack_full(sol: Solution) -> np.ndarray:
    """Solution in the unknown order of `full_system`."""
    return np.concatenate([sol.uedge, sol.uint.ravel()])


def relerr_res(A: np.ndarray, b: np.ndarray, u: np.ndarray) -> float:
    """eq. (accuracy_formula), left, on the full system with its Dirichlet rows."""
    return float(np.linalg.norm(A @ u - b) / np.linalg.norm(b))
