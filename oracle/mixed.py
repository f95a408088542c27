"""Mixed orders within one problem (oracle; test infrastructure only).

Sec. 2 notes that p may be chosen per leaf from a fixed set of values (the
hp-adaptivity it mentions) but does not say how two leaves of different
order meet.  Reading (the minimum rule of conforming hp finite elements):

* the unknowns of a shared edge sit at the edge nodes of the LOWER-order
  leaf (its p-2 interior Chebyshev extreme points of the edge);
* the higher-order leaf's values on that edge are the polynomial through
  the unknowns (degree m_e - 1), evaluated at its own edge nodes
  (interpolation P, m_leaf x m_e);
* its outward flux, known at its own edge nodes, is carried to the edge's
  nodes by the polynomial through those values (degree m_leaf - 1;
  interpolation R, m_e x m_leaf), and the fluxes of the two leaves balance
  at the edge's nodes (Sec. 2: continuity of the flux across the edge).

Equal orders give P = R = I, the uniform scheme of `interface`.  An edge
on the outer boundary belongs to one leaf and carries its own nodes, with
Dirichlet data.  The reduced system is then

    A~ = sum_t  R_t S_t P_t   over the leaf's interface edges,
    f~ = -sum_t R_t (w_t + S_t[:, D] g_D),

and a leaf's boundary values are u_b = P_t u~ on interface edges, g on the
outer boundary.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.sparse

from . import cheb
from . import leaf as lf
from .interface import LeafData, solve_reduced


def edge_nodes(m: int) -> np.ndarray:
    """The m interior points of the order-(m+2) Chebyshev extreme points."""
    return cheb.nodes(m + 2)[1:-1]


def interp_matrix(m_from: int, m_to: int) -> np.ndarray:
    """[m_to, m_from]: values at edge_nodes(m_to) of the degree-(m_from-1)
    polynomial through the values at edge_nodes(m_from) (Lagrange basis)."""
    s = edge_nodes(m_from)
    t = edge_nodes(m_to)
    M = np.ones((m_to, m_from))
    for k in range(m_from):
        for q in range(m_from):
            if q != k:
                M[:, k] *= (t - s[q]) / (s[k] - s[q])
    return M


@dataclass
class MixedNumbering:
    """Edges: vertical (line ix = 0..nx, leaf row iy) first, then horizontal
    (leaf column ix, line iy = 0..ny).  Edge e carries m_edge[e] nodes with
    global ids off[e] .. off[e+1]-1, in increasing coordinate."""

    nx: int
    ny: int
    orders: np.ndarray        # [nleaf]
    m_edge: np.ndarray        # [nedge]
    off: np.ndarray           # [nedge + 1]
    dirichlet: np.ndarray     # [nedge] bool
    leaf_edges: np.ndarray    # [nleaf, 4] edge of the W, E, S, N side
    unknown: np.ndarray       # [nnode] reduced-system index, -1 on Dirichlet nodes
    nunknown: int

    @property
    def nnode(self) -> int:
        return int(self.off[-1])

    def nodes_of(self, e: int) -> np.ndarray:
        return np.arange(self.off[e], self.off[e + 1])


def numbering(nx: int, ny: int, orders) -> MixedNumbering:
    orders = np.asarray(orders, dtype=np.int64)
    nv = (nx + 1) * ny
    nedge = nv + nx * (ny + 1)
    m_edge = np.zeros(nedge, dtype=np.int64)
    dirichlet = np.zeros(nedge, dtype=bool)
    leaf_edges = np.zeros((nx * ny, 4), dtype=np.int64)
    owners: List[List[int]] = [[] for _ in range(nedge)]
    for iy in range(ny):
        for ix in range(nx):
            t = ix + nx * iy
            sides = [ix + (nx + 1) * iy, ix + 1 + (nx + 1) * iy,
                     nv + ix + nx * iy, nv + ix + nx * (iy + 1)]
            leaf_edges[t] = sides
            for e in sides:
                owners[e].append(t)
    for e in range(nedge):
        ms = [int(orders[t]) - 2 for t in owners[e]]
        m_edge[e] = min(ms)
        dirichlet[e] = len(owners[e]) == 1
    off = np.zeros(nedge + 1, dtype=np.int64)
    off[1:] = np.cumsum(m_edge)
    unknown = -np.ones(int(off[-1]), dtype=np.int64)
    k = 0
    for e in range(nedge):
        if not dirichlet[e]:
            unknown[off[e]:off[e + 1]] = np.arange(k, k + m_edge[e])
            k += int(m_edge[e])
    return MixedNumbering(nx=nx, ny=ny, orders=orders, m_edge=m_edge, off=off,
                          dirichlet=dirichlet, leaf_edges=leaf_edges, unknown=unknown,
                          nunknown=k)


def side_maps(num: MixedNumbering, t: int):
    """Per side of leaf t: (edge, P [m_leaf, m_e], R [m_e, m_leaf])."""
    m = int(num.orders[t]) - 2
    out = []
    for s in range(4):
        e = int(num.leaf_edges[t, s])
        me = int(num.m_edge[e])
        out.append((e, interp_matrix(me, m), interp_matrix(m, me)))
    return out


def edge_coordinates(problem, num: MixedNumbering):
    """(x, y) of every edge node."""
    x0, x1, y0, y1 = problem.domain
    hx, hy = (x1 - x0) / num.nx, (y1 - y0) / num.ny
    nv = (num.nx + 1) * num.ny
    X = np.empty(num.nnode)
    Y = np.empty(num.nnode)
    for e in range(num.m_edge.size):
        t = edge_nodes(int(num.m_edge[e]))
        sl = slice(num.off[e], num.off[e + 1])
        if e < nv:
            line, iy = e % (num.nx + 1), e // (num.nx + 1)
            X[sl] = x0 + line * hx
            Y[sl] = y0 + iy * hy + (t + 1.0) * hy / 2.0
        else:
            ix, line = (e - nv) % num.nx, (e - nv) // num.nx
            X[sl] = x0 + ix * hx + (t + 1.0) * hx / 2.0
            Y[sl] = y0 + line * hy
    return X, Y


def build_leaves(problem) -> List[LeafData]:
    """Each leaf condensed at its own order (plain per-leaf oracle)."""
    boxes = problem.boxes()
    out = []
    for t in range(problem.nleaf):
        p = int(problem.orders[t])
        coef = lf.sample_coefficients(problem, boxes[t], p)
        bl = lf.blocks(boxes[t], p, coef)
        fi = None
        if problem.f is not None:
            X, Y = lf.grid(boxes[t], p)
            fi = np.asarray(problem.f(X, Y, np), dtype=np.float64)[lf.flat(p, lf.interior_nodes(p))]
        out.append(LeafData(blocks=bl, cond=lf.condense(bl, fi), fi=fi))
    return out


def assemble(num: MixedNumbering, leaves: List[LeafData], gedge: np.ndarray):
    """Reduced matrix (CSC) and right-hand side, with the interpolations."""
    rows, cols, vals = [], [], []
    rhs = np.zeros(num.nunknown)
    for t, ld in enumerate(leaves):
        m = int(num.orders[t]) - 2
        maps = side_maps(num, t)
        S, w = ld.cond.S, ld.cond.w
        gb = np.zeros(4 * m)                    # the leaf's Dirichlet values
        for s, (e, P, R) in enumerate(maps):
            if num.dirichlet[e]:
                gb[s * m:(s + 1) * m] = gedge[num.nodes_of(e)]
        flux0 = w + S @ gb                      # flux of the known part
        for s, (e, P, R) in enumerate(maps):
            if num.dirichlet[e]:
                continue
            ru = num.unknown[num.nodes_of(e)]
            np.subtract.at(rhs, ru, R @ flux0[s * m:(s + 1) * m])
            for q, (e2, P2, R2) in enumerate(maps):
                if num.dirichlet[e2]:
                    continue
                cu = num.unknown[num.nodes_of(e2)]
                blk = R @ S[s * m:(s + 1) * m, q * m:(q + 1) * m] @ P2
                rr, cc = np.meshgrid(ru, cu, indexing="ij")
                rows.append(rr.ravel())
                cols.append(cc.ravel())
                vals.append(blk.ravel())
    A = scipy.sparse.coo_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
        shape=(num.nunknown, num.nunknown)).tocsc()
    return A, rhs


def leaf_boundary_values(num: MixedNumbering, t: int, uedge: np.ndarray) -> np.ndarray:
    """u_b of leaf t: P u on interface edges, the edge values (its own nodes)
    on the outer boundary."""
    m = int(num.orders[t]) - 2
    ub = np.empty(4 * m)
    for s, (e, P, R) in enumerate(side_maps(num, t)):
        ub[s * m:(s + 1) * m] = P @ uedge[num.nodes_of(e)]
    return ub


@dataclass
class MixedSolution:
    uedge: np.ndarray          # [nnode]
    ub: List[np.ndarray]       # per leaf, at its own boundary slots
    uint: List[np.ndarray]     # per leaf interiors
    num: MixedNumbering


def dirichlet_values(problem, num: MixedNumbering) -> np.ndarray:
    X, Y = edge_coordinates(problem, num)
    return np.asarray(problem.g(X, Y, np), dtype=np.float64)


def solve(problem, leaves=None) -> MixedSolution:
    num = numbering(problem.nx, problem.ny, problem.orders)
    if leaves is None:
        leaves = build_leaves(problem)
    gedge = dirichlet_values(problem, num)
    A, rhs = assemble(num, leaves, gedge)
    uedge = gedge.copy()
    uedge[num.unknown >= 0] = 0.0
    ut = solve_reduced(A, rhs)
    idx = np.flatnonzero(num.unknown >= 0)
    uedge[idx] = ut[num.unknown[idx]]
    ub = [leaf_boundary_values(num, t, uedge) for t in range(problem.nleaf)]
    uint = [lf.recover(ld.cond, ub[t]) for t, ld in enumerate(leaves)]
    return MixedSolution(uedge=uedge, ub=ub, uint=uint, num=num)


def full_system(problem, leaves: List[LeafData]):
    """Dense full system over the edge nodes and every leaf's interior:
    identity rows at Dirichlet nodes, flux-balance rows (R applied to each
    leaf's flux) at interface nodes, PDE rows at interiors, with every
    leaf's boundary values taken through P."""
    num = numbering(problem.nx, problem.ny, problem.orders)
    ni = [(int(p) - 2) ** 2 for p in problem.orders]
    ioff = np.concatenate([[0], np.cumsum(ni)]) + num.nnode
    n = int(ioff[-1])
    A = np.zeros((n, n))
    b = np.zeros(n)
    gedge = dirichlet_values(problem, num)
    for e in np.flatnonzero(num.dirichlet):
        nd = num.nodes_of(e)
        A[nd, nd] = 1.0
        b[nd] = gedge[nd]
    for t, ld in enumerate(leaves):
        m = int(num.orders[t]) - 2
        bl = ld.blocks
        icol = np.arange(ioff[t], ioff[t + 1])
        maps = side_maps(num, t)
        # u_b = Pi u_edge: [4m, nnode] sparse in effect
        Pi = np.zeros((4 * m, num.nnode))
        for s, (e, P, R) in enumerate(maps):
            Pi[s * m:(s + 1) * m, num.nodes_of(e)] = P
        A[np.ix_(icol, icol)] += bl.Aii
        A[icol, :num.nnode] += bl.Aib @ Pi
        if ld.fi is not None:
            b[icol] = ld.fi
        for s, (e, P, R) in enumerate(maps):
            if num.dirichlet[e]:
                continue
            rows = num.nodes_of(e)
            A[np.ix_(rows, icol)] += R @ bl.Abi[s * m:(s + 1) * m]
            A[rows, :num.nnode] += R @ bl.Abb[s * m:(s + 1) * m] @ Pi
    return A, b, num


def stack_full(sol: MixedSolution) -> np.ndarray:
    return np.concatenate([sol.uedge] + [u for u in sol.uint])


def relerr_true(sol: MixedSolution, problem) -> float:
    """eq. (accuracy_formula), right: l2 error against the exact solution over
    every edge node (each once) and every leaf interior node."""
    X, Y = edge_coordinates(problem, sol.num)
    ue = np.asarray(problem.exact(X, Y, np))
    boxes = problem.boxes()
    d2 = np.sum((sol.uedge - ue) ** 2)
    n2 = np.sum(ue ** 2)
    for t in range(problem.nleaf):
        p = int(problem.orders[t])
        Xi, Yi = lf.grid(boxes[t], p)
        I = lf.flat(p, lf.interior_nodes(p))
        ui = np.asarray(problem.exact(Xi[I], Yi[I], np))
        d2 += np.sum((sol.uint[t] - ui) ** 2)
        n2 += np.sum(ui ** 2)
    return float(np.sqrt(d2 / n2))
