"""Host-side harness around the HIP library.

* prepares the device inputs of one or several problems (leaf boxes and the
  coefficient fields sampled at the node coordinates the library reports);
* calls the library's condense / recover entry points;
* drives the library's FP64 interface solve (nested dissection on the
  device) and, for comparison, a host solve of the same reduced system
  (SciPy SuperLU with COLAMD, Sec. 3.1).  The interface solve is not part of
  the timed leaf-condensation path.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import hps
from .inputs import FIELDS, Problem


def _torch():
    import torch
    return torch


@dataclass
class GroupView:
    problem: Problem
    p: int
    nleaf: int
    ni: int
    nb: int
    leaf0: int
    box: object
    coef: dict
    xy: object


class LeafBatch:
    """One library batch holding one group per problem."""

    def __init__(self, problems: Sequence[Problem], device: str = "cuda", stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no ROCm device visible to torch")
        self.device = torch.device(device)
        self.problems = list(problems)
        self.ctx = hps.hps_ctx_create(stream)
        descs = []
        self.groups: List[GroupView] = []
        leaf0 = 0
        for prob in self.problems:
            box = torch.as_tensor(prob.boxes(), dtype=torch.float64, device=self.device).contiguous()
            coef = {}
            for name in FIELDS:
                if prob.has(name):
                    coef[name] = torch.empty((prob.nleaf, prob.p * prob.p), dtype=torch.float64,
                                             device=self.device)
            d = {"p": prob.p, "box": box}
            d.update(coef)
            descs.append(d)
            self.groups.append(GroupView(prob, prob.p, prob.nleaf, (prob.p - 2) ** 2,
                                         4 * (prob.p - 2), leaf0, box, coef, None))
            leaf0 += prob.nleaf
        self.nleaf = leaf0
        self.batch = hps.hps_leaf_build(self.ctx, descs)
        for gi, G in enumerate(self.groups):
            xy = torch.empty((G.nleaf, G.p * G.p, 2), dtype=torch.float64, device=self.device)
            hps.hps_leaf_nodes(self.batch, gi, xy)
            G.xy = xy
            X, Y = xy[..., 0], xy[..., 1]
            for name, t in G.coef.items():
                t.copy_(G.problem.sample(name, X, Y, torch))
        self.ni_total = sum(G.nleaf * G.ni for G in self.groups)
        self.nb_total = sum(G.nleaf * G.nb for G in self.groups)
        self.s_total = sum(G.nleaf * G.nb * G.nb for G in self.groups)

    # -- outputs -----------------------------------------------------------
    def alloc_outputs(self):
        torch = _torch()
        S = torch.empty(self.s_total, dtype=torch.float64, device=self.device)
        w = torch.empty(self.nb_total, dtype=torch.float64, device=self.device)
        info = torch.empty(self.nleaf, dtype=torch.int32, device=self.device)
        return S, w, info

    def split(self, flat, kind: str):
        """Per-group views of a flat output: kind in S, w, ui, f, Xt."""
        out, off = [], 0
        for G in self.groups:
            if kind == "S":
                n, shape = G.nleaf * G.nb * G.nb, (G.nleaf, G.nb, G.nb)
            elif kind in ("w", "ub"):
                n, shape = G.nleaf * G.nb, (G.nleaf, G.nb)
            elif kind in ("ui", "f", "h"):
                n, shape = G.nleaf * G.ni, (G.nleaf, G.ni)
            elif kind == "Xt":
                n, shape = G.nleaf * G.nb * G.ni, (G.nleaf, G.nb, G.ni)
            else:
                raise ValueError(kind)
            out.append(flat[off:off + n].view(shape))
            off += n
        return out

    def interior_f(self):
        """f at the interior nodes of every leaf, flat (None if no problem has f)."""
        torch = _torch()
        if all(G.problem.f is None for G in self.groups):
            return None
        parts = []
        for G in self.groups:
            m = G.p - 2
            ij = [(i, j) for j in range(1, G.p - 1) for i in range(1, G.p - 1)]
            idx = torch.tensor([i + G.p * j for (i, j) in ij], device=self.device)
            xy = G.xy[:, idx, :]
            if G.problem.f is None:
                parts.append(torch.zeros((G.nleaf, m * m), dtype=torch.float64, device=self.device))
            else:
                parts.append(G.problem.f(xy[..., 0], xy[..., 1], torch))
        return torch.cat([t.reshape(-1) for t in parts]).contiguous()

    def condense(self, prec=hps.HPS_FP64, tol: float = 0.0, max_refine: int = 2, f=None,
                 S=None, w=None, info=None, sync: bool = False, allow=(hps.HPS_OK,)):
        if S is None:
            S, w, info = self.alloc_outputs()
        st = hps.hps_leaf_condense(self.batch, prec, tol, max_refine, f, S, w, info,
                                   hps.HPS_SYNC if sync else 0, allow=allow)
        return S, w, info, st

    def recover(self, ub, f=None, refactor: bool = False, ui=None, sync: bool = False):
        torch = _torch()
        if ui is None:
            ui = torch.empty(self.ni_total, dtype=torch.float64, device=self.device)
        flags = (hps.HPS_RECOVER_REFACTOR if refactor else 0) | (hps.HPS_SYNC if sync else 0)
        hps.hps_leaf_recover(self.batch, ub, f, ui, flags)
        return ui

    def export(self):
        torch = _torch()
        xt_total = sum(G.nleaf * G.nb * G.ni for G in self.groups)
        Xt = torch.empty(xt_total, dtype=torch.float64, device=self.device)
        h = torch.empty(self.ni_total, dtype=torch.float64, device=self.device)
        hps.hps_batch_export(self.batch, Xt, h)
        return Xt, h

    def close(self):
        if getattr(self, "batch", None):
            hps.hps_batch_destroy(self.batch)
            self.batch = None
        if getattr(self, "ctx", None):
            hps.hps_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# interface solve on the device (include/hps_iface.h)
# ---------------------------------------------------------------------------

def boundary_index(p: int):
    """Flat grid index (i + p*j) of each boundary slot, in the W, E, S, N order."""
    r = range(1, p - 1)
    return ([p * j for j in r] + [p - 1 + p * j for j in r] + [i for i in r]
            + [i + p * (p - 1) for i in r])


def dirichlet_data(G: GroupView):
    """g at every boundary slot of every leaf of the group, [nleaf, nb] on the
    device (the interface solve reads only the slots on the outer boundary)."""
    torch = _torch()
    idx = torch.tensor(boundary_index(G.p), device=G.xy.device)
    xy = G.xy[:, idx, :]
    return G.problem.g(xy[..., 0], xy[..., 1], torch).contiguous()


def dirichlet_data_batch(batch: "LeafBatch"):
    """dirichlet_data of every group, concatenated in the batch's slot layout."""
    torch = _torch()
    return torch.cat([dirichlet_data(G).reshape(-1) for G in batch.groups]).contiguous()


def interface_unknowns(problem) -> int:
    """Unknowns of the reduced system: the nodes of every edge shared by two
    leaves, at the lower of the two orders."""
    nx, ny = problem.nx, problem.ny
    orders = getattr(problem, "orders", None)
    if orders is None:
        return ((nx - 1) * ny + nx * (ny - 1)) * (problem.p - 2)
    o = np.asarray(orders).reshape(ny, nx) - 2
    return int(np.minimum(o[:, :-1], o[:, 1:]).sum() + np.minimum(o[:-1, :], o[1:, :]).sum())


def batch_offsets(batch: "LeafBatch", problem):
    """Offsets of every grid leaf's S and boundary slots in a batch whose
    groups are `problem`'s leaf sets (one per order, in `problem.groups()`
    order): leaf t's S starts at s_off[t] doubles, its slots at b_off[t]."""
    s_off = np.zeros(problem.nleaf, dtype=np.int64)
    b_off = np.zeros(problem.nleaf, dtype=np.int64)
    s0 = b0 = 0
    for G in batch.groups:
        k = np.arange(G.nleaf)
        s_off[G.problem.leaves] = s0 + k * G.nb * G.nb
        b_off[G.problem.leaves] = b0 + k * G.nb
        s0 += G.nleaf * G.nb * G.nb
        b0 += G.nleaf * G.nb
    return s_off, b_off


class InterfaceSolver:
    """The library's nested-dissection solve of the reduced system for one
    problem: a rectangle of nx x ny leaves of one order, or a MixedProblem
    (orders per leaf) condensed by `batch` with one group per order."""

    def __init__(self, ctx: int, problem, batch: "LeafBatch" = None):
        self.problem = problem
        orders = getattr(problem, "orders", None)
        if orders is None:
            self.plan = hps.hps_iface_plan(problem.p, problem.nx, problem.ny)
            self.it = hps.hps_iface_create(ctx, problem.p, problem.nx, problem.ny)
        else:
            if batch is None:
                raise ValueError("a problem with per-leaf orders needs its batch for the layout")
            s_off, b_off = batch_offsets(batch, problem)
            self.plan = hps.hps_iface_plan_orders(problem.nx, problem.ny, orders)
            self.it = hps.hps_iface_create_orders(ctx, problem.nx, problem.ny, orders, s_off, b_off)

    def factor(self, S, info=None, sync: bool = False, allow=(hps.HPS_OK,)):
        return hps.hps_iface_factor(self.it, S, info, hps.HPS_SYNC if sync else 0, allow=allow)

    def solve(self, S, w, g, ub=None, sync: bool = False):
        torch = _torch()
        if ub is None:
            ub = torch.empty(g.numel(), dtype=torch.float64, device=g.device)
        hps.hps_iface_solve(self.it, S, w, g, ub, hps.HPS_SYNC if sync else 0)
        return ub

    def close(self):
        if getattr(self, "it", None):
            hps.hps_iface_destroy(self.it)
            self.it = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# host interface solve (eq. (hps_reduced)), for end-to-end runs
# ---------------------------------------------------------------------------

def edge_ids(nx: int, ny: int, p: int):
    """Global edge-node ids of each leaf's boundary slots (W, E, S, N) and a
    Dirichlet mask.  Vertical edge lines ix = 0..nx come first, then the
    horizontal lines iy = 0..ny; p-2 nodes per leaf edge."""
    m = p - 2
    nv = (nx + 1) * ny * m
    ids = np.empty((nx * ny, 4 * m), dtype=np.int64)
    r = np.arange(m)
    for iy in range(ny):
        for ix in range(nx):
            t = ix + nx * iy
            ids[t, 0:m] = (ix + (nx + 1) * iy) * m + r
            ids[t, m:2 * m] = (ix + 1 + (nx + 1) * iy) * m + r
            ids[t, 2 * m:3 * m] = nv + (ix + nx * iy) * m + r
            ids[t, 3 * m:4 * m] = nv + (ix + nx * (iy + 1)) * m + r
    nedge = nv + nx * (ny + 1) * m
    dir_mask = np.zeros(nedge, dtype=bool)
    for iy in range(ny):
        dir_mask[(0 + (nx + 1) * iy) * m + r] = True
        dir_mask[(nx + (nx + 1) * iy) * m + r] = True
    for ix in range(nx):
        dir_mask[nv + ix * m + r] = True
        dir_mask[nv + (ix + nx * ny) * m + r] = True
    return ids, dir_mask


def interface_solve(problem: Problem, S: np.ndarray, w: Optional[np.ndarray], xy_b: np.ndarray):
    """Solve the reduced system for one problem.

    S: [nleaf, nb, nb]; w: [nleaf, nb] or None; xy_b: [nleaf, nb, 2] boundary
    node coordinates.  Returns ub [nleaf, nb] (interface values solved,
    Dirichlet values from problem.g)."""
    import scipy.sparse
    import scipy.sparse.linalg

    ids, dmask = edge_ids(problem.nx, problem.ny, problem.p)
    nedge = dmask.size
    g = np.zeros(nedge)
    gx = np.zeros(nedge)
    gy = np.zeros(nedge)
    gx[ids.ravel()] = xy_b[..., 0].ravel()
    gy[ids.ravel()] = xy_b[..., 1].ravel()
    g[dmask] = np.asarray(problem.g(gx[dmask], gy[dmask], np))
    unk = -np.ones(nedge, dtype=np.int64)
    unk[~dmask] = np.arange(int((~dmask).sum()))
    n = int((~dmask).sum())
    rows, cols, vals = [], [], []
    rhs = np.zeros(n)
    for t in range(problem.nleaf):
        e = ids[t]
        U = np.flatnonzero(~dmask[e])
        Dn = np.flatnonzero(dmask[e])
        gu = unk[e[U]]
        St = S[t]
        rows.append(np.repeat(gu, U.size))
        cols.append(np.tile(gu, U.size))
        vals.append(St[np.ix_(U, U)].ravel())
        r = St[np.ix_(U, Dn)] @ g[e[Dn]]
        if w is not None:
            r = r + w[t][U]
        np.subtract.at(rhs, gu, r)
    A = scipy.sparse.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                shape=(n, n))
    sol = scipy.sparse.linalg.splu(A, permc_spec="COLAMD").solve(rhs)
    u = g.copy()
    u[~dmask] = sol
    return u[ids]
