"""Shared helpers for the GPU parity tests (oracle side + error measures)."""
import sys

import numpy as np

from oracle import leaf as lf

EPS64 = 2.0 ** -53


def oracle_leaf(problem, t, fi=None):
    """Oracle blocks and condensation of leaf t of `problem`."""
    box = problem.boxes()[t]
    coef = lf.sample_coefficients(problem, box, problem.p)
    bl = lf.blocks(box, problem.p, coef)
    return bl, lf.condense(bl, fi)


def oracle_interior_f(problem, t):
    if problem.f is None:
        return None
    p = problem.p
    X, Y = lf.grid(problem.boxes()[t], p)
    I = lf.flat(p, lf.interior_nodes(p))
    return np.asarray(problem.f(X[I], Y[I], np), dtype=np.float64)


def relerr(a, b):
    """Normwise relative error ||a - b||_F / ||b||_F (0 if both are 0)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    na = np.linalg.norm(a - b)
    if nb == 0.0:
        return float(na)
    return float(na / nb)


def sample_leaves(nleaf, count, seed=0):
    """A seeded sample of leaf indices that always includes the first and last."""
    rng = np.random.default_rng(seed)
    k = min(count, nleaf)
    idx = set(rng.choice(nleaf, size=k, replace=False).tolist())
    idx.update({0, nleaf - 1})
    return sorted(idx)


def fp64_floor(Aii):
    """10 cond_2(A_ii) 2^-53: how far two correct FP64 results for the leaf may
    lie apart.  Rounding the operator entries alone (a relative change of at
    most 2^-53 each, by which two correct FP64 builds of A_ii may differ) moves
    X = A_ii^{-1} A_ib by up to about cond_2(A_ii) 2^-53 relative."""
    return 10.0 * float(np.linalg.cond(Aii)) * EPS64


def leaf_bar(Aii, tol):
    """Per-leaf error bar: `tol`, or the FP64 floor where that is larger."""
    return max(tol, fp64_floor(Aii))


def backward_error(Aii, Aib, X):
    """||A_ib - A_ii X||_F / (||A_ii||_F ||X||_F + ||A_ib||_F), in FP64 on the
    host: independent of the conditioning of A_ii, so it checks a computed X
    tightly even on a leaf whose forward error may sit at the FP64 floor."""
    r = Aib - Aii @ X
    return float(np.linalg.norm(r) /
                 (np.linalg.norm(Aii) * np.linalg.norm(X) + np.linalg.norm(Aib)))


def p7_bar(ni):
    """Bar for the backward error of X: 10 ni 2^-53."""
    return 10.0 * ni * EPS64


class BarLog:
    """Checks errors against the fixed tolerance, raising the bar to the FP64
    floor of a leaf only where the error exceeds the tolerance, and reports
    how many leaves needed that (with their condition numbers)."""

    def __init__(self, label):
        self.label = label
        self.checked = 0
        self.raised = []          # (leaf id, quantity, error, cond)
        self.worst = {}

    def check(self, leaf, name, err, tol, Aii):
        self.checked += 1
        self.worst[name] = max(self.worst.get(name, 0.0), err)
        if err <= tol:
            return True
        floor = fp64_floor(Aii)
        self.raised.append((leaf, name, err, floor / (10.0 * EPS64)))
        return err <= floor

    def report(self):
        conds = [c for (_, _, _, c) in self.raised]
        msg = (f"  {self.label}: {self.checked} checks, worst "
               + ", ".join(f"{k} {v:.2e}" for k, v in sorted(self.worst.items()))
               + f"; raised to the FP64 floor on {len(self.raised)}")
        if conds:
            msg += f" (cond {min(conds):.1e} .. {max(conds):.1e}: " + ", ".join(
                f"leaf {l} {n} {e:.1e}" for (l, n, e, _) in self.raised[:6]) + ")"
        print(msg, file=sys.stderr, flush=True)
        return msg


def cond1_estimate(A) -> float:
    """cond_1 of a sparse matrix: ||A||_1 exactly, ||A^{-1}||_1 by the
    Hager-Higham block estimator (scipy onenormest) on SuperLU factors.
    For the FP64 floor of large reduced systems, where a dense cond_2 is out
    of reach."""
    import scipy.sparse.linalg as sla
    lu = sla.splu(A.tocsc(), permc_spec="COLAMD")
    n = A.shape[0]
    inv = sla.LinearOperator((n, n), matvec=lu.solve,
                             rmatvec=lambda x: lu.solve(x, trans="T"), dtype=np.float64)
    a1 = float(abs(A).sum(axis=0).max())
    return a1 * float(sla.onenormest(inv))
