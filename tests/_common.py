"""Shared helpers for the GPU parity tests (oracle side + error measures)."""
import numpy as np

from oracle import leaf as lf


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


def leaf_bar(Aii, tol):
    """Per-leaf error bar: `tol`, or the FP64 floor 10 * cond_2(A_ii) * 2^-53
    where that is larger.  A leaf close to a Dirichlet resonance of its box
    has a nearly singular A_ii; the rounding of the operator entries alone
    (a relative change of 2^-53 each, which two correct FP64 builds may
    differ by) moves X by up to about cond(A_ii) * 2^-53 relative."""
    return max(tol, 10.0 * float(np.linalg.cond(Aii)) * 2.0 ** -53)
