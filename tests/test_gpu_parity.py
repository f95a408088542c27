"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances, normwise relative error per leaf.  FP64 path: 1e-10 on X, h, S,
w.  FP32 + FP64 refinement: 1e-9 on S, h, w and on the recovered u, the
target the method is built for (1e-8 on X).  Either bar is raised to the
FP64 floor 10 cond_2(A_ii) 2^-53 on a leaf where that is larger: a leaf near
a Dirichlet resonance of its box (cond up to ~1e8 on the p = 32 grids here)
cannot be pinned closer than that by any FP64 computation, since rounding
the operator entries alone moves X that far.
"""
import math
import sys

import numpy as np
import pytest

from _common import leaf_bar, oracle_interior_f, oracle_leaf, relerr, sample_leaves
from oracle import leaf as lf
from oracle import interface as itf
from paper_2211_14969_amd import hps, inputs

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL_MIXED = 1e-9


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.fail("no GPU visible")
    hps.load()          # fails loudly if the library is missing
    return T


def _batch(problems):
    from paper_2211_14969_amd.harness import LeafBatch
    return LeafBatch(problems)


def _small(p, nx=2, ny=2, kappa=None, kind="bump"):
    if kind == "tiny":
        return inputs.tiny(p=p, n=nx, kappa=kappa or 10.0)
    if kind == "annulus":
        return inputs.annulus(p=p, ntheta=nx, nr=ny, kappa=kappa or 12.0)
    pr = inputs.multi_bump(p=p, n=nx, kappa=kappa or 3.0 * p, seed=3)
    return pr


# --------------------------------------------------------------------------
# operator blocks
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p,kind", [(4, "bump"), (8, "tiny"), (12, "annulus"), (16, "bump"),
                                    (21, "annulus"), (32, "bump")])
def test_operator_blocks(torch, p, kind):
    prob = _small(p, 2, 2, kind=kind)
    _say(f"operator p={p} {kind}")
    B = _batch([prob])
    ni, nb = (p - 2) ** 2, 4 * (p - 2)
    L = prob.nleaf
    mk = lambda *s: torch.empty(s, dtype=torch.float64, device="cuda")
    Aii, Aib, Abi, Abb = mk(L, ni, ni), mk(L, ni, nb), mk(L, nb, ni), mk(L, nb, nb)
    hps.hps_leaf_operator(B.batch, 0, Aii, Aib, Abi, Abb)
    torch.cuda.synchronize()
    for t in range(L):
        bl, _ = oracle_leaf(prob, t)
        for name, got in (("Aii", Aii), ("Aib", Aib), ("Abi", Abi), ("Abb", Abb)):
            assert relerr(got[t].cpu().numpy(), getattr(bl, name)) < 1e-13, (name, t)
    B.close()


# --------------------------------------------------------------------------
# condensation, FP64 and FP32 + refinement, across orders (ragged tiles)
# --------------------------------------------------------------------------
ORDERS = [4, 5, 6, 8, 12, 13, 16, 20, 24, 30, 32]


def _check_condense(torch, prob, prec, tol, with_x=True, leaves=None, max_refine=3):
    B = _batch([prob])
    S, w, info, st = B.condense(prec=prec, max_refine=max_refine, sync=True)
    assert st == hps.HPS_OK
    Xt, h = B.export()
    torch.cuda.synchronize()
    nb, ni = 4 * (prob.p - 2), (prob.p - 2) ** 2
    S = S.view(prob.nleaf, nb, nb).cpu().numpy()
    Xt = Xt.view(prob.nleaf, nb, ni).cpu().numpy()
    assert np.all(info.cpu().numpy() == 0)
    worst = {"S": 0.0, "X": 0.0, "S/bar": 0.0}
    for t in (leaves if leaves is not None else range(prob.nleaf)):
        bl, c = oracle_leaf(prob, t)
        bar = leaf_bar(bl.Aii, tol)
        eS, eX = relerr(S[t], c.S), relerr(Xt[t].T, c.X)
        worst["S"] = max(worst["S"], eS)
        worst["X"] = max(worst["X"], eX)
        worst["S/bar"] = max(worst["S/bar"], eS / bar)
        assert eS <= bar, (t, eS, bar)
        if with_x:
            assert eX <= (bar if prec == hps.HPS_FP64 else max(bar, 1e-8)), (t, eX, bar)
    _say(f"  {prob.name} prec={prec} worst {worst}")
    B.close()
    return worst


@pytest.mark.parametrize("p", ORDERS)
def test_condense_fp64_orders(torch, p):
    _say(f"condense fp64 p={p}")
    _check_condense(torch, _small(p, 3), hps.HPS_FP64, TOL64)


@pytest.mark.parametrize("p", ORDERS)
def test_condense_fp32_refine_orders(torch, p):
    _say(f"condense fp32+refine p={p}")
    _check_condense(torch, _small(p, 3), hps.HPS_FP32_REFINE, TOL_MIXED)


@pytest.mark.parametrize("p", [o for o in ORDERS if o <= 16])
def test_condense_fp32_register_resident(torch, p):
    """The register-resident FP32 factorisation (tuning variant 3) meets the
    same bar as the streaming one, with the f column present too."""
    _say(f"condense fp32 register-resident p={p}")
    prob = _small(p, 3)
    B = _batch([prob])
    hps.hps_batch_set_tuning(B.batch, 0, 3, 0)
    S, w, info, st = B.condense(prec=hps.HPS_FP32_REFINE, max_refine=3, sync=True)
    assert st == hps.HPS_OK and bool((info == 0).all())
    nb = 4 * (p - 2)
    Sg = S.view(prob.nleaf, nb, nb).cpu().numpy()
    for t in range(prob.nleaf):
        bl, c = oracle_leaf(prob, t)
        assert relerr(Sg[t], c.S) <= leaf_bar(bl.Aii, TOL_MIXED), t
    B.close()
    fp = _forced_problem(p if p >= 6 else 6)
    B = _batch([fp])
    hps.hps_batch_set_tuning(B.batch, 0, 3, 0)
    f = B.interior_f()
    S, w, info, st = B.condense(prec=hps.HPS_FP32_REFINE, f=f, max_refine=3, sync=True)
    assert st == hps.HPS_OK
    nb, ni = 4 * (fp.p - 2), (fp.p - 2) ** 2
    _, h = B.export()
    Sg, wg, hg = (S.view(-1, nb, nb).cpu().numpy(), w.view(-1, nb).cpu().numpy(),
                  h.view(-1, ni).cpu().numpy())
    for t in range(fp.nleaf):
        bl, c = oracle_leaf(fp, t, oracle_interior_f(fp, t))
        bar = leaf_bar(bl.Aii, TOL_MIXED)
        assert relerr(Sg[t], c.S) <= bar and relerr(wg[t], c.w) <= bar and relerr(hg[t], c.h) <= bar
    B.close()


# Work matrices above 256 rows: panels in pairs with the first panel's
# multipliers re-read from the work matrix (variant 2), at both occupancies
# (64 and 128 column chunks select one or two workgroups per CU), with an
# even and an odd number of row tiles (p = 23: 28 tiles; p = 20, 32: odd),
# the single-panel variant on an even tile count, and the FP64 default at
# exactly 256 rows (p = 18), which takes the one-panel-in-LDS pairs.
@pytest.mark.parametrize("p,prec,variant,chunk", [
    (23, hps.HPS_FP64, 2, 0), (23, hps.HPS_FP32_REFINE, 2, 0), (20, hps.HPS_FP64, 2, 64),
    (20, hps.HPS_FP32_REFINE, 2, 0), (32, hps.HPS_FP32_REFINE, 2, 128), (32, hps.HPS_FP64, 2, 64),
    (26, hps.HPS_FP64, 1, 0), (18, hps.HPS_FP64, 0, 0)])
def test_condense_large_factor_variants(torch, p, prec, variant, chunk):
    _say(f"condense large p={p} prec={prec} variant={variant} chunk={chunk}")
    prob = _small(p, 2)
    B = _batch([prob])
    hps.hps_batch_set_tuning(B.batch, 0, variant, chunk)
    S, w, info, st = B.condense(prec=prec, max_refine=3, sync=True)
    assert st == hps.HPS_OK and bool((info == 0).all())
    Xt, _ = B.export()
    nb, ni = 4 * (p - 2), (p - 2) ** 2
    Sg, Xg = S.view(-1, nb, nb).cpu().numpy(), Xt.view(-1, nb, ni).cpu().numpy()
    tol = TOL64 if prec == hps.HPS_FP64 else TOL_MIXED
    for t in range(prob.nleaf):
        bl, c = oracle_leaf(prob, t)
        bar = leaf_bar(bl.Aii, tol)
        assert relerr(Sg[t], c.S) <= bar, t
        assert relerr(Xg[t].T, c.X) <= (bar if prec == hps.HPS_FP64 else max(bar, 1e-8)), t
    B.close()
    # with the body-load column
    fp = _forced_problem(p)
    B = _batch([fp])
    hps.hps_batch_set_tuning(B.batch, 0, variant, chunk)
    f = B.interior_f()
    S, w, info, st = B.condense(prec=prec, f=f, max_refine=3, sync=True)
    assert st == hps.HPS_OK
    _, h = B.export()
    Sg, wg, hg = (S.view(-1, nb, nb).cpu().numpy(), w.view(-1, nb).cpu().numpy(),
                  h.view(-1, ni).cpu().numpy())
    for t in range(fp.nleaf):
        bl, c = oracle_leaf(fp, t, oracle_interior_f(fp, t))
        bar = leaf_bar(bl.Aii, tol)
        assert relerr(Sg[t], c.S) <= bar and relerr(wg[t], c.w) <= bar and relerr(hg[t], c.h) <= bar
    B.close()


@pytest.mark.parametrize("prec", [hps.HPS_FP64, hps.HPS_FP32_REFINE])
def test_annulus_variable_coefficients(torch, prec):
    _say(f"annulus prec={prec}")
    _check_condense(torch, inputs.annulus(p=20, ntheta=4, nr=2, kappa=150.0), prec,
                    TOL64 if prec == hps.HPS_FP64 else TOL_MIXED)


def test_single_leaf(torch):
    _say("single leaf p=16")
    _check_condense(torch, _small(16, 1, 1), hps.HPS_FP64, TOL64)


# --------------------------------------------------------------------------
# body load f: h and w
# --------------------------------------------------------------------------
def _forced_problem(p, nx=2, ny=2):
    kappa = 6.0
    u = lambda x, y, xp: xp.sin(3 * x) * xp.cos(2 * y) + x * y
    f = lambda x, y, xp: (13.0 - kappa ** 2) * xp.sin(3 * x) * xp.cos(2 * y) - kappa ** 2 * x * y
    return inputs.Problem(name=f"forced_p{p}", nx=nx, ny=ny, p=p, kappa=kappa,
                          coef={"k2b": lambda x, y, xp: xp.zeros_like(x) + kappa ** 2},
                          g=u, exact=u, f=f)


# p = 18 with f: five right-hand-side column tiles (the widest register-
# resident solves); p = 28 with f: the 2 x 2-tile MFMA residual's f column.
@pytest.mark.parametrize("prec,p", [(hps.HPS_FP64, 10), (hps.HPS_FP64, 17), (hps.HPS_FP64, 18),
                                    (hps.HPS_FP32_REFINE, 10), (hps.HPS_FP32_REFINE, 17),
                                    (hps.HPS_FP32_REFINE, 18), (hps.HPS_FP32_REFINE, 28)])
def test_condense_with_body_load(torch, prec, p):
    _say(f"forced prec={prec} p={p}")
    prob = _forced_problem(p)
    B = _batch([prob])
    f = B.interior_f()
    S, w, info, st = B.condense(prec=prec, f=f, max_refine=3, sync=True)
    Xt, h = B.export()
    nb, ni = 4 * (p - 2), (p - 2) ** 2
    S, w, h = (S.view(-1, nb, nb).cpu().numpy(), w.view(-1, nb).cpu().numpy(),
               h.view(-1, ni).cpu().numpy())
    tol = TOL64 if prec == hps.HPS_FP64 else TOL_MIXED
    for t in range(prob.nleaf):
        _, c = oracle_leaf(prob, t, oracle_interior_f(prob, t))
        assert relerr(S[t], c.S) <= tol
        assert relerr(h[t], c.h) <= tol
        assert relerr(w[t], c.w) <= tol
    B.close()


# --------------------------------------------------------------------------
# recovery: stored X and the re-factor mode, fed the oracle's u_b
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [hps.HPS_FP64, hps.HPS_FP32_REFINE])
def test_recover_with_oracle_boundary_values(torch, prec):
    prob = inputs.tiny()
    _say(f"recover tiny prec={prec}")
    sol = itf.solve(prob)
    ub = np.stack([sol.uedge[sol.num.slot[t]] for t in range(prob.nleaf)])
    B = _batch([prob])
    B.condense(prec=prec, max_refine=3, sync=True)
    ub_d = torch.as_tensor(ub.ravel(), device="cuda")
    ui = B.recover(ub_d, sync=True).view(prob.nleaf, -1).cpu().numpy()
    ui_rf = B.recover(ub_d, refactor=True, sync=True).view(prob.nleaf, -1).cpu().numpy()
    tol = TOL64 if prec == hps.HPS_FP64 else TOL_MIXED
    assert relerr(ui, sol.uint) <= tol
    assert relerr(ui_rf, sol.uint) <= TOL64
    B.close()


def test_recover_refactor_with_body_load(torch):
    prob = _forced_problem(12, 3, 2)
    _say("recover refactor forced")
    leaves = itf.build_leaves(prob)
    sol = itf.solve(prob, leaves)
    ub = np.stack([sol.uedge[sol.num.slot[t]] for t in range(prob.nleaf)])
    B = _batch([prob])
    f = B.interior_f()
    ui = B.recover(torch.as_tensor(ub.ravel(), device="cuda"), f=f, refactor=True, sync=True)
    assert relerr(ui.view(prob.nleaf, -1).cpu().numpy(), sol.uint) <= TOL64
    B.close()


# --------------------------------------------------------------------------
# end to end on the tiny workload: GPU condense -> host interface solve ->
# GPU recover, against the exact solution and the oracle's solution
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [hps.HPS_FP64, hps.HPS_FP32_REFINE])
def test_end_to_end_tiny(torch, prec):
    from paper_2211_14969_amd.harness import interface_solve
    prob = inputs.tiny()
    _say(f"end-to-end tiny prec={prec}")
    B = _batch([prob])
    S, w, info, st = B.condense(prec=prec, max_refine=3, sync=True)
    nb = 4 * (prob.p - 2)
    Bidx = lf.flat(prob.p, lf.boundary_nodes(prob.p))
    xy_b = B.groups[0].xy[:, Bidx, :].cpu().numpy()
    ub = interface_solve(prob, S.view(-1, nb, nb).cpu().numpy(), w.view(-1, nb).cpu().numpy(), xy_b)
    ui = B.recover(torch.as_tensor(ub.ravel(), device="cuda"), sync=True)
    ui = ui.view(prob.nleaf, -1).cpu().numpy()
    sol = itf.solve(prob)
    ub_o = np.stack([sol.uedge[sol.num.slot[t]] for t in range(prob.nleaf)])
    assert relerr(ui, sol.uint) <= 1e-9
    assert relerr(ub, ub_o) <= 1e-9
    # exact solution sin(kappa x1) at the interior nodes
    I = lf.flat(prob.p, lf.interior_nodes(prob.p))
    xy_i = B.groups[0].xy[:, I, :].cpu().numpy()
    exact = np.sin(prob.kappa * xy_i[..., 0])
    assert relerr(ui, exact) < 1e-3
    B.close()


# --------------------------------------------------------------------------
# failure reporting
# --------------------------------------------------------------------------
def test_singular_leaf_reports_zero_pivot(torch):
    zero = lambda x, y, xp: xp.zeros_like(x)
    prob = inputs.Problem(name="zero", nx=2, ny=1, p=8, kappa=0.0,
                          coef={"a11": zero, "a22": zero, "k2b": zero})
    _say("singular")
    B = _batch([prob])
    S, w, info, st = B.condense(prec=hps.HPS_FP64, sync=True, allow=(hps.HPS_ERR_SINGULAR,))
    assert st == hps.HPS_ERR_SINGULAR
    assert np.all(info.cpu().numpy() == 1)
    B.close()


def test_nonfinite_coefficient_is_flagged(torch):
    prob = inputs.tiny(p=8, n=2)
    # NaN in the interior of the leaves right of x1 = 0.5 (leaves 1 and 3)
    prob.coef["k2b"] = lambda x, y, xp: xp.where(x > 0.5, xp.zeros_like(x) + float("nan"),
                                                  xp.zeros_like(x) + 100.0)
    _say("nonfinite")
    B = _batch([prob])
    S, w, info, st = B.condense(prec=hps.HPS_FP64, sync=True,
                                allow=(hps.HPS_ERR_NONFINITE, hps.HPS_ERR_SINGULAR))
    assert st in (hps.HPS_ERR_NONFINITE, hps.HPS_ERR_SINGULAR)
    inf = info.cpu().numpy()
    assert inf[0] == 0 and inf[2] == 0 and inf[1] != 0 and inf[3] != 0
    B.close()


def test_fp64_fallback_when_refinement_cannot_meet_tol(torch):
    """An unreachable refinement target sends every leaf to the FP64 redo;
    the results are then FP64-accurate and the redo count is reported."""
    prob = _small(12, 2, 2)
    _say("fallback")
    B = _batch([prob])
    S, w, info = B.alloc_outputs()
    st = hps.hps_leaf_condense(B.batch, hps.HPS_FP32_REFINE, 1e-300, 1, None, S, w, info,
                               hps.HPS_SYNC)
    assert st == hps.HPS_OK
    assert hps.hps_batch_stats(B.batch) == (1, prob.nleaf)
    assert np.all(info.cpu().numpy() == 0)
    nb = 4 * (prob.p - 2)
    Sg = S.view(-1, nb, nb).cpu().numpy()
    for t in range(prob.nleaf):
        _, c = oracle_leaf(prob, t)
        assert relerr(Sg[t], c.S) <= TOL64
    B.close()


def test_refinement_stats_typical_leaves(torch):
    """Well-conditioned leaves (the annulus workload's) meet the default
    target within three corrections, without the FP64 redo."""
    prob = inputs.annulus(p=20, ntheta=8, nr=2, kappa=150.0)
    B = _batch([prob])
    S, w, info, st = B.condense(prec=hps.HPS_FP32_REFINE, max_refine=3, sync=True)
    assert hps.hps_batch_stats(B.batch) == (3, 0)
    B.close()


@pytest.mark.parametrize("p", [6, 8, 12, 16, 18])
def test_refinement_converges_without_redo_small_orders(torch, p):
    """The residual kernels of the orders up to 18 (interior lines of at most
    16 nodes) drive the refinement to the default target within three
    corrections on well-conditioned leaves: a wrong residual would show as leaves handed to the FP64 redo
    (which would still return correct results)."""
    _say(f"refinement without redo p={p}")
    prob = _small(p, 3)
    B = _batch([prob])
    S, w, info, st = B.condense(prec=hps.HPS_FP32_REFINE, max_refine=3, sync=True)
    assert st == hps.HPS_OK
    assert hps.hps_batch_stats(B.batch) == (3, 0)
    B.close()


def test_fixed_step_count_without_stop_test(torch):
    """tol >= 1 applies exactly max_refine corrections with no test and no
    FP64 redo: the error in X falls with every step (the contraction of
    LU-based refinement) until it reaches FP64 level."""
    prob = _small(24, 2, 1)
    _say("fixed step count")
    B = _batch([prob])
    ni, nb = (prob.p - 2) ** 2, 4 * (prob.p - 2)
    ref = [oracle_leaf(prob, t)[1].X for t in range(prob.nleaf)]
    errs = []
    for k in range(4):
        S, w, info = B.alloc_outputs()
        st = hps.hps_leaf_condense(B.batch, hps.HPS_FP32_REFINE, 2.0, k, None, S, w, info,
                                   hps.HPS_SYNC)
        assert st == hps.HPS_OK
        assert hps.hps_batch_stats(B.batch) == (k, 0)
        Xt, _ = B.export()
        Xt = Xt.view(prob.nleaf, nb, ni).cpu().numpy()
        errs.append(max(relerr(Xt[t].T, ref[t]) for t in range(prob.nleaf)))
    floor = max(leaf_bar(oracle_leaf(prob, t)[0].Aii, 0.0) for t in range(prob.nleaf))
    _say(f"  X error after 0..3 corrections {errs}, FP64 floor {floor:.1e}")
    assert 1e-9 < errs[0] < 1e-3
    assert errs[1] < 1e-2 * errs[0]
    assert errs[2] <= max(1e-2 * errs[1], floor) and errs[3] <= floor
    B.close()


def test_invalid_arguments_enqueue_nothing(torch):
    prob = _small(8, 1, 1)
    B = _batch([prob])
    S, w, info = B.alloc_outputs()
    with pytest.raises(hps.HpsError):
        hps.hps_leaf_condense(B.batch, 7, 0.0, 1, None, S, w, info)
    with pytest.raises(hps.HpsError):
        hps.hps_leaf_condense(B.batch, hps.HPS_FP64, 0.0, 99, None, S, w, info)
    with pytest.raises(hps.HpsError):
        hps.hps_leaf_recover(B.batch, S, None, S)    # recover before any condense
    box = torch.zeros((1, 4), dtype=torch.float64, device="cuda")
    empty = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    for bad in ({"p": 3, "box": box}, {"p": 33, "box": box}, {"p": 8, "box": empty}):
        with pytest.raises(hps.HpsError):
            hps.hps_leaf_build(B.ctx, [bad])
    B.close()


@pytest.mark.parametrize("prec", [hps.HPS_FP64, hps.HPS_FP32_REFINE])
def test_workspace_chunking_matches_single_pass(torch, prec, monkeypatch):
    """A workspace cap smaller than the batch condenses the leaves in several
    passes; every leaf's results are the same as in one pass (the leaves are
    independent), and recovery from the stored X agrees too."""
    probs = [_small(16, 4), _small(12, 3)]
    _say(f"workspace chunking prec={prec}")
    B1 = _batch(probs)
    S1, w1, i1, _ = B1.condense(prec=prec, max_refine=3, sync=True)
    ub = torch.randn(B1.nb_total, dtype=torch.float64, device="cuda")
    u1 = B1.recover(ub, sync=True)
    monkeypatch.setenv("HPS_WORKSPACE_MB", "1")     # about two p = 16 leaves per pass
    B2 = _batch(probs)
    S2, w2, i2, _ = B2.condense(prec=prec, max_refine=3, sync=True)
    u2 = B2.recover(ub, sync=True)
    assert torch.equal(S1, S2) and torch.equal(i1, i2)
    assert torch.equal(u1, u2)
    B1.close()
    B2.close()


# --------------------------------------------------------------------------
# concurrent lanes, redo flags, a leaf near a Dirichlet resonance
# --------------------------------------------------------------------------
@pytest.mark.parametrize("prec", [hps.HPS_FP64, hps.HPS_FP32_REFINE])
def test_lanes_match_serial_order(torch, prec):
    """Groups of different orders condensed on concurrent lanes give the
    same bits as the same groups one after another on the context stream
    (the per-phase timing mode runs the lanes serially)."""
    probs = [_small(p, 3) for p in (8, 12, 16, 20, 24, 30)]
    _say(f"lanes vs serial prec={prec}")
    B = _batch(probs)
    assert hps.hps_batch_lanes(B.batch) == 4
    S1, w1, i1, st = B.condense(prec=prec, max_refine=3, sync=True)
    assert st == hps.HPS_OK
    u_b = torch.randn(B.nb_total, dtype=torch.float64, device="cuda")
    u1 = B.recover(u_b, refactor=True, sync=True)
    hps.hps_ctx_set_timing(B.ctx, True)
    S2, w2, i2, st = B.condense(prec=prec, max_refine=3, sync=True)
    u2 = B.recover(u_b, refactor=True, sync=True)
    hps.hps_ctx_phase_times(B.ctx)
    hps.hps_ctx_set_timing(B.ctx, False)
    assert torch.equal(S1, S2) and torch.equal(i1, i2) and torch.equal(u1, u2)
    for G, Sg in zip(B.groups, B.split(S1, "S")):
        for t in (0, G.nleaf - 1):
            bl, c = oracle_leaf(G.problem, t)
            tol = TOL64 if prec == hps.HPS_FP64 else TOL_MIXED
            assert relerr(Sg[t].cpu().numpy(), c.S) <= leaf_bar(bl.Aii, tol)
    B.close()


def test_redo_flags_follow_the_fallback(torch):
    prob = _small(12, 2, 2)
    B = _batch([prob])
    S, w, info = B.alloc_outputs()
    flags = torch.full((prob.nleaf,), 7, dtype=torch.int32, device="cuda")
    hps.hps_leaf_condense(B.batch, hps.HPS_FP32_REFINE, 1e-300, 1, None, S, w, info, hps.HPS_SYNC)
    hps.hps_batch_redo_flags(B.batch, flags)
    torch.cuda.synchronize()
    assert bool((flags == 1).all())
    hps.hps_leaf_condense(B.batch, hps.HPS_FP32_REFINE, 0.0, 3, None, S, w, info, hps.HPS_SYNC)
    hps.hps_batch_redo_flags(B.batch, flags)
    torch.cuda.synchronize()
    assert bool((flags == 0).all()) and hps.hps_batch_stats(B.batch)[1] == 0
    hps.hps_leaf_condense(B.batch, hps.HPS_FP64, 0.0, 3, None, S, w, info, hps.HPS_SYNC)
    hps.hps_batch_redo_flags(B.batch, flags)
    torch.cuda.synchronize()
    assert bool((flags == 0).all())
    B.close()


def _near_resonant_problem(p=16, h=0.125, target_cond=1e8):
    """Two leaves of side h with b == 1: on the left one kappa^2 sits just
    above the smallest eigenvalue lambda_1 of the discrete Dirichlet operator
    (A_ii at kappa = 0), so A_ii(kappa) = A_ii(0) - kappa^2 I is nearly
    singular (cond ~ target_cond); on the right one kappa^2 = lambda_1 / 2."""
    box = (0.0, h, 0.0, h)
    bl0 = lf.blocks(box, p, {})
    lam = np.linalg.eigvals(bl0.Aii)
    lam1 = float(np.min(lam.real))
    lo, hi = 0.0, 1e-2              # bisection on the relative offset
    for _ in range(60):
        d = 0.5 * (lo + hi) if hi > 0 else lo
        k2 = lam1 * (1.0 + d)
        c = np.linalg.cond(bl0.Aii - k2 * np.eye(bl0.Aii.shape[0]))
        if c > target_cond:
            lo = d
        else:
            hi = d
    k2_left = lam1 * (1.0 + hi)
    k2 = lambda x, y, xp: xp.where(x < h, xp.zeros_like(x) + k2_left,
                                   xp.zeros_like(x) + 0.5 * lam1)
    return inputs.Problem(name="near_resonance", nx=2, ny=1, p=p, kappa=float(np.sqrt(k2_left)),
                          domain=(0.0, 2 * h, 0.0, h), coef={"k2b": k2})


def test_leaf_near_a_dirichlet_resonance(torch):
    """The method's own edge case: A_ii nearly singular when kappa^2 b meets
    a Dirichlet eigenvalue of the leaf.  FP64 meets the leaf's FP64 floor;
    the FP32 factorisation cannot serve the left leaf (cond * 2^-24 > 1), so
    the mixed path hands that leaf, and only that leaf, to the FP64 redo,
    and both precisions then give S, X and u at the FP64 floor, with the
    backward error of X at rounding level."""
    from _common import backward_error, fp64_floor, p7_bar
    prob = _near_resonant_problem()
    bls = [oracle_leaf(prob, t) for t in range(2)]
    conds = [float(np.linalg.cond(bl.Aii)) for bl, _ in bls]
    _say(f"near resonance: cond(A_ii) = {conds[0]:.2e} (left), {conds[1]:.2e} (right)")
    assert 1e7 <= conds[0] <= 1e9 and conds[1] < 1e4
    B = _batch([prob])
    nb, ni = 4 * (prob.p - 2), (prob.p - 2) ** 2
    ub = torch.randn(B.nb_total, dtype=torch.float64, device="cuda")
    flags = torch.empty(2, dtype=torch.int32, device="cuda")
    for prec in (hps.HPS_FP64, hps.HPS_FP32_REFINE):
        S, w, info, st = B.condense(prec=prec, max_refine=4, sync=True)
        assert st == hps.HPS_OK and bool((info == 0).all())
        hps.hps_batch_redo_flags(B.batch, flags)
        Xt, _ = B.export()
        ui = B.recover(ub, sync=True).view(2, ni).cpu().numpy()
        fl = flags.cpu().numpy().tolist()
        _say(f"  prec={prec}: redo flags {fl}")
        if prec == hps.HPS_FP32_REFINE:
            assert fl == [1, 0]
        Sg = S.view(2, nb, nb).cpu().numpy()
        Xg = Xt.view(2, nb, ni).cpu().numpy()
        ubh = ub.view(2, nb).cpu().numpy()
        for t, (bl, c) in enumerate(bls):
            tol = TOL64 if prec == hps.HPS_FP64 else TOL_MIXED
            bar = max(tol, fp64_floor(bl.Aii))
            eS, eX = relerr(Sg[t], c.S), relerr(Xg[t].T, c.X)
            eu = relerr(ui[t], lf.recover(c, ubh[t]))
            be = backward_error(bl.Aii, bl.Aib, Xg[t].T)
            _say(f"    leaf {t}: S {eS:.1e} X {eX:.1e} u {eu:.1e} (bar {bar:.1e}), "
                 f"backward {be:.1e}")
            assert eS <= bar and eX <= bar and eu <= bar, t
            assert be <= p7_bar(ni), t
    B.close()


# --------------------------------------------------------------------------
# left-looking factorisation (tuning variant 4)
# --------------------------------------------------------------------------
LL_ORDERS = [4, 5, 8, 12, 13, 16, 18, 19, 20, 23, 24, 30, 32]


@pytest.mark.parametrize("prec", [hps.HPS_FP64, hps.HPS_FP32_REFINE])
@pytest.mark.parametrize("p", LL_ORDERS)
def test_condense_left_looking(torch, p, prec):
    """Variant 4 at every block-column shape: one or two row-tile groups per
    wavefront, block columns straddling the pivot panels and the right-hand
    sides, odd and even tile counts; with the body-load column too."""
    _say(f"left-looking p={p} prec={prec}")
    prob = _small(p, 2)
    B = _batch([prob])
    hps.hps_batch_set_tuning(B.batch, 0, 4, 0)
    S, w, info, st = B.condense(prec=prec, max_refine=3, sync=True)
    assert st == hps.HPS_OK and bool((info == 0).all())
    Xt, _ = B.export()
    nb, ni = 4 * (p - 2), (p - 2) ** 2
    Sg, Xg = S.view(-1, nb, nb).cpu().numpy(), Xt.view(-1, nb, ni).cpu().numpy()
    tol = TOL64 if prec == hps.HPS_FP64 else TOL_MIXED
    for t in range(prob.nleaf):
        bl, c = oracle_leaf(prob, t)
        bar = leaf_bar(bl.Aii, tol)
        assert relerr(Sg[t], c.S) <= bar, t
        assert relerr(Xg[t].T, c.X) <= (bar if prec == hps.HPS_FP64 else max(bar, 1e-8)), t
    B.close()
    if p < 6:
        return
    fp = _forced_problem(p)
    B = _batch([fp])
    hps.hps_batch_set_tuning(B.batch, 0, 4, 0)
    f = B.interior_f()
    S, w, info, st = B.condense(prec=prec, f=f, max_refine=3, sync=True)
    assert st == hps.HPS_OK
    _, h = B.export()
    Sg, wg, hg = (S.view(-1, nb, nb).cpu().numpy(), w.view(-1, nb).cpu().numpy(),
                  h.view(-1, ni).cpu().numpy())
    for t in range(fp.nleaf):
        bl, c = oracle_leaf(fp, t, oracle_interior_f(fp, t))
        bar = leaf_bar(bl.Aii, tol)
        assert relerr(Sg[t], c.S) <= bar and relerr(wg[t], c.w) <= bar and relerr(hg[t], c.h) <= bar
    # the paper's re-factor recovery on the same variant
    ub = torch.randn(B.nb_total, dtype=torch.float64, device="cuda")
    u_rf = B.recover(ub, f=f, refactor=True, sync=True).view(-1, ni).cpu().numpy()
    ubh = ub.view(-1, nb).cpu().numpy()
    for t in range(fp.nleaf):
        bl, c = oracle_leaf(fp, t, oracle_interior_f(fp, t))
        assert relerr(u_rf[t], lf.recover(c, ubh[t])) <= leaf_bar(bl.Aii, TOL64)
    B.close()
