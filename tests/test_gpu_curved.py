"""GPU parity of the general operator with a mixed term (Sec. 3.2: the
paper's curved domain, eq. (chain_rule), a12 = psi' x2 / psi != 0), against
the oracle:

* the leaf blocks, with the interior rows' corner columns folded into A_ib
  (each corner the mean of its two edges' degree-(p-3) extrapolants);
* FP64 condensation (S, X) at orders across every factorisation kernel,
  and each forced factorisation variant;
* recovery, stored and re-factored;
* end to end on the device (condense, interface solve, recover) against the
  exact plane-wave solution;
* FP32 + refinement is refused for such operators (its structured residual
  has no mixed term).
"""
import sys

import numpy as np
import pytest

from _common import leaf_bar, oracle_leaf, relerr
from oracle import interface as itf
from oracle import leaf as lf
from paper_2211_14969_amd import hps, inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.fail("no GPU visible")
    hps.load()
    return T


def _batch(problems):
    from paper_2211_14969_amd.harness import LeafBatch
    return LeafBatch(problems)


@pytest.mark.parametrize("p", [4, 8, 13, 16, 24, 32])
def test_curved_operator_blocks(torch, p):
    prob = inputs.curved(p=p, n=2, kappa=3.0 * p)
    _say(f"curved operator p={p}")
    B = _batch([prob])
    ni, nb, L = (p - 2) ** 2, 4 * (p - 2), prob.nleaf
    mk = lambda *s: torch.empty(s, dtype=torch.float64, device="cuda")
    Aii, Aib, Abi, Abb = mk(L, ni, ni), mk(L, ni, nb), mk(L, nb, ni), mk(L, nb, nb)
    hps.hps_leaf_operator(B.batch, 0, Aii, Aib, Abi, Abb)
    torch.cuda.synchronize()
    for t in range(L):
        bl, _ = oracle_leaf(prob, t)
        for name, got in (("Aii", Aii), ("Aib", Aib), ("Abi", Abi), ("Abb", Abb)):
            assert relerr(got[t].cpu().numpy(), getattr(bl, name)) < 1e-13, (name, t)
    B.close()


def _check(torch, prob, variant=None, tol=1e-10):
    B = _batch([prob])
    if variant is not None:
        hps.hps_batch_set_tuning(B.batch, 0, variant, 0)
    S, w, info, st = B.condense(prec=hps.HPS_FP64, sync=True)
    assert st == hps.HPS_OK
    Xt, h = B.export()
    nb, ni = 4 * (prob.p - 2), (prob.p - 2) ** 2
    S = S.view(prob.nleaf, nb, nb).cpu().numpy()
    Xt = Xt.view(prob.nleaf, nb, ni).cpu().numpy()
    worst = 0.0
    for t in range(prob.nleaf):
        bl, c = oracle_leaf(prob, t)
        bar = leaf_bar(bl.Aii, tol)
        eS, eX = relerr(S[t], c.S), relerr(Xt[t].T, c.X)
        worst = max(worst, eS, eX)
        assert eS <= bar and eX <= bar, (prob.name, variant, t, eS, eX, bar)
    _say(f"  {prob.name} variant {variant}: worst {worst:.2e}")
    return B


@pytest.mark.parametrize("p", [5, 8, 12, 16, 20, 24, 28, 32])
def test_curved_condense_fp64(torch, p):
    prob = inputs.curved(p=p, n=2, kappa=3.0 * p)
    _say(f"curved condense p={p}")
    _check(torch, prob).close()


@pytest.mark.parametrize("p,variant", [(16, 1), (16, 2), (16, 4), (24, 1), (24, 2), (24, 4)])
def test_curved_factor_variants(torch, p, variant):
    prob = inputs.curved(p=p, n=2, kappa=40.0)
    _say(f"curved condense p={p} variant {variant}")
    _check(torch, prob, variant).close()


@pytest.mark.parametrize("p", [12, 24])
def test_curved_recover(torch, p):
    prob = inputs.curved(p=p, n=2, kappa=30.0)
    _say(f"curved recover p={p}")
    B = _check(torch, prob)
    nb = 4 * (p - 2)
    rng = np.random.default_rng(p)
    ub = rng.standard_normal((prob.nleaf, nb))
    ub_d = torch.as_tensor(ub.ravel(), device="cuda")
    u1 = B.recover(ub_d, sync=True).view(prob.nleaf, -1).cpu().numpy()
    u2 = B.recover(ub_d, refactor=True, sync=True).view(prob.nleaf, -1).cpu().numpy()
    for t in range(prob.nleaf):
        bl, c = oracle_leaf(prob, t)
        ref = lf.recover(c, ub[t])
        assert relerr(u1[t], ref) <= 1e-10, t
        assert relerr(u2[t], ref) <= 1e-10, t
    B.close()


def test_curved_fp32_refused(torch):
    prob = inputs.curved(p=12, n=2)
    _say("curved fp32 refused")
    B = _batch([prob])
    S, w, info = B.alloc_outputs()
    with pytest.raises(hps.HpsError) as e:
        hps.hps_leaf_condense(B.batch, hps.HPS_FP32_REFINE, 0.0, 2, None, S, w, info, 0)
    assert e.value.status == hps.HPS_ERR_INVALID
    B.close()


@pytest.mark.parametrize("n,p,kappa,tol", [(2, 12, 8.0, 1e-7), (8, 16, 20.0, 1e-9)])
def test_curved_end_to_end(torch, n, p, kappa, tol):
    """Condense, interface solve and recover on the device; the plane wave in
    the physical coordinates is the exact solution.  On the small grid the
    result must also match the oracle's own solve."""
    from paper_2211_14969_amd.harness import InterfaceSolver, dirichlet_data
    prob = inputs.curved(p=p, n=n, kappa=kappa)
    _say(f"curved end to end {prob.name}")
    B = _batch([prob])
    S, w, info, st = B.condense(prec=hps.HPS_FP64, sync=True)
    assert st == hps.HPS_OK
    it = InterfaceSolver(B.ctx, prob)
    it.factor(S, sync=True)
    ub = it.solve(S, w, dirichlet_data(B.groups[0]), sync=True)
    ui = B.recover(ub, sync=True)
    L = prob.nleaf
    uih = ui.view(L, -1).cpu().numpy()
    ubh = ub.view(L, -1).cpu().numpy()
    xy = B.groups[0].xy.cpu().numpy()
    I = lf.flat(p, lf.interior_nodes(p))
    Bn = lf.flat(p, lf.boundary_nodes(p))
    ex_i = prob.exact(xy[:, I, 0], xy[:, I, 1], np)
    ex_b = prob.exact(xy[:, Bn, 0], xy[:, Bn, 1], np)
    err = np.sqrt(np.sum((uih - ex_i) ** 2) + np.sum((ubh - ex_b) ** 2)) / np.sqrt(
        np.sum(ex_i ** 2) + np.sum(ex_b ** 2))
    _say(f"  error against the exact solution {err:.2e}")
    assert err <= tol
    if L <= 16:
        sol = itf.solve(prob)
        assert relerr(uih, sol.uint) <= 1e-10
    it.close()
    B.close()
