"""hps_leaf_condense_noalloc: the entry point for callers that cannot
allocate device memory (pass scratch in the library's static device array)
gives the results of hps_leaf_condense, through the C ABI, on two calls in a
row, the second on a smaller batch, in both precisions and with a body load;
and leaves the batch's stored X usable for recovery."""
import sys

import numpy as np
import pytest

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


def _forced(p, nx, ny):
    kappa = 6.0
    u = lambda x, y, xp: xp.sin(3 * x) * xp.cos(2 * y) + x * y
    f = lambda x, y, xp: (13.0 - kappa ** 2) * xp.sin(3 * x) * xp.cos(2 * y) - kappa ** 2 * x * y
    return inputs.Problem(name=f"forced_p{p}", nx=nx, ny=ny, p=p, kappa=kappa,
                          coef={"k2b": lambda x, y, xp: xp.zeros_like(x) + kappa ** 2},
                          g=u, exact=u, f=f)


def _rel(a, b):
    return ((a - b).norm() / b.norm()).item()


@pytest.mark.parametrize("prec", [hps.HPS_FP64, hps.HPS_FP32_REFINE])
def test_noalloc_matches_condense_twice(torch, prec):
    from paper_2211_14969_amd.harness import LeafBatch
    big = [inputs.multi_bump(p=p, n=n, kappa=3.0 * p, seed=3) for p, n in ((32, 12), (16, 8), (9, 5))]
    small = [inputs.multi_bump(p=p, n=n, kappa=3.0 * p, seed=4) for p, n in ((20, 3), (8, 2))]
    for probs in (big, small):
        _say(f"noalloc prec={prec} orders {[q.p for q in probs]} leaves {[q.nleaf for q in probs]}")
        B = LeafBatch(probs)
        S1, w1, i1, st = B.condense(prec=prec, max_refine=3, sync=True)
        assert st == hps.HPS_OK
        ub = torch.randn(B.nb_total, dtype=torch.float64, device="cuda")
        u1 = B.recover(ub, sync=True)
        S2, w2, i2 = B.alloc_outputs()
        S2.fill_(float("nan"))
        st = hps.hps_leaf_condense_noalloc(B.batch, prec, 0.0, 3, None, S2, w2, i2, hps.HPS_SYNC)
        assert st == hps.HPS_OK
        u2 = B.recover(ub, sync=True)
        assert torch.equal(i1, i2) and bool((i2 == 0).all())
        assert bool(torch.isfinite(S2).all())
        tol = 1e-12 if prec == hps.HPS_FP64 else 1e-9
        for G, a, b in zip(B.groups, B.split(S1, "S"), B.split(S2, "S")):
            r = ((a - b).flatten(1).norm(dim=1) / a.flatten(1).norm(dim=1)).max().item()
            assert r <= tol, (G.p, r)
        assert _rel(u2, u1) <= tol
        B.close()


def test_noalloc_with_body_load(torch):
    from paper_2211_14969_amd.harness import LeafBatch
    for prob in (_forced(24, 4, 3), _forced(12, 2, 2)):
        B = LeafBatch([prob])
        f = B.interior_f()
        for prec in (hps.HPS_FP64, hps.HPS_FP32_REFINE):
            S1, w1, i1, st = B.condense(prec=prec, f=f, max_refine=3, sync=True)
            _, h1 = B.export()
            S2, w2, i2 = B.alloc_outputs()
            st = hps.hps_leaf_condense_noalloc(B.batch, prec, 0.0, 3, f, S2, w2, i2, hps.HPS_SYNC)
            assert st == hps.HPS_OK
            _, h2 = B.export()
            tol = 1e-12 if prec == hps.HPS_FP64 else 1e-9
            assert _rel(S2, S1) <= tol and _rel(w2, w1) <= tol and _rel(h2, h1) <= tol
        B.close()


def test_noalloc_rejects_bad_arguments(torch):
    from paper_2211_14969_amd.harness import LeafBatch
    B = LeafBatch([inputs.tiny()])
    S, w, info = B.alloc_outputs()
    with pytest.raises(hps.HpsError):
        hps.hps_leaf_condense_noalloc(B.batch, 9, 0.0, 1, None, S, w, info)
    with pytest.raises(hps.HpsError):
        hps.hps_leaf_condense_noalloc(B.batch, hps.HPS_FP64, 0.0, 99, None, S, w, info)
    B.close()
