"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (one condense call over the whole batch), checked on a
seeded sample of leaves against the oracle, plus properties that hold at
any size (finite output, no failure flags, FP64 and FP32+refinement agree).

Workloads: 64x64 leaves p=16 (single bump, FP64), 32x32 leaves p=32 (eight
bumps, FP64 and FP32+refinement), the quarter annulus 128x16 leaves p=20,
and the eight-problem uneven batch (p = 8 ... 32, one batch).
"""
import sys

import numpy as np
import pytest

from _common import leaf_bar, oracle_leaf, relerr, sample_leaves
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
    hps.load()
    return T


def _run(torch, problems, prec, max_refine=2):
    from paper_2211_14969_amd.harness import LeafBatch
    B = LeafBatch(problems)
    S, w, info, st = B.condense(prec=prec, max_refine=max_refine, sync=True,
                                allow=(hps.HPS_OK, hps.HPS_ERR_NOT_CONVERGED))
    Xt, h = B.export()
    torch.cuda.synchronize()
    return B, S, Xt, info, st


def _check_sample(B, S, Xt, problems, tol, nsample, seed):
    worst = 0.0
    for G, Sg, Xg in zip(B.groups, B.split(S, "S"), B.split(Xt, "Xt")):
        prob = G.problem
        assert bool(torch_isfinite(Sg)), prob.name
        for t in sample_leaves(prob.nleaf, nsample, seed):
            bl, c = oracle_leaf(prob, t)
            bar = leaf_bar(bl.Aii, tol)
            eS = relerr(Sg[t].cpu().numpy(), c.S)
            eX = relerr(Xg[t].cpu().numpy().T, c.X)
            worst = max(worst, eS)
            assert eS <= bar, (prob.name, t, eS, bar)
            assert eX <= max(bar, 1e-8), (prob.name, t, eX, bar)
    return worst


def torch_isfinite(t):
    import torch
    return torch.isfinite(t).all().item()


def test_bump_64x64_p16_fp64(torch):
    prob = inputs.single_bump()
    _say("full size: bump 64x64 p16 fp64")
    B, S, Xt, info, st = _run(torch, [prob], hps.HPS_FP64)
    assert st == hps.HPS_OK and int((info != 0).sum()) == 0
    w = _check_sample(B, S, Xt, [prob], TOL64, 6, 2)
    _say(f"  worst sampled rel err S {w:.2e}")
    B.close()


@pytest.mark.parametrize("prec", [hps.HPS_FP64, hps.HPS_FP32_REFINE])
def test_bumps_32x32_p32(torch, prec):
    prob = inputs.multi_bump()
    _say(f"full size: bumps 32x32 p32 prec={prec}")
    B, S, Xt, info, st = _run(torch, [prob], prec)
    assert st == hps.HPS_OK and int((info != 0).sum()) == 0
    w = _check_sample(B, S, Xt, [prob], TOL64 if prec == hps.HPS_FP64 else TOL_MIXED, 3, 3)
    _say(f"  worst sampled rel err S {w:.2e}")
    B.close()


@pytest.mark.parametrize("prec", [hps.HPS_FP64, hps.HPS_FP32_REFINE])
def test_annulus_128x16_p20(torch, prec):
    prob = inputs.annulus()
    _say(f"full size: annulus 128x16 p20 prec={prec}")
    B, S, Xt, info, st = _run(torch, [prob], prec)
    assert st == hps.HPS_OK and int((info != 0).sum()) == 0
    w = _check_sample(B, S, Xt, [prob], TOL64 if prec == hps.HPS_FP64 else TOL_MIXED, 6, 4)
    _say(f"  worst sampled rel err S {w:.2e}")
    # any size: the FP64 and mixed results agree on every leaf
    other = hps.HPS_FP32_REFINE if prec == hps.HPS_FP64 else hps.HPS_FP64
    S2, _, _, _ = B.condense(prec=other, max_refine=2, sync=True)
    nb = 4 * (prob.p - 2)
    a, b = S.view(-1, nb, nb), S2.view(-1, nb, nb)
    rel = ((a - b).flatten(1).norm(dim=1) / b.flatten(1).norm(dim=1)).max().item()
    assert rel <= TOL_MIXED
    B.close()


def test_uneven_eight_problems(torch):
    probs = inputs.uneven_batch()
    _say("full size: uneven batch " + ", ".join(f"p{q.p}:{q.nleaf}" for q in probs))
    B, S, Xt, info, st = _run(torch, probs, hps.HPS_FP32_REFINE)
    assert st == hps.HPS_OK, hps.status_string(st)
    assert int((info != 0).sum()) == 0
    w = _check_sample(B, S, Xt, probs, TOL_MIXED, 1, 5)
    _say(f"  worst sampled rel err S {w:.2e}")
    B.close()
