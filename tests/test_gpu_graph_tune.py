"""GPU: condensation captured in a HIP graph and replayed, and the autotuner.

The graph test captures one hps_leaf_condense of a multi-order batch (the
uneven-batch shape at small size) and replays it several times with other
device work and synchronisations in between; every replay must reproduce the
eager result.  The autotuner must pick a setting whose results agree with the
default ones."""
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


def _problems():
    return [inputs.multi_bump(p=p, n=2, kappa=2.0 * p, seed=5 + p) for p in (8, 12, 16, 20, 24)]


@pytest.mark.parametrize("prec", [hps.HPS_FP64, hps.HPS_FP32_REFINE])
def test_graph_replay_matches_eager(torch, prec):
    from paper_2211_14969_amd.harness import LeafBatch
    _say(f"graph replay prec={prec}")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        B = LeafBatch(_problems(), stream=stream)
        S, w, info = B.alloc_outputs()
        hps.hps_leaf_condense(B.batch, prec, 0.0, 2, None, S, w, info, 0)
    stream.synchronize()
    S_ref = S.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        hps.hps_leaf_condense(B.batch, prec, 0.0, 2, None, S, w, info, 0)
    for rep in range(3):
        S.fill_(float("nan"))
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(S, S_ref), f"replay {rep} differs"
        assert bool((info == 0).all())
        del junk
    B.close()


def test_autotuner_setting_keeps_results(torch, tmp_path):
    from paper_2211_14969_amd import tune
    from paper_2211_14969_amd.harness import LeafBatch
    probs = [inputs.multi_bump(p=16, n=8, kappa=60.0), inputs.annulus(p=20, ntheta=16, nr=4, kappa=60.0)]
    B = LeafBatch(probs)
    S0, w0, i0, _ = B.condense(prec=hps.HPS_FP64, sync=True)
    res = tune.tune_batch(B, prec=hps.HPS_FP64, reps=1, cache_path=str(tmp_path / "t.json"))
    _say(f"tuned: {res}")
    assert set(res) == {0, 1}
    for gi, r in res.items():
        assert tuple(r["setting"]) in tune.candidates(B.groups[gi].p)
    S1, w1, i1, _ = B.condense(prec=hps.HPS_FP64, sync=True)
    for a, b in zip(B.split(S0, "S"), B.split(S1, "S")):
        rel = ((a - b).flatten(1).norm(dim=1) / a.flatten(1).norm(dim=1)).max().item()
        assert rel <= 1e-12
    # second call is served from the cache
    res2 = tune.tune_batch(B, prec=hps.HPS_FP64, reps=1, cache_path=str(tmp_path / "t.json"))
    assert all(r["cached"] for r in res2.values())
    B.close()
