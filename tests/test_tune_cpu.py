"""Host logic of the autotuner: candidates, cache keys, cache round trip."""
import os

from paper_2211_14969_amd import hps, tune


def test_buckets_and_keys():
    assert tune.bucket(1) == 64 and tune.bucket(64) == 64 and tune.bucket(65) == 128
    assert tune.bucket(4096) == 4096 and tune.bucket(4097) == 8192
    assert tune.cache_key(16, hps.HPS_FP64, 4096) == "p16_fp64_L4096"
    assert tune.cache_key(32, hps.HPS_FP32_REFINE, 1000) == "p32_fp32r_L1024"


def test_candidates_respect_kernel_limits():
    for p in (4, 8, 12, 16, 17, 18, 20, 32):
        cands = tune.candidates(p)
        assert cands and len(set(cands)) == len(cands)
        ni = (p - 2) ** 2
        for v, c in cands:
            assert v in (1, 2, 4) and c % 16 == 0 and 0 <= c <= 1024
            if v == 2 and ni > 256:
                assert c in (0, 64, 128)
        assert any(v == 1 for v, _ in cands) and any(v == 2 for v, _ in cands)


def test_register_resident_candidate_only_for_small_fp32():
    for p in range(4, 33):
        R = ((p - 2) ** 2 + 15) // 16 * 16
        has = (3, 0) in tune.candidates(p, hps.HPS_FP32_REFINE)
        assert has == (R <= 208), p
        assert all(v != 3 for v, _ in tune.candidates(p, hps.HPS_FP64))


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert tune.load_cache(path) == {}
    tune.save_cache(path, {"p16_fp64_L4096": {"setting": [2, 64], "ms": 5.0}})
    assert os.path.exists(path)
    assert tune.load_cache(path)["p16_fp64_L4096"]["setting"] == [2, 64]


def test_tuning_problem_keeps_the_leaf_boxes():
    """The tuning sub-problem is the leading rows of the real leaves: same
    boxes, hence the same conditioning and refinement behaviour."""
    from paper_2211_14969_amd import inputs
    import numpy as np
    for prob in (inputs.uneven_batch()[1], inputs.multi_bump()):
        sub = tune.tuning_problem(prob, 1024)
        assert sub.nleaf <= 1024 and sub.nx == prob.nx
        np.testing.assert_allclose(sub.boxes(), prob.boxes()[:sub.nleaf], rtol=0, atol=1e-15)
    small = inputs.tiny()
    assert tune.tuning_problem(small, 1024) is small
