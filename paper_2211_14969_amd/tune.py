"""Autotuner of the factorisation per (order p, precision, batch size).

For every order group of a batch it times the candidate settings of
`hps_batch_set_tuning` -- the factorisation variant (one 16-column panel per
trailing pass, panels in pairs, or for FP32 and p <= 16 the work matrix held
in registers) and the column chunk of the U12 / trailing passes -- on a batch
of that group's own leaves, keeps the fastest, applies
it to the batch, and remembers it in a JSON cache keyed by
``p<order>_<precision>_L<leaf-count bucket>``.  Timing uses the library's
per-phase HIP events (`hps_ctx_phase_times`).
"""
from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Tuple

from . import hps

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hps_leaf_tune.json")


def bucket(nleaf: int) -> int:
    """Leaf-count bucket: the power of two at or above nleaf (min 64)."""
    b = 64
    while b < nleaf:
        b *= 2
    return b


def cache_key(p: int, prec: int, nleaf: int) -> str:
    return f"p{p}_{'fp64' if prec == hps.HPS_FP64 else 'fp32r'}_L{bucket(nleaf)}"


def candidates(p: int, prec: int = hps.HPS_FP64) -> List[Tuple[int, int]]:
    """(variant, chunk_cols) pairs worth timing for order p: the streaming
    variants over their column chunks (the paired one of large work matrices
    only at 64 and 128 columns), for FP32 work matrices of at most 208 rows
    the register-resident variant (which has no chunk), and the left-looking
    variant."""
    ni, nb = (p - 2) ** 2, 4 * (p - 2)
    cols = ((ni + 15) // 16) * 16 + ((nb + 1 + 15) // 16) * 16
    chunks = [c for c in (32, 64, 128, 256, 512) if c < cols] + [0]
    if ni <= 256:
        out = [(v, c) for v in (1, 2) for c in chunks]
    else:
        # paired panels with a large work matrix: only strips of whole
        # four-tile groups pay (64 or 128 columns)
        out = [(1, c) for c in chunks] + [(2, c) for c in (64, 128) if c < cols] + [(2, 0)]
    if prec == hps.HPS_FP32_REFINE and ((ni + 15) // 16) * 16 <= 208:
        out.append((3, 0))
    # left-looking, block column in registers
    out.append((4, 0))
    return out


def tuning_problem(prob, max_leaves: int):
    """The leading leaf rows of `prob` (at most `max_leaves` leaves) as a
    problem of its own: the domain is cut in x2 so that every leaf keeps its
    box, hence its conditioning and refinement behaviour."""
    from .inputs import Problem
    if prob.nleaf <= max_leaves:
        return prob
    ny = max(1, min(prob.ny, max_leaves // prob.nx))
    x0, x1, y0, y1 = prob.domain
    hy = (y1 - y0) / prob.ny
    return Problem(name=prob.name + "_tune", nx=prob.nx, ny=ny, p=prob.p, kappa=prob.kappa,
                   domain=(x0, x1, y0, y0 + ny * hy), coef=prob.coef, g=prob.g,
                   exact=prob.exact, f=prob.f, meta=prob.meta)


def load_cache(path: Optional[str]) -> Dict[str, list]:
    if path and os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def save_cache(path: Optional[str], cache: Dict[str, list]) -> None:
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_setting(sub, prec: int, max_refine: int, setting: Tuple[int, int], reps: int) -> float:
    """Milliseconds per condense of the one-group batch `sub` with `setting`."""
    hps.hps_batch_set_tuning(sub.batch, 0, *setting)
    S, w, info = sub.alloc_outputs()
    hps.hps_leaf_condense(sub.batch, prec, 0.0, max_refine, None, S, w, info, hps.HPS_SYNC)
    hps.hps_ctx_set_timing(sub.ctx, True)
    hps.hps_ctx_phase_times(sub.ctx)
    for _ in range(reps):
        hps.hps_leaf_condense(sub.batch, prec, 0.0, max_refine, None, S, w, info, 0)
    ph = hps.hps_ctx_phase_times(sub.ctx)
    hps.hps_ctx_set_timing(sub.ctx, False)
    return sum(v[0] for v in ph.values()) / reps


def tune_batch(lb, prec: int = hps.HPS_FP64, max_refine: int = 1, reps: int = 2,
               cache_path: Optional[str] = DEFAULT_CACHE, max_leaves: int = 4096,
               retune: bool = False) -> Dict[int, dict]:
    """Tune every group of the LeafBatch `lb` and apply the winners.

    Each group is timed on a batch of at most `max_leaves` of its leaves (the
    leading ones).  Returns {group: {"key", "setting", "ms", "timings"}}."""
    from .harness import LeafBatch
    from .inputs import Problem

    cache = load_cache(cache_path)
    out = {}
    for gi, G in enumerate(lb.groups):
        key = cache_key(G.p, prec, G.nleaf)
        if key in cache and not retune:
            setting = tuple(cache[key]["setting"])
            hps.hps_batch_set_tuning(lb.batch, gi, *setting)
            out[gi] = {"key": key, "setting": setting, "ms": cache[key]["ms"], "cached": True}
            continue
        prob: Problem = tuning_problem(G.problem, max_leaves)
        sub = LeafBatch([prob])
        timings = {}
        for setting in candidates(G.p, prec):
            timings[setting] = _time_setting(sub, prec, max_refine, setting, reps)
        sub.close()
        best = min(timings, key=timings.get)
        hps.hps_batch_set_tuning(lb.batch, gi, *best)
        cache[key] = {"setting": list(best), "ms": timings[best]}
        out[gi] = {"key": key, "setting": best, "ms": timings[best],
                   "timings": {f"{v}/{c}": t for (v, c), t in timings.items()}, "cached": False}
    save_cache(cache_path, cache)
    return out
