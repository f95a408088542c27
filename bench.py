#!/usr/bin/env python3
"""Throughput of batched HPS leaf condensation on one MI355X.

One step = one pass of the whole hot path over the batch: form every leaf's
collocation operator on the device, factor A_ii, solve for X = A_ii^{-1} A_ib
and form S = A_bb - A_bi X (plus the FP64 refinement of X in the mixed
precision mode).  Inputs (leaf boxes, coefficient samples) are resident in
HBM before the timed region; nothing is copied to or from the host inside it.

Default workload: the precision study, the unit square split into 32 x 32
leaves of order p = 32, kappa = 300, b(x) = 1 - 0.3 sum of eight Gaussian
bumps (width 0.03, centres from seed 3).  The headline is FP64; the same
batch is timed in FP32 + FP64 refinement beside it ("compare").  For the
uneven eight-problem batch each precision is autotuned and its step is the
replay of one condense captured in a HIP graph.

Accuracy, reported with the timing: every leaf's S from the two precisions
is compared on the device, and for the leaves where they differ most plus a
seeded sample the relative errors of S, X and the recovered u_i = h - X u_b
(from a seeded u_b) against the FP64 CPU oracle are stated for both
precisions.  Recovery is timed separately against the HBM roofline.  The
CPU oracle is timed on the host's cores on a bounded sample of the same
leaves, in two schedules (a leaf-parallel process pool with one BLAS thread
per process, and one process with threaded BLAS), the faster reported.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}

# Calibrated HBM traffic of one factorisation launch, from rocprofv3 --pmc
# FETCH_SIZE / WRITE_SIZE (KiB per dispatch, FETCH scaled by 2.0 and WRITE by
# 1.0 against a 1 GiB device copy), keyed by the hash of the kernel source it
# was measured on (kernel_source_hash), the workload and the precision.
MEASURED_TRAFFIC = {
    ("fa33572667cedb58", "bumps_32x32_p32", "fp64"): {
        "kernel": "k_factor_ll<double, 8, 8, 2, 1>",
        "fetch_bytes": 39873461.542 * 2.0 * 1024, "write_bytes": 8804062.776 * 1.0 * 1024},
}

WORKLOADS = {
    "bumps": ("multi_bump", "32x32 leaves p=32 kappa=300, eight bumps (default)"),
    "bump": ("single_bump", "64x64 leaves p=16 kappa=100, one bump"),
    "annulus": ("annulus", "quarter annulus 128x16 leaves p=20 kappa=150"),
    "uneven": ("uneven_batch", "eight problems p=8..32 in one batch"),
    "tiny": ("tiny", "4x4 leaves p=8 kappa=10"),
    "mixed": ("mixed_bump", "32x32 leaves of orders 12 / 20 / 28 (one problem, by distance to a "
                            "bump), kappa=150"),
    "curved": ("curved", "the paper's curved domain (mixed term a12), 48x48 leaves p=20 kappa=150",
               {"p": 20, "n": 48, "kappa": 150.0}),
}


def kernel_source_hash(kernel: str = "k_factor_ll") -> str:
    """sha256 prefix of the kernel file up to the end of `kernel`'s
    definition (its helpers come before it; the solves and launchers after
    it do not change its traffic), with comments and whitespace removed:
    edits of comments keep a traffic measurement valid, any change of that
    code invalidates it."""
    import hashlib
    import re
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "paper_2211_14969_amd", "csrc", "hps_kernels.hip")
    with open(path) as fh:
        src = fh.read()
    head = src.index(kernel + "(Geom g")
    src = src[:src.index("\n}\n", head) + 3]
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = re.sub(r"\s+", " ", src).strip()
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def algorithmic_flops(p: int):
    """Useful FLOP per leaf, per kernel: LU of A_ii together with the forward
    elimination of the nb columns of A_ib (2/3 ni^3 + ni^2 nb), the back
    substitution (ni^2 nb), and S with A_bi's p-2 nonzeros per row
    (2 nb^2 (p-2))."""
    ni, nb = (p - 2) ** 2, 4 * (p - 2)
    factor = (2.0 / 3.0) * ni ** 3 + ni * ni * nb
    back = ni * ni * nb
    schur = 2.0 * nb * nb * (p - 2)
    return {"factor": factor, "backsolve": back, "schur": schur,
            "total": factor + back + schur}


def make_problems(workload: str):
    from paper_2211_14969_amd import inputs
    entry = WORKLOADS[workload]
    made = getattr(inputs, entry[0])(**(entry[2] if len(entry) > 2 else {}))
    if hasattr(made, "groups"):      # one problem, leaves of several orders
        return made.groups()
    return made if isinstance(made, list) else [made]


# --------------------------------------------------------------------------
# CPU baseline: the oracle on the host's cores
# --------------------------------------------------------------------------
def _pool_init():
    """One BLAS thread per worker: set before numpy loads its BLAS, and
    limited again once it is loaded (threadpoolctl only sees loaded
    libraries)."""
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"
    import numpy  # noqa: F401
    import scipy.linalg  # noqa: F401
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)


def _oracle_leaves(args):
    """Condense leaves `ts` of problem `gi` of `workload` with the oracle
    (operator build + LAPACK condensation); returns the count."""
    workload, gi, ts = args
    from oracle import leaf as lf
    prob = make_problems(workload)[gi]
    boxes = prob.boxes()
    for t in ts:
        coef = lf.sample_coefficients(prob, boxes[t], prob.p)
        lf.condense(lf.blocks(boxes[t], prob.p, coef))
    return len(ts)


def cpu_baseline(workload: str, budget_s: float):
    """The FP64 oracle on a bounded sample of the workload's leaves (the
    first problem's, for a multi-problem batch), in two schedules, each
    timed five times (median): a leaf-parallel process pool with one BLAS
    thread per process, and one process with threaded BLAS.  The faster is
    reported, with its name and the threads it used."""
    import multiprocessing as mp
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    cores = min(16, len(os.sched_getaffinity(0)))     # the host share of one GPU
    prob = make_problems(workload)[0]
    rng = np.random.default_rng(7)
    t0 = time.perf_counter()
    _oracle_leaves((workload, 0, [0]))
    per_leaf = time.perf_counter() - t0
    res = {}
    # (a) process pool, one BLAS thread per process; each run holds about
    # budget/10 seconds of oracle work per process
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores, initializer=_pool_init) as pool:
        t0 = time.perf_counter()
        pool.map(_oracle_leaves, [(workload, 0, [0])] * cores)     # warm the workers
        t1 = time.perf_counter()
        pool.map(_oracle_leaves, [(workload, 0, [1 % prob.nleaf])] * cores)
        per_leaf_1 = time.perf_counter() - t1          # one leaf per worker, in parallel
        n_pool = max(cores, int(budget_s / 10.0 * cores / max(per_leaf_1, 1e-3)))
        runs = []
        for _ in range(5):
            ts = rng.choice(prob.nleaf, size=n_pool, replace=n_pool > prob.nleaf).tolist()
            chunks = [(workload, 0, ts[k::cores]) for k in range(cores)]
            t0 = time.perf_counter()
            n = sum(pool.map(_oracle_leaves, chunks))
            runs.append(n / (time.perf_counter() - t0))
            print(f"# cpu oracle, process pool: {runs[-1]:.1f} leaves/s", file=sys.stderr,
                  flush=True)
    res["process_pool"] = {"value": statistics.median(runs), "cores": cores,
                           "leaves_per_run": n_pool, "runs": runs}
    # (b) one process, threaded BLAS
    n_thr = max(2, int(budget_s / 10.0 / per_leaf))
    with threadpool_limits(limits=cores):
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        runs = []
        for _ in range(5):
            ts = rng.choice(prob.nleaf, size=n_thr, replace=n_thr > prob.nleaf).tolist()
            t0 = time.perf_counter()
            n = _oracle_leaves((workload, 0, ts))
            runs.append(n / (time.perf_counter() - t0))
            print(f"# cpu oracle, threaded BLAS: {runs[-1]:.1f} leaves/s", file=sys.stderr,
                  flush=True)
    res["threaded_blas"] = {"value": statistics.median(runs), "cores": threads,
                            "leaves_per_run": n_thr, "runs": runs}
    best = max(res, key=lambda k: res[k]["value"])
    return {"value": res[best]["value"], "unit": "leaves/s", "cores": res[best]["cores"],
            "kind": "oracle", "schedule": best,
            "sample": f"median of 5 runs of {res[best]['leaves_per_run']} random leaves of "
                      f"{prob.name} (p={prob.p}): operator build + LU condensation per leaf "
                      f"in numpy/LAPACK FP64",
            "schedules": {k: {kk: vv for kk, vv in v.items() if kk != "runs"}
                          for k, v in res.items()},
            "host_cpus_visible": len(os.sched_getaffinity(0))}


# --------------------------------------------------------------------------
# GPU timing
# --------------------------------------------------------------------------
def time_precision(B, prec, steps, warmup, max_refine, use_graph, use_tune, phases_on):
    """Tune (optionally), warm up, optionally capture one condense in a HIP
    graph, then time `steps` steps between HIP events on the library stream.
    Returns (ms per step, sorted per-step ms, phase times or None, tuned)."""
    import torch
    from paper_2211_14969_amd import hps
    S, w, info = B.alloc_outputs()
    tuned = None
    if use_tune:
        from paper_2211_14969_amd import tune
        res = tune.tune_batch(B, prec=prec, max_refine=max_refine, reps=1, cache_path=None)
        tuned = {B.groups[g].p: list(r["setting"]) for g, r in res.items()}

    def condense():
        hps.hps_leaf_condense(B.batch, prec, 0.0, max_refine, None, S, w, info, 0)

    for _ in range(max(warmup, 1)):
        condense()
    torch.cuda.synchronize()
    step = condense
    if use_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=torch.cuda.current_stream()):
            condense()
        torch.cuda.synchronize()
        step = graph.replay
        step()
        torch.cuda.synchronize()
    timing = phases_on and not use_graph
    hps.hps_ctx_set_timing(B.ctx, timing)
    hps.hps_ctx_phase_times(B.ctx)          # reset
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    evs[0].record()
    for i in range(steps):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    per = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    ms = evs[0].elapsed_time(evs[-1]) / steps
    phases = hps.hps_ctx_phase_times(B.ctx) if timing else None
    hps.hps_ctx_set_timing(B.ctx, False)
    assert int((info != 0).sum().item()) == 0, "a leaf reported a failure"
    return ms, per, phases, tuned


def accuracy(B, max_refine, nworst=2, nrand=2, seed=11):
    """Both precisions on the same batch: the largest per-leaf S gap between
    them over every leaf, and, for the leaves where it is largest plus a
    seeded sample (per problem), the relative errors of S, X and u against
    the FP64 oracle."""
    import numpy as np
    import torch
    from oracle import leaf as lf
    from paper_2211_14969_amd import hps
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    from _common import oracle_leaf, relerr

    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    ub = torch.randn(B.nb_total, generator=gen, dtype=torch.float64, device="cuda")
    out = {}
    precs = [("fp64", hps.HPS_FP64), ("fp32+refine", hps.HPS_FP32_REFINE)]
    if any(G.problem.has("a12") for G in B.groups):   # FP64 only for a mixed term
        precs = precs[:1]
    for name, prec in precs:
        S, _, info, st = B.condense(prec=prec, max_refine=max_refine, sync=True)
        Xt, _ = B.export()
        u = B.recover(ub, sync=True)
        out[name] = (S, Xt, u, hps.hps_batch_stats(B.batch)[1])
    gap_max, checked = 0.0, 0
    err = {k: {"S": 0.0, "X": 0.0, "u": 0.0} for k in out}
    rng = np.random.default_rng(seed)
    views = {k: (B.split(v[0], "S"), B.split(v[1], "Xt"), B.split(v[2], "ui"))
             for k, v in out.items()}
    ubs = B.split(ub, "ub")
    for gi, G in enumerate(B.groups):
        leaves = set()
        if "fp32+refine" in views:
            s64, s32 = views["fp64"][0][gi], views["fp32+refine"][0][gi]
            gap = (s32 - s64).flatten(1).norm(dim=1) / s64.flatten(1).norm(dim=1)
            gap_max = max(gap_max, gap.max().item())
            leaves.update(torch.topk(gap, min(nworst, G.nleaf)).indices.tolist())
        leaves.update(rng.choice(G.nleaf, size=min(nrand, G.nleaf), replace=False).tolist())
        ubh = ubs[gi].cpu().numpy()
        for t in sorted(leaves):
            bl, c = oracle_leaf(G.problem, t)
            u_or = lf.recover(c, ubh[t])
            checked += 1
            for k, (Sv, Xv, uv) in views.items():
                e = err[k]
                e["S"] = max(e["S"], relerr(Sv[gi][t].cpu().numpy(), c.S))
                e["X"] = max(e["X"], relerr(Xv[gi][t].cpu().numpy().T, c.X))
                e["u"] = max(e["u"], relerr(uv[gi][t].cpu().numpy(), u_or))
    return {"leaves_checked_vs_oracle": checked,
            "selection": (f"per problem the {nworst} leaves with the largest FP32-vs-FP64 S gap "
                          f"and {nrand} random (seed {seed})" if "fp32+refine" in out else
                          f"per problem {nrand} random leaves (seed {seed}); FP64 only"),
            "max_relerr_vs_oracle": err,
            "max_leaf_gap_S_fp32_vs_fp64_all_leaves": gap_max,
            "leaves_redone_fp64": out["fp32+refine"][3] if "fp32+refine" in out else None}


def recover_timing(B, steps: int):
    """Time hps_leaf_recover (stored X) on the condensed batch: u_i = h - X u_b
    per leaf.  HBM-bound: reads X (8 ni nb bytes per leaf) and u_b, writes u_i.
    Also the paper's alternative (Remark in Sec. 2): re-form and re-factor
    A_ii and solve for the one right-hand side f_i - A_ib u_b, nothing
    stored."""
    import torch
    from paper_2211_14969_amd import hps
    ub = torch.randn(B.nb_total, dtype=torch.float64, device="cuda")
    ui = torch.empty(B.ni_total, dtype=torch.float64, device="cuda")
    out = {}
    for name, flags in (("stored_x", 0), ("refactor", hps.HPS_RECOVER_REFACTOR)):
        hps.hps_leaf_recover(B.batch, ub, None, ui, flags)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            hps.hps_leaf_recover(B.batch, ub, None, ui, flags)
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / steps
    nbytes = sum(8.0 * G.nleaf * (G.ni * G.nb + G.nb + G.ni) for G in B.groups)
    gbs = nbytes / (out["stored_x"] * 1e-3) / 1e9
    return {"ms": out["stored_x"], "leaves_per_s": B.nleaf / (out["stored_x"] * 1e-3),
            "bytes": nbytes, "GB_per_s": gbs, "frac_hbm_peak": gbs / 8000.0, "bound": "hbm",
            "refactor_mode": {"ms": out["refactor"],
                              "leaves_per_s": B.nleaf / (out["refactor"] * 1e-3),
                              "precision": "fp64"}}


def iface_timing(B, prob, prec, max_refine: int, steps: int):
    """Time the FP64 interface solve (nested dissection on the device) of a
    single-problem batch (one group, or one group per order of a problem
    with mixed orders): the factorisation from the leaves' S and one solve
    for u_b.  Not part of the condensation step."""
    import torch
    from paper_2211_14969_amd.harness import (InterfaceSolver, dirichlet_data_batch,
                                              interface_unknowns)
    S, w, _, _ = B.condense(prec=prec, max_refine=max_refine, sync=True)
    g = dirichlet_data_batch(B)
    it = InterfaceSolver(B.ctx, prob, B)
    ub = torch.empty_like(w)
    it.factor(S, sync=True)
    it.solve(S, w, g, ub, sync=True)
    out = {}
    for name, fn in (("factor", lambda: it.factor(S)), ("solve", lambda: it.solve(S, w, g, ub))):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / steps
    plan = it.plan
    it.close()
    tf = plan["factor_flop"] / (out["factor"] * 1e-3) / 1e12
    return {"unknowns": interface_unknowns(prob),
            "fronts": plan["fronts"], "levels": plan["levels"],
            "max_separator": plan["max_separator"], "factor_ms": out["factor"],
            "solve_ms": out["solve"], "factor_flop": plan["factor_flop"],
            "factor_tflops": tf, "factor_frac_fp64_peak": tf / PEAK_TFLOPS["fp64"],
            "bytes": plan["bytes"], "precision": "fp64"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", choices=("fp64", "fp32"), default="fp64",
                    help="precision of the headline (fp32 = FP32 + FP64 refinement)")
    ap.add_argument("--max-refine", type=int, default=4)
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="approximate CPU time budget of the oracle baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the timing of the other precision")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the accuracy check against the oracle")
    ap.add_argument("--no-recover", action="store_true", help="skip the recovery timing")
    ap.add_argument("--no-iface", action="store_true",
                    help="skip the timing of the interface solve")
    ap.add_argument("--workload", default="bumps", choices=tuple(WORKLOADS),
                    help="; ".join(f"{k}: {v[1]}" for k, v in WORKLOADS.items()))
    ap.add_argument("--graph", choices=("auto", "on", "off"), default="auto",
                    help="time replays of one condense captured in a HIP graph "
                         "(auto: on for the uneven batch)")
    ap.add_argument("--tune", choices=("auto", "on", "off"), default="auto",
                    help="autotune every order group before timing (auto: on for the uneven batch)")
    ap.add_argument("--factor-variant", type=int, default=None,
                    help="force the factorisation variant of every order group "
                         "(hps_batch_set_tuning; default: the library's choice or the tuner's)")
    ap.add_argument("--factor-chunk", type=int, default=0,
                    help="tuning chunk passed with --factor-variant")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB three times "
                         "(calibrates the HBM traffic counters against a known byte count)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: leaves are independent, so a multi-GPU run "
              "would shard the batch; that path is not built (use --gpus 1).", file=sys.stderr)
        return 2

    import torch
    from paper_2211_14969_amd import hps
    from paper_2211_14969_amd.harness import LeafBatch

    if not torch.cuda.is_available():
        print("no ROCm device visible", file=sys.stderr)
        return 1
    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.copy_mib, "copies": 3}))
        return 0
    hps.load()
    uneven = args.workload == "uneven"
    use_graph = args.graph == "on" or (args.graph == "auto" and uneven)
    use_tune = args.tune == "on" or (args.tune == "auto" and uneven)
    # graph capture needs a stream other than the legacy default one; the
    # library context binds to the current stream when the batch is built
    torch.cuda.set_stream(torch.cuda.Stream())
    probs = make_problems(args.workload)
    prob = probs[0]
    L = sum(q.nleaf for q in probs)
    print(f"# workload {args.workload}: {L} leaves, p={[q.p for q in probs]}", file=sys.stderr,
          flush=True)
    B = LeafBatch(probs)
    if args.factor_variant is not None:
        for gi in range(len(B.groups)):
            hps.hps_batch_set_tuning(B.batch, gi, args.factor_variant, args.factor_chunk)
    prec_name = args.prec
    prec = hps.HPS_FP64 if prec_name == "fp64" else hps.HPS_FP32_REFINE
    ms, per, phases, tuned = time_precision(B, prec, args.steps, args.warmup, args.max_refine,
                                            use_graph, use_tune, phases_on=True)
    redo = hps.hps_batch_stats(B.batch)[1]
    print(f"# timed {prec_name}: {ms:.3f} ms per step", file=sys.stderr, flush=True)

    fl = {k: sum(algorithmic_flops(q.p)[k] * q.nleaf for q in probs) / L
          for k in ("factor", "backsolve", "schur", "total")}
    value = L / (ms * 1e-3)
    parent = getattr(prob, "parent", None)    # the problem of a mixed-order batch
    workload_name = (prob.name if len(probs) == 1 else
                     parent.name if parent is not None else "uneven_8_problems")
    line = {
        "metric": "leaf condensations/s + % MFMA peak; FP64 vs FP32+refine at <=1e-9 rel err",
        "value": value,
        "unit": "leaves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_step_median": per[len(per) // 2],
        "ms_per_step_min": per[0],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec_name == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": workload_name,
                   "leaves": L, "p": prob.p if len(probs) == 1 else [q.p for q in probs],
                   "kappa": prob.kappa if len(probs) == 1 else [q.kappa for q in probs],
                   "b": prob.meta.get("b"), "precision": prec_name, "max_refine": args.max_refine,
                   "graph_replay": use_graph, "tuned": tuned,
                   "factor_variant": args.factor_variant, "factor_chunk": args.factor_chunk,
                   "lanes": hps.hps_batch_lanes(B.batch), "parallelism": "single-gpu"},
        "useful_tflops": fl["total"] * L / (ms * 1e-3) / 1e12,
        "useful_frac_fp64_peak": fl["total"] * L / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"],
        "leaves_redone_fp64": redo,
    }
    if phases is not None:
        f_ms, f_n = phases["factor"]
        achieved = fl["factor"] * L * args.steps / (f_ms * 1e-3) / 1e12
        line["phases_ms_per_step"] = {k: v[0] / args.steps for k, v in phases.items() if v[1]}
        line["roofline"] = {"bound": "mfma", "kernel": "factorisation", "achieved": achieved,
                            "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                            "frac": achieved / PEAK_TFLOPS["fp64"], "traffic": None,
                            "per_launch_flop": fl["factor"] * L * args.steps / max(f_n, 1),
                            "launch_ms": f_ms / max(f_n, 1),
                            "launches_per_step": f_n / args.steps,
                            "timing": "HIP events around each launch on the library stream, "
                                      "inside the timed region"}
        tr = MEASURED_TRAFFIC.get((kernel_source_hash(), workload_name, prec_name))
        if tr is not None:
            line["roofline"]["kernel"] = tr["kernel"]
            line["roofline"]["traffic"] = tr["fetch_bytes"] + tr["write_bytes"]
            line["roofline"]["traffic_detail"] = dict(tr, unit="bytes per launch",
                                                      source="rocprofv3 --pmc, calibrated")

    mixed_term = any(q.has("a12") for q in probs)
    if mixed_term and prec == hps.HPS_FP32_REFINE:
        raise SystemExit("FP32 + refinement does not take operators with a mixed term")
    if not args.no_compare and not mixed_term:
        other = hps.HPS_FP32_REFINE if prec == hps.HPS_FP64 else hps.HPS_FP64
        ms2, per2, ph2, tuned2 = time_precision(B, other, max(5, args.steps // 2), 2,
                                                args.max_refine, use_graph, use_tune,
                                                phases_on=True)
        cmp_ = {"precision": "fp32+refine" if other == hps.HPS_FP32_REFINE else "fp64",
                "leaves_per_s": L / (ms2 * 1e-3), "ms_per_step": ms2,
                "ms_per_step_median": per2[len(per2) // 2], "graph_replay": use_graph,
                "tuned": tuned2, "leaves_redone_fp64": hps.hps_batch_stats(B.batch)[1],
                "speedup_vs_headline": ms / ms2}
        if ph2 is not None:
            cmp_["phases_ms_per_step"] = {k: v[0] / len(per2) for k, v in ph2.items() if v[1]}
        line["compare"] = cmp_
        print(f"# timed the other precision: {ms2:.3f} ms per step", file=sys.stderr, flush=True)

    if not args.no_accuracy:
        line["accuracy"] = accuracy(B, args.max_refine)
        print("# accuracy checked", file=sys.stderr, flush=True)

    if not args.no_recover:
        B.condense(prec=prec, max_refine=args.max_refine, sync=True)
        line["recover"] = recover_timing(B, max(3, args.steps // 2))

    if not args.no_iface and (len(probs) == 1 or parent is not None):
        try:
            line["interface_solve"] = iface_timing(B, parent if parent is not None else prob,
                                                   prec, args.max_refine, max(3, args.steps // 4))
            print("# timed the interface solve", file=sys.stderr, flush=True)
        except hps.HpsError as e:   # e.g. a separator above the build's limit
            line["interface_solve"] = {"skipped": str(e)}

    if not args.no_cpu:
        print("# timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
        if len(probs) > 1:
            line["cpu_baseline"]["sample"] += " (first problem of the batch)"
    B.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
