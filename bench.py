#!/usr/bin/env python3
"""Throughput of batched HPS leaf condensation on one MI355X.

One step = one pass of the whole hot path over the batch: form every leaf's
collocation operator on the device, factor A_ii, solve for X = A_ii^{-1} A_ib
and form S = A_bb - A_bi X (plus the FP64 refinement of X in the mixed
precision mode).  Inputs (leaf boxes, coefficient samples) are resident in
HBM before the timed region; nothing is copied to or from the host inside it.
For the uneven eight-problem batch the step is the replay of one condense
captured in a HIP graph, after the autotuner has picked the factorisation
variant per order.  Recovery u_i = h - X u_b is timed separately against the
HBM roofline.

Workload: the unit square split into 64 x 64 leaves of order p = 16,
kappa = 100, b(x) = 1 - 0.5 exp(-|x - (0.5, 0.5)|^2 / 0.05), in FP64.  The
same batch is also condensed in FP32 + FP64 refinement and compared against
the FP64 result; the plain FP64 CPU oracle is timed on a bounded sample of
the same leaves.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}

# Calibrated HBM traffic of one factorisation launch, from rocprofv3 --pmc
# FETCH_SIZE / WRITE_SIZE (KiB per dispatch, FETCH scaled by 2.0 and WRITE by
# 1.0 against a 1 GiB device copy), keyed by the sha256 prefix of the kernel
# source it was measured on, the workload and the precision.
MEASURED_TRAFFIC = {
    ("d795a6e2ac355df0", "bump_64x64_p16", "fp64"): {
        "kernel": "k_factor2_t<double, 2>",
        "fetch_bytes": 3003746.896 * 2.0 * 1024, "write_bytes": 8168543.906 * 1.0 * 1024},
    ("d795a6e2ac355df0", "bump_64x64_p16", "fp32"): {
        "kernel": "k_factor2_t<float, 3>",
        "fetch_bytes": 1477504.146 * 2.0 * 1024, "write_bytes": 4122125.177 * 1.0 * 1024},
    ("d795a6e2ac355df0", "bumps_32x32_p32", "fp64"): {
        "kernel": "k_factorP<double, 512, 2>",
        "fetch_bytes": 51446724.896 * 2.0 * 1024, "write_bytes": 93056184.031 * 1.0 * 1024},
}


def kernel_source_hash() -> str:
    import hashlib
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "paper_2211_14969_amd", "csrc", "hps_kernels.hip")
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


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


def cpu_baseline(problem, seconds: float):
    """Time the FP64 CPU oracle (operator build + LAPACK condensation) on
    consecutive leaves of the workload until `seconds` have elapsed."""
    import numpy as np
    from oracle import leaf as lf
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = 1
    boxes = problem.boxes()
    t0 = time.perf_counter()
    n = 0
    while True:
        box = boxes[n % problem.nleaf]
        coef = lf.sample_coefficients(problem, box, problem.p)
        lf.condense(lf.blocks(box, problem.p, coef))
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds and n >= 4:
            break
    return {"value": n / el, "unit": "leaves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} consecutive leaves of the same workload, {el:.1f} s, "
                      f"operator build + LU condensation per leaf in numpy/LAPACK FP64",
            "host_cpus": len(os.sched_getaffinity(0))}


def recover_timing(B, steps: int):
    """Time hps_leaf_recover (stored X) on the condensed batch: u_i = h - X u_b
    per leaf.  HBM-bound: reads X (8 ni nb bytes per leaf) and u_b, writes u_i."""
    import torch
    from paper_2211_14969_amd import hps
    ub = torch.randn(B.nb_total, dtype=torch.float64, device="cuda")
    ui = torch.empty(B.ni_total, dtype=torch.float64, device="cuda")
    hps.hps_leaf_recover(B.batch, ub, None, ui, 0)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        hps.hps_leaf_recover(B.batch, ub, None, ui, 0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nbytes = sum(8.0 * G.nleaf * (G.ni * G.nb + G.nb + G.ni) for G in B.groups)
    gbs = nbytes / (ms * 1e-3) / 1e9
    # the paper's alternative (Remark in Sec. 2): re-form and re-factor A_ii
    # and solve for the one right-hand side f_i - A_ib u_b, nothing stored
    flags = hps.HPS_RECOVER_REFACTOR
    hps.hps_leaf_recover(B.batch, ub, None, ui, flags)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        hps.hps_leaf_recover(B.batch, ub, None, ui, flags)
    e1.record()
    torch.cuda.synchronize()
    ms_rf = e0.elapsed_time(e1) / steps
    return {"ms": ms, "leaves_per_s": B.nleaf / (ms * 1e-3), "bytes": nbytes, "GB_per_s": gbs,
            "frac_hbm_peak": gbs / 8000.0, "bound": "hbm",
            "refactor_mode": {"ms": ms_rf, "leaves_per_s": B.nleaf / (ms_rf * 1e-3),
                              "precision": "fp64"}}


def worst_leaf_floor(B, gi: int, t: int) -> dict:
    """Order, cond_2(A_ii) and the FP64 floor 10 cond 2^-53 of leaf t of group
    gi: two correct FP64 results for that leaf may differ by about that much
    (rounding the operator entries alone moves X so far)."""
    import numpy as np
    import torch
    from paper_2211_14969_amd import hps
    G = B.groups[gi]
    d = {"p": G.p, "box": G.box[t:t + 1].contiguous()}
    for name, c in G.coef.items():
        d[name] = c[t:t + 1].contiguous()
    one = hps.hps_leaf_build(B.ctx, [d])
    Aii = torch.empty((1, G.ni, G.ni), dtype=torch.float64, device="cuda")
    hps.hps_leaf_operator(one, 0, Aii)
    torch.cuda.synchronize()
    hps.hps_batch_destroy(one)
    cond = float(np.linalg.cond(Aii[0].cpu().numpy()))
    return {"p": G.p, "leaf": t, "cond_Aii": cond, "fp64_floor": 10.0 * cond * 2.0 ** -53}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", choices=("fp64", "fp32"), default=None,
                    help="precision of the timed path (fp32 = FP32 + FP64 refinement); "
                         "default fp64, fp32 for the uneven batch")
    ap.add_argument("--max-refine", type=int, default=4)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the run of the other precision on the same batch")
    ap.add_argument("--no-recover", action="store_true", help="skip the recovery timing")
    ap.add_argument("--workload", default="bump",
                    choices=("bump", "tiny", "bumps", "annulus", "uneven"),
                    help="bump: 64x64 leaves p=16 (default, the headline configuration); "
                         "tiny: 4x4 p=8; bumps: 32x32 p=32; annulus: 128x16 p=20; "
                         "uneven: the eight-problem batch p=8..32 in one batch")
    ap.add_argument("--graph", choices=("auto", "on", "off"), default="auto",
                    help="time replays of one condense captured in a HIP graph "
                         "(auto: on for the uneven batch)")
    ap.add_argument("--tune", choices=("auto", "on", "off"), default="auto",
                    help="autotune every order group before timing (auto: on for the uneven batch)")
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
    from paper_2211_14969_amd import hps, inputs
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
    prec_name = args.prec or ("fp32" if uneven else "fp64")
    use_graph = args.graph == "on" or (args.graph == "auto" and uneven)
    use_tune = args.tune == "on" or (args.tune == "auto" and uneven)
    if use_graph:
        # capture needs a stream other than the legacy default one; the
        # library context binds to the current stream when the batch is built
        torch.cuda.set_stream(torch.cuda.Stream())
    probs = {"bump": lambda: [inputs.single_bump()], "tiny": lambda: [inputs.tiny()],
             "bumps": lambda: [inputs.multi_bump()], "annulus": lambda: [inputs.annulus()],
             "uneven": lambda: inputs.uneven_batch()}[args.workload]()
    prob = probs[0]
    p, L = prob.p, sum(q.nleaf for q in probs)
    print(f"# workload {args.workload}: {L} leaves, p={[q.p for q in probs]}", file=sys.stderr,
          flush=True)
    B = LeafBatch(probs)
    S, w, info = B.alloc_outputs()
    prec = hps.HPS_FP64 if prec_name == "fp64" else hps.HPS_FP32_REFINE
    tuned = None
    if use_tune:
        from paper_2211_14969_amd import tune
        tuned = tune.tune_batch(B, prec=prec, max_refine=args.max_refine, reps=1, cache_path=None)
        tuned = {B.groups[g].p: list(r["setting"]) for g, r in tuned.items()}
        print(f"# tuned (variant, chunk) per order: {tuned}", file=sys.stderr, flush=True)

    def condense(pr=prec, S_=S):
        hps.hps_leaf_condense(B.batch, pr, 0.0, args.max_refine, None, S_, w, info, 0)

    for _ in range(max(args.warmup, 1)):
        condense()
    torch.cuda.synchronize()
    st = hps.hps_leaf_condense(B.batch, prec, 0.0, args.max_refine, None, S, w, info, hps.HPS_SYNC)
    print(f"# warmup done, status {st}", file=sys.stderr, flush=True)
    step = condense
    if use_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=torch.cuda.current_stream()):
            condense()
        torch.cuda.synchronize()
        step = graph.replay

    hps.hps_ctx_set_timing(B.ctx, not use_graph)
    hps.hps_ctx_phase_times(B.ctx)          # reset
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    evs[0].record()
    for i in range(args.steps):
        step()
        evs[i + 1].record()
    torch.cuda.synchronize()
    per = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
    ms = evs[0].elapsed_time(evs[-1]) / args.steps
    phases = hps.hps_ctx_phase_times(B.ctx)
    hps.hps_ctx_set_timing(B.ctx, False)
    bad = int((info != 0).sum().item())
    redo = hps.hps_batch_stats(B.batch)[1]

    fl = {k: sum(algorithmic_flops(q.p)[k] * q.nleaf for q in probs) / L
          for k in ("factor", "backsolve", "schur", "total")}
    dtype = "f64" if prec_name == "fp64" else "f32+f64"
    peak = PEAK_TFLOPS["fp64"]
    value = L / (ms * 1e-3)
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
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": prob.name if len(probs) == 1 else "uneven_8_problems",
                   "leaves": L, "p": p if len(probs) == 1 else [q.p for q in probs],
                   "kappa": prob.kappa if len(probs) == 1 else [q.kappa for q in probs],
                   "b": prob.meta.get("b"), "precision": prec_name, "max_refine": args.max_refine,
                   "graph_replay": use_graph, "tuned": tuned, "parallelism": "single-gpu"},
        "useful_tflops": fl["total"] * L / (ms * 1e-3) / 1e12,
        "useful_frac_fp64_peak": fl["total"] * L / (ms * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"],
        "leaves_with_nonzero_info": bad,
        "leaves_redone_fp64": redo,
    }
    if not use_graph:
        f_ms, f_n = phases["factor"]
        t_factor = f_ms / args.steps          # ms of factorisation launches per step
        achieved = fl["factor"] * L / (t_factor * 1e-3) / 1e12
        line["phases_ms_per_step"] = {k: v[0] / args.steps for k, v in phases.items() if v[1]}
        # every tile product runs on the FP64 MFMA in both precisions
        line["roofline"] = {"bound": "mfma", "kernel": "factorisation", "achieved": achieved,
                            "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                            "traffic": None,
                            "per_launch_flop": fl["factor"] * L * args.steps / max(f_n, 1),
                            "launch_ms": f_ms / max(f_n, 1),
                            "launches_per_step": f_n / args.steps}
        tr = MEASURED_TRAFFIC.get((kernel_source_hash(), line["config"]["workload"], prec_name))
        if tr is not None:
            line["roofline"]["kernel"] = tr["kernel"]
            line["roofline"]["traffic"] = tr["fetch_bytes"] + tr["write_bytes"]
            line["roofline"]["traffic_detail"] = dict(tr, unit="bytes per launch",
                                                      source="rocprofv3 --pmc, calibrated")

    if not args.no_compare:
        other = hps.HPS_FP32_REFINE if prec == hps.HPS_FP64 else hps.HPS_FP64
        S2 = torch.empty_like(S)
        for _ in range(2):
            condense(other, S2)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        n2 = max(3, args.steps // 2)
        e0.record()
        for _ in range(n2):
            condense(other, S2)
        e1.record()
        torch.cuda.synchronize()
        ms2 = e0.elapsed_time(e1) / n2
        rel, worst, above = 0.0, (0, 0), 0
        for gi, (Sa, Sb) in enumerate(zip(B.split(S, "S"), B.split(S2, "S"))):
            r = (Sa - Sb).flatten(1).norm(dim=1) / Sb.flatten(1).norm(dim=1)
            above += int((r > 1e-9).sum().item())
            m, t = r.max(dim=0)
            if m.item() > rel:
                rel, worst = m.item(), (gi, int(t.item()))
        redo2 = hps.hps_batch_stats(B.batch)[1]
        line["compare"] = {"precision": "fp32+refine" if other == hps.HPS_FP32_REFINE else "fp64",
                           "leaves_redone_fp64": redo2,
                           "leaves_per_s": L / (ms2 * 1e-3), "ms_per_step": ms2,
                           "eager": True,
                           "max_leaf_relerr_S_vs_other": rel,
                           "leaves_above_1e-9": above,
                           "worst_leaf": worst_leaf_floor(B, *worst)}
        condense()               # leave the timed precision's X in the batch
        torch.cuda.synchronize()

    if not args.no_recover:
        line["recover"] = recover_timing(B, max(3, args.steps // 2))

    if not args.no_cpu:
        print("# timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
        if len(probs) > 1:
            line["cpu_baseline"]["sample"] += f" (first problem, p={prob.p})"
    B.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
