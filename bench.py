#!/usr/bin/env python3
"""Benchmark: one step = the whole hot path on one synthetic LP, on one GPU:
pdhg_create_device (ingest from HBM, transpose, scaling, step size),
pdhg_solve to the relative KKT tolerance, pdhg_corner_push (Algorithm 1 and
its early stop).  The default workload is the 2,000 x 5,000 transportation
LP (10M columns) in the FP32-mixed mode.

Prints ONE JSON line.  `value` is PDHG iterations per second over the timed
steps (solve + push iterations / wall time), with the LP already in device
memory when a step starts (it is copied there once, before the warm-up).
The roofline object covers the dominant iteration kernel: algorithmic bytes
per launch / mean launch duration measured live with HIP events on the
solver's stream during the timed steps.  Outside the timed region: the
learned-vs-plain comparison of the corner push and the CPU oracle's rate.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PDHG iter/s + HBM GB/s; time to 1e-6 KKT corner, learned vs plain"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c1": ("random sparse LP m=100000 n=400000 (power-law column degree 1..200, alpha 1.75; half the rows '<' "
           "with implicit slacks; 30% of columns with u~U(1,10); planted degenerate optimum, 15% dual-degenerate "
           "zeros; seed 1)"),
    "c2": "transportation LP 2000 sources x 5000 sinks (n=10M arcs, m=7000 rows, integer data; seed 2)",
    "c0": "random sparse LP m=200 n=500 (5 nnz per column, planted degenerate optimum; seed 0)",
    "c3": ("batch of 256 independent random sparse LPs, m log-uniform in [500, 20000], n = 2.5m, 4-8 nnz per "
           "column, planted degenerate optima (seeds 3000+i)"),
    "c4": ("multicommodity flow LP: 50000 nodes, 400000 arcs, 8 commodities (m=800000 node-balance + arc-capacity "
           "rows, n=3.2M, nnz=9.6M; seed 4100)"),
    "c5": ("random sparse LP m=100000 n=400000 with the c1 structure and a primal-degenerate planted optimum (85% "
           "of columns at zero, none dual-degenerate: fewer variables off their bounds than rows, a large dual "
           "optimal face; seed 5)"),
}


# oracle iterations timed for the CPU baseline (all cores, one thread): about
# 10-20 s each on a 16-thread host (c2 and c4 hold 10M and 3.2M columns)
CPU_ITERS = {"c0": (20000, 5000), "c1": (2000, 200), "c2": (200, 30), "c4": (400, 60), "c5": (2000, 200)}

PUSH_WORDS = {"primal": "corner push", "dual": "dual corner push",
              "both": "corner push + dual corner push from its pushed x"}


def make_lp(cfg):
    from paper_2511_13894_amd import lpgen

    if cfg == "c1":
        return lpgen.config1(1)
    if cfg == "c2":
        return lpgen.config2(2)
    if cfg == "c4":
        return lpgen.config4()
    if cfg == "c5":
        return lpgen.config5()
    return lpgen.config0(0)


# Everything that shapes a profiled run of the solve and the pushes: the
# iteration, check, setup, push, compaction and batch sources, the host code
# that drives them, and the input generator (the predictor's network and
# features play no part in it).  A counter summary counts only while this
# hash is unchanged.
SOURCE_FILES = ("pdhg_iter.hip", "pdhg_kernels.hpp", "pdhg_device.hpp", "pdhg_internal.hpp", "pdhg_setup.hip",
                "pdhg_compact.hip", "pdhg_sell.hip", "pdhg_batch.hip", "pdhg_capi.cpp", "../lpgen.py")


def kernel_source_hash(files=SOURCE_FILES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2511_13894_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(cfg, kernel, precision, push, push_compact):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this workload (config, precision, push mode, push on free columns), if
    it was taken on the current sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{cfg}_{precision}_counters.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    fields = dict(re.findall(r"^(\w+):\s*(\S+)", txt, flags=re.M))
    want = {"kernel_source_hash": kernel_source_hash(), "precision": precision, "push": push,
            "push_compact": str(int(push_compact))}
    if any(fields.get(k) != v for k, v in want.items()) or "hbm_bytes_per_launch" not in fields:
        return None
    return float(fields["hbm_bytes_per_launch"])


def cpu_baseline(lp, iters, iters_one, cfg):
    """The CPU oracle as it stands, timed on this host after its setup: `iters`
    float64 PDHG iterations of the same LP on every core it uses, then
    `iters_one` on one thread."""
    from oracle import OracleSolver, num_threads, set_threads

    o = OracleSolver(lp, eps_rel=1e-30)
    cores = num_threads()
    t0 = time.perf_counter()
    o.iterate(iters)
    dt = time.perf_counter() - t0
    set_threads(1)
    t1 = time.perf_counter()
    o.iterate(iters_one)
    dt1 = time.perf_counter() - t1
    set_threads(cores)
    return {"value": iters / dt, "unit": "iter/s", "cores": cores, "kind": "oracle",
            "sample": f"{cfg}, {iters} float64 PDHG iterations after setup on {cores} threads ({dt:.1f} s)",
            "single_thread": {"value": iters_one / dt1, "unit": "iter/s", "cores": 1,
                              "sample": f"the next {iters_one} iterations on 1 thread ({dt1:.1f} s)"}}


PREDICTOR = os.path.join(ROOT, "paper_2511_13894_amd", "predictor.json")


def learned_vs_plain(path):
    """Outside the timed region: the corner push with the committed learned
    warm start against the plain push, on the multicommodity evaluation LP
    (single LP) and on 64 held-out LPs of the batched family (learned+batched
    against plain batched), both FP32-mixed.  Each arm's time to the corner is
    create + solve + push; max(p - m, 0) and the candidate count are the
    pushed point's."""
    from paper_2511_13894_amd import learned, lpgen

    net, theta, meta = learned.load_predictor(path)
    keys = ("seconds", "push_iters", "push_lockstep", "push_lp_iters", "est_primal_after", "candidates_after",
            "off_bound_after", "learned_fix", "learned_undo", "push_status", "push_done", "optimal")
    pick = lambda d: None if d is None else {k: d[k] for k in keys if k in d}  # noqa: E731
    out = {"predictor": os.path.relpath(path, ROOT), "theta": theta, "trained_by": meta.get("command")}
    lp = lpgen.config4()
    print("[bench] learned vs plain: multicommodity LP", file=sys.stderr, flush=True)
    plain = learned.time_to_corner(lp, 4100, "fp32")
    lrn = learned.time_to_corner(lp, 4100, "fp32", net, theta)
    out["c4"] = {"workload": WORKLOADS["c4"], "plain": pick(plain), "learned": pick(lrn)}
    m_range = tuple(meta.get("val_lps", [0, 0, [500, 20000]])[2])
    ev = [lpgen.config3_instance(i, base_seed=43000, m_range=m_range) for i in range(64)]
    seeds = [500 + i for i in range(len(ev))]
    print("[bench] learned vs plain: 64 held-out LPs, batched", file=sys.stderr, flush=True)
    out["batched_64"] = {"workload": f"64 held-out LPs of the batched family (seeds 43000+i, m in {list(m_range)})",
                         "plain": pick(learned.batch_time_to_corner(ev, seeds, "fp32")),
                         "learned": pick(learned.batch_time_to_corner(ev, seeds, "fp32", net, theta))}
    return out


def bench_batch(args, pdhg, copy_gbs):
    """The batched family: one step = batch create + solve + corner push (or dual corner push) of all 256 LPs."""
    from paper_2511_13894_amd import lpgen

    lps = [lpgen.config3_instance(i) for i in range(256)]
    seeds = [args.seed + i for i in range(len(lps))]
    tot_m, tot_n, tot_nz = sum(l.m for l in lps), sum(l.n for l in lps), sum(l.nnz for l in lps)
    print(f"[bench] c3: {len(lps)} LPs, {tot_m} rows, {tot_n} columns, {tot_nz} nonzeros", file=sys.stderr,
          flush=True)

    # the LPs are copied to HBM once, before any timed step: a step starts from
    # them in device memory (pdhg_batch_create_device)
    dlps = pdhg.DeviceBatch(lps)

    def step(timing):
        b = pdhg.Batch(dlps, precision=args.precision, timing=timing, use_graph=0 if args.no_graph else 1,
                       push_compact=args.push_compact)
        res = b.solve()
        push = b.corner_push(seeds) if args.push == "primal" else b.dual_push(seeds)
        rep = b.report()
        b.destroy()
        return res, push, rep

    for w in range(args.warmup):
        res, push, _ = step(0)
        print(f"[bench] warmup {w}: {sum(r.iters for r in res)} solve + {sum(p.iters for p in push)} push "
              f"LP-iterations", file=sys.stderr, flush=True)
    lp_iters, prim, dual, samples, bp, bd = 0, 0.0, 0.0, 0, 0.0, 0.0
    details = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        res, push, rep = step(1)
        te = time.perf_counter()
        si, pi = sum(r.iters for r in res), sum(p.iters for p in push)
        lp_iters += si + pi
        prim += rep.primal_ms * rep.samples
        dual += rep.dual_ms * rep.samples
        bp += rep.bytes_primal * rep.samples
        bd += rep.bytes_dual * rep.samples
        samples += rep.samples
        status = {}
        for r in res:
            status[pdhg.STATUS[r.status]] = status.get(pdhg.STATUS[r.status], 0) + 1
        d = {"step_s": te - ts, "solve_s": rep.solve_seconds, "solve_lp_iters": si, "push_lp_iters": pi,
             "solve_lockstep": rep.solve_lockstep_iters, "solve_status": status, "kernels": [rep.lanes_at, rep.lanes_a]}
        if args.push == "primal":
            d.update({"push_s": rep.push_seconds, "push_lockstep": rep.push_lockstep_iters,
                      "off_bound_before": sum(p.before.p_off for p in push),
                      "off_bound_after": sum(p.after.p_off for p in push),
                      "est_primal_before": sum(p.before.est_primal for p in push),
                      "est_primal_after": sum(p.after.est_primal for p in push)})
        else:
            d.update({"push_s": push[0].seconds if push else 0.0, "push_lockstep": max(p.iters for p in push),
                      "est_dual_before": sum(p.before.est_dual for p in push),
                      "est_dual_after": sum(p.after.est_dual for p in push),
                      "push_status": sorted({pdhg.STATUS[p.status] for p in push})})
        details.append(d)
        print(f"[bench] step {k}: {te - ts:.3f}s, {si} solve + {pi} push LP-iterations, status {status}",
              file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t_start
    n = max(samples, 1)
    prim_ms, dual_ms, bytes_p, bytes_d = prim / n, dual / n, bp / n, bd / n
    if prim_ms >= dual_ms:
        kname, ms, nbytes, other = "kb_primal", prim_ms, bytes_p, ("kb_dual", dual_ms, bytes_d)
    else:
        kname, ms, nbytes, other = "kb_dual", dual_ms, bytes_d, ("kb_primal", prim_ms, bytes_p)
    achieved = nbytes / (ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(lp_iters / elapsed, 1), "unit": "LP-iter/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64norms", "data": "synthetic",
        "config": {"workload": f"c3: {WORKLOADS['c3']}; step = batch create from the LPs in HBM + solve to 1e-6 relative KKT + "
                               f"{'corner push' if args.push == 'primal' else 'dual corner push'} of every LP",
                   "lps": len(lps), "m": tot_m, "n": tot_n, "nnz": tot_nz, "precision": args.precision,
                   "eps_rel": 1e-6, "push_on_free_columns": bool(args.push_compact) and args.push == "primal",
                   "push": args.push},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile("c3", kname, args.precision, args.push,
                                                                    args.push_compact),
                     "kernel": kname,
                     "launch_us": round(ms * 1e3, 2), "algorithmic_bytes_per_launch": int(nbytes),
                     "other_kernel": {"name": other[0], "launch_us": round(other[1] * 1e3, 2),
                                      "algorithmic_bytes_per_launch": int(other[2])},
                     "timed_launches": int(samples), "copy_probe_gbs": round(copy_gbs, 1),
                     "iteration_pair": {"algorithmic_bytes": int(bytes_p + bytes_d),
                                        "us": round((prim_ms + dual_ms) * 1e3, 2),
                                        "achieved": round((bytes_p + bytes_d) / ((prim_ms + dual_ms) * 1e-3) / 1e9, 1),
                                        "frac": round((bytes_p + bytes_d) / ((prim_ms + dual_ms) * 1e-3) / 1e9
                                                      / HBM_PEAK_GBS, 4)}},
        "detail": {"steps": details},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        from oracle import OracleSolver, num_threads

        sample, it_each, dt = lps[:32], 2 * (args.cpu_iters or 2000), 0.0
        for lp in sample:
            o = OracleSolver(lp, eps_rel=1e-30)
            t0 = time.perf_counter()
            o.iterate(it_each)
            dt += time.perf_counter() - t0
        out["cpu_baseline"] = {"value": len(sample) * it_each / dt, "unit": "LP-iter/s", "cores": num_threads(),
                               "kind": "oracle",
                               "sample": f"the first {len(sample)} LPs of c3, {it_each} float64 PDHG iterations each "
                                         f"after setup, one LP at a time ({dt:.1f} s)"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32"],
                    help="fp32: FP32-mixed (float matrix, n-vectors as float differences from float64 anchors, float64 checks); fp64")
    ap.add_argument("--learned", default=PREDICTOR,
                    help="predictor file for the learned-vs-plain comparison outside the timed region ('' skips it)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="oracle iterations for the CPU baseline (0: the workload's default)")
    ap.add_argument("--iters-only", type=int, default=0,
                    help="profiling runs: create + this many iterations per step, no push, no JSON roofline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--push-compact", type=int, default=1, choices=[0, 1],
                    help="1 (default): the push iterates on its free columns; 0: on the full push model")
    ap.add_argument("--push", default="primal", choices=["primal", "dual", "both"],
                    help="primal (default): the corner push of Algorithm 1; dual: the dual corner push; both: "
                         "the corner push, then the dual push from its pushed x (single LP only)")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every cycle eagerly instead of replaying captured hipGraphs (profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a design note, "
              "not a built path", file=sys.stderr)
        sys.exit(2)
    if args.config == "c3" and args.push == "both":
        print("--push both is a single-LP option; c3 is a batch", file=sys.stderr)
        sys.exit(2)

    from paper_2511_13894_amd import pdhg

    t0 = time.perf_counter()
    lp = make_lp(args.config) if args.config != "c3" else None
    gen_s = time.perf_counter() - t0
    if lp is not None:
        print(f"[bench] {args.config} m={lp.m} n={lp.n} nnz={lp.nnz} generated in {gen_s:.1f}s", file=sys.stderr,
              flush=True)
    copy_gbs = pdhg.copy_probe(1 << 30, 20)
    print(f"[bench] copy probe 1 GiB: {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    if args.config == "c3":
        return bench_batch(args, pdhg, copy_gbs)

    if args.iters_only:
        for k in range(args.steps):
            s = pdhg.Solver(pdhg.DeviceLP(lp), precision=args.precision, use_graph=0 if args.no_graph else 1)
            r = s.iterate(args.iters_only)
            s.destroy()
            print(f"[bench] profiling step {k}: {r.iters} iterations", file=sys.stderr, flush=True)
        return

    # the inputs are copied to HBM once, before any timed step: a step starts
    # from the LP in device memory (pdhg_create_device), as the metric asks
    dlp = pdhg.DeviceLP(lp)

    def step(timing):
        t0 = time.perf_counter()
        s = pdhg.Solver(dlp, precision=args.precision, timing=timing, use_graph=0 if args.no_graph else 1,
                        push_compact=args.push_compact)
        step.create_s = time.perf_counter() - t0
        r = s.solve()
        p = s.corner_push(args.seed) if args.push != "dual" else s.dual_push(args.seed)
        d = s.dual_push(args.seed) if args.push == "both" else None
        t = s.get_timing() if timing else None
        s.destroy()
        return r, p, t, d

    for w in range(args.warmup):
        r, p, _, _ = step(0)
        print(f"[bench] warmup {w}: solve {r.iters} it ({pdhg.STATUS[r.status]}), push {p.iters} it "
              f"({pdhg.STATUS[p.status]})", file=sys.stderr, flush=True)
    iters = 0
    prim_ms = dual_ms = 0.0
    samples = 0
    tim = None
    details = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        r, p, tim, dp = step(1)
        te = time.perf_counter()
        iters += r.iters + p.iters + (dp.iters if dp is not None else 0)
        prim_ms += tim.primal_ms * tim.samples
        dual_ms += tim.dual_ms * tim.samples
        samples += tim.samples
        d = {"solve_iters": r.iters, "solve_status": pdhg.STATUS[r.status], "push_iters": p.iters,
             "push_status": pdhg.STATUS[p.status], "step_s": te - ts, "create_s": step.create_s,
             "solve_s": r.seconds, "push_s": p.seconds,
             "rel_kkt": [r.rel_p, r.rel_d, r.rel_gap], "pobj": r.pobj}
        if args.push != "dual":
            d.update({"off_bound_before": p.before.p_off, "off_bound_after": p.after.p_off,
                      "candidates_before": p.before.candidates, "candidates_after": p.after.candidates,
                      "est_primal_before": p.before.est_primal, "est_primal_after": p.after.est_primal,
                      "fixed": p.n_fix_lower + p.n_fix_upper, "rows_to_eq": p.n_rows_to_eq})
        else:
            d.update({"zero_rc_before": p.before.d_zero, "zero_rc_after": p.after.d_zero,
                      "est_dual_before": p.before.est_dual, "est_dual_after": p.after.est_dual,
                      "cols_free": p.n_cols_free, "rows_fixed": p.n_rows_fixed,
                      "rel_d_push": p.rel_d_push})
        if dp is not None:
            d.update({"dual_push_iters": dp.iters, "dual_push_status": pdhg.STATUS[dp.status],
                      "dual_push_s": dp.seconds, "est_dual_before": dp.before.est_dual,
                      "est_dual_after": dp.after.est_dual, "zero_rc_before": dp.before.d_zero,
                      "zero_rc_after": dp.after.d_zero, "cols_free": dp.n_cols_free, "rows_fixed": dp.n_rows_fixed,
                      "final_rel_kkt": [dp.after.rel_p, dp.after.rel_d, dp.after.rel_gap]})
        details.append(d)
        print(f"[bench] step {k}: {te - ts:.3f}s solve {r.iters} push {p.iters}"
              + (f" dual push {dp.iters}" if dp is not None else ""), file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t_start
    value = iters / elapsed
    prim_ms /= max(samples, 1)
    dual_ms /= max(samples, 1)
    # dominant kernel: larger share of the iteration time
    if prim_ms >= dual_ms:
        kname, ms, nbytes = "k_primal", prim_ms, tim.bytes_primal
    else:
        kname, ms, nbytes = "k_dual", dual_ms, tim.bytes_dual
    achieved = nbytes / (ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_from_profile(args.config, kname, args.precision, args.push, args.push_compact),
            "kernel": kname, "launch_us": round(ms * 1e3, 2), "algorithmic_bytes_per_launch": int(nbytes),
            "other_kernel": {"name": "k_dual" if kname == "k_primal" else "k_primal",
                             "launch_us": round((dual_ms if kname == "k_primal" else prim_ms) * 1e3, 2),
                             "algorithmic_bytes_per_launch": int(tim.bytes_dual if kname == "k_primal"
                                                                 else tim.bytes_primal)},
            "timed_launches": int(samples), "copy_probe_gbs": round(copy_gbs, 1)}
    # the two halves of one PDHG iteration together (they take about the same time)
    pair_bytes, pair_ms = tim.bytes_primal + tim.bytes_dual, prim_ms + dual_ms
    roof["iteration_pair"] = {"algorithmic_bytes": int(pair_bytes), "us": round(pair_ms * 1e3, 2),
                              "achieved": round(pair_bytes / (pair_ms * 1e-3) / 1e9, 1),
                              "frac": round(pair_bytes / (pair_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 2), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64norms", "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}; step = create + solve to 1e-6 relative "
                               f"KKT + {PUSH_WORDS[args.push]}",
                   "m": lp.m, "n": lp.n, "nnz": lp.nnz,
                   "precision": args.precision, "eps_rel": 1e-6, "push_seed": args.seed,
                   "push_on_free_columns": bool(args.push_compact) and args.push != "dual",
                   "push": args.push},
        "roofline": roof,
        "detail": {"steps": details, "time_to_corner_s": round(elapsed / args.steps, 4),
                   "lanes_at": tim.lanes_at, "lanes_a": tim.lanes_a},
    }
    if args.learned and os.path.exists(args.learned):
        out["learned_vs_plain"] = learned_vs_plain(args.learned)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        n_all, n_one = CPU_ITERS.get(args.config, (2000, 200))
        if args.cpu_iters:
            n_all, n_one = args.cpu_iters, max(1, args.cpu_iters // 10)
        out["cpu_baseline"] = cpu_baseline(lp, n_all, n_one, f"{args.config} at full size")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
