"""Learned warm start of the corner push: data, training, evaluation.

The training data are the method's own trajectories: every LP is solved with
restart history recorded, its 16 features are read from the device, the plain
corner push (Algorithm 1) runs, and the label of a column is 1 iff the pushed
x ends at one of its bounds (within 1e-6).  The network is trained on the GPU
by the library's BF16 MFMA kernels; theta is chosen on a validation split so
that, among the columns the plain rule leaves free, the predicted fixes are
right at least `min_precision` of the time.  The comparison of the two arms
times create + solve + push (the time to the corner) and reports the primal
push estimate max(p - m, 0) and the off-bound/small-|z| count after the push.

Command line: python -m paper_2511_13894_amd.learned --train 200 --val 40 --eval 20
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import lpgen, pdhg


USE_GRAPH = 1  # 0: every cycle launched eagerly (profiler runs)


def solve_and_label(lp, seed, precision="fp64", eps=1e-6, eps_abs=1e-6):
    """(features, labels, mask, solve result, push result) of one LP, or None.

    The mask selects the columns a learned fix may touch: left free by the
    plain rule (|z_j| <= eps_abs) and bounded on at least one side."""
    s = pdhg.Solver(lp, precision=precision, record_history=1, eps_rel=eps, eps_abs=eps_abs, use_graph=USE_GRAPH)
    r = s.solve()
    if r.status != pdhg.PDHG_OPTIMAL:
        return None
    _, _, z = s.get_solution()
    f = s.features(seed)
    p = s.corner_push(seed)
    x, _, _ = s.get_solution()
    at_bound = (x - lp.l <= 1e-6) | (lp.u - x <= 1e-6)
    mask = (np.abs(z) <= eps_abs) & (np.isfinite(lp.l) | np.isfinite(lp.u))
    return f, at_bound.astype(np.float32), mask, r, p


def build_dataset(lps, seeds, precision="fp64", log=None):
    """Features and labels of the masked columns of every LP that solves."""
    feats, labels = [], []
    t0 = time.time()
    for i, (lp, sd) in enumerate(zip(lps, seeds)):
        out = solve_and_label(lp, sd, precision)
        if out is None:
            continue
        f, y, mask, _, _ = out
        feats.append(f[mask])
        labels.append(y[mask])
        if log and (i + 1) % 20 == 0:
            log(f"[learned] data {i + 1}/{len(lps)} LPs, {sum(a.shape[0] for a in feats)} free columns, "
                f"{time.time() - t0:.1f}s")
    return np.concatenate(feats), np.concatenate(labels)


def build_dataset_batched(lps, seeds, precision="fp64", eps=1e-6, eps_abs=1e-6):
    """The same data, produced by the batch engine: every LP solved, its
    features read and its plain push run in one batch."""
    b = pdhg.Batch(lps, precision=precision, record_history=1, eps_rel=eps, eps_abs=eps_abs, use_graph=USE_GRAPH)
    res = b.solve()
    feats = b.features(seeds)
    zs = []
    for i in range(len(lps)):
        zs.append(b.get_solution(i)[2])
    b.corner_push(seeds)
    fs, ys = [], []
    for i, lp in enumerate(lps):
        if res[i].status != pdhg.PDHG_OPTIMAL:
            continue
        x = b.get_solution(i)[0]
        at_bound = (x - lp.l <= 1e-6) | (lp.u - x <= 1e-6)
        mask = (np.abs(zs[i]) <= eps_abs) & (np.isfinite(lp.l) | np.isfinite(lp.u))
        fs.append(feats[i][mask])
        ys.append(at_bound[mask].astype(np.float32))
    b.destroy()
    return np.concatenate(fs), np.concatenate(ys)


def batch_time_to_corner(lps, seeds, precision="fp64", net=None, theta=0.9, eps=1e-6):
    """create + solve + push of the whole batch, plain or learned."""
    t0 = time.perf_counter()
    b = pdhg.Batch(lps, precision=precision, record_history=1 if net is not None else 0, eps_rel=eps,
                   use_graph=USE_GRAPH)
    res = b.solve()
    push = b.corner_push(seeds) if net is None else b.corner_push_learned(net, theta, seeds)
    dt = time.perf_counter() - t0
    rep = b.report()
    b.destroy()
    ok = [i for i, r in enumerate(res) if r.status == pdhg.PDHG_OPTIMAL]
    return {"seconds": dt, "push_lockstep": rep.push_lockstep_iters, "solve_lockstep": rep.solve_lockstep_iters,
            "push_lp_iters": sum(push[i].iters for i in ok), "push_done": sum(push[i].status == pdhg.PDHG_PUSH_DONE
                                                                              for i in ok),
            "est_primal_after": sum(push[i].after.est_primal for i in ok),
            "candidates_after": sum(push[i].after.candidates for i in ok),
            "off_bound_after": sum(push[i].after.p_off for i in ok),
            "learned_fix": sum(push[i].n_learned_fix for i in ok),
            "learned_undo": sum(push[i].n_learned_undo for i in ok), "optimal": len(ok)}


THETAS = (0.5, 0.6, 0.7, 0.8, 0.85, 0.9, 0.95, 0.98, 0.99, 0.995, 0.999)


def theta_table(net, f, y):
    """(theta, precision of the fixes, fraction of free columns fixed) per theta."""
    p = 1.0 / (1.0 + np.exp(-net.forward(f).astype(np.float64)))
    rows = []
    for th in THETAS:
        sel = p >= th
        k = int(sel.sum())
        rows.append((th, float(np.mean(y[sel] > 0.5)) if k else float("nan"), k / max(1, len(y))))
    return rows


def choose_theta(rows, min_precision=0.95):
    """Smallest theta whose fixes are right at least min_precision of the time."""
    for th, prec, frac in rows:
        if frac > 0 and prec >= min_precision:
            return th
    return None


def time_to_corner(lp, seed, precision="fp64", net=None, theta=0.9, eps=1e-6):
    """create + solve + push wall time, and the corner statistics."""
    t0 = time.perf_counter()
    s = pdhg.Solver(lp, precision=precision, record_history=1 if net is not None else 0, eps_rel=eps,
                    use_graph=USE_GRAPH)
    r = s.solve()
    if r.status != pdhg.PDHG_OPTIMAL:
        return None
    p = s.corner_push(seed) if net is None else s.corner_push_learned(net, theta, seed)
    dt = time.perf_counter() - t0
    return {"seconds": dt, "solve_iters": r.iters, "push_iters": p.iters, "push_status": pdhg.STATUS[p.status],
            "est_primal_after": p.after.est_primal, "candidates_after": p.after.candidates,
            "off_bound_after": p.after.p_off, "est_primal_before": p.before.est_primal,
            "rel_p_after": p.after.rel_p, "learned_fix": p.n_learned_fix, "learned_undo": p.n_learned_undo}


def save_predictor(path, net, theta, meta):
    """The trained network's float32 parameters, its theta and how it was
    made, as JSON."""
    out = dict(meta)
    out.update({"theta": theta, "n_params": pdhg.MLP_NPARAMS,
                "params": [float(v) for v in np.asarray(net.get_params(), dtype=np.float32)]})
    with open(path, "w") as fh:
        json.dump(out, fh)


def load_predictor(path):
    """(network, theta, metadata) from a file written by save_predictor."""
    with open(path) as fh:
        d = json.load(fh)
    if d.get("n_params") != pdhg.MLP_NPARAMS or len(d.get("params", [])) != pdhg.MLP_NPARAMS:
        raise ValueError(f"{path}: not a predictor of {pdhg.MLP_NPARAMS} parameters")
    net = pdhg.Mlp(seed=0)
    net.set_params(np.asarray(d.pop("params"), dtype=np.float32))
    return net, d["theta"], d


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--val", type=int, default=40)
    ap.add_argument("--eval", type=int, default=20)
    ap.add_argument("--m-lo", type=int, default=300)
    ap.add_argument("--m-hi", type=int, default=3000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--min-precision", type=float, default=0.95)
    ap.add_argument("--mcf", default="", help="nodes,arcs,commodities of a multicommodity evaluation LP")
    ap.add_argument("--mcf-precision", default="fp32", choices=["fp64", "fp32"])
    ap.add_argument("--mcf-seeds", type=int, default=1)
    ap.add_argument("--no-graph", action="store_true", help="launch every cycle eagerly (profiler runs)")
    ap.add_argument("--theta-by-time", action="store_true",
                    help="with --batched: choose theta by the validation batch's measured time to the corner")
    ap.add_argument("--batched", action="store_true",
                    help="training data from the batch engine, and learned+batched vs plain batched push")
    ap.add_argument("--save", default="", help="write the trained network and its theta to this JSON file")
    args = ap.parse_args(argv)
    global USE_GRAPH
    USE_GRAPH = 0 if args.no_graph else 1
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
    rng_range = (args.m_lo, args.m_hi)
    tr = [lpgen.config3_instance(i, base_seed=40000, m_range=rng_range) for i in range(args.train)]
    va = [lpgen.config3_instance(i, base_seed=42000, m_range=rng_range) for i in range(args.val)]
    ev = [lpgen.config3_instance(i, base_seed=43000, m_range=rng_range) for i in range(args.eval)]
    t_data = time.time()
    if args.batched:
        f, y = build_dataset_batched(tr, [17 + i for i in range(len(tr))], args.precision)
        fv, yv = build_dataset_batched(va, [91 + i for i in range(len(va))], args.precision)
    else:
        f, y = build_dataset(tr, [17 + i for i in range(len(tr))], args.precision, log)
        fv, yv = build_dataset(va, [91 + i for i in range(len(va))], args.precision, log)
    log(f"[learned] data generation {time.time() - t_data:.1f}s ({'batch engine' if args.batched else 'one LP at a time'})")
    log(f"[learned] train {f.shape[0]} free columns ({y.mean():.3f} end at a bound), val {fv.shape[0]}")
    net = pdhg.Mlp(seed=7)
    rep = net.train(f, y, epochs=args.epochs, batch=4096, lr=1e-3, seed=3)
    log(f"[learned] training: loss {rep.loss_first:.4f} -> {rep.loss_last:.4f}, {rep.seconds:.2f}s, "
        f"{rep.samples_per_s:.3e} samples/s, pos_weight {rep.pos_weight:.3f}")
    rows = theta_table(net, fv, yv)
    for th, prec, frac in rows:
        log(f"[learned] validation theta {th}: precision {prec:.4f}, fixes {frac:.4f} of free columns")
    theta = choose_theta(rows, args.min_precision)
    if args.save:
        cmd = "python -m paper_2511_13894_amd.learned " + " ".join(argv if argv is not None else sys.argv[1:])
        save_predictor(args.save, net, theta,
                       {"command": cmd, "train_columns": int(f.shape[0]), "val_columns": int(fv.shape[0]),
                        "train_loss": [rep.loss_first, rep.loss_last], "theta_table": rows,
                        "min_precision": args.min_precision,
                        "train_lps": [args.train, "base seed 40000", [args.m_lo, args.m_hi]],
                        "val_lps": [args.val, "base seed 42000", [args.m_lo, args.m_hi]]})
        log(f"[learned] saved the network and theta {theta} to {args.save}")
    if args.batched and args.theta_by_time:
        sd = [91 + i for i in range(len(va))]
        base = batch_time_to_corner(va, sd, args.precision)
        best = (base["seconds"], None)
        for th in (0.9, 0.95, 0.98, 0.99, 0.995):
            r = batch_time_to_corner(va, sd, args.precision, net, th)
            log(f"[learned] validation batch, theta {th}: {r['seconds']:.3f}s (plain {base['seconds']:.3f}s), push "
                f"lockstep {r['push_lockstep']} (plain {base['push_lockstep']})")
            if r["seconds"] < best[0]:
                best = (r["seconds"], th)
        theta = best[1]
        log(f"[learned] theta by validation time: {theta} (None: the plain push was fastest)")
    out = {"train_columns": int(f.shape[0]), "val_columns": int(fv.shape[0]), "theta": theta,
           "theta_table": rows, "train_loss": [rep.loss_first, rep.loss_last], "train_seconds": rep.seconds,
           "train_samples_per_s": rep.samples_per_s, "eval": []}
    if theta is None or (not ev and not args.mcf):
        print(json.dumps(out))
        return
    if args.batched and ev:
        sd = [500 + i for i in range(len(ev))]
        plain = batch_time_to_corner(ev, sd, args.precision)
        lrn = batch_time_to_corner(ev, sd, args.precision, net, theta)
        out["batched_eval"] = {"lps": len(ev), "plain": plain, "learned": lrn}
        log(f"[learned] batched: {len(ev)} LPs, time to corner {plain['seconds']:.3f}s -> {lrn['seconds']:.3f}s, push "
            f"lockstep {plain['push_lockstep']} -> {lrn['push_lockstep']}, push LP-iterations {plain['push_lp_iters']} "
            f"-> {lrn['push_lp_iters']}, primal push estimate {plain['est_primal_after']} -> "
            f"{lrn['est_primal_after']}, candidates {plain['candidates_after']} -> {lrn['candidates_after']}, "
            f"learned fixes {lrn['learned_fix']} (undone {lrn['learned_undo']})")
    cases = [(lambda lp=lp: lp, 500 + i, args.precision) for i, lp in enumerate(ev)]
    if args.mcf:
        nn, na, nk = (int(v) for v in args.mcf.split(","))
        for k in range(args.mcf_seeds):
            cases.append((lambda k=k: lpgen.multicommodity(nn, na, nk, seed=4100 + k), 4100 + k, args.mcf_precision))
    for make, sd, prec in cases:
        lp = make()
        plain = time_to_corner(lp, sd, prec)
        learned = time_to_corner(lp, sd, prec, net, theta)
        out["eval"].append({"lp": lp.name, "m": lp.m, "n": lp.n, "precision": prec, "plain": plain,
                            "learned": learned})
        if plain and learned:
            log(f"[learned] {lp.name} ({prec}): time {plain['seconds']:.3f}s -> {learned['seconds']:.3f}s, push "
                f"iters {plain['push_iters']} -> {learned['push_iters']}, est_primal {plain['est_primal_after']} -> "
                f"{learned['est_primal_after']}, candidates {plain['candidates_after']} -> "
                f"{learned['candidates_after']}, learned fixes {learned['learned_fix']} (undone "
                f"{learned['learned_undo']})")
        else:
            log(f"[learned] {lp.name} ({prec}): solve did not reach optimality")
    both = [e for e in out["eval"] if e["plain"] and e["learned"]]
    for tag, sel in (("batched family", [e for e in both if e["lp"].startswith("c3")]),
                     ("multicommodity", [e for e in both if e["lp"].startswith("mcf")])):
        if not sel:
            continue
        ratio = np.exp(np.mean([np.log(e["learned"]["seconds"] / e["plain"]["seconds"]) for e in sel]))
        pi = sum(e["plain"]["push_iters"] for e in sel), sum(e["learned"]["push_iters"] for e in sel)
        ep = sum(e["plain"]["est_primal_after"] for e in sel), sum(e["learned"]["est_primal_after"] for e in sel)
        out[f"summary_{tag.split()[0]}"] = {"lps": len(sel), "geomean_time_ratio": ratio, "push_iters": pi,
                                             "est_primal_after": ep}
        log(f"[learned] {tag}: {len(sel)} LPs, time-to-corner learned/plain geomean {ratio:.3f}, push iterations "
            f"{pi[0]} -> {pi[1]}, primal push estimate {ep[0]} -> {ep[1]}")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
