"""Learned warm start of the corner push: data, training, evaluation.

The training data are the method's own trajectories: every LP is solved with
restart history recorded, its 12 features are read from the device, the plain
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


def solve_and_label(lp, seed, precision="fp64", eps=1e-6, eps_abs=1e-6):
    """(features, labels, free-column mask, solve result, push result) of one LP, or None."""
    s = pdhg.Solver(lp, precision=precision, record_history=1, eps_rel=eps, eps_abs=eps_abs)
    r = s.solve()
    if r.status != pdhg.PDHG_OPTIMAL:
        return None
    _, _, z = s.get_solution()
    f = s.features()
    p = s.corner_push(seed)
    x, _, _ = s.get_solution()
    at_bound = (x - lp.l <= 1e-6) | (lp.u - x <= 1e-6)
    free = np.abs(z) <= eps_abs
    return f, at_bound.astype(np.float32), free, r, p


def build_dataset(lps, seeds, precision="fp64", log=None):
    feats, labels, frees = [], [], []
    t0 = time.time()
    for i, (lp, sd) in enumerate(zip(lps, seeds)):
        out = solve_and_label(lp, sd, precision)
        if out is None:
            continue
        f, y, free, _, _ = out
        feats.append(f)
        labels.append(y)
        frees.append(free)
        if log and (i + 1) % 20 == 0:
            log(f"[learned] data {i + 1}/{len(lps)} LPs, {sum(a.shape[0] for a in feats)} columns, "
                f"{time.time() - t0:.1f}s")
    return np.concatenate(feats), np.concatenate(labels), np.concatenate(frees)


def choose_theta(net, f, y, free, min_precision=0.98):
    """Smallest theta whose fixes among free columns are right >= min_precision."""
    z = net.forward(f)
    p = 1.0 / (1.0 + np.exp(-z.astype(np.float64)))
    best = None
    for th in (0.5, 0.6, 0.7, 0.8, 0.9, 0.95, 0.98, 0.99, 0.995):
        sel = free & (p >= th)
        if sel.sum() == 0:
            continue
        prec = float(np.mean(y[sel] > 0.5))
        if prec >= min_precision:
            best = (th, prec, int(sel.sum()), int(free.sum()))
            break
    return best


def time_to_corner(lp, seed, precision="fp64", net=None, theta=0.9, eps=1e-6):
    """create + solve + push wall time, and the corner statistics."""
    t0 = time.perf_counter()
    s = pdhg.Solver(lp, precision=precision, record_history=1 if net is not None else 0, eps_rel=eps)
    r = s.solve()
    if r.status != pdhg.PDHG_OPTIMAL:
        return None
    p = s.corner_push(seed) if net is None else s.corner_push_learned(net, theta, seed)
    dt = time.perf_counter() - t0
    return {"seconds": dt, "solve_iters": r.iters, "push_iters": p.iters, "push_status": pdhg.STATUS[p.status],
            "est_primal_after": p.after.est_primal, "candidates_after": p.after.candidates,
            "off_bound_after": p.after.p_off, "est_primal_before": p.before.est_primal,
            "rel_p_after": p.after.rel_p, "learned_fix": p.n_learned_fix, "learned_undo": p.n_learned_undo}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--val", type=int, default=40)
    ap.add_argument("--eval", type=int, default=20)
    ap.add_argument("--m-lo", type=int, default=300)
    ap.add_argument("--m-hi", type=int, default=3000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--mcf", default="", help="nodes,arcs,commodities of a multicommodity evaluation LP")
    args = ap.parse_args(argv)
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
    rng_range = (args.m_lo, args.m_hi)
    tr = [lpgen.config3_instance(i, base_seed=40000, m_range=rng_range) for i in range(args.train)]
    va = [lpgen.config3_instance(i, base_seed=42000, m_range=rng_range) for i in range(args.val)]
    ev = [lpgen.config3_instance(i, base_seed=43000, m_range=rng_range) for i in range(args.eval)]
    f, y, free = build_dataset(tr, [17 + i for i in range(len(tr))], args.precision, log)
    fv, yv, freev = build_dataset(va, [91 + i for i in range(len(va))], args.precision, log)
    log(f"[learned] train {f.shape[0]} columns ({y.mean():.3f} positive), val {fv.shape[0]}")
    net = pdhg.Mlp(seed=7)
    rep = net.train(f, y, epochs=args.epochs, batch=4096, lr=1e-3, seed=3)
    log(f"[learned] training: loss {rep.loss_first:.4f} -> {rep.loss_last:.4f}, {rep.seconds:.2f}s, "
        f"{rep.samples_per_s:.3e} samples/s, pos_weight {rep.pos_weight:.3f}")
    th = choose_theta(net, fv, yv, freev)
    theta = th[0] if th else 0.99
    log(f"[learned] theta {theta} (validation precision on free columns: {th})")
    out = {"train_columns": int(f.shape[0]), "val_columns": int(fv.shape[0]), "theta": theta,
           "theta_detail": th, "train_loss": [rep.loss_first, rep.loss_last], "train_seconds": rep.seconds,
           "train_samples_per_s": rep.samples_per_s, "eval": []}
    cases = [(lp, 500 + i) for i, lp in enumerate(ev)]
    if args.mcf:
        nn, na, nk = (int(v) for v in args.mcf.split(","))
        cases.append((lpgen.multicommodity(nn, na, nk, seed=4100), 4100))
    for lp, sd in cases:
        plain = time_to_corner(lp, sd, args.precision)
        learned = time_to_corner(lp, sd, args.precision, net, theta)
        out["eval"].append({"lp": lp.name, "m": lp.m, "n": lp.n, "plain": plain, "learned": learned})
        if plain and learned:
            log(f"[learned] {lp.name}: time {plain['seconds']:.3f}s -> {learned['seconds']:.3f}s, push iters "
                f"{plain['push_iters']} -> {learned['push_iters']}, est_primal {plain['est_primal_after']} -> "
                f"{learned['est_primal_after']}, learned fixes {learned['learned_fix']} (undone "
                f"{learned['learned_undo']})")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
