"""Train and evaluate the learned large-kernel correction on engine-generated pairs.

python -m paper_2512_18863_amd.train_learned --train 2000 --steps 3000 --eval 100 \
    --out paper_2512_18863_amd/data/learned_c4.npz --report <json>

Training pairs: randomised 128^3 pelvis plans p in [0, train) (seed 4000 + p,
60-180 control points, jaws 20-50 mm), input = the 9 x 9 FP32 dose and the
density, target = the 61 x 61 FP32 dose, both from the HIP engine.  Held-out
plans p in [2000, 2000 + eval): the learned dose (with its fallback) is compared
with the plain 61 x 61 FP32 dose (1 %/1 mm global gamma, 10 % threshold; max
error).  The trained parameters (optionally with the Adam state) are written
with numpy (no pickles).  The learning rate follows a cosine decay over the
step budget or the time budget, whichever runs out first.  `--load` skips
training and evaluates stored parameters.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import engine as E
from . import gamma, inputs, learned


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def make_pair(p):
    case = inputs.config_c4_plan(p, n_taps=61)
    es = E.DoseEngine(case, n_taps=9)
    el = E.DoseEngine(case, n_taps=61)
    lv, jw, mu = _t(case.leaves), _t(case.jaws), _t(case.mu)
    ds = es.forward(lv, jw, mu).reshape(-1).clone()
    dl = el.forward(lv, jw, mu).reshape(-1).clone()
    mask = (dl >= 0.05 * dl.max()).float()
    return (ds, dl, es.rho.reshape(-1).clone(), mask, float(mask.sum())), case


def evaluate(net, plans, log):
    rows = []
    for p in plans:
        case = inputs.config_c4_plan(p, n_taps=61)
        lv, jw, mu = _t(case.leaves), _t(case.jaws), _t(case.mu)
        ld = learned.LearnedDose(net, case)
        plain = E.DoseEngine(case, n_taps=61).forward(lv, jw, mu).cpu().numpy()
        raw = learned.LearnedDose(net, case, mode="never").forward(lv, jw, mu).cpu().numpy()
        out = ld.forward(lv, jw, mu).cpu().numpy()
        err_raw = float(np.abs(raw - plain).max() / plain.max())
        err = float(np.abs(out - plain).max() / plain.max())
        g_raw = gamma.pass_rate(plain, raw, case.spacing, 1.0, 1.0)
        g = 1.0 if ld.fell_back else g_raw
        rows.append({"plan": p, "n_cp": case.n_cp, "fallback": ld.fell_back, "gamma_raw": g_raw, "gamma": g,
                     "max_err_raw": err_raw, "max_err": err})
        log("[eval] plan %d: fallback %s, gamma raw %.4f, used %.4f, max err raw %.3e" %
            (p, ld.fell_back, 100 * g_raw, 100 * g, err_raw))
    return rows


def summarize(rows, head):
    g = np.array([r["gamma"] for r in rows])
    return dict(head, **{
        "eval_plans": len(rows), "fallback_rate": float(np.mean([r["fallback"] for r in rows])),
        "gamma_mean": float(g.mean()), "gamma_min": float(g.min()),
        "gamma_raw_mean": float(np.mean([r["gamma_raw"] for r in rows])),
        "gamma_raw_min": float(np.min([r["gamma_raw"] for r in rows])),
        "plans_raw_gamma_at_least_99_5": int(sum(r["gamma_raw"] >= 0.995 for r in rows)),
        "max_err_raw_mean": float(np.mean([r["max_err_raw"] for r in rows])), "rows": rows})


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--eval", type=int, default=100)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--budget", type=float, default=600.0, help="seconds for pair generation + training")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "data", "learned_c4.npz"))
    ap.add_argument("--report", default=None)
    ap.add_argument("--save-optimizer", action="store_true", help="also store the Adam moments (to resume training)")
    ap.add_argument("--load", default=None, help="evaluate these stored parameters instead of training")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    if args.load:
        net = learned.Net3D.from_file(args.load, (128, 128, 128))
        rows = evaluate(net, range(2000, 2000 + args.eval), log)
        report = summarize(rows, {"weights": args.load})
        if args.report:
            with open(args.report, "w") as fh:
                json.dump(report, fh, indent=1)
        log(json.dumps({k: v for k, v in report.items() if k != "rows"}))
        return 0

    t0 = time.perf_counter()
    pairs = []
    for p in range(args.train):
        pr, _ = make_pair(p)
        pairs.append(pr)
        if (p + 1) % 50 == 0:
            log("[pairs] %d generated (%.0f s)" % (p + 1, time.perf_counter() - t0))
        if time.perf_counter() - t0 > 0.5 * args.budget:
            log("[pairs] time budget reached after %d plans" % (p + 1))
            break
    t_pairs = time.perf_counter() - t0
    n_pairs = len(pairs)
    net = learned.Net3D((128, 128, 128), seed=0)
    t1 = time.perf_counter()
    steps_done = 0
    hist = []
    chunk = 100
    train_budget = max(1.0, args.budget - t_pairs)
    while steps_done < args.steps and time.perf_counter() - t0 < args.budget:
        frac = max(steps_done / args.steps, (time.perf_counter() - t1) / train_budget)
        lr = args.lr * max(0.02, 0.5 * (1.0 + math.cos(math.pi * min(1.0, frac))))
        n = min(chunk, args.steps - steps_done)
        order = [pairs[(steps_done + i) % len(pairs)] for i in range(n)]
        h = learned.train(net, order, n, lr=lr, log_every=n, log=lambda m: None)
        steps_done += n
        hist.append((steps_done, h[-1][1]))
        log("[train] step %d lr %.2e loss %.4e (%.0f s)" % (steps_done, lr, h[-1][1], time.perf_counter() - t1))
    t_train = time.perf_counter() - t1
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    st = net.state()
    extra = dict(m=st["m"], v=st["v"]) if args.save_optimizer else {}
    np.savez(args.out, params=st["params"], t=np.array(st["t"]), layers=np.array([l[0] for l in learned.LAYERS]),
             **extra)
    log("[train] saved %s" % args.out)
    del pairs
    torch.cuda.empty_cache()
    rows = evaluate(net, range(2000, 2000 + args.eval), log)
    report = summarize(rows, {"train_plans": n_pairs, "steps": steps_done, "pair_seconds": t_pairs,
                              "train_seconds": t_train, "loss_history": hist})
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)
    log(json.dumps({k: v for k, v in report.items() if k != "rows"}))


if __name__ == "__main__":
    sys.exit(main())
