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

`--finetune-error-head <npz> --quantile q` starts from stored parameters and
trains only the error head, on the pinball loss of the q-quantile of the local
error |prediction - target| (the prediction, and so the learned dose, is left as
it is); the fallback then compares the largest such upper estimate with 1 % of
the largest dose.  The report also runs the held-out plan 2000 on anatomies no
training phantom resembles (`inputs.config_c4_ood`), where the estimate should
make the correction fall back.  `--calibrate n` then scales the error head on a
calibration split of held-out plans p in [2100, 2100 + n) (disjoint from the
evaluation plans) so that its largest estimate reaches the largest error of the
learned dose on a fraction `--calibrate-quantile` of them.
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


def evaluate_case(net, case):
    """Learned dose (with its fallback) against the plain 61 x 61 FP32 dose."""
    lv, jw, mu = _t(case.leaves), _t(case.jaws), _t(case.mu)
    ld = learned.LearnedDose(net, case)
    plain = E.DoseEngine(case, n_taps=61).forward(lv, jw, mu).cpu().numpy()
    raw = learned.LearnedDose(net, case, mode="never").forward(lv, jw, mu).cpu().numpy()
    out = ld.forward(lv, jw, mu).cpu().numpy()
    st = net.stats.cpu().numpy()
    err_raw = float(np.abs(raw - plain).max() / plain.max())
    err = float(np.abs(out - plain).max() / plain.max())
    g_raw = gamma.pass_rate(plain, raw, case.spacing, 1.0, 1.0)
    g = 1.0 if ld.fell_back else g_raw
    return {"n_cp": case.n_cp, "fallback": ld.fell_back, "estimate": float(st[1] / st[0]), "gamma_raw": g_raw,
            "gamma": g, "max_err_raw": err_raw, "max_err": err}


def calibrate(net, plans, q, log):
    """Ratio k of the largest error to the largest estimate whose q-quantile over
    the calibration plans scales the error head."""
    ratios = []
    for p in plans:
        case = inputs.config_c4_plan(p, n_taps=61)
        lv, jw, mu = _t(case.leaves), _t(case.jaws), _t(case.mu)
        raw = learned.LearnedDose(net, case, mode="never").forward(lv, jw, mu)
        st = net.stats.cpu().numpy()
        plain = E.DoseEngine(case, n_taps=61).forward(lv, jw, mu)
        err = float((raw - plain).abs().max() / plain.max())
        est = float(st[1] / st[0])
        if not est > 0.0:
            raise RuntimeError("plan %d: non-positive error estimate %g" % (p, est))
        ratios.append(err / est)
        log("[calibrate] plan %d: max err %.3e estimate %.3e ratio %.3f" % (p, err, est, ratios[-1]))
        torch.cuda.empty_cache()
    k = float(np.quantile(ratios, q))
    net.scale_error_head(k)
    log("[calibrate] error head scaled by %.4f (%.2f-quantile of %d ratios)" % (k, q, len(ratios)))
    return k, ratios


def evaluate(net, plans, log):
    rows = []
    for p in plans:
        r = dict({"plan": p}, **evaluate_case(net, inputs.config_c4_plan(p, n_taps=61)))
        rows.append(r)
        log("[eval] plan %d: fallback %s, estimate %.3e, gamma raw %.4f, used %.4f, max err raw %.3e" %
            (p, r["fallback"], r["estimate"], 100 * r["gamma_raw"], 100 * r["gamma"], r["max_err_raw"]))
    return rows


def evaluate_ood(net, log, plan=2000):
    rows = []
    for kind in inputs.C4_OOD_KINDS:
        r = dict({"plan": plan, "anatomy": kind}, **evaluate_case(net, inputs.config_c4_ood(kind, plan)))
        rows.append(r)
        log("[ood] plan %d %s: fallback %s, estimate %.3e, gamma raw %.4f, max err raw %.3e" %
            (plan, kind, r["fallback"], r["estimate"], 100 * r["gamma_raw"], r["max_err_raw"]))
    return rows


def summarize(rows, head, ood=None):
    g = np.array([r["gamma"] for r in rows])
    est = np.array([r["estimate"] for r in rows])
    err = np.array([r["max_err_raw"] for r in rows])
    return dict(head, **{
        "estimate_max": float(est.max()), "estimate_mean": float(est.mean()),
        "estimate_below_error": int(np.sum(est < err)), "ood": ood or [],
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
    ap.add_argument("--finetune-error-head", default=None, metavar="NPZ",
                    help="start from these parameters and train the error head only")
    ap.add_argument("--quantile", type=float, default=0.0,
                    help="train the error head on this quantile of |error| (pinball loss); 0: squared loss")
    ap.add_argument("--lam", type=float, default=1.0, help="weight of the error head's loss")
    ap.add_argument("--calibrate", type=int, default=0, help="calibration plans 2100.. for the error head's scale")
    ap.add_argument("--calibrate-quantile", type=float, default=0.9)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    if args.load:
        net = learned.Net3D.from_file(args.load, (128, 128, 128))
        rows = evaluate(net, range(2000, 2000 + args.eval), log)
        report = summarize(rows, {"weights": args.load}, evaluate_ood(net, log))
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
    head_only = args.finetune_error_head is not None
    if head_only:
        net = learned.Net3D.from_file(args.finetune_error_head, (128, 128, 128))
        net.m.zero_()
        net.v.zero_()
        net.t = 0
    else:
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
        h = learned.train(net, order, n, lr=lr, log_every=n, log=lambda m: None, lam=args.lam,
                          quantile=args.quantile, error_head_only=head_only)
        steps_done += n
        hist.append((steps_done, h[-1][1]))
        log("[train] step %d lr %.2e loss %.4e (%.0f s)" % (steps_done, lr, h[-1][1], time.perf_counter() - t1))
    t_train = time.perf_counter() - t1
    del pairs
    torch.cuda.empty_cache()
    calib = {}
    if args.calibrate > 0:
        k, ratios = calibrate(net, range(2100, 2100 + args.calibrate), args.calibrate_quantile, log)
        calib = {"calibration_plans": args.calibrate, "calibration_quantile": args.calibrate_quantile,
                 "error_head_scale": k, "calibration_ratios": ratios}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    st = net.state()
    extra = dict(m=st["m"], v=st["v"]) if args.save_optimizer else {}
    np.savez(args.out, params=st["params"], t=np.array(st["t"]), layers=np.array([l[0] for l in learned.LAYERS]),
             **extra)
    log("[train] saved %s" % args.out)
    rows = evaluate(net, range(2000, 2000 + args.eval), log)
    report = summarize(rows, {"train_plans": n_pairs, "steps": steps_done, "pair_seconds": t_pairs,
                              "train_seconds": t_train, "loss_history": hist, "quantile": args.quantile,
                              "error_head_only": head_only, "init": args.finetune_error_head, **calib},
                       evaluate_ood(net, log))
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(report, fh, indent=1)
    log(json.dumps({k: v for k, v in report.items() if k != "rows"}))


if __name__ == "__main__":
    sys.exit(main())
