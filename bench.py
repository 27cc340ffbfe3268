#!/usr/bin/env python3
"""Throughput of the dose path: forward + backward control points per second.

Workload (the 128^3 benchmark plan): a randomised synthetic pelvis CT of 128^3
voxels at 3 mm, a two-arc VMAT plan of 180 control points, 60 leaf pairs of
5 mm, jaws +-40 mm, 61 x 61 lateral kernel; one step = the dose forward plus the
backward of L = sum w D to leaves, jaws and MU (all 180 control points).
Inputs are resident in HBM before the timed region.  The plain FP32 path gives
`value`; the BF16 convolution variant is timed the same way and its dose is
compared with the FP32 dose (max error, 1 %/1 mm gamma).  Per-kernel times come
from HIP events recorded by the library around every launch in the timed
region.  The FP64 CPU oracle is timed on a bounded sample of the same plan.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
PEAK_FP32_MFMA_TFLOPS = 157.3     # MI355X dense FP32 matrix peak
PEAK_BF16_MFMA_TFLOPS = 2500.0    # MI355X dense BF16 matrix peak
PEAK_HBM_GBS = 8000.0


# sources that make up each kernel whose counters are recorded in profiles/traffic.json
KERNEL_SOURCES = {
    "conv_mfma_f32": ["conv_mfma.hip", "conv_common.hpp", "taps.hpp", "device_math.hpp", "pdrt_internal.hpp"],
}


def kernel_source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2512_18863_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they were
    taken on the kernel's current sources; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    e = rec.get(workload, {}).get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash(kernel):
        return None
    return e.get("bytes_per_launch")


# the FP32 convolution's two kernels (forward on the aperture's inputs, adjoint on its outputs)
KERNEL_SYMBOLS = {"conv_mfma_f32": ("k_conv_mfma_f32<", "k_conv_mfma_f32_adj<")}
COPY_BYTES = 1 << 30   # the counter run's calibration copy


def traffic_from_counters(fetch_csv, write_csv, workload="c4bench_fp32"):
    """Write profiles/traffic.json from two rocprofv3 --pmc runs of `bench.py
    --counter-run` (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).  Each counter is
    scaled by what it reads for the run's 1 GiB copy, so that the copy counts as
    1 GiB read and 1 GiB written."""
    import csv
    import re

    def load(path):
        rows = list(csv.DictReader(open(path)))
        return [(r["Kernel_Name"], float(r["Counter_Value"])) for r in rows]

    fetch, write = load(fetch_csv), load(write_csv)
    f_copy = max(v for n, v in fetch if "copyBuffer" in n)
    w_copy = max(v for n, v in write if "copyBuffer" in n)
    kf, kw = COPY_BYTES / (f_copy * 1024.0), COPY_BYTES / (w_copy * 1024.0)

    def short(name):
        m = re.search(r"pdrt::(k_\w+(<[^(]*>)?)", name)
        return m.group(1).replace(" ", "") if m else None

    per = {}
    for (n, v), (n2, v2) in zip(fetch, write):
        if n != n2:
            raise ValueError("the two counter runs dispatched different kernels")
        k = short(n)
        if k:
            e = per.setdefault(k, [0, 0.0, 0.0])
            e[0] += 1
            e[1] += v * 1024.0 * kf
            e[2] += v2 * 1024.0 * kw
    rec = {"calibration": {"copy_bytes": COPY_BYTES, "fetch_kib_for_copy": f_copy, "write_kib_for_copy": w_copy,
                           "fetch_factor": kf, "write_factor": kw},
           "commands": ["rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir> -o fetch -- python3 bench.py --counter-run",
                        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir> -o write -- python3 bench.py --counter-run"],
           workload: {}, "all_kernels_" + workload: {}}
    for k, (cnt, fb, wb) in per.items():
        rec["all_kernels_" + workload][k] = {"dispatches": cnt, "fetch_bytes_per_launch": fb / cnt,
                                             "write_bytes_per_launch": wb / cnt}
    for name, syms in KERNEL_SYMBOLS.items():
        hits = [(n, v, v2) for (n, v), (_, v2) in zip(fetch, write) if any(sy in n for sy in syms)]
        if hits:
            fb = sum(h[1] for h in hits) * 1024.0 * kf / len(hits)
            wb = sum(h[2] for h in hits) * 1024.0 * kw / len(hits)
            rec[workload][name] = {"bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
                                   "dispatches": len(hits), "source_hash": kernel_source_hash(name)}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("wrote", path)


def aperture_pixels(jaws, lat, Nu, Nv):
    """Per control point, the fan pixels that overlap the jaw opening: the fluence
    (hence the primary P = F G) is zero elsewhere, and the parameter gradients read
    the adjoint only there.  These are the nodes the lateral convolution has to
    process, in either direction: 2 n^2 flops per aperture node and plane."""
    import numpy as np
    def count(a, b, N):
        c = (np.arange(N) - (N - 1) / 2.0) * lat
        return int(((c + lat / 2 > a) & (c - lat / 2 < b)).sum())
    return np.array([count(j[0], j[1], Nu) * count(j[2], j[3], Nv) for j in np.asarray(jaws)])


def hbm_table(kernels, steps, n_cp, nodes, ap_nodes, plane, vox):
    """Achieved bandwidth of the memory-bound kernels from their algorithmic bytes
    (each byte the kernel must move once): nodes = beam-frame nodes of the plan,
    ap_nodes = those on the control points' apertures (the only rays the march
    and its adjoint process), plane = fluence pixels per control point, vox = CT
    voxels."""
    b = {
        "march": 4 * ap_nodes + 4 * n_cp * plane + 4 * vox,           # write P on the aperture; read F, rho
        "gather": 4 * nodes + 2 * 4 * vox,                            # read Dfan; write dose + compensation
        "backproject_adj": 4 * nodes + 4 * vox,                       # write G; read g
        "march_adj": 4 * ap_nodes + 4 * n_cp * plane + 4 * vox,       # read H on the aperture; write A; read rho
    }
    out = {}
    for k, by in b.items():
        if k not in kernels:
            continue
        launches, total = kernels[k]
        avg = total / max(launches, 1) / 1e3
        gbs = by / avg / 1e9 if avg > 0 else 0.0
        out[k] = {"algorithmic_bytes": by, "avg_launch_ms": round(avg * 1e3, 4), "achieved_GBs": round(gbs, 1),
                  "frac": round(gbs / PEAK_HBM_GBS, 4)}
    return out


def run_gpu(case, conv, steps, warmup, w, cache=None):
    """Forward + backward timed over `steps`; with cache = "fp32" / "bf16" the plan's
    geometry cache is built first (outside the timed region: once per plan)."""
    import torch
    from paper_2512_18863_amd import engine as E
    eng = E.DoseEngine(case, conv=conv)
    dev = eng.device
    if cache:
        torch.cuda.synchronize()
        tb = time.perf_counter()
        eng.cache_bytes = eng.build_cache(cache)
        torch.cuda.synchronize()
        eng.cache_build_ms = (time.perf_counter() - tb) * 1e3
    lv = torch.tensor(case.leaves, dtype=torch.float32, device=dev)
    jw = torch.tensor(case.jaws, dtype=torch.float32, device=dev)
    mu = torch.tensor(case.mu, dtype=torch.float32, device=dev)
    g = torch.tensor(w, dtype=torch.float32, device=dev)
    dose = torch.empty(eng.vol_shape, dtype=torch.float32, device=dev)

    def step():
        eng.forward(lv, jw, mu, out=dose)
        return eng.backward(lv, jw, mu, g)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    E.profile_begin(64 * steps + 64)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    kernels = E.profile_end()
    ms = t0.elapsed_time(t1) / steps
    fwd_dose = eng.forward(lv, jw, mu).cpu().numpy()
    torch.cuda.synchronize()
    return ms, kernels, fwd_dose, eng


LEARNED_WEIGHTS = os.path.join(ROOT, "paper_2512_18863_amd", "data", "learned_c4.npz")


def run_learned(case, steps, warmup, w, d_ref, cache=None):
    """The learned path (9 x 9 dose + U-Net, falling back to the plain 61 x 61 path
    when its own error estimate is too large), forward + backward, timed like the
    plain path; its dose is compared with the plain FP32 61 x 61 dose.  With cache
    the 9 x 9 engine uses a geometry cache built before the timed region."""
    import numpy as np
    import torch
    from paper_2512_18863_amd import engine as E
    from paper_2512_18863_amd import gamma, learned
    net = learned.Net3D.from_file(LEARNED_WEIGHTS, case.shape)
    ld = learned.LearnedDose(net, case, mode="auto")
    dev = ld.small.device
    if cache:
        ld.small.build_cache(cache)
    lv = torch.tensor(case.leaves, dtype=torch.float32, device=dev)
    jw = torch.tensor(case.jaws, dtype=torch.float32, device=dev)
    mu = torch.tensor(case.mu, dtype=torch.float32, device=dev)
    g = torch.tensor(w, dtype=torch.float32, device=dev)

    def step():
        ld.forward(lv, jw, mu)
        return ld.backward(lv, jw, mu, g)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    E.profile_begin(64 * steps + 64)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    kernels = E.profile_end()
    dose = ld.forward(lv, jw, mu).cpu().numpy().astype(np.float64)
    fell_back = ld.fell_back
    raw = learned.LearnedDose(net, case, mode="never").forward(lv, jw, mu).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    return {"value": round(case.n_cp / (ms / 1e3), 3), "ms_per_step": round(ms, 4), "fell_back": fell_back,
            "max_abs_err_vs_fp32_61_over_max": float(np.abs(dose - d_ref).max() / np.abs(d_ref).max()),
            "gamma_1pct_1mm_vs_fp32_61": round(gamma.pass_rate(d_ref, dose, case.spacing, 1.0, 1.0), 6),
            "network_only": {"max_abs_err_over_max": float(np.abs(raw - d_ref).max() / np.abs(d_ref).max()),
                             "gamma_1pct_1mm": round(gamma.pass_rate(d_ref, raw, case.spacing, 1.0, 1.0), 6)},
            "kernels_ms_per_step": {k: round(v[1] / steps, 4) for k, v in sorted(kernels.items())},
            "note": "wall clock per step (the fallback decision reads two numbers back to the host)"}


def cpu_baseline(case, w, budget_s=12.0, max_cp=24):
    """The FP64 oracle, as it stands, on a sample of the plan's control points."""
    import numpy as np
    import oracle
    m = oracle.Model(case)
    rho = oracle.density(m)
    order = np.random.default_rng(0).permutation(case.n_cp)
    t0 = time.perf_counter()
    done = 0
    for b in order[:max_cp]:
        sl = slice(b, b + 1)
        oracle.forward(m, rho, case.gantry[sl], case.leaves[sl], case.jaws[sl], case.mu[sl])
        oracle.backward(m, rho, case.gantry[sl], case.leaves[sl], case.jaws[sl], case.mu[sl], w)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": round(done / dt, 4), "unit": "control points/s (fwd+bwd)", "cores": threads,
            "kind": "oracle",
            "sample": "%d of the %d control points of the same plan, forward + backward, one at a time, "
                      "%.1f s" % (done, case.n_cp, dt)}


def counter_run(case, w):
    """A copy kernel of known size (1 GiB read + 1 GiB written) followed by one
    FP32 forward and one backward of the benchmark plan."""
    import torch
    from paper_2512_18863_amd import engine as E
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    eng = E.DoseEngine(case, conv="fp32")
    dev = eng.device
    lv = torch.tensor(case.leaves, dtype=torch.float32, device=dev)
    jw = torch.tensor(case.jaws, dtype=torch.float32, device=dev)
    mu = torch.tensor(case.mu, dtype=torch.float32, device=dev)
    eng.forward(lv, jw, mu)
    eng.backward(lv, jw, mu, torch.tensor(w, dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    print("counter run done", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-fluence-corr", action="store_true")
    ap.add_argument("--no-cache", action="store_true", help="skip the geometry-cache variants")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from the two counter runs' CSV files and exit")
    ap.add_argument("--counter-run", action="store_true",
                    help="one copy of 1 GiB (the counter calibration) then one FP32 forward + backward; "
                         "for rocprofv3 --pmc runs")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from_counters(*args.traffic_from)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the dose path is built and timed on a single MI355X; "
              "multi-GPU control-point sharding is a design note only (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2512_18863_amd import gamma, inputs

    case = inputs.config_c4_plan(2000, bench=True)
    w = np.random.default_rng(4001).uniform(0.0, 1.0, size=case.shape)
    if args.counter_run:
        counter_run(case, w)
        return
    n_cp = case.n_cp
    print("[bench] fp32 fwd+bwd, %d CPs, 128^3, n=61: warmup %d, steps %d" % (n_cp, args.warmup, args.steps),
          file=sys.stderr, flush=True)
    ms, kernels, d32, eng = run_gpu(case, "fp32", args.steps, args.warmup, w)
    nodes = n_cp * eng.Nk * eng.Nu * eng.Nv
    n = eng.spec.n_taps
    conv_name = "conv_mfma_f32"
    launches, total_ms = kernels.get(conv_name, (0, 0.0))
    avg_s = total_ms / max(launches, 1) / 1e3
    ap_nodes = int(aperture_pixels(case.jaws, case.lat_step, eng.Nu, eng.Nv).sum()) * eng.Nk
    flops = 2.0 * n * n * ap_nodes           # the convolution's work on the aperture nodes
    dense_flops = 2.0 * n * n * nodes        # every beam-frame node (what a dense convolution does)
    achieved = flops / avg_s / 1e12 if avg_s > 0 else 0.0
    traffic = measured_traffic(conv_name, "c4bench_fp32")
    out = {
        "metric": "fwd+bwd control points/s at 128^3",
        "value": round(n_cp / (ms / 1e3), 3),
        "unit": "control points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "128^3 pelvis at 3 mm, two arcs of 180 control points, 60 leaf pairs, "
                               "jaws +-40 mm, 61x61 kernel, per-ray depth, FP32 convolution",
                   "grid": [128, 128, 128], "n_cp": n_cp, "n_taps": n,
                   "beam_frame_grid": [eng.Nu, eng.Nv, eng.Nk]},
        "roofline": {"kernel": conv_name, "bound": "mfma", "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4),
                     "traffic": traffic,
                     "flops_per_launch": flops, "avg_launch_ms": round(avg_s * 1e3, 4),
                     "launches": launches,
                     "work": "2 n^2 flops per aperture node (fan pixels overlapping the jaw opening x planes): "
                             "%d of %d nodes" % (ap_nodes, nodes),
                     "dense_equivalent_TFLOPs": round(dense_flops / avg_s / 1e12, 3) if avg_s > 0 else 0.0},
        "kernels_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in sorted(kernels.items())},
        "hbm_kernels": hbm_table(kernels, args.steps, n_cp, nodes, ap_nodes, eng.Nu * eng.Nv,
                                 int(np.prod(case.shape))),
        "paper_context": {"value": 35.3, "unit": "control points/s (fwd+bwd)", "hardware": "NVIDIA A40",
                          "workload": "105x224x224 grid, 180 control points, kernel 55 (Table 6: 5.102 s)"},
    }
    del eng
    torch.cuda.empty_cache()
    if not args.no_bf16:
        print("[bench] bf16 variant", file=sys.stderr, flush=True)
        ms16, k16, d16, eng16 = run_gpu(case, "bf16", args.steps, args.warmup, w)
        l16, t16 = k16.get("conv_mfma_bf16", (0, 0.0))
        a16 = flops / (t16 / max(l16, 1) / 1e3) / 1e12 if t16 > 0 else 0.0
        err = float(np.abs(d16.astype(np.float64) - d32).max() / np.abs(d32).max())
        print("[bench] gamma 1%/1mm bf16 vs fp32", file=sys.stderr, flush=True)
        gp = gamma.pass_rate(d32, d16, case.spacing, 1.0, 1.0)
        out["variants"] = {"bf16": {
            "value": round(n_cp / (ms16 / 1e3), 3), "ms_per_step": round(ms16, 4),
            "max_abs_err_vs_fp32_over_max": err, "gamma_1pct_1mm_vs_fp32": round(gp, 6),
            "roofline": {"kernel": "conv_mfma_bf16", "bound": "mfma", "achieved": round(a16, 3),
                         "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(a16 / PEAK_BF16_MFMA_TFLOPS, 4)},
            "kernels_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in sorted(k16.items())}}}
        del eng16
    if not args.no_fluence_corr:
        print("[bench] fp32 with fluence corrections", file=sys.stderr, flush=True)
        import copy
        cc = copy.copy(case)
        cc.machine = inputs.with_fluence_corrections(case.machine)
        msc, kc, _, engc = run_gpu(cc, "fp32", args.steps, args.warmup, w)
        out.setdefault("variants", {})["fp32_fluence_corrections"] = {
            "value": round(n_cp / (msc / 1e3), 3), "ms_per_step": round(msc, 4),
            "corrections": "penumbra FWHM 3.5/4.5 mm, head scatter 4 % (sigma 20 mm), off-axis +4 % at 100 mm",
            "kernels_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in sorted(kc.items())}}
        del engc
        torch.cuda.empty_cache()
    if not args.no_cache:
        for name, conv, kind in (("fp32_geometry_cache", "fp32", "fp32"), ("bf16_geometry_cache", "bf16", "bf16")):
            print("[bench] %s" % name, file=sys.stderr, flush=True)
            msg, kg, dg, engg = run_gpu(case, conv, args.steps, args.warmup, w, cache=kind)
            v = {"value": round(n_cp / (msg / 1e3), 3), "ms_per_step": round(msg, 4),
                 "cache": "%s factor, %.2f GB, built once per plan in %.2f ms (not in the step)"
                          % (kind.upper(), engg.cache_bytes / 1e9, engg.cache_build_ms),
                 "kernels_ms_per_step": {k: round(x[1] / args.steps, 4) for k, x in sorted(kg.items())}}
            if kind == "fp32":
                v["identical_to_uncached_fp32"] = bool(np.array_equal(dg, d32))
            else:
                v["max_abs_err_vs_fp32_over_max"] = float(np.abs(dg.astype(np.float64) - d32).max()
                                                          / np.abs(d32).max())
                v["gamma_1pct_1mm_vs_fp32"] = round(gamma.pass_rate(d32, dg, case.spacing, 1.0, 1.0), 6)
            out.setdefault("variants", {})[name] = v
            del engg
            torch.cuda.empty_cache()
    if not args.no_learned and os.path.exists(LEARNED_WEIGHTS):
        print("[bench] learned variant", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out.setdefault("variants", {})["learned"] = run_learned(case, args.steps, args.warmup, w, d32)
        if not args.no_cache:
            print("[bench] learned variant with geometry cache", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
            out["variants"]["learned_geometry_cache"] = run_learned(case, args.steps, args.warmup, w, d32,
                                                                    cache="fp32")
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
