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
import fnmatch
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
PEAK_FP32_MFMA_TFLOPS = 157.3     # MI355X dense FP32 matrix peak
PEAK_BF16_MFMA_TFLOPS = 2500.0    # MI355X dense BF16 matrix peak
PEAK_HBM_GBS = 8000.0


# kernels whose HBM counters are recorded in profiles/traffic.json: the library's
# profile name -> (patterns of the kernel-trace symbol with blanks removed, sources
# the kernel is built from)
_CONV = ["conv_mfma.hip", "conv_common.hpp", "taps.hpp", "device_math.hpp", "pdrt_internal.hpp"]
_CONV16 = ["conv_bf16.hip", "conv_common.hpp", "taps.hpp", "device_math.hpp", "pdrt_internal.hpp"]
_FWDREG = ["conv_fwd_reg.hip", "conv_mfma.hip", "conv_bf16.hip", "conv_common.hpp", "taps.hpp", "device_math.hpp",
           "pdrt_internal.hpp"]
_FWD = ["dose_fwd.hip", "taps.hpp", "device_math.hpp", "pdrt_internal.hpp"]
_BWD = ["dose_bwd.hip", "device_math.hpp", "pdrt_internal.hpp"]
KERNELS = {
    # forwards: the register-resident kernel <BF16?, T, SU>
    "conv_mfma_f32": (("k_conv_fwd_reg<false,",), _FWDREG),
    # adjoint: the window kernel <NW, TPW> (the region kernel serves the fluence corrections)
    "conv_mfma_f32_adj": (("k_conv_f32_adj_win<", "k_conv_mfma_f32_adj<"), _CONV),
    "conv_mfma_bf16": (("k_conv_fwd_reg<true,",), _FWDREG),
    # BF16 adjoint: the window kernel <NK> (the tiled kernel <NK, BR, BC, NWB, NWP, SUP> with
    # 2 x 2 tiles in four wavefronts serves the fluence corrections)
    "conv_mfma_bf16_adj": (("k_conv_bf16_adj_win<", "k_conv_bf16<*,2,2,1,4,*"), _CONV16),
    "march": (("k_march_serial<float,0,",), _FWD),
    "march_adj": (("k_march_serial<float,1,",), _FWD),
    "gather": (("k_gather<float",), _FWD),
    "backproject_adj": (("k_backproject_reg<float", "k_backproject_adj<float"), _BWD),
}


def _symbol_match(name, pattern):
    return fnmatch.fnmatchcase(name.replace(" ", ""), "*" + pattern + "*")


def kernel_source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNELS[kernel][1]:
        with open(os.path.join(ROOT, "paper_2512_18863_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they were
    taken on the kernel's current sources; otherwise None."""
    if kernel not in KERNELS:
        return None
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


COPY_BYTES = 1 << 30   # the counter run's calibration copy


def traffic_from_counters(fetch_csv, write_csv, workload="c4bench"):
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
    for name, (syms, _src) in KERNELS.items():
        hits = [(n, v, v2) for (n, v), (_, v2) in zip(fetch, write) if any(_symbol_match(n, sy) for sy in syms)]
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


class Work:
    """Algorithmic work of one dose-path step (per launch of each kernel): flops of
    the convolutions (2 n^2 per aperture node), bytes of the memory-bound kernels
    (each byte the kernel must move once)."""

    def __init__(self, case, eng):
        import numpy as np
        n = eng.spec.n_taps
        self.n_cp = case.n_cp
        self.nodes = case.n_cp * eng.Nk * eng.Nu * eng.Nv
        self.ap_nodes = int(aperture_pixels(case.jaws, case.lat_step, eng.Nu, eng.Nv).sum()) * eng.Nk
        self.plane = eng.Nu * eng.Nv
        self.vox = int(np.prod(case.shape))
        self.conv_flops = 2.0 * n * n * self.ap_nodes
        self.dense_conv_flops = 2.0 * n * n * self.nodes

    def entry(self, kernel):
        """(bound, algorithmic units per launch, peak, unit) of a kernel, or None."""
        hbm = {
            "march": 4 * self.ap_nodes + 4 * self.n_cp * self.plane + 4 * self.vox,      # write P; read F, rho
            "march_adj": 4 * self.ap_nodes + 4 * self.n_cp * self.plane + 4 * self.vox,  # read H; write A; read rho
            "gather": 4 * self.nodes + 2 * 4 * self.vox,                                # read Dfan; write dose + comp
            "backproject_adj": 4 * self.nodes + 4 * self.vox,                           # write G; read g
        }
        if kernel in hbm:
            return "hbm", float(hbm[kernel]), PEAK_HBM_GBS, "GB/s"
        if kernel.startswith("conv_mfma_f32"):
            return "mfma", self.conv_flops, PEAK_FP32_MFMA_TFLOPS, "TFLOP/s"
        if kernel.startswith("conv_mfma_bf16"):
            return "mfma", self.conv_flops, PEAK_BF16_MFMA_TFLOPS, "TFLOP/s"
        return None


def roofline_entry(kernel, kernels, steps, work, traffic=None):
    """Achieved rate of one kernel from its algorithmic work per launch and its
    average launch time (HIP events around every launch in the timed region)."""
    e = work.entry(kernel)
    if e is None or kernel not in kernels:
        return None
    bound, units, peak, unit = e
    launches, total_ms = kernels[kernel]
    avg_s = total_ms / max(launches, 1) / 1e3
    scale = 1e9 if unit == "GB/s" else 1e12
    ach = units / avg_s / scale if avg_s > 0 else 0.0
    out = {"kernel": kernel, "bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
           "frac": round(ach / peak, 4), "traffic": traffic, "avg_launch_ms": round(avg_s * 1e3, 4),
           "launches": launches}
    if unit == "TFLOP/s":
        out["flops_per_launch"] = units
        out["dense_equivalent_TFLOPs"] = round(ach * work.dense_conv_flops / work.conv_flops, 3)
        # the FP32 planes it must move once: the aperture nodes on one side, every node on the other
        out["algorithmic_bytes_per_launch"] = 4 * work.ap_nodes + 4 * work.nodes
    else:
        out["algorithmic_bytes_per_launch"] = units
    if traffic:
        out["traffic_over_algorithmic"] = round(traffic / out["algorithmic_bytes_per_launch"], 3)
    return out


def _tensors(case, dev):
    import torch
    return (torch.tensor(case.leaves, dtype=torch.float32, device=dev),
            torch.tensor(case.jaws, dtype=torch.float32, device=dev),
            torch.tensor(case.mu, dtype=torch.float32, device=dev))


def timed(fn, steps, warmup, profile=True):
    """Median and mean ms of `fn` over `steps` calls after `warmup` (torch events on
    the current stream, which every library kernel is launched on), and the
    library's per-kernel times over the timed calls."""
    import numpy as np
    import torch
    from paper_2512_18863_amd import engine as E
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if profile:
        E.profile_begin(256 * steps + 256)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    kernels = E.profile_end() if profile else {}
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return float(np.median(per)), float(per.mean()), kernels


def per_step(kernels, steps):
    return {k: round(v[1] / steps, 4) for k, v in sorted(kernels.items())}


def run_gpu(case, conv, steps, warmup, w, cache=None, forward_only=False, march_scan=False):
    """Forward + backward (or forward only) timed over `steps`; with cache = "fp32" /
    "bf16" the plan's geometry cache is built first (once per plan, not timed)."""
    import torch
    from paper_2512_18863_amd import engine as E
    eng = E.DoseEngine(case, conv=conv, march_scan=march_scan)
    dev = eng.device
    if cache:
        torch.cuda.synchronize()
        tb = time.perf_counter()
        eng.cache_bytes = eng.build_cache(cache)
        torch.cuda.synchronize()
        eng.cache_build_ms = (time.perf_counter() - tb) * 1e3
    lv, jw, mu = _tensors(case, dev)
    g = torch.tensor(w, dtype=torch.float32, device=dev)
    dose = torch.empty(eng.vol_shape, dtype=torch.float32, device=dev)

    def step():
        eng.forward(lv, jw, mu, out=dose)
        if not forward_only:
            eng.backward(lv, jw, mu, g)

    med, mean, kernels = timed(step, steps, warmup)
    fwd_dose = eng.forward(lv, jw, mu).cpu().numpy()
    grads = None if forward_only else [t.cpu().numpy() for t in eng.backward(lv, jw, mu, g)]
    torch.cuda.synchronize()
    return {"median_ms": med, "mean_ms": mean, "kernels": kernels, "dose": fwd_dose, "grads": grads, "eng": eng}


LEARNED_WEIGHTS = os.path.join(ROOT, "paper_2512_18863_amd", "data", "learned_c4.npz")


def net_flops(shape):
    """Matrix work of one network pass over a volume: 2 * 27 * Cin * Cout flops per
    output position of each 3 x 3 x 3 convolution at its level's resolution."""
    from paper_2512_18863_amd import learned
    import numpy as np
    P = int(np.prod(shape))
    tot = 0.0
    for (name, c1, c2, cout, lvl) in learned.LAYERS:
        tot += 2.0 * 27 * (c1 + c2) * cout * P / (8 ** lvl)
    return tot


def run_learned(case, steps, warmup, w, d_ref, cache=None):
    """The learned path (9 x 9 dose + U-Net, falling back to the plain 61 x 61 path
    when its own error estimate is too large), forward + backward; its dose is
    compared with the plain FP32 61 x 61 dose.  Timed by wall clock: the fallback
    decision reads two numbers back to the host every step."""
    import numpy as np
    import torch
    from paper_2512_18863_amd import engine as E
    from paper_2512_18863_amd import gamma, learned
    net = learned.Net3D.from_file(LEARNED_WEIGHTS, case.shape)
    ld = learned.LearnedDose(net, case, mode="auto")
    dev = ld.small.device
    if cache:
        ld.small.build_cache(cache)
    lv, jw, mu = _tensors(case, dev)
    g = torch.tensor(w, dtype=torch.float32, device=dev)

    def step():
        ld.forward(lv, jw, mu)
        return ld.backward(lv, jw, mu, g)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    E.profile_begin(256 * steps + 256)
    per = []
    for _ in range(steps):
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t0) * 1e3)
    kernels = E.profile_end()
    ms = float(np.median(per))
    dose = ld.forward(lv, jw, mu).cpu().numpy().astype(np.float64)
    fell_back = ld.fell_back
    est = net.stats.cpu().numpy()
    raw = learned.LearnedDose(net, case, mode="never").forward(lv, jw, mu).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    fl = net_flops(case.shape)
    conv3d = {}
    for k in ("conv3d_fwd", "conv3d_dgrad"):
        if k in kernels:
            t = kernels[k][1] / steps / 1e3
            conv3d[k] = {"bound": "mfma", "achieved": round(fl / t / 1e12, 3), "peak": PEAK_BF16_MFMA_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(fl / t / 1e12 / PEAK_BF16_MFMA_TFLOPS, 4),
                         "ms_per_step": round(t * 1e3, 4), "flops_per_pass": fl}
    return {"value": round(case.n_cp / (ms / 1e3), 3), "ms_per_step": round(ms, 4), "fell_back": fell_back,
            "error_estimate_over_max": float(est[1] / est[0]),
            "max_abs_err_vs_fp32_61_over_max": float(np.abs(dose - d_ref).max() / np.abs(d_ref).max()),
            "gamma_1pct_1mm_vs_fp32_61": round(gamma.pass_rate(d_ref, dose, case.spacing, 1.0, 1.0), 6),
            "network_only": {"max_abs_err_over_max": float(np.abs(raw - d_ref).max() / np.abs(d_ref).max()),
                             "gamma_1pct_1mm": round(gamma.pass_rate(d_ref, raw, case.spacing, 1.0, 1.0), 6)},
            "roofline_conv3d": conv3d,
            "kernels_ms_per_step": per_step(kernels, steps),
            "note": "median wall clock per step (the fallback decision reads two numbers back)"}


def errors_vs_oracle(case, w, engines, idx):
    """FP32 and BF16 dose and gradient errors against the FP64 oracle on the control
    points idx of the benchmark plan, in the benchmark's launch configuration."""
    import copy
    import numpy as np
    import torch
    import oracle
    sub = copy.copy(case)
    sub.gantry, sub.leaves, sub.jaws, sub.mu = case.gantry[idx], case.leaves[idx], case.jaws[idx], case.mu[idx]
    m = oracle.Model(sub)
    rho = oracle.density(m)
    ref = oracle.forward(m, rho, sub.gantry, sub.leaves, sub.jaws, sub.mu)
    rg = oracle.backward(m, rho, sub.gantry, sub.leaves, sub.jaws, sub.mu, w)
    out = {"control_points": [int(i) for i in idx]}
    for name, eng in engines.items():
        lv, jw, mu = _tensors(case, eng.device)
        mu0 = torch.zeros_like(mu)
        mu0[torch.as_tensor(idx, device=eng.device)] = mu[torch.as_tensor(idx, device=eng.device)]
        d = eng.forward(lv, jw, mu0).cpu().numpy().astype(np.float64)
        g = [t.cpu().numpy() for t in eng.backward(lv, jw, mu, torch.tensor(w, dtype=torch.float32,
                                                                          device=eng.device))]
        e = {"dose_max_abs_err_over_max": float(np.abs(d - ref).max() / np.abs(ref).max())}
        for gname, got, r in zip(("leaves", "jaws", "mu"), g, rg):
            e["grad_%s_max_abs_err_over_max" % gname] = float(np.abs(got[idx] - r).max() / np.abs(r).max())
        out[name] = e
    return out


def config_lines(steps, warmup):
    """Forward and forward + backward CP/s of the C1 and C2 workloads and of the
    paper's timing shape (P0, Table 6)."""
    import numpy as np
    import torch
    from paper_2512_18863_amd import inputs
    out = {}
    for name, mk, desc in (
            ("c1", inputs.config_c1, "128x128x96 pelvis at 3 mm, 90 control points, 15x15 kernel"),
            ("c2", inputs.config_c2, "192x192x128 pelvis at 2.5 mm, 180 control points (two arcs), 31x31 kernel"),
            ("p0_paper_shape", inputs.config_p0,
             "224x224x105 pelvis at 2 mm, 180 control points (two arcs), 55x55 kernel: the dose-grid, "
             "control-point and kernel sizes of the paper's Table 6")):
        print("[bench] %s" % name, file=sys.stderr, flush=True)
        case = mk()
        w = case.loss_w
        fwd = run_gpu(case, "fp32", steps, warmup, w, forward_only=True)
        both = run_gpu(case, "fp32", steps, warmup, w)
        eng = both["eng"]
        line = {"workload": desc, "beam_frame_grid": [eng.Nu, eng.Nv, eng.Nk],
                "forward": {"value": round(case.n_cp / (fwd["median_ms"] / 1e3), 3), "unit": "control points/s",
                            "ms": round(fwd["median_ms"], 4)},
                "fwd_bwd": {"value": round(case.n_cp / (both["median_ms"] / 1e3), 3), "unit": "control points/s",
                            "ms": round(both["median_ms"], 4)},
                "kernels_ms_per_step": per_step(both["kernels"], steps)}
        if name == "p0_paper_shape":
            line["paper_context"] = {"forward_s": 2.051, "fwd_bwd_s": 5.102, "hardware": "NVIDIA A40",
                                     "source": "Table 6 (mean over 100 iterations; precision not stated)"}
        out[name] = line
        del fwd, both, eng
        torch.cuda.empty_cache()
    return out


def c3_line():
    """The optimisation workload: 200 Adam steps of the quadratic objective from the
    closed start on the 192x192x128 two-arc geometry (31x31 kernel), time per step,
    and the final objective against the oracle's recomputation of the final dose."""
    import numpy as np
    import torch
    import oracle
    from paper_2512_18863_amd import inputs, optimize
    print("[bench] c3 optimisation (200 Adam steps)", file=sys.stderr, flush=True)
    case = optimize.c3_case()
    masks = inputs.structures_c3(case)
    opt = optimize.PlanOptimizer(case, masks)
    losses, sec = opt.run(200)
    lv, jw, mu, dose = opt.final()
    L_gpu = float(optimize.objective(dose, opt.masks))
    print("[bench] c3 oracle recomputation of the final dose (%d control points)" % case.n_cp, file=sys.stderr,
          flush=True)
    m = oracle.Model(case)
    ref = oracle.forward(m, oracle.density(m), case.gantry, lv, jw, mu)
    L_ref = float(optimize.objective(torch.tensor(ref), {k: torch.tensor(v) for k, v in masks.items()}))
    d = dose.cpu().numpy().astype(np.float64)
    return {"workload": "192x192x128 pelvis at 2.5 mm, 180 control points, 31x31 kernel, quadratic "
                        "dose-volume objective, Adam from closed apertures",
            "steps": 200, "ms_per_step": round(1e3 * sec, 4), "objective_start": losses[0],
            "objective_final_gpu": L_gpu, "objective_final_oracle_dose": L_ref,
            "final_dose_max_abs_err_vs_oracle_over_max": float(np.abs(d - ref).max() / ref.max())}


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def cpu_baseline(case, w, runs=3, cps=8):
    """The FP64 oracle, as it stands, on samples of the plan's control points
    (forward + backward, one control point at a time): median of `runs` runs."""
    import numpy as np
    import oracle
    m = oracle.Model(case)
    rho = oracle.density(m)
    order = np.random.default_rng(0).permutation(case.n_cp)
    rates, total = [], 0.0
    for r in range(runs):
        t0 = time.perf_counter()
        for b in order[r * cps:(r + 1) * cps]:
            sl = slice(b, b + 1)
            oracle.forward(m, rho, case.gantry[sl], case.leaves[sl], case.jaws[sl], case.mu[sl])
            oracle.backward(m, rho, case.gantry[sl], case.leaves[sl], case.jaws[sl], case.mu[sl], w)
        dt = time.perf_counter() - t0
        total += dt
        rates.append(cps / dt)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": round(float(np.median(rates)), 4), "unit": "control points/s (fwd+bwd)", "cores": threads,
            "kind": "oracle", "runs": [round(x, 4) for x in rates], "nproc": os.cpu_count(), "cpu": cpu_info(),
            "sample": "median of %d runs, each %d distinct control points of the same plan, forward + backward, "
                      "one at a time (%.1f s in total); the oracle is a plain FP64 reference, not a tuned "
                      "CPU engine" % (runs, cps, total)}


def counter_run(case, w):
    """A copy kernel of known size (1 GiB read + 1 GiB written) followed by one
    forward and one backward of the benchmark plan with the FP32 convolution, then
    one of each with the BF16 convolution."""
    import torch
    from paper_2512_18863_amd import engine as E
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    for conv in ("fp32", "bf16"):
        eng = E.DoseEngine(case, conv=conv)
        dev = eng.device
        lv, jw, mu = _tensors(case, dev)
        eng.forward(lv, jw, mu)
        eng.backward(lv, jw, mu, torch.tensor(w, dtype=torch.float32, device=dev))
        torch.cuda.synchronize()
        del eng
        torch.cuda.empty_cache()
    print("counter run done", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-fluence-corr", action="store_true")
    ap.add_argument("--no-cache", action="store_true", help="skip the geometry-cache variants")
    ap.add_argument("--no-configs", action="store_true", help="skip the C1, C2, C3 and paper-shape lines")
    ap.add_argument("--no-oracle-errors", action="store_true")
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
    K, W = args.steps, args.warmup
    print("[bench] fp32 fwd+bwd, %d CPs, 128^3, n=61: warmup %d, steps %d" % (n_cp, W, K),
          file=sys.stderr, flush=True)
    r32 = run_gpu(case, "fp32", K, W, w)
    eng = r32["eng"]
    work = Work(case, eng)
    kernels = r32["kernels"]
    d32 = r32["dose"]
    rl = {}
    for k in sorted(kernels):
        e = roofline_entry(k, kernels, K, work, measured_traffic(k, "c4bench"))
        if e:
            rl[k] = e
    # the dominant kernel of the step: the one with the largest time per step
    dom = max((k for k in rl), key=lambda k: kernels[k][1])
    roof = {key: rl[dom][key] for key in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
    roof.update({"kernel": dom, "avg_launch_ms": rl[dom]["avg_launch_ms"], "launches": rl[dom]["launches"],
                 "work": "2 n^2 flops per aperture node (fan pixels overlapping the jaw opening x planes): "
                         "%d of %d nodes" % (work.ap_nodes, work.nodes)})
    for key in ("flops_per_launch", "dense_equivalent_TFLOPs"):
        if key in rl[dom]:
            roof[key] = rl[dom][key]
    out = {
        "metric": "fwd+bwd control points/s at 128^3",
        "value": round(n_cp / (r32["median_ms"] / 1e3), 3),
        "unit": "control points/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(r32["median_ms"], 4),
        "ms_per_step_mean": round(r32["mean_ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "128^3 pelvis at 3 mm, two arcs of 180 control points, 60 leaf pairs, "
                               "jaws +-40 mm, 61x61 kernel, per-ray depth, FP32 convolution",
                   "grid": [128, 128, 128], "n_cp": n_cp, "n_taps": eng.spec.n_taps,
                   "beam_frame_grid": [eng.Nu, eng.Nv, eng.Nk]},
        "roofline": roof,
        "roofline_kernels": rl,
        "kernels_ms_per_step": per_step(kernels, K),
        "paper_context": {"value": 35.3, "unit": "control points/s (fwd+bwd)", "hardware": "NVIDIA A40",
                          "workload": "105x224x224 grid, 180 control points, kernel 55 (Table 6: 5.102 s); "
                                      "see config_lines.p0_paper_shape for this build on that shape"},
    }
    print("[bench] fp32 forward only", file=sys.stderr, flush=True)
    f32 = run_gpu(case, "fp32", K, W, w, forward_only=True)
    out["forward_only"] = {"value": round(n_cp / (f32["median_ms"] / 1e3), 3), "unit": "control points/s",
                           "ms": round(f32["median_ms"], 4), "kernels_ms_per_step": per_step(f32["kernels"], K)}
    del f32
    engines = {"fp32": eng}
    variants = {}
    print("[bench] fp32 with the segmented-scan ray march", file=sys.stderr, flush=True)
    rs = run_gpu(case, "fp32", K, W, w, march_scan=True)
    variants["fp32_march_scan"] = {
        "value": round(n_cp / (rs["median_ms"] / 1e3), 3), "ms_per_step": round(rs["median_ms"], 4),
        "march": "depth integral as a segmented scan over the wavefronts of a workgroup (spec.march_scan = 1); "
                 "the default is one thread per ray",
        "max_abs_err_vs_default_over_max": float(np.abs(rs["dose"].astype(np.float64) - d32).max()
                                                 / np.abs(d32).max()),
        "roofline_kernels": {k: roofline_entry(k, rs["kernels"], K, work) for k in ("march", "march_adj")},
        "kernels_ms_per_step": per_step(rs["kernels"], K)}
    del rs
    torch.cuda.empty_cache()
    if not args.no_bf16:
        print("[bench] bf16 variant", file=sys.stderr, flush=True)
        r16 = run_gpu(case, "bf16", K, W, w)
        d16 = r16["dose"]
        err = float(np.abs(d16.astype(np.float64) - d32).max() / np.abs(d32).max())
        print("[bench] gamma 1%/1mm bf16 vs fp32", file=sys.stderr, flush=True)
        gp = gamma.pass_rate(d32, d16, case.spacing, 1.0, 1.0)
        f16 = run_gpu(case, "bf16", K, W, w, forward_only=True)
        variants["bf16"] = {
            "value": round(n_cp / (r16["median_ms"] / 1e3), 3), "ms_per_step": round(r16["median_ms"], 4),
            "forward_only": {"value": round(n_cp / (f16["median_ms"] / 1e3), 3), "ms": round(f16["median_ms"], 4)},
            "max_abs_err_vs_fp32_over_max": err, "gamma_1pct_1mm_vs_fp32": round(gp, 6),
            "roofline_kernels": {k: roofline_entry(k, r16["kernels"], K, work, measured_traffic(k, "c4bench"))
                                 for k in r16["kernels"] if k.startswith("conv_mfma_bf16")},
            "kernels_ms_per_step": per_step(r16["kernels"], K)}
        engines["bf16"] = r16["eng"]
        del f16
    if not args.no_oracle_errors:
        print("[bench] errors against the oracle (6 control points)", file=sys.stderr, flush=True)
        out["errors_vs_oracle"] = errors_vs_oracle(case, w, engines, np.array([3, 60, 91, 122, 150, 177]))
    del engines, eng
    r32.pop("eng")
    torch.cuda.empty_cache()
    if "bf16" in variants:
        del r16
        torch.cuda.empty_cache()
    if not args.no_fluence_corr:
        print("[bench] fp32 with fluence corrections", file=sys.stderr, flush=True)
        import copy
        cc = copy.copy(case)
        cc.machine = inputs.with_fluence_corrections(case.machine)
        rc = run_gpu(cc, "fp32", K, W, w)
        variants["fp32_fluence_corrections"] = {
            "value": round(n_cp / (rc["median_ms"] / 1e3), 3), "ms_per_step": round(rc["median_ms"], 4),
            "corrections": "penumbra FWHM 3.5/4.5 mm, head scatter 4 % (sigma 20 mm), off-axis +4 % at 100 mm",
            "kernels_ms_per_step": per_step(rc["kernels"], K)}
        print("[bench] fp32 with collimator rotation", file=sys.stderr, flush=True)
        cr = copy.copy(case)
        cr.collimator = np.linspace(-45.0, 45.0, n_cp)
        rr = run_gpu(cr, "fp32", K, W, w)
        variants["fp32_collimator_rotation"] = {
            "value": round(n_cp / (rr["median_ms"] / 1e3), 3), "ms_per_step": round(rr["median_ms"], 4),
            "collimator": "angles -45 ... 45 degrees over the plan; square beam-frame grid %s"
                          % [rr["eng"].Nu, rr["eng"].Nv, rr["eng"].Nk],
            "kernels_ms_per_step": per_step(rr["kernels"], K)}
        del rc, rr
        torch.cuda.empty_cache()
    if not args.no_cache:
        for name, conv, kind in (("fp32_geometry_cache", "fp32", "fp32"), ("bf16_geometry_cache", "bf16", "bf16")):
            print("[bench] %s" % name, file=sys.stderr, flush=True)
            rg = run_gpu(case, conv, K, W, w, cache=kind)
            engg = rg["eng"]
            v = {"value": round(n_cp / (rg["median_ms"] / 1e3), 3), "ms_per_step": round(rg["median_ms"], 4),
                 "cache": "%s factor, %.2f GB, built once per plan in %.2f ms (not in the step)"
                          % (kind.upper(), engg.cache_bytes / 1e9, engg.cache_build_ms),
                 "kernels_ms_per_step": per_step(rg["kernels"], K)}
            if kind == "fp32":
                v["identical_to_uncached_fp32"] = bool(np.array_equal(rg["dose"], d32))
            else:
                v["max_abs_err_vs_fp32_over_max"] = float(np.abs(rg["dose"].astype(np.float64) - d32).max()
                                                          / np.abs(d32).max())
                v["gamma_1pct_1mm_vs_fp32"] = round(gamma.pass_rate(d32, rg["dose"], case.spacing, 1.0, 1.0), 6)
            variants[name] = v
            del rg, engg
            torch.cuda.empty_cache()
    if not args.no_learned and os.path.exists(LEARNED_WEIGHTS):
        print("[bench] learned variant", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        variants["learned"] = run_learned(case, K, W, w, d32)
        if not args.no_cache:
            print("[bench] learned variant with geometry cache", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
            variants["learned_geometry_cache"] = run_learned(case, K, W, w, d32, cache="fp32")
    out["variants"] = variants
    if not args.no_configs:
        torch.cuda.empty_cache()
        out["config_lines"] = config_lines(K, W)
        out["config_lines"]["c3"] = c3_line()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
