#!/usr/bin/env python3
"""Benchmark: supernodal selected inversion on one MI355X.

One step = one pass of the whole hot path over one matrix whose factors are
already in HBM: diagonal-block inversion, normalisation, then the level sweep
(gather, products of steps 3 and 5, product of step 4) and the extraction of
the selected entries into a device buffer.  Throughput is algorithmic GFLOP/s
(flop convention: F_K = 4 s cL cU + 2 s^2 cU + s^2 (cL + cU) + 4/3 s^3 per
supernode, the same for every precision) over the timed steps.

Default workload: 2D 9-point asymmetric stencil on a 256x256 grid (n = 65536),
nested dissection, supernodes <= 128, FP64 (the plain-FP64 GPU configuration);
the mixed form is measured on the same matrix and reported beside it.

Prints ONE JSON line.  --gpus N with N > 1 exits: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "mixed_fp32": 157.3, "mixed_bf16x3": 2500.0}  # dense TFLOP/s, MI355X
HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c1", choices=["c0", "c1", "c2", "c4", "u1", "u4", "z1"])
    ap.add_argument("--symbolic", default=None, choices=["symmetrized", "exact"],
                    help="analysis form (default: symmetrized for c*, exact for the upwind u* configs)")
    ap.add_argument("--precision", default=None, help="fp64 | mixed_fp32 | mixed_bf16x3 (default: per config)")
    ap.add_argument("--mixed", default="mixed_fp32", help="mixed form reported beside the main one")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--sweep", default="auto", choices=["auto", "levels", "persistent"])
    ap.add_argument("--no-tune", action="store_true", help="size policy instead of the autotuner's choices")
    ap.add_argument("--tune-reps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-device-lu", action="store_true", help="skip timing the LU on the device (setup)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="bound on the oracle's CPU time")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for scaling HBM counters) and exit")
    return ap.parse_args()


WORKLOADS = {
    "c0": "2D 32x32 5-point asymmetric convection-diffusion, n=1024, ND, supernodes<=32",
    "c1": "2D 256x256 9-point asymmetric stencil, n=65536, ND, supernodes<=128",
    "c2": "3D 48^3 7-point asymmetric convection-diffusion, n=110592, ND, supernodes<=256",
    "c4": "3D 64^3 27-point asymmetric stencil, n=262144, ND, supernodes<=512",
    "u1": "2D 256x256 9-point upwind stencil (non-symmetric pattern), n=65536, ND, supernodes<=128",
    "u4": "3D 64^3 27-point upwind stencil (non-symmetric pattern), n=262144, ND, supernodes<=512",
    "z1": "complex 2D 256x256 9-point shifted stencil, n=65536 (real form of order 131072), ND, supernodes<=128 nodes",
}


def timed_steps(s, prec, steps, warmup, graph, out, stream):
    import torch
    for _ in range(warmup):
        s.run(prec, stream=stream, graph=graph)
        s.get_selected_device(out, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        s.run(prec, stream=stream, graph=graph)
        s.get_selected_device(out, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return max(e0.elapsed_time(e1) / 1e3, 0.0), wall


def phase_profile(s, prec, stream, reps=5):
    """Per-phase device times from HIP events recorded on the run's stream.

    Returns per-class totals and, per level, the time and work of each launch,
    so that a kernel class can be priced against its roofline."""
    import numpy as np
    import torch
    s.set_profiling(True)
    acc = None
    for _ in range(reps):
        s.run(prec, stream=stream)
        t = s.timings()
        acc = t if acc is None else acc + t
    torch.cuda.synchronize()
    s.set_profiling(False)
    t = acc / reps
    L = s.info["nlevels"]
    lev = [s.level_stats(d) for d in range(L)]
    ph = {
        "tri_inv_ms": float(t[0]),
        "normalise_ms": float(t[1]),
        "diag_init_ms": float(t[2]),
        "small_ms": float(sum(t[3 + 4 * d] for d in range(L))),
        "gather_ms": float(sum(t[4 + 4 * d] for d in range(L))),
        "gemm35_ms": float(sum(t[5 + 4 * d] for d in range(L))),
        "gemm4_ms": float(sum(t[6 + 4 * d] for d in range(L))),
    }
    # An interval between two events that holds no launch measures the cost of
    # the event pair itself (a few us on this device); it is subtracted from
    # every launch's interval, so that launch times compare with the kernel
    # durations rocprofv3 reports.
    empty = [float(t[3 + 4 * d]) for d in range(L) if lev[d]["small_count"] == 0]
    empty += [float(t[4 + 4 * d]) for d in range(L) if lev[d]["gather_tiles"] == 0]
    ph["event_overhead_ms"] = float(np.median(empty)) if empty else 0.0
    launches = []
    for d in range(L):
        if lev[d]["small_count"] > 0:
            launches.append({"cls": "small", "tile": 64, "ms": float(t[3 + 4 * d]),
                             "flops": lev[d]["small_flops"]})
        if lev[d]["gather_tiles"] > 0:
            launches.append({"cls": "gather", "tile": 64, "ms": float(t[4 + 4 * d]),
                             "elems": lev[d]["gather_elems"]})
        if lev[d]["tiles35"] > 0:
            launches.append({"cls": "gemm35", "tile": int(lev[d]["tile35"]), "ms": float(t[5 + 4 * d]),
                             "flops": lev[d]["flops35"]})
        if lev[d]["tiles4"] > 0:
            launches.append({"cls": "gemm4", "tile": int(lev[d]["tile4"]), "ms": float(t[6 + 4 * d]),
                             "flops": lev[d]["flops4"]})
    ph["launches"] = launches
    return ph


KERNEL_SYMBOL = {
    # (class, precision, tile) -> kernel symbol as rocprofv3 prints it
    "gemm35": "selinv::gemm_v2<{mode}, {t}, {t}, {T}, {T}, 1>",
    "gemm4": "selinv::step4_gather<{mode}, {t}, {t}, {T}>",
    "gather": "selinv::gather_kernel<{T}>",
    "small": "selinv::small_kernel<{mode}>",
}


def roofline(ph, prec):
    """Dominant level-sweep kernel (largest total device time) priced against
    its bound: MFMA peak of its arithmetic for the products, HBM for the
    gather.  achieved = algorithmic work per launch / mean launch duration."""
    groups = {}
    for l in ph["launches"]:
        groups.setdefault((l["cls"], l["tile"]), []).append(l)
    key = max(groups, key=lambda k: sum(l["ms"] for l in groups[k]))
    g = groups[key]
    raw = sum(l["ms"] for l in g) / len(g)
    ovh = ph.get("event_overhead_ms", 0.0)
    ms = max(raw - ovh, 0.5 * raw)
    mode = {"fp64": 0, "mixed_fp32": 1, "mixed_bf16x3": 2}[prec]
    T = "double" if prec == "fp64" else "float"
    sym = KERNEL_SYMBOL[key[0]].format(mode=mode, t=key[1], T=T)
    if key[0] == "gather":
        e = 8 if prec == "fp64" else 4
        work = sum(2 * e * l["elems"] for l in g) / len(g)  # read the source entry, write G
        achieved = work / (ms / 1e3) / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_GBS, "unit": "GB/s",
                "frac": achieved / HBM_GBS, "traffic": None, "kernel": sym, "launches": len(g),
                "mean_launch_ms": ms, "mean_event_interval_ms": raw, "event_overhead_ms": ovh,
                "bytes_per_launch": work}
    work = sum(l["flops"] for l in g) / len(g)
    achieved = work / (ms / 1e3) / 1e12
    return {"bound": "mfma", "achieved": achieved, "peak": PEAK[prec], "unit": "TFLOP/s",
            "frac": achieved / PEAK[prec], "traffic": None, "kernel": sym, "launches": len(g),
            "mean_launch_ms": ms, "mean_event_interval_ms": raw, "event_overhead_ms": ovh,
            "flops_per_launch": work}


def source_digest():
    """SHA-256 over the library's kernel and runtime sources (sorted by name)."""
    import hashlib
    d = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1708_04539_amd", "csrc")
    for name in sorted(os.listdir(src)):
        if name.endswith((".hip", ".hpp", ".cpp")):
            d.update(name.encode())
            with open(os.path.join(src, name), "rb") as f:
                d.update(f.read())
    return d.hexdigest()


def load_traffic(config, prec, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    profiles/traffic_<config>_<prec>.md (FETCH_SIZE and WRITE_SIZE per
    dispatch, scaled by a plain copy of known size).  None when there is no
    summary for this kernel or the sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{config}_{prec}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    try:
        if vals.get("kernel") != kernel or vals.get("source_sha256") != source_digest():
            return None
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mib):
    """A plain device-to-device copy of `mib` MiB, timed; the reference for
    scaling the FETCH_SIZE / WRITE_SIZE counters of the sweep kernels."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "ms": ms,
                      "GBps_read_plus_write": 2 * n * 8 / ms / 1e6}))


def cpu_baseline(w, budget_s):
    import numpy as np
    import oracle
    from oracle import Oracle
    oracle.build(force=False)
    threads = oracle.get_threads()
    o = Oracle(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, 0, w.pad_pct).factor(w.values)
    times = []
    t_start = time.perf_counter()
    sel = None
    while True:
        t0 = time.perf_counter()
        o.selinv()
        sel = o.get_selected()
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s or len(times) >= 10:
            break
    return o, sel, float(np.mean(times)), len(times), threads


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the library runs on one GPU only; multi-GPU sharding is a design note, "
                                   "not an implemented path", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1708_04539_amd.selinv import SelInv
    from workloads import get_config

    prec = args.precision or "fp64"
    w = get_config(args.config)
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()  # graphs cannot be captured on the legacy null stream
    t0 = time.perf_counter()
    symbolic = args.symbolic or ("exact" if args.config.startswith("u") else "symmetrized")
    cplx = bool(w.extra.get("complex"))
    s = SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct, symbolic=symbolic,
               complex_values=cplx)
    s.set_sweep_mode(args.sweep)
    t_an = time.perf_counter() - t0
    t0 = time.perf_counter()
    s.factor(w.values)
    t_fa = time.perf_counter() - t0
    info = s.info
    F = info["flops"]
    out = torch.empty(w.nnz, dtype=torch.complex128 if cplx else torch.float64, device="cuda")
    graph = not args.no_graph

    # autotuner (setup, untimed): launch choices measured on this device
    tuning = {"tuned": False}
    precs = [prec] + ([args.mixed] if args.mixed and args.mixed != prec else [])
    if not args.no_tune:
        from paper_1708_04539_amd.autotune import describe
        t0 = time.perf_counter()
        for p in precs:
            ms_pol, ms_tun = s.tune(p, args.tune_reps, stream)
            tuning[p] = dict(describe(s.get_tuning(p)), ms_policy_graph=ms_pol, ms_tuned_graph=ms_tun)
        tuning["tuned"] = True
        tuning["tune_s"] = time.perf_counter() - t0

    dev_s, wall_s = timed_steps(s, prec, args.steps, args.warmup, graph, out, stream)
    ms = 1e3 * dev_s / args.steps
    value = F / (dev_s / args.steps) / 1e9
    sel_main = out.cpu().numpy()

    # mixed form on the same matrix
    mixed = None
    if args.mixed and args.mixed != prec:
        mdev, _ = timed_steps(s, args.mixed, args.steps, args.warmup, graph, out, stream)
        mixed = {"precision": args.mixed, "ms_per_matrix": 1e3 * mdev / args.steps,
                 "gflops": F / (mdev / args.steps) / 1e9}
        sel_mixed = out.cpu().numpy()

    ph = phase_profile(s, prec, stream)
    roof = roofline(ph, prec)
    traffic = load_traffic(args.config, prec, roof["kernel"])
    roof["traffic"] = traffic
    roof["traffic_unit"] = "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)"

    res = {
        "metric": "selinv GFLOP/s & ms/matrix, mixed vs FP64 on 1 MI355X at stated max rel err",
        "value": value,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_matrix": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else ("f32" if prec == "mixed_fp32" else "bf16x3/f32"),
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "n": w.n, "nnz": w.nnz, "precision": prec,
                   "symbolic": symbolic, "nnz_lu": info["nnz_lu"],
                   "complex": "real form of order 2n: GFLOP counts the real form's flops, twice those of "
                              "native complex arithmetic" if cplx else False,
                   "supernodes": info["nsuper"], "levels": info["nlevels"], "gflop": F / 1e9,
                   "hip_graph": graph, "sweep": "persistent" if s.sweep_is_persistent(prec) == 1 else "levels",
                   "parallelism": "single GPU"},
        "wall_s_timed": wall_s,
        "setup_s": {"analyze": t_an, "factor_host_lu_and_h2d": t_fa, "tune": tuning.get("tune_s", 0.0)},
        "tuning": tuning,
        "phases_ms": {k: v for k, v in ph.items() if k.endswith("_ms") and k != "event_overhead_ms"},
        "phase_note": "phases from HIP events around each launch class in separate eager runs",
        "roofline": roof,
    }
    if mixed:
        res["mixed"] = mixed
        res["mixed_speedup_vs_main"] = ms / mixed["ms_per_matrix"]

    # LU factorisation on the device (setup, not part of a step): first call
    # (work lists built and uploaded) and the mean of repeats, then one run on
    # its factors against the run on the host factors
    if not args.no_device_lu:
        dvals = torch.from_numpy(np.ascontiguousarray(w.values)).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.factor_device(dvals, stream)
        t_first = time.perf_counter() - t0
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            s.factor_device(dvals, stream)
        t_dev = (time.perf_counter() - t0) / reps
        with torch.cuda.stream(stream):
            s.run(prec, stream)
            s.get_selected_device(out, stream)
        stream.synchronize()
        sel_dev = out.cpu().numpy()
        res["device_lu"] = {"ms": 1e3 * t_dev, "first_call_s": t_first,
                            "host_lu_and_h2d_ms": 1e3 * t_fa,
                            "max_rel_diff_vs_host_lu": float(np.abs(sel_dev - sel_main).max()
                                                             / np.abs(sel_main).max()),
                            "note": "wall clock of selinv_factor_device (values resident in HBM; ends with "
                                    "a stream synchronisation), mean of %d calls" % reps}

    if not args.no_cpu_baseline and args.config in ("c0", "c1", "u1"):
        o, sel_ref, t_cpu, reps, threads = cpu_baseline(w, args.cpu_seconds)
        res["cpu_baseline"] = {"value": F / t_cpu / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
                               "sample": f"full matrix, oracle steps 2-6 (selected inversion + extraction), "
                                         f"mean of {reps} runs, {t_cpu * 1e3:.1f} ms each"}
        scale = np.abs(sel_ref).max()
        res["max_rel_err"] = {prec: float(np.abs(sel_main - sel_ref).max() / scale)}
        if mixed:
            res["max_rel_err"][args.mixed] = float(np.abs(sel_mixed - sel_ref).max() / scale)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
