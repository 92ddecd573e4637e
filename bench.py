#!/usr/bin/env python3
"""Benchmark: supernodal selected inversion on one MI355X.

One step = one pass of the whole hot path over one matrix whose factors are
already in HBM: diagonal-block inversion, normalisation, then the level sweep
(gather, products of steps 3 and 5, product of step 4) and the extraction of
the selected entries into a device buffer.  Throughput is algorithmic GFLOP/s
(flop convention: F_K = 4 s cL cU + 2 s^2 cU + s^2 (cL + cU) + 4/3 s^3 per
supernode, the same for every precision) over the timed steps.

Default workload: 3D 64^3 27-point asymmetric stencil (n = 262,144), nested
dissection, supernodes <= 512, in FP64 (the headline value); the split-BF16
and FP32 mixed forms run on the same matrix and are reported beside it with
their speed-up over FP64.  Errors are measured against columns of A^{-1}
solved from the definition, over every computed entry of those columns.

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

# MI355X published dense peaks (TFLOP/s) of the arithmetic each form's
# products run on; split-BF16 issues three BF16 MFMA products per useful one
PEAK_TF = {"fp64": 78.6, "mixed_fp32": 157.3, "mixed_bf16x3": 2500.0}
HBM_GBS = 8000.0
FORMS = ["fp64", "mixed_fp32", "mixed_bf16x3"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c4", choices=["c0", "c1", "c2", "c3", "c4", "u1", "u4", "z1"])
    ap.add_argument("--symbolic", default=None, choices=["symmetrized", "exact"],
                    help="analysis form (default: symmetrized for c*, exact for the upwind u* configs)")
    ap.add_argument("--precision", default="fp64", help="form of the headline value")
    ap.add_argument("--mixed", default="mixed_bf16x3,mixed_fp32",
                    help="forms timed beside the headline one (comma list; empty: none)")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--sweep", default="auto", choices=["auto", "levels", "persistent"])
    ap.add_argument("--no-tune", action="store_true", help="size policy instead of the autotuner's choices")
    ap.add_argument("--tune-reps", type=int, default=5)
    ap.add_argument("--tuning-cache", default=None,
                    help="JSON cache of tuning tables (read if present, else tuned and written)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-device-lu", action="store_true", help="skip timing the LU on the device (setup)")
    ap.add_argument("--no-errors", action="store_true", help="skip the error measurement")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="bound on the oracle's CPU time")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for scaling HBM counters) and exit")
    return ap.parse_args()


WORKLOADS = {
    "c0": "2D 32x32 5-point asymmetric convection-diffusion, n=1024, ND, supernodes<=32",
    "c1": "2D 256x256 9-point asymmetric stencil, n=65536, ND, supernodes<=128",
    "c2": "3D 48^3 7-point asymmetric convection-diffusion, n=110592, ND, supernodes<=256",
    "c3": "batch of 32 2D 5-point asymmetric convection-diffusion matrices, grid sides uniform in 64..256 "
          "(n 4k..64k), ND, supernodes<=128, one level-batched sweep",
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
    """Per-launch device times from HIP events recorded on the run's stream
    (eager runs with profiling on), with the algorithmic work of each launch
    (selinv_level_stats).  Returns per-class totals and the launch list."""
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
    pro = s.level_stats(-1)
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
    bulk = PEAK_TF[prec]
    launches = [
        {"cls": "tri", "tile": 0, "level": -1, "ms": float(t[0]), "flops": pro["tri_flops"],
         "bytes": pro["tri_bytes"], "peak_tf": PEAK_TF["fp64"]},
        {"cls": "norm", "tile": 0, "level": -1, "ms": float(t[1]), "flops": pro["norm_flops"],
         "bytes": pro["norm_bytes"], "peak_tf": PEAK_TF["fp64"] if prec == "fp64" else bulk},
    ]
    if prec != "fp64":
        launches.append({"cls": "dt", "tile": 0, "level": -1, "ms": float(t[2]), "flops": pro["dt_flops"],
                         "bytes": pro["dt_bytes"], "peak_tf": PEAK_TF["fp64"]})
    for d in range(L):
        if lev[d]["small_count"] > 0:
            launches.append({"cls": "small", "tile": 64, "level": d, "ms": float(t[3 + 4 * d]),
                             "flops": lev[d]["small_flops"], "bytes": lev[d]["bytes_small"], "peak_tf": bulk})
        if lev[d]["gather_tiles"] > 0:
            launches.append({"cls": "gather", "tile": 64, "level": d, "ms": float(t[4 + 4 * d]), "flops": 0.0,
                             "bytes": lev[d]["bytes_gather"], "peak_tf": bulk})
        if lev[d]["tiles35"] > 0:
            # gather_fused == 2: the level's products read G_K from its sources (gemm_g35)
            cls35 = "gemm35g" if lev[d]["gather_fused"] == 2 else "gemm35"
            launches.append({"cls": cls35, "tile": int(lev[d]["tile35"]), "level": d,
                             "ms": float(t[5 + 4 * d]), "flops": lev[d]["flops35"], "bytes": lev[d]["bytes35"],
                             "peak_tf": bulk, "max_prod_flops": lev[d]["max_prod_flops"]})
        if lev[d]["tiles4"] > 0:
            launches.append({"cls": "gemm4", "tile": int(lev[d]["tile4"]), "level": d, "ms": float(t[6 + 4 * d]),
                             "flops": lev[d]["flops4"], "bytes": lev[d]["bytes4"], "peak_tf": bulk})
    ph["launches"] = launches
    return ph


KERNEL_SYMBOL = {
    # (class, precision, tile) -> kernel symbol as rocprofv3 prints it
    "gemm35": "selinv::gemm_v2<{mode}, {t}, {t}, {T}, {T}, 1>",
    "gemm35g": "selinv::gemm_g35<{mode}, {t}, {t}, {T}>",
    "gemm4": "selinv::step4_gather<{mode}, {t}, {t}, {T}>",
    "gather": "selinv::gather_kernel<{T}>",
    "small": "selinv::small_kernel<{mode}>",
    "tri": "selinv::tri_base_kernel<4> (+ doubling rounds)",
    "norm": "selinv::gemm_v2<{pm}, *, *, double, {T}, 0>",
    "dt": "selinv::gemm_v2<0, *, *, double, double, 0>",
}


def price(g, ovh, hbm_gbs=HBM_GBS):
    """One launch class priced against its roofline: per launch, the time
    its algorithmic flops need at the MFMA peak and the time its algorithmic
    bytes need at the HBM peak; the larger names the bound."""
    raw = sum(l["ms"] for l in g) / len(g)
    ms = max(raw - ovh, 0.5 * raw)
    F = sum(l["flops"] for l in g) / len(g)
    B = sum(l["bytes"] for l in g) / len(g)
    peak = g[0]["peak_tf"]
    t_f = F / (peak * 1e12)
    t_b = B / (hbm_gbs * 1e9)
    if t_f >= t_b:
        achieved = F / (ms / 1e3) / 1e12
        return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "mean_launch_ms": ms, "mean_event_interval_ms": raw, "flops_per_launch": F,
                "bytes_per_launch": B, "intensity_flop_per_byte": F / B if B else None}
    achieved = B / (ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": hbm_gbs, "unit": "GB/s", "frac": achieved / hbm_gbs,
            "mean_launch_ms": ms, "mean_event_interval_ms": raw, "flops_per_launch": F, "bytes_per_launch": B,
            "intensity_flop_per_byte": F / B if B else None}


def roofline(ph, prec):
    """The dominant launch class (largest total device time, prologue classes
    included) priced against its bound."""
    groups = {}
    for l in ph["launches"]:
        if l["ms"] > 0:
            groups.setdefault((l["cls"], l["tile"]), []).append(l)
    key = max(groups, key=lambda k: sum(l["ms"] for l in groups[k]))
    g = groups[key]
    ovh = ph.get("event_overhead_ms", 0.0)
    mode = {"fp64": 0, "mixed_fp32": 1, "mixed_bf16x3": 2}[prec]
    T = "double" if prec == "fp64" else "float"
    r = price(g, ovh)
    r.update({"traffic": None, "class": key[0],
              "kernel": KERNEL_SYMBOL[key[0]].format(mode=mode, t=key[1], T=T, pm=0 if prec == "fp64" else 3),
              "launches": len(g), "event_overhead_ms": ovh,
              "class_total_ms": sum(l["ms"] for l in g)})
    return r


def largest_product(ph, prec):
    """The steps-3/5 launch of the level that holds the largest single
    supernode product: its useful rate and, for split-BF16, the rate of the
    BF16 products it issues (three per useful product)."""
    g35 = [l for l in ph["launches"] if l["cls"] in ("gemm35", "gemm35g")]
    if not g35:
        return None
    l = max(g35, key=lambda x: (x["max_prod_flops"], x["flops"]))
    ms = max(l["ms"] - ph.get("event_overhead_ms", 0.0), 0.5 * l["ms"])
    useful = l["flops"] / (ms / 1e3) / 1e12
    out = {"level": l["level"], "launch_ms": ms, "launch_flops": l["flops"],
           "largest_product_flops": l["max_prod_flops"], "useful_tflops": useful,
           "useful_frac_of_peak": useful / PEAK_TF[prec] if prec != "mixed_bf16x3" else None}
    if prec == "mixed_bf16x3":
        out["issued_bf16_tflops"] = 3 * useful
        out["issued_frac_of_bf16_peak"] = 3 * useful / PEAK_TF[prec]
    return out


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


def column_entries(st, r):
    """Columns c of the computed entries At^{-T}(r, c) in row r of the block
    pattern: the columns of sup(r), R_U(sup(r)), and the columns of every
    supernode J with r in R_L(J)."""
    import numpy as np
    xsup, rlp, rl, rup, ru = st["xsup"], st["rl_ptr"], st["rl"], st["ru_ptr"], st["ru"]
    K = int(np.searchsorted(xsup, r, side="right") - 1)
    parts = [np.arange(xsup[K], xsup[K + 1]), ru[rup[K]:rup[K + 1]]]
    for J in np.searchsorted(rlp, np.nonzero(rl == r)[0], side="right") - 1:
        parts.append(np.arange(xsup[J], xsup[J + 1]))
    return np.concatenate(parts).astype(np.int64)


def reference_columns_complex(s, w):
    """As reference_columns for a complex matrix (held in its real form of
    order 2n): columns of A^{-1} solved from the definition with a sparse
    complex LU and refinement (oracle.complex_ref); the computed entries of
    complex column j are the nodes of the real form's computed entries in row
    q[2j]."""
    import numpy as np
    from oracle.complex_ref import solve_columns
    st = s.structure()
    xsup, lev, cl = st["xsup"], st["level"], np.diff(st["rl_ptr"])
    ns = len(xsup) - 1
    rows = [int(xsup[ns - 1]), int(xsup[ns]) - 2]
    for d in (int(lev.max()) // 2, int(lev.max())):
        ks = np.nonzero(lev == d)[0]
        rows.append(int(xsup[ks[np.argmax(cl[ks])]]))
    perm = st["perm"].astype(np.int64)
    js = [int(perm[r]) // 2 for r in rows]
    out = []
    for r, j, x in zip(rows, js, solve_columns(w.n, w.colptr, w.rowind, w.values, js)):
        i = np.unique(perm[column_entries(st, r)] // 2)
        out.append((j, i, x[i], float("nan")))
    return out


def reference_columns(s, w):
    """Error reference at full size: a few columns of A^{-1} solved from the
    definition A x = e_j (oracle.sampled, certified bounds): the first and last
    column of the root supernode, and the first column of the supernode with
    the largest |R_L| on the middle and on the deepest level.  Returns
    [(j, rows i of the computed entries of column j, A^{-1}(i, j))]."""
    import numpy as np
    from oracle.sampled import solve_columns
    st = s.structure()
    xsup, lev, cl = st["xsup"], st["level"], np.diff(st["rl_ptr"])
    ns = len(xsup) - 1
    rows = [int(xsup[ns - 1]), int(xsup[ns]) - 1]
    for d in (int(lev.max()) // 2, int(lev.max())):
        ks = np.nonzero(lev == d)[0]
        rows.append(int(xsup[ks[np.argmax(cl[ks])]]))
    perm = st["perm"].astype(np.int64)
    js = [int(perm[r]) for r in rows]
    out = []
    for r, j, (x, bound) in zip(rows, js, solve_columns(w.to_scipy(), js)):
        i = perm[column_entries(st, r)]
        out.append((j, i, x[i], bound))
    return out


def cpu_baseline(config, budget_s, w_full):
    """The oracle (steps 2-6: selected inversion and extraction) timed on the
    host cores.  Full matrix for the 2D configurations; for the 3D ones a
    smaller grid of the same recipe, so that the leg stays within about
    budget_s seconds of CPU work."""
    import numpy as np
    import oracle
    from oracle import Oracle
    from paper_1708_04539_amd.selinv import SelInv
    from workloads import config_grid, get_config
    oracle.build(force=False)
    threads = oracle.get_threads()
    if config in ("c4", "u4"):
        w = config_grid("c4-sample", (40, 40, 40), "box", "sym_perturbed", 0.1, 0, 512, 64, delta=0.15)
        sample = "40^3 27-point stencil of the 64^3 recipe (n=64000, supernodes<=512)"
    elif config == "c2":
        w = config_grid("c2-sample", (32, 32, 32), "star", "convection", 0.1, None, 256, 64)
        sample = "32^3 7-point stencil of the 48^3 recipe (n=32768, supernodes<=256)"
    else:
        w = w_full
        sample = "full matrix"
    F = SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct).info["flops"]
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
    t = float(np.mean(times))
    return {"value": F / t / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample}: oracle steps 2-6 (selected inversion + extraction), {F / 1e9:.1f} GFLOP, "
                      f"mean of {len(times)} runs, {t * 1e3:.1f} ms each"}, (w, o, sel)


def bench_c3(args, prec, mixed_forms):
    """Batch of 32 matrices: one level-batched sweep (HIP graph, tuned per
    form) plus the extraction of every matrix's selected entries per step;
    the same matrices run one by one are timed beside it."""
    import numpy as np
    import torch
    from paper_1708_04539_amd.selinv import Batch, SelInv
    from workloads import config_c3

    ws = config_c3()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    mats = [SelInv(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, w.pad_pct).factor(w.values) for w in ws]
    t_setup = time.perf_counter() - t0
    b = Batch(mats)
    F = b.info["flops"]
    offs = np.concatenate([[0], np.cumsum([w.nnz for w in ws])])
    out = torch.empty(int(offs[-1]), dtype=torch.float64, device="cuda")
    views = [out[int(offs[k]):int(offs[k + 1])] for k in range(len(ws))]
    graph = not args.no_graph
    tuning = {"tuned": False}
    if not args.no_tune:
        from paper_1708_04539_amd.autotune import describe
        t0 = time.perf_counter()
        for p in [prec] + mixed_forms:
            ms_pol, ms_tun = b.tune(p, args.tune_reps, stream)
            tuning[p] = dict(describe(b.get_tuning(p)), ms_policy_graph=ms_pol, ms_tuned_graph=ms_tun)
        tuning["tuned"] = True
        tuning["tune_s"] = time.perf_counter() - t0

    class Step:  # one step: the batched sweep and every matrix's extraction
        def __init__(self):
            self.info = b.info

        def run(self, p, stream=None, graph=False):
            b.run(p, stream=stream, graph=graph)

        def get_selected_device(self, _out, stream=None):
            for m, v in zip(mats, views):
                m.get_selected_device(v, stream=stream)

    st = Step()
    forms = {}
    for p in [prec] + mixed_forms:
        dev, wall = timed_steps(st, p, args.steps, args.warmup, graph, out, stream)
        forms[p] = {"ms_per_batch": 1e3 * dev / args.steps, "ms_per_matrix": 1e3 * dev / args.steps / len(ws),
                    "gflops": F / (dev / args.steps) / 1e9}
        if p == prec:
            wall_main = wall
        print(f"# {p}: {forms[p]['ms_per_matrix']:.4f} ms per matrix", file=sys.stderr, flush=True)
    ms = forms[prec]["ms_per_matrix"]
    for p in mixed_forms:
        forms[p]["speedup_vs_" + prec] = ms / forms[p]["ms_per_matrix"]
    # the same matrices one by one (each its own graph, tuned by the size policy)
    for m in mats:
        m.run(prec, stream=stream, graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        for m, v in zip(mats, views):
            m.run(prec, stream=stream, graph=True)
            m.get_selected_device(v, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1) / args.steps / len(ws)

    ph = phase_profile(b, prec, stream)
    roof = roofline(ph, prec)
    roof["traffic"] = load_traffic("c3", prec, roof["kernel"])
    roof["traffic_unit"] = "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)"
    forms[prec]["largest_product_launch"] = largest_product(ph, prec)
    for p in mixed_forms:
        php = phase_profile(b, p, stream)
        forms[p]["largest_product_launch"] = largest_product(php, p)
        forms[p]["roofline"] = roofline(php, p)
    res = {
        "metric": "selinv GFLOP/s & ms/matrix, mixed vs FP64 on 1 MI355X at stated max rel err",
        "value": forms[prec]["gflops"], "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": forms[prec]["ms_per_batch"], "ms_per_matrix": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else ("f32" if prec == "mixed_fp32" else "bf16x3/f32"),
        "data": "synthetic",
        "config": {"workload": WORKLOADS["c3"], "matrices": len(ws), "n_total": int(sum(w.n for w in ws)),
                   "nnz_total": int(offs[-1]), "precision": prec, "gflop": F / 1e9,
                   "aligned_levels": b.info["nlevels"], "hip_graph": graph, "parallelism": "single GPU"},
        "forms": forms,
        "unbatched_ms_per_matrix": ms_single,
        "batching_speedup": ms_single / ms,
        "wall_s_timed": wall_main,
        "setup_s": {"analyze_and_host_lu": t_setup, "tune": tuning.get("tune_s", 0.0)},
        "tuning": tuning,
        "roofline": roof,
    }
    if mixed_forms:
        best = max(mixed_forms, key=lambda p: forms[p]["gflops"])
        res["mixed_best"] = best
        res["mixed_speedup_vs_fp64"] = forms[best]["speedup_vs_" + prec] if prec == "fp64" else None
    if not args.no_cpu_baseline:
        print("# cpu baseline", file=sys.stderr, flush=True)
        import oracle
        from oracle import Oracle
        oracle.build(force=False)
        done, t_cpu, f_cpu, refs = 0, 0.0, 0.0, []
        for k, w in enumerate(ws):  # matrices in order while the budget lasts
            o = Oracle(w.n, w.colptr, w.rowind, w.perm, w.max_super, w.relax, 0, w.pad_pct).factor(w.values)
            t0 = time.perf_counter()
            o.selinv()
            refs.append(o.get_selected())
            t_cpu += time.perf_counter() - t0
            f_cpu += mats[k].info["flops"]
            done += 1
            o.close()
            if t_cpu > args.cpu_seconds:
                break
        res["cpu_baseline"] = {"value": f_cpu / t_cpu / 1e9, "unit": "GFLOP/s", "cores": oracle.get_threads(),
                               "kind": "oracle",
                               "sample": f"the first {done} of the 32 matrices, one oracle pass each (steps 2-6), "
                                         f"{f_cpu / 1e9:.2f} GFLOP in {t_cpu:.1f} s"}
        if not args.no_errors:
            errs = {}
            for p in [prec] + mixed_forms:
                b.run(p, stream=stream, graph=graph)
                e = 0.0
                for k in range(done):
                    got = mats[k].get_selected()
                    e = max(e, float(np.abs(got - refs[k]).max() / np.abs(refs[k]).max()))
                errs[p] = e
            res["max_rel_err"] = errs
            res["max_rel_err_on"] = f"every selected entry of the first {done} matrices, against the FP64 oracle"
    print(json.dumps(res))


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

    prec = args.precision
    mixed_forms = [m for m in args.mixed.split(",") if m and m != prec]
    for p in [prec] + mixed_forms:
        if p not in FORMS:
            raise SystemExit(f"unknown form {p}")
    if args.config == "c3":
        return bench_c3(args, prec, mixed_forms)
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
    print(f"# setup: analyze {t_an:.1f} s, host LU + H2D {t_fa:.1f} s", file=sys.stderr, flush=True)

    # autotuner (setup, untimed): launch choices measured on this device
    tuning = {"tuned": False}
    if not args.no_tune:
        from paper_1708_04539_amd.autotune import describe, tuned
        t0 = time.perf_counter()
        for p in [prec] + mixed_forms:
            r = tuned(s, p, args.tuning_cache, reps=args.tune_reps, stream=stream)
            tuning[p] = dict(describe(r["table"]), ms_policy_graph=r["ms_policy"], ms_tuned_graph=r["ms_tuned"],
                             cached=r["cached"])
        tuning["tuned"] = True
        tuning["tune_s"] = time.perf_counter() - t0
        print(f"# tuned in {tuning['tune_s']:.1f} s", file=sys.stderr, flush=True)

    dev_s, wall_s = timed_steps(s, prec, args.steps, args.warmup, graph, out, stream)
    ms = 1e3 * dev_s / args.steps
    value = F / (dev_s / args.steps) / 1e9
    sel_main = out.cpu().numpy()
    print(f"# {prec}: {ms:.3f} ms per matrix", file=sys.stderr, flush=True)

    forms = {prec: {"ms_per_matrix": ms, "gflops": value}}
    for p in mixed_forms:
        mdev, _ = timed_steps(s, p, args.steps, args.warmup, graph, out, stream)
        forms[p] = {"ms_per_matrix": 1e3 * mdev / args.steps, "gflops": F / (mdev / args.steps) / 1e9,
                    "speedup_vs_" + prec: ms / (1e3 * mdev / args.steps)}
        print(f"# {p}: {forms[p]['ms_per_matrix']:.3f} ms per matrix", file=sys.stderr, flush=True)

    # roofline of the dominant launch class, and the rate of the launch that
    # holds the largest supernode product, per form
    ph = phase_profile(s, prec, stream)
    roof = roofline(ph, prec)
    traffic = load_traffic(args.config, prec, roof["kernel"])
    roof["traffic"] = traffic
    roof["traffic_unit"] = "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)"
    forms[prec]["largest_product_launch"] = largest_product(ph, prec)
    forms[prec]["phases_ms"] = {k: v for k, v in ph.items() if k.endswith("_ms") and k != "event_overhead_ms"}
    for p in mixed_forms:
        php = phase_profile(s, p, stream)
        forms[p]["largest_product_launch"] = largest_product(php, p)
        forms[p]["phases_ms"] = {k: v for k, v in php.items() if k.endswith("_ms") and k != "event_overhead_ms"}
        forms[p]["roofline"] = roofline(php, p)

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
                   "largest_product_mnk": [info["max_gemm_m"], info["max_gemm_n"], info["max_gemm_k"]],
                   "hip_graph": graph, "sweep": "persistent" if s.sweep_is_persistent(prec) == 1 else "levels",
                   "parallelism": "single GPU"},
        "forms": forms,
        "wall_s_timed": wall_s,
        "setup_s": {"analyze": t_an, "factor_host_lu_and_h2d": t_fa, "tune": tuning.get("tune_s", 0.0)},
        "tuning": tuning,
        "phase_note": "phases from HIP events around each launch class in separate eager runs",
        "roofline": roof,
    }
    if mixed_forms:
        best = max(mixed_forms, key=lambda p: forms[p]["gflops"])
        res["mixed_best"] = best
        res["mixed_speedup_vs_fp64"] = forms[best]["speedup_vs_" + prec] if prec == "fp64" else None

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
        s.factor(w.values)  # back to the host factors for the error measurement

    # CPU baseline and error reference (the only leg that uses the oracle)
    if not args.no_cpu_baseline and cplx:
        # the supernodal oracle is real: complex matrices are checked against
        # columns from the definition and have no CPU-baseline timing
        if not args.no_errors:
            cols = reference_columns_complex(s, w)
            errs = {}
            for p in [prec] + mixed_forms:
                s.run(p, stream=stream, graph=graph)
                X = np.concatenate([s.get_many(i, np.full(len(i), j)) for j, i, _, _ in cols])
                R = np.concatenate([c[2] for c in cols])
                D = np.concatenate([c[1] == c[0] for c in cols])
                en = np.abs(X - R).max() / np.abs(R).max()
                ed = (np.abs(X[D] - R[D]) / np.abs(R[D])).max()
                errs[p] = float(max(en, ed))
            res["max_rel_err"] = errs
            res["max_rel_err_on"] = (f"every computed entry of {len(cols)} complex columns of A^-1 "
                                     f"({sum(len(c[1]) for c in cols)} entries) against sparse complex LU "
                                     f"solves with refinement; max(err_norm, err_diag)")
    elif not args.no_cpu_baseline:
        print("# cpu baseline", file=sys.stderr, flush=True)
        cb, (wo, o, sel_ref) = cpu_baseline(args.config, args.cpu_seconds, w)
        res["cpu_baseline"] = cb
        if not args.no_errors:
            errs = {}
            if wo is w:  # full-matrix oracle: every selected entry
                scale = np.abs(sel_ref).max()
                for p in [prec] + mixed_forms:
                    s.run(p, stream=stream, graph=graph)
                    got = s.get_selected()
                    errs[p] = float(np.abs(got - sel_ref).max() / scale)
                res["max_rel_err"] = errs
                res["max_rel_err_on"] = "every selected entry (A(j,i) != 0), against the supernodal FP64 oracle"
            else:
                cols = reference_columns(s, w)
                for p in [prec] + mixed_forms:
                    s.run(p, stream=stream, graph=graph)
                    X, R, D = [], [], []
                    for j, i, ref, _ in cols:
                        X.append(s.get_many(i, np.full(len(i), j)))
                        R.append(ref)
                        D.append(i == j)
                    X, R, D = np.concatenate(X), np.concatenate(R), np.concatenate(D)
                    en = np.abs(X - R).max() / np.abs(R).max()
                    ed = (np.abs(X[D] - R[D]) / np.abs(R[D])).max()
                    errs[p] = float(max(en, ed))
                res["max_rel_err"] = errs
                res["max_rel_err_on"] = (f"every computed entry of {len(cols)} columns of A^-1 "
                                         f"({sum(len(c[1]) for c in cols)} entries: root supernode first and last "
                                         f"column, widest supernode of the middle and deepest level), against "
                                         f"A x = e_j solved in extended precision (error bound "
                                         f"{max(c[3] for c in cols):.1e}); max(err_norm, err_diag)")
    print(json.dumps(res))


if __name__ == "__main__":
    main()
