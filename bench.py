#!/usr/bin/env python3
"""PDHG iterations per second on one MI355X.

Workload (default, --workload block_angular): a plain PDHG solve to
eps_rel = 1e-4 of the block-angular LP (64 diagonal blocks 30,000 x 120,000
with 6 nonzeros per column, plus 2,000 linking rows of 1,200 nonzeros drawn
over all columns: m = 1,922,000, n = 7,680,000, about 48.5M nonzeros, values
N(0,1), planted optimum), float32 iterates with float64 SpMV sums, float64
termination tests on the original model.  It is the one workload whose
matrix does not fit the 256 MB last-level cache, so its kernels are the ones
HBM bandwidth bounds.  One step is one whole solve from device-resident
inputs: validation, scaling, power iteration, the iterations, and the final
evaluation.  value = iterations / second over the K timed steps.
--workload power_law puts the 3.2M-nonzero power-law LP on the main line.

Also reported, on the same JSON line:
  roofline          the slower iteration kernel's algorithmic bytes per launch
                    over its mean launch time (HIP events on the solver's
                    stream around 256 back-to-back launches), against MI355X's
                    8 TB/s HBM peak; traffic = measured HBM-side bytes per
                    launch from the committed counter record, while the kernel
                    sources match it;
  cpu_baseline      the float64 NumPy/SciPy oracle on the host, single thread,
                    on a bounded sample of the same workload;
  power_law, tolerance_ratios, differentiation, batched, general, ipm_hybrid:
                    the other workloads (see their docstrings below), each
                    with its error against the float64 oracle or the
                    closed-form optimum.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "power_law": ("power-law LP m=100000 n=400000 (~3.2M nnz, column counts k^-2.1423 on [2,2000], "
                  "N(0,1) x row factor U(0.1,10), planted optimum), plain PDHG, FP32 iterates, "
                  "FP64 termination tests, eps_rel=1e-4"),
    "block_angular": ("block-angular LP m=1922000 n=7680000 (64 blocks 30000x120000 with 6 nnz/col, "
                      "2000 link rows x 1200 nnz, ~48.5M nnz, planted optimum), plain PDHG, FP32 iterates, "
                      "FP64 termination tests, eps_rel=1e-4"),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16", "fp32acc32", "fp32a"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-iters", type=int, default=1024,
                    help="iterations of the per-kernel HIP-event timing leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-LP leg")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--plain-sample", type=int, default=32,
                    help="instances of the batch solved one at a time by the plain FP64 path")
    ap.add_argument("--no-other", action="store_true",
                    help="skip the leg of the workload that is not on the main line")
    ap.add_argument("--no-ratios", action="store_true", help="skip the tolerance-ratio leg")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiation leg")
    ap.add_argument("--no-general", action="store_true", help="skip the general-form LP leg")
    ap.add_argument("--no-ipm", action="store_true", help="skip the PDHG / interior-point hybrid leg")
    ap.add_argument("--profile", action="store_true",
                    help="only a short capped solve (256 iterations) of --workload (for hardware counters)")
    ap.add_argument("--shape", default="",
                    help="SpMV shape instead of the autotuner's, e.g. spmv_kind=0,tile_nnz=4096,tile_rows=512,short_row=-1")
    ap.add_argument("--workload", default="block_angular", choices=["power_law", "block_angular", "batched"],
                    help="LP of the main line (the other one runs as a leg); batched: only with --counter-summary")
    ap.add_argument("--infeas-tol", type=float, default=None,
                    help="infeasibility-certificate tolerance of the main-line solves (default: the library's)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only a plain device copy and a streaming read of known sizes (to calibrate hardware "
                         "byte counters)")
    ap.add_argument("--profile-batched", action="store_true",
                    help="only one batched solve of the 4,096-LP workload (for hardware counters)")
    ap.add_argument("--counter-summary", default="",
                    help="no GPU: write profiles/traffic_<workload>.json and the profile summary of --workload "
                         "from the rocprofv3 outputs under this folder (see counter_summary)")
    return ap.parse_args()


def cpu_baseline(lp, gpu_iters: int, eps: float) -> dict:
    """The oracle as it stands, one thread, on a bounded sample (about 10 s of
    CPU work on the power-law LP): two runs capped at 128 and 768 iterations
    give its setup time and per-iteration time; the rate is quoted for a
    solve of the GPU's iteration count."""
    import oracle
    from oracle.pdhg import OracleOptions
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    times = {}
    ctx = threadpool_limits(1) if threadpool_limits else None
    if ctx:
        ctx.__enter__()
    try:
        for n in (128, 768):
            t0 = time.perf_counter()
            oracle.solve(lp.A, lp.AT, lp.b, lp.c, eps, opts=OracleOptions(max_iter=n))
            times[n] = time.perf_counter() - t0
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    per_iter = (times[768] - times[128]) / 640.0
    setup = max(0.0, times[128] - 128 * per_iter)
    value = gpu_iters / (setup + gpu_iters * per_iter)
    return {"value": value, "unit": "iter/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle capped at 128 and 768 iterations on the same LP: setup {setup:.2f} s, "
                       f"{per_iter * 1e3:.1f} ms/iteration, rate quoted for a {gpu_iters}-iteration solve")}


def cpu_baseline_block_angular(gpu_iters: int, eps: float, seed: int) -> dict:
    """The oracle as it stands, one thread, over the first 100 iterations of
    a 1/16 sample of the block-angular LP: 4 blocks of the same shape and
    density and 125 linking rows of 1,200 nonzeros (3.03M nonzeros, the same
    structure per nonzero).  Two runs (capped at 2 and 100 iterations) split
    its setup (validation, scaling, power iteration) from its time per
    iteration; both are scaled by the ratio of nonzeros to the full LP (the
    oracle's work is linear in them) and the rate is quoted for a solve of
    the GPU's iteration count.  About 20 s of CPU work; the full LP's setup
    alone takes the oracle over two minutes."""
    import lpgen
    import oracle
    from oracle.pdhg import OracleOptions
    from threadpoolctl import threadpool_limits
    full_nnz = 64 * 120_000 * 6 + 2_000 * 1_200
    lp = lpgen.cfg3(seed, nblocks=4, nlink=125)
    times = {}
    with threadpool_limits(1):
        for n in (2, 100):
            t0 = time.perf_counter()
            oracle.solve(lp.A, lp.AT, lp.b, lp.c, eps, opts=OracleOptions(max_iter=n))
            times[n] = time.perf_counter() - t0
    per_iter = (times[100] - times[2]) / 98.0
    setup = max(0.0, times[2] - 2 * per_iter)
    r = full_nnz / lp.nnz
    value = gpu_iters / (r * setup + gpu_iters * r * per_iter)
    return {"value": value, "unit": "iter/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle on a 1/16 block-angular LP (4 blocks, 125 link rows, {lp.nnz} nnz), runs capped "
                       f"at 2 and 100 iterations: setup {setup:.2f} s, {per_iter * 1e3:.1f} ms/iteration, both "
                       f"scaled by {r:.2f} (nonzeros of the full LP), rate quoted for a {gpu_iters}-iteration "
                       f"solve")}


KERNEL_SOURCES = ("paper_2603_03150_amd/csrc/common.h", "paper_2603_03150_amd/csrc/plain.h",
                  "paper_2603_03150_amd/csrc/plain.hip", "paper_2603_03150_amd/csrc/panel.h",
                  "paper_2603_03150_amd/csrc/panel.hip")
PANEL_DUAL = "k_panel_spmv+k_panel_rows<dual>"


def kernel_names(shape: dict) -> dict:
    """Names of the kernels of one primal and one dual step for an SpMV
    shape; the panel layout's dual step is two kernels."""
    kind = int(shape.get("spmv_kind", 0))
    base = {0: "k_iter_tiled", 1: "k_iter", 2: "k_iter_persist", 3: "k_iter_tiled", 4: "k_rowpanel_primal"}[kind]
    return {"primal": f"{base}<primal>", "dual": PANEL_DUAL if kind >= 3 else f"{base}<dual>"}


def short_kernel(symbol: str):
    """The name kernel_names() uses for a kernel symbol of a profile (the
    panel kernels under their own names), or None for other kernels."""
    import re
    m = re.search(r"mip::(k_iter_tiled|k_iter_persist|k_iter|k_panel_spmv|k_panel_rows|k_rowpanel_primal)<([^()]*)>",
                  symbol)
    if not m:
        return None
    name, targs = m.group(1), [t.strip() for t in m.group(2).split(",")]
    if name.startswith("k_panel"):
        return name
    if name == "k_rowpanel_primal":
        return "k_rowpanel_primal<primal>"
    primal = targs[4 if name == "k_iter" else 3] == "true"
    return f"{name}<{'primal' if primal else 'dual'}>"


BATCHED_SOURCES = ("paper_2603_03150_amd/csrc/common.h", "paper_2603_03150_amd/csrc/inst_common.h",
                   "paper_2603_03150_amd/csrc/batched.hip")


def kernel_source_sha(sources=KERNEL_SOURCES) -> str:
    """Hash of the sources that define the iteration kernels: a stored
    hardware-counter record is used only while they are unchanged."""
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def batched_traffic_record(split: int):
    """Measured HBM bytes of the batched launch on the 4,096-LP workload,
    from profiles/traffic_batched.json, or None if there is none, or the
    batched kernel's sources or the launch split differ from its own."""
    path = os.path.join(ROOT, "profiles", "traffic_batched.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != kernel_source_sha(BATCHED_SOURCES) or rec.get("batch_split") != split:
        return None
    return rec


def traffic_record(workload_key: str, kernel: str, shape: dict):
    """Measured HBM bytes per launch of `kernel` on `workload_key`, from the
    committed counter summary (profiles/traffic_<workload_key>.json), or None
    if there is none, or the kernel sources or the kernel's side of the SpMV
    shape differ from the ones it was taken with."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_key}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    # the kernel's own side of the shape: A's tiles (or panels) for the dual, A^T's tiles for the primal
    if kernel.startswith("k_rowpanel_primal"):
        side = ("spmv_kind", "panel_width")
    elif kernel.endswith("<primal>"):
        side = ("spmv_kind", "tile_nnz_at", "tile_rows_at", "short_row_at")
    elif kernel == PANEL_DUAL:
        side = ("spmv_kind", "panel_width")
    else:
        side = ("spmv_kind", "tile_nnz", "tile_rows", "short_row")
    stored = rec.get("spmv_shape", {})
    if (rec.get("source_sha256") != kernel_source_sha() or kernel not in rec.get("kernels", {})
            or any(stored.get(k, 0) != shape.get(k, 0) for k in side)):
        return None
    return rec["kernels"][kernel]


def read_ceiling(P, torch, nbytes: int = 2 << 30, reps: int = 20) -> dict:
    """The device's streaming-read rate: mipdhg_read_probe over a buffer of
    nbytes, timed by HIP events on the current stream (the stream it runs
    on), mean over reps launches after one untimed launch."""
    buf = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    P.read_probe(buf)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        P.read_probe(buf)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del buf
    torch.cuda.empty_cache()
    return {"bytes": nbytes, "ms": ms, "GBs": nbytes / (ms * 1e-3) / 1e9}


def tuned_shape(P, dlp, precision: str) -> tuple[dict, float]:
    """The SpMV shape mipdhg_autotune picks for this LP (a one-off per
    matrix, outside the timed region)."""
    t0 = time.perf_counter()
    best = P.autotune(dlp, precision, iters=64)
    keys = ("spmv_kind", "tile_nnz", "tile_rows", "short_row", "tile_nnz_at", "tile_rows_at", "short_row_at")
    return {k: best[k] for k in keys}, time.perf_counter() - t0


def kernel_roofline(P, dlp, ws, precision: str, iters: int, workload_key: str, shape: dict) -> dict:
    """Algorithmic bytes per launch of the slower iteration kernel over its
    mean launch time, against the 8 TB/s HBM peak.  The launch time is from
    HIP events on the solver's stream around 256 back-to-back launches of each
    kernel (kernel_timing=2); the mean with events around every launch of a
    solve (kernel_timing=1, which adds the event cost to each launch) is
    reported beside it."""
    tsol = P.solve(dlp, 0.0, precision, workspace=ws, max_iter=64, kernel_timing=2, validate=0, **shape)
    ti = tsol.info
    each = P.solve(dlp, 0.0, precision, workspace=ws, max_iter=iters, kernel_timing=1, validate=0, **shape).info
    kern = {"primal": (ti["bytes_primal"], ti["ms_primal"]), "dual": (ti["bytes_dual"], ti["ms_dual"])}
    dom = max(kern, key=lambda k: kern[k][1])
    b, ms = kern[dom]
    achieved = b / (ms * 1e-3) / 1e9
    names = kernel_names(shape)
    name = names[dom]
    rec = traffic_record(workload_key, name, shape)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": rec["bytes_per_launch"] if rec else None,
            "kernel": name, "bytes_per_launch": b, "ms_per_launch": ms, "launches_timed": int(ti["n_primal"]),
            "ms_primal": ti["ms_primal"], "ms_dual": ti["ms_dual"],
            "ms_per_launch_events_each": each["ms_" + dom],
            "traffic_source": f"profiles/traffic_{workload_key}.json" if rec else None,
            "other_kernel": {names[k]: {"bytes": v[0], "ms": v[1], "GBs": v[0] / (v[1] * 1e-3) / 1e9,
                                        "traffic": (traffic_record(workload_key, names[k], shape) or {}).get(
                                            "bytes_per_launch")}
                             for k, v in kern.items() if k != dom}}


def bf16_values(P, dlp, lp, eps: float, shape: dict, max_iter: int) -> dict:
    """The same LP with the scaled values stored in BF16 (2 bytes per value
    instead of 4), iterates in float32: a capped solve, its float64 measures
    and its objective against the planted optimum."""
    bsol = P.solve(dlp, eps, "bf16", max_iter=max_iter, **shape)
    bi = bsol.info
    return {"status": bsol.status_name, "iters": int(bi["iters"]), "rel_rp": bi["rel_rp"], "rel_rd": bi["rel_rd"],
            "rel_gap": bi["rel_gap"], "rel_obj_err_vs_planted": abs(bi["pobj"] - lp.p_star) / max(1.0, abs(lp.p_star)),
            "ms_total": bi["ms_total"], "iter_only_rate": int(bi["iters"]) / (bi["ms_iter"] * 1e-3),
            "bytes_per_iter": bi["bytes_per_iter"]}


def workload_leg(P, torch, key: str, eps: float, precision: str, timing_iters: int, seed: int,
                 cpu: bool) -> dict:
    """The workload that is not on the main line: a solve to eps (mean of
    three), the per-kernel roofline, the BF16-value variant, and for the
    power-law LP the tolerance ratios and its own oracle baseline.  The
    power-law LP (64 MB per iteration in FP32) fits the 256 MB last-level
    cache, so its 'HBM' fraction is a cache-resident rate."""
    import lpgen
    t0 = time.perf_counter()
    lp = lpgen.cfg3(seed) if key == "block_angular" else lpgen.cfg2(seed)
    gen_s = time.perf_counter() - t0
    dlp = P.DeviceLP.from_lp(lp, "cuda:0")
    dlp.p_star = lp.p_star
    shape, tune_s = tuned_shape(P, dlp, precision)
    ws = torch.empty(P.workspace_bytes(dlp, precision, **shape), dtype=torch.uint8, device="cuda:0")
    P.solve(dlp, eps, precision, workspace=ws, max_iter=64, **shape)  # warm-up
    runs = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sol = P.solve(dlp, eps, precision, workspace=ws, max_iter=200_000, **shape)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
    dt = sum(runs) / len(runs)
    inf = sol.info
    roof = kernel_roofline(P, dlp, ws, precision, timing_iters, key, shape)
    out = {"workload": WORKLOADS[key], "m": lp.m, "n": lp.n, "nnz": lp.nnz, "precision": precision,
           "eps_rel": eps, "status": sol.status_name, "iters": int(inf["iters"]), "restarts": int(inf["restarts"]),
           "seconds": dt, "iter_per_s": int(inf["iters"]) / dt,
           "iter_only_rate": int(inf["iters"]) / (inf["ms_iter"] * 1e-3), "ms_setup": inf["ms_setup"],
           "bytes_per_iter": inf["bytes_per_iter"],
           "iter_only_GBs": inf["bytes_per_iter"] * int(inf["iters"]) / (inf["ms_iter"] * 1e-3) / 1e9,
           "rel_obj_err_vs_planted": abs(inf["pobj"] - lp.p_star) / max(1.0, abs(lp.p_star)),
           "rel_rp": inf["rel_rp"], "rel_rd": inf["rel_rd"], "rel_gap": inf["rel_gap"],
           "max_violation": inf["max_violation"], "generate_s": gen_s, "roofline": roof,
           "spmv_shape": shape, "autotune_s": tune_s,
           "bf16_values": bf16_values(P, dlp, lp, eps, shape, 20_000)}
    if key == "power_law":
        out["cache_note"] = ("64 MB per FP32 iteration: resident in the 256 MB last-level cache, so the "
                             "roofline fraction is a cache-resident rate, not an HBM one")
        out["tolerance_ratios"] = ratio_leg(P, torch, dlp, ws, precision, dt, int(inf["iters"]), shape)
        if cpu:
            out["cpu_baseline"] = cpu_baseline(lp, int(inf["iters"]), eps)
    del dlp, ws
    torch.cuda.empty_cache()
    return out


def general_leg(P, torch, eps: float, precision: str) -> dict:
    """The general form (bounds l <= x <= u, rows of sense =, >= or <=) on a
    power-law LP of the main workload's shape (100,000 x 400,000, ~3.2M
    nonzeros) with a planted KKT point: a solve to eps, the general kernels'
    roofline, and the same kernels' standard-form variants on the same matrix
    (what the bounds and senses cost per launch)."""
    import lpgen
    t0 = time.perf_counter()
    lp = lpgen.general_cfg2(0)
    gen_s = time.perf_counter() - t0
    dlp = P.DeviceLP.from_lp(lp, "cuda:0")
    shape, tune_s = tuned_shape(P, dlp, precision)
    ws = torch.empty(P.workspace_bytes(dlp, precision, **shape), dtype=torch.uint8, device="cuda:0")
    P.solve(dlp, eps, precision, workspace=ws, max_iter=64, **shape)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol = P.solve(dlp, eps, precision, workspace=ws, max_iter=200_000, **shape)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    inf = sol.info
    roof = kernel_roofline(P, dlp, ws, precision, 256, "general", shape)
    std = P.DeviceLP(lp.A, lp.AT, lp.b, lp.c, "cuda:0")
    sroof = kernel_roofline(P, std, ws, precision, 256, "general_std", shape)
    out = {"workload": "power-law LP m=100000 n=400000 in general form (30% x>=0, 25% boxes, 10% free, "
                       "15% upper-only, 20% shifted lower bounds; rows 50% =, 25% >=, 25% <=), planted KKT point",
           "m": lp.m, "n": lp.n, "nnz": lp.nnz, "precision": precision, "eps_rel": eps,
           "status": sol.status_name, "iters": int(inf["iters"]), "restarts": int(inf["restarts"]),
           "seconds": dt, "iter_per_s": int(inf["iters"]) / dt,
           "iter_only_rate": int(inf["iters"]) / (inf["ms_iter"] * 1e-3), "ms_setup": inf["ms_setup"],
           "rel_obj_err_vs_planted": abs(inf["pobj"] - lp.p_star) / max(1.0, abs(lp.p_star)),
           "rel_rp": inf["rel_rp"], "rel_rd": inf["rel_rd"], "rel_gap": inf["rel_gap"],
           "max_violation": inf["max_violation"], "generate_s": gen_s, "roofline": roof,
           "standard_kernels_same_matrix": {"ms_primal": sroof["ms_primal"], "ms_dual": sroof["ms_dual"]},
           "spmv_shape": shape, "autotune_s": tune_s}
    del dlp, std, ws
    torch.cuda.empty_cache()
    return out


def lp_star(dlp) -> float:
    """The planted optimum c^T x* kept beside a device LP by the caller."""
    return float(getattr(dlp, "p_star"))


def ratio_leg(P, torch, dlp2, ws2, precision: str, t_main: float, iters_main: int, shape: dict) -> dict:
    """Solve time at a tighter tolerance over solve time at 1e-4: the small
    LP in FP64 at 1e-8; the power-law LP at 1e-6 in the bench precision,
    with float32 values and float64 iterates (fp32a), with BF16 values, and
    in FP64 (each capped at 200,000 iterations), with each 1e-6 objective's
    error against the planted optimum."""
    import lpgen
    d1 = P.DeviceLP.from_lp(lpgen.cfg1(0), "cuda:0")

    def timed(dlp, eps, prec, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = P.solve(dlp, eps, prec, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, s

    timed(d1, 1e-4, "fp64")
    a_t, a = timed(d1, 1e-4, "fp64")
    b_t, b = timed(d1, 1e-8, "fp64", max_iter=1_000_000)
    c_t, c = timed(dlp2, 1e-6, precision, workspace=ws2, max_iter=200_000, **shape)
    p_star = lp_star(dlp2)
    out = {"small_fp64": {"t_1e-4_s": a_t, "t_1e-8_s": b_t, "ratio": b_t / a_t, "iters_1e-4": int(a.info["iters"]),
                          "iters_1e-8": int(b.info["iters"]), "status_1e-8": b.status_name},
           "power_law": {"precision": precision, "t_1e-4_s": t_main, "t_1e-6_s": c_t, "ratio": c_t / t_main,
                         "iters_1e-4": iters_main, "iters_1e-6": int(c.info["iters"]), "status_1e-6": c.status_name,
                         "rel_rp_1e-6": c.info["rel_rp"], "omega_1e-6": c.info["omega"],
                         "rel_obj_err_vs_planted_1e-6": abs(c.info["pobj"] - p_star) / max(1.0, abs(p_star))}}
    for prec in ("fp32a", "bf16", "fp64"):
        timed(dlp2, 1e-4, prec, **shape)
        u_t, u = timed(dlp2, 1e-4, prec, **shape)
        v_t, v = timed(dlp2, 1e-6, prec, max_iter=200_000, **shape)
        out["power_law_" + prec] = {"t_1e-4_s": u_t, "t_1e-6_s": v_t, "ratio": v_t / u_t,
                                    "iters_1e-4": int(u.info["iters"]), "iters_1e-6": int(v.info["iters"]),
                                    "status_1e-6": v.status_name,
                                    "rel_obj_err_vs_planted_1e-6": abs(v.info["pobj"] - p_star) / max(1.0, abs(p_star))}
    out["paper_context"] = "geomean runtime ratios over its LP set: 2.29 (1e-6), 3.56 (1e-8)"
    return out



def diff_leg(P, torch) -> dict:
    """256 LPs (m=500, n=1,500, 5 nonzeros per column): K=2,000 unrolled FP32
    iterations with checkpoints every 100, forward and hand-written backward;
    x_K, dL/dc and dL/db of four instances against the float64 oracle's
    reverse mode (its own schedule of restarts and steps)."""
    import numpy as np

    import lpgen
    import oracle
    from oracle.pdhg import OracleOptions, Schedule
    lps, ws = lpgen.cfg5_batch(256)
    batch = P.DeviceBatch.from_lps(lps, "cuda:0")
    umap = P.UnrolledMap(batch, K=2000, ckpt_every=100, precision="fp32")
    w = torch.tensor(np.concatenate(ws), device="cuda:0")
    xk, tape = umap.forward_raw(batch.lp.c, batch.lp.b)
    umap.backward_raw(batch.lp.c, batch.lp.b, tape, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xk, tape = umap.forward_raw(batch.lp.c, batch.lp.b, tape=tape)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gc, gb = umap.backward_raw(batch.lp.c, batch.lp.b, tape, w)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    xk, gc, gb = (v.cpu().numpy() for v in (xk, gc, gb))
    errs = []
    for i in (0, 85, 170, 255):
        rc, rb, rx, _ = oracle.unrolled_grad(lps[i].A, lps[i].b, lps[i].c, 2000, ws[i], OracleOptions())
        # the float64 oracle on the schedule this FP32 run recorded (restart
        # iterations and steps): what remains is FP32 arithmetic
        ra, ta, sa = umap.schedule(tape, i)
        sc, _, _, _ = oracle.unrolled_grad(lps[i].A, lps[i].b, lps[i].c, 2000, ws[i], OracleOptions(),
                                           schedule=Schedule(list(ra), list(ta), list(sa)))
        c0, c1, r0, r1 = batch.col_off[i], batch.col_off[i + 1], batch.row_off[i], batch.row_off[i + 1]

        def rel(a, b):
            return float(np.linalg.norm(a - b) / max(1e-300, np.linalg.norm(b)))
        # coordinates whose final projection mask (x_j > 0) differs from the
        # oracle's: the map is piecewise linear, its piece fixed by the masks
        flips = int(np.count_nonzero((xk[c0:c1] > 0) != (rx > 0)))
        errs.append({"instance": i, "x_K": rel(xk[c0:c1], rx), "dL_dc": rel(gc[c0:c1], rc),
                     "dL_db": rel(gb[r0:r1], rb), "final_mask_flips": flips, "n": int(c1 - c0),
                     "dL_dc_vs_oracle_on_this_schedule": rel(gc[c0:c1], sc)})
    return {"instances": 256, "K": 2000, "ckpt_every": 100, "precision": "fp32", "forward_s": t1 - t0,
            "backward_s": t2 - t1, "tape_bytes": umap.tape_bytes,
            "error_vs_fp64_oracle": {"instances": errs,
                                     "max_rel_x_K": max(e["x_K"] for e in errs),
                                     "max_rel_dL_dc": max(e["dL_dc"] for e in errs),
                                     "max_rel_dL_db": max(e["dL_db"] for e in errs)}}


def _oracle_solve(args):
    import oracle
    from oracle.pdhg import OracleOptions
    A, AT, b, c, eps = args
    return oracle.solve(A, AT, b, c, eps, opts=OracleOptions(max_iter=100_000)).iters


def _oracle_objective(args):
    import oracle
    from oracle.pdhg import OracleOptions
    A, AT, b, c = args
    r = oracle.solve(A, AT, b, c, 1e-8, opts=OracleOptions(max_iter=400_000))
    return r.status, r.meas.pobj


def oracle_objectives(lps) -> list:
    """The oracle's objective at 1e-8 on each LP, one single-threaded process
    per host core (at most 16)."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    cores = max(1, min(16, os.cpu_count() or 1))
    env_threads = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        with ProcessPoolExecutor(max_workers=cores, mp_context=multiprocessing.get_context("spawn")) as ex:
            return list(ex.map(_oracle_objective, [(lp.A, lp.AT, lp.b, lp.c) for lp in lps], timeout=600))
    finally:
        if env_threads is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = env_threads


def batched_cpu_baseline(lps, eps: float) -> dict:
    """The oracle on the same stratified sample, one process per host core
    (at most 16), each single-threaded: LPs/s of the host."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    cores = max(1, min(16, os.cpu_count() or 1))
    env_threads = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        t0 = time.perf_counter()
        # fresh interpreters (spawn): the workers import only the oracle and
        # never touch the GPU this process holds
        with ProcessPoolExecutor(max_workers=cores, mp_context=multiprocessing.get_context("spawn")) as ex:
            list(ex.map(_oracle_solve, [(lp.A, lp.AT, lp.b, lp.c, eps) for lp in lps], timeout=300))
        dt = time.perf_counter() - t0
    finally:
        if env_threads is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = env_threads
    return {"value": len(lps) / dt, "unit": "LPs/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(lps)} instances spread over the size range, {cores} processes of one thread each"}


def batched_leg(P, torch, count: int, sample: int, eps: float) -> dict:
    """4,096 LPs (m log-uniform on [20, 2000], n = 2.5 m, 4 nonzeros per
    column) in one persistent launch, FP32 iterates with FP64 per-instance
    tests, against the plain FP64 single-LP path on a stratified sample."""
    import numpy as np

    import lpgen
    t0 = time.perf_counter()
    sizes = lpgen.cfg4_sizes(count)
    lps = [lpgen.cfg4_instance(i, int(m)) for i, m in enumerate(sizes)]
    batch = P.DeviceBatch.from_lps(lps, "cuda:0")
    gen_s = time.perf_counter() - t0
    ws = torch.empty(P.batch_workspace_bytes(batch, "fp32"), dtype=torch.uint8, device="cuda:0")
    # the launch split mipdhg_autotune_batched picks (one timed solve per
    # candidate; it also warms the kernels up)
    t0 = time.perf_counter()
    split = P.autotune_batched(batch, eps, "fp32", max_iter=100_000)["batch_split"]
    tune_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol = P.solve_batched(batch, eps, "fp32", workspace=ws, max_iter=100_000, batch_split=split)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = np.array([inf["iters"] for inf in sol.infos])
    solved = sum(1 for inf in sol.infos if inf["status"] == 0)
    # the same batch with BF16 matrix values (a side record, not the headline)
    ws16 = torch.empty(P.batch_workspace_bytes(batch, "bf16"), dtype=torch.uint8, device="cuda:0")
    P.solve_batched(batch, eps, "bf16", workspace=ws16, max_iter=100_000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sol16 = P.solve_batched(batch, eps, "bf16", workspace=ws16, max_iter=100_000)
    torch.cuda.synchronize()
    dt16 = time.perf_counter() - t1
    x16 = sol16.x.cpu().numpy()
    err16 = max(abs(float(lp.c @ x16[batch.col_off[i]:batch.col_off[i + 1]]) - lp.p_star) / max(1.0, abs(lp.p_star))
                for i, lp in enumerate(lps))
    bf16_rec = {"value": count / dt16, "unit": "LPs/s", "seconds": dt16,
                "solved": sum(1 for inf in sol16.infos if inf["status"] == 0),
                "iters_p50": float(np.median([inf["iters"] for inf in sol16.infos])),
                "max_rel_obj_err_vs_planted": err16}
    del ws16
    # plain FP64 path, one LP at a time, on every (count/sample)-th instance by size
    order = np.argsort(sizes, kind="stable")
    pick = order[np.linspace(0, count - 1, sample).round().astype(int)]
    t_plain = 0.0
    for i in pick:
        dl = P.DeviceLP.from_lp(lps[i], "cuda:0")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P.solve(dl, eps, "fp64", max_iter=100_000)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t1
    plain_lps = sample / t_plain
    cpu = batched_cpu_baseline([lps[i] for i in pick], eps)
    # algorithmic bytes: per instance and iteration 12 nnz + 28 n + 24 m in
    # FP32 (values of A and A^T and their 16-bit instance-local columns, row
    # pointers, vectors touched once), over the whole launch time
    alg = sum(int(inf["iters"]) * (12.0 * lp.nnz + 28.0 * lp.n + 24.0 * lp.m) for inf, lp in zip(sol.infos, lps))
    mat_mb = 12.0 * sum(lp.nnz for lp in lps) / 1e6
    gbs = alg / dt / 1e9
    trec = batched_traffic_record(split)
    # objectives: every instance against its planted optimum, and a sample of
    # 16 (spread over the sizes) against the oracle run to 1e-8
    x = sol.x.cpu().numpy()
    errs_planted = []
    for i, lp in enumerate(lps):
        c0, c1 = batch.col_off[i], batch.col_off[i + 1]
        pv = float(lp.c @ x[c0:c1])
        errs_planted.append(abs(pv - lp.p_star) / max(1.0, abs(lp.p_star)))
    osample = order[np.linspace(0, count - 1, 16).round().astype(int)]
    refs = oracle_objectives([lps[i] for i in osample])
    errs_oracle = []
    for i, (st, pref) in zip(osample, refs):
        c0, c1 = batch.col_off[i], batch.col_off[i + 1]
        pv = float(lps[i].c @ x[c0:c1])
        errs_oracle.append(abs(pv - pref) / max(1.0, abs(pref)))
    return {"metric": "batched LPs/s to eps_rel=1e-4", "value": count / dt, "unit": "LPs/s",
            "cpu_baseline": cpu,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS,
                         "traffic": None if trec is None else trec["bytes_per_launch"],
                         "traffic_over_algorithmic": None if trec is None else trec["bytes_per_launch"] / alg,
                         "kernel": "k_batched",
                         "bytes_total": alg, "seconds": dt,
                         "note": "algorithmic bytes summed over every instance's iterations (12 nnz + 28 n + 24 m "
                                 f"each, FP32) over the launch; the batch's iteration copy of A and A^T is {mat_mb:.0f} MB "
                                 "against a 256 MB last-level cache, and each instance's vectors live in LDS"},
            "error_vs_planted": {"max": max(errs_planted), "p99": float(np.percentile(errs_planted, 99)),
                                 "p50": float(np.percentile(errs_planted, 50))},
            "error_vs_fp64_oracle": {"instances": [int(i) for i in osample], "max": max(errs_oracle),
                                     "p50": float(np.percentile(errs_oracle, 50)),
                                     "oracle_status": [int(st) for st, _ in refs],
                                     "reference": "objective of the oracle run to 1e-8"},
            "count": count, "solved": solved, "seconds": dt, "batch_split": split, "autotune_s": tune_s,
            "bf16_values": bf16_rec,
            "iters_p50": float(np.percentile(iters, 50)), "iters_p99": float(np.percentile(iters, 99)),
            "plain_fp64_lps_per_s": plain_lps, "plain_sample": int(sample),
            "speedup_vs_plain": (count / dt) / plain_lps, "generate_s": gen_s,
            "workload": "4096 LPs, m log-uniform [20,2000], n=2.5m, 4 nnz/col, N(0,1), planted optima, "
                        "FP32 iterates, FP64 per-instance tests"}


def ipm_leg(P, torch, eps: float = 1e-4) -> dict:
    """The hybrid of Section 3.1 on synthetic LPs: the GPU PDHG solve to
    eps_rel (float64), Algorithm 1's centered start and the GPU interior-point
    method from it (mipdhg_ipm_warm, with the alpha_min loop), against the same
    interior-point method from Mehrotra's point on the same scaled LP.  Reports
    the Newton-step counts, their ratio (the quantity of the paper's Section
    4.6 tables), how many warm runs finish within 10 steps, and the objective
    error against the planted optimum."""
    import math
    import lpgen
    cases = [(f"cfg1 seed {s} (200 x 500)", lpgen.cfg1(s)) for s in range(4)] + \
            [(f"power-law 1/100 seed {s} (1,000 x 4,000)", lpgen.cfg2_sub(s, 100)) for s in range(4)] + \
            [("power-law 1/25 seed 0 (4,000 x 16,000)", lpgen.cfg2_sub(0, 25))]
    rows = []
    for name, lp in cases:
        dlp = P.DeviceLP.from_lp(lp)
        pd = P.solve(dlp, eps, "fp64")
        torch.cuda.synchronize()
        warm = P.ipm_warm(dlp, pd)
        cold = P.ipm_solve(dlp, pd.d_row, pd.d_col)
        wi, ci = warm.info, cold.info
        rows.append({"lp": name, "pdhg_iters": int(pd.info["iters"]), "pdhg_ms": pd.info["ms_total"],
                     "warm_status": warm.status_name, "warm_iters": wi["iters"], "lifts": wi["lifts"],
                     "cold_status": cold.status_name, "cold_iters": ci["iters"],
                     "ratio": wi["iters"] / max(1, ci["iters"]), "warm_ms": wi["ms_total"], "cold_ms": ci["ms_total"],
                     "rel_obj_err_vs_planted": abs(wi["pobj"] - lp.p_star) / max(1.0, abs(lp.p_star))})
        del dlp, pd, warm, cold
        torch.cuda.empty_cache()
    ok = [r for r in rows if r["warm_status"] == "OPTIMAL" and r["cold_status"] == "OPTIMAL"]
    return {"pdhg_eps_rel": eps, "ipm_tol": 1e-8, "instances": len(rows), "solved": len(ok),
            "ratio_geomean": math.exp(sum(math.log(max(r["ratio"], 1e-12)) for r in ok) / max(1, len(ok))),
            "warm_le_10_rate": sum(1 for r in ok if r["warm_iters"] <= 10) / max(1, len(rows)),
            "max_rel_obj_err_vs_planted": max((r["rel_obj_err_vs_planted"] for r in ok), default=None),
            "runs": rows}


def _counter_rows(folder: str) -> dict:
    """Per kernel symbol of a rocprofv3 --pmc csv output: {counter: mean per
    dispatch} (rows of one dispatch and counter are added first)."""
    import csv
    import glob
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {folder}")
    per = {}
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                key = (row["Kernel_Name"], row["Counter_Name"], row.get("Dispatch_Id", ""))
                per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    out = {}
    for (kern, ctr, _), v in per.items():
        d = out.setdefault(kern, {}).setdefault(ctr, [])
        d.append(v)
    return {k: {c: (sum(v) / len(v), len(v)) for c, v in cs.items()} for k, cs in out.items()}


def batched_counter_summary(folder: str) -> int:
    """Write profiles/traffic_batched.json and profiles/batched_kernels_4096.md
    from the rocprofv3 outputs of the commands listed in them (run from the
    repository root, outputs under `folder`): FETCH_SIZE and WRITE_SIZE of
    the batched launch (bench.py --profile-batched, the default launch
    split), calibrated like the plain kernels' (bench.py --calibrate-copy),
    and the launch's kernel statistics."""
    import csv
    import glob
    prof = "python3 bench.py --profile-batched"
    cmds = {
        "fetch": f"timeout -s KILL 240 rocprofv3 --pmc FETCH_SIZE -d {folder}/pmc_batched_FETCH_SIZE -o run "
                 f"--output-format csv -- {prof}",
        "write": f"timeout -s KILL 240 rocprofv3 --pmc WRITE_SIZE -d {folder}/pmc_batched_WRITE_SIZE -o run "
                 f"--output-format csv -- {prof}",
        "cfetch": f"timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -d {folder}/pmc_copy_FETCH_SIZE -o run "
                  "--output-format csv -- python3 bench.py --calibrate-copy",
        "cwrite": f"timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d {folder}/pmc_copy_WRITE_SIZE -o run "
                  "--output-format csv -- python3 bench.py --calibrate-copy",
        "trace": f"rocprofv3 --kernel-trace --stats -d {folder}/profb_batched -o run --output-format csv -- {prof}",
    }
    fetch = _counter_rows(f"{folder}/pmc_batched_FETCH_SIZE")
    write = _counter_rows(f"{folder}/pmc_batched_WRITE_SIZE")
    cf = _counter_rows(f"{folder}/pmc_copy_FETCH_SIZE")
    cw = _counter_rows(f"{folder}/pmc_copy_WRITE_SIZE")
    gib = float(1 << 30)
    probe_f = [v["FETCH_SIZE"][0] for k, v in cf.items() if "k_read_probe" in k]
    copy_w = [v["WRITE_SIZE"][0] for k, v in cw.items() if "copyBuffer" in k]
    if not probe_f or not copy_w:
        raise RuntimeError("calibration kernels not found in the copy profiles")
    ff, wf = gib / (probe_f[0] * 1024.0), gib / (copy_w[0] * 1024.0)
    kernels = {}
    for sym, cs in fetch.items():
        if "k_batched" not in sym or "FETCH_SIZE" not in cs or sym not in write:
            continue
        fk, nd = cs["FETCH_SIZE"]
        wk = write[sym]["WRITE_SIZE"][0]
        kernels[sym.split("(")[0]] = {"dispatches": nd, "fetch_kib": fk, "write_kib": wk,
                                      "bytes_per_launch": fk * 1024.0 * ff + wk * 1024.0 * wf}
    if not kernels:
        raise RuntimeError("k_batched not found in the counter profiles")
    total = sum(v["bytes_per_launch"] for v in kernels.values())
    rec = {"workload": "4096 LPs, m log-uniform [20,2000], n=2.5m, 4 nnz/col, FP32 iterates, eps_rel=1e-4",
           "batch_split": 0, "source_sha256": kernel_source_sha(BATCHED_SOURCES),
           "kernel_sources": list(BATCHED_SOURCES), "fetch_factor": ff, "write_factor": wf,
           "calibration": (f"FETCH_SIZE {probe_f[0]:.1f} KiB per 1 GiB streaming read (k_read_probe), WRITE_SIZE "
                           f"{copy_w[0]:.1f} KiB per 1 GiB device copy (__amd_rocclr_copyBuffer), bench.py "
                           "--calibrate-copy"),
           "commands": [cmds["fetch"], cmds["write"], cmds["cfetch"], cmds["cwrite"]], "kernels": kernels,
           "bytes_per_launch": total}
    with open(os.path.join(ROOT, "profiles", "traffic_batched.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    stats = []
    for f in glob.glob(os.path.join(folder, "profb_batched", "**", "*kernel_stats.csv"), recursive=True):
        with open(f, newline="") as fh:
            stats += list(csv.DictReader(fh))
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Batched kernel, 4,096 LPs, FP32 iterates, eps_rel 1e-4, one launch", "",
             "Kernel statistics (rocprofv3 --kernel-trace --stats):", "", "```", cmds["trace"], "```", "",
             "| kernel | calls | avg ms | total ms |", "|---|---|---|---|"]
    for r in stats[:6]:
        lines.append(f"| `{r['Name'].split('(')[0]}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.2f} |")
    lines += ["", "## HBM-side traffic (rocprofv3 --pmc, one counter per run)", "", "```"]
    lines += [cmds[k] for k in ("fetch", "write", "cfetch", "cwrite")]
    lines += ["```", "", rec["calibration"] + f": factors {ff:.3f} (FETCH_SIZE) and {wf:.3f} (WRITE_SIZE).", "",
              "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | calibrated GB per launch |", "|---|---|---|---|"]
    for k, v in kernels.items():
        lines.append(f"| `{k}` | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | {v['bytes_per_launch'] / 1e9:.1f} |")
    lines += ["", f"Kernel sources sha256 {rec['source_sha256']} ({', '.join(BATCHED_SOURCES)}); the bench's "
              "batched leg uses this record while they are unchanged and its launch split is 0."]
    with open(os.path.join(ROOT, "profiles", "batched_kernels_4096.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps({"wrote": ["profiles/traffic_batched.json", "profiles/batched_kernels_4096.md"],
                      "bytes_per_launch": total}))
    return 0


def counter_summary(folder: str, workload: str, precision: str, shape_text: str) -> int:
    """Write profiles/traffic_<workload>.json from the rocprofv3 outputs of
    the commands listed in it (run from the repository root, outputs under
    `folder`): FETCH_SIZE and WRITE_SIZE of the iteration kernels (bench.py
    --profile), each scaled by what the same counter reads for reads and
    writes of known size (bench.py --calibrate-copy: FETCH_SIZE from the
    streaming-read probe, WRITE_SIZE from the device copy), and the per-kernel
    statistics of the bench command (kernel trace) beside them in
    profiles/iteration_kernels_<workload>_<precision>.md."""
    import csv
    shape = {k: int(v) for k, v in (kv.split("=") for kv in shape_text.split(","))} if shape_text else {}
    prof = f"python3 bench.py --profile --workload {workload} --precision {precision} --shape {shape_text}"
    cmds = {
        "fetch": f"timeout -s KILL 240 rocprofv3 --pmc FETCH_SIZE -d {folder}/pmc_{workload}_FETCH_SIZE -o run "
                 f"--output-format csv -- {prof}",
        "write": f"timeout -s KILL 240 rocprofv3 --pmc WRITE_SIZE -d {folder}/pmc_{workload}_WRITE_SIZE -o run "
                 f"--output-format csv -- {prof}",
        "cfetch": f"timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -d {folder}/pmc_copy_FETCH_SIZE -o run "
                  "--output-format csv -- python3 bench.py --calibrate-copy",
        "cwrite": f"timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d {folder}/pmc_copy_WRITE_SIZE -o run "
                  "--output-format csv -- python3 bench.py --calibrate-copy",
        "trace": f"rocprofv3 --kernel-trace --stats -d {folder}/profb_{workload} -o run --output-format csv -- "
                 f"python3 bench.py --workload {workload} --precision {precision} --shape {shape_text} --steps 2 "
                 "--warmup 1 --no-batched --no-ratios --no-diff --no-cpu-baseline --no-other --no-general --no-ipm",
    }
    fetch = _counter_rows(f"{folder}/pmc_{workload}_FETCH_SIZE")
    write = _counter_rows(f"{folder}/pmc_{workload}_WRITE_SIZE")
    cf = _counter_rows(f"{folder}/pmc_copy_FETCH_SIZE")
    cw = _counter_rows(f"{folder}/pmc_copy_WRITE_SIZE")
    gib = float(1 << 30)
    probe_f = [v["FETCH_SIZE"][0] for k, v in cf.items() if "k_read_probe" in k]
    copy_w = [v["WRITE_SIZE"][0] for k, v in cw.items() if "copyBuffer" in k]
    if not probe_f or not copy_w:
        raise RuntimeError("calibration kernels not found in the copy profiles")
    ff, wf = gib / (probe_f[0] * 1024.0), gib / (copy_w[0] * 1024.0)
    kernels = {}
    for sym, cs in fetch.items():
        short = short_kernel(sym)
        if short is None or "FETCH_SIZE" not in cs or sym not in write:
            continue
        fk, nd = cs["FETCH_SIZE"]
        wk = write[sym]["WRITE_SIZE"][0]
        kernels[short] = {"kernel_symbol": sym.split("(")[0], "dispatches": nd, "fetch_kib": fk, "write_kib": wk,
                          "bytes_per_launch": fk * 1024.0 * ff + wk * 1024.0 * wf}
    if "k_panel_spmv" in kernels and "k_panel_rows" in kernels:
        kernels[PANEL_DUAL] = {"parts": ["k_panel_spmv", "k_panel_rows"],
                               "bytes_per_launch": kernels["k_panel_spmv"]["bytes_per_launch"]
                               + kernels["k_panel_rows"]["bytes_per_launch"]}
    rec = {"workload": workload, "precision": precision, "spmv_shape": shape, "source_sha256": kernel_source_sha(),
           "kernel_sources": list(KERNEL_SOURCES), "fetch_factor": ff, "write_factor": wf,
           "calibration": (f"FETCH_SIZE {probe_f[0]:.1f} KiB per 1 GiB streaming read (k_read_probe), WRITE_SIZE "
                           f"{copy_w[0]:.1f} KiB per 1 GiB device copy (__amd_rocclr_copyBuffer), bench.py "
                           "--calibrate-copy"),
           "commands": [cmds["fetch"], cmds["write"], cmds["cfetch"], cmds["cwrite"]], "kernels": kernels}
    with open(os.path.join(ROOT, "profiles", f"traffic_{workload}.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    # the kernel statistics of the bench command, and its bench line if it was kept
    stats = []
    import glob
    for f in glob.glob(os.path.join(folder, f"profb_{workload}", "**", "*kernel_stats.csv"), recursive=True):
        with open(f, newline="") as fh:
            stats += list(csv.DictReader(fh))
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# Iteration kernels, {workload} LP, {precision}, SpMV shape {shape_text}", "",
             "Kernel statistics (rocprofv3 --kernel-trace --stats) of the single-workload bench command:", "",
             "```", cmds["trace"] + f" > {folder}/bench_{workload}.json", "```", "",
             "| kernel | calls | avg us | min us | max us | total ms |", "|---|---|---|---|---|---|"]
    for r in stats[:12]:
        lines.append(f"| `{r['Name'].replace('(anonymous namespace)::', '').split('(')[0]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.1f} |")
    bj = os.path.join(folder, f"bench_{workload}.json")
    if os.path.exists(bj):
        with open(bj) as fh:
            line = [ln for ln in fh if ln.startswith("{")]
        if line:
            roof = json.loads(line[-1])["roofline"]
            lines += ["", "The same run's bench line (HIP events on the solver's stream around 256 back-to-back "
                      "launches of each kernel):", "",
                      f"* {roof['kernel']}: {roof['ms_per_launch'] * 1e3:.2f} us per launch, "
                      f"{roof['bytes_per_launch'] / 1e6:.1f} MB algorithmic -> {roof['achieved']:.0f} GB/s, "
                      f"frac {roof['frac']:.3f} of 8 TB/s"]
            for k, v in roof.get("other_kernel", {}).items():
                lines.append(f"* {k}: {v['ms'] * 1e3:.2f} us per launch, {v['bytes'] / 1e6:.1f} MB -> "
                             f"{v['GBs']:.0f} GB/s")
            if "read_probe" in roof:
                rp = roof["read_probe"]
                lines.append(f"* streaming-read probe (mipdhg_read_probe, {rp['bytes'] / 2**30:.0f} GiB): "
                             f"{rp['GBs']:.0f} GB/s")
    lines += ["", "## HBM-side traffic (rocprofv3 --pmc, one counter per run)", "", "```"]
    lines += [cmds[k] for k in ("fetch", "write", "cfetch", "cwrite")]
    lines += ["```", "", rec["calibration"] + f": factors {ff:.3f} (FETCH_SIZE) and {wf:.3f} (WRITE_SIZE).", "",
              "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | calibrated MB per launch |",
              "|---|---|---|---|---|"]
    for k, v in kernels.items():
        if "parts" in v:
            lines.append(f"| {k} (sum) | | | | {v['bytes_per_launch'] / 1e6:.1f} |")
        else:
            lines.append(f"| `{v['kernel_symbol']}` ({k}) | {v['dispatches']} | {v['fetch_kib']:.1f} | "
                         f"{v['write_kib']:.1f} | {v['bytes_per_launch'] / 1e6:.1f} |")
    lines += ["", f"Kernel sources sha256 {rec['source_sha256']} ({', '.join(KERNEL_SOURCES)}); bench.py reports "
              f"`traffic` from profiles/traffic_{workload}.json only while they match."]
    with open(os.path.join(ROOT, "profiles", f"iteration_kernels_{workload}_{precision}.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps({k: v["bytes_per_launch"] for k, v in kernels.items()}))
    return 0


def main() -> int:
    args = parse()
    if args.counter_summary:
        if args.workload == "batched":
            return batched_counter_summary(args.counter_summary)
        return counter_summary(args.counter_summary, args.workload, args.precision, args.shape)
    if args.workload == "batched":
        print("--workload batched is for --counter-summary only", file=sys.stderr)
        return 2
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the solver runs on a single GPU; how it would shard is described, not built)", file=sys.stderr)
        return 2
    import torch

    import lpgen
    import paper_2603_03150_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.profile_batched:
        lps = [lpgen.cfg4_instance(i, int(m)) for i, m in enumerate(lpgen.cfg4_sizes(args.batch_count))]
        batch = P.DeviceBatch.from_lps(lps, "cuda:0")
        sol = P.solve_batched(batch, args.eps, "fp32", max_iter=100_000)
        torch.cuda.synchronize()
        print(json.dumps({"profile_batched_count": args.batch_count, "status": sol.status,
                          "instance_iterations": sum(int(i["iters"]) for i in sol.infos),
                          "ms_kernel": sol.infos[0]["ms_iter"]}))
        return 0
    if args.calibrate_copy:
        # 1 GiB read + 1 GiB written per copy, four copies; then four 1 GiB
        # streaming reads with the SpMV kernels' loads (mipdhg_read_probe)
        a = torch.empty(256 * 2**20, dtype=torch.float32, device="cuda:0")
        a.fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        for _ in range(4):
            P.read_probe(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "copies": 4,
                          "read_probe_bytes": a.numel() * 4, "read_probes": 4}))
        return 0
    t0 = time.perf_counter()
    lp = lpgen.cfg3(args.seed) if args.workload == "block_angular" else lpgen.cfg2(args.seed)
    gen_s = time.perf_counter() - t0
    print(f"# generated m={lp.m} n={lp.n} nnz={lp.nnz} in {gen_s:.1f}s", file=sys.stderr, flush=True)
    dlp = P.DeviceLP.from_lp(lp, "cuda:0")
    dlp.p_star = lp.p_star
    if args.shape:
        shape = {k: int(v) for k, v in (kv.split("=") for kv in args.shape.split(","))}
        tune_s = 0.0
    else:
        shape, tune_s = tuned_shape(P, dlp, args.precision)
    print(f"# SpMV shape {shape} (autotune {tune_s:.1f}s)", file=sys.stderr, flush=True)
    ws = torch.empty(P.workspace_bytes(dlp, args.precision, **shape), dtype=torch.uint8, device="cuda:0")

    extra = {} if args.infeas_tol is None else {"infeas_tol": args.infeas_tol}

    def step():
        return P.solve(dlp, args.eps, args.precision, workspace=ws, max_iter=200_000, **shape, **extra)

    if args.profile:
        s = P.solve(dlp, 0.0, args.precision, workspace=ws, max_iter=256, **shape)
        torch.cuda.synchronize()
        print(json.dumps({"profile_solve_iters": int(s.info["iters"]), "precision": args.precision}))
        return 0

    for i in range(args.warmup):
        s = step()
        print(f"# warmup {i}: {s.status_name} iters={s.info['iters']} ms={s.info['ms_total']:.1f}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sols = []
    for i in range(args.steps):
        sols.append(step())
        print(f"# step {i}: iters={sols[-1].info['iters']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    iters = sum(int(s.info["iters"]) for s in sols)
    last = sols[-1]
    value = iters / elapsed

    # per-kernel timing leg: HIP events around every primal and dual launch
    roofline = kernel_roofline(P, dlp, ws, args.precision, args.timing_iters, args.workload, shape)
    rc = read_ceiling(P, torch)
    roofline["read_probe"] = rc
    roofline["frac_of_read_probe"] = roofline["achieved"] / rc["GBs"]

    out = {
        "metric": "PDHG iter/s (plain solve to eps_rel=1e-4)",
        "value": value,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "f32+bf16(A)", "fp32acc32": "f32",
                  "fp32a": "f32(A)+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "m": lp.m, "n": lp.n, "nnz": lp.nnz, "seed": args.seed,
                   "eps_rel": args.eps, "precision": args.precision},
        "roofline": roofline,
        "solve": {"status": last.status_name, "iters": int(last.info["iters"]),
                  "restarts": int(last.info["restarts"]), "ms_setup": last.info["ms_setup"],
                  "ms_iter": last.info["ms_iter"], "pobj": last.info["pobj"], "p_star": lp.p_star,
                  "rel_obj_err_vs_planted": abs(last.info["pobj"] - lp.p_star) / max(1.0, abs(lp.p_star)),
                  "objective_reference": "planted optimum p* = c^T x* (closed form; an oracle run to 1e-8 is "
                                         "out of reach at this size)",
                  "rel_rp": last.info["rel_rp"], "rel_rd": last.info["rel_rd"],
                  "rel_gap": last.info["rel_gap"], "max_violation": last.info["max_violation"],
                  "bytes_per_iter": last.info["bytes_per_iter"],
                  "iter_only_rate": int(last.info["iters"]) / (last.info["ms_iter"] * 1e-3),
                  "iter_only_GBs": last.info["bytes_per_iter"] * int(last.info["iters"])
                  / (last.info["ms_iter"] * 1e-3) / 1e9,
                  "spmv_shape": shape, "autotune_s": tune_s, "generate_s": gen_s},
    }
    print("# BF16 values", file=sys.stderr, flush=True)
    out["solve"]["bf16_values"] = bf16_values(P, dlp, lp, args.eps, shape, 20_000)
    if args.workload == "power_law" and not args.no_ratios:
        print("# tolerance ratios", file=sys.stderr, flush=True)
        out["tolerance_ratios"] = ratio_leg(P, torch, dlp, ws, args.precision, elapsed / args.steps,
                                            int(last.info["iters"]), shape)
    main_iters = int(last.info["iters"])
    del ws, dlp
    torch.cuda.empty_cache()
    if not args.no_other:
        other = "power_law" if args.workload == "block_angular" else "block_angular"
        print(f"# {other} leg", file=sys.stderr, flush=True)
        out[other] = workload_leg(P, torch, other, args.eps, args.precision, 256, args.seed,
                                  cpu=not args.no_cpu_baseline)
    if not args.no_diff:
        print("# differentiation leg", file=sys.stderr, flush=True)
        out["differentiation"] = diff_leg(P, torch)
    if not args.no_general:
        print("# general-form leg", file=sys.stderr, flush=True)
        out["general"] = general_leg(P, torch, args.eps, args.precision)
    if not args.no_ipm:
        print("# hybrid leg (PDHG, centered start, interior point)", file=sys.stderr, flush=True)
        out["ipm_hybrid"] = ipm_leg(P, torch)
    if not args.no_batched:
        print("# batched leg", file=sys.stderr, flush=True)
        out["batched"] = batched_leg(P, torch, args.batch_count, args.plain_sample, args.eps)
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle, 1 thread)", file=sys.stderr, flush=True)
        if args.workload == "block_angular":
            out["cpu_baseline"] = cpu_baseline_block_angular(main_iters, args.eps, args.seed)
        else:
            out["cpu_baseline"] = cpu_baseline(lp, main_iters, args.eps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
