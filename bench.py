#!/usr/bin/env python3
"""PDHG iterations per second on one MI355X.

Workload: a plain PDHG solve to eps_rel = 1e-4 of the power-law LP with
m = 100,000, n = 400,000 (column counts p(k) ~ k^-2.1423 on [2, 2000], about
3.2M nonzeros, values N(0,1) times a per-row factor U(0.1, 10), planted
optimum), float32 iterates and SpMV accumulation, float64 termination tests on
the original model.  One step is one whole solve from device-resident inputs:
validation, scaling, power iteration, the iterations, and the final
evaluation.  value = iterations / second over the K timed steps.

Also reported, on the same JSON line:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                mean launch time (HIP events on the solver's stream), against
                MI355X's 8 TB/s HBM peak;
  cpu_baseline  the float64 NumPy/SciPy oracle on the host, single thread, on
                a bounded sample of the same workload.
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
WORKLOAD = ("power-law LP m=100000 n=400000 (~3.2M nnz, column counts k^-2.1423 on [2,2000], "
            "N(0,1) x row factor U(0.1,10), planted optimum), plain PDHG, FP32 iterates, "
            "FP64 termination tests, eps_rel=1e-4")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "bf16", "fp32acc32"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing-iters", type=int, default=1024,
                    help="iterations of the per-kernel HIP-event timing leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-LP leg")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--plain-sample", type=int, default=32,
                    help="instances of the batch solved one at a time by the plain FP64 path")
    return ap.parse_args()


def cpu_baseline(lp, gpu_iters: int, eps: float) -> dict:
    """The oracle as it stands, one thread, on a bounded sample: two runs
    capped at 64 and 192 iterations give its setup time and per-iteration
    time; the rate is quoted for a solve of the GPU's iteration count."""
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
        for n in (64, 192):
            t0 = time.perf_counter()
            oracle.solve(lp.A, lp.AT, lp.b, lp.c, eps, opts=OracleOptions(max_iter=n))
            times[n] = time.perf_counter() - t0
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    per_iter = (times[192] - times[64]) / 128.0
    setup = max(0.0, times[64] - 64 * per_iter)
    value = gpu_iters / (setup + gpu_iters * per_iter)
    return {"value": value, "unit": "iter/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle capped at 64 and 192 iterations on the same LP: setup {setup:.2f} s, "
                       f"{per_iter * 1e3:.1f} ms/iteration, rate quoted for a {gpu_iters}-iteration solve")}


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
    P.solve_batched(batch, eps, "fp32", workspace=ws, max_iter=100_000)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol = P.solve_batched(batch, eps, "fp32", workspace=ws, max_iter=100_000)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = np.array([inf["iters"] for inf in sol.infos])
    solved = sum(1 for inf in sol.infos if inf["status"] == 0)
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
    return {"metric": "batched LPs/s to eps_rel=1e-4", "value": count / dt, "unit": "LPs/s",
            "count": count, "solved": solved, "seconds": dt,
            "iters_p50": float(np.percentile(iters, 50)), "iters_p99": float(np.percentile(iters, 99)),
            "plain_fp64_lps_per_s": plain_lps, "plain_sample": int(sample),
            "speedup_vs_plain": (count / dt) / plain_lps, "generate_s": gen_s,
            "workload": "4096 LPs, m log-uniform [20,2000], n=2.5m, 4 nnz/col, N(0,1), planted optima, "
                        "FP32 iterates, FP64 per-instance tests"}


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(this build is single-GPU; sharding is described, not built)", file=sys.stderr)
        return 2
    import torch

    import lpgen
    import paper_2603_03150_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    lp = lpgen.cfg2(args.seed)
    gen_s = time.perf_counter() - t0
    print(f"# generated m={lp.m} n={lp.n} nnz={lp.nnz} in {gen_s:.1f}s", file=sys.stderr, flush=True)
    dlp = P.DeviceLP.from_lp(lp, "cuda:0")
    ws = torch.empty(P.workspace_bytes(dlp, args.precision), dtype=torch.uint8, device="cuda:0")

    def step():
        return P.solve(dlp, args.eps, args.precision, workspace=ws, max_iter=200_000)

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
    tsol = P.solve(dlp, 0.0, args.precision, workspace=ws, max_iter=args.timing_iters, kernel_timing=1)
    ti = tsol.info
    kern = {"primal": (ti["bytes_primal"], ti["ms_primal"]), "dual": (ti["bytes_dual"], ti["ms_dual"])}
    dom = max(kern, key=lambda k: kern[k][1])
    b, ms = kern[dom]
    achieved = b / (ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": f"k_iter<{'dual' if dom == 'dual' else 'primal'}>",
                "bytes_per_launch": b, "ms_per_launch": ms,
                "other_kernel": {k: {"bytes": v[0], "ms": v[1], "GBs": v[0] / (v[1] * 1e-3) / 1e9}
                                 for k, v in kern.items() if k != dom}}

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
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "f32+bf16(A)", "fp32acc32": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "m": lp.m, "n": lp.n, "nnz": lp.nnz, "seed": args.seed,
                   "eps_rel": args.eps, "precision": args.precision},
        "roofline": roofline,
        "solve": {"status": last.status_name, "iters": int(last.info["iters"]),
                  "restarts": int(last.info["restarts"]), "ms_setup": last.info["ms_setup"],
                  "ms_iter": last.info["ms_iter"], "pobj": last.info["pobj"], "p_star": lp.p_star,
                  "rel_obj_err_vs_planted": abs(last.info["pobj"] - lp.p_star) / max(1.0, abs(lp.p_star)),
                  "rel_rp": last.info["rel_rp"], "rel_rd": last.info["rel_rd"],
                  "rel_gap": last.info["rel_gap"], "max_violation": last.info["max_violation"],
                  "bytes_per_iter": last.info["bytes_per_iter"],
                  "iter_only_rate": int(last.info["iters"]) / (last.info["ms_iter"] * 1e-3),
                  "plan": {k: last.info[k] for k in ("lanes_a", "lanes_at", "long_a", "long_at")}},
    }
    if not args.no_batched:
        print("# batched leg", file=sys.stderr, flush=True)
        out["batched"] = batched_leg(P, torch, args.batch_count, args.plain_sample, args.eps)
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle, 1 thread)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(lp, int(last.info["iters"]), args.eps)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
