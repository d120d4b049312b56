"""Throughput of the hybrid LB / finite-difference step on one MI355X.

Workload: the 256^3 D3Q19 planar nematic slab (random director, 1e-4 noise
on Q, gamma = 2.7, A0 = 1, K = 0.04, Gamma = 0.3, xi = 0.7, tau = 1) in the
FP32 deviation storage form; a "step" is one full lattice update (molecular
field, stress, body force, moments, Heun update of Q, collision, streaming).
The same grid is also timed in double precision for the FP32/FP64 ratio.

Prints one JSON line.  Inputs are resident in HBM before the timed region;
timing uses HIP events recorded on the stream the library launches on.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS & %HBM roofline, FP32-dev vs FP64 at stated error; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def alg_bytes_per_site(q, es):
    """Compulsory traffic of one site update: read and write f (q values)
    and Q (5 values)."""
    return 2 * (q + 5) * es


def time_steps(lc, torch, solver, steps, warmup):
    stream = solver.stream
    solver.step(warmup)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    solver.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps  # ms per step


def cpu_baseline(n=128, steps=6):
    """The oracle (as written) on the host cores: the same slab recipe at
    n^3 for a few steps."""
    import numpy as np
    import oracle
    from paper_1907_13415_amd import inputs
    rng = np.random.default_rng(2)
    q5, _ = inputs.slab_3d(n, rng)
    f = oracle.rest_populations(oracle.D3Q19, q5.shape[1:])
    oracle.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t = time.perf_counter()
    oracle.run(oracle.D3Q19, f, q5, inputs.WORKLOAD_PARAMS, steps)
    dt = time.perf_counter() - t
    return dict(value=round(n ** 3 * steps / dt / 1e6, 4), unit="MLUPS", cores=threads, kind="oracle",
                sample="oracle FP64, D3Q19 slab recipe at %d^3, %d steps (%.1f s)" % (n, steps, dt))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=256, help="edge of the cubic grid")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--calibrate", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the slab decomposition over xGMI is a design note).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1907_13415_amd import inputs, lc

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    if args.calibrate:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4}))
        return
    w = inputs.config2(args.n)
    res = {}
    for prec in ("fp32dev",) + (() if args.no_fp64 else ("fp64",)):
        with torch.cuda.stream(stream):
            s = lc.Solver("D3Q19", prec, w.shape, w.params, device=dev, stream=stream, variant=args.variant)
            s.load(w.q5)
            steps = args.steps if prec == "fp32dev" else max(1, args.steps // 2)
            ms = time_steps(lc, torch, s, steps, args.warmup)
            obs = s.observe(half_axis=2)
            res[prec] = dict(ms=ms, steps=steps, obs=obs)
            del s
            torch.cuda.empty_cache()
    N = args.n ** 3
    ms32 = res["fp32dev"]["ms"]
    mlups32 = N / (ms32 * 1e-3) / 1e6
    bytes_site = alg_bytes_per_site(19, 4)
    achieved = bytes_site * N / (ms32 * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(mlups32, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "slab%d^3_d3q19_fp32dev" % args.n, "lattice": "D3Q19", "grid": [args.n] * 3,
                   "storage": "fp32 deviation", "gamma": 2.7, "steps_in_config": 500},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_site": bytes_site, "kernel": "whole step"},
    }
    if "fp64" in res:
        ms64 = res["fp64"]["ms"]
        mlups64 = N / (ms64 * 1e-3) / 1e6
        out["fp64"] = {"mlups": round(mlups64, 2), "ms_per_step": round(ms64, 5),
                       "roofline_frac": round(alg_bytes_per_site(19, 8) * N / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        out["fp32_over_fp64"] = round(mlups32 / mlups64, 3)
    out["observables_fp32"] = {k: (float(v) if not hasattr(v, "tolist") else v.tolist())
                               for k, v in res["fp32dev"]["obs"].items() if k in ("mass", "umax", "ssum_half")}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
