"""Throughput of the hybrid LB / finite-difference step on one MI355X.

Headline workload: the 256^3 D3Q19 planar nematic slab (random director,
1e-4 noise on Q, gamma = 2.7, A0 = 1, K = 0.04, Gamma = 0.3, xi = 0.7,
tau = 1) in the FP32 deviation storage form.  A step is one full lattice
update (molecular field, stress, body force, moments, Heun update of Q,
collision, streaming).  The same grid is timed in double precision for the
FP32/FP64 ratio and the FP32 error in S, and in the float form with
stochastic rounding.  Each of these legs runs W untimed steps and then
`--repeats` timed runs of exactly K steps; ms_per_step is the median run.
Also reported: the single-pass variant, the mixed form, the 64-grid
temperature sweep in the batched form, the same slab with the MRT
collision, the isotropic difference stencils (staged kernels), the 256^2
droplets over 20000 steps, and the cost of the checkpointed reverse sweep on
the 256^2 droplet.

Prints one JSON line.  Inputs are resident in HBM before the timed region;
timings use HIP events recorded on the stream the library launches on.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--repeats R] [--no-cpu]
                  [--quick] [--only batch|adjoint|mrt|fused|stencil] [--calibrate]
"""
import argparse
import hashlib
import json
import math
import os
import re
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS & %HBM roofline, FP32-dev vs FP64 at stated error; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
COUNTERS = os.path.join(ROOT, "profiles", "split_sweeps_slab256_d3q19_fp32dev_counters.md")
# what the two sweeps are compiled from (sources, tile configuration, flags)
KERNEL_SOURCES = ["csrc/lc_device.h", "csrc/lc_staged.h", "csrc/lc_split.h", "build.py"]


def note(msg):
    """Progress line on stderr (the JSON record alone goes to stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def alg_bytes_per_site(q, es):
    """Compulsory traffic of one site update: read and write f (q values)
    and Q (5 values)."""
    return 2 * (q + 5) * es


def kernel_hash():
    h = hashlib.sha1()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1907_13415_amd", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def measured_traffic(key="hbm_bytes_per_step"):
    """HBM bytes (per step, or per launch of one sweep) from the committed
    counter summary, if it was taken on the current kernel sources (else
    None)."""
    if not os.path.exists(COUNTERS):
        return None
    txt = open(COUNTERS).read()
    m = re.search(r"kernel_sources_sha1:\s*([0-9a-f]+)", txt)
    t = re.search(r"^" + key + r":\s*([0-9.eE+]+)", txt, re.M)
    if not m or not t or m.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def _oracle_rate(oracle, inputs, n, min_s, max_steps):
    """Steps of the oracle on the slab recipe at n^3, one at a time until
    about min_s seconds have passed: (MLUPS, steps, seconds)."""
    import numpy as np
    rng = np.random.default_rng(2)
    q5, _ = inputs.slab_3d(n, rng)
    f = oracle.rest_populations(oracle.D3Q19, q5.shape[1:])
    steps = 0
    t = time.perf_counter()
    while steps < max_steps and time.perf_counter() - t < min_s:
        f, q5 = oracle.run(oracle.D3Q19, f, q5, inputs.WORKLOAD_PARAMS, 1)
        steps += 1
    dt = time.perf_counter() - t
    return n ** 3 * steps / dt / 1e6, steps, dt


def cpu_baseline(n=128, min_s=10.0, max_steps=200):
    """The oracle (as written) on the host cores: the slab recipe at n^3,
    one step at a time until about min_s seconds have passed; then the same
    on one thread at 64^3 for about a third of that."""
    import oracle
    from paper_1907_13415_amd import inputs
    oracle.build()
    threads = oracle.threads()
    rate, steps, dt = _oracle_rate(oracle, inputs, n, min_s, max_steps)
    oracle.set_threads(1)
    try:
        rate1, steps1, dt1 = _oracle_rate(oracle, inputs, 64, min_s / 3, max_steps)
    finally:
        oracle.set_threads(threads)
    # the oracle's own operation count of one D3Q19 step (oracle/opcount.cpp)
    try:
        flops = oracle.opcount(oracle.D3Q19, 4)["flops_per_site"]
    except (OSError, subprocess.CalledProcessError, ValueError):
        flops = None
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=round(rate, 4), unit="MLUPS", cores=threads, kind="oracle",
                sample="oracle FP64 on the D3Q19 slab recipe at %d^3, %d steps in %.1f s" % (n, steps, dt),
                single_thread=dict(value=round(rate1, 4), unit="MLUPS", cores=1,
                                   sample="the same at 64^3, %d steps in %.1f s" % (steps1, dt1)),
                oracle_flops_per_site=flops,
                gflops=None if flops is None else round(rate * flops / 1e3, 2),
                cpu_model=model, nproc=os.cpu_count())


# ghost-group rates of the MRT leg (s_e, s_eps, s_q, s_pi, s_m); the paper's
# are not given, these are of the usual size
MRT_RATES = (1.19, 1.4, 1.2, 1.4, 1.98)


def run_slab(torch, lc, w, prec, steps, warmup, dev, stream, mrt=False, repeats=1, variant=None, stencil=None):
    """The slab for `warmup` untimed steps, then `repeats` timed runs of
    exactly `steps` steps each (HIP events on the library stream around each
    run, and around each kernel launch): the median run's ms per step and
    the launches' average durations over all runs."""
    with torch.cuda.stream(stream):
        s = lc.Solver("D3Q19", prec, w.shape, w.params, device=dev, stream=stream)
        if variant is not None:
            s.set_variant(variant)
        if stencil is not None:
            s.set_stencil(stencil)
        if mrt:
            s.set_collision(lc.LC_COLL_MRT, MRT_RATES)
        s.load(w.q5)
        s.step(warmup)
        torch.cuda.synchronize()
        lc.lc_set_timing(s.ctx, True)
        lc.lc_get_timing(s.ctx)  # clear
        runs = []
        for _ in range(repeats):
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            t0.record(stream)
            s.step(steps)
            t1.record(stream)
            torch.cuda.synchronize()
            runs.append(t0.elapsed_time(t1) / steps)
        ms_k, n_k = lc.lc_get_timing(s.ctx)
        lc.lc_set_timing(s.ctx, False)
        S = torch.empty((1,) + w.shape, dtype=torch.float64, device=dev)
        lc.lc_export(s.ctx, lc.LC_FIELD_S, S.data_ptr())
        obs = s.observe(half_axis=2)
        torch.cuda.synchronize()
        del s
    return dict(ms=statistics.median(runs), runs=runs, steps_total=warmup + repeats * steps,
                kernel_ms=[ms_k[0] / max(n_k[0], 1), ms_k[1] / max(n_k[1], 1)], launches=list(n_k), S=S, obs=obs)


def fused_leg(torch, lc, w, args, dev, stream, N, bytes_site, ms_split32, ms_split64):
    """The single-pass variant on the slab (FP32 and FP64), beside the two
    sweeps timed above."""
    out = {}
    for prec, es, ref in (("fp32dev", 4, ms_split32), ("fp64", 8, ms_split64)):
        r = run_slab(torch, lc, w, prec, args.steps, args.warmup, dev, stream, repeats=min(3, args.repeats),
                     variant=lc.LC_VARIANT_FUSED)
        del r["S"]
        b = alg_bytes_per_site(19, es)
        out[prec] = {"mlups": round(N / (r["ms"] * 1e-3) / 1e6, 2), "ms_per_step": round(r["ms"], 5),
                     "kernel_ms": round(r["kernel_ms"][0], 5),
                     "roofline_frac": round(b * N / (r["kernel_ms"][0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "over_split": round(r["ms"] / ref, 3)}
        torch.cuda.empty_cache()
    return out


def mixed_leg(torch, lc, w, args, dev, stream, N, S64):
    """The slab in the mixed form (float populations, double Q): throughput,
    roofline on its own compulsory bytes and |S - S64| after the same steps."""
    rm = run_slab(torch, lc, w, "mixed", args.steps, args.warmup, dev, stream, repeats=args.repeats)
    dS = float((rm["S"] - S64).abs().max().item())
    b = 2 * (19 * 4 + 5 * 8)
    return {"mlups": round(N / (rm["ms"] * 1e-3) / 1e6, 2), "ms_per_step": round(rm["ms"], 5),
            "kernel_ms": [round(v, 5) for v in rm["kernel_ms"]], "bytes_per_site": b,
            "roofline_frac": round(b * N / (sum(rm["kernel_ms"]) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "max_abs_dS_vs_fp64": dS}


def mrt_leg(torch, lc, w, args, dev, stream, N, bytes_site):
    rm = run_slab(torch, lc, w, "fp32dev", args.steps, args.warmup, dev, stream, mrt=True)
    return {"mlups": round(N / (rm["ms"] * 1e-3) / 1e6, 2), "ms_per_step": round(rm["ms"], 5),
            "kernel_ms": [round(v, 5) for v in rm["kernel_ms"]], "rates": list(MRT_RATES),
            "roofline_frac": round(bytes_site * N / (sum(rm["kernel_ms"]) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def _time_2d(torch, lc, q5, params, prec, variant, stencil, steps, dev, stream):
    """ms per step of a D2Q9 grid (HIP events on the library stream)."""
    with torch.cuda.stream(stream):
        s = lc.Solver("D2Q9", prec, q5.shape[1:], params, device=dev, stream=stream)
        s.set_variant(variant)
        s.set_stencil(stencil)
        s.load(q5)
        s.step(20)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        s.step(steps)
        t1.record(stream)
        torch.cuda.synchronize()
        del s
    return t0.elapsed_time(t1) / steps


def stencil_leg(torch, lc, inputs, w, args, dev, stream, N):
    """The isotropic difference stencils in the two-sweep and staged kernels,
    beside the compact stencils: on the slab in FP32 and FP64, and on a
    2048^2 D2Q9 grid (the circle recipe scaled up) in FP32."""
    out = {}
    for prec in ("fp32dev", "fp64"):
        leg = {}
        for name, variant, st in (("split_compact", lc.LC_VARIANT_SPLIT, lc.LC_STENCIL_COMPACT),
                                  ("split_isotropic", lc.LC_VARIANT_SPLIT, lc.LC_STENCIL_ISOTROPIC),
                                  ("staged_compact", lc.LC_VARIANT_STAGED, lc.LC_STENCIL_COMPACT),
                                  ("staged_isotropic", lc.LC_VARIANT_STAGED, lc.LC_STENCIL_ISOTROPIC)):
            r = run_slab(torch, lc, w, prec, min(args.steps, 100), min(args.warmup, 10), dev, stream,
                         variant=variant, stencil=st)
            del r["S"]
            leg[name] = {"mlups": round(N / (r["ms"] * 1e-3) / 1e6, 2), "ms_per_step": round(r["ms"], 5),
                         "kernel_ms": [round(v, 5) for v in r["kernel_ms"]]}
            torch.cuda.empty_cache()
        out["slab_%s" % prec] = leg
    n2 = 2048
    q5 = inputs.paper_circle(n2, n2 / 4.0)
    params = inputs.with_gamma(inputs.PAPER_PARAMS, 2.7076)
    d2 = {}
    for name, variant, st in (("split_compact", lc.LC_VARIANT_SPLIT, lc.LC_STENCIL_COMPACT),
                              ("split_isotropic", lc.LC_VARIANT_SPLIT, lc.LC_STENCIL_ISOTROPIC),
                              ("staged_isotropic", lc.LC_VARIANT_STAGED, lc.LC_STENCIL_ISOTROPIC)):
        ms = _time_2d(torch, lc, q5, params, "fp32dev", variant, st, 200, dev, stream)
        d2[name] = {"mlups": round(n2 * n2 / (ms * 1e-3) / 1e6, 2), "ms_per_step": round(ms, 5)}
        torch.cuda.empty_cache()
    out["circle2048_d2q9_fp32dev"] = d2
    return out


def s_nematic(g):
    """Nematic minimum of the uniaxial bulk free energy (Eq. 3), for
    converting sums of S into lengths and areas (0 below gamma = 8/3)."""
    return 0.25 + 0.75 * math.sqrt(1.0 - 8.0 / (3.0 * g)) if g >= 8.0 / 3.0 else 0.0


def _vel_err(x, ref):
    """Relative error of the mean interface velocity (radius drift over the
    run) of one form against the double-precision run."""
    return abs((x["r1"] - x["r0"]) - (ref["r1"] - ref["r0"])) / abs(ref["r1"] - ref["r0"])


def run_droplets(torch, lc, dev, stream, steps=20000):
    """256^2 droplet at gamma = 2.7, 2.705, 2.71 for 20000 steps in FP64,
    FP32 and the mixed form: max |u|, radius drift and the errors of the
    other two forms against FP64 (S, interface position and velocity, max
    |u|)."""
    from paper_1907_13415_amd import inputs
    recs = []
    for dg in (0.0, 0.005, 0.01):
        w = inputs.config1(dg)
        g = w.params[1]
        sn = s_nematic(g)
        res = {}
        for prec in ("fp64", "fp32dev", "mixed", "fp32sr"):
            with torch.cuda.stream(stream):
                s = lc.Solver("D2Q9", prec, w.shape, w.params, device=dev, stream=stream)
                s.load(w.q5)
                r0 = math.sqrt(s.observe()["ssum"] / (math.pi * sn))
                t0 = time.perf_counter()
                s.step(steps)
                o = s.observe()
                dt = time.perf_counter() - t0
                res[prec] = dict(umax=o["umax"], r0=r0, r1=math.sqrt(o["ssum"] / (math.pi * sn)),
                                 S=s.export(lc.LC_FIELD_S), mlups=w.shape[1] * w.shape[2] * steps / dt / 1e6)
                del s
        a, b, m, r = res["fp64"], res["fp32dev"], res["mixed"], res["fp32sr"]
        recs.append({"gamma": round(g, 4), "umax": a["umax"], "radius": [round(a["r0"], 4), round(a["r1"], 4)],
                     "radius_drift_per_step": (a["r1"] - a["r0"]) / steps,
                     "fp32_max_abs_dS": float(abs(a["S"] - b["S"]).max()),
                     "fp32_umax_rel_err": abs(b["umax"] - a["umax"]) / a["umax"],
                     "fp32_radius_err": abs(b["r1"] - a["r1"]),
                     "fp32_interface_velocity_rel_err": _vel_err(b, a),
                     "mixed_max_abs_dS": float(abs(a["S"] - m["S"]).max()),
                     "mixed_umax_rel_err": abs(m["umax"] - a["umax"]) / a["umax"],
                     "mixed_radius_err": abs(m["r1"] - a["r1"]),
                     "mixed_interface_velocity_rel_err": _vel_err(m, a),
                     "fp32sr_max_abs_dS": float(abs(a["S"] - r["S"]).max()),
                     "fp32sr_umax_rel_err": abs(r["umax"] - a["umax"]) / a["umax"],
                     "fp32sr_radius_err": abs(r["r1"] - a["r1"]),
                     "fp32sr_interface_velocity_rel_err": _vel_err(r, a),
                     "mlups_fp64": round(a["mlups"], 1), "mlups_fp32": round(b["mlups"], 1),
                     "mlups_mixed": round(m["mlups"], 1), "mlups_fp32sr": round(r["mlups"], 1)})
    return dict(workload="droplet256_d2q9", steps=steps, runs=recs)


def batch_velocities(b, ws, t0=1000, t1=5000):
    """Per-grid interface velocity of the sweep (the right interface of each
    slab, from the half-domain sum of S) between steps t0 and t1, and the
    grids that melt (gamma < 8/3, or all isotropic by t1) or fill instead."""
    for k, w in enumerate(ws):
        b.load(k, w.q5)
    b.step(t0)
    o0 = b.observe(half_axis=0)
    b.step(t1 - t0)
    o1 = b.observe(half_axis=0)
    vel, melted, filled = [], 0, 0
    for w, a, c in zip(ws, o0, o1):
        L = w.shape[2]
        g = w.params[1]
        sn = s_nematic(g)
        if sn == 0.0 or c["ssum"] < 1e-6 * L * L:  # below 8/3 the nematic is unstable
            melted += 1
            vel.append(None)
        elif sn > 0 and c["ssum"] > 0.99 * sn * L * L:
            filled += 1
            vel.append(None)
        else:
            vel.append(round((c["ssum_half"] - a["ssum_half"]) / (sn * L) / (t1 - t0), 8))
    return dict(steps=[t0, t1], melted=melted, filled=filled,
                velocity_per_grid=[{"gamma": round(w.params[1], 5), "L": w.shape[2], "v": v}
                                   for w, v in zip(ws, vel)])


def run_batch(torch, lc, stream, dev, steps, tiles=None, physics=True):
    from paper_1907_13415_amd import inputs
    ws = inputs.config3()
    shapes = [w.shape[1:] for w in ws]
    with torch.cuda.stream(stream):
        b = lc.BatchSolver("fp32dev", shapes, [w.params for w in ws], device=dev, stream=stream)
        for k, w in enumerate(ws):
            b.load(k, w.q5)
        if tiles is None:
            tile, _ = b.autotune(10)
        else:
            b.set_tiles(*tiles)
            tile = tiles[0] + 7 * tiles[1]
        for k, w in enumerate(ws):
            b.load(k, w.q5)
        b.step(64)
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        b.step(steps)
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / steps
        obs = b.observe()
        sweep = batch_velocities(b, ws) if physics else None
        del b
        # the same batch in the float form with stochastic rounding, on the
        # tile shapes just chosen
        bs = lc.BatchSolver("fp32sr", shapes, [w.params for w in ws], device=dev, stream=stream)
        for k, w in enumerate(ws):
            bs.load(k, w.q5)
        bs.set_tiles(tile % 7, tile // 7)
        bs.step(64)
        torch.cuda.synchronize()
        t0.record(stream)
        bs.step(steps)
        t1.record(stream)
        torch.cuda.synchronize()
        ms_sr = t0.elapsed_time(t1) / steps
        del bs
    sites = sum(w.shape[1] * w.shape[2] for w in ws)
    shapes_ = ["32x8", "64x4", "16x16", "32x16", "64x8", "64x16", "128x8"]
    return dict(grids=len(ws), sites=sites, tiles={"lb": shapes_[tile % 7], "q": shapes_[tile // 7]},
                ms_per_step=round(ms, 5),
                mlups=round(sites / (ms * 1e-3) / 1e6, 2),
                roofline_frac=round(alg_bytes_per_site(9, 4) * sites / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                nonfinite=int(sum(o["nonfinite"] for o in obs)), sweep=sweep,
                fp32sr={"ms_per_step": round(ms_sr, 5), "mlups": round(sites / (ms_sr * 1e-3) / 1e6, 2)})


def run_adjoint(torch, repeats=5):
    """Gradient of a 2000-step droplet loss: wall time of the forward and of
    the backward (median of `repeats` runs after one warm-up)."""
    from paper_1907_13415_amd import adjoint, inputs
    w = inputs.config4()
    dev = torch.device("cuda:0")
    A0, g, K, G, xi, tau = w.params
    cfg = dict(A0=A0, xi=xi, tau=tau, steps=w.steps, every=100)
    f64 = dict(dtype=torch.float64)
    q0 = torch.tensor(w.q5, device=dev, requires_grad=True)
    tg, tK, tG = (torch.tensor(v, requires_grad=True, **f64) for v in (g, K, G))
    st = torch.tensor(w.extra["s_target"], device=dev)

    def loss(qf):
        xx, xy, xz, yy, yz = qf
        qq = xx * xx + yy * yy + (xx + yy) * (xx + yy) + 2 * (xy * xy + xz * xz + yz * yz)
        return ((torch.sqrt((1.5 * qq).clamp_min(1e-300)) - st) ** 2).sum()

    loss(adjoint.solve(q0, tg, tK, tG, **cfg)).backward()  # warm-up
    fwds, bwds = [], []
    for _ in range(repeats):
        q0.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = loss(adjoint.solve(q0, tg, tK, tG, **cfg))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fwds.append(t1 - t0)
        bwds.append(t2 - t1)
    fwd, bwd = statistics.median(fwds), statistics.median(bwds)
    # the backward replays every segment once (a forward pass with recording,
    # on a second stream, overlapping the reverse steps of the next segment)
    return dict(workload="adjoint_droplet256_d2q9_fp64", steps=w.steps, checkpoint_every=100,
                repeats=repeats, forward_s=round(fwd, 4), backward_s=round(bwd, 4),
                backward_over_forward=round(bwd / fwd, 2), includes_replay=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the slab workload is 500 steps: time all of them after 50 untimed ones
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=256, help="edge of the cubic grid")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--repeats", type=int, default=5, help="timed runs of --steps steps; the median is reported")
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--calibrate", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM counters)")
    ap.add_argument("--batch-tiles", help="LB,Q tile shapes of the batched leg instead of tuning (0..6)")
    ap.add_argument("--no-physics", action="store_true",
                    help="with --only batch: skip the 5000-step front-speed window (for counter runs)")
    ap.add_argument("--only", choices=["batch", "adjoint", "mrt", "fused", "stencil", "droplets"],
                    help="run one secondary leg alone and print its record (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
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

    if args.only == "batch":
        tiles = tuple(int(v) for v in args.batch_tiles.split(",")) if args.batch_tiles else None
        print(json.dumps({"batch_sweep": run_batch(torch, lc, stream, dev, args.steps, tiles,
                                                   physics=not args.no_physics)}), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps({"adjoint": run_adjoint(torch)}), flush=True)
        return
    if args.only == "droplets":
        print(json.dumps({"droplets": run_droplets(torch, lc, dev, stream)}), flush=True)
        return

    w = inputs.config2(args.n)
    N = args.n ** 3
    bytes_site = alg_bytes_per_site(19, 4)
    if args.only == "mrt":
        print(json.dumps({"mrt_fp32": mrt_leg(torch, lc, w, args, dev, stream, N, bytes_site)}), flush=True)
        return
    if args.only == "stencil":
        print(json.dumps({"stencil_iso": stencil_leg(torch, lc, inputs, w, args, dev, stream, N)}), flush=True)
        return
    if args.only == "fused":
        print(json.dumps({"fused": fused_leg(torch, lc, w, args, dev, stream, N, bytes_site, 1.0, 1.0)}), flush=True)
        return
    rep = args.repeats
    r32 = run_slab(torch, lc, w, "fp32dev", args.steps, args.warmup, dev, stream, repeats=rep)
    note("slab fp32dev %.4f ms/step" % r32["ms"])
    r64 = run_slab(torch, lc, w, "fp64", args.steps, args.warmup, dev, stream, repeats=rep)
    note("slab fp64 %.4f ms/step" % r64["ms"])
    rsr = run_slab(torch, lc, w, "fp32sr", args.steps, args.warmup, dev, stream, repeats=rep)
    note("slab fp32sr %.4f ms/step" % rsr["ms"])
    dS = float((r32["S"] - r64["S"]).abs().max().item())
    dS_sr = float((rsr["S"] - r64["S"]).abs().max().item())
    mixed = None if args.quick else mixed_leg(torch, lc, w, args, dev, stream, N, r64["S"])
    del r32["S"], r64["S"], rsr["S"]
    torch.cuda.empty_cache()

    ms32 = r32["ms"]
    mlups32 = N / (ms32 * 1e-3) / 1e6
    mlups64 = N / (r64["ms"] * 1e-3) / 1e6
    mlups_sr = N / (rsr["ms"] * 1e-3) / 1e6
    kernel_ms = sum(r32["kernel_ms"])  # the two sweeps of one step
    achieved = bytes_site * N / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    # measured HBM rate of each sweep: counter bytes per launch over its
    # event-timed duration
    per_launch = [measured_traffic("hbm_bytes_per_launch_split_lb"), measured_traffic("hbm_bytes_per_launch_split_q")]
    measured_gbs = [None if b is None else round(b / (ms * 1e-3) / 1e9, 1)
                    for b, ms in zip(per_launch, r32["kernel_ms"])]
    out = {
        "metric": METRIC,
        "value": round(mlups32, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "repeats": rep,
        "ms_per_step": round(ms32, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "slab%d^3_d3q19_fp32dev" % args.n, "lattice": "D3Q19", "grid": [args.n] * 3,
                   "storage": "fp32 deviation", "gamma": 2.7, "steps_in_config": 500},
        # achieved: the algorithmic bytes of one step over the summed average
        # durations of the step's two launches (kernel time, HIP events on
        # the library stream); frac_step_wall: the same bytes over the whole
        # step's wall time (ms_per_step)
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "frac_basis": "kernel time",
                     "frac_step_wall": round(bytes_site * N / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "measured_gbs_per_sweep": measured_gbs,
                     "kernel": "split_lb + split_q (the two launches of one step)",
                     "bytes_per_site": bytes_site, "sites_per_launch": N,
                     "kernel_ms": [round(v, 5) for v in r32["kernel_ms"]]},
        "fp64": {"mlups": round(mlups64, 2), "ms_per_step": round(r64["ms"], 5),
                 "kernel_ms": [round(v, 5) for v in r64["kernel_ms"]],
                 "roofline_frac": round(alg_bytes_per_site(19, 8) * N / (sum(r64["kernel_ms"]) * 1e-3) / 1e9
                                        / HBM_PEAK_GBS, 4)},
        "fp32_over_fp64": round(mlups32 / mlups64, 3),
        "fp32_max_abs_dS_vs_fp64": dS,
        "fp32_steps_compared": r32["steps_total"],
        # float storage with the molecular field summed in double and
        # stochastic rounding of the Q update (within 1e-5 on the droplets)
        "fp32sr": {"mlups": round(mlups_sr, 2), "ms_per_step": round(rsr["ms"], 5),
                   "kernel_ms": [round(v, 5) for v in rsr["kernel_ms"]],
                   "roofline_frac": round(bytes_site * N / (sum(rsr["kernel_ms"]) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "over_fp64": round(mlups_sr / mlups64, 3), "max_abs_dS_vs_fp64": dS_sr},
    }
    if not args.quick:
        out["fused"] = fused_leg(torch, lc, w, args, dev, stream, N, bytes_site, r32["ms"], r64["ms"])
        note("fused leg done")
        out["mixed"] = mixed
        out["mrt_fp32"] = mrt_leg(torch, lc, w, args, dev, stream, N, bytes_site)
        note("mrt leg done")
        out["stencil_iso"] = stencil_leg(torch, lc, inputs, w, args, dev, stream, N)
        note("stencil leg done")
        out["batch_sweep"] = run_batch(torch, lc, stream, dev, 128)
        note("batch leg done")
        out["droplets"] = run_droplets(torch, lc, dev, stream)
        note("droplets done")
        out["adjoint"] = run_adjoint(torch)
        note("adjoint done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
        note("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
