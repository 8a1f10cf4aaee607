#!/usr/bin/env python3
"""Benchmark of the direct-sum N-body hot path on one MI355X.

Default workload: the 10,425-body Solar-System system (Sun, 30 major bodies,
100 minor moons, 19 heavy and 10,275 small asteroids; seed 1), dt = 0.1 day.
A step is one velocity-Verlet step (one all-pairs force pass plus the fused
kick-drift-kick epilogue).  The line reports pair interactions/s and steps/s
for the FP64 form (the headline `value`) and for the split-precision form,
with both forms' energy errors, the force kernel's roofline fraction and the
CPU oracle's rate on this host.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --workload {solar-131,solar-131072,ensemble,adjoint}
    python bench.py --workload dt-scan    # accuracy against the step size (Sec. 4)
    python bench.py --workload n-scan     # throughput against N, GPU and oracle (Sec. 5)
    python bench.py --workload force      # force passes only (for counter profiles)
    python bench.py --workload shard      # one GPU's share of the targets (8-way split)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def metric_at(n):
    """The headline metric's name for a single system of n bodies."""
    return f"pair interactions/s + steps/s at N={n:,}: FP64 vs split-precision at fixed ΔE/E"


FP64_PEAK_TFLOPS = 78.6          # MI355X vector FP64, 256 CU x 64 lanes x 2 x 2.4 GHz
FP32_PEAK_TFLOPS = 157.3         # MI355X vector FP32 (packed)
VJP_FLOPS_PER_PAIR = 47         # transpose-Jacobian pass of the adjoint, per ordered pair
HBM_PEAK_GBS = 8000.0
# algorithmic work of one force pass: 20 flops per ordered pair interaction,
# N (N - 1) of them, whichever kernel evaluates them
FLOPS_PER_PAIR = 20
# the each-pair-once kernel's own arithmetic per unordered pair: the pair's 20
# flops serve the target, and the reaction on the source adds 7 (the
# source-side mass scale and three fused multiply-adds)
FLOPS_PER_MUTUAL_PAIR = 27


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="solar-10425",
                    choices=["solar-10425", "solar-131", "solar-131072", "ensemble", "adjoint",
                             "dt-scan", "n-scan", "copy", "force", "shard"])
    ap.add_argument("--tune", action="store_true",
                    help="single-system workloads: autotune the force tiles first (the default "
                         "is the library's sweep-derived heuristic; the ensemble always autotunes)")
    ap.add_argument("--settle-ms", type=float, default=60.0,
                    help="untimed force passes (about this many ms of GPU work) right before "
                         "each timed run, so that the GPU's clock has reached its sustained "
                         "level under load (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-legs", action="store_true",
                    help="solar-10425: skip the paper-shaped run and the RK4 leg (counter passes)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate CPU time budget of the oracle sample")
    ap.add_argument("--fd-coords", type=int, default=64, help="adjoint workload: FD coordinates")
    ap.add_argument("--force-reps", type=int, default=None,
                    help="launches timed for the force kernel's roofline figure (default: ~0.1 s)")
    ap.add_argument("--tile", default=None,
                    help="fix the FP64 force tile as T,W,C[,variant] (skips autotune)")
    ap.add_argument("--split-tile", default=None, help="fix the split force tile as T,W,C[,variant]")
    return ap.parse_args()


def tile_str(t):
    return f"{t['targets_per_lane']},{t['waves']},{t['chunks']},{t['variant']}"


def read_profile(name, tile):
    """The 'key: value' lines of a committed rocprofv3 summary
    (profiles/<name>.txt) if it was taken with this tile shape, else None."""
    path = os.path.join(ROOT, "profiles", f"{name}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.lstrip().startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    return vals if vals.get("tile") == tile_str(tile) else None


def read_traffic(kernel_key, tile):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary
    (profiles/<kernel_key>_traffic.txt), if it was taken with this tile
    shape; None otherwise."""
    vals = read_profile(f"{kernel_key}_traffic", tile)
    try:
        return float(vals["hbm_bytes_per_launch"]) if vals else None
    except (KeyError, ValueError):
        return None


def counter_fractions(kernel_key, tile, ms, alg_flops):
    """The force kernel's fraction of peak taken apart, from committed
    rocprofv3 summaries taken with this tile and the launch time measured
    now (ms):
      counter_frac_fp64 / _fp32: FP64 / FP32 vector FLOP/s by the counters
        (64 (ADD + MUL + TRANS + 2 FMA) per launch,
        profiles/<kernel_key>_counters.txt) over the chip's peaks;
      sclk_sustained_ghz: the shader clock held while the kernel runs
        back to back (profiles/sclk_<kernel_key>.txt); the nominal peak
        assumes 2.4 GHz;
      issue_efficiency: the kernel's VALU work (SQ_ACTIVE_INST_VALU: busy
        quad-cycles, spread evenly over the 1024 SIMDs) at the sustained
        clock, over the launch time;
      mix_efficiency: algorithmic flops (20 N (N - 1)) over the flops that
        those VALU quad-cycles could issue at 128 per SIMD quad-cycle (one
        FP64 FMA per lane);
    so that frac = (sclk / 2.4) * issue_efficiency * mix_efficiency.
    None where no summary matches."""
    vals = read_profile(f"{kernel_key}_counters", tile)
    if not vals:
        return None
    try:
        f64 = float(vals["fp64_flops_per_launch"])
        f32 = float(vals["fp32_flops_per_launch"])
        quad = float(vals["SQ_ACTIVE_INST_VALU"])
    except (KeyError, ValueError):
        return None
    s = ms * 1e-3
    out = {"counter_frac_fp64": round(f64 / s / 1e12 / FP64_PEAK_TFLOPS, 4),
           "counter_frac_fp32": round(f32 / s / 1e12 / FP32_PEAK_TFLOPS, 4)}
    clk = read_profile(f"sclk_{kernel_key}", tile)
    if clk and "sclk_sustained_ghz" in clk:
        ghz = float(clk["sclk_sustained_ghz"])
        issue_s = quad / 1024 * 4 / (ghz * 1e9)
        out.update({"sclk_sustained_ghz": ghz,
                    "clock_frac": round(ghz / 2.4, 4),
                    "frac_of_sustained_clock_peak": round(
                        alg_flops / s / 1e12 / (FP64_PEAK_TFLOPS * ghz / 2.4), 4),
                    "issue_efficiency": round(issue_s / s, 4),
                    "mix_efficiency": round(alg_flops / (quad * 128), 4)})
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the force pass would "
              "shard by targets with a per-step all-gather of positions). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import solar_ics as S
    import paper_2112_15079_amd as nb

    if not torch.cuda.is_available():
        print("no GPU visible: the benchmark needs an MI355X", file=sys.stderr)
        sys.exit(3)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.workload == "copy":
        return bench_copy(torch, dev)
    if args.workload == "ensemble":
        return bench_ensemble(args, S, nb, torch, np, dev)
    if args.workload == "adjoint":
        return bench_adjoint(args, S, nb, torch, np, dev)
    if args.workload == "dt-scan":
        return bench_dt_scan(args, S, nb, torch, np, dev)
    if args.workload == "n-scan":
        return bench_n_scan(args, S, nb, torch, np, dev)
    if args.workload == "force":
        return bench_force(args, S, nb, torch, np, dev)
    if args.workload == "shard":
        return bench_shard(args, S, nb, torch, np, dev)
    k = {"solar-131": 0, "solar-10425": 1, "solar-131072": 2}[args.workload]
    return bench_single(args, k, S, nb, torch, np, dev)


def _t(a, torch, dev):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)


def settle_clock(nb, pos, m, G, prec, ms):
    """Untimed force passes on `pos` for about `ms` milliseconds of GPU work.
    The GPU raises its clock over the first tens of milliseconds of sustained
    load (a trace of one 1000-step run at N = 10,425 shows the force pass
    falling from 54 to 46.7 us over its first ~30 ms), so a timed window of a
    few steps that starts from an idle GPU measures that ramp rather than the
    kernels' sustained rate.  Nothing here changes the state of the run."""
    if ms <= 0:
        return
    per = nb.time_force(pos, m, G, prec, reps=3)
    nb.time_force(pos, m, G, prec, reps=max(1, int(ms / max(per, 1e-3))))


def bench_single(args, k, S, nb, torch, np_, dev):
    s = S.config(k)
    n, G, dt = s.n, s.G, s.dt
    K = args.steps if args.steps is not None else {0: 3650, 1: 10000, 2: 1000}[k]
    W = args.warmup if args.warmup is not None else {0: 365, 1: 200, 2: 10}[k]
    log(f"workload {s.name}: n={n}, dt={dt}, steps={K}, warmup={W}")
    pos0, vel0, m = _t(s.pos, torch, dev), _t(s.vel, torch, dev), _t(s.mass, torch, dev)

    tiles = {}
    for prec, fixed in (("fp64", args.tile), ("split", args.split_tile)):
        if fixed:
            nb.set_tile(0, prec, n, *[int(x) for x in fixed.split(",")])
        elif args.tune:
            tile, ms = nb.autotune(pos0, m, G, prec)
            log(f"autotune {prec}: {tile} {ms:.4f} ms per force pass")
        tiles[prec] = nb.get_tile(0, prec, n)

    E0 = nb.energy(pos0, vel0, m, G)[2].item()
    results = {}
    for prec in ("fp64", "split", "compensated"):
        # the same buffers for the warm-up and the timed run: captured step
        # graphs are keyed by the buffers they run on
        p, v = pos0.clone(), vel0.clone()
        nb.verlet_run(p, v, m, G, dt, W, precision=prec)        # warm-up (graphs, caches)
        p.copy_(pos0)
        v.copy_(vel0)
        settle_clock(nb, pos0, m, G, prec, args.settle_ms)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record()
        nb.verlet_run(p, v, m, G, dt, K, precision=prec)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_s = ev0.elapsed_time(ev1) / 1e3
        E1 = nb.energy(p, v, m, G)[2].item()
        results[prec] = dict(wall=wall, gpu=gpu_s, E=E1, pos=p, vel=v)
        log(f"{prec}: {K} steps in {wall:.4f} s wall ({gpu_s:.4f} s events), "
            f"dE/E = {(E1 - E0) / abs(E0):.3e}")

    pairs = n * (n - 1)
    r64, rsp = results["fp64"], results["split"]

    def rate(r):
        return (K + 1) * pairs / r["wall"], K / r["wall"]

    v64, sps64 = rate(r64)
    vsp, spssp = rate(rsp)

    rcp = results["compensated"]
    vcp, spscp = rate(rcp)
    reps = args.force_reps or max(20, min(2000, int(2e11 / pairs)))
    mscp = nb.time_force(pos0, m, G, "compensated", reps=reps)
    comp = {"pairs_per_s": vcp, "steps_per_s": spscp, "ms_per_step": 1e3 * rcp["wall"] / K,
            "dE_over_E": (rcp["E"] - E0) / abs(E0),
            "E_minus_E_fp64_over_E0": (rcp["E"] - r64["E"]) / abs(E0),
            "speedup_vs_fp64": vcp / v64, "ms_per_launch": round(mscp, 5),
            "tile": nb.get_tile(0, "compensated", n), "gpu_event_s": rcp["gpu"],
            "form": "split as specified: FP64 d and r^2, FP32 rsqrt + one FP64 Newton step, "
                    "light terms in FP32 Kahan sums"}

    # force-kernel timing for the roofline (HIP events around the force kernels only)
    ms64 = nb.time_force(pos0, m, G, "fp64", reps=reps)
    mssp = nb.time_force(pos0, m, G, "split", reps=reps)
    t64 = tiles["fp64"]
    roof = roofline(n, t64, ms64, mssp)
    log(f"force pass: fp64 {ms64:.4f} ms ({roof['achieved']:.2f} TFLOP/s alg.), "
        f"split {mssp:.4f} ms")

    line = {
        "metric": metric_at(n),
        "value": v64,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "settle_ms": args.settle_ms,
        "ms_per_step": 1e3 * r64["wall"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{s.name}: Sun, {s.counts.get('major', 0)} major, "
                               f"{s.counts.get('moons', 0)} moons, {s.counts.get('heavy', 0)} heavy, "
                               f"{s.counts.get('small', 0)} small asteroids; seed {k if k < 3 else ''}",
                   "n": n, "dt_days": dt, "steps": K, "tile": tiles["fp64"]},
        "steps_per_s": sps64,
        "fp64": {"pairs_per_s": v64, "steps_per_s": sps64, "dE_over_E": (r64["E"] - E0) / abs(E0),
                 "gpu_event_s": r64["gpu"]},
        "split": {"pairs_per_s": vsp, "steps_per_s": spssp, "ms_per_step": 1e3 * rsp["wall"] / K,
                  "dE_over_E": (rsp["E"] - E0) / abs(E0),
                  "E_split_minus_E_fp64_over_E0": (rsp["E"] - r64["E"]) / abs(E0),
                  "speedup_vs_fp64": vsp / v64,
                  "tile": tiles["split"], "gpu_event_s": rsp["gpu"]},
        "split_compensated": comp,
        "roofline": roof,
    }
    if k == 1 and not args.no_extra_legs:
        line["paper_run"] = paper_run(nb, torch, pos0, vel0, m, G, dt)
        line["rk4"] = rk4_rate(nb, torch, pos0, vel0, m, G, dt, n)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds, k)
        line["cpu_baseline"]["accel_max_rel_err_of_gpu"] = oracle_accel_errors(nb, s, pos0, m, G)
    print(json.dumps(line), flush=True)


KERNEL_NAMES = {0: "k_force (LDS tiles)", 1: "k_force_s (scalar operands)",
                2: "k_force_s (shared targets)", 3: "k_run_small (one workgroup)",
                4: "k_step_fused (force pass and step)", 5: "k_force_mutual (each pair once)"}


def roofline(n, tile, ms64, mssp):
    """Roofline object of the FP64 force kernel: algorithmic flops per launch
    (20 N (N - 1)) over its measured launch time against the FP64 vector peak;
    for the each-pair-once kernel also its own arithmetic (27 flops per
    unordered pair); counter fractions and HBM traffic from committed
    rocprofv3 summaries taken with the same tile."""
    pairs = n * (n - 1)
    flops = FLOPS_PER_PAIR * pairs
    achieved = flops / (ms64 * 1e-3) / 1e12
    roof = {"bound": "alu",
            "kernel": KERNEL_NAMES[tile["variant"]] + f" FP64, tile {tile_str(tile)}",
            "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
            "traffic": read_traffic(f"force_fp64_n{n}", tile),
            "ms_per_launch": round(ms64, 5), "flops_per_launch": flops,
            "split_ms_per_launch": round(mssp, 5)}
    if tile["variant"] == 5:
        own = FLOPS_PER_MUTUAL_PAIR * pairs // 2
        a = own / (ms64 * 1e-3) / 1e12
        roof["own_arithmetic"] = {"flops_per_launch": own, "achieved": round(a, 3),
                                  "frac": round(a / FP64_PEAK_TFLOPS, 4)}
    cf = counter_fractions(f"force_fp64_n{n}", tile, ms64, flops)
    if cf:
        roof.update(cf)
    return roof


def bench_force(args, S, nb, torch, np_, dev):
    """The force passes alone on the 10,425-body system (no step loop, no
    graphs): the command the counter profiles are taken with."""
    s = S.config(1)
    n, G = s.n, s.G
    pos0, m = _t(s.pos, torch, dev), _t(s.mass, torch, dev)
    reps = args.force_reps or 200
    out = {"metric": "force pass time", "unit": "ms", "n": n, "reps": reps, "n_gpus": 1,
           "dtype": "f64", "data": "synthetic"}
    for prec in ("fp64", "split", "compensated"):
        settle_clock(nb, pos0, m, G, prec, args.settle_ms)
        out[prec] = {"ms_per_launch": nb.time_force(pos0, m, G, prec, reps=reps),
                     "tile": nb.get_tile(0, prec, n)}
        log(f"force {prec}: {out[prec]['ms_per_launch']:.4f} ms per launch")
    out["roofline"] = roofline(n, out["fp64"]["tile"], out["fp64"]["ms_per_launch"],
                               out["split"]["ms_per_launch"])
    # the adjoint's transpose-Jacobian pass at the same size: 47 flops per
    # ordered pair (d 3, |d|^2 5, rsqrt 1, the powers 3, m_q u_j - m_j u_q 9,
    # d.w 5, its scale 2, the tidal product 12, the mass term 7)
    # (the default tile: each pair once at this size; the one-way pass beside it)
    settle_clock(nb, pos0, m, G, "fp64", args.settle_ms)
    for key, tile in (("vjp", None), ("vjp_one_way", (1, 2, 64, 1))):
        if tile is not None:
            nb.set_tile(1, "fp64", n, *tile)
        msv = nb.time_force(pos0, m, G, "fp64", kind=1, reps=max(20, reps // 4))
        tfv = VJP_FLOPS_PER_PAIR * n * (n - 1) / (msv * 1e-3) / 1e12
        out[key] = {"ms_per_launch": msv, "tile": nb.get_tile(1, "fp64", n),
                    "flops_per_ordered_pair": VJP_FLOPS_PER_PAIR, "achieved_tflops": tfv,
                    "frac": tfv / FP64_PEAK_TFLOPS}
        log(f"{key}: {msv:.4f} ms per launch, {tfv:.2f} TFLOP/s "
            f"({tfv / FP64_PEAK_TFLOPS:.3f} of peak)")
    nb.reset_caches()
    print(json.dumps(out), flush=True)


def bench_shard(args, S, nb, torch, np_, dev):
    """One GPU's share of the force pass when the 131,072-body system's
    targets are split over 8 GPUs (16,384 targets against all 131,072
    sources each): every share timed on this GPU with HIP events around
    back-to-back calls of nbody_accel_shard (work-list upload, G m, the
    one-way force kernel and the fixed-order sum), beside the single-GPU
    each-pair-once pass over the whole system."""
    s = S.config(2)
    n, G, gpus = s.n, s.G, 8
    pos, m = _t(s.pos, torch, dev), _t(s.mass, torch, dev)
    reps = args.force_reps or 20
    w = -(-n // gpus)
    rows = []
    outs = [nb.accel_shard(pos, m, G, k * w, min(w, n - k * w)) for k in range(gpus)]  # work lists
    settle_clock(nb, pos, m, G, "fp64", args.settle_ms)
    for k in range(gpus):
        t0, nt = k * w, min(w, n - k * w)
        out = outs[k]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            nb.accel_shard(pos, m, G, t0, nt, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        pairs = nt * (n - 1)
        tf = FLOPS_PER_PAIR * pairs / (ms * 1e-3) / 1e12
        rows.append({"t0": t0, "nt": nt, "ms": ms, "pairs_per_s": pairs / (ms * 1e-3),
                     "achieved_tflops": tf, "frac": tf / FP64_PEAK_TFLOPS})
        log(f"share {k}: targets [{t0}, {t0 + nt}) {ms:.4f} ms, {pairs / (ms * 1e-3):.3e} pairs/s, "
            f"frac {tf / FP64_PEAK_TFLOPS:.3f}")
    ms_full = nb.time_force(pos, m, G, "fp64", reps=reps)
    worst = max(r["ms"] for r in rows)
    print(json.dumps({"metric": "one GPU's share of the force pass, 8-way split of the targets",
                      "unit": "pair interactions/s", "n": n, "gpus_modelled": gpus, "reps": reps,
                      "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "solar-131072, seed 2; shares of 16,384 targets"},
                      "tile": "one-way force kernel (the full pass's one-way tile, chunks per share)",
                      "shares": rows, "slowest_share_ms": worst,
                      "whole_pass_one_gpu_ms": ms_full,
                      "whole_pass_one_gpu_tile": nb.get_tile(0, "fp64", n),
                      "force_pass_speedup_8_shares_vs_one_gpu": ms_full / worst}), flush=True)


def rk4_rate(nb, torch, pos0, vel0, m, G, dt, n, steps=1000):
    """Throughput of the fourth-order Runge-Kutta method (four force passes
    per step) on the same system, FP64, state resident on the GPU."""
    p, v = pos0.clone(), vel0.clone()
    nb.rk4_run(p, v, m, G, dt, 64)                          # warm-up on these buffers
    p.copy_(pos0)
    v.copy_(vel0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nb.rk4_run(p, v, m, G, dt, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"rk4: {steps} steps in {wall:.4f} s")
    return {"steps": steps, "steps_per_s": steps / wall,
            "pairs_per_s": 4 * steps * n * (n - 1) / wall, "force_passes_per_step": 4}


PAPER_RUN_S = 23 * 60.0   # Sec. 5: 10^4 bodies, 10^2 days at 0.1 day, 176 CPU processors


def paper_run(nb, torch, pos0, vel0, m, G, dt):
    """The paper's production-run shape on this system: 10^2 days = 10^3
    steps, wall clock with the state resident on the GPU; the paper's time
    on 176 CPU processors is context (other hardware, 10^4 bodies)."""
    out = {"steps": 1000, "days": 1000 * dt, "paper_wall_s": PAPER_RUN_S,
           "paper_hardware": "176 CPU processors, vectorised MPI, 10^4 bodies (Sec. 5)"}
    for prec in ("fp64", "split"):
        p, v = pos0.clone(), vel0.clone()
        nb.verlet_run(p, v, m, G, dt, 1000, precision=prec)     # warm-up on these buffers
        p.copy_(pos0)
        v.copy_(vel0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nb.verlet_run(p, v, m, G, dt, 1000, precision=prec)
        torch.cuda.synchronize()
        out[f"{prec}_wall_s"] = time.perf_counter() - t0
    out["fp64_speedup_vs_paper"] = PAPER_RUN_S / out["fp64_wall_s"]
    log(f"paper-shaped run (10^3 steps): fp64 {out['fp64_wall_s']:.4f} s, "
        f"split {out['split_wall_s']:.4f} s (paper: {PAPER_RUN_S:.0f} s on 176 CPUs)")
    return out


def cpu_baseline(s, budget_s, k):
    """The oracle (plain FP64 C, OpenMP over targets) on this host's cores, on
    a bounded prefix of the same run."""
    import oracle
    n = s.n
    t1, _, _ = oracle.timed_verlet(s.pos, s.vel, s.mass, s.G, s.dt, 1)   # 2 force passes
    per_pass = t1 / 2
    # a prefix of the workload's own run (all of it when that fits the budget)
    steps = int(max(1, min(s.steps or 2000, budget_s / max(per_pass, 1e-9) - 1)))
    log(f"cpu baseline: oracle on {oracle.get_threads()} threads, {steps} steps")
    t, _, _ = oracle.timed_verlet(s.pos, s.vel, s.mass, s.G, s.dt, steps)
    pairs = (steps + 1) * n * (n - 1)
    return {"value": pairs / t, "unit": "pair interactions/s", "cores": oracle.get_threads(),
            "kind": "oracle", "steps_per_s": steps / t,
            "sample": f"first {steps} steps of the same {n}-body run ({steps + 1} force passes, "
                      f"{t:.1f} s)",
            "host_cpus": os.cpu_count()}


def oracle_accel_errors(nb, s, pos0, m, G):
    """Part of the CPU-baseline leg: the largest relative error of each
    precision form's accelerations at the initial state against the oracle
    (all bodies up to 20,000, else the first, the last and 254 seeded ones)."""
    import oracle
    n = s.n
    if n <= 20000:
        a_ref = oracle.accel(s.pos, s.mass, G)
        idx = None
    else:
        rng = np.random.default_rng(0)
        idx = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 254, replace=False)]))
        a_ref = oracle.accel_targets(s.pos, s.mass, G, idx)
    out = {}
    for prec in ("fp64", "split", "compensated"):
        a = nb.accel(pos0, m, G, precision=prec).cpu().numpy()
        if idx is not None:
            a = a[:, idx]
        out[prec] = float(np.max(np.linalg.norm(a - a_ref, axis=0)
                                 / np.linalg.norm(a_ref, axis=0)))
    out["targets"] = "all" if idx is None else f"{len(idx)} sampled"
    return out


def bench_copy(torch, dev):
    """A plain streaming kernel of known size (y = 1.0 * x over 256 MiB: reads
    256 MiB, writes 256 MiB): the reference that scales the FETCH_SIZE /
    WRITE_SIZE counters to bytes."""
    nbytes = 256 << 20
    x = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for _ in range(5):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        torch.mul(x, 1.0, out=y)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 10
    print(json.dumps({"metric": "device copy", "bytes_read": nbytes, "bytes_written": nbytes,
                      "ms": ms, "GB_per_s": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)


def bench_ensemble(args, S, nb, torch, np, dev):
    K = args.steps if args.steps is not None else 1000
    W = args.warmup if args.warmup is not None else 5
    log("building the 512-system ensemble")
    systems, offs = S.ensemble(512)
    cat = lambda f: np.ascontiguousarray(np.concatenate([f(x) for x in systems], axis=-1))
    pos0, vel0, m = (_t(cat(lambda x: x.pos), torch, dev), _t(cat(lambda x: x.vel), torch, dev),
                     _t(cat(lambda x: x.mass), torch, dev))
    G, dt = S.G_AU_DAY_MSUN, 0.1
    pairs = int(sum(x.n * (x.n - 1) for x in systems))
    out = {"metric": "ensemble pair interactions/s", "unit": "pair interactions/s", "steps": K,
           "warmup": W, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "512 systems: Sun, 30 majors, U{100..8192} asteroids, seeds 100..611",
                      "bodies": int(offs[-1]), "pairs_per_step": pairs}}
    for prec in ("fp64", "split"):
        tile, ms = nb.autotune_batched(pos0, m, offs, G, prec)
        log(f"autotune ensemble {prec}: {tile} {ms:.3f} ms per force pass")
        out.setdefault("tiles", {})[prec] = tile
        p, v = pos0.clone(), vel0.clone()
        nb.verlet_run_batched(p, v, m, offs, G, dt, W, precision=prec)
        torch.cuda.synchronize()
        p, v = pos0.clone(), vel0.clone()
        t0 = time.perf_counter()
        nb.verlet_run_batched(p, v, m, offs, G, dt, K, precision=prec)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[prec] = {"pairs_per_s": (K + 1) * pairs / wall, "steps_per_s": K / wall, "wall_s": wall}
        log(f"ensemble {prec}: {wall:.3f} s, {(K + 1) * pairs / wall:.3e} pairs/s")
    out["value"] = out["fp64"]["pairs_per_s"]
    print(json.dumps(out), flush=True)


def bench_adjoint(args, S, nb, torch, np, dev):
    """The adjoint workload: 2,079 bodies, 36,500 steps, checkpoints every
    100; its gradient against central finite differences (relative step
    1e-7) on 64 coordinates.  For L = sum_asteroids |delta|^2 (delta = final
    position minus the target run's) the two-point quotient of L equals the
    two-point difference of delta applied to dL/dr_T (2 delta0 . J) plus a
    curvature term h^2 J . H known exactly from the same three runs; both
    are reported against the adjoint, with each coordinate's finite-
    difference error bound: how far the same quotient moves when its step is
    doubled and halved."""
    s = S.config(4)
    K = args.steps if args.steps is not None else s.steps
    n, G, dt = s.n, s.G, s.dt
    first = 1 + s.counts["major"]
    m = _t(s.mass, torch, dev)
    pt, vt = _t(S.adjoint_target_perturbation(s), torch, dev), _t(s.vel, torch, dev)
    nb.verlet_run(pt, vt, m, G, dt, K)
    tgt = pt.cpu().numpy()[:, first:]

    def delta(p0, v0, m0):
        p, v = _t(p0, torch, dev), _t(v0, torch, dev)
        nb.verlet_run(p, v, _t(m0, torch, dev), G, dt, K)
        return p.cpu().numpy()[:, first:] - tgt

    d0 = delta(s.pos, s.vel, s.mass)
    lam = np.zeros((3, n))
    lam[:, first:] = 2 * d0
    args_adj = (_t(s.pos, torch, dev), _t(s.vel, torch, dev), m, G, dt, K, 100,
                _t(lam, torch, dev), _t(np.zeros_like(lam), torch, dev))
    nb.verlet_adjoint(*args_adj)                       # warm-up (graphs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gr, gv, gm, _, _ = nb.verlet_adjoint(*args_adj)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    # the same gradient in two calls: the forward run keeping its checkpoints
    # (what an autograd forward pass runs), then the reverse sweep alone
    r0, v0 = args_adj[0], args_adj[1]
    lam_r, lam_v = args_adj[7], args_adj[8]
    _, _, ck = nb.verlet_checkpoints(r0, v0, m, G, dt, K, 100)
    nb.verlet_adjoint_from_checkpoints(ck, m, G, dt, K, 100, lam_r, lam_v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, ck = nb.verlet_checkpoints(r0, v0, m, G, dt, K, 100)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    g2 = nb.verlet_adjoint_from_checkpoints(ck, m, G, dt, K, 100, lam_r, lam_v)
    torch.cuda.synchronize()
    t_rev = time.perf_counter() - t0 - t_fwd
    same = all(torch.equal(x, y) for x, y in zip(g2, (gr, gv, gm)))
    log(f"adjoint of {K} steps: {t_adj:.3f} s in one call; forward with checkpoints "
        f"{t_fwd:.3f} s + reverse sweep {t_rev:.3f} s (bitwise equal: {same})")
    grad = np.concatenate([gr.cpu().numpy().ravel(), gv.cpu().numpy().ravel(),
                           gm.cpu().numpy()[1:31]])
    coords = S.fd_coordinates(s, args.fd_coords)
    rows = []
    for idx in coords:
        p0, v0, m0 = s.pos.copy(), s.vel.copy(), s.mass.copy()
        if idx < 3 * n:
            arr, flat, scale = p0, idx, max(abs(p0.ravel()[idx]), 1.0)
        elif idx < 6 * n:
            arr, flat = v0, idx - 3 * n
            scale = max(abs(v0.ravel()[flat]), 0.01)
        else:
            arr, flat = m0, 1 + idx - 6 * n
            scale = m0[flat]
        base = arr.ravel()[flat]
        h = 1e-7 * scale

        def pair(k):
            arr.ravel()[flat] = base + k
            a = delta(p0, v0, m0)
            arr.ravel()[flat] = base - k
            b = delta(p0, v0, m0)
            arr.ravel()[flat] = base
            return a, b

        dp, dm = pair(h)
        J = (dp - dm) / (2 * h)
        fd_state = float(2 * np.sum(d0 * J))
        curv = float(np.sum(J * ((dp - d0) + (dm - d0))))
        fd_loss = float(np.sum((dp - dm) * (dp + dm)) / (2 * h))
        # the quotient's own error: how far it moves for steps 2h and h/2
        fd_k = [float(2 * np.sum(d0 * (a - b)) / (2 * k))
                for k in (2 * h, 0.5 * h) for a, b in (pair(k),)]
        bound = abs(fd_k[0] - fd_state) + abs(fd_k[1] - fd_state)
        rows.append((int(idx), float(grad[idx]), fd_state, fd_loss, curv, bound))
        log(f"coord {idx}: adjoint {grad[idx]: .9e} fd_state {fd_state: .9e} "
            f"fd_loss {fd_loss: .9e} curvature {curv: .3e} fd error bound {bound: .3e}")
    g, fs, fl, cv, bd = (np.array([r[i] for r in rows]) for i in range(1, 6))
    floor = 1e-9 * np.abs(fs).max()
    big = np.abs(fs) > floor
    rel_s = np.abs(g - fs) / np.maximum(np.abs(fs), 1e-300)
    rel_l = np.abs(g - fl) / np.maximum(np.abs(fl), 1e-300)
    resolved = bd <= 1e-7 * np.abs(fs)
    out = {"metric": "adjoint vs central finite differences", "steps": K, "n": n,
           "checkpoint_every": 100, "adjoint_s": t_adj, "forward_with_checkpoints_s": t_fwd,
           "reverse_sweep_s": t_rev, "split_calls_bitwise_equal": bool(same), "coords": len(rows),
           "rel_step": 1e-7, "rows": rows,
           "fd_state": {"pass_1e-6": int(((rel_s <= 1e-6) | ~big).sum()),
                        "resolved": int((resolved & big).sum()),
                        "resolved_pass_1e-6": int(((rel_s <= 1e-6) & resolved & big).sum()),
                        "pass_1e-6_plus_fd_error_bound": int(((np.abs(g - fs) <= 1e-6 * np.abs(fs)
                                                              + bd) | ~big).sum()),
                        "median_fd_error_bound_rel": float(np.median(bd[big] / np.abs(fs[big])))
                        if big.any() else 0.0,
                        "max_rel_err": float(rel_s[big].max()) if big.any() else 0.0,
                        "median_rel_err": float(np.median(rel_s[big])) if big.any() else 0.0},
           "fd_loss": {"pass_1e-6": int(((rel_l <= 1e-6) | ~big).sum()),
                       "pass_1e-6_plus_curvature": int(((np.abs(g - fl) <= 1e-6 * np.abs(fl)
                                                        + np.abs(cv)) | ~big).sum()),
                       "max_rel_err": float(rel_l[big].max()) if big.any() else 0.0,
                       "median_rel_err": float(np.median(rel_l[big])) if big.any() else 0.0,
                       "median_curvature_share": float(np.median(np.abs(cv[big]) / np.abs(fl[big])))
                       if big.any() else 0.0},
           "negligible_coords": int((~big).sum())}
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# accuracy against the step size (the paper's Sec. 4 study, on synthetic data)

def orbit_energy(pos, vel, mass, G, bodies, parents):
    """Two-body orbital energy per unit mass of each body about its parent:
    |v_b - v_P|^2 / 2 - G (m_P + m_b) / |r_b - r_P|."""
    dr = pos[:, bodies] - pos[:, parents]
    dv = vel[:, bodies] - vel[:, parents]
    return (0.5 * np.einsum("ki,ki->i", dv, dv)
            - G * (mass[parents] + mass[bodies]) / np.sqrt(np.einsum("ki,ki->i", dr, dr)))


def dt_scan_system(S, n=5000, seed=20, n_moons=100, n_heavy=19):
    """Sun, 30 major bodies, minor moons, heavy asteroids and small asteroids
    (by default the 10,425-body workload's populations at N = 5000)."""
    return S.solar_system(seed, n - 31 - n_moons - n_heavy, n_moons=n_moons, n_heavy=n_heavy,
                          n_major=30, name=f"solar-{n}-dt-scan")


def gpu_stepper(nb, torch, dev, s, precision="fp64", integrator="verlet"):
    """advance(dt) -> step(k) running k steps of size dt on the GPU from the
    system's initial state (velocity Verlet, or the fourth-order Runge-Kutta
    method with integrator="rk4"); step returns (pos, vel, total energy) on
    the host."""
    run = nb.verlet_run if integrator == "verlet" else nb.rk4_run
    m = torch.tensor(s.mass, dtype=torch.float64, device=dev)

    def start(dt):
        p = torch.tensor(s.pos, dtype=torch.float64, device=dev)
        v = torch.tensor(s.vel, dtype=torch.float64, device=dev)

        def step(k):
            run(p, v, m, s.G, dt, k, precision=precision)
            return p.cpu().numpy(), v.cpu().numpy(), nb.energy(p, v, m, s.G)[2].item()
        return step
    return start


def dt_scan(start, s, dts, days, sample_days, dt_ref):
    """Runs the system for `days` at each step size and at dt_ref (the
    reference), sampling every `sample_days`; returns per-dt errors against
    the reference: the orbital energy about its parent of the innermost major
    body and of the moon with the shortest period, positions, and the
    total-energy error."""
    G = s.G
    nmaj = s.counts["major"]
    parents = s.parent          # the body each body was placed about (0: the Sun)
    majors = np.arange(1, 1 + nmaj)
    a = np.linalg.norm(s.pos[:, majors] - s.pos[:, :1], axis=0)
    inner = int(majors[np.argmin(a)])
    moons = np.nonzero(parents > 0)[0]
    dr = np.linalg.norm(s.pos[:, moons] - s.pos[:, parents[moons]], axis=0)
    period = 2 * np.pi * np.sqrt(dr ** 3 / (G * (s.mass[parents[moons]] + s.mass[moons])))
    moon = int(moons[np.argmin(period)]) if moons.size else inner
    bodies = np.array([inner, moon])
    samples = int(round(days / sample_days))
    E0 = None

    def run(dt):
        nonlocal E0
        k = int(round(sample_days / dt))
        if abs(k * dt - sample_days) > 1e-9 * sample_days:
            raise ValueError(f"dt = {dt} does not divide the sampling interval {sample_days}")
        step = start(dt)
        if E0 is None:
            E0 = step(0)[2]
        eps, dE, t0 = [], [], time.perf_counter()
        for _ in range(samples):
            P, V, E = step(k)
            eps.append(orbit_energy(P, V, s.mass, G, bodies, parents[bodies]))
            dE.append((E - E0) / abs(E0))
        return np.array(eps), np.array(dE), P, time.perf_counter() - t0, samples * k

    eps_ref, dE_ref, P_ref, wall_ref, steps_ref = run(dt_ref)
    rows = []
    for dt in dts:
        eps, dE, P, wall, steps = run(dt)
        err = np.max(np.abs(eps - eps_ref) / np.abs(eps_ref), axis=0)
        pos_err = np.linalg.norm(P - P_ref, axis=0)
        rows.append({"dt": dt, "steps": steps, "wall_s": wall,
                     "dE_over_E_max": float(np.max(np.abs(dE))),
                     "inner_major_orbit_energy_err": float(err[0]),
                     "moon_orbit_energy_err": float(err[1]),
                     "max_pos_err_au": float(pos_err.max()),
                     "inner_major_pos_err_au": float(pos_err[inner]),
                     "moon_pos_err_au": float(pos_err[moon])})
        log(f"dt={dt}: {steps} steps {wall:.2f} s, max|dE/E|={rows[-1]['dE_over_E_max']:.3e}, "
            f"orbit energy err: inner major {err[0]:.3e}, moon {err[1]:.3e}")
    orders = {}
    # (the largest position error over all bodies is set by chaotic close
    # encounters and does not converge; the two tracked bodies do)
    for key in ("dE_over_E_max", "inner_major_orbit_energy_err", "moon_orbit_energy_err",
                "inner_major_pos_err_au", "moon_pos_err_au"):
        orders[key] = [float(np.log2(rows[i][key] / rows[i + 1][key]))
                       for i in range(len(rows) - 1)]
    return {"bodies": {"inner_major": inner, "moon": moon,
                       "moon_period_days": float(period.min()) if moons.size else None,
                       "inner_major_distance_au": float(a.min())},
            "reference": {"dt": dt_ref, "steps": steps_ref, "wall_s": wall_ref,
                          "dE_over_E_max": float(np.max(np.abs(dE_ref)))},
            "rows": rows, "orders_log2_ratio": orders}


def bench_dt_scan(args, S, nb, torch, np_, dev):
    s = dt_scan_system(S)
    dts = [0.4, 0.2, 0.1, 0.05, 0.025]
    days = 1500.0
    log(f"dt scan: n={s.n}, {days:.0f} days, dt in {dts}, reference dt 0.00625")
    res = dt_scan(gpu_stepper(nb, torch, dev, s), s, dts, days, 10.0, 0.00625)
    log("the fourth-order Runge-Kutta method, dt in [0.4, 0.2, 0.1, 0.05], reference dt 0.0125")
    res_rk4 = dt_scan(gpu_stepper(nb, torch, dev, s, integrator="rk4"), s, [0.4, 0.2, 0.1, 0.05],
                      days, 10.0, 0.0125)
    out = {"metric": "accuracy against the step size", "unit": "relative error",
           "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{s.name}: Sun, 30 major, 100 moons, 19 heavy, "
                                  f"{s.n - 150} small asteroids; seed 20",
                      "n": s.n, "days": days, "sample_every_days": 10.0}}
    out.update(res)
    out["rk4"] = res_rk4
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# throughput against N (the paper's Sec. 5 scaling study, GPU beside the oracle)

SCAN_N = (100, 131, 300, 1000, 3000, 10425, 30000, 131072)


def oracle_scan_rates(s, n):
    """CPU-baseline leg of the N scan: the oracle's force-pass rate on one
    thread and on all of them, over a sample of targets."""
    import oracle
    row = {}
    all_threads = oracle.get_threads()
    for threads, budget in ((1, 1.5e8), (all_threads, 2.5e9)):
        oracle.set_threads(threads)
        count = int(min(n, max(1, budget / n)))
        idx = np.linspace(0, n - 1, count).astype(np.int64)
        reps, t0 = 0, time.perf_counter()
        while reps == 0 or time.perf_counter() - t0 < 0.3:
            oracle.accel_targets(s.pos, s.mass, s.G, idx)
            reps += 1
        dt_cpu = (time.perf_counter() - t0) / reps
        row[f"oracle_{'all' if threads == all_threads else 1}t_pairs_per_s"] = \
            count * (n - 1) / dt_cpu
    oracle.set_threads(all_threads)
    row["oracle_threads"] = all_threads
    return row


def bench_n_scan(args, S, nb, torch, np_, dev):
    rows = []
    for i, n in enumerate(SCAN_N):
        s = S.solar_system(30 + i, n - 31, n_major=30, name=f"scan-{n}")
        pairs = n * (n - 1)
        m = _t(s.mass, torch, dev)
        K = int(min(4000, max(10, 2e11 / pairs)))
        row = {"n": n, "steps": K}
        for prec in ("fp64", "split"):
            if args.tune:
                nb.autotune(_t(s.pos, torch, dev), m, s.G, prec)
            pos0, vel0 = _t(s.pos, torch, dev), _t(s.vel, torch, dev)
            p, v = pos0.clone(), vel0.clone()
            nb.verlet_run(p, v, m, s.G, s.dt, max(2, K // 10), precision=prec)
            p.copy_(pos0)
            v.copy_(vel0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nb.verlet_run(p, v, m, s.G, s.dt, K, precision=prec)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            row[prec] = {"pairs_per_s": (K + 1) * pairs / wall, "steps_per_s": K / wall,
                         "tile": nb.get_tile(0, prec, n)}
        msg = (f"n={n}: fp64 {row['fp64']['pairs_per_s']:.3e} pairs/s "
               f"({row['fp64']['steps_per_s']:.0f} steps/s), split {row['split']['pairs_per_s']:.3e}")
        if not args.no_cpu_baseline:
            row.update(oracle_scan_rates(s, n))
            msg += (f"; oracle 1t {row['oracle_1t_pairs_per_s']:.3e}, "
                    f"{row['oracle_threads']}t {row['oracle_allt_pairs_per_s']:.3e}")
        log(msg)
        rows.append(row)
    print(json.dumps({"metric": "pair interactions/s against N", "unit": "pair interactions/s",
                      "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": "Sun + 30 major bodies + N - 31 small asteroids, "
                                             "seeds 30..37, dt 0.1 day"},
                      "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
