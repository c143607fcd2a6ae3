"""Throughput benchmark of the TENO7X operator on MI355X: 2D Euler, 4096 x 4096, FP64, SSP-RK3.

One step = one SSP-RK3 step of the whole hot path: CFL dt from the state on the device, three
evaluations of the semi-discrete operator (x- and y-sweeps: Roe-averaged characteristic
projection, GLF splitting, TENO5 flags, neighbour-vector selection (Table 3), Table 2
reconstruction, conservative difference) and the three stage updates with the wave-speed
maxima of each produced state. Input: the seeded four-quadrant Riemann state with a vortex,
resident in HBM before the timed region. The step is captured once in a HIP graph and replayed.

value = cells * 3 * steps / wall time  (cell-updates per second, one GPU), reported in Gcell-updates/s.

Prints one JSON line: the throughput; `roofline` for the x-sweep + stage kernel (algorithmic FP64
flops per launch over its HIP-event launch time, against the FP64 vector peak, with the HBM bytes per
launch from the committed rocprofv3 counter summary while its kernel-source hash matches); `hbm`;
per-kernel times; the batched, FP32, TENO5 and adjoint side runs; and `cpu_baseline`, the oracle
timed on one host core over a bounded strip of the same state.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM = 8.0e12           # B/s
PEAK_FP64_VALU = 78.6e12    # FLOP/s (vector FP64)

# Algorithmic work per cell of one sweep kernel, 2D Euler FP64 (derivation in the design notes):
# per face 1156 flops (Roe average 23, L 15, R 6, projection 368, GLF split 160, smoothness and
# cut-off of 2 sides x 4 fields 456, reconstruction 108, back-projection 20), per cell 16 (primitive
# variables, H, sqrt(rho), physical flux) + 8 (conservative difference).
FLOPS_YSWEEP = 1156 + 16 + 8
# the x-sweep also adds the y-part (4), applies the RK stage (16) and the wave speeds of the
# produced state (25)
FLOPS_XSTAGE = 1156 + 16 + 8 + 4 + 16 + 25
# algorithmic HBM bytes per cell-update of a fused stage: read U^(k) and write U^(k+1) (64 B),
# plus U^n at stages 2 and 3 (32 B): mean 85.3 B
BYTES_PER_CELL_UPDATE = (64 + 96 + 96) / 3.0

METRIC = "2D Euler RHS Gcell-updates/s, %HBM peak; batched vs plain; adjoint/fwd cost"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("teno_device.hpp", "teno_lib.hip"):
        with open(os.path.join(ROOT, "paper_1808_00037_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_x_stage_euler2d_4096_traffic.txt")


def measured_traffic():
    """HBM bytes per launch of the x-sweep stage kernel from the committed rocprofv3 --pmc
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the same counters' reading for a plain copy
    kernel), if it was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != kernel_source_hash():
        return None
    try:
        return float(kv["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_peaks():
    """Peaks measured on this device beside the published ones: a plain device-to-device copy of
    1 GiB (read + write bytes over its time, best of 5) and the library's FP64 vector FMA probe."""
    import torch
    from paper_1808_00037_amd import teno as T

    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    copy_gbps = 2 * src.numel() * 8 / (best / 1e3) / 1e9
    del src, dst
    fma = max(T.probe_fp64_fma(32768) for _ in range(3))
    return {"copy_GBps": copy_gbps, "fp64_fma_TFLOPs": fma}


def cpu_baseline(problem, budget_s=12.0):
    """The oracle (plain C, one thread) on a bounded sample of the same workload: one operator
    evaluation on a horizontal strip of the 4096^2 state (periodic), the strip height chosen so
    that the sample takes about budget_s seconds."""
    import numpy as np
    from oracle import oracle as O

    def timed(rows):
        U = np.ascontiguousarray(problem.U0[:, :rows, :])
        cfg = O.Config(O.EULER2D, problem.nx, rows, 0.0, 1.0, 0.0, rows / problem.ny)
        t0 = time.perf_counter()
        O.rhs(cfg, U)
        return time.perf_counter() - t0

    t_probe = timed(16)
    rate = problem.nx * 16 / t_probe
    rows = int(min(problem.ny, max(16, budget_s * rate / problem.nx)))
    t = timed(rows)
    cells = problem.nx * rows
    return {"value": cells / t / 1e9, "unit": "Gcell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one operator evaluation (FP64, single thread) on a {problem.nx}x{rows} periodic strip "
                      f"of the {problem.nx}x{problem.ny} state, {t:.1f} s"}


def batched_speedup(seed=3, nsteps=20):
    """512 Euler instances (256 1D, N log-uniform in [256, 65536]; 256 2D squares, side log-uniform in
    [64, 1024]) advanced nsteps SSP-RK3 steps: one persistent graph-captured launch sequence (mode 0,
    autotuned tiles) vs one launch per instance per kernel (mode 1); states must be bitwise equal."""
    import torch
    from paper_1808_00037_amd import teno as T
    from paper_1808_00037_amd import workloads as W

    probs = W.batch(seed, nsteps=nsteps)
    b = T.Batch(probs)
    buf0 = b.pack([torch.from_numpy(p.U0) for p in probs])
    cells = sum(p.ncells for p in probs)
    # mode 0 first call tunes the launch shape and captures the graph
    warm = buf0.clone()
    b.run(warm, nsteps, mode=0)
    b.run(warm.copy_(buf0), nsteps, mode=1)
    torch.cuda.synchronize()
    b.poll()
    # each mode timed three times from the same initial state, alternating; the medians are reported
    times = {0: [], 1: []}
    outs = {}
    for rep in range(3):
        for mode in (0, 1):
            U = buf0.clone()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.run(U, nsteps, mode=mode)
            e1.record()
            torch.cuda.synchronize()
            times[mode].append(e0.elapsed_time(e1))
            outs.setdefault(mode, U)
    b.poll()
    equal = bool(torch.equal(outs[0], outs[1]))
    b.close()
    res = {m: sorted(t)[1] for m, t in times.items()}
    return {"instances": len(probs), "cells": cells, "steps": nsteps, "ms_batched": res[0], "ms_per_instance": res[1],
            "speedup": res[1] / res[0], "bitwise_equal": equal, "repeats": 3,
            "batched_Gcell_updates_per_s": cells * 3 * nsteps / (res[0] / 1e3) / 1e9}


def adjoint_cost(n=1024, nsteps=400, ckpt=20, seed=21):
    """Frozen-selection adjoint of 2D Euler n x n, nsteps steps, checkpoints every ckpt steps:
    backward (segment recomputation + reverse sweep) time over the plain forward run time."""
    import torch
    from paper_1808_00037_amd import teno as T
    from paper_1808_00037_amd import workloads as W

    pr = W.euler2d(seed, n=n)
    sv = T.Solver.for_problem(pr)
    U0 = torch.from_numpy(pr.U0).cuda()
    target = torch.from_numpy(W.density_target(seed, n)).cuda()

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    U = U0.clone()
    sv.run(U, 2, graph=True)          # warm-up (graph capture)
    U = U0.clone()
    t_fwd = timed(lambda: sv.run(U, nsteps, graph=True))
    U = U0.clone()
    box = {}
    t_rec = timed(lambda: box.setdefault("rec", sv.run_record(U, nsteps, ckpt)))
    rec = box["rec"]
    area = pr.dx * pr.dy
    J = torch.sqrt(torch.sum((U[0] - target) ** 2) * area)
    lam = torch.zeros_like(U)
    lam[0] = (U[0] - target) * area / J
    t_bwd = timed(lambda: sv.run_vjp(rec, lam))
    sv.poll()
    # central differences of the frozen map in a few seeded directions (the full 32-direction check
    # is a GPU test)
    worst = 0.0
    for k, dn in enumerate(W.random_directions(77, pr.U0, 2)):
        d = torch.from_numpy(dn).cuda()
        h = 1e-6 * U0.abs().max() / d.abs().max()
        Up, Um = U0 + h * d, U0 - h * d
        sv.run_replay(Up, rec)
        sv.run_replay(Um, rec)
        Jp = torch.sqrt(torch.sum((Up[0] - target) ** 2) * area)
        Jm = torch.sqrt(torch.sum((Um[0] - target) ** 2) * area)
        fd = float((Jp - Jm) / (2 * h))
        an = float(torch.sum(lam * d))
        worst = max(worst, abs(fd - an) / abs(an))
    # the unfrozen map in the first direction: each perturbed run measures its own selection; report
    # its central difference and the mask words that differ from the base run's
    d = torch.from_numpy(W.random_directions(77, pr.U0, 1)[0]).cuda()
    h = 1e-6 * U0.abs().max() / d.abs().max()
    Js, flips = [], 0
    for sgn in (1.0, -1.0):
        Uq = U0 + sgn * h * d
        rq = sv.run_record(Uq, nsteps, ckpt)
        Js.append(torch.sqrt(torch.sum((Uq[0] - target) ** 2) * area))
        flips += int((rq["masks"] != rec["masks"]).sum())
        del rq
    sv.poll()
    an = float(torch.sum(lam * d))
    fd_unfrozen = float((Js[0] - Js[1]) / (2 * h))
    return {"n": n, "steps": nsteps, "ckpt_every": ckpt, "ms_forward": t_fwd, "ms_record": t_rec,
            "ms_backward": t_bwd, "bwd_over_fwd": t_bwd / t_fwd, "fwd_plus_bwd_over_fwd": (t_fwd + t_bwd) / t_fwd,
            "fd_rel_err_2dirs": worst, "unfrozen_fd_rel_err": abs(fd_unfrozen - an) / abs(an),
            "unfrozen_mask_flips": flips, "mask_words_per_run": int(rec["masks"].numel())}


def scheme_cost(n=4096, steps=10, seed=1):
    """The paper's efficiency claim, quantified: SSP-RK3 step time of TENO7X and of its TENO5 base
    (Table 1, eps = 1e-40) on the same 2D Euler state, same kernels apart from the selection."""
    import torch
    from paper_1808_00037_amd import teno as T
    from paper_1808_00037_amd import workloads as W

    pr = W.euler2d(seed, n=n)
    res = {}
    for name, scheme in (("teno7x", T.TENO7X), ("teno5", T.TENO5)):
        sv = T.Solver.for_problem(pr, scheme=scheme)
        U = torch.from_numpy(pr.U0).cuda()
        sv.run(U, 2, graph=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sv.run(U, steps, graph=True)
        e1.record()
        torch.cuda.synchronize()
        sv.poll()
        res[f"ms_per_step_{name}"] = e0.elapsed_time(e1) / steps
        del sv, U
        torch.cuda.empty_cache()
    res["teno7x_over_teno5"] = res["ms_per_step_teno7x"] / res["ms_per_step_teno5"]
    res["n"] = n
    res["steps"] = steps
    return res


def fp32_run(n=4096, steps=10, n_err=256, steps_err=20, seed=1):
    """Single precision: SSP-RK3 throughput on the same 4096^2 state, and the error of a 256^2 run of
    steps_err steps against the FP64 oracle's trajectory (L1 and max norms, relative to the
    oracle's state)."""
    import numpy as np
    import torch
    from oracle import oracle as O
    from paper_1808_00037_amd import teno as T
    from paper_1808_00037_amd import workloads as W

    pr = W.euler2d(seed, n=n)
    sv = T.Solver.for_problem(pr, dtype=torch.float32)
    U = torch.from_numpy(pr.U0.astype(np.float32)).cuda()
    sv.run(U, 2, graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    sv.run(U, steps, graph=True)
    e1.record()
    torch.cuda.synchronize()
    sv.poll()
    ms = e0.elapsed_time(e1) / steps
    del sv, U
    pe = W.euler2d(seed, n=n_err)
    cfg = O.Config(O.EULER2D, n_err, n_err, 0.0, 1.0, 0.0, 1.0)
    Uo = O.run(cfg, pe.U0, steps_err, cfl=pe.cfl)
    sv = T.Solver.for_problem(pe, dtype=torch.float32)
    Ug = torch.from_numpy(pe.U0.astype(np.float32)).cuda()
    sv.run(Ug, steps_err, graph=False)
    sv.poll()
    d = Ug.double().cpu().numpy() - Uo
    return {"n": n, "ms_per_step": ms, "Gcell_updates_per_s": n * n * 3 / (ms / 1e3) / 1e9,
            "error_run": f"{n_err}x{n_err}, {steps_err} steps vs the FP64 oracle",
            "rel_L1": float(np.abs(d).sum() / np.abs(Uo).sum()), "rel_Linf": float(np.abs(d).max() / np.abs(Uo).max())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and adjoint side runs")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after the timed region, one plain device-to-device copy of this many bytes "
                         "(a reference kernel for calibrating profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_1808_00037_amd import teno as T
    from paper_1808_00037_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n = args.n
    log(f"building the 2D Euler {n}x{n} state")
    pr = W.euler2d(args.seed, n=n, nsteps=args.steps)
    U = torch.from_numpy(pr.U0).cuda()
    sv = T.Solver.for_problem(pr)
    cells = n * n

    log("warmup")
    sv.run(U, args.warmup, graph=True)
    torch.cuda.synchronize()
    sv.poll()

    log(f"timed region: {args.steps} steps")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sv.run(U, args.steps, graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    sv.poll()
    ms_per_step = ms / args.steps
    value = cells * 3 * args.steps / (ms / 1e3) / 1e9
    log(f"{ms_per_step:.3f} ms/step, {value:.2f} Gcell-updates/s (wall {wall:.2f} s)")

    # per-kernel durations: the same K steps again, launched one kernel at a time with HIP events
    # recorded around every sweep launch on the stream the kernels run on
    sv.set_timing(True)
    torch.cuda.synchronize()
    e0.record(stream)
    sv.run(U, args.steps, graph=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1)
    kt = sv.read_timing()
    sv.set_timing(False)
    sv.poll()
    x_ms = kt["x"][0] / max(kt["x"][1], 1)
    y_ms = kt["y"][0] / max(kt["y"][1], 1)
    log(f"x-sweep+stage {x_ms:.3f} ms, y-sweep {y_ms:.3f} ms per launch ({kt['x'][1]} + {kt['y'][1]} launches), "
        f"eager step {ms_eager / args.steps:.3f} ms")
    flops_x = FLOPS_XSTAGE * cells
    achieved = flops_x / (x_ms / 1e3)
    log("measured peaks (copy, FP64 FMA)")
    peaks = measured_peaks()
    roofline = {"bound": "alu", "kernel": "sweep_kernel<double,EULER2D,x,stage>", "achieved": achieved / 1e12,
                "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU,
                "traffic": measured_traffic(), "avg_launch_ms": x_ms,
                "flops_per_cell": FLOPS_XSTAGE, "measured_peak": peaks["fp64_fma_TFLOPs"],
                "frac_of_measured": achieved / 1e12 / peaks["fp64_fma_TFLOPs"]}
    hbm_frac = value * 1e9 * BYTES_PER_CELL_UPDATE / PEAK_HBM

    out = {"metric": METRIC, "value": value, "unit": "Gcell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"euler2d_{n}x{n}_fp64_ssprk3", "nx": n, "ny": n, "cfl": pr.cfl,
                      "seed": args.seed, "bc": "periodic", "scheme": "TENO7X", "eps": "dx^3", "C_T": 1e-5},
           "roofline": roofline,
           "hbm": {"algorithmic_bytes_per_cell_update": BYTES_PER_CELL_UPDATE,
                   "achieved_GBps": value * BYTES_PER_CELL_UPDATE, "peak_GBps": PEAK_HBM / 1e9, "frac": hbm_frac,
                   "copy_GBps": peaks["copy_GBps"],
                   "frac_of_copy": value * BYTES_PER_CELL_UPDATE / peaks["copy_GBps"],
                   # the x-stage kernel's HBM bytes per launch measured by rocprofv3 (FETCH_SIZE +
                   # WRITE_SIZE, calibrated) over its live launch time
                   "x_stage_measured_GBps": (roofline["traffic"] / (x_ms / 1e3) / 1e9
                                             if roofline["traffic"] else None)},
           "kernels_ms": {"x_sweep_stage": x_ms, "y_sweep": y_ms, "launches_x": kt["x"][1],
                          "launches_y": kt["y"][1], "eager_ms_per_step": ms_eager / args.steps}}

    if args.copy_bytes > 0:
        # an elementwise kernel that reads copy_bytes and writes copy_bytes
        src = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    del sv, U
    torch.cuda.empty_cache()
    if not args.no_extras:
        log("batched vs one launch per instance (512 instances)")
        out["batched"] = batched_speedup()
        log(json.dumps(out["batched"]))
        torch.cuda.empty_cache()
        log("FP32 throughput and error against the FP64 oracle")
        out["fp32"] = fp32_run(n=n)
        log(json.dumps(out["fp32"]))
        torch.cuda.empty_cache()
        log("TENO7X vs TENO5 step cost")
        out["scheme_cost"] = scheme_cost(n=n)
        log(json.dumps(out["scheme_cost"]))
        torch.cuda.empty_cache()
        log("adjoint cost (1024^2, 400 steps, checkpoints every 20)")
        out["adjoint"] = adjoint_cost()
        log(json.dumps(out["adjoint"]))
        torch.cuda.empty_cache()
    if not args.no_cpu:
        log("oracle CPU baseline")
        out["cpu_baseline"] = cpu_baseline(pr)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
