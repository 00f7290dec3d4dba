"""Benchmark: block-BP solves of a 16x16 open PEPS (D=4, 4x4 blocks, chi=32)
on one MI355X.

One step is one complete solve on device-resident buffers: tensor setup and
rotation (bbp_set_tensors), the synchronous sweeps needed to bring the
message residual below 1e-10 (the count is found in the warm-up), every
<sigma_z> (256) and bond <S.S> (480), and the log-norm.  The reported value
is directed-message updates per second over the whole step; per-phase times,
the counted fit TFLOP/s, per-step latency percentiles, the dominant kernel's
roofline figures (HIP events on its launch stream) and the FP64 CPU oracle
timed on the host are added to the same JSON line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--no-cpu-baseline]
    python bench.py --calibrate-copy   (plain 1 GiB device copy, for counters)

The roofline's `traffic` (HBM bytes per launch of the dominant kernel) comes
from the rocprofv3 FETCH_SIZE / WRITE_SIZE summary under profiles/ and is
reported only while the HIP sources match the ones the counters were taken
on; otherwise it is null.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from bbp_inputs import CONFIGS, op_heis, op_sz, peps_finite  # noqa: E402

WORKLOAD = "obc16x16_D4_b4_chi32"
TOL = 1e-10
MAX_SWEEPS = 40
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (vector and matrix)
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
RIDGE = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fit_visit_obc16x16_D4_chi32.json")
COPY_BYTES = 1 << 30


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sync():
    import torch
    torch.cuda.synchronize()


def solve(ctx, A, sweeps, sites, bonds, times=None):
    t0 = time.perf_counter()
    ctx.set_tensors(A)
    sync()
    t1 = time.perf_counter()
    res = ctx.sweep(sweeps)
    sync()
    t2 = time.perf_counter()
    sz = ctx.expect_sites(sites[:, 0], sites[:, 1], op_sz())
    ss = ctx.expect_bonds(bonds, op_heis())
    ln = ctx.log_norm()
    sync()
    t3 = time.perf_counter()
    if times is not None:
        times.append((t1 - t0, t2 - t1, t3 - t2))
    return res, sz, ss, ln


def roofline(stats):
    """Dominant kernel class by summed time; achieved rate of its launches."""
    dom = max(stats, key=lambda s: s["ms"])
    n = max(dom["launches"], 1)
    avg_s = dom["ms"] / n * 1e-3
    flops, bytes_ = dom["flops"] / n, dom["bytes"] / n
    intensity = flops / bytes_ if bytes_ else float("inf")
    if intensity < RIDGE:
        achieved = bytes_ / avg_s / 1e9
        r = dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s",
                 frac=achieved / PEAK_HBM_GBS)
    else:
        achieved = flops / avg_s / 1e12
        r = dict(bound="mfma", achieved=achieved, peak=PEAK_FP64_TFLOPS,
                 unit="TFLOP/s", frac=achieved / PEAK_FP64_TFLOPS)
    r.update(traffic=measured_traffic(dom["name"]), kernel=dom["name"], launches=dom["launches"],
             avg_us=dom["ms"] / n * 1e3, flops_per_launch=flops,
             bytes_per_launch=bytes_, intensity=intensity)
    return r


def measured_traffic(cls):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernels (same source hash) for this kernel class."""
    from paper_2301_05844_amd.profiling import source_sha
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != source_sha() or t.get("kernel_class") != cls:
        return None
    return t["bytes_per_launch"]


def calibrate_copy():
    """A plain device copy of COPY_BYTES (read and written once), five times:
    the reference for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes=COPY_BYTES, kernel="neg (elementwise)")), flush=True)


def cpu_baseline(cfg, A):
    """The FP64 oracle on the host: one untimed sweep, then one timed sweep
    with every bond at its cap (48 directed-message updates)."""
    from oracle.blockbp import BlockBP
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    bp = BlockBP(A, D=cfg["D"], chi=cfg["chi"], bx=cfg["bx"], by=cfg["by"],
                 Lx=cfg["Lx"], Ly=cfg["Ly"])
    bp.sweep()
    t0 = time.perf_counter()
    bp.sweep()
    dt = time.perf_counter() - t0
    n = len(bp.order)
    return dict(value=n / dt, unit="message updates/s", cores=threads,
                kind="oracle",
                sample=f"second sweep of the same solve ({n} message updates, "
                       f"bonds at chi), {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: every message update of this "
              "workload runs on a single MI355X; --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)

    from paper_2301_05844_amd import bbp
    cfg = CONFIGS[WORKLOAD]
    A = peps_finite(cfg["Lx"], cfg["Ly"], cfg["D"], seed=0)
    sites = np.array([(x, y) for y in range(cfg["Ly"]) for x in range(cfg["Lx"])],
                     dtype=np.int32)
    bonds = [(x, y, x + 1, y) for y in range(cfg["Ly"]) for x in range(cfg["Lx"] - 1)]
    bonds += [(x, y, x, y + 1) for y in range(cfg["Ly"] - 1) for x in range(cfg["Lx"])]
    ctx = bbp.BlockBP(Lx=cfg["Lx"], Ly=cfg["Ly"], bx=cfg["bx"], by=cfg["by"],
                      D=cfg["D"], chi=cfg["chi"])

    # warm-up: find the sweep count that reaches the tolerance
    log("warm-up: sweeping to the tolerance")
    ctx.set_tensors(A)
    sweeps, res = 0, 1.0
    while res >= TOL and sweeps < MAX_SWEEPS:
        res = ctx.sweep(1)
        sweeps += 1
    n_msgs, flops_sweep = ctx.stats()
    log(f"{sweeps} sweeps reach residual {res:.2e}")
    for _ in range(args.warmup):
        solve(ctx, A, sweeps, sites, bonds)
        log("warm-up solve done")

    ctx.set_option("timing", 1)
    times = []
    sync()
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = solve(ctx, A, sweeps, sites, bonds, times)
        log(f"step {k}: {sum(times[-1]) * 1e3:.1f} ms")
    sync()
    total = time.perf_counter() - t0
    stats = ctx.kernel_stats()
    ctx.set_option("timing", 0)

    step_s = np.array([sum(t) for t in times])
    sweep_s = np.array([t[1] for t in times])
    updates = sweeps * n_msgs * args.steps
    line = dict(
        metric="BP message updates/s + achieved TFLOP/s vs MFMA peak; "
               "p50/p99 solve latency",
        value=updates / total,
        unit="message updates/s",
        n_gpus=1,
        steps=args.steps,
        warmup=args.warmup,
        ms_per_step=total / args.steps * 1e3,
        higher_is_better=True,
        scaling="weak",
        vs_baseline=None,
        dtype="f64",
        data="synthetic",
        config=dict(workload=WORKLOAD, lattice="16x16 open", D=cfg["D"],
                    chi=cfg["chi"], block="4x4", chi_env=2 * cfg["D"] ** 2 + 10,
                    n_fit=2, sweeps_per_solve=sweeps, messages_per_sweep=n_msgs,
                    residual=out[0],
                    outputs="256 sigma_z, 480 S.S, log-norm"),
        fit_tflops=flops_sweep * sweeps / sweep_s.mean() / 1e12,
        fit_tflops_frac=flops_sweep * sweeps / sweep_s.mean() / 1e12
        / PEAK_FP64_TFLOPS,
        phase_ms=dict(set_tensors=float(np.mean([t[0] for t in times]) * 1e3),
                      sweeps=float(sweep_s.mean() * 1e3),
                      observables=float(np.mean([t[2] for t in times]) * 1e3)),
        solve_latency_ms=dict(p50=float(np.percentile(step_s, 50) * 1e3),
                              p99=float(np.percentile(step_s, 99) * 1e3)),
        roofline=roofline(stats),
        kernels={s["name"]: dict(launches=s["launches"], ms=s["ms"])
                 for s in stats},
        cpu_baseline=None,
    )
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(cfg, A)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
