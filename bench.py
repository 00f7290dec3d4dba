"""Benchmark: block-BP solves of a 16x16 open PEPS (D=4, 4x4 blocks, chi=32)
on one MI355X (the default workload; --workload picks the 4x4 open D=2 case,
the infinite 2x2-cell D=4 case or the 16x16 D=6 chi=64 case instead).

One step is one complete solve on device-resident buffers: tensor setup and
rotation (bbp_set_tensors), the synchronous sweeps needed to bring the
message residual below 1e-10 (the count is found in the warm-up), every
<sigma_z> (256) and bond <S.S> (480), and the log-norm.  The reported value
is directed-message updates per second over the whole step; per-phase times,
the counted fit TFLOP/s, per-step latency percentiles, the dominant kernel's
roofline figures (HIP events on its launch stream) and the FP64 CPU oracle
timed on the host are added to the same JSON line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--no-cpu-baseline] [--no-mixed]
    python bench.py --workload obc4x4_D2_b2_chi4 | inf2x2_D4_b4_chi32 | obc16x16_D6_b4_chi64
    python bench.py --calibrate-copy   (plain 1 GiB device copy, for counters)
    python bench.py --serve [--requests 256] [--slots 8] [--rates 0.5 1 2 4]
    python bench.py --ite ite_ti_obc10x10_D2_b5 | ite_afh_obc14x14_D3_b7  (blockBP update)

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

from bbp_inputs import (CONFIGS, op_heis, op_sx, op_sz, op_szsz,  # noqa: E402
                        peps_finite, peps_infinite)

WORKLOAD = "obc16x16_D4_b4_chi32"
WORKLOADS = (WORKLOAD, "obc4x4_D2_b2_chi4", "inf2x2_D4_b4_chi32", "obc16x16_D6_b4_chi64")
TOL = 1e-10
MAX_SWEEPS = 40
SEARCH_MAX_SWEEPS = 80   # the sweep-count search (the D=6 lattice needs about 50)
PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (vector and matrix)
PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 matrix
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 matrix
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
RIDGE = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fit_visit_obc16x16_D4_chi32.json")
COPY_BYTES = 1 << 30


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sync():
    import torch
    torch.cuda.synchronize()


def lattice_terms(cfg):
    """Sites and nearest-neighbour bonds whose terms a solve evaluates: every
    site and bond of a finite lattice; the unit cell's sites and its
    right/down bonds on the infinite lattice."""
    if cfg["infinite"]:
        cells = [(x, y) for y in range(cfg["ucy"]) for x in range(cfg["ucx"])]
        bonds = [(x, y, x + 1, y) for (x, y) in cells] + [(x, y, x, y + 1) for (x, y) in cells]
        return np.array(cells, dtype=np.int32), bonds
    Lx, Ly = cfg["Lx"], cfg["Ly"]
    sites = np.array([(x, y) for y in range(Ly) for x in range(Lx)], dtype=np.int32)
    bonds = [(x, y, x + 1, y) for y in range(Ly) for x in range(Lx - 1)]
    bonds += [(x, y, x, y + 1) for y in range(Ly - 1) for x in range(Lx)]
    return sites, bonds


def observables(ctx, cfg, sites, bonds):
    """Finite lattice: <sigma_z> and <S.S>; infinite lattice: the transverse-Ising
    terms <sigma_z>, <sigma_x>, <sigma_z sigma_z>.  Returns (site terms, bond terms)."""
    if cfg["infinite"]:
        sz, zz = ctx.expect_terms(sites[:, 0], sites[:, 1], op_sz(), bonds, op_szsz())
        sx = ctx.expect_sites(sites[:, 0], sites[:, 1], op_sx())
        return np.concatenate([np.asarray(sz), np.asarray(sx)]), zz
    return ctx.expect_terms(sites[:, 0], sites[:, 1], op_sz(), bonds, op_heis())


def solve(ctx, cfg, A, sweeps, sites, bonds, times=None, phase_ms=None):
    """One solve; with ``phase_ms`` (a dict, timing on) the event-timed
    kernel milliseconds of its sweeps and of its observables are added to
    ``phase_ms["sweeps"]`` and ``phase_ms["observables"]`` per class."""
    t0 = time.perf_counter()
    ctx.set_tensors(A)
    sync()
    t1 = time.perf_counter()
    if sweeps <= 20:
        res = ctx.sweep(sweeps)
    else:   # long solves report their progress (a run silent for minutes looks hung)
        done = 0
        while done < sweeps:
            k = min(20, sweeps - done)
            res = ctx.sweep(k)
            done += k
            log(f"    {done}/{sweeps} sweeps")
    sync()
    t2 = time.perf_counter()
    if phase_ms is not None:
        mid = {k["name"]: k["ms"] for k in ctx.kernel_stats()}
    sz, ss = observables(ctx, cfg, sites, bonds)
    ln = ctx.log_norm()
    sync()
    t3 = time.perf_counter()
    if phase_ms is not None:
        end = {k["name"]: k["ms"] for k in ctx.kernel_stats()}
        for name, ms in mid.items():
            sw = phase_ms.setdefault("sweeps", {})
            ob = phase_ms.setdefault("observables", {})
            sw[name] = sw.get(name, 0.0) + ms - phase_ms.get("_last", {}).get(name, 0.0)
            ob[name] = ob.get(name, 0.0) + end[name] - ms
        phase_ms["_last"] = end
    if times is not None:
        times.append((t1 - t0, t2 - t1, t3 - t2))
    return res, sz, ss, ln


def class_rates(s):
    """One kernel class's launches and time with its counted rate against
    both rooflines: TFLOP/s against the FP64 peak and the algorithmic bytes
    (operands read and results written once, on the true extents) in GB/s
    against HBM; the small-panel classes (QR, end sites) are latency- and
    HBM-bound, so the GB/s figure is theirs to read."""
    ms = max(s["ms"], 1e-9)
    tf = s["flops"] / ms / 1e9
    gbs = s["bytes"] / ms / 1e6
    return dict(launches=s["launches"], ms=s["ms"], tflops=tf, frac_fp64=tf / PEAK_FP64_TFLOPS,
                gbs=gbs, frac_hbm=gbs / PEAK_HBM_GBS)


def roofline(stats, workload=WORKLOAD):
    """Roofline of the fit visit (the contraction class with the most time:
    the fused visit, or the unfused T1/ket/bra/local chain where the fused
    tiles do not fit): achieved rate of its launches from the FLOPs and
    algorithmic bytes counted on every item's true bond dimensions; the same
    launches counted at the padded bond cap are reported beside them.  The
    kernel class with the most time overall is named too."""
    by = {s["name"]: s for s in stats}
    dom_all = max(stats, key=lambda s: s["ms"])
    fused = by["fit_visit"]
    chain = [by[k] for k in ("fit_T1", "fit_ket", "fit_bra", "fit_local")]
    if sum(c["ms"] for c in chain) > fused["ms"]:
        dom = dict(name="fit_T1+fit_ket+fit_bra+fit_local",
                   launches=max(c["launches"] for c in chain),
                   **{k: sum(c[k] for c in chain)
                      for k in ("ms", "flops", "bytes", "padded_flops", "padded_bytes")})
    else:
        dom = fused
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
    pf = dom["padded_flops"] / n
    r.update(traffic=measured_traffic(dom["name"]) if workload == WORKLOAD else None,
             kernel=dom["name"], launches=dom["launches"],
             avg_us=dom["ms"] / n * 1e3, flops_per_launch=flops,
             algorithmic_bytes_per_launch=bytes_, intensity=intensity,
             counted_on="true bond dimensions of every item (split-layer schedule)",
             padded=dict(flops_per_launch=pf, kernel_bytes_per_launch=dom["padded_bytes"] / n,
                         achieved_tflops=pf / avg_s / 1e12,
                         frac=pf / avg_s / 1e12 / PEAK_FP64_TFLOPS),
             most_time_class=dom_all["name"])
    return r


def host_cpu():
    """The host's CPU model and the BLAS the oracle's NumPy calls."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        for p in threadpool_info():
            if p.get("user_api") == "blas":
                blas = f"{p.get('internal_api')} {p.get('version')}"
                break
    except Exception:
        pass
    return dict(cpu_model=model, logical_cpus=os.cpu_count(), blas=blas)


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


def serve_stream(n, seed):
    """The request stream of the serving workload: lattice side uniform in
    {6, 8, ..., 20}, D uniform in {2, 3, 4}, chi = 2 D^2, block side uniform in
    {2, 3, 4} (lattices padded with trivial sites), seeded tensors."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        side = int(rng.choice(np.arange(6, 21, 2)))
        D = int(rng.choice([2, 3, 4]))
        b = int(rng.choice([2, 3, 4]))
        reqs.append(dict(Lx=side, Ly=side, bx=b, by=b, D=D, chi=2 * D * D,
                         tensor_seed=int(rng.integers(1 << 31))))
    return reqs


def serve(args):
    """Serving pattern: every request on a plain context of its own, one at a
    time; every request through the request server one at a time; then the
    same stream through the server (continuous batching) with Poisson
    arrivals at several multiples of the one-at-a-time service rate, and all
    of it submitted at once."""
    import threading
    import torch
    from paper_2301_05844_amd import bbp
    reqs = serve_stream(args.requests, args.seed)
    tens = [peps_finite(r["Lx"], r["Ly"], r["D"], seed=r["tensor_seed"]) for r in reqs]
    spec = [{k: v for k, v in r.items() if k != "tensor_seed"} for r in reqs]
    free, total = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    kw = dict(tol=TOL, max_sweeps=MAX_SWEEPS)

    def run(rate, slots):
        srv = bbp.Server(budget_bytes=budget, max_slots=slots)
        gaps = np.random.default_rng(args.seed + 1).exponential(1.0 / rate, len(reqs)) \
            if rate and rate != float("inf") else np.zeros(len(reqs))
        tickets = []
        t0 = time.perf_counter()

        def feed():
            nxt = t0
            for g, r, A in zip(gaps, spec, tens):
                nxt += g
                dt = nxt - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                tickets.append(srv.submit(A, **r, **kw))
        if slots == 1 and not rate:   # the plain path: one at a time
            res = []
            for i, (r, A) in enumerate(zip(spec, tens)):
                t = srv.submit(A, **r, **kw)
                res.append(srv.wait(t, timeout=600))
                tickets.append(t)
                if (i + 1) % 16 == 0:
                    log(f"  {i + 1} requests done ({time.perf_counter() - t0:.1f} s)")
        else:
            th = threading.Thread(target=feed)
            th.start()
            th.join()
            res = [srv.wait(t, timeout=600) for t in tickets]
        wall = time.perf_counter() - t0
        st = srv.stats()
        errs = [srv.error(t) for t in tickets]
        srv.close()
        bad = [e for (s, _, _), e in zip(res, errs) if s != "done"]
        if bad:
            raise RuntimeError(f"{len(bad)} requests failed: {bad[0]}")
        lat = np.array([tm[2] - tm[0] for _, _, tm in res])
        return res, dict(wall_s=wall, solves_per_s=len(res) / wall,
                         p50_ms=float(np.percentile(lat, 50) * 1e3),
                         p99_ms=float(np.percentile(lat, 99) * 1e3),
                         max_running=st["max_running"], shared_sweeps=st["shared_sweeps"],
                         request_sweeps=st["request_sweeps"],
                         max_together=st["max_together"],
                         busy_s=dict(sweeps=st["sweep_s"], admit=st["admit_s"],
                                     outputs=st["outputs_s"]))

    # the plain per-context path: each request its own context, one at a time
    log(f"serving: {len(reqs)} requests on plain contexts, one at a time")
    t0 = time.perf_counter()
    lat_plain = []
    for i, (r, A) in enumerate(zip(spec, tens)):
        ts = time.perf_counter()
        g = bbp.BlockBP(Lx=r["Lx"], Ly=r["Ly"], bx=r["bx"], by=r["by"], D=r["D"], chi=r["chi"],
                        chi_env=max(r["chi"], min(128, 2 * r["D"] ** 2 + 10)))
        g.set_tensors(A)
        res_ = 1.0
        n = 0
        while res_ >= TOL and n < MAX_SWEEPS:
            res_ = g.sweep(1)
            n += 1
        sites, bonds = lattice_terms(dict(infinite=False, Lx=r["Lx"], Ly=r["Ly"]))
        g.expect_terms(sites[:, 0], sites[:, 1], op_sz(), bonds, op_heis())
        g.log_norm()
        g.close()
        lat_plain.append(time.perf_counter() - ts)
        if (i + 1) % 32 == 0:
            log(f"  {i + 1} plain solves done ({time.perf_counter() - t0:.1f} s)")
    wall_plain = time.perf_counter() - t0
    plain_ctx = dict(wall_s=wall_plain, solves_per_s=len(reqs) / wall_plain,
                     p50_ms=float(np.percentile(lat_plain, 50) * 1e3),
                     p99_ms=float(np.percentile(lat_plain, 99) * 1e3))
    log(f"serving: {len(reqs)} requests one at a time")
    plain_res, plain = run(0.0, 1)
    service = np.array([tm[2] - tm[1] for _, _, tm in plain_res])
    mu = len(reqs) / service.sum()
    log(f"one-at-a-time service rate {mu:.2f} solves/s")
    lines = []
    for mult in args.rates:
        log(f"serving at {mult} x the one-at-a-time rate")
        res, m = run(mult * mu, args.slots)
        same = all(a[1]["residual"] == b[1]["residual"] and
                   np.array_equal(a[1]["sz"], b[1]["sz"]) and
                   np.array_equal(a[1]["ss"], b[1]["ss"]) for a, b in zip(plain_res, res))
        m.update(rate_multiple=mult, arrival_rate=mult * mu, equal_to_alone=bool(same))
        lines.append(m)
    updates = sum(r[1]["sweeps"] for r in plain_res)
    log("serving: the whole stream submitted at once")
    res_all, burst = run(float("inf"), args.slots)
    out = dict(metric="p50/p99 solve latency and solves/s under Poisson arrivals",
               workload="serving stream (side 6..20, D 2..4, chi 2D^2, block 2..4)",
               requests=len(reqs), slots=args.slots, budget_bytes=budget,
               plain_contexts=plain_ctx,
               one_at_a_time=dict(plain, service_rate=mu, total_sweeps=updates),
               served=lines, all_at_once=burst, data="synthetic", dtype="f64")
    print(json.dumps(out), flush=True)


def mixed_precision(ctx, cfg, A, sites, bonds, ref, sweeps, steps, fp64_ms):
    """The precision pattern on the same workload, two protocols: FP32 sweeps
    until the residual stops falling (or drops below the tolerance), then
    FP64 sweeps to the tolerance; and BF16, then FP32, then FP64 the same
    way.  Observables are computed in FP64.  Reports each stage's error
    against a tightly converged FP64 solve, each protocol's time per solve
    against the all-FP64 one, and each precision's sweep time and fit rate."""
    err = lambda a, b: float(np.max(np.abs(np.array(a) - np.array(b))))

    def observables():
        ctx.set_option("precision", 64)
        sz, ss = ctx.expect_terms(sites[:, 0], sites[:, 1], op_sz(), bonds, op_heis())
        return np.array(sz), np.array(ss)

    # tightly converged FP64 reference: how close each stage is to the fixed point
    ctx.set_option("precision", 64)
    ctx.set_tensors(A)
    rt, nt = 1.0, 0
    while rt >= 1e-14 and nt < SEARCH_MAX_SWEEPS:
        rt = ctx.sweep(1)
        nt += 1
        if nt % 10 == 0:
            log(f"  reference sweep {nt}: residual {rt:.2e}")
    szt, sst = observables()

    def chunked(n):
        r, done = None, 0
        while done < n:
            k = min(20, n - done)
            r = ctx.sweep(k)
            done += k
            if n > 20:
                log(f"    {done}/{n} sweeps")
        return r

    def protocol(stages):
        # search: the sweep count of each stage, and its error at the end
        ctx.set_option("precision", stages[0])
        ctx.set_tensors(A)
        counts, stage_err, res = [], {}, 1.0
        for p in stages:
            ctx.set_option("precision", p)
            n, prev = 0, None
            while n < SEARCH_MAX_SWEEPS:
                res = ctx.sweep(1)
                n += 1
                if res < TOL or (p != 64 and prev is not None and res >= prev):
                    break   # converged, or at this precision's floor
                prev = res
                if n % 10 == 0:
                    log(f"  precision {p} sweep {n}: residual {res:.2e}")
            counts.append(n)
            sz, ss = observables()
            stage_err[f"fp{p}" if p != 16 else "bf16"] = dict(
                sweeps=n, residual=res, err_sz=err(sz, szt), err_ss=err(ss, sst))
        name = ">".join("bf16" if p == 16 else f"fp{p}" for p in stages)
        log(f"{name}: sweeps {counts}, residual {res:.2e}")
        times = []
        for _ in range(steps):
            sync()
            t0 = time.perf_counter()
            ctx.set_option("precision", stages[0])
            ctx.set_tensors(A)
            for p, n in zip(stages, counts):
                ctx.set_option("precision", p)
                res = chunked(n)
            sz, ss = ctx.expect_terms(sites[:, 0], sites[:, 1], op_sz(), bonds, op_heis())
            ln = ctx.log_norm()
            sync()
            times.append(time.perf_counter() - t0)
        ms = float(np.mean(times) * 1e3)
        return dict(stages=stage_err, residual=res, ms_per_solve=ms,
                    speedup_vs_fp64=fp64_ms / ms,
                    max_abs_diff_sz_vs_fp64=err(sz, ref[1]),
                    max_abs_diff_ss_vs_fp64=err(ss, ref[2]),
                    abs_err_log_norm=float(abs(ln[0] - ref[3][0])),
                    err_sz_vs_converged=err(sz, szt), err_ss_vs_converged=err(ss, sst))

    protocols = {"fp32>fp64": protocol((32, 64)), "bf16>fp32>fp64": protocol((16, 32, 64))}
    # the plain per-message FP64 form: every directed message updated as a
    # batch of its own, one after another on one stream (message_split 0,
    # lanes 1), the same sweeps and observables; its results are the
    # batched FP64 solve's bits
    pm = None
    if fp64_ms < 1000.0:
        from paper_2301_05844_amd import bbp
        g = bbp.BlockBP(Lx=cfg["Lx"], Ly=cfg["Ly"], bx=cfg["bx"], by=cfg["by"], D=cfg["D"],
                        chi=cfg["chi"], message_split=0, lanes=1)
        n64 = sweeps
        g.set_tensors(A)
        g.sweep(n64)   # warm-up: the per-message graphs are captured here
        sync()
        t0 = time.perf_counter()
        g.set_tensors(A)
        res_pm = g.sweep(n64)
        sz_pm, ss_pm = g.expect_terms(sites[:, 0], sites[:, 1], op_sz(), bonds, op_heis())
        g.log_norm()
        sync()
        ms_pm = (time.perf_counter() - t0) * 1e3
        g.close()
        log(f"per-message FP64: {ms_pm:.0f} ms per solve")
        pm = dict(ms_per_solve=ms_pm, sweeps=n64, residual=res_pm,
                  equals_batched_fp64=bool(np.array_equal(sz_pm, ref[1]) and
                                           np.array_equal(ss_pm, ref[2])),
                  batched_fp64_speedup=ms_pm / fp64_ms)
        for pr in protocols.values():
            pr["speedup_vs_per_message_fp64"] = ms_pm / pr["ms_per_solve"]
    per = {}
    names = {16: "bf16", 32: "fp32", 64: "fp64"}
    peaks = {16: PEAK_BF16_TFLOPS, 32: PEAK_FP32_TFLOPS, 64: PEAK_FP64_TFLOPS}
    for prec in (16, 32, 64):   # time per sweep in each precision, same state
        ctx.set_option("precision", prec)
        sync()
        t0 = time.perf_counter()
        ctx.sweep(2)
        sync()
        ms = (time.perf_counter() - t0) / 2 * 1e3
        _, fl = ctx.stats()   # fit FLOPs of the last sweep, true bonds
        tf = fl / (ms * 1e-3) / 1e12
        per[names[prec]] = dict(ms_per_sweep=ms, fit_tflops=tf, frac_of_peak=tf / peaks[prec])
    ctx.set_option("precision", 64)
    return dict(protocols=protocols, per_precision=per, per_message_fp64=pm,
                peaks_tflops=dict(fp64=PEAK_FP64_TFLOPS, fp32=PEAK_FP32_TFLOPS,
                                  bf16=PEAK_BF16_TFLOPS),
                reference=f"FP64, {nt} sweeps to residual {rt:.1e}",
                fp64_err_sz=err(ref[1], szt), fp64_err_ss=err(ref[2], sst),
                note="each stage until the residual stops falling, the last (FP64) to the "
                     "tolerance; BF16 and FP32 stages run the fused visit and environment "
                     "contractions on BF16 / FP32 MFMA with FP32 accumulation (the BF16 "
                     "stage in the generic fused visit); QR, normalisation and messages "
                     "FP64; observables FP64; errors against the all-FP64 solve and "
                     "against a tightly converged FP64 reference")


def cpu_baseline(cfg, A):
    """The FP64 oracle on the host: one untimed sweep, then timed sweeps of
    the same solve (bonds at their caps) until about two seconds have passed
    (one sweep on the 16x16 lattice).  Workloads with D >= 6 (a sweep is
    tens of minutes there) time the first message updates of the first
    sweep instead, about 20 s of them: inside each column fit the bonds
    already reach their caps."""
    from oracle.blockbp import BlockBP
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    geo = dict(infinite=True, ucx=cfg["ucx"], ucy=cfg["ucy"]) if cfg["infinite"] \
        else dict(Lx=cfg["Lx"], Ly=cfg["Ly"])
    bp = BlockBP(A, D=cfg["D"], chi=cfg["chi"], bx=cfg["bx"], by=cfg["by"], **geo)
    if cfg["D"] >= 6:
        t0 = time.perf_counter()
        n = 0
        for e, key in enumerate(bp.order):
            bp.update_message(e, key, bp.msgs)
            n += 1
            log(f"  oracle message update {n}: {time.perf_counter() - t0:.1f} s")
            if time.perf_counter() - t0 >= 20.0:
                break
        dt = time.perf_counter() - t0
        return dict(value=n / dt, unit="message updates/s", cores=threads, kind="oracle",
                    sample=f"first {n} message updates of the first sweep, {dt:.1f} s",
                    **host_cpu())
    bp.sweep()
    nsw = 0
    t0 = time.perf_counter()
    while True:
        bp.sweep()
        nsw += 1
        dt = time.perf_counter() - t0
        if dt >= 2.0 or nsw >= 50:
            break
    n = len(bp.order) * nsw
    what = "second sweep" if nsw == 1 else f"sweeps 2..{nsw + 1}"
    out = dict(value=n / dt, unit="message updates/s", cores=threads,
               kind="oracle",
               sample=f"{what} of the same solve ({n} message updates, "
                      f"bonds at chi), {dt:.1f} s", **host_cpu())
    try:  # the same updates on one thread: the first messages of the next sweep
        from threadpoolctl import threadpool_limits
        n1 = min(12, len(bp.order))
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            for e, key in enumerate(bp.order[:n1]):
                bp.update_message(e, key, bp.msgs)
            d1 = time.perf_counter() - t0
        out["one_thread"] = dict(value=n1 / d1, unit="message updates/s", cores=1,
                                 sample=f"first {n1} message updates of sweep {nsw + 2}, "
                                        f"{d1:.1f} s")
    except ImportError:
        pass
    return out


ITE_WORKLOADS = {
    # transverse-field Ising (B = 3) on a 10x10 open lattice in 5x5 blocks, D = 2
    "ite_ti_obc10x10_D2_b5": dict(model="ti", B=3.0, Lx=10, Ly=10, bx=5, by=5, D=2, chi=4,
                                  chi_env=18, dtau=0.05),
    # antiferromagnetic Heisenberg on a 14x14 open lattice in 7x7 blocks, D = 3
    "ite_afh_obc14x14_D3_b7": dict(model="afh", Lx=14, Ly=14, bx=7, by=7, D=3, chi=9,
                                   chi_env=28, dtau=0.05),
}
ITE_TOL, ITE_MAX_SWEEPS = 1e-6, 10


def ite_hamiltonian(w):
    """Bond Hamiltonian h (d^2 x d^2) of an ITE workload: transverse-field
    Ising -sz sz - B/4 (sx 1 + 1 sx) with Pauli-type op_sz/op_sx, or the
    Heisenberg S.S."""
    if w["model"] == "afh":
        return op_heis()
    sz, sx = op_sz(), op_sx()
    return -np.kron(sz, sz) - w["B"] / 4 * (np.kron(sx, np.eye(2)) + np.kron(np.eye(2), sx))


def ite_bench(args):
    """ITE steps of the blockBP update (App. B): each step sweeps block BP
    from the previous step's messages until the residual is below 1e-6 (at
    most 10 sweeps), then applies the Trotter gates exp(-h dtau) to every
    bond (bbp_ite_step, 4 ALS passes).  Reports ITE steps/s over K timed
    steps after W warm-up steps, the phase split, the energy per bond after
    the run, the fit-visit roofline of a second, event-timed step, and the
    oracle's per-step time on a bounded sample of the same step."""
    from scipy.linalg import expm
    from paper_2301_05844_amd import bbp
    w = ITE_WORKLOADS[args.ite]
    h = ite_hamiltonian(w)
    G = expm(-w["dtau"] * h)
    A0 = peps_finite(w["Lx"], w["Ly"], w["D"], seed=args.seed)
    ctx = bbp.BlockBP(Lx=w["Lx"], Ly=w["Ly"], bx=w["bx"], by=w["by"], D=w["D"],
                      chi=w["chi"], chi_env=w["chi_env"])
    ctx.set_tensors(A0)
    _, bonds = lattice_terms(dict(infinite=False, Lx=w["Lx"], Ly=w["Ly"]))

    def step(times=None, sweeps_log=None):
        t0 = time.perf_counter()
        n, res = 0, 1.0
        while n < ITE_MAX_SWEEPS and res >= ITE_TOL:
            res = ctx.sweep(1)
            n += 1
        sync()
        t1 = time.perf_counter()
        gates, loss = ctx.ite_step(G, n_als=4)
        sync()
        t2 = time.perf_counter()
        if times is not None:
            times.append((t1 - t0, t2 - t1, n, res, gates, loss, ctx.ite_info))
        return gates

    e0 = float(np.mean(ctx.expect_bonds(bonds, h)))
    log(f"ITE {args.ite}: energy per bond {e0:.8f} at the start")
    for k in range(args.warmup):
        step()
        log(f"warm-up ITE step {k} done")
    times = []
    sync()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(times)
        t = times[-1]
        log(f"ITE step {k}: {t[2]} sweeps ({t[0] * 1e3:.1f} ms, residual {t[3]:.1e}), "
            f"{t[4]} gates ({t[1] * 1e3:.1f} ms)")
    sync()
    total = time.perf_counter() - t0
    ctx.sweep(ITE_MAX_SWEEPS)
    e1 = float(np.mean(ctx.expect_bonds(bonds, h)))
    log(f"energy per bond {e1:.8f} after {args.warmup + args.steps} steps")
    # one more step with every launch bracketed by HIP events (process-wide)
    stats = None
    if not args.no_kernel_pass:
        ctx.set_option("timing", 1)
        step()
        stats = ctx.kernel_stats()
        ctx.set_option("timing", 0)
    gates = times[0][4]
    line = dict(
        metric="ITE steps/s (blockBP update: BP sweeps to 1e-6 plus one Trotter step of "
               "gates on every bond)",
        value=args.steps / total,
        unit="ITE steps/s",
        n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=total / args.steps * 1e3,
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=args.ite, model=w["model"], lattice=f"{w['Lx']}x{w['Ly']} open",
                    block=f"{w['bx']}x{w['by']}", D=w["D"], chi=w["chi"],
                    chi_env=w["chi_env"], dtau=w["dtau"], n_als=4, gates_per_step=gates,
                    sweep_tol=ITE_TOL, max_sweeps=ITE_MAX_SWEEPS),
        gates_per_s=gates * args.steps / total,
        phase_ms=dict(sweeps=float(np.mean([t[0] for t in times]) * 1e3),
                      update=float(np.mean([t[1] for t in times]) * 1e3),
                      update_environments=float(np.mean([t[6]["env_s"] for t in times]) * 1e3),
                      update_host_fits=float(np.mean([t[6]["host_s"] for t in times]) * 1e3)),
        gate_levels=times[0][6]["levels"],
        sweeps_per_step=[t[2] for t in times],
        fit_error_per_step=[t[5] for t in times],
        energy_per_bond=dict(start=e0, end=e1),
        roofline=None if stats is None else dict(
            roofline(stats, None), measured_in="one further ITE step with every launch "
            "bracketed by HIP events (sweeps and the environment contractions)"),
        kernels=None if stats is None else {
            s["name"]: class_rates(s) for s in stats},
        cpu_baseline=None if args.no_cpu_baseline else ite_cpu_baseline(w, A0, G, gates),
    )
    print(json.dumps(line), flush=True)


SVD_BATCH, SVD_M, SVD_N = 48, 512, 32


def svd_bench(args):
    """bbp_svd_jacobi on one batch of 48 message-panel shaped matrices (512 x
    32, the (chi D^2) x chi panels of the 16x16 D=4 chi=32 workload's message
    batch), all 32 singular triplets kept: K timed calls after W warm-up
    calls, HIP events on the stream the kernel runs on, the FP64 vector-ALU
    roofline on the rotations' arithmetic, and the oracle (LAPACK SVD) on
    the same matrices on the host."""
    import torch
    from paper_2301_05844_amd import bbp
    from bbp_inputs import dense_matrices
    A = dense_matrices(SVD_BATCH, SVD_M, SVD_N, seed=args.seed)
    t = torch.from_numpy(A).cuda()
    for _ in range(args.warmup):
        bbp.svd_jacobi(t)
    sync()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(args.steps):
        U, S, V, e2, sw = bbp.svd_jacobi(t)
    e1.record(st)
    sync()
    total = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1) / args.steps
    sweeps = sw.cpu().numpy()
    if np.any(sweeps <= 0):
        raise SystemExit("bbp_svd_jacobi: an item did not converge")
    # every pair of every sweep: three length-m dot products (6 m flops); the
    # rotation of two columns of A and of V (6 m + 6 n) for every pair of
    # every sweep but the last, which rotates nothing (an upper bound: pairs
    # already orthogonal are skipped); the final column norms (2 m n)
    m, n = SVD_M, SVD_N
    P = n * (n - 1) / 2
    flops = float(np.sum(sweeps) * P * 6 * m + np.sum(sweeps - 1) * P * (6 * m + 6 * n)
                  + SVD_BATCH * 2 * m * n)
    achieved = flops / (ev_ms * 1e-3) / 1e12
    S_gpu = S.cpu().numpy()
    from oracle.svd import truncated_svd
    c0 = time.perf_counter()
    err = 0.0
    for b in range(SVD_BATCH):
        _, So, _, _ = truncated_svd(A[b])
        err = max(err, float(np.abs(S_gpu[b] - So).max() / So[0]))
    cpu_s = time.perf_counter() - c0
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    line = dict(
        metric="matrices/s (batched truncated SVD by one-sided Jacobi, FP64)",
        value=SVD_BATCH * args.steps / total, unit="matrices/s",
        n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=total / args.steps * 1e3,
        higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=f"svd_{SVD_BATCH}x{m}x{n}", batch=SVD_BATCH, m=m, n=n, k=n),
        sweeps=dict(mean=float(np.mean(sweeps)), max=int(np.max(sweeps))),
        max_rel_err_singular_values_vs_oracle=err,
        roofline=dict(bound="alu", achieved=achieved, peak=78.6, unit="TFLOP/s",
                      frac=achieved / 78.6, traffic=None, kernel="k_svd_jacobi",
                      avg_us=ev_ms * 1e3, flops_per_launch=flops,
                      counted_on="pair sums of every sweep each item took, rotations of "
                                 "every pair of every sweep but the last (an upper bound)"),
        cpu_baseline=dict(value=SVD_BATCH / cpu_s, unit="matrices/s", cores=threads,
                          kind="oracle", sample=f"the same {SVD_BATCH} matrices, LAPACK "
                          "SVD (numpy.linalg.svd) one by one", **host_cpu()),
    )
    print(json.dumps(line), flush=True)


def ite_cpu_baseline(w, A, G, gates):
    """The oracle's blockBP update on the host, on a bounded sample: block BP
    converged to 1e-6 (at most 10 sweeps) from the start, then gates of the
    first Trotter step in order until about 20 s have passed; the per-step
    time is sweeps + gates x the mean gate time."""
    from oracle import blockbp as ob
    from oracle import ite
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    Lx, Ly, D = w["Lx"], w["Ly"], w["D"]
    bp = ob.BlockBP(A, D=D, chi=w["chi"], bx=w["bx"], by=w["by"], Lx=Lx, Ly=Ly,
                    chi_env=w["chi_env"])
    t0 = time.perf_counter()
    n = 0
    while n < ITE_MAX_SWEEPS:
        n += 1
        if bp.sweep() < ITE_TOL:
            break
        log(f"  oracle sweep {n}: {time.perf_counter() - t0:.1f} s")
    t_sweeps = time.perf_counter() - t0
    A = np.array(A, dtype=np.float64)
    t0 = time.perf_counter()
    done = 0
    for (a, b) in ite.bond_order(Lx, Ly):
        horizontal = a[1] == b[1]
        ia, ib = a[1] * Lx + a[0], b[1] * Lx + b[0]
        da, db = ite.leg_dims(a[0], a[1], Lx, Ly, D), ite.leg_dims(b[0], b[1], Lx, Ly, D)
        Xa, Ra, Lb, Yb, oa, ob_, sa, sb = ite.split_pair(A[ia], A[ib], horizontal, da, db)
        k, kb = Xa.shape[1], Yb.shape[0]
        N = ite.bond_environment(bp, A, a, b, Xa, Yb, oa, ob_, sa, sb, k, kb, da, db)
        R, L = ite.fit_pair(N, np.einsum("asr,rtb->astb", Ra, Lb), G, D, 4)
        A[ia], A[ib] = ite.rebuild(Xa, R, L, Yb, oa, ob_, sa, sb, A.shape[1], D, da, db)
        done += 1
        if time.perf_counter() - t0 >= 20.0:
            break
    t_gate = (time.perf_counter() - t0) / done
    per_step = t_sweeps + gates * t_gate
    log(f"  oracle: {n} sweeps {t_sweeps:.1f} s, {done} gates at {t_gate:.2f} s each")
    return dict(value=1.0 / per_step, unit="ITE steps/s", cores=threads, kind="oracle",
                sample=f"{n} block-BP sweeps ({t_sweeps:.1f} s) and the first {done} of "
                       f"{gates} gates of a step ({t_gate:.2f} s per gate); per step = "
                       "sweeps + gates x mean gate time", **host_cpu())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-pass", action="store_true",
                    help="skip the second, event-timed pass (no roofline figures)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision pattern (profiling runs: the timed "
                         "solves are then the last kernels of the run)")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--serve", action="store_true",
                    help="serving pattern instead of the default solve")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--rates", type=float, nargs="+", default=[0.5, 1.0, 2.0, 4.0])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", choices=WORKLOADS, default=WORKLOAD,
                    help="workload of the solve (default: the 16x16 open lattice)")
    ap.add_argument("--ite", choices=sorted(ITE_WORKLOADS), default=None,
                    help="ITE steps of the blockBP update on this workload instead of the "
                         "default solve")
    ap.add_argument("--svd", action="store_true",
                    help="the batched truncated SVD (bbp_svd_jacobi) on 48 512x32 panels")
    ap.add_argument("--lanes", type=int, default=None,
                    help="streams the message and boundary-stack batches spread over "
                         "(library default when absent)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: every message update of this "
              "workload runs on a single MI355X; --gpus must be 1",
              file=sys.stderr)
        sys.exit(2)
    if args.serve:
        serve(args)
        return
    if args.ite:
        ite_bench(args)
        return
    if args.svd:
        svd_bench(args)
        return

    from paper_2301_05844_amd import bbp
    cfg = CONFIGS[args.workload]
    opts = {} if args.lanes is None else dict(lanes=args.lanes)
    if cfg["infinite"]:
        A = peps_infinite(cfg["ucx"], cfg["ucy"], cfg["D"], seed=0)
        geo = dict(infinite=True, ucx=cfg["ucx"], ucy=cfg["ucy"])
        lattice = f"infinite, {cfg['ucx']}x{cfg['ucy']} unit cell"
        outputs = "unit cell's sigma_z and sigma_x, sigma_z sigma_z on its bonds, log-norm"
    else:
        A = peps_finite(cfg["Lx"], cfg["Ly"], cfg["D"], seed=0)
        geo = dict(Lx=cfg["Lx"], Ly=cfg["Ly"])
        lattice = f"{cfg['Lx']}x{cfg['Ly']} open"
        outputs = None
    sites, bonds = lattice_terms(cfg)
    if outputs is None:
        outputs = f"{len(sites)} sigma_z, {len(bonds)} S.S, log-norm"
    ctx = bbp.BlockBP(bx=cfg["bx"], by=cfg["by"], D=cfg["D"], chi=cfg["chi"], **geo, **opts)

    ctx.set_tensors(A)
    if "sweeps" in cfg:   # a fixed sweep count
        sweeps = cfg["sweeps"]
        res = ctx.sweep(sweeps)
        log(f"{sweeps} sweeps (fixed) reach residual {res:.2e}")
    else:                 # warm-up: find the sweep count that reaches the tolerance
        log("warm-up: sweeping to the tolerance")
        sweeps, res = 0, 1.0
        while res >= TOL and sweeps < SEARCH_MAX_SWEEPS:
            res = ctx.sweep(1)
            sweeps += 1
            log(f"  sweep {sweeps}: residual {res:.2e}")
        log(f"{sweeps} sweeps reach residual {res:.2e}")
    n_msgs, flops_sweep = ctx.stats()
    for _ in range(args.warmup):
        solve(ctx, cfg, A, sweeps, sites, bonds)
        log("warm-up solve done")

    # timed region: K solves, no instrumentation (per-launch timing events
    # would add a marker before and after every kernel)
    times = []
    sync()
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = solve(ctx, cfg, A, sweeps, sites, bonds, times)
        log(f"step {k}: {sum(times[-1]) * 1e3:.1f} ms")
    sync()
    total = time.perf_counter() - t0
    # the same K solves again with every launch bracketed by HIP events on its
    # stream: per-kernel-class durations for the roofline.  A context on one
    # stream runs them, so that no two kernels overlap (the bracket of a kernel
    # that shares the GPU with another lane's would include the other's time)
    stats, timed_total = None, None
    phase_kernels = {}
    if not args.no_kernel_pass:
        log("event-timed pass")
        # the first context's buffers are released first: at D=6 one
        # context's observables hold over 100 GB of the 288
        ctx.close()
        ctx = None
        ctx1 = bbp.BlockBP(bx=cfg["bx"], by=cfg["by"], D=cfg["D"], chi=cfg["chi"], **geo,
                           lanes=1)
        ctx1.set_option("timing", 1)
        sync()
        ti0 = time.perf_counter()
        for k in range(args.steps):
            solve(ctx1, cfg, A, sweeps, sites, bonds, phase_ms=phase_kernels)
        sync()
        timed_total = time.perf_counter() - ti0
        stats = ctx1.kernel_stats()
        ctx1.set_option("timing", 0)   # the timing switch is process-wide
        ctx1.close()

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
        config=dict(workload=args.workload, lattice=lattice, D=cfg["D"],
                    chi=cfg["chi"], block=f"{cfg['bx']}x{cfg['by']}",
                    chi_env=cfg.get("chi_env", 2 * cfg["D"] ** 2 + 10),
                    n_fit=2, sweeps_per_solve=sweeps, messages_per_sweep=n_msgs,
                    residual=out[0],
                    outputs=outputs),
        fit_tflops=flops_sweep * sweeps / sweep_s.mean() / 1e12,
        fit_tflops_frac=flops_sweep * sweeps / sweep_s.mean() / 1e12
        / PEAK_FP64_TFLOPS,
        phase_ms=dict(set_tensors=float(np.mean([t[0] for t in times]) * 1e3),
                      sweeps=float(sweep_s.mean() * 1e3),
                      observables=float(np.mean([t[2] for t in times]) * 1e3)),
        solve_latency_ms=dict(p50=float(np.percentile(step_s, 50) * 1e3),
                              p99=float(np.percentile(step_s, 99) * 1e3)),
        roofline=None if stats is None else dict(
            roofline(stats, args.workload), measured_in="second pass of the same K "
            "solves on a one-stream context (lanes 1), every launch bracketed by HIP events",
            pass_ms_per_step=timed_total / args.steps * 1e3),
        kernels=None if stats is None else {
            s["name"]: class_rates(s) for s in stats},
        kernel_ms_per_solve_by_phase=None if stats is None else {
            ph: {n: v / args.steps for n, v in d.items() if v > 0}
            for ph, d in phase_kernels.items() if not ph.startswith("_")},
        cpu_baseline=None,
    )
    # the precision pattern (BF16 / FP32 contractions in the fused visits)
    if not args.no_mixed and "tol" in cfg and not cfg["infinite"]:
        if ctx is None:
            ctx = bbp.BlockBP(bx=cfg["bx"], by=cfg["by"], D=cfg["D"], chi=cfg["chi"], **geo,
                              **opts)
        line["mixed_precision"] = mixed_precision(ctx, cfg, A, sites, bonds, out, sweeps,
                                                  args.steps, line["ms_per_step"])
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(cfg, A)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
