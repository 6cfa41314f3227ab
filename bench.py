#!/usr/bin/env python3
"""Benchmark of the Sakurai-Sugiura shifted-CG eigensolver on one MI355X.

One step is one pass of the whole hot path over one set of synthetic inputs that
are already resident in HBM: quadrature on the two lines, the shifted CG for all
N nodes and L sources (one seed system per source), the moment sums and the
Rayleigh-Ritz extraction with acceptance (sscg_ss_eigs). The throughput is
shift-updates per second: the number of (source, shift) vector updates the
shifted CG performs, summed over the timed steps, divided by their wall time.

Printed as one JSON line on rank 0. Besides the throughput it carries:
  roofline      the dominant kernel (by measured time), its algorithmic bytes per
                launch over its average launch duration from HIP events recorded
                around every launch inside the timed region, against 8 TB/s;
                traffic from committed rocprofv3 counter summaries when they match
                the current kernel source, else null
  dslash        the same figures for the Wilson dslash
  dslash_24x48  the dslash alone on the 24^3 x 48 lattice with 8 sources (FP32 with
                12-real links, FP64 with 18-real links), autotuned launch shape
  tts           time to solution of the step in FP64 and FP64-seed / FP32-shift
                precision, with stored solutions and with in-loop moments
  tts_window    the same comparison on a window of the field's spectrum that holds
                eigenvalues, with both modes' eigenvalues and residuals
  cpu_baseline  the FP64 CPU oracle (numpy/scipy) on the host: one source's full
                shifted CG (all N shifts) on the same workload, bounded in time
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

METRIC = "shift-updates/sec & dslash HBM GB/s (frac of peak), mixed/batched vs FP64 plain"
HBM_PEAK_GBS = 8000.0
DEFAULT_CONFIG = "wilson8_fp64"
STAGES = ["dslash", "seed_alpha", "seed_r_update", "unused", "shift_update", "reliable_update",
          "solve_loop"]
KERNEL_SOURCES = {"shift_update": "paper_1004_0292_amd/csrc/vec.hip",
                  "dslash": "paper_1004_0292_amd/csrc/dslash.hip",
                  "dslash_fp32_links12": "paper_1004_0292_amd/csrc/dslash.hip",
                  "dslash_fp64_links18": "paper_1004_0292_amd/csrc/dslash.hip"}


def source_hash(rel):
    return hashlib.sha256((ROOT / rel).read_bytes()).hexdigest()[:16]


def pmc_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, if it still matches."""
    f = ROOT / "profiles" / f"{kernel}_{workload}_pmc.txt"
    if not f.exists():
        return None
    d = json.loads(f.read_text())
    if d.get("source_sha256_16") != source_hash(KERNEL_SOURCES[kernel]):
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_model():
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, budget_s=20.0):
    """Oracle shifted CG (all N shifts) on the workload's sources, one after another,
    stopped after budget_s seconds of wall time."""
    import numpy as np
    from oracle import quadrature as quad
    from oracle import solvers, wilson
    import synth

    t_setup = time.perf_counter()
    U = w.gauge()
    A = wilson.hermitian_wilson(U, w.dims, w.kappa)
    V = w.sources().reshape(w.L, -1)
    z, zeta = quad.line_nodes(w.N, w.gamma, w.rho, w.beta)
    setup = time.perf_counter() - t_setup
    updates = [0]
    t0 = time.perf_counter()
    c0 = time.process_time()

    class Stop(Exception):
        pass

    def rec(k, st):
        updates[0] += st["updated"]
        if time.perf_counter() - t0 > budget_s:
            raise Stop()

    done = 0
    try:
        for l in range(w.L):
            solvers.shifted_cg(lambda x: A @ x, V[l], z, w.gamma, w.tol, record=rec)
            done += 1
    except Stop:
        pass
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    return {"value": updates[0] / wall, "unit": "shift-updates/s", "cores": max(1, round(cpu / wall)),
            "kind": "oracle",
            "sample": (f"FP64 shifted CG for all {w.N} shifts on the explicit sparse A (scipy CSR), sources "
                       f"solved one after another: {done} of {w.L} to convergence"
                       f"{'' if done == w.L else ', the next stopped at the time limit'}; "
                       f"{updates[0]} shift-updates in {wall:.1f} s; cores = process CPU time / wall time; "
                       f"matrix assembly ({setup:.1f} s) excluded"),
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}


def tts_compare(S, ctx, params, vd, max_eigs, steps):
    """Time to solution of the whole step in FP64 and in the FP64-seed / FP32-shift mode,
    each with stored solutions and with the moments summed inside the solve, on the
    same inputs (graph replay, no per-launch events)."""
    import copy
    import torch
    out = {}
    ctx.set_profiling(False)
    for name, prec, in_loop in (("fp64", S.FP64, 0), ("mixed_shifts", S.MIXED_SHIFTS, 0),
                                ("fp64_inloop", S.FP64, 1), ("mixed_shifts_inloop", S.MIXED_SHIFTS, 1)):
        p = copy.copy(params)
        p.solve = copy.copy(params.solve)
        p.solve.prec = prec
        p.moments_in_loop = in_loop
        ctx.ss_eigs(p, vd, max_eigs=max_eigs)          # tune for this mode
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = ctx.ss_eigs(p, vd, max_eigs=max_eigs)
        torch.cuda.synchronize()
        out[name + "_ms_per_step"] = round((time.perf_counter() - t0) / steps * 1e3, 3)
        out[name + "_eigs"] = r.lam.round(12).tolist()
        out[name + "_max_res"] = float(r.res.max()) if len(r.res) else None
    out["speedup_mixed_vs_fp64"] = round(out["fp64_ms_per_step"] / out["mixed_shifts_ms_per_step"], 3)
    out["speedup_mixed_inloop_vs_fp64"] = round(out["fp64_ms_per_step"] / out["mixed_shifts_inloop_ms_per_step"], 3)
    return out


# Eigenvalue windows that do contain eigenvalues of a workload's field (from its
# reference spectrum), for the time-to-solution comparison at equal accuracy.
WINDOWS = {"wilson8_fp64": dict(lo=0.3700, hi=0.3735, beta=0.5, N=32, M=8)}


def tts_window(S, ctx, w, vd, steps):
    """Time to solution and accuracy of FP64 against the FP32-shift mode on a window
    with eigenvalues: per-step time, the eigenvalues and residuals of each mode, and
    the largest relative eigenvalue difference between the two."""
    import numpy as np
    import torch
    win = WINDOWS.get(w.name)
    if win is None:
        return None
    gamma, rho = 0.5 * (win["lo"] + win["hi"]), 0.5 * (win["hi"] - win["lo"])
    out = {"window": [win["lo"], win["hi"]], "beta": win["beta"], "N": win["N"], "M": win["M"]}
    ctx.set_profiling(False)
    lams = {}
    for name, prec in (("fp64", S.FP64), ("mixed_shifts", S.MIXED_SHIFTS)):
        opts = S.default_opts(tol=w.tol, prec=prec, ru_interval=w.ru_interval, switch_tol=w.switch_tol)
        p = S.default_ss_params(gamma=gamma, rho=rho, beta=win["beta"], N=win["N"], M=win["M"], rank_tol=1e-7,
                                spur_tol=1e-6, solve=opts)
        ctx.ss_eigs(p, vd, max_eigs=32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = ctx.ss_eigs(p, vd, max_eigs=32)
        torch.cuda.synchronize()
        out[name + "_ms_per_step"] = round((time.perf_counter() - t0) / steps * 1e3, 3)
        out[name + "_eigs"] = r.lam.round(13).tolist()
        out[name + "_max_res"] = float(r.res.max()) if len(r.res) else None
        lams[name] = r.lam
    a, b = lams["fp64"], lams["mixed_shifts"]
    out["eigs_found"] = [len(a), len(b)]
    out["max_rel_eig_diff"] = float(np.max(np.abs(a - b) / np.abs(a))) if len(a) == len(b) and len(a) else None
    out["speedup_mixed_vs_fp64"] = round(out["fp64_ms_per_step"] / out["mixed_shifts_ms_per_step"], 3)
    return out


def bench_batch(args):
    """The batched workload: three lattices (8^4, 12^4, 16^4) with their own intervals,
    N and 4 sources solved together (one grouped launch per stage, graphs between polls)
    versus the same three problems solved one after another in plain FP64."""
    import numpy as np
    import torch
    import paper_1004_0292_amd as S
    import synth
    ws = [synth.CONFIGS[nm] for nm in synth.BATCH]
    ctxs, vs, zs, ys = [], [], [], []
    for w in ws:
        c = S.Context(w.dims, w.kappa)
        c.set_gauge(w.gauge())
        ctxs.append(c)
        vs.append(torch.from_numpy(w.sources()).to("cuda:0"))
        z, _, _ = S.quad_lines(w.N, w.gamma, w.rho, w.beta)
        zs.append(z)
        ys.append(torch.zeros((w.L, w.N, w.n), dtype=torch.complex128, device="cuda:0"))
    mixed = S.default_opts(prec=S.MIXED_SHIFTS, ru_interval=50, switch_tol=1e-6)
    fp64 = S.default_opts(prec=S.FP64)

    def batched():
        return S.batch_solve(ctxs, vs, zs, [w.gamma for w in ws], ys, mixed, true_res=False)

    def sequential():
        return [c.shifted_cg_solve(v, z, w.gamma, y, fp64, true_res=False) for c, v, z, w, y in zip(ctxs, vs, zs, ws, ys)]

    res = {}
    for name, fn in (("batched_mixed", batched), ("sequential_fp64", sequential)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rr = fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        su = sum(int(np.where(r.conv_iter >= 0, r.conv_iter, r.iters[:, None]).sum()) for r in rr)
        res[name] = {"ms_per_step": round(dt * 1e3, 3), "shift_updates": su, "value": round(su / dt, 1),
                     "status": [int(r.status) for r in rr]}
    line = {
        "metric": METRIC, "value": res["batched_mixed"]["value"], "unit": "shift-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["batched_mixed"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batch_8_12_16", "problems": [
            {"lattice": list(w.dims), "kappa": w.kappa, "interval": [w.gamma - w.rho, w.gamma + w.rho], "N": w.N,
             "L": w.L} for w in ws], "prec": "mixed_shifts", "parallelism": "single GPU, one grouped launch per stage"},
        "tts": {"batched_mixed_ms": res["batched_mixed"]["ms_per_step"],
                "sequential_fp64_ms": res["sequential_fp64"]["ms_per_step"],
                "speedup": round(res["sequential_fp64"]["ms_per_step"] / res["batched_mixed"]["ms_per_step"], 3)},
        "detail": res,
    }
    print(json.dumps(line), flush=True)


def dslash_large(S, reps=10):
    """The Wilson dslash alone on the large single-GPU lattice (24^3 x 48, 8 sources):
    FP32 spinors with 12-real links and FP64 spinors with 18-real links, in the launch
    shape the library's autotuner picks, timed with HIP events around every launch,
    against its compulsory HBM bytes (spinors in and out once, links once)."""
    import torch
    import synth
    w = synth.CONFIGS["wilson24x48_mixed12"]
    U = w.gauge()
    x = torch.from_numpy(w.sources()).to("cuda:0")
    y = torch.empty_like(x)
    out = {"lattice": list(w.dims), "sources": w.L}
    for name, prec, lr, wb in (("fp32_links12", S.MIXED, 12, 4), ("fp64_links18", S.FP64, 18, 8)):
        c = S.Context(w.dims, w.kappa)
        c.set_gauge(U, lr)
        c.apply_A(x, y, prec)            # chooses the launch shape
        c.set_profiling(True)
        for _ in range(reps):
            c.apply_A(x, y, prec)
        ms, calls = c.stage_times()
        avg_s = ms[0] / 1e3 / calls[0]
        nbytes = w.L * w.V * 24 * wb * 2 + w.V * 4 * lr * wb
        ach = nbytes / avg_s / 1e9
        out[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": pmc_traffic("dslash_" + name, w.name), "avg_launch_us": round(avg_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": nbytes, "launches": int(calls[0])}
        c.close()
    del x, y
    torch.cuda.empty_cache()
    return out


def copy_bandwidth(nbytes=2 << 30, reps=5):
    """Device-to-device copy rate (read + write bytes per second) as the achievable
    HBM reference next to the 8 TB/s peak."""
    import torch
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return round(gbs, 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default=DEFAULT_CONFIG)
    ap.add_argument("--method", default="rr", choices=["rr", "hankel"])
    ap.add_argument("--prec", default=None, choices=["fp64", "mixed", "mixed_shifts"],
                    help="override the workload's precision mode")
    ap.add_argument("--moments-in-loop", action="store_true",
                    help="accumulate the moments inside the solve (no stored solutions)")
    ap.add_argument("--weighted-tol", action="store_true", help="moment-weighted per-shift stopping")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dslash-large", action="store_true",
                    help="skip the dslash-only measurement on the 24^3 x 48 lattice")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 vs mixed time-to-solution comparison")
    ap.add_argument("--no-events", action="store_true", help="time without per-launch events")
    ap.add_argument("--sample-every", type=int, default=None,
                    help="time the dslash and shift update of every k-th iteration (graph replay kept; "
                         "default 25 for FP64 solves, 10 for the mixed modes); 1 times every launch with "
                         "direct launches")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy five times (for counter scaling) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU sharding is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8, "launches": 5}))
        return

    import paper_1004_0292_amd as S
    import synth

    if args.config == "batch":
        bench_batch(args)
        return
    w = synth.CONFIGS[args.config]
    mode = args.prec or w.prec
    prec = {"fp64": S.FP64, "mixed": S.MIXED, "mixed_shifts": S.MIXED_SHIFTS}[mode]
    seed32 = prec == S.MIXED
    U = w.gauge()
    V = w.sources()
    ctx = S.Context(w.dims, w.kappa, device=0)
    ctx.set_gauge(U, w.link_reals)
    vd = torch.from_numpy(V).to("cuda:0")
    del V
    opts = S.default_opts(tol=w.tol, prec=prec, ru_interval=w.ru_interval, switch_tol=w.switch_tol)
    params = S.default_ss_params(gamma=w.gamma, rho=w.rho, beta=w.beta, N=w.N, M=w.M,
                                 method=S.RR if args.method == "rr" else S.HANKEL, rank_tol=1e-7,
                                 spur_tol=1e-6, solve=opts, moments_in_loop=int(args.moments_in_loop),
                                 weighted_tol=int(args.weighted_tol))
    max_eigs = min(w.M * w.L, 32)
    if args.sample_every is None:
        # the sample must hit every poll interval at the same rate: FP64 solves poll
        # every 50 iterations; the FP64 phase of the mixed modes polls every 10
        args.sample_every = 25 if prec == S.FP64 else 10
    ctx.set_profiling(0 if args.no_events else args.sample_every)
    for _ in range(args.warmup):
        ctx.ss_eigs(params, vd, max_eigs=max_eigs)
    torch.cuda.synchronize()
    stage_ms = np.zeros(8)
    stage_calls = np.zeros(8, dtype=np.int64)
    tot = dict(shift_updates=0, shift_updates_fp32=0, seed_iters=0, seed_iters_fp32=0, matvecs=0,
               t_solve=0.0, t_moments=0.0, t_extract=0.0)
    link_launches = [0, 0]   # dslash launches doing work in the FP64 and FP32 phases
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = ctx.ss_eigs(params, vd, max_eigs=max_eigs)
        ms, calls = ctx.stage_times()
        stage_ms += ms
        stage_calls += calls
        for k in tot:
            tot[k] += getattr(out.info, k)
        sw = out.info.switch_iter if out.info.switch_iter >= 0 else out.info.iters
        link_launches[0] += min(out.info.iters, sw)
        link_launches[1] += max(0, out.info.iters - sw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    n = w.n
    value = tot["shift_updates"] / elapsed
    graph_value = None
    if not args.no_events:
        # the same steps again without events (shows what the timing costs)
        ctx.set_profiling(False)
        su = 0
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(args.steps):
            su += ctx.ss_eigs(params, vd, max_eigs=max_eigs).info.shift_updates
        torch.cuda.synchronize()
        graph_value = su / (time.perf_counter() - g0)

    # algorithmic bytes (compulsory traffic) per kernel over the timed steps
    su64 = tot["shift_updates"] - tot["shift_updates_fp32"]
    su32 = tot["shift_updates_fp32"]
    it64 = tot["seed_iters"] - tot["seed_iters_fp32"]
    it32 = tot["seed_iters_fp32"]
    # shift update: read and write x_j and p_j per active (shift, source, entry); seed r
    # read once and seed p read and written once per (source, entry, iteration)
    # (the seed vectors are FP32 in the FP32 phase only in the "mixed" mode)
    shift_bytes = (su64 * 64 + it64 * 48) * n + (su32 * 32 + it32 * (24 if seed32 else 48)) * n
    if args.moments_in_loop:
        # p_j read and written per active (shift, source, entry); per (source, entry,
        # iteration) the seed r read, the seed p read and written, and the M moments read
        # and written
        shift_bytes = (su64 * 32 + su32 * 16 + (it64 + it32) * (48 + 32 * w.M)) * n
    # dslash: spinor in and out per (source, site) and the four forward links per site
    dslash_bytes = (it64 * 48 * 8 + it32 * 48 * (4 if seed32 else 8)) * w.V
    dslash_bytes += (link_launches[0] * 18 * 8 +
                     link_launches[1] * (w.link_reals * 4 if seed32 else 18 * 8)) * 4 * w.V
    rep = {}
    launched = int(stage_calls[6])   # iterations launched (one dslash and one shift update each)
    for name, idx, b in (("shift_update", 4, shift_bytes), ("dslash", 0, dslash_bytes)):
        calls = int(stage_calls[idx])  # launches timed (every k-th when sampling)
        if calls == 0 or stage_ms[idx] <= 0 or launched == 0:
            rep[name] = None
            continue
        avg_s = stage_ms[idx] / 1e3 / calls
        per_launch = b / launched
        ach = per_launch / avg_s / 1e9
        rep[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": pmc_traffic(name, w.name),
                     "kernel": name, "launches": launched, "launches_timed": calls, "avg_launch_us": round(avg_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": round(per_launch)}
    dominant = "shift_update" if stage_ms[4] >= stage_ms[0] else "dslash"
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "shift-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == S.FP64 else "f32+f64",
        "prec_mode": mode,
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": list(w.dims), "kappa": w.kappa, "eps": w.eps, "seed": w.seed,
                   "interval": [w.gamma - w.rho, w.gamma + w.rho], "beta": w.beta, "N": w.N, "L": w.L,
                   "M": w.M, "tol": w.tol, "prec": mode, "link_reals": w.link_reals,
                   "method": args.method, "moments_in_loop": bool(args.moments_in_loop),
                   "weighted_tol": bool(args.weighted_tol), "parallelism": "single GPU"},
        "roofline": rep[dominant],
        "dslash": rep["dslash"],
        "site_shift_updates_per_s": round(value * w.V, 1),
        "seed_iters_per_step": tot["seed_iters"] / args.steps / w.L,
        "eigenpairs_found": int(out.n_found),
        "stage_ms_per_step": {STAGES[i]: round(stage_ms[i] / args.steps, 3) for i in range(7) if i != 3},
        "phase_ms_per_step": {k: round(tot[k] * 1e3 / args.steps, 3) for k in ("t_solve", "t_moments", "t_extract")},
        "timing": ("graph replay, no events" if args.no_events else
                   "direct launches, HIP events around every launch" if args.sample_every == 1 else
                   f"graph replay, HIP event-record nodes around the dslash and shift update of every "
                   f"{args.sample_every}th iteration (offset {args.sample_every // 2} in each poll interval)"),
        "value_without_events": round(graph_value, 1) if graph_value else None,
    }
    if not args.no_compare:
        line["tts"] = tts_compare(S, ctx, params, vd, max_eigs, args.steps)
        tw = tts_window(S, ctx, w, vd, args.steps)
        if tw is not None:
            line["tts_window"] = tw
    line["copy_bw_GBs"] = copy_bandwidth()
    if not args.no_dslash_large:
        line["dslash_24x48"] = dslash_large(S)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
