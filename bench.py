#!/usr/bin/env python3
"""Benchmark of the Sakurai-Sugiura shifted-CG eigensolver on one MI355X.

One step is one pass of the whole hot path over one set of synthetic inputs that
are already resident in HBM: quadrature on the two lines, the shifted CG for all
N nodes and L sources (one seed system per source), the moment sums and the
Rayleigh-Ritz extraction with acceptance (sscg_ss_eigs). The throughput is
shift-updates per second: the number of (source, shift) vector updates the
shifted CG performs, summed over the timed steps, divided by their wall time.

The default workload is the largest single-GPU one, a 24^3 x 48 lattice with 64
nodes, 8 sources and 24 moments, timed in FP64 (the paper's arithmetic) with the
moments summed inside the solve (each shift's step added to the moments as it is
made). Printed as one JSON line; besides the throughput it carries:
  roofline      the dominant kernel (by time per step): algorithmic bytes per launch
                over its average launch duration from HIP events recorded inside the
                solve's graphs, against 8 TB/s; traffic from the committed rocprofv3
                counter summary when it matches the current kernel source, else null
  dslash        the same figures for the Wilson dslash of the solve
  stage_ms_per_step  every stage of the solve, from the sampled launch times scaled
                by the launches of that stage (the split of the paper's Table 2:
                matrix-vector products against everything else)
  tts           time to solution of the same step in its other forms: FP64 with the
                solutions stored, FP32 shift directions with the moments inside or the
                solutions stored (and SSCG_MIXED with --with-mixed-seed), with each
                mode's largest FP64 true residual where solutions are stored
  tts_window    the same on an interval that holds eigenvalues, with the eigenvalues
                of each mode, their agreement with FP64 and with the reference spectrum
  extraction    Rayleigh-Ritz against block Hankel on that window: extraction time,
                device memory, residuals and eigenvalue error
  dslash_24x48  the dslash alone on the 24^3 x 48 lattice with 8 sources (FP32 with
                12-real links, FP64 with 18-real links), autotuned launch shape
  cpu_baseline  the FP64 CPU oracle (numpy/scipy) on the host, on a bounded sample of
                the same workload, and the solve time extrapolated from it
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME] [--prec P]
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
MALL_BYTES = 256 << 20          # Infinity Cache of the MI355X
DEFAULT_CONFIG = "wilson24x48"
STAGES = ["dslash", "seed_alpha", "seed_r_update", "unused", "shift_update", "reliable_update",
          "solve_loop", "block_sweep"]
TIMED_STAGES = (0, 1, 2, 4, 5, 7)
BLOCK_DEFAULT = 24    # block length of the in-loop moment update (SSCG_BLOCK, unless set)
KERNEL_SOURCES = {"shift_update": "paper_1004_0292_amd/csrc/vec.hip",
                  "shift_moments": "paper_1004_0292_amd/csrc/vec.hip",
                  "block_sweep": "paper_1004_0292_amd/csrc/vec.hip",
                  "dslash": "paper_1004_0292_amd/csrc/dslash.hip",
                  "dslash_fp32_links12": "paper_1004_0292_amd/csrc/dslash.hip",
                  "dslash_fp64_links18": "paper_1004_0292_amd/csrc/dslash.hip"}


def source_hash(rel):
    return hashlib.sha256((ROOT / rel).read_bytes()).hexdigest()[:16]


def pmc_traffic(kernel, workload, prec):
    """HBM bytes per launch from the committed counter summary, if it still matches."""
    f = ROOT / "profiles" / f"{kernel}_{workload}_{prec}_pmc.txt"
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


def cpu_baseline(w, gpu_iters, budget_s=20.0, max_shifts=16):
    """The FP64 oracle's shifted CG on the host, on a bounded sample of the workload:
    source 0 with every (N / max_shifts)-th node, iterated until budget_s seconds or 25
    iterations. Reports the oracle's shift-updates per second on that sample, and the
    solve of the whole workload extrapolated from it (oracle matrix-vector product
    time plus per-shift vector time, times the GPU's seed iterations)."""
    import numpy as np
    from oracle import quadrature as quad
    from oracle import solvers, wilson

    t_setup = time.perf_counter()
    U = w.gauge()
    A = wilson.hermitian_wilson(U, w.dims, w.kappa)
    del U
    v = w.sources()[0].reshape(-1)
    z, _ = quad.line_nodes(w.N, w.gamma, w.rho, w.beta)
    stride = max(1, w.N // max_shifts)
    zs = z[::stride]
    setup = time.perf_counter() - t_setup
    # the oracle's matrix-vector product alone
    t0 = time.perf_counter()
    for _ in range(3):
        _ = A @ v
    t_mv = (time.perf_counter() - t0) / 3
    updates = [0]
    iters = [0]
    t0 = time.perf_counter()
    c0 = time.process_time()

    class Stop(Exception):
        pass

    def rec(k, st):
        updates[0] += st["updated"]
        iters[0] += 1
        if time.perf_counter() - t0 > budget_s or iters[0] >= 25:
            raise Stop()

    try:
        solvers.shifted_cg(lambda x: A @ x, v, zs, w.gamma, w.tol, record=rec)
    except Stop:
        pass
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    t_it = wall / max(iters[0], 1)
    per_shift = max(t_it - t_mv, 0.0) / len(zs)
    t_it_full = t_mv + per_shift * w.N
    return {"value": round(updates[0] / wall, 2), "unit": "shift-updates/s", "cores": max(1, round(cpu / wall)),
            "kind": "oracle",
            "sample": (f"FP64 oracle shifted CG (scipy CSR matrix, numpy vectors) on source 0 of {w.L} with "
                       f"{len(zs)} of the {w.N} nodes (every {stride}th), {iters[0]} iterations, "
                       f"{updates[0]} shift-updates in {wall:.1f} s; cores = process CPU time / wall time; "
                       f"matrix assembly ({setup:.1f} s) excluded"),
            "oracle_matvec_s": round(t_mv, 4),
            "oracle_iteration_s_all_nodes": round(t_it_full, 3),
            "extrapolated_solve_s": round(t_it_full * gpu_iters, 1),
            "extrapolation": (f"oracle iteration with all {w.N} nodes (matrix-vector product + {w.N} x the "
                              f"measured per-node vector time) times the {gpu_iters} seed iterations the GPU "
                              f"ran over all sources in one step: extrapolated, not run"),
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model()}


PRECS = {"fp64": 0, "mixed": 1, "mixed_shifts": 2}


def solve_steps(S, ctx, params, vd, max_eigs, steps, warmup=1):
    """Run ss_eigs warmup + steps times; per-step wall time and the last result."""
    import torch
    for _ in range(warmup):
        ctx.ss_eigs(params, vd, max_eigs=max_eigs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = ctx.ss_eigs(params, vd, max_eigs=max_eigs)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, r


def mode_summary(r, ms, nsrc):
    i = r.info
    return {"ms_per_step": round(ms, 2), "status": int(r.status), "seed_iters_per_source": i.seed_iters / nsrc,
            "switch_iter": int(i.switch_iter), "max_true_res": float(i.max_true_res),
            "shift_updates": int(i.shift_updates), "shift_updates_fp32": int(i.shift_updates_fp32),
            "eigenpairs_found": int(r.n_found), "eigs": r.lam.round(13).tolist(),
            "max_res": float(r.res.max()) if len(r.res) else None,
            "t_solve_s": round(i.t_solve, 4), "t_extract_s": round(i.t_extract, 4)}


def tts_compare(S, ctx, params, vd, max_eigs, steps, base_ms, base_res, with_mixed_seed, deadline):
    """Time to solution of the whole step on the same inputs and interval as the timed
    steps, in the other precision modes and moment forms (graph replay, sampled events
    off): FP64 with stored solutions, FP32 shift vectors with moments in the loop and
    with stored solutions, and (when asked for) the FP32-seed mode."""
    import copy
    ctx.set_profiling(0)
    out = {"timed_steps": dict(base_res)}
    modes = [("fp64_stored", S.FP64, 0), ("mixed_shifts", S.MIXED_SHIFTS, params.moments_in_loop),
             ("mixed_shifts_stored", S.MIXED_SHIFTS, 0)]
    if with_mixed_seed:
        modes.append(("mixed_seed32", S.MIXED, 0))
    for name, prec, in_loop in modes:
        if time.perf_counter() > deadline:
            out[name] = "skipped: time budget of the benchmark"
            continue
        p = copy.copy(params)
        p.solve = copy.copy(params.solve)
        p.solve.prec = prec
        p.moments_in_loop = in_loop
        dt, r = solve_steps(S, ctx, p, vd, max_eigs, steps)
        out[name] = mode_summary(r, dt * 1e3, vd.shape[0])
        out[name]["moments_in_loop"] = bool(in_loop)
        out[name]["speedup_vs_timed_steps"] = round(base_ms / (dt * 1e3), 3)
    return out


# Intervals of a workload's field that hold eigenvalues (from its reference
# spectrum), for the time-to-solution comparison at equal accuracy: the interval
# [lo, hi], the line offset beta, N nodes, M moments and L sources.
WINDOWS = {"wilson8_fp64": dict(lo=0.3700, hi=0.3735, beta=0.5, N=32, M=8, L=4),
           "wilson16x32_mixed": dict(lo=0.3650, hi=0.3661, beta=0.5, N=32, M=8, L=4),
           # one eigenvalue (0.3454946 in the oracle's reference spectrum); SSCG_MIXED
           # is left out at this size (its FP32 seed does not converge here)
           "wilson24x48": dict(lo=0.3450, hi=0.3457, beta=0.5, N=32, M=8, L=2,
                               modes=("fp64", "mixed_shifts", "fp64_inloop", "mixed_shifts_inloop",
                                      "fp64_hankel"))}


def reference_spectrum(name):
    """Reference eigenvalues of a workload's field (written by the oracle scripts under
    tests/golden), or None."""
    g = ROOT / "tests" / "golden"
    if name == "wilson8_fp64":
        f = g / "wilson8.json"
        return json.loads(f.read_text())["lowest_eigs"]["lam"] if f.exists() else None
    f = g / f"spectrum_{name}.json"
    return json.loads(f.read_text())["lam"] if f.exists() else None


def tts_window(S, ctx, w, vd_all, steps):
    """FP64 against both mixed modes on a window that holds eigenvalues: per-step time,
    eigenvalues and residuals, the largest relative eigenvalue difference from FP64 and
    from the reference spectrum; and Rayleigh-Ritz against block Hankel (extraction
    time, device memory, accuracy) on the FP64 solve of that window."""
    import numpy as np
    win = WINDOWS.get(w.name)
    if not win:
        return None, None
    ref = reference_spectrum(w.name)
    gamma, rho = 0.5 * (win["lo"] + win["hi"]), 0.5 * (win["hi"] - win["lo"])
    vd = vd_all[:win["L"]].contiguous()
    out = {"window": [win["lo"], win["hi"]], "beta": win["beta"], "N": win["N"], "M": win["M"], "L": win["L"]}
    truth = None
    if ref is not None:
        lam_ref = np.array(ref)
        truth = np.sort(lam_ref[(lam_ref >= win["lo"]) & (lam_ref <= win["hi"])])
        out["reference_eigs"] = truth.round(13).tolist()
    ctx.set_profiling(0)
    lams = {}
    ext = {}
    for name in win.get("modes", ("fp64", "mixed_shifts", "mixed", "fp64_hankel")):
        # "_inloop": moments summed inside the solve (block form); otherwise stored solutions
        base = name.replace("_hankel", "").replace("_inloop", "")
        opts = S.default_opts(tol=w.tol, prec=PRECS[base], ru_interval=w.ru_interval, switch_tol=w.switch_tol)
        p = S.default_ss_params(gamma=gamma, rho=rho, beta=win["beta"], N=win["N"], M=win["M"], rank_tol=1e-7,
                                spur_tol=1e-6, solve=opts, method=S.HANKEL if name.endswith("hankel") else S.RR,
                                moments_in_loop=int(name.endswith("_inloop")))
        dt, r = solve_steps(S, ctx, p, vd, 32, steps)
        s = mode_summary(r, dt * 1e3, win["L"])
        if truth is not None and len(r.lam) == len(truth) and len(truth):
            s["max_rel_err_vs_reference"] = float(np.max(np.abs(r.lam - truth) / np.abs(truth)))
        lams[name] = r.lam
        if name in ("fp64", "fp64_hankel"):
            ext["rr" if name == "fp64" else "hankel"] = {
                "t_extract_ms": round(r.info.t_extract * 1e3, 2), "extract_bytes": int(r.info.extract_bytes),
                "rank": int(r.info.rank), "eigenpairs_found": int(r.n_found),
                "max_res": s["max_res"], "max_rel_err_vs_reference": s.get("max_rel_err_vs_reference")}
        if name == "fp64_hankel":
            continue
        out[name] = s
    a = lams["fp64"]
    for name in lams:
        if name in ("fp64", "fp64_hankel"):
            continue
        b = lams[name]
        out[name]["max_rel_eig_diff_vs_fp64"] = (float(np.max(np.abs(a - b) / np.abs(a)))
                                                 if len(a) == len(b) and len(a) else None)
        out[name]["speedup_vs_fp64"] = round(out["fp64"]["ms_per_step"] / out[name]["ms_per_step"], 3)
    return out, ext


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
    w = synth.CONFIGS["wilson24x48"]
    U = w.gauge()
    x = torch.from_numpy(w.sources()).to("cuda:0")
    y = torch.empty_like(x)
    out = {"lattice": list(w.dims), "sources": w.L}
    for name, prec, lr, wb in (("fp32_links12", S.MIXED, 12, 4), ("fp64_links18", S.FP64, 18, 8)):
        c = S.Context(w.dims, w.kappa)
        c.set_gauge(U, lr)
        c.apply_A(x, y, prec)            # chooses the launch shape
        c.set_profiling(1)
        for _ in range(reps):
            c.apply_A(x, y, prec)
        ms, calls = c.stage_times()
        avg_s = ms[0] / 1e3 / calls[0]
        nbytes = w.L * w.V * 24 * wb * 2 + w.V * 4 * lr * wb
        ach = nbytes / avg_s / 1e9
        out[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": pmc_traffic("dslash_" + name, w.name, "apply"), "avg_launch_us": round(avg_s * 1e6, 2),
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


def kernel_bytes(w, prec, tot, link_launches, moments_in_loop, blk=0):
    """Algorithmic (compulsory) HBM bytes of the shift update and the dslash over the
    timed steps. Shift update: read and write x_j and p_j per active (shift, source,
    entry) (64 B FP64, 32 B FP32), the seed r read once and the seed p read and written
    once per (source, entry, iteration) (48 B FP64, 24 B FP32 for the FP32 seed of the
    "mixed" mode). Dslash: the spinor in and out per (source, site) and the four
    forward links per site once per launch."""
    n = w.n
    seed32 = prec == PRECS["mixed"]
    su64 = tot["shift_updates"] - tot["shift_updates_fp32"]
    su32 = tot["shift_updates_fp32"]
    it64 = tot["seed_iters"] - tot["seed_iters_fp32"]
    it32 = tot["seed_iters_fp32"]
    shift = (su64 * 64 + it64 * 48) * n + (su32 * 32 + it32 * (24 if seed32 else 48)) * n
    if moments_in_loop and blk:
        # block form: the shift stage is the table launch (a few hundred bytes per
        # shift, not counted) and the seed direction update (r read, p read and
        # written per (source, entry, iteration)); the sweep is counted per pass
        shift = (it64 + it32) * 48 * n
    elif moments_in_loop:
        # p_j read and written per active (shift, source, entry); per (source, entry,
        # iteration) the seed r read, the seed p read and written, the M moments read
        # and written (the stage also holds the table launch that forms the shift
        # scalars, a few hundred bytes per shift, not counted)
        shift = (su64 * 32 + su32 * 16 + (it64 + it32) * (48 + 32 * w.M)) * n
    dslash = (it64 * 48 * 8 + it32 * 48 * (4 if seed32 else 8)) * w.V
    dslash += (link_launches[0] * 18 * 8 + link_launches[1] * (w.link_reals * 4 if seed32 else 18 * 8)) * 4 * w.V
    return shift, dslash


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tts-steps", type=int, default=2, help="steps per mode of the time-to-solution comparisons")
    ap.add_argument("--config", default=DEFAULT_CONFIG)
    ap.add_argument("--method", default="rr", choices=["rr", "hankel"])
    ap.add_argument("--prec", default="fp64", choices=["fp64", "mixed", "mixed_shifts", "workload"],
                    help="precision of the timed steps (default FP64; 'workload' = the workload's own mode)")
    ap.add_argument("--stored", action="store_true",
                    help="store the shifted solutions and form the moments after the solve (default: the moments "
                         "are accumulated inside the solve when the extraction allows it, Rayleigh-Ritz with "
                         "at most 32 moments)")
    ap.add_argument("--with-mixed-seed", action="store_true",
                    help="also time the FP32-seed mode (SSCG_MIXED) in the comparison")
    ap.add_argument("--budget", type=float, default=420.0,
                    help="seconds after which the optional comparisons are skipped")
    ap.add_argument("--weighted-tol", action="store_true", help="moment-weighted per-shift stopping")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dslash-large", action="store_true",
                    help="skip the dslash-only measurement on the 24^3 x 48 lattice")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 vs mixed time-to-solution comparisons")
    ap.add_argument("--sample-every", type=int, default=None,
                    help="time every stage of every k-th iteration (graph replay kept; default 25 for FP64 "
                         "solves, 10 for the mixed modes); 1 times every launch with direct launches")
    ap.add_argument("--only-dslash-large", action="store_true",
                    help="run only the dslash measurement on the 24^3 x 48 lattice and print it (for profiling)")
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

    if args.only_dslash_large:
        print(json.dumps({"dslash_24x48": dslash_large(S)}), flush=True)
        return
    if args.config == "batch":
        bench_batch(args)
        return
    t_start = time.perf_counter()
    w = synth.CONFIGS[args.config]
    mode = w.prec if args.prec == "workload" else args.prec
    args.moments_in_loop = (not args.stored and args.method == "rr" and w.M <= 32 and mode != "mixed")
    # the block length is set here for the library too (it reads SSCG_BLOCK at each solve)
    os.environ.setdefault("SSCG_BLOCK", str(BLOCK_DEFAULT))
    blk = int(os.environ["SSCG_BLOCK"]) if args.moments_in_loop else 0
    prec = PRECS[mode]
    print(f"[bench] {w.name} {w.dims} N={w.N} L={w.L} M={w.M} prec={mode}", file=sys.stderr, flush=True)
    U = w.gauge()
    ctx = S.Context(w.dims, w.kappa, device=0)
    ctx.set_gauge(U, w.link_reals)
    del U
    vd = torch.from_numpy(w.sources()).to("cuda:0")
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
    ctx.set_profiling(args.sample_every)
    for _ in range(args.warmup):
        ctx.ss_eigs(params, vd, max_eigs=max_eigs)
    torch.cuda.synchronize()
    print("[bench] warm-up done", file=sys.stderr, flush=True)
    stage_ms = np.zeros(8)
    stage_calls = np.zeros(8, dtype=np.int64)
    stage_launched = np.zeros(8, dtype=np.int64)
    sweep_bytes = 0          # algorithmic bytes of the block sweeps (library count)
    stage_est = np.zeros(8)          # sampled average times launches, summed over steps
    tot = dict(shift_updates=0, shift_updates_fp32=0, seed_iters=0, seed_iters_fp32=0, matvecs=0,
               t_solve=0.0, t_moments=0.0, t_extract=0.0)
    link_launches = [0, 0]   # dslash launches doing work in the FP64 and FP32 phases
    launched_tot = 0
    work_launches = 0        # launches with a source still iterating (the others exit at once)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = ctx.ss_eigs(params, vd, max_eigs=max_eigs)
        ms, calls = ctx.stage_times()
        launched = ctx.stage_launches()
        stage_ms += ms
        stage_calls += calls
        stage_launched += launched
        sweep_bytes += ctx.sweep_bytes()
        for k in TIMED_STAGES:
            if calls[k] > 0:
                stage_est[k] += ms[k] / calls[k] * launched[k]
        launched_tot += int(launched[6])
        work_launches += int(out.info.iters)
        for k in tot:
            tot[k] += getattr(out.info, k)
        sw = out.info.switch_iter if out.info.switch_iter >= 0 else out.info.iters
        link_launches[0] += min(out.info.iters, sw)
        link_launches[1] += max(0, out.info.iters - sw)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print("[bench] timed steps done", file=sys.stderr, flush=True)
    value = tot["shift_updates"] / elapsed
    step_ms = elapsed / args.steps * 1e3

    shift_bytes, dslash_bytes = kernel_bytes(w, prec, tot, link_launches, args.moments_in_loop, blk)
    # working set of the solve: the FP64 shift slots and solutions (or moments) of every
    # (source, node), the seed vectors and the links; above the 256 MB Infinity Cache
    # the streams come from HBM, below it they can stay in the cache
    ws_bytes = w.L * w.N * w.n * 16 * (1 if args.moments_in_loop else 2) + 4 * w.L * w.n * 16 + w.V * 4 * 144
    resident = "hbm" if ws_bytes > MALL_BYTES else "mall"
    rep = {}
    upd_name = ("seed_p_update" if blk else "shift_moments") if args.moments_in_loop else "shift_update"
    for name, idx, b in ((upd_name, 4, shift_bytes), ("dslash", 0, dslash_bytes)):
        calls = int(stage_calls[idx])  # launches timed (every k-th when sampling)
        if calls == 0 or stage_ms[idx] <= 0 or work_launches == 0:
            rep[name] = None
            continue
        avg_s = stage_ms[idx] / 1e3 / calls
        # the sampled iterations lie inside the run of every source, so their launches
        # do work: the bytes are averaged over the launches that do work (iterations
        # launched after the last source finished exit at once)
        per_launch = b / work_launches
        ach = per_launch / avg_s / 1e9
        rep[name] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": pmc_traffic(name, w.name, mode), "kernel": name,
                     "working_set_resident_in": resident,
                     "launches": launched_tot, "launches_doing_work": work_launches, "launches_timed": calls,
                     "avg_launch_us": round(avg_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": round(per_launch)}
    if blk:
        # the sweep: the library counts the algorithmic bytes of every sweep of the
        # solve (the directions actually read and written, the residuals and moment
        # sums); divided by the sweeps' time estimated from the sampled ones (every
        # sweep is timed when the sampling period is at most the block length)
        calls = int(stage_calls[7])
        if calls > 0 and stage_ms[7] > 0 and stage_launched[7] > 0:
            avg_s = stage_ms[7] / 1e3 / calls
            per_pass = sweep_bytes / stage_launched[7]
            ach = sweep_bytes / (stage_est[7] / 1e3) / 1e9
            rep["block_sweep"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(ach / HBM_PEAK_GBS, 4),
                                  "traffic": pmc_traffic("block_sweep", w.name, mode), "kernel": "block_sweep",
                                  "kernels": ["blk_compose_kernel", "blk_moments_kernel", "blk_dirs_kernel"],
                                  "block": blk, "working_set_resident_in": resident,
                                  "launches": int(stage_launched[7]), "launches_timed": calls,
                                  "avg_launch_us": round(avg_s * 1e6, 2),
                                  "algorithmic_bytes_per_launch": round(per_pass)}
        else:
            rep["block_sweep"] = None
    per_step = stage_est / args.steps
    cands = ([("block_sweep", 7)] if blk else []) + [(upd_name, 4), ("dslash", 0)]
    dominant = max(cands, key=lambda kv: per_step[kv[1]])[0]
    stage_split = {STAGES[i]: round(float(per_step[i]), 3) for i in TIMED_STAGES if i != 3}
    matvec_ms = float(per_step[0])
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "shift-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == S.FP64 else "f32+f64",
        "prec_mode": mode,
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": list(w.dims), "kappa": w.kappa, "eps": w.eps, "seed": w.seed,
                   "interval": [w.gamma - w.rho, w.gamma + w.rho], "beta": w.beta, "N": w.N, "L": w.L,
                   "M": w.M, "tol": w.tol, "prec": mode,
                   "link_reals": w.link_reals if prec == S.MIXED else 18,
                   "method": args.method, "moments_in_loop": bool(args.moments_in_loop), "block": blk,
                   "weighted_tol": bool(args.weighted_tol), "parallelism": "single GPU"},
        "roofline": rep[dominant],
        "dslash": rep["dslash"],
        "site_shift_updates_per_s": round(value * w.V, 1),
        "seed_iters_per_source": tot["seed_iters"] / args.steps / w.L,
        "eigenpairs_found": int(out.n_found),
        "stage_ms_per_step": stage_split,
        "table2_split": {"total_ms_per_step": round(step_ms, 2), "matvec_ms_per_step": round(matvec_ms, 2),
                         "matvec_fraction": round(matvec_ms / step_ms, 4),
                         "note": ("the paper's Table 2 reports matrix-vector time against total time; here "
                                  "the seed dslash (the only product with A in the solve) against the step")},
        "phase_ms_per_step": {k: round(tot[k] * 1e3 / args.steps, 3) for k in ("t_solve", "t_moments", "t_extract")},
        "timing": ("direct launches, HIP events around every launch" if args.sample_every == 1 else
                   (f"graph replay, HIP event-record nodes around every stage of the last iteration of about "
                    f"one block in every {args.sample_every} iterations (its launches include the block "
                    f"sweep); stage times per step = sampled average x launches of the stage") if blk else
                   f"graph replay, HIP event-record nodes around every stage of every {args.sample_every}th "
                   f"iteration (offset {args.sample_every // 2} in each poll interval) and around every "
                   f"reliable update; stage times per step = sampled average x launches of the stage"),
    }
    base_res = mode_summary(out, step_ms, w.L)
    if not args.no_compare:
        print("[bench] mixed-precision comparison", file=sys.stderr, flush=True)
        line["tts"] = tts_compare(S, ctx, params, vd, max_eigs, args.tts_steps, step_ms, base_res,
                                  args.with_mixed_seed, t_start + args.budget)
        print("[bench] eigen window", file=sys.stderr, flush=True)
        tw, ext = (tts_window(S, ctx, w, vd, 1) if time.perf_counter() < t_start + args.budget
                   else ({"skipped": "time budget of the benchmark"}, None))
        if tw is not None:
            line["tts_window"] = tw
            line["extraction"] = ext
    ctx.close()
    del vd
    torch.cuda.empty_cache()
    line["copy_bw_GBs"] = copy_bandwidth()
    if not args.no_dslash_large:
        print("[bench] dslash alone on 24^3 x 48", file=sys.stderr, flush=True)
        line["dslash_24x48"] = dslash_large(S)
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, tot["seed_iters"] // args.steps)
    line["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
