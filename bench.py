#!/usr/bin/env python3
"""Benchmark: Chebyshev-filtered subspace iteration on one MI355X.

Workload (default, ``seq8192``): the 5-cycle sequence of correlated generalized problems,
complex128, n = 8192, S = I + G G^H / n, A_0 in designed form with 1/8 of the spectrum clustered in
[-1, -0.5], A_{l+1} = A_l + 5e-3 0.6^l (E + E^H)/2, nev = 400, nex = 80, FP64 filter of degree 12.
``seq2048`` is the 10-cycle n = 2048 sequence (nev 128, nex 64, eps_l = 1e-2 0.5^l).

A step is one warm-started solve of one cycle (reduction, Lanczos, filter/QR/Rayleigh-Ritz/locking
loop, back-transform and verification), with the inputs resident in HBM.  Before the timed region
the whole sequence is solved once (cycle 0 from a random block, each later cycle from the previous
solution); timed step s re-solves cycle 1 + (s mod (cycles - 1)) from the stored solution of the
cycle before it.

Printed JSON (one line): value = filter TFLOP/s over the timed steps (8 n^2 flops per filtered
vector and degree, divided by the filter phase time), ms_per_step = time to solution per cycle,
the roofline of the dominant kernel (the FP64 filter step) from the dispatches' own timestamps
(the main kernel alone and the whole step with its split-K reduction), and the CPU reference timed
on a bounded sample.  Extras: the n = 8192 sequence at degrees 8/12/16/20 with the FP64, FP32,
BF16x3 and BF16x6 filters, and with the analytic and learned per-vector degrees in FP64 and BF16x3,
and their per-eigenpair errors against the CPU reference's eigenvalues
(tests/golden/c3_oracle_eigenvalues.json), the n = 2048 sequence (warm vs random start, mixed
precision), the batched k-point cycle (32 problems, sequential vs one batch) and the learned
per-vector degree against fixed degrees and the analytic rule (20-cycle n = 4096 sequence).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}   # TFLOP/s, MI355X dense matrix peaks
HBM_PEAK_GBS = 8000.0
GOLDEN_C3 = os.path.join(ROOT, "tests", "golden", "c3_oracle_eigenvalues.json")
WORKLOADS = {
    "seq8192": "seq8192: 5-cycle correlated generalized sequence, complex128, n=8192, nev=400, nex=80, "
               "degree 12, warm start, FP64 filter",
    "seq2048": "seq2048: 10-cycle correlated generalized sequence, complex128, n=2048, nev=128, nex=64, "
               "degree 12, warm start, FP64 filter",
}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def spec_of(workload: str):
    from paper_1206_3768_amd import synth
    if workload == "seq8192":
        return synth.config_mixed_precision()
    return synth.config_generalized_sequence()


PREC_NAMES = {0: "fp64", 1: "fp32", 2: "bf16x3", 3: "bf16x6"}
PREC_DTYPE = {0: "f64", 1: "f32", 2: "bf16x3", 3: "bf16x6"}
PREC_PROFILE = {0: "f64", 1: "f32", 2: "bf16x3", 3: "bf16x6"}


def kernel_symbol(prec: int, bm: int, bn: int, mode: int) -> str:
    """Symbol of the filter-step kernel of a launch-log row (as rocprofv3 names it)."""
    if prec == 0:
        return f"k_zgemm<double, 0, 0, 1, {bm}, {bn}, {mode}>"
    if prec == 1:
        return f"k_zgemm<float, 0, 0, 1, {bm}, {bn}, {mode}>"
    split = 'true' if mode else 'false'
    if prec == 2 and bm == 128:
        return f"k_filter_bf16_p<{split}>"
    return f"k_filter_bf16<{2 if prec == 2 else 3}, {split}, {bm // 32}>"


def peak_and_products(prec: int):
    """MFMA peak of the arithmetic of `prec` (TFLOP/s) and the executed products per counted one:
    the BF16-split filters run 3 or 6 BF16 products for each complex product of the standard count."""
    if prec == 0:
        return PEAK["f64"], 1
    if prec == 1:
        return PEAK["f32"], 1
    return PEAK["bf16"], (3 if prec == 2 else 6)


def load_traffic(workload: str, kernel: str, prec: int = 0):
    """The committed rocprofv3 counter summary of `kernel` on this workload, if it was taken on the
    current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"filter_{PREC_PROFILE[prec]}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    from paper_1206_3768_amd.traffic import kernel_source_hash
    if t.get("kernel_source_sha256_16") != kernel_source_hash() or t.get("kernel") != kernel:
        return None
    return t


def golden_c3():
    """Eigenvalues of the n = 8192 sequence computed by the CPU reference (dict cycle -> array)."""
    if not os.path.exists(GOLDEN_C3):
        return {}
    with open(GOLDEN_C3) as fh:
        g = json.load(fh)
    return {c["cycle"]: np.array([float(v) for v in c["lam"]]) for c in g["cycles"]}


def pair_errors(lam, ref):
    """Per-eigenpair relative errors |lam_i - ref_i| / max(|ref_i|, 1e-3) and their summary."""
    e = np.abs(lam[:len(ref)] - ref) / np.maximum(np.abs(ref), 1e-3)
    hist = {}
    for lo in range(-17, -9):
        hist[f"1e{lo}"] = int(np.sum((e >= 10.0 ** lo) & (e < 10.0 ** (lo + 1))))
    hist["below_1e-17"] = int(np.sum(e < 1e-17))
    hist["above_1e-10"] = int(np.sum(e >= 1e-10))
    return e, {"max": float(e.max()), "median": float(np.median(e)), "argmax": int(np.argmax(e)), "decades": hist}


def cpu_baseline(workload: str, seq_spec, A_host) -> dict:
    """The CPU reference as it stands (plain loops, all host threads) on a bounded sample of the
    workload: one filter of the first `cols` columns of the block at the workload's degree with the
    workload's H = A_1 of the sequence."""
    import oracle
    n, d = seq_spec.n, seq_spec.deg
    cols = 8 if n > 4096 else seq_spec.nev + seq_spec.nex
    rng = np.random.default_rng(0)
    Y = (rng.standard_normal((n, cols)) + 1j * rng.standard_normal((n, cols))) / np.sqrt(2)
    t0 = time.perf_counter()
    oracle.cheb_filter(A_host, Y, -0.3, 1.5, -1.0, deg=d)
    tf = time.perf_counter() - t0
    flops = 8.0 * n * n * cols * d
    return {"value": round(flops / tf / 1e12, 5), "unit": "TFLOP/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{workload}: oracle filter (plain loops, FP64) of a {n} x {cols} block at degree {d} with "
                      f"the sequence's A_1 ({tf:.2f} s, {flops / 1e9:.1f} GFLOP)", "seconds": round(tf, 2)}


def roofline(rows: np.ndarray, workload: str, prec: int = 0) -> dict:
    """Dominant filter kernel of precision `prec` (the (tile, split mode) group with the largest
    summed main-kernel time): algorithmic flops per launch over its average dispatch duration, alone
    and with its split-K reduction; HBM traffic from the committed counter summary when it matches
    the sources."""
    groups = {}
    for nn, w, pr, bm, bn, ks, mode, t_main, t_step in rows:
        if int(pr) != prec:
            continue
        key = (int(pr), int(bm), int(bn), int(mode))   # one kernel symbol per (tile, split mode)
        g = groups.setdefault(key, [0.0, 0.0, 0.0, 0, 0.0, 0.0])
        g[0] += 8.0 * nn * nn * w
        g[1] += t_main * 1e-3
        g[2] += t_step * 1e-3
        g[3] += 1
        g[4] += 16.0 * nn * nn + 3.0 * 16.0 * nn * w      # algorithmic bytes: H, Y_k, Y_{k-1} read, Y_{k+1} written
        g[5] = nn
    key, (g_flops, g_time, g_step, g_count, g_bytes, g_n) = max(groups.items(), key=lambda kv: kv[1][1])
    achieved = g_flops / g_time / 1e12
    achieved_step = g_flops / g_step / 1e12
    kernel = kernel_symbol(prec, key[1], key[2], key[3])
    tr = load_traffic(workload, kernel, prec)
    alg_bytes = g_bytes / g_count
    peak, products = peak_and_products(prec)
    out = {"bound": "mfma", "achieved": round(achieved * products, 3), "peak": peak, "unit": "TFLOP/s",
           "frac": round(achieved * products / peak, 4),
           "traffic": tr["bytes_per_launch"] if tr else None,
           "kernel": kernel, "flops_per_launch": g_flops / g_count, "avg_launch_ms": g_time / g_count * 1e3,
           "launches": g_count,
           # the whole filter step: the main kernel and, for a split-K plan, the kernel summing its
           # partial tiles and applying the recurrence
           "step_achieved": round(achieved_step * products, 3),
           "step_frac": round(achieved_step * products / peak, 4),
           "avg_step_ms": g_step / g_count * 1e3,
           "standard_count_tflops": round(achieved, 3),
           # the three-product complex MFMA executes 6 of the 8 counted flops per complex multiply-add
           "mfma_frac": round((0.75 if prec < 2 else 1.0) * achieved * products / peak, 4),
           "algorithmic_bytes_per_launch": alg_bytes,
           "all_filter_launches": {"count": int(len(rows)),
                                   "tflops": round(float(np.sum(8.0 * rows[:, 0] ** 2 * rows[:, 1]) /
                                                         np.sum(rows[:, 7] * 1e-3) / 1e12), 3),
                                   "tflops_with_reduce": round(float(np.sum(8.0 * rows[:, 0] ** 2 * rows[:, 1]) /
                                                                     np.sum(rows[:, 8] * 1e-3) / 1e12), 3)}}
    if tr:
        out["traffic_over_algorithmic"] = round(tr["bytes_per_launch"] / alg_bytes, 3)
        out["traffic_source"] = f"profiles/filter_{PREC_PROFILE[prec]}_{workload}_traffic.json"
    return out


def timed_sequence(seq, spec, steps: int, warmup: int, prec: int = 0):
    """Warm-started solves of cycles 1 .. cycles-1 in turn (filter precision `prec`); returns
    results and launch logs."""
    import torch
    cycles = [1 + (s % (spec.cycles - 1)) for s in range(warmup + steps)]
    work = seq.new_block()
    for c in cycles[:warmup]:
        seq.solve(c, warm=True, X=work, filter_precision=prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed, launch_rows = [], []
    for c in cycles[warmup:]:
        timed.append(seq.solve(c, warm=True, X=work, filter_precision=prec))
        launch_rows.append(seq.h.filter_launch_log())   # host-side copy of this solve's event log
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rows = np.concatenate(launch_rows) if launch_rows else np.zeros((0, 9))
    return timed, rows, wall, work


def correlation_summary(seq, spec) -> dict:
    """Angles between the eigenvectors of successive cycles of the sequence (the stored solutions of
    the reference pass): sines of the principal angles between the spans of the nev wanted vectors
    and of the angle each vector turns by (chfsi_correlation), per cycle."""
    out = {}
    nev = spec.nev
    for c in range(1, spec.cycles):
        Xp, Xc = seq.X[c - 1], seq.X[c]
        if Xp is None or Xc is None:
            continue
        _, sp, ss = seq.h.correlation(Xp[:nev], Xc[:nev], seq.S, n=spec.n, m=nev)
        out[f"{c - 1}->{c}"] = {"max_sin_principal": float(ss.max()), "median_sin_principal": float(np.median(ss)),
                                "max_sin_pair": float(sp.max()), "median_sin_pair": float(np.median(sp))}
    return out


def phase_summary(timed) -> dict:
    phase = {k: round(sum(r.stats[k] for r in timed) / len(timed), 3)
             for k in ("t_reduce", "t_lanczos", "t_filter", "t_qr", "t_rr", "t_resid", "t_lock", "t_back", "t_total")}
    return phase


def bench_c3_sweep(seq, spec, golden) -> dict:
    """The n = 8192 sequence at degrees 8, 12, 16, 20 with every filter precision, then with the
    analytic and learned per-vector degrees in FP64 and BF16x3: warm cycles 1..cycles-1, time to
    solution, loops, matrix-vector products, precision switches, and the per-eigenpair error of
    every converged eigenvalue against the CPU reference."""
    out = {"workload": f"n={spec.n} generalized sequence, nev {spec.nev}, nex {spec.nex}, warm cycles 1..{spec.cycles - 1}",
           "reference": "tests/golden/c3_oracle_eigenvalues.json (CPU oracle, FP64)" if golden else None}
    work = seq.new_block()

    def run(base, **kw):
        seq.solve(1, warm=True, X=work, **kw)   # untimed: workspace, H copies
        rs = [seq.solve(c, warm=True, X=work, **kw) for c in range(1, spec.cycles)]
        tot = sum(r.wall_ms for r in rs)
        rec = {"all_converged": all(r.status == 0 for r in rs), "time_to_solution_ms": round(tot, 1),
               "speedup_vs_fp64": round(base / tot, 3) if base else None,
               "filter_ms": round(sum(r.stats["t_filter"] for r in rs), 1),
               "matvecs": sum(r.stats["matvecs"] for r in rs), "loops": [r.stats["loops"] for r in rs],
               "precision_switches": [r.stats["precision_switches"] for r in rs],
               "max_resid": float(max(r.resid[:spec.nev].max() for r in rs))}
        if golden:
            per = {}
            for r in rs:
                if r.status == 0 and r.cycle in golden:
                    _, summ = pair_errors(r.lam, golden[r.cycle])
                    per[str(r.cycle)] = summ
            rec["rel_eig_err_vs_oracle"] = per
        return rec, tot

    best_fixed = None
    for d in (8, 12, 16, 20):
        base = None
        for name in ("fp64", "fp32", "bf16x3", "bf16x6"):
            rec, tot = run(base, filter_precision=name, deg=d)
            if name == "fp64":
                base = tot
                rec["speedup_vs_fp64"] = 1.0
                best_fixed = tot if best_fixed is None else min(best_fixed, tot)
            out[f"d{d}_{name}"] = rec
            log(f"c3 degree {d} {name}: {rec['time_to_solution_ms']} ms, loops {rec['loops']}")
    # per-vector degrees on the same warm cycles: the analytic rule and the network (trained on the
    # n = 4096 traces), with the margins chosen on the network's selection seed, never on this
    # sequence; speedups against the fastest fixed degree in FP64
    from paper_1206_3768_amd import chfsi, degree_model
    info = degree_model.meta()
    margin = int(info.get("margin", degree_model.LEARNED_MARGIN))
    margin_an = int(info.get("analytic_margin", margin))
    blob = degree_model.load()
    policies = [("analytic", chfsi.DEG_ANALYTIC, margin_an)]
    if blob is not None:
        policies.append(("learned", chfsi.DEG_LEARNED, margin))
        seq.h.set_degree_model(blob)
    try:
        for pol, code, mg in policies:
            for name in ("fp64", "bf16x3"):
                rec, _ = run(best_fixed, filter_precision=name, degree_policy=code, deg_margin=mg)
                rec["speedup_vs_best_fixed_fp64"] = rec.pop("speedup_vs_fp64")
                out[f"{pol}+{mg}_{name}"] = rec
                log(f"c3 {pol}+{mg} {name}: {rec['time_to_solution_ms']} ms, loops {rec['loops']}")
    finally:
        if blob is not None:
            seq.h.set_degree_model(None)
    return out


def bench_seq2048(h, steps: int = 9) -> dict:
    """The n = 2048 sequence: timed warm solves, the dominant kernel, warm vs random start, the
    low-precision filters and the analytic degree on the same cycles, phase times."""
    from paper_1206_3768_amd import sequence
    spec = spec_of("seq2048")
    seq = sequence.Sequence(spec, handle=h)
    ref = seq.run_reference()
    if any(r.status != 0 for r in ref):
        return {"failed": "reference pass"}
    timed, rows, wall, work = timed_sequence(seq, spec, steps, 1)
    flops = sum(r.stats["filter_flops"] for r in timed)
    t_filter = sum(r.stats["t_filter"] for r in timed) * 1e-3
    out = {"workload": WORKLOADS["seq2048"], "filter_tflops": round(flops / t_filter / 1e12, 3),
           "ms_per_step": round(wall / len(timed) * 1e3, 3), "roofline": roofline(rows, "seq2048")}
    warm_ms = {}
    for r in timed:
        warm_ms.setdefault(r.cycle, r.wall_ms)
    rnd = {c: seq.solve(c, warm=False, X=work) for c in range(1, spec.cycles)}
    out["warm_vs_random"] = {
        str(c): {"t_app_ms": round(warm_ms.get(c, float("nan")), 3), "t_rnd_ms": round(rnd[c].wall_ms, 3),
                 "speedup": round(rnd[c].wall_ms / warm_ms[c], 3) if c in warm_ms else None,
                 "loops_app": next((r.stats["loops"] for r in timed if r.cycle == c), None),
                 "loops_rnd": rnd[c].stats["loops"]} for c in range(1, spec.cycles)}
    mixed = {}
    for name in ("fp32", "bf16x6", "bf16x3"):
        rs = [seq.solve(c, warm=True, X=work, filter_precision=name) for c in range(1, spec.cycles)]
        mixed[name] = {"all_converged": all(r.status == 0 for r in rs),
                       "time_to_solution_ms_total": round(sum(r.wall_ms for r in rs), 3),
                       "fp64_total_ms": round(sum(warm_ms.get(r.cycle, float("nan")) for r in rs), 3),
                       "max_resid": float(max(r.resid[:spec.nev].max() for r in rs)),
                       "loops": [r.stats["loops"] for r in rs],
                       "precision_switches": [r.stats["precision_switches"] for r in rs]}
    out["mixed_precision"] = mixed
    an = [seq.solve(c, warm=True, X=work, degree_policy=1) for c in range(1, spec.cycles)]
    out["analytic_degree"] = {"time_to_solution_ms_total": round(sum(r.wall_ms for r in an), 3),
                              "all_converged": all(r.status == 0 for r in an),
                              "matvecs": [r.stats["matvecs"] for r in an]}
    phase = phase_summary(timed)
    out["phase_ms_per_solve"] = phase
    out["solve_only_ms_per_solve"] = round(sum(phase[k] for k in ("t_lanczos", "t_filter", "t_qr", "t_rr",
                                                                   "t_resid", "t_lock")), 3)
    return out


def bench_lobpcg(h, kappa: float = 1e6, maxiter_gen: int = 300) -> dict:
    """Table 2's comparison on a synthetic pencil: block LOBPCG iterating on the pencil (GEN) and on
    the reduced problem (STD, reduction included in its time), tolerances 1e-6, 1e-8, 1e-10, from a
    random block and from the previous cycle's eigenvectors; ChFSI on the same problem beside it.
    Cycle 1 of the n = 2048 sequence with an overlap of condition number `kappa`, nev 128, block
    1.05 nev (Table 3).  GEN runs are capped at `maxiter_gen` iterations (status 3 when they stop)."""
    import torch
    from paper_1206_3768_amd import chfsi, synth
    spec = synth.config_ill_conditioned(kappa=kappa, cycles=2)
    pens = list(synth.sequence(spec))
    nev = spec.nev
    bs = int(np.ceil(1.05 * nev))
    dA0, dA1 = chfsi.to_device(pens[0].A), chfsi.to_device(pens[1].A)
    dS = chfsi.to_device(pens[0].S)
    # the approximate start: cycle 0's eigenvectors (STD LOBPCG at 1e-10)
    X0 = torch.zeros((bs, spec.n), dtype=torch.complex128, device="cuda")
    r0 = h.lobpcg(dA0, dS, X0, False, nev=nev, tol=1e-10, seed=1)
    out = {"workload": f"n={spec.n} generalized, kappa(S)={kappa:g}, cycle 1 of the sequence, nev {nev}, block {bs}",
           "cycle0_status": r0.status}
    work = X0.clone()
    for tol in (1e-6, 1e-8, 1e-10):
        for start in ("random", "approx"):
            for gen in (False, True):
                work.copy_(X0)
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = h.lobpcg(dA1, dS, work, start == "approx", nev=nev, tol=tol, gen=gen, seed=2,
                             maxiter=maxiter_gen if gen else 1000, raise_on_error=False)
                ms = (time.perf_counter() - t) * 1e3
                key = f"tol{tol:g}_{start}_{'gen' if gen else 'std'}"
                out[key] = {"status": r.status, "ms": round(ms, 1), "iters": r.stats["iters"],
                            "matvecs": r.stats["matvecs"], "bmatvecs": r.stats["bmatvecs"],
                            "nconv": r.stats["nconv"], "restarts": r.stats["restarts"],
                            "max_resid": float(np.max(r.resid[:nev]))}
                log(f"LOBPCG {key}: status {r.status}, {ms:.0f} ms, {r.stats['iters']} iterations")
    # ChFSI on the same cycle, same starts, tolerance 1e-10
    m = spec.nev + spec.nex
    for start in ("random", "approx"):
        Xc = torch.zeros((m, spec.n), dtype=torch.complex128, device="cuda")
        if start == "approx":
            Xc[:bs].copy_(X0)
            Xc[bs:].copy_(h.random_block(3, 1, spec.n, m - bs))
        prm = chfsi.default_params(nev=nev, nex=spec.nex, deg=spec.deg, tol=1e-10, seed=2)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = h.solve(dA1, dS, Xc, start == "approx", prm, raise_on_error=False)
        out[f"chfsi_tol1e-10_{start}"] = {"status": r.status, "ms": round((time.perf_counter() - t) * 1e3, 1),
                                         "loops": r.stats["loops"], "matvecs": r.stats["matvecs"]}
    return out


def bench_kpoints(h, count: int = 32) -> dict:
    """Batched SCF cycle: `count` k-point problems (n uniform in [1500, 6000], nev = ceil(0.06 n),
    nex = ceil(0.2 nev), warm start from the unperturbed eigenvectors, perturbation 1e-3), solved
    one after another with chfsi_solve and as one batch with chfsi_solve_batched (persistent
    filter launch with the autotuned tile, graph replay and without it, the per-problem phases
    spread over three streams with a host thread each)."""
    import torch
    from paper_1206_3768_amd import chfsi, synth
    t0 = time.perf_counter()
    sizes = synth.kpoint_sizes(count)
    probs, x0 = [], []
    for k, n in enumerate(sizes):
        kp = synth.kpoint_problem(k, n)
        probs.append(dict(A=chfsi.to_device(kp.A), S=chfsi.to_device(kp.S), X=chfsi.to_device(kp.X0),
                          nev=kp.nev, nex=kp.nex, x_is_guess=1))
        x0.append(probs[-1]["X"].clone())
        del kp
    log(f"k-points: {count} problems generated and resident ({time.perf_counter() - t0:.1f} s)")

    def reset():
        for p, x in zip(probs, x0):
            p["X"].copy_(x)
        torch.cuda.synchronize()

    seq_ms, seq_lam, seq_loops, seq_flops, seq_filter_ms, seq_phase_ms = 0.0, [], [], 0.0, 0.0, 0.0
    reset()
    p = probs[0]   # warm-up of the sequential path on the first problem
    h.solve(p["A"], p["S"], p["X"], True, chfsi.default_params(nev=p["nev"], nex=p["nex"], deg=12, tol=1e-10))
    reset()
    for p in probs:
        prm = chfsi.default_params(nev=p["nev"], nex=p["nex"], deg=12, tol=1e-10)
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = h.solve(p["A"], p["S"], p["X"], True, prm)
        seq_ms += (time.perf_counter() - t) * 1e3
        if r.status != 0:
            raise RuntimeError(f"sequential k-point solve failed: status {r.status}")
        seq_lam.append(r.lam[:p["nev"]].copy())
        seq_loops.append(r.stats["loops"])
        seq_flops += r.stats["filter_flops"]
        seq_filter_ms += r.stats["t_filter_kernels"]
        seq_phase_ms += r.stats["t_filter"]
    reset()
    plan, plan_ms = h.autotune_batched(probs)
    out = {"count": count, "n_range": [min(sizes), max(sizes)], "sequential_ms": round(seq_ms, 1),
           "sequential_filter_tflops": round(seq_flops / seq_filter_ms / 1e9, 2),
           "sequential_filter_phase_tflops": round(seq_flops / seq_phase_ms / 1e9, 2),
           "autotuned_tile": list(plan), "autotune_step_ms": round(plan_ms, 3)}
    prm = chfsi.default_params(nev=1, nex=0, deg=12, tol=1e-10)
    for lanes in (3, 1):
        for use_graph in ((True, False) if lanes == 3 else (True,)):
            h.set_batched_plan(*plan, use_graph=use_graph, lanes=lanes)
            best = None
            for _ in range(2):
                reset()
                t = time.perf_counter()
                st, res = h.solve_batched(probs, prm)
                ms = (time.perf_counter() - t) * 1e3
                if st != 0:
                    raise RuntimeError(f"batched k-point solve failed: status {st}")
                best = ms if best is None else min(best, ms)
            info = h.batched_info()
            dl = max(float(np.max(np.abs(r.lam[:p["nev"]] - l) / np.maximum(np.abs(l), 1e-3)))
                     for r, p, l in zip(res, probs, seq_lam))
            key = ("graph" if use_graph else "no_graph") + ("" if lanes == 3 else "_one_lane")
            out[key] = {
                "lanes": lanes, "batched_ms": round(best, 1), "speedup_vs_sequential": round(seq_ms / best, 3),
                "filter_ms": round(info["filter_ms"], 1),
                "filter_tflops": round(info["filter_flops"] / info["filter_ms"] / 1e9, 2),
                "graph_replays": info["graph_launches"], "persistent_launches": info["kernel_launches"],
                "max_rel_eig_diff_vs_sequential": dl,
                "max_resid": max(float(r.resid[:p["nev"]].max()) for r, p in zip(res, probs)),
                "loops_equal_to_sequential": [r.stats["loops"] for r in res] == seq_loops}
    # a tile per problem (per order and width), tuned problem by problem
    reset()
    tiles, tiles_ms = h.autotune_batched_tiles(probs)
    h.set_batched_plan(use_graph=True, lanes=3)
    best = None
    for _ in range(2):
        reset()
        t = time.perf_counter()
        st, res = h.solve_batched(probs, prm)
        ms = (time.perf_counter() - t) * 1e3
        if st != 0:
            raise RuntimeError(f"batched k-point solve (tile per problem) failed: status {st}")
        best = ms if best is None else min(best, ms)
    info = h.batched_info()
    counts = {}
    for bm, bn in tiles:
        counts[f"{bm}x{bn}"] = counts.get(f"{bm}x{bn}", 0) + 1
    out["graph_tile_per_problem"] = {
        "lanes": 3, "tiles": counts, "autotune_step_ms": round(tiles_ms, 3), "batched_ms": round(best, 1),
        "speedup_vs_sequential": round(seq_ms / best, 3), "filter_ms": round(info["filter_ms"], 1),
        "filter_tflops": round(info["filter_flops"] / info["filter_ms"] / 1e9, 2),
        "max_rel_eig_diff_vs_sequential": max(float(np.max(np.abs(r.lam[:p["nev"]] - l) / np.maximum(np.abs(l), 1e-3)))
                                              for r, p, l in zip(res, probs, seq_lam)),
        "max_resid": max(float(r.resid[:p["nev"]].max()) for r, p in zip(res, probs))}
    h.set_batched_tiles(None, None)
    h.set_batched_plan(64, 64, use_graph=True, lanes=3)
    return out


def bench_learned_degree(h, cycles: int = 20) -> dict:
    """Learned per-vector degree on the held-out seed 0 of the n = 4096 standard sequence (warm
    cycles 1 .. cycles-1), against the analytic rule it falls back to (with the same margin and
    without one) and every fixed degree; the margin and the best fixed degree come from the
    network's selection seed (degree_model_meta.json), never from this sequence.  FP64 and FP32
    filters."""
    from paper_1206_3768_amd import chfsi, degree_model, sequence, synth
    blob = degree_model.load()
    if blob is None:
        return {"skipped": "no trained network"}
    info = degree_model.meta()
    margin = int(info.get("margin", degree_model.LEARNED_MARGIN))
    margin_an = int(info.get("analytic_margin", margin))
    best = int(info.get("best_fixed_degree", 20))
    h.set_degree_model(blob)
    seq = sequence.Sequence(synth.config_learned_degree(seed=degree_model.EVAL_SEED, n=4096, cycles=cycles), handle=h)
    res = {}
    for d in degree_model.FIXED_DEGREES:
        res[f"fixed{d}"] = degree_model.run_policy(h, seq, chfsi.DEG_FIXED, deg=d)
    for mg in sorted({0, margin, margin_an}):
        res[f"analytic+{mg}"] = degree_model.run_policy(h, seq, chfsi.DEG_ANALYTIC, margin=mg)
    res["learned"] = degree_model.run_policy(h, seq, chfsi.DEG_LEARNED, margin=margin)
    res[f"fixed{best}_fp32"] = degree_model.run_policy(h, seq, chfsi.DEG_FIXED, deg=best, precision=chfsi.FP32)
    res[f"analytic+{margin}_fp32"] = degree_model.run_policy(h, seq, chfsi.DEG_ANALYTIC, margin=margin,
                                                             precision=chfsi.FP32)
    res["learned_fp32"] = degree_model.run_policy(h, seq, chfsi.DEG_LEARNED, margin=margin, precision=chfsi.FP32)
    h.set_degree_model(None)
    out = {k: {"time_to_solution_ms": round(v["ms"], 1), "matvecs": v["matvecs"], "loops": v["loops"],
               "filter_ms": round(v["filter_ms"], 1), "all_converged": v["ok"], "max_resid": v["max_resid"]}
           for k, v in res.items()}
    an = f"analytic+{margin}"
    ans = f"analytic+{margin_an}"
    post = min((f"fixed{d}" for d in degree_model.FIXED_DEGREES), key=lambda k: res[k]["ms"])
    out["margin"] = margin
    out["selection"] = {"seed": info.get("selection_seed"), "best_fixed": f"fixed{best}",
                        "analytic_margin": margin_an, "train_seeds": info.get("train_seeds"),
                        "train_cycles": info.get("cycles")}
    out["learned_vs_analytic_selected_margin_time"] = round(res[ans]["ms"] / res["learned"]["ms"], 3)
    out["learned_vs_analytic_selected_margin_matvecs"] = round(res[ans]["matvecs"] / res["learned"]["matvecs"], 3)
    out["best_fixed_on_this_sequence"] = post
    out["learned_vs_selected_fixed_time"] = round(res[f"fixed{best}"]["ms"] / res["learned"]["ms"], 3)
    out["learned_vs_selected_fixed_matvecs"] = round(res[f"fixed{best}"]["matvecs"] / res["learned"]["matvecs"], 3)
    out["learned_vs_analytic_same_margin_time"] = round(res[an]["ms"] / res["learned"]["ms"], 3)
    out["learned_vs_analytic_same_margin_matvecs"] = round(res[an]["matvecs"] / res["learned"]["matvecs"], 3)
    out["learned_fp32_vs_selected_fixed_fp64_time"] = round(res[f"fixed{best}"]["ms"] / res["learned_fp32"]["ms"], 3)
    out["learned_fp32_vs_analytic_fp32_time"] = round(res[an + "_fp32"]["ms"] / res["learned_fp32"]["ms"], 3)
    out["workload"] = f"n=4096 standard sequence, seed 0 (held out), warm cycles 1..{cycles - 1}, nev 256, nex 64"
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="seq8192", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the timed headline solves")
    ap.add_argument("--precision", default="fp64", choices=sorted(PREC_NAMES.values()),
                    help="filter arithmetic of the timed solves (the headline is FP64)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one MI355X; --gpus {args.gpus} is not supported: the solver drives "
              "one GPU and has no multi-GPU path", file=sys.stderr)
        return 2
    import torch
    from paper_1206_3768_amd import chfsi, sequence

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    spec = spec_of(args.workload)
    n = spec.n
    log(f"generating {spec.cycles} cycles, n={n}, nev={spec.nev}, nex={spec.nex}")
    t0 = time.perf_counter()
    seq = sequence.Sequence(spec, keep_host=False)
    log(f"inputs resident in HBM ({time.perf_counter() - t0:.1f} s); {seq.tuned_entries} tuned plans loaded")

    ref = seq.run_reference()
    bad = [r.cycle for r in ref if r.status != 0]
    if bad:
        log(f"reference pass failed on cycles {bad}")
        return 1
    log("reference pass: loops per cycle " + " ".join(str(r.stats["loops"]) for r in ref))
    corr = correlation_summary(seq, spec)

    prec = {v: k for k, v in PREC_NAMES.items()}[args.precision]
    timed, rows, wall, work = timed_sequence(seq, spec, args.steps, args.warmup, prec)
    for r in timed:
        if r.status != 0 or r.resid[:spec.nev].max() > 1e-10:
            log(f"timed solve of cycle {r.cycle} failed: status {r.status}, max resid {r.resid[:spec.nev].max():.2e}")
            return 1
    flops = sum(r.stats["filter_flops"] for r in timed)
    t_filter = sum(r.stats["t_filter"] for r in timed) * 1e-3
    value = flops / t_filter / 1e12
    rl = roofline(rows, args.workload, prec)
    log(f"timed {args.steps} warm solves: {wall / args.steps * 1e3:.2f} ms/solve, filter phase {value:.2f} TFLOP/s; "
        f"dominant kernel {rl['kernel']}: {rl['launches']} launches, {rl['achieved']:.2f} TFLOP/s "
        f"({rl['step_achieved']:.2f} with its reduction)")

    out = {
        "metric": "Filter TFLOP/s + time-to-solution @res<=1e-10, mixed/learned vs FP64",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PREC_DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload].replace("FP64 filter", f"{args.precision.upper()} filter"),
                   "n": n, "nev": spec.nev, "nex": spec.nex, "deg": spec.deg,
                   "cycles": spec.cycles},
        "time_to_solution_ms": {"median": round(statistics.median(r.wall_ms for r in timed), 3),
                                "per_cycle": {str(r.cycle): round(r.wall_ms, 3) for r in timed}},
        "roofline": rl,
        "phase_ms_per_solve": phase_summary(timed),
        "loops_per_cycle": {str(r.cycle): r.stats["loops"] for r in ref},
        "eigenvector_correlation": corr,
    }
    golden = golden_c3() if args.workload == "seq8192" else {}
    if golden:
        errs = {}
        for r in ref:
            if r.cycle in golden:
                _, errs[str(r.cycle)] = pair_errors(r.lam, golden[r.cycle])
        out["rel_eig_err_vs_oracle_fp64"] = errs

    if not args.no_extras:
        if args.workload == "seq8192":
            log("n=8192: degrees x precisions ...")
            out["c3_degrees_precisions"] = bench_c3_sweep(seq, spec, golden)
        A1 = None if args.no_cpu_baseline else chfsi.to_numpy(seq.A[1])
        seq.A.clear()
        torch.cuda.empty_cache()
        if args.workload != "seq2048":
            log("n=2048 sequence ...")
            out["seq2048"] = bench_seq2048(seq.h)
        log("LOBPCG GEN vs STD (n=2048, kappa 1e6) ...")
        out["lobpcg_gen_vs_std"] = bench_lobpcg(seq.h)
        log("k-point batch ...")
        out["batched_kpoints"] = bench_kpoints(seq.h)
        log("learned degree (n=4096, 20 cycles) ...")
        out["learned_degree"] = bench_learned_degree(seq.h)
    else:
        A1 = None if args.no_cpu_baseline else chfsi.to_numpy(seq.A[1])

    if not args.no_cpu_baseline:
        log("CPU baseline (oracle) on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(args.workload, spec, A1)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
