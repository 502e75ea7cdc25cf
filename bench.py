"""Benchmark: remainder-operator apply throughput (Gpts/s) and time to a 1e-8 solution.

Workload (N = 1 GPU): the ellipsoid with semi-axes (1, 0.8, 0.6) as a cube-sphere
with 1,536 patches of 10 x 10 Gauss-Legendre nodes (153,600 nodes),
a(x) = exp(0.3 x1 x2), right-hand side = 20 solid harmonics with N(0, 1)
coefficients (seed 1).  All inputs are synthetic and seeded.

One step = one application of the discretized operator of the integral equation
(source preparation, far field, near/self correction, combination) to one
density already resident in device memory, on the chosen path:
  mixed : FP32 interpolation-FMM far field (M2L on MFMA), FP64 near field
  fp64  : FP64 direct far field, FP64 near field
value = N * n_rhs * K / (wall time of K steps), in Gpts/s.

The same run also reports the other path's apply rate, the time to reach a
relative residual of 1e-8 on both paths (mixed: iterative refinement with FP64
residuals), the representation u = K[sigma] of the mixed solution, the roofline
of the dominant kernel (device time from HIP events on the library's stream),
and, in the CPU leg (skipped with --no-cpu, the only part that runs the oracle),
the oracle's checks of the apply, the solutions and the representation on
sampled rows and the oracle timed on the host cores on a bounded sample of rows.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "operator-apply Gpts/s @1e-8 rel err, mixed vs FP64; solves/s + p50/p99 latency"
# MI355X peaks: FP64 vector and FP32 MFMA as published; FP32 vector 157.3 needs packed FP32
# instructions, which this build does not emit (they are disabled at compile time), so FP32 VALU
# kernels are rated against the non-packed rate, 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
# = 78.6 TFLOP/s (the packed figure is reported beside it).
PEAK = {"fp64_valu": 78.6, "fp32_valu": 78.6, "fp32_valu_packed": 157.3, "fp32_mfma": 157.3, "hbm": 8000.0}

# HBM traffic per launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (KiB) on this workload
# (ellipsoid, 153,600 nodes, mixed path, 1 RHS; the M2L in the layout it runs in beside the
# second stream, as in the timed region), scaled by what the counters read for a plain
# 256 MiB device copy (FETCH_SIZE 131,088 KiB -> x2.0, WRITE_SIZE 262,144 KiB -> x1.0).  Each
# record is tied to its kernel's source text (the definition in its file, comments removed); a
# different text means a changed kernel and the traffic is reported as null.
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
TRAFFIC = {
    "fmm_m2l": {"src": "paper_2401_12501_amd/csrc/fmm.hip", "fn": "k_m2l", "sha": "d9444ab3830a46d6",
                "kib": [("k_m2l", 12065.9, 372009.3)]},
    "fmm_m2l_sum": {"src": "paper_2401_12501_amd/csrc/fmm.hip", "fn": "k_m2l_reduce", "sha": "13d98ce94106f035",
                    "kib": [("k_m2l_reduce", 166728.6, 7382.5)]},
    "fmm_p2p": {"src": "paper_2401_12501_amd/csrc/fmm.hip", "fn": "k_p2p", "sha": "eebd985a1eecaf25",
                "kib": [("k_p2p", 46446.4, 9602.3)]},
    "near": {"src": "paper_2401_12501_amd/csrc/nearapply.hip", "fn": "k_near_combine", "sha": "dbbc8c35cbb2ac42",
             "kib": [("k_near_combine", 281884.5, 1266.4)]},
}


def code_hash(path: str, fn: str | None = None) -> str:
    """Hash of source code with line comments, trailing spaces and blank lines removed (editing a
    comment does not count as changing the kernel): the whole file, or with ``fn`` the definition of
    that kernel (from its __global__ line to the closing brace in the first column)."""
    import hashlib
    import re
    with open(path, encoding="utf-8") as fh:
        src = fh.read().splitlines()
    if fn is not None:
        start = next(i for i, l in enumerate(src) if l.startswith("__global__") and f" {fn}(" in l)
        end = next(i for i in range(start, len(src)) if src[i] == "}")
        src = src[start:end + 1]
    lines = []
    for line in src:
        line = re.sub(r"//.*$", "", line).rstrip()
        if line:
            lines.append(line)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def traffic_bytes(phase: str, n_rhs: int, k: int):
    """Measured HBM bytes per launch of a phase, or None if not measured for this kernel/workload."""
    rec = TRAFFIC.get(phase)
    if rec is None or n_rhs != 1 or k != 16:
        return None
    if code_hash(os.path.join(ROOT, rec["src"]), rec.get("fn")) != rec["sha"]:
        return None
    return sum((f * FETCH_SCALE + w * WRITE_SCALE) * 1024.0 for _, f, w in rec["kib"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measure_representation(op, s_dev, N: int, n_rhs: int):
    """u = K[sigma] of the mixed solution: the FP64 direct log-kernel sum plus the parametrix near
    blocks D, minus its weighted mean.  The first call also builds the D blocks.  Returns (record,
    u on the host); the CPU leg checks u on sampled rows."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = op.represent(s_dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    u = op.represent(s_dev, out=u)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    u_h = u.cpu().numpy().T.copy()                # (N, n_rhs)
    rep = {"ms": round((t2 - t1) * 1e3, 3), "first_call_ms": round((t1 - t0) * 1e3, 3),
           "gpts_per_s": round(N * n_rhs / (t2 - t1) / 1e9, 5)}
    log(f"[bench] representation u = K[sigma]: {rep}")
    return rep, u_h


def algorithmic_work(phase: str, st, N: int, q: int, n_rhs: int, fmm_order: int, path: str = "mixed"):
    """(amount per launch, unit, bound, peak) of a phase's kernel(s)."""
    p3 = fmm_order ** 3
    if phase in ("direct64", "direct32"):
        flops = float(N) * N * (24 + 2 * n_rhs)          # per ordered pair: 24 + 2 per rhs
        return flops / 1e12, "TFLOP/s", "alu", PEAK["fp64_valu" if phase == "direct64" else "fp32_valu"]
    if phase == "near":
        # blocks C, sigma read and y written per rhs, near lists; the FP64 path also reads its far-field
        # partials (counted as one array), the mixed path's far field is added later by L2P
        vecs = 3 if path == "fp64" else 2
        byts = 8.0 * st.near_pairs * q * q + 8.0 * N * n_rhs * vecs + 8.0 * (N + 1) + 4.0 * st.near_pairs
        return byts / 1e9, "GB/s", "hbm", PEAK["hbm"]
    if phase == "fmm_m2l":
        return 2.0 * 9 * p3 * p3 * st.fmm_m2l_pairs * n_rhs / 1e12, "TFLOP/s", "mfma", PEAK["fp32_mfma"]
    if phase == "fmm_m2l_sum":
        byts = 4.0 * 9 * p3 * (st.fmm_m2l_pairs + st.fmm_boxes) * n_rhs + 4.0 * st.fmm_m2l_pairs
        return byts / 1e9, "GB/s", "hbm", PEAK["hbm"]
    if phase == "fmm_p2p":
        return float(st.fmm_p2p_pairs) * (24 + 2 * n_rhs) / 1e12, "TFLOP/s", "alu", PEAK["fp32_valu"]
    return None


def host_cpu():
    """Host core count and CPU model (the oracle's timing runs on the GPU machine's host)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(prob, factory, sigma, budget_s: float, checks: dict):
    """The CPU leg: the only part of this script that runs the oracle.  It checks the GPU results
    kept in `checks` on 1,024 sampled rows (apply error, solve residuals, representation) and then
    times the oracle's apply on batches of random rows: each batch's near/self correction blocks are
    built first (worker processes, timed separately as setup), then the rows are applied (smooth-rule
    sums over all sources in C on every host core, plus the block products).  Returns
    (cpu_baseline record, check results)."""
    from oracle import cfar
    from oracle.operator import OracleOperator
    from oracle.system import BlockPool, rows_from_blocks
    orc = OracleOperator.from_problem(prob)
    N = prob.n
    q2 = prob.surface.q ** 2
    workers = max(1, min(8, os.cpu_count() or 1))   # few processes: the box limits processes that map the GPU runtime
    host = host_cpu()
    threads = cfar.threads()
    res = {}
    with BlockPool(factory, ROOT, workers) as pool:
        rng = np.random.default_rng(5)
        patches = rng.choice(N // q2, 128, replace=False)
        tg = np.unique(np.concatenate([[0, N - 1], patches * q2, patches * q2 + q2 - 1,
                                       rng.choice(N, 1024 - 258, replace=False)]))
        blocks = pool.blocks(tg, ("R",), chunk=16)
        ref = rows_from_blocks(orc, blocks, tg, sigma)
        scale = np.abs(ref).max()
        res["apply_rel_err_vs_oracle"] = {k: float(np.abs(v[tg] - ref).max() / scale) for k, v in checks["y"].items()}
        res["rows_checked"] = int(len(tg))
        log(f"[bench] {len(tg)} sampled rows, apply error vs oracle: {res['apply_rel_err_vs_oracle']}")
        # residual of each returned density in the oracle's discrete system
        f_rows = prob.f[tg] - (prob.f * orc.w[:, None]).sum(0) / orc.w.sum()   # mean-zero data at the rows
        res["solve_rows"] = {}
        for path, s_h in checks["sigma"].items():
            r_rows = f_rows - rows_from_blocks(orc, blocks, tg, s_h)
            res["solve_rows"][path] = float(np.abs(r_rows).max() / np.abs(f_rows).max())
        log(f"[bench] sampled-row relative residual of the solves: {res['solve_rows']}")
        # representation: the GPU rows differ from the oracle's rows before the mean is removed by one
        # constant per right-hand side (the weighted mean), so the spread of the differences is the
        # error, relative to the spread of the oracle rows
        if checks.get("u") is not None:
            u_h, s_h = checks["u"], checks["sigma"]["mixed"]
            ref_u = rows_from_blocks(orc, pool.blocks(tg, ("K",), chunk=16), tg, s_h, "K")
            d = u_h[tg] - ref_u
            res["representation"] = {
                "rows_rel_err_vs_oracle": float(np.abs(d - d.mean(0)).max() / np.abs(ref_u - ref_u.mean(0)).max()),
                "weighted_mean_rel": float(np.abs(orc.w @ u_h).max() / orc.w.sum() / np.abs(u_h).max())}
            log(f"[bench] representation vs oracle rows: {res['representation']}")
        rng = np.random.default_rng(7)
        n_rows, t_apply, t_setup = 0, 0.0, 0.0
        t_start = time.perf_counter()
        while time.perf_counter() - t_start < budget_s:
            batch = rng.choice(N, min(N, 1024), replace=False)
            t0 = time.perf_counter()
            bl = pool.blocks(batch, ("R",), chunk=16)
            t1 = time.perf_counter()
            rows_from_blocks(orc, bl, batch, sigma)
            t2 = time.perf_counter()
            n_rows += len(batch)
            t_setup += t1 - t0
            t_apply += t2 - t1
    rec = {"value": n_rows / t_apply / 1e9, "unit": "Gpts/s", "cores": threads, "kind": "oracle",
           "sample": f"{n_rows} random target rows of the {N}-node apply in batches of 1,024: smooth-rule sums over "
                     f"all {N} sources (C, FP64, {threads} OpenMP threads) plus the rows' near/self block products "
                     f"(numpy); the blocks themselves built beforehand on {workers} processes, "
                     f"{t_setup / n_rows * 1e3:.2f} ms/row wall, timed separately",
           "setup_ms_per_row": round(t_setup / n_rows * 1e3, 3), "host": host}
    log(f"[bench] cpu baseline: {rec}")
    return rec, res


def _percentiles(x):
    x = np.asarray(x, dtype=np.float64)
    return round(float(np.percentile(x, 50)), 4), round(float(np.percentile(x, 99)), 4)


def serving(n_req: int, slots: int, loads, budget_bytes: int, n_cal: int = 64):
    """Serving workload: requests from the sphere / random-axis ellipsoid / torus families with
    2e3..2e5 nodes (log-uniform), mixed path, admitted by slots and by the HBM budget of their
    context.  A separate closed-loop run of n_cal requests (another seed) measures the saturated
    rate mu; then the n_req requests arrive as a Poisson stream at each load * mu.  Latency =
    submit -> result ready (server clock), split into queue wait and service."""
    from paper_2401_12501_amd import pmx
    from paper_2401_12501_amd.inputs import serving_requests
    log(f"[serve] generating {n_req} + {n_cal} requests ...")
    reqs = [p for _, p in serving_requests(n_req, seed=3)]
    cal = [p for _, p in serving_requests(n_cal, seed=4)]
    o = pmx.pmx_default_options()
    o.precision = pmx.PMX_PREC_MIXED_FMM
    ctx = pmx.Context(0, hbm_budget_bytes=budget_bytes)

    def run(problems, arrivals):
        sv = pmx.Server(ctx, o, max_active=slots)
        out, done = set(), []
        t0 = time.perf_counter()
        nxt = 0
        while nxt < len(problems) or out:
            now = time.perf_counter() - t0
            while nxt < len(problems) and (arrivals is None or arrivals[nxt] <= now):
                p = problems[nxt]
                out.add(sv.submit(p.surface, p.a, p.grad_a, p.f[:, 0]))
                nxt += 1
            sv.step()
            for t in list(out):
                r = sv.poll(t)
                if r is not None:
                    out.remove(t)
                    done.append((r[0], r[4].copy()))
            time.sleep(0.0005)
        wall = time.perf_counter() - t0
        st = sv.stats()
        sv.close()
        bad = [c for c, _ in done if c != pmx.PMX_OK]
        if bad:
            raise RuntimeError(f"serving: {len(bad)} requests did not return PMX_OK: {sorted(set(bad))}")
        return wall, np.array([t for _, t in done]), st

    wall, _, _ = run(cal, None)
    mu = n_cal / wall
    log(f"[serve] saturated rate {mu:.2f} solves/s ({n_cal} requests, closed loop)")
    per_load = []
    for load in loads:
        lam = load * mu
        arrivals = np.cumsum(np.random.default_rng(33).exponential(1.0 / lam, n_req))
        wall, times, st = run(reqs, arrivals)
        p50, p99 = _percentiles(times[:, 2])
        q50, q99 = _percentiles(times[:, 0])
        s50, s99 = _percentiles(times[:, 1])
        rec = {"load": load, "arrival_rate_per_s": round(lam, 3), "solves_per_s": round(n_req / wall, 3),
               "p50_latency_s": p50, "p99_latency_s": p99, "queue_p50_s": q50, "queue_p99_s": q99,
               "service_p50_s": s50, "service_p99_s": s99, "held_for_memory": st["held_for_memory"],
               "peak_reserved_gib": round(st["peak_reserved_bytes"] / 2 ** 30, 3),
               "mean_batch": round(st["applies"] / max(st["batches"], 1), 2), "max_batch": st["max_batch"],
               "shared_launches": st["batches"], "applies": st["applies"]}
        log(f"[serve] {rec}")
        per_load.append(rec)
    main = next((r for r in per_load if abs(r["load"] - 0.7) < 1e-9), per_load[0])
    return {"requests": n_req, "ok": n_req, "calibration_requests": n_cal, "slots": slots,
            "hbm_budget_bytes": budget_bytes, "saturated_solves_per_s": round(mu, 3),
            "p50_latency_s": main["p50_latency_s"], "p99_latency_s": main["p99_latency_s"],
            "at_load": main["load"], "loads": per_load,
            "nodes_min_max": [int(min(p.n for p in reqs)), int(max(p.n for p in reqs))]}


# Operation count per ordered pair of the FP64 direct far field with c < 0 (the kernel's evaluation,
# each add, mul, division, reciprocal square root, logarithm or exponential 1 flop, an FMA 2): the
# geometry and the factored remainder 44, plus K0 and K1 of z = kappa r either by four degree-12
# Horner polynomials of the ascending series for z <= 2 (111, the "series" entry) or by the power
# forms of two degree-22 interpolants in 4/z - 1 (Horner's rule) times exp(-z) / sqrt(z) for z > 2
# (95, the "chebyshev" entry).
C_PAIR_FLOPS = {"pair": 44, "series": 111, "chebyshev": 95}
# The same count for c > 0 (complex kernel, one complex density): geometry, the factored remainder's
# real and imaginary parts and the complex multiply-add 54, plus J0, J1, Y0, Y1 of z = k r either by
# four degree-16 polynomials in z^2 (Horner's rule) and a logarithm for z <= 8 (142, the "series"
# entry) or by four degree-14 polynomials in 8 / z, a sine, a cosine and the envelope
# sqrt(2 / (pi z)) for z > 8 (138, the "chebyshev" entry).
C_PAIR_FLOPS_POS = {"pair": 54, "series": 142, "chebyshev": 138}


def c_pair_flops(prob, n_sample: int = 200_000, seed: int = 7) -> tuple[float, float]:
    """(flops per pair, fraction of pairs on the first branch: z <= 2 for c < 0, z <= 8 for c > 0)
    from seeded sample pairs."""
    rng = np.random.default_rng(seed)
    x = prob.surface.x
    i = rng.integers(prob.n, size=n_sample)
    j = rng.integers(prob.n, size=n_sample)
    keep = i != j
    pos = bool(prob.c[0] > 0)
    kap = np.sqrt(np.abs(prob.c[j[keep]]) / prob.a[j[keep]])
    z = kap * np.linalg.norm(x[i[keep]] - x[j[keep]], axis=1)
    f = float(np.mean(z <= (8.0 if pos else 2.0)))
    cnt = C_PAIR_FLOPS_POS if pos else C_PAIR_FLOPS
    return (cnt["pair"] + f * cnt["series"] + (1 - f) * cnt["chebyshev"], f)


def helmholtz_bench(args):
    """The c != 0 path with advection (variable a and c of Section 7.4's kind, a non-tangent advection
    field) on the 153,600-node ellipsoid surface: FP64 applies, a solve to 1e-8, the roofline of the
    direct sum, and (CPU leg) oracle rows.  Workload helmholtz: c = -4 - exp(x1/2) < 0; helmholtz_pos:
    c = 2 (1 + 0.2 x2) > 0, the complex Helmholtz-type kernel (one complex density, timed in the
    library's layout of two real columns)."""
    import torch
    from paper_2401_12501_amd import pmx
    from paper_2401_12501_amd.inputs import helmholtz_ellipsoid_problem, random_density
    pos = args.workload == "helmholtz_pos"
    prob = helmholtz_ellipsoid_problem(k=args.k, q=10, swirl=True, positive=pos)
    N = prob.n
    tag = "c > 0" if pos else "c < 0"
    log(f"[bench] workload {prob.name} N={N} path=fp64 ({tag} with advection)")
    ctx = pmx.Context(0)
    surf = pmx.Surface.from_inputs(ctx, prob.surface)
    t0 = time.perf_counter()
    op = pmx.Operator(surf, prob.a, prob.grad_a, c=prob.c, b=prob.b)
    t_setup = time.perf_counter() - t0
    sig_h = random_density(N, 1, seed=3)
    if pos:
        sig_h = sig_h + 1j * random_density(N, 1, seed=4)
        sig = torch.tensor(np.ascontiguousarray(np.stack([sig_h.real.T, sig_h.imag.T], axis=1)), device="cuda:0")
    else:
        sig = torch.tensor(np.ascontiguousarray(sig_h.T), device="cuda:0")
    y = torch.empty_like(sig)
    P64 = pmx.PMX_PREC_FP64_DIRECT
    run = (lambda: op.apply_planar(sig, P64, out=y)) if pos else (lambda: op.apply(sig, P64, out=y))
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    op.profile_read()
    op.profile(True)
    ts = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - ts) / args.steps
    op.profile(False)
    phases = op.profile_read()
    log(f"[bench] fp64 ({tag}, advection): {step_s * 1e3:.3f} ms/apply; phases " +
        ", ".join(f"{k} {v[0] / max(v[1], 1):.3f} ms" for k, v in phases.items() if v[1]))
    fpp, f_series = c_pair_flops(prob)
    d_ms = phases["direct64"][0] / max(phases["direct64"][1], 1)
    achieved = N * (N - 1.0) * fpp / (d_ms * 1e-3) / 1e12
    near_ms = phases["near"][0] / max(phases["near"][1], 1)
    near_bytes = op.stats().near_pairs * 8.0 * 100 * (2 if pos else 1) + 24.0 * N * (2 if pos else 1)
    o = pmx.pmx_default_options()
    o.gmres_tol = 1e-8
    ts = time.perf_counter()
    s_sol, _, info = op.solve(np.ascontiguousarray(prob.f.T), o)
    t_solve = time.perf_counter() - ts
    log(f"[bench] solve to 1e-8: {t_solve:.3f} s, {info[0].iters_total} iterations, residual {info[0].rel_residual:.2e}")
    y_h = y.cpu().numpy()
    y_h = (y_h[:, 0] + 1j * y_h[:, 1]).T.copy() if pos else y_h.T.copy()
    err = None
    if not args.no_cpu:
        from oracle.operator import OracleOperator
        from oracle.system import blocks_parallel
        orc = OracleOperator.from_problem(prob)
        tg = np.sort(np.random.default_rng(11).choice(N, size=48, replace=False))
        blocks = blocks_parallel(("paper_2401_12501_amd.inputs", "helmholtz_ellipsoid_problem",
                                  {"k": args.k, "q": 10, "swirl": True, "positive": pos}), ROOT, tg, kernels=("R",),
                                 workers=min(8, os.cpu_count() or 1))
        ref = orc.apply_rows(tg, sig_h, blocks)
        err = float(np.abs(y_h[tg] - ref).max() / np.abs(ref).max())
        log(f"[bench] 48 sampled rows vs oracle: {err:.2e}")
    cdesc = "c=2(1+0.2x2)" if pos else "c=-4-exp(x1/2)"
    out = {"metric": f"{'c>0' if pos else 'c<0'} + advection operator-apply Gpts/s (FP64 direct far field)",
           "value": round(N / step_s / 1e9, 5),
           "unit": "Gpts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(step_s * 1e3, 3), "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": (f"ellipsoid (1, 0.8, 0.6), {prob.surface.n_patches} patches x 10x10, N={N}, "
                                   f"a=2+x3, {cdesc}, b=(0.6-x2, x1+0.4x3, 0.5x1x2)"), "path": "fp64"},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK["fp64_valu"], "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK["fp64_valu"], 4), "traffic": None,
                        "kernel": "k_direct64_cz" if pos else "k_direct64_c",
                        "avg_ms": round(d_ms, 4), "flops_per_pair": round(fpp, 1), "series_fraction": round(f_series, 4)},
           "near": {"ms": round(near_ms, 4), "achieved": round(near_bytes / (near_ms * 1e-3) / 1e9, 1), "unit": "GB/s",
                    "frac": round(near_bytes / (near_ms * 1e-3) / 1e9 / PEAK["hbm"], 4)},
           "setup_s": round(t_setup, 3),
           "solve_to_1e-8": {"seconds": round(t_solve, 3), "iters": info[0].iters_total,
                             "rel_residual": info[0].rel_residual},
           "apply_rel_err_vs_oracle": err}
    print(json.dumps(out), flush=True)


# Algorithmic FP64 flops per (target, fine point) pair of the edge-operator kernels, one density:
# the difference and r^2 (9); K: the logarithm (counted as 1) and its scale (2); N: the reciprocal,
# nu.r (5), the logarithm term (3) and the combination (3); R: the reciprocal, n'.r and h.r (10) and
# Phi (4); T: R's 15 plus nu.r, n'.nu, h.nu (15), the derivative's bracket (10), its scale (3) and the
# combination with Phi (2); and 2 for the accumulation.
EDGE_PAIR_FLOPS = {"K": 13, "N": 23, "R": 26, "T": 56}


def edge_bench(args):
    """Open surfaces: the edge operators K, N, R, T (Section 5) applied from the boundary circles of
    the wavy-torus band 4 pi / 3 < u < 2 pi (17 x 18 patches of 8 x 8 nodes, 19,584 targets) with 200
    samples per circle oversampled 64 times (25,600 fine points, Section 7.5's setting), a =
    exp(0.3 x1 x2), mu = exp(x1).  Reports each kind's apply time, the roofline of the T pair kernel
    (device time from HIP events on the launch stream), Section 7.5's error against oversampling, and
    (CPU leg) the oracle's rows and its rate on a bounded sample."""
    import torch
    from paper_2401_12501_amd import pmx
    from paper_2401_12501_amd.inputs import wavy_torus_piece_problem
    m_over = 64
    prob = wavy_torus_piece_problem(n_u=17, n_v=18, q=8, n_edge=200, variable_a=True, n_rhs=1)
    edge = prob.meta["edge"]
    N = prob.n
    ctx = pmx.Context(0)
    surf = pmx.Surface.from_inputs(ctx, prob.surface)
    op = pmx.Operator(surf, prob.a, prob.grad_a)
    t0 = time.perf_counter()
    E = pmx.Edge.from_inputs(ctx, edge, m_over)
    t_edge = time.perf_counter() - t0
    Mf = E.n_fine
    log(f"[bench] workload {prob.name} N={N}, {edge.m} samples, oversampling {m_over}: {Mf} fine points "
        f"(edge setup {t_edge * 1e3:.1f} ms)")
    mu = torch.tensor(np.ascontiguousarray(edge.mu.T), device="cuda:0")
    y = torch.empty((1, N), dtype=torch.float64, device="cuda:0")
    res = {}
    for kind in ("K", "N", "R", "T"):
        for _ in range(args.warmup):
            E.apply(op, kind, mu, out=y)
        torch.cuda.synchronize()
        op.profile_read()
        op.profile(True)
        ts = time.perf_counter()
        for _ in range(args.steps):
            E.apply(op, kind, mu, out=y)
        torch.cuda.synchronize()
        step_s = (time.perf_counter() - ts) / args.steps
        op.profile(False)
        ph = op.profile_read()["edge"]
        pair_ms = ph[0] / max(ph[1], 1)
        tf = N * Mf * EDGE_PAIR_FLOPS[kind] / (pair_ms * 1e-3) / 1e12
        res[kind] = {"ms": round(step_s * 1e3, 4), "pair_kernel_ms": round(pair_ms, 4), "tflops": round(tf, 3),
                     "frac": round(tf / PEAK["fp64_valu"], 4)}
        log(f"[bench] edge {kind}: {step_s * 1e3:.4f} ms/apply, pair kernel {pair_ms:.4f} ms, "
            f"{tf:.2f} TFLOP/s ({tf / PEAK['fp64_valu']:.3f} of FP64)")
    # K'_gamma: targets on the curves (the samples), trapezoid rule on the samples
    yk = torch.empty_like(mu)
    for _ in range(args.warmup):
        E.kprime(mu, out=yk)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        E.kprime(mu, out=yk)
    torch.cuda.synchronize()
    kp_ms = (time.perf_counter() - ts) / args.steps * 1e3
    res["Kprime_gamma"] = {"ms": round(kp_ms, 4), "pairs": edge.m * edge.m}
    log(f"[bench] edge K'_gamma at the {edge.m} samples: {kp_ms:.4f} ms/apply")
    # Section 7.5: error of R and T against the finest rule as the oversampling grows, on this surface
    # and on one refined twice across the band (its nodes twice as close to the curves)
    study = {}
    fine_prob = wavy_torus_piece_problem(n_u=34, n_v=18, q=8, n_edge=200, variable_a=True, n_rhs=1)
    fine_op = pmx.Operator(pmx.Surface.from_inputs(ctx, fine_prob.surface), fine_prob.a, fine_prob.grad_a)
    for label, o in (("17x18", op), ("34x18", fine_op)):
        for kind in ("R", "T"):
            ref = pmx.Edge.from_inputs(ctx, edge, 128).apply(o, kind, mu).cpu().numpy()
            errs = {}
            for m in (1, 2, 4, 8, 16, 32, 64):
                v = pmx.Edge.from_inputs(ctx, edge, m).apply(o, kind, mu).cpu().numpy()
                errs[m] = float(np.abs(v - ref).max() / np.abs(ref).max())
            study[f"{kind}_{label}"] = {str(k): float(f"{v:.3g}") for k, v in errs.items()}
            log(f"[bench] edge {kind} on {label} patches, error vs oversampling (max over nodes, against m = 128): " +
                ", ".join(f"m={k} {v:.2e}" for k, v in errs.items()))
    E.apply(op, "T", mu, out=y)
    y_t = y.cpu().numpy()[0]
    cpu, err = None, None
    if not args.no_cpu:
        from oracle.edge import edge_apply, targets_of
        from oracle.operator import OracleOperator
        tgt = targets_of(OracleOperator.from_problem(prob))
        tg = np.sort(np.random.default_rng(13).choice(N, size=48, replace=False))
        ts = time.perf_counter()
        ref = edge_apply("T", tgt, edge, edge.mu, m_over, targets=tg)[:, 0]
        t_cpu = time.perf_counter() - ts
        err = float(np.abs(y_t[tg] - ref).max() / np.abs(ref).max())
        cpu = {"value": round(len(tg) * Mf / t_cpu / 1e9, 6), "unit": "Gpairs/s", "cores": 1, "kind": "oracle",
               "sample": f"T_gamma at {len(tg)} seeded targets x {Mf} fine points (NumPy, one thread), "
                         f"{t_cpu:.2f} s", **host_cpu()}
        log(f"[bench] oracle T rows: {len(tg)} targets in {t_cpu:.2f} s; GPU vs oracle {err:.2e} of the column")
    t = res["T"]
    out = {"metric": "open-surface edge operators: target-source pairs/s (T_gamma, FP64, trapezoid x64)",
           "value": round(N * Mf / (t["ms"] * 1e-3) / 1e9, 3), "unit": "Gpairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": t["ms"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": (f"wavy torus band 4pi/3 < u < 2pi, 17 x 18 patches x 8x8, N={N}; 2 boundary "
                                   f"circles x 200 samples, oversampling {m_over} ({Mf} fine points); "
                                   f"a=exp(0.3 x1 x2), mu=exp(x1)"), "kinds": res},
           "roofline": {"bound": "alu", "achieved": t["tflops"], "peak": PEAK["fp64_valu"], "unit": "TFLOP/s",
                        "frac": t["frac"], "traffic": None, "kernel": "k_edge_pairs<3,1>",
                        "avg_ms": t["pair_kernel_ms"], "flops_per_pair": EDGE_PAIR_FLOPS["T"]},
           "oversampling_study": study, "edge_setup_ms": round(t_edge * 1e3, 2),
           "apply_rel_err_vs_oracle": err, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--path", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--n-rhs", type=int, default=1)
    ap.add_argument("--workload", choices=["ellipsoid", "star", "torus", "helmholtz", "helmholtz_pos", "edge"],
                    default="ellipsoid",
                    help="ellipsoid: 153,600 nodes, 1 RHS (default); star: 525,696 nodes, 1 RHS; "
                         "torus: wobbly torus, 2,097,152 nodes, 16 RHS; helmholtz: the c < 0 path with advection "
                         "on the ellipsoid's surface (FP64); helmholtz_pos: the same with c > 0 (complex kernel); "
                         "edge: the open-surface edge operators on the wavy-torus band")
    ap.add_argument("--k", type=int, default=16, help="ellipsoid: cube-sphere patches per face edge (16: 153,600 nodes)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--fmm-leaf", type=int, default=0, help="FMM leaf occupancy target (0: library default)")
    ap.add_argument("--fmm-order", type=int, default=0, help="FMM interpolation order (0: library default)")
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="mixed solve: inner GMRES tolerance (0: library default)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="mixed applies on one stream (no near/P2P overlap with the M2L chain)")
    ap.add_argument("--serve", type=int, default=256,
                    help="serving requests per load (0: skip); a separate closed-loop run calibrates the saturated rate")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-loads", default="0.5,0.7,0.9",
                    help="serving: Poisson arrival rates as fractions of the measured saturated rate")
    ap.add_argument("--serve-budget-mib", type=int, default=2048,
                    help="serving: HBM budget of the server's context (admission by memory)")
    ap.add_argument("--calib-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (a known-size kernel for traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): sharding the apply over several GPUs "
              f"(by target ownership along the octree's Morton order) is designed but not implemented.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload in ("helmholtz", "helmholtz_pos"):
        helmholtz_bench(args)
        return
    if args.workload == "edge":
        edge_bench(args)
        return
    import torch
    from paper_2401_12501_amd import pmx
    from paper_2401_12501_amd.inputs import ellipsoid_problem, star_problem, wobbly_torus_problem, random_density

    if args.calib_mb:
        src = torch.ones(args.calib_mb * 2 ** 18, device="cuda:0", dtype=torch.float32)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    INPUTS = "paper_2401_12501_amd.inputs"
    if args.workload == "ellipsoid":
        prob = ellipsoid_problem(k=args.k, q=10, n_rhs=args.n_rhs)
        factory = (INPUTS, "ellipsoid_problem", {"k": args.k, "q": 10, "n_rhs": args.n_rhs})
        n_rhs = args.n_rhs
        desc = (f"ellipsoid (1, 0.8, 0.6), {prob.surface.n_patches} patches x 10x10 Gauss-Legendre nodes, "
                f"N={prob.n}, a=exp(0.3 x1 x2)")
    elif args.workload == "star":
        prob = star_problem()
        factory = (INPUTS, "star_problem", {})
        n_rhs = 1
        desc = (f"star r = 1 + 0.25 (8 real spherical harmonics, l <= 4), {prob.surface.n_patches} patches x 8x8 "
                f"Gauss-Legendre nodes, N={prob.n}, a = 2^tanh(smooth seed field)")
    else:
        prob = wobbly_torus_problem()
        factory = (INPUTS, "wobbly_torus_problem", {})
        n_rhs = prob.f.shape[1]
        desc = (f"wobbly torus R=1, r=0.4(1+0.2 cos 5t sin 3p), {prob.surface.n_patches} patches x 8x8 "
                f"Gauss-Legendre nodes, N={prob.n}, a=1+0.5 tanh(sin 3 x1), {n_rhs} right-hand sides")
    N = prob.n
    log(f"[bench] workload {prob.name} N={N} n_rhs={n_rhs} path={args.path}")
    ctx = pmx.Context(0)
    surf = pmx.Surface.from_inputs(ctx, prob.surface)
    t0 = time.perf_counter()
    opts = pmx.pmx_default_options()
    if args.fmm_leaf:
        opts.fmm_leaf = args.fmm_leaf
    if args.fmm_order:
        opts.fmm_order = args.fmm_order
    if args.no_overlap:
        opts.overlap = 0
    op = pmx.Operator(surf, prob.a, prob.grad_a, opts)
    t_setup = time.perf_counter() - t0
    prec = {"mixed": pmx.PMX_PREC_MIXED_FMM, "fp64": pmx.PMX_PREC_FP64_DIRECT,
            "fp32_direct": pmx.PMX_PREC_FP32_DIRECT}
    other = "fp64" if args.path == "mixed" else "mixed"
    sig_h = random_density(N, n_rhs, seed=3)
    sig = torch.tensor(np.ascontiguousarray(sig_h.T), device="cuda:0")
    y = torch.empty_like(sig)
    t0 = time.perf_counter()
    op.apply(sig, prec[args.path], out=y)          # first call builds the FMM tree on the mixed path
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    log(f"[bench] setup {t_setup:.2f} s, first apply {t_first:.3f} s")

    def timed(path, steps, warmup, profile):
        for _ in range(warmup):
            op.apply(sig, prec[path], out=y)
        torch.cuda.synchronize()
        op.profile_read()
        op.profile(profile)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(steps):
            op.apply(sig, prec[path], out=y)
        torch.cuda.synchronize()
        te = time.perf_counter()
        op.profile(False)
        return (te - ts) / steps, op.profile_read()

    step_s, phases = timed(args.path, args.steps, args.warmup, True)
    log(f"[bench] {args.path}: {step_s * 1e3:.3f} ms/apply; phases " +
        ", ".join(f"{k} {v[0] / max(v[1], 1):.3f} ms" for k, v in phases.items() if v[1]))
    y_main = y.cpu().numpy().T.copy()
    try:
        other_s, other_phases = timed(other, max(3, args.steps // 4), 1, True)
        y_other = y.cpu().numpy().T.copy()
        log(f"[bench] {other}: {other_s * 1e3:.3f} ms/apply")
    except pmx.PmxError as e:
        log(f"[bench] {other} path unavailable: {e}")
        other_s, y_other, other_phases = None, None, {}
    # the optional FP32 direct far field (same pair kernel as the FP64 path, in FP32)
    try:
        d32_s, _ = timed("fp32_direct", max(3, args.steps // 4), 1, False)
        y_d32 = y.cpu().numpy().T.copy()
        d32_tf = float(N) * (N - 1) * (24 + 2 * n_rhs) / d32_s / 1e12
        fp32_direct = {"ms_per_apply": round(d32_s * 1e3, 4), "gpts_per_s": round(N * n_rhs / d32_s / 1e9, 4),
                       "achieved": round(d32_tf, 3), "unit": "TFLOP/s", "peak": PEAK["fp32_valu"],
                       "frac": round(d32_tf / PEAK["fp32_valu"], 4), "peak_packed": PEAK["fp32_valu_packed"],
                       "note": "pair flops over the whole apply time (the FP64 near correction included)"}
        log(f"[bench] fp32 direct: {fp32_direct}")
    except pmx.PmxError as e:
        log(f"[bench] fp32 direct path unavailable: {e}")
        fp32_direct, y_d32 = None, None

    st = op.stats()
    # the same mixed apply with every kernel on one stream (operator option overlap = 0): the
    # kernels' own durations without the second stream sharing the CUs, and the overlap's gain
    one_stream = None
    if args.path == "mixed" and not args.no_overlap:
        opts1 = pmx.pmx_default_options()
        for fld in ("fmm_order", "fmm_leaf"):
            setattr(opts1, fld, getattr(opts, fld))
        opts1.overlap = 0
        op1 = pmx.Operator(surf, prob.a, prob.grad_a, opts1)
        y1 = torch.empty_like(sig)
        for _ in range(args.warmup + 1):
            op1.apply(sig, prec["mixed"], out=y1)
        torch.cuda.synchronize()
        op1.profile_read()
        op1.profile(True)
        ts1 = time.perf_counter()
        for _ in range(args.steps):
            op1.apply(sig, prec["mixed"], out=y1)
        torch.cuda.synchronize()
        one_s = (time.perf_counter() - ts1) / args.steps
        op1.profile(False)
        ph1 = op1.profile_read()
        same = bool(np.array_equal(y1.cpu().numpy().T, y_main))
        one_stream = {"ms_per_apply": round(one_s * 1e3, 4), "overlap_speedup": round(one_s / step_s, 3),
                      "bitwise_equal": same, "kernels": []}
        for name, (ms, cnt) in ph1.items():
            w = algorithmic_work(name, st, N, prob.surface.q, n_rhs, op.opts.fmm_order, "mixed") if cnt else None
            if w:
                amount, unit, bound, peak = w
                t = ms / 1e3 / args.steps
                one_stream["kernels"].append({"kernel": name, "ms": round(t * 1e3, 4), "achieved": round(amount / t, 3),
                                              "unit": unit, "frac": round(amount / t / peak, 4)})
        log(f"[bench] mixed on one stream: {one_s * 1e3:.3f} ms/apply (two streams {step_s * 1e3:.3f}), "
            f"identical output {same}; " + ", ".join(f"{k['kernel']} {k['ms']:.3f} ms ({k['frac']:.3f})"
                                                    for k in one_stream["kernels"]))
        del op1

    # dominant kernel of the timed path: the longest one alone (one-stream run) when the second
    # stream shares the CUs, since overlapped durations also count waiting for the other stream;
    # its rate below still comes from the timed (two-stream) region
    cands = [(k, v) for k, v in phases.items() if v[1] and k != "prep"]
    if one_stream and one_stream["kernels"]:
        alone = max(one_stream["kernels"], key=lambda k: k["ms"])["kernel"]
        dom = next(((k, v) for k, v in cands if k == alone), max(cands, key=lambda kv: kv[1][0]))
    else:
        dom = max(cands, key=lambda kv: kv[1][0])
    work = algorithmic_work(dom[0], st, N, prob.surface.q, n_rhs, op.opts.fmm_order, args.path)
    roof = None
    if work:
        amount, unit, bound, peak = work
        avg_s = dom[1][0] / dom[1][1] / 1e3
        launches_per_step = dom[1][1] / args.steps
        achieved = amount / (avg_s * launches_per_step)
        tb = traffic_bytes(dom[0], n_rhs, args.k if args.workload == "ellipsoid" else -1)
        roof = {"bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": (round(tb / 1e9, 4) if tb else None),
                "traffic_unit": "GB per launch", "kernel": dom[0],
                "avg_ms": round(avg_s * launches_per_step * 1e3, 4)}

    # every kernel with a defined algorithmic work, both paths
    kernels = []
    for path, ph, steps in ((args.path, phases, args.steps), (other, other_phases, max(3, args.steps // 4))):
        for name, (ms, cnt) in ph.items():
            w = algorithmic_work(name, st, N, prob.surface.q, n_rhs, op.opts.fmm_order, path) if cnt else None
            if w:
                amount, unit, bound, peak = w
                t = ms / 1e3 / steps
                kernels.append({"path": path, "kernel": name, "bound": bound, "ms": round(t * 1e3, 4),
                                "achieved": round(amount / t, 3), "peak": peak, "unit": unit,
                                "frac": round(amount / t / peak, 4)})

    # PCIe-inclusive rate: the same apply with host arrays (staged through device buffers)
    sig_host = np.ascontiguousarray(sig_h.T)
    op.apply(sig_host, prec[args.path])
    th0 = time.perf_counter()
    for _ in range(5):
        op.apply(sig_host, prec[args.path])
    host_s = (time.perf_counter() - th0) / 5

    # GPU results that the CPU leg checks against the oracle on sampled rows
    checks = {"y": {args.path: y_main, other: y_other} if y_other is not None else {args.path: y_main},
              "sigma": {}, "u": None}
    if y_d32 is not None:
        checks["y"]["fp32_direct"] = y_d32
    solve = {}
    representation = None
    if not args.no_solve:
        f = torch.tensor(np.ascontiguousarray(prob.f.T), device="cuda:0")
        for path in ("mixed", "fp64"):
            if path == "fp64" and N * n_rhs > 4_000_000:
                log(f"[bench] solve fp64 skipped at N*n_rhs = {N * n_rhs} (one FP64 apply is timed above)")
                continue
            o = pmx.pmx_default_options()
            o.precision = prec[path]
            o.gmres_tol = 1e-8
            o.ir_tol = 1e-8
            if args.inner_tol:
                o.inner_tol = args.inner_tol
            torch.cuda.synchronize()
            ts = time.perf_counter()
            try:
                s_out, _, info = op.solve(f, o)
            except pmx.PmxError as e:
                log(f"[bench] solve {path} unavailable: {e}")
                continue
            torch.cuda.synchronize()
            dt = time.perf_counter() - ts
            checks["sigma"][path] = s_out.T if isinstance(s_out, np.ndarray) else s_out.cpu().numpy().T.copy()
            if path == "mixed":
                s_mixed = s_out
            solve[path] = {"seconds": round(dt, 4), "iters": max(i.iters_total for i in info),
                           "ir_steps": max(i.ir_steps for i in info),
                           "applies_fp64": info[0].applies_fp64, "applies_fp32": info[0].applies_low,
                           "rel_residual": max(i.rel_residual for i in info),
                           "oracle_rows_rel_residual": None}
            log(f"[bench] solve {path}: {dt:.3f} s {solve[path]}")
        if "mixed" in solve:
            solve["solves_per_s_mixed"] = round(1.0 / solve["mixed"]["seconds"], 3)
            representation, checks["u"] = measure_representation(op, s_mixed, N, n_rhs)

    value = N * n_rhs / step_s / 1e9
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "Gpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(step_s * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.path == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": desc, "n_rhs": n_rhs,
                   "path": args.path, "fmm_order": op.opts.fmm_order, "fmm_leaf": op.opts.fmm_leaf},
        "roofline": roof,
        "other_path": ({"path": other, "gpts_per_s": round(N * n_rhs / other_s / 1e9, 4),
                        "ms_per_apply": round(other_s * 1e3, 4)} if other_s else None),
        "one_stream": one_stream,
        "fp32_direct": fp32_direct,
        "apply_rel_err_vs_oracle": None,
        "solve_to_1e-8": solve,
        "representation": representation,
        "setup_s": round(t_setup, 3),
        "kernels": kernels,
        "host_buffers_gpts_per_s": round(N * n_rhs / host_s / 1e9, 4),
        "phases_ms": {k: round(v[0] / v[1], 4) for k, v in phases.items() if v[1]},
        "fmm": {"levels": st.fmm_levels, "boxes": st.fmm_boxes, "m2l_pairs": st.fmm_m2l_pairs,
                "p2p_pairs": st.fmm_p2p_pairs},
        "near_pairs": st.near_pairs,
    }
    if args.serve:
        out["serving"] = serving(args.serve, args.serve_slots, [float(v) for v in args.serve_loads.split(",")],
                                 args.serve_budget_mib << 20)
    if not args.no_cpu:
        log("[bench] cpu leg: oracle checks on sampled rows and the oracle's own rate ...")
        out["cpu_baseline"], res = cpu_baseline(prob, factory, sig_h, args.cpu_budget, checks)
        out["rows_checked_vs_oracle"] = res["rows_checked"]
        out["apply_rel_err_vs_oracle"] = res["apply_rel_err_vs_oracle"]
        for path, r in res["solve_rows"].items():
            solve[path]["oracle_rows_rel_residual"] = r
        if representation is not None:
            representation.update(res["representation"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
