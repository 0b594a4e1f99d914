#!/usr/bin/env python3
"""Benchmark of the HPS hot path on one MI355X.

Workload (default): Omega = [-1, 1]^2, 64 x 64 leaves of 16 x 16 Chebyshev
points (N = 961^2 grid points), k = 80, contrast = 40 Gaussian bumps rescaled
to max 0.5 (seed 3), 256 incident directions, 256 measurement angles on the
circle R = 2, complex128 throughout.

One step = the whole hot path over that input: factor(q, k) + solve(256
directions) + far field + Frechet derivative (jvp, 256 right-hand sides) +
adjoint (vjp, 256 right-hand sides).  value = RHS solves per second over the
step: 3 * 256 right-hand sides (forward, derivative, adjoint) / step time,
factorisation included.  The per-wavenumber exterior set-up (host quadrature
of the layer potentials) is done once before timing and reported as
t_wavenumber_ms.

Prints one JSON line (see the keys below).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    # name: (nleaf, k, ndir, ntheta, nbumps, seed, amp, rescale)
    "k80_L64_M256": (64, 80.0, 256, 256, 40, 3, (0.0, 0.5), 0.5),
    "k10_L4_M16": (4, 10.0, 16, 64, 5, 1, (0.1, 0.3), None),
}
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def inputs(xy, cfg):
    import synth
    L, k, M, P, nb, seed, amp, resc = cfg
    q = synth.gaussian_bumps(xy, nb, seed, amp=amp, width=0.15, rescale_max=resc)
    dq = synth.gaussian_bumps(xy, 3, seed + 100, amp=(0.01, 0.02), width=0.3)
    rng = np.random.default_rng(seed + 200)
    r = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    return q, dq, r


def cpu_baseline(cfg, L_sample=8):
    """The oracle on a bounded sample of the workload: the same k, directions,
    angles and contrast generator on L_sample x L_sample leaves."""
    from oracle.bie import circle_points
    from oracle.forward import Problem, directions
    L, k, M, P = cfg[0], cfg[1], cfg[2], cfg[3]
    Ls = min(L, L_sample)
    prob = Problem(Ls, k)
    xy = prob.grid.pde_coords()
    q, dq, r = inputs(xy, cfg)
    _, th = circle_points(2.0, P)
    prob.set_measurement(th, 2.0)
    t0 = time.perf_counter()
    prob.factor(q)
    prob.solve(directions(M))
    prob.far_field()
    prob.jvp(dq)
    prob.vjp(r)
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas = 1
    return {"value": 3 * M / dt, "unit": "RHS solves/s", "cores": int(blas),
            "kind": "oracle",
            "sample": f"oracle step (factor + {M}-direction solve + far field + jvp + vjp) at k={k:g}, "
                      f"{Ls}x{Ls} leaves (1/{(L // Ls) ** 2} of the workload's leaves), "
                      f"{P} angles: {dt:.1f} s; SuperLU on 1 thread, dense parts on {blas} BLAS threads"}


def sine_truth(S, seed=4):
    """Sine coefficients of a smooth contrast: c_mn = 0.3 g_mn exp(-(m^2 + n^2)
    / 800), g ~ N(0, 1), later rescaled so that max q = 0.5 at the nodes."""
    rng = np.random.default_rng(seed)
    m = np.arange(1, S + 1)
    env = np.exp(-(m[:, None] ** 2 + m[None, :] ** 2) / 800.0)
    return 0.3 * rng.standard_normal((S, S)) * env


def gn_timing(s, k, dirs, th, R, steps, S=160, cg_iters=30):
    """Gauss-Newton steps on the sine model (S x S modes) at the benchmark's
    k, grid and directions: factor + solve at the current coefficients, then
    a fixed number of CG iterations, each one JVP and one VJP over all
    directions.  The data are the far field of a known contrast."""
    import torch
    c = torch.from_numpy(sine_truth(S).ravel()).cuda()
    q = s.sine_eval(c)
    scale = 0.5 / float(q.abs().max())
    c *= scale
    s.factor(s.sine_eval(c), k)
    s.solve(dirs)
    data = s.far_field(th, R).clone()
    c0 = 0.5 * c
    out = torch.empty_like(c)
    s.gn_step(k, dirs, th, R, c0, data, max_iter=cg_iters, tol=0.0, out=out)
    torch.cuda.synchronize()
    times, info = [], None
    for i in range(steps):
        t0 = time.perf_counter()
        _, info = s.gn_step(k, dirs, th, R, c0, data, max_iter=cg_iters, tol=0.0, out=out)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        log(f"gn step {i + 1}/{steps}: {times[-1]:.0f} ms, {info['cg_iters']} CG iterations")
    ms = float(np.median(times))
    M = len(dirs)
    # relative model error after the step (the data are exact, so one
    # Gauss-Newton step from half the true contrast should close most of it)
    err = float((out - c).norm() / c.norm())
    return {"ms_per_gn_step": ms, "modes": S * S, "cg_iters": int(info["cg_iters"]),
            "cg_rel_res": float(info["cg_rel_res"]), "misfit_before": float(info["misfit"]),
            "rhs_solves_per_step": (2 * int(info["cg_iters"]) + 1) * M,
            "rhs_solves_per_s": (2 * int(info["cg_iters"]) + 1) * M / (ms * 1e-3),
            "model_rel_err_after_step": err, "start": "half the true coefficients"}


def level_table(L, p=16):
    """Merge levels of the L x L leaf tree (alternating x / y merges):
    [(count, s = shared nodes, m = exterior nodes per child)] per level."""
    e = p - 2
    out = []
    nlev = 2 * int(round(np.log2(L)))
    for l in range(1, nlev + 1):
        s = e * 2 ** (l // 2)
        out.append((L * L // 2 ** l, s))
    return out


def child_boundary(l, e):
    """Boundary nodes of a box one level below merge level l (a leaf for
    l = 1): boxes alternate square (2^a x 2^a leaves) and 2:1 rectangles."""
    a = (l - 1) // 2
    if (l - 1) % 2 == 0:
        return 4 * e * 2 ** a
    return 6 * e * 2 ** a


def algorithmic_work(L, M, p=16):
    """Algorithmic flops (complex multiply-add = 8) of the factorisation stages
    as this library executes them, the part of each spent in explicit
    inverses (8 n^3 per order-n matrix by Gauss-Jordan), and the operator
    bytes one sweep must read (16 bytes per complex entry)."""
    e = p - 2
    mi, ne = e * e, 4 * e
    nl = L * L
    nb = 4 * L * e
    # leaves: the interior impedance problem (order mi) is inverted explicitly
    inv = {"leaf": nl * 8.0 * mi ** 3, "merge": 0.0, "top": 8.0 * nb ** 3}
    D_bytes = 0.0
    for l, (cnt, s) in enumerate(level_table(L, p), start=1):
        nc = child_boundary(l, e)
        m = nc - s
        inv["merge"] += cnt * 8.0 * s ** 3
        D_bytes += cnt * 16.0 * (2 * s) * (2 * m)
    ops = {
        # Z^-1, R_root, [S, -(K - I/2)], D per level, Y; u0 written once
        "solve": 16.0 * (2 * nb * nb + 2 * nb * nb) + D_bytes + 16.0 * nl * mi * ne + 16.0 * nl * mi * M,
        # H (read, scaled copy written and read), U per level, A2, Z^-1, R_root; u0 read
        "jvp": 16.0 * 3 * nl * ne * mi + D_bytes + 16.0 * 3 * nb * nb + 16.0 * nl * mi * M,
        # conjugate-transposed top operators, U per level, H; u0 read
        "vjp": 16.0 * 2 * nl * ne * mi + D_bytes + 16.0 * 3 * nb * nb + 16.0 * nl * mi * M,
    }
    return inv, ops


def phase_report(kernels, stats, L, M):
    """Per stage: wall time (HIP events around the stage), kernel time and
    algorithmic flops from the launch profiler, the rate against the FP64
    matrix-core peak counting explicit inverses as executed (8 n^3) and
    LU-equivalent (8 n^3 / 3, as a factorisation by LU would count them), and
    for the sweeps the operator bytes and their rate against HBM."""
    inv, ops = algorithmic_work(L, M)
    out = {}
    wall = {"leaf": stats["t_leaf_ms"], "merge": stats["t_merge_ms"], "top": stats["t_top_ms"],
            "solve": stats["t_solve_ms"], "jvp": stats["t_jvp_ms"], "vjp": stats["t_vjp_ms"]}
    for ph, ms in wall.items():
        k = kernels.get(f"phase:{ph}")
        if k is None or ms <= 0:
            continue
        r = {"wall_ms": ms, "kernel_ms": k["total_ms"], "launches": k["launches"], "flops": k["flops"],
             "tflops": k["flops"] / (ms * 1e-3) / 1e12}
        r["frac_peak"] = r["tflops"] / PEAK_FP64_TFLOPS
        if ph in inv:
            lu = k["flops"] - (2.0 / 3.0) * inv[ph]
            r.update({"flops_explicit_inverses": inv[ph], "flops_lu_equivalent": lu,
                      "tflops_lu_equivalent": lu / (ms * 1e-3) / 1e12,
                      "frac_peak_lu_equivalent": lu / (ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS})
        if ph in ops:
            r.update({"operator_bytes": ops[ph], "gbs": ops[ph] / (ms * 1e-3) / 1e9,
                      "frac_hbm": ops[ph] / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                      "arithmetic_intensity": k["flops"] / ops[ph]})
        out[ph] = r
    return out


def sweep_small_m(s, k, q, th, R, L, dq, M=16, reps=5):
    """Sweeps with few right-hand sides on the benchmark grid (the regime
    where they are bound by HBM, not by the matrix cores): solve, jvp and vjp
    with M directions, median of reps, with the operator bytes they read."""
    import torch
    import synth
    dirs = synth.equispaced_angles(M)
    rng = np.random.default_rng(5)
    r = torch.from_numpy(rng.standard_normal((M, len(th))) + 1j * rng.standard_normal((M, len(th)))).cuda()
    t = {"solve": [], "jvp": [], "vjp": []}
    for i in range(reps + 1):
        s.solve(dirs)
        s.far_field(th, R)
        s.jvp(dq)
        s.vjp(r)
        st = s.stats()
        if i > 0:
            for ph in t:
                t[ph].append(st[f"t_{ph}_ms"])
    _, ops = algorithmic_work(L, M)
    out = {"ndir": M}
    for ph, v in t.items():
        ms = float(np.median(v))
        out[ph] = {"ms": ms, "operator_bytes": ops[ph], "gbs": ops[ph] / (ms * 1e-3) / 1e9,
                   "frac_hbm": ops[ph] / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    return out


def recursive_linearization_timing(k_max=20.0):
    """The recursive linearization of Section 3.4 with the Section 4 protocol
    (k_j = 1 + j/4 up to k_max, M = floor 2k directions, P = floor 4k
    receivers at R = 20, band m + n <= floor 2k, leaves per k for >= 10
    points per wavelength, one Newton step per k with the CG (LSQR) tolerance
    1e-3, q_1 the projection onto the modes (1,1), (1,2), (2,1)); data from
    the generator on another discretisation (p = 20, >= 15 points per
    wavelength), no noise.  Times the inversion only (data made first)."""
    import torch
    import synth
    from paper_1608_06871_amd.drivers import (DataGenerator, RecursiveLinearization, initial_projection,
                                              paper_schedule)
    qfn = lambda xy: synth.gaussian_bumps(xy, 5, 2, amp=(0.1, 0.3), width=0.15)
    sched = paper_schedule(k_max, ppw=10.0)
    gen = DataGenerator(qfn, p=20, ppw=15.0)
    data = [gen(st) for st in sched]
    rl = RecursiveLinearization(sched, lambda st: data[st["j"]], newton_max=1, cg_tol=1e-3, cg_max=200)
    s0 = rl.solver(sched[0]["L"])
    coef0 = initial_projection(s0, torch.from_numpy(qfn(s0.node_coords())).cuda(), S=2)
    # contexts and per-k set-up outside the timed run: one pass at the first k
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    coef, S, log = rl.run(coef0, S0=2, resume=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sl = rl.solver(sched[-1]["L"])
    qm = sl.sine_eval(coef).cpu().numpy()
    qt = qfn(sl.node_coords())
    its = [e["newton"][0]["cg_iters"] for e in log]
    solves = sum((2 * i + 1) * e["M"] for i, e in zip(its, log))
    return {"k_max": k_max, "frequencies": len(sched), "seconds": dt, "ms_per_frequency": dt / len(sched) * 1e3,
            "cg_iters_total": int(sum(its)), "rhs_solves": int(solves), "rhs_solves_per_s": solves / dt,
            "final_grid_leaves": sched[-1]["L"], "final_modes": sched[-1]["modes"],
            "final_misfit_rel": log[-1]["newton"][0]["misfit_before"],
            "model_rel_err": float(np.linalg.norm(qm - qt) / np.linalg.norm(qt)),
            "protocol": "Section 4 schedule, 10 ppw inversion grids, p=20 data grids at 15 ppw, no noise, "
                        "1 Newton step per k, CG tol 1e-3; inversion only (data generated before timing)"}


# the GEMM kernels and the sources that decide which GEMM calls a step makes
# (shapes, counts): the stored per-launch traffic holds while none changes
GEMM_SOURCES = [os.path.join(ROOT, "paper_1608_06871_amd", "csrc", f) for f in ("zgemm.hip", "zinv.hip", "hps.cpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "zgemm_traffic_k80_L64_M256_fp64.json")


def source_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(hashlib.sha256(f.read()).digest())
    return h.hexdigest()


def stored_traffic():
    """HBM bytes per launch of the complex FP64 GEMM class from the committed
    counter summary, or None when the GEMM kernels or the code that issues the
    GEMM calls have changed since the counters were taken (or no summary
    exists)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sha256") != source_sha256(GEMM_SOURCES):
        return None
    return t.get("traffic_bytes_per_launch")


def copy_probe(mib, reps=4):
    """Plain device copies of `mib` MiB (hipMemcpy kernels): the calibration
    of the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * (1 << 20)
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": reps + 1}), flush=True)


STEP_MARK = r"k_leaf_assemble"  # first kernel of every benchmark step


def pmc_sum(csv_path, pattern, counter, after=None):
    """Sum of `counter` (KiB) and the dispatch count over the kernels whose
    name matches `pattern` in a rocprofv3 counter_collection.csv; with
    `after`, only dispatches issued after the last kernel matching it (the
    last benchmark step, without the warm-up's tuning trials)."""
    import csv
    import re
    rows = []
    with open(csv_path) as f:
        rows = [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]
    lo = -1
    if after:
        ra = re.compile(after)
        marks = [int(r["Dispatch_Id"]) for r in rows if ra.search(r["Kernel_Name"])]
        lo = max(marks) if marks else -1
    tot, disp = 0.0, set()
    rx = re.compile(pattern)
    for r in rows:
        if rx.search(r["Kernel_Name"]) and int(r["Dispatch_Id"]) > lo:
            tot += float(r["Counter_Value"])
            disp.add(r["Dispatch_Id"])
    return tot, len(disp)


def traffic_summary(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, out_path):
    """Writes the GEMM-class HBM traffic per launch from four counter runs:
    FETCH_SIZE and WRITE_SIZE of the benchmark's last step (the dispatches
    after its leaf assembly) and of a plain copy of copy_bytes bytes, which
    calibrates each counter (bytes per KiB counted)."""
    # bytes of every kernel of a GEMM call (split-K slices and their
    # reduction included); launches = GEMM calls = main-kernel dispatches
    gemm = r"zgemm_kernel|gemm_kernel<double|k_splitk_reduce"
    main = r"zgemm_kernel|gemm_kernel<double"
    copy = r"copyBuffer"
    f_kib, _ = pmc_sum(fetch_csv, gemm, "FETCH_SIZE", STEP_MARK)
    w_kib, _ = pmc_sum(write_csv, gemm, "WRITE_SIZE", STEP_MARK)
    _, nf = pmc_sum(fetch_csv, main, "FETCH_SIZE", STEP_MARK)
    _, nw = pmc_sum(write_csv, main, "WRITE_SIZE", STEP_MARK)
    cf_kib, ncf = pmc_sum(copy_fetch_csv, copy, "FETCH_SIZE")
    cw_kib, ncw = pmc_sum(copy_write_csv, copy, "WRITE_SIZE")
    # each copy reads and writes copy_bytes once
    sf = copy_bytes * ncf / (cf_kib * 1024.0)
    sw = copy_bytes * ncw / (cw_kib * 1024.0)
    launches = max(nf, nw)
    per = (f_kib * 1024.0 * sf + w_kib * 1024.0 * sw) / launches
    res = {"sources": [os.path.relpath(p, ROOT) for p in GEMM_SOURCES], "sha256": source_sha256(GEMM_SOURCES),
           "launches": launches, "fetch_kib": f_kib, "write_kib": w_kib,
           "copy_bytes": copy_bytes, "copy_fetch_kib_per_copy": cf_kib / ncf, "copy_write_kib_per_copy": cw_kib / ncw,
           "scale_fetch": sf, "scale_write": sw, "traffic_bytes_per_launch": per}
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res), flush=True)


def trace_summary(trace_csv, out_path, skip_steps=1):
    """Per-step kernel table from a rocprofv3 kernel trace (--kernel-trace
    --output-format csv) of a benchmark run: the trace is cut into steps at
    every k_leaf_assemble (the first kernel of a step), the first skip_steps
    (warm-up, with the GEMM tile-tuning trials) are left out, and each kernel
    name's calls and time are averaged over the remaining steps.  Also: the
    GEMM family per call (compare roofline.avg_launch_ms of the bench line),
    kernel time, window (first start to last end) and GPU-busy time (union of
    the kernel intervals) per step."""
    import csv
    import re
    with open(trace_csv) as f:
        rows = list(csv.DictReader(f))
    key = lambda r, *names: next(r[n] for n in names if n in r)
    ev = sorted((int(key(r, "Start_Timestamp", "start")), int(key(r, "End_Timestamp", "end")),
                 key(r, "Kernel_Name", "kernel_name", "name")) for r in rows)
    marks = [i for i, e in enumerate(ev) if re.search(STEP_MARK, e[2])]
    if len(marks) <= skip_steps:
        raise SystemExit("trace holds no step after the skipped ones")
    sel = ev[marks[skip_steps]:]
    nsteps = len(marks) - skip_steps

    def short(n):
        n = re.sub(r"^void ", "", n)
        n = n.replace("hps::(anonymous namespace)::", "").replace("hps::", "")
        n = re.sub(r"\(.*$", "", n)
        return n.replace("HIP_vector_type<double, 2u>", "double2").replace("HIP_vector_type<float, 2u>", "float2")

    tot = {}
    for s0, e0, n in sel:
        k = short(n)
        c, t = tot.get(k, (0, 0.0))
        tot[k] = (c + 1, t + (e0 - s0) * 1e-6)
    ktime = sum(t for _, t in tot.values())
    busy, cur_s, cur_e = 0.0, None, None
    for s0, e0, _ in sel:
        if cur_e is None or s0 > cur_e:
            if cur_e is not None:
                busy += (cur_e - cur_s) * 1e-6
            cur_s, cur_e = s0, e0
        else:
            cur_e = max(cur_e, e0)
    busy += (cur_e - cur_s) * 1e-6
    window = (max(e for _, e, _ in sel) - sel[0][0]) * 1e-6
    gemm = [(c, t) for k, (c, t) in tot.items() if re.search(r"zgemm_kernel|gemm_kernel<double|k_splitk_reduce", k)]
    main_calls = sum(c for k, (c, _) in tot.items() if re.search(r"zgemm_kernel|gemm_kernel<double", k))
    gt = sum(t for _, t in gemm)
    lines = [f"Steps summarised: {nsteps} (after {skip_steps} warm-up step(s) left out).", "",
             f"Per step: kernel time {ktime / nsteps:.2f} ms, window {window / nsteps:.2f} ms, GPU busy "
             f"{busy / nsteps:.2f} ms (kernel time above the window: kernels overlapping on a second stream).", "",
             f"Complex FP64 GEMM family (`zgemm_kernel`, FP64 `gemm_kernel`, `k_splitk_reduce`): "
             f"{main_calls / nsteps:.0f} calls per step, {gt / nsteps:.2f} ms per step, "
             f"{gt / max(main_calls, 1) * 1e3:.1f} us per call.", "",
             "| kernel | calls per step | ms per step | avg us | % of kernel time |", "|---|---|---|---|---|"]
    for k, (c, t) in sorted(tot.items(), key=lambda x: -x[1][1]):
        if t / ktime < 0.001:
            continue
        lines.append(f"| `{k}` | {c / nsteps:.1f} | {t / nsteps:.2f} | {t / c * 1e3:.1f} | {100 * t / ktime:.1f} |")
    text = "\n".join(lines) + "\n"
    with open(out_path, "w") as f:
        f.write(text)
    print(text, flush=True)


def batch_problems(n=32, seed0=100):
    """32 independent problems: k ~ U[10, 60], leaf grids 8, 16 or 32 per
    side, 16 to 256 directions, contrasts from the 5-bump generator."""
    import synth
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed0 + i)
        out.append({"seed": seed0 + i, "k": float(rng.uniform(10.0, 60.0)), "L": int(rng.choice([8, 16, 32])),
                    "M": int(rng.choice([16, 32, 64, 128, 256]))})
    return out


def run_batch(args, emit=True):
    """Batched forward solves (factor + solve + far field) of 32 problems in
    one context per leaf grid, against the same problems solved one by one."""
    import torch
    import paper_1608_06871_amd as hps
    from paper_1608_06871_amd.drivers import BatchForward
    import synth
    specs = batch_problems()
    P, R = 64, 2.0
    th = synth.equispaced_angles(P)
    probs = [dict(sp) for sp in specs]
    # node coordinates per grid (the same for every problem on it)
    coords = {}
    for L in sorted({sp["L"] for sp in specs}):
        coords[L] = hps.Solver(nleaf=L, p=16, keep_derivs=False).node_coords()
    for pr in probs:
        xy = coords[pr["L"]]
        pr["q"] = torch.from_numpy(synth.gaussian_bumps(xy, 5, pr["seed"], amp=(0.1, 0.3), width=0.15)).cuda()
        pr["dirs"] = synth.equispaced_angles(pr["M"])
    nrhs = sum(pr["M"] for pr in probs)
    log(f"batch: {len(probs)} problems, {nrhs} directions, grids " +
        ", ".join(f"L={L}: {sum(1 for p in probs if p['L'] == L)}" for L in sorted(coords)))
    prec = getattr(args, "batch_precision", "fp64")
    bf = BatchForward(keep_derivs=False, precision=prec)
    t0 = time.perf_counter()
    bf.prepare(probs)
    t_set = time.perf_counter() - t0
    for w in range(args.warmup):
        bf.run(probs, th, R)
        torch.cuda.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = bf.run(probs, th, R)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    log(f"batched: {dt * 1e3:.1f} ms per pass")
    # the same problems one by one, each in its own single-problem context
    singles = []
    for pr in probs:
        s = hps.Solver(nleaf=pr["L"], p=16, keep_derivs=False)
        s.set_wavenumber(pr["k"])
        singles.append(s)

    def one_by_one():
        res = []
        for s, pr in zip(singles, probs):
            s.factor(pr["q"], pr["k"])
            s.solve(pr["dirs"])
            res.append(s.far_field(th, R))
        return res
    for w in range(args.warmup):
        one_by_one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ref = one_by_one()
    torch.cuda.synchronize()
    dt1 = (time.perf_counter() - t0) / args.steps
    log(f"one by one: {dt1 * 1e3:.1f} ms per pass")
    maxdiff = max(float((a - b).abs().max() / b.abs().max()) for a, b in zip(out, ref))
    res = {
        "metric": "RHS solves/sec, 32 independent (q,k) problems, batched per leaf grid",
        "value": nrhs / dt, "unit": "RHS solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "c64 sweeps + f64 refinement", "data": "synthetic",
        "config": {"workload": "32 problems (seeds 100-131): k ~ U[10,60], 8x8/16x16/32x32 leaves of 16x16, "
                               f"16-256 directions, 64 angles, R=2, factor + solve + far field, {prec}",
                   "problems": len(probs), "rhs": nrhs, "precision": prec},
        "one_by_one_ms": dt1 * 1e3, "one_by_one_rhs_per_s": nrhs / dt1, "speedup_vs_one_by_one": dt1 / dt,
        "max_rel_diff_vs_one_by_one": maxdiff, "t_wavenumber_setup_s": t_set,
        "gemm_tuning": hps.gemm_tuning_info(),
    }
    if emit:
        print(json.dumps(res), flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="k80_L64_M256", choices=sorted(CONFIGS) + ["batch32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event timing")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision comparison")
    ap.add_argument("--no-gn", action="store_true", help="skip the Gauss-Newton step timing")
    ap.add_argument("--no-small-m", action="store_true", help="skip the 16-direction sweep timing")
    ap.add_argument("--no-rl", action="store_true", help="skip the recursive-linearization timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the 32-problem batch")
    ap.add_argument("--streams", type=int, choices=[1, 2], default=2,
                    help="streams of the benchmark context (hps_opts.streams)")
    ap.add_argument("--batch-precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--tune", choices=["auto", "on", "off"], default="auto",
                    help="GEMM tile autotuning (every distinct GEMM shape times its candidate tile shapes on its "
                         "first call, in the untimed warm-up; results are bitwise the same); auto: on whenever "
                         "there is a warm-up step")
    ap.add_argument("--copy-probe", type=int, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--trace-summary", nargs=2, metavar=("KERNEL_TRACE_CSV", "OUT"),
                    help="per-step kernel table of a rocprofv3 kernel trace of a benchmark run")
    ap.add_argument("--traffic-summary", nargs=5, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV",
                                                           "COPY_WRITE_CSV", "COPY_BYTES"),
                    help="write the GEMM traffic summary from four rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.traffic_summary:
        a = args.traffic_summary
        return traffic_summary(a[0], a[1], a[2], a[3], int(a[4]), TRAFFIC_FILE)
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    if args.trace_summary:
        return trace_summary(args.trace_summary[0], args.trace_summary[1])
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (--gpus {args.gpus} "
              "requested). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1608_06871_amd as hps
    import synth
    tune = args.warmup >= 1 and args.tune in ("on", "auto")
    if tune:
        # every GEMM shape is tuned on its first call, in the untimed warm-up
        hps.gemm_tuning(1)
    if args.config == "batch32":
        return run_batch(args)

    cfg = CONFIGS[args.config]
    L, k, M, P = cfg[0], cfg[1], cfg[2], cfg[3]
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    log(f"config {args.config}: L={L} k={k} M={M} P={P}")
    s = hps.Solver(nleaf=L, p=16, keep_derivs=True, streams=args.streams)
    xy = s.node_coords()
    q_np, dq_np, r_np = inputs(xy, cfg)
    q = torch.from_numpy(q_np).cuda()
    dq = torch.from_numpy(dq_np).cuda()
    r = torch.from_numpy(r_np).cuda()
    dirs = synth.equispaced_angles(M)
    th = synth.equispaced_angles(P)
    R = 2.0
    t0 = time.perf_counter()
    s.set_wavenumber(k)
    t_wave = (time.perf_counter() - t0) * 1e3
    log(f"exterior set-up (host quadrature) {t_wave:.0f} ms")
    ufar = torch.empty((M, P), dtype=torch.complex128, device="cuda")
    dfar = torch.empty((M, P), dtype=torch.complex128, device="cuda")
    grad = torch.empty(s.npde, dtype=torch.float64, device="cuda")

    def step():
        s.factor(q, k)
        s.solve(dirs)
        s.far_field(th, R, out=ufar)
        s.jvp(dq, out=dfar)
        s.vjp(r, out=grad)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done")
    phases = {"factor": [], "solve": [], "far_field": [], "jvp": [], "vjp": [], "leaf": [], "merge": [], "top": []}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        st = s.stats()
        for ph in phases:
            phases[ph].append(st[f"t_{ph}_ms"])
        log(f"step {i + 1}/{args.steps}: factor {st['t_factor_ms']:.1f} ms, solve {st['t_solve_ms']:.1f} ms, "
            f"jvp {st['t_jvp_ms']:.1f} ms, vjp {st['t_vjp_ms']:.1f} ms")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = 3 * M * args.steps / dt
    dev_bytes = s.stats()["device_bytes"]

    roofline = None
    kernels = None
    if not args.no_profile:
        # one more step with every kernel launch bracketed by HIP events on
        # the launch stream; the dominant kernel class gives the roofline
        torch.cuda.synchronize()
        hps.profile_start()
        step()
        kernels = hps.profile_stop()
        dom = max((n for n in kernels if not n.startswith("phase:")), key=lambda n: kernels[n]["total_ms"])
        kd = kernels[dom]
        per_launch_ms = kd["total_ms"] / kd["launches"]
        if kd["flops"] > 0:
            achieved = kd["flops"] / (kd["total_ms"] * 1e-3) / 1e12
            roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": achieved / PEAK_FP64_TFLOPS,
                        "traffic": stored_traffic() if dom == "zgemm" else None, "kernel": dom,
                        "launches": kd["launches"], "avg_launch_ms": per_launch_ms,
                        "flops_per_launch": kd["flops"] / kd["launches"]}
        else:
            achieved = kd["bytes"] / (kd["total_ms"] * 1e-3) / 1e9
            roofline = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": achieved / PEAK_HBM_GBS, "traffic": None, "kernel": dom,
                        "launches": kd["launches"], "avg_launch_ms": per_launch_ms,
                        "bytes_per_launch": kd["bytes"] / kd["launches"]}
        log("kernel classes: " + ", ".join(f"{n} {v['total_ms']:.1f} ms/{v['launches']}" for n, v in kernels.items()))
        # the same step with the factorisation on one stream: the dominant
        # class's launches then never share the chip with the other stream's
        # (one untimed step first: the full leaf batch is a new GEMM shape)
        s.set_streams(1)
        step()
        torch.cuda.synchronize()
        hps.profile_start()
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        t1 = time.perf_counter() - t1
        k1 = hps.profile_stop()[dom]
        s.set_streams(args.streams)
        a1 = (k1["flops"] if roofline["bound"] == "mfma" else k1["bytes"]) / (k1["total_ms"] * 1e-3)
        a1 = a1 / 1e12 if roofline["bound"] == "mfma" else a1 / 1e9
        roofline["one_stream"] = {"achieved": a1, "frac": a1 / roofline["peak"], "launches": k1["launches"],
                                  "avg_launch_ms": k1["total_ms"] / k1["launches"],
                                  "profiled_step_ms": t1 * 1e3}
        log(f"one-stream step: {t1 * 1e3:.1f} ms, {dom} {a1:.1f} {roofline['unit']}")
        med_now = {ph: float(np.median(v)) for ph, v in phases.items()}
        stage = phase_report(kernels, {f"t_{ph}_ms": v for ph, v in med_now.items()}, L, M)
        log("stages: " + ", ".join(f"{ph} {v['wall_ms']:.1f} ms {v['tflops']:.1f} TF" for ph, v in stage.items()))
    else:
        stage = None

    small_m = None
    if not args.no_small_m:
        small_m = sweep_small_m(s, k, q, th, R, L, dq)
        log("16-direction sweeps: " + ", ".join(f"{ph} {v['ms']:.2f} ms {v['gbs']:.0f} GB/s" for ph, v in small_m.items()
                                               if isinstance(v, dict)))

    gn = None
    if not args.no_gn:
        log("Gauss-Newton steps (160 x 160 sine modes, 30 CG iterations) ...")
        gn = gn_timing(s, k, dirs, th, R, max(1, min(args.steps, 2)))
        log(f"gn: {gn['ms_per_gn_step']:.0f} ms per step, model error after the step "
            f"{gn['model_rel_err_after_step']:.2e}")

    mixed = None
    if not args.no_mixed:
        # far-field error after a fixed number of corrections (the refinement
        # target set out of reach so that exactly that many are made)
        del s
        torch.cuda.empty_cache()
        per_corr = []
        for nref in (0, 1, 2):
            sm = hps.Solver(nleaf=L, p=16, keep_derivs=False, precision="mixed", max_refine=nref, refine_tol=1e-300,
                            fallback_fp64=False)
            sm.factor(q, k)
            try:
                sm.solve(dirs)
            except hps.HpsError as e:
                if e.code != hps.HPS_ENOCONV:
                    raise
            um = sm.far_field(th, R)
            st = sm.stats()
            per_corr.append({"corrections": nref, "residual": float(st["refine_residual"]),
                             "far_field_rel_err_vs_fp64": float((um - ufar).abs().max() / ufar.abs().max())})
            del sm
        log("mixed per correction: " + ", ".join(f"{c['corrections']}: res {c['residual']:.1e} "
                                                 f"err {c['far_field_rel_err_vs_fp64']:.1e}" for c in per_corr))
        # the same workload in mixed precision (complex64 sweeps + refinement),
        # timed the same way, with its far-field error against complex128
        torch.cuda.empty_cache()
        sm = hps.Solver(nleaf=L, p=16, keep_derivs=False, precision="mixed")
        sm.set_wavenumber(k)
        um = torch.empty((M, P), dtype=torch.complex128, device="cuda")

        def mstep():
            sm.factor(q, k)
            sm.solve(dirs)
            sm.far_field(th, R, out=um)
        mstep()
        torch.cuda.synchronize()
        mf, ms = [], []
        t0 = time.perf_counter()
        for i in range(args.steps):
            mstep()
            st = sm.stats()
            mf.append(st["t_factor_ms"])
            ms.append(st["t_solve_ms"])
        torch.cuda.synchronize()
        dtm = (time.perf_counter() - t0) / args.steps
        err = float((um - ufar).abs().max() / ufar.abs().max())
        mixed = {"ms_per_factor_solve_farfield": dtm * 1e3, "factor_ms": float(np.median(mf)),
                 "solve_ms": float(np.median(ms)), "rhs_per_s_incl_factor": M / dtm,
                 "solve_only_rhs_per_s": M / (float(np.median(ms)) * 1e-3),
                 "refine_iters": int(st["refine_iters"]), "refine_residual": float(st["refine_residual"]),
                 "refine_tol": sm.refine_tol, "far_field_rel_err_vs_fp64": err, "per_correction": per_corr}
        log(f"mixed: factor {mixed['factor_ms']:.1f} ms, solve {mixed['solve_ms']:.1f} ms, "
            f"{mixed['refine_iters']} corrections, far-field error vs fp64 {err:.2e}")
        del sm
        if not args.no_gn:
            torch.cuda.empty_cache()
            sg = hps.Solver(nleaf=L, p=16, keep_derivs=True, precision="mixed")
            sg.set_wavenumber(k)
            mixed["gauss_newton"] = gn_timing(sg, k, dirs, th, R, 1)
            log(f"mixed gn: {mixed['gauss_newton']['ms_per_gn_step']:.0f} ms per step")
            del sg

    rl = None
    if not args.no_rl:
        torch.cuda.empty_cache()
        log("recursive linearization to k = 20 ...")
        rl = recursive_linearization_timing(20.0)
        log(f"recursive linearization: {rl['frequencies']} frequencies in {rl['seconds']:.2f} s, "
            f"model error {rl['model_rel_err']:.2e}")

    batch = None
    if not args.no_batch:
        torch.cuda.empty_cache()
        batch = run_batch(args, emit=False)
        log(f"batch32: {batch['value']:.0f} RHS solves/s ({batch['config']['precision']})")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(cfg)
        log(f"cpu baseline: {cpu['value']:.2f} RHS solves/s")

    med = {ph: float(np.median(v)) for ph, v in phases.items()}
    if mixed is not None:
        mixed["fp64_factor_solve_farfield_ms"] = med["factor"] + med["solve"] + med["far_field"]
    out = {
        "metric": "RHS solves/sec + factor time at k=80, mixed vs FP64 at <=1e-8 rel far-field err",
        "value": value,
        "unit": "RHS solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"HPS forward+jvp+vjp, k={k:g}, {L}x{L} leaves of 16x16, "
                               f"{M} directions, {P} angles, R={R:g}, FP64",
                   "k": k, "nleaf": L, "p": 16, "ndir": M, "ntheta": P, "precision": "fp64",
                   "streams": args.streams},
        "factor_ms": med["factor"],
        "solve_ms": med["solve"],
        "far_field_ms": med["far_field"],
        "jvp_ms": med["jvp"],
        "vjp_ms": med["vjp"],
        "solve_only_rhs_per_s": M / (med["solve"] * 1e-3) if med["solve"] > 0 else None,
        "t_wavenumber_ms": t_wave,
        "device_bytes": dev_bytes,
        "roofline": roofline,
        "stages": stage,
        "sweeps_16_directions": small_m,
        "kernels": {n: v for n, v in kernels.items() if not n.startswith("phase:")} if kernels else None,
        "cpu_baseline": cpu,
        "mixed": mixed,
        "gauss_newton": gn,
        "recursive_linearization": rl,
        "batch32": batch,
        "zinv_pivoting": hps.zinv_pivoting_info(),
        "gemm_tuning": dict(hps.gemm_tuning_info(), mode="autotuned" if tune else "fixed rules"),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
