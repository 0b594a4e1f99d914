"""Drivers above the C ABI.

Recursive linearization (the algorithm box of Section 3.4, with the protocol
of Section 4): for ascending wavenumbers k_j, zero-extend the sine-model
coefficients to the new band S(k_j) and take Gauss-Newton steps (Section 3.3)
with the library's hps_gn_step.  Only the schedule and the coefficient
bookkeeping happen here; every solve, derivative and CG iteration runs in the
library.  Batched forward solves of many independent problems: BatchForward.
"""
import json
import math
import os
import time

import numpy as np
import torch


def recursive_linearization(solver, ks, bands, data, dirs, thetas, R, newton_steps=1,
                            max_iter=50, tol=1e-12, coef0=None, S0=0):
    """ks: ascending wavenumbers; bands: sine band S per k; data: list of
    complex128 GPU tensors [ndir, ntheta] per k.  Returns the final
    coefficients and a per-step log."""
    coef = coef0 if coef0 is not None else torch.zeros(0, dtype=torch.float64, device="cuda")
    S_prev = S0
    log = []
    for k, S, d in zip(ks, bands, data):
        coef = extend(coef, S_prev, S)
        for it in range(newton_steps):
            coef, info = solver.gn_step(k, dirs, thetas, R, coef, d, max_iter=max_iter, tol=tol)
            log.append({"k": float(k), "S": int(S), "newton": it, **info})
        S_prev = S
    return coef, log


def leaves_for(k, ppw, p=16, width=2.0, min_leaves=1, max_leaves=256):
    """Leaves per side for a wavenumber (Section 4: 2^l x 2^l leaves of p x p
    points, l chosen so that there are at least ppw points per wavelength):
    the smallest power of two L >= min_leaves with (p - 1) L intervals over
    the width spanning at least ppw per wavelength, width k / (2 pi)
    wavelengths across."""
    need = ppw * k * width / (2.0 * math.pi) / (p - 1)
    L = 1
    while L < need or L < min_leaves:
        L *= 2
    if L > max_leaves:
        raise ValueError(f"k = {k} needs more than {max_leaves} leaves per side at {ppw} points per wavelength")
    return L


def grid_for(k, ppw, width=2.0, p_range=(12, 20), min_leaves=1, max_leaves=256):
    """(L, p) for a wavenumber: L leaves per side (a power of two) of p x p
    points, with at least ppw points per wavelength over the width (Section 4)
    and as few points as that allows: the fewest intervals (p - 1) L per side
    with (p - 1) L >= ppw k width / (2 pi), p in p_range, ties to the higher
    order.  The leaf order supplies the granularity that a power-of-two leaf
    count alone lacks (doubling L can double the points per side)."""
    need = ppw * k * width / (2.0 * math.pi)
    best = None
    L = 1
    while L <= max_leaves:
        if L >= min_leaves:
            p = max(p_range[0], int(math.ceil(need / L - 1e-9)) + 1)
            if p <= p_range[1]:
                key = ((p - 1) * L, -p)
                if best is None or key < best[0]:
                    best = (key, L, p)
        L *= 2
    if best is None:
        raise ValueError(f"k = {k} needs more than {max_leaves} leaves per side at {ppw} points per wavelength")
    return best[1], best[2]


def paper_schedule(k_max, k0=1.0, dk=0.25, ppw=10.0, p=16, width=2.0, angles_per_k=4, R=20.0, min_leaves=1,
                   leaves=None):
    """The frequency schedule of Section 4: k_j = k0 + j dk up to k_max,
    M_j = floor(2 k_j) incident directions at 2 pi m / M_j, P_j =
    floor(angles_per_k k_j) receivers at 2 pi p / P_j on the circle of radius
    R, band S(k_j) = floor(2 k_j) (eq. sineseries: modes m + n <= S), and the
    leaf grid per k from the points-per-wavelength rule (or `leaves` for a
    fixed grid; p = "auto" picks leaf count and order per k with grid_for,
    each step then carrying its own "p").  The text gives P_j = floor(4 k_j);
    Tables 2-3 list M P = 16 k^2, i.e. P = 8 k (angles_per_k = 8)."""
    out = []
    j = 0
    while True:
        k = k0 + j * dk
        if k > k_max + 1e-12:
            break
        M = max(1, int(math.floor(2.0 * k + 1e-12)))
        P = max(1, int(math.floor(angles_per_k * k + 1e-12)))
        S = int(math.floor(2.0 * k + 1e-12))
        if p == "auto":
            L, pk = grid_for(k, ppw, width, min_leaves=min_leaves) if leaves is None else (leaves, 16)
        else:
            L, pk = (leaves if leaves is not None else leaves_for(k, ppw, p, width, min_leaves)), p
        out.append({"j": j, "k": k, "M": M, "P": P, "band": S, "modes": S * (S - 1) // 2, "L": L, "p": pk,
                    "R": R})
        j += 1
    return out


def extend(coef, S_old, S_new):
    """Zero-extension of an [S_old, S_old] coefficient block to [S_new, S_new]
    (Section 3.4: the previous band-limited model is the initial guess)."""
    out = torch.zeros(S_new * S_new, dtype=torch.float64, device=coef.device)
    if S_old > 0:
        m = min(S_old, S_new)
        out.view(S_new, S_new)[:m, :m] = coef.view(S_old, S_old)[:m, :m]
    return out


def initial_projection(solver, q_nodes, modes=((1, 1), (1, 2), (2, 1)), S=2):
    """q_1 of Section 4: the coefficients of the given modes of the sine model
    that best fit a contrast q at the solver's PDE nodes in the least-squares
    sense (the projection of q onto those modes), as an [S, S] block.  The
    normal-equation matrix E^T E and E^T q come from the library's sine maps;
    the small (#modes x #modes) system is solved on the host."""
    nm = len(modes)
    cols = []
    for (m, n) in modes:
        e = torch.zeros(S * S, dtype=torch.float64, device="cuda")
        e[(m - 1) * S + (n - 1)] = 1.0
        cols.append(e)
    idx = [(m - 1) * S + (n - 1) for (m, n) in modes]
    G = np.zeros((nm, nm))
    for a in range(nm):
        ETe = solver.sine_adjoint(solver.sine_eval(cols[a]), S).cpu().numpy()
        G[:, a] = ETe[idx]
    b = solver.sine_adjoint(q_nodes.contiguous(), S).cpu().numpy()[idx]
    c = np.linalg.solve(G, b)
    out = torch.zeros(S * S, dtype=torch.float64, device="cuda")
    for v, i in zip(c, idx):
        out[i] = float(v)
    return out


class DataGenerator:
    """Measured data for the recursive linearization: the scattered field of
    a known contrast on the circle of radius R (Section 1), computed by the
    library on a discretisation other than the inversion's (another Chebyshev
    order p and its own leaf grid per k) so that the inversion does not
    reproduce its own discretisation error (the inverse crime Section 4
    avoids), with the noise model of Section 4 (synth.add_noise) when
    delta > 0.  q_fn maps node coordinates [n, 2] to contrast values."""

    def __init__(self, q_fn, p=20, ppw=15.0, delta=0.0, seed=0, box=(-1.0, 1.0, -1.0, 1.0), min_leaves=1):
        self.q_fn, self.p, self.ppw, self.delta, self.seed = q_fn, p, ppw, delta, seed
        self.box, self.min_leaves = box, min_leaves
        self._ctx = {}

    def solver(self, L):
        from . import Solver
        if L not in self._ctx:
            s = Solver(nleaf=L, p=self.p, box=self.box, keep_derivs=False)
            s.q_true = torch.from_numpy(np.ascontiguousarray(self.q_fn(s.node_coords()))).cuda()
            self._ctx[L] = s
        return self._ctx[L]

    def __call__(self, step):
        import synth
        L = leaves_for(step["k"], self.ppw, self.p, self.box[1] - self.box[0], self.min_leaves)
        s = self.solver(L)
        s.factor(s.q_true, step["k"])
        s.solve(synth.equispaced_angles(step["M"]))
        ff = s.far_field(synth.equispaced_angles(step["P"]), step["R"]).cpu().numpy()
        if self.delta > 0.0:
            ff = synth.add_noise(ff, self.delta, self.seed + step["j"])
        return torch.from_numpy(np.ascontiguousarray(ff)).cuda()


class RecursiveLinearization:
    """Recursive linearization with Newton's method (the algorithm box of
    Section 3.4; Section 3.3 for the Newton iteration):

      for each k_j of the schedule (paper_schedule):
        a leaf grid for k_j (schedule "L"), the band S(k_j) (modes m + n <= S);
        the coefficients of the previous frequency as the initial guess
        (zero-extended; the first from coef0, e.g. initial_projection);
        Newton steps: solve the normal equations (eq. normaleq) by CG on the
        library (hps_gn_step: one JVP and one VJP per iteration) until the
        CG residual falls to cg_tol times its initial norm (the LSQR
        tolerance of Section 4, 1e-3) or cg_max iterations; update the
        coefficients; stop when the data misfit ||d - F[q]|| is below
        newton_tol ||d|| (the paper's stopping test, relative here), when a
        step no longer lowers it, or after newton_max steps.

    checkpoint: a JSON file rewritten after every frequency with the
    coefficients and the log; run(resume=True) continues after the last
    frequency it holds.  Contexts are kept per leaf grid."""

    def __init__(self, schedule, data, p=16, newton_max=1, newton_tol=0.0, cg_tol=1e-3, cg_max=200,
                 box=(-1.0, 1.0, -1.0, 1.0), checkpoint=None):
        self.schedule, self.data, self.p, self.box = schedule, data, p, box
        self.newton_max, self.newton_tol = newton_max, newton_tol
        self.cg_tol, self.cg_max = cg_tol, cg_max
        self.checkpoint = checkpoint
        self._ctx = {}

    def solver(self, L, p=None):
        from . import Solver
        p = self.p if p is None else p
        if (L, p) not in self._ctx:
            self._ctx[(L, p)] = Solver(nleaf=L, p=p, box=self.box, keep_derivs=True)
        return self._ctx[(L, p)]

    def _save(self, j, coef, S, log):
        tmp = self.checkpoint + ".tmp"
        with open(tmp, "w") as f:
            json.dump({"j": j, "S": S, "coef": coef.cpu().numpy().tolist(), "log": log}, f)
        os.replace(tmp, self.checkpoint)

    def _load(self):
        if not self.checkpoint or not os.path.exists(self.checkpoint):
            return None
        with open(self.checkpoint) as f:
            return json.load(f)

    def run(self, coef0=None, S0=0, resume=True, stop_after=None):
        """Returns (coef [S*S] GPU tensor, S, log).  stop_after: number of
        frequencies to process in this call (the rest is left to a resumed
        call)."""
        import synth
        coef = coef0 if coef0 is not None else torch.zeros(0, dtype=torch.float64, device="cuda")
        S = S0
        log = []
        start = 0
        ck = self._load() if resume else None
        if ck is not None:
            S = int(ck["S"])
            coef = torch.tensor(ck["coef"], dtype=torch.float64, device="cuda")
            log = ck["log"]
            start = int(ck["j"]) + 1
        done = 0
        for step in self.schedule[start:]:
            if stop_after is not None and done >= stop_after:
                break
            t0 = time.perf_counter()
            k, band = step["k"], step["band"]
            S_new = max(S, band - 1)  # largest mode number in the band m + n <= S(k)
            coef = extend(coef, S, S_new)
            S = S_new
            s = self.solver(step["L"], step.get("p"))
            d = self.data(step)
            dnorm = float(d.abs().pow(2).sum().sqrt())
            dirs = synth.equispaced_angles(step["M"])
            th = synth.equispaced_angles(step["P"])
            entry = {k_: step[k_] for k_ in ("j", "k", "M", "P", "band", "modes", "L", "p") if k_ in step}
            entry["newton"] = []
            prev_mis = None
            for it in range(self.newton_max):
                new, info = s.gn_step(k, dirs, th, step["R"], coef, d, max_iter=self.cg_max, tol=self.cg_tol,
                                      band=band)
                rel = info["misfit"] / dnorm if dnorm > 0 else 0.0
                entry["newton"].append({"misfit_before": rel, "cg_iters": info["cg_iters"],
                                        "cg_rel_res": info["cg_rel_res"]})
                # the misfit reported is that of the current coefficients:
                # stop before accepting this step if they already meet the
                # test, or if the previous step did not lower the misfit
                if it > 0 and (rel < self.newton_tol or rel >= prev_mis):
                    entry["newton"][-1]["accepted"] = False
                    break
                coef = new
                entry["newton"][-1]["accepted"] = True
                prev_mis = rel
            torch.cuda.synchronize()
            entry["seconds"] = time.perf_counter() - t0
            log.append(entry)
            if self.checkpoint:
                self._save(step["j"], coef, S, log)
            done += 1
        return coef, S, log


class BatchForward:
    """Forward solves of many independent (q, k) problems (the uncoupled
    solves of the recursive linearization): problems on the same leaf grid
    share one batched context, so each leaf stage, merge level and top system
    runs once per group.  Problems with many directions (more than m_split)
    form their own group on a grid; within a group the direction count is
    padded to the largest one by cycling each problem's own directions
    (padded columns are computed and dropped).  Groups run concurrently, each
    on its own stream and host thread (the library releases the interpreter
    lock during its calls), so the launches of small groups overlap the work
    of large ones.  Contexts and streams are kept between calls.  streams:
    the contexts' own stream count (hps_opts.streams); by default 1 when the
    groups run concurrently (they already overlap), else 2."""

    def __init__(self, p=16, keep_derivs=False, m_split=64, concurrent=True, precision="fp64", streams=None):
        self.p = p
        self.streams = streams if streams is not None else (1 if concurrent else 2)
        self.keep_derivs = keep_derivs
        self.precision = precision
        self.m_split = m_split  # problems with more directions than this batch separately
        self.concurrent = concurrent
        self._ctx = {}

    def _solver(self, key, L, nprob):
        from . import Solver
        key = key + (nprob,)
        if key not in self._ctx:
            stream = torch.cuda.Stream() if self.concurrent else None
            self._ctx[key] = Solver(nleaf=L, p=self.p, nprob=nprob, keep_derivs=self.keep_derivs, stream=stream,
                                    precision=self.precision, streams=self.streams)
        return self._ctx[key]

    def groups(self, problems):
        """{(L, many-directions flag): problem indices}"""
        g = {}
        for i, pr in enumerate(problems):
            key = (int(pr["L"]), len(pr["dirs"]) > self.m_split)
            g.setdefault(key, []).append(i)
        return g

    def prepare(self, problems):
        """Per-wavenumber host set-up of every group (kept out of timed runs)."""
        for key, idx in self.groups(problems).items():
            self._solver(key, key[0], len(idx)).set_wavenumber([problems[i]["k"] for i in idx])

    def _run_group(self, s, problems, idx, thetas, R, ready):
        with torch.cuda.stream(s.stream):
            s.stream.wait_event(ready)
            M = max(len(problems[i]["dirs"]) for i in idx)
            dirs = np.stack([np.resize(np.asarray(problems[i]["dirs"], dtype=np.float64), M) for i in idx])
            q = torch.stack([problems[i]["q"] for i in idx]).contiguous()
            s.factor(q, [problems[i]["k"] for i in idx])
            s.solve(dirs)
            ff = s.far_field(thetas, R)
        if ff.dim() == 2:  # a group of one problem has no problem axis
            ff = ff.unsqueeze(0)
        return ff

    def run(self, problems, thetas, R):
        """problems: dicts with L, k, q (float64 GPU tensor [npde]) and dirs
        (angles).  Returns the far fields (complex128 GPU tensors [M_i, P]),
        ready for use on the caller's current stream."""
        out = [None] * len(problems)
        cur = torch.cuda.current_stream()
        ready = torch.cuda.Event()
        ready.record(cur)  # the inputs were produced on the caller's stream
        work = [(self._solver(key, key[0], len(idx)), idx) for key, idx in self.groups(problems).items()]
        if self.concurrent and len(work) > 1:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(max_workers=len(work)) as ex:
                futs = [ex.submit(self._run_group, s, problems, idx, thetas, R, ready) for s, idx in work]
                results = [f.result() for f in futs]
        else:
            results = [self._run_group(s, problems, idx, thetas, R, ready) for s, idx in work]
        for (s, idx), ff in zip(work, results):
            cur.wait_stream(s.stream)
            ff.record_stream(cur)
            for j, i in enumerate(idx):
                out[i] = ff[j, :len(problems[i]["dirs"])]
        return out
