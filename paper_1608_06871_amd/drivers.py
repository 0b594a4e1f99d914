"""Recursive linearization (the algorithm box of Section 3.4): for ascending
wavenumbers k_j, zero-extend the sine-model coefficients to the new band
S(k_j) and take Gauss-Newton steps (Section 3.3) with the library's
hps_gn_step.  Only the coefficient bookkeeping happens here."""
import numpy as np
import torch


def extend(coef, S_old, S_new):
    """Zero-extension of an [S_old, S_old] coefficient block to [S_new, S_new]
    (Section 3.4: the previous band-limited model is the initial guess)."""
    out = torch.zeros(S_new * S_new, dtype=torch.float64, device=coef.device)
    if S_old > 0:
        m = min(S_old, S_new)
        out.view(S_new, S_new)[:m, :m] = coef.view(S_old, S_old)[:m, :m]
    return out


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
    of large ones.  Contexts and streams are kept between calls."""

    def __init__(self, p=16, keep_derivs=False, m_split=64, concurrent=True):
        self.p = p
        self.keep_derivs = keep_derivs
        self.m_split = m_split  # problems with more directions than this batch separately
        self.concurrent = concurrent
        self._ctx = {}

    def _solver(self, key, L, nprob):
        from . import Solver
        key = key + (nprob,)
        if key not in self._ctx:
            stream = torch.cuda.Stream() if self.concurrent else None
            self._ctx[key] = Solver(nleaf=L, p=self.p, nprob=nprob, keep_derivs=self.keep_derivs, stream=stream)
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
