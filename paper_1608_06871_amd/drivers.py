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
