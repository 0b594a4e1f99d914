"""The paper-scale recursive linearization driver (algorithm box of Section
3.4, protocol of Section 4) through the C ABI against the oracle, its
checkpoint/resume, and the data generator on another discretisation."""
import numpy as np
import pytest

import synth
from oracle import gn as ogn
from oracle import sine as osine
from oracle.forward import Problem
from oracle.grid import Grid

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _qtrue(xy):
    return synth.gaussian_bumps(xy, 3, 5, amp=(0.1, 0.3), width=0.3)


def _oracle_data(sched, L=4):
    """Far-field data of the true contrast from the oracle on a finer grid
    (a different discretisation than the inversion's)."""
    out = []
    for st in sched:
        prob = Problem(L, st["k"])
        prob.set_measurement(synth.equispaced_angles(st["P"]), st["R"])
        prob.factor(_qtrue(prob.grid.pde_coords()))
        prob.solve(synth.equispaced_angles(st["M"]))
        out.append(np.ascontiguousarray(prob.far_field()))
    return out


def test_paper_schedule_matches_oracle_first_frequencies():
    """k = 1, 1.25, ..., 2.75 (M = floor 2k, P = floor 4k, R = 20, band
    m + n <= floor 2k) on a fixed 2 x 2-leaf grid, one Newton step per k from
    the projection q_1 onto the modes (1,1), (1,2), (2,1); CG to 1e-14 on
    the GPU against the oracle's dense least squares with the same band."""
    torch = _torch()
    from paper_1608_06871_amd.drivers import RecursiveLinearization, initial_projection, paper_schedule
    sched = paper_schedule(2.75, leaves=2)
    assert len(sched) == 8
    data = _oracle_data(sched)
    # oracle recursion
    xy = Grid(2).pde_coords()
    q2 = _qtrue(xy)
    E = osine.basis(xy, 2)
    idx = [0, 1, 2]  # (1,1), (1,2), (2,1) in the [S, S] = [2, 2] layout
    c, *_ = np.linalg.lstsq(E[:, idx], q2, rcond=None)
    C = np.zeros((2, 2))
    C.ravel()[idx] = c
    C0 = C.copy()
    S = 2
    for st, d in zip(sched, data):
        Sn = max(S, st["band"] - 1)
        Cn = np.zeros((Sn, Sn))
        Cn[:S, :S] = C
        C, S = Cn, Sn
        C, _, _, _ = ogn.gauss_newton_step(2, st["k"], C, d, synth.equispaced_angles(st["M"]), st["P"], st["R"],
                                           band=st["band"])
    # library recursion
    rl = RecursiveLinearization(sched, lambda st: torch.from_numpy(data[st["j"]]).cuda(), newton_max=1,
                                cg_tol=1e-14, cg_max=500)
    coef0 = initial_projection(rl.solver(2), torch.from_numpy(q2).cuda(), S=2)
    assert np.max(np.abs(coef0.cpu().numpy().reshape(2, 2) - C0)) < 1e-12 * np.max(np.abs(C0))
    coef, Sg, log = rl.run(coef0, S0=2, resume=False)
    got = coef.cpu().numpy().reshape(Sg, Sg)
    print("coefficients per k:", [e["newton"][0]["cg_iters"] for e in log], flush=True)
    assert Sg == S
    err = np.max(np.abs(got - C)) / np.max(np.abs(C))
    print(f"recursive linearization vs oracle: {err:.2e}", flush=True)
    assert err < 1e-8
    # coefficients outside the band of the last frequency were never updated
    keep = ogn.band_mask(S, sched[-1]["band"])
    assert np.all(got[~keep] == 0.0)


def test_checkpoint_resume_equals_one_run(tmp_path):
    torch = _torch()
    from paper_1608_06871_amd.drivers import RecursiveLinearization, paper_schedule
    sched = paper_schedule(2.5, leaves=2)
    data = _oracle_data(sched, L=2)
    get = lambda st: torch.from_numpy(data[st["j"]]).cuda()
    full, S1, _ = RecursiveLinearization(sched, get, newton_max=2, newton_tol=1e-3).run(resume=False)
    ck = str(tmp_path / "rl.json")
    a = RecursiveLinearization(sched, get, newton_max=2, newton_tol=1e-3, checkpoint=ck)
    a.run(resume=True, stop_after=3)
    b = RecursiveLinearization(sched, get, newton_max=2, newton_tol=1e-3, checkpoint=ck)
    part, S2, log = b.run(resume=True)
    assert S1 == S2 and len(log) == len(sched)
    assert torch.equal(full, part)


def test_data_generator_p20_matches_oracle():
    """The data generator's discretisation (20 x 20 points per leaf) against
    the oracle at the same order, with and without the noise model."""
    torch = _torch()
    from paper_1608_06871_amd.drivers import DataGenerator
    st = {"j": 0, "k": 6.0, "M": 4, "P": 10, "R": 20.0}
    gen = DataGenerator(_qtrue, p=20, ppw=15.0, min_leaves=2)
    got = gen(st).cpu().numpy()
    L = gen._ctx and list(gen._ctx)[0]
    prob = Problem(L, st["k"], p=20)
    prob.set_measurement(synth.equispaced_angles(st["P"]), st["R"])
    prob.factor(_qtrue(prob.grid.pde_coords()))
    prob.solve(synth.equispaced_angles(st["M"]))
    ref = prob.far_field()
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))
    noisy = DataGenerator(_qtrue, p=20, ppw=15.0, delta=0.05, seed=3, min_leaves=2)(st).cpu().numpy()
    rel = np.linalg.norm(noisy - got, axis=1) / np.linalg.norm(got, axis=1)
    assert np.allclose(rel, 0.05, rtol=1e-9)
