"""GPU parity of the HPS solver (through the C ABI) with the CPU oracle:
forward far field, total field, Frechet derivative, adjoint, sine model."""
import numpy as np
import pytest

import synth
from oracle import sine as osine
from oracle.bie import circle_points
from oracle.forward import Problem, directions

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


_CACHE = {}


def _case(L, k, M, P, seed, nbumps=5, R=2.0):
    key = (L, k, M, P, seed, nbumps, R)
    if key not in _CACHE:
        prob = Problem(L, k)
        q = synth.gaussian_bumps(prob.grid.pde_coords(), nbumps, seed)
        prob.factor(q)
        prob.solve(directions(M))
        _, th = circle_points(R, P)
        prob.set_measurement(th, R)
        _CACHE[key] = (prob, q, th)
    return _CACHE[key]


def _solver(L, **kw):
    import paper_1608_06871_amd as hps
    return hps.Solver(nleaf=L, p=16, **kw)


def test_node_coords_match_oracle():
    _torch()
    for L in (1, 2, 4):
        s = _solver(L)
        prob = Problem.__new__(Problem)
        from oracle.grid import Grid
        assert np.max(np.abs(s.node_coords() - Grid(L).pde_coords())) < 1e-15


@pytest.mark.parametrize("L,k,M,P,seed", [(1, 3.0, 3, 8, 4), (2, 5.0, 4, 16, 3), (4, 10.0, 16, 64, 1)])
def test_forward_far_field_matches_oracle(L, k, M, P, seed):
    torch = _torch()
    print(f"forward L={L} k={k} M={M} P={P} seed={seed}", flush=True)
    prob, q, th = _case(L, k, M, P, seed)
    s = _solver(L)
    s.factor(torch.from_numpy(q).cuda(), k)
    s.solve(directions(M))
    uf = s.far_field(th, 2.0).cpu().numpy()
    ref = prob.far_field()
    assert _rel(uf, ref) < 1e-9
    u = s.total_field().cpu().numpy()
    assert _rel(u, prob.u_pde().T) < 1e-9


def test_zero_contrast_gpu():
    torch = _torch()
    s = _solver(4)
    s.factor(torch.zeros(s.npde, dtype=torch.float64, device="cuda"), 10.0)
    s.solve(directions(8))
    uf = s.far_field(circle_points(2.0, 32)[1], 2.0).cpu().numpy()
    assert np.max(np.abs(uf)) < 1e-8


def test_jvp_vjp_match_oracle():
    torch = _torch()
    L, k, M, P = 2, 5.0, 4, 16
    prob, q, th = _case(L, k, M, P, 3)
    s = _solver(L)
    s.factor(torch.from_numpy(q).cuda(), k)
    s.solve(directions(M))
    s.far_field(th, 2.0)
    rng = np.random.default_rng(9)
    dq = synth.gaussian_bumps(prob.grid.pde_coords(), 3, 7) + 0.1 * rng.standard_normal(prob.grid.npde)
    jv = s.jvp(torch.from_numpy(dq).cuda()).cpu().numpy()
    assert _rel(jv, prob.jvp(dq)) < 1e-9
    r = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    g = s.vjp(torch.from_numpy(r).cuda()).cpu().numpy()
    assert _rel(g, prob.vjp(r)) < 1e-9
    # adjoint identity on the GPU results themselves
    assert abs(np.real(np.vdot(r, jv)) - dq @ g) < 1e-10 * abs(dq @ g)


def test_sine_maps_match_oracle():
    torch = _torch()
    s = _solver(4)
    xy = s.node_coords()
    rng = np.random.default_rng(1)
    for S in (1, 3, 10):
        C = rng.standard_normal((S, S))
        q = s.sine_eval(torch.from_numpy(C.ravel()).cuda()).cpu().numpy()
        assert np.max(np.abs(q - osine.evaluate(xy, C))) < 1e-12 * max(1.0, np.abs(C).sum())
        gvals = rng.standard_normal(s.npde)
        a = s.sine_adjoint(torch.from_numpy(gvals).cuda(), S).cpu().numpy().reshape(S, S)
        ref = osine.adjoint(xy, gvals, S)
        assert np.max(np.abs(a - ref)) < 1e-11 * np.max(np.abs(ref))


def test_call_order_errors():
    torch = _torch()
    import paper_1608_06871_amd as hps
    s = _solver(2)
    with pytest.raises(hps.HpsError) as e:
        s.solve([0.0])
    assert e.value.code == hps.HPS_ESTATE
    q = torch.zeros(s.npde, dtype=torch.float64, device="cuda")
    with pytest.raises(hps.HpsError) as e:
        s.factor(q, -1.0)
    assert e.value.code == hps.HPS_EINVAL


def test_nonfinite_contrast_is_reported():
    """A NaN or an infinity in q is found on the device during the factor
    (no extra synchronisation) and reported as HPS_ENONFINITE; the context
    stays usable for the next, finite contrast."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    L, k, M, P = 2, 5.0, 4, 16
    prob, q, th = _case(L, k, M, P, 3)
    s = _solver(L)
    for bad in (np.nan, np.inf):
        qb = q.copy()
        qb[17] = bad
        with pytest.raises(hps.HpsError) as e:
            s.factor(torch.from_numpy(qb).cuda(), k)
        assert e.value.code == hps.HPS_ENONFINITE
        assert s.stats()["nonfinite"] & 1
    s.factor(torch.from_numpy(q).cuda(), k)
    assert s.stats()["nonfinite"] == 0
    s.solve(directions(M))
    assert _rel(s.far_field(th, 2.0).cpu().numpy(), prob.far_field()) < 1e-9


@pytest.mark.parametrize("M", [4, 55, 56, 64])
def test_jvp_vjp_leaf_orders_match_oracle(M):
    """The leaf terms of the derivatives are formed in one of two orders by
    the direction count (fewer than the 56 edge nodes: scaled fields and
    H^H g; else scaled H and g u0^H); both against the oracle."""
    torch = _torch()
    L, k, P = 2, 5.0, 8
    print(f"jvp/vjp leaf order M={M}", flush=True)
    prob, q, th = _case(L, k, M, P, 3)
    s = _solver(L)
    s.factor(torch.from_numpy(q).cuda(), k)
    s.solve(directions(M))
    s.far_field(th, 2.0)
    rng = np.random.default_rng(M)
    dq = synth.gaussian_bumps(prob.grid.pde_coords(), 3, 7) + 0.1 * rng.standard_normal(prob.grid.npde)
    assert _rel(s.jvp(torch.from_numpy(dq).cuda()).cpu().numpy(), prob.jvp(dq)) < 1e-9
    r = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    assert _rel(s.vjp(torch.from_numpy(r).cuda()).cpu().numpy(), prob.vjp(r)) < 1e-9


@pytest.mark.parametrize("p,L,k", [(12, 2, 6.0), (13, 2, 8.0), (17, 4, 12.0), (20, 2, 9.0)])
def test_leaf_orders_of_the_grid_rule_match_oracle(p, L, k):
    """Leaf orders other than 16 (the grid rule picks p in [12, 20] per k):
    far field, total field, J dq and Re J^H r element by element against
    the oracle on the same grid."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    M, P, R = 4, 16, 2.0
    print(f"leaf order p={p} L={L} k={k}", flush=True)
    s = hps.Solver(nleaf=L, p=p)
    inp = synth.parity_inputs(s.node_coords(), M, P, seed=p)
    prob = Problem(L, k, p)
    assert np.max(np.abs(s.node_coords() - prob.grid.pde_coords())) < 1e-15
    _, th = circle_points(R, P)
    prob.set_measurement(th, R)
    prob.factor(inp["q"])
    prob.solve(directions(M))
    s.factor(torch.from_numpy(inp["q"]).cuda(), k)
    s.solve(synth.equispaced_angles(M))
    ff = s.far_field(synth.equispaced_angles(P), R).cpu().numpy()
    u = s.total_field().cpu().numpy()
    jv = s.jvp(torch.from_numpy(inp["dq"]).cuda()).cpu().numpy()
    g = s.vjp(torch.from_numpy(inp["r"]).cuda()).cpu().numpy()
    errs = {"far": _rel(ff, prob.far_field()), "u": _rel(u, prob.u_pde().T), "jvp": _rel(jv, prob.jvp(inp["dq"])),
            "vjp": _rel(g, prob.vjp(inp["r"]))}
    print("  " + ", ".join(f"{n} {e:.1e}" for n, e in errs.items()), flush=True)
    for n, e in errs.items():
        assert e <= 1e-9, (n, e)


def test_degenerate_and_empty_inputs():
    """One direction and one angle against the oracle; a zero perturbation and
    a zero residual give exactly zero; empty direction or angle lists, R <= 0
    and non-finite angles are rejected with HPS_EINVAL."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    L, k = 2, 5.0
    prob, q, _ = _case(L, k, 1, 1, 3)
    s = _solver(L)
    s.factor(torch.from_numpy(q).cuda(), k)
    s.solve(directions(1))
    _, th = circle_points(2.0, 1)
    ff = s.far_field(th, 2.0).cpu().numpy()
    assert ff.shape == (1, 1)
    assert _rel(ff, prob.far_field()) <= 1e-9
    jv = s.jvp(torch.zeros(s.npde, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert np.all(jv == 0.0)
    g = s.vjp(torch.zeros((1, 1), dtype=torch.complex128, device="cuda")).cpu().numpy()
    assert np.all(g == 0.0)
    for bad in (lambda: s.solve([]), lambda: s.far_field([], 2.0), lambda: s.far_field(th, 0.0),
                lambda: s.far_field(th, -1.0), lambda: s.solve([np.nan])):
        with pytest.raises(hps.HpsError) as e:
            bad()
        assert e.value.code == hps.HPS_EINVAL


def test_deferred_butterfly_check_redoes_factorisation_pivoted():
    """The factorisation reads its butterfly inverses' probe checks once, at
    its own synchronisation.  Forced from the host (probe tolerance 0, so
    every check fails), it must count one fallback per factorisation, redo
    the pass on the pivoted path and give exactly the always-pivoted result;
    with the default tolerance it matches the oracle golden path to 1e-9."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    L, k, M, P = 16, 40.0, 4, 16
    s = hps.Solver(nleaf=L, p=16)
    inp = synth.parity_inputs(s.node_coords(), M, P, seed=7)
    q = torch.from_numpy(inp["q"]).cuda()
    th = synth.equispaced_angles(P)

    def run():
        s.factor(q, k)
        s.solve(synth.equispaced_angles(M))
        return s.far_field(th, 2.0).cpu(), s.vjp(torch.from_numpy(inp["r"]).cuda()).cpu()

    try:
        hps.zinv_pivoting(0)
        ref = run()
        hps.zinv_pivoting(-1, 0.0)
        before = hps.zinv_pivoting_info()
        got = run()
        after = hps.zinv_pivoting_info()
        print(f"fallbacks {after['fallbacks'] - before['fallbacks']}, calls {after['calls'] - before['calls']}",
              flush=True)
        assert after["fallbacks"] == before["fallbacks"] + 1
        assert after["calls"] > before["calls"]
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    finally:
        hps.zinv_pivoting(-1, 1e-10)
    ok = run()
    assert _rel(ok[0].numpy(), ref[0].numpy()) <= 1e-9


@pytest.mark.parametrize("case", ["L32", "mixed_L32", "batch_L16"])
def test_second_stream_gives_identical_results(case):
    """hps_opts.streams = 2 (half the leaf stage and the merge levels' V, U
    products on the context's second stream) runs the same kernels on the
    same operands as streams = 1: far field, total field, jvp and vjp agree
    bit for bit (32 x 32 leaves: the leaf stage splits within the problem;
    a 2-problem batch on 16 x 16 leaves: at the problem boundary)."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    L = 16 if case == "batch_L16" else 32
    nprob = 2 if case == "batch_L16" else 1
    prec = "mixed" if case.startswith("mixed") else "fp64"
    k, M, P = 40.0, 8, 16
    print(f"streams 1 vs 2: {case}", flush=True)
    out = {}
    for ns in (1, 2):
        s = hps.Solver(nleaf=L, p=16, nprob=nprob, precision=prec, streams=ns)
        xy = s.node_coords()
        qs = [synth.parity_inputs(xy, M, P, seed=11 + b) for b in range(nprob)]
        q = torch.from_numpy(np.stack([x["q"] for x in qs]) if nprob > 1 else qs[0]["q"]).cuda()
        r = torch.from_numpy(np.stack([x["r"] for x in qs]) if nprob > 1 else qs[0]["r"]).cuda()
        dq = torch.from_numpy(np.stack([x["dq"] for x in qs]) if nprob > 1 else qs[0]["dq"]).cuda()
        s.factor(q, [k + 3.0 * b for b in range(nprob)] if nprob > 1 else k)
        s.solve(synth.equispaced_angles(M))
        ff = s.far_field(synth.equispaced_angles(P), 2.0).cpu()
        out[ns] = (ff, s.total_field().cpu(), s.jvp(dq).cpu(), s.vjp(r).cpu())
    for a, b in zip(out[1], out[2]):
        assert torch.equal(a, b)
    # the count can be changed between factorisations; others are refused
    s.set_streams(1)
    with pytest.raises(hps.HpsError) as e:
        s.set_streams(3)
    assert e.value.code == hps.HPS_EINVAL
