"""The combined-field (Burton-Miller) exterior relation on the GPU, through
the C ABI, against the oracle's combined-field problem (the same discrete
system, independent quadrature and a sparse direct solve), element by
element: far field [M, P], total field at sampled nodes, J dq and Re J^H r.

The cases include k = pi/sqrt(2), the lowest Dirichlet eigenvalue of
[-1, 1]^2, where the Green relation of the Remark in Section 2 is singular:
there the library must also match the radial reference by separation of
variables."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

K_EIG = np.pi / np.sqrt(2.0)


def maxrel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def _oracle(L, k, inp, M, P, R):
    from oracle.bie import circle_points
    from oracle.forward import Problem, directions
    prob = Problem(L, k, exterior="burton_miller")
    _, th = circle_points(R, P)
    prob.set_measurement(th, R)
    prob.factor(inp["q"])
    prob.solve(directions(M))
    return {"far": prob.far_field(), "u": prob.u_pde()[inp["iu"], :].T, "jvp": prob.jvp(inp["dq"]),
            "g": prob.vjp(inp["r"])}


def _library(hps, L, k, inp, M, P, R, precision="fp64"):
    s = hps.Solver(nleaf=L, p=16, precision=precision, exterior="burton_miller")
    s.factor(torch.from_numpy(inp["q"]).cuda(), k)
    s.solve(synth.equispaced_angles(M))
    out = {"far": s.far_field(synth.equispaced_angles(P), R).cpu().numpy(),
           "u": s.total_field().cpu().numpy()[:, inp["iu"]],
           "jvp": s.jvp(torch.from_numpy(inp["dq"]).cuda()).cpu().numpy(),
           "g": s.vjp(torch.from_numpy(inp["r"]).cuda()).cpu().numpy()}
    return s, out


@pytest.mark.parametrize("L,k,precision,tol", [(4, K_EIG, "fp64", 1e-9), (8, 20.0, "fp64", 1e-9),
                                               (8, 20.0, "mixed", 1e-8)])
def test_combined_field_matches_oracle(L, k, precision, tol):
    import paper_1608_06871_amd as hps
    M, P, R = 8, 32, 2.0
    print(f"combined field L={L} k={k:.4f} {precision}", flush=True)
    xy = hps.Solver(nleaf=L, p=16, keep_derivs=False).node_coords()
    inp = synth.parity_inputs(xy, M, P, seed=11)
    _, lib = _library(hps, L, k, inp, M, P, R, precision)
    ref = _oracle(L, k, inp, M, P, R)
    errs = {n: maxrel(lib[n], ref[n]) for n in ref}
    print("  " + ", ".join(f"{n} {e:.1e}" for n, e in errs.items()), flush=True)
    for n, e in errs.items():
        assert e <= tol, (n, e)


def test_combined_field_at_eigenvalue_matches_radial_reference():
    import paper_1608_06871_amd as hps
    from oracle.radial import scattered_on_circle
    amp, sig, d = 0.4, 0.2, 0.7
    th = synth.equispaced_angles(16)
    ref = scattered_on_circle(K_EIG, lambda r: amp * np.exp(-r * r / sig ** 2), 1.0, d, 2.0, th)
    s = hps.Solver(nleaf=8, p=16, keep_derivs=False, exterior="burton_miller")
    q = synth.radial_gaussian(s.node_coords(), amp, sig)
    s.factor(torch.from_numpy(q).cuda(), K_EIG)
    s.solve(np.array([d]))
    ff = s.far_field(th, 2.0).cpu().numpy()[0]
    err = maxrel(ff, ref)
    print(f"eigenvalue vs radial {err:.1e}", flush=True)
    assert err <= 1e-8


def test_combined_field_batch_matches_single_contexts():
    """Two problems of one batched context (one at the eigenvalue) against
    two single contexts."""
    import paper_1608_06871_amd as hps
    L, M, P, R = 4, 8, 32, 2.0
    ks = [K_EIG, 9.0]
    xy = hps.Solver(nleaf=L, p=16, keep_derivs=False).node_coords()
    inps = [synth.parity_inputs(xy, M, P, seed=21 + i) for i in range(2)]
    b = hps.Solver(nleaf=L, p=16, nprob=2, exterior="burton_miller")
    b.factor(torch.from_numpy(np.stack([i["q"] for i in inps])).cuda(), ks)
    b.solve(synth.equispaced_angles(M))
    ff = b.far_field(synth.equispaced_angles(P), R).cpu().numpy()
    g = b.vjp(torch.from_numpy(np.stack([i["r"] for i in inps])).cuda()).cpu().numpy()
    for j in range(2):
        _, one = _library(hps, L, ks[j], inps[j], M, P, R)
        e1, e2 = maxrel(ff[j], one["far"]), maxrel(g[j], one["g"])
        print(f"  problem {j}: far {e1:.1e}, vjp {e2:.1e}", flush=True)
        assert e1 <= 1e-12 and e2 <= 1e-12
