"""Writes the oracle's results for the library-vs-oracle parity cases at
larger grids (tests/golden/parity_<case>.json).  Calls only oracle/ and the
seeded input recipe synth.parity_inputs; nothing here touches the library.

Cases (Omega = [-1, 1]^2, leaves of 16 x 16 Chebyshev-Lobatto points, 5
Gaussian bumps, M = 8 equispaced directions, P = 32 equispaced angles on the
circle R = 2):
  L8_k20    8 x 8 leaves,   k = 20  (outer boundary 448 nodes)
  L16_k40  16 x 16 leaves,  k = 40  (896 nodes: the top system takes the
                                     tournament-pivoted inverse)
  L32_k70  32 x 32 leaves,  k = 70  (1792 nodes; order-448 merge inverses,
                                     split-K top products at M = 8)
Stored per case: the far field u_far [M, P] (Section 1 data), the total
field at sampled PDE nodes, the Frechet derivative J dq (Theorem 1) and the
adjoint Re(J^H r) (Theorem 2, discrete) at sampled nodes plus its dot
products with seeded probe vectors.  The oracle assembles the global sparse
system and solves it with SuperLU: about 1 min for L16_k40 and 20 min (and
~15 GB) for L32_k70 on 8 cores.

usage: python tests/golden/make_parity_goldens.py [case ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle.forward import Problem, directions  # noqa: E402

CASES = {
    "L8_k20": dict(L=8, k=20.0, M=8, P=32, R=2.0, seed=31),
    "L16_k40": dict(L=16, k=40.0, M=8, P=32, R=2.0, seed=32),
    "L32_k70": dict(L=32, k=70.0, M=8, P=32, R=2.0, seed=33),
}


def cplx(a):
    a = np.asarray(a)
    return {"re": np.real(a).tolist(), "im": np.imag(a).tolist()}


def make(name):
    c = CASES[name]
    t0 = time.perf_counter()
    prob = Problem(c["L"], c["k"])
    xy = prob.grid.pde_coords()
    inp = synth.parity_inputs(xy, c["M"], c["P"], c["seed"])
    prob.factor(inp["q"])
    prob.solve(directions(c["M"]))
    th = synth.equispaced_angles(c["P"])
    prob.set_measurement(th, c["R"])
    far = prob.far_field()
    u = prob.u_pde()[inp["iu"], :]          # [nsample, M]
    jv = prob.jvp(inp["dq"])
    g = prob.vjp(inp["r"])
    out = {"case": dict(c, name=name, p=16, nbumps=5,
                        recipe="synth.parity_inputs(xy, M, P, seed); directions and angles equispaced"),
           "far": cplx(far), "u_at_iu": cplx(u), "jvp": cplx(jv),
           "vjp_at_ig": np.asarray(g[inp["ig"]]).tolist(),
           "vjp_probe_dots": (inp["probes"] @ g).tolist(),
           "vjp_norm": float(np.linalg.norm(g)),
           "oracle_seconds": time.perf_counter() - t0}
    path = os.path.join(HERE, f"parity_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"{name}: {out['oracle_seconds']:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        make(name)
