"""Library (through the C ABI) against the oracle's stored results on larger
grids (tests/golden/parity_<case>.json, written by make_parity_goldens.py
from oracle/ only): 8 x 8, 16 x 16 and 32 x 32 leaves at k = 20, 40, 70.

These reach the code paths of the benchmark that the small cases do not:
the tournament-pivoted top inverse (outer boundary 896 and 1792 nodes) in
both column blockings, order-224/448 merge inverses, split-K top products
(1792 x 8 x 1792), the mixed-precision refinement and batched contexts.

Comparison is element by element: max |lib - oracle| / max |oracle| over
each array (far field [M, P], total field at sampled nodes, J dq [M, P],
Re J^H r at sampled nodes), <= 1e-9 in FP64 and <= 1e-8 in mixed precision;
the adjoint is also compared through dot products with seeded probe
vectors over every node."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CASES = ["L8_k20", "L16_k40", "L32_k70"]


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _load(name):
    path = os.path.join(GOLD, f"parity_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        d = json.load(f)
    c = lambda v: np.asarray(v["re"]) + 1j * np.asarray(v["im"])
    return d["case"], {"far": c(d["far"]), "u": c(d["u_at_iu"]), "jvp": c(d["jvp"]),
                       "g": np.asarray(d["vjp_at_ig"]), "dots": np.asarray(d["vjp_probe_dots"]),
                       "gnorm": d["vjp_norm"]}


def maxrel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def _check(case, ref, inp, ff, u, jv, g, tol, label):
    errs = {"far": maxrel(ff, ref["far"]), "u": maxrel(u[:, inp["iu"]].T, ref["u"]),
            "jvp": maxrel(jv, ref["jvp"]), "vjp": maxrel(g[inp["ig"]], ref["g"])}
    pn = np.linalg.norm(inp["probes"], axis=1)
    errs["vjp_dots"] = float(np.max(np.abs(inp["probes"] @ g - ref["dots"]) / (pn * ref["gnorm"])))
    print(f"{label} {case['name']}: " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()), flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)


def _run(hps, torch, case, precision="fp64"):
    s = hps.Solver(nleaf=case["L"], p=16, precision=precision)
    inp = synth.parity_inputs(s.node_coords(), case["M"], case["P"], case["seed"])
    s.factor(torch.from_numpy(inp["q"]).cuda(), case["k"])
    s.solve(synth.equispaced_angles(case["M"]))
    ff = s.far_field(synth.equispaced_angles(case["P"]), case["R"]).cpu().numpy()
    u = s.total_field().cpu().numpy()
    jv = s.jvp(torch.from_numpy(inp["dq"]).cuda()).cpu().numpy()
    g = s.vjp(torch.from_numpy(inp["r"]).cuda()).cpu().numpy()
    return s, inp, ff, u, jv, g


@pytest.mark.parametrize("name,blocking", [("L8_k20", -1), ("L16_k40", 0), ("L16_k40", 1),
                                           ("L32_k70", 0), ("L32_k70", 1)])
def test_fp64_matches_oracle_goldens(name, blocking):
    torch = _torch()
    import paper_1608_06871_amd as hps
    case, ref = _load(name)
    print(f"fp64 golden {name} blocking={blocking}", flush=True)
    hps.zinv_blocking(blocking)
    try:
        _, inp, ff, u, jv, g = _run(hps, torch, case)
    finally:
        hps.zinv_blocking(-1)
    _check(case, ref, inp, ff, u, jv, g, 1e-9, f"fp64 blocking {blocking}")


@pytest.mark.parametrize("name", ["L16_k40", "L32_k70"])
def test_mixed_matches_oracle_goldens(name):
    torch = _torch()
    import paper_1608_06871_amd as hps
    case, ref = _load(name)
    print(f"mixed golden {name}", flush=True)
    s, inp, ff, u, jv, g = _run(hps, torch, case, precision="mixed")
    st = s.stats()
    print(f"  {st['refine_iters']} corrections, residual {st['refine_residual']:.1e}", flush=True)
    _check(case, ref, inp, ff, u, jv, g, 1e-8, "mixed")


@pytest.mark.parametrize("name", CASES)
def test_batch_matches_oracle_goldens(name):
    """The golden problem as problem 1 of a two-problem batched context (the
    other problem has its own contrast and wavenumber)."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    case, ref = _load(name)
    print(f"batch golden {name}", flush=True)
    b = hps.Solver(nleaf=case["L"], p=16, nprob=2)
    xy = b.node_coords()
    inp = synth.parity_inputs(xy, case["M"], case["P"], case["seed"])
    other = synth.parity_inputs(xy, case["M"], case["P"], case["seed"] + 1000)
    ks = [0.75 * case["k"], case["k"]]
    b.factor(torch.from_numpy(np.stack([other["q"], inp["q"]])).cuda(), ks)
    b.solve(synth.equispaced_angles(case["M"]))
    ff = b.far_field(synth.equispaced_angles(case["P"]), case["R"]).cpu().numpy()[1]
    u = b.total_field().cpu().numpy()[1]
    jv = b.jvp(torch.from_numpy(np.stack([other["dq"], inp["dq"]])).cuda()).cpu().numpy()[1]
    g = b.vjp(torch.from_numpy(np.stack([other["r"], inp["r"]])).cuda()).cpu().numpy()[1]
    _check(case, ref, inp, ff, u, jv, g, 1e-9, "batch")
