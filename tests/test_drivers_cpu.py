"""Host logic of the drivers (no GPU): the frequency schedule of Section 4
against the columns of Table 2, and the noise model of Section 4."""
import math
import os

import numpy as np

import synth
from paper_1608_06871_amd.drivers import grid_for, leaves_for, paper_schedule

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table2_schedule.txt")


def test_schedule_reproduces_table2():
    """k_j = 1 + j/4, M = floor(2k), P = floor(8k) (Table 2's M P; the text
    says floor(4k)), band S = floor(2k) with S(S-1)/2 modes, and 2^l leaves
    from >= 6 points per wavelength on [-pi/2, pi/2]^2 (coarsest 4 x 4)."""
    tab = np.loadtxt(GOLD)
    sched = {round(s["k"], 6): s for s in paper_schedule(64.0, ppw=6.0, width=math.pi, angles_per_k=8,
                                                          min_leaves=4)}
    assert len(sched) == 253  # k = 1, 1.25, ..., 64
    for k, N, modes, M, MP in tab:
        s = sched[round(k, 6)]
        assert (15 * s["L"] + 1) ** 2 == N, k
        assert s["modes"] == modes and s["M"] == M and s["M"] * s["P"] == MP, k


def test_leaves_rule_points_per_wavelength():
    # width 2, p = 16: L = 8 gives 120 intervals; at k = 20 there are 20/pi
    # wavelengths across, i.e. 18.8 points per wavelength (L = 4: 9.4)
    assert leaves_for(20.0, 9.0) == 4 and leaves_for(20.0, 10.0) == 8 and leaves_for(20.0, 18.0) == 8 and leaves_for(20.0, 19.0) == 16
    assert leaves_for(80.0, 10.0) == 32
    assert leaves_for(0.5, 10.0, min_leaves=2) == 2


def test_grid_rule_meets_ppw_with_fewest_points():
    """grid_for: (p - 1) L >= ppw k width / (2 pi), p in [12, 20], and no
    admissible (L, p) has fewer intervals per side (brute force over the
    powers of two)."""
    for k in (1.0, 3.3, 20.0, 37.5, 80.0, 150.0):
        for ppw in (6.0, 10.0, 15.0):
            L, p = grid_for(k, ppw)
            need = ppw * k * 2.0 / (2.0 * math.pi)
            assert 12 <= p <= 20 and L & (L - 1) == 0
            assert (p - 1) * L >= need - 1e-9
            best = min((q - 1) * M for M in (2 ** i for i in range(9)) for q in range(12, 21)
                       if (q - 1) * M >= need - 1e-9)
            assert (p - 1) * L == best
            # never more points per side than the fixed-order rule
            assert (p - 1) * L <= 15 * leaves_for(k, ppw)
    assert grid_for(80.0, 10.0) == (16, 17)
    assert grid_for(20.0, 10.0) == (4, 17)


def test_schedule_with_leaf_order_per_k():
    sched = paper_schedule(10.0, ppw=10.0, p="auto")
    assert all("p" in s and 12 <= s["p"] <= 20 for s in sched)
    assert all((s["p"] - 1) * s["L"] >= 10.0 * s["k"] / math.pi - 1e-9 for s in sched)


def test_noise_model_has_the_stated_size():
    rng = np.random.default_rng(0)
    u = rng.standard_normal((5, 12)) + 1j * rng.standard_normal((5, 12))
    v = synth.add_noise(u, 0.05, 7)
    rel = np.linalg.norm(v - u, axis=1) / np.linalg.norm(u, axis=1)
    assert np.allclose(rel, 0.05, rtol=1e-13)
    assert np.array_equal(v, synth.add_noise(u, 0.05, 7))  # seeded
    assert np.array_equal(synth.add_noise(u, 0.0, 7), u)
