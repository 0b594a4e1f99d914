"""GPU parity of the dense building blocks (complex GEMM on MFMA, batched
Gauss-Jordan inverse) against CPU float64/complex128 references."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rand(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _colmajor(torch, a):
    # numpy [batch, rows, cols] -> torch storage [batch, cols, rows] (column-major)
    return torch.from_numpy(np.ascontiguousarray(np.swapaxes(a, 1, 2))).cuda()


def _back(t):
    return np.swapaxes(t.cpu().numpy(), 1, 2)


@pytest.mark.parametrize("M,N,K,batch", [(16, 16, 4, 1), (64, 64, 16, 2), (1, 1, 1, 1), (37, 130, 19, 3),
                                         (130, 7, 70, 2), (252, 56, 252, 5), (200, 300, 33, 1)])
@pytest.mark.parametrize("opA,opB", [(0, 0), (1, 0), (2, 0), (0, 1), (0, 2), (2, 2)])
def test_zgemm_matches_cpu(M, N, K, batch, opA, opB):
    torch = _torch()
    import paper_1608_06871_amd as hps
    print(f"zgemm M={M} N={N} K={K} batch={batch} ops={opA},{opB}", flush=True)
    rng = np.random.default_rng(M * 1000 + N + K + opA * 7 + opB)
    A = _rand(rng, (batch, M, K) if opA == 0 else (batch, K, M))
    B = _rand(rng, (batch, K, N) if opB == 0 else (batch, N, K))
    C0 = _rand(rng, (batch, M, N))
    f = {0: lambda x: x, 1: lambda x: np.swapaxes(x, 1, 2), 2: lambda x: np.conj(np.swapaxes(x, 1, 2))}
    alpha, beta = 0.7 - 0.3j, -0.5 + 0.25j
    ref = alpha * (f[opA](A) @ f[opB](B)) + beta * C0
    C = _colmajor(torch, C0)
    hps.zgemm(_colmajor(torch, A), _colmajor(torch, B), C, opA=opA, opB=opB, alpha=alpha, beta=beta)
    torch.cuda.synchronize()
    got = _back(C)
    scale = np.abs(f[opA](A)) @ np.abs(f[opB](B)) + np.abs(C0)
    assert np.max(np.abs(got - ref) / scale) < 1e-14


@pytest.mark.parametrize("M,N,K,batch,opA", [(256, 256, 7168, 1, 0), (100, 40, 3000, 3, 0), (200, 64, 1030, 2, 2),
                                             (33, 17, 5000, 1, 1)])
def test_zgemm_split_k(M, N, K, batch, opA):
    """Few output tiles and a long K: the K range is split over workgroups
    and reduced in a fixed order (same result on every call)."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    print(f"zgemm split-K M={M} N={N} K={K} batch={batch} opA={opA}", flush=True)
    rng = np.random.default_rng(K + M)
    A = _rand(rng, (batch, M, K) if opA == 0 else (batch, K, M))
    B = _rand(rng, (batch, K, N))
    C0 = _rand(rng, (batch, M, N))
    f = {0: lambda x: x, 1: lambda x: np.swapaxes(x, 1, 2), 2: lambda x: np.conj(np.swapaxes(x, 1, 2))}
    alpha, beta = 0.7 - 0.3j, -0.5 + 0.25j
    ref = alpha * (f[opA](A) @ B) + beta * C0
    outs = []
    for rep in range(2):
        C = _colmajor(torch, C0)
        hps.zgemm(_colmajor(torch, A), _colmajor(torch, B), C, opA=opA, alpha=alpha, beta=beta)
        torch.cuda.synchronize()
        outs.append(_back(C))
    scale = np.abs(f[opA](A)) @ np.abs(B) + np.abs(C0)
    assert np.max(np.abs(outs[0] - ref) / scale) < 1e-14
    assert np.array_equal(outs[0], outs[1])


def test_zgemm_beta_zero_ignores_nan():
    torch = _torch()
    import paper_1608_06871_amd as hps
    rng = np.random.default_rng(5)
    A, B = _rand(rng, (1, 20, 9)), _rand(rng, (1, 9, 11))
    C = torch.full((1, 11, 20), float("nan"), dtype=torch.complex128, device="cuda")
    hps.zgemm(_colmajor(torch, A), _colmajor(torch, B), C)
    assert np.allclose(_back(C), A @ B, atol=1e-13)


@pytest.mark.parametrize("n,batch", [(1, 3), (5, 4), (14, 7), (33, 2), (64, 3), (100, 2), (252, 3),
                                     (300, 1), (513, 1), (700, 1), (1100, 2)])
def test_zinv_matches_numpy(n, batch):
    torch = _torch()
    import paper_1608_06871_amd as hps
    print(f"zinv n={n} batch={batch}", flush=True)
    rng = np.random.default_rng(n + batch)
    A = _rand(rng, (batch, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[None]
    # force pivoting: a tiny leading entry
    A[:, 0, 0] = 1e-12
    inv = _back(hps.zinv(_colmajor(torch, A)))
    torch.cuda.synchronize()
    ref = np.linalg.inv(A)
    for b in range(batch):
        cond = np.linalg.cond(A[b])
        assert np.max(np.abs(inv[b] - ref[b])) < 1e-13 * cond * np.max(np.abs(ref[b]))
        assert np.max(np.abs(inv[b] @ A[b] - np.eye(n))) < 1e-12 * cond


def test_zinv_reports_singular():
    torch = _torch()
    import paper_1608_06871_amd as hps
    A = np.zeros((2, 6, 6), dtype=np.complex128)
    A[0] = np.eye(6)
    with pytest.raises(hps.HpsError) as e:
        hps.zinv(_colmajor(torch, A))
    assert e.value.code == hps.HPS_ESINGULAR


def test_zinv_large_multilevel_tournament():
    """n = 4200 needs more candidate sets than one reduction merges (the
    multi-level tournament path): inv A = I to rounding, checked with the
    library's own GEMM."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    n = 4200
    rng = np.random.default_rng(n)
    A = _rand(rng, (1, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[None]
    Ag = _colmajor(torch, A)
    inv = hps.zinv(Ag.clone())
    prod = hps.zgemm(inv, Ag)
    err = np.max(np.abs(_back(prod)[0] - np.eye(n)))
    print(f"zinv n={n}: max |inv A - I| = {err:.2e}", flush=True)
    assert err < 1e-11


@pytest.mark.parametrize("n,batch", [(513, 1), (1100, 2), (4200, 1)])
@pytest.mark.parametrize("mode", [0, 1])
def test_zinv_blockings_agree(n, batch, mode):
    """Both column blockings of the orders above 512 (recursive; right-looking
    with look-ahead, whose last panel is partial for 513 and 1100) give
    inv A = I to rounding; 4200 also takes the multi-level tournament."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    print(f"zinv n={n} batch={batch} blocking={mode}", flush=True)
    rng = np.random.default_rng(n + 7 * batch)
    A = _rand(rng, (batch, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[None]
    A[:, 0, 0] = 1e-12
    Ag = _colmajor(torch, A)
    hps.zinv_blocking(mode)
    try:
        inv = hps.zinv(Ag.clone())
    finally:
        hps.zinv_blocking(-1)
    prod = _back(hps.zgemm(inv, Ag))
    for b in range(batch):
        err = np.max(np.abs(prod[b] - np.eye(n)))
        assert err < 1e-11, (b, err)


@pytest.mark.parametrize("n", [224, 320, 448, 452])
@pytest.mark.parametrize("mode", [0, 1])
def test_zinv_butterfly_blockings_agree(n, mode):
    """Butterfly-transformed orders from 224 up to the register-panel limit
    take the look-ahead with wide pivot-free panels under blocking 1 (and the
    default rule) and the recursive 32-column panels under 0: both give
    inv A = I to rounding with no fallback to the pivoted path; 452 ends with
    a 4-column panel."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    batch = 2
    print(f"zinv butterfly n={n} blocking={mode}", flush=True)
    rng = np.random.default_rng(n + 11 * mode)
    A = _rand(rng, (batch, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[None]
    Ag = _colmajor(torch, A)
    before = hps.zinv_pivoting_info()
    hps.zinv_blocking(mode)
    try:
        inv = hps.zinv(Ag.clone())
    finally:
        hps.zinv_blocking(-1)
    after = hps.zinv_pivoting_info()
    assert after["calls"] == before["calls"] + 1 and after["fallbacks"] == before["fallbacks"]
    prod = _back(hps.zgemm(inv, Ag))
    for b in range(batch):
        err = np.max(np.abs(prod[b] - np.eye(n)))
        assert err < 1e-11, (b, err)


@pytest.mark.parametrize("mode", [0, 1])
def test_zinv_reports_singular_tournament(mode):
    """A zero column in an order-700 matrix (tournament path; the zero pivot is
    met in the last reduction of its panel) is reported as singular by both
    column blockings."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    n = 700
    print(f"zinv singular n={n} blocking={mode}", flush=True)
    rng = np.random.default_rng(11)
    A = _rand(rng, (1, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[None]
    A[:, :, 37] = 0.0
    hps.zinv_blocking(mode)
    try:
        with pytest.raises(hps.HpsError) as e:
            hps.zinv(_colmajor(torch, A))
    finally:
        hps.zinv_blocking(-1)
    assert e.value.code == hps.HPS_ESINGULAR


@pytest.mark.parametrize("n", [64, 600])
def test_zinv_equal_magnitudes(n):
    """Every entry of a Fourier matrix has the same magnitude, so every pivot
    search is a tie (broken towards the lowest row); the inverse is exact up
    to rounding (the matrix is unitary up to scale)."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    j = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(j, j) / n)[None]
    inv = _back(hps.zinv(_colmajor(torch, F)))[0]
    ref = np.conj(F[0]).T / n
    assert np.max(np.abs(inv - ref)) < 1e-13


@pytest.mark.parametrize("n", [40, 700])
def test_zinv_nan_entry_propagates(n):
    """A NaN entry ranks as the largest pivot candidate: the call completes and
    the NaN reaches the inverse instead of being hidden."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    rng = np.random.default_rng(n)
    A = _rand(rng, (1, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[None]
    A[0, n // 3, 0] = np.nan
    inv = _back(hps.zinv(_colmajor(torch, A)))
    torch.cuda.synchronize()
    assert np.isnan(inv).any()


@pytest.mark.parametrize("n", [252, 700])
def test_zinv_row_scaled_keeps_accuracy(n):
    """Rows scaled by 1e6 (like the PDE rows of a small leaf next to its
    impedance rows): the inverse keeps the accuracy of the unscaled matrix
    (row scaling only rescales the columns of the inverse)."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    rng = np.random.default_rng(n)
    B = _rand(rng, (1, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[None]
    d = np.where(np.arange(n) % 2 == 0, 1e6, 1.0)
    A = d[None, :, None] * B
    inv = _back(hps.zinv(_colmajor(torch, A)))[0]
    ref = np.linalg.inv(B[0]) / d[None, :]
    cond = np.linalg.cond(B[0])
    # compare column by column relative to each column's scale
    err = np.max(np.abs(inv - ref), axis=0) / np.max(np.abs(ref), axis=0)
    assert np.max(err) < 1e-13 * cond


# 3M tile variants (tile shape, K step, waves per SIMD, one or two LDS buffers)
VARIANTS_3M = [12, 8, 11, 1, 10, 4, 9, 13, 14, 15, 16, 17, 18]


def test_gemm_tile_variants_agree_bitwise():
    """Every 3M tile variant accumulates the products of an output element in
    the same order, so all of them, and the autotuner's choice, give the same
    bits (the autotuner relies on this)."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    rng = np.random.default_rng(11)
    M, N, K, batch = 130, 70, 90, 2
    A = _colmajor(torch, _rand(rng, (batch, M, K)))
    B = _colmajor(torch, _rand(rng, (batch, K, N)))
    C0 = _colmajor(torch, _rand(rng, (batch, M, N)))
    beta = 0.5 + 0.25j
    outs = []
    try:
        for v in VARIANTS_3M:
            hps.gemm_tuning(0, v)
            C = C0.clone()
            hps.zgemm(A, B, C, alpha=1.0 - 2.0j, beta=beta)
            outs.append(C.cpu())
        hps.gemm_tuning(1, -1)
        n0 = hps.gemm_tuning_info()["shapes_tuned"]
        C = C0.clone()
        hps.zgemm(A, B, C, alpha=1.0 - 2.0j, beta=beta)
        tuned = C.cpu()
        assert hps.gemm_tuning_info()["shapes_tuned"] == n0 + 1
        C = C0.clone()
        hps.zgemm(A, B, C, alpha=1.0 - 2.0j, beta=beta)  # the tuned shape again
        again = C.cpu()
    finally:
        hps.gemm_tuning(0, -1)
    for v, o in zip(VARIANTS_3M, outs):
        assert torch.equal(o, outs[0]), f"variant {v}"
    assert torch.equal(tuned, outs[0]) and torch.equal(again, outs[0])
    ref = np.einsum("bmk,bkn->bmn", _back(A), _back(B)) * (1.0 - 2.0j) + beta * _back(C0)
    assert np.max(np.abs(_back(outs[0]) - ref)) < 1e-12 * np.max(np.abs(ref))


def test_autotuned_solver_gives_identical_results():
    """A factorisation and solve with GEMM autotuning on (every shape tuned on
    its first call, the output saved and restored around the trials) gives the
    same far field, bit for bit, as with the fixed tile rules."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    import synth
    L, k, M, P = 4, 10.0, 16, 32
    s = hps.Solver(nleaf=L, p=16, keep_derivs=False)
    q = torch.from_numpy(synth.gaussian_bumps(s.node_coords(), 5, 1, amp=(0.1, 0.3), width=0.15)).cuda()
    dirs, th = synth.equispaced_angles(M), synth.equispaced_angles(P)
    s.factor(q, k)
    s.solve(dirs)
    ref = s.far_field(th, 2.0).cpu()
    try:
        hps.gemm_tuning(1, -1)
        s.factor(q, k)
        s.solve(dirs)
        tuned = s.far_field(th, 2.0).cpu()
    finally:
        hps.gemm_tuning(0, -1)
    assert hps.gemm_tuning_info()["shapes_tuned"] > 0
    assert torch.equal(tuned, ref)


def test_autotuned_lookahead_inverse_is_bitwise_identical():
    """Autotuning inside the look-ahead inverse (order 1100, two matrices):
    the two streams update disjoint column ranges of the same matrices, and
    each tuning call saves and restores only its own output block, so the
    result equals the untuned one bit for bit."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    n, batch = 1100, 2
    print(f"zinv tuned look-ahead n={n} batch={batch}", flush=True)
    rng = np.random.default_rng(1234)
    A = _rand(rng, (batch, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[None]
    Ag = _colmajor(torch, A)
    hps.zinv_blocking(1)
    try:
        ref = hps.zinv(Ag.clone())
        hps.gemm_tuning(1, -1)
        tuned = hps.zinv(Ag.clone())
        again = hps.zinv(Ag.clone())  # tuned shapes reused
    finally:
        hps.gemm_tuning(0, -1)
        hps.zinv_blocking(-1)
    torch.cuda.synchronize()
    assert torch.equal(tuned, ref) and torch.equal(again, ref)


@pytest.mark.parametrize("n,batch,mode", [(8, 3, 1), (64, 2, 1), (100, 3, 1), (252, 2, 1), (516, 1, -1),
                                          (700, 2, -1), (1100, 1, -1), (700, 2, 0)])
@pytest.mark.parametrize("blocking", [0, 1])
def test_zinv_butterfly_path_matches_numpy(n, batch, mode, blocking):
    """Random butterfly transform + pivot-free elimination (mode 1 forces it
    at small orders; -1 is the default rule, which takes it above 512), in
    both column blockings, against numpy; a tiny leading entry would stop a
    plain pivot-free elimination."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    print(f"zinv butterfly n={n} batch={batch} mode={mode} blocking={blocking}", flush=True)
    rng = np.random.default_rng(n + 31 * batch)
    A = _rand(rng, (batch, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[None]
    A[:, 0, 0] = 1e-12
    before = hps.zinv_pivoting_info()
    hps.zinv_pivoting(mode)
    hps.zinv_blocking(blocking)
    try:
        inv = _back(hps.zinv(_colmajor(torch, A)))
    finally:
        hps.zinv_pivoting(-1)
        hps.zinv_blocking(-1)
    after = hps.zinv_pivoting_info()
    took = after["calls"] - before["calls"]
    assert took == (0 if (mode == 0 or (mode == -1 and n < 224)) else 1)
    assert after["fallbacks"] == before["fallbacks"]
    ref = np.linalg.inv(A)
    for b in range(batch):
        cond = np.linalg.cond(A[b])
        assert np.max(np.abs(inv[b] - ref[b])) < 1e-13 * cond * np.max(np.abs(ref[b]))


def test_zinv_butterfly_fallback_forced_from_host():
    """A probe tolerance of 0 fails every check: the batch is inverted again
    with pivoting, which still gives the inverse, and the fallback is counted."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    n = 600
    rng = np.random.default_rng(3)
    A = _rand(rng, (2, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[None]
    before = hps.zinv_pivoting_info()
    hps.zinv_pivoting(-1, 0.0)
    try:
        inv = _back(hps.zinv(_colmajor(torch, A)))
    finally:
        hps.zinv_pivoting(-1, 1e-10)
    after = hps.zinv_pivoting_info()
    assert after["fallbacks"] == before["fallbacks"] + 1
    ref = np.linalg.inv(A)
    assert np.max(np.abs(inv - ref)) < 1e-11 * np.max(np.abs(ref))


def test_zinv_butterfly_singular_falls_back_and_reports():
    """An exactly singular order-700 matrix: the butterfly path's check fails,
    the pivoted fallback meets the zero pivot and reports it."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    n = 700
    rng = np.random.default_rng(11)
    A = _rand(rng, (1, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[None]
    A[:, :, 37] = 0.0
    with pytest.raises(hps.HpsError) as e:
        hps.zinv(_colmajor(torch, A))
    assert e.value.code == hps.HPS_ESINGULAR


@pytest.mark.parametrize("M,N,K,batch", [(2000, 16, 4000, 1), (100, 5, 3000, 3), (28, 16, 84, 50), (1, 1, 2000, 2),
                                         (130, 9, 17, 4), (700, 3, 1024, 2), (64, 16, 1, 1)])
def test_zgemm_few_columns_matches_cpu(M, N, K, batch):
    """Products with at most 16 columns (the sweeps with few right-hand
    sides; long K is split into thin slices reduced in a fixed order):
    against complex128 on the CPU, and the same bits on a second call."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    print(f"zgemm few columns M={M} N={N} K={K} batch={batch}", flush=True)
    rng = np.random.default_rng(M + 7 * N + K)
    A, B, C0 = _rand(rng, (batch, M, K)), _rand(rng, (batch, K, N)), _rand(rng, (batch, M, N))
    alpha, beta = 0.7 - 0.3j, -0.5 + 0.25j
    ref = alpha * (A @ B) + beta * C0
    outs = []
    for rep in range(2):
        C = _colmajor(torch, C0)
        hps.zgemm(_colmajor(torch, A), _colmajor(torch, B), C, alpha=alpha, beta=beta)
        torch.cuda.synchronize()
        outs.append(_back(C))
    scale = np.abs(A) @ np.abs(B) + np.abs(C0)
    assert np.max(np.abs(outs[0] - ref) / scale) < 1e-14
    assert np.array_equal(outs[0], outs[1])
