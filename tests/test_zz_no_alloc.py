"""The allocation-free inverse hps_zinv_noalloc (static device scratch array)
against the allocating hps_zinv, through the C ABI: two calls in a row, the
second smaller, synchronous and asynchronous status, and the size limit."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _mats(torch, rng, n, batch):
    a = rng.standard_normal((batch, n, n)) + 1j * rng.standard_normal((batch, n, n))
    a += 2.0 * np.sqrt(n) * np.eye(n)[None]  # moderate condition numbers
    return a, torch.from_numpy(np.ascontiguousarray(np.swapaxes(a, 1, 2))).cuda()


def _inv_ref(hps, torch, A):
    return hps.zinv(A.clone())


@pytest.mark.parametrize("shapes", [((300, 40), (100, 3)), ((512, 20), (252, 64))])
def test_noalloc_matches_zinv_two_calls(shapes):
    torch = _torch()
    import paper_1608_06871_amd as hps
    rng = np.random.default_rng(sum(n * b for n, b in shapes))
    for n, batch in shapes:  # second call smaller than the first
        print(f"zinv_noalloc n={n} batch={batch}", flush=True)
        a, A = _mats(torch, rng, n, batch)
        ref = _inv_ref(hps, torch, A)
        got = hps.zinv_noalloc(A.clone())
        torch.cuda.synchronize()
        d = (got - ref).abs().max().item() / ref.abs().max().item()
        assert d <= 1e-13, d
        # and an inverse in its own right (residual against the matrix)
        inv = np.swapaxes(got.cpu().numpy(), 1, 2)
        res = max(np.max(np.abs(a[b] @ inv[b] - np.eye(n))) for b in range(min(batch, 3)))
        assert res < 1e-10


def test_noalloc_async_status_and_singular():
    torch = _torch()
    import paper_1608_06871_amd as hps
    rng = np.random.default_rng(7)
    _, A = _mats(torch, rng, 64, 4)
    st = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    hps.zinv_noalloc(A.clone(), status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    # an exactly singular matrix in the batch: a zero column
    S = A.clone()
    S[2, 7, :] = 0.0  # column 7 of matrix 2 (column-major storage)
    hps.zinv_noalloc(S.clone(), status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 1
    with pytest.raises(hps.HpsError) as e:
        hps.zinv_noalloc(S.clone())
    assert e.value.code == hps.HPS_ESINGULAR
    # the next call starts from a cleared status
    hps.zinv_noalloc(A.clone(), status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0


def test_noalloc_rejects_sizes_beyond_the_array():
    torch = _torch()
    import paper_1608_06871_amd as hps
    L = hps.lib()
    dummy = torch.zeros(1, dtype=torch.complex128, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # order above 512, and a batch whose workspace exceeds 64 MiB: both
    # rejected on the host before any launch
    assert L.hps_zinv_noalloc(st, 513, 1, p, p, None) == hps.HPS_EINVAL
    assert L.hps_zinv_noalloc(st, 512, 4096, p, p, None) == hps.HPS_EINVAL
    assert L.hps_zinv_noalloc(st, 0, 4, p, p, None) == hps.HPS_OK
