"""CPU checks of the C-ABI library: it builds, loads, and exports every entry
point that include/*.h declare (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hps.h")


def _declared():
    text = "".join(open(os.path.join(ROOT, "include", f)).read()
                   for f in sorted(os.listdir(os.path.join(ROOT, "include"))) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hps_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_interface():
    names = _declared()
    for must in ("hps_create", "hps_factor", "hps_solve", "hps_far_field", "hps_jvp", "hps_vjp"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1608_06871_amd as hps
    if not os.path.exists(hps.LIB_PATH):
        pytest.skip("libhps.so not built")
    so = ctypes.CDLL(hps.LIB_PATH)
    for name in _declared():
        assert hasattr(so, name), name
    bound = {n for n, _, _ in hps.SIGNATURES}
    assert set(_declared()) == bound


def test_default_opts_and_invalid_create_on_cpu():
    import paper_1608_06871_amd as hps
    if not os.path.exists(hps.LIB_PATH):
        pytest.skip("libhps.so not built")
    L = hps.lib()
    o = hps.Opts()
    L.hps_default_opts(ctypes.byref(o))
    assert (o.x0, o.x1, o.nleaf, o.p, o.keep_derivs) == (-1.0, 1.0, 4, 16, 1)
    h = ctypes.c_void_p()
    bad = hps.Opts()
    L.hps_default_opts(ctypes.byref(bad))
    bad.nleaf = 3  # not a power of two: rejected before any device call
    assert L.hps_create(ctypes.byref(bad), ctypes.byref(h)) == hps.HPS_EINVAL
    bad.nleaf, bad.p = 4, 2
    assert L.hps_create(ctypes.byref(bad), ctypes.byref(h)) == hps.HPS_EINVAL
    bad.p, bad.x1 = 16, 3.0  # not square
    assert L.hps_create(ctypes.byref(bad), ctypes.byref(h)) == hps.HPS_EINVAL
    bad.x1, bad.exterior = 1.0, 2  # no such exterior relation
    assert L.hps_create(ctypes.byref(bad), ctypes.byref(h)) == hps.HPS_EINVAL
    for n in (0, 3):  # one or two streams only
        bad.exterior, bad.streams = 0, n
        assert L.hps_create(ctypes.byref(bad), ctypes.byref(h)) == hps.HPS_EINVAL
    assert o.exterior == 0 and o.streams == 2


def test_status_codes_match_the_header():
    """The binding's status constants equal the header's enum values."""
    import paper_1608_06871_amd as hps
    text = open(HEADER).read()
    enum = dict((n, int(v)) for n, v in re.findall(r"\b(HPS_E[A-Z]+|HPS_OK)\s*=\s*(-?\d+)", text))
    assert enum["HPS_OK"] == 0
    for name, val in enum.items():
        assert getattr(hps, name) == val, name
        assert hps._NAMES[val] == name


def test_noalloc_rejects_oversized_calls_on_the_host():
    """hps_zinv_noalloc refuses orders above 512 and workspaces beyond its
    static array before touching the device (so this runs without a GPU)."""
    import paper_1608_06871_amd as hps
    if not os.path.exists(hps.LIB_PATH):
        pytest.skip("libhps.so not built")
    L = hps.lib()
    p = ctypes.c_void_p(16)  # never dereferenced: the calls stop at the size checks
    assert L.hps_zinv_noalloc(None, 513, 1, p, p, None) == hps.HPS_EINVAL
    assert L.hps_zinv_noalloc(None, 512, 64, p, p, None) == hps.HPS_EINVAL   # 64 MiB + headers
    assert L.hps_zinv_noalloc(None, 252, 263, p, p, None) == hps.HPS_EINVAL
    assert L.hps_zinv_noalloc(None, 128, 1009, p, p, None) == hps.HPS_EINVAL
    assert L.hps_zinv_noalloc(None, -1, 1, p, p, None) == hps.HPS_EINVAL
    assert L.hps_zinv_noalloc(None, 0, 5, p, p, None) == hps.HPS_OK
    assert L.hps_zinv_noalloc(None, 16, 2, None, p, None) == hps.HPS_EINVAL
