"""Python binding of libhps, the MI355X HPS/ItI Helmholtz scattering library.

Argument marshalling only: every computation runs in the HIP kernels behind
the C ABI of include/hps.h and include/hps_blocks.h.  Device arrays are torch tensors on the GPU
(float64 / complex128, contiguous); the library enqueues on the stream given
at construction (default: torch's current stream).  If libhps.so is missing
the first call raises: there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhps.so")
_LIB = None

HPS_OK, HPS_EINVAL, HPS_ENOMEM, HPS_EDEVICE, HPS_ESTATE, HPS_ESINGULAR, HPS_ENOCONV, HPS_ENONFINITE = \
    0, -1, -2, -3, -4, -5, -6, -7
_NAMES = {0: "HPS_OK", -1: "HPS_EINVAL", -2: "HPS_ENOMEM", -3: "HPS_EDEVICE", -4: "HPS_ESTATE",
          -5: "HPS_ESINGULAR", -6: "HPS_ENOCONV", -7: "HPS_ENONFINITE"}


class HpsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double), ("nleaf", ctypes.c_int), ("p", ctypes.c_int),
                ("eta_scale", ctypes.c_double), ("keep_derivs", ctypes.c_int),
                ("precision", ctypes.c_int), ("host_threads", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("nprob", ctypes.c_int), ("max_refine", ctypes.c_int),
                ("refine_tol", ctypes.c_double), ("fallback_fp64", ctypes.c_int), ("exterior", ctypes.c_int),
                ("streams", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("t_wavenumber_ms", ctypes.c_double), ("t_factor_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("t_far_field_ms", ctypes.c_double),
                ("t_jvp_ms", ctypes.c_double), ("t_vjp_ms", ctypes.c_double),
                ("t_leaf_ms", ctypes.c_double), ("t_merge_ms", ctypes.c_double), ("t_top_ms", ctypes.c_double),
                ("device_bytes", ctypes.c_int64), ("ndir", ctypes.c_int), ("singular", ctypes.c_int),
                ("nonfinite", ctypes.c_int), ("refine_iters", ctypes.c_int), ("refine_residual", ctypes.c_double),
                ("refine_fallback", ctypes.c_int), ("cg_graph_iters", ctypes.c_int)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


# (name, restype, argtypes) of every exported entry point
_P, _D, _I, _L = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64
SIGNATURES = [
    ("hps_default_opts", None, [ctypes.POINTER(Opts)]),
    ("hps_create", _I, [ctypes.POINTER(Opts), ctypes.POINTER(_P)]),
    ("hps_destroy", None, [_P]),
    ("hps_last_error", ctypes.c_char_p, [_P]),
    ("hps_num_nodes", _L, [_P]),
    ("hps_num_boundary_nodes", _L, [_P]),
    ("hps_node_coords", _I, [_P, _P]),
    ("hps_set_wavenumber", _I, [_P, _D]),
    ("hps_set_wavenumbers", _I, [_P, _P]),
    ("hps_set_streams", _I, [_P, _I]),
    ("hps_factor", _I, [_P, _P, _D]),
    ("hps_factor_batch", _I, [_P, _P, _P]),
    ("hps_solve", _I, [_P, _I, _P]),
    ("hps_solve_batch", _I, [_P, _I, _P]),
    ("hps_far_field", _I, [_P, _I, _P, _D, _P]),
    ("hps_total_field", _I, [_P, _P]),
    ("hps_jvp", _I, [_P, _P, _P]),
    ("hps_vjp", _I, [_P, _P, _P]),
    ("hps_sine_eval", _I, [_P, _I, _P, _P]),
    ("hps_sine_adjoint", _I, [_P, _I, _P, _P]),
    ("hps_get_stats", _I, [_P, ctypes.POINTER(Stats)]),
    ("hps_gn_step", _I, [_P, _D, _I, _P, _I, _P, _D, _I, _I, _P, _P, _I, _D, _P, _P, _P, _P]),
    ("hps_boundary_operators", _I, [ctypes.POINTER(Opts), _D, _P, _P, _P]),
    ("hps_combined_field_operators", _I, [ctypes.POINTER(Opts), _D, _P, _P]),
    ("hps_zgemm", _I, [_P, _I, _I, _I, _I, _I, _P, _P, _L, _L, _P, _L, _L, _P, _P, _L, _L, _I]),
    ("hps_zinv", _I, [_P, _I, _I, _P, _P]),
    ("hps_zinv_noalloc", _I, [_P, _I, _I, _P, _P, _P]),
    ("hps_gemm_tuning", _I, [_I, _I]),
    ("hps_zinv_blocking", _I, [_I]),
    ("hps_zinv_pivoting", _I, [_I, _D]),
    ("hps_zinv_pivoting_info", _I, [_P, _P, _P]),
    ("hps_gemm_tuning_info", _I, [_P, _P, _P]),
    ("hps_profile_start", _I, []),
    ("hps_profile_stop", _I, [ctypes.POINTER(KernelStat), _I]),
]


def lib():
    """Loads libhps.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1608_06871_amd.build` (no CPU fallback exists)")
        so = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(so, name)
            f.restype = res
            f.argtypes = args
        _LIB = so
    return _LIB


def _torch():
    import torch
    return torch


def _dev(t, dtype, numel=None, name="array"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


# exterior relations of hps_opts.exterior
EXTERIORS = {"green": 0, "burton_miller": 1}


class Solver:
    """One HPS context: geometry fixed at construction; factor/solve/... as in
    the C ABI (include/hps.h).  With nprob > 1 the context holds a batch of
    independent problems on the same grid: per-problem arrays get a leading
    problem axis (q [nprob, npde], far field [nprob, ndir, ntheta], ...).
    streams: 2 lets hps_factor overlap work on a second stream of the
    context, 1 keeps everything on `stream` (hps_opts.streams)."""

    def __init__(self, nleaf=4, p=16, box=(-1.0, 1.0, -1.0, 1.0), eta_scale=1.0,
                 keep_derivs=True, host_threads=0, stream=None, nprob=1, precision="fp64",
                 max_refine=None, refine_tol=None, fallback_fp64=None, exterior="green", streams=2):
        torch = _torch()
        L = lib()
        o = Opts()
        L.hps_default_opts(ctypes.byref(o))
        o.x0, o.x1, o.y0, o.y1 = map(float, box)
        o.nleaf, o.p = int(nleaf), int(p)
        o.eta_scale = float(eta_scale)
        o.keep_derivs = 1 if keep_derivs else 0
        o.host_threads = int(host_threads)
        o.nprob = int(nprob)
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        o.precision = 0 if precision == "fp64" else 1
        if max_refine is not None:
            o.max_refine = int(max_refine)
        if refine_tol is not None:
            o.refine_tol = float(refine_tol)
        if fallback_fp64 is not None:
            o.fallback_fp64 = 1 if fallback_fp64 else 0
        if exterior not in EXTERIORS:
            raise ValueError(f"exterior must be one of {sorted(EXTERIORS)}")
        o.exterior = EXTERIORS[exterior]
        self.exterior = exterior
        o.streams = int(streams)
        self.precision = precision
        self.max_refine, self.refine_tol = o.max_refine, o.refine_tol
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        o.stream = ctypes.c_void_p(stream.cuda_stream)
        h = ctypes.c_void_p()
        rc = L.hps_create(ctypes.byref(o), ctypes.byref(h))
        if rc != HPS_OK:
            raise HpsError(rc, "hps_create failed (invalid options?)")
        self._h = h
        self.nleaf, self.p, self.box = o.nleaf, o.p, (o.x0, o.x1, o.y0, o.y1)
        self.nprob = o.nprob
        self.npde = int(L.hps_num_nodes(h))
        self.nb = int(L.hps_num_boundary_nodes(h))
        self.ndir = 0
        self.ntheta = 0
        self.generation = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            _LIB.hps_destroy(h)
            self._h = None

    def _check(self, rc, what):
        if rc != HPS_OK:
            msg = lib().hps_last_error(self._h)
            raise HpsError(rc, f"{what}: {msg.decode() if msg else ''}")

    def node_coords(self):
        """[npde, 2] numpy array of PDE-node coordinates (interface order)."""
        xy = np.zeros((self.npde, 2), dtype=np.float64)
        self._check(lib().hps_node_coords(self._h, xy.ctypes.data_as(ctypes.c_void_p)), "node_coords")
        return xy

    def _shape(self, *dims):
        return tuple(dims) if self.nprob == 1 else (self.nprob,) + tuple(dims)

    def set_wavenumber(self, k):
        """k: one wavenumber for every problem, or one per problem."""
        kv = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.float64), (self.nprob,)))
        self._check(lib().hps_set_wavenumbers(self._h, kv.ctypes.data_as(ctypes.c_void_p)), "set_wavenumber")

    def set_streams(self, streams):
        """hps_set_streams: 1 or 2 streams for the next factorisations."""
        self._check(lib().hps_set_streams(self._h, int(streams)), "set_streams")

    def factor(self, q, k):
        """q: [npde] (or [nprob, npde]) float64 GPU tensor; k: scalar or one per problem."""
        torch = _torch()
        self._q = q
        qp = _dev(q, torch.float64, self.nprob * self.npde, "q")
        if np.ndim(k) == 0:
            self._check(lib().hps_factor(self._h, qp, float(k)), "factor")
            self.k = float(k)
        else:
            kv = np.ascontiguousarray(np.asarray(k, dtype=np.float64).ravel())
            if kv.size != self.nprob:
                raise ValueError(f"need {self.nprob} wavenumbers, got {kv.size}")
            self._check(lib().hps_factor_batch(self._h, qp, kv.ctypes.data_as(ctypes.c_void_p)), "factor")
            self.k = kv.copy()
        self.generation += 1

    def solve(self, angles):
        """angles: [ndir] (the same for every problem) or [nprob, ndir]."""
        a = np.asarray(angles, dtype=np.float64)
        if a.ndim <= 1:
            a = np.ascontiguousarray(a.ravel())
            rc = lib().hps_solve(self._h, int(a.size), a.ctypes.data_as(ctypes.c_void_p))
            nd = int(a.size)
        else:
            if a.shape[0] != self.nprob:
                raise ValueError(f"need directions for {self.nprob} problems, got {a.shape[0]}")
            a = np.ascontiguousarray(a.reshape(self.nprob, -1))
            rc = lib().hps_solve_batch(self._h, int(a.shape[1]), a.ctypes.data_as(ctypes.c_void_p))
            nd = int(a.shape[1])
        if rc in (HPS_OK, HPS_ENOCONV):  # HPS_ENOCONV keeps the (unrefined) fields
            self.ndir = nd
            self.generation += 1
        self._check(rc, "solve")

    def far_field(self, thetas, R, out=None):
        torch = _torch()
        th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64).ravel())
        if out is None:
            out = torch.empty(self._shape(self.ndir, th.size), dtype=torch.complex128, device="cuda")
        ptr = _dev(out, torch.complex128, self.nprob * self.ndir * th.size, "out")
        self._check(lib().hps_far_field(self._h, int(th.size), th.ctypes.data_as(ctypes.c_void_p),
                                        float(R), ptr), "far_field")
        self.ntheta = int(th.size)
        return out

    def total_field(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self._shape(self.ndir, self.npde), dtype=torch.complex128, device="cuda")
        self._check(lib().hps_total_field(self._h, _dev(out, torch.complex128,
                                                        self.nprob * self.ndir * self.npde, "out")),
                    "total_field")
        return out

    def jvp(self, dq, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self._shape(self.ndir, self.ntheta), dtype=torch.complex128, device="cuda")
        self._check(lib().hps_jvp(self._h, _dev(dq, torch.float64, self.nprob * self.npde, "dq"),
                                  _dev(out, torch.complex128, self.nprob * self.ndir * self.ntheta, "out")),
                    "jvp")
        return out

    def vjp(self, r, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self._shape(self.npde), dtype=torch.float64, device="cuda")
        self._check(lib().hps_vjp(self._h, _dev(r, torch.complex128, self.nprob * self.ndir * self.ntheta, "r"),
                                  _dev(out, torch.float64, self.nprob * self.npde, "grad")), "vjp")
        return out

    def sine_eval(self, coef, out=None):
        torch = _torch()
        S = int(round(np.sqrt(coef.numel())))
        if out is None:
            out = torch.empty(self.npde, dtype=torch.float64, device="cuda")
        self._check(lib().hps_sine_eval(self._h, S, _dev(coef, torch.float64, S * S, "coef"),
                                        _dev(out, torch.float64, self.npde, "q")), "sine_eval")
        return out

    def sine_adjoint(self, g, S, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(S * S, dtype=torch.float64, device="cuda")
        self._check(lib().hps_sine_adjoint(self._h, int(S), _dev(g, torch.float64, self.npde, "g"),
                                           _dev(out, torch.float64, S * S, "coef")), "sine_adjoint")
        return out

    def gn_step(self, k, dirs, thetas, R, coef, data, max_iter=50, tol=1e-12, out=None, band=0):
        """One Gauss-Newton step on the sine model; returns (coef_out, info).
        band > 0: only the modes with m + n <= band are unknowns."""
        torch = _torch()
        a = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).ravel())
        th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64).ravel())
        S = int(round(np.sqrt(coef.numel())))
        if out is None:
            out = torch.empty(S * S, dtype=torch.float64, device="cuda")
        it = ctypes.c_int(0)
        rel = ctypes.c_double(0.0)
        mis = ctypes.c_double(0.0)
        self._check(lib().hps_gn_step(self._h, float(k), int(a.size), a.ctypes.data_as(ctypes.c_void_p),
                                      int(th.size), th.ctypes.data_as(ctypes.c_void_p), float(R), S, int(band),
                                      _dev(coef, torch.float64, S * S, "coef"),
                                      _dev(data, torch.complex128, a.size * th.size, "data"),
                                      int(max_iter), float(tol), _dev(out, torch.float64, S * S, "coef_out"),
                                      ctypes.byref(it), ctypes.byref(rel), ctypes.byref(mis)), "gn_step")
        self.ndir, self.ntheta, self.k = int(a.size), int(th.size), float(k)
        self.generation += 1
        return out, {"cg_iters": it.value, "cg_rel_res": rel.value, "misfit": mis.value}

    def stats(self):
        s = Stats()
        self._check(lib().hps_get_stats(self._h, ctypes.byref(s)), "stats")
        return {f: getattr(s, f) for f, _ in Stats._fields_}


def boundary_operators(nleaf, p, k, box=(-1.0, 1.0, -1.0, 1.0)):
    """Host-side S, K ([nb, nb] complex128 numpy) and boundary-node
    coordinates ([nb, 2]) in the library's root order (no GPU needed)."""
    L = lib()
    o = Opts()
    L.hps_default_opts(ctypes.byref(o))
    o.x0, o.x1, o.y0, o.y1 = map(float, box)
    o.nleaf, o.p = int(nleaf), int(p)
    nb = 4 * o.nleaf * (o.p - 2)
    xy = np.zeros((nb, 2))
    S = np.zeros((nb, nb), dtype=np.complex128)
    K = np.zeros((nb, nb), dtype=np.complex128)
    rc = L.hps_boundary_operators(ctypes.byref(o), float(k), xy.ctypes.data_as(ctypes.c_void_p),
                                  S.ctypes.data_as(ctypes.c_void_p), K.ctypes.data_as(ctypes.c_void_p))
    if rc != HPS_OK:
        raise HpsError(rc, "hps_boundary_operators")
    return xy, S, K


def combined_field_operators(nleaf, p, k, box=(-1.0, 1.0, -1.0, 1.0)):
    """Host-side K' (adjoint double layer) and T (hypersingular) [nb, nb]
    complex128 numpy, in the order of boundary_operators (no GPU needed)."""
    L = lib()
    o = Opts()
    L.hps_default_opts(ctypes.byref(o))
    o.x0, o.x1, o.y0, o.y1 = map(float, box)
    o.nleaf, o.p = int(nleaf), int(p)
    nb = 4 * o.nleaf * (o.p - 2)
    Kp = np.zeros((nb, nb), dtype=np.complex128)
    T = np.zeros((nb, nb), dtype=np.complex128)
    rc = L.hps_combined_field_operators(ctypes.byref(o), float(k), Kp.ctypes.data_as(ctypes.c_void_p),
                                        T.ctypes.data_as(ctypes.c_void_p))
    if rc != HPS_OK:
        raise HpsError(rc, "hps_combined_field_operators")
    return Kp, T


def zgemm(A, B, C=None, opA=0, opB=0, alpha=1.0, beta=0.0, stream=None):
    """Batched complex GEMM on [batch, rows, cols] column-major views: each
    torch tensor X of shape [batch, cols, rows] (row-major storage of the
    column-major matrix).  Used by the kernel tests."""
    torch = _torch()
    for t in (A, B):
        _dev(t, torch.complex128)
    batch, ka, ra = A.shape
    _, kb, rb = B.shape
    M = ra if opA == 0 else ka
    K = ka if opA == 0 else ra
    N = kb if opB == 0 else rb
    if C is None:
        C = torch.zeros((batch, N, M), dtype=torch.complex128, device=A.device)
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    st = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
    rc = lib().hps_zgemm(st, opA, opB, M, N, K, al, _dev(A, torch.complex128), ra, ka * ra,
                         _dev(B, torch.complex128), rb, kb * rb, be, _dev(C, torch.complex128), M, N * M, batch)
    if rc != HPS_OK:
        raise HpsError(rc, "hps_zgemm")
    return C


def zinv(A, stream=None):
    """Batched inverse of [batch, n, n] complex128 GPU matrices (column-major
    storage, i.e. each [n, n] slice holds the transpose); A is destroyed."""
    torch = _torch()
    batch, n, _ = A.shape
    inv = torch.empty_like(A)
    st = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
    rc = lib().hps_zinv(st, n, batch, _dev(A, torch.complex128), _dev(inv, torch.complex128))
    if rc != HPS_OK:
        raise HpsError(rc, "hps_zinv")
    return inv


def zinv_noalloc(A, inv=None, status=None, stream=None):
    """hps_zinv_noalloc: the inverse of [batch, n, n] complex128 GPU matrices
    (A destroyed) with the library's static scratch array as workspace.
    status: optional int32 GPU tensor of one element (asynchronous call);
    without it the call is synchronous and raises on a zero pivot."""
    torch = _torch()
    batch, n, _ = A.shape
    if inv is None:
        inv = torch.empty_like(A)
    sp = _dev(status, torch.int32, 1, "status") if status is not None else None
    st = ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
    rc = lib().hps_zinv_noalloc(st, n, batch, _dev(A, torch.complex128), _dev(inv, torch.complex128), sp)
    if rc != HPS_OK:
        raise HpsError(rc, "hps_zinv_noalloc")
    return inv


def gemm_tuning(mode=1, force=-1):
    """Tile-shape selection of the library's complex GEMM (process-wide):
    mode 0 fixed rules, 1 autotuning per distinct shape (tune in a warm-up
    pass); force >= 0 pins one tile variant.  Results do not depend on it."""
    rc = lib().hps_gemm_tuning(int(mode), int(force))
    if rc != HPS_OK:
        raise HpsError(rc, "hps_gemm_tuning")


def zinv_blocking(mode=-1):
    """Column blocking of the inverses of order above 512 and of the
    butterfly-transformed ones below it (process-wide): 1 right-looking with
    look-ahead, 0 recursive, -1 by size (look-ahead while the batch fits the
    last-level cache, and below order 512 for at most 32 matrices)."""
    rc = lib().hps_zinv_blocking(int(mode))
    if rc != HPS_OK:
        raise HpsError(rc, "hps_zinv_blocking")


def zinv_pivoting(mode=-1, tol=-1.0):
    """Pivoting of the large explicit inverses (process-wide): -1 butterfly
    transform + pivot-free elimination from order 224 (probe-checked, with a
    pivoted fallback), 0 always pivoted, 1 butterfly for every multiple of 4;
    tol >= 0 sets the probe tolerance (-1 keeps it)."""
    rc = lib().hps_zinv_pivoting(int(mode), float(tol))
    if rc != HPS_OK:
        raise HpsError(rc, "hps_zinv_pivoting")


def zinv_pivoting_info():
    """{calls, fallbacks, max_err} of the butterfly-path inverses so far."""
    c, f, e = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_double(0.0)
    rc = lib().hps_zinv_pivoting_info(ctypes.byref(c), ctypes.byref(f), ctypes.byref(e))
    if rc != HPS_OK:
        raise HpsError(rc, "hps_zinv_pivoting_info")
    return {"calls": c.value, "fallbacks": f.value, "max_err": e.value}


def gemm_tuning_info():
    """{variants, shapes_tuned, seconds} of the GEMM tile-shape tuning."""
    v, n, t = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    rc = lib().hps_gemm_tuning_info(ctypes.byref(v), ctypes.byref(n), ctypes.byref(t))
    if rc != HPS_OK:
        raise HpsError(rc, "hps_gemm_tuning_info")
    return {"variants": v.value, "shapes_tuned": n.value, "seconds": t.value}


def profile_start():
    """Times every following kernel launch of the library (HIP events)."""
    rc = lib().hps_profile_start()
    if rc != HPS_OK:
        raise HpsError(rc, "hps_profile_start")


def profile_stop():
    """Stops timing; returns {kernel class: {launches, total_ms, flops, bytes}},
    plus "phase:<name>" entries grouping the same launches by stage."""
    buf = (KernelStat * 32)()
    n = lib().hps_profile_stop(buf, 32)
    if n < 0:
        raise HpsError(n, "hps_profile_stop")
    return {buf[i].name.decode(): {"launches": buf[i].launches, "total_ms": buf[i].total_ms,
                                   "flops": buf[i].flops, "bytes": buf[i].bytes} for i in range(n)}
