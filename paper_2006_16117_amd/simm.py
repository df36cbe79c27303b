"""Thin ctypes binding of the SIM-M HIP library (libsimm.so, C ABI in include/simm.h).

Only argument marshalling lives here: every step of the method runs in the
library's HIP kernels.  Device memory comes from torch (ROCm) tensors, host
memory from numpy arrays.  If the built library is missing this module raises
at import time; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsimm.so")

SIMM_OK = 0
SIMM_MEM_HOST = 0
SIMM_MEM_DEVICE = 1
SIMM_FLAG_PROJECT = 1
SIMM_FLAG_KERNEL_TIMING = 2
SIMM_FLAG_RELEASE_FACTORS = 4
SIMM_FLAG_MIXED_PROJECT = 8
SIMM_PREC_FP64 = 0
SIMM_PREC_MIXED = 1
SIMM_PROJ_FP64 = 0
SIMM_PROJ_FP32 = 1
SIMM_PROJ_BF16 = 2
KERNEL_NAMES = ["band_lu", "band_sweep", "gram_schmidt", "schur", "indicators", "project", "spike_prep"]
REJECTED, ADMISSIBLE, UNRESOLVED = 0, 1, 2

STATUS_NAMES = {0: "SIMM_OK", -1: "SIMM_EINVAL", -2: "SIMM_ENODEV", -3: "SIMM_ENOMEM", -4: "SIMM_EHIP",
                -5: "SIMM_ESINGULAR_SHIFT", -6: "SIMM_ENOCONV", -7: "SIMM_ELIMIT", -8: "SIMM_EUNSUPPORTED",
                -9: "SIMM_EREFINE", -10: "SIMM_EUNRESOLVED"}


class SimmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class simm_params(C.Structure):
    _fields_ = [("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("n1", C.c_int32), ("gauss_per_edge", C.c_int32), ("m", C.c_int32), ("levels", C.c_int32),
                ("h0", C.c_double), ("eps0", C.c_double), ("delta0", C.c_double), ("tau", C.c_double),
                ("max_regions_per_level", C.c_int64), ("flags", C.c_uint32),
                ("lookahead", C.c_int32), ("precision", C.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2006_16117_amd.build`")
# One HIP runtime per process.  ROCm builds of torch ship their own libamdhip64; loaded
# first, it also serves the library (its libamdhip64.so.7 dependency resolves to the
# runtime already in the process), so torch tensors and the library's allocations and
# streams live in the same runtime.  Loading the library first pulls in /opt/rocm's
# runtime and a later torch import adds a second one.
try:
    import torch  # noqa: F401
except ImportError:
    pass
_lib = C.CDLL(LIB_PATH)

_vp, _dp, _ip64, _i32, _i64, _d = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32, C.c_int64, C.c_double

EXPORTS = {
    "simm_last_error": (C.c_char_p, []),
    "simm_version": (C.c_int32, []),
    "simm_params_default": (C.c_int, [C.POINTER(simm_params)]),
    "simm_pencil_create_banded": (C.c_int, [_i64, _i32, _i32, _vp, _i32, _i32, _vp, _i32, _vp, C.POINTER(_vp)]),
    "simm_pencil_create_csr": (C.c_int, [_i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_vp)]),
    "simm_pencil_info": (C.c_int, [_vp, C.POINTER(_i64), C.POINTER(_i32), C.POINTER(_i32)]),
    "simm_pencil_destroy": (None, [_vp]),
    "simm_shift_build": (C.c_int, [_vp, _d, _d, _vp, _i32, _i32, _i32, _vp, C.POINTER(_vp)]),
    "simm_shift_refine_stats": (C.c_int, [_vp, _vp, _vp, _vp]),
    "simm_shift_factor_info": (C.c_int, [_vp, _vp, _vp, _vp]),
    "simm_shift_from_hessenberg": (C.c_int, [_d, _d, _d, _vp, _i32, _vp, C.POINTER(_vp)]),
    "simm_shift_info": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "simm_shift_basis": (C.c_int, [_vp, _vp, _i32, _vp]),
    "simm_shift_apply": (C.c_int, [_vp, _vp, _vp, _i32, _vp]),
    "simm_shift_apply_many": (C.c_int, [_vp, _vp, _vp, _i32, _i32, _vp]),
    "simm_shift_destroy": (None, [_vp]),
    "simm_indicators": (C.c_int, [_vp, _i32, _vp, _i64, C.POINTER(simm_params), _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                  _i32, _i32, _vp]),
    "simm_cell_residuals": (C.c_int, [_vp, _i32, _vp, _i64, C.POINTER(simm_params), _vp, _i32, _vp]),
    "simm_project": (C.c_int, [_vp, _vp, _i64, _vp, _vp, _i32, _vp]),
    "simm_project_noalloc": (C.c_int, [_vp, _vp, _i64, _vp, _vp, _i32, _vp]),
    "simm_gradient": (C.c_int, [_vp, _i32, _vp, _i64, C.POINTER(simm_params), _i32, _i32, _vp, _vp, _vp, _vp, _i32,
                                _vp]),
    "simm_run": (C.c_int, [_vp, C.POINTER(simm_params), _vp, _i32, _vp, C.POINTER(_vp)]),
    "simm_run_batch": (C.c_int, [C.POINTER(_vp), C.POINTER(simm_params), C.POINTER(_vp), _i32, _i32, _i32,
                                 C.POINTER(_vp)]),
    "simm_batch_tuning": (C.c_int, [_vp, _vp, _vp, _vp, _i64]),
    "simm_multiplicities": (C.c_int, [_vp, _vp, _i32, _i32, _d, _vp, _vp, _vp, _i64]),
    "simm_result_summary": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "simm_result_level": (C.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64]),
    "simm_result_full_indicators": (C.c_int, [_vp, _i32, _vp, _i64]),
    "simm_result_shift": (C.c_int, [_vp, _i32, C.POINTER(_vp)]),
    "simm_result_clusters": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _i64]),
    "simm_result_stats": (C.c_int, [_vp, _vp, _vp]),
    "simm_result_kernel_stats": (C.c_int, [_vp, _vp, _vp]),
    "simm_result_refine_stats": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "simm_result_destroy": (None, [_vp]),
}
for _name, (_res, _args) in EXPORTS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(status: int) -> None:
    if status != SIMM_OK:
        raise SimmError(status, _lib.simm_last_error().decode(errors="replace"))


def _ptr(a):
    """(pointer, mem kind) of a numpy array or a torch tensor."""
    if a is None:
        return None, SIMM_MEM_HOST
    if isinstance(a, np.ndarray):
        if not a.flags["F_CONTIGUOUS"] and not a.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be contiguous")
        return a.ctypes.data, SIMM_MEM_HOST
    if hasattr(a, "data_ptr"):
        return a.data_ptr(), (SIMM_MEM_DEVICE if a.is_cuda else SIMM_MEM_HOST)
    raise TypeError(type(a))


def _stream(stream):
    if stream is not None:
        return stream
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:  # noqa: BLE001
        pass
    return None


def params_default(**overrides) -> simm_params:
    p = simm_params()
    _check(_lib.simm_params_default(C.byref(p)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def params_from_dict(d: dict, **extra) -> simm_params:
    keys = {f[0] for f in simm_params._fields_}
    p = params_default()
    for k, v in {**d, **extra}.items():
        if k in keys:
            setattr(p, k, v)
    return p


class Pencil:
    """simm_pencil: banded A and B (LAPACK band layout, complex128)."""

    def __init__(self, n, kl_a, ku_a, a_band, kl_b=0, ku_b=0, b_band=None, stream=None):
        a = np.asfortranarray(a_band, dtype=np.complex128) if isinstance(a_band, np.ndarray) else a_band
        b = (np.asfortranarray(b_band, dtype=np.complex128) if isinstance(b_band, np.ndarray) else b_band)
        pa, mem = _ptr(a)
        pb, _ = _ptr(b)
        h = _vp()
        _check(_lib.simm_pencil_create_banded(n, kl_a, ku_a, pa, kl_b, ku_b, pb, mem, _stream(stream), C.byref(h)))
        self.handle = h
        self.n = n

    @classmethod
    def from_workload(cls, pen, stream=None):
        return cls(pen.n, pen.kl_a, pen.ku_a, pen.a_band, pen.kl_b, pen.ku_b, pen.b_band, stream)

    @classmethod
    def from_csr(cls, n, a_rowptr, a_col, a_val, b_rowptr=None, b_col=None, b_val=None, stream=None):
        """simm_pencil_create_csr: host CSR arrays (int64 row pointers, int32 columns,
        complex128 values); B = I when b_rowptr is None."""
        self = cls.__new__(cls)
        keep = [np.ascontiguousarray(a_rowptr, np.int64), np.ascontiguousarray(a_col, np.int32),
                np.ascontiguousarray(a_val, np.complex128)]
        if b_rowptr is not None:
            keep += [np.ascontiguousarray(b_rowptr, np.int64), np.ascontiguousarray(b_col, np.int32),
                     np.ascontiguousarray(b_val, np.complex128)]
        ptrs = [x.ctypes.data_as(_vp) for x in keep] + [None] * (6 - len(keep))
        h = _vp()
        _check(_lib.simm_pencil_create_csr(n, *ptrs, _stream(stream), C.byref(h)))
        self.handle = h
        self.n = n
        return self

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.simm_pencil_destroy(self.handle)
            self.handle = None


class Shift:
    """simm_shift: LU, Arnoldi basis and Schur data of one shift."""

    def __init__(self, handle, owner=None):
        self.handle = handle
        self._owner = owner          # a Result keeps borrowed shifts alive

    def info(self):
        sig = np.zeros(2)
        beta = C.c_double()
        me = C.c_int32()
        _check(_lib.simm_shift_info(self.handle, sig.ctypes.data, C.addressof(beta), C.addressof(me), None, None))
        m = me.value
        H = np.zeros((m + 1, m), dtype=np.complex128, order="F")
        ritz = np.zeros(m, dtype=np.complex128)
        _check(_lib.simm_shift_info(self.handle, None, None, None, H.ctypes.data, ritz.ctypes.data))
        return dict(sigma=complex(sig[0], sig[1]), beta=beta.value, m_eff=m, H=H, ritz=ritz)

    def basis(self, out=None, stream=None):
        if out is None:
            inf = self.info()
            n = _lib_n(self)
            out = np.zeros((n, inf["m_eff"] + 1), dtype=np.complex128, order="F")
        p, mem = _ptr(out)
        _check(_lib.simm_shift_basis(self.handle, p, mem, _stream(stream)))
        return out

    def refine_stats(self):
        sv = C.c_int64()
        co = C.c_int64()
        eta = C.c_double()
        _check(_lib.simm_shift_refine_stats(self.handle, C.addressof(sv), C.addressof(co), C.addressof(eta)))
        return dict(solves=sv.value, corrections=co.value, max_eta=eta.value)

    def factor_info(self):
        bl = C.c_int64()
        fb = C.c_int32()
        eta = C.c_double()
        _check(_lib.simm_shift_factor_info(self.handle, C.addressof(bl), C.addressof(fb), C.addressof(eta)))
        return dict(block_len=bl.value, fallback=bool(fb.value), eta=eta.value)

    def apply(self, x, y, stream=None):
        px, mem = _ptr(x)
        py, _ = _ptr(y)
        _check(_lib.simm_shift_apply(self.handle, px, py, mem, _stream(stream)))
        return y

    def apply_many(self, X, Y, stream=None):
        """X, Y: n x k column-major complex (numpy arrays in Fortran order, or device
        tensors whose storage is column-major)."""
        px, mem = _ptr(X)
        py, _ = _ptr(Y)
        k = X.shape[1] if len(X.shape) > 1 else 1
        _check(_lib.simm_shift_apply_many(self.handle, px, py, int(k), mem, _stream(stream)))
        return Y

    def __del__(self):
        if getattr(self, "handle", None) and self._owner is None and _lib is not None:
            _lib.simm_shift_destroy(self.handle)
            self.handle = None


def _lib_n(shift: Shift) -> int:
    return shift._n


def simm_shift_build(pencil: Pencil, sigma: complex, f, m: int, precision: int = SIMM_PREC_FP64,
                     stream=None) -> Shift:
    pf, mem = _ptr(np.ascontiguousarray(f, dtype=np.complex128) if isinstance(f, np.ndarray) else f)
    h = _vp()
    _check(_lib.simm_shift_build(pencil.handle, float(np.real(sigma)), float(np.imag(sigma)), pf, mem, m,
                                 int(precision), _stream(stream), C.byref(h)))
    s = Shift(h)
    s._n = pencil.n
    return s


def simm_shift_from_hessenberg(sigma: complex, beta: float, H, stream=None) -> Shift:
    """A shift from (sigma, beta, H_{m+1,m}) alone: H is an (m+1) x m complex array."""
    H = np.asfortranarray(H, dtype=np.complex128)
    m = H.shape[1]
    assert H.shape[0] == m + 1, "H must be (m + 1) x m"
    h = _vp()
    _check(_lib.simm_shift_from_hessenberg(float(np.real(sigma)), float(np.imag(sigma)), float(beta), H.ctypes.data,
                                           m, _stream(stream), C.byref(h)))
    s = Shift(h)
    s._n = 0
    return s


def simm_indicators(shifts, regions: np.ndarray, params: simm_params, want_sums: bool = False, m_max: int = 0,
                    stream=None) -> dict:
    """Host-memory convenience form: regions (N, 4) int64 (level, ix, iy, shift)."""
    regions = np.ascontiguousarray(regions, dtype=np.int64).reshape(-1, 4)
    N = regions.shape[0]
    arr = (_vp * len(shifts))(*[s.handle for s in shifts])
    out = {k: np.zeros(N) for k in ("indicator", "rho_max", "nsf", "nsc", "Tf")}
    out["decision"] = np.zeros(N, dtype=np.uint8)
    sums = None
    if want_sums:
        if m_max <= 0:
            m_max = max(s.info()["m_eff"] for s in shifts)
        sums = np.zeros((N, 2, m_max), dtype=np.complex128)
    _check(_lib.simm_indicators(arr, len(shifts), regions.ctypes.data, N, C.byref(params),
                                out["indicator"].ctypes.data, out["rho_max"].ctypes.data, out["nsf"].ctypes.data,
                                out["nsc"].ctypes.data, out["Tf"].ctypes.data, out["decision"].ctypes.data,
                                sums.ctypes.data if sums is not None else None, m_max, SIMM_MEM_HOST,
                                _stream(stream)))
    if sums is not None:
        out["sums"] = sums
    return out


def simm_cell_residuals(shift: Shift, level: int, squares: np.ndarray, params: simm_params, stream=None) -> np.ndarray:
    """Host-memory form: squares (N, 2) int64 (ix, iy) of one level; returns rho_max (N)."""
    squares = np.ascontiguousarray(squares, dtype=np.int64).reshape(-1, 2)
    out = np.zeros(squares.shape[0])
    _check(_lib.simm_cell_residuals(shift.handle, int(level), squares.ctypes.data, squares.shape[0], C.byref(params),
                                    out.ctypes.data, SIMM_MEM_HOST, _stream(stream)))
    return out


def simm_project(shift: Shift, Y, X, col_norms=None, precision: int = SIMM_PROJ_FP64, stream=None):
    """Device tensors: Y (m_eff x c), X (n x c) column-major complex128 (torch tensors
    whose storage is column-major: pass the transposed-contiguous view).  X may be
    None when col_norms is given (norms only).  precision: SIMM_PROJ_*."""
    py, _ = _ptr(Y)
    px, _ = _ptr(X)
    pn, _ = _ptr(col_norms)
    c = Y.shape[1]
    _check(_lib.simm_project(shift.handle, py, c, px, pn, int(precision), _stream(stream)))
    return X


def simm_project_noalloc(shift: Shift, Y, X, col_norms=None, precision: int = SIMM_PROJ_FP64, stream=None):
    """simm_project_noalloc: the arguments of simm_project; the call only enqueues its
    kernels (no device allocation, no synchronisation)."""
    py, _ = _ptr(Y)
    px, _ = _ptr(X)
    pn, _ = _ptr(col_norms)
    c = Y.shape[1]
    _check(_lib.simm_project_noalloc(shift.handle, py, c, px, pn, int(precision), _stream(stream)))
    return X


def simm_gradient(shifts, regions: np.ndarray, params: simm_params, a1_band=None, kl1: int = 0, ku1: int = 0,
                  want_diag: bool = True, want_dp: bool = True, n: int | None = None, stream=None):
    """Host-memory form of simm_gradient: regions (N, 4) int64 (level, ix, iy, shift);
    a1_band (kl1 + ku1 + 1, n) complex band of A1 or None.  Returns
    (J, dJ/dp or None, dJ/dRe A_ii + i dJ/dIm A_ii as an (n,) complex array or None)."""
    regions = np.ascontiguousarray(regions, dtype=np.int64).reshape(-1, 4)
    arr = (_vp * len(shifts))(*[s.handle for s in shifts])
    n = n if n is not None else shifts[0]._n
    J = C.c_double()
    dp = C.c_double()
    a1 = np.asfortranarray(a1_band, dtype=np.complex128) if (a1_band is not None and want_dp) else None
    gd = np.zeros(n, dtype=np.complex128) if want_diag else None
    _check(_lib.simm_gradient(arr, len(shifts), regions.ctypes.data, regions.shape[0], C.byref(params), kl1, ku1,
                              a1.ctypes.data if a1 is not None else None, C.addressof(J),
                              C.addressof(dp) if a1 is not None else None, gd.ctypes.data if gd is not None else None,
                              SIMM_MEM_HOST, _stream(stream)))
    return J.value, (dp.value if a1 is not None else None), gd


def _band_sum(n, parts):
    """Band (kl, ku, array) of the sum of bands given as (kl, ku, band) triples."""
    kl = max(p[0] for p in parts)
    ku = max(p[1] for p in parts)
    out = np.zeros((kl + ku + 1, n), dtype=np.complex128, order="F")
    for pkl, pku, band in parts:
        out[ku - pku: ku + pkl + 1, :] += band
    return kl, ku, out


class ProjectedNorms:
    """J(p, d) = sum_R ||x_R||^2 (the quantity of simm_gradient) for the pencil
    A = A0 + p A1 + diag(d), B, with the squares and shifts held fixed, as a
    torch.autograd.Function of the real scalar p and the complex n-vector d:
    backward returns dJ/dp and dJ/dRe d + i dJ/dIm d (torch's convention for a real
    function of complex inputs) from the adjoint kernels.  Host-memory bands."""

    def __init__(self, n, kl0, ku0, a0_band, kl1, ku1, a1_band, f, sigmas, regions, params, m, kl_b=0, ku_b=0,
                 b_band=None):
        self.n = n
        self.a0 = (kl0, ku0, np.asarray(a0_band, dtype=np.complex128))
        self.a1 = (kl1, ku1, np.asarray(a1_band, dtype=np.complex128))
        self.b = (kl_b, ku_b, b_band)
        self.f = np.asarray(f, dtype=np.complex128)
        self.sigmas = list(sigmas)
        self.regions = np.ascontiguousarray(regions, dtype=np.int64).reshape(-1, 4)
        self.params = params
        self.m = m

    def evaluate(self, p: float, d: np.ndarray, derivatives: bool = True):
        """(J, dJ/dp, grad_diag) at (p, d); with derivatives=False, (J, None, None)."""
        dband = (0, 0, np.asarray(d, dtype=np.complex128).reshape(1, -1))
        kl, ku, band = _band_sum(self.n, [self.a0, (self.a1[0], self.a1[1], p * self.a1[2]), dband])
        pen = Pencil(self.n, kl, ku, band, self.b[0], self.b[1], self.b[2])
        shifts = [simm_shift_build(pen, s, self.f, self.m) for s in self.sigmas]
        out = simm_gradient(shifts, self.regions, self.params, self.a1[2], self.a1[0], self.a1[1],
                            want_diag=derivatives, want_dp=derivatives)
        del shifts, pen
        return out

    def function(self):
        import torch
        prob = self

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, p, d):
                J, dp, gd = prob.evaluate(float(p.detach().cpu()), d.detach().cpu().numpy())
                ctx.save_for_backward(torch.tensor(dp, dtype=torch.float64, device=p.device),
                                      torch.from_numpy(gd).to(d.device))
                return torch.tensor(J, dtype=torch.float64, device=p.device)

            @staticmethod
            def backward(ctx, gJ):
                dp, gd = ctx.saved_tensors
                return gJ * dp, gJ.to(gd.device) * gd

        return _Fn.apply


@dataclasses.dataclass
class LevelOut:
    level: int
    keys: np.ndarray
    shift: np.ndarray
    indicator: np.ndarray
    rho_max: np.ndarray
    decision: np.ndarray
    full_indicator: np.ndarray     # ||V_m s_f|| / ||V_m s_c|| (NaN unless the run projected)


class Result:
    def __init__(self, handle):
        self.handle = handle
        K = C.c_int32()
        ns = C.c_int32()
        nc = C.c_int64()
        nu = C.c_int64()
        _check(_lib.simm_result_summary(handle, C.addressof(K), C.addressof(ns), C.addressof(nc), C.addressof(nu)))
        self.K, self.n_shifts, self.n_clusters, self.n_unresolved = K.value, ns.value, nc.value, nu.value
        self.levels = []
        for k in range(1, self.K + 1):
            cnt = C.c_int64()
            _lib.simm_result_level(handle, k, C.addressof(cnt), None, None, None, None, None, None, 0)
            N = cnt.value
            ix = np.zeros(N, np.int64)
            iy = np.zeros(N, np.int64)
            sh = np.zeros(N, np.int32)
            ind = np.zeros(N)
            rho = np.zeros(N)
            dec = np.zeros(N, np.uint8)
            _check(_lib.simm_result_level(handle, k, C.addressof(cnt), ix.ctypes.data, iy.ctypes.data, sh.ctypes.data,
                                          ind.ctypes.data, rho.ctypes.data, dec.ctypes.data, N))
            full = np.zeros(N)
            _check(_lib.simm_result_full_indicators(handle, k, full.ctypes.data, N))
            self.levels.append(LevelOut(k, np.stack([ix, iy], 1), sh, ind, rho, dec, full))
        nc_ = self.n_clusters
        lam = np.zeros(nc_, np.complex128)
        lr = np.zeros(nc_, np.complex128)
        cs = np.zeros(nc_, np.int32)
        fl = np.zeros(nc_, np.int32)
        cnt = C.c_int64()
        _check(_lib.simm_result_clusters(handle, C.addressof(cnt), lam.ctypes.data, lr.ctypes.data, cs.ctypes.data,
                                         fl.ctypes.data, nc_))
        self.lam, self.lam_ritz, self.cluster_shift, self.cluster_flags = lam, lr, cs, fl
        ms = np.zeros(4)
        ctr = np.zeros(3, np.int64)
        _check(_lib.simm_result_stats(handle, ms.ctypes.data, ctr.ctypes.data))
        self.ms = dict(shift_builds=ms[0], indicators=ms[1], projection=ms[2], total=ms[3])
        self.counters = dict(quadrature_systems=int(ctr[0]), squares=int(ctr[1]), m_applications=int(ctr[2]))
        kms = np.zeros(len(KERNEL_NAMES))
        kcnt = np.zeros(len(KERNEL_NAMES), np.int64)
        _check(_lib.simm_result_kernel_stats(handle, kms.ctypes.data, kcnt.ctypes.data))
        self.kernel_ms = {k: float(v) for k, v in zip(KERNEL_NAMES, kms)}
        self.kernel_launches = {k: int(v) for k, v in zip(KERNEL_NAMES, kcnt)}
        sv = C.c_int64()
        co = C.c_int64()
        fb = C.c_int32()
        eta = C.c_double()
        _check(_lib.simm_result_refine_stats(handle, C.addressof(sv), C.addressof(co), C.addressof(fb),
                                             C.addressof(eta)))
        self.refine = dict(solves=sv.value, corrections=co.value, fallbacks=fb.value, max_eta=eta.value)

    def shift(self, idx: int) -> Shift:
        h = _vp()
        _check(_lib.simm_result_shift(self.handle, idx, C.byref(h)))
        return Shift(h, owner=self)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.simm_result_destroy(self.handle)
            self.handle = None


def simm_run(pencil: Pencil, f, params: simm_params, stream=None) -> Result:
    pf, mem = _ptr(np.ascontiguousarray(f, dtype=np.complex128) if isinstance(f, np.ndarray) else f)
    h = _vp()
    _check(_lib.simm_run(pencil.handle, C.byref(params), pf, mem, _stream(stream), C.byref(h)))
    res = Result(h)
    res.pencil = pencil      # the result's shifts refer to the pencil: keep it alive with the result
    return res


def simm_multiplicities(result: "Result", F, rel_tol: float = 1e-6, stream=None):
    """Multiplicity of every cluster of `result` from the k start vectors in the
    columns of F (n x k complex; host array or device tensor, column-major).
    Returns (mult int32[n_clusters], singular values [n_clusters, k])."""
    if isinstance(F, np.ndarray):
        F = np.asfortranarray(F, dtype=np.complex128)
        k = F.shape[1]
        pf, mem = F.ctypes.data, SIMM_MEM_HOST
    else:
        k = F.shape[1]
        assert F.stride(0) == 1 and F.stride(1) == F.shape[0], "F must be column-major"
        pf, mem = F.data_ptr(), SIMM_MEM_DEVICE
    ncl = result.n_clusters
    mult = np.zeros(max(ncl, 1), np.int32)
    sv = np.zeros((max(ncl, 1), k))
    _check(_lib.simm_multiplicities(result.handle, pf, k, mem, rel_tol, _stream(stream), mult.ctypes.data,
                                    sv.ctypes.data, ncl))
    return mult[:ncl], sv[:ncl]


def simm_run_batch(pencils, fs, params_list, workers: int = 8):
    """simm_run_batch: one run per pencil, up to `workers` in flight on streams of
    their own.  fs are host complex vectors; returns one Result per pencil."""
    count = len(pencils)
    assert len(fs) == count and len(params_list) == count
    keep = [np.ascontiguousarray(f, dtype=np.complex128) for f in fs]
    ph = (_vp * count)(*[p.handle for p in pencils])
    pp = (simm_params * count)(*params_list)
    pf = (_vp * count)(*[k.ctypes.data_as(_vp) for k in keep])
    out = (_vp * count)()
    _check(_lib.simm_run_batch(ph, pp, pf, 0, count, workers, out))
    results = [Result(_vp(out[i])) for i in range(count)]
    for r, p in zip(results, pencils):
        r.pencil = p
    return results


def simm_batch_tuning(cap: int = 64):
    """The batched form's autotuner cache: shape classes, tuning rounds, and the chosen
    workgroup counts of the indicator and projection launches."""
    ne = C.c_int64()
    tr = C.c_int64()
    ig = np.zeros(cap, np.int32)
    pg = np.zeros(cap, np.int32)
    _check(_lib.simm_batch_tuning(C.addressof(ne), C.addressof(tr), ig.ctypes.data, pg.ctypes.data, cap))
    return dict(entries=ne.value, trials=tr.value, indicator_grids=[int(x) for x in ig if x],
                projection_grids=[int(x) for x in pg if x])
