"""Python access to the plain FP64 CPU oracle (``kr_oracle.c``).

TEST INFRASTRUCTURE ONLY: tests, the package smoke check and the benchmark's
CPU-baseline leg may use it; the product library never does.  The C source
is compiled with gcc into ``oracle/libkr_oracle.so`` by :func:`build`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kr_oracle.c")
_LIB = os.path.join(_HERE, "libkr_oracle.so")
_lib = None

ADAPTIVE, FIXED, REPLAY = 0, 1, 2
POST_CLIPPED, POST_BROKEN_UP = 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle (plain C, OpenMP) with gcc."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Extras(C.Structure):
    _fields_ = [("h_hint", C.c_void_p), ("h_log", C.c_void_p), ("h_log_ld", C.c_int64),
                ("h_log_cap", C.c_int32), ("h_log_n", C.c_void_p), ("post", C.c_void_p),
                ("photo_flux", C.c_void_p), ("photo_length", C.c_void_p)]


class Opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("floor", C.c_double), ("newton_tol", C.c_double),
                ("rho_floor", C.c_double), ("max_newton", C.c_int32),
                ("max_substeps", C.c_int32), ("mode", C.c_int32), ("n_fixed", C.c_int32)]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.kro_net_create.restype = C.c_void_p
        L.kro_net_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                     C.c_double, C.POINTER(C.c_int)]
        L.kro_net_destroy.argtypes = [C.c_void_p]
        L.kro_net_set_heat_capacity.argtypes = [C.c_void_p, C.c_double, C.c_void_p]
        L.kro_net_set_tables.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double,
                                         C.c_void_p, C.c_void_p]
        L.kro_species_thermo.argtypes = [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]
        L.kro_net_set_photo.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.kro_rhs_photo.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p,
                                    C.POINTER(C.c_double)]
        L.kro_jacobian_photo.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p]
        for name in ("kro_arrhenius",):
            getattr(L, name).argtypes = [C.c_void_p, C.c_void_p]
        L.kro_rate_coeffs.argtypes = [C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]
        L.kro_rhs.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
        L.kro_jacobian.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.kro_residual.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
        L.kro_newton_matrix.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]
        L.kro_lu_decompose.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
        L.kro_lu_solve.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.kro_gauss_full_pivot.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.kro_default_opts.argtypes = [C.POINTER(Opts)]
        L.kro_integrate.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_double, C.POINTER(Opts),
                                    C.c_void_p, C.c_void_p, C.c_int]
        L.kro_integrate_ex.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_double, C.POINTER(Opts),
                                       C.c_void_p, C.c_void_p, C.POINTER(Extras), C.c_int]
        L.kro_postprocess_flags.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.kro_be_substep.argtypes = [C.c_void_p, C.POINTER(Opts), C.c_void_p, C.c_void_p,
                                     C.c_double, C.c_void_p, C.POINTER(C.c_int32)]
        L.kro_element_residual.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                           C.c_int64, C.c_void_p]
        L.kro_postprocess.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.kro_fastest_timescale.restype = C.c_double
        L.kro_fastest_timescale.argtypes = [C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().kro_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class OracleNet:
    """The oracle's own copy of a network description (any object with the
    description's attributes: composition, reservoir, cv, h_form, s_form,
    reac, prod, arr_f, arr_r, n_elem, p_ref, T_min, T_max)."""

    def __init__(self, desc):
        L = lib()
        self.S = int(np.asarray(desc.composition).shape[1])
        self.N = self.S + 1
        self.n_rows = int(np.asarray(desc.composition).shape[0])
        self.R = int(np.asarray(desc.reac).shape[0])
        self._keep = [np.ascontiguousarray(desc.composition, np.int32),
                      np.ascontiguousarray(desc.reservoir, np.int32),
                      np.ascontiguousarray(desc.cv, np.float64),
                      np.ascontiguousarray(desc.h_form, np.float64),
                      np.ascontiguousarray(desc.s_form, np.float64),
                      np.ascontiguousarray(desc.reac, np.int32).reshape(-1, 3),
                      np.ascontiguousarray(desc.prod, np.int32).reshape(-1, 3),
                      np.ascontiguousarray(desc.arr_f, np.float64).reshape(-1, 3)]
        arr_r = None if desc.arr_r is None else np.ascontiguousarray(desc.arr_r, np.float64)
        self._keep.append(arr_r)
        err = C.c_int(0)
        k = self._keep
        self.h = L.kro_net_create(self.S, self.n_rows, int(desc.n_elem), k[0].ctypes.data,
                                  k[1].ctypes.data, k[2].ctypes.data, k[3].ctypes.data,
                                  k[4].ctypes.data, self.R, k[5].ctypes.data, k[6].ctypes.data,
                                  k[7].ctypes.data, None if arr_r is None else arr_r.ctypes.data,
                                  float(desc.p_ref), float(desc.T_min), float(desc.T_max), C.byref(err))
        if not self.h:
            raise ValueError(f"oracle rejected the network (code {err.value})")
        cvp = getattr(desc, "cv_poly", None)
        if cvp is not None:
            cvp = np.ascontiguousarray(cvp, np.float64).reshape(self.S, 2, 5)
            self._keep.append(cvp)
            if L.kro_net_set_heat_capacity(self.h, float(desc.T_mid), cvp.ctypes.data):
                raise ValueError("oracle rejected the heat-capacity polynomials")
        tab_of = getattr(desc, "tab_of", None)
        if tab_of is not None:
            tab_of = np.ascontiguousarray(tab_of, np.int32)
            tab = np.ascontiguousarray(desc.tab_log2k, np.float64)
            self._keep += [tab_of, tab]
            if L.kro_net_set_tables(self.h, int(tab.shape[0]), int(tab.shape[1]), float(desc.tab_log2T0),
                                    float(desc.tab_dlog2T), tab_of.ctypes.data, tab.ctypes.data):
                raise ValueError("oracle rejected the rate tables")
        sig = getattr(desc, "sigma_abs", None)
        photo = getattr(desc, "photo", None)
        qx = getattr(desc, "heat_extra", None)
        if sig is not None or photo is not None or qx is not None:
            arrs = [None if sig is None else np.ascontiguousarray(sig, np.float64),
                    None if photo is None else np.ascontiguousarray(photo, np.int32),
                    None if qx is None else np.ascontiguousarray(qx, np.float64).reshape(-1, 3)]
            self._keep += arrs
            if L.kro_net_set_photo(self.h, *[None if a is None else a.ctypes.data for a in arrs]):
                raise ValueError("oracle rejected the photoreaction data")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.kro_net_destroy(self.h)
            self.h = None

    # -- pieces of the method, one cell at a time --------------------------
    def arrhenius(self) -> np.ndarray:
        out = np.zeros((self.R, 2, 3))
        lib().kro_arrhenius(self.h, out.ctypes.data)
        return out

    def species_thermo(self, T: float):
        """(e_s(T), c_V,s(T)) per species, k_B units."""
        e, c = np.zeros(self.S), np.zeros(self.S)
        lib().kro_species_thermo(self.h, float(T), e.ctypes.data, c.ctypes.data)
        return e, c

    def rate_coeffs(self, T: float):
        kf, kr = np.zeros(self.R), np.zeros(self.R)
        lib().kro_rate_coeffs(self.h, float(T), kf.ctypes.data, kr.ctypes.data)
        return kf, kr

    def rhs(self, y):
        y = np.ascontiguousarray(y, np.float64)
        f = np.zeros(self.S)
        Q = C.c_double(0.0)
        lib().kro_rhs(self.h, y.ctypes.data, f.ctypes.data, C.byref(Q))
        return f, Q.value

    def jacobian(self, y):
        y = np.ascontiguousarray(y, np.float64)
        J = np.zeros((self.N, self.N))
        lib().kro_jacobian(self.h, y.ctypes.data, J.ctypes.data)
        return J

    def residual(self, y, yn, h):
        y = np.ascontiguousarray(y, np.float64)
        yn = np.ascontiguousarray(yn, np.float64)
        R = np.zeros(self.N)
        lib().kro_residual(self.h, y.ctypes.data, yn.ctypes.data, float(h), R.ctypes.data)
        return R

    def newton_matrix(self, y, h):
        y = np.ascontiguousarray(y, np.float64)
        M = np.zeros((self.N, self.N))
        lib().kro_newton_matrix(self.h, y.ctypes.data, float(h), M.ctypes.data)
        return M

    def be_substep(self, yn, h, atol, opts=None):
        o = opts or default_opts()
        yn = np.ascontiguousarray(yn, np.float64)
        atol = np.ascontiguousarray(atol, np.float64)
        y = np.zeros(self.N)
        it = C.c_int32(0)
        rc = lib().kro_be_substep(self.h, C.byref(o), yn.ctypes.data, atol.ctypes.data,
                                  float(h), y.ctypes.data, C.byref(it))
        return rc, y, it.value

    def postprocess(self, E0, n):
        E0 = np.ascontiguousarray(E0, np.float64)
        n = np.array(n, np.float64)
        lib().kro_postprocess(self.h, E0.ctypes.data, n.ctypes.data)
        return n

    def postprocess_flags(self, E0, n):
        """(post-processed copy of n, KRO_POST_* flags)."""
        E0 = np.ascontiguousarray(E0, np.float64)
        n = np.array(n, np.float64)
        flags = lib().kro_postprocess_flags(self.h, E0.ctypes.data, n.ctypes.data)
        return n, flags

    def fastest_timescale(self, y) -> float:
        y = np.ascontiguousarray(y, np.float64)
        return lib().kro_fastest_timescale(self.h, y.ctypes.data)

    # -- whole batches -------------------------------------------------------
    def integrate(self, n, T, rho=None, dt=None, dt_scalar=0.0, opts=None, nthreads=0):
        """Integrates copies of the batch; returns (n, T, status, cell_stats)."""
        o = opts or default_opts()
        n = np.array(n, np.float64, order="C")
        T = np.array(T, np.float64)
        ncell = T.shape[0]
        status = np.zeros(ncell, np.int32)
        stats = np.zeros((ncell, 4), np.int32)
        rho_a = None if rho is None else np.ascontiguousarray(rho, np.float64)
        dt_a = None if dt is None else np.ascontiguousarray(dt, np.float64)
        rc = lib().kro_integrate(self.h, ncell, n.ctypes.data, ncell, T.ctypes.data,
                                 None if rho_a is None else rho_a.ctypes.data,
                                 None if dt_a is None else dt_a.ctypes.data, float(dt_scalar),
                                 C.byref(o), status.ctypes.data, stats.ctypes.data, int(nthreads))
        if rc != 0:
            raise ValueError("oracle rejected the integrate arguments")
        return n, T, status, stats

    def rhs_photo(self, y, F, L):
        y = np.ascontiguousarray(y, np.float64)
        f = np.zeros(self.S)
        Q = C.c_double(0.0)
        lib().kro_rhs_photo(self.h, y.ctypes.data, float(F), float(L), f.ctypes.data, C.byref(Q))
        return f, Q.value

    def jacobian_photo(self, y, F, L):
        y = np.ascontiguousarray(y, np.float64)
        J = np.zeros((self.N, self.N))
        lib().kro_jacobian_photo(self.h, y.ctypes.data, float(F), float(L), J.ctypes.data)
        return J

    def integrate_ex(self, n, T, rho=None, dt=None, dt_scalar=0.0, opts=None, nthreads=0,
                     h_hint=None, log_cap=0, replay=None, replay_n=None, photo_flux=None,
                     photo_length=None):
        """kro_integrate_ex on copies of the batch.  h_hint: per-cell first
        substep (in/out copy).  log_cap > 0 records the accepted substep
        lengths (first log_cap per cell).  replay, replay_n: the substep
        lengths [cap, n_cells] and counts to replay (sets mode KRO_REPLAY).
        photo_flux, photo_length: per-cell radiation field (photoreactions).
        Returns a dict with n, T, status, stats, h_hint, h_log, h_log_n,
        post."""
        o = opts or default_opts()
        n = np.array(n, np.float64, order="C")
        T = np.array(T, np.float64)
        ncell = T.shape[0]
        status = np.zeros(ncell, np.int32)
        stats = np.zeros((ncell, 4), np.int32)
        post = np.zeros(ncell, np.int32)
        rho_a = None if rho is None else np.ascontiguousarray(rho, np.float64)
        dt_a = None if dt is None else np.ascontiguousarray(dt, np.float64)
        ex = Extras()
        hint = None if h_hint is None else np.array(h_hint, np.float64)
        ex.h_hint = None if hint is None else hint.ctypes.data
        if replay is not None:
            o = Opts.from_buffer_copy(o)
            o.mode = REPLAY
            log = np.array(replay, np.float64, order="C").reshape(-1, ncell)
            log_n = np.array(replay_n, np.int32)
        else:
            log = np.zeros((max(log_cap, 0), ncell))
            log_n = np.zeros(ncell, np.int32)
        ex.h_log = log.ctypes.data if log.size else None
        ex.h_log_ld = ncell
        ex.h_log_cap = log.shape[0]
        ex.h_log_n = log_n.ctypes.data
        ex.post = post.ctypes.data
        pf = None if photo_flux is None else np.ascontiguousarray(np.broadcast_to(photo_flux, (ncell,)), np.float64)
        pl = None if photo_length is None else np.ascontiguousarray(np.broadcast_to(photo_length, (ncell,)),
                                                                   np.float64)
        ex.photo_flux = None if pf is None else pf.ctypes.data
        ex.photo_length = None if pl is None else pl.ctypes.data
        rc = lib().kro_integrate_ex(self.h, ncell, n.ctypes.data, ncell, T.ctypes.data,
                                    None if rho_a is None else rho_a.ctypes.data,
                                    None if dt_a is None else dt_a.ctypes.data, float(dt_scalar),
                                    C.byref(o), status.ctypes.data, stats.ctypes.data, C.byref(ex),
                                    int(nthreads))
        if rc != 0:
            raise ValueError("oracle rejected the integrate arguments")
        return {"n": n, "T": T, "status": status, "stats": stats, "h_hint": hint,
                "h_log": log, "h_log_n": log_n, "post": post}

    def element_residual(self, before, after):
        before = np.ascontiguousarray(before, np.float64)
        after = np.ascontiguousarray(after, np.float64)
        nc = before.shape[1]
        out = np.zeros(nc)
        lib().kro_element_residual(self.h, nc, before.ctypes.data, after.ctypes.data, nc,
                                   out.ctypes.data)
        return out


def lu_decompose(a):
    a = np.array(a, np.float64, order="C")
    N = a.shape[0]
    p = np.zeros(N, np.int32)
    rc = lib().kro_lu_decompose(N, a.ctypes.data, p.ctypes.data)
    return rc, a, p


def lu_solve(lu, p, b):
    b = np.array(b, np.float64)
    lib().kro_lu_solve(lu.shape[0], np.ascontiguousarray(lu).ctypes.data,
                       np.ascontiguousarray(p, np.int32).ctypes.data, b.ctypes.data)
    return b


def gauss_full_pivot(a, b):
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros(a.shape[0])
    rc = lib().kro_gauss_full_pivot(a.shape[0], a.ctypes.data, b.ctypes.data, x.ctypes.data)
    return rc, x
