"""Python binding of libkr.so: per-cell implicit thermochemistry on MI355X.

Argument marshalling only.  Every step of the integration runs in the
library's HIP kernels; PyTorch provides device memory (tensors) and the
stream.  The names mirror the C ABI in include/kr.h:

    net = Network(desc)                       # kr_network_create
    chem_integrate(net, states, T, ...)        # kr_chem_integrate
    element_residual(net, before, after, ...)  # kr_element_residual

``desc`` is any object with the network-description attributes
(composition, reservoir, cv, h_form, s_form, reac, prod, arr_f, arr_r,
n_elem, p_ref, T_min, T_max).  There is no CPU fallback: without the built
library, or without a GPU, these functions raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkr.so")

KR_OK, KR_EINVAL, KR_EDEVICE, KR_ENOMEM, KR_ECOMPILE = 0, -1, -2, -3, -4
KR_FP64, KR_FP32LU_REFINE, KR_SINGLE, KR_MIXED = 0, 1, 2, 3
KR_ADAPTIVE, KR_FIXED_STEP = 0, 1
KR_ORDER_INPUT, KR_ORDER_WORK = 0, 1
KR_LAYOUT_AUTO, KR_LAYOUT_LANE, KR_LAYOUT_WAVE, KR_LAYOUT_GROUP16, KR_LAYOUT_GROUP32 = 0, 1, 2, 3, 4
KR_WIDE_MIN_SPECIES = 16
KR_NOALLOC_SCRATCH_BYTES = 8 << 20
KR_NOALLOC_MAX_ORDER_CELLS = (KR_NOALLOC_SCRATCH_BYTES - 4096) // 5

EXPORTED = ("kr_network_create", "kr_network_destroy", "kr_network_unknowns", "kr_network_layout",
            "kr_network_arrhenius", "kr_network_source", "kr_network_check", "kr_network_check_ex",
            "kr_default_options", "kr_chem_integrate", "kr_element_residual", "kr_postprocess",
            "kr_advect_plm", "kr_advect_plm_ssprk2", "kr_chem_integrate_noalloc",
            "kr_last_error", "kr_guess_create", "kr_guess_destroy", "kr_guess_num_params",
            "kr_guess_get_params", "kr_guess_set_params", "kr_guess_get_normalization",
            "kr_guess_set_normalization", "kr_guess_features", "kr_guess_targets",
            "kr_guess_fit_normalization", "kr_guess_gradients", "kr_guess_train",
            "kr_guess_forward", "kr_guess_predict")


class KrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libkr error {code}: {msg}")
        self.code = code


class _Desc(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("n_rows", C.c_int32), ("n_elem", C.c_int32),
                ("n_reactions", C.c_int32), ("composition", C.c_void_p),
                ("reservoir", C.c_void_p), ("cv", C.c_void_p), ("h_form", C.c_void_p),
                ("s_form", C.c_void_p), ("reac", C.c_void_p), ("prod", C.c_void_p),
                ("arr_f", C.c_void_p), ("arr_r", C.c_void_p), ("p_ref", C.c_double),
                ("T_min", C.c_double), ("T_max", C.c_double), ("cv_poly", C.c_void_p),
                ("T_mid", C.c_double), ("n_tables", C.c_int32), ("n_tab_nodes", C.c_int32),
                ("tab_of", C.c_void_p), ("tab_log2k", C.c_void_p), ("tab_log2T0", C.c_double),
                ("tab_dlog2T", C.c_double), ("sigma_abs", C.c_void_p), ("photo", C.c_void_p),
                ("heat_extra", C.c_void_p)]


class Stats(C.Structure):
    """kr_stats: totals of one kr_chem_integrate call."""
    _fields_ = [("cells", C.c_int64), ("substeps", C.c_int64), ("newton_iterations", C.c_int64),
                ("rejected", C.c_int64), ("newton_failures", C.c_int64), ("retried", C.c_int64),
                ("reverted", C.c_int64), ("refinement_sweeps", C.c_int64),
                ("fp64_fallbacks", C.c_int64), ("guess_fallbacks", C.c_int64),
                ("max_element_residual", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Options(C.Structure):
    """kr_options; defaults from kr_default_options."""
    _fields_ = [("precision", C.c_int32), ("mode", C.c_int32), ("n_fixed", C.c_int32),
                ("max_newton", C.c_int32), ("max_substeps", C.c_int32), ("order", C.c_int32),
                ("floor", C.c_double), ("newton_tol", C.c_double), ("rho_floor", C.c_double),
                ("guess", C.c_void_p), ("guess_ld", C.c_int64), ("counters", C.c_void_p),
                ("h_hint", C.c_void_p), ("h_log", C.c_void_p), ("h_log_ld", C.c_int64),
                ("h_log_cap", C.c_int32), ("reserved", C.c_int32), ("h_log_n", C.c_void_p),
                ("stats", C.POINTER(Stats)), ("photo_flux", C.c_void_p), ("photo_length", C.c_void_p)]


class BuildOpts(C.Structure):
    """kr_build_opts: compile-time tuning of the generated kernels."""
    _fields_ = [("waves_per_eu", C.c_int32), ("pivot_tau", C.c_float), ("layout", C.c_int32),
                ("lu_mfma", C.c_int32)]


class Batch(C.Structure):
    """kr_batch: one network's cells in a multi-network launch."""
    _fields_ = [("n_cells", C.c_int64), ("states", C.c_void_p), ("ld", C.c_int64),
                ("T", C.c_void_p), ("rho", C.c_void_p), ("dt", C.c_void_p),
                ("dt_scalar", C.c_double), ("status", C.c_void_p), ("cell_stats", C.c_void_p)]


class TrainOpts(C.Structure):
    """kr_train_opts."""
    _fields_ = [("steps", C.c_int64), ("batch", C.c_int32), ("reserved", C.c_int32),
                ("lr", C.c_float), ("lr_min", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2504_04941_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        L.kr_network_create.argtypes = [C.POINTER(_Desc), C.POINTER(C.c_void_p)]
        L.kr_network_create.restype = C.c_int
        L.kr_network_destroy.argtypes = [C.c_void_p]
        L.kr_network_destroy.restype = None
        L.kr_network_unknowns.argtypes = [C.c_void_p]
        L.kr_network_arrhenius.argtypes = [C.c_void_p, C.c_void_p]
        L.kr_network_source.argtypes = [C.c_void_p, C.c_char_p, C.c_int64]
        L.kr_network_source.restype = C.c_int64
        L.kr_network_check.argtypes = [C.POINTER(_Desc), C.c_int, C.c_char_p, C.c_int64]
        L.kr_default_options.argtypes = [C.POINTER(Options)]
        L.kr_default_options.restype = None
        L.kr_chem_integrate.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                        C.POINTER(Options), C.c_void_p, C.c_void_p, C.c_void_p]
        L.kr_element_residual.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                          C.c_int64, C.c_void_p, C.POINTER(C.c_double),
                                          C.c_void_p]
        L.kr_chem_integrate_noalloc.argtypes = L.kr_chem_integrate.argtypes
        L.kr_advect_plm.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                    C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                    C.c_void_p, C.c_double, C.c_double, C.c_int32, C.c_void_p]
        L.kr_advect_plm_ssprk2.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                           C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_void_p]
        L.kr_postprocess.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.c_void_p, C.c_void_p]
        L.kr_last_error.restype = C.c_char_p
        vp, i64 = C.c_void_p, C.c_int64
        L.kr_default_build_options.argtypes = [C.POINTER(BuildOpts)]
        L.kr_default_build_options.restype = None
        L.kr_network_create_ex.argtypes = [C.POINTER(_Desc), C.POINTER(BuildOpts), C.POINTER(vp)]
        L.kr_fastest_timescale.argtypes = [vp, i64, vp, i64, vp, vp, vp]
        L.kr_work_order.argtypes = [vp, i64, vp, i64, vp, vp, vp, C.c_double, C.POINTER(Options), vp, vp]
        L.kr_multi_create.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(BuildOpts), C.POINTER(vp)]
        L.kr_multi_destroy.argtypes = [vp]
        L.kr_multi_destroy.restype = None
        L.kr_chem_integrate_multi.argtypes = [vp, C.POINTER(Batch), C.c_double, C.POINTER(Options),
                                              C.c_int32, vp]
        L.kr_multi_graph_stats.argtypes = [vp, C.POINTER(i64)]
        L.kr_multi_graph_stats.restype = i64
        L.kr_multi_check.argtypes = [C.POINTER(C.POINTER(_Desc)), C.c_int32, C.c_int, C.c_char_p, i64]
        L.kr_guess_create.argtypes = [vp, C.c_int32, C.c_int32, C.c_uint64, C.POINTER(vp)]
        L.kr_guess_destroy.argtypes = [vp]
        L.kr_guess_destroy.restype = None
        L.kr_guess_num_params.argtypes = [vp]
        L.kr_guess_num_params.restype = i64
        for name in ("kr_guess_get_params", "kr_guess_set_params", "kr_guess_get_normalization",
                     "kr_guess_set_normalization"):
            getattr(L, name).argtypes = [vp, vp]
        L.kr_guess_features.argtypes = [vp, i64, vp, i64, vp, vp, C.c_double, vp, vp]
        L.kr_guess_targets.argtypes = [vp, i64, vp, vp, vp, vp, i64, vp, vp]
        L.kr_guess_fit_normalization.argtypes = [vp, i64, vp, vp, vp]
        L.kr_guess_gradients.argtypes = [vp, C.c_int32, vp, vp, vp, C.POINTER(C.c_double), vp]
        L.kr_guess_train.argtypes = [vp, i64, vp, vp, C.POINTER(TrainOpts), C.POINTER(C.c_double), vp]
        L.kr_guess_forward.argtypes = [vp, i64, vp, vp, vp]
        L.kr_guess_predict.argtypes = [vp, i64, vp, i64, vp, vp, C.c_double, vp, vp, i64, vp]
        _lib = L
    return _lib


def _check(rc):
    if rc != KR_OK:
        raise KrError(rc, lib().kr_last_error().decode())


def default_options(**kw) -> Options:
    o = Options()
    lib().kr_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": KR_FP64, "fp32lu": KR_FP32LU_REFINE, "single": KR_SINGLE, "mixed": KR_MIXED}[v]
        if k == "mode" and isinstance(v, str):
            v = {"adaptive": KR_ADAPTIVE, "fixed": KR_FIXED_STEP}[v]
        setattr(o, k, v)
    return o


def _pack_desc(desc):
    keep = [np.ascontiguousarray(desc.composition, np.int32),
            np.ascontiguousarray(desc.reservoir, np.int32),
            np.ascontiguousarray(desc.cv, np.float64),
            np.ascontiguousarray(desc.h_form, np.float64),
            np.ascontiguousarray(desc.s_form, np.float64),
            np.ascontiguousarray(desc.reac, np.int32).reshape(-1, 3),
            np.ascontiguousarray(desc.prod, np.int32).reshape(-1, 3),
            np.ascontiguousarray(desc.arr_f, np.float64).reshape(-1, 3)]
    arr_r = None if desc.arr_r is None else np.ascontiguousarray(desc.arr_r, np.float64).reshape(-1, 3)
    keep.append(arr_r)
    d = _Desc()
    d.n_rows, d.n_species = keep[0].shape if keep[0].ndim == 2 else (0, keep[2].shape[0])
    d.n_elem = int(desc.n_elem)
    d.n_reactions = keep[5].shape[0]
    (d.composition, d.reservoir, d.cv, d.h_form, d.s_form, d.reac, d.prod,
     d.arr_f) = (a.ctypes.data for a in keep[:8])
    d.arr_r = None if arr_r is None else arr_r.ctypes.data
    d.p_ref, d.T_min, d.T_max = float(desc.p_ref), float(desc.T_min), float(desc.T_max)
    sig, photo, qx = (getattr(desc, k, None) for k in ("sigma_abs", "photo", "heat_extra"))
    if sig is not None:
        sig = np.ascontiguousarray(sig, np.float64)
        keep.append(sig)
        d.sigma_abs = sig.ctypes.data
    if photo is not None:
        photo = np.ascontiguousarray(photo, np.int32)
        keep.append(photo)
        d.photo = photo.ctypes.data
    if qx is not None:
        qx = np.ascontiguousarray(qx, np.float64).reshape(-1, 3)
        keep.append(qx)
        d.heat_extra = qx.ctypes.data
    cvp = getattr(desc, "cv_poly", None)
    if cvp is not None:
        cvp = np.ascontiguousarray(cvp, np.float64)
        keep.append(cvp)
        d.cv_poly, d.T_mid = cvp.ctypes.data, float(desc.T_mid)
    tab_of = getattr(desc, "tab_of", None)
    if tab_of is not None:
        tab_of = np.ascontiguousarray(tab_of, np.int32)
        tab = np.ascontiguousarray(desc.tab_log2k, np.float64)
        keep += [tab_of, tab]
        d.tab_of, d.tab_log2k = tab_of.ctypes.data, tab.ctypes.data
        d.n_tables, d.n_tab_nodes = tab.shape
        d.tab_log2T0, d.tab_dlog2T = float(desc.tab_log2T0), float(desc.tab_dlog2T)
    return d, keep


def network_check(desc, compile: bool = False, build: BuildOpts | None = None) -> str:
    """Validates (and optionally compiles, without a device) a description;
    returns the generated device source."""
    d, keep = _pack_desc(desc)
    buf = C.create_string_buffer(1 << 23)
    _check(lib().kr_network_check_ex(C.byref(d), C.byref(build) if build is not None else None,
                                     int(bool(compile)), buf, len(buf)))
    return buf.value.decode()


def build_options(**kw) -> BuildOpts:
    o = BuildOpts()
    lib().kr_default_build_options(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def multi_check(descs, compile: bool = False) -> str:
    packed = [_pack_desc(d) for d in descs]
    arr = (C.POINTER(_Desc) * len(descs))(*[C.pointer(p[0]) for p in packed])
    buf = C.create_string_buffer(1 << 23)
    _check(lib().kr_multi_check(arr, len(descs), int(bool(compile)), buf, len(buf)))
    return buf.value.decode()


class Network:
    """A compiled network (kr_network_create_ex / kr_network_destroy)."""

    def __init__(self, desc, build: BuildOpts | None = None):
        d, keep = _pack_desc(desc)
        h = C.c_void_p()
        _check(lib().kr_network_create_ex(C.byref(d), None if build is None else C.byref(build),
                                          C.byref(h)))
        self._h = h
        self.n_species = d.n_species
        self.n_reactions = d.n_reactions
        self.n_unknowns = lib().kr_network_unknowns(h)
        self.layout = lib().kr_network_layout(h)
        # lanes per cell: 1, 16, 32 or 64
        self.group = {KR_LAYOUT_LANE: 1, KR_LAYOUT_GROUP16: 16, KR_LAYOUT_GROUP32: 32}.get(self.layout, 64)
        self.wide = self.group > 1

    @property
    def handle(self):
        if not self._h:
            raise ValueError("network destroyed")
        return self._h

    def arrhenius(self) -> np.ndarray:
        out = np.zeros((self.n_reactions, 2, 3))
        _check(lib().kr_network_arrhenius(self.handle, out.ctypes.data))
        return out

    def source(self) -> str:
        n = lib().kr_network_source(self.handle, None, 0)
        buf = C.create_string_buffer(int(n))
        lib().kr_network_source(self.handle, buf, n)
        return buf.value.decode()

    def close(self):
        if getattr(self, "_h", None):
            lib().kr_network_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dev_ptr(t, dtype, name):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    return t.data_ptr()


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def chem_integrate(net: Network, states, T, rho=None, dt=None, dt_scalar: float = 0.0,
                   rtol: float = 1e-6, opts: Options | None = None, status=None,
                   cell_stats=None, stream=None, h_hint=None, h_log=None, h_log_n=None,
                   stats: bool = False, noalloc: bool = False, photo_flux=None, photo_length=None):
    """kr_chem_integrate on device tensors.

    states: float64 [S, ld] with unit stride along cells (row stride = ld);
    T, rho, dt: float64 [n_cells]; status: int32 [n_cells];
    cell_stats: int32 [n_cells, 4]; h_hint: float64 [n_cells] in/out;
    h_log: float64 [cap, ld] (unit stride along cells) with h_log_n int32
    [n_cells].  Asynchronous on the stream unless stats=True, which returns
    the call's kr_stats totals as a dict (and synchronises).  noalloc=True
    calls kr_chem_integrate_noalloc (no allocation; a static per-GPU
    workspace).  photo_flux, photo_length: float64 [n_cells], the cells'
    radiation field for networks with photoreactions."""
    import torch
    if (h_hint is not None or h_log is not None or h_log_n is not None or stats or photo_flux is not None
            or photo_length is not None):
        o = Options.from_buffer_copy(opts if opts is not None else default_options())
        n_cells = int(T.numel())
        if h_hint is not None:
            if h_hint.numel() != n_cells or not h_hint.is_contiguous():
                raise ValueError("h_hint must be float64 [n_cells]")
            o.h_hint = _dev_ptr(h_hint, torch.float64, "h_hint")
        if h_log is not None:
            if h_log.dim() != 2 or h_log.stride(1) != 1 or h_log.shape[1] < n_cells:
                raise ValueError("h_log must be [cap, ld >= n_cells] with unit stride along cells")
            o.h_log = _dev_ptr(h_log, torch.float64, "h_log")
            o.h_log_ld = int(h_log.stride(0)) if h_log.shape[0] > 1 else int(h_log.shape[1])
            o.h_log_cap = int(h_log.shape[0])
        if h_log_n is not None:
            if h_log_n.numel() != n_cells:
                raise ValueError("h_log_n must be int32 [n_cells]")
            o.h_log_n = _dev_ptr(h_log_n, torch.int32, "h_log_n")
        for name, arr in (("photo_flux", photo_flux), ("photo_length", photo_length)):
            if arr is not None:
                if arr.numel() != n_cells or not arr.is_contiguous():
                    raise ValueError(f"{name} must be float64 [n_cells]")
                setattr(o, name, _dev_ptr(arr, torch.float64, name))
        st = Stats()
        if stats:
            o.stats = C.pointer(st)
        chem_integrate(net, states, T, rho=rho, dt=dt, dt_scalar=dt_scalar, rtol=rtol, opts=o,
                       status=status, cell_stats=cell_stats, stream=stream, noalloc=noalloc)
        return st.as_dict() if stats else None
    n_cells = int(T.numel())
    if states.dim() != 2 or states.shape[0] != net.n_species or states.stride(1) != 1:
        raise ValueError("states must be [n_species, ld] with unit stride along cells")
    ld = int(states.stride(0))
    if states.shape[1] < n_cells:
        raise ValueError("states has fewer columns than cells")
    if not T.is_contiguous() or (dt is not None and dt.numel() != n_cells):
        raise ValueError("T must be contiguous; dt must have one entry per cell")
    if cell_stats is not None and (cell_stats.numel() != 4 * n_cells or not cell_stats.is_contiguous()):
        raise ValueError("cell_stats must be int32 [n_cells, 4]")
    if status is not None and status.numel() != n_cells:
        raise ValueError("status must have one entry per cell")
    o = opts if opts is not None else default_options()
    fn = lib().kr_chem_integrate_noalloc if noalloc else lib().kr_chem_integrate
    _check(fn(
        net.handle, n_cells, _dev_ptr(states, torch.float64, "states"), ld,
        _dev_ptr(T, torch.float64, "T"), _dev_ptr(rho, torch.float64, "rho"),
        _dev_ptr(dt, torch.float64, "dt"), float(dt_scalar), float(rtol), C.byref(o),
        _dev_ptr(status, torch.int32, "status"), _dev_ptr(cell_stats, torch.int32, "cell_stats"),
        _stream_ptr(stream)))


def postprocess(net: Network, before, after, flags=None, stream=None) -> None:
    """kr_postprocess: the three post-processing stages (Sec. 2.2.3) of
    `after` in place, with the conserved totals of `before` (both float64
    [S, ld], unit stride along cells, same ld); flags int32 [n_cells] or
    None."""
    import torch
    if after.dim() != 2 or after.stride(1) != 1 or before.stride() != after.stride() or \
            before.shape != after.shape:
        raise ValueError("before/after must be [n_species, ld] with the same layout")
    n = int(after.shape[1]) if flags is None else int(flags.numel())
    _check(lib().kr_postprocess(net.handle, n, _dev_ptr(before, torch.float64, "before"),
                                _dev_ptr(after, torch.float64, "after"), int(after.stride(0)),
                                _dev_ptr(flags, torch.int32, "flags"), _stream_ptr(stream)))


ADVECT_PLAIN, ADVECT_PROJECTED, ADVECT_DONOR = 0, 1, 2


def advect_plm(net: Network, n_in, n_out, rho, flux, xc, xf, dt: float, n_lines: int = 1,
               line_stride: int | None = None, base=None, alpha: float = 0.0, beta: float = 1.0,
               mode: int = ADVECT_PROJECTED, stream=None) -> None:
    """kr_advect_plm: one forward-Euler stage of the stoichiometry-compatible
    PLM advection of the species along n_lines periodic lines.  n_in, n_out,
    base: float64 [S, ld] (unit stride along cells); rho, flux: float64
    [cells]; xc [n_cells], xf [n_cells + 1]."""
    import torch
    if n_in.dim() != 2 or n_in.stride(1) != 1 or n_out.stride() != n_in.stride():
        raise ValueError("n_in/n_out must be [n_species, ld] with the same layout")
    if base is not None and base.stride() != n_in.stride():
        raise ValueError("base must share the layout of n_in")
    n_cells = int(xc.numel())
    stride = n_cells if line_stride is None else int(line_stride)
    _check(lib().kr_advect_plm(net.handle, int(n_lines), n_cells, stride,
                               _dev_ptr(n_in, torch.float64, "n_in"), _dev_ptr(n_out, torch.float64, "n_out"),
                               int(n_in.stride(0)), _dev_ptr(rho, torch.float64, "rho"),
                               _dev_ptr(flux, torch.float64, "flux"), _dev_ptr(xc, torch.float64, "xc"),
                               _dev_ptr(xf, torch.float64, "xf"), float(dt),
                               _dev_ptr(base, torch.float64, "base"), float(alpha), float(beta), int(mode),
                               _stream_ptr(stream)))


def advect_plm_ssprk2(net: Network, n_in, n_out, rho0, flux0, rho1, flux1, xc, xf, dt: float, n_lines: int = 1,
                      line_stride: int | None = None, mode: int = ADVECT_PROJECTED, stream=None) -> None:
    """kr_advect_plm_ssprk2: one whole SSP-RK2 step of the same advection in
    one pass: rho0/flux0 the density and face
    mass fluxes of the step's start, rho1/flux1 those after the first stage.
    n_in, n_out: float64 [S, ld] (unit stride along cells)."""
    import torch
    if n_in.dim() != 2 or n_in.stride(1) != 1 or n_out.stride() != n_in.stride():
        raise ValueError("n_in/n_out must be [n_species, ld] with the same layout")
    n_cells = int(xc.numel())
    stride = n_cells if line_stride is None else int(line_stride)
    _check(lib().kr_advect_plm_ssprk2(net.handle, int(n_lines), n_cells, stride,
                                      _dev_ptr(n_in, torch.float64, "n_in"), _dev_ptr(n_out, torch.float64, "n_out"),
                                      int(n_in.stride(0)), _dev_ptr(rho0, torch.float64, "rho0"),
                                      _dev_ptr(flux0, torch.float64, "flux0"), _dev_ptr(rho1, torch.float64, "rho1"),
                                      _dev_ptr(flux1, torch.float64, "flux1"), _dev_ptr(xc, torch.float64, "xc"),
                                      _dev_ptr(xf, torch.float64, "xf"), float(dt), int(mode), _stream_ptr(stream)))


def work_order(net: Network, states, T, rho=None, dt=None, dt_scalar: float = 0.0,
               opts: Options | None = None, out=None, stream=None):
    """kr_work_order: the order (int32 view of uint32 cell indices) in which
    kr_chem_integrate with KR_ORDER_WORK hands out the cells, largest
    expected work first."""
    import torch
    n = int(T.numel())
    if states.dim() != 2 or states.stride(1) != 1 or states.shape[1] < n:
        raise ValueError("states must be [n_species, ld] with unit stride along cells")
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=T.device)
    o = opts if opts is not None else default_options()
    _check(lib().kr_work_order(net.handle, n, _dev_ptr(states, torch.float64, "states"),
                               int(states.stride(0)), _dev_ptr(T, torch.float64, "T"),
                               _dev_ptr(rho, torch.float64, "rho"), _dev_ptr(dt, torch.float64, "dt"),
                               float(dt_scalar), C.byref(o), _dev_ptr(out, torch.int32, "out"),
                               _stream_ptr(stream)))
    return out


def fastest_timescale(net: Network, states, T, out=None, stream=None):
    """kr_fastest_timescale: per-cell fastest self-coupling timescale (s)."""
    import torch
    n = int(T.numel())
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=T.device)
    _check(lib().kr_fastest_timescale(net.handle, n, _dev_ptr(states, torch.float64, "states"),
                                      int(states.stride(0)), _dev_ptr(T, torch.float64, "T"),
                                      _dev_ptr(out, torch.float64, "out"), _stream_ptr(stream)))
    return out


class Multi:
    """Several networks in one persistent launch (kr_multi_*)."""

    def __init__(self, nets, build: BuildOpts | None = None):
        self.nets = list(nets)   # keep the networks alive
        arr = (C.c_void_p * len(self.nets))(*[n.handle.value for n in self.nets])
        h = C.c_void_p()
        _check(lib().kr_multi_create(arr, len(self.nets), None if build is None else C.byref(build),
                                     C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().kr_multi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def graph_stats(self):
        cap = C.c_int64(0)
        launches = lib().kr_multi_graph_stats(self._h, C.byref(cap))
        return int(launches), int(cap.value)

    def integrate(self, batches, rtol=1e-6, opts: Options | None = None, use_graph=False,
                  stream=None, stats: bool = False):
        """batches: list of dicts with states [S_k, ld], T, and optional
        rho, dt, dt_scalar, status, cell_stats (device tensors).  stats=True
        returns the launch's kr_stats totals (all networks) as a dict and
        synchronises."""
        import torch
        arr = (Batch * len(batches))()
        for k, b in enumerate(batches):
            st = b["states"]
            n = int(b["T"].numel())
            if st.stride(1) != 1 or st.shape[0] != self.nets[k].n_species:
                raise ValueError(f"batch {k}: states must be [n_species, ld] with unit cell stride")
            arr[k] = Batch(n, _dev_ptr(st, torch.float64, "states"), int(st.stride(0)),
                           _dev_ptr(b["T"], torch.float64, "T"),
                           _dev_ptr(b.get("rho"), torch.float64, "rho"),
                           _dev_ptr(b.get("dt"), torch.float64, "dt"), float(b.get("dt_scalar", 0.0)),
                           _dev_ptr(b.get("status"), torch.int32, "status"),
                           _dev_ptr(b.get("cell_stats"), torch.int32, "cell_stats"))
        o = Options.from_buffer_copy(opts if opts is not None else default_options())
        st = Stats()
        if stats:
            o.stats = C.pointer(st)
        _check(lib().kr_chem_integrate_multi(self._h, arr, float(rtol), C.byref(o),
                                             int(bool(use_graph)), _stream_ptr(stream)))
        return st.as_dict() if stats else None


def element_residual(net: Network, before, after, resid=None, want_max: bool = False,
                     stream=None):
    """kr_element_residual on device tensors [S, ld]; returns the host max
    when want_max (the call then synchronises the stream)."""
    import torch
    n_cells = int(before.shape[1]) if resid is None else int(resid.numel())
    if before.stride() != after.stride() or before.stride(1) != 1:
        raise ValueError("before/after must share a [S, ld] layout with unit cell stride")
    mx = C.c_double(0.0)
    _check(lib().kr_element_residual(
        net.handle, n_cells, _dev_ptr(before, torch.float64, "before"),
        _dev_ptr(after, torch.float64, "after"), int(before.stride(0)),
        _dev_ptr(resid, torch.float64, "resid"), C.byref(mx) if want_max else None,
        _stream_ptr(stream)))
    return mx.value if want_max else None


class GuessModel:
    """The learned Newton guess (kr_guess_*): an MLP with BF16-MFMA training
    and inference kernels.  Tensors are device tensors; features X are
    float32 [n, S+2], targets Y float32 [n, S+1]."""

    def __init__(self, net: Network, hidden: int = 256, layers: int = 3, seed: int = 0):
        h = C.c_void_p()
        _check(lib().kr_guess_create(net.handle, int(hidden), int(layers), int(seed), C.byref(h)))
        self._h = h
        self.S = net.n_species
        self.n_in, self.n_out = self.S + 2, self.S + 1
        self.hidden, self.layers = hidden, layers
        self.n_params = int(lib().kr_guess_num_params(h))

    @property
    def handle(self):
        if not self._h:
            raise ValueError("guess model destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().kr_guess_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, np.float32)
        _check(lib().kr_guess_get_params(self.handle, out.ctypes.data))
        return out

    def set_params(self, w) -> None:
        w = np.ascontiguousarray(w, np.float32)
        assert w.size == self.n_params
        _check(lib().kr_guess_set_params(self.handle, w.ctypes.data))

    def get_normalization(self) -> np.ndarray:
        out = np.zeros(64, np.float32)
        _check(lib().kr_guess_get_normalization(self.handle, out.ctypes.data))
        return out

    def set_normalization(self, norm64) -> None:
        norm64 = np.ascontiguousarray(norm64, np.float32)
        _check(lib().kr_guess_set_normalization(self.handle, norm64.ctypes.data))

    def layer_slices(self):
        """[(W slice, b slice, fan_out, fan_in)] of the flat parameter vector."""
        out, off = [], 0
        for l in range(self.layers + 1):
            fi = self.n_in if l == 0 else self.hidden
            fo = self.n_out if l == self.layers else self.hidden
            out.append((slice(off, off + fi * fo), slice(off + fi * fo, off + fi * fo + fo), fo, fi))
            off += fi * fo + fo
        return out

    def features(self, states, T, dt=None, dt_scalar=0.0, X=None, stream=None):
        import torch
        n = int(T.numel())
        if X is None:
            X = torch.empty((n, self.n_in), dtype=torch.float32, device=T.device)
        _check(lib().kr_guess_features(self.handle, n, _dev_ptr(states, torch.float64, "states"),
                                       int(states.stride(0)), _dev_ptr(T, torch.float64, "T"),
                                       _dev_ptr(dt, torch.float64, "dt"), float(dt_scalar),
                                       _dev_ptr(X, torch.float32, "X"), _stream_ptr(stream)))
        return X

    def targets(self, before, T_before, after, T_after, Y=None, stream=None):
        import torch
        n = int(T_before.numel())
        if Y is None:
            Y = torch.empty((n, self.n_out), dtype=torch.float32, device=T_before.device)
        assert before.stride() == after.stride()
        _check(lib().kr_guess_targets(self.handle, n, _dev_ptr(before, torch.float64, "before"),
                                      _dev_ptr(T_before, torch.float64, "T_before"),
                                      _dev_ptr(after, torch.float64, "after"),
                                      _dev_ptr(T_after, torch.float64, "T_after"),
                                      int(before.stride(0)), _dev_ptr(Y, torch.float32, "Y"),
                                      _stream_ptr(stream)))
        return Y

    def fit_normalization(self, X, Y, stream=None):
        import torch
        _check(lib().kr_guess_fit_normalization(self.handle, int(X.shape[0]),
                                                _dev_ptr(X, torch.float32, "X"),
                                                _dev_ptr(Y, torch.float32, "Y"), _stream_ptr(stream)))

    def gradients(self, X, Y, stream=None):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=X.device)
        loss = C.c_double(0.0)
        _check(lib().kr_guess_gradients(self.handle, int(X.shape[0]), _dev_ptr(X, torch.float32, "X"),
                                        _dev_ptr(Y, torch.float32, "Y"), _dev_ptr(g, torch.float32, "g"),
                                        C.byref(loss), _stream_ptr(stream)))
        return g, loss.value

    def train(self, X, Y, steps, batch=4096, lr=1e-3, lr_min=1e-5, seed=1, beta1=0.9,
              beta2=0.999, eps=1e-8, stream=None) -> float:
        import torch
        o = TrainOpts(int(steps), int(batch), 0, float(lr), float(lr_min), float(beta1),
                      float(beta2), float(eps), int(seed))
        loss = C.c_double(0.0)
        _check(lib().kr_guess_train(self.handle, int(X.shape[0]), _dev_ptr(X, torch.float32, "X"),
                                    _dev_ptr(Y, torch.float32, "Y"), C.byref(o), C.byref(loss),
                                    _stream_ptr(stream)))
        return loss.value

    def forward(self, X, stream=None):
        import torch
        out = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device=X.device)
        _check(lib().kr_guess_forward(self.handle, int(X.shape[0]), _dev_ptr(X, torch.float32, "X"),
                                      _dev_ptr(out, torch.float32, "out"), _stream_ptr(stream)))
        return out

    def predict(self, states, T, dt=None, dt_scalar=0.0, guess=None, X_scratch=None, stream=None):
        """Newton starting points [S+1, n] (float64) for one substep of
        length dt of each cell."""
        import torch
        n = int(T.numel())
        if guess is None:
            guess = torch.empty((self.S + 1, n), dtype=torch.float64, device=T.device)
        if X_scratch is None:
            X_scratch = torch.empty((n, self.n_in), dtype=torch.float32, device=T.device)
        _check(lib().kr_guess_predict(self.handle, n, _dev_ptr(states, torch.float64, "states"),
                                      int(states.stride(0)), _dev_ptr(T, torch.float64, "T"),
                                      _dev_ptr(dt, torch.float64, "dt"), float(dt_scalar),
                                      _dev_ptr(X_scratch, torch.float32, "X"),
                                      _dev_ptr(guess, torch.float64, "guess"), int(guess.stride(0)),
                                      _stream_ptr(stream)))
        return guess


def guess_options(guess, counters=None, **kw) -> Options:
    """Options that start each cell's first substep from `guess` [S+1, ld]."""
    import torch
    o = default_options(**kw)
    o.guess = _dev_ptr(guess, torch.float64, "guess")
    o.guess_ld = int(guess.stride(0))
    if counters is not None:
        o.counters = counters.data_ptr()
    return o
