"""ctypes binding of libxsec.so (include/xsec.h). Argument marshalling only: every step of
the computation runs in the library's HIP kernels. PyTorch is used by callers for device
memory and streams; this module accepts raw device pointers or torch tensors.

The library is loaded from this package directory; if it is missing, LibraryMissing is
raised (there is no fallback implementation)."""
from __future__ import annotations

import ctypes as C
import os
import threading
from typing import Dict, Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# XSEC_LIB selects another build of the same library (same ABI)
LIB_PATH = os.environ.get("XSEC_LIB") or os.path.join(PKG, "libxsec.so")

XS_OK, XS_EINVAL, XS_ENOMEM, XS_EDEVICE, XS_ENOTFOUND = 0, -1, -2, -3, -4
XS_EUNSORTED, XS_EBUSY, XS_ECANCELLED, XS_ETIMEOUT = -5, -6, -7, -8
XS_EINSTEIN_A, XS_REF_STRENGTH = 0, 1
XS_Q_POWER, XS_Q_TABLE = 0, 1
XS_CUT_FIXED, XS_CUT_MIN_FWHM = 0, 1
XS_FP32_KAHAN, XS_FP64 = 0, 1
XS_F64, XS_F32 = 0, 1            # element type of sigma outputs
XS_REGRID_LINEAR, XS_REGRID_BIN_MEAN = 0, 1
XS_N_EVAL_TIERS = 10
# names of the evaluation tiers counted by Context.count_evals_by_tier
EVAL_TIERS = ("lorentz_shifted", "series2", "series3", "series4", "series6",
              "core16", "core20_24", "core32", "core40", "core_small_y")

_STATUS = {0: "XS_OK", -1: "XS_EINVAL", -2: "XS_ENOMEM", -3: "XS_EDEVICE",
           -4: "XS_ENOTFOUND", -5: "XS_EUNSORTED", -6: "XS_EBUSY", -7: "XS_ECANCELLED",
           -8: "XS_ETIMEOUT"}


class LibraryMissing(RuntimeError):
    pass


class XsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class LinesDesc(C.Structure):
    _fields_ = [("n", C.c_size_t), ("nu0", C.c_void_p), ("A_or_Sref", C.c_void_p),
                ("E_low", C.c_void_p), ("gamma_ref", C.c_void_p), ("n_T", C.c_void_p),
                ("g_up", C.c_void_p), ("J_low", C.c_void_p)]


class SpeciesDesc(C.Structure):
    _fields_ = [("strength_form", C.c_int), ("mass_amu", C.c_double), ("T_ref", C.c_double),
                ("P_ref", C.c_double), ("q_kind", C.c_int), ("q_a", C.c_double),
                ("q_b", C.c_double), ("q_T", C.c_void_p), ("q_val", C.c_void_p),
                ("q_n", C.c_size_t), ("n_broad", C.c_int), ("broad_nj", C.c_size_t),
                ("broad_vmr", C.c_void_p), ("broad_gamma", C.c_void_p),
                ("broad_n", C.c_void_p)]


class Pt(C.Structure):
    _fields_ = [("P_bar", C.c_double), ("T_K", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("cutoff_kind", C.c_int), ("cut_cm1", C.c_double), ("fwhm_mult", C.c_double),
                ("precision", C.c_int), ("pts_per_lane", C.c_int), ("split", C.c_int),
                ("waves_per_simd", C.c_int), ("select_eps", C.c_double),
                ("out_dtype", C.c_int), ("tile_group", C.c_int), ("tol", C.c_double)]


class ServeOpts(C.Structure):
    _fields_ = [("max_inflight", C.c_int), ("mem_bytes", C.c_size_t), ("max_bypass", C.c_int),
                ("start_paused", C.c_int), ("max_admitted", C.c_int),
                ("step_items", C.c_int)]


class TuneResult(C.Structure):
    _fields_ = [("pts_per_lane", C.c_int), ("split", C.c_int), ("waves_per_simd", C.c_int),
                ("items_per_slot", C.c_int), ("probe_ms", C.c_double),
                ("default_probe_ms", C.c_double), ("candidates", C.c_int),
                ("key", C.c_char * 192)]


_lib = None
_lib_lock = threading.Lock()

_SIGS = {
    "xs_abi_version": ([], C.c_int),
    "xs_create": ([C.c_int, C.c_size_t, C.POINTER(C.c_void_p)], C.c_int),
    "xs_destroy": ([C.c_void_p], None),
    "xs_last_error": ([C.c_void_p], C.c_char_p),
    "xs_device_info": ([C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_size_t), C.c_char_p,
                        C.c_size_t], C.c_int),
    "xs_memory_used": ([C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)], C.c_int),
    "xs_load_lines": ([C.c_void_p, C.POINTER(LinesDesc), C.POINTER(SpeciesDesc),
                       C.POINTER(C.c_uint64)], C.c_int),
    "xs_unload_lines": ([C.c_void_p, C.c_uint64], C.c_int),
    "xs_lines_info": ([C.c_void_p, C.c_uint64, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)],
                      C.c_int),
    "xs_set_grid": ([C.c_void_p, C.c_void_p, C.c_size_t, C.POINTER(C.c_uint64)], C.c_int),
    "xs_free_grid": ([C.c_void_p, C.c_uint64], C.c_int),
    "xs_grid_info": ([C.c_void_p, C.c_uint64, C.POINTER(C.c_size_t)], C.c_int),
    "xs_compute": ([C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(Pt), C.c_size_t,
                    C.POINTER(Opts), C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "xs_compute_noalloc": ([C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(Pt), C.c_size_t,
                            C.POINTER(Opts), C.c_void_p, C.c_void_p], C.c_int),
    "xs_count_evals": ([C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(Pt), C.c_size_t,
                        C.POINTER(Opts), C.c_void_p], C.c_int),
    "xs_count_evals_by_tier": ([C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(Pt),
                                C.c_size_t, C.POINTER(Opts), C.c_void_p], C.c_int),
    "xs_graph_create": ([C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(Pt), C.c_size_t,
                         C.POINTER(Opts), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "xs_graph_launch": ([C.c_void_p, C.c_void_p], C.c_int),
    "xs_graph_destroy": ([C.c_void_p], None),
    "xs_serve_start": ([C.c_void_p, C.POINTER(ServeOpts)], C.c_int),
    "xs_serve_pause": ([C.c_void_p, C.c_int], C.c_int),
    "xs_submit": ([C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(Pt), C.c_size_t,
                   C.POINTER(Opts), C.c_void_p, C.c_int, C.POINTER(C.c_uint64)], C.c_int),
    "xs_submit_window": ([C.c_void_p, C.c_uint64, C.c_double, C.c_double, C.c_size_t,
                          C.POINTER(Pt), C.c_size_t, C.POINTER(Opts), C.c_void_p, C.c_int,
                          C.POINTER(C.c_uint64)], C.c_int),
    "xs_poll": ([C.c_void_p, C.c_uint64, C.POINTER(C.c_int)], C.c_int),
    "xs_wait": ([C.c_void_p, C.c_uint64, C.c_double], C.c_int),
    "xs_cancel": ([C.c_void_p, C.c_uint64], C.c_int),
    "xs_request_times": ([C.c_void_p, C.c_uint64, C.POINTER(C.c_double),
                          C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "xs_release": ([C.c_void_p, C.c_uint64], C.c_int),
    "xs_sched_simulate": ([C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_int,
                           C.c_int, C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64)], C.c_int),
    "xs_autotune": ([C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(Pt), C.c_size_t,
                     C.POINTER(Opts), C.POINTER(TuneResult)], C.c_int),
    "xs_tune_key": ([C.c_void_p, C.c_uint64, C.c_uint64, C.c_size_t, C.POINTER(Opts),
                     C.c_char_p, C.c_size_t], C.c_int),
    "xs_tune_cache_put": ([C.c_char_p, C.c_int, C.c_int, C.c_int, C.c_double], C.c_int),
    "xs_tune_cache_get": ([C.c_char_p, C.POINTER(C.c_int), C.POINTER(C.c_int),
                           C.POINTER(C.c_int), C.POINTER(C.c_double)], C.c_int),
    "xs_tune_cache_clear": ([], C.c_int),
    "xs_tune_cache_size": ([C.POINTER(C.c_size_t)], C.c_int),
    "xs_tune_cache_load": ([C.c_char_p], C.c_int),
    "xs_tune_cache_save": ([C.c_char_p], C.c_int),
    "xs_set_kernel_timing": ([C.c_void_p, C.c_int], C.c_int),
    "xs_kernel_time": ([C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)], C.c_int),
    "xs_eval_voigt": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p],
                      C.c_int),
    "xs_eval_voigt_host": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p],
                           C.c_int),
    "xs_eval_series_host": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_double,
                             C.c_void_p, C.c_void_p], C.c_int),
    "xs_eval_far_host": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                          C.c_double, C.c_void_p, C.c_void_p], C.c_int),
    "xs_eval_bounds_host": ([C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p],
                            C.c_int),
    "xs_regrid": ([C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p, C.c_size_t, C.c_int,
                   C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "xs_cia_regrid": ([C.c_void_p, C.c_uint64, C.c_void_p, C.c_size_t, C.c_void_p,
                       C.c_void_p, C.c_void_p], C.c_int),
    "xs_wavelength_grid_host": ([C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_size_t,
                                 C.POINTER(C.c_size_t)], C.c_int),
    "xs_set_grid_wavelength": ([C.c_void_p, C.c_double, C.c_double, C.c_double,
                                C.POINTER(C.c_uint64), C.POINTER(C.c_size_t)], C.c_int),
}


def lib():
    """The loaded library (raises LibraryMissing when it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise LibraryMissing(
                    f"{LIB_PATH} is missing: build it with `python -m paper_2510_20870_amd.build`")
            L = C.CDLL(LIB_PATH)
            for name, (args, res) in _SIGS.items():
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
            _lib = L
        return _lib


def exported_symbols() -> Sequence[str]:
    return tuple(_SIGS)


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def eval_voigt_host(x, y, precision: int = XS_FP32_KAHAN) -> np.ndarray:
    """K(x, y) as the kernels compute it, evaluated by the same source compiled for the host."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    out = np.empty_like(x)
    rc = lib().xs_eval_voigt_host(_ptr(x), _ptr(y), x.size, precision, _ptr(out))
    if rc:
        raise XsError(rc, lib().xs_last_error(None).decode())
    return out


def eval_series_host(x, y, variant: int = -1, tol: float = 0.0):
    """The tile kernel's FP32 far-region forms on the host: (K, variant used per point).
    variant 0 = shifted Lorentzian, 1..4 = asymptotic series with 2, 3, 4, 6 terms, -1 =
    the variant the kernel picks for a nearest point at (x, y) under error budget tol
    (0: the default 2e-7)."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    out = np.empty_like(x)
    var = np.empty(x.shape, np.int32)
    rc = lib().xs_eval_series_host(_ptr(x), _ptr(y), x.size, int(variant), float(tol),
                                   _ptr(out), _ptr(var))
    if rc:
        raise XsError(rc, lib().xs_last_error(None).decode())
    return out, var


def eval_far_host(X, H, y, t, with_kind: bool = False, tol: float = 0.0):
    """The tile kernel's polynomial for far lines on the host: K at x = X + H t from the
    degree-13 expansion over a tile of half-width H centred at X (Doppler units), with the
    thresholds of error budget tol (0: the default 2e-7); with with_kind also the
    expansion taken per case (0 shifted, 1 doubly shifted Lorentzian)."""
    X, H, y, t = (np.ascontiguousarray(a, np.float64) for a in np.broadcast_arrays(X, H, y, t))
    out = np.empty_like(X)
    kind = np.empty(X.shape, np.int32)
    rc = lib().xs_eval_far_host(_ptr(X), _ptr(H), _ptr(y), _ptr(t), X.size, float(tol),
                                _ptr(out), _ptr(kind))
    if rc:
        raise XsError(rc, lib().xs_last_error(None).decode())
    return (out, kind) if with_kind else out


def wavelength_grid(lambda_min_um: float, lambda_max_um: float, R: float) -> np.ndarray:
    """Wavenumbers (increasing) of the fixed-resolving-power wavelength grid, as the
    library builds it (xs_wavelength_grid_host)."""
    n = C.c_size_t()
    _lib_check(lib().xs_wavelength_grid_host(float(lambda_min_um), float(lambda_max_um),
                                             float(R), None, 0, C.byref(n)))
    out = np.empty(n.value, np.float64)
    _lib_check(lib().xs_wavelength_grid_host(float(lambda_min_um), float(lambda_max_um),
                                             float(R), _ptr(out), out.size, C.byref(n)))
    return out


def eval_bounds_host(x, y):
    """(K_lo, K_hi): the bounds of K(x, y) used by main-contributor selection."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    lo = np.empty_like(x)
    hi = np.empty_like(x)
    rc = lib().xs_eval_bounds_host(_ptr(x), _ptr(y), x.size, _ptr(lo), _ptr(hi))
    if rc:
        raise XsError(rc, lib().xs_last_error(None).decode())
    return lo, hi


def _out_np_dtype(opts: "Opts"):
    return np.float32 if opts.out_dtype == XS_F32 else np.float64


def _dev_ptr(t) -> int:
    if hasattr(t, "data_ptr"):
        return int(t.data_ptr())
    return int(t)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream)
    return int(stream)


def sched_simulate(arrive, duration, footprint, mem_bytes: int, max_admitted: int,
                   max_bypass: int = 0):
    """The server's admission rule on a simulated clock (host only): returns
    (admit times, done times, peak arena bytes)."""
    a = np.ascontiguousarray(arrive, np.float64)
    d = np.ascontiguousarray(duration, np.float64)
    f = np.ascontiguousarray(footprint, np.uint64)
    if not (len(a) == len(d) == len(f)):
        raise ValueError("arrive, duration and footprint differ in length")
    ad = np.zeros(len(a))
    dn = np.zeros(len(a))
    peak = C.c_uint64()
    rc = lib().xs_sched_simulate(len(a), _ptr(a), _ptr(d), _ptr(f), int(mem_bytes),
                                 int(max_admitted), int(max_bypass), _ptr(ad), _ptr(dn),
                                 C.byref(peak))
    if rc:
        raise XsError(rc, lib().xs_last_error(None).decode())
    return ad, dn, peak.value


def _lib_check(rc: int):
    if rc != XS_OK:
        raise XsError(rc, lib().xs_last_error(None).decode())


def tune_cache_put(key: str, pts_per_lane: int, waves_per_simd: int, items_per_slot: int,
                   probe_ms: float = 0.0):
    _lib_check(lib().xs_tune_cache_put(key.encode(), pts_per_lane, waves_per_simd,
                                       items_per_slot, probe_ms))


def tune_cache_get(key: str):
    """(pts_per_lane, waves_per_simd, items_per_slot, probe_ms) or None."""
    P, W, I, ms = C.c_int(), C.c_int(), C.c_int(), C.c_double()
    rc = lib().xs_tune_cache_get(key.encode(), C.byref(P), C.byref(W), C.byref(I), C.byref(ms))
    if rc == XS_ENOTFOUND:
        return None
    _lib_check(rc)
    return P.value, W.value, I.value, ms.value


def tune_cache_clear():
    _lib_check(lib().xs_tune_cache_clear())


def tune_cache_size() -> int:
    n = C.c_size_t()
    _lib_check(lib().xs_tune_cache_size(C.byref(n)))
    return n.value


def tune_cache_load(path: str):
    _lib_check(lib().xs_tune_cache_load(os.fsencode(path)))


def tune_cache_save(path: str):
    _lib_check(lib().xs_tune_cache_save(os.fsencode(path)))


class Request:
    """A submitted cross-section request (see Context.submit)."""

    def __init__(self, ctx: "Context", h: int, out, keep=()):
        self.ctx = ctx
        self.h = h
        self.out = out
        self._keep = keep   # host buffers that must outlive the request

    def poll(self) -> bool:
        d = C.c_int()
        self.ctx._check(self.ctx._L.xs_poll(self.ctx.h, self.h, C.byref(d)))
        return bool(d.value)

    def wait(self, timeout_s: float = -1.0):
        """Wait and return the output (raises XsError on failure or cancellation)."""
        self.ctx._check(self.ctx._L.xs_wait(self.ctx.h, self.h, float(timeout_s)))
        return self.out

    def status(self, timeout_s: float = -1.0) -> int:
        return self.ctx._L.xs_wait(self.ctx.h, self.h, float(timeout_s))

    def cancel(self) -> int:
        return self.ctx._L.xs_cancel(self.ctx.h, self.h)

    def times(self):
        ts, ta, td = C.c_double(), C.c_double(), C.c_double()
        self.ctx._check(self.ctx._L.xs_request_times(self.ctx.h, self.h, C.byref(ts),
                                                     C.byref(ta), C.byref(td)))
        return ts.value, ta.value, td.value

    def release(self):
        if self.h:
            self.ctx._check(self.ctx._L.xs_release(self.ctx.h, self.h))
            self.h = None


class Context:
    """One xs_ctx on one device. Closes on close()/__exit__/garbage collection."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._L = lib()
        h = C.c_void_p()
        self._check(self._L.xs_create(device, hbm_budget_bytes, C.byref(h)))
        self.h = h.value
        self.device = device

    # ------------------------------------------------------------------ plumbing
    def _check(self, rc: int):
        if rc != XS_OK:
            raise XsError(rc, self._L.xs_last_error(None).decode())

    def close(self):
        if getattr(self, "h", None):
            self._L.xs_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ queries
    def device_info(self) -> Dict[str, object]:
        n_cu = C.c_int()
        lds = C.c_size_t()
        arch = C.create_string_buffer(64)
        self._check(self._L.xs_device_info(self.h, C.byref(n_cu), C.byref(lds), arch, 64))
        return {"n_cu": n_cu.value, "lds_bytes": lds.value, "arch": arch.value.decode()}

    def memory_used(self):
        u, b = C.c_size_t(), C.c_size_t()
        self._check(self._L.xs_memory_used(self.h, C.byref(u), C.byref(b)))
        return u.value, b.value

    # ------------------------------------------------------------------ residency
    def load_lines(self, lines: Dict[str, np.ndarray], mass_amu: float,
                   strength_form: int = XS_EINSTEIN_A, q_a: float = 0.0343, q_b: float = 1.5,
                   q_table: Optional[Sequence[Sequence[float]]] = None,
                   T_ref: float = 296.0, P_ref: float = 1.0,
                   broadening: Optional[Dict[str, np.ndarray]] = None) -> int:
        """Load a line list. broadening (optional): {"vmr": [B], "gamma": [B][nj],
        "n": [B][nj]} partner tables over J, with the lines' "J_low"."""
        arrs = {
            "nu0": np.ascontiguousarray(lines["nu0"], np.float64),
            "A": np.ascontiguousarray(lines["A"], np.float32),
            "E_low": np.ascontiguousarray(lines["E_low"], np.float32),
            "gamma": np.ascontiguousarray(lines["gamma"], np.float32),
            "n_T": np.ascontiguousarray(lines["n_T"], np.float32),
            "g_up": np.ascontiguousarray(lines["g_up"], np.uint16),
        }
        if "J_low" in lines:
            arrs["J_low"] = np.ascontiguousarray(lines["J_low"], np.uint16)
        n = len(arrs["nu0"])
        d = LinesDesc(n, _ptr(arrs["nu0"]), _ptr(arrs["A"]), _ptr(arrs["E_low"]),
                      _ptr(arrs["gamma"]), _ptr(arrs["n_T"]), _ptr(arrs["g_up"]),
                      _ptr(arrs["J_low"]) if "J_low" in arrs else None)
        if q_table is not None:
            qT = np.ascontiguousarray(q_table[0], np.float64)
            qV = np.ascontiguousarray(q_table[1], np.float64)
            sp = SpeciesDesc(strength_form, mass_amu, T_ref, P_ref, XS_Q_TABLE, 0.0, 0.0,
                             _ptr(qT), _ptr(qV), len(qT))
        else:
            sp = SpeciesDesc(strength_form, mass_amu, T_ref, P_ref, XS_Q_POWER, q_a, q_b,
                             None, None, 0)
        if broadening is not None:
            bv = np.ascontiguousarray(broadening["vmr"], np.float64).ravel()
            bg = np.ascontiguousarray(broadening["gamma"], np.float64).reshape(len(bv), -1)
            bn = np.ascontiguousarray(broadening["n"], np.float64).reshape(bg.shape)
            arrs.update(bv=bv, bg=bg, bn=bn)   # kept alive until the call returns
            sp.n_broad = len(bv)
            sp.broad_nj = bg.shape[1]
            sp.broad_vmr, sp.broad_gamma, sp.broad_n = _ptr(bv), _ptr(bg), _ptr(bn)
        h = C.c_uint64()
        self._check(self._L.xs_load_lines(self.h, C.byref(d), C.byref(sp), C.byref(h)))
        return h.value

    def unload_lines(self, h: int):
        self._check(self._L.xs_unload_lines(self.h, h))

    def lines_info(self, h: int):
        n, b = C.c_size_t(), C.c_size_t()
        self._check(self._L.xs_lines_info(self.h, h, C.byref(n), C.byref(b)))
        return n.value, b.value

    def set_grid(self, nu: np.ndarray) -> int:
        nu = np.ascontiguousarray(nu, np.float64)
        h = C.c_uint64()
        self._check(self._L.xs_set_grid(self.h, _ptr(nu), nu.size, C.byref(h)))
        return h.value

    def set_grid_wavelength(self, lambda_min_um: float, lambda_max_um: float, R: float):
        """Resident grid of fixed resolving power R over [lambda_min, lambda_max] (um):
        (handle, wavenumbers in increasing order). Point j of a result is at wavelength
        1e4 / nu[j]; reverse a row for increasing wavelength."""
        h = C.c_uint64()
        n = C.c_size_t()
        self._check(self._L.xs_set_grid_wavelength(self.h, float(lambda_min_um),
                                                   float(lambda_max_um), float(R),
                                                   C.byref(h), C.byref(n)))
        return h.value, wavelength_grid(lambda_min_um, lambda_max_um, R)

    def cia_regrid(self, grid: int, blocks) -> np.ndarray:
        """Collision-induced absorption: blocks = [(nu, alpha), ...] (one per temperature,
        nu increasing), each interpolated linearly onto the grid (zero outside its range):
        [n_blocks, n_grid]."""
        nus = [np.ascontiguousarray(b[0], np.float64) for b in blocks]
        als = [np.ascontiguousarray(b[1], np.float64) for b in blocks]
        off = np.zeros(len(blocks) + 1, np.uint64)
        off[1:] = np.cumsum([len(v) for v in nus])
        nu = np.ascontiguousarray(np.concatenate(nus) if nus else np.zeros(0), np.float64)
        al = np.ascontiguousarray(np.concatenate(als) if als else np.zeros(0), np.float64)
        out = np.empty((len(blocks), self.grid_len(grid)), np.float64)
        self._check(self._L.xs_cia_regrid(self.h, grid, _ptr(off), len(blocks), _ptr(nu),
                                          _ptr(al), _ptr(out)))
        return out

    def regrid(self, src_grid: int, dst_grid: int, sigma, mode: int = XS_REGRID_BIN_MEAN,
               out=None, stream=None):
        """Rows of sigma on src_grid resampled onto dst_grid (float64): a host array in,
        a new host array out; or device tensors (out required), enqueued on `stream`."""
        n_dst = self.grid_len(dst_grid)
        if isinstance(sigma, np.ndarray):
            src = np.ascontiguousarray(sigma, np.float64).reshape(-1, self.grid_len(src_grid))
            host = np.empty((src.shape[0], n_dst), np.float64)
            self._check(self._L.xs_regrid(self.h, src_grid, dst_grid, _ptr(src), src.shape[0],
                                          int(mode), _ptr(host), 0, None))
            return host
        n_rows = int(sigma.numel()) // self.grid_len(src_grid)
        self._check(self._L.xs_regrid(self.h, src_grid, dst_grid, _dev_ptr(sigma), n_rows,
                                      int(mode), _dev_ptr(out), 1, _stream_handle(stream)))
        return out

    def free_grid(self, h: int):
        self._check(self._L.xs_free_grid(self.h, h))

    # ------------------------------------------------------------------ compute
    @staticmethod
    def opts(cutoff_kind: int = XS_CUT_FIXED, cut_cm1: float = 25.0, fwhm_mult: float = 100.0,
             precision: int = XS_FP32_KAHAN, pts_per_lane: int = 0, split: int = 0,
             waves_per_simd: int = 0, select_eps: float = 0.0,
             out_dtype: int = XS_F64, tile_group: int = 0, tol: float = 0.0) -> Opts:
        """Options of a computation (xs_opts). tol: the FP32 path's error budget of its far
        forms relative to each contribution, 0 (the default 2e-7) or in [2e-7, 1e-5]."""
        return Opts(cutoff_kind, cut_cm1, fwhm_mult, precision, pts_per_lane, split,
                    waves_per_simd, float(select_eps), int(out_dtype), int(tile_group),
                    float(tol))

    @staticmethod
    def _pts(pts) -> C.Array:
        pts = np.asarray(pts, np.float64).reshape(-1, 2)
        arr = (Pt * len(pts))()
        for k, (p, t) in enumerate(pts):
            arr[k] = Pt(float(p), float(t))
        return arr

    def compute(self, lines: int, grid: int, pts, opts: Opts, out=None, stream=None):
        """sigma[npts, n_grid] (float64, or float32 with opts.out_dtype = XS_F32). With
        `out` a device tensor (or pointer) the work is enqueued on `stream` and `out` is
        returned; otherwise a host numpy array is returned."""
        p = self._pts(pts)
        if out is None:
            n_grid = self.grid_len(grid)
            host = np.empty((len(p), n_grid), _out_np_dtype(opts))
            self._check(self._L.xs_compute(self.h, lines, grid, p, len(p), C.byref(opts),
                                           _ptr(host), 0, None))
            return host
        self._check(self._L.xs_compute(self.h, lines, grid, p, len(p), C.byref(opts),
                                       _dev_ptr(out), 1, _stream_handle(stream)))
        return out

    def compute_noalloc(self, lines: int, grid: int, pts, opts: Opts, out, stream=None):
        """xs_compute_noalloc: sigma into the device tensor (or pointer) `out`, enqueued on
        `stream`, with no device allocation (the library's static scratch array)."""
        p = self._pts(pts)
        self._check(self._L.xs_compute_noalloc(self.h, lines, grid, p, len(p), C.byref(opts),
                                               _dev_ptr(out), _stream_handle(stream)))
        return out

    def count_evals(self, lines: int, grid: int, pts, opts: Opts) -> np.ndarray:
        p = self._pts(pts)
        out = np.zeros(len(p), np.uint64)
        self._check(self._L.xs_count_evals(self.h, lines, grid, p, len(p), C.byref(opts),
                                           _ptr(out)))
        return out

    def count_evals_by_tier(self, lines: int, grid: int, pts, opts: Opts) -> np.ndarray:
        """[npts, XS_N_EVAL_TIERS] counts of in-cut pairs by the tier each point needs."""
        p = self._pts(pts)
        out = np.zeros((len(p), XS_N_EVAL_TIERS), np.uint64)
        self._check(self._L.xs_count_evals_by_tier(self.h, lines, grid, p, len(p),
                                                   C.byref(opts), _ptr(out)))
        return out

    def grid_len(self, grid: int) -> int:
        n = C.c_size_t()
        self._check(self._L.xs_grid_info(self.h, grid, C.byref(n)))
        return n.value

    def eval_voigt(self, x, y, precision: int = XS_FP32_KAHAN) -> np.ndarray:
        x = np.ascontiguousarray(x, np.float64)
        y = np.ascontiguousarray(y, np.float64)
        out = np.empty_like(x)
        self._check(self._L.xs_eval_voigt(self.h, _ptr(x), _ptr(y), x.size, precision,
                                          _ptr(out)))
        return out

    # ------------------------------------------------------------------ serving
    def serve_start(self, max_inflight: int = 0, mem_bytes: int = 0, max_bypass: int = 0,
                    paused: bool = False, max_admitted: int = 0, step_items: int = 0):
        o = ServeOpts(max_inflight, mem_bytes, max_bypass, int(bool(paused)), max_admitted,
                      int(step_items))
        self._check(self._L.xs_serve_start(self.h, C.byref(o)))

    def serve_pause(self, paused: bool = True):
        self._check(self._L.xs_serve_pause(self.h, int(bool(paused))))

    def submit(self, lines: int, grid: int, pts, opts: Opts, out=None) -> Request:
        """Queue sigma(grid; pts). out: None (a new host array), a host float64 array of
        [npts, n_grid], or a device tensor (written by the server's streams)."""
        p = self._pts(pts)
        if out is None:
            out = np.empty((len(p), self.grid_len(grid)), _out_np_dtype(opts))
        on_dev = not isinstance(out, np.ndarray)
        if not on_dev and (out.dtype != _out_np_dtype(opts) or not out.flags.c_contiguous):
            raise ValueError(f"host out must be C-contiguous {_out_np_dtype(opts).__name__}")
        h = C.c_uint64()
        self._check(self._L.xs_submit(self.h, lines, grid, p, len(p), C.byref(opts),
                                      _dev_ptr(out) if on_dev else _ptr(out), int(on_dev),
                                      C.byref(h)))
        return Request(self, h.value, out, (p,))

    def submit_window(self, lines: int, nu_start: float, step: float, n_points: int, pts,
                      opts: Opts, out=None) -> Request:
        """Queue sigma on the uniform grid nu_start + j*step, j < n_points."""
        p = self._pts(pts)
        if out is None:
            out = np.empty((len(p), n_points), _out_np_dtype(opts))
        on_dev = not isinstance(out, np.ndarray)
        if not on_dev and (out.dtype != _out_np_dtype(opts) or not out.flags.c_contiguous):
            raise ValueError(f"host out must be C-contiguous {_out_np_dtype(opts).__name__}")
        h = C.c_uint64()
        self._check(self._L.xs_submit_window(self.h, lines, float(nu_start), float(step),
                                             int(n_points), p, len(p), C.byref(opts),
                                             _dev_ptr(out) if on_dev else _ptr(out),
                                             int(on_dev), C.byref(h)))
        return Request(self, h.value, out, (p,))

    # ------------------------------------------------------------------ tuning
    def autotune(self, lines: int, grid: int, pts, opts: Opts) -> Dict[str, object]:
        """Time launch shapes on probes of this workload and cache the fastest for its
        class; returns the shape this workload now gets."""
        p = self._pts(pts)
        r = TuneResult()
        self._check(self._L.xs_autotune(self.h, lines, grid, p, len(p), C.byref(opts),
                                        C.byref(r)))
        return {"pts_per_lane": r.pts_per_lane, "split": r.split,
                "waves_per_simd": r.waves_per_simd, "items_per_slot": r.items_per_slot,
                "probe_ms": r.probe_ms, "default_probe_ms": r.default_probe_ms,
                "candidates": r.candidates, "key": r.key.decode()}

    def tune_key(self, lines: int, grid: int, npts: int, opts: Opts) -> str:
        buf = C.create_string_buffer(192)
        self._check(self._L.xs_tune_key(self.h, lines, grid, npts, C.byref(opts), buf, 192))
        return buf.value.decode()

    # ------------------------------------------------------------------ timing
    def set_kernel_timing(self, enable: bool = True):
        self._check(self._L.xs_set_kernel_timing(self.h, int(bool(enable))))

    def kernel_time(self):
        """(summed ms, launches) of the tile kernel since the previous call."""
        ms = C.c_double()
        n = C.c_int()
        self._check(self._L.xs_kernel_time(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # ------------------------------------------------------------------ graphs
    def graph_create(self, lines: int, grid: int, pts, opts: Opts, out) -> "Graph":
        p = self._pts(pts)
        g = C.c_void_p()
        self._check(self._L.xs_graph_create(self.h, lines, grid, p, len(p), C.byref(opts),
                                            _dev_ptr(out), C.byref(g)))
        return Graph(self, g.value)


class Graph:
    def __init__(self, ctx: Context, h: int):
        self.ctx = ctx
        self.h = h

    def launch(self, stream=None):
        self.ctx._check(self.ctx._L.xs_graph_launch(self.h, _stream_handle(stream)))

    def close(self):
        if self.h:
            self.ctx._L.xs_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
