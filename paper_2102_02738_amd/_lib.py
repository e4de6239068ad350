"""ctypes binding of libsimus (include/simus.h): argument marshalling only.

Every computation runs in the HIP library; if the library is missing the
functions raise -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsimus.so")

SIMUS_OK = 0
ERRORS = {-1: "SIMUS_EINVAL", -2: "SIMUS_EDOMAIN", -3: "SIMUS_ENOMEM", -4: "SIMUS_EHIP",
          -5: "SIMUS_ETOOBIG"}
FLAG_NO_MFMA = 1
FLAG_PERSISTENT = 2
FLAG_NO_DELTA_TABLE = 4
FLAG_2D = 8
FLAG_STATIC = 16
FLAG_ALT_SHAPE = 32
FLAG_FP32_PRODUCTS = 64

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = ["simus_version", "simus_last_error", "simus_rf_grid", "simus_rf_spectrum", "simus_rf",
           "simus_rf_noalloc",
           "simus_spectrum_to_rf", "simus_rf_backward", "simus_pfield_nf", "simus_pfield",
           "simus_rf_plan_create", "simus_rf_plan_execute", "simus_rf_plan_graph_launch",
           "simus_rf_plan_autotune", "simus_tune_cache", "simus_tune_cache_hits", "simus_rf_plan_destroy",
           "simus_release_workspace", "simus_profile_enable", "simus_profile_read", "simus_profile_reset"]


class SimusError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Probe(C.Structure):
    _fields_ = [("n_elements", C.c_int32), ("baffle", C.c_int32), ("fc", C.c_double),
                ("pitch", C.c_double), ("width", C.c_double), ("height", C.c_double),
                ("elev_focus", C.c_double), ("bandwidth", C.c_double), ("radius", C.c_double),
                ("zeta", C.c_double)]


class Medium(C.Structure):
    _fields_ = [("c", C.c_double), ("alpha_db", C.c_double)]


class Options(C.Structure):
    _fields_ = [("fs", C.c_double), ("n_cycles", C.c_double), ("spectral_eps", C.c_double),
                ("nu", C.c_int32), ("nfft", C.c_int32), ("n_t", C.c_int32), ("flags", C.c_int32),
                ("n_gauss", C.c_int32), ("tile_scat", C.c_int32), ("gauss", C.c_void_p)]


class Grid(C.Structure):
    _fields_ = [("nfft", C.c_int32), ("n_t", C.c_int32), ("j_lo", C.c_int32), ("n_bins", C.c_int32),
                ("nu", C.c_int32), ("reserved", C.c_int32), ("df", C.c_double)]

    def as_dict(self):
        return dict(nfft=self.nfft, n_t=self.n_t, j_lo=self.j_lo, n_bins=self.n_bins, nu=self.nu,
                    df=self.df)


_lib = None


def lib():
    """Loads libsimus.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SimusError(-4, f"{LIB_PATH} is missing: run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        i32, i64, vp = C.c_int32, C.c_int64, C.c_void_p
        pd, pf, pi64, pi32 = P(C.c_double), P(C.c_float), P(C.c_int64), P(C.c_int32)
        pP, pM, pO, pG = P(Probe), P(Medium), P(Options), P(Grid)
        sig = {
            "simus_version": (C.c_int, []),
            "simus_last_error": (C.c_char_p, []),
            "simus_rf_grid": (C.c_int, [pP, pM, pO, i32, pd, i64, pf, pf, pf, pG]),
            "simus_rf_spectrum": (C.c_int, [pP, pM, pO, i32, pd, pf, i32, pi64, vp, vp, vp, vp, vp, vp]),
            "simus_rf": (C.c_int, [pP, pM, pO, i32, pd, pf, i32, pi64, vp, vp, vp, vp, vp, vp]),
            "simus_rf_noalloc": (C.c_int, [pP, pM, pO, i32, pd, pf, i32, pi64, vp, vp, vp, vp, vp, vp]),
            "simus_spectrum_to_rf": (C.c_int, [i32, i32, i32, i32, i64, vp, vp, vp]),
            "simus_rf_backward": (C.c_int, [pP, pM, pO, i32, pd, pf, i32, pi64, vp, vp, vp, vp, vp,
                                            vp, vp, vp, vp, vp]),
            "simus_pfield_nf": (C.c_int, [pP, pM, pO, pd, i64, pf, pf, pf, pi32]),
            "simus_pfield": (C.c_int, [pP, pM, pO, i32, pd, pf, i64, vp, vp, vp, vp, vp]),
            "simus_rf_plan_create": (C.c_int, [pP, pM, pO, i32, pd, pf, i32, pi64, i32, vp,
                                               P(C.c_void_p)]),
            "simus_rf_plan_execute": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
            "simus_rf_plan_graph_launch": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
            "simus_rf_plan_autotune": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, pi64, pi32]),
            "simus_tune_cache": (C.c_int, [C.c_char_p]),
            "simus_tune_cache_hits": (C.c_int64, []),
            "simus_rf_plan_destroy": (None, [vp]),
            "simus_release_workspace": (None, []),
            "simus_profile_enable": (C.c_int, [C.c_int]),
            "simus_profile_read": (C.c_int, [C.c_char_p, pd, pi64]),
            "simus_profile_reset": (None, []),
        }
        for name, (res, args) in sig.items():
            if not hasattr(L, name):
                continue
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int):
    if code != SIMUS_OK:
        raise SimusError(code, lib().simus_last_error().decode())


# ------------------------------------------------------------------ structs
def make_probe(p: dict) -> Probe:
    return Probe(int(p["n_elements"]), int(p.get("baffle", 0)), p["fc"], p["pitch"], p["width"],
                 p["height"], p.get("elev_focus", math.inf), p["bandwidth"], p.get("radius", 0.0),
                 p.get("zeta", 1.75))


def make_medium(m: dict) -> Medium:
    return Medium(m.get("c", 1540.0), m.get("alpha_db", 0.0))


def gauss_table(gset) -> np.ndarray:
    """A set of Gaussians (Eq. 12) as the ABI's [G][4] FP64 table (Re A, Im A,
    Re B, Im B); gset: (G, 2) complex (A_g, B_g), e.g. from gaussians.fit."""
    g = np.asarray(gset, dtype=np.complex128).reshape(-1, 2)
    return np.ascontiguousarray(np.stack([g[:, 0].real, g[:, 0].imag, g[:, 1].real, g[:, 1].imag], -1))


def make_options(o: dict, **over) -> Options:
    """options dict -> simus_options; o['gauss'] (optional) is a (G, 2) complex
    set of Gaussians, kept alive with the returned structure."""
    d = dict(o)
    d.update(over)
    gs = d.get("gauss")
    tab = None if gs is None else gauss_table(gs)
    opt = Options(d["fs"], d.get("n_cycles", 1.0), d.get("spectral_eps", 1e-7), int(d.get("nu", 0)),
                  int(d.get("nfft", 0)), int(d.get("n_t", 0)), int(d.get("flags", 0)),
                  0 if tab is None else tab.shape[0], int(d.get("tile_scat", 0)),
                  None if tab is None else tab.ctypes.data)
    opt._gauss_table = tab
    return opt


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(C.POINTER(t))


def _dev(t, like=None):
    """Device pointer of a contiguous float32 CUDA/HIP tensor (or None); with
    `like`, the tensor must sit on the same device."""
    if t is None:
        return None
    if not t.is_cuda:
        raise SimusError(-1, "device tensor expected")
    if not t.is_contiguous():
        raise SimusError(-1, "contiguous tensor expected")
    if like is not None and t.device != like.device:
        raise SimusError(-1, f"tensors on different devices ({t.device} and {like.device})")
    return C.c_void_p(t.data_ptr())


def _need(t, n: int, name: str):
    """The library takes raw device pointers to float32 data: refuse a tensor
    of another dtype, or one holding fewer than the n floats the call will
    read or write."""
    if t is None:
        return
    if str(t.dtype) != "torch.float32":
        raise SimusError(-1, f"{name} must be float32, not {t.dtype}")
    if t.numel() < n:
        raise SimusError(-1, f"{name} holds {t.numel() * t.element_size()} bytes, {4 * n} needed")


def _n_t(options: dict) -> int:
    """RF samples per channel the library writes: options n_t, else nfft."""
    return max(int(options.get("n_t", 0) or options.get("nfft", 0) or 0), 0)


def _scatterers(x, y, z, refl, offsets=None):
    """Scatterers the call reads (the last offset, else all of x); every
    array must hold that many floats."""
    n = x.numel() if offsets is None else int(np.asarray(offsets, dtype=np.int64)[-1])
    if offsets is not None and n > x.numel():
        raise SimusError(-1, f"scat_offsets end at {n}, x holds {x.numel()} scatterers")
    for t, name in ((x, "x"), (y, "y"), (z, "z"), (refl, "refl")):
        _need(t, n, name)
    return n


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ host-only
def rf_grid(probe: dict, medium: dict, options: dict, delays, x, y, z) -> dict:
    d = _f64(delays)
    n_tx = d.size // max(int(probe["n_elements"]), 1)
    xs, zs = _f32(x), _f32(z)
    ys = None if y is None else _f32(y)
    g = Grid()
    check(lib().simus_rf_grid(C.byref(make_probe(probe)), C.byref(make_medium(medium)),
                              C.byref(make_options(options)), n_tx, _p(d, C.c_double), xs.size,
                              _p(xs, C.c_float), None if ys is None else _p(ys, C.c_float),
                              _p(zs, C.c_float), C.byref(g)))
    return g.as_dict()


def pfield_nf(probe: dict, medium: dict, options: dict, delays, X, Y, Z) -> int:
    d = _f64(delays)
    Xs, Zs = _f32(X), _f32(Z)
    Ys = None if Y is None else _f32(Y)
    out = C.c_int32()
    check(lib().simus_pfield_nf(C.byref(make_probe(probe)), C.byref(make_medium(medium)),
                                C.byref(make_options(options)), _p(d, C.c_double), Xs.size,
                                _p(Xs, C.c_float), None if Ys is None else _p(Ys, C.c_float),
                                _p(Zs, C.c_float), C.byref(out)))
    return int(out.value)


# ------------------------------------------------------------------ device calls
def _tx(probe, delays, apod):
    d = _f64(delays)
    N = max(int(probe["n_elements"]), 1)
    n_tx = d.size // N
    if d.size != n_tx * N or n_tx < 1:
        raise SimusError(-1, f"delays hold {d.size} values, not n_tx x {N}")
    a = _f32(np.ones((n_tx, N)) if apod is None else apod)
    if a.size != n_tx * N:
        raise SimusError(-1, f"apod holds {a.size} values, delays {n_tx} x {N}")
    return d, a, n_tx


def _offsets(offsets, n_scat):
    o = np.ascontiguousarray(np.asarray([0, n_scat] if offsets is None else offsets, dtype=np.int64))
    return o, o.size - 1


def rf_spectrum_into(spec, probe, medium, options, delays, apod, x, y, z, refl,
                     offsets=None, stream=None):
    """spec must hold [n_phantoms][n_tx][N][n_bins] complex64 (as float32
    pairs), n_bins from rf_grid."""
    d, a, n_tx = _tx(probe, delays, apod)
    o, n_ph = _offsets(offsets, _scatterers(x, y, z, refl, offsets))
    n_bins = rf_grid(probe, medium, options, d.reshape(n_tx, -1), [], None, [])["n_bins"]
    _need(spec, 2 * n_ph * n_tx * int(probe["n_elements"]) * n_bins, "spec")
    check(lib().simus_rf_spectrum(C.byref(make_probe(probe)), C.byref(make_medium(medium)),
                                  C.byref(make_options(options)), n_tx, _p(d, C.c_double),
                                  _p(a, C.c_float), n_ph, _p(o, C.c_int64), _dev(x), _dev(y, x),
                                  _dev(z, x), _dev(refl, x), _dev(spec, x), _stream(stream)))


def rf_into(rf, probe, medium, options, delays, apod, x, y, z, refl, offsets=None, stream=None):
    d, a, n_tx = _tx(probe, delays, apod)
    o, n_ph = _offsets(offsets, _scatterers(x, y, z, refl, offsets))
    _need(rf, n_ph * n_tx * int(probe["n_elements"]) * _n_t(options), "rf")
    check(lib().simus_rf(C.byref(make_probe(probe)), C.byref(make_medium(medium)),
                         C.byref(make_options(options)), n_tx, _p(d, C.c_double), _p(a, C.c_float),
                         n_ph, _p(o, C.c_int64), _dev(x), _dev(y, x), _dev(z, x), _dev(refl, x),
                         _dev(rf, x), _stream(stream)))


def rf_noalloc_into(rf, probe, medium, options, delays, apod, x, y, z, refl, offsets=None,
                    stream=None):
    """simus_rf_noalloc: as rf_into, with the library's static scratch as
    workspace (no allocation)."""
    d, a, n_tx = _tx(probe, delays, apod)
    o, n_ph = _offsets(offsets, _scatterers(x, y, z, refl, offsets))
    _need(rf, n_ph * n_tx * int(probe["n_elements"]) * _n_t(options), "rf")
    check(lib().simus_rf_noalloc(C.byref(make_probe(probe)), C.byref(make_medium(medium)),
                                 C.byref(make_options(options)), n_tx, _p(d, C.c_double),
                                 _p(a, C.c_float), n_ph, _p(o, C.c_int64), _dev(x), _dev(y, x),
                                 _dev(z, x), _dev(refl, x), _dev(rf, x), _stream(stream)))


def spectrum_to_rf_into(rf, spec, nfft, n_t, j_lo, n_bins, n_chan, stream=None):
    _need(rf, max(int(n_chan), 0) * max(int(n_t), 0), "rf")
    _need(spec, 2 * max(int(n_chan), 0) * max(int(n_bins), 0), "spec")
    check(lib().simus_spectrum_to_rf(int(nfft), int(n_t), int(j_lo), int(n_bins), int(n_chan),
                                     _dev(spec), _dev(rf, spec), _stream(stream)))


def rf_backward_into(grads, probe, medium, options, delays, apod, x, y, z, refl, drf,
                     offsets=None, stream=None):
    """grads: dict with optional device tensors 'refl', 'x', 'y', 'z'."""
    d, a, n_tx = _tx(probe, delays, apod)
    n = _scatterers(x, y, z, refl, offsets)
    o, n_ph = _offsets(offsets, n)
    _need(drf, n_ph * n_tx * int(probe["n_elements"]) * _n_t(options), "drf")
    for k in ("refl", "x", "y", "z"):
        _need(grads.get(k), n, "gradient " + k)
    check(lib().simus_rf_backward(C.byref(make_probe(probe)), C.byref(make_medium(medium)),
                                  C.byref(make_options(options)), n_tx, _p(d, C.c_double),
                                  _p(a, C.c_float), n_ph, _p(o, C.c_int64), _dev(x), _dev(y, x),
                                  _dev(z, x), _dev(refl, x), _dev(drf, x),
                                  _dev(grads.get("refl"), x), _dev(grads.get("x"), x),
                                  _dev(grads.get("y"), x), _dev(grads.get("z"), x),
                                  _stream(stream)))


def pfield_into(p_rms, probe, medium, options, n_f, delays, apod, X, Y, Z, stream=None):
    n = X.numel()
    for t, name in ((X, "X"), (Y, "Y"), (Z, "Z"), (p_rms, "p_rms")):
        _need(t, n, name)
    d = _f64(delays)
    N = int(probe["n_elements"])
    if d.size != N:
        raise SimusError(-1, f"delays hold {d.size} values, the probe has {N} elements")
    a = _f32(np.ones(d.size) if apod is None else apod)
    if a.size != N:
        raise SimusError(-1, f"apod holds {a.size} values, the probe has {N} elements")
    check(lib().simus_pfield(C.byref(make_probe(probe)), C.byref(make_medium(medium)),
                             C.byref(make_options(options)), int(n_f), _p(d, C.c_double),
                             _p(a, C.c_float), X.numel(), _dev(X), _dev(Y, X), _dev(Z, X),
                             _dev(p_rms, X), _stream(stream)))


class RFPlan:
    """simus_rf_plan: the host work of simus_rf done once for a probe, medium,
    options, transmit sequence and partition into phantoms.  Executions take
    device scatterer tensors and write rf [n_phantoms, n_tx, N, n_t]."""

    def __init__(self, probe, medium, options, delays, apod, n_scat=None, offsets=None,
                 has_y=False, stream=None):
        d, a, n_tx = _tx(probe, delays, apod)
        if offsets is None and n_scat is None:
            raise SimusError(-1, "n_scat or offsets is required")
        o, n_ph = _offsets(offsets, n_scat)
        h = C.c_void_p()
        check(lib().simus_rf_plan_create(C.byref(make_probe(probe)), C.byref(make_medium(medium)),
                                         C.byref(make_options(options)), n_tx, _p(d, C.c_double),
                                         _p(a, C.c_float), n_ph, _p(o, C.c_int64),
                                         1 if has_y else 0, _stream(stream), C.byref(h)))
        self._h = h
        self.n_phantoms, self.n_tx, self.n_elements = n_ph, n_tx, int(probe["n_elements"])
        self.n_scat, self.n_t = int(o[-1]), _n_t(options)

    def _check_sizes(self, rf, x, y, z, refl):
        _need(x, self.n_scat, "x")
        _scatterers(x, y, z, refl, [0, self.n_scat])
        _need(rf, self.n_phantoms * self.n_tx * self.n_elements * self.n_t, "rf")

    def _ptrs(self, rf, x, y, z, refl):
        return _dev(x), _dev(y, x), _dev(z, x), _dev(refl, x), _dev(rf, x)

    def execute_into(self, rf, x, y, z, refl, stream=None):
        self._check_sizes(rf, x, y, z, refl)
        check(lib().simus_rf_plan_execute(self._handle(), *self._ptrs(rf, x, y, z, refl),
                                          _stream(stream)))

    def graph_launch_into(self, rf, x, y, z, refl, stream=None):
        self._check_sizes(rf, x, y, z, refl)
        check(lib().simus_rf_plan_graph_launch(self._handle(), *self._ptrs(rf, x, y, z, refl),
                                               _stream(stream)))

    def autotune_into(self, rf, x, y, z, refl, stream=None) -> dict:
        """Runs the plan's autotuner on these scatterers; returns the chosen
        options (tile_scat, flags)."""
        self._check_sizes(rf, x, y, z, refl)
        ts = C.c_int64()
        fl = C.c_int32()
        check(lib().simus_rf_plan_autotune(self._handle(), *self._ptrs(rf, x, y, z, refl),
                                           _stream(stream), C.byref(ts), C.byref(fl)))
        return dict(tile_scat=int(ts.value), flags=int(fl.value))

    def _handle(self):
        if not self._h:
            raise SimusError(-1, "plan is closed")
        return self._h

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _lib is not None:
            _lib.simus_rf_plan_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def release_workspace():
    lib().simus_release_workspace()


def tune_cache(path):
    """Sets (or, with None, clears) the autotuner's file cache of choices."""
    check(lib().simus_tune_cache(os.fsencode(path) if path else None))


def tune_cache_hits() -> int:
    """Autotuner calls of this process answered from the cache."""
    return int(lib().simus_tune_cache_hits())


def profile_enable(on: bool = True):
    check(lib().simus_profile_enable(1 if on else 0))


def profile_reset():
    lib().simus_profile_reset()


def profile_read(kernel: str):
    """(total_ms, launches) of one library kernel since the last reset."""
    ms = C.c_double()
    n = C.c_int64()
    check(lib().simus_profile_read(kernel.encode(), C.byref(ms), C.byref(n)))
    return float(ms.value), int(n.value)
