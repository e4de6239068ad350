"""Python face of the FP64 SIMUS oracle (``oracle/simus_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg are the only callers.  The product library never imports this
module, and this module imports nothing from the product package.

The functions below marshal numpy arrays into the C oracle; every piece of
arithmetic lives in the C file, written term by term from the paper
(Eqs. 10-42 of SIMUS Part I).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "simus_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
            "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Setup(C.Structure):
    _fields_ = [
        ("n_elements", C.c_int32), ("nu", C.c_int32),
        ("fc", C.c_double), ("pitch", C.c_double), ("width", C.c_double),
        ("height", C.c_double), ("elev_focus", C.c_double),
        ("bandwidth", C.c_double), ("radius", C.c_double),
        ("baffle", C.c_int32), ("pad0", C.c_int32), ("zeta", C.c_double),
        ("c", C.c_double), ("alpha_db", C.c_double),
        ("fs", C.c_double), ("n_cycles", C.c_double),
        ("dim2", C.c_int32), ("pad1", C.c_int32),
        ("n_gauss", C.c_int32), ("pad2", C.c_int32), ("gauss", C.c_void_p),
    ]


@dataclass
class Setup:
    """Probe + medium + pulse, SI units (mirrors the C struct)."""
    n_elements: int
    fc: float
    pitch: float
    width: float
    height: float
    elev_focus: float
    bandwidth: float
    c: float = 1540.0
    alpha_db: float = 0.0
    fs: float = 0.0
    n_cycles: float = 1.0
    radius: float = 0.0
    baffle: int = 0
    zeta: float = 1.75
    nu: int = 0          # 0: Eq. (21)
    dim2: int = 0        # 1: 2-D acoustics (Section V)
    gauss: object = None  # Gaussians of Eq. (12): complex pairs [(A_g, B_g)], None: Eq. (18)

    def resolved_nu(self) -> int:
        if self.nu > 0:
            return self.nu
        return nu_eq21(self.width, self.fc, self.bandwidth, self.c)

    def to_c(self) -> _Setup:
        n_g, ptr = 0, None
        if self.gauss is not None:
            ab = np.asarray(self.gauss, dtype=np.complex128).reshape(-1, 2)
            self._gbuf = np.ascontiguousarray(np.stack([ab[:, 0].real, ab[:, 0].imag,
                                                        ab[:, 1].real, ab[:, 1].imag], -1))
            n_g, ptr = ab.shape[0], self._gbuf.ctypes.data
        return _Setup(self.n_elements, self.resolved_nu(), self.fc, self.pitch,
                      self.width, self.height, self.elev_focus, self.bandwidth,
                      self.radius, self.baffle, 0, self.zeta, self.c,
                      self.alpha_db, self.fs, self.n_cycles, int(self.dim2), 0, n_g, 0, ptr)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        pd, pi32, pi64 = P(d), P(i32), P(i64)
        ps = P(_Setup)
        sig = {
            "oracle_nu": (i32, [d, d, d, d]),
            "oracle_subelements": (None, [ps, pd, pd, pd, pd, pd, pd]),
            "oracle_pulse_spectrum": (None, [ps, d, pd]),
            "oracle_transducer_spectrum": (d, [ps, d]),
            "oracle_green": (None, [ps, i32, d, d, d, d, pd]),
            "oracle_delta": (None, [ps, d, d, d, pd]),
            "oracle_directivity": (d, [ps, d, d, d, d]),
            "oracle_band": (None, [ps, i32, d, pi32]),
            "oracle_grid": (None, [ps, i32, i32, d, i32, pd, i64, pd, pd, pd, pi32]),
            "oracle_spectrum": (None, [ps, i32, i32, pd, pd, i64, pd, pd, pd, pd, i32, pi32, pd]),
            "oracle_rf_from_spectrum": (None, [i32, i32, i32, pi32, i64, pd, pd]),
            "oracle_residual_spectrum": (None, [i32, i32, i32, pi32, i64, pd, pd]),
            "oracle_adjoint": (None, [ps, i32, i32, pd, pd, pd, pd, pd, pd, i32, pi32, pd,
                                      i32, pi64, pd, pd, pd, pd]),
            "oracle_pfield_nf": (i32, [ps, pd, i64, pd, pd, pd]),
            "oracle_field": (None, [ps, pd, pd, i32, pd, i64, pd, pd, pd, pd]),
            "oracle_pfield": (None, [ps, pd, pd, i32, i64, pd, pd, pd, pd]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray, ctype=C.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


# ---------------------------------------------------------------- scalars
def nu_eq21(width, fc, bandwidth, c) -> int:
    return int(lib().oracle_nu(width, fc, bandwidth, c))


def subelements(su: Setup):
    """Sub-element centroids, tangents and normals (Eq. 24; convex reading)."""
    M = su.n_elements * su.resolved_nu()
    arrs = [np.zeros(M) for _ in range(6)]
    lib().oracle_subelements(C.byref(su.to_c()), *[_ptr(a) for a in arrs])
    return dict(zip(["xc", "zc", "tx", "tz", "nx", "nz"], arrs))


def pulse_spectrum(su: Setup, w: float) -> complex:
    out = np.zeros(2)
    lib().oracle_pulse_spectrum(C.byref(su.to_c()), float(w), _ptr(out))
    return complex(out[0], out[1])


def transducer_spectrum(su: Setup, w: float) -> float:
    return float(lib().oracle_transducer_spectrum(C.byref(su.to_c()), float(w)))


def green(su: Setup, n: int, X: float, Y: float, Z: float, w: float) -> complex:
    out = np.zeros(2)
    lib().oracle_green(C.byref(su.to_c()), int(n), X, Y, Z, w, _ptr(out))
    return complex(out[0], out[1])


def delta(su: Setup, y: float, r: float, k: float) -> complex:
    out = np.zeros(2)
    lib().oracle_delta(C.byref(su.to_c()), y, r, k, _ptr(out))
    return complex(out[0], out[1])


def directivity(su: Setup, sin_t, cos_t, k, b_sub) -> float:
    return float(lib().oracle_directivity(C.byref(su.to_c()), sin_t, cos_t, k, b_sub))


# ---------------------------------------------------------------- grid
def band(su: Setup, nfft: int, eps: float = 1e-7):
    out = (C.c_int32 * 2)()
    lib().oracle_band(C.byref(su.to_c()), int(nfft), float(eps), out)
    return int(out[0]), int(out[1])


def grid(su: Setup, delays, x, y, z, n_t: int = 0, nfft: int = 0, eps: float = 1e-7):
    """Returns dict(nfft, n_t, j_lo, n_bins)."""
    delays = _f64(delays)
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = (C.c_int32 * 4)()
    n_tx = delays.size // su.n_elements
    lib().oracle_grid(C.byref(su.to_c()), int(n_t), int(nfft), float(eps), n_tx,
                      _ptr(delays), x.size, _ptr(x), _ptr(y), _ptr(z), out)
    return dict(nfft=int(out[0]), n_t=int(out[1]), j_lo=int(out[2]), n_bins=int(out[3]))


# ---------------------------------------------------------------- spectra / RF
def spectrum(su: Setup, nfft: int, delays, apod, x, y, z, R, bins) -> np.ndarray:
    """Direct-sum element spectra X[t, e, b] (complex128) at absolute bins."""
    delays, apod = _f64(delays), _f64(apod)
    x, y, z, R = _f64(x), _f64(y), _f64(z), _f64(R)
    bins = np.ascontiguousarray(np.asarray(bins, dtype=np.int32))
    N = su.n_elements
    n_tx = delays.size // N
    out = np.zeros((n_tx, N, bins.size, 2))
    lib().oracle_spectrum(C.byref(su.to_c()), int(nfft), n_tx, _ptr(delays), _ptr(apod),
                          x.size, _ptr(x), _ptr(y), _ptr(z), _ptr(R),
                          bins.size, _ptr(bins, C.c_int32), _ptr(out))
    return out[..., 0] + 1j * out[..., 1]


def rf_from_spectrum(X: np.ndarray, bins, nfft: int, n_t: int) -> np.ndarray:
    """Explicit inverse DFT of Eq. (1): X[..., b] -> rf[..., q]."""
    bins = np.ascontiguousarray(np.asarray(bins, dtype=np.int32))
    lead = X.shape[:-1]
    Xc = np.ascontiguousarray(np.stack([X.real, X.imag], -1).reshape(-1, bins.size, 2))
    rf = np.zeros((Xc.shape[0], n_t))
    lib().oracle_rf_from_spectrum(int(nfft), int(n_t), bins.size, _ptr(bins, C.c_int32),
                                  Xc.shape[0], _ptr(Xc), _ptr(rf))
    return rf.reshape(*lead, n_t)


def residual_spectrum(rho: np.ndarray, bins, nfft: int) -> np.ndarray:
    bins = np.ascontiguousarray(np.asarray(bins, dtype=np.int32))
    lead = rho.shape[:-1]
    n_t = rho.shape[-1]
    r = _f64(rho).reshape(-1, n_t)
    lam = np.zeros((r.shape[0], bins.size, 2))
    lib().oracle_residual_spectrum(int(nfft), int(n_t), bins.size, _ptr(bins, C.c_int32),
                                   r.shape[0], _ptr(r), _ptr(lam))
    return (lam[..., 0] + 1j * lam[..., 1]).reshape(*lead, bins.size)


def all_bins(g) -> np.ndarray:
    return np.arange(g["j_lo"], g["j_lo"] + g["n_bins"], dtype=np.int32)


def rf(su: Setup, g, delays, apod, x, y, z, R) -> np.ndarray:
    """Full RF [n_tx, N, n_t] by the direct sum + explicit inverse DFT."""
    bins = all_bins(g)
    X = spectrum(su, g["nfft"], delays, apod, x, y, z, R, bins)
    return rf_from_spectrum(X, bins, g["nfft"], g["n_t"])


def adjoint(su: Setup, g, delays, apod, x, y, z, R, rho, sel=None):
    """Gradients of L = 1/2 sum rho^2 (rho = dL/drf) w.r.t. R, x, y, z."""
    bins = all_bins(g)
    lam = residual_spectrum(np.asarray(rho), bins, g["nfft"])
    lam2 = np.ascontiguousarray(np.stack([lam.real, lam.imag], -1))
    delays, apod = _f64(delays), _f64(apod)
    x, y, z, R = _f64(x), _f64(y), _f64(z), _f64(R)
    if sel is None:
        sel = np.arange(x.size)
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    outs = [np.zeros(sel.size) for _ in range(4)]
    n_tx = delays.size // su.n_elements
    lib().oracle_adjoint(C.byref(su.to_c()), g["nfft"], n_tx, _ptr(delays), _ptr(apod),
                         _ptr(x), _ptr(y), _ptr(z), _ptr(R), bins.size, _ptr(bins, C.c_int32),
                         _ptr(lam2), sel.size, _ptr(sel, C.c_int64), *[_ptr(o) for o in outs])
    return dict(zip(["R", "x", "y", "z"], outs))


# ---------------------------------------------------------------- field
def pfield_nf(su: Setup, delays, X, Y, Z) -> int:
    delays = _f64(delays)
    X, Y, Z = _f64(X), _f64(Y), _f64(Z)
    return int(lib().oracle_pfield_nf(C.byref(su.to_c()), _ptr(delays), X.size,
                                      _ptr(X), _ptr(Y), _ptr(Z)))


def field(su: Setup, delays, apod, ws, X, Y, Z) -> np.ndarray:
    delays, apod, ws = _f64(delays), _f64(apod), _f64(ws)
    X, Y, Z = _f64(X), _f64(Y), _f64(Z)
    out = np.zeros((X.size, ws.size, 2))
    lib().oracle_field(C.byref(su.to_c()), _ptr(delays), _ptr(apod), ws.size, _ptr(ws),
                       X.size, _ptr(X), _ptr(Y), _ptr(Z), _ptr(out))
    return out[..., 0] + 1j * out[..., 1]


def pfield(su: Setup, delays, apod, n_f: int, X, Y, Z) -> np.ndarray:
    delays, apod = _f64(delays), _f64(apod)
    X, Y, Z = _f64(X), _f64(Y), _f64(Z)
    out = np.zeros(X.size)
    lib().oracle_pfield(C.byref(su.to_c()), _ptr(delays), _ptr(apod), int(n_f), X.size,
                        _ptr(X), _ptr(Y), _ptr(Z), _ptr(out))
    return out
