"""Coefficient sets of the Gaussian superposition that replaces the element's
rectangular elevation aperture (SIMUS Part I, Section II-B, Eqs. 12-18):

    Pi(u) ~ sum_g A_g exp(-B_g u^2),  u = y' / h.

A set is an input of the model, like the probe's geometry: the library
(options ``gauss``) and the FP64 oracle (``Setup.gauss``) both take it as an
argument.  This module computes none of the RF synthesis.  It gives

* ``EQ18``: the four Gaussians printed in Eq. (18), the default of both;
* ``fit(G)``: G Gaussians (G/2 conjugate pairs, so that the sum is real)
  fitted by the criterion the paper states for its sets: least squares of
  the difference rectangle - sum of Gaussians over u in [-2, 2];
* ``l2_error(set)``: that criterion's value for a set.

Sets are arrays of shape (G, 2), complex: column 0 = A_g, column 1 = B_g.
"""
from __future__ import annotations

import functools

import numpy as np

EQ18 = np.array([[0.187 + 0.275j, 4.558 - 25.59j],
                 [0.288 - 1.954j, 8.598 - 7.924j],
                 [0.187 - 0.275j, 4.558 + 25.59j],
                 [0.288 + 1.954j, 8.598 + 7.924j]])

# Least-squares nodes: u in [0, 2] (the criterion is even in u; weights
# doubled for [-2, 0]), Simpson's rule on each piece where Pi is constant,
# [0, 1/2] (Pi = 1) and [1/2, 2] (Pi = 0), so that the jump at the
# rectangle's edge costs no accuracy (u = 1/2 is a node of both pieces).
def _piece(a: float, b: float, n: int, value: float):
    u = np.linspace(a, b, n)          # n odd
    w = np.full(n, 2.0)
    w[1::2] = 4.0
    w[0] = w[-1] = 1.0
    return u, w * (u[1] - u[0]) / 3.0, np.full(n, value)


_P1, _P2 = _piece(0.0, 0.5, 1001, 1.0), _piece(0.5, 2.0, 3001, 0.0)
_U = np.concatenate([_P1[0], _P2[0]])
_W = np.concatenate([_P1[1], _P2[1]])
_RECT = np.concatenate([_P1[2], _P2[2]])
_NU = _U.size
_SW = np.sqrt(2.0 * _W)


def expand(pairs: np.ndarray) -> np.ndarray:
    """(P, 2) complex pairs (A, B) -> the (2P, 2) set with their conjugates."""
    pairs = np.asarray(pairs, dtype=np.complex128).reshape(-1, 2)
    return np.concatenate([pairs, np.conj(pairs)])


def _pairs_of(params: np.ndarray) -> np.ndarray:
    a = params[0::4] + 1j * params[1::4]
    b = params[2::4] + 1j * params[3::4]
    return np.stack([a, b], -1)


def _params_of(pairs: np.ndarray) -> np.ndarray:
    pairs = np.asarray(pairs, dtype=np.complex128).reshape(-1, 2)
    return np.stack([pairs[:, 0].real, pairs[:, 0].imag, pairs[:, 1].real, pairs[:, 1].imag],
                    -1).ravel()


def _residual(params: np.ndarray) -> np.ndarray:
    p = _pairs_of(params)
    e = np.exp(-p[None, :, 1] * _U[:, None] ** 2)
    return _SW * (_RECT - 2.0 * np.real(e @ p[:, 0]))


def _jacobian(params: np.ndarray) -> np.ndarray:
    p = _pairs_of(params)
    e = np.exp(-p[None, :, 1] * _U[:, None] ** 2)          # [u, pair]
    ae = e * p[None, :, 0]
    u2 = _U[:, None] ** 2
    J = np.empty((_NU, params.size))
    # d/d(Re A, Im A, Re B, Im B) of 2 Re(A e^{-B u^2})
    J[:, 0::4] = 2.0 * e.real
    J[:, 1::4] = -2.0 * e.imag
    J[:, 2::4] = -2.0 * (u2 * ae).real
    J[:, 3::4] = 2.0 * (u2 * ae).imag
    return -_SW[:, None] * J


def l2_error(gset) -> float:
    """sqrt of the integral over [-2, 2] of |Pi(u) - sum_g A_g e^{-B_g u^2}|^2
    (Simpson's rule with 0.5e-3 steps on each piece; imaginary parts count
    too)."""
    g = np.asarray(gset, dtype=np.complex128).reshape(-1, 2)
    s = np.exp(-g[None, :, 1] * _U[:, None] ** 2) @ g[:, 0]
    return float(np.sqrt(np.sum(2.0 * _W * np.abs(_RECT - s) ** 2)))


def _lsq(params0: np.ndarray, max_nfev: int) -> np.ndarray:
    from scipy.optimize import least_squares
    with np.errstate(all="ignore"):
        r = least_squares(_residual, params0, jac=_jacobian, method="lm", xtol=1e-15,
                          ftol=1e-15, max_nfev=max_nfev)
    return r.x


@functools.lru_cache(maxsize=None)
def _fit_pairs(n_pairs: int) -> tuple:
    if n_pairs < 1:
        raise ValueError("at least one conjugate pair")
    if n_pairs == 1:
        starts = [_params_of(EQ18[:1])]
    elif n_pairs == 2:
        starts = [_params_of(EQ18[:2])]
    else:
        # continuation: the best set of one pair fewer, plus a new pair tried
        # from a fixed grid of starting exponents
        prev = _params_of(np.asarray(_fit_pairs(n_pairs - 1)))
        starts = [np.concatenate([prev, [0.05, 0.05, br, bi]])
                  for br in (2.0, 5.0, 10.0, 15.0) for bi in (-80.0, -50.0, -30.0, -10.0)]
    best, best_err = None, np.inf
    for p0 in starts:
        x = _lsq(p0, 20000)
        if not np.all(np.isfinite(x)) or not np.all(x[2::4] > 0):
            continue
        err = float(np.sqrt(np.sum(_residual(x) ** 2)))
        if err < best_err:
            best, best_err = x, err
    if best is None:
        raise RuntimeError(f"no fit of {2 * n_pairs} Gaussians converged")
    return tuple(map(tuple, _pairs_of(best)))


def fit(G: int) -> np.ndarray:
    """G Gaussians (G even: G/2 conjugate pairs) minimising l2_error; the
    two-pair fit starts from Eq. (18), each larger one from the fit with one
    pair fewer.  Deterministic.  Returns the (G, 2) set."""
    if G < 2 or G % 2:
        raise ValueError("G must be even and >= 2 (conjugate pairs)")
    return expand(np.asarray(_fit_pairs(G // 2), dtype=np.complex128))
