"""MI355X (gfx950) implementation of the SIMUS radio-frequency synthesis
(D. Garcia, "SIMUS: an open-source simulator for medical ultrasound
imaging. Part I: theory & examples").

The compute path is libsimus.so (HIP kernels behind the C ABI declared in
include/simus.h).  This package only marshals arguments: PyTorch provides
device memory and streams.  Nothing here computes RF on the host, and every
call raises if the library has not been built.

    probe, medium, options: dicts (see inputs.linear_probe / inputs.workload)
    delays, apod: host arrays [n_tx, N]
    x, y, z, refl: device float32 tensors [S] (y may be None: y = 0)
"""
from __future__ import annotations

from . import _lib
from ._lib import SimusError, FLAG_NO_MFMA, FLAG_PERSISTENT, FLAG_NO_DELTA_TABLE, FLAG_2D, FLAG_STATIC, FLAG_ALT_SHAPE, FLAG_FP32_PRODUCTS  # noqa: F401

__all__ = ["grid", "rf", "rf_spectrum", "spectrum_to_rf", "rf_backward", "pfield", "pfield_nf",
           "RFPlan", "rf_plan", "SimusRF", "simus_rf_autograd", "release_workspace", "tune_cache",
           "tune_cache_hits", "SimusError"]


def _opts_with_grid(options: dict, g: dict) -> dict:
    o = dict(options)
    o["nfft"] = g["nfft"]
    o["n_t"] = g["n_t"]
    if g.get("nu"):
        o["nu"] = g["nu"]
    return o


def grid(probe, medium, options, delays, x, y, z) -> dict:
    """Frequency grid of a call (host-only, see simus_rf_grid).  x, y, z may be
    host arrays or device tensors (copied to the host once)."""
    def host(a):
        if a is None:
            return None
        if hasattr(a, "detach"):
            return a.detach().float().cpu().numpy()
        return a
    return _lib.rf_grid(probe, medium, options, delays, host(x), host(y), host(z))


def _n_phantoms(offsets):
    return 1 if offsets is None else len(offsets) - 1


def rf(probe, medium, options, delays, apod, x, y, z, refl, offsets=None, stream=None):
    """RF signals [n_phantoms, n_tx, N, n_t] (device float32).  options['nfft']
    must be set (use grid())."""
    import torch
    n_tx = len(delays)
    N = int(probe["n_elements"])
    n_t = options["n_t"] or options["nfft"]
    out = torch.empty((_n_phantoms(offsets), n_tx, N, n_t), dtype=torch.float32, device=x.device)
    _lib.rf_into(out, probe, medium, options, delays, apod, x, y, z, refl, offsets, stream)
    return out


def rf_spectrum(probe, medium, options, delays, apod, x, y, z, refl, offsets=None, stream=None,
                n_bins=None):
    """Element spectra [n_phantoms, n_tx, N, n_bins] as complex64 (device)."""
    import torch
    if n_bins is None:
        n_bins = _lib.rf_grid(probe, medium, options, delays, [], None, [])["n_bins"]
    n_tx = len(delays)
    N = int(probe["n_elements"])
    out = torch.empty((_n_phantoms(offsets), n_tx, N, n_bins, 2), dtype=torch.float32, device=x.device)
    _lib.rf_spectrum_into(out, probe, medium, options, delays, apod, x, y, z, refl, offsets, stream)
    return torch.view_as_complex(out)


def spectrum_to_rf(spec, nfft, n_t, j_lo, stream=None):
    """Inverse transform alone: spec complex64 [..., n_bins] -> rf [..., n_t]."""
    import torch
    s = torch.view_as_real(spec.contiguous()).contiguous()
    lead = spec.shape[:-1]
    n_chan = 1
    for d in lead:
        n_chan *= d
    out = torch.empty((*lead, n_t), dtype=torch.float32, device=spec.device)
    _lib.spectrum_to_rf_into(out, s, nfft, n_t, j_lo, spec.shape[-1], n_chan, stream)
    return out


def rf_backward(probe, medium, options, delays, apod, x, y, z, refl, drf, offsets=None,
                stream=None, need=("refl", "x", "y", "z")):
    """Gradients dL/d{refl, x, y, z} given drf = dL/drf (device tensors)."""
    import torch
    grads = {}
    for k in need:
        if k == "y" and y is None:
            continue
        grads[k] = torch.empty_like(x)
    _lib.rf_backward_into(grads, probe, medium, options, delays, apod, x, y, z, refl,
                          drf.contiguous(), offsets, stream)
    return grads


def pfield_nf(probe, medium, options, delays, X, Y, Z) -> int:
    return _lib.pfield_nf(probe, medium, options, delays, X, Y, Z)


def pfield(probe, medium, options, n_f, delays, apod, X, Y, Z, stream=None):
    """RMS pressure field at device points X, Y, Z (Y may be None)."""
    import torch
    out = torch.empty_like(X)
    _lib.pfield_into(out, probe, medium, options, n_f, delays, apod, X, Y, Z, stream)
    return out


class RFPlan(_lib.RFPlan):
    """Forward plan (see rf_plan)."""

    def _out(self, x, n_t):
        import torch
        if n_t is not None and int(n_t) != self.n_t:
            raise SimusError(-1, f"the plan writes {self.n_t} samples per channel, not {n_t}")
        return torch.empty((self.n_phantoms, self.n_tx, self.n_elements, self.n_t),
                           dtype=torch.float32, device=x.device)

    def rf(self, x, y, z, refl, n_t=None, graph=False, stream=None):
        """RF [n_phantoms, n_tx, N, n_t] of the plan for device scatterers; with
        graph=True through the plan's captured HIP graph.  n_t, if given, must
        be the plan's."""
        out = self._out(x, n_t)
        (self.graph_launch_into if graph else self.execute_into)(out, x, y, z, refl, stream)
        return out

    def autotune(self, x, y, z, refl, n_t=None, stream=None) -> dict:
        """Times launch shapes on these scatterers and keeps the fastest in the
        plan; returns the chosen options (tile_scat, flags)."""
        out = self._out(x, n_t)
        return self.autotune_into(out, x, y, z, refl, stream)


def rf_plan(probe, medium, options, delays, apod, n_scat=None, offsets=None, has_y=False,
            stream=None) -> RFPlan:
    """Plans simus_rf once for a fixed probe, transmit sequence and phantom
    partition (offsets, or one phantom of n_scat scatterers); options['nfft']
    must be set (use grid())."""
    return RFPlan(probe, medium, options, delays, apod, n_scat, offsets, has_y, stream)


def release_workspace():
    _lib.release_workspace()


def tune_cache(path):
    """File cache of the autotuner's choices per problem class (None: off)."""
    _lib.tune_cache(path)


def tune_cache_hits() -> int:
    return _lib.tune_cache_hits()


def __getattr__(name):
    if name in ("SimusRF", "simus_rf_autograd"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
