"""torch.autograd.Function over simus_rf / simus_rf_backward.

The forward call runs the HIP synthesis; the backward call runs the
hand-written adjoint kernels, which recompute the Green's terms per
frequency bin (nothing but the inputs is kept from the forward pass).
Gradients flow to the reflectivities and the scatterer positions.

The frequency grid must be frozen across calls: pass options with 'nfft'
and 'n_t' set (see paper_2102_02738_amd.grid).
"""
from __future__ import annotations

import torch

from . import _lib


class SimusRF(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, z, refl, call: dict):
        o = call["options"]
        if not o.get("nfft"):
            raise _lib.SimusError(-1, "options['nfft'] must be fixed for differentiation")
        offsets = call.get("offsets")
        n_ph = 1 if offsets is None else len(offsets) - 1
        T = len(call["delays"])
        N = int(call["probe"]["n_elements"])
        n_t = o.get("n_t") or o["nfft"]
        rf = torch.empty((n_ph, T, N, n_t), dtype=torch.float32, device=x.device)
        _lib.rf_into(rf, call["probe"], call["medium"], o, call["delays"], call.get("apod"),
                     x.contiguous(), None if y is None else y.contiguous(), z.contiguous(),
                     refl.contiguous(), offsets)
        ctx.call = call
        ctx.has_y = y is not None
        ctx.save_for_backward(x, y if y is not None else x, z, refl)
        return rf

    @staticmethod
    def backward(ctx, grad_rf):
        x, y, z, refl = ctx.saved_tensors
        y = y if ctx.has_y else None
        c = ctx.call
        need = {}
        if ctx.needs_input_grad[0]:
            need["x"] = torch.empty_like(x)
        if ctx.needs_input_grad[1] and y is not None:
            need["y"] = torch.empty_like(x)
        if ctx.needs_input_grad[2]:
            need["z"] = torch.empty_like(x)
        if ctx.needs_input_grad[3]:
            need["refl"] = torch.empty_like(x)
        if need:
            _lib.rf_backward_into(need, c["probe"], c["medium"], c["options"], c["delays"],
                                  c.get("apod"), x.contiguous(), None if y is None else y.contiguous(),
                                  z.contiguous(), refl.contiguous(), grad_rf.contiguous(),
                                  c.get("offsets"))
        return need.get("x"), need.get("y"), need.get("z"), need.get("refl"), None


def simus_rf_autograd(probe, medium, options, delays, apod, x, y, z, refl, offsets=None):
    """Differentiable RF [n_phantoms, n_tx, N, n_t]."""
    call = dict(probe=probe, medium=medium, options=options, delays=delays, apod=apod,
                offsets=offsets)
    return SimusRF.apply(x, y, z, refl, call)
