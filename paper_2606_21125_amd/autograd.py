"""torch.autograd.Functions for the band-energy functional.

E(psi, V) = sum_i f_i <psi_i | H[V] | psi_i> with fixed weights f.  Forward and
backward call the HIP library (``dcdft_band_energy`` for one fragment,
``dcdft_band_energy_all`` for every fragment at once), which recomputes H psi
instead of storing it; the gradients are dE/dpsi_i = 2 f_i dV H psi_i and
dE/dV = dV sum_i f_i psi_i^2.  The binding only moves pointers.
"""
from __future__ import annotations

import torch

from .binding import PREC_FP64, PREC_MIXED


class BandEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi, veff, f, dcdft, frag):
        if psi.dtype not in (torch.float64, torch.float32):
            raise TypeError("psi must be float64 or float32")
        prec = PREC_FP64 if psi.dtype == torch.float64 else PREC_MIXED
        psi_c = psi.contiguous()
        veff_c = veff.contiguous().to(torch.float64)
        f_c = f.contiguous().to(torch.float64)
        energy = torch.empty(1, dtype=torch.float64, device=psi.device)
        dcdft.dcdft_band_energy(frag, psi_c, f_c, veff=veff_c, energy=energy, prec=prec)
        ctx.save_for_backward(psi_c, veff_c, f_c)
        ctx.dcdft = dcdft
        ctx.frag = frag
        ctx.prec = prec
        return energy[0]

    @staticmethod
    def backward(ctx, grad_out):
        psi, veff, f = ctx.saved_tensors
        gpsi = torch.empty_like(psi) if ctx.needs_input_grad[0] else None
        gv = torch.empty(veff.numel(), dtype=torch.float64, device=psi.device) \
            if ctx.needs_input_grad[1] else None
        ctx.dcdft.dcdft_band_energy(ctx.frag, psi, f, veff=veff, grad_psi=gpsi, grad_v=gv,
                                    prec=ctx.prec)
        g = grad_out.to(torch.float64)
        out_psi = None if gpsi is None else gpsi * g.to(gpsi.dtype)
        out_v = None if gv is None else (gv * g).reshape(veff.shape)
        return out_psi, out_v, None, None, None


def band_energy(dcdft, frag: int, psi, veff, f):
    """E(psi, V) of fragment frag through the HIP library, differentiable in psi and V."""
    return BandEnergy.apply(psi, veff, f, dcdft, frag)


class BandEnergyAll(torch.autograd.Function):
    """E of every fragment's vectors (fragment order, each fragment's V_eff of the
    last step), differentiable in psi."""

    @staticmethod
    def forward(ctx, psi, f, dcdft):
        if psi.dtype not in (torch.float64, torch.float32):
            raise TypeError("psi must be float64 or float32")
        prec = PREC_FP64 if psi.dtype == torch.float64 else PREC_MIXED
        psi_c = psi.contiguous()
        f_c = f.contiguous().to(torch.float64)
        energy = torch.empty(1, dtype=torch.float64, device=psi.device)
        # H psi needs a buffer of psi's type when the context's own is narrower
        hbuf = torch.empty_like(psi_c) if (prec == PREC_FP64 and
                                           int(dcdft.params.precision) != PREC_FP64) else None
        dcdft.dcdft_band_energy_all(psi_c, f_c, energy=energy, grad_psi=hbuf, prec=prec)
        ctx.save_for_backward(psi_c, f_c)
        ctx.dcdft = dcdft
        ctx.prec = prec
        return energy[0]

    @staticmethod
    def backward(ctx, grad_out):
        psi, f = ctx.saved_tensors
        if not ctx.needs_input_grad[0]:
            return None, None, None
        gpsi = torch.empty_like(psi)
        ctx.dcdft.dcdft_band_energy_all(psi, f, grad_psi=gpsi, prec=ctx.prec)
        return gpsi * grad_out.to(gpsi.dtype), None, None


def band_energy_all(dcdft, psi, f):
    """E of every fragment's vectors through the HIP library, differentiable in psi."""
    return BandEnergyAll.apply(psi, f, dcdft)
