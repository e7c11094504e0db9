"""The fit's chi2 as a differentiable function of the barrel-layer alignment
and the field scale.

`FitChi2` wraps the library's forward fit (run with a checkpoint of the
filtered state after every hit) and its hand-written reverse sweep
(kfx_fit_tracks_backward).  Both run on the GPU; torch only holds the device
memory and orders the calls on its current stream.

The paper (arXiv 2002.06295, Sec. 1) fits tracks with the Kalman filter over
the hits found by building; the alignment and field-scale parameters are an
addition for calibration, not part of the paper.
"""
from __future__ import annotations

import torch

from .kfx import Context, DeviceHits

DEFAULT_PRIOR = (0.1, 0.5, 0.05, 0.05)


class FitChi2(torch.autograd.Function):
    """chi2 per track (float32 [n_tracks], 0 for tracks that failed) as a
    function of align ([n_layers, 3] or [3 n_layers]: dr, drphi, dz; only
    barrel layers enter) and field_scale (a one-element tensor)."""

    @staticmethod
    def forward(ctx, align, field_scale, kctx: Context, hits: DeviceHits, trk_off, trk_hits, prior):
        a = align.detach().to(device=kctx.device, dtype=torch.float32).contiguous().reshape(-1)
        fs = float(field_scale.detach().reshape(-1)[0].item())
        out = kctx.fit_tracks(hits, trk_off, trk_hits, prior=prior, align=a, field_scale=fs, ckpt=True)
        n = int(trk_off.shape[0] - 1)
        ctx.kctx, ctx.hits, ctx.trk_off, ctx.trk_hits, ctx.prior = kctx, hits, trk_off, trk_hits, prior
        ctx.fit_out, ctx.a, ctx.fs = out, a, fs
        ctx.align_meta = (align.shape, align.dtype, align.device)
        ctx.fs_meta = (field_scale.shape, field_scale.dtype, field_scale.device)
        return out["chi2"][:n].clone()

    @staticmethod
    def backward(ctx, grad_chi2):
        dalign, dfield = ctx.kctx.fit_tracks_backward(ctx.hits, ctx.trk_off, ctx.trk_hits, ctx.fit_out, grad_chi2,
                                                      prior=ctx.prior, align=ctx.a, field_scale=ctx.fs)
        shape, dtype, dev = ctx.align_meta
        ga = dalign.to(device=dev, dtype=dtype).reshape(shape)
        shape, dtype, dev = ctx.fs_meta
        gf = dfield.to(device=dev, dtype=dtype).reshape(shape)
        return ga, gf, None, None, None, None, None


def fit_chi2(kctx: Context, hits: DeviceHits, trk_off, trk_hits, align, field_scale, prior=DEFAULT_PRIOR):
    """chi2 per track; differentiable in align and field_scale."""
    if not isinstance(field_scale, torch.Tensor):
        field_scale = torch.tensor([float(field_scale)], dtype=torch.float64)
    return FitChi2.apply(align, field_scale, kctx, hits, trk_off, trk_hits, prior)
