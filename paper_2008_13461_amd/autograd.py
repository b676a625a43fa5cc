"""torch.autograd.Function around the broken-line fit and its adjoint.

    params, chi2 = broken_line_fit(x, y, z, layer, module, tuplets, nhits, offsets)

Forward runs pt_fit_broken_line; backward runs pt_fit_broken_line_bwd, which
recomputes the fit in registers instead of storing it.  Gradients flow to the
hit coordinates (x, y, z) and to the per-module alignment offsets.  Hits in
double select the double-precision fit; hits in float the single-precision
fit with the double refit of stiff tracks.
"""
from __future__ import annotations

import torch

from . import _abi as A
from . import api


class _Fit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, z, offsets, layer, module, tuplets, nhits, cfg_holder):
        cfg = cfg_holder.cfg
        precision = A.PT_FIT_F64 if x.dtype == torch.float64 else A.PT_FIT_F32_F64SOLVE
        hits = api.Hits(x.detach().contiguous(), y.detach().contiguous(), z.detach().contiguous(), layer, module,
                        torch.tensor([0, x.shape[0]], dtype=torch.int32, device=x.device))
        n = int(tuplets.shape[0])
        tup = api.Tuplets.from_rows(tuplets, nhits)
        tracks = api.Tracks.empty(n, precision, device=x.device)
        status = api.new_status(x.device)
        ws = api.new_workspace(api.workspace_size(cfg, hits.n_hits, 1, 0, 0, n), x.device)
        off = offsets.detach().contiguous() if offsets is not None else None
        api.fit_broken_line(hits, cfg, tup, off, precision, tracks, status, ws)
        ctx.save_for_backward(x, y, z, offsets if offsets is not None else torch.empty(0, device=x.device), layer,
                              module, tuplets, nhits)
        ctx.has_offsets = offsets is not None
        ctx.cfg_holder = cfg_holder
        ctx.precision = precision
        ctx.mark_non_differentiable(tracks.status)
        return tracks.params, tracks.chi2, tracks.status

    @staticmethod
    def backward(ctx, g_params, g_chi2, _g_status):
        x, y, z, offsets, layer, module, tuplets, nhits = ctx.saved_tensors
        cfg = ctx.cfg_holder.cfg
        hits = api.Hits(x.detach().contiguous(), y.detach().contiguous(), z.detach().contiguous(), layer, module,
                        torch.tensor([0, x.shape[0]], dtype=torch.int32, device=x.device))
        n = int(tuplets.shape[0])
        tup = api.Tuplets.from_rows(tuplets, nhits)
        status = api.new_status(x.device)
        ws = api.new_workspace(api.workspace_size(cfg, hits.n_hits, 1, 0, 0, n), x.device)
        # cotangents in the fit's precision: double for the double fit
        gdt = torch.float64 if ctx.precision == A.PT_FIT_F64 else torch.float32
        gp = (g_params if g_params is not None else torch.zeros((n, 5), device=x.device)).to(gdt).contiguous()
        gc = (g_chi2 if g_chi2 is not None else torch.zeros(n, device=x.device)).to(gdt).contiguous()
        gh = torch.zeros((hits.n_hits, 3), dtype=gdt, device=x.device)
        off = offsets if ctx.has_offsets else None
        go = torch.zeros((cfg.n_modules, 3), dtype=torch.float64, device=x.device) if ctx.has_offsets else None
        api.fit_broken_line_bwd(hits, cfg, tup, off, ctx.precision, gp, gc, gh, go, status, ws)
        gx, gy, gz = (gh[:, i].to(x.dtype) for i in range(3))
        goff = go.to(offsets.dtype) if go is not None else None
        return gx, gy, gz, goff, None, None, None, None, None


class FitConfig:
    """Holds the pt_config of a fit (an object, so autograd does not try to differentiate it)."""

    def __init__(self, cfg_dict: dict, **perf):
        self.cfg = A.make_config(cfg_dict, **perf)


def broken_line_fit(x, y, z, layer, module, tuplets, nhits, offsets=None, cfg: FitConfig | None = None):
    """Differentiable broken-line fit of the rows of `tuplets` ([n, 8] hit indices, -1 padded).

    Returns params [n, 5] = (kappa, phi0, cot(theta), d0, z0), chi2 [n], status [n].
    """
    if cfg is None:
        raise ValueError("pass a FitConfig")
    return _Fit.apply(x, y, z, offsets, layer, module, tuplets, nhits, cfg)
