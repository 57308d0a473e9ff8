"""torch.autograd binding of the differentiable refit: chi2 per track as a
function of raw hit coordinates and the 16 calibration parameters.  The
backward pass is the library's hand-written adjoint."""
from __future__ import annotations

import torch

from . import api


class RefitFunction(torch.autograd.Function):
    """chi2[k] = refit chi2 of track k.  Inputs: y, z raw hit coordinates
    (one per hit entry, or one per cluster when the track CSR carries
    cluster ids), theta [16]; non-tensor context: the library context, the
    track CSR (TrackHits), row geometry and parameters."""

    @staticmethod
    def forward(fctx, y, z, theta, tctx, hits, row_x, prm, cm=None):
        y = y.detach().contiguous()
        z = z.detach().contiguous()
        out = api.refit(tctx, hits, row_x, prm, theta, checkpoints=True, cm=cm, y=y, z=z)
        fctx.tctx, fctx.hits, fctx.row_x, fctx.prm, fctx.cm = tctx, hits, row_x, prm, cm
        fctx.fwd = out
        fctx.save_for_backward(y, z, theta)
        fctx.mark_non_differentiable(out["status"])
        return out["chi2"], out["status"]

    @staticmethod
    def backward(fctx, grad_chi2, _grad_status):
        y, z, theta = fctx.saved_tensors
        hits = fctx.hits
        out = None
        if hits.idx is not None:
            # per-entry gradients start at zero, so entries past the device
            # track count (never written) add nothing below
            m = max(hits.n_hits, 1)
            out = dict(gy=torch.zeros(m, dtype=torch.float32, device=y.device),
                       gz=torch.zeros(m, dtype=torch.float32, device=y.device))
        gy, gz, gt = api.refit_adjoint(fctx.tctx, hits, fctx.row_x, fctx.prm, theta,
                                       fctx.fwd, grad_chi2, cm=fctx.cm, y=y, z=z, out=out)
        if hits.idx is not None:
            # entry j of the track list is cluster idx[j]: scatter to clusters
            # (ids of unwritten entries are clamped; their gradient is zero)
            idx = hits.idx[:gy.shape[0]].long().clamp(0, y.shape[0] - 1)
            gy = torch.zeros_like(y).index_add_(0, idx, gy)
            gz = torch.zeros_like(z).index_add_(0, idx, gz)
        return gy, gz, gt.to(theta.dtype), None, None, None, None, None


def refit_chi2(tctx, hits, row_x, prm, y, z, theta, cm=None):
    """Differentiable per-track chi2 (and the non-differentiable status)."""
    return RefitFunction.apply(y, z, theta, tctx, hits, row_x, prm, cm)
