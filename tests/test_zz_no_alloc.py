"""The refit adjoint's entry point for callers that cannot allocate
(tpc_refit_adjoint_noalloc: theta partials in the library's static device
array) against tpc_refit_adjoint with a caller workspace, through the C
ABI: the same bits for every output, on two calls in a row, the second on a
smaller input (the array keeps the first call's contents)."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from gpu_common import ctx
from paper_1905_05515_amd import _lib as L
from paper_1905_05515_amd import api

pytestmark = pytest.mark.gpu
TPC_ERR_INVALID_ARG = 1     # include/tpc.h


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _case(n_tracks, seed_shift):
    rs = synth.make_config5(n_tracks=n_tracks)
    dev = "cuda"
    h = api.TrackHits(torch.as_tensor(rs.trk_off).to(dev), torch.as_tensor(rs.row).to(dev),
                      torch.as_tensor(rs.y).to(dev), torch.as_tensor(rs.z).to(dev))
    rx = torch.as_tensor(rs.row_x).to(dev)
    th = torch.as_tensor(rs.theta_eval).to(dev)
    prm = synth.default_params()
    out = api.refit(ctx(), h, rx, prm, th)
    g = torch.linspace(0.5, 1.5 + seed_shift, rs.n_tracks, device=dev)
    return rs, h, rx, th, prm, out, g


def _noalloc(h, rx, th, prm, out, g):
    n_hits = h.n_hits
    gy = torch.full((max(n_hits, 1),), float("nan"), device="cuda")
    gz = torch.full((max(n_hits, 1),), float("nan"), device="cuda")
    gt = torch.full((16,), float("nan"), device="cuda")
    P = api.params_struct(prm)
    CM = api.calib_struct(None)
    ck = out["checkpoints"]
    rc = L.lib().tpc_refit_adjoint_noalloc(
        ctx().handle, h.struct(), int(rx.shape[0]), _ptr(rx), C.byref(P), C.byref(CM),
        _ptr(th.float().contiguous()), _ptr(ck), ck.numel() * 4, _ptr(out["status"]),
        _ptr(g), _ptr(gy), _ptr(gz), _ptr(gt), None)
    L.check(rc, "tpc_refit_adjoint_noalloc")
    torch.cuda.synchronize()
    return gy[:n_hits], gz[:n_hits], gt


def test_noalloc_adjoint_equals_the_workspace_form_twice():
    for n_tracks, shift in ((20000, 0.0), (3000, 0.25)):
        print(f"case noalloc adjoint tracks={n_tracks}", flush=True)
        rs, h, rx, th, prm, out, g = _case(n_tracks, shift)
        ny, nz, nt = _noalloc(h, rx, th, prm, out, g)
        wy, wz, wt = api.refit_adjoint(ctx(), h, rx, prm, th, out, g)
        torch.cuda.synchronize()
        assert torch.equal(ny, wy) and torch.equal(nz, wz) and torch.equal(nt, wt)
        assert bool(torch.isfinite(nt).all()) and float(nt.abs().sum()) > 0.0


def test_noalloc_adjoint_argument_errors():
    print("case noalloc adjoint bad arguments", flush=True)
    rs, h, rx, th, prm, out, g = _case(100, 0.0)
    P = api.params_struct(prm)
    CM = api.calib_struct(None)
    ck = out["checkpoints"]
    gy = torch.empty(h.n_hits, device="cuda")
    gt = torch.empty(16, device="cuda")
    # checkpoint buffer shorter than the tracks need
    rc = L.lib().tpc_refit_adjoint_noalloc(
        ctx().handle, h.struct(), int(rx.shape[0]), _ptr(rx), C.byref(P), C.byref(CM), _ptr(th),
        _ptr(ck), 64, _ptr(out["status"]), _ptr(g), _ptr(gy), _ptr(gy), _ptr(gt), None)
    assert rc == TPC_ERR_INVALID_ARG
    # missing output
    rc = L.lib().tpc_refit_adjoint_noalloc(
        ctx().handle, h.struct(), int(rx.shape[0]), _ptr(rx), C.byref(P), C.byref(CM), _ptr(th),
        _ptr(ck), ck.numel() * 4, _ptr(out["status"]), _ptr(g), None, _ptr(gy), _ptr(gt), None)
    assert rc == TPC_ERR_INVALID_ARG
