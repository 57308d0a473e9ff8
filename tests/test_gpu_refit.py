"""GPU refit and adjoint against the float64 oracle, through the C ABI.

Forward: every track's parameters within relative 1e-4 of max(|p|, floor)
(floors 1 cm, 1 cm, 0.01, 0.01, 0.1 c/GeV for parameters near zero), chi2
relative 1e-4.
Adjoint: against the float64 reverse-mode gradient of the oracle refit on
every hit of 10k tracks and against float64 central differences on a few
tracks, relative 1e-3 per gradient block (hit y, hit z, theta) and per
component to 1e-3 of the block's largest entry, plus exact chain-rule
identities of the calibration model at full size."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import ctx
from paper_1905_05515_amd import api
from paper_1905_05515_amd.autograd import refit_chi2

pytestmark = pytest.mark.gpu
FLOOR = np.array([1.0, 1.0, 0.01, 0.01, 0.1])


def _hits(rs, dev="cuda"):
    return api.TrackHits(torch.as_tensor(rs.trk_off).to(dev), torch.as_tensor(rs.row).to(dev),
                         torch.as_tensor(rs.y).to(dev), torch.as_tensor(rs.z).to(dev))


def _subset(rs, idx):
    off = rs.trk_off
    parts = [np.arange(off[i], off[i + 1]) for i in idx]
    sel = np.concatenate(parts)
    new_off = np.zeros(len(idx) + 1, np.int32)
    new_off[1:] = np.cumsum([p.shape[0] for p in parts])
    return synth.RefitSet(new_off, rs.row[sel], rs.y[sel], rs.z[sel], rs.row_x, rs.theta_true,
                          rs.theta_eval, {}, {})


def _fwd(rs):
    h = _hits(rs)
    rx = torch.as_tensor(rs.row_x).cuda()
    th = torch.as_tensor(rs.theta_eval).cuda()
    out = api.refit(ctx(), h, rx, synth.default_params(), th)
    return h, rx, th, out


def _par_errors(par32, par64):
    scale = np.maximum(np.abs(par64), FLOOR)
    return (np.abs(par32.astype(np.float64) - par64) / scale).max(1)


def test_refit_forward_matches_fp64():
    rs = synth.make_config5(n_tracks=3000)
    _, _, _, out = _fwd(rs)
    o = oracle.refit(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, synth.default_params(),
                     rs.theta_eval.astype(np.float64), fp64=True)
    st = out["status"].cpu().numpy()
    assert np.array_equal(st, o["status"])
    ok = st == 0
    err = _par_errors(out["par"].cpu().numpy()[ok], o["par"][ok])
    assert err.max() <= 1e-4, (np.mean(err > 1e-4), err.max())
    c32 = out["chi2"].cpu().numpy()[ok]
    assert np.allclose(c32, o["chi2"][ok], rtol=1e-4, atol=1e-3)


def _block_ok(g, ref, tol=1e-3):
    return np.linalg.norm(g - ref) <= tol * np.linalg.norm(ref)


def test_adjoint_matches_fp64_central_differences():
    rs = synth.make_config5(n_tracks=400)
    sub = _subset(rs, np.arange(0, 400, 8))
    h, rx, th, out = _fwd(sub)
    g = torch.linspace(0.5, 1.5, sub.n_tracks, device="cuda")
    gy, gz, gt = api.refit_adjoint(ctx(), h, rx, synth.default_params(), th, out, g)
    fy, fz, ft = oracle.refit_fd_grad(sub.trk_off, sub.row, sub.y, sub.z, sub.row_x,
                                      synth.default_params(), sub.theta_eval.astype(np.float64),
                                      g.cpu().numpy().astype(np.float64))
    gy, gz, gt = (x.cpu().numpy().astype(np.float64) for x in (gy, gz, gt))
    assert _block_ok(gy, fy) and _block_ok(gz, fz) and _block_ok(gt, ft), (
        np.linalg.norm(gy - fy) / np.linalg.norm(fy), np.linalg.norm(gz - fz) / np.linalg.norm(fz),
        np.linalg.norm(gt - ft) / np.linalg.norm(ft))
    # component-wise with a floor of 1e-3 of the block's largest entry
    for a, b in ((gy, fy), (gz, fz), (gt, ft)):
        assert np.all(np.abs(a - b) <= 1e-3 * np.abs(b).max() + 3e-3 * np.abs(b))


@pytest.mark.timeout(600)
def test_adjoint_matches_fp64_adjoint_on_10k_tracks():
    rs = synth.make_config5(n_tracks=10000)
    print(f"case adjoint 10k tracks hits={rs.n_hits}", flush=True)
    h, rx, th, out = _fwd(rs)
    g = torch.linspace(0.5, 1.5, rs.n_tracks, device="cuda")
    gy, gz, gt = api.refit_adjoint(ctx(), h, rx, synth.default_params(), th, out, g)
    st = out["status"].cpu().numpy()
    ok = st == 0
    assert ok.mean() > 0.99
    # stopped tracks carry no gradient on the library's side
    g64 = g.cpu().numpy().astype(np.float64) * ok
    ry, rz, rt = oracle.refit_adjoint64(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x,
                                        synth.default_params(),
                                        rs.theta_eval.astype(np.float64), g64)
    hit_ok = np.repeat(ok, np.diff(rs.trk_off))
    gy, gz, gt = (x.cpu().numpy().astype(np.float64) for x in (gy, gz, gt))
    assert np.all(gy[~hit_ok] == 0) and np.all(gz[~hit_ok] == 0)
    for name, a, b in (("y", gy, ry), ("z", gz, rz), ("theta", gt, rt)):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        worst = np.abs(a - b).max() / np.abs(b).max()
        assert rel <= 1e-3 and worst <= 1e-3, (name, rel, worst)


def test_autograd_function_uses_the_adjoint():
    rs = synth.make_config5(n_tracks=64)
    h = _hits(rs)
    rx = torch.as_tensor(rs.row_x).cuda()
    y = h.y.clone().requires_grad_(True)
    z = h.z.clone().requires_grad_(True)
    th = torch.as_tensor(rs.theta_eval).cuda().requires_grad_(True)
    chi2, status = refit_chi2(ctx(), h, rx, synth.default_params(), y, z, th)
    w = torch.arange(chi2.shape[0], device="cuda", dtype=torch.float32) / 64.0
    (chi2 * w).sum().backward()
    out = api.refit(ctx(), h, rx, synth.default_params(), th.detach())
    gy, gz, gt = api.refit_adjoint(ctx(), h, rx, synth.default_params(), th.detach(), out, w)
    assert torch.equal(y.grad, gy) and torch.equal(z.grad, gz) and torch.equal(th.grad, gt)
    assert torch.equal(chi2, out["chi2"])


def test_autograd_through_the_trackers_own_tracks():
    """The differentiable refit on the tracker's output (track entries are
    cluster ids, y and z are per cluster): autograd returns per-cluster
    gradients, the ABI adjoint's per-entry gradients summed onto clusters."""
    from gpu_common import run_gpu
    ev = synth.make_config1()
    print(f"case autograd found tracks n={ev.n_clusters}", flush=True)
    e, g = run_gpu(ev)
    hits = api.found_track_hits(e)
    rx = e.t["row_x"]
    prm = synth.default_params()
    th = torch.as_tensor(rs_theta()).cuda().requires_grad_(True)
    y = e.t["y"].clone().requires_grad_(True)
    z = e.t["z"].clone().requires_grad_(True)
    chi2, status = refit_chi2(ctx(), hits, rx, prm, y, z, th)
    n_trk = len(g["trk_off"]) - 1
    w = torch.zeros_like(chi2)
    w[:n_trk] = torch.linspace(0.5, 1.5, n_trk, device="cuda")
    (chi2 * w).sum().backward()
    assert y.grad.shape == y.shape and z.grad.shape == z.shape
    out = api.refit(ctx(), hits, rx, prm, th.detach())
    gy, gz, gt = api.refit_adjoint(ctx(), hits, rx, prm, th.detach(), out, w)
    m = int(g["trk_off"][-1])
    ids = torch.as_tensor(g["trk_hits"][:m].astype(np.int64)).cuda()
    ey = torch.zeros_like(y).index_add_(0, ids, gy[:m])
    ez = torch.zeros_like(z).index_add_(0, ids, gz[:m])
    assert torch.equal(y.grad, ey) and torch.equal(z.grad, ez) and torch.equal(th.grad, gt)
    assert float(y.grad.abs().sum()) > 0.0
    # clusters on no track get no gradient
    on = torch.zeros(y.shape[0], dtype=torch.bool, device="cuda")
    on[ids] = True
    assert not bool((y.grad[~on] != 0).any())


def test_track_ordered_hit_copies_give_the_same_refit():
    """The selection's track-ordered copies of the hits' rows and
    coordinates equal the clusters gathered through the track's ids, and
    the refit and its adjoint on the copies (contiguous reads) equal those
    through the ids bit for bit, in the staged and the persistent form."""
    from gpu_common import run_gpu
    ev = synth.make_config2()
    print(f"case track hit copies n={ev.n_clusters}", flush=True)
    prm = synth.default_params()
    th = torch.as_tensor(rs_theta()).cuda()
    for mode in ("staged", "persistent"):
        e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x, prm,
                           sector_side=ev.sector_side)
        api.track_batch(ctx(), e, mode=mode)
        torch.cuda.synchronize()
        st = api.get_status(e)
        m = int(st["n_track_hits"])
        ids = e.t["trk_hits"][:m].long()
        assert torch.equal(e.t["trk_row"][:m], e.t["row"][ids]), mode
        assert torch.equal(e.t["trk_y"][:m].view(torch.int32), e.t["y"][ids].view(torch.int32))
        assert torch.equal(e.t["trk_z"][:m].view(torch.int32), e.t["z"][ids].view(torch.int32))
        rx = e.t["row_x"]
        w = torch.linspace(0.5, 1.5, e.track_capacity, device="cuda")
        res = []
        for copies in (False, True):
            hits = api.found_track_hits(e, copies=copies)
            out = api.refit(ctx(), hits, rx, prm, th)
            gy, gz, gt = api.refit_adjoint(ctx(), hits, rx, prm, th, out, w)
            res.append((out, gy, gz, gt))
        nt = int(st["n_tracks"])
        (o0, y0, z0, t0), (o1, y1, z1, t1) = res
        for k in ("par", "cov", "chi2", "status"):
            a, b = o0[k][:nt], o1[k][:nt]
            if a.dtype == torch.float32:
                a, b = a.view(torch.int32), b.view(torch.int32)
            assert torch.equal(a, b), (mode, k)
        assert torch.equal(y0[:m].view(torch.int32), y1[:m].view(torch.int32))
        assert torch.equal(z0[:m].view(torch.int32), z1[:m].view(torch.int32))
        assert torch.equal(t0.view(torch.int32), t1.view(torch.int32))


def rs_theta():
    return synth.make_config5(n_tracks=1).theta_eval


@pytest.mark.timeout(900)
def test_full_size_refit_and_adjoint_properties():
    """1M tracks at the benchmark's launch configuration: sampled tracks
    against the float64 oracle, and exact identities of the calibration
    model over all hits (z_raw enters only through the drift length)."""
    rs = synth.make_config5()
    print(f"case c5 tracks={rs.n_tracks} hits={rs.n_hits}", flush=True)
    h, rx, th, out = _fwd(rs)
    g = torch.ones(rs.n_tracks, device="cuda")
    gy, gz, gt = api.refit_adjoint(ctx(), h, rx, synth.default_params(), th, out, g)
    st = out["status"].cpu().numpy()
    assert np.mean(st == 0) > 0.999
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(rs.n_tracks, 2000, replace=False))
    sub = _subset(rs, idx)
    o = oracle.refit(sub.trk_off, sub.row, sub.y, sub.z, sub.row_x, synth.default_params(),
                     rs.theta_eval.astype(np.float64), fp64=True)
    ok = (o["status"] == 0) & (st[idx] == 0)
    err = _par_errors(out["par"].cpu().numpy()[idx][ok], o["par"][ok])
    assert err.max() <= 1e-4, (np.mean(err > 1e-4), err.max())
    assert np.allclose(out["chi2"].cpu().numpy()[idx][ok], o["chi2"][ok], rtol=1e-4, atol=1e-3)
    cm = api.CALIB_MODEL
    vd = float(np.float32(cm["vd"]))
    gz64 = gz.double()
    gt64 = gt.double().cpu().numpy()
    sum_gz = float(gz64.sum())
    assert abs(gt64[1] - vd * sum_gz) <= 2e-3 * float((vd * gz64.abs()).sum())
    d_raw = float(np.float32(cm["drift_len"])) - h.z.double()
    th64 = rs.theta_eval.astype(np.float64)
    expect = float((gz64 * (d_raw - vd * th64[1]) / (-(1.0 + th64[0]))).sum())
    assert abs(gt64[0] - expect) <= 2e-3 * float((gz64 * d_raw).abs().sum())
    # deterministic: a second adjoint pass gives the same bits
    gy2, gz2, gt2 = api.refit_adjoint(ctx(), h, rx, synth.default_params(), th, out, g)
    assert torch.equal(gy, gy2) and torch.equal(gz, gz2) and torch.equal(gt, gt2)
