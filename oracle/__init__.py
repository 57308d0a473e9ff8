"""Oracle of the TPC track-finding hot path -- TEST INFRASTRUCTURE ONLY.

Thin numpy/ctypes wrapper around liboracle.so (plain single-threaded C,
oracle.c).  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the library under
paper_1905_05515_amd never does.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class Params(C.Structure):
    _fields_ = [(n, C.c_float) for n in (
        "curv", "nb_win_y", "nb_win_z", "nb_d2max", "sigma_y2", "sigma_z2",
        "chi2_max", "search_nsigma", "s_max", "c_ss0", "c_tt0", "c_ww0")] + \
        [(n, C.c_int) for n in ("max_miss", "min_tracklet_hits", "min_track_hits")]


class CalibModel(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("drift_len", "vd", "tan_half", "u_centre", "u_scale")]


SECTOR_DTYPE = np.dtype([
    ("y0", np.float32), ("z0", np.float32), ("inv_by", np.float32), ("inv_bz", np.float32),
    ("nby", np.int32), ("nbz", np.int32), ("bin_base", np.int32), ("side", np.int32),
    ("begin", np.int64), ("end", np.int64)])


def lib():
    """The oracle library; TPC_ORACLE_SO names another build of oracle.c
    (for checking that a pin fails under a deliberate change of the
    oracle)."""
    global _lib
    if _lib is None:
        so = os.environ.get("TPC_ORACLE_SO") or _build.SO
        if so == _build.SO and not os.path.exists(so):
            _build.build()
        _lib = C.CDLL(so)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def params(d: dict) -> Params:
    p = Params()
    for name, _ in Params._fields_:
        setattr(p, name, d[name])
    return p


def calib_model(drift_len=250.0, vd=2.58, tan_half=0.17632698070846498,
                u_centre=165.0, u_scale=80.0) -> CalibModel:
    return CalibModel(drift_len, vd, tan_half, u_centre, u_scale)


def _sectors(layout):
    tab = np.ascontiguousarray(layout, dtype=SECTOR_DTYPE)
    return tab


def build_grid(row, y, z, layout, n_bins, n_rows=152):
    L = lib()
    tab = _sectors(layout)
    n = row.shape[0]
    bin_start = np.zeros(n_bins + 1, np.int32)
    yg = np.zeros(n, np.float32)
    zg = np.zeros(n, np.float32)
    idg = np.zeros(n, np.int32)
    L.orc_build_grid.restype = C.c_int
    placed = L.orc_build_grid(C.c_int(tab.shape[0]), _p(tab), C.c_int(n_rows), _p(row), _p(y),
                              _p(z), C.c_int(n_bins), _p(bin_start), _p(yg), _p(zg), _p(idg))
    if placed < 0:
        raise MemoryError("oracle grid")
    return dict(bin_start=bin_start, yg=yg[:placed], zg=zg[:placed], idg=idg[:placed])


def find_neighbours(layout, row_x, prm, grid, n_clusters, n_rows=152):
    L = lib()
    tab = _sectors(layout)
    up0 = np.empty(n_clusters, np.int32)
    down0 = np.empty(n_clusters, np.int32)
    P = params(prm)
    L.orc_find_neighbours(C.c_int(tab.shape[0]), _p(tab), C.c_int(n_rows), _p(row_x),
                          C.byref(P), _p(grid["bin_start"]), _p(grid["yg"]), _p(grid["zg"]),
                          _p(grid["idg"]), C.c_int64(n_clusters), _p(up0), _p(down0))
    return up0, down0


def clean_links(up0, down0):
    n = up0.shape[0]
    up = np.empty(n, np.int32)
    down = np.empty(n, np.int32)
    lib().orc_clean_links(C.c_int64(n), _p(up0), _p(down0), _p(up), _p(down))
    return up, down


def select_starts(up, down):
    n = up.shape[0]
    starts = np.empty(max(n // 3, 1), np.int32)
    L = lib()
    L.orc_select_starts.restype = C.c_int64
    m = L.orc_select_starts(C.c_int64(n), _p(up), _p(down), _p(starts))
    return starts[:m].copy()


def construct_tracklets(layout, row_x, prm, grid, row, y, z, up, starts, n_rows=152,
                        brute=False):
    L = lib()
    tab = _sectors(layout)
    m = starts.shape[0]
    hits = np.empty((m, n_rows), np.int32)
    nhits = np.empty(m, np.int32)
    rin = np.empty(m, np.int32)
    par = np.empty((m, 5), np.float32)
    cov = np.empty((m, 15), np.float32)
    chi2 = np.empty(m, np.float32)
    P = params(prm)
    L.orc_construct_tracklets(C.c_int(tab.shape[0]), _p(tab), C.c_int(n_rows), _p(row_x),
                              C.byref(P), _p(grid["bin_start"]), _p(grid["yg"]),
                              _p(grid["zg"]), _p(grid["idg"]), _p(row), _p(y), _p(z), _p(up),
                              C.c_int64(m), _p(starts), C.c_int(1 if brute else 0), _p(hits),
                              _p(nhits), _p(rin), _p(par), _p(cov), _p(chi2))
    return dict(hits=hits, nhits=nhits, row_inner=rin, par=par, cov=cov, chi2=chi2)


def tracklet_work():
    """(transports, updates, chi2 evaluations) of the last tracklet construction."""
    out = np.zeros(3, np.int64)
    lib().orc_tracklet_work(_p(out))
    return tuple(int(v) for v in out)


def tracklet_replay64(row_x, prm, y, z, start_row, hits_by_row, n_rows=152):
    L = lib()
    P = params(prm)
    par = np.empty(5, np.float64)
    cov = np.empty(15, np.float64)
    chi2 = np.empty(1, np.float64)
    hb = np.ascontiguousarray(hits_by_row, np.int32)
    st = L.orc_tracklet_replay64(C.c_int(n_rows), _p(row_x), C.byref(P), _p(y), _p(z),
                                 C.c_int(int(start_row)), _p(hb), _p(par), _p(cov), _p(chi2))
    return st, par, cov, float(chi2[0])


def select_tracks(n_clusters, prm, tracklets, starts, n_rows=152):
    L = lib()
    P = params(prm)
    m = starts.shape[0]
    off = np.zeros(m + 1, np.int32)
    th = np.empty(max(n_clusters, 1), np.int32)
    tt = np.empty(max(m, 1), np.int32)
    L.orc_select_tracks.restype = C.c_int64
    nt = L.orc_select_tracks(C.c_int64(n_clusters), C.c_int(n_rows), C.byref(P), C.c_int64(m),
                             _p(tracklets["hits"]), _p(tracklets["nhits"]), _p(starts),
                             _p(off), _p(th), _p(tt))
    off = off[:nt + 1].copy()
    return dict(trk_off=off, trk_hits=th[:off[-1]].copy(), trk_tracklet=tt[:nt].copy())


def attach_clusters(sector_offsets, row, y, z, row_x, prm, trk_off, trk_hits, par, rin,
                    radius=1.5, pt_good=0.05, n_rows=152):
    """Track-based cluster attachment (section 6).  par/rin: the state of
    each track (5 floats at the plane of row rin).  Returns (track, state)
    per cluster id: owning or adjacent track (-1 none); state bits 1
    attached, 2 adjacent, 4 protected, 8 removed."""
    L = lib()
    offs = np.ascontiguousarray(sector_offsets, np.int64)
    n = row.shape[0]
    nt = trk_off.shape[0] - 1
    track = np.empty(max(n, 1), np.int32)
    state = np.empty(max(n, 1), np.uint8)
    P = params(prm)
    w_good = np.float32(1.0) / np.float32(pt_good)
    L.orc_attach_clusters(C.c_int(offs.shape[0] - 1), _p(offs), C.c_int(n_rows),
                          _p(np.ascontiguousarray(row_x, np.float32)), C.byref(P),
                          _p(np.ascontiguousarray(row, np.uint8)),
                          _p(np.ascontiguousarray(y, np.float32)),
                          _p(np.ascontiguousarray(z, np.float32)), C.c_int64(n), C.c_int64(nt),
                          _p(np.ascontiguousarray(trk_off, np.int32)),
                          _p(np.ascontiguousarray(trk_hits, np.int32)),
                          _p(np.ascontiguousarray(par, np.float32)),
                          _p(np.ascontiguousarray(rin, np.int32)), C.c_float(radius),
                          C.c_float(w_good), _p(track), _p(state))
    return track[:n], state[:n]


MERGE_WINDOWS = (3.0, 2.0, 0.1, 0.02, 2.0)   # y, z [cm], sin(phi), tan(lambda), q/pT


def merge_windows_inv(windows=MERGE_WINDOWS):
    """Inverse window widths as float32 (the form both sides take)."""
    return (np.float32(1.0) / np.asarray(windows, np.float32)).astype(np.float32)


def sector_width_cs(width_deg=20.0):
    """cos and sin of the sector width as float32 inputs."""
    import math
    w = math.radians(width_deg)
    return np.float32(math.cos(w)), np.float32(math.sin(w))


def merge_transform(pj, xj, c, sd, x_to, curv, s_max=0.95):
    """One state rotated into a frame turned by D (cos c, sin sd) and
    transported to the plane x_to; None where invalid."""
    out = np.empty(5, np.float32)
    ok = lib().orc_merge_transform(_p(np.ascontiguousarray(pj, np.float32)), C.c_float(xj),
                                   C.c_float(c), C.c_float(sd), C.c_float(x_to),
                                   C.c_float(curv), C.c_float(s_max), _p(out))
    return out if ok else None


def merge_sector_tracks(sector_offsets, sectors_per_side, row_x, prm, trk_off, trk_hits, par,
                        rin, iw=None, cos_w=None, sin_w=None):
    """Sector-track merging (sections 2 and 3).  par/rin: the state of every
    track.  Returns (link_up, link_dn, group) per track."""
    offs = np.ascontiguousarray(sector_offsets, np.int64)
    n_sec = offs.shape[0] - 1
    if sectors_per_side < 3 or n_sec % sectors_per_side:
        raise ValueError("sectors must form sides of at least 3 sectors")
    if cos_w is None:
        cos_w, sin_w = sector_width_cs(360.0 / sectors_per_side)
    iw = merge_windows_inv() if iw is None else np.ascontiguousarray(iw, np.float32)
    nt = trk_off.shape[0] - 1
    up = np.empty(max(nt, 1), np.int32)
    dn = np.empty(max(nt, 1), np.int32)
    grp = np.empty(max(nt, 1), np.int32)
    P = params(prm)
    lib().orc_merge_sector_tracks(C.c_int(n_sec), _p(offs), C.c_int(sectors_per_side),
                                  _p(np.ascontiguousarray(row_x, np.float32)), C.byref(P),
                                  C.c_int64(nt), _p(np.ascontiguousarray(trk_off, np.int32)),
                                  _p(np.ascontiguousarray(trk_hits, np.int32)),
                                  _p(np.ascontiguousarray(par, np.float32)),
                                  _p(np.ascontiguousarray(rin, np.int32)), C.c_float(cos_w),
                                  C.c_float(sin_w), _p(iw), _p(up), _p(dn), _p(grp))
    return up[:nt], dn[:nt], grp[:nt]


def track_t0(par, x_in, side, prm, vd=2.58):
    """Interaction time of every track (section 2, continuous read-out):
    returns (z0, y0, t0, ok) at the plane x = 0 of each track's frame."""
    par = np.ascontiguousarray(par, np.float32).reshape(-1, 5)
    n = par.shape[0]
    out = [np.empty(max(n, 1), np.float32) for _ in range(3)]
    ok = np.empty(max(n, 1), np.int8)
    lib().orc_track_t0(C.c_int64(n), _p(par), _p(np.ascontiguousarray(x_in, np.float32)),
                       _p(np.ascontiguousarray(side, np.int8)), C.c_float(prm["curv"]),
                       C.c_float(prm["s_max"]), C.c_float(vd), *[_p(o) for o in out], _p(ok))
    return out[0][:n], out[1][:n], out[2][:n], ok[:n]


def track_event(row, y, z, layout, n_bins, row_x, prm, n_rows=152, brute=False):
    """The whole chain: grid, neighbours, cleaning, starts, tracklets,
    selection.  Returns a dict of every intermediate (id space)."""
    grid = build_grid(row, y, z, layout, n_bins, n_rows)
    n = row.shape[0]
    up0, down0 = find_neighbours(layout, row_x, prm, grid, n, n_rows)
    up, down = clean_links(up0, down0)
    starts = select_starts(up, down)
    trl = construct_tracklets(layout, row_x, prm, grid, row, y, z, up, starts, n_rows, brute)
    trl["work"] = tracklet_work()
    trk = select_tracks(n, prm, trl, starts, n_rows)
    return dict(grid=grid, up0=up0, down0=down0, up=up, down=down, starts=starts,
                tracklets=trl, tracks=trk)


def refit(trk_off, row, y, z, row_x, prm, theta, side=None, cm=None, fp64=False):
    L = lib()
    P = params(prm)
    cm = cm or calib_model()
    n = trk_off.shape[0] - 1
    dt = np.float64 if fp64 else np.float32
    y = np.ascontiguousarray(y, dt)
    z = np.ascontiguousarray(z, dt)
    th = np.ascontiguousarray(theta, dt)
    par = np.empty((n, 5), dt)
    cov = np.empty((n, 15), dt)
    chi2 = np.empty(n, dt)
    status = np.empty(n, np.int32)
    sd = None if side is None else np.ascontiguousarray(side, np.int8)
    fn = L.orc_refit64 if fp64 else L.orc_refit32
    fn(C.c_int64(n), _p(np.ascontiguousarray(trk_off, np.int32)), _p(row), _p(y), _p(z),
       _p(sd), _p(row_x), C.byref(P), C.byref(cm), _p(th), _p(par), _p(cov), _p(chi2),
       _p(status))
    return dict(par=par, cov=cov, chi2=chi2, status=status)


def refit_fd_grad(trk_off, row, y, z, row_x, prm, theta, g, side=None, cm=None,
                  h_hit=1e-4, h_theta=1e-5):
    """FP64 central differences of L = sum_t g_t chi2_t."""
    L = lib()
    P = params(prm)
    cm = cm or calib_model()
    n = trk_off.shape[0] - 1
    nh = row.shape[0]
    gy = np.zeros(nh, np.float64)
    gz = np.zeros(nh, np.float64)
    gt = np.zeros(16, np.float64)
    sd = None if side is None else np.ascontiguousarray(side, np.int8)
    L.orc_refit64_fd_grad(C.c_int64(n), _p(np.ascontiguousarray(trk_off, np.int32)), _p(row),
                          _p(np.ascontiguousarray(y, np.float64)),
                          _p(np.ascontiguousarray(z, np.float64)), _p(sd), _p(row_x),
                          C.byref(P), C.byref(cm), _p(np.ascontiguousarray(theta, np.float64)),
                          _p(np.ascontiguousarray(g, np.float64)), C.c_double(h_hit),
                          C.c_double(h_theta), _p(gy), _p(gz), _p(gt))
    return gy, gz, gt


def fit_merged(sector_offsets, sectors_per_side, row_x, prm, row, y, z, trk_off, trk_hits, par,
               cov, rin, link_up, link_dn, group, n_pass=3, cov_scale=100.0, cos_w=None,
               sin_w=None, fp64=True):
    """Full-track fit of merged sector tracks (float64, or float32 with the
    same expressions in the same order): per track index, filled for group
    leaders.  Returns dict(par_in, par_out, cov_out, chi2, n_hits,
    n_members, status)."""
    offs = np.ascontiguousarray(sector_offsets, np.int64)
    n_sec = offs.shape[0] - 1
    if cos_w is None:
        cos_w, sin_w = sector_width_cs(360.0 / sectors_per_side)
    nt = trk_off.shape[0] - 1
    m = max(nt, 1)
    dt = np.float64 if fp64 else np.float32
    out = dict(par_in=np.zeros((m, 5), dt), par_out=np.zeros((m, 5), dt),
               cov_out=np.zeros((m, 15), dt), chi2=np.zeros(m, dt),
               n_hits=np.zeros(m, np.int32), n_members=np.zeros(m, np.int32),
               status=np.zeros(m, np.int32))
    P = params(prm)
    i32 = lambda a: _p(np.ascontiguousarray(a, np.int32))
    fn = lib().orc_fit_merged64 if fp64 else lib().orc_fit_merged32
    fn(C.c_int(n_sec), _p(offs), C.c_int(sectors_per_side),
                           _p(np.ascontiguousarray(row_x, np.float32)), C.byref(P),
                           _p(np.ascontiguousarray(row, np.uint8)),
                           _p(np.ascontiguousarray(y, np.float32)),
                           _p(np.ascontiguousarray(z, np.float32)), C.c_int64(nt), i32(trk_off),
                           i32(trk_hits), _p(np.ascontiguousarray(par, np.float32)),
                           _p(np.ascontiguousarray(cov, np.float32)), i32(rin),
                           i32(link_up), i32(link_dn), i32(group), C.c_float(cos_w),
                           C.c_float(sin_w), C.c_int(n_pass), C.c_float(cov_scale),
                           _p(out["par_in"]),
                           _p(out["par_out"]), _p(out["cov_out"]), _p(out["chi2"]),
                           _p(out["n_hits"]), _p(out["n_members"]), _p(out["status"]))
    return {k: v[:nt] for k, v in out.items()}


def rotate(x, p, Cov, c, sd, curv, s_max=0.95):
    """One frame turn (float64); returns (ok, x', p', C')."""
    xx = C.c_double(x)
    p = np.array(p, np.float64)
    Cv = np.array(Cov, np.float64)
    ok = lib().orc_rotate64(C.byref(xx), _p(p), _p(Cv), C.c_double(c), C.c_double(sd),
                            C.c_double(curv), C.c_double(s_max))
    return bool(ok), xx.value, p, Cv


def vertex_weights(trk_off, row, y, z, row_x, prm, theta, sigma_v=0.01, side=None, cm=None):
    """Per-track weights (w00, w01, w11) of the beam-axis term at theta
    (float64) and the tracks that have one."""
    cm = cm or calib_model()
    n = trk_off.shape[0] - 1
    w = np.zeros((max(n, 1), 3), np.float64)
    ok = np.zeros(max(n, 1), np.int32)
    sd = None if side is None else np.ascontiguousarray(side, np.int8)
    lib().orc_vertex_weights64(C.c_int64(n), _p(np.ascontiguousarray(trk_off, np.int32)), _p(row),
                               _p(np.ascontiguousarray(y, np.float64)),
                               _p(np.ascontiguousarray(z, np.float64)), _p(sd), _p(row_x),
                               C.byref(params(prm)), C.byref(cm),
                               _p(np.ascontiguousarray(theta, np.float64)),
                               C.c_double(sigma_v * sigma_v), _p(w), _p(ok))
    return w[:n], ok[:n]


def calib_objective(trk_off, row, y, z, row_x, prm, theta, w, g=None, side=None, cm=None,
                    grad=True):
    """Calibration objective with the beam-axis constraint (float64):
    L = sum_t g_t (chi2_t + r_t^T W_t r_t) with the per-track weights w
    (vertex_weights; None: chi2 only).  Returns (L, dL/dtheta or None,
    per-track terms, vertex-term flags)."""
    L = lib()
    L.orc_calib_objective64.restype = C.c_double
    P = params(prm)
    cm = cm or calib_model()
    n = trk_off.shape[0] - 1
    g = np.ones(n) if g is None else np.ascontiguousarray(g, np.float64)
    gt = np.zeros(16, np.float64) if grad else None
    per = np.zeros(max(n, 1), np.float64)
    vok = np.zeros(max(n, 1), np.int32)
    sd = None if side is None else np.ascontiguousarray(side, np.int8)
    wv = None if w is None else np.ascontiguousarray(w, np.float64)
    val = L.orc_calib_objective64(C.c_int64(n), _p(np.ascontiguousarray(trk_off, np.int32)),
                                  _p(row), _p(np.ascontiguousarray(y, np.float64)),
                                  _p(np.ascontiguousarray(z, np.float64)), _p(sd), _p(row_x),
                                  C.byref(P), C.byref(cm),
                                  _p(np.ascontiguousarray(theta, np.float64)), _p(g), _p(wv),
                                  _p(gt), _p(per), _p(vok))
    return val, gt, per[:n], vok[:n]


class CmpParams(C.Structure):
    _fields_ = [("qbits", C.c_int32), ("cbits", C.c_int32), ("chunk", C.c_int32)]


def compress(layout, n_rows, row_x, prm, row, y, z, charge, grid, trk_off, trk_hits, tpar,
             trin, qbits=5, cbits=5, chunk=4096):
    """Cluster compression (section 6): the blob (uint8 array).  grid: the
    grid of the same clusters (bin_start, idg); tpar, trin: each track's
    tracklet state and innermost row."""
    L = lib()
    L.orc_compress.restype = C.c_int64
    tab = _sectors(layout)
    cp = CmpParams(qbits, cbits, chunk)
    n = row.shape[0]
    nt = trk_off.shape[0] - 1
    i32 = lambda a: _p(np.ascontiguousarray(a, np.int32))
    args = (C.c_int(tab.shape[0]), _p(tab), C.c_int(n_rows),
            _p(np.ascontiguousarray(row_x, np.float32)), C.byref(params(prm)),
            _p(np.ascontiguousarray(row, np.uint8)), _p(np.ascontiguousarray(y, np.float32)),
            _p(np.ascontiguousarray(z, np.float32)), _p(np.ascontiguousarray(charge, np.float32)),
            C.c_int64(n), i32(grid["bin_start"]), i32(grid["idg"]), C.c_int64(nt), i32(trk_off),
            i32(trk_hits), _p(np.ascontiguousarray(tpar, np.float32)), i32(trin), C.byref(cp))
    cap = 64 * n + 4096 + 32 * nt
    out = np.zeros(cap, np.uint8)
    size = L.orc_compress(*args, _p(out), C.c_int64(cap))
    if size < 0:
        out = np.zeros(-size, np.uint8)
        size = L.orc_compress(*args, _p(out), C.c_int64(-size))
    return out[:size]


def decompress(blob, n_clusters, row_x, prm):
    """Clusters of a blob in its order: dict(row, yq, zq, qcode, track,
    sector) (track -1 for clusters on no track; sector -1 for clusters on
    tracks)."""
    L = lib()
    L.orc_decompress.restype = C.c_int64
    m = max(n_clusters, 1)
    o = dict(row=np.zeros(m, np.uint8), yq=np.zeros(m, np.int32), zq=np.zeros(m, np.int32),
             qcode=np.zeros(m, np.int32), track=np.zeros(m, np.int32),
             sector=np.zeros(m, np.int32))
    blob = np.ascontiguousarray(blob, np.uint8)
    n = L.orc_decompress(_p(blob), C.c_int64(blob.shape[0]),
                         _p(np.ascontiguousarray(row_x, np.float32)), C.byref(params(prm)),
                         _p(o["row"]), _p(o["yq"]), _p(o["zq"]), _p(o["qcode"]),
                         _p(o["track"]), _p(o["sector"]), C.c_int64(m))
    if n < 0:
        raise ValueError("malformed blob")
    return {k: v[:n] for k, v in o.items()}


def charge_decode(code, cbits=5):
    return lib().orc_charge_decode(C.c_int(int(code)), C.c_int(cbits))


def rans_roundtrip(sym):
    """rANS code of a byte stream with its own table: (bytes, decoded)."""
    L = lib()
    L.orc_rans_roundtrip.restype = C.c_int64
    sym = np.ascontiguousarray(sym, np.uint8)
    out = np.zeros(2 * sym.shape[0] + 8, np.uint8)
    back = np.zeros(max(sym.shape[0], 1), np.uint8)
    nb = L.orc_rans_roundtrip(_p(sym), C.c_int64(sym.shape[0]), _p(out), _p(back))
    if nb < 0:
        raise ValueError("rANS decode failed")
    return out[:nb], back[:sym.shape[0]]


def refit_adjoint64(trk_off, row, y, z, row_x, prm, theta, g, side=None, cm=None):
    """Gradient of L = sum_t g_t chi2_t of the float64 refit with respect to
    the raw hit y, z and the 16 calibration parameters, by reverse-mode
    differentiation of the float64 forward (a recorded tape)."""
    L = lib()
    P = params(prm)
    cm = cm or calib_model()
    n = trk_off.shape[0] - 1
    nh = row.shape[0]
    gy = np.zeros(nh, np.float64)
    gz = np.zeros(nh, np.float64)
    gt = np.zeros(16, np.float64)
    sd = None if side is None else np.ascontiguousarray(side, np.int8)
    L.orc_refit64_adjoint(C.c_int64(n), _p(np.ascontiguousarray(trk_off, np.int32)), _p(row),
                          _p(np.ascontiguousarray(y, np.float64)),
                          _p(np.ascontiguousarray(z, np.float64)), _p(sd), _p(row_x),
                          C.byref(P), C.byref(cm), _p(np.ascontiguousarray(theta, np.float64)),
                          _p(np.ascontiguousarray(g, np.float64)), _p(gy), _p(gz), _p(gt))
    return gy, gz, gt


def propagate(p, Cov, dx, curv, s_max=0.95, fp64=True):
    """One propagation step; returns (ok, p', C')."""
    dt = np.float64 if fp64 else np.float32
    p = np.array(p, dt)
    Cv = np.array(Cov, dt)
    L = lib()
    if fp64:
        ok = L.orc_propagate64(_p(p), _p(Cv), C.c_double(dx), C.c_double(curv), C.c_double(s_max))
    else:
        ok = L.orc_propagate32(_p(p), _p(Cv), C.c_float(dx), C.c_float(curv), C.c_float(s_max))
    return bool(ok), p, Cv


def update(p, Cov, my, mz, sy2, sz2, fp64=True):
    """One Kalman update; returns (chi2, p', C')."""
    dt = np.float64 if fp64 else np.float32
    p = np.array(p, dt)
    Cv = np.array(Cov, dt)
    L = lib()
    if fp64:
        L.orc_update64.restype = C.c_double
        c2 = L.orc_update64(_p(p), _p(Cv), C.c_double(my), C.c_double(mz), C.c_double(sy2),
                            C.c_double(sz2))
    else:
        L.orc_update32.restype = C.c_float
        c2 = L.orc_update32(_p(p), _p(Cv), C.c_float(my), C.c_float(mz), C.c_float(sy2),
                            C.c_float(sz2))
    return c2, p, Cv


def calibrate(theta, xr, yr, zr, side=1.0, cm=None):
    out = np.empty(3, np.float64)
    cm = cm or calib_model()
    lib().orc_calibrate64(_p(np.ascontiguousarray(theta, np.float64)), C.c_double(xr),
                          C.c_double(yr), C.c_double(zr), C.c_double(side), C.byref(cm),
                          _p(out))
    return out
