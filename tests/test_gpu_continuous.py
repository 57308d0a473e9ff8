"""The continuous read-out slice at full size (100 overlapping collisions,
tens of millions of clusters) through the launch form the benchmark times
(staged stages, graph replay).  The oracle cannot track the whole slice in
seconds, but sectors are independent for every step, so the oracle run on
single sectors must reproduce the library's outputs for those sectors bit
for bit; properties that hold at any size are checked over the whole
slice."""
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import assert_same_tracking, ctx, run_gpu, run_oracle
from paper_1905_05515_amd import api
from paper_1905_05515_amd.layout import grid_layout

pytestmark = pytest.mark.gpu

# sectors checked against the oracle one by one: both z sides, first and
# last of each side, and sectors in between
SAMPLED_SECTORS = (0, 3, 13, 17, 18, 24, 30, 35)


@pytest.fixture(scope="module")
def slice_run():
    t0 = time.time()
    ev = synth.make_config3()
    print(f"case c3 n={ev.n_clusters} generated in {time.time() - t0:.1f}s", flush=True)
    prm = synth.default_params()
    e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x, prm,
                       sector_side=ev.sector_side)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        for _ in range(2):                   # capture, then replay
            api.track_batch(ctx(), e, mode="staged", use_graph=True, stream=side)
    side.synchronize()
    st = api.get_status(e, side)
    print(f"case c3 tracked: starts {st['n_starts']} tracks {st['n_tracks']}", flush=True)
    return ev, e, st, prm


def _sector_slice(ev, e, st, s):
    """The library's outputs for sector s, in the coordinates of the sector
    as a stand-alone event (ids and positions minus its first id)."""
    t = e.t
    b0, b1 = int(ev.sector_offsets[s]), int(ev.sector_offsets[s + 1])
    tab, _ = e.layout
    bb0 = int(tab[s]["bin_base"])
    nb = e.n_rows * int(tab[s]["nby"]) * int(tab[s]["nbz"]) + 1
    cpu = lambda x: x.cpu().numpy()

    def shift(a):
        return np.where(a >= 0, a - b0, -1).astype(np.int32)

    out = dict(status=dict(st))
    out["bin_start"] = cpu(t["bin_start"][bb0:bb0 + nb + 1]) - b0
    out["yg"] = cpu(t["yg"][b0:b1])
    out["zg"] = cpu(t["zg"][b0:b1])
    out["idg"] = cpu(t["idg"][b0:b1]) - b0
    for k in ("up0", "down0", "up", "down"):
        out[k] = shift(cpu(t[k][b0:b1]))
    m = min(int(st["n_starts"]), e.start_capacity)
    starts = cpu(t["starts"][:m])
    t_lo, t_hi = np.searchsorted(starts >= b0, True), np.searchsorted(starts >= b1, True)
    # starts are in id order, so the sector's starts are one block
    assert np.all((starts[t_lo:t_hi] >= b0) & (starts[t_lo:t_hi] < b1))
    out["starts"] = starts[t_lo:t_hi] - b0
    hits = cpu(t["t_hits"].view(e.n_rows, e.start_capacity)[:, t_lo:t_hi]).T
    out["t_hits"] = shift(np.ascontiguousarray(hits))
    for k, w in (("t_nhits", 1), ("t_rin", 1), ("t_chi2", 1)):
        out[k] = cpu(t[k][t_lo:t_hi])
    out["t_par"] = cpu(t["t_par"][t_lo * 5:t_hi * 5]).reshape(-1, 5)
    out["t_cov"] = cpu(t["t_cov"][t_lo * 15:t_hi * 15]).reshape(-1, 15)
    nt = min(int(st["n_tracks"]), e.track_capacity)
    trk_t = cpu(t["trk_tracklet"][:nt])
    k_lo, k_hi = np.searchsorted(trk_t, t_lo), np.searchsorted(trk_t, t_hi)
    off = cpu(t["trk_off"][k_lo:k_hi + 1])
    out["trk_off"] = (off - off[0]).astype(np.int32)
    out["trk_hits"] = cpu(t["trk_hits"][int(off[0]):int(off[-1])]) - b0
    out["trk_tracklet"] = (trk_t[k_lo:k_hi] - t_lo).astype(np.int32)
    out["status"]["n_grid"] = b1 - b0
    return out


def test_slice_status_and_any_size_properties(slice_run):
    ev, e, st, _ = slice_run
    assert st["overflow"] == 0
    assert st["n_grid"] == ev.n_clusters
    assert 0 < st["n_tracks"] <= st["n_starts"] <= e.start_capacity
    nt = int(st["n_tracks"])
    off = e.t["trk_off"][:nt + 1].cpu().numpy()
    ids = e.t["trk_hits"][:int(off[-1])].cpu().numpy()
    # every cluster is in at most one track; every track has hits of one
    # sector only, at increasing rows
    assert np.unique(ids).shape[0] == ids.shape[0]
    sec = np.searchsorted(ev.sector_offsets, ids, side="right") - 1
    first = np.repeat(sec[off[:-1]], np.diff(off))
    assert np.array_equal(sec, first)
    rows = ev.row[ids].astype(np.int64)
    inc = np.diff(rows)
    inner = np.ones(ids.shape[0] - 1, bool)
    inner[off[1:-1] - 1] = False
    assert np.all(inc[inner] > 0)


@pytest.mark.parametrize("s", SAMPLED_SECTORS)
def test_sampled_sectors_match_the_oracle(slice_run, s):
    ev, e, st, prm = slice_run
    sub = ev.sector(s)
    print(f"case c3 sector {s} n={sub.n_clusters}", flush=True)
    tab, nb = grid_layout(sub.sector_offsets, sub.sector_range, occupancy=e.occupancy,
                          sides=sub.sector_side)
    full_tab, _ = e.layout
    for f in ("y0", "z0", "inv_by", "inv_bz", "nby", "nbz"):
        assert tab[0][f] == full_tab[s][f], f
    o = oracle.track_event(sub.row, sub.y, sub.z, tab, nb, sub.row_x, prm)
    g = _sector_slice(ev, e, st, s)
    # the work counters are whole-slice totals: compare them as the oracle's
    g["status"]["n_propagations"], g["status"]["n_updates"], g["status"]["n_candidates"] = \
        o["tracklets"]["work"]
    assert_same_tracking(g, o, sub.n_clusters)


@pytest.mark.timeout(600)
def test_big_sector_between_small_ones(slice_run):
    """A sector of the slice (millions of clusters: the selection takes its
    row form there, one block per pad row) between two central-event sectors
    (row chunks in LDS) in one problem: staged and per-sector launches equal
    the oracle."""
    ev3 = slice_run[0]
    ev2 = synth.make_config2()
    parts = [ev2.sector(0), ev3.sector(SAMPLED_SECTORS[0]), ev2.sector(1)]
    cat = lambda f: np.concatenate([getattr(p, f) for p in parts])
    offs = np.concatenate([[0], np.cumsum([p.n_clusters for p in parts])]).astype(np.int64)
    ev = synth.Event(cat("row"), cat("y"), cat("z"), cat("charge"), offs,
                     np.concatenate([p.sector_range for p in parts]), ev2.row_x, cat("label"),
                     ev2.tracks, {}, cat("sector_side"))
    print(f"case mixed sectors n={ev.n_clusters} sizes={np.diff(offs).tolist()}", flush=True)
    o = run_oracle(ev)
    for mode in ("staged", "per_sector"):
        _, g = run_gpu(ev, mode=mode)
        assert g["status"]["overflow"] == 0
        assert_same_tracking(g, o, ev.n_clusters)


@pytest.mark.timeout(600)
def test_dense_sector_rows_beyond_one_key_table(slice_run):
    """Two sectors of the slice laid over each other as one sector (3.7M
    clusters, ~24k per pad row: more grid positions per row than one LDS key
    table of the selection's row form holds, so rows take several slices)
    between two central-event sectors: staged and per-sector launches equal
    the oracle."""
    ev3 = slice_run[0]
    ev2 = synth.make_config2()
    a, b = ev3.sector(SAMPLED_SECTORS[1]), ev3.sector(SAMPLED_SECTORS[1] + 1)
    assert np.array_equal(a.sector_range, b.sector_range)
    assert np.array_equal(a.sector_side, b.sector_side)
    dense = synth.Event(np.concatenate([a.row, b.row]), np.concatenate([a.y, b.y]),
                        np.concatenate([a.z, b.z]), np.concatenate([a.charge, b.charge]),
                        np.array([0, a.n_clusters + b.n_clusters], np.int64), a.sector_range,
                        a.row_x, np.concatenate([a.label, b.label]), a.tracks, {}, a.sector_side)
    parts = [ev2.sector(0), dense, ev2.sector(1)]
    cat = lambda f: np.concatenate([getattr(p, f) for p in parts])
    offs = np.concatenate([[0], np.cumsum([p.n_clusters for p in parts])]).astype(np.int64)
    ev = synth.Event(cat("row"), cat("y"), cat("z"), cat("charge"), offs,
                     np.concatenate([p.sector_range for p in parts]), ev2.row_x, cat("label"),
                     ev2.tracks, {}, cat("sector_side"))
    per_row = np.bincount(dense.row, minlength=152).max()
    print(f"case dense sector n={ev.n_clusters} sizes={np.diff(offs).tolist()} "
          f"max clusters per row {per_row}", flush=True)
    assert per_row > 16384
    o = run_oracle(ev)
    for mode in ("staged", "per_sector"):
        _, g = run_gpu(ev, mode=mode)
        assert g["status"]["overflow"] == 0
        assert_same_tracking(g, o, ev.n_clusters)


@pytest.mark.timeout(600)
def test_merging_links_of_sampled_sector_pair(slice_run):
    """Sector-track merging on the whole slice (1M tracks), checked where the
    oracle can compute it: the links between two adjacent sectors of one
    side for the tracks of a tan(lambda) band.  A link is a mutual best
    match and candidates lie within the tan(lambda) window (0.02) of the
    track, so the oracle, merging its own tracks of sector s with
    tan(lambda) in the band +-0.04 and of sector s+1 in the band +-0.02,
    sees every candidate of both best matches of every track of the band."""
    ev, e, st, prm = slice_run
    up, dn, _ = api.merge_sector_tracks(ctx(), e)
    torch.cuda.synchronize()
    nt = int(st["n_tracks"])
    up, dn = up[:nt].cpu().numpy(), dn[:nt].cpu().numpy()
    off = e.t["trk_off"][:nt + 1].cpu().numpy()
    hits = e.t["trk_hits"][:int(off[-1])].cpu().numpy()
    gsec = np.searchsorted(ev.sector_offsets, hits[off[:-1]], side="right") - 1
    by_first = {int(h): k for k, h in enumerate(hits[off[:-1]])}
    s = SAMPLED_SECTORS[1]
    lo_band, hi_band, w3 = 0.0, 0.02, api.MERGE_WINDOWS[3]
    sub_off, sub_hits, sub_par, sub_rin, sub_gpu, in_band = [0], [], [], [], [], []
    # margins a little wider than the window: the float window test may pass
    # a candidate a rounding step beyond it
    for q, margin in ((s, 2 * w3 + 1e-3), (s + 1, w3 + 5e-4)):
        sv = ev.sector(q)
        tab, nb = grid_layout(sv.sector_offsets, sv.sector_range, occupancy=e.occupancy,
                              sides=sv.sector_side)
        o = oracle.track_event(sv.row, sv.y, sv.z, tab, nb, sv.row_x, prm)
        trk, trl = o["tracks"], o["tracklets"]
        b0 = int(ev.sector_offsets[q])
        for k in range(len(trk["trk_off"]) - 1):
            t = trk["trk_tracklet"][k]
            tl = float(trl["par"][t][3])
            if not (lo_band - margin <= tl <= hi_band + margin):
                continue
            h = trk["trk_hits"][trk["trk_off"][k]:trk["trk_off"][k + 1]] + b0
            sub_hits.append(h)
            sub_off.append(sub_off[-1] + len(h))
            sub_par.append(trl["par"][t])
            sub_rin.append(trl["row_inner"][t])
            sub_gpu.append(by_first[int(h[0])])   # the same track on the GPU (same hits)
            in_band.append(q == s and lo_band <= tl <= hi_band)
    print(f"case merge slice sectors {s},{s + 1}: {len(sub_gpu)} tracks, "
          f"{sum(in_band)} in the band", flush=True)
    ou, od, _ = oracle.merge_sector_tracks(
        ev.sector_offsets, 18, ev.row_x, prm, np.array(sub_off, np.int32),
        np.concatenate(sub_hits).astype(np.int32), np.array(sub_par, np.float32),
        np.array(sub_rin, np.int32), iw=oracle.merge_windows_inv(api.MERGE_WINDOWS))
    sub_gpu = np.array(sub_gpu)
    n_links = 0
    for i in np.nonzero(in_band)[0]:
        o_part = ou[i] if ou[i] >= 0 else od[i]          # only sector s + 1 is there
        o_gpu = int(sub_gpu[o_part]) if o_part >= 0 else -1
        g = int(sub_gpu[i])
        g_part = -1
        for c in (up[g], dn[g]):
            if c >= 0 and gsec[c] == s + 1:
                g_part = int(c)
        assert g_part == o_gpu, (i, g, g_part, o_gpu)
        n_links += o_gpu >= 0
    print(f"  {n_links} links checked", flush=True)
    assert n_links > 50
