"""Pins of the oracle's track-finding chain: grid, neighbours, cleaning,
chain starts, tracklets and selection.

The paper names the method (cellular-automaton seeding, then single-hypothesis
Kalman following, section 3) but no rule of it; the rules the oracle follows
are this project's readings.  They are pinned here by:
  * a library sort (grid), pure-Python brute force on tiny inputs
    (neighbour pairs, selection), hand-built geometric cases;
  * invariants that hold by construction (mutual links, disjoint chains,
    results independent of the bin layout and of the search acceleration);
  * generator truth: isolated helices are found exactly, hit for hit.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from paper_1905_05515_amd.layout import grid_layout

F32 = np.float32


def _single_sector(row, y, z, yr=None, zr=(0.0, 250.0), occupancy=2.0, n_rows=152):
    off = np.array([0, row.shape[0]], np.int64)
    if yr is None:
        yr = (float(y.min()) if y.size else -1.0, float(y.max()) if y.size else 1.0)
    rng_ = np.array([[yr[0], yr[1], zr[0], zr[1]]], np.float32)
    return grid_layout(off, rng_, n_rows=n_rows, occupancy=occupancy)


# ---------------------------------------------------------------- grid

def _bin_key(row, y, z, tab, sector_of, n_rows=152):
    """Global bin of each cluster, same clamp-and-truncate definition; rows
    >= n_rows in the sector's last bin."""
    s = tab[sector_of]
    fy = (y - s["y0"]) * s["inv_by"]
    fz = (z - s["z0"]) * s["inv_bz"]
    fy = np.where(fy >= 0, fy, F32(0))
    fz = np.where(fz >= 0, fz, F32(0))
    fy = np.minimum(fy, (s["nby"] - 1).astype(np.float32))
    fz = np.minimum(fz, (s["nbz"] - 1).astype(np.float32))
    key = s["bin_base"] + (row.astype(np.int64) * s["nbz"] + fz.astype(np.int64)) * s["nby"] \
        + fy.astype(np.int64)
    bad = row >= n_rows
    return np.where(bad, s["bin_base"] + n_rows * s["nbz"] * s["nby"], key)


@pytest.mark.parametrize("occ", [0.5, 2.0, 7.0])
def test_grid_is_stable_sort_by_bin(occ):
    ev = synth.make_config2().sector(3)
    big = synth.make_config1()
    for e in (ev, big):
        tab, nb = grid_layout(e.sector_offsets, e.sector_range, occupancy=occ)
        g = oracle.build_grid(e.row, e.y, e.z, tab, nb)
        sec = np.zeros(e.n_clusters, np.int64)
        key = _bin_key(e.row, e.y, e.z, tab, sec)
        order = np.argsort(key, kind="stable")
        assert np.array_equal(g["idg"], order.astype(np.int32))
        assert np.array_equal(g["yg"], e.y[order]) and np.array_equal(g["zg"], e.z[order])
        counts = np.bincount(key, minlength=nb)
        assert np.array_equal(g["bin_start"], np.concatenate([[0], np.cumsum(counts)]).astype(np.int32))


def test_grid_multi_sector_and_bad_rows():
    """Sectors occupy their own id range of grid positions; a cluster with an
    invalid row lands in its sector's last bin, after every valid one."""
    ev = synth.make_config2()
    sel = np.concatenate([np.arange(ev.sector_offsets[s], ev.sector_offsets[s] + 500) for s in range(5)])
    row = ev.row[sel].copy()
    row[7] = 200
    row[1203] = 152
    off = np.arange(6, dtype=np.int64) * 500
    tab, nb = grid_layout(off, ev.sector_range[:5])
    g = oracle.build_grid(row, ev.y[sel], ev.z[sel], tab, nb)
    assert g["idg"].shape[0] == 2500
    sec = np.repeat(np.arange(5), 500)
    key = _bin_key(row, ev.y[sel], ev.z[sel], tab, sec)
    order = np.argsort(key, kind="stable")
    assert np.array_equal(g["idg"], order.astype(np.int32))
    assert g["idg"][499] == 7 and g["idg"][1499] == 1203
    for s in range(5):
        assert g["bin_start"][tab["bin_base"][s]] == 500 * s
        assert np.all(g["idg"][500 * s:500 * (s + 1)] // 500 == s)


# ---------------------------------------------------------------- neighbours

def brute_neighbours(row, y, z, sector, X, prm, n_rows):
    """All pairs, straight from the definition (pure Python, float32)."""
    n = row.shape[0]
    up0 = -np.ones(n, np.int32)
    down0 = -np.ones(n, np.int32)
    Wy, Wz, D2m = F32(prm["nb_win_y"]), F32(prm["nb_win_z"]), F32(prm["nb_d2max"])
    for h in range(n):
        r = int(row[h])
        if r == 0 or r >= n_rows - 1:
            continue
        slope = y[h] / X[r]
        yu_c, yd_c = slope * X[r + 1], slope * X[r - 1]
        U = [u for u in range(n) if sector[u] == sector[h] and row[u] == r + 1
             and abs(y[u] - yu_c) <= Wy and abs(z[u] - z[h]) <= Wz]
        D = [d for d in range(n) if sector[d] == sector[h] and row[d] == r - 1
             and abs(y[d] - yd_c) <= Wy and abs(z[d] - z[h]) <= Wz]
        best = None
        for u in U:
            for d in D:
                dy = (y[u] + y[d]) - (y[h] + y[h])
                dz = (z[u] + z[d]) - (z[h] + z[h])
                d2 = dy * dy + dz * dz
                if d2 <= D2m and (best is None or (d2, u, d) < best):
                    best = (d2, u, d)
        if best is not None:
            up0[h], down0[h] = best[1], best[2]
    return up0, down0


def _tiny_event(seed, n=220, n_rows=10, n_sec=2):
    rng = np.random.default_rng(seed)
    X = (100.0 + np.arange(n_rows) * 1.0596026).astype(np.float32)
    sec = np.sort(rng.integers(0, n_sec, n))
    # a few straight tracks plus dense noise on a small patch: many candidates
    row = rng.integers(0, n_rows, n).astype(np.uint8)
    y = rng.uniform(-4, 4, n).astype(np.float32)
    z = rng.uniform(0, 8, n).astype(np.float32)
    # snap some values to a coarse lattice to create exact D2 ties
    snap = rng.random(n) < 0.3
    y[snap] = np.round(y[snap] * 4) / 4
    z[snap] = np.round(z[snap] * 4) / 4
    off = np.searchsorted(sec, np.arange(n_sec + 1)).astype(np.int64)
    rng_ = np.array([[-4.0, 4.0, 0.0, 8.0]] * n_sec, np.float32)
    return row, y, z, sec, X, off, rng_


@pytest.mark.parametrize("seed", range(6))
def test_neighbours_match_brute_force(seed):
    row, y, z, sec, X, off, rng_ = _tiny_event(seed)
    prm = synth.default_params()
    for occ in (0.3, 1.0, 4.0):
        tab, nb = grid_layout(off, rng_, n_rows=X.shape[0], occupancy=occ)
        g = oracle.build_grid(row, y, z, tab, nb, n_rows=X.shape[0])
        up0, down0 = oracle.find_neighbours(tab, X, prm, g, row.shape[0], n_rows=X.shape[0])
        bu, bd = brute_neighbours(row, y, z, sec, X, prm, X.shape[0])
        assert np.array_equal(up0, bu) and np.array_equal(down0, bd)
    assert (up0 >= 0).sum() > 10


def _hand(rows, ys, zs, prm=None, n_rows=3):
    X = np.array([100.0, 101.0, 102.0][:n_rows], np.float32)
    row = np.array(rows, np.uint8)
    y = np.array(ys, np.float32)
    z = np.array(zs, np.float32)
    tab, nb = _single_sector(row, y, z, yr=(-20, 20), zr=(0, 20), n_rows=n_rows)
    g = oracle.build_grid(row, y, z, tab, nb, n_rows=n_rows)
    prm = prm or synth.default_params()
    return oracle.find_neighbours(tab, X, prm, g, row.shape[0], n_rows=n_rows)


def test_neighbour_hand_cases():
    # collinear triple (uniform spacing): D2 = 0, both links
    up0, down0 = _hand([1, 2, 0], [10.0, 11.0, 9.0], [5.0, 5.5, 4.5])
    assert up0.tolist() == [1, -1, -1] and down0.tolist() == [2, -1, -1]
    # exact tie in D2 (0.25 each way): the lower id of the up hit wins, then of the down hit
    up0, down0 = _hand([1, 2, 2, 0, 0], [10.0, 11.5, 10.5, 9.0, 9.0], [5.0, 5.0, 5.0, 5.0, 5.0])
    assert (up0[0], down0[0]) == (1, 3)
    up0, down0 = _hand([1, 2, 2, 0, 0], [10.0, 10.5, 11.5, 9.0, 9.0], [5.0, 5.0, 5.0, 5.0, 5.0])
    assert (up0[0], down0[0]) == (1, 3)
    # smaller deviation beats lower id
    up0, down0 = _hand([1, 2, 2, 0], [10.0, 11.6, 11.1, 9.0], [5.0, 5.0, 5.0, 5.0])
    assert up0[0] == 2
    # D2 just above the cut (1.0): no link; exactly at it: link
    up0, _ = _hand([1, 2, 0], [10.0, 12.0, 9.0], [5.0, 5.0, 5.0])       # dy = 1 -> D2 = 1
    assert up0[0] == 1
    up0, _ = _hand([1, 2, 0], [10.0, 12.0625, 9.0], [5.0, 5.0, 5.0])
    assert up0[0] == -1
    # straight line but outside the origin-pointing window (|dy| > 2.5 around 10*102/101)
    up0, _ = _hand([1, 2, 0], [10.0, 13.0, 7.0], [5.0, 5.0, 5.0])
    assert up0[0] == -1
    # outside the z window
    up0, _ = _hand([1, 2, 0], [10.0, 11.0, 9.0], [5.0, 8.0, 2.0])
    assert up0[0] == -1
    # first and last rows never get links
    up0, down0 = _hand([0, 1, 2], [9.0, 10.0, 11.0], [5.0, 5.0, 5.0])
    assert up0[0] == -1 and down0[0] == -1 and up0[2] == -1 and down0[2] == -1 and up0[1] == 2


# ---------------------------------------------------------------- cleaning and starts

def test_clean_and_starts_hand_cases():
    #             0   1   2   3   4   5   6   7
    up0 = np.array([1, 2, 3, -1, 5, 6, -1, 0], np.int32)
    down0 = np.array([-1, 0, 1, 2, -1, 7, 5, -1], np.int32)
    up, down = oracle.clean_links(up0, down0)
    # 0-1-2-3 mutual; 4->5 not mutual (down0[5] = 7); 5<->6 mutual; 7->0 not (down0[0] = -1)
    assert up.tolist() == [1, 2, 3, -1, -1, 6, -1, -1]
    assert down.tolist() == [-1, 0, 1, 2, -1, -1, 5, -1]
    starts = oracle.select_starts(up, down)
    assert starts.tolist() == [0]              # 5-6 is a chain of two: no start


def test_clean_links_invariants_on_event():
    ev = synth.make_config2().sector(7)
    tab, nb = grid_layout(ev.sector_offsets, ev.sector_range)
    res = oracle.track_event(ev.row, ev.y, ev.z, tab, nb, ev.row_x, synth.default_params())
    up, down = res["up"], res["down"]
    h = np.nonzero(up >= 0)[0]
    assert np.all(down[up[h]] == h)
    h = np.nonzero(down >= 0)[0]
    assert np.all(up[down[h]] == h)
    # chains are disjoint paths: following up from every start visits each hit once
    seen = np.zeros(ev.n_clusters, bool)
    for s in res["starts"]:
        c = s
        n = 0
        while c >= 0:
            assert not seen[c]
            seen[c] = True
            c = up[c]
            n += 1
        assert n >= 3
    # starts in ascending id, and every chain of >= 3 hits has exactly one start
    st = res["starts"]
    assert np.all(np.diff(st) > 0)
    lowest = np.nonzero((up >= 0) & (down < 0))[0]
    long = lowest[up[up[lowest]] >= 0]
    assert np.array_equal(np.sort(long), st)


# ---------------------------------------------------------------- tracklets

def _run(ev, occ=2.0, brute=False):
    tab, nb = grid_layout(ev.sector_offsets, ev.sector_range, occupancy=occ)
    return oracle.track_event(ev.row, ev.y, ev.z, tab, nb, ev.row_x, synth.default_params(),
                              brute=brute)


def _track_sets(res):
    off, hits = res["tracks"]["trk_off"], res["tracks"]["trk_hits"]
    return [tuple(hits[off[i]:off[i + 1]]) for i in range(off.shape[0] - 1)]


def test_results_independent_of_bin_layout_and_search_acceleration():
    """The grid accelerates but never decides: links, starts, tracklets and
    tracks are identical for any bin occupancy and with whole-row scans."""
    for ev in (synth.make_config1(), synth.make_config2().sector(11)):
        ref = _run(ev, 2.0)
        for occ, brute in ((0.25, False), (9.0, False), (2.0, True)):
            res = _run(ev, occ, brute)
            for key in ("up0", "down0", "starts"):
                assert np.array_equal(res[key], ref[key]), key
            for key in ("hits", "nhits", "par", "cov", "chi2"):
                assert np.array_equal(res["tracklets"][key], ref["tracklets"][key]), key
            assert _track_sets(res) == _track_sets(ref)


def test_isolated_helices_are_found_hit_for_hit():
    """Well separated tracks: every track is found once, with exactly the
    clusters its helix left, in every row it crossed."""
    rng = np.random.default_rng(17)
    for n_trk, noise in ((6, 0.0), (6, 0.05)):
        trk = synth.events._sample_tracks(rng, n_trk, 0.0, 1.0, 0.1, 0.8, 0.6)
        trk["phi0"] = np.radians(np.linspace(1.0, 19.0, n_trk))      # > 3 degrees apart
        trk["tanl"] = np.linspace(0.15, 0.9, n_trk)
        row, y, z, lab = synth.events._instance_clusters(rng, trk)
        ylim = synth.events.ROW_X64 * synth.TAN10
        row, y, z, lab = synth.events._add_noise_and_pack(rng, row, y, z, lab, noise, ylim,
                                                          0.0, 250.0)
        off = np.array([0, row.shape[0]], np.int64)
        rng_ = np.array([[y.min(), y.max(), 0.0, 250.0]], np.float32)
        tab, nb = grid_layout(off, rng_)
        res = oracle.track_event(row, y, z, tab, nb, synth.ROW_X, synth.default_params())
        found = _track_sets(res)
        truth = [tuple(np.sort(np.nonzero(lab == t)[0])) for t in range(n_trk)]
        got = sorted(tuple(sorted(f)) for f in found)
        assert got == sorted(truth)


PAR_FLOOR = np.array([1.0, 1.0, 0.01, 0.01, 0.1])   # cm, cm, -, -, (GeV/c)^-1


def rel_par_error(p32, p64, c64):
    """|a - b| / max(|b|, floor, sigma): relative to the parameter, to a floor
    of its natural scale, or to its own uncertainty, whichever is largest."""
    sig = np.sqrt(np.asarray(c64)[[0, 2, 5, 9, 14]])
    return np.abs(np.asarray(p32, np.float64) - p64) / np.maximum(np.maximum(np.abs(p64), PAR_FLOOR), sig)


def test_tracklet_hit_lists_and_fit_are_consistent():
    """Hit lists sit on their rows; the float fit equals its double-precision
    replay over the same hits to 1e-4 (relative, see rel_par_error) for all
    but a rare few tracklets, and to 1e-3 for all: the float filter's own
    rounding."""
    ev = synth.make_config2().sector(2)
    res = _run(ev)
    trl = res["tracklets"]
    prm = synth.default_params()
    starts = res["starts"]
    assert trl["hits"].shape[0] == starts.shape[0]
    errs = []
    for t in range(starts.shape[0]):
        hb = trl["hits"][t]
        rows = np.nonzero(hb >= 0)[0]
        assert trl["nhits"][t] == rows.shape[0]
        assert np.all(ev.row[hb[rows]] == rows)           # each hit sits on its row
        assert trl["row_inner"][t] == rows.min()
        st, p64, c64, chi64 = oracle.tracklet_replay64(ev.row_x, prm, ev.y, ev.z,
                                                      int(ev.row[starts[t]]), hb)
        if st != 0 or trl["nhits"][t] < prm["min_tracklet_hits"]:
            continue
        errs.append(rel_par_error(trl["par"][t], p64, c64).max())
        assert abs(trl["chi2"][t] - chi64) <= 1e-3 * max(1.0, chi64)
    errs = np.array(errs)
    assert errs.shape[0] > 200
    assert np.mean(errs > 1e-4) < 2e-3 and errs.max() < 1e-3


# ---------------------------------------------------------------- selection

def brute_select(n_clusters, hits, nhits, starts, prm):
    keys = [((int(nhits[t]) << 32) | (0xFFFFFFFF - int(starts[t])))
            if nhits[t] >= prm["min_tracklet_hits"] else 0 for t in range(len(starts))]
    owner = {}
    for t, k in enumerate(keys):
        if k:
            for c in hits[t]:
                if c >= 0:
                    owner[c] = max(owner.get(c, 0), k)
    out = []
    for t, k in enumerate(keys):
        if not k:
            continue
        kept = [c for c in hits[t] if c >= 0 and owner[c] == k]
        if len(kept) >= prm["min_track_hits"]:
            out.append((t, tuple(kept)))
    return out


@pytest.mark.parametrize("seed", range(5))
def test_selection_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    n_clusters, n_rows, m = 300, 40, 60
    prm = synth.default_params()
    hits = -np.ones((m, n_rows), np.int32)
    for t in range(m):
        k = rng.integers(3, 35)
        rows = np.sort(rng.choice(n_rows, k, replace=False))
        hits[t, rows] = rng.choice(n_clusters, k, replace=False)
    nhits = (hits >= 0).sum(1).astype(np.int32)
    nhits[rng.random(m) < 0.2] = 25                  # force equal lengths: ties on start id
    starts = np.sort(rng.choice(10**6, m, replace=False)).astype(np.int32)
    res = oracle.select_tracks(n_clusters, prm, dict(hits=hits, nhits=nhits), starts,
                               n_rows=n_rows)
    got = [(int(res["trk_tracklet"][i]),
            tuple(res["trk_hits"][res["trk_off"][i]:res["trk_off"][i + 1]]))
           for i in range(res["trk_tracklet"].shape[0])]
    assert got == brute_select(n_clusters, hits, nhits, starts, prm)


def test_selection_hand_cases():
    prm = dict(synth.default_params(), min_tracklet_hits=3, min_track_hits=2)
    n_rows = 8
    hits = -np.ones((4, n_rows), np.int32)
    hits[0, :4] = [10, 11, 12, 13]        # 4 hits
    hits[1, :5] = [10, 11, 20, 21, 22]    # 5 hits: takes 10, 11 from tracklet 0
    hits[2, :5] = [30, 31, 32, 33, 34]    # 5 hits, start id 7 (higher than tracklet 3)
    hits[3, :5] = [30, 31, 40, 41, 42]    # 5 hits, start id 5: wins 30, 31
    nhits = (hits >= 0).sum(1).astype(np.int32)
    starts = np.array([1, 2, 7, 5], np.int32)
    res = oracle.select_tracks(50, prm, dict(hits=hits, nhits=nhits), starts, n_rows=n_rows)
    off, th = res["trk_off"], res["trk_hits"]
    tracks = {int(t): th[off[i]:off[i + 1]].tolist() for i, t in enumerate(res["trk_tracklet"])}
    assert tracks == {0: [12, 13], 1: [10, 11, 20, 21, 22], 2: [32, 33, 34],
                      3: [30, 31, 40, 41, 42]}
    prm["min_track_hits"] = 3
    res = oracle.select_tracks(50, prm, dict(hits=hits, nhits=nhits), starts, n_rows=n_rows)
    assert res["trk_tracklet"].tolist() == [1, 2, 3]


def test_each_cluster_in_at_most_one_track():
    ev = synth.make_config2().sector(20)
    res = _run(ev)
    hits = res["tracks"]["trk_hits"]
    assert np.unique(hits).shape[0] == hits.shape[0]
    off = res["tracks"]["trk_off"]
    for i in range(off.shape[0] - 1):
        h = hits[off[i]:off[i + 1]]
        assert np.all(np.diff(ev.row[h].astype(int)) > 0)
