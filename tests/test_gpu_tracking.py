"""GPU parity of the tracking chain against the oracle, through the C ABI.

Bit-exact: grid permutation and bin starts, raw and cleaned links, chain
starts, tracklet hit lists, tracklet parameters, covariances and chi2 (both
sides evaluate the same binary32 expressions in the same order, without
contraction), and track lists.  Inputs are the seeded synthetic events."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import assert_same_tracking, ctx, run_gpu, run_oracle, to_ids
from paper_1905_05515_amd import api
from paper_1905_05515_amd.layout import grid_layout

pytestmark = pytest.mark.gpu


def _ev(name):
    if name == "c1":
        return synth.make_config1()
    if name == "c2_sector":
        return synth.make_config2().sector(9)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["c1", "c2_sector"])
def test_parity_small(name):
    ev = _ev(name)
    print(f"case {name} n={ev.n_clusters}", flush=True)
    _, g = run_gpu(ev)
    o = run_oracle(ev)
    assert_same_tracking(g, o, ev.n_clusters)
    assert g["status"]["n_tracks"] > 0


def test_parity_central_event_full():
    """One central Pb-Pb-like event, 36 sectors, ~1.3M clusters, every output."""
    ev = synth.make_config2()
    print(f"case c2 n={ev.n_clusters}", flush=True)
    _, g = run_gpu(ev)
    o = run_oracle(ev)
    assert_same_tracking(g, o, ev.n_clusters)
    assert g["status"]["n_tracks"] > 10000


@pytest.mark.parametrize("occ", [0.3, 6.0])
def test_parity_other_bin_layouts(occ):
    """Tracks do not depend on the bin layout; grids follow it exactly."""
    ev = synth.make_config2().sector(20)
    _, g = run_gpu(ev, occupancy=occ)
    o = run_oracle(ev, occupancy=occ)
    assert_same_tracking(g, o, ev.n_clusters)
    _, g2 = run_gpu(ev, occupancy=2.0)
    assert np.array_equal(g["trk_hits"], g2["trk_hits"])
    assert np.array_equal(g["trk_off"], g2["trk_off"])


def test_edge_cases_empty_sector_bad_rows_single_bin():
    ev = synth.make_config2()
    # three sectors: a normal one, an empty one, and one with a bad row
    a0, a1 = int(ev.sector_offsets[4]), int(ev.sector_offsets[5])
    b0, b1 = int(ev.sector_offsets[7]), int(ev.sector_offsets[7]) + 3000
    sel = np.concatenate([np.arange(a0, a1), np.arange(b0, b1)])
    row = ev.row[sel].copy()
    row[10] = 200
    row[a1 - a0 + 5] = 152
    offs = np.array([0, a1 - a0, a1 - a0, sel.shape[0]], np.int64)
    rng_ = ev.sector_range[[4, 5, 7]]
    sub = synth.Event(row, ev.y[sel], ev.z[sel], ev.charge[sel], offs, rng_, ev.row_x,
                      ev.label[sel], ev.tracks, {})
    _, g = run_gpu(sub)
    o = run_oracle(sub)
    assert g["status"]["n_bad_rows"] == 2
    assert g["status"]["n_grid"] == sub.n_clusters
    assert_same_tracking(g, o, sub.n_clusters)
    # every sector in a single bin per row: the searches scan whole rows
    lay = grid_layout(offs, rng_, occupancy=1e9)
    assert int(lay[0]["nby"].max()) == 1 and int(lay[0]["nbz"].max()) == 1
    _, g1 = run_gpu(sub, layout=lay)
    o1 = run_oracle(sub, layout=lay)
    assert_same_tracking(g1, o1, sub.n_clusters)
    assert np.array_equal(g1["trk_hits"], g["trk_hits"])


def test_tiny_events():
    prm = synth.default_params()
    # a lone cluster; three collinear clusters (a chain too short for a track)
    for rows, ys, zs in (([5], [1.0], [2.0]), ([4, 5, 6], [10.0, 10.1, 10.2], [5.0, 5.0, 5.0])):
        row = np.array(rows, np.uint8)
        y = np.array(ys, np.float32)
        z = np.array(zs, np.float32)
        ev = synth.Event(row, y, z, np.zeros_like(y), np.array([0, len(rows)], np.int64),
                         np.array([[-50, 50, 0, 250]], np.float32), synth.ROW_X,
                         np.zeros(len(rows), np.int32), {}, {})
        _, g = run_gpu(ev, prm)
        o = run_oracle(ev, prm)
        assert_same_tracking(g, o, ev.n_clusters)
        assert g["status"]["n_tracks"] == 0


def test_capacity_overflow_is_flagged():
    ev = synth.make_config1()
    _, g = run_gpu(ev, start_capacity=5, track_capacity=5)
    st = g["status"]
    assert st["overflow"] & 1 and st["n_starts"] > 5
    o = run_oracle(ev)
    # the starts that fit are the first ones, in id order
    assert np.array_equal(to_ids(g, ev.n_clusters)["starts"], o["starts"][:5])


def test_deterministic_repeat_and_graph_replay():
    ev = synth.make_config2().sector(3)
    e, g = run_gpu(ev)
    c = ctx()
    for rep in range(3):
        api.track(c, e)
        r = api.results(e)
        assert np.array_equal(r["trk_hits"], g["trk_hits"])
        assert np.array_equal(r["t_par"].view(np.uint32), g["t_par"].view(np.uint32))
    side = torch.cuda.Stream()           # graphs are captured on a non-default stream
    e2, _ = run_gpu(ev)
    for rep in range(4):
        e2.t["trk_hits"].fill_(-7)           # eager work between replays
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            api.track_batch(c, e2, mode="staged", use_graph=True)
        side.synchronize()
        r = api.results(e2)
        assert np.array_equal(r["trk_off"], g["trk_off"])
        assert np.array_equal(r["trk_hits"], g["trk_hits"])
        assert np.array_equal(r["idg"], g["idg"])


def test_track_parameters_match_fp64_replay():
    """Tracklet parameters of the selected tracks against a float64 replay
    of the same hit sequence: relative 1e-4 of max(|p|, floor, sigma) for all
    but the rare tracks where the float filter's own rounding shows, 1e-3
    for every track."""
    ev = synth.make_config2().sector(14)
    _, g = run_gpu(ev)
    prm = synth.default_params()
    ids = to_ids(g, ev.n_clusters)
    floor = np.array([1.0, 1.0, 0.01, 0.01, 0.1])
    errs = []
    for t in g["trk_tracklet"]:
        st, p64, c64, _ = oracle.tracklet_replay64(ev.row_x, prm, ev.y, ev.z,
                                                   int(ev.row[ids["starts"][t]]), ids["hits"][t])
        if st:
            continue
        sig = np.sqrt(c64[[0, 2, 5, 9, 14]])
        d = np.abs(g["t_par"][t].astype(np.float64) - p64) / np.maximum(np.maximum(np.abs(p64), floor), sig)
        errs.append(d.max())
    errs = np.array(errs)
    assert errs.shape[0] > 100
    assert np.mean(errs > 1e-4) < 2e-3 and errs.max() < 1e-3


def test_autotuned_layout_gives_the_same_tracks():
    """The autotuner only picks a bin layout: the tracks found with its pick
    are the oracle's, and equal to those of a fixed layout."""
    ev = synth.make_config2()
    print(f"case c2 autotune n={ev.n_clusters}", flush=True)
    prm = synth.default_params()
    e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x, prm,
                       occupancy=2.0, sector_side=ev.sector_side)
    best, times = api.autotune(ctx(), e, candidates=(0.125, 0.5, 2.0), reps=2)
    assert best in times and all(v > 0 for v in times.values())
    assert ctx().tuned[(e.problem.n_sectors, e.problem.n_clusters, "staged")] == best
    api.track(ctx(), e)
    g = api.results(e)
    o = run_oracle(ev, occupancy=best)
    assert_same_tracking(g, o, ev.n_clusters)
    _, g2 = run_gpu(ev, occupancy=2.0)
    assert np.array_equal(g["trk_hits"], g2["trk_hits"])
    assert np.array_equal(g["trk_off"], g2["trk_off"])
