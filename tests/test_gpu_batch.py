"""Launch forms of the tracking chain through tpc_track_batch: one launch per
stage over all sectors, one launch sequence per sector, and (when built) one
persistent launch over a device work queue; with and without graph replay.
Every form gives bit-identical outputs, equal to the oracle's."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import assert_same_tracking, ctx, run_gpu, run_oracle
from paper_1905_05515_amd import api

pytestmark = pytest.mark.gpu

KEYS = ("bin_start", "yg", "zg", "idg", "up0", "down0", "up", "down", "starts", "t_start",
        "t_hits", "t_nhits", "t_rin", "t_par", "t_cov", "t_chi2", "trk_off", "trk_hits",
        "trk_tracklet", "trk_side")


def _same(a, b):
    for k in KEYS:
        x, y = a[k], b[k]
        if x.dtype.kind == "f":
            x, y = x.view(np.uint32), y.view(np.uint32)
        assert np.array_equal(x, y), k
    for k in ("n_grid", "n_starts", "n_tracks", "n_track_hits", "n_propagations", "n_updates",
              "n_candidates", "overflow", "n_bad_rows"):
        assert a["status"][k] == b["status"][k], k


def _forms(ev, forms):
    side = torch.cuda.Stream()
    out = {}
    for mode, graph in forms:
        e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x,
                           synth.default_params(), sector_side=ev.sector_side)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            for _ in range(2 if graph else 1):      # a graph is captured, then replayed
                api.track_batch(ctx(), e, mode=mode, use_graph=graph)
        side.synchronize()
        out[(mode, graph)] = api.results(e)
    return out


def test_per_sector_form_equals_staged_and_oracle():
    ev = synth.make_config2()
    print(f"case c2 forms n={ev.n_clusters}", flush=True)
    r = _forms(ev, [("staged", False), ("per_sector", False), ("per_sector", True)])
    o = run_oracle(ev)
    assert_same_tracking(r[("per_sector", False)], o, ev.n_clusters)
    _same(r[("staged", False)], r[("per_sector", False)])
    _same(r[("staged", False)], r[("per_sector", True)])


def test_persistent_form_equals_staged_and_oracle():
    ev = synth.make_config2()
    print(f"case c2 persistent n={ev.n_clusters}", flush=True)
    r = _forms(ev, [("staged", False), ("persistent", False), ("persistent", True)])
    o = run_oracle(ev)
    assert r[("persistent", False)]["status"]["overflow"] == 0
    assert_same_tracking(r[("persistent", False)], o, ev.n_clusters)
    _same(r[("staged", False)], r[("persistent", False)])
    _same(r[("staged", False)], r[("persistent", True)])


def test_persistent_small_and_edge_events():
    """Single sector, an empty sector in the middle, invalid rows."""
    for ev in (synth.make_config1(), synth.make_config2().sector(5)):
        r = _forms(ev, [("staged", False), ("persistent", False)])
        _same(r[("staged", False)], r[("persistent", False)])
    ev = synth.make_config2()
    a0, a1 = int(ev.sector_offsets[4]), int(ev.sector_offsets[5])
    b0, b1 = int(ev.sector_offsets[7]), int(ev.sector_offsets[7]) + 3000
    sel = np.concatenate([np.arange(a0, a1), np.arange(b0, b1)])
    row = ev.row[sel].copy()
    row[10] = 200
    offs = np.array([0, a1 - a0, a1 - a0, sel.shape[0]], np.int64)
    sub = synth.Event(row, ev.y[sel], ev.z[sel], ev.charge[sel], offs, ev.sector_range[[4, 5, 7]],
                      ev.row_x, ev.label[sel], ev.tracks, {})
    r = _forms(sub, [("staged", False), ("persistent", False), ("per_sector", False)])
    _same(r[("staged", False)], r[("persistent", False)])
    _same(r[("staged", False)], r[("per_sector", False)])


@pytest.mark.timeout(900)
def test_batched_uneven_instances_full_size():
    """512 single-sector instances of very uneven size (~14M clusters): the
    staged and per-sector forms agree bit for bit, and match the oracle."""
    ev = synth.make_config4()
    print(f"case c4 n={ev.n_clusters} instances={ev.n_sectors}", flush=True)
    r = _forms(ev, [("staged", True), ("per_sector", False), ("persistent", True)])
    _same(r[("staged", True)], r[("per_sector", False)])
    _same(r[("staged", True)], r[("persistent", True)])
    o = run_oracle(ev)
    assert_same_tracking(r[("staged", True)], o, ev.n_clusters)


@pytest.mark.timeout(600)
def test_persistent_tile_scales():
    """The persistent form grows its tiles with the clusters per resident
    block (scale 1, 2 or 4).  The central event and the full 512-instance set
    cover the smallest and the largest scale on this part; the first
    instances of the set, about 4.5M clusters, the middle one.  Every scale
    gives the staged form's outputs."""
    ev = synth.make_config4()
    k = int(np.searchsorted(ev.sector_offsets, 4_500_000))
    n = int(ev.sector_offsets[k])
    sub = synth.Event(ev.row[:n], ev.y[:n], ev.z[:n], ev.charge[:n],
                      ev.sector_offsets[:k + 1].copy(), ev.sector_range[:k].copy(), ev.row_x,
                      ev.label[:n], ev.tracks, {}, ev.sector_side[:k].copy())
    print(f"case c4 first {k} instances n={n}", flush=True)
    r = _forms(sub, [("staged", False), ("persistent", False), ("persistent", True)])
    assert r[("persistent", False)]["status"]["overflow"] == 0
    _same(r[("staged", False)], r[("persistent", False)])
    _same(r[("staged", False)], r[("persistent", True)])


@pytest.mark.timeout(600)
def test_launch_shapes_change_no_output():
    """Every launch shape the context accepts (tracklet hit lists in LDS or
    written directly, starts dealt by a device queue, neighbour blocks of 64-256 threads, persistent tile
    scales 1-8 and 1-2 blocks per compute unit) gives the outputs of the
    automatic shapes bit for bit; the shape tuner keeps the tracks and
    leaves valid shapes set; invalid shapes are refused."""
    ev = synth.make_config2()
    print(f"case c2 launch shapes n={ev.n_clusters}", flush=True)
    c = api.Context(0)
    e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x,
                       synth.default_params(), sector_side=ev.sector_side)
    side = torch.cuda.Stream()             # graphs are captured on a stream of their own
    torch.cuda.synchronize()
    api.track_batch(c, e, mode="staged", stream=side)
    ref = api.results(e, side)
    cases = [("staged", dict(tracklet_form=1)), ("staged", dict(tracklet_form=2)),
             ("staged", dict(tracklet_form=3)), ("per_sector", dict(tracklet_form=3)),
             ("staged", dict(neighbour_block=64)), ("staged", dict(neighbour_block=128)),
             ("per_sector", dict(tracklet_form=2, neighbour_block=128)),
             ("persistent", dict(persistent_scale=1)), ("persistent", dict(persistent_scale=8)),
             ("persistent", dict(persistent_scale=2, persistent_blocks_per_cu=1))]
    for mode, kw in cases:
        api.set_tuning(c, **{k: 0 for k in api.TUNING_FIELDS})
        api.set_tuning(c, **kw)
        for graph in (False, True, True):
            with torch.cuda.stream(side):
                api.track_batch(c, e, mode=mode, use_graph=graph, stream=side)
            print(f"  {mode} {kw} graph={graph}", flush=True)
            _same(ref, api.results(e, side))
    api.set_tuning(c, **{k: 0 for k in api.TUNING_FIELDS})
    for mode in ("staged", "persistent"):
        shapes, times = api.autotune_shapes(c, e, mode=mode, reps=1, stream=side)
        print(f"  tuned {mode}: {shapes} {times}", flush=True)
        _same(ref, api.results(e, side))
    for bad in (dict(tracklet_form=4), dict(neighbour_block=96), dict(persistent_scale=3),
                dict(persistent_blocks_per_cu=-1)):
        with pytest.raises(api.L.TPCError):
            api.set_tuning(c, **bad)
    c.close()
