"""Helpers shared by the GPU tests: run the library and the oracle on the
same seeded event and map the library's grid-position outputs to cluster
ids."""
import numpy as np

import oracle
import synth
from paper_1905_05515_amd import api
from paper_1905_05515_amd.layout import grid_layout

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = api.Context(0)
    return _CTX


def run_gpu(ev, prm=None, occupancy=api.DEFAULT_OCCUPANCY, mode=None, use_graph=False, layout=None, **kw):
    prm = prm or synth.default_params()
    e = api.make_event(ev.row, ev.y, ev.z, ev.sector_offsets, ev.sector_range, ev.row_x, prm,
                       occupancy=occupancy, layout=layout, sector_side=ev.sector_side, **kw)
    if mode is None:
        api.track(ctx(), e)
    else:
        api.track_batch(ctx(), e, mode=mode, use_graph=use_graph)
    return e, api.results(e)


def run_oracle(ev, prm=None, occupancy=api.DEFAULT_OCCUPANCY, layout=None):
    prm = prm or synth.default_params()
    tab, nb = layout if layout is not None else grid_layout(ev.sector_offsets, ev.sector_range,
                                                            occupancy=occupancy,
                                                            sides=ev.sector_side)
    return oracle.track_event(ev.row, ev.y, ev.z, tab, nb, ev.row_x, prm)


def to_ids(g, n_clusters):
    """Library outputs in cluster-id space."""
    idg = g["idg"]

    def link(a):
        out = -np.ones(n_clusters, np.int32)
        v = np.where(a >= 0, idg[np.maximum(a, 0)], -1)
        out[idg] = v
        return out

    hits = np.where(g["t_hits"] >= 0, idg[np.maximum(g["t_hits"], 0)], -1).astype(np.int32)
    return dict(up0=link(g["up0"]), down0=link(g["down0"]), up=link(g["up"]),
                down=link(g["down"]), starts=idg[g["starts"]], hits=hits)


def same_floats(a, b):
    """Bit-for-bit equality of float32 arrays, where any NaN equals any NaN:
    IEEE 754 leaves the sign and payload of the NaN an invalid operation
    returns to the implementation (x86 returns the negative quiet NaN, the
    GPU the positive one), so only NaN-ness is compared."""
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    if a.shape != b.shape:
        return False
    na, nb = np.isnan(a), np.isnan(b)
    if not np.array_equal(na, nb):
        return False
    return np.array_equal(a.view(np.uint32)[~na], b.view(np.uint32)[~nb])


def assert_same_tracking(g, o, n_clusters):
    """Bit-exact equality of every stage, in id space."""
    s = g["status"]
    assert s["overflow"] == 0
    assert s["n_grid"] == o["grid"]["idg"].shape[0]
    assert np.array_equal(g["bin_start"], o["grid"]["bin_start"])
    assert np.array_equal(g["idg"], o["grid"]["idg"])
    assert same_floats(g["yg"], o["grid"]["yg"])
    assert same_floats(g["zg"], o["grid"]["zg"])
    gi = to_ids(g, n_clusters)
    for k in ("up0", "down0", "up", "down"):
        assert np.array_equal(gi[k], o[k]), k
    assert np.array_equal(gi["starts"], o["starts"])
    tr = o["tracklets"]
    # the transport stops on |sin(phi)| >= s_max at either end of a step, so
    # no state leaves its domain and no output is NaN
    for k in ("par", "cov", "chi2"):
        assert np.isfinite(tr[k]).all(), k
    assert np.array_equal(gi["hits"], tr["hits"])
    assert np.array_equal(g["t_nhits"], tr["nhits"])
    assert np.array_equal(g["t_rin"], tr["row_inner"])
    assert same_floats(g["t_par"], tr["par"])
    assert same_floats(g["t_cov"], tr["cov"])
    assert same_floats(g["t_chi2"], tr["chi2"])
    # the same transports, updates and candidate evaluations were made
    assert (s["n_propagations"], s["n_updates"], s["n_candidates"]) == tr["work"]
    t = o["tracks"]
    assert np.array_equal(g["trk_off"], t["trk_off"])
    assert np.array_equal(g["trk_hits"], t["trk_hits"])
    assert np.array_equal(g["trk_tracklet"], t["trk_tracklet"])
