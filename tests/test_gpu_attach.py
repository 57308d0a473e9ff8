"""Track-based cluster attachment on the GPU (tpc_attach_clusters) against
the oracle, cluster by cluster: the owning or adjacent track and the state
bits (attached, adjacent, protected, removed) of every cluster id, after the
tracking chain of the same event on both sides."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import ctx, run_gpu, run_oracle
from paper_1905_05515_amd import api

pytestmark = pytest.mark.gpu


def _oracle_attach(ev, o, radius=1.5, pt_good=0.05):
    trk = o["tracks"]
    trl = o["tracklets"]
    tt = trk["trk_tracklet"]
    return oracle.attach_clusters(ev.sector_offsets, ev.row, ev.y, ev.z, ev.row_x,
                                  synth.default_params(), trk["trk_off"], trk["trk_hits"],
                                  trl["par"][tt], trl["row_inner"][tt], radius, pt_good)


def _gpu_attach(ev, radius=1.5, pt_good=0.05, **kw):
    e, g = run_gpu(ev, **kw)
    track, state = api.attach_clusters(ctx(), e, radius, pt_good)
    torch.cuda.synchronize()
    return e, g, track.cpu().numpy(), state.cpu().numpy()


def _check(ev, radius=1.5, pt_good=0.05):
    e, g, track, state = _gpu_attach(ev, radius, pt_good)
    o = run_oracle(ev, layout=e.layout)
    assert np.array_equal(g["trk_off"], o["tracks"]["trk_off"])
    ot, os_ = _oracle_attach(ev, o, radius, pt_good)
    assert np.array_equal(track, ot)
    assert np.array_equal(state, os_)
    return g, track, state


@pytest.mark.parametrize("cfg", ["c1", "c2_sector"])
def test_attachment_matches_the_oracle(cfg):
    ev = synth.make_config1() if cfg == "c1" else synth.make_config2().sector(7)
    print(f"case attach {cfg} n={ev.n_clusters}", flush=True)
    _, track, state = _check(ev)
    assert (state & 1).any() and (state & 2).any()
    # every attached cluster is owned by its track, every adjacent one is not
    assert np.all((track >= 0) == ((state & 3) != 0))


@pytest.mark.timeout(600)
def test_attachment_central_event_and_fake_rate():
    """The whole central event, and the paper's figure of merit: the share
    of attached and of adjacent clusters that do not carry the generating
    track of their track (practically none of the attached ones; more of
    the adjacent ones, which a tube may collect from other tracks and
    noise)."""
    ev = synth.make_config2()
    print(f"case attach c2 n={ev.n_clusters}", flush=True)
    g, track, state = _check(ev)
    # majority generating track of every found track
    off, hits = g["trk_off"], g["trk_hits"]
    maj = np.array([np.bincount(np.maximum(ev.label[hits[off[k]:off[k + 1]]], 0)).argmax()
                    for k in range(len(off) - 1)])
    att = (state & 1) != 0
    adj = (state & 2) != 0
    fake_att = np.mean(ev.label[att] != maj[track[att]])
    fake_adj = np.mean(ev.label[adj] != maj[track[adj]])
    print(f"attached {att.sum()} (fake {fake_att:.4f}), adjacent {adj.sum()} "
          f"(fake {fake_adj:.4f})", flush=True)
    assert fake_att < 0.05
    assert fake_adj > fake_att


def test_attachment_parameters_and_empty_event():
    """Another tube radius and pT threshold; and an event without tracks
    (every cluster unmarked)."""
    ev = synth.make_config2().sector(3)
    _check(ev, radius=0.7, pt_good=0.4)
    rng = np.random.default_rng(1)
    n = 500
    row = rng.integers(0, 152, n).astype(np.uint8)
    y = rng.uniform(-20, 20, n).astype(np.float32)
    z = rng.uniform(0, 250, n).astype(np.float32)
    off = np.array([0, n], np.int64)
    rr = np.array([[-25, 25, 0, 250]], np.float32)
    noise = synth.Event(row, y, z, np.zeros(n, np.float32), off, rr, synth.ROW_X,
                        -np.ones(n, np.int32), {}, {})
    e, g, track, state = _gpu_attach(noise)
    assert g["status"]["n_tracks"] == 0
    assert np.all(track == -1) and np.all(state == 0)


@pytest.mark.timeout(600)
def test_attachment_batched_uneven_instances():
    """Many small and large single-sector instances in one problem (the
    tracks of every instance stay in it)."""
    ev = synth.make_config4()
    k = 40
    n = int(ev.sector_offsets[k])
    sub = synth.Event(ev.row[:n], ev.y[:n], ev.z[:n], ev.charge[:n],
                      ev.sector_offsets[:k + 1].copy(), ev.sector_range[:k].copy(), ev.row_x,
                      ev.label[:n], ev.tracks, {}, ev.sector_side[:k].copy())
    print(f"case attach c4 first {k} instances n={n}", flush=True)
    _check(sub)
