"""Sector-track merging on the GPU (tpc_merge_sector_tracks) against the
oracle, track by track: the links to the up and down neighbour sectors and
the chain group of every track, after the tracking chain of the same event
on both sides."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import ctx, run_gpu, run_oracle
from paper_1905_05515_amd import _lib as L
from paper_1905_05515_amd import api

pytestmark = pytest.mark.gpu


def _oracle_merge(ev, o, windows=api.MERGE_WINDOWS, sps=18):
    trk, trl = o["tracks"], o["tracklets"]
    tt = trk["trk_tracklet"]
    return oracle.merge_sector_tracks(ev.sector_offsets, sps, ev.row_x, synth.default_params(),
                                      trk["trk_off"], trk["trk_hits"], trl["par"][tt],
                                      trl["row_inner"][tt],
                                      iw=oracle.merge_windows_inv(windows))


def _check(ev, windows=api.MERGE_WINDOWS, sps=18):
    e, g = run_gpu(ev)
    up, dn, grp = api.merge_sector_tracks(ctx(), e, sps, windows)
    torch.cuda.synchronize()
    nt = len(g["trk_off"]) - 1
    up, dn, grp = (t[:nt].cpu().numpy() for t in (up, dn, grp))
    o = run_oracle(ev, layout=e.layout)
    assert np.array_equal(g["trk_off"], o["tracks"]["trk_off"])
    ou, od, og = _oracle_merge(ev, o, windows, sps)
    assert np.array_equal(up, ou)
    assert np.array_equal(dn, od)
    assert np.array_equal(grp, og)
    return g, up, dn, grp


@pytest.mark.timeout(600)
def test_merging_central_event_matches_the_oracle():
    ev = synth.make_config2()
    print(f"case merge c2 n={ev.n_clusters}", flush=True)
    g, up, dn, grp = _check(ev)
    k = np.nonzero(up >= 0)[0]
    assert len(k) > 5000 and np.all(dn[up[k]] == k)


@pytest.mark.timeout(600)
def test_merging_other_windows_and_a_smaller_event():
    ev = synth.make_config2(seed=77, n_primary=1500)
    print(f"case merge small n={ev.n_clusters}", flush=True)
    _check(ev)
    _check(ev, windows=(1.0, 0.5, 0.03, 0.006, 1.0))
    _check(ev, windows=(30.0, 20.0, 1.0, 0.2, 20.0))


@pytest.mark.timeout(600)
def test_merging_continuous_slice_matches_the_oracle():
    """Three collisions of continuous read-out (several collisions' tracks
    in every sector bucket; the oracle compares every pair)."""
    ev = synth.make_config3(n_collisions=3)
    print(f"case merge c3 3 collisions n={ev.n_clusters}", flush=True)
    _check(ev)
    _check(ev, windows=(3.0, 2.0, 0.1, float("inf"), 2.0))     # no tan(lambda) cut


def _canonical_groups(grp):
    """Group ids renamed to the least member, as a partition of the tracks."""
    first = {}
    for i, gid in enumerate(grp):
        first.setdefault(gid, i)
    return np.array([first[gid] for gid in grp])


@pytest.mark.timeout(600)
def test_merging_does_not_depend_on_track_order():
    """The same tracks handed over in a shuffled order through the C ABI:
    the links are the same tracks' links and the groups the same
    partition (no two candidates of these events are at exactly the same
    distance, so the index tie rule does not come in)."""
    ev = synth.make_config2(seed=77, n_primary=1500)
    print(f"case merge shuffled n={ev.n_clusters}", flush=True)
    e, g = run_gpu(ev)
    nt = len(g["trk_off"]) - 1
    up, dn, grp = (t[:nt].cpu().numpy() for t in api.merge_sector_tracks(ctx(), e))
    perm = np.random.default_rng(4).permutation(nt)         # new track i is old perm[i]
    off, hits, tt = g["trk_off"], g["trk_hits"], g["trk_tracklet"]
    noff = np.concatenate([[0], np.cumsum(np.diff(off)[perm])]).astype(np.int32)
    nhits = np.concatenate([hits[off[p]:off[p + 1]] for p in perm]).astype(np.int32)
    dev = torch.device("cuda", 0)
    d_off = torch.as_tensor(noff, device=dev)
    d_hits = torch.as_tensor(nhits, device=dev)
    d_tt = torch.as_tensor(tt[perm].astype(np.int32), device=dev)
    d_n = torch.tensor([nt], dtype=torch.int64, device=dev)
    tracks = L.Tracks(C.c_void_p(d_off.data_ptr()), C.c_void_p(d_hits.data_ptr()),
                      C.c_void_p(d_tt.data_ptr()), None, nt, len(nhits))
    need = C.c_size_t(0)
    L.check(L.lib().tpc_merge_workspace_size(C.byref(e.problem), nt, C.byref(need)), "size")
    ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=dev)
    out = [torch.empty(max(nt, 1), dtype=torch.int32, device=dev) for _ in range(3)]
    L.check(L.lib().tpc_merge_sector_tracks(
        ctx().handle, C.byref(e.problem), api._tracklets(e), tracks, C.c_void_p(d_n.data_ptr()),
        api.merge_cuts(), *[C.c_void_p(o.data_ptr()) for o in out], C.c_void_p(ws.data_ptr()),
        ws.numel(), C.c_void_p(torch.cuda.current_stream().cuda_stream)), "merge")
    torch.cuda.synchronize()
    up2, dn2, grp2 = (o[:nt].cpu().numpy() for o in out)
    back = lambda a: np.where(a >= 0, perm[np.maximum(a, 0)], -1)
    assert np.array_equal(back(up2), up[perm])
    assert np.array_equal(back(dn2), dn[perm])
    assert (up >= 0).sum() > 100
    # the same partition into groups
    assert np.array_equal(_canonical_groups(grp2), _canonical_groups(grp[perm]))


def test_merging_without_tracks_and_bad_arguments():
    rng = np.random.default_rng(3)
    n = 720
    sec = np.repeat(np.arange(36), 20)
    row = rng.integers(0, 152, n).astype(np.uint8)
    y = rng.uniform(-10, 10, n).astype(np.float32)
    z = np.where(sec < 18, 1, -1) * rng.uniform(1, 240, n).astype(np.float32)
    off = np.arange(37, dtype=np.int64) * 20
    rr = np.array([[-45, 45, 0, 250]] * 18 + [[-45, 45, -250, 0]] * 18, np.float32)
    side = np.array([1] * 18 + [-1] * 18, np.int8)
    noise = synth.Event(row, y, z.astype(np.float32), np.zeros(n, np.float32), off, rr,
                        synth.ROW_X, -np.ones(n, np.int32), {}, {}, side)
    print("case merge noise", flush=True)
    e, g = run_gpu(noise)
    assert g["status"]["n_tracks"] == 0
    up, dn, grp = api.merge_sector_tracks(ctx(), e)
    torch.cuda.synchronize()
    for sps in (2, 5):          # fewer than 3 sectors a side; 36 not a multiple of 5
        with pytest.raises(L.TPCError):
            api.merge_sector_tracks(ctx(), e, sectors_per_side=sps)
