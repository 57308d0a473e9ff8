"""Full-track fit of merged sector tracks on the GPU (tpc_fit_merged_tracks)
against the oracle, track by track, after the tracking and merging chains of
the same event on both sides (the oracle's inputs are its own tracking and
merging results):
  * bit for bit against the float32 oracle (the same expressions in the same
    order): statuses, hit and member counts, both states, the covariance and
    the chi2;
  * against the float64 oracle: every state within 2% of the float64 fit's
    own standard deviation of each parameter, at least 99% of them within
    relative 1e-4 (floors 1 cm, 1 cm, 0.01, 0.01, 0.1 c/GeV), chi2 within
    relative 1e-3.  The float32 filter's rounding reaches a relative 1e-3 on
    q/pT of short tracks whose q/pT is loosely measured: 0.3% to 0.7% of the
    tracks of the 1500-primary events of seeds 77 to 80 (with the products
    summed by fused multiply-adds or not alike), all below 0.01 sigma."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import ctx, run_gpu, run_oracle, same_floats
from paper_1905_05515_amd import _lib as L
from paper_1905_05515_amd import api

pytestmark = pytest.mark.gpu
FLOOR = np.array([1.0, 1.0, 0.01, 0.01, 0.1])


def _check(ev, n_pass=3):
    e, g = run_gpu(ev)
    links = api.merge_sector_tracks(ctx(), e, 18)
    f = api.fit_merged_tracks(ctx(), e, links, 18, n_pass=n_pass)
    torch.cuda.synchronize()
    nt = len(g["trk_off"]) - 1
    f = {k: v[:nt].cpu().numpy() for k, v in f.items()}
    o = run_oracle(ev, layout=e.layout)
    trk, trl = o["tracks"], o["tracklets"]
    tt = trk["trk_tracklet"]
    prm = synth.default_params()
    up, dn, grp = oracle.merge_sector_tracks(ev.sector_offsets, 18, ev.row_x, prm, trk["trk_off"],
                                             trk["trk_hits"], trl["par"][tt],
                                             trl["row_inner"][tt])
    args = (ev.sector_offsets, 18, ev.row_x, prm, ev.row, ev.y, ev.z, trk["trk_off"],
            trk["trk_hits"], trl["par"][tt], trl["cov"][tt], trl["row_inner"][tt], up, dn, grp)
    r32 = oracle.fit_merged(*args, n_pass=n_pass, fp64=False)
    for k in ("status", "n_hits", "n_members"):
        assert np.array_equal(f[k], r32[k]), k
    for k in ("par_in", "par_out", "cov_out", "chi2"):
        assert same_floats(f[k], r32[k]), k
    r = oracle.fit_merged(*args, n_pass=n_pass)
    assert np.array_equal(f["status"], r["status"])
    ok = r["status"] == 0
    sig = np.sqrt(r["cov_out"][ok][:, [0, 2, 5, 9, 14]])
    keys = ("par_out", "par_in") if n_pass > 1 else ("par_out",)
    for key in keys:
        a = f[key][ok].astype(np.float64)
        b = r[key][ok]
        assert np.all(np.abs(a - b) <= 0.02 * sig), (key, (np.abs(a - b) / sig).max())
        err = (np.abs(a - b) / np.maximum(np.abs(b), FLOOR)).max(1)
        assert np.mean(err > 1e-4) <= 0.01, (key, err.max(), np.mean(err > 1e-4))
    c32, c64 = f["chi2"][ok].astype(np.float64), r["chi2"][ok]
    assert np.all(np.abs(c32 - c64) <= 1e-3 * np.abs(c64)), (np.abs(c32 - c64) / c64).max()
    return f, r


@pytest.mark.timeout(600)
def test_fullfit_central_event_matches_the_oracle():
    ev = synth.make_config2()
    print(f"case fullfit c2 n={ev.n_clusters}", flush=True)
    f, r = _check(ev)
    ok = r["status"] == 0
    multi = ok & (r["n_members"] > 1)
    assert multi.sum() > 1000
    # per-track chi2 / ndf (the median: a few tracks carry a wrong hit)
    ndf = 2 * r["n_hits"][ok] - 5
    assert 0.85 < np.median(r["chi2"][ok] / ndf) < 1.15


@pytest.mark.timeout(600)
def test_fullfit_one_pass_and_a_continuous_slice():
    ev = synth.make_config2(seed=77, n_primary=1500)
    print(f"case fullfit small one pass n={ev.n_clusters}", flush=True)
    _check(ev, n_pass=1)
    _check(ev, n_pass=4)
    ev = synth.make_config3(n_collisions=3)
    print(f"case fullfit c3 3 collisions n={ev.n_clusters}", flush=True)
    _check(ev)


def test_fullfit_bad_arguments():
    ev = synth.make_config1()
    print("case fullfit bad arguments", flush=True)
    e, _ = run_gpu(ev)
    up = torch.full((max(e.track_capacity, 1),), -1, dtype=torch.int32, device="cuda")
    grp = torch.arange(max(e.track_capacity, 1), dtype=torch.int32, device="cuda")
    # a pass count outside [1, 64]; fewer than three sectors per side, or a
    # count that does not divide the sectors
    for sps, n_pass in ((1, 0), (1, 65), (1, 3), (3, 3)):
        with pytest.raises(L.TPCError):
            api.fit_merged_tracks(ctx(), e, (up, up, grp), sps, n_pass=n_pass)
