"""Per-track interaction time on the GPU (tpc_track_t0) against the oracle,
track by track and bit for bit (z0, y0, t0, ok), after the tracking chain of
the same event on both sides: the central event (both z sides) and a
continuous read-out slice of three collisions."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import ctx, run_gpu, run_oracle, same_floats
from paper_1905_05515_amd import _lib as L
from paper_1905_05515_amd import api
from synth.events import VD_CM_PER_US

pytestmark = pytest.mark.gpu


def _check(ev):
    e, g = run_gpu(ev)
    z0, y0, t0, ok = api.track_t0(ctx(), e, VD_CM_PER_US)
    torch.cuda.synchronize()
    nt = len(g["trk_off"]) - 1
    z0, y0, t0, ok = (t[:nt].cpu().numpy() for t in (z0, y0, t0, ok))
    o = run_oracle(ev, layout=e.layout)
    assert np.array_equal(g["trk_off"], o["tracks"]["trk_off"])
    trk, trl = o["tracks"], o["tracklets"]
    tt = trk["trk_tracklet"]
    off, hits = trk["trk_off"], trk["trk_hits"]
    sec = np.searchsorted(ev.sector_offsets, hits[off[:-1]], side="right") - 1
    oz, oy, ot, ook = oracle.track_t0(trl["par"][tt], ev.row_x[trl["row_inner"][tt]],
                                      ev.sector_side[sec], synth.default_params(),
                                      vd=VD_CM_PER_US)
    assert np.array_equal(ok, ook)
    assert same_floats(z0, oz) and same_floats(y0, oy) and same_floats(t0, ot)
    return e, t0, ok


@pytest.mark.timeout(600)
def test_t0_central_event_matches_the_oracle():
    ev = synth.make_config2()
    print(f"case t0 c2 n={ev.n_clusters}", flush=True)
    _, t0, ok = _check(ev)
    # one collision at t = 0: the estimates of the found tracks centre on it
    assert ok.mean() > 0.8 and abs(np.median(t0[ok == 1])) < 0.05


@pytest.mark.timeout(600)
def test_t0_continuous_slice_matches_the_oracle():
    ev = synth.make_config3(n_collisions=3)
    print(f"case t0 c3 3 collisions n={ev.n_clusters}", flush=True)
    _check(ev)


def test_t0_bad_velocity():
    ev = synth.make_config1()
    print("case t0 bad vd", flush=True)
    e, _ = run_gpu(ev)
    for vd in (0.0, -1.0, float("nan")):
        with pytest.raises(L.TPCError):
            api.track_t0(ctx(), e, vd)
