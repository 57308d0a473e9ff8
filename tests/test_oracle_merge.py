"""Pins of the oracle's sector-track merging (section 2: the first fit of the
sector tracks serves to find the whole track; section 3: sector boundaries).

Pinned against helix geometry, not against the oracle's own arithmetic: the
state of a helix from the origin at any sector-local plane is known in
closed form (float64 here), so the state of one segment taken into the
neighbour sector's frame and moved to the other segment's plane must equal
the closed-form state there, in both directions of rotation; segments of one
helix in neighbouring sectors must link and those of others must not; the
mutual-best rule, the tie rule, the wrap of a side's last sector to its
first, the separation of the two sides, chains over three sectors and the
invariance under a cyclic relabelling of the sectors are fixed by hand-built
cases; on the seeded central event the links must join the segments of one
generating particle."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth.events import CURV_PER_QPT64

W = math.radians(20.0)
CURV = float(CURV_PER_QPT64)
X = synth.ROW_X.astype(np.float64)
PRM = synth.default_params()
COS_W, SIN_W = oracle.sector_width_cs(20.0)


def _alpha(i):
    return (i + 0.5) * W


def _state(phi0, qpt, tanl, alpha, x):
    """Closed-form state (y, z, sin(phi), tan(lambda), q/pT) of the helix from
    the origin (direction phi0, dip tanl) at the plane x of the frame rotated
    by alpha, on its outgoing branch."""
    k = CURV * qpt
    xc, yc = -math.sin(phi0) / k, math.cos(phi0) / k
    xcl = xc * math.cos(alpha) + yc * math.sin(alpha)
    ycl = -xc * math.sin(alpha) + yc * math.cos(alpha)
    s = k * (x - xcl)
    assert abs(s) < 0.9
    phi = math.asin(s)
    y = ycl - math.cos(phi) / k
    phi0l = math.remainder(phi0 - alpha, 2 * math.pi)
    arc = (phi - phi0l) / k
    assert arc > 0
    return np.array([y, tanl * arc, s, tanl, qpt])


def test_transform_matches_the_helix_in_both_directions():
    rng = np.random.default_rng(11)
    for _ in range(200):
        i = int(rng.integers(0, 18))
        phi0 = (i + 1) * W + rng.uniform(-0.06, 0.06)      # near the boundary i | i+1
        qpt = rng.choice([-1, 1]) / rng.uniform(0.8, 5.0)
        tanl = rng.uniform(-1.0, 1.0)
        ra, rb = int(rng.integers(0, 40)), int(rng.integers(60, 152))
        a = _state(phi0, qpt, tanl, _alpha(i), X[ra])
        b = _state(phi0, qpt, tanl, _alpha(i + 1), X[rb])
        # b (up neighbour) into a's frame: D = alpha_b - alpha_a = +w
        q = oracle.merge_transform(b.astype(np.float32), synth.ROW_X[rb], COS_W, SIN_W,
                                   synth.ROW_X[ra], PRM["curv"])
        assert q is not None
        np.testing.assert_allclose(q[:2], a[:2], atol=2e-3)
        np.testing.assert_allclose(q[2], a[2], atol=2e-5)
        assert q[3] == np.float32(tanl) and q[4] == np.float32(qpt)
        # a (down neighbour) into b's frame: D = -w
        q = oracle.merge_transform(a.astype(np.float32), synth.ROW_X[ra], COS_W, -SIN_W,
                                   synth.ROW_X[rb], PRM["curv"])
        assert q is not None
        np.testing.assert_allclose(q[:2], b[:2], atol=2e-3)
        np.testing.assert_allclose(q[2], b[2], atol=2e-5)


def test_transform_rejects_states_turned_past_the_frame():
    # a state at sin(phi) = 0.9 turned by another 20 degrees leaves |sin| < s_max
    p = np.array([0.0, 0.0, 0.9, 0.0, 0.0], np.float32)
    assert oracle.merge_transform(p, 150.0, COS_W, SIN_W, 100.0, PRM["curv"]) is None
    # a straight track is moved along its line
    p = np.array([1.0, 2.0, 0.1, 0.5, 0.0], np.float32)
    q = oracle.merge_transform(p, 150.0, np.float32(1.0), np.float32(0.0), 110.0, PRM["curv"])
    c = math.sqrt(1 - 0.01)
    np.testing.assert_allclose(q[:2], [1.0 - 40 * 0.1 / c, 2.0 - 40 * 0.5 / c], atol=1e-4)


def _merge(tracks, sps=18, n_sec=36, **kw):
    """tracks: list of (sector, row of the state, state) -> oracle links.
    Each track has one hit, whose id lies in its sector."""
    n = len(tracks)
    offs = np.arange(n_sec + 1, dtype=np.int64) * 1000
    hits = np.array([s * 1000 + k for k, (s, _, _) in enumerate(tracks)], np.int32)
    off = np.arange(n + 1, dtype=np.int32)
    par = np.array([p for _, _, p in tracks], np.float32).reshape(-1, 5)
    rin = np.array([r for _, r, _ in tracks], np.int32)
    return oracle.merge_sector_tracks(offs, sps, synth.ROW_X, PRM, off, hits, par, rin, **kw)


def _seg(phi0, qpt, tanl, i, r, sector=None):
    return (i if sector is None else sector, r, _state(phi0, qpt, tanl, _alpha(i % 18), X[r]))


def test_segments_of_one_helix_link_and_others_do_not():
    h = dict(phi0=4 * W + 0.02, qpt=1.0 / 1.5, tanl=0.3)
    g = dict(phi0=4 * W - 0.03, qpt=-1.0 / 0.9, tanl=-0.4)
    tracks = [_seg(i=3, r=5, **h), _seg(i=3, r=12, **g), _seg(i=4, r=90, **h),
              _seg(i=4, r=70, **g), _seg(i=5, r=80, phi0=6 * W, qpt=0.5, tanl=0.1)]
    up, dn, grp = _merge(tracks)
    assert list(up) == [2, 3, -1, -1, -1]
    assert list(dn) == [-1, -1, 0, 1, -1]
    assert list(grp) == [0, 1, 0, 1, 4]


def test_window_edges():
    h = dict(phi0=4 * W + 0.02, qpt=1.0 / 1.5, tanl=0.3)
    a, b = _seg(i=3, r=5, **h), _seg(i=4, r=90, **h)
    for shift, linked in ((1.0, True), (4.0, False)):
        pb = b[2].copy()
        pb[0] += shift                       # y of the outer segment, its own frame
        up, _, _ = _merge([a, (b[0], b[1], pb)])
        assert (up[0] == 1) == linked
    # tan(lambda) off by twice its window
    pb = b[2].copy()
    pb[3] += 0.04
    up, _, _ = _merge([a, (b[0], b[1], pb)])
    assert up[0] == -1


def test_mutual_best_and_ties():
    h = dict(phi0=4 * W + 0.02, qpt=1.0 / 1.5, tanl=0.3)
    a, b = _seg(i=3, r=5, **h), _seg(i=4, r=90, **h)
    a_off = (a[0], a[1], a[2] + np.array([1.0, 0, 0, 0, 0]))
    # a' (index 0) wants b, but b prefers the exact a (index 1): only a-b
    up, dn, grp = _merge([a_off, a, b])
    assert list(up) == [-1, 2, -1] and list(dn) == [-1, -1, 1]
    assert list(grp) == [0, 1, 1]
    # an exact duplicate: equal distances go to the lower index
    up, dn, _ = _merge([b, a, a])
    assert list(dn) == [1, -1, -1] and list(up) == [-1, 0, -1]


def test_wrap_of_a_side_and_separation_of_sides():
    h = dict(phi0=18 * W + 0.01, qpt=1.0 / 2.0, tanl=0.2)
    a = _seg(i=17, r=8, **h)
    b = _seg(i=18, r=100, **h)          # index 0 of side A, frame angle 18.5 w = 0.5 w
    up, dn, _ = _merge([a, (0, b[1], b[2])])
    assert list(up) == [1, -1] and list(dn) == [-1, 0]
    # the same states with the outer segment on the other side: no link
    up, dn, _ = _merge([a, (18, b[1], b[2])])
    assert list(up) == [-1, -1] and list(dn) == [-1, -1]
    # both on side C (sectors 35 and 18)
    up, dn, _ = _merge([(35, a[1], a[2]), (18, b[1], b[2])])
    assert list(up) == [1, -1] and list(dn) == [-1, 0]


def test_chain_over_three_sectors():
    # a helix of 0.25 GeV/c bends through sectors 8, 9 and 10
    qpt, tanl, phi0 = -4.0, 0.5, 8 * W
    segs = [_seg(phi0=phi0, qpt=qpt, tanl=tanl, i=i, r=r) for i, r in ((8, 0), (9, 30), (10, 122))]
    # the helix lies inside each sector at those planes
    for i, r, p in segs:
        assert abs(p[0]) < X[r] * math.tan(W / 2), (i, p[0])
    up, dn, grp = _merge([segs[2], segs[0], segs[1]])
    assert list(up) == [-1, 2, 0] and list(dn) == [2, -1, 1]
    assert list(grp) == [0, 0, 0]


def test_empty_and_hitless_tracks_and_arguments():
    up, dn, grp = _merge([])
    assert len(up) == len(dn) == len(grp) == 0
    offs = np.arange(37, dtype=np.int64) * 10
    off = np.array([0, 0, 1], np.int32)     # track 0 has no hits
    par = np.zeros((2, 5), np.float32)
    up, dn, grp = oracle.merge_sector_tracks(offs, 18, synth.ROW_X, PRM, off,
                                             np.array([5], np.int32), par,
                                             np.zeros(2, np.int32))
    assert list(up) == [-1, -1] and list(grp) == [0, 1]
    with pytest.raises(ValueError):
        oracle.merge_sector_tracks(offs, 2, synth.ROW_X, PRM, off, np.array([5], np.int32), par,
                                   np.zeros(2, np.int32))
    with pytest.raises(ValueError):
        oracle.merge_sector_tracks(offs, 5, synth.ROW_X, PRM, off, np.array([5], np.int32), par,
                                   np.zeros(2, np.int32))


@pytest.fixture(scope="module")
def central():
    from paper_1905_05515_amd.layout import grid_layout
    ev = synth.make_config2()
    tab, nb = grid_layout(ev.sector_offsets, ev.sector_range, occupancy=0.25,
                          sides=ev.sector_side)
    o = oracle.track_event(ev.row, ev.y, ev.z, tab, nb, ev.row_x, PRM)
    return ev, o


def _inputs(ev, o):
    trk, trl = o["tracks"], o["tracklets"]
    tt = trk["trk_tracklet"]
    return trk["trk_off"], trk["trk_hits"], trl["par"][tt], trl["row_inner"][tt]


def test_central_event_links_join_one_particle(central):
    ev, o = central
    off, hits, par, rin = _inputs(ev, o)
    up, dn, grp = oracle.merge_sector_tracks(ev.sector_offsets, 18, ev.row_x, PRM, off, hits,
                                             par, rin)
    k = np.nonzero(up >= 0)[0]
    assert np.all(dn[up[k]] == k) and np.sum(dn >= 0) == len(k)
    maj = np.array([np.bincount(np.maximum(ev.label[hits[off[t]:off[t + 1]]], 0)).argmax()
                    for t in range(len(off) - 1)])
    assert len(k) > 5000
    assert np.mean(maj[k] == maj[up[k]]) > 0.995
    # groups: the least index of every chain, shared along it
    assert np.all(grp <= np.arange(len(grp)))
    assert np.all(grp[k] == grp[up[k]])
    # a particle whose segments both became tracks in neighbouring sectors is
    # linked in most cases
    sec = np.searchsorted(ev.sector_offsets, hits[off[:-1]], side="right") - 1
    nxt = (sec // 18) * 18 + (sec % 18 + 1) % 18
    by = {}
    for t, m in enumerate(maj):
        if m > 0:
            by.setdefault((m, sec[t]), []).append(t)
    pairs = found = 0
    for t, m in enumerate(maj):
        for u in by.get((m, nxt[t]), []) if m > 0 else []:
            pairs += 1
            found += up[t] == u
    assert pairs > 6000 and found / pairs > 0.75


def test_cyclic_relabelling_of_sectors(central):
    """Local states do not depend on the sector's angle: turning every
    sector index by three within its side (hit ids moved with it) leaves the
    links unchanged."""
    ev, o = central
    off, hits, par, rin = _inputs(ev, o)
    up, dn, grp = oracle.merge_sector_tracks(ev.sector_offsets, 18, ev.row_x, PRM, off, hits,
                                             par, rin)
    offs = np.asarray(ev.sector_offsets, np.int64)
    sec = np.searchsorted(offs, hits, side="right") - 1
    new_sec = (sec // 18) * 18 + (sec % 18 + 3) % 18
    big = int(np.max(np.diff(offs))) + 1
    moved = (new_sec * big + (hits - offs[sec])).astype(np.int32)
    offs2 = np.arange(37, dtype=np.int64) * big
    up2, dn2, grp2 = oracle.merge_sector_tracks(offs2, 18, ev.row_x, PRM, off, moved, par, rin)
    assert np.array_equal(up, up2) and np.array_equal(dn, dn2) and np.array_equal(grp, grp2)
