"""Pins of the oracle's full-track fit of merged sector tracks (section 2:
the first fit of the sector tracks finds the whole track, which is then
fitted; section 3: several fit iterations in and out, sector boundaries).

Pinned against helix geometry and statistics, not the oracle's arithmetic:
  * the frame turn: its state equals the closed-form helix in the turned
    frame, and the Jacobian it applies to the covariance (read off by turning
    unit covariances) equals central differences of the exact geometric map
    (state at a plane of one frame -> state at the plane through the same
    point in the turned frame), computed here in numpy from the circle;
  * noiseless helices crossing one or two sector boundaries, members given
    in any order and chains walked up or down: the fit returns the helix
    state at the last hit in that hit's frame and a chi2 near zero;
  * smeared helices: the pulls of the fitted outer state against the truth
    have unit width and no bias, and chi2 / ndf is about 1 (a wrong
    covariance turn or transport would widen or narrow them);
  * bookkeeping: leaders only, member and hit counts, fewer than three hits.
"""
import math

import numpy as np

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


def _centre(p, x, k):
    """Circle centre of the state p at plane x (d(sin phi)/dx = k)."""
    c = math.sqrt(1.0 - p[2] * p[2])
    return x - p[2] / k, p[0] + c / k


def _turned(p, x, k, c, sd, X_to):
    """Exact state, in the frame turned by D (cos c, sin sd), of the helix
    through state p at plane x, at the plane X_to (outgoing branch)."""
    xc, yc = _centre(p, x, k)
    xc2, yc2 = xc * c - yc * sd, xc * sd + yc * c
    phi_pt = math.atan2(p[2], math.sqrt(1 - p[2] ** 2)) + math.atan2(sd, c)
    s2 = k * (X_to - xc2)
    phi2 = math.asin(s2)
    y2 = yc2 - math.cos(phi2) / k
    arc = (phi2 - phi_pt) / k
    return np.array([y2, p[1] + p[3] * arc, s2, p[3], p[4]])


def _lower(M):
    return np.array([M[i, j] for i in range(5) for j in range(i + 1)])


def _full(v):
    M = np.zeros((5, 5))
    k = 0
    for i in range(5):
        for j in range(i + 1):
            M[i, j] = M[j, i] = v[k]
            k += 1
    return M


def test_turn_matches_the_helix_and_its_jacobian():
    rng = np.random.default_rng(21)
    for _ in range(80):
        x = rng.uniform(90.0, 240.0)
        p = np.array([rng.uniform(-20, 20), rng.uniform(-100, 100), rng.uniform(-0.6, 0.6),
                      rng.uniform(-1, 1), rng.choice([-1, 1]) / rng.uniform(0.3, 5.0)])
        k = CURV * p[4]
        # an exact rotation (the float32 cos and sin of the width are off
        # the unit circle by ~1e-8, which the closed form would see)
        sd = math.sin(W) * float(rng.choice([1.0, -1.0]))
        c = math.cos(W)
        ok, x2, p2, _ = oracle.rotate(x, p, _lower(np.eye(5)), c, sd, CURV)
        assert ok
        assert abs(x2 - (x * c - p[0] * sd)) < 1e-12
        np.testing.assert_allclose(p2, _turned(p, x, k, c, sd, x2), rtol=0, atol=1e-9)
        J = np.zeros((5, 5))
        for j in range(5):
            h = 1e-6 * max(1.0, abs(p[j]))
            e = np.zeros(5)
            e[j] = h
            J[:, j] = (_turned(p + e, x, CURV * (p + e)[4], c, sd, x2) -
                       _turned(p - e, x, CURV * (p - e)[4], c, sd, x2)) / (2 * h)
        F = np.zeros((5, 5))
        for j in range(5):
            E = np.zeros((5, 5))
            E[j, j] = 1.0
            _, _, _, C2 = oracle.rotate(x, p, _lower(E), c, sd, CURV)
            # C' = J e_j e_j^T J^T: column j is J[:, j] J[j, j], and J[j, j] > 0
            col = _full(C2)[:, j]
            F[:, j] = col / math.sqrt(col[j])
        assert np.all(np.abs(F - J) <= 1e-6 * (1.0 + np.abs(J))), np.abs(F - J).max()


def test_turn_refuses_a_direction_past_the_frame():
    p = np.array([0.0, 0.0, 0.9, 0.0, 0.0])
    ok, x2, p2, _ = oracle.rotate(150.0, p, _lower(np.eye(5)), float(COS_W), float(SIN_W), CURV)
    assert not ok and x2 == 150.0 and np.array_equal(p2, p)


def _helix_hits(phi0, qpt, tanl, sectors, rows_per_sector, smear=0.0, rng=None):
    """Clusters of one helix from the origin in the given sectors (side A),
    rows_per_sector[i] rows each; returns per member (sector, rows, y, z) and
    the truth state at every hit."""
    members = []
    for i, rows in zip(sectors, rows_per_sector):
        ys, zs, truth = [], [], []
        for r in rows:
            st = _state(phi0, qpt, tanl, _alpha(i), X[r])
            truth.append(st)
            dy = rng.normal(0, smear) if smear else 0.0
            dz = rng.normal(0, smear) if smear else 0.0
            ys.append(st[0] + dy)
            zs.append(st[1] + dz)
        members.append((i, np.array(rows), np.array(ys), np.array(zs), truth))
    return members


def _state(phi0, qpt, tanl, alpha, x):
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


def _event(tracks, n_sec=36, order=None):
    """tracks: list of member lists (as _helix_hits returns).  Builds the
    clusters (ids per sector block), the track CSR (one track per member,
    in `order`), the links along each chain and the groups; the prior of
    each member is its truth state at its first hit."""
    per_sec = [[] for _ in range(n_sec)]
    mem = []
    for t, members in enumerate(tracks):
        for m, (i, rows, ys, zs, truth) in enumerate(members):
            ids = []
            for r, yy, zz in zip(rows, ys, zs):
                ids.append((i, len(per_sec[i])))
                per_sec[i].append((r, yy, zz))
            mem.append((t, m, ids, rows[0], truth[0]))
    offs = np.zeros(n_sec + 1, np.int64)
    for s in range(n_sec):
        offs[s + 1] = offs[s] + len(per_sec[s])
    row = np.zeros(offs[-1], np.uint8)
    y = np.zeros(offs[-1], np.float32)
    z = np.zeros(offs[-1], np.float32)
    for s in range(n_sec):
        for j, (r, yy, zz) in enumerate(per_sec[s]):
            row[offs[s] + j], y[offs[s] + j], z[offs[s] + j] = r, yy, zz
    order = list(range(len(mem))) if order is None else order
    mem = [mem[o] for o in order]
    off = [0]
    hits = []
    for (_, _, ids, _, _) in mem:
        hits += [int(offs[i] + j) for i, j in ids]
        off.append(len(hits))
    par = np.array([m[4] for m in mem], np.float32)
    rin = np.array([m[3] for m in mem], np.int32)
    n = len(mem)
    up = -np.ones(n, np.int32)
    dn = -np.ones(n, np.int32)
    key = {(m[0], m[1]): k for k, m in enumerate(mem)}
    sec = {k: tracks[m[0]][m[1]][0] for k, m in enumerate(mem)}
    for k, m in enumerate(mem):
        nxt = key.get((m[0], m[1] + 1))
        if nxt is not None:
            if sec[nxt] == (sec[k] % 18 + 1) % 18 + 18 * (sec[k] // 18):
                up[k], dn[nxt] = nxt, k
            else:
                dn[k], up[nxt] = nxt, k
    grp = np.arange(n, dtype=np.int32)
    for k in range(n):
        same = [j for j in range(n) if mem[j][0] == mem[k][0]]
        grp[k] = min(same)
    return dict(offs=offs, row=row, y=y, z=z, off=np.array(off, np.int32),
                hits=np.array(hits, np.int32), par=par, rin=rin, up=up, dn=dn, grp=grp, mem=mem)


TOL = np.array([2e-4, 2e-4, 2e-6, 2e-6, 2e-5])


def _close(a, b, tol=TOL):
    d = np.abs(np.asarray(a) - np.asarray(b))
    assert np.all(d <= tol), (a, b, d)


# tracklet covariance of every member: a diagonal of the size a fitted
# tracklet has (the fit restarts from these variances times cov_scale)
COV0 = np.array([0.01 if i in (0, 2) else 1e-4 if i in (5, 9) else 1e-2 if i == 14 else 0.0
                 for i in range(15)], np.float32)


def _fit(ev, n_pass=3, fp64=True):
    cov = np.tile(COV0, (len(ev["par"]), 1))
    return oracle.fit_merged(ev["offs"], 18, synth.ROW_X, PRM, ev["row"], ev["y"], ev["z"],
                             ev["off"], ev["hits"], ev["par"], cov, ev["rin"], ev["up"],
                             ev["dn"], ev["grp"], n_pass=n_pass, fp64=fp64)


def test_noiseless_helices_across_boundaries():
    # up-going (phi0 grows into sector i+1), down-going (into i-1), and one
    # over three sectors; members listed in scrambled order
    cases = [
        (dict(phi0=4 * W - 0.05, qpt=-1 / 1.2, tanl=0.3), [3, 4],
         [range(0, 50), range(60, 151)]),
        (dict(phi0=5 * W + 0.05, qpt=1 / 1.1, tanl=-0.5), [5, 4],
         [range(2, 40), range(45, 140)]),
        (dict(phi0=7 * W - 0.02, qpt=-1 / 0.6, tanl=0.1), [6, 7, 8],
         [range(0, 25), range(30, 100), range(105, 150)]),
    ]
    tracks, truth_last = [], []
    for h, secs, rows in cases:
        m = _helix_hits(h["phi0"], h["qpt"], h["tanl"], secs, [list(r) for r in rows])
        tracks.append(m)
        truth_last.append(m[-1][4][-1])
    order = [6, 2, 0, 4, 1, 5, 3]
    ev = _event(tracks, order=order)
    f = _fit(ev)
    leaders = np.nonzero(ev["grp"] == np.arange(len(order)))[0]
    assert len(leaders) == 3
    assert np.all(f["status"][~np.isin(np.arange(len(order)), leaders)] == -1)
    for L in leaders:
        t = ev["mem"][L][0]
        assert f["status"][L] == 0
        assert f["n_members"][L] == len(cases[t][1])
        assert f["n_hits"][L] == sum(len(r) for r in cases[t][2])
        _close(f["par_out"][L], truth_last[t])
        assert f["chi2"][L] < 1e-3
        # the inward pass ends at the first hit, in its frame
        _close(f["par_in"][L], tracks[t][0][4][0])


def test_pulls_of_smeared_helices():
    rng = np.random.default_rng(5)
    tracks, truth = [], []
    sigma = math.sqrt(PRM["sigma_y2"])
    while len(tracks) < 300:
        i = int(rng.integers(0, 17))
        qpt = rng.choice([-1, 1]) / rng.uniform(0.5, 3.0)
        phi0 = (i + 1) * W + rng.uniform(-0.15, 0.05) * np.sign(-qpt)
        tanl = rng.uniform(-0.8, 0.8)
        # the row where the helix crosses into the next sector
        rows_a, rows_b = [], []
        for r in range(152):
            try:
                _state(phi0, qpt, tanl, _alpha(i), X[r])
                sa = True
            except AssertionError:
                sa = False
            if sa:
                st = _state(phi0, qpt, tanl, _alpha(i), X[r])
                inside = abs(st[0]) <= X[r] * math.tan(W / 2)
            else:
                inside = False
            j = i + 1 if qpt < 0 else i - 1
            if inside:
                rows_a.append(r)
            else:
                try:
                    st = _state(phi0, qpt, tanl, _alpha(j % 18), X[r])
                    if abs(st[0]) <= X[r] * math.tan(W / 2) and abs(st[2]) < 0.8:
                        rows_b.append(r)
                except AssertionError:
                    pass
        if len(rows_a) < 10 or len(rows_b) < 10 or (rows_b and rows_a and rows_b[0] < rows_a[-1]):
            continue
        m = _helix_hits(phi0, qpt, tanl, [i, j % 18], [rows_a, rows_b], smear=sigma, rng=rng)
        tracks.append(m)
        truth.append(m[-1][4][-1])
    ev = _event(tracks)
    f = _fit(ev)
    L = np.nonzero(ev["grp"] == np.arange(len(ev["grp"])))[0]
    assert np.all(f["status"][L] == 0)
    tr = np.array([truth[ev["mem"][k][0]] for k in L])
    d = f["par_out"][L] - tr
    sig = np.sqrt(f["cov_out"][L][:, [0, 2, 5, 9, 14]])
    pull = d / sig
    assert np.all(np.abs(pull.mean(0)) < 0.2), pull.mean(0)
    assert np.all(np.abs(pull.std(0) - 1.0) < 0.15), pull.std(0)
    ndf = 2 * f["n_hits"][L] - 5
    assert abs(f["chi2"][L].sum() / ndf.sum() - 1.0) < 0.05


def test_short_and_single_member_tracks():
    h = dict(phi0=2 * W + 0.05, qpt=1 / 2.0, tanl=0.2)
    a = _helix_hits(h["phi0"], h["qpt"], h["tanl"], [2], [[10, 11]])
    b = _helix_hits(h["phi0"], h["qpt"], h["tanl"], [2], [list(range(20, 60))])
    ev = _event([a, b])
    f = _fit(ev)
    assert f["status"][0] == 1 and f["n_hits"][0] == 2
    assert f["status"][1] == 0 and f["n_members"][1] == 1
    _close(f["par_out"][1], b[0][4][-1])
