"""Pins of the tracklet construction's rules (section 3: Kalman-filter track
following after the cellular-automaton seeding; the rules are this project's
readings, the paper states none).

Every case is a hand-built track in the y = 0 plane of one sector, z = t x:
there sin(phi) stays exactly 0 and the z, tan(lambda) block of the filter is
a linear Gaussian model, so its prediction, its posterior and the sum of its
update chi2 have closed forms (regularised least squares with the filter's
prior, solved here in float64 numpy, no oracle code).  The cases pin:
  * the miss limit: a gap of max_miss - 1 empty rows is bridged, a gap of
    max_miss rows ends the pass (outwards and, below the start, inwards);
  * the chi2 gate: a lone candidate at predicted chi2 16 - eps is taken, one
    at 16 + eps is not;
  * ties: two candidates of bit-identical predicted chi2 resolve to the lower
    cluster id whichever of them the search meets first;
  * the inward pass: its state, covariance and chi2 sum equal the least-
    squares fit whose prior is the outermost hit and the outward pass's
    direction with the initial covariance (a pass that kept the outward
    covariance, or another prior, is off by orders of magnitude);
  * the stop on |sin(phi)|: an update that pushes the state past s_max ends
    the tracklet without a NaN.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_1905_05515_amd.layout import grid_layout

X = synth.ROW_X                     # float32 row planes
X64 = X.astype(np.float64)
PRM = synth.default_params()
SIG2 = float(np.float32(PRM["sigma_z2"]))
CTT = float(np.float32(PRM["c_tt0"]))


def _event(rows, z, extra=(), y=None):
    """Clusters at (row, y, z) for the track, then the extra clusters
    (row, y, z, id) placed at the given ids (the track fills the others)."""
    n = len(rows) + len(extra)
    row = np.zeros(n, np.uint8)
    yy = np.zeros(n, np.float32)
    zz = np.zeros(n, np.float32)
    taken = {e[3] for e in extra}
    free = [i for i in range(n) if i not in taken]
    ids = {}
    for k, r in enumerate(rows):
        i = free[k]
        row[i], zz[i] = r, z[k]
        if y is not None:
            yy[i] = y[k]
        ids[r] = i
    for (r, ey, ez, i) in extra:
        row[i], yy[i], zz[i] = r, ey, ez
    return row, yy, zz, ids


def _track(row, y, z, prm=PRM, occupancy=0.5):
    off = np.array([0, row.shape[0]], np.int64)
    rng_ = np.array([[-30.0, 30.0, 0.0, 250.0]], np.float32)
    tab, nb = grid_layout(off, rng_, occupancy=occupancy)
    res = oracle.track_event(row, y, z, tab, nb, X, prm)
    return res, tab


def _tracklet_of(res, start_id):
    t = int(np.nonzero(res["starts"] == start_id)[0][0])
    trl = res["tracklets"]
    return {k: trl[k][t] for k in ("hits", "nhits", "row_inner", "par", "cov", "chi2")}


def _lsq(x_ref, z_prior, t_prior, xs, zs):
    """Least squares of z = z_ref + t (x - x_ref) with the Gaussian prior
    z_ref ~ N(z_prior, sigma^2), t ~ N(t_prior, c_tt0): posterior mean,
    covariance and minimum of the objective (float64)."""
    H = np.stack([np.ones(len(xs)), np.asarray(xs, np.float64) - x_ref], 1)
    P0 = np.diag([1.0 / SIG2, 1.0 / CTT])
    A = P0 + H.T @ H / SIG2
    b = P0 @ np.array([z_prior, t_prior]) + H.T @ np.asarray(zs, np.float64) / SIG2
    mu = np.linalg.solve(A, b)
    cov = np.linalg.inv(A)
    r = np.asarray(zs, np.float64) - H @ mu
    d = mu - np.array([z_prior, t_prior])
    jmin = d @ P0 @ d + r @ r / SIG2
    return mu, cov, jmin


def _moved(mu, cov, dx):
    """The (z, t) posterior carried to a plane dx further (z += t dx)."""
    A = np.array([[1.0, dx], [0.0, 1.0]])
    return A @ mu, A @ cov @ A.T


def _outward_prediction(ids, z, rows, r0, r_last_fit, r_pred):
    """Prediction at row r_pred of the outward pass that started at chain
    start row r0 and updated every hit of rows r0+1 .. r_last_fit."""
    zr = {r: float(z[ids[r]]) for r in rows}
    t0 = (zr[r0 + 2] - zr[r0]) / (X64[r0 + 2] - X64[r0])
    fit_rows = [r for r in rows if r0 < r <= r_last_fit]
    mu, cov, _ = _lsq(X64[r0], zr[r0], t0, X64[fit_rows], [zr[r] for r in fit_rows])
    return _moved(mu, cov, X64[r_pred] - X64[r0])


TANL = 0.3


def _line_z(rows, tanl=TANL):
    return (tanl * X64[list(rows)]).astype(np.float32)


# ---------------------------------------------------------------- miss limit

@pytest.mark.parametrize("gap", [PRM["max_miss"] - 1, PRM["max_miss"]])
def test_outward_gap_of_max_miss_rows_ends_the_pass(gap):
    lo = list(range(2, 31))
    hi = list(range(31 + gap, 61))
    rows = lo + hi
    row, y, z, ids = _event(rows, _line_z(rows))
    res, _ = _track(row, y, z)
    # the chain of the first segment starts on its second row (its first row
    # has no pair below it)
    tr = _tracklet_of(res, ids[3])
    bridged = gap < PRM["max_miss"]
    for r in hi:
        assert (tr["hits"][r] == ids[r]) == bridged, r
    for r in lo:
        assert tr["hits"][r] == ids[r]


@pytest.mark.parametrize("gap", [PRM["max_miss"] - 1, PRM["max_miss"]])
def test_inward_gap_of_max_miss_rows_ends_the_pass(gap):
    hi = list(range(20, 80))
    lo = list(range(4, 20 - gap))
    rows = lo + hi
    row, y, z, ids = _event(rows, _line_z(rows))
    res, _ = _track(row, y, z)
    tr = _tracklet_of(res, ids[21])          # start of the upper segment
    assert tr["hits"][20] == ids[20]         # searched below the start, found
    bridged = gap < PRM["max_miss"]
    for r in lo:
        assert (tr["hits"][r] == ids[r]) == bridged, r
    assert tr["row_inner"] == (4 if bridged else 20)


# ---------------------------------------------------------------- chi2 gate

@pytest.mark.parametrize("sign", [-1, 1])
def test_chi2_gate(sign):
    """A lone candidate two rows past the chain's end (one empty row between:
    no link can reach it) at predicted chi2 = 16 (1 -+ 1e-3)."""
    rows = list(range(2, 41))
    z = _line_z(rows)
    row, y, z, ids = _event(rows, z)
    mu, cov = _outward_prediction(ids, z, rows, 3, 40, 42)
    s11 = cov[0, 0] + SIG2
    for frac, taken in ((1.0 - 1e-3, True), (1.0 + 1e-3, False)):
        dz = sign * np.sqrt(PRM["chi2_max"] * frac * s11)
        zc = np.float32(mu[0] + dz)
        c2 = (float(zc) - mu[0]) ** 2 / s11
        assert (c2 <= PRM["chi2_max"]) == taken
        extra = [(42, 0.0, zc, len(rows))]
        row2, y2, z2, ids2 = _event(rows, z, extra)
        res, _ = _track(row2, y2, z2)
        tr = _tracklet_of(res, ids2[3])
        assert (tr["hits"][42] == len(rows)) == taken, (frac, c2)


# ---------------------------------------------------------------- ties

@pytest.mark.parametrize("lower_first", [False, True])
def test_equal_chi2_goes_to_the_lower_id(lower_first):
    """Candidates at (+a, z) and (-a, z) on the predicted z: the y residuals
    are exact negatives (the predicted y is exactly 0), so their chi2 are the
    same bits.  -a lies in a lower y bin and is met first; the lower id wins
    whether it is the first or the second one met."""
    rows = list(range(2, 41))
    z = _line_z(rows)
    _, _, _, ids0 = _event(rows, z)
    mu, _ = _outward_prediction(ids0, z, rows, 3, 40, 42)
    zc = np.float32(mu[0])
    a = np.float32(0.3)
    n = len(rows)
    lo_id, hi_id = 5, n + 1           # both ids inside the array
    if lower_first:
        extra = [(42, -a, zc, lo_id), (42, a, zc, hi_id)]
    else:
        extra = [(42, a, zc, lo_id), (42, -a, zc, hi_id)]
    row, y, zz, ids = _event(rows, z, extra)
    res, tab = _track(row, y, zz, occupancy=0.005)     # 4 y bins: y = 0 is a bin edge
    g = res["grid"]["idg"]
    pos_m = int(np.nonzero(g == extra[0 if lower_first else 1][3])[0][0])
    pos_p = int(np.nonzero(g == extra[1 if lower_first else 0][3])[0][0])
    assert pos_m < pos_p                      # -a comes first in grid (search) order
    y_bin = lambda v: int((np.float32(v) - tab["y0"][0]) * tab["inv_by"][0])
    assert y_bin(-a) < y_bin(a)
    tr = _tracklet_of(res, ids[3])
    assert tr["hits"][42] == lo_id


# ---------------------------------------------------------------- inward pass

def test_inward_pass_equals_least_squares_with_its_prior():
    rng = np.random.default_rng(2024)
    rows = list(range(0, 152))
    z = (0.5 * X64[rows] + rng.normal(0.0, 0.1, len(rows))).astype(np.float32)
    row, y, z, ids = _event(rows, z)
    res, _ = _track(row, y, z)
    tr = _tracklet_of(res, ids[1])           # row 0 gets no links: the chain starts on row 1
    assert tr["nhits"] == 152 and tr["row_inner"] == 0
    zr = z[[ids[r] for r in rows]].astype(np.float64)
    # outward: prior from the chain start (row 1) and the hit two rows up,
    # every hit of rows 2..151 updated
    t0 = (zr[3] - zr[1]) / (X64[3] - X64[1])
    mu_o, _, _ = _lsq(X64[1], zr[1], t0, X64[2:], zr[2:])
    t_out = mu_o[1]
    # inward: prior = the outermost hit's z and the outward direction, with
    # the initial covariance; rows 150..0 updated; output at row 0
    mu_i, cov_i, jmin = _lsq(X64[151], zr[151], t_out, X64[:151], zr[:151])
    m0, c0 = _moved(mu_i, cov_i, X64[0] - X64[151])
    par, cov = tr["par"].astype(np.float64), tr["cov"].astype(np.float64)
    assert par[0] == 0.0 and par[2] == 0.0 and par[4] == 0.0
    np.testing.assert_allclose(par[[1, 3]], m0, rtol=2e-5, atol=2e-6)
    # lower-triangle entries (z,z) = 2, (t,z) = 7, (t,t) = 9
    np.testing.assert_allclose(cov[[2, 7, 9]], [c0[0, 0], c0[1, 0], c0[1, 1]], rtol=1e-4)
    np.testing.assert_allclose(tr["chi2"], jmin, rtol=1e-4)
    # the float64 replay of the same hit list to 1e-10
    st, p64, c64, chi64 = oracle.tracklet_replay64(X, PRM, y, z, 1, tr["hits"])
    assert st == 0
    np.testing.assert_allclose(p64[[1, 3]], m0, rtol=1e-10)
    np.testing.assert_allclose(c64[[2, 7, 9]], [c0[0, 0], c0[1, 0], c0[1, 1]], rtol=1e-10)
    np.testing.assert_allclose(chi64, jmin, rtol=1e-10)


# ---------------------------------------------------------------- |sin(phi)| stop

def test_update_past_s_max_ends_the_tracklet_without_nan():
    """A steep chain (slope 0.75, sin(phi) = 0.6) whose second hit lies
    0.9 cm off the line (a straight-line cut wide enough to link it), with
    wide initial sin(phi) and q/pT variances: the update with that hit
    carries sin(phi) past 1 and q/pT to a curvature that, on the way back
    inwards, would bring sin(phi) below s_max within one row.  Every
    transport from a state with |sin(phi)| >= s_max must stop instead of
    taking the square root of a negative number: the outward pass ends after
    that hit and the inward pass stops at once, with finite outputs."""
    prm = dict(PRM, c_ss0=1.0, c_ww0=1e6, nb_d2max=9.0)
    rows = list(range(9, 20))            # row 9 has no pair below: the chain starts on row 10
    yv = (0.75 * (X64[rows] - X64[10])).astype(np.float32)
    yv[2] += np.float32(0.9)
    zv = _line_z(rows)
    row, y, z, ids = _event(rows, zv, y=yv)
    res, _ = _track(row, y, z, prm)
    assert ids[10] in res["starts"]
    tr = _tracklet_of(res, ids[10])
    assert abs(tr["par"][2]) >= 1.0              # the state the update produced
    assert tr["nhits"] == 1 and tr["hits"][11] == ids[11]
    assert tr["row_inner"] == 11
    for key in ("par", "cov", "chi2"):
        assert np.isfinite(res["tracklets"][key]).all()
