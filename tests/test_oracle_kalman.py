"""Pins of the oracle's Kalman-filter primitives against closed forms.

The paper states that track following uses a Kalman filter (section 3) but
gives no formulas; the oracle's propagator, transport Jacobian and update
are pinned here against mathematics written independently of them:
  * helix arcs from circle geometry (asin / cos, no series),
  * the transport Jacobian against central differences of that closed form,
  * the update against Gaussian conditioning in information form,
  * a filter on noiseless tracks against the exact generating helix,
  * fit pulls and chi2 against their distributions on smeared tracks.
"""
import math

import numpy as np
import pytest

import oracle
import synth

CURV = float(synth.CURV_PER_QPT)


def helix_step(p, dx, curv):
    """Exact state after moving a helix from plane x to x + dx (closed form:
    circle centre, sin(phi) linear in x, arc = dphi / k)."""
    y, z, s, t, w = p
    k = curv * w
    s2 = s + k * dx
    if k == 0.0:
        tanphi = s / math.sqrt(1 - s * s)
        return np.array([y + dx * tanphi, z + t * dx * math.sqrt(1 + tanphi**2), s, t, w])
    c1, c2 = math.sqrt(1 - s * s), math.sqrt(1 - s2 * s2)
    y2 = y + (c1 - c2) / k
    arc = (math.asin(s2) - math.asin(s)) / k
    return np.array([y2, z + t * arc, s2, t, w])


def full(Cl):
    M = np.zeros((5, 5))
    k = 0
    for i in range(5):
        for j in range(i + 1):
            M[i, j] = M[j, i] = Cl[k]
            k += 1
    return M


def lower(M):
    return np.array([M[i, j] for i in range(5) for j in range(i + 1)])


def rand_state(rng):
    return np.array([rng.uniform(-20, 20), rng.uniform(-100, 100), rng.uniform(-0.7, 0.7),
                     rng.uniform(-1, 1), rng.uniform(-8, 8)])


def rand_cov(rng):
    A = rng.normal(size=(5, 5)) * np.array([0.1, 0.1, 0.01, 0.01, 0.5])[:, None]
    return A @ A.T + np.diag([0.01, 0.01, 1e-4, 1e-4, 0.01])


def test_propagate_matches_exact_helix():
    rng = np.random.default_rng(7)
    worst = 0.0
    for _ in range(500):
        p = rand_state(rng)
        dx = rng.choice([1.0596026, -1.0596026, 3.2, -7.5])
        ok, p2, _ = oracle.propagate(p, lower(np.eye(5)), dx, CURV)
        ref = helix_step(p, dx, CURV)
        if abs(ref[2]) >= 0.95:
            assert not ok
            continue
        assert ok
        scale = np.array([1, 1, 1e-3, 1, 1])
        worst = max(worst, np.max(np.abs(p2 - ref) / (np.abs(ref) + scale)))
    assert worst < 1e-11


def test_propagate_straight_line_limit():
    p = np.array([1.0, 2.0, 0.3, 0.5, 0.0])
    ok, p2, _ = oracle.propagate(p, lower(np.eye(5)), 10.0, 0.0)
    assert ok
    tanphi = 0.3 / math.sqrt(1 - 0.09)
    assert abs(p2[0] - (1 + 10 * tanphi)) < 1e-12
    assert abs(p2[1] - (2 + 0.5 * 10 * math.sqrt(1 + tanphi**2))) < 1e-12
    assert p2[2] == 0.3


def test_propagate_stops_at_s_max():
    p = np.array([0.0, 0.0, 0.94, 0.1, -5.0])   # k = curv*w > 0 -> s grows
    ok, p2, _ = oracle.propagate(p, lower(np.eye(5)), 5.0, CURV, 0.95)
    assert not ok and np.all(p2 == p)


def test_propagate_stops_on_an_incoming_state_past_s_max():
    """An update can leave |sin(phi)| >= s_max (even > 1); a transport from
    there stops (state untouched) even when the step's curvature would bring
    sin(phi) back below s_max: no square root of a negative number."""
    for s in (0.95, 0.97, 1.02, -1.02):
        w = -np.sign(s) * 60.0 / abs(CURV) / 1.0596026 * 0.1     # k dx pulls s back by 0.1
        p = np.array([0.0, 0.0, s, 0.1, w])
        for fp64 in (True, False):
            ok, p2, C2 = oracle.propagate(p, lower(np.eye(5)), 1.0596026, CURV, 0.95, fp64=fp64)
            assert not ok and np.all(p2 == p.astype(p2.dtype)) and np.isfinite(C2).all()


def test_straight_line_kalman_equals_least_squares():
    """B = 0 (curv = 0), the track in the plane y = 0 (so sin(phi) stays
    exactly 0 and the filter's transport is linear): the filter run plane by
    plane over measurements with noisy z (and y = 0) equals the regularised
    least-squares fit with the same Gaussian prior -- mean, full covariance
    and the sum of the update chi2 (= the minimum of the objective), in
    float64 to 1e-10.  The y, sin(phi) block is pinned through the
    covariance, the z, tan(lambda) block through mean and covariance."""
    rng = np.random.default_rng(8)
    sy2, sz2 = 0.01, 0.02
    for _ in range(20):
        n = int(rng.integers(3, 40))
        xs = 85.0 + np.cumsum(rng.uniform(0.5, 3.0, n))
        x0 = 85.0 - rng.uniform(0.0, 5.0)
        t_true, z_true = rng.uniform(-1, 1), rng.uniform(-50, 50)
        zm = z_true + t_true * (xs - x0) + rng.normal(0, math.sqrt(sz2), n)
        # prior: block diagonal {y, s}, {z, t}, {w}
        Ays = rng.normal(size=(2, 2)) * [[0.2], [0.02]]
        Azt = rng.normal(size=(2, 2)) * [[0.3], [0.05]]
        P0 = np.zeros((5, 5))
        P0[np.ix_([0, 2], [0, 2])] = Ays @ Ays.T + np.diag([0.01, 1e-4])
        P0[np.ix_([1, 3], [1, 3])] = Azt @ Azt.T + np.diag([0.01, 1e-4])
        P0[4, 4] = rng.uniform(1, 100)
        mu0 = np.array([0.0, z_true + rng.normal(0, 0.3), 0.0, t_true + rng.normal(0, 0.05),
                        rng.normal(0, 3)])
        p, Cl = mu0.copy(), lower(P0)
        xp, csum = x0, 0.0
        for i in range(n):
            ok, p, Cl = oracle.propagate(p, Cl, xs[i] - xp, 0.0, 0.95)
            assert ok
            c2, p, Cl = oracle.update(p, Cl, 0.0, zm[i], sy2, sz2)
            csum += c2
            xp = xs[i]
        # least squares for the state at x0: y_i = y + d_i s, z_i = z + d_i t
        d = xs - x0
        H = np.zeros((2 * n, 5))
        H[0::2, 0] = 1.0
        H[0::2, 2] = d
        H[1::2, 1] = 1.0
        H[1::2, 3] = d
        m = np.zeros(2 * n)
        m[1::2] = zm
        Ri = np.tile([1.0 / sy2, 1.0 / sz2], n)
        P0i = np.linalg.inv(P0)
        A = P0i + H.T @ (Ri[:, None] * H)
        mu = np.linalg.solve(A, P0i @ mu0 + H.T @ (Ri * m))
        cov = np.linalg.inv(A)
        r = m - H @ mu
        jmin = (mu - mu0) @ P0i @ (mu - mu0) + r @ (Ri * r)
        # carried to the last plane
        D = xs[-1] - x0
        T = np.eye(5)
        T[0, 2] = T[1, 3] = D
        mu_n, cov_n = T @ mu, T @ cov @ T.T
        np.testing.assert_allclose(p, mu_n, rtol=1e-10, atol=1e-10)
        scale = np.sqrt(np.outer(np.diag(cov_n), np.diag(cov_n)))
        assert np.all(np.abs(full(Cl) - cov_n) <= 1e-10 * scale)
        assert abs(csum - jmin) <= 1e-10 * max(1.0, jmin)


def test_transport_jacobian_matches_central_differences():
    """Covariance transport C' = F C F^T: the F it applies (read off by
    transporting unit covariances) equals the central-difference Jacobian of
    the closed-form helix step, and random covariances transport as F C F^T."""
    rng = np.random.default_rng(11)
    for _ in range(60):
        p = rand_state(rng)
        p[2] = rng.uniform(-0.5, 0.5)
        dx = rng.choice([1.0596026, -1.0596026, 4.0, -9.0])
        J = np.zeros((5, 5))
        for j in range(5):
            h = 1e-5 * max(1.0, abs(p[j]))
            e = np.zeros(5)
            e[j] = h
            J[:, j] = (helix_step(p + e, dx, CURV) - helix_step(p - e, dx, CURV)) / (2 * h)
        F = np.zeros((5, 5))
        for j in range(5):
            E = np.zeros((5, 5))
            E[j, j] = 1.0
            ok, _, C2 = oracle.propagate(p, lower(E), dx, CURV)
            assert ok
            # with C = e_j e_j^T, C' = F_j F_j^T; column j of C' is F[:, j] F[j, j]
            F[:, j] = full(C2)[:, j]
        assert np.all(np.abs(F - J) <= 1e-7 * (1.0 + np.abs(J))), np.abs(F - J).max()
        Cm = rand_cov(rng)
        ok, _, C2 = oracle.propagate(p, lower(Cm), dx, CURV)
        ref = F @ Cm @ F.T
        scale = np.sqrt(np.outer(np.diag(ref), np.diag(ref)))
        assert np.all(np.abs(full(C2) - ref) <= 1e-12 * scale + 1e-15)


def test_update_equals_gaussian_conditioning():
    rng = np.random.default_rng(3)
    R = np.diag([0.01, 0.02])
    H = np.zeros((2, 5))
    H[0, 0] = H[1, 1] = 1
    for _ in range(200):
        p = rand_state(rng)
        P = rand_cov(rng)
        m = p[:2] + rng.normal(size=2) * 0.2
        c2, p2, C2 = oracle.update(p, lower(P), m[0], m[1], 0.01, 0.02)
        # information form, independent of the gain form used by the oracle
        Pi = np.linalg.inv(P)
        Ri = np.linalg.inv(R)
        Ppost = np.linalg.inv(Pi + H.T @ Ri @ H)
        mpost = Ppost @ (Pi @ p + H.T @ Ri @ m)
        r = m - H @ p
        chi2 = r @ np.linalg.solve(H @ P @ H.T + R, r)
        assert np.allclose(p2, mpost, rtol=1e-9, atol=1e-10)
        assert np.allclose(full(C2), Ppost, rtol=1e-7, atol=1e-12)
        assert abs(c2 - chi2) <= 1e-9 * max(1.0, chi2)


def _truth_hits(rng, n_tracks, pt_min=0.3):
    trk = synth.events._sample_tracks(rng, n_tracks, 0.0, math.radians(20), 0.1, 0.9, pt_min)
    rows = np.arange(20, 140)
    ti = np.repeat(np.arange(n_tracks), rows.shape[0])
    ri = np.tile(rows, n_tracks)
    X = synth.ROW_X.astype(np.float64)       # the planes the fit uses
    u, y, z, turn = synth.events._segment_points(trk, ti, X[ri])
    ok = (np.abs(u) < 0.85).reshape(n_tracks, -1).all(1)
    return trk, ri.reshape(n_tracks, -1), y.reshape(n_tracks, -1), z.reshape(n_tracks, -1), ok


def _exact_state_at(trk, i, x):
    """Exact helix state (y, z, s, t, w) at the local plane x."""
    u, y, z, _ = synth.events._segment_points(trk, np.array([i]), np.array([x]))
    return np.array([y[0], z[0], u[0], trk["tanl"][i], trk["qpt"][i]])


def test_filter_on_noiseless_helix_recovers_truth():
    """Exact hits of a helix, diffuse prior: the filtered state at the last
    hit is the helix state there and chi2 vanishes (the prior's pull and the
    linearisation error are below 1e-7)."""
    rng = np.random.default_rng(5)
    trk, ri, Y, Z, ok = _truth_hits(rng, 40)
    prm = synth.default_params()
    prm.update(c_ss0=1e4, c_tt0=1e4, c_ww0=1e6)
    theta = np.zeros(16)
    for i in np.nonzero(ok)[0][:20]:
        n = ri.shape[1]
        off = np.array([0, n], np.int32)
        res = oracle.refit(off, ri[i].astype(np.uint8), Y[i], Z[i], synth.ROW_X,
                           prm, theta, fp64=True)
        assert res["status"][0] == 0
        ref = _exact_state_at(trk, i, float(synth.ROW_X[ri[i, -1]]))
        d = res["par"][0] - ref
        assert np.all(np.abs(d[:2]) < 5e-7) and np.all(np.abs(d[2:4]) < 1e-7), d
        assert abs(d[4]) < 1e-6 * max(1.0, abs(ref[4])), d
        assert res["chi2"][0] < 1e-5


def test_filter_pulls_and_chi2_on_smeared_tracks():
    """With Gaussian smear equal to the assumed measurement error the fitted
    parameters scatter around the truth with unit pulls, and chi2 follows
    its distribution (mean 2(n-1) minus the parameters fixed by the three
    initialisation constraints: about 2n - 5)."""
    rng = np.random.default_rng(9)
    trk, ri, Y, Z, ok = _truth_hits(rng, 600)
    prm = synth.default_params()
    idx = np.nonzero(ok)[0]
    n = ri.shape[1]
    Ys = Y[idx] + rng.normal(0, 0.1, Y[idx].shape)
    Zs = Z[idx] + rng.normal(0, 0.1, Z[idx].shape)
    m = idx.shape[0]
    off = (np.arange(m + 1) * n).astype(np.int32)
    res = oracle.refit(off, ri[idx].ravel().astype(np.uint8), Ys.ravel(), Zs.ravel(),
                       synth.ROW_X, prm, np.zeros(16), fp64=True)
    assert np.all(res["status"] == 0)
    pulls = []
    for j, i in enumerate(idx):
        ref = _exact_state_at(trk, i, float(synth.ROW_X[ri[i, -1]]))
        var = np.diag(full(res["cov"][j]))
        pulls.append((res["par"][j] - ref) / np.sqrt(var))
    pulls = np.array(pulls)
    assert np.all(np.abs(pulls.mean(0)) < 0.15), pulls.mean(0)
    assert np.all(np.abs(pulls.std(0) - 1) < 0.12), pulls.std(0)
    ndf = 2 * n - 5
    assert abs(res["chi2"].mean() / ndf - 1) < 0.03, res["chi2"].mean() / ndf


def test_calibration_hand_values():
    cm = oracle.calib_model()
    th = np.zeros(16)
    # identity at theta = 0
    assert np.allclose(oracle.calibrate(th, 245.0, 10.0, 100.0), [245.0, 10.0, 100.0])
    assert np.allclose(oracle.calibrate(th, 85.0, -3.0, -40.0, side=-1.0), [85.0, -3.0, -40.0])
    # drift-velocity scale: drift 150 cm -> 151.5 cm, z 100 -> 98.5
    th[0] = 0.01
    assert np.allclose(oracle.calibrate(th, 165.0, 0.0, 100.0), [165.0, 0.0, 98.5], atol=1e-5)
    # t0 of 1 us removes vd * 1 us = 2.58 cm of drift (float32 model constant)
    th[:] = 0
    th[1] = 1.0
    vd = float(np.float32(2.58))
    assert np.allclose(oracle.calibrate(th, 165.0, 0.0, 100.0), [165.0, 0.0, 100.0 + vd])
    # side C mirrors z
    assert np.allclose(oracle.calibrate(th, 165.0, 0.0, -100.0, side=-1.0), [165.0, 0.0, -100.0 - vd])
    # radial and azimuthal basis terms, at x = 245 (u = 1), y = 245 tan10 (v = 1),
    # z = 0 (w = 1)
    yv = 245.0 * float(np.float32(cm.tan_half))
    for j, val in enumerate([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0]):
        th[:] = 0
        th[2 + j] = 0.5
        x, y, z = oracle.calibrate(th, 245.0, yv, 0.0)
        assert abs(x - (245.0 + 0.5 * val)) < 1e-5 and abs(y - yv) < 1e-9
        th[:] = 0
        th[9 + j] = 0.25
        x, y, z = oracle.calibrate(th, 245.0, yv, 0.0)
        assert abs(x - 245.0) < 1e-12 and abs(y - (yv + 0.25 * val)) < 1e-5
    # u = -1 at x = 85 flips the odd u terms
    th[:] = 0
    th[3] = 0.5        # a1 * u
    th[5] = 0.25       # a3 * u^2
    x, _, _ = oracle.calibrate(th, 85.0, 0.0, 250.0)
    assert abs(x - (85.0 - 0.5 + 0.25)) < 1e-6


def test_calibration_inverts_generator_distortion():
    """The generator distorts true points with its own inverse iteration; the
    oracle's calibration maps the raw points back onto the true helix, so
    the residuals to the truth are the smear alone (RMS 0.1 cm), while the
    uncalibrated points are off by the distortion."""
    rs = synth.make_config5(n_tracks=40)
    res = {True: [], False: []}
    for calibrated in (True, False):
        theta = rs.theta_true if calibrated else np.zeros(16)
        for t in range(40):
            for i in range(rs.trk_off[t], rs.trk_off[t + 1]):
                xr = float(rs.row_x[rs.row[i]])
                x, y, z = oracle.calibrate(theta, xr, float(rs.y[i]), float(rs.z[i]))
                _, yt, zt, _ = synth.events._segment_points(rs.tracks, np.array([t]),
                                                            np.array([x]))
                res[calibrated] += [y - yt[0], z - zt[0]]
    rms_cal = float(np.sqrt(np.mean(np.square(res[True]))))
    rms_raw = float(np.sqrt(np.mean(np.square(res[False]))))
    assert 0.095 < rms_cal < 0.105, rms_cal
    assert rms_raw > 1.15 * rms_cal, (rms_raw, rms_cal)
