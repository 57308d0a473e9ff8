"""Pins of the oracle's calibration objective with the beam-axis constraint
(section 3: online calibration of drift velocity, t0 and distortions from
tracks; section 2: primaries from the origin; the objective is this
project's reading):
L(theta) = sum_t chi2_t(theta) + r_t^T W_t r_t, r_t the refit state of the
last hit transported to the beam-axis plane and W_t the inverse of its
transported covariance plus the vertex spread (held while theta moves).

  * its float64 reverse-mode gradient equals converged central differences;
  * the transport to the axis plane returns a helix from the origin to the
    origin: with the true calibration, y0 and z0 of noiseless tracks vanish;
  * minimising it over t0 and the 14 distortion coefficients (the drift
    velocity scale held at its true value: with primaries of a known vertex
    on one z side only the combination of scale and t0 that moves z at the
    vertex is seen) recovers the distortion the data were made with, within
    four standard deviations of the estimator (covariance 2 H^-1 from the
    Hessian of L at the minimum).
"""
import numpy as np
import pytest

import oracle
import synth

PRM = synth.default_params()


def _set(n, seed_shift=0):
    return synth.make_config5(n_tracks=n)


def test_objective_gradient_matches_central_differences():
    rs = _set(40)
    th = rs.theta_eval.astype(np.float64)
    g = np.linspace(0.5, 1.5, rs.n_tracks)
    w, wok = oracle.vertex_weights(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, PRM, th)
    assert wok.all()
    v, gt, per, vok = oracle.calib_objective(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, PRM, th,
                                             w, g=g)
    assert vok.all() and np.isclose(v, np.sum(g * per))
    fd = np.zeros(16)
    for k in range(16):
        h = 1e-6 if k == 0 else 1e-5
        e = np.zeros(16)
        e[k] = h
        fp = oracle.calib_objective(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, PRM, th + e, w,
                                    g=g, grad=False)[0]
        fm = oracle.calib_objective(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, PRM, th - e, w,
                                    g=g, grad=False)[0]
        fd[k] = (fp - fm) / (2 * h)
    assert np.linalg.norm(gt - fd) <= 1e-6 * np.linalg.norm(fd), np.abs(gt - fd) / np.abs(fd)


def test_noiseless_primaries_reach_the_origin():
    """Undistorted, unsmeared helices from the origin (theta = 0 and raw =
    true points): the beam-axis term is zero to the transport's accuracy."""
    rs = _set(60)
    tr = rs.tracks
    # rebuild the points of the segments without distortion or smear
    from synth.events import _segment_points, ROW_X64
    off = rs.trk_off
    ti = np.repeat(np.arange(rs.n_tracks), np.diff(off))
    xr = ROW_X64[rs.row]
    _, y, z, _ = _segment_points(tr, ti, xr)
    # unit weights: the term is y0^2 + z0^2
    w = np.tile([1.0, 0.0, 1.0], (rs.n_tracks, 1))
    v, _, per, vok = oracle.calib_objective(off, rs.row, y.astype(np.float32),
                                            z.astype(np.float32), rs.row_x, PRM, np.zeros(16), w,
                                            grad=False)
    assert vok.all()
    chi2 = oracle.refit(off, rs.row, y.astype(np.float32), z.astype(np.float32), rs.row_x, PRM,
                        np.zeros(16), fp64=True)["chi2"]
    # y0^2 + z0^2: every track within 0.03 cm of the origin
    # (the refit's priors pull the fitted state of noiseless hits slightly),
    # most within 0.003 cm
    r2 = per - chi2
    assert np.all(r2 < 9e-4) and np.median(r2) < 1e-5, (r2.max(), np.median(r2))


CALIB_FREE = (1, 9, 10, 12, 15)


@pytest.mark.slow
def test_damped_newton_recovers_the_distortion():
    """Levenberg-Marquardt steps from the evaluation point (weights taken at
    each iterate and held, Hessian by central differences of the reverse-mode
    gradient) over t0 and the azimuthal terms in 1, u, u^2 and w, the other
    parameters at their true values."""
    rs = _set(400)
    th_true = rs.theta_true.astype(np.float64)
    free = np.array(CALIB_FREE)
    th = th_true.copy()
    th[free] = rs.theta_eval.astype(np.float64)[free]
    lam = 1e-3

    def f(t, w, grad=True):
        return oracle.calib_objective(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, PRM, t, w,
                                      grad=grad)

    for _ in range(8):
        w, _ = oracle.vertex_weights(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, PRM, th)
        v, g, _, _ = f(th, w)
        H = np.zeros((free.size, free.size))
        for j, k in enumerate(free):
            e = np.zeros(16)
            e[k] = 1e-4
            H[:, j] = (f(th + e, w)[1][free] - f(th - e, w)[1][free]) / 2e-4
        H = 0.5 * (H + H.T)
        while lam < 1e12:
            cand = th.copy()
            cand[free] -= np.linalg.solve(H + lam * np.diag(np.diag(H)), g[free])
            if f(cand, w, grad=False)[0] < v:
                th, lam = cand, max(lam / 3, 1e-9)
                break
            lam *= 10
    sig = np.sqrt(np.diag(2.0 * np.linalg.inv(H)))
    dev = np.abs(th[free] - th_true[free]) / sig
    assert np.all(dev < 4.0), dev
    w, _ = oracle.vertex_weights(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, PRM, th)
    assert f(th, w, grad=False)[0] <= f(th_true, w, grad=False)[0]
