"""Pins of the oracle's calibrated refit and its finite-difference gradient.

The paper's reconstruction refits tracks once the calibration is applied
(section 2) and calibrates the drift velocity online (section 3); the
refit's calibration model is this project's reading (drift-velocity
scale, t0 and 14 smooth distortion coefficients).  Pinned here:
  * the double-precision central differences are converged (two step sizes
    agree);
  * exact chain-rule identities of the model: z_raw enters only through
    the drift length d = (1 + vd_scale)(d_raw - vd t0), so the t0 and
    vd-scale gradients are fixed sums of the z_raw gradients;
  * the reverse-mode (tape) gradient of the double refit, the reference
    for the library's adjoint, equals the converged central differences to
    1e-6 per block and per component, for both z sides;
  * float and double refits agree to the float filter's rounding;
  * chi2 at the true calibration is the smear's chi2 (ndf about 2n - 5), and
    a distortion the helix cannot absorb raises it.
"""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def small_set():
    return synth.make_config5(n_tracks=60)


def test_fd_gradient_converged(small_set):
    rs = small_set
    prm = synth.default_params()
    g = np.linspace(0.5, 1.5, rs.n_tracks)
    th = rs.theta_eval.astype(np.float64)
    a = oracle.refit_fd_grad(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, prm, th, g,
                             h_hit=1e-4, h_theta=1e-5)
    b = oracle.refit_fd_grad(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, prm, th, g,
                             h_hit=3e-5, h_theta=3e-6)
    for x, y in zip(a, b):
        assert np.linalg.norm(x - y) <= 1e-6 * np.linalg.norm(y)


def test_gradient_chain_rule_identities(small_set):
    rs = small_set
    prm = synth.default_params()
    g = np.ones(rs.n_tracks)
    th = rs.theta_eval.astype(np.float64)
    gy, gz, gt = oracle.refit_fd_grad(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, prm, th, g)
    cm = oracle.calib_model()
    vd = float(np.float32(cm.vd))
    dl = float(np.float32(cm.drift_len))
    side = 1.0
    # dL/dt0 = (vd / side) * sum dL/dz_raw
    assert abs(gt[1] - vd / side * gz.sum()) <= 1e-6 * np.abs(vd * gz).sum()
    # dL/dvd_scale = sum dL/dz_raw * (d_raw - vd t0) / (-side (1 + vd_scale))
    d_raw = dl - side * rs.z.astype(np.float64)
    expect = np.sum(gz * (d_raw - vd * th[1]) / (-side * (1.0 + th[0])))
    assert abs(gt[0] - expect) <= 1e-6 * np.sum(np.abs(gz * d_raw))


def test_tape_adjoint_matches_central_differences(small_set):
    rs = small_set
    prm = synth.default_params()
    g = np.linspace(0.5, 1.5, rs.n_tracks)
    th = rs.theta_eval.astype(np.float64)
    side = np.where(np.arange(rs.n_tracks) % 3 == 0, -1, 1).astype(np.int8)
    ad = oracle.refit_adjoint64(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, prm, th, g, side=side)
    fd = oracle.refit_fd_grad(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, prm, th, g, side=side)
    for a, b in zip(ad, fd):
        assert np.linalg.norm(a - b) <= 1e-6 * np.linalg.norm(b)
        assert np.all(np.abs(a - b) <= 1e-6 * np.abs(b).max())


def test_tape_adjoint_chain_rule_identities(small_set):
    """z_raw enters only through the drift length, so the t0 and vd-scale
    gradients are exact sums of the z_raw gradients (to double rounding)."""
    rs = small_set
    prm = synth.default_params()
    th = rs.theta_eval.astype(np.float64)
    gy, gz, gt = oracle.refit_adjoint64(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, prm, th,
                                        np.ones(rs.n_tracks))
    cm = oracle.calib_model()
    vd = float(np.float32(cm.vd))
    dl = float(np.float32(cm.drift_len))
    assert abs(gt[1] - vd * gz.sum()) <= 1e-12 * np.abs(vd * gz).sum()
    d_raw = dl - rs.z.astype(np.float64)
    expect = np.sum(gz * (d_raw - vd * th[1]) / (-(1.0 + th[0])))
    assert abs(gt[0] - expect) <= 1e-12 * np.sum(np.abs(gz * d_raw))


def test_float_refit_matches_double(small_set):
    rs = small_set
    prm = synth.default_params()
    r32 = oracle.refit(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, prm, rs.theta_eval)
    r64 = oracle.refit(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, prm, rs.theta_eval, fp64=True)
    assert np.all(r32["status"] == 0) and np.all(r64["status"] == 0)
    sig = np.sqrt(r64["cov"][:, [0, 2, 5, 9, 14]])
    scale = np.maximum(np.maximum(np.abs(r64["par"]), [1.0, 1.0, 0.01, 0.01, 0.1]), sig)
    rel = np.abs(r32["par"] - r64["par"]) / scale
    assert np.quantile(rel.max(1), 0.95) < 1e-4 and rel.max() < 1e-3
    assert np.allclose(r32["chi2"], r64["chi2"], rtol=1e-3)


def test_chi2_at_true_calibration(small_set):
    rs = small_set
    prm = synth.default_params()
    n = np.diff(rs.trk_off)
    true = oracle.refit(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, prm, rs.theta_true, fp64=True)
    ratio = true["chi2"].sum() / np.sum(2 * n - 5)
    assert 0.93 < ratio < 1.07, ratio
    # a distortion the helix cannot absorb (curvature-like radial u^2 term)
    th = rs.theta_true + 0.5 * np.eye(16)[5]
    off = oracle.refit(rs.trk_off, rs.row, rs.y, rs.z, rs.row_x, prm, th, fp64=True)
    assert off["chi2"].sum() > 1.05 * true["chi2"].sum()
