/*
 * Reference gradient of the calibrated refit in double precision --
 * TEST INFRASTRUCTURE ONLY.
 *
 * The refit's chi2 sum (the refit reading of section 2's track fit, with the
 * calibration of the drift velocity, t0 and the distortion map that
 * section 3 calibrates online) is differentiated by plain reverse-mode
 * automatic differentiation: the very same double-precision forward code
 * (kalman_impl.h, instantiated here with a recording number type) writes
 * every elementary operation and its local partial derivatives to a tape,
 * and one backward sweep over the tape accumulates d(sum_t g_t chi2_t) with
 * respect to each raw hit coordinate and the 16 calibration parameters.
 * Nothing is derived by hand: the gradient is exact (up to rounding) for
 * whatever the forward computes, branches included (a branch is taken on
 * values, as in the forward).
 */
#include <cmath>
#include <cstring>
#include <vector>

extern "C" {
#include "oracle.h"
}

namespace {

/* One tape entry: the value it produced depends on at most two earlier
 * entries a, b (-1: none) with partial derivatives da, db. */
struct Node {
    int a, b;
    double da, db;
};

std::vector<Node> g_tape;

struct AD {
    double v;
    int i;   /* tape index, -1 for a constant */
    AD() : v(0.0), i(-1) {}
    AD(double x) : v(x), i(-1) {}
};

static AD rec(double v, int a, double da, int b, double db)
{
    AD r;
    r.v = v;
    if (a < 0 && b < 0) return r;   /* constant folding: no dependence */
    g_tape.push_back(Node{a, b, da, db});
    r.i = (int)g_tape.size() - 1;
    return r;
}

static AD variable(double v)
{
    g_tape.push_back(Node{-1, -1, 0.0, 0.0});
    AD r;
    r.v = v;
    r.i = (int)g_tape.size() - 1;
    return r;
}

static AD operator+(const AD& x, const AD& y) { return rec(x.v + y.v, x.i, 1.0, y.i, 1.0); }
static AD operator-(const AD& x, const AD& y) { return rec(x.v - y.v, x.i, 1.0, y.i, -1.0); }
static AD operator*(const AD& x, const AD& y) { return rec(x.v * y.v, x.i, y.v, y.i, x.v); }
static AD operator/(const AD& x, const AD& y)
{
    const double q = x.v / y.v;
    return rec(q, x.i, 1.0 / y.v, y.i, -q / y.v);
}
static AD operator-(const AD& x) { return rec(-x.v, x.i, -1.0, -1, 0.0); }
static bool operator<(const AD& x, const AD& y) { return x.v < y.v; }
static AD ad_sqrt(const AD& x)
{
    const double r = std::sqrt(x.v);
    return rec(r, x.i, 0.5 / r, -1, 0.0);
}
static AD ad_fabs(const AD& x) { return rec(std::fabs(x.v), x.i, x.v < 0.0 ? -1.0 : 1.0, -1, 0.0); }

}  // namespace

/* The double-precision forward, instantiated on the recording type. */
#define REAL AD
#define SUF _ad
#define SQRT ad_sqrt
#define FABS ad_fabs
#define FMA(a, b, c) ((a) * (b) + (c))
#define C_1_6 (AD(1.0 / 6.0))
#define C_3_40 (AD(3.0 / 40.0))
#define C_5_112 (AD(5.0 / 112.0))
#define C_3_8 (AD(3.0 / 8.0))
#define C_5_16 (AD(5.0 / 16.0))
#define C_3_20 (AD(3.0 / 20.0))
#define C_15_112 (AD(15.0 / 112.0))
namespace {
#include "kalman_impl.h"
}

/* ---- calibration objective with the beam-axis constraint -----------------
 * Reading of section 3 (online calibration of the drift velocity, t0 and
 * distortions) with section 2's primaries from the origin: per track, the
 * refit chi2 plus r^T W r, where r = (y0, z0) is the refit state of the last
 * hit (at the calibrated plane of that hit) transported to the beam-axis
 * plane x = 0 of the sector frame in ceil(x / 20 cm) equal steps, and W a
 * per-track weight (2x2, given, held fixed: the inverse of the refit
 * covariance transported there plus the vertex spread, taken at the current
 * calibration; see orc_vertex_weights64).  A track whose refit or transport
 * stops adds only what it has (its chi2 up to the stop, no vertex term).
 * L = sum_t g_t L_t.  The gradient is the tape gradient of exactly this
 * computation. */
static AD vertex_term(const AD* p_in, AD x, const orc_params* prm, const double* w, int* ok)
{
    AD p[5], C[15];
    for (int i = 0; i < 5; i++) p[i] = p_in[i];
    for (int i = 0; i < 15; i++) C[i] = AD(0.0);
    int n = (int)std::ceil(x.v / 20.0);
    if (n < 1) n = 1;
    AD dx = (AD(0.0) - x) / AD((double)n);
    *ok = 1;
    for (int i = 0; i < n; i++)
        if (!propagate_ad(p, C, dx, AD((double)prm->curv), AD((double)prm->s_max))) {
            *ok = 0;
            return AD(0.0);
        }
    /* r^T W r, W = [[w0, w1], [w1, w2]] */
    return p[0] * (AD(w[0]) * p[0] + AD(w[1]) * p[1]) + p[1] * (AD(w[1]) * p[0] + AD(w[2]) * p[1]);
}

extern "C" double orc_calib_objective64(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                                        const double* y, const double* z,
                                        const signed char* side, const float* row_x,
                                        const orc_params* prm, const orc_calib_model* cm,
                                        const double* theta, const double* g, const double* wv,
                                        double* grad_theta, double* per_track, int* vertex_ok)
{
    double total = 0.0;
    if (grad_theta)
        for (int k = 0; k < 16; k++) grad_theta[k] = 0.0;
    std::vector<AD> vy, vz;
    std::vector<double> adj;
    for (int64_t t = 0; t < n_tracks; t++) {
        const int a = trk_off[t], n = trk_off[t + 1] - a;
        g_tape.clear();
        AD th[16];
        for (int k = 0; k < 16; k++) th[k] = variable(theta[k]);
        vy.resize((size_t)n);
        vz.resize((size_t)n);
        for (int i = 0; i < n; i++) {
            vy[i] = AD(y[a + i]);
            vz[i] = AD(z[a + i]);
        }
        AD p[5], C[15], chi2;
        const AD sd(side ? (double)side[t] : 1.0);
        const int st = refit_track_ad(n, row + a, vy.data(), vz.data(), sd, row_x, prm, cm, th, p,
                                      C, &chi2);
        AD lt = chi2;
        int vok = 0;
        if (st == 0 && wv) {
            AD xl, yl, zl;
            calibrate_ad(th, AD((double)row_x[row[a + n - 1]]), vy[n - 1], vz[n - 1], sd,
                         AD((double)cm->drift_len), AD((double)cm->vd), AD((double)cm->tan_half),
                         AD((double)cm->u_centre), AD((double)cm->u_scale), &xl, &yl, &zl);
            AD v = vertex_term(p, xl, prm, wv + 3 * t, &vok);
            if (vok) lt = lt + v;
        }
        if (per_track) per_track[t] = lt.v;
        if (vertex_ok) vertex_ok[t] = vok;
        total += g[t] * lt.v;
        if (!grad_theta) continue;
        adj.assign(g_tape.size(), 0.0);
        if (lt.i >= 0) adj[(size_t)lt.i] = g[t];
        for (int j = (int)g_tape.size() - 1; j >= 0; j--) {
            const Node& nd = g_tape[(size_t)j];
            const double aj = adj[(size_t)j];
            if (aj == 0.0) continue;
            if (nd.a >= 0) adj[(size_t)nd.a] += nd.da * aj;
            if (nd.b >= 0) adj[(size_t)nd.b] += nd.db * aj;
        }
        for (int k = 0; k < 16; k++) grad_theta[k] += adj[(size_t)th[k].i];
    }
    g_tape.clear();
    g_tape.shrink_to_fit();
    return total;
}

extern "C" void orc_refit64_adjoint(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                                    const double* y, const double* z, const signed char* side,
                                    const float* row_x, const orc_params* prm,
                                    const orc_calib_model* cm, const double* theta,
                                    const double* g, double* grad_y, double* grad_z,
                                    double* grad_theta)
{
    for (int k = 0; k < 16; k++) grad_theta[k] = 0.0;
    std::vector<AD> vy, vz;
    std::vector<double> adj;
    for (int64_t t = 0; t < n_tracks; t++) {
        const int a = trk_off[t], n = trk_off[t + 1] - a;
        g_tape.clear();
        AD th[16];
        for (int k = 0; k < 16; k++) th[k] = variable(theta[k]);
        vy.resize((size_t)n);
        vz.resize((size_t)n);
        for (int i = 0; i < n; i++) {
            vy[i] = variable(y[a + i]);
            vz[i] = variable(z[a + i]);
        }
        AD p[5], C[15], chi2;
        const AD sd(side ? (double)side[t] : 1.0);
        refit_track_ad(n, row + a, vy.data(), vz.data(), sd, row_x, prm, cm, th, p, C, &chi2);
        adj.assign(g_tape.size(), 0.0);
        if (chi2.i >= 0) adj[(size_t)chi2.i] = g[t];
        for (int j = (int)g_tape.size() - 1; j >= 0; j--) {
            const Node& nd = g_tape[(size_t)j];
            const double aj = adj[(size_t)j];
            if (aj == 0.0) continue;
            if (nd.a >= 0) adj[(size_t)nd.a] += nd.da * aj;
            if (nd.b >= 0) adj[(size_t)nd.b] += nd.db * aj;
        }
        for (int k = 0; k < 16; k++) grad_theta[k] += adj[(size_t)th[k].i];
        for (int i = 0; i < n; i++) {
            grad_y[a + i] = adj[(size_t)vy[i].i];
            grad_z[a + i] = adj[(size_t)vz[i].i];
        }
    }
    g_tape.clear();
    g_tape.shrink_to_fit();
}
