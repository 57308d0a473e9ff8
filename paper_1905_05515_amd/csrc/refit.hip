// Calibrated Kalman refit of found tracks and its adjoint.
//
// Forward (one thread per track): calibrate every raw cluster with the 16
// parameters theta, start from the first and third hits, filter outwards and
// sum the chi2 of the updates; the state after every update but the last is
// written as a checkpoint (5 parameters + 15 covariance entries).
//
// Adjoint (one thread per track): with L = sum_k g_k chi2_k, a reverse sweep
// from the last hit reloads each checkpoint, recomputes the transport and
// update, and applies their exact derivatives: of the update (gain, chi2,
// covariance) and of the transport including the dependence of the Jacobian
// on the state and on the step length, which the calibration moves.  The
// symmetric covariance carries a symmetric adjoint G with
// dL = sum_ij G_ij dC_ij.  Hit gradients are written per hit; the theta
// gradient is reduced per block in a fixed order, then over blocks.
#include <mutex>

#include "tpc_internal.hpp"

namespace tpc {

namespace {

__device__ __forceinline__ int lt(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

struct CalibModel {
    float DL, VD, TH, UC, US;
    float iUS, iDL;      // 1 / US, 1 / DL (taken once on the host)
};

inline CalibModel make_calib(const tpc_calib_model& m)
{
    return CalibModel{m.drift_len, m.vd, m.tan_half, m.u_centre, m.u_scale, 1.0f / m.u_scale,
                      1.0f / m.drift_len};
}

struct CalHit {
    float x, y, z;      // calibrated plane, y, z
    float xr, yr, dr;   // raw plane x_r, raw y, raw drift length
    float d, u, v;      // calibrated drift, basis coordinates
};

__device__ __forceinline__ CalHit calibrate(const float* th, float xr, float yr, float zr, float sd,
                                            const CalibModel& cm)
{
#pragma clang fp contract(fast)
    CalHit h;
    h.xr = xr;
    h.yr = yr;
    h.dr = cm.DL - sd * zr;
    h.d = (1.0f + th[0]) * (h.dr - cm.VD * th[1]);
    h.z = sd * (cm.DL - h.d);
    h.u = (xr - cm.UC) * cm.iUS;
    h.v = yr / (xr * cm.TH);
    const float w = h.d * cm.iDL;
    const float b[7] = {1.0f, h.u, h.v, h.u * h.u, h.u * h.v, h.v * h.v, w};
    float dr = 0.0f, drphi = 0.0f;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        dr += th[2 + j] * b[j];
        drphi += th[9 + j] * b[j];
    }
    h.x = xr + dr;
    h.y = yr + drphi;
    return h;
}

// reverse of calibrate: adjoints (X, Y, Z) of the calibrated point ->
// raw (y, z) adjoints, accumulated theta adjoint
__device__ __forceinline__ void calibrate_adj(const float* th, const CalHit& h, float sd,
                                              const CalibModel& cm, float X, float Y, float Z,
                                              double* gth, float& gyr, float& gzr)
{
    // reverse-mode arithmetic: compared with the float64 adjoint within a
    // tolerance, so products and sums may contract into fused multiply-adds.
    // The theta adjoint is summed in float64 (per lane over its hits, then
    // over lanes and blocks): it is a sum of ~1e8 terms that cancel at the
    // calibration's minimum, where float32 sums would leave a noise floor
    // that stops the fit short of it.
#pragma clang fp contract(fast)
    const float w = h.d * cm.iDL;
    const float b[7] = {1.0f, h.u, h.v, h.u * h.u, h.u * h.v, h.v * h.v, w};
    float bb[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        gth[2 + j] += (double)(X * b[j]);
        gth[9 + j] += (double)(Y * b[j]);
        bb[j] = X * th[2 + j] + Y * th[9 + j];
    }
    const float vb = bb[2] + bb[4] * h.u + 2.0f * bb[5] * h.v;
    gyr = Y + vb / (h.xr * cm.TH);
    const float db = bb[6] * cm.iDL - Z * sd;
    gth[0] += (double)(db * (h.dr - cm.VD * th[1]));
    gth[1] += (double)(-db * (1.0f + th[0]) * cm.VD);
    gzr = -sd * (1.0f + th[0]) * db;
}

// hit i of a track: entry a + i of the CSR, cluster idx[a + i] if given
struct HitRef {
    const int32_t* idx;
    const uint8_t* row_;
    const float* y_;
    const float* z_;
    int a;
    __device__ __forceinline__ int cl(int i) const { return idx ? idx[a + i] : a + i; }
    __device__ __forceinline__ int row(int i) const { return row_[cl(i)]; }
    __device__ __forceinline__ CalHit cal(int i, const float* th, const float* xs, float sd,
                                          const CalibModel& cm) const
    {
        const int c = cl(i);
        return calibrate(th, xs[row_[c]], y_[c], z_[c], sd, cm);
    }
    // raw plane, y, z of cluster c (an index from cl)
    __device__ __forceinline__ void raw(int c, const float* xs, float* r) const
    {
        r[0] = xs[row_[c]];
        r[1] = y_[c];
        r[2] = z_[c];
    }
};

struct Prop {
    float dx, k, s2, c1, c2, cc, T, q, L, a, a2, g, S, Ts, kdx, Tw, LT, G1, Sk;
    float ys, yw, zs, zt, zw, sw;   // non-trivial Jacobian entries
    float FC[5][5];                 // F C
};

// transport of (p, C) by dx; fills the intermediates; false when |s| at
// either end of the step is not below s_max
__device__ __forceinline__ bool prop_fwd(float* p, float* C, float dx, float curv, float s_max,
                                         Prop& P)
{
    // the refit is compared with the float64 refit within a tolerance (it
    // takes no decision but the transport stop), so products and sums may
    // contract into fused multiply-adds, as in the reverse sweep
#pragma clang fp contract(fast)
    const float s = p[2], t = p[3], w = p[4];
    P.dx = dx;
    P.k = curv * w;
    P.s2 = s + P.k * dx;
    if (!(fabsf(s) < s_max) || !(fabsf(P.s2) < s_max)) return false;
    P.c1 = sqrtf((1.0f - s) * (1.0f + s));
    P.c2 = sqrtf((1.0f - P.s2) * (1.0f + P.s2));
    P.cc = P.c1 + P.c2;
    const float icc = 1.0f / P.cc;   // three quotients by c1 + c2
    P.T = (s + P.s2) * icc;
    P.q = sqrtf(1.0f + P.T * P.T);
    P.L = dx * P.q;
    P.a = 0.5f * P.k * P.L;
    P.a2 = P.a * P.a;
    P.g = 1.0f + P.a2 * ((1.0f / 6.0f) + P.a2 * ((3.0f / 40.0f) + P.a2 * (5.0f / 112.0f)));
    P.S = P.L * P.g;
    P.Ts = (2.0f + P.T * (s / P.c1 + P.s2 / P.c2)) * icc;
    P.kdx = curv * dx;
    P.Tw = P.kdx * (1.0f + P.T * (P.s2 / P.c2)) * icc;
    P.LT = dx * P.T / P.q;
    P.G1 = 1.0f + P.a2 * (0.5f + P.a2 * ((3.0f / 8.0f) + P.a2 * (5.0f / 16.0f)));
    P.Sk = P.L * P.L * P.a * ((1.0f / 6.0f) + P.a2 * ((3.0f / 20.0f) + P.a2 * (15.0f / 112.0f)));
    P.ys = dx * P.Ts;
    P.yw = dx * P.Tw;
    const float m1 = P.G1 * P.LT;
    P.zs = t * m1 * P.Ts;
    P.zt = P.S;
    P.zw = t * (m1 * P.Tw + P.Sk * curv);
    P.sw = P.kdx;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const float cy = C[lt(0, j)], cz = C[lt(1, j)], cs = C[lt(2, j)];
        const float ct = C[lt(3, j)], cw = C[lt(4, j)];
        P.FC[0][j] = cy + P.ys * cs + P.yw * cw;
        P.FC[1][j] = cz + P.zs * cs + P.zt * ct + P.zw * cw;
        P.FC[2][j] = cs + P.sw * cw;
        P.FC[3][j] = ct;
        P.FC[4][j] = cw;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const float* B = P.FC[i];
        C[lt(i, 0)] = B[0] + P.ys * B[2] + P.yw * B[4];
        if (i >= 1) C[lt(i, 1)] = B[1] + P.zs * B[2] + P.zt * B[3] + P.zw * B[4];
        if (i >= 2) C[lt(i, 2)] = B[2] + P.sw * B[4];
        if (i >= 3) C[lt(i, 3)] = B[3];
        if (i >= 4) C[lt(i, 4)] = B[4];
    }
    p[0] = p[0] + dx * P.T;
    p[1] = p[1] + t * P.S;
    p[2] = P.s2;
    return true;
}

struct Upd {
    float r0, r1, B00, B10, B11;
    float A0[5], A1[5], K0[5], K1[5];
};

__device__ __forceinline__ float upd_fwd(float* p, float* C, float my, float mz, float sy2,
                                         float sz2, Upd& U)
{
#pragma clang fp contract(fast)
    U.r0 = my - p[0];
    U.r1 = mz - p[1];
    const float S00 = C[0] + sy2, S10 = C[1], S11 = C[2] + sz2;
    const float idet = 1.0f / (S00 * S11 - S10 * S10);
    U.B00 = S11 * idet;
    U.B10 = -S10 * idet;
    U.B11 = S00 * idet;
    const float chi2 = U.r0 * (U.B00 * U.r0 + U.B10 * U.r1) + U.r1 * (U.B10 * U.r0 + U.B11 * U.r1);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        U.A0[i] = C[lt(i, 0)];
        U.A1[i] = C[lt(i, 1)];
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        U.K0[i] = U.A0[i] * U.B00 + U.A1[i] * U.B10;
        U.K1[i] = U.A0[i] * U.B10 + U.A1[i] * U.B11;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        p[i] += U.K0[i] * U.r0 + U.K1[i] * U.r1;
#pragma unroll
        for (int j = 0; j <= i; ++j) C[lt(i, j)] -= U.K0[i] * U.A0[j] + U.K1[i] * U.A1[j];
    }
    return chi2;
}

// adjoint of the update: in pb (5), G (15, symmetric adjoint) of the
// updated state; out the same for the predicted state, and the adjoints of
// the measurement
__device__ __forceinline__ void upd_adj(const Upd& U, float cb, float* pb, float* G, float& myb,
                                        float& mzb)
{
    // reverse-mode arithmetic: compared with the float64 adjoint within a
    // tolerance, so products and sums may contract into fused multiply-adds
#pragma clang fp contract(fast)
    float Kb0[5], Kb1[5];
    float rb0 = 0.0f, rb1 = 0.0f;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        Kb0[i] = pb[i] * U.r0;
        Kb1[i] = pb[i] * U.r1;
        rb0 += U.K0[i] * pb[i];
        rb1 += U.K1[i] * pb[i];
    }
    // M = G A (5x2)
    float M0[5], M1[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        float m0 = 0.0f, m1 = 0.0f;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const float gij = G[lt(i, j)];
            m0 += gij * U.A0[j];
            m1 += gij * U.A1[j];
        }
        M0[i] = m0;
        M1[i] = m1;
    }
    // Ab = -2 M B + Kb B ; Bb = -A^T M + A^T Kb + cb r r^T
    float Ab0[5], Ab1[5];
    float Bb00 = cb * U.r0 * U.r0, Bb01 = cb * U.r0 * U.r1, Bb10 = Bb01, Bb11 = cb * U.r1 * U.r1;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const float e0 = Kb0[i] - 2.0f * M0[i], e1 = Kb1[i] - 2.0f * M1[i];
        Ab0[i] = e0 * U.B00 + e1 * U.B10;
        Ab1[i] = e0 * U.B10 + e1 * U.B11;
        const float f0 = Kb0[i] - M0[i], f1 = Kb1[i] - M1[i];
        Bb00 += U.A0[i] * f0;
        Bb01 += U.A0[i] * f1;
        Bb10 += U.A1[i] * f0;
        Bb11 += U.A1[i] * f1;
    }
    // r: chi2 term
    rb0 += 2.0f * cb * (U.B00 * U.r0 + U.B10 * U.r1);
    rb1 += 2.0f * cb * (U.B10 * U.r0 + U.B11 * U.r1);
    // S adjoint: -B sym(Bb) B
    const float s00 = Bb00, s11 = Bb11, s01 = 0.5f * (Bb01 + Bb10);
    const float t00 = U.B00 * s00 + U.B10 * s01, t01 = U.B00 * s01 + U.B10 * s11;
    const float t10 = U.B10 * s00 + U.B11 * s01, t11 = U.B10 * s01 + U.B11 * s11;
    const float Sb00 = -(t00 * U.B00 + t01 * U.B10);
    const float Sb10 = -(t10 * U.B00 + t11 * U.B10);
    const float Sb11 = -(t10 * U.B10 + t11 * U.B11);
    G[0] += Sb00;
    G[1] += Sb10;
    G[2] += Sb11;
    // A = C[:, 0:2], symmetric embedding
    G[0] += Ab0[0];
    G[2] += Ab1[1];
    G[1] += 0.5f * (Ab0[1] + Ab1[0]);
#pragma unroll
    for (int i = 2; i < 5; ++i) {
        G[lt(i, 0)] += 0.5f * Ab0[i];
        G[lt(i, 1)] += 0.5f * Ab1[i];
    }
    myb = rb0;
    mzb = rb1;
    pb[0] -= rb0;
    pb[1] -= rb1;
}

// adjoint of the transport: in pb, G of the transported state; out those of
// the state before it (p0: that state), and the step-length adjoint
__device__ __forceinline__ float prop_adj(const Prop& P, const float* p0, const float* C0,
                                          float curv, float* pb, float* G)
{
    // reverse-mode arithmetic: compared with the float64 adjoint within a
    // tolerance, so products and sums may contract into fused multiply-adds
#pragma clang fp contract(fast)
    const float s = p0[2], t = p0[3];
    // F-bar = 2 G F C for the six free entries
    auto gfc = [&](int a, int b) {
        float v = 0.0f;
#pragma unroll
        for (int j = 0; j < 5; ++j) v += G[lt(a, j)] * P.FC[j][b];
        return 2.0f * v;
    };
    const float Fys = gfc(0, 2), Fyw = gfc(0, 4), Fzs = gfc(1, 2), Fzt = gfc(1, 3),
                Fzw = gfc(1, 4), Fsw = gfc(2, 4);
    // G <- F^T G F
    float E[5][5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const float g0 = G[lt(i, 0)], g1 = G[lt(i, 1)], g2 = G[lt(i, 2)];
        E[i][0] = g0;
        E[i][1] = g1;
        E[i][2] = g2 + g0 * P.ys + g1 * P.zs;
        E[i][3] = G[lt(i, 3)] + g1 * P.zt;
        E[i][4] = G[lt(i, 4)] + g0 * P.yw + g1 * P.zw + g2 * P.sw;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            float v = E[i][j];
            if (i == 2) v += P.ys * E[0][j] + P.zs * E[1][j];
            if (i == 3) v += P.zt * E[1][j];
            if (i == 4) v += P.yw * E[0][j] + P.zw * E[1][j] + P.sw * E[2][j];
            G[lt(i, j)] = v;
        }
    }
    (void)C0;
    // state part: y' = y + dx T, z' = z + t S, s' = s2, t' = t, w' = w
    float Tb = pb[0] * P.dx, dxb = pb[0] * P.T, Sb = pb[1] * t, s2b = pb[2];
    float tb = pb[3] + pb[1] * P.S, wb = pb[4];
    // Jacobian entries
    const float m1 = P.G1 * P.LT;
    float Tsb = 0.0f, Twb = 0.0f, m1b = 0.0f, Skb = 0.0f, kdxb = 0.0f;
    dxb += Fys * P.Ts;
    Tsb += Fys * P.dx;
    dxb += Fyw * P.Tw;
    Twb += Fyw * P.dx;
    tb += Fzs * m1 * P.Ts;
    m1b += Fzs * t * P.Ts;
    Tsb += Fzs * t * m1;
    Sb += Fzt;
    tb += Fzw * (m1 * P.Tw + P.Sk * curv);
    m1b += Fzw * t * P.Tw;
    Twb += Fzw * t * m1;
    Skb += Fzw * t * curv;
    kdxb += Fsw;
    const float G1b = m1b * P.LT;
    float LTb = m1b * P.G1;
    // Sk = L^2 a h(a2)
    const float h = (1.0f / 6.0f) + P.a2 * ((3.0f / 20.0f) + P.a2 * (15.0f / 112.0f));
    const float hp = (3.0f / 20.0f) + 2.0f * P.a2 * (15.0f / 112.0f);
    float Lb = Skb * 2.0f * P.L * P.a * h;
    float ab = Skb * P.L * P.L * h;
    float a2b = Skb * P.L * P.L * P.a * hp;
    // G1 = 1 + a2 (1/2 + a2 (3/8 + a2 5/16))
    a2b += G1b * (0.5f + P.a2 * (2.0f * (3.0f / 8.0f) + P.a2 * (3.0f * (5.0f / 16.0f))));
    // the reverse sweep divides by four quantities only: their reciprocals
    // once (the gradient is compared within a tolerance, not bit for bit,
    // and a correctly rounded division costs a dozen instructions)
    const float iq = 1.0f / P.q, icc = 1.0f / P.cc, ic1 = 1.0f / P.c1, ic2 = 1.0f / P.c2;
    // LT = dx T / q
    dxb += LTb * P.T * iq;
    Tb += LTb * P.dx * iq;
    float qb = -LTb * P.dx * P.T * (iq * iq);
    // Tw = kdx n / cc, n = 1 + T s2 / c2
    const float n = 1.0f + P.T * (P.s2 * ic2);
    kdxb += Twb * n * icc;
    const float nb = Twb * P.kdx * icc;
    float ccb = -Twb * P.Tw * icc;
    Tb += nb * P.s2 * ic2;
    s2b += nb * P.T * ic2;
    float c2b = -nb * P.T * P.s2 * (ic2 * ic2);
    // kdx = curv dx
    dxb += kdxb * curv;
    // Ts = (2 + T e) / cc, e = s/c1 + s2/c2
    const float e = s * ic1 + P.s2 * ic2;
    const float numb = Tsb * icc;
    ccb += -Tsb * P.Ts * icc;
    Tb += numb * e;
    const float eb = numb * P.T;
    float sb = eb * ic1;
    float c1b = -eb * s * (ic1 * ic1);
    s2b += eb * ic2;
    c2b += -eb * P.s2 * (ic2 * ic2);
    // S = L g, g = 1 + a2 (1/6 + a2 (3/40 + a2 5/112))
    Lb += Sb * P.g;
    const float gb = Sb * P.L;
    a2b += gb * ((1.0f / 6.0f) + P.a2 * (2.0f * (3.0f / 40.0f) + P.a2 * (3.0f * (5.0f / 112.0f))));
    // a2 = a^2 ; a = k L / 2
    ab += a2b * 2.0f * P.a;
    float kb = ab * 0.5f * P.L;
    Lb += ab * 0.5f * P.k;
    // L = dx q ; q = sqrt(1 + T^2)
    dxb += Lb * P.q;
    qb += Lb * P.dx;
    Tb += qb * P.T * iq;
    // T = (s + s2) / cc ; cc = c1 + c2
    sb += Tb * icc;
    s2b += Tb * icc;
    ccb += -Tb * P.T * icc;
    c1b += ccb;
    c2b += ccb;
    s2b += c2b * (-P.s2 * ic2);
    sb += c1b * (-s * ic1);
    // s2 = s + k dx ; k = curv w
    sb += s2b;
    kb += s2b * P.dx;
    dxb += s2b * P.k;
    wb += kb * curv;
    pb[0] = pb[0];        // y' = y + ...: dy'/dy = 1
    pb[1] = pb[1];        // z' = z + ...
    pb[2] = sb;
    pb[3] = tb;
    pb[4] = wb;
    return dxb;
}

// Checkpoints are kept in tiles of 64 tracks (one wave): slot i of the
// track in lane l of tile g holds 20 floats (p, C) as five float4 at
// ck4[((g * n_rows + i) * 5 + q) * 64 + l].  The lanes of a wave that stand
// at the same slot store and load five contiguous 1 KB blocks, and one
// wave's checkpoints are one contiguous block.
__device__ __forceinline__ float4* ck_tile(float* ck, int64_t t, int n_rows)
{
    return reinterpret_cast<float4*>(ck) + (t / kWave) * (int64_t)n_rows * 5 * kWave +
           (t & (kWave - 1));
}

__device__ __forceinline__ void store_ck(float4* o, int i, const float* p, const float* C)
{
    o += (int64_t)i * 5 * kWave;
    o[0 * kWave] = make_float4(p[0], p[1], p[2], p[3]);
    o[1 * kWave] = make_float4(p[4], C[0], C[1], C[2]);
    o[2 * kWave] = make_float4(C[3], C[4], C[5], C[6]);
    o[3 * kWave] = make_float4(C[7], C[8], C[9], C[10]);
    o[4 * kWave] = make_float4(C[11], C[12], C[13], C[14]);
}

__device__ __forceinline__ void load_ck(const float4* o, int i, float4* q)
{
    o += (int64_t)i * 5 * kWave;
#pragma unroll
    for (int k = 0; k < 5; ++k) q[k] = o[k * kWave];
}

__device__ __forceinline__ void unpack_ck(const float4* q, float* p, float* C)
{
    p[0] = q[0].x; p[1] = q[0].y; p[2] = q[0].z; p[3] = q[0].w;
    p[4] = q[1].x; C[0] = q[1].y; C[1] = q[1].z; C[2] = q[1].w;
    C[3] = q[2].x; C[4] = q[2].y; C[5] = q[2].z; C[6] = q[2].w;
    C[7] = q[3].x; C[8] = q[3].y; C[9] = q[3].z; C[10] = q[3].w;
    C[11] = q[4].x; C[12] = q[4].y; C[13] = q[4].z; C[14] = q[4].w;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const int w = __shfl_xor(v, o, kWave);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ void load_theta(const float* __restrict__ d_theta, float* th)
{
    if (threadIdx.x < 16) th[threadIdx.x] = d_theta[threadIdx.x];
    __syncthreads();
}

// ---- staging of a wave's hits through LDS ---------------------------------
// The 64 tracks of a wave are consecutive in the CSR, so hits [i0, i0 + K)
// of all of them are 64 short contiguous runs.  The wave loads them
// cooperatively (item e of a chunk: track e / K, hit i0 + e % K), K runs of
// K hits per load instruction instead of 64 scattered words, and each lane
// then reads its own hits from LDS.  Gradients leave the same way.
constexpr int kChunk = 8;

struct Stage {
    float x[kChunk][kWave];   // raw plane position of the hit's row
    float y[kChunk][kWave];
    float z[kChunk][kWave];
};

// stage hits [i0, i0 + kChunk) of the wave's tracks (a, n of each lane);
// flags a hit row >= n_rows in bad[lane of the track]
__device__ __forceinline__ void stage_hits(Stage& S, int* bad, int i0, int a, int n,
                                           const int32_t* __restrict__ idx,
                                           const uint8_t* __restrict__ row,
                                           const float* __restrict__ y,
                                           const float* __restrict__ z, const float* xs,
                                           int n_rows)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
        const int e = lane + kWave * j;
        const int l = e / kChunk, k = e % kChunk;
        const int al = __shfl(a, l, kWave), nl = __shfl(n, l, kWave);
        const int i = i0 + k;
        if (i < nl) {
            const int c = idx ? idx[al + i] : al + i;
            const int r = row[c];
            if (r >= n_rows) bad[l] = 1;
            S.x[k][l] = xs[r];
            S.y[k][l] = y[c];
            S.z[k][l] = z[c];
        }
    }
}

}  // namespace

// ---- tile order ---------------------------------------------------------------
// With a checkpoint buffer the tracks are taken in order of decreasing hit
// count (stable: equal counts in track order), so that the 64 tracks of a
// tile have similar lengths: a tile steps to its longest track, storing and
// loading whole checkpoint lines, and tiles of uniformly drawn lengths would
// otherwise move about 1.5 times the checkpoint bytes their tracks need.
// A counting sort by key (n_rows + 1) - min(n, n_rows + 1): per block of
// 256 tracks the key counts (one wave's equal keys found by nine ballots),
// an exclusive scan over (key, block), then every track's position.
constexpr int kOrdBlock = 256;

__device__ __forceinline__ int order_key(const int32_t* __restrict__ off, int64_t t, int n_rows)
{
    const int n = off[t + 1] - off[t];
    const int c = n < 0 ? 0 : n > n_rows + 1 ? n_rows + 1 : n;
    return n_rows + 1 - c;
}

// lanes of the wave holding the same key as this lane (keys below 512)
__device__ __forceinline__ uint64_t same_key(int key)
{
    uint64_t m = ~0ull;
#pragma unroll
    for (int b = 0; b < 9; ++b) {
        const uint64_t v = __ballot((key >> b) & 1);
        m &= ((key >> b) & 1) ? v : ~v;
    }
    return m;
}

// wc[w][key]: count of the key among wave w's tracks of the block
__device__ __forceinline__ void order_counts(const int32_t* __restrict__ off, int64_t nt,
                                             int n_rows, int nkeys, int (*wc)[256 + 2], int& key,
                                             int& rank)
{
    for (int i = threadIdx.x; i < (kOrdBlock / kWave) * nkeys; i += kOrdBlock)
        wc[i / nkeys][i % nkeys] = 0;
    __syncthreads();
    const int64_t t = blockIdx.x * (int64_t)kOrdBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    key = t < nt ? order_key(off, t, n_rows) : 511;   // 511: no track, no key
    const uint64_t m = same_key(key);
    rank = __popcll(m & ((1ull << lane) - 1ull));
    if (key != 511 && rank == 0) wc[threadIdx.x / kWave][key] = __popcll(m);
    __syncthreads();
}

__global__ __launch_bounds__(kOrdBlock) void k_order_count(const int32_t* __restrict__ off,
                                                           const int64_t* __restrict__ d_count,
                                                           int64_t n_tracks, int n_rows,
                                                           int32_t* __restrict__ cnt)
{
    __shared__ int wc[kOrdBlock / kWave][256 + 2];
    const int64_t nt = d_count && *d_count < n_tracks ? *d_count : n_tracks;
    const int nkeys = n_rows + 2;
    int key, rank;
    order_counts(off, nt, n_rows, nkeys, wc, key, rank);
    for (int k = threadIdx.x; k < nkeys; k += kOrdBlock) {
        int c = 0;
#pragma unroll
        for (int w = 0; w < kOrdBlock / kWave; ++w) c += wc[w][k];
        cnt[(int64_t)k * gridDim.x + blockIdx.x] = c;
    }
}

// after the scan of cnt: position of every track t < nt, order[pos] = t
__global__ __launch_bounds__(kOrdBlock) void k_order_place(const int32_t* __restrict__ off,
                                                           const int64_t* __restrict__ d_count,
                                                           int64_t n_tracks, int n_rows,
                                                           const int32_t* __restrict__ base,
                                                           int32_t* __restrict__ order)
{
    __shared__ int wc[kOrdBlock / kWave][256 + 2];
    const int64_t nt = d_count && *d_count < n_tracks ? *d_count : n_tracks;
    int key, rank;
    order_counts(off, nt, n_rows, n_rows + 2, wc, key, rank);
    if (key == 511) return;
    int pos = base[(int64_t)key * gridDim.x + blockIdx.x] + rank;
    for (int w = 0; w < (int)(threadIdx.x / kWave); ++w) pos += wc[w][key];
    order[pos] = (int32_t)(blockIdx.x * (int64_t)kOrdBlock + threadIdx.x);
}

// track of tile position q (q itself past the count, or without an order)
__device__ __forceinline__ int64_t track_at(const int32_t* __restrict__ order, int64_t q,
                                            int64_t nt)
{
    return order && q < nt ? (int64_t)order[q] : q;
}

__global__ __launch_bounds__(kWave) void k_refit_fwd(
    const int32_t* __restrict__ off, const int32_t* __restrict__ idx,
    const uint8_t* __restrict__ row, const float* __restrict__ y, const float* __restrict__ z,
    const int8_t* __restrict__ side, const int64_t* __restrict__ d_count, int64_t n_tracks,
    int n_rows,
    const float* __restrict__ row_x, tpc_params prm, CalibModel cm,
    const float* __restrict__ d_theta, float* __restrict__ par, float* __restrict__ cov,
    float* __restrict__ chi2_out, int32_t* __restrict__ status, float* __restrict__ ck,
    const int32_t* __restrict__ order)
{
    __shared__ float th[16];
    __shared__ float xs[256];
    __shared__ Stage S;
    __shared__ int bad[kWave];
    load_theta(d_theta, th);
    for (int i = threadIdx.x; i < n_rows; i += blockDim.x) xs[i] = row_x[i];
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t nt = d_count && *d_count < n_tracks ? *d_count : n_tracks;
    // one wave per tile of 64 tracks (consecutive in the tile order)
    for (int64_t tb = blockIdx.x * (int64_t)kWave; tb < nt; tb += (int64_t)gridDim.x * kWave) {
        const int64_t t = track_at(order, tb + lane, nt);
        int a = 0, n = 0;
        if (t < nt) {
            a = off[t];
            n = off[t + 1] - a;
        }
        // tracks filtered: at least 3 hits, not more hits than rows (a hit
        // row outside the table is found while staging)
        const bool fit = t < nt && n >= 3 && n <= n_rows;
        const int M = wave_max(t < nt && n >= 3 ? n : 0);
        bad[lane] = 0;
        float p[5] = {0, 0, 0, 0, 0}, C[15];
#pragma unroll
        for (int i = 0; i < 15; ++i) C[i] = 0.0f;
        float chi2 = 0.0f, xp = 0.0f;
        bool alive = fit;
        int stat = 0;
        const float sd = t < nt && side ? (float)side[t] : 1.0f;
        // every lane of a tile stores every slot up to the wave's longest
        // track (a lane past its own track stores its unchanged state, which
        // nothing reads), so that each store writes whole lines; the tile of
        // the last, partial wave is allocated in full
        float4* ckt = ck ? ck_tile(ck, tb + lane, n_rows) : nullptr;
        const int M_ck = M < n_rows ? M : n_rows;
        for (int i0 = 0; i0 < M; i0 += kChunk) {
            __syncthreads();      // the previous chunk is consumed
            stage_hits(S, bad, i0, a, t < nt && n >= 3 ? n : 0, idx, row, y, z, xs, n_rows);
            __syncthreads();
            if (i0 == 0 && alive) {
                // state from the first and third hits
                const CalHit h0 = calibrate(th, S.x[0][lane], S.y[0][lane], S.z[0][lane], sd, cm);
                const CalHit h2 = calibrate(th, S.x[2][lane], S.y[2][lane], S.z[2][lane], sd, cm);
                const float dX = h2.x - h0.x;
                const float T0 = (h2.y - h0.y) / dX;
                const float q0 = sqrtf(1.0f + T0 * T0);
                p[0] = h0.y;
                p[1] = h0.z;
                p[2] = T0 / q0;
                p[3] = (h2.z - h0.z) / (dX * q0);
                p[4] = 0.0f;
                C[0] = prm.sigma_y2;
                C[2] = prm.sigma_z2;
                C[5] = prm.c_ss0;
                C[9] = prm.c_tt0;
                C[14] = prm.c_ww0;
                xp = h0.x;
            }
            if (i0 == 0 && ckt && M_ck > 1) store_ck(ckt, 0, p, C);
            const int i_hi = i0 + kChunk < M ? i0 + kChunk : M;
            for (int i = i0 > 1 ? i0 : 1; i < i_hi; ++i) {
                if (alive && i < n) {
                    const int k = i - i0;
                    const CalHit h =
                        calibrate(th, S.x[k][lane], S.y[k][lane], S.z[k][lane], sd, cm);
                    Prop P;
                    if (prop_fwd(p, C, h.x - xp, prm.curv, prm.s_max, P)) {
                        Upd U;
                        chi2 += upd_fwd(p, C, h.y, h.z, prm.sigma_y2, prm.sigma_z2, U);
                        xp = h.x;
                    } else {
                        stat = 2;
                        alive = false;
                    }
                }
                if (ckt && i + 1 < M_ck) store_ck(ckt, i, p, C);
            }
        }
        __syncthreads();
        if (t < nt) {
            if (n < 3) stat = 1;
            else if (bad[lane]) stat = 3;
            else if (n > n_rows) stat = 4;
            if (stat == 1 || stat == 3 || stat == 4) {
                chi2 = 0.0f;
#pragma unroll
                for (int i = 0; i < 5; ++i) p[i] = 0.0f;
#pragma unroll
                for (int i = 0; i < 15; ++i) C[i] = 0.0f;
            }
#pragma unroll
            for (int i = 0; i < 5; ++i) par[t * 5 + i] = p[i];
#pragma unroll
            for (int i = 0; i < 15; ++i) cov[t * 15 + i] = C[i];
            chi2_out[t] = chi2;
            status[t] = stat;
        }
    }
}

__global__ __launch_bounds__(kWave) void k_refit_adj(
    const int32_t* __restrict__ off, const int32_t* __restrict__ idx,
    const uint8_t* __restrict__ row, const float* __restrict__ y, const float* __restrict__ z,
    const int8_t* __restrict__ side, const int64_t* __restrict__ d_count, int64_t n_tracks,
    int n_rows,
    const float* __restrict__ row_x, tpc_params prm, CalibModel cm,
    const float* __restrict__ d_theta, const float* __restrict__ ck,
    const int32_t* __restrict__ status, const float* __restrict__ gchi2,
    const float* __restrict__ seed_p, const float* __restrict__ seed_x,
    float* __restrict__ gy, float* __restrict__ gz, double* __restrict__ partials,
    const int32_t* __restrict__ order)
{
    __shared__ float th[16];
    __shared__ float xs[256];
    __shared__ Stage S;
    __shared__ float Gy[kChunk][kWave], Gz[kChunk][kWave];
    __shared__ int bad[kWave];
    load_theta(d_theta, th);
    for (int i = threadIdx.x; i < n_rows; i += blockDim.x) xs[i] = row_x[i];
    __syncthreads();
    double gth[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) gth[k] = 0.0;
    const int64_t nt = d_count && *d_count < n_tracks ? *d_count : n_tracks;
    const int lane = threadIdx.x & (kWave - 1);
    // one wave per tile of 64 tracks; the reverse sweep runs over the slots
    // of the tile in lockstep (slot i is active in the lanes whose track has
    // more than i hits), so that checkpoint loads are whole lines; hits come
    // through LDS in chunks, from the top down
    for (int64_t tb = blockIdx.x * (int64_t)kWave; tb < nt; tb += (int64_t)gridDim.x * kWave) {
        const int64_t t = track_at(order, tb + lane, nt);
        int a = 0, n = 0;
        if (t < nt) {
            a = off[t];
            n = off[t + 1] - a;
        }
        const bool fit = t < nt && n >= 3 && status[t] == 0;
        if (t < nt && !fit)
            for (int i = 0; i < n; ++i) {
                gy[a + i] = 0.0f;
                gz[a + i] = 0.0f;
            }
        const int ne = fit ? n : 0;
        const int M = wave_max(ne);
        if (M == 0) continue;
        HitRef H{idx, row, y, z, a};
        const float4* ckt = ck_tile(const_cast<float*>(ck), tb + lane, n_rows);
        const float sd = fit && side ? (float)side[t] : 1.0f;
        const float cb = fit ? gchi2[t] : 0.0f;
        // adjoint of the final state: the seed of the caller's terms in the
        // state after the last update (dL/dp), zero without one
        float pb[5] = {0, 0, 0, 0, 0}, G[15];
        if (fit && seed_p)
#pragma unroll
            for (int i = 0; i < 5; ++i) pb[i] = seed_p[t * 5 + i];
#pragma unroll
        for (int i = 0; i < 15; ++i) G[i] = 0.0f;
        CalHit cur{};
        // checkpoint of the coming step (slot i - 1), loaded a step ahead
        float4 ck4[5];
        if (fit) {
            cur = H.cal(n - 1, th, xs, sd, cm);
            load_ck(ckt, n - 2, ck4);
        }
        // dL/dx of the last hit's calibrated plane from the caller's terms
        float Xcarry = fit && seed_x ? seed_x[t] : 0.0f;
        float X2 = 0.0f, Y2 = 0.0f, Z2 = 0.0f;
        // steps i = top .. lo need hits lo - 1 .. top - 1 (the previous hit)
        for (int top = M - 1; top >= 1;) {
            const int lo = top - kChunk + 1 > 1 ? top - kChunk + 1 : 1;
            __syncthreads();
            stage_hits(S, bad, lo - 1, a, ne, idx, row, y, z, xs, n_rows);
            __syncthreads();
            for (int i = top; i >= lo; --i) {
                if (i >= ne) continue;
                const int k = i - lo;             // slot of hit i - 1
                const CalHit prev = calibrate(th, S.x[k][lane], S.y[k][lane], S.z[k][lane], sd, cm);
                float p[5], C[15];
                unpack_ck(ck4, p, C);
                if (i >= 2) load_ck(ckt, i - 2, ck4);
                const float p0[5] = {p[0], p[1], p[2], p[3], p[4]};
                Prop P;
                prop_fwd(p, C, cur.x - prev.x, prm.curv, prm.s_max, P);
                Upd U;
                upd_fwd(p, C, cur.y, cur.z, prm.sigma_y2, prm.sigma_z2, U);
                float myb, mzb;
                upd_adj(U, cb, pb, G, myb, mzb);
                const float dxb = prop_adj(P, p0, nullptr, prm.curv, pb, G);
                const float Xi = Xcarry + dxb;
                if (i == 2) {
                    X2 = Xi;
                    Y2 = myb;
                    Z2 = mzb;
                } else {
                    float gyr, gzr;
                    calibrate_adj(th, cur, sd, cm, Xi, myb, mzb, gth, gyr, gzr);
                    Gy[i - lo][lane] = gyr;
                    Gz[i - lo][lane] = gzr;
                }
                Xcarry = -dxb;
                cur = prev;
            }
            __syncthreads();
            // write the chunk's hit gradients (hits lo .. top, but hit 2),
            // the same runs as the staging
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                const int e = lane + kWave * j;
                const int l = e / kChunk, kk = e % kChunk;
                const int al = __shfl(a, l, kWave), nl = __shfl(ne, l, kWave);
                const int i = lo + kk;
                if (i <= top && i < nl && i != 2) {
                    gy[al + i] = Gy[kk][l];
                    gz[al + i] = Gz[kk][l];
                }
            }
            top = lo - 1;
        }
        if (!fit) continue;
        // initial state: y, z of hit 0, direction from hit 0 to hit 2
        const CalHit h0 = cur;
        const CalHit h2 = H.cal(2, th, xs, sd, cm);
        const float dX = h2.x - h0.x;
        const float T0 = (h2.y - h0.y) / dX;
        const float q0 = sqrtf(1.0f + T0 * T0);
        const float tt = (h2.z - h0.z) / (dX * q0);
        float Y0 = pb[0], Z0 = pb[1], X0 = Xcarry;
        float T0b = pb[2] / (q0 * q0 * q0);
        const float den = dX * q0;
        Z2 += pb[3] / den;
        Z0 -= pb[3] / den;
        const float denb = -pb[3] * tt / den;
        float dXb = denb * q0;
        const float q0b = denb * dX;
        T0b += q0b * T0 / q0;
        Y2 += T0b / dX;
        Y0 -= T0b / dX;
        dXb -= T0b * T0 / dX;
        X2 += dXb;
        X0 -= dXb;
        float gyr, gzr;
        calibrate_adj(th, h0, sd, cm, X0, Y0, Z0, gth, gyr, gzr);
        gy[a] = gyr;
        gz[a] = gzr;
        calibrate_adj(th, h2, sd, cm, X2, Y2, Z2, gth, gyr, gzr);
        gy[a + 2] = gyr;
        gz[a + 2] = gzr;
    }
    // deterministic wave reduction of the theta adjoint (one wave per block)
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        double v = gth[k];
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
        if (lane == k) partials[blockIdx.x * 16 + k] = v;
    }
}

// sum of the per-block partials in a fixed order: block k sums parameter k;
// thread j adds partials j, j + 256, ... of it, then a fixed tree
__global__ __launch_bounds__(kBlock) void k_reduce_theta(const double* __restrict__ partials,
                                                         int nb, float* __restrict__ out)
{
    __shared__ double red[kBlock];
    const int k = blockIdx.x;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) v += partials[b * 16 + k];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = (float)red[0];
}

// Beam-axis term of the calibration objective (section 3's online
// calibration with section 2's primaries from the origin): the refit state of
// a track's last hit (par, cov at the calibrated plane of that hit) is
// transported to the plane x = 0 of its sector frame, which holds the beam
// axis, in ceil(x / 20 cm) equal steps; r = (y0, z0) there and
// loss = r^T W r, with W = S^-1, S the transported (y, z) covariance plus
// sigma_v^2 on the diagonal (the chi2 increment of a vertex measurement) --
// or W given by the caller (w_in: held fixed while the calibration moves).
// Derivatives: with respect to the state through the product of the step
// Jacobians, and to the plane of the last hit (moving the plane with the
// state held translates the track along x: dr/dx = -(s0, t) / c0 at the axis
// plane).  Zero (ok = 0) for tracks without a fit or whose transport stops.
// One thread per track.
__global__ __launch_bounds__(kBlock) void k_vertex_residual(
    const int32_t* __restrict__ off, const int32_t* __restrict__ idx,
    const uint8_t* __restrict__ row, const float* __restrict__ y, const float* __restrict__ z,
    const int8_t* __restrict__ side, const int64_t* __restrict__ d_count, int64_t n_tracks,
    const float* __restrict__ row_x, tpc_params prm, CalibModel cm,
    const float* __restrict__ d_theta, const float* __restrict__ par,
    const float* __restrict__ cov, const int32_t* __restrict__ status, float sv2,
    const float* __restrict__ w_in, float* __restrict__ w_out, float* __restrict__ loss,
    float* __restrict__ seed_p, float* __restrict__ seed_x, int8_t* __restrict__ ok)
{
    __shared__ float th[16];
    if (threadIdx.x < 16) th[threadIdx.x] = d_theta[threadIdx.x];
    __syncthreads();
    const int64_t nt = d_count && *d_count < n_tracks ? *d_count : n_tracks;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nt;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int a = off[t], n = off[t + 1] - a;
        float l = 0.0f, gx = 0.0f, gp[5] = {0, 0, 0, 0, 0}, w[3] = {0, 0, 0};
        bool good = status[t] == 0 && n >= 3;
        if (good) {
            const HitRef H{idx, row, y, z, a};
            const int c = H.cl(n - 1);
            const float sd = side ? (float)side[t] : 1.0f;
            const float xl = calibrate(th, row_x[row[c]], y[c], z[c], sd, cm).x;
            float p[5], C[15];
#pragma unroll
            for (int i = 0; i < 5; ++i) p[i] = par[t * 5 + i];
#pragma unroll
            for (int i = 0; i < 15; ++i) C[i] = cov[t * 15 + i];
            // rows y, z, sin of the accumulated Jacobian d(p at x)/d(p at xl)
            float J0[5] = {1, 0, 0, 0, 0}, J1[5] = {0, 1, 0, 0, 0}, J2[5] = {0, 0, 1, 0, 0};
            int n_step = (int)ceilf(xl / 20.0f);
            if (n_step < 1) n_step = 1;
            const float dx = (0.0f - xl) / (float)n_step;
            for (int i = 0; i < n_step && good; ++i) {
                Prop P;
                if (!prop_fwd(p, C, dx, prm.curv, prm.s_max, P)) {
                    good = false;
                    break;
                }
                // rows 3, 4 of every step Jacobian are those of the identity
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const float e3 = k == 3 ? 1.0f : 0.0f, e4 = k == 4 ? 1.0f : 0.0f;
                    const float n0 = J0[k] + P.ys * J2[k] + P.yw * e4;
                    const float n1 = J1[k] + P.zs * J2[k] + P.zt * e3 + P.zw * e4;
                    J2[k] = J2[k] + P.sw * e4;
                    J0[k] = n0;
                    J1[k] = n1;
                }
            }
            if (good) {
                if (w_in) {
                    w[0] = w_in[t * 3];
                    w[1] = w_in[t * 3 + 1];
                    w[2] = w_in[t * 3 + 2];
                } else {
                    const float s00 = C[0] + sv2, s10 = C[1], s11 = C[2] + sv2;
                    const float det = s00 * s11 - s10 * s10;
                    w[0] = s11 / det;
                    w[1] = -s10 / det;
                    w[2] = s00 / det;
                }
                const float y0 = p[0], z0 = p[1];
                const float u0 = w[0] * y0 + w[1] * z0, u1 = w[1] * y0 + w[2] * z0;
                l = y0 * u0 + z0 * u1;
#pragma unroll
                for (int k = 0; k < 5; ++k) gp[k] = 2.0f * (u0 * J0[k] + u1 * J1[k]);
                const float c0 = sqrtf((1.0f - p[2]) * (1.0f + p[2]));
                gx = -2.0f * (u0 * p[2] + u1 * p[3]) / c0;
            }
        }
        loss[t] = l;
#pragma unroll
        for (int k = 0; k < 5; ++k) seed_p[t * 5 + k] = gp[k];
        seed_x[t] = gx;
        if (w_out) {
            w_out[t * 3] = w[0];
            w_out[t * 3 + 1] = w[1];
            w_out[t * 3 + 2] = w[2];
        }
        if (ok) ok[t] = good ? 1 : 0;
    }
}

constexpr int64_t kRefitMaxBlocks = 16384;

static unsigned refit_grid(int64_t n_tracks)
{
    return grid_for_block(n_tracks, kWave, kRefitMaxBlocks);
}

// The checkpoint buffer: the tiles, then the tile order (int32 per track),
// the per-(key, block) counts of the ordering and its scan partials.
struct CkLayout {
    size_t order_off, cnt_off, part_off, total;
    int64_t nblk;
    int nkeys;
};

static size_t ck_align(size_t v) { return (v + 255) & ~(size_t)255; }

static CkLayout ck_layout(int64_t n_tracks, int n_rows)
{
    CkLayout L;
    const int64_t tiles = (n_tracks + kWave - 1) / kWave;
    L.nblk = ceil_div(n_tracks > 0 ? n_tracks : 1, kOrdBlock);
    L.nkeys = n_rows + 2;
    const int64_t ncnt = L.nblk * L.nkeys;
    L.order_off = ck_align(sizeof(float) * (size_t)tiles * kWave * (size_t)n_rows * 20);
    L.cnt_off = L.order_off + ck_align(sizeof(int32_t) * (size_t)(n_tracks > 0 ? n_tracks : 1));
    L.part_off = L.cnt_off + ck_align(sizeof(int32_t) * (size_t)ncnt);
    L.total = L.part_off + sizeof(int64_t) * (size_t)(ceil_div(ncnt, kScanTile) + 1);
    return L;
}

static const int32_t* ck_order(const float* ck, int64_t n_tracks, int n_rows)
{
    return reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(ck) +
                                            ck_layout(n_tracks, n_rows).order_off);
}

// the tile order of the forward pass, into the checkpoint buffer
static void launch_order(const tpc_track_hits& hits, int n_rows, float* ck, hipStream_t st)
{
    const CkLayout L = ck_layout(hits.n_tracks, n_rows);
    char* b = reinterpret_cast<char*>(ck);
    int32_t* order = reinterpret_cast<int32_t*>(b + L.order_off);
    int32_t* cnt = reinterpret_cast<int32_t*>(b + L.cnt_off);
    int64_t* part = reinterpret_cast<int64_t*>(b + L.part_off);
    TPC_LAUNCH(k_order_count, dim3((unsigned)L.nblk), dim3(kOrdBlock), 0, st, hits.off,
               hits.d_count, hits.n_tracks, n_rows, cnt);
    launch_scan<int32_t>(cnt, cnt, L.nblk * L.nkeys, false, nullptr, nullptr, part, st);
    TPC_LAUNCH(k_order_place, dim3((unsigned)L.nblk), dim3(kOrdBlock), 0, st, hits.off,
               hits.d_count, hits.n_tracks, n_rows, (const int32_t*)cnt, order);
}

// the adjoint and its theta reduction, partials[16 * refit_grid(n_tracks)]
static int launch_refit_adjoint(tpc_track_hits hits, int32_t n_rows, const float* d_row_x,
                                const tpc_params& prm, const tpc_calib_model& m,
                                const float* d_theta, const float* checkpoints,
                                const int32_t* status, const float* grad_chi2,
                                const float* seed_p, const float* seed_x, float* grad_y,
                                float* grad_z, float* grad_theta, double* partials,
                                hipStream_t st)
{
    const CalibModel cm = make_calib(m);
    const unsigned nb = refit_grid(hits.n_tracks);
    TPC_LAUNCH(k_refit_adj, dim3(nb), dim3(kWave), 0, st, hits.off, hits.idx, hits.row, hits.y,
               hits.z, hits.side, hits.d_count, hits.n_tracks, n_rows, d_row_x, prm, cm,
               d_theta, checkpoints, status, grad_chi2, seed_p, seed_x, grad_y, grad_z, partials,
               ck_order(checkpoints, hits.n_tracks, n_rows));
    TPC_LAUNCH(k_reduce_theta, dim3(16), dim3(kBlock), 0, st, (const double*)partials, (int)nb,
               grad_theta);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // namespace tpc

// Theta partials of the adjoint's blocks for callers that cannot allocate
// (tpc_refit_adjoint_noalloc): one copy per GPU, held until the process
// ends, shared by every call on that GPU (calls that overlap on one GPU
// race on it).  Every block of the adjoint writes its 16 partials before the
// reduction reads them, so nothing needs clearing between calls.
static __device__ __align__(256) double scratch[16 * tpc::kRefitMaxBlocks];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices];   // device address of `scratch` per GPU

}  // namespace

namespace tpc {

// Device address of this GPU's copy of `scratch`, taken once per device at
// context creation with that device current (the array's name is only a
// host-side stand-in and cannot be passed to a kernel).
int refit_scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return TPC_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return TPC_OK;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return TPC_ERR_HIP;
    if (prev != device && hipSetDevice(device) != hipSuccess) return TPC_ERR_HIP;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !ptr) return TPC_ERR_HIP;
    g_scratch_ptr[device] = static_cast<double*>(ptr);
    return TPC_OK;
}

}  // namespace tpc

extern "C" {

int tpc_refit_workspace_size(int64_t n_tracks, size_t* h_bytes)
{
    if (!h_bytes || n_tracks < 0) return TPC_ERR_INVALID_ARG;
    *h_bytes = sizeof(double) * 16 * (size_t)tpc::refit_grid(n_tracks);
    return TPC_OK;
}

int tpc_refit_checkpoint_size(int64_t n_tracks, int32_t n_rows, size_t* h_bytes)
{
    if (!h_bytes || n_tracks < 0 || n_rows < 3 || n_rows > 255) return TPC_ERR_INVALID_ARG;
    *h_bytes = tpc::ck_layout(n_tracks, n_rows).total;
    return TPC_OK;
}

int tpc_refit(tpc_context* ctx, tpc_track_hits hits, int32_t n_rows, const float* d_row_x,
              const tpc_params* h_params, const tpc_calib_model* h_model, const float* d_theta,
              float* par, float* cov, float* chi2, int32_t* status, float* checkpoints,
              size_t ck_bytes, void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    if (!ctx || !h_params || !h_model || !d_theta || !d_row_x || !par || !cov || !chi2 ||
        !status || hits.n_tracks < 0 || hits.n_hits < 0 || n_rows < 3 || n_rows > 255 ||
        (hits.n_tracks > 0 && (!hits.off || !hits.row || !hits.y || !hits.z)) ||
        hits.n_hits >= (int64_t(1) << 31) || hits.n_tracks >= (int64_t(1) << 31))
        return TPC_ERR_INVALID_ARG;
    size_t ck_need = 0;
    if (checkpoints && (tpc_refit_checkpoint_size(hits.n_tracks, n_rows, &ck_need) ||
                        ck_bytes < ck_need))
        return TPC_ERR_INVALID_ARG;
    if (hits.n_tracks == 0) return TPC_OK;
    const tpc::CalibModel cm = tpc::make_calib(*h_model);
    hipStream_t st = (hipStream_t)stream;
    if (checkpoints) tpc::launch_order(hits, n_rows, checkpoints, st);
    TPC_LAUNCH(tpc::k_refit_fwd, dim3(tpc::refit_grid(hits.n_tracks)), dim3(tpc::kWave),
                       0, st, hits.off, hits.idx, hits.row, hits.y, hits.z,
                       hits.side, hits.d_count, hits.n_tracks, n_rows, d_row_x, *h_params, cm,
                       d_theta, par, cov, chi2, status, checkpoints,
                       checkpoints ? tpc::ck_order(checkpoints, hits.n_tracks, n_rows) : nullptr);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

int tpc_refit_adjoint(tpc_context* ctx, tpc_track_hits hits, int32_t n_rows,
                      const float* d_row_x, const tpc_params* h_params,
                      const tpc_calib_model* h_model, const float* d_theta,
                      const float* checkpoints, size_t ck_bytes, const int32_t* status,
                      const float* grad_chi2,
                      float* grad_y, float* grad_z, float* grad_theta, void* d_ws,
                      size_t ws_bytes, void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    size_t need = 0;
    if (!ctx || !h_params || !h_model || !d_theta || !d_row_x || !checkpoints || !status ||
        !grad_chi2 || !grad_y || !grad_z || !grad_theta || !d_ws || hits.n_tracks < 0 ||
        n_rows < 3 || n_rows > 255 ||
        (hits.n_tracks > 0 && (!hits.off || !hits.row || !hits.y || !hits.z)) ||
        tpc_refit_workspace_size(hits.n_tracks, &need) || need > ws_bytes ||
        tpc_refit_checkpoint_size(hits.n_tracks, n_rows, &need) || need > ck_bytes)
        return TPC_ERR_INVALID_ARG;
    return tpc::launch_refit_adjoint(hits, n_rows, d_row_x, *h_params, *h_model, d_theta,
                                     checkpoints, status, grad_chi2, nullptr, nullptr, grad_y,
                                     grad_z, grad_theta, (double*)d_ws, (hipStream_t)stream);
}

int tpc_refit_adjoint_seeded(tpc_context* ctx, tpc_track_hits hits, int32_t n_rows,
                             const float* d_row_x, const tpc_params* h_params,
                             const tpc_calib_model* h_model, const float* d_theta,
                             const float* checkpoints, size_t ck_bytes, const int32_t* status,
                             const float* grad_chi2, const float* grad_par, const float* grad_x,
                             float* grad_y, float* grad_z, float* grad_theta, void* d_ws,
                             size_t ws_bytes, void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    size_t need = 0;
    if (!ctx || !h_params || !h_model || !d_theta || !d_row_x || !checkpoints || !status ||
        !grad_chi2 || !grad_y || !grad_z || !grad_theta || !d_ws || hits.n_tracks < 0 ||
        n_rows < 3 || n_rows > 255 ||
        (hits.n_tracks > 0 && (!hits.off || !hits.row || !hits.y || !hits.z)) ||
        tpc_refit_workspace_size(hits.n_tracks, &need) || need > ws_bytes ||
        tpc_refit_checkpoint_size(hits.n_tracks, n_rows, &need) || need > ck_bytes)
        return TPC_ERR_INVALID_ARG;
    return tpc::launch_refit_adjoint(hits, n_rows, d_row_x, *h_params, *h_model, d_theta,
                                     checkpoints, status, grad_chi2, grad_par, grad_x, grad_y,
                                     grad_z, grad_theta, (double*)d_ws, (hipStream_t)stream);
}

int tpc_vertex_residual(tpc_context* ctx, tpc_track_hits hits, int32_t n_rows,
                        const float* d_row_x, const tpc_params* h_params,
                        const tpc_calib_model* h_model, const float* d_theta, const float* par,
                        const float* cov, const int32_t* status, float sigma_v,
                        const float* w_in, float* w_out, float* loss, float* grad_par,
                        float* grad_x, int8_t* ok, void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    if (!ctx || !h_params || !h_model || !d_theta || !d_row_x || !par || !cov || !status ||
        !loss || !grad_par || !grad_x || hits.n_tracks < 0 || n_rows < 3 || n_rows > 255 ||
        (hits.n_tracks > 0 && (!hits.off || !hits.row || !hits.y || !hits.z)) ||
        !(sigma_v >= 0.0f) || !std::isfinite(sigma_v))
        return TPC_ERR_INVALID_ARG;
    if (hits.n_tracks == 0) return TPC_OK;
    const tpc::CalibModel cm = tpc::make_calib(*h_model);
    TPC_LAUNCH(tpc::k_vertex_residual, dim3(tpc::grid_for(hits.n_tracks)), dim3(tpc::kBlock), 0,
               (hipStream_t)stream, hits.off, hits.idx, hits.row, hits.y, hits.z, hits.side,
               hits.d_count, hits.n_tracks, d_row_x, *h_params, cm, d_theta, par, cov, status,
               sigma_v * sigma_v, w_in, w_out, loss, grad_par, grad_x, ok);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

int tpc_refit_adjoint_noalloc(tpc_context* ctx, tpc_track_hits hits, int32_t n_rows,
                              const float* d_row_x, const tpc_params* h_params,
                              const tpc_calib_model* h_model, const float* d_theta,
                              const float* checkpoints, size_t ck_bytes, const int32_t* status,
                              const float* grad_chi2, float* grad_y, float* grad_z,
                              float* grad_theta, void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    size_t need = 0;
    if (!ctx || !h_params || !h_model || !d_theta || !d_row_x || !checkpoints || !status ||
        !grad_chi2 || !grad_y || !grad_z || !grad_theta || hits.n_tracks < 0 ||
        n_rows < 3 || n_rows > 255 ||
        (hits.n_tracks > 0 && (!hits.off || !hits.row || !hits.y || !hits.z)) ||
        tpc_refit_checkpoint_size(hits.n_tracks, n_rows, &need) || need > ck_bytes)
        return TPC_ERR_INVALID_ARG;
    if (tpc::refit_grid(hits.n_tracks) > tpc::kRefitMaxBlocks) return TPC_ERR_CAPACITY;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TPC_ERR_HIP;
    if (dev != ctx->device || dev < 0 || dev >= kMaxDevices) return TPC_ERR_INVALID_ARG;
    double* partials = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        partials = g_scratch_ptr[dev];
    }
    if (!partials) return TPC_ERR_HIP;   // set up when the context was created
    return tpc::launch_refit_adjoint(hits, n_rows, d_row_x, *h_params, *h_model, d_theta,
                                     checkpoints, status, grad_chi2, nullptr, nullptr, grad_y,
                                     grad_z, grad_theta, partials, (hipStream_t)stream);
}

}  // extern "C"
