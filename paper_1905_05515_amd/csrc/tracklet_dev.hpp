// Kalman-filter tracklet construction of one chain start (device code shared
// by the staged kernel and the persistent kernel).
//
// State at the sector-local plane x: (y, z, s = sin(phi), t = tan(lambda),
// w = q/pT), covariance as the lower triangle of the symmetric 5x5 matrix
// (i*(i+1)/2 + j).  In a uniform field along z the curvature k = curv * w is
// constant: s grows linearly with x, the y step is dx (s1 + s2)/(c1 + c2)
// with c = sqrt(1 - s^2), and the arc length over the step is
// chord * asin(a)/a, a = k chord / 2, expanded to a^6.  Every expression
// below keeps the association order of its comment's formula, and sums of
// products are written as explicit fused multiply-adds (fmaf, one
// rounding); with contraction off otherwise and IEEE division and square
// root the results are the same bits on any conforming implementation.
#pragma once
#include "tpc_internal.hpp"

namespace tpc {

__device__ __forceinline__ int lt(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

struct KState {
    float p[5];
    float C[15];
};

// Transport from plane x1 to x1 + dx.  Returns false (state untouched) when
// |sin(phi)| at either end of the step is not below s_max: at the far end
// the track turns back before the plane, at the near end an update has
// pushed the state out of the transport's domain (|s| >= 1 has no cosine).
__device__ __forceinline__ bool propagate(KState& st, float dx, float curv, float s_max)
{
    const float s = st.p[2], t = st.p[3], w = st.p[4];
    const float k = curv * w;
    const float s2 = fmaf(k, dx, s);
    if (!(fabsf(s) < s_max) || !(fabsf(s2) < s_max)) return false;
    const float c1 = sqrtf((1.0f - s) * (1.0f + s));
    const float c2 = sqrtf((1.0f - s2) * (1.0f + s2));
    const float cc = c1 + c2;
    const float icc = 1.0f / cc;   // one reciprocal for the three quotients by cc
    const float T = (s + s2) * icc;
    const float q = sqrtf(fmaf(T, T, 1.0f));
    const float L = dx * q;
    const float a = 0.5f * (k * L);
    const float a2 = a * a;
    const float g = fmaf(a2, fmaf(a2, fmaf(a2, 5.0f / 112.0f, 3.0f / 40.0f), 1.0f / 6.0f), 1.0f);
    const float S = L * g;
    const float Ts = fmaf(T, s / c1 + s2 / c2, 2.0f) * icc;
    const float kdx = curv * dx;
    const float Tw = (kdx * fmaf(T, s2 / c2, 1.0f)) * icc;
    const float LT = dx * (T / q);
    const float G1 = fmaf(a2, fmaf(a2, fmaf(a2, 5.0f / 16.0f, 3.0f / 8.0f), 0.5f), 1.0f);
    const float Sk = (L * (L * a)) * fmaf(a2, fmaf(a2, 15.0f / 112.0f, 3.0f / 20.0f), 1.0f / 6.0f);
    const float Fys = dx * Ts;
    const float Fyw = dx * Tw;
    const float Fzs = t * ((G1 * LT) * Ts);
    const float Fzt = S;
    const float Fzw = t * fmaf(Sk, curv, (G1 * LT) * Tw);
    const float Fsw = kdx;

    // B = F C, then C' = B F^T, sums over the non-zero entries of F in
    // increasing column order, each product added by a fused multiply-add
    float B[5][5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const float cy = st.C[lt(0, j)], cz = st.C[lt(1, j)], cs = st.C[lt(2, j)];
        const float ct = st.C[lt(3, j)], cw = st.C[lt(4, j)];
        B[0][j] = fmaf(Fyw, cw, fmaf(Fys, cs, cy));
        B[1][j] = fmaf(Fzw, cw, fmaf(Fzt, ct, fmaf(Fzs, cs, cz)));
        B[2][j] = fmaf(Fsw, cw, cs);
        B[3][j] = ct;
        B[4][j] = cw;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        st.C[lt(i, 0)] = fmaf(Fyw, B[i][4], fmaf(Fys, B[i][2], B[i][0]));
        if (i >= 1) st.C[lt(i, 1)] = fmaf(Fzw, B[i][4], fmaf(Fzt, B[i][3], fmaf(Fzs, B[i][2], B[i][1])));
        if (i >= 2) st.C[lt(i, 2)] = fmaf(Fsw, B[i][4], B[i][2]);
        if (i >= 3) st.C[lt(i, 3)] = B[i][3];
        if (i >= 4) st.C[lt(i, 4)] = B[i][4];
    }
    st.p[0] = fmaf(dx, T, st.p[0]);
    st.p[1] = fmaf(t, S, st.p[1]);
    st.p[2] = s2;
    return true;
}

__device__ __forceinline__ float chi2_pred(const KState& st, float my, float mz, float sy2, float sz2)
{
    const float r0 = my - st.p[0], r1 = mz - st.p[1];
    const float S00 = st.C[0] + sy2, S10 = st.C[1], S11 = st.C[2] + sz2;
    const float det = fmaf(S00, S11, -(S10 * S10));
    const float idet = 1.0f / det;
    const float B00 = S11 * idet, B10 = -(S10 * idet), B11 = S00 * idet;
    return fmaf(r1, fmaf(B11, r1, B10 * r0), r0 * fmaf(B10, r1, B00 * r0));
}

__device__ __forceinline__ float kupdate(KState& st, float my, float mz, float sy2, float sz2)
{
    const float r0 = my - st.p[0], r1 = mz - st.p[1];
    const float S00 = st.C[0] + sy2, S10 = st.C[1], S11 = st.C[2] + sz2;
    const float det = fmaf(S00, S11, -(S10 * S10));
    const float idet = 1.0f / det;
    const float B00 = S11 * idet, B10 = -(S10 * idet), B11 = S00 * idet;
    const float chi2 = fmaf(r1, fmaf(B11, r1, B10 * r0), r0 * fmaf(B10, r1, B00 * r0));
    float A0[5], A1[5], K0[5], K1[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        A0[i] = st.C[lt(i, 0)];
        A1[i] = st.C[lt(i, 1)];
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        K0[i] = fmaf(A1[i], B10, A0[i] * B00);
        K1[i] = fmaf(A1[i], B11, A0[i] * B10);
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        st.p[i] = st.p[i] + fmaf(K1[i], r1, K0[i] * r0);
#pragma unroll
        for (int j = 0; j <= i; ++j)
            st.C[lt(i, j)] = st.C[lt(i, j)] - fmaf(K1[i], A1[j], K0[i] * A0[j]);
    }
    return chi2;
}

__device__ __forceinline__ void reset_cov(KState& st, const tpc_params& prm)
{
#pragma unroll
    for (int i = 0; i < 15; ++i) st.C[i] = 0.0f;
    st.C[0] = prm.sigma_y2;
    st.C[2] = prm.sigma_z2;
    st.C[5] = prm.c_ss0;
    st.C[9] = prm.c_tt0;
    st.C[14] = prm.c_ww0;
}

constexpr int kCandBatch = 4;   // candidate loads issued together

// Hit of least predicted chi2 <= chi2_max on row r of sector s, ties to the
// lower cluster id; -1 if none, else its grid position with its coordinates
// in (my, mz).  The bins scanned cover +-nsigma of the prediction (every hit
// passing the gate lies inside); the gate decides.  Two z rows of bins are
// opened at a time so that their bin bounds load together.
__device__ __forceinline__ int search_row(const KState& st, const tpc_sector& s, int r,
                                          const tpc_params& prm, int& n_cand,
                                          const int32_t* __restrict__ bin_start,
                                          const float* __restrict__ yg,
                                          const float* __restrict__ zg,
                                          const int32_t* __restrict__ idg, float& my, float& mz)
{
    // The window only has to contain every hit the gate can accept: the
    // hardware square root (within 1 ulp) is far inside the 1/64 widening,
    // so it needs none of the correctly rounded sequence the decisions use.
    const float S00 = st.C[0] + prm.sigma_y2, S11 = st.C[2] + prm.sigma_z2;
    const float hy = prm.search_nsigma * __builtin_amdgcn_sqrtf(S00) * TPC_WIDEN + 0.01f;
    const float hz = prm.search_nsigma * __builtin_amdgcn_sqrtf(S11) * TPC_WIDEN + 0.01f;
    const int iy0 = bin_of(st.p[0] - hy, s.y0, s.inv_by, s.nby);
    const int iy1 = bin_of(st.p[0] + hy, s.y0, s.inv_by, s.nby);
    const int iz0 = bin_of(st.p[1] - hz, s.z0, s.inv_bz, s.nbz);
    const int iz1 = bin_of(st.p[1] + hz, s.z0, s.inv_bz, s.nbz);
    float best = 0.0f;
    int bpos = -1;
    for (int iz = iz0; iz <= iz1; iz += 2) {
        const int g = s.bin_base + (r * s.nbz + iz) * s.nby;
        int lo[2], hi[2];
        lo[0] = bin_start[g + iy0];
        hi[0] = bin_start[g + iy1 + 1];
        lo[1] = hi[1] = 0;
        if (iz + 1 <= iz1) {
            lo[1] = bin_start[g + s.nby + iy0];
            hi[1] = bin_start[g + s.nby + iy1 + 1];
        }
        // the candidates of both z rows as one stream (row iz first, each in
        // grid order: the order of evaluation decides nothing but ties,
        // which go to the lower id anyway), loaded kCandBatch at a time so
        // that one memory round trip serves several candidates
        const int n0 = hi[0] - lo[0] > 0 ? hi[0] - lo[0] : 0;
        const int n1 = hi[1] - lo[1] > 0 ? hi[1] - lo[1] : 0;
        n_cand += n0 + n1;
        for (int b = 0; b < n0 + n1; b += kCandBatch) {
            float yb[kCandBatch], zb[kCandBatch];
            int pb[kCandBatch];
#pragma unroll
            for (int j = 0; j < kCandBatch; ++j) {
                const int e = b + j;
                pb[j] = e < n0 ? lo[0] + e : lo[1] + (e - n0);
                if (e < n0 + n1) {
                    yb[j] = yg[pb[j]];
                    zb[j] = zg[pb[j]];
                }
            }
#pragma unroll
            for (int j = 0; j < kCandBatch; ++j) {
                if (b + j >= n0 + n1) break;
                const float c2 = chi2_pred(st, yb[j], zb[j], prm.sigma_y2, prm.sigma_z2);
                if (!(c2 <= prm.chi2_max)) continue;
                // equal chi2 (rare): the lower cluster id wins
                if (bpos < 0 || c2 < best || (c2 == best && idg[pb[j]] < idg[bpos])) {
                    best = c2;
                    bpos = pb[j];
                    my = yb[j];
                    mz = zb[j];
                }
            }
        }
    }
    return bpos;
}

// Build tracklet t (one thread).  xs holds the row positions; the hit list
// (grid position per row, -1 where none) goes to th[r * ths], which is either
// the tracklet's column of the [row][tracklet] output or a scratch column in
// LDS that the caller copies out.
//
// Up pass: from the start hit, one row at a time, the next hit is the next
// link of the chain while there is one (links always join adjacent rows),
// then the least-chi2 hit of a window search.  Down pass: from the outermost
// hit with the initial covariance, the hits already assigned are refitted and
// rows below the start are searched.  The loads of the next chain hit (up
// pass) and of the next assigned hit (down pass) are issued one row ahead.
__device__ __forceinline__ void build_tracklet(
    int64_t t, const tpc_sector* __restrict__ sec, int n_rows, const float* xs,
    const tpc_params& prm, const int32_t* __restrict__ bin_start, const float* __restrict__ yg,
    const float* __restrict__ zg, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ gsr, const int32_t* __restrict__ up,
    const int32_t* __restrict__ starts, int32_t* th, int64_t ths, int32_t* __restrict__ t_start,
    int32_t* __restrict__ t_nhits, int32_t* __restrict__ t_rin,
    float* __restrict__ t_par, float* __restrict__ t_cov, float* __restrict__ t_chi2,
    int& n_prop, int& n_upd, int& n_cand)
{
    const float sy2 = prm.sigma_y2, sz2 = prm.sigma_z2;
    for (int r = 0; r < n_rows; ++r) th[r * ths] = -1;
    const int h0 = starts[t];
    const int v0 = gsr[h0];
    const tpc_sector s = sec[v0 >> 8];
    const int r0 = v0 & 255;
    const int h1 = up[h0], h2 = up[h1];
    const int r2 = gsr[h2] & 255;
    KState st;
    {   // state from the first and third chain hits
        const float dX = xs[r2] - xs[r0];
        const float T0 = (yg[h2] - yg[h0]) / dX;
        const float q0 = sqrtf(1.0f + T0 * T0);
        st.p[0] = yg[h0];
        st.p[1] = zg[h0];
        st.p[2] = T0 / q0;
        st.p[3] = (zg[h2] - zg[h0]) / (dX * q0);
        st.p[4] = 0.0f;
        reset_cov(st, prm);
    }
    th[r0 * ths] = h0;
    int last = r0;
    float plast[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) plast[i] = st.p[i];

    // ---- up pass
    int cc = h1, cn = h2;                 // chain hit of this row, of the next
    float cy = yg[h1], cz = zg[h1];
    int miss = 0;
    for (int r = r0 + 1; r < n_rows; ++r) {
        const bool chain = cc >= 0;
        float ny = 0.0f, nz = 0.0f;
        int cnn = -1;
        if (cn >= 0) {
            ny = yg[cn];
            nz = zg[cn];
            cnn = up[cn];
        }
        ++n_prop;
        if (!propagate(st, xs[r] - xs[r - 1], prm.curv, prm.s_max)) break;
        int c = cc;
        float my = cy, mz = cz;
        if (!chain) {
            c = search_row(st, s, r, prm, n_cand, bin_start, yg, zg, idg, my, mz);
            if (c < 0) {
                if (++miss >= prm.max_miss) break;
                continue;
            }
            miss = 0;
        }
        ++n_upd;
        kupdate(st, my, mz, sy2, sz2);
        th[r * ths] = c;
        last = r;
#pragma unroll
        for (int i = 0; i < 5; ++i) plast[i] = st.p[i];
        if (chain) {
            cc = cn;
            cy = ny;
            cz = nz;
            cn = cnn;
        }
    }

    // ---- down pass
    const int hl = th[last * ths];
#pragma unroll
    for (int i = 0; i < 5; ++i) st.p[i] = plast[i];
    st.p[0] = yg[hl];
    st.p[1] = zg[hl];
    reset_cov(st, prm);
    KState in = st;
    float csum = 0.0f;
    int rin = last;
    miss = 0;
    // assigned hits of the next two rows down: the hit list entry of row
    // r - 2 loads during step r, the coordinates of the hit of row r - 1
    // during step r (its entry loaded a step before), so that no step waits
    // on a load it issued itself
    int an = -1, an2 = -1;
    float ay = 0.0f, az = 0.0f;
    if (last - 1 >= r0) {
        an = th[(last - 1) * ths];
        if (an >= 0) {
            ay = yg[an];
            az = zg[an];
        }
    }
    if (last - 2 >= r0) an2 = th[(last - 2) * ths];
    for (int r = last - 1; r >= 0; --r) {
        int c = an;
        float my = ay, mz = az;
        an = an2;                         // the hit of row r - 1, or -1
        an2 = -1;
        if (an >= 0) {
            ay = yg[an];
            az = zg[an];
        }
        if (r - 2 >= r0) an2 = th[(r - 2) * ths];
        ++n_prop;
        if (!propagate(st, xs[r] - xs[r + 1], prm.curv, prm.s_max)) {
            for (int q = r; q >= 0; --q) th[q * ths] = -1;
            break;
        }
        if (r < r0) {
            c = search_row(st, s, r, prm, n_cand, bin_start, yg, zg, idg, my, mz);
            if (c < 0) {
                if (++miss >= prm.max_miss) break;
                continue;
            }
            miss = 0;
        }
        if (c >= 0) {
            ++n_upd;
            csum = csum + kupdate(st, my, mz, sy2, sz2);
            th[r * ths] = c;
            rin = r;
            in = st;
        }
    }
    int nh = 0;
    for (int r = 0; r < n_rows; ++r) nh += th[r * ths] >= 0;
    t_start[t] = h0;
    t_nhits[t] = nh;
    t_rin[t] = rin;
#pragma unroll
    for (int i = 0; i < 5; ++i) t_par[t * 5 + i] = in.p[i];
#pragma unroll
    for (int i = 0; i < 15; ++i) t_cov[t * 15 + i] = in.C[i];
    t_chi2[t] = csum;
}

// ---- queue form ------------------------------------------------------------
// One thread per tracklet at a time, every lane at its own row and pass:
// a loop step advances each lane by one row of its current pass (the same
// transport, search and update code for both passes), and a lane that
// finishes takes the next start from a device queue.  Lanes wait idle
// until kRefill of them are free (or no lane of the wave works), so that
// the refill (the tracklet's column of -1 entries and its first state) is
// issued for several lanes at once.  Per tracklet the arithmetic is the
// same sequence of operations as build_tracklet's.
constexpr int kRefill = 8;

enum : int { kLaneIdle = 0, kLaneUp = 1, kLaneDown = 2, kLaneDone = 3, kLaneOut = 4 };

struct LaneTracklet {
    int64_t t;
    int32_t* th;          // the tracklet's column: th[r * cap]
    tpc_sector s;
    int ph, r, r0, last, miss, nh, rin, h0, hl;
    int cc, cn, an;       // chain hit of this row, of the next (up); assigned hit below (down)
    float cy, cz, ay, az, csum;
    KState st, in;
    float plast[5];
};

// start of the down pass from the outermost hit (state at the up pass's
// last update, position of that hit, initial covariance)
__device__ __forceinline__ void lane_begin_down(LaneTracklet& L, const tpc_params& prm,
                                                const float* __restrict__ yg,
                                                const float* __restrict__ zg, int64_t cap)
{
#pragma unroll
    for (int i = 0; i < 5; ++i) L.st.p[i] = L.plast[i];
    L.st.p[0] = yg[L.hl];
    L.st.p[1] = zg[L.hl];
    reset_cov(L.st, prm);
    L.in = L.st;
    L.csum = 0.0f;
    L.rin = L.last;
    L.miss = 0;
    L.an = -1;
    if (L.last - 1 >= L.r0) {
        L.an = L.th[(int64_t)(L.last - 1) * cap];
        if (L.an >= 0) {
            L.ay = yg[L.an];
            L.az = zg[L.an];
        }
    }
    L.r = L.last - 1;
    L.ph = L.r >= 0 ? kLaneDown : kLaneDone;
}

// first state of tracklet t (its column already holds -1 everywhere)
__device__ __forceinline__ void lane_init(LaneTracklet& L, int64_t t,
                                          const tpc_sector* __restrict__ sec, int n_rows,
                                          const float* xs, const tpc_params& prm,
                                          const float* __restrict__ yg,
                                          const float* __restrict__ zg,
                                          const int32_t* __restrict__ gsr,
                                          const int32_t* __restrict__ up,
                                          const int32_t* __restrict__ starts, int64_t cap)
{
    const int h0 = starts[t];
    const int v0 = gsr[h0];
    L.s = sec[v0 >> 8];
    L.r0 = v0 & 255;
    const int h1 = up[h0], h2 = up[h1];
    const int r2 = gsr[h2] & 255;
    const float dX = xs[r2] - xs[L.r0];
    const float T0 = (yg[h2] - yg[h0]) / dX;
    const float q0 = sqrtf(1.0f + T0 * T0);
    L.st.p[0] = yg[h0];
    L.st.p[1] = zg[h0];
    L.st.p[2] = T0 / q0;
    L.st.p[3] = (zg[h2] - zg[h0]) / (dX * q0);
    L.st.p[4] = 0.0f;
    reset_cov(L.st, prm);
    L.th[(int64_t)L.r0 * cap] = h0;
    L.h0 = h0;
    L.hl = h0;
    L.last = L.r0;
    L.nh = 1;
#pragma unroll
    for (int i = 0; i < 5; ++i) L.plast[i] = L.st.p[i];
    L.cc = h1;
    L.cn = h2;
    L.cy = yg[h1];
    L.cz = zg[h1];
    L.miss = 0;
    L.r = L.r0 + 1;
    L.ph = kLaneUp;
    if (L.r >= n_rows) lane_begin_down(L, prm, yg, zg, cap);
}

// one row of the lane's current pass
__device__ __forceinline__ void lane_step(LaneTracklet& L, int n_rows, const float* xs,
                                          const tpc_params& prm,
                                          const int32_t* __restrict__ bin_start,
                                          const float* __restrict__ yg,
                                          const float* __restrict__ zg,
                                          const int32_t* __restrict__ idg,
                                          const int32_t* __restrict__ up, int64_t cap,
                                          int& n_prop, int& n_upd, int& n_cand)
{
    const bool upp = L.ph == kLaneUp;
    const int r = L.r;
    int c;
    float my, mz, ny = 0.0f, nz = 0.0f;
    int cnn = -1;
    if (upp) {
        if (L.cn >= 0) {
            ny = yg[L.cn];
            nz = zg[L.cn];
            cnn = up[L.cn];
        }
        c = L.cc;
        my = L.cy;
        mz = L.cz;
    } else {
        c = L.an;
        my = L.ay;
        mz = L.az;
        L.an = -1;
        if (r - 1 >= L.r0) {
            L.an = L.th[(int64_t)(r - 1) * cap];
            if (L.an >= 0) {
                L.ay = yg[L.an];
                L.az = zg[L.an];
            }
        }
    }
    ++n_prop;
    const float dx = upp ? xs[r] - xs[r - 1] : xs[r] - xs[r + 1];
    if (!propagate(L.st, dx, prm.curv, prm.s_max)) {
        if (upp) {
            lane_begin_down(L, prm, yg, zg, cap);
        } else {
            for (int q = r; q >= 0; --q) {
                L.nh -= L.th[(int64_t)q * cap] >= 0;
                L.th[(int64_t)q * cap] = -1;
            }
            L.ph = kLaneDone;
        }
        return;
    }
    const bool search = upp ? c < 0 : r < L.r0;
    if (search) {
        c = search_row(L.st, L.s, r, prm, n_cand, bin_start, yg, zg, idg, my, mz);
        if (c < 0) {
            if (++L.miss >= prm.max_miss) {
                if (upp) lane_begin_down(L, prm, yg, zg, cap);
                else L.ph = kLaneDone;
                return;
            }
        } else {
            L.miss = 0;
        }
    }
    if (c >= 0) {
        ++n_upd;
        const float chi = kupdate(L.st, my, mz, prm.sigma_y2, prm.sigma_z2);
        L.th[(int64_t)r * cap] = c;
        if (upp) {
            L.last = r;
            L.hl = c;
            ++L.nh;
#pragma unroll
            for (int i = 0; i < 5; ++i) L.plast[i] = L.st.p[i];
        } else {
            L.csum = L.csum + chi;
            L.rin = r;
            L.in = L.st;
            L.nh += r < L.r0;
        }
    }
    if (upp) {
        if (!search) {
            L.cc = L.cn;
            L.cy = ny;
            L.cz = nz;
            L.cn = cnn;
        }
        L.r = r + 1;
        if (L.r >= n_rows) lane_begin_down(L, prm, yg, zg, cap);
    } else {
        L.r = r - 1;
        if (L.r < 0) L.ph = kLaneDone;
    }
}

// per-wave sum of the work counters into the status block
__device__ __forceinline__ void add_work(tpc_status* status, int n_prop, int n_upd, int n_cand)
{
    unsigned long long a = n_prop, b = n_upd, c = n_cand;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, kWave);
        b += __shfl_xor(b, o, kWave);
        c += __shfl_xor(c, o, kWave);
    }
    if ((threadIdx.x & (kWave - 1)) == 0 && (a | b | c)) {
        atomicAdd((unsigned long long*)&status->n_propagations, a);
        atomicAdd((unsigned long long*)&status->n_updates, b);
        atomicAdd((unsigned long long*)&status->n_candidates, c);
    }
}

}  // namespace tpc
