// Full-track fit of merged sector tracks (section 2: the first fit of the
// sector tracks serves to find the whole track, which is then fitted;
// section 3: several fit iterations, inwards and outwards, across sector
// boundaries).
//
// One thread per chain: blocks list the chains' least track indices (their
// groups) and fit those, the other tracks are marked.  The chain is walked
// from its down end along the up links, or from its up end along the down
// links when the up end's first hit lies on a lower row than the down end's;
// the hits are the members' hits in that order, each member's row-ascending.
// Passes alternate outwards and inwards over all hits, each from the
// previous pass's parameters and a diagonal covariance (the variances of the
// first member's tracklet, then of the previous pass's end, times
// cov_scale); between hits of
// neighbouring sectors the state is turned into the next sector's frame
// (D = alpha_now - alpha_next) and then transported to the hit's row plane
// with the tracklet transport.  Float32 throughout, with the expressions
// and order of the float32 reference.
#include "tracklet_dev.hpp"

namespace tpc {

namespace {

// Turn the frame by D (cos c, sin sd): the point (x, y) becomes
// (x c - y sd, x sd + y c) and the state is taken at the plane through it;
// the covariance follows the first-order map of that change (a change of y
// slides the point back onto the plane along the track, a change of sin(phi)
// turns the direction).  False (nothing changed) when the direction would
// not point along +x or |sin(phi)| would reach s_max.
__device__ __forceinline__ bool turn_frame(float& x, KState& st, float c, float sd, float curv,
                                           float s_max)
{
    const float y = st.p[0], s = st.p[2], t = st.p[3];
    const float cs = sqrtf((1.0f - s) * (1.0f + s));
    const float s2 = s * c + cs * sd;
    const float c2 = cs * c - s * sd;
    if (!(0.0f < c2) || !(fabsf(s2) < s_max)) return false;
    const float jyy = c + (sd * s2) / c2;
    const float jzy = (t * sd) / c2;
    const float jsy = (curv * st.p[4]) * sd;
    const float jss = c2 / cs;
    float B[5][5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const float cy = st.C[lt(0, j)], cz = st.C[lt(1, j)], cc = st.C[lt(2, j)];
        B[0][j] = jyy * cy;
        B[1][j] = cz + jzy * cy;
        B[2][j] = jsy * cy + jss * cc;
        B[3][j] = st.C[lt(3, j)];
        B[4][j] = st.C[lt(4, j)];
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        st.C[lt(i, 0)] = jyy * B[i][0];
        if (i >= 1) st.C[lt(i, 1)] = B[i][1] + jzy * B[i][0];
        if (i >= 2) st.C[lt(i, 2)] = jsy * B[i][0] + jss * B[i][2];
        if (i >= 3) st.C[lt(i, 3)] = B[i][3];
        if (i >= 4) st.C[lt(i, 4)] = B[i][4];
    }
    const float x0 = x;
    x = x0 * c - y * sd;
    st.p[0] = x0 * sd + y * c;
    st.p[2] = s2;
    return true;
}

// diagonal entries of the lower-triangle covariance (y, z, sin, tan, q/pT)
constexpr int kDiag[5] = {0, 2, 5, 9, 14};

__device__ __forceinline__ int first_row(const uint8_t* __restrict__ row,
                                         const int32_t* __restrict__ off,
                                         const int32_t* __restrict__ hits, int j)
{
    return off[j + 1] > off[j] ? row[hits[off[j]]] : 0;
}

// Fit of track g (a chain's least index) or, for any other track, its
// marks (status -1).  xs: the row positions (LDS).
__device__ __forceinline__ void fit_track(
    int64_t g, const tpc_sector* __restrict__ sec, int n_sec, int sps, const float* xs,
    const tpc_params& prm, const uint8_t* __restrict__ row, const float* __restrict__ cy,
    const float* __restrict__ cz, const int32_t* __restrict__ off,
    const int32_t* __restrict__ hits, const int32_t* __restrict__ trk_tracklet,
    const float* __restrict__ t_par, const float* __restrict__ t_cov,
    const int32_t* __restrict__ t_rin, const int32_t* __restrict__ link_up,
    const int32_t* __restrict__ link_dn, const int32_t* __restrict__ group, float cos_w,
    float sin_w, int n_pass, float cov_scale, const tpc_fit_out& out)
{
    {
        float pin[5] = {0, 0, 0, 0, 0}, pout[5] = {0, 0, 0, 0, 0}, Cout[15];
#pragma unroll
        for (int i = 0; i < 15; ++i) Cout[i] = 0.0f;
        KState st;
        float chi2 = 0.0f;
        int n_hits = 0, n_mem = 0, status = -1;
        if (group[g] == (int32_t)g) {
            // down end (at most n_sec steps; a closed chain stops before g)
            int a = (int)g;
            for (int step = 0; step < n_sec && link_dn[a] >= 0 && link_dn[a] != (int)g; ++step)
                a = link_dn[a];
            // up end and the member and hit counts
            int b = a, j = a;
            while (j >= 0 && n_mem < n_sec) {
                ++n_mem;
                n_hits += off[j + 1] - off[j];
                b = j;
                j = link_up[j];
                if (j == a) break;
            }
            const bool rev = first_row(row, off, hits, b) < first_row(row, off, hits, a);
            const int first = rev ? b : a, last = rev ? a : b;
            const int32_t* fwd = rev ? link_dn : link_up;
            const int32_t* bwd = rev ? link_up : link_dn;
            if (n_hits < 3) {
                status = 1;
            } else {
                const int tf = trk_tracklet[first];
#pragma unroll
                for (int i = 0; i < 5; ++i) st.p[i] = t_par[(int64_t)tf * 5 + i];
                // each pass starts from a diagonal covariance: the variances of
                // the first member's tracklet (first pass) or of the previous
                // pass's end, times cov_scale; the initial variances stand in
                // for any that is not positive and finite
                const float v0[5] = {prm.sigma_y2, prm.sigma_z2, prm.c_ss0, prm.c_tt0, prm.c_ww0};
                float dg[5];
#pragma unroll
                for (int j = 0; j < 5; ++j) {
                    const float v = t_cov[(int64_t)tf * 15 + kDiag[j]];
                    dg[j] = v > 0.0f && v < 1e30f ? v : v0[j];
                }
                float x = xs[t_rin[tf]];
                int cur = -1;     // frame of the state: the sector of the first hit
                bool ok = true;
                for (int pass = 0; pass < n_pass && ok; ++pass) {
                    const bool outw = (pass & 1) == 0;
#pragma unroll
                    for (int i = 0; i < 15; ++i) st.C[i] = 0.0f;
#pragma unroll
                    for (int j = 0; j < 5; ++j) st.C[kDiag[j]] = dg[j] * cov_scale;
                    chi2 = 0.0f;
                    int m = outw ? first : last;
                    for (int mi = 0; mi < n_mem && ok && m >= 0; ++mi) {
                        const int h0 = off[m], h1 = off[m + 1];
                        if (h1 > h0) {
                            const int ms = find_sector(sec, n_sec, hits[h0]);
                            if (cur < 0) {
                                cur = ms;
                            } else if (ms != cur) {
                                // neighbouring sectors of one side
                                const int side = cur / sps, ic = cur % sps;
                                const int up = side * sps + (ic + 1) % sps;
                                const float sd = ms == up ? -sin_w : sin_w;
                                if (!turn_frame(x, st, cos_w, sd, prm.curv, prm.s_max)) {
                                    ok = false;
                                    break;
                                }
                                cur = ms;
                            }
                            // the member's hits in order; the row and
                            // coordinates of hit q + 1 load during step q,
                            // the index of hit q + 2 a step earlier still
                            const int nh = h1 - h0;
                            const int32_t* hp = hits + (outw ? h0 : h1 - 1);
                            const int dq = outw ? 1 : -1;
                            int ca = nh > 1 ? hp[dq] : -1;
                            const int c0 = hp[0];
                            int rb = row[c0];
                            float yb = cy[c0], zb = cz[c0];
                            for (int q = 0; q < nh; ++q) {
                                const int rr = rb;
                                const float my = yb, mz = zb;
                                if (ca >= 0) {
                                    rb = row[ca];
                                    yb = cy[ca];
                                    zb = cz[ca];
                                }
                                ca = q + 2 < nh ? hp[(q + 2) * dq] : -1;
                                const float xh = xs[rr];
                                if (!propagate(st, xh - x, prm.curv, prm.s_max)) {
                                    ok = false;
                                    break;
                                }
                                x = xh;
                                chi2 = chi2 + kupdate(st, my, mz, prm.sigma_y2, prm.sigma_z2);
                            }
                        }
                        m = outw ? fwd[m] : bwd[m];
                    }
                    if (!ok) break;
#pragma unroll
                    for (int j = 0; j < 5; ++j) {
                        const float v = st.C[kDiag[j]];
                        dg[j] = v > 0.0f && v < 1e30f ? v : v0[j];
                    }
                    if (outw) {
#pragma unroll
                        for (int i = 0; i < 5; ++i) pout[i] = st.p[i];
#pragma unroll
                        for (int i = 0; i < 15; ++i) Cout[i] = st.C[i];
                    } else {
#pragma unroll
                        for (int i = 0; i < 5; ++i) pin[i] = st.p[i];
                    }
                }
                status = ok ? 0 : 2;
                if (!ok) {
                    chi2 = 0.0f;
#pragma unroll
                    for (int i = 0; i < 5; ++i) pin[i] = pout[i] = 0.0f;
#pragma unroll
                    for (int i = 0; i < 15; ++i) Cout[i] = 0.0f;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            out.par_in[g * 5 + i] = pin[i];
            out.par_out[g * 5 + i] = pout[i];
        }
#pragma unroll
        for (int i = 0; i < 15; ++i) out.cov_out[g * 15 + i] = Cout[i];
        out.chi2[g] = chi2;
        out.n_hits[g] = status == -1 ? 0 : n_hits;
        out.n_members[g] = status == -1 ? 0 : n_mem;
        out.status[g] = status;
    }
}

// A block takes kFitIds consecutive track ids at a time, marks the tracks
// that lead no chain and lists the chain leaders in LDS, then its first
// threads fit the listed chains: about 60% of the tracks lead a chain, and
// without the list the lanes of the others would idle through every fit;
// with it, waves left without a chain end at once.  (Blocks of four times
// as many ids, fitted in rounds, took twice as long on the central event:
// a quarter of the waves, and every round waits for its longest chain.)
constexpr int kFitIds = kBlock;

__global__ __launch_bounds__(kBlock) void k_fit_merged(
    const tpc_sector* __restrict__ sec, int n_sec, int sps, int n_rows,
    const float* __restrict__ row_x, tpc_params prm, const uint8_t* __restrict__ row,
    const float* __restrict__ cy, const float* __restrict__ cz, const int32_t* __restrict__ off,
    const int32_t* __restrict__ hits, const int32_t* __restrict__ trk_tracklet,
    const float* __restrict__ t_par, const float* __restrict__ t_cov,
    const int32_t* __restrict__ t_rin,
    const int64_t* __restrict__ d_n_tracks, int64_t cap, const int32_t* __restrict__ link_up,
    const int32_t* __restrict__ link_dn, const int32_t* __restrict__ group, float cos_w,
    float sin_w, int n_pass, float cov_scale, tpc_fit_out out)
{
    __shared__ float xs[256];
    __shared__ int lead[kFitIds];
    __shared__ int n_lead;
    for (int i = threadIdx.x; i < n_rows; i += blockDim.x) xs[i] = row_x[i];
    const int64_t n = *d_n_tracks;
    const int64_t nt = n < cap ? n : cap;
    for (int64_t b0 = blockIdx.x * (int64_t)kFitIds; b0 < nt; b0 += (int64_t)gridDim.x * kFitIds) {
        if (threadIdx.x == 0) n_lead = 0;
        __syncthreads();
        for (int k = threadIdx.x; k < kFitIds && b0 + k < nt; k += blockDim.x) {
            const int64_t g = b0 + k;
            if (group[g] == (int32_t)g) {
                lead[atomicAdd(&n_lead, 1)] = k;
            } else {
                fit_track(g, sec, n_sec, sps, xs, prm, row, cy, cz, off, hits, trk_tracklet,
                          t_par, t_cov, t_rin, link_up, link_dn, group, cos_w, sin_w, n_pass,
                          cov_scale, out);
            }
        }
        __syncthreads();
        const int m = n_lead;
        for (int i = threadIdx.x; i < m; i += blockDim.x)
            fit_track(b0 + lead[i], sec, n_sec, sps, xs, prm, row, cy, cz, off, hits,
                      trk_tracklet, t_par, t_cov, t_rin, link_up, link_dn, group, cos_w, sin_w,
                      n_pass, cov_scale, out);
        // the list is reused only by a next round (none when the grid covers
        // every track: waves without a chain then end at once)
        if (b0 + (int64_t)gridDim.x * kFitIds < nt) __syncthreads();
    }
}

}  // namespace

}  // namespace tpc

extern "C" int tpc_check_problem(const tpc_problem* p);

extern "C" {

int tpc_fit_merged_tracks(tpc_context* ctx, const tpc_problem* h_prob, tpc_clusters clusters,
                          tpc_tracklets tracklets, tpc_tracks tracks, const int64_t* d_n_tracks,
                          const int32_t* link_up, const int32_t* link_dn, const int32_t* group,
                          int32_t sectors_per_side, float cos_width, float sin_width,
                          int32_t n_pass, float cov_scale, tpc_fit_out out, void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    if (!ctx || !clusters.row || !clusters.y || !clusters.z || !tracklets.par ||
        !tracklets.row_inner || !tracklets.cov || !tracks.off || !tracks.hits || !tracks.tracklet ||
        !d_n_tracks || !link_up || !link_dn || !group || !out.par_in || !out.par_out ||
        !out.cov_out || !out.chi2 || !out.n_hits || !out.n_members || !out.status ||
        tracks.capacity < 0 || tracks.capacity >= (int64_t(1) << 31) || n_pass < 1 ||
        n_pass > 64 || !std::isfinite(cos_width) || !std::isfinite(sin_width) ||
        !(cov_scale > 0.0f) || !std::isfinite(cov_scale))
        return TPC_ERR_INVALID_ARG;
    const int e = tpc_check_problem(h_prob);
    if (e) return e;
    const int sps = sectors_per_side;
    if (sps < 3 || h_prob->n_sectors % sps != 0) return TPC_ERR_INVALID_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TPC_ERR_HIP;
    if (dev != ctx->device && hipSetDevice(ctx->device) != hipSuccess) return TPC_ERR_HIP;
    if (tracks.capacity > 0)
        TPC_LAUNCH(tpc::k_fit_merged,
                   dim3(tpc::grid_for_block(tracks.capacity, tpc::kFitIds, 65536)),
                   dim3(tpc::kBlock), 0, (hipStream_t)stream, h_prob->d_sectors,
                   h_prob->n_sectors, sps, h_prob->n_rows, h_prob->d_row_x, h_prob->params, clusters.row, clusters.y, clusters.z,
                   (const int32_t*)tracks.off, (const int32_t*)tracks.hits,
                   (const int32_t*)tracks.tracklet, (const float*)tracklets.par,
                   (const float*)tracklets.cov, (const int32_t*)tracklets.row_inner, d_n_tracks,
                   tracks.capacity, link_up, link_dn, group, cos_width, sin_width, (int)n_pass,
                   cov_scale, out);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // extern "C"
