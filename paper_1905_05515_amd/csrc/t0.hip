// Per-track interaction time in continuous read-out (section 2: the z of a
// hit depends on the unknown time of its collision; the first fit of a
// track, taken as primary, improves its z).  A primary comes from the beam
// axis at z = 0 and the tracker sees z* = z - side * vd * t for a collision
// at time t; the track's state (its tracklet's, at the plane of its
// innermost fitted row) is transported to the plane x = 0 of its sector
// frame, which holds the beam axis.  There y0 is the track's distance from
// the axis (0 for a primary) and z0 = -side * vd * t, so
// t0 = (side > 0 ? -z0 : z0) / vd.  One thread per track; the transport is
// the tracklet construction's, in ceil(x_in / 20 cm) equal steps: over a
// step of at most 20 cm the arc-length series of the transport stays
// accurate down to pT = 0.05 GeV/c, where one step over the whole distance
// would be off by up to a percent of the arc.
#include "tracklet_dev.hpp"

namespace tpc {

namespace {

constexpr float kT0Step = 20.0f;   // longest transport step to the axis plane [cm]

__global__ __launch_bounds__(kBlock) void k_track_t0(
    const tpc_sector* __restrict__ sec, int n_sec, const float* __restrict__ row_x, float curv,
    float s_max, const int32_t* __restrict__ trk_off, const int32_t* __restrict__ trk_hits,
    const int32_t* __restrict__ trk_tracklet, const float* __restrict__ t_par,
    const int32_t* __restrict__ t_rin, const int64_t* __restrict__ d_n_tracks, int64_t cap,
    float vd, float* __restrict__ z0, float* __restrict__ y0, float* __restrict__ t0,
    int8_t* __restrict__ ok)
{
    const int64_t n = *d_n_tracks;
    const int64_t nt = n < cap ? n : cap;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nt;
         k += (int64_t)gridDim.x * blockDim.x) {
        int side = 1;
        if (trk_off[k + 1] > trk_off[k]) side = sec[find_sector(sec, n_sec, trk_hits[trk_off[k]])].side;
        const int32_t t = trk_tracklet[k];
        KState st;
#pragma unroll
        for (int i = 0; i < 5; ++i) st.p[i] = t_par[(int64_t)t * 5 + i];
#pragma unroll
        for (int i = 0; i < 15; ++i) st.C[i] = 0.0f;
        const float x_in = row_x[t_rin[t]];
        int n_step = (int)ceilf(x_in / kT0Step);
        if (n_step < 1) n_step = 1;
        const float dx = (0.0f - x_in) / (float)n_step;
        bool alive = true;
        for (int i = 0; i < n_step && alive; ++i) alive = propagate(st, dx, curv, s_max);
        if (!alive) {
            z0[k] = 0.0f;
            y0[k] = 0.0f;
            t0[k] = 0.0f;
            ok[k] = 0;
            continue;
        }
        y0[k] = st.p[0];
        z0[k] = st.p[1];
        t0[k] = (side > 0 ? -st.p[1] : st.p[1]) / vd;
        ok[k] = 1;
    }
}

}  // namespace

}  // namespace tpc

extern "C" int tpc_check_problem(const tpc_problem* p);

extern "C" {

int tpc_track_t0(tpc_context* ctx, const tpc_problem* h_prob, tpc_tracklets tracklets,
                 tpc_tracks tracks, const int64_t* d_n_tracks, float vd, float* z0, float* y0,
                 float* t0, int8_t* ok, void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    if (!ctx || !tracklets.par || !tracklets.row_inner || !tracks.off || !tracks.hits ||
        !tracks.tracklet || !d_n_tracks || !z0 || !y0 || !t0 || !ok || !(vd > 0.0f) ||
        !std::isfinite(vd) || tracks.capacity < 0)
        return TPC_ERR_INVALID_ARG;
    const int e = tpc_check_problem(h_prob);
    if (e) return e;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TPC_ERR_HIP;
    if (dev != ctx->device && hipSetDevice(ctx->device) != hipSuccess) return TPC_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    if (tracks.capacity > 0)
        TPC_LAUNCH(tpc::k_track_t0, dim3(tpc::grid_for(tracks.capacity)), dim3(tpc::kBlock), 0,
                   st, h_prob->d_sectors, h_prob->n_sectors, h_prob->d_row_x,
                   h_prob->params.curv, h_prob->params.s_max, (const int32_t*)tracks.off,
                   (const int32_t*)tracks.hits, (const int32_t*)tracks.tracklet,
                   (const float*)tracklets.par, (const int32_t*)tracklets.row_inner, d_n_tracks,
                   tracks.capacity, vd, z0, y0, t0, ok);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // extern "C"
