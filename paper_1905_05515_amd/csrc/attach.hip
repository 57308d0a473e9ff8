// Track-based cluster attachment (section 6, cluster rejection): a tube of
// fixed radius around every found track; clusters no track owns that lie in
// tubes are adjacent to the track of highest transverse momentum among
// them; clusters in the tubes of good tracks are protected; attached or
// adjacent clusters that are not protected are removed.
//
// One thread per track walks its rows: the track state (the tracklet's,
// at the plane of its innermost fitted row) is transported outwards row by
// row with the tracklet construction's transport, and on every row from the
// track's first to its last hit the grid bins covering the tube's cross
// section are scanned; the exact test dy*dy + dz*dz <= radius^2 decides.
// The working flags are kept by grid position, so that a candidate's flags
// load with its coordinates; the bin bounds of a row are loaded before the
// transport to the next row is computed, which hides their latency.
// The adjacent track of a cluster is a 64-bit atomic max over tubes of the
// key (~bits(|q/pT|), ~track): for non-negative floats the bit pattern
// orders like the value, so the largest key is the least |q/pT| and, among
// equal ones, the lowest track index; the result does not depend on the
// order of the atomics.
#include "tracklet_dev.hpp"

namespace tpc {

namespace {

constexpr uint32_t kAttached = 1, kAdjacent = 2, kProtected = 4, kRemoved = 8;

struct AttachWs {
    unsigned long long* adj;   // [n] by grid position: best adjacent key
    uint32_t* flags;           // [n] by grid position: attached, in a good tube
    int32_t* pos;              // [n] by cluster id: grid position
};

bool layout_attach(const tpc_problem* p, void* base, AttachWs* w, size_t* bytes)
{
    const size_t n = (size_t)(p->n_clusters > 0 ? p->n_clusters : 1);
    const size_t a = (sizeof(unsigned long long) * n + 255) & ~(size_t)255;
    const size_t f = (sizeof(uint32_t) * n + 255) & ~(size_t)255;
    *bytes = a + f + sizeof(int32_t) * n;
    if (w) {
        w->adj = (unsigned long long*)base;
        w->flags = (uint32_t*)((char*)base + a);
        w->pos = (int32_t*)((char*)base + a + f);
    }
    return true;
}

__device__ __forceinline__ int64_t track_count(const int64_t* d_n, int64_t cap)
{
    const int64_t n = *d_n;
    return n < cap ? n : cap;
}

// per grid position: clear the working arrays and the cluster's output
// track; record the position of every cluster id
__global__ __launch_bounds__(kBlock) void k_attach_init(int64_t n,
                                                        const int32_t* __restrict__ idg,
                                                        int32_t* __restrict__ track, AttachWs w)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = idg[q];
        track[c] = -1;
        w.pos[c] = (int32_t)q;
        w.adj[q] = 0ull;
        w.flags[q] = 0u;
    }
}

// the clusters of every track are attached to it (a cluster is in at most
// one track); one wave per track, its lanes over the hits
__global__ __launch_bounds__(kWave) void k_attach_own(
    const int32_t* __restrict__ trk_off, const int32_t* __restrict__ trk_hits,
    const int64_t* __restrict__ d_n_tracks, int64_t trk_cap, int32_t* __restrict__ track,
    AttachWs w)
{
    const int64_t nt = track_count(d_n_tracks, trk_cap);
    for (int64_t k = blockIdx.x; k < nt; k += gridDim.x)
        for (int32_t i = trk_off[k] + (int32_t)threadIdx.x; i < trk_off[k + 1]; i += kWave) {
            const int32_t c = trk_hits[i];
            track[c] = (int32_t)k;
            w.flags[w.pos[c]] = kAttached;
        }
}

// One thread per track: its tube, row by row.
__global__ __launch_bounds__(kWave) void k_attach_tube(
    const tpc_sector* __restrict__ sec, int n_sec, int n_rows, const float* __restrict__ row_x,
    tpc_params prm, const uint8_t* __restrict__ row, const int32_t* __restrict__ bin_start,
    const float* __restrict__ yg, const float* __restrict__ zg, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ trk_off, const int32_t* __restrict__ trk_hits,
    const int32_t* __restrict__ trk_tracklet, const float* __restrict__ t_par,
    const int32_t* __restrict__ t_rin, const int64_t* __restrict__ d_n_tracks, int64_t trk_cap,
    float radius, float r2, float w_good, AttachWs w)
{
    __shared__ float xs[256];
    for (int i = threadIdx.x; i < n_rows; i += blockDim.x) xs[i] = row_x[i];
    __syncthreads();
    const int64_t nt = track_count(d_n_tracks, trk_cap);
    // tube cross section widened before taking bins: a rounding difference
    // at its edge never drops a cluster, the exact test decides
    const float hw = radius * TPC_WIDEN + 0.01f;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nt;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = trk_off[k], b = trk_off[k + 1];
        if (b <= a) continue;
        const int32_t c0 = trk_hits[a];
        const int r_first = row[c0], r_last = row[trk_hits[b - 1]];
        const tpc_sector s = sec[find_sector(sec, n_sec, c0)];
        const int32_t t = trk_tracklet[k];
        KState st;
#pragma unroll
        for (int i = 0; i < 5; ++i) st.p[i] = t_par[(int64_t)t * 5 + i];
#pragma unroll
        for (int i = 0; i < 15; ++i) st.C[i] = 0.0f;
        const float aw = fabsf(st.p[4]);
        const bool good = aw <= w_good;
        const unsigned long long key =
            ((unsigned long long)(0xFFFFFFFFu - __float_as_uint(aw)) << 32) |
            (unsigned long long)(0xFFFFFFFFu - (uint32_t)k);
        const int r0 = t_rin[t];
        bool alive = true;
        for (int r = r0; alive && r <= r_last && r < n_rows; ++r) {
            const float py = st.p[0], pz = st.p[1];
            const bool in_tube_rows = r >= r_first;
            int iy0 = 0, iy1 = -1, iz0 = 0, iz1 = -1;
            int lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
            if (in_tube_rows) {
                iy0 = bin_of(py - hw, s.y0, s.inv_by, s.nby);
                iy1 = bin_of(py + hw, s.y0, s.inv_by, s.nby);
                iz0 = bin_of(pz - hw, s.z0, s.inv_bz, s.nbz);
                iz1 = bin_of(pz + hw, s.z0, s.inv_bz, s.nbz);
                const int g = s.bin_base + (r * s.nbz + iz0) * s.nby;
                lo0 = bin_start[g + iy0];
                hi0 = bin_start[g + iy1 + 1];
                if (iz0 + 1 <= iz1) {
                    lo1 = bin_start[g + s.nby + iy0];
                    hi1 = bin_start[g + s.nby + iy1 + 1];
                }
            }
            // the next row's transport while the bounds load
            if (r < r_last && r + 1 < n_rows)
                alive = propagate(st, xs[r + 1] - xs[r], prm.curv, prm.s_max);
            if (!in_tube_rows) continue;
            for (int iz = iz0; iz <= iz1; iz += 2) {
                if (iz > iz0) {
                    const int g = s.bin_base + (r * s.nbz + iz) * s.nby;
                    lo0 = bin_start[g + iy0];
                    hi0 = bin_start[g + iy1 + 1];
                    lo1 = hi1 = 0;
                    if (iz + 1 <= iz1) {
                        lo1 = bin_start[g + s.nby + iy0];
                        hi1 = bin_start[g + s.nby + iy1 + 1];
                    }
                }
                // the candidates of both z rows as one stream, kCandBatch
                // loads at a time
                const int n0 = hi0 - lo0 > 0 ? hi0 - lo0 : 0;
                const int n1 = hi1 - lo1 > 0 ? hi1 - lo1 : 0;
                for (int bb = 0; bb < n0 + n1; bb += kCandBatch) {
                    float yb[kCandBatch], zb[kCandBatch];
                    uint32_t fb[kCandBatch];
                    int pb[kCandBatch];
#pragma unroll
                    for (int j = 0; j < kCandBatch; ++j) {
                        const int e = bb + j;
                        pb[j] = e < n0 ? lo0 + e : lo1 + (e - n0);
                        if (e < n0 + n1) {
                            yb[j] = yg[pb[j]];
                            zb[j] = zg[pb[j]];
                            // the attached bit is fixed before this kernel; a
                            // stale protected bit only costs an atomic
                            fb[j] = w.flags[pb[j]];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < kCandBatch; ++j) {
                        if (bb + j >= n0 + n1) break;
                        const float dy = yb[j] - py, dz = zb[j] - pz;
                        if (!(dy * dy + dz * dz <= r2)) continue;
                        if (good && !(fb[j] & kProtected)) atomicOr(&w.flags[pb[j]], kProtected);
                        if (!(fb[j] & kAttached)) atomicMax(&w.adj[pb[j]], key);
                    }
                }
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_attach_final(
    int64_t n, const int32_t* __restrict__ idg, const int32_t* __restrict__ trk_tracklet,
    const float* __restrict__ t_par, float w_good, int32_t* __restrict__ track,
    uint8_t* __restrict__ state, AttachWs w)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = idg[q];
        const uint32_t f = w.flags[q];
        uint32_t out = f & kProtected;
        if (f & kAttached) {
            out |= kAttached;
            const int32_t k = track[c];
            if (fabsf(t_par[(int64_t)trk_tracklet[k] * 5 + 4]) <= w_good) out |= kProtected;
        } else if (w.adj[q]) {
            track[c] = (int32_t)(0xFFFFFFFFu - (uint32_t)(w.adj[q] & 0xFFFFFFFFull));
            out |= kAdjacent;
        }
        if ((out & (kAttached | kAdjacent)) && !(out & kProtected)) out |= kRemoved;
        state[c] = (uint8_t)out;
    }
}

}  // namespace

}  // namespace tpc

extern "C" int tpc_check_problem(const tpc_problem* p);

extern "C" {

int tpc_attach_workspace_size(const tpc_problem* h_prob, size_t* h_bytes)
{
    if (!h_bytes) return TPC_ERR_INVALID_ARG;
    const int e = tpc_check_problem(h_prob);
    if (e) return e;
    tpc::layout_attach(h_prob, nullptr, nullptr, h_bytes);
    return TPC_OK;
}

int tpc_attach_clusters(tpc_context* ctx, const tpc_problem* h_prob, tpc_clusters in,
                        tpc_grid grid, tpc_tracklets tracklets, tpc_tracks tracks,
                        const int64_t* d_n_tracks, float radius, float pt_good,
                        int32_t* track, uint8_t* state, void* d_ws, size_t ws_bytes,
                        void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    if (!ctx || !d_ws || !in.row || !grid.bin_start || !grid.y || !grid.z || !grid.id ||
        !tracklets.par || !tracklets.row_inner || !tracks.off || !tracks.hits ||
        !tracks.tracklet || !d_n_tracks || !track || !state || !(radius > 0.0f) ||
        !(pt_good > 0.0f) || tracks.capacity < 0)
        return TPC_ERR_INVALID_ARG;
    int e = tpc_check_problem(h_prob);
    if (e) return e;
    size_t need = 0;
    tpc::AttachWs w;
    tpc::layout_attach(h_prob, d_ws, &w, &need);
    if (need > ws_bytes) return TPC_ERR_INVALID_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TPC_ERR_HIP;
    if (dev != ctx->device && hipSetDevice(ctx->device) != hipSuccess) return TPC_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = h_prob->n_clusters;
    const float r2 = radius * radius;
    const float w_good = 1.0f / pt_good;
    TPC_LAUNCH(tpc::k_attach_init, dim3(tpc::grid_for(n)), dim3(tpc::kBlock), 0, st, n,
               (const int32_t*)grid.id, track, w);
    TPC_LAUNCH(tpc::k_attach_own,
               dim3((unsigned)(tracks.capacity < 65536 ? (tracks.capacity > 0 ? tracks.capacity : 1)
                                                       : 65536)),
               dim3(tpc::kWave), 0, st, (const int32_t*)tracks.off, (const int32_t*)tracks.hits, d_n_tracks,
               tracks.capacity, track, w);
    TPC_LAUNCH(tpc::k_attach_tube,
               dim3(tpc::grid_for_block(tracks.capacity, tpc::kWave, 65536)), dim3(tpc::kWave),
               0, st, h_prob->d_sectors, h_prob->n_sectors, h_prob->n_rows, h_prob->d_row_x,
               h_prob->params, in.row, (const int32_t*)grid.bin_start, (const float*)grid.y,
               (const float*)grid.z, (const int32_t*)grid.id, (const int32_t*)tracks.off,
               (const int32_t*)tracks.hits, (const int32_t*)tracks.tracklet,
               (const float*)tracklets.par, (const int32_t*)tracklets.row_inner, d_n_tracks,
               tracks.capacity, radius, r2, w_good, w);
    TPC_LAUNCH(tpc::k_attach_final, dim3(tpc::grid_for(n)), dim3(tpc::kBlock), 0, st, n,
               (const int32_t*)grid.id, (const int32_t*)tracks.tracklet,
               (const float*)tracklets.par, w_good, track, state, w);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // extern "C"
