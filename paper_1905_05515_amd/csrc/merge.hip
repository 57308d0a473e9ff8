// Sector-track merging (section 2: the first fit of the sector tracks serves
// to find the whole track; section 3: sector boundaries).  Tracks found in
// two neighbouring sectors of one side are linked when each is the other's
// best partner: the partner's state, turned into the frame of the track's
// sector and transported to the track's plane, must lie within a windowed
// distance d2 = sum ((p'_i - p_i) / win_i)^2 < 1; the least d2 wins, ties
// to the lower track index.  Chains of links over several sectors form one
// group, named by its least track index.
//
// Work layout: the tracks are bucketed by sector (any input order); the
// bucket of every sector stores, per candidate, its state already turned
// into the frames of both neighbour sectors (the turn does not depend on
// the track it is compared with), 32 bytes per direction, so the pair loop
// streams contiguous records.  Every bucket is sorted by tan(lambda), which
// neither the turn nor the transport changes: a candidate passes only if
// r3 = (tl_j - tl_k) / win_3 lies in (-1, 1) (else r3^2 >= 1 and so
// d2 >= 1), and r3 grows with tl_j, so the candidates that can pass form one
// range of the sorted bucket, found by two binary searches with the same
// float expression; the result is the brute-force one.  The pair loop over
// that range is split over kSlices threads
// per (track, direction), each taking every kSlices-th candidate, with the
// lanes of a wave on consecutive tracks of one sector reading the same
// record; the slices' minima meet in a 64-bit atomic min of the key
// (bits(d2) << 32 | index): d2 >= +0 orders like its bit pattern, so the
// least key is the least d2 and, among equal ones, the lower index, and the
// result does not depend on the bucket order or the order of the atomics.
#include "tracklet_dev.hpp"

namespace tpc {

namespace {

constexpr int kSlices = 16;
constexpr int kMergeRows = 512;   // waves per (slice, direction) of the pair kernel

struct MergeWs {
    int32_t* sec;              // [cap] sector of every track (-1: no hits)
    int32_t* cnt;              // [n_sec + 1] tracks per sector
    int32_t* fill;             // [n_sec + 1] bucket fill counters
    int32_t* first;            // [n_sec + 1] first bucket slot of every sector
    unsigned long long* key;   // [2 * cap] best partner key per (track, direction)
    float4* rec;               // [2][cap][2] bucketed candidate records (fill order)
    float4* rec_s;             // [2][cap][2] the same, each bucket sorted by tan(lambda)
    float* tl;                 // [cap] sorted tan(lambda) (NaN as +inf)
    uint32_t* key_in;          // [cap] order-preserving bits of tan(lambda)
    uint32_t* key_out;
    int32_t* val_in;           // [cap] fill slot
    int32_t* val_out;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bool layout_merge(const tpc_problem* p, int64_t cap, void* base, MergeWs* w, size_t* bytes)
{
    const size_t c = (size_t)(cap > 0 ? cap : 1);
    const size_t ns = (size_t)p->n_sectors + 1;
    size_t o = 0;
    const size_t o_key = o;  o += align256(sizeof(unsigned long long) * 2 * c);
    const size_t o_rec = o;  o += align256(sizeof(float4) * 4 * c);
    const size_t o_sec = o;  o += align256(sizeof(int32_t) * c);
    const size_t o_cnt = o;  o += align256(sizeof(int32_t) * 3 * ns);
    const size_t o_rs = o;   o += align256(sizeof(float4) * 4 * c);
    const size_t o_tl = o;   o += align256(sizeof(float) * c);
    const size_t o_ki = o;   o += align256(sizeof(uint32_t) * c);
    const size_t o_ko = o;   o += align256(sizeof(uint32_t) * c);
    const size_t o_vi = o;   o += align256(sizeof(int32_t) * c);
    const size_t o_vo = o;   o += align256(sizeof(int32_t) * c);
    *bytes = o;
    if (w) {
        char* b = (char*)base;
        w->key = (unsigned long long*)(b + o_key);
        w->rec = (float4*)(b + o_rec);
        w->sec = (int32_t*)(b + o_sec);
        w->cnt = (int32_t*)(b + o_cnt);
        w->fill = w->cnt + ns;
        w->first = w->fill + ns;
        w->rec_s = (float4*)(b + o_rs);
        w->tl = (float*)(b + o_tl);
        w->key_in = (uint32_t*)(b + o_ki);
        w->key_out = (uint32_t*)(b + o_ko);
        w->val_in = (int32_t*)(b + o_vi);
        w->val_out = (int32_t*)(b + o_vo);
    }
    return true;
}

__device__ __forceinline__ int64_t n_tracks_of(const int64_t* d_n, int64_t cap)
{
    const int64_t n = *d_n;
    return n < cap ? n : cap;
}

// neighbour sector of s in direction d (0: next index of the side, 1: previous)
__device__ __forceinline__ int neighbour(int s, int d, int sps)
{
    const int side = s / sps, i = s % sps;
    return side * sps + (d == 0 ? (i + 1) % sps : (i + sps - 1) % sps);
}

// ctr[s] += 1 for every active lane, one atomic per distinct s among the
// wave's active lanes (tracks arrive mostly grouped by sector, so a wave
// usually holds one or two); returns the lane's slot: the counter's old
// value plus the lane's rank among the lanes of its s.
__device__ __forceinline__ int wave_bucket_add(int32_t* ctr, int s, bool active)
{
    const int lane = __lane_id();
    unsigned long long pending = __ballot(active);
    int slot = 0;
    while (pending) {
        const int leader = __ffsll(pending) - 1;
        const int sl = __shfl(s, leader);
        const unsigned long long same = __ballot(s == sl) & pending;
        int base = 0;
        if (lane == leader) base = atomicAdd(&ctr[sl], (int)__popcll(same));
        base = __shfl(base, leader);
        if ((same >> lane) & 1ull) slot = base + (int)__popcll(same & ((1ull << lane) - 1ull));
        pending &= ~same;
    }
    return slot;
}

__global__ __launch_bounds__(kBlock) void k_merge_init(int n_sec, MergeWs w)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 3 * (n_sec + 1);
         i += gridDim.x * blockDim.x)
        w.cnt[i] = 0;   // cnt, fill, first
}

__global__ __launch_bounds__(kBlock) void k_merge_count(
    const tpc_sector* __restrict__ sec, int n_sec, const int32_t* __restrict__ trk_off,
    const int32_t* __restrict__ trk_hits, const int64_t* __restrict__ d_n_tracks, int64_t cap,
    MergeWs w)
{
    const int64_t nt = n_tracks_of(d_n_tracks, cap);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nt;
         k += (int64_t)gridDim.x * blockDim.x) {
        int s = -1;
        if (trk_off[k + 1] > trk_off[k]) s = find_sector(sec, n_sec, trk_hits[trk_off[k]]);
        wave_bucket_add(w.cnt, s, s >= 0);
        w.sec[k] = s;
        w.key[2 * k] = ~0ull;
        w.key[2 * k + 1] = ~0ull;
    }
}

// exclusive prefix of the per-sector counts (a few dozen sectors)
__global__ void k_merge_scan(int n_sec, MergeWs w)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int acc = 0;
    for (int s = 0; s < n_sec; ++s) {
        w.first[s] = acc;
        acc += w.cnt[s];
    }
    w.first[n_sec] = acc;
}

// Every track into its sector's bucket, with its state turned into the frame
// of the down neighbour (d = 0: compared with the tracks of that sector
// looking up, turn D = +width) and of the up neighbour (d = 1, D = -width):
//   x' = x c - y sd, y' = x sd + y c, sin' = sin c + cos sd,
//   cos' = cos c - sin sd, valid when cos' > 0 and |sin'| < s_max.
__global__ __launch_bounds__(kBlock) void k_merge_fill(
    const float* __restrict__ row_x, float s_max, const int32_t* __restrict__ trk_tracklet,
    const float* __restrict__ t_par, const int32_t* __restrict__ t_rin,
    const int64_t* __restrict__ d_n_tracks, int64_t cap, float cw, float sw, MergeWs w)
{
    const int64_t nt = n_tracks_of(d_n_tracks, cap);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nt;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int s = w.sec[k];
        const int rank = wave_bucket_add(w.fill, s, s >= 0);
        if (s < 0) continue;
        const int64_t slot = w.first[s] + rank;
        const int32_t t = trk_tracklet[k];
        const float* p = t_par + (int64_t)t * 5;
        const float x = row_x[t_rin[t]];
        const float y = p[0], z = p[1], sn = p[2], tl = p[3], qp = p[4];
        const float cs = sqrtf((1.0f - sn) * (1.0f + sn));
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const float sd = d == 0 ? sw : -sw;
            const float xr = x * cw - y * sd;
            const float yr = x * sd + y * cw;
            const float sr = sn * cw + cs * sd;
            const float cr = cs * cw - sn * sd;
            const bool ok = (cr > 0.0f) && (fabsf(sr) < s_max);
            float4* r = w.rec + ((int64_t)d * cap + slot) * 2;
            r[0] = make_float4(xr, yr, z, sr);
            r[1] = make_float4(tl, qp, ok ? 1.0f : 0.0f, __int_as_float((int32_t)k));
        }
        // bits that order like the value: sign bit set for >= +0, all bits
        // flipped for negatives; NaN last (it is read as +inf below)
        const uint32_t u = __float_as_uint(tl);
        w.key_in[slot] = tl != tl ? 0xFFFFFFFFu : (u & 0x80000000u) ? ~u : (u | 0x80000000u);
        w.val_in[slot] = (int32_t)slot;
    }
}

// Sort of every sector bucket by its tan(lambda) key bits: one 1024-thread
// block per bucket runs a least-significant-digit radix sort, 8-bit digits,
// through key_in/val_in and key_out/val_out in turn, leaving the bucket's
// slots in key order in val_out.  A digit pass is a histogram of the
// bucket's digits (LDS atomics), its exclusive scan, and a stable scatter of
// 1024-key tiles: within a wave the keys of one digit are found with one
// ballot per digit bit, a key's rank is the number of such keys on lower
// lanes, and the per-wave digit counts are scanned across the waves in LDS,
// so equal digits keep their order.  A pass whose digit is the same for the
// whole bucket moves nothing.
constexpr int kSortBlock = 1024;
constexpr int kSortWaves = kSortBlock / kWave;

__global__ __launch_bounds__(kSortBlock) void k_merge_sort(int n_sec, MergeWs w)
{
    __shared__ int hist[256];
    __shared__ int off[256];
    __shared__ int wcnt[kSortWaves * 256];
    __shared__ int same;
    const int s = blockIdx.x;
    if (s >= n_sec) return;
    const int b0 = w.first[s], n = w.first[s + 1] - b0;
    const int lane = (int)threadIdx.x & (kWave - 1), wv = (int)threadIdx.x / kWave;
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t* ks = w.key_in + b0;
    int32_t* vs = w.val_in + b0;
    uint32_t* kd = w.key_out + b0;
    int32_t* vd = w.val_out + b0;
    for (int shift = 0; shift < 32; shift += 8) {
        for (int d = threadIdx.x; d < 256; d += kSortBlock) hist[d] = 0;
        if (threadIdx.x == 0) same = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += kSortBlock) atomicAdd(&hist[(ks[i] >> shift) & 255u], 1);
        __syncthreads();
        if (threadIdx.x < 256 && hist[threadIdx.x] == n) same = 1;
        if (threadIdx.x == 0) {
            int a = 0;
            for (int d = 0; d < 256; ++d) {
                off[d] = a;
                a += hist[d];
            }
        }
        __syncthreads();
        const bool skip = same != 0;        // every key has this digit
        __syncthreads();
        if (skip) continue;
        for (int t0 = 0; t0 < n; t0 += kSortBlock) {
            for (int e = threadIdx.x; e < kSortWaves * 256; e += kSortBlock) wcnt[e] = 0;
            const int i = t0 + (int)threadIdx.x;
            const bool valid = i < n;
            uint32_t key = 0;
            int32_t val = 0;
            if (valid) {
                key = ks[i];
                val = vs[i];
            }
            const int d = (int)((key >> shift) & 255u);
            uint64_t m = __ballot(valid);
#pragma unroll
            for (int bit = 0; bit < 8; ++bit) {
                const uint64_t b = __ballot((d >> bit) & 1);
                m &= ((d >> bit) & 1) ? b : ~b;
            }
            __syncthreads();
            if (valid && (m & below) == 0) wcnt[wv * 256 + d] = __popcll(m);
            __syncthreads();
            if (threadIdx.x < 256) {
                int a = 0;
                for (int q = 0; q < kSortWaves; ++q) {
                    const int c = wcnt[q * 256 + threadIdx.x];
                    wcnt[q * 256 + threadIdx.x] = a;
                    a += c;
                }
                hist[threadIdx.x] = a;       // the tile's count of this digit
            }
            __syncthreads();
            if (valid) {
                const int pos = off[d] + wcnt[wv * 256 + d] + __popcll(m & below);
                kd[pos] = key;
                vd[pos] = val;
            }
            __syncthreads();
            if (threadIdx.x < 256) off[threadIdx.x] += hist[threadIdx.x];
            __syncthreads();
        }
        uint32_t* tk = ks; ks = kd; kd = tk;
        int32_t* tv = vs; vs = vd; vd = tv;
    }
    // the sorted slots are in vs: leave them in val_out
    if (vs != w.val_out + b0)
        for (int i = threadIdx.x; i < n; i += kSortBlock) w.val_out[b0 + i] = vs[i];
}

// bucket records into tan(lambda) order (both directions)
__global__ __launch_bounds__(kBlock) void k_merge_gather(int n_sec, int64_t cap, MergeWs w)
{
    const int64_t total = w.first[n_sec];
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < total;
         m += (int64_t)gridDim.x * blockDim.x) {
        const int64_t src = w.val_out[m];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const float4* a = w.rec + ((int64_t)d * cap + src) * 2;
            float4* b = w.rec_s + ((int64_t)d * cap + m) * 2;
            b[0] = a[0];
            b[1] = a[1];
        }
        const float t = w.rec[src * 2 + 1].x;
        w.tl[m] = t != t ? __int_as_float(0x7f800000) : t;
    }
}

// first m in [lo, hi) with pred(m), pred monotone (false ... true)
template <typename P>
__device__ __forceinline__ int first_true(int lo, int hi, P pred)
{
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (pred(mid)) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// (track, direction, slice): the least key over every kSlices-th candidate
// of the neighbour sector's bucket.  Threads walk the tracks in sorted
// bucket order, so the lanes of a wave hold tracks of one sector with close
// tan(lambda) and nearly the same candidate range.
__global__ __launch_bounds__(kWave) void k_merge_best(
    int n_sec, int sps, const float* __restrict__ row_x, float curv, float s_max,
    const int32_t* __restrict__ trk_tracklet, const float* __restrict__ t_par,
    const int32_t* __restrict__ t_rin, int64_t cap, float iw0, float iw1, float iw2, float iw3,
    float iw4, MergeWs w)
{
    const int slice = blockIdx.y, d = blockIdx.z;
    const float iw[5] = {iw0, iw1, iw2, iw3, iw4};
    const float4* rec = w.rec_s + (int64_t)d * cap * 2;
    const int64_t total = w.first[n_sec];
    const float4* own = w.rec_s;      // direction 0 records carry the track index
    for (int64_t q = blockIdx.x * (int64_t)kWave + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * kWave) {
        const int64_t k = __float_as_int(own[q * 2 + 1].w);
        const int s = w.sec[k];
        const int nb = neighbour(s, d, sps);
        const int32_t t = trk_tracklet[k];
        const float xk = row_x[t_rin[t]];
        float pk[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) pk[i] = t_par[(int64_t)t * 5 + i];
        unsigned long long best = ~0ull;
        // candidates with r3 = (tl_j - tl_k) * iw3 in (-1, 1); a window
        // without a tan(lambda) cut takes the whole bucket, a NaN track none
        int m0 = w.first[nb], m1 = w.first[nb + 1];
        if (pk[3] != pk[3]) {
            m1 = m0;
        } else if (iw[3] != 0.0f) {
            const float* tl = w.tl;
            const float tk = pk[3], i3 = iw[3];
            const int a = first_true(m0, m1, [&](int m) { return (tl[m] - tk) * i3 > -1.0f; });
            m1 = first_true(a, m1, [&](int m) { return (tl[m] - tk) * i3 >= 1.0f; });
            m0 = a;
        }
        for (int m = m0 + slice; m < m1; m += kSlices) {
            const float4 a = rec[(int64_t)m * 2], b = rec[(int64_t)m * 2 + 1];
            if (!(b.z != 0.0f)) continue;
            // the transport's covariance part is dead code here and drops out
            KState st;
            st.p[0] = a.y;
            st.p[1] = a.z;
            st.p[2] = a.w;
            st.p[3] = b.x;
            st.p[4] = b.y;
#pragma unroll
            for (int i = 0; i < 15; ++i) st.C[i] = 0.0f;
            if (!propagate(st, xk - a.x, curv, s_max)) continue;
            float d2 = 0.0f;
#pragma unroll
            for (int e = 0; e < 5; ++e) {
                const float r = (st.p[e] - pk[e]) * iw[e];
                d2 = d2 + r * r;
            }
            if (!(d2 < 1.0f)) continue;
            const unsigned long long key =
                ((unsigned long long)__float_as_uint(d2) << 32) | (uint32_t)__float_as_int(b.w);
            best = key < best ? key : best;
        }
        if (best != ~0ull) atomicMin(&w.key[2 * k + d], best);
    }
}

__device__ __forceinline__ int32_t partner(unsigned long long key)
{
    return key == ~0ull ? -1 : (int32_t)(key & 0xFFFFFFFFull);
}

__global__ __launch_bounds__(kBlock) void k_merge_link(const int64_t* __restrict__ d_n_tracks,
                                                       int64_t cap, int32_t* __restrict__ link_up,
                                                       int32_t* __restrict__ link_dn, MergeWs w)
{
    const int64_t nt = n_tracks_of(d_n_tracks, cap);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nt;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = partner(w.key[2 * k]);
        const int32_t v = partner(w.key[2 * k + 1]);
        link_up[k] = (u >= 0 && partner(w.key[2 * (int64_t)u + 1]) == (int32_t)k) ? u : -1;
        link_dn[k] = (v >= 0 && partner(w.key[2 * (int64_t)v]) == (int32_t)k) ? v : -1;
    }
}

// least index over the chain through every track; a chain visits each
// sector of a side at most once, so n_sec steps bound each walk
__global__ __launch_bounds__(kBlock) void k_merge_group(int n_sec,
                                                        const int64_t* __restrict__ d_n_tracks,
                                                        int64_t cap,
                                                        const int32_t* __restrict__ link_up,
                                                        const int32_t* __restrict__ link_dn,
                                                        int32_t* __restrict__ group)
{
    const int64_t nt = n_tracks_of(d_n_tracks, cap);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nt;
         k += (int64_t)gridDim.x * blockDim.x) {
        int32_t g = (int32_t)k;
        for (int d = 0; d < 2; ++d) {
            const int32_t* lk = d == 0 ? link_up : link_dn;
            int32_t j = lk[k];
            for (int step = 0; j >= 0 && j != (int32_t)k && step < n_sec; ++step) {
                g = j < g ? j : g;
                j = lk[j];
            }
        }
        group[k] = g;
    }
}

}  // namespace

}  // namespace tpc

extern "C" int tpc_check_problem(const tpc_problem* p);

extern "C" {

int tpc_merge_workspace_size(const tpc_problem* h_prob, int64_t track_capacity, size_t* h_bytes)
{
    if (!h_bytes || track_capacity < 0) return TPC_ERR_INVALID_ARG;
    const int e = tpc_check_problem(h_prob);
    if (e) return e;
    return tpc::layout_merge(h_prob, track_capacity, nullptr, nullptr, h_bytes) ? TPC_OK
                                                                                : TPC_ERR_HIP;
}

int tpc_merge_sector_tracks(tpc_context* ctx, const tpc_problem* h_prob,
                            tpc_tracklets tracklets, tpc_tracks tracks,
                            const int64_t* d_n_tracks, tpc_merge_cuts cuts, int32_t* link_up,
                            int32_t* link_dn, int32_t* group, void* d_ws, size_t ws_bytes,
                            void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    if (!ctx || !d_ws || !tracklets.par || !tracklets.row_inner || !tracks.off ||
        !tracks.hits || !tracks.tracklet || !d_n_tracks || !link_up || !link_dn || !group ||
        tracks.capacity < 0 || tracks.capacity >= ((int64_t)1 << 31))
        return TPC_ERR_INVALID_ARG;
    int e = tpc_check_problem(h_prob);
    if (e) return e;
    const int sps = cuts.sectors_per_side;
    if (sps < 3 || h_prob->n_sectors % sps != 0 || !std::isfinite(cuts.cos_width) ||
        !std::isfinite(cuts.sin_width))
        return TPC_ERR_INVALID_ARG;
    for (int i = 0; i < 5; ++i)
        if (!(cuts.inv_window[i] >= 0.0f) || !std::isfinite(cuts.inv_window[i]))
            return TPC_ERR_INVALID_ARG;
    const int64_t cap = tracks.capacity;
    size_t need = 0;
    tpc::MergeWs w;
    if (!tpc::layout_merge(h_prob, cap, d_ws, &w, &need)) return TPC_ERR_HIP;
    if (need > ws_bytes) return TPC_ERR_INVALID_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TPC_ERR_HIP;
    if (dev != ctx->device && hipSetDevice(ctx->device) != hipSuccess) return TPC_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    const int n_sec = h_prob->n_sectors;
    const tpc_params& prm = h_prob->params;
    TPC_LAUNCH(tpc::k_merge_init, dim3(tpc::grid_for(3 * (int64_t)(n_sec + 1))),
               dim3(tpc::kBlock), 0, st, n_sec, w);
    if (cap > 0) {
        TPC_LAUNCH(tpc::k_merge_count, dim3(tpc::grid_for(cap)), dim3(tpc::kBlock), 0, st,
                   h_prob->d_sectors, n_sec, (const int32_t*)tracks.off,
                   (const int32_t*)tracks.hits, d_n_tracks, cap, w);
        TPC_LAUNCH(tpc::k_merge_scan, dim3(1), dim3(1), 0, st, n_sec, w);
        TPC_LAUNCH(tpc::k_merge_fill, dim3(tpc::grid_for(cap)), dim3(tpc::kBlock), 0, st,
                   h_prob->d_row_x, prm.s_max, (const int32_t*)tracks.tracklet,
                   (const float*)tracklets.par, (const int32_t*)tracklets.row_inner, d_n_tracks,
                   cap, cuts.cos_width, cuts.sin_width, w);
        TPC_LAUNCH(tpc::k_merge_sort, dim3((unsigned)n_sec), dim3(tpc::kSortBlock), 0, st,
                   n_sec, w);
        TPC_LAUNCH(tpc::k_merge_gather, dim3(tpc::grid_for(cap)), dim3(tpc::kBlock), 0, st, n_sec,
                   cap, w);
        TPC_LAUNCH(tpc::k_merge_best,
                   dim3(tpc::grid_for_block(cap, tpc::kWave, tpc::kMergeRows), tpc::kSlices, 2),
                   dim3(tpc::kWave), 0, st, n_sec, sps, h_prob->d_row_x, prm.curv, prm.s_max,
                   (const int32_t*)tracks.tracklet, (const float*)tracklets.par,
                   (const int32_t*)tracklets.row_inner, cap, cuts.inv_window[0],
                   cuts.inv_window[1], cuts.inv_window[2], cuts.inv_window[3],
                   cuts.inv_window[4], w);
        TPC_LAUNCH(tpc::k_merge_link, dim3(tpc::grid_for(cap)), dim3(tpc::kBlock), 0, st,
                   d_n_tracks, cap, link_up, link_dn, w);
        TPC_LAUNCH(tpc::k_merge_group, dim3(tpc::grid_for(cap)), dim3(tpc::kBlock), 0, st,
                   n_sec, d_n_tracks, cap, (const int32_t*)link_up, (const int32_t*)link_dn,
                   group);
    }
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // extern "C"
