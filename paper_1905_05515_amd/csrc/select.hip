// Tracklet selection: every cluster goes to the tracklet of largest key
// (hits << 32 | (2^32 - 1 - start id)) containing it, among tracklets with
// at least min_tracklet_hits hits (64-bit atomic max, order independent); a
// tracklet keeping at least min_track_hits clusters becomes a track.
// Tracks are compacted in tracklet order by a scan of (accepted, kept).
#include "select_dev.hpp"

namespace tpc {

// Sectors whose row chunks hold on average several times more positions
// than the LDS table take the row form below instead (same keys and
// counts).  A chunk just over the table still uses its
// block (with device-wide keys).  Host and device decide alike from the
// sector's size.
__host__ __device__ inline bool sel_big(const tpc_sector& s, int n_rows)
{
    return (s.end - s.begin) * (int64_t)kSelRows > (int64_t)(8 * kSelLds) * n_rows;
}

// one block per (sector, row chunk) of sectors [sec_lo, ...)
__global__ __launch_bounds__(kBlock) void k_sel_chunk(
    const tpc_sector* __restrict__ sec, int sec_lo, int n_rows, tpc_params prm,
    const int32_t* __restrict__ bin_start, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_hits,
    const int32_t* __restrict__ t_nhits, const int64_t* __restrict__ sec_start,
    int64_t count_cap, int64_t cap, unsigned long long* __restrict__ hitkey,
    uint8_t* __restrict__ ccnt)
{
    __shared__ unsigned long long kl[kSelLds];
    const int nq = (n_rows + kSelRows - 1) / kSelRows;
    const int si = sec_lo + (int)(blockIdx.x / nq);
    const int q = (int)(blockIdx.x % nq);
    const tpc_sector s = sec[si];
    if (sel_big(s, n_rows)) return;   // the row kernels take this sector
    int64_t lo = sec_start[si], hi = sec_start[si + 1];
    if (lo < 0) lo = 0;
    sel_chunk_block(s, q, n_rows, prm, bin_start, idg, t_start, t_hits, t_nhits, lo, hi,
                    count_cap, cap, hitkey, ccnt, kl, kSelLds);
}

// Row form for big sectors.  One block per (sector, pad row) keeps the
// ownership keys of the row's grid positions in LDS (in slices of 64 KB of
// keys when the row has more), reads the row's entry of
// every tracklet of the sector, claims with a 64-bit LDS atomic max, writes
// the keys out and records which tracklets keep their hit on the row as one
// bit per tracklet (kbits[row][t / 64], bit t % 64).  A second kernel sums
// the bits of every row chunk into the kept counts.  No device-wide atomic
// per hit: on a continuous read-out slice (3.4M tracklets over 36 sectors
// of 1.9M clusters) the tracklet-parallel form with one 64-bit device atomic
// per hit took 11 + 3.5 ms, this form with 64-bit keys in slices of 8192
// positions (two per row there) 5.1 + 0.7 ms.
constexpr int kSelRowBytes = 65536;      // LDS key table of one block
constexpr int kSelRowBlock = 1024;
constexpr int kSelRowUnroll = 4;          // tracklet entries loaded together
constexpr unsigned long long kKeyNotBig = ~0ull;   // tracklet of a sector that is not big

// tkey[t]: the tracklet's key (0: takes no part), kKeyNotBig outside big
// sectors; kbits cleared over the words of tracklets [lo, m).
__global__ __launch_bounds__(kBlock) void k_sel_prep_big(
    const tpc_sector* __restrict__ sec, int n_rows, tpc_params prm,
    const int32_t* __restrict__ idg, const int32_t* __restrict__ gsr,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_nhits,
    const int64_t* __restrict__ t_lo, const int64_t* __restrict__ t_hi, int64_t count_cap,
    int64_t n_words, unsigned long long* __restrict__ tkey,
    unsigned long long* __restrict__ kbits)
{
    const int64_t lo = *t_lo < count_cap ? *t_lo : count_cap;
    const int64_t m = *t_hi < count_cap ? *t_hi : count_cap;
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = lo + g; t < m; t += stride)
        tkey[t] = sel_big(sec[gsr[t_start[t]] >> 8], n_rows) ? key_of(t, prm, idg, t_start, t_nhits)
                                                            : kKeyNotBig;
    if (m <= lo) return;
    const int64_t w0 = lo >> 6, nw = ((m - 1) >> 6) - w0 + 1;
    for (int64_t i = g; i < nw * n_rows; i += stride)
        kbits[(i / nw) * n_words + w0 + i % nw] = 0ull;
}

// Keys in LDS: 32 bits when the sector has at most 2^24 clusters
// (hits << 24 | (2^24 - 1 - start id + first id of the sector), the same
// order as the 64-bit key), else the 64-bit key.
struct Key32 {
    using T = unsigned int;
    int64_t begin;
    __device__ T pack(unsigned long long k) const
    {
        if (!k) return 0u;
        const unsigned nh = (unsigned)(k >> 32);
        const int64_t id = (int64_t)(0xFFFFFFFFull - (k & 0xFFFFFFFFull));
        return (nh << 24) | (0xFFFFFFu - (unsigned)(id - begin));
    }
    __device__ unsigned long long unpack(T k) const
    {
        if (!k) return 0ull;
        const int64_t id = begin + (int64_t)(0xFFFFFFu - (k & 0xFFFFFFu));
        return ((unsigned long long)(k >> 24) << 32) | (0xFFFFFFFFull - (unsigned long long)id);
    }
};
struct Key64 {
    using T = unsigned long long;
    int64_t begin;
    __device__ T pack(unsigned long long k) const { return k; }
    __device__ unsigned long long unpack(T k) const { return k; }
};

template <typename KF>
__global__ __launch_bounds__(kSelRowBlock) void k_sel_rows_big(
    const tpc_sector* __restrict__ sec, int sec_lo, int n_rows,
    const int32_t* __restrict__ bin_start, const int32_t* __restrict__ t_hits,
    const int64_t* __restrict__ sec_start, int64_t count_cap, int64_t cap, int64_t n_words,
    const unsigned long long* __restrict__ tkey, unsigned long long* __restrict__ hitkey,
    unsigned long long* __restrict__ kbits)
{
    using T = typename KF::T;
    constexpr int kLds = kSelRowBytes / (int)sizeof(T);
    __shared__ T kl[kLds];
    const int si = sec_lo + (int)(blockIdx.x / n_rows);
    const int r = (int)(blockIdx.x % n_rows);
    const tpc_sector s = sec[si];
    if (!sel_big(s, n_rows)) return;
    const KF kf{s.begin};
    const int per_row = s.nbz * s.nby;
    const int p0 = bin_start[s.bin_base + r * per_row];
    const int p1 = bin_start[s.bin_base + (r + 1) * per_row];
    int64_t lo = sec_start[si], hi = sec_start[si + 1];
    if (hi > count_cap) hi = count_cap;
    if (lo < 0) lo = 0;
    if (lo > hi) lo = hi;
    // whole waves over 64-aligned tracklet ranges: lane 0 of a wave owns one
    // word of kbits; words shared with a neighbouring sector (the first and
    // the last) are merged with an atomic or, the others written by their
    // owner alone
    const int64_t a0 = lo & ~(int64_t)63, a1 = (hi + 63) & ~(int64_t)63;
    const int64_t w_first = lo >> 6, w_last = (hi - 1) >> 6;
    const int32_t* __restrict__ row = t_hits + (int64_t)r * cap;
    unsigned long long* __restrict__ kb = kbits + (int64_t)r * n_words;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t bd = blockDim.x;
    for (int ps = p0, slice = 0; ps < p1; ps += kLds, ++slice) {
        const int np = p1 - ps < kLds ? p1 - ps : kLds;
        for (int k = threadIdx.x; k < np; k += blockDim.x) kl[k] = 0;
        __syncthreads();
        // claims: kSelRowUnroll entries per thread in flight
        for (int64_t t0 = a0 + threadIdx.x; t0 < hi; t0 += bd * kSelRowUnroll) {
            int h[kSelRowUnroll];
#pragma unroll
            for (int u = 0; u < kSelRowUnroll; ++u) {
                const int64_t t = t0 + u * bd;
                h[u] = t >= lo && t < hi ? row[t] : -1;
            }
#pragma unroll
            for (int u = 0; u < kSelRowUnroll; ++u) {
                const unsigned o = (unsigned)(h[u] - ps);
                if (h[u] < 0 || o >= (unsigned)np) continue;
                const T key = kf.pack(tkey[t0 + u * bd]);
                if (key) atomicMax(&kl[o], key);
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < np; k += blockDim.x) hitkey[ps + k] = kf.unpack(kl[k]);
        // kept bits, kSelRowUnroll waves' worth of entries per thread in flight
        for (int64_t t0 = a0 + threadIdx.x; t0 < a1; t0 += bd * kSelRowUnroll) {
            int h[kSelRowUnroll];
#pragma unroll
            for (int u = 0; u < kSelRowUnroll; ++u) {
                const int64_t t = t0 + u * bd;
                h[u] = t >= lo && t < hi ? row[t] : -1;
            }
#pragma unroll
            for (int u = 0; u < kSelRowUnroll; ++u) {
                const int64_t t = t0 + u * bd;
                if (t >= a1) break;   // whole waves: t's wave is a 64-aligned block
                bool kept = false;
                const unsigned o = (unsigned)(h[u] - ps);
                if (h[u] >= 0 && o < (unsigned)np) {
                    const T key = kf.pack(tkey[t]);
                    kept = key && kl[o] == key;
                }
                const unsigned long long mask = __ballot(kept);
                if (lane == 0 && mask) {
                    const int64_t w = t >> 6;
                    if (slice == 0 && w != w_first && w != w_last) kb[w] = mask;
                    else atomicOr(&kb[w], mask);
                }
            }
        }
        __syncthreads();
    }
}

// Kept counts per row chunk of the tracklets of big sectors from the bits.
__global__ __launch_bounds__(kBlock) void k_sel_count_bits(
    int n_rows, const int64_t* __restrict__ t_lo, const int64_t* __restrict__ t_hi,
    int64_t count_cap, int64_t n_words, const unsigned long long* __restrict__ tkey,
    const unsigned long long* __restrict__ kbits, uint8_t* __restrict__ ccnt)
{
    const int64_t lo = *t_lo < count_cap ? *t_lo : count_cap;
    const int64_t m = *t_hi < count_cap ? *t_hi : count_cap;
    for (int64_t t = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (tkey[t] == kKeyNotBig) continue;     // k_sel_chunk counts it
        const int64_t w = t >> 6;
        const int b = (int)(t & 63);
        for (int ra = 0, q = 0; ra < n_rows; ra += kSelRows, ++q) {
            const int rb = ra + kSelRows < n_rows ? ra + kSelRows : n_rows;
            int kept = 0;
            for (int rr = ra; rr < rb; ++rr) kept += (int)((kbits[(int64_t)rr * n_words + w] >> b) & 1ull);
            ccnt[q * count_cap + t] = (uint8_t)kept;
        }
    }
}

// per tracklet: 1 << 32 | kept if it becomes a track, else 0
__global__ __launch_bounds__(kBlock) void k_sel_len(
    int n_chunks, tpc_params prm, const int64_t* __restrict__ t_lo,
    const int64_t* __restrict__ t_hi, int64_t count_cap, const uint8_t* __restrict__ ccnt,
    uint64_t* __restrict__ tlen)
{
    const int64_t lo = *t_lo < count_cap ? *t_lo : count_cap;
    const int64_t m = *t_hi < count_cap ? *t_hi : count_cap;
    for (int64_t t = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
         t += (int64_t)gridDim.x * blockDim.x) {
        int kept = 0;
        for (int q = 0; q < n_chunks; ++q) kept += ccnt[q * count_cap + t];
        tlen[t] = kept >= prm.min_track_hits ? ((1ull << 32) | (uint64_t)kept) : 0ull;
    }
}

__global__ __launch_bounds__(kBlock) void k_sel_write(
    int n_rows, tpc_params prm, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_hits,
    const int32_t* __restrict__ t_nhits, const tpc_status* __restrict__ status, int64_t count_cap,
    int64_t cap, const unsigned long long* __restrict__ hitkey, const uint64_t* __restrict__ tlen,
    const uint64_t* __restrict__ toff, const uint8_t* __restrict__ ccnt,
    const tpc_sector* __restrict__ sec, const int32_t* __restrict__ gsr,
    int32_t* __restrict__ trk_off, TrkHitOut out, int32_t* __restrict__ trk_tracklet,
    int8_t* __restrict__ trk_side, int64_t trk_cap, int64_t hit_cap)
{
    int64_t m = status->n_starts;
    if (m > count_cap) m = count_cap;
    const int q = blockIdx.y;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (!tlen[t]) continue;
        const uint64_t to = toff[t];
        int64_t o = (int64_t)(to & 0xFFFFFFFFull);
        if (q == 0)
            sel_write_track(t, (int64_t)(to >> 32), o, t_start, sec, gsr, trk_off, trk_tracklet,
                            trk_side, trk_cap);
        if (!ccnt[q * count_cap + t]) continue;     // the chunk keeps nothing
        for (int j = 0; j < q; ++j) o += ccnt[j * count_cap + t];
        const uint64_t key = key_of(t, prm, idg, t_start, t_nhits);
        sel_write_chunk(t, q * kSelRows, n_rows, key, o, idg, t_hits, cap, hitkey, out, hit_cap);
    }
}

__global__ void k_sel_finish(const uint64_t* __restrict__ toff_total, tpc_status* status,
                             int32_t* __restrict__ trk_off, int64_t trk_cap, int64_t hit_cap)
{
    if (blockIdx.x || threadIdx.x) return;
    const uint64_t tot = *toff_total;
    const int64_t nt = (int64_t)(tot >> 32), nh = (int64_t)(tot & 0xFFFFFFFFull);
    status->n_tracks = nt;
    status->n_track_hits = nh;
    if (nt <= trk_cap) trk_off[nt] = (int32_t)nh;
    if (nt > trk_cap) status->overflow |= 2;
    if (nh > hit_cap) status->overflow |= 4;
}

// Track hits from their grid positions (written by k_sel_write in track
// order, with the rows): cluster ids and, when asked for, coordinates, one thread
// per hit, coalesced writes (the positions of one track lie in one sector's
// part of the grid).  Writing all of them from k_sel_write, whose threads
// hold a tracklet's row chunk each and write short runs at scattered
// offsets, took 923 us on the 512-instance set against 175 us for the ids
// alone.
__global__ __launch_bounds__(kBlock) void k_trk_copy(
    const tpc_status* __restrict__ status, int64_t cap, const int32_t* __restrict__ tpos,
    const int32_t* __restrict__ idg, const float* __restrict__ yg,
    const float* __restrict__ zg, int32_t* __restrict__ trk_hits, float* __restrict__ trk_y,
    float* __restrict__ trk_z)
{
    int64_t n = status->n_track_hits;
    if (n > cap) n = cap;
    // tiles of kCopyItems hits per thread (every load of a tile in flight
    // before its stores: the gathers are latency-bound), dealt to the XCDs
    // in contiguous ranges: the tracks of one sector, and the grid rows
    // their hits lie in, stay in one L2
    constexpr int kCopyItems = 4;
    const int64_t tile = (int64_t)blockDim.x * kCopyItems;
    const int64_t nb = (n + tile - 1) / tile;
    for (int64_t b0 = 0; b0 < nb; b0 += gridDim.x) {
        const int64_t chunk = nb - b0 < (int64_t)gridDim.x ? nb - b0 : (int64_t)gridDim.x;
        if ((int64_t)blockIdx.x >= chunk) break;
        const int64_t j0 = (b0 + xcd_remap(blockIdx.x, (int)chunk)) * tile + threadIdx.x;
        int p[kCopyItems];
#pragma unroll
        for (int u = 0; u < kCopyItems; ++u) {
            const int64_t j = j0 + (int64_t)u * blockDim.x;
            p[u] = j < n ? tpos[j] : -1;
        }
        int32_t id[kCopyItems];
        float yv[kCopyItems], zv[kCopyItems];
#pragma unroll
        for (int u = 0; u < kCopyItems; ++u) {
            if (p[u] < 0) continue;
            id[u] = idg[p[u]];
            if (trk_y) {
                yv[u] = yg[p[u]];
                zv[u] = zg[p[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < kCopyItems; ++u) {
            if (p[u] < 0) continue;
            const int64_t j = j0 + (int64_t)u * blockDim.x;
            trk_hits[j] = id[u];
            if (trk_y) {
                trk_y[j] = yv[u];
                trk_z[j] = zv[u];
            }
        }
    }
}

static unsigned sel_grid_x(int64_t n) { return grid_for_block(n, kBlock, 1024); }

// Ownership keys and kept-hit counts of the tracklets of sectors
// [sec_lo, sec_hi) (their hits are grid positions of those sectors).
int run_select_keys(const tpc_problem* p, int sec_lo, int sec_hi, tpc_grid grid,
                    int64_t count_cap, tpc_tracklets trl, const Workspace& ws, hipStream_t st)
{
    const int64_t c0 = p->h_sectors[sec_lo].begin, c1 = p->h_sectors[sec_hi - 1].end;
    const int64_t bound = (c1 - c0) / 3 + 1;
    const unsigned gx = sel_grid_x(bound < count_cap ? bound : count_cap);
    const int nq = sel_chunks(p->n_rows);
    const int64_t* lo = ws.sec_start + sec_lo;
    const int64_t* hi = ws.sec_start + sec_hi;
    TPC_LAUNCH(k_sel_chunk, dim3((unsigned)((sec_hi - sec_lo) * nq)), dim3(kBlock), 0, st,
               p->d_sectors, sec_lo, p->n_rows, p->params, (const int32_t*)grid.bin_start,
               (const int32_t*)grid.id, (const int32_t*)trl.start, (const int32_t*)trl.hits,
               (const int32_t*)trl.nhits, (const int64_t*)ws.sec_start, count_cap,
               trl.capacity, (unsigned long long*)ws.hitkey, ws.ccnt);
    bool any_big = false;
    for (int s = sec_lo; s < sec_hi && !any_big; ++s) any_big = sel_big(p->h_sectors[s], p->n_rows);
    if (any_big) {
        const int64_t n_words = sel_words(count_cap);
        TPC_LAUNCH(k_sel_prep_big, dim3(gx), dim3(kBlock), 0, st, p->d_sectors, p->n_rows,
                   p->params, (const int32_t*)grid.id, (const int32_t*)ws.gsr,
                   (const int32_t*)trl.start, (const int32_t*)trl.nhits, lo, hi, count_cap,
                   n_words, (unsigned long long*)ws.tkey, (unsigned long long*)ws.kbits);
        // 32-bit keys in LDS when every big sector has at most 2^24 clusters
        bool k32 = true;
        for (int s = sec_lo; s < sec_hi; ++s)
            if (sel_big(p->h_sectors[s], p->n_rows) &&
                p->h_sectors[s].end - p->h_sectors[s].begin > (int64_t(1) << 24))
                k32 = false;
        const dim3 gr((unsigned)((sec_hi - sec_lo) * p->n_rows));
        if (k32)
            TPC_LAUNCH(k_sel_rows_big<Key32>, gr, dim3(kSelRowBlock), 0, st, p->d_sectors, sec_lo,
                       p->n_rows, (const int32_t*)grid.bin_start, (const int32_t*)trl.hits,
                       (const int64_t*)ws.sec_start, count_cap, trl.capacity, n_words,
                       (const unsigned long long*)ws.tkey, (unsigned long long*)ws.hitkey,
                       (unsigned long long*)ws.kbits);
        else
            TPC_LAUNCH(k_sel_rows_big<Key64>, gr, dim3(kSelRowBlock), 0, st, p->d_sectors, sec_lo,
                       p->n_rows, (const int32_t*)grid.bin_start, (const int32_t*)trl.hits,
                       (const int64_t*)ws.sec_start, count_cap, trl.capacity, n_words,
                       (const unsigned long long*)ws.tkey, (unsigned long long*)ws.hitkey,
                       (unsigned long long*)ws.kbits);
        TPC_LAUNCH(k_sel_count_bits, dim3(gx), dim3(kBlock), 0, st, p->n_rows, lo, hi, count_cap,
                   n_words, (const unsigned long long*)ws.tkey,
                   (const unsigned long long*)ws.kbits, ws.ccnt);
    }
    TPC_LAUNCH(k_sel_len, dim3(gx), dim3(kBlock), 0, st, nq, p->params, lo, hi, count_cap,
               (const uint8_t*)ws.ccnt, ws.tlen);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

// Dense track list in tracklet order from the kept-hit counts of all
// tracklets [0, count_cap) (tlen zero where no track).
int run_select_compact(const tpc_problem* p, tpc_grid grid, int64_t count_cap,
                       tpc_tracklets trl, tpc_tracks trk, const Workspace& ws, hipStream_t st)
{
    const unsigned gx = sel_grid_x(count_cap);
    launch_scan<uint64_t>(ws.tlen, ws.toff, count_cap, true, nullptr, nullptr, ws.partials, st);
    TPC_LAUNCH(k_sel_write, dim3(gx, sel_chunks(p->n_rows)), dim3(kBlock), 0, st, p->n_rows,
               p->params, (const int32_t*)grid.id, (const int32_t*)trl.start,
               (const int32_t*)trl.hits, (const int32_t*)trl.nhits, (const tpc_status*)ws.status,
               count_cap, trl.capacity, (const unsigned long long*)ws.hitkey,
               (const uint64_t*)ws.tlen, (const uint64_t*)ws.toff, (const uint8_t*)ws.ccnt,
               p->d_sectors, (const int32_t*)ws.gsr, trk.off,
               TrkHitOut{ws.tpos, nullptr, trk.hit_y ? trk.hit_row : nullptr, nullptr, nullptr,
                         nullptr, nullptr},
               trk.tracklet, trk.side,
               trk.capacity, trk.hit_capacity);
    TPC_LAUNCH(k_sel_finish, dim3(1), dim3(1), 0, st, (const uint64_t*)(ws.toff + count_cap),
               ws.status, trk.off, trk.capacity, trk.hit_capacity);
    const int64_t hb = trk.hit_capacity < p->n_clusters ? trk.hit_capacity : p->n_clusters;
    TPC_LAUNCH(k_trk_copy, dim3(grid_for(ceil_div(hb, 4))), dim3(kBlock), 0, st,
               (const tpc_status*)ws.status, hb, (const int32_t*)ws.tpos,
               (const int32_t*)grid.id, (const float*)grid.y, (const float*)grid.z, trk.hits,
               trk.hit_y, trk.hit_z);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

int run_select_tracks(const tpc_problem* p, tpc_grid grid, int64_t count_cap,
                      tpc_tracklets trl, tpc_tracks trk, const Workspace& ws, hipStream_t st)
{
    launch_fill<uint64_t>(ws.tlen, 0ull, count_cap + 1, st);
    int r = run_select_keys(p, 0, p->n_sectors, grid, count_cap, trl, ws, st);
    if (!r) r = run_select_compact(p, grid, count_cap, trl, trk, ws, st);
    return r;
}

}  // namespace tpc
