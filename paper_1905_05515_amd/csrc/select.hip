// Tracklet selection: every cluster goes to the tracklet of largest key
// (hits << 32 | (2^32 - 1 - start id)) containing it, among tracklets with
// at least min_tracklet_hits hits (64-bit atomic max, order independent); a
// tracklet keeping at least min_track_hits clusters becomes a track.
// Tracks are compacted in tracklet order by a scan of (accepted, kept).
#include "select_dev.hpp"

namespace tpc {

// Sectors whose row chunks hold on average several times more positions
// than the LDS table take the tracklet-parallel form with device-wide
// atomics instead (same keys and counts): one block per chunk would loop
// over too many tracklets.  A chunk just over the table still uses its
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
    if (sel_big(s, n_rows)) {   // the tracklet-parallel kernels take this sector
        const int ra = q * kSelRows, rb = ra + kSelRows < n_rows ? ra + kSelRows : n_rows;
        const int per_row = s.nbz * s.nby;
        const int p0 = bin_start[s.bin_base + ra * per_row];
        const int np = bin_start[s.bin_base + rb * per_row] - p0;
        for (int k = threadIdx.x; k < np; k += blockDim.x) hitkey[p0 + k] = 0ull;
        return;
    }
    int64_t lo = sec_start[si], hi = sec_start[si + 1];
    if (lo < 0) lo = 0;
    sel_chunk_block(s, q, n_rows, prm, bin_start, idg, t_start, t_hits, t_nhits, lo, hi,
                    count_cap, cap, hitkey, ccnt, kl, kSelLds);
}

// Tracklet-parallel form for big sectors.  Keys: one thread per tracklet
// claims its hits with device-wide 64-bit atomics, reading its rows upwards
// from its innermost hit until all its hits are seen (every hit row lies in
// [t_rin, last hit row]), and records that row span.  Tracklets of other
// sectors are left to k_sel_chunk.
constexpr uint16_t kSpanOther = 0xFFFE;   // tracklet of a sector that is not big
constexpr uint16_t kSpanNone = 0xFFFF;    // takes no part in the selection

__global__ __launch_bounds__(kBlock) void k_sel_keys_big(
    const tpc_sector* __restrict__ sec, int n_rows, tpc_params prm,
    const int32_t* __restrict__ idg, const int32_t* __restrict__ gsr,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_hits,
    const int32_t* __restrict__ t_nhits, const int32_t* __restrict__ t_rin,
    const int64_t* __restrict__ t_lo, const int64_t* __restrict__ t_hi, int64_t count_cap,
    int64_t cap, unsigned long long* __restrict__ hitkey, uint16_t* __restrict__ tspan)
{
    const int64_t lo = *t_lo < count_cap ? *t_lo : count_cap;
    const int64_t m = *t_hi < count_cap ? *t_hi : count_cap;
    for (int64_t t = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (!sel_big(sec[gsr[t_start[t]] >> 8], n_rows)) {
            tspan[t] = kSpanOther;
            continue;
        }
        const uint64_t key = key_of(t, prm, idg, t_start, t_nhits);
        const int nh = t_nhits[t];
        int r = t_rin[t];
        if (!key || r < 0 || r >= n_rows) {
            tspan[t] = kSpanNone;
            continue;
        }
        const int first = r;
        int last = r, seen = 0;
        for (; r < n_rows && seen < nh; ++r) {
            const int h = t_hits[(int64_t)r * cap + t];
            if (h < 0) continue;
            // keys only grow: a value seen here is a lower bound of the
            // current one, so a hit that already holds a key >= ours needs
            // no atomic (most hits are claimed by several tracklets)
            const unsigned long long seen_key =
                __hip_atomic_load(&hitkey[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (seen_key < key) atomicMax(&hitkey[h], (unsigned long long)key);
            ++seen;
            last = r;
        }
        tspan[t] = (uint16_t)(first | (last << 8));
    }
}

// Counts: item (t, blockIdx.y) handles rows [8 y, 8 y + 8) of tracklet t;
// a chunk outside the tracklet's row span is zero without a load.
__global__ __launch_bounds__(kBlock) void k_sel_count_big(
    int n_rows, tpc_params prm, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_hits,
    const int32_t* __restrict__ t_nhits, const int64_t* __restrict__ t_lo,
    const int64_t* __restrict__ t_hi, int64_t count_cap, int64_t cap,
    const unsigned long long* __restrict__ hitkey, const uint16_t* __restrict__ tspan,
    uint8_t* __restrict__ ccnt)
{
    const int64_t lo = *t_lo < count_cap ? *t_lo : count_cap;
    const int64_t m = *t_hi < count_cap ? *t_hi : count_cap;
    const int ra = blockIdx.y * kSelRows;
    for (int64_t t = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int sp = tspan[t];
        if (sp == kSpanOther) continue;
        int kept = 0;
        if (sp != kSpanNone && ra + kSelRows > (sp & 255) && ra <= (sp >> 8))
            kept = sel_count_chunk(t, ra, n_rows, key_of(t, prm, idg, t_start, t_nhits), t_hits,
                                   cap, hitkey);
        ccnt[blockIdx.y * count_cap + t] = (uint8_t)kept;
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
    int32_t* __restrict__ trk_off, int32_t* __restrict__ trk_hits,
    int32_t* __restrict__ trk_tracklet, int8_t* __restrict__ trk_side, int64_t trk_cap,
    int64_t hit_cap)
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
        sel_write_chunk(t, q * kSelRows, n_rows, key, o, idg, t_hits, cap, hitkey, trk_hits,
                        hit_cap);
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
        TPC_LAUNCH(k_sel_keys_big, dim3(gx), dim3(kBlock), 0, st, p->d_sectors, p->n_rows,
                   p->params, (const int32_t*)grid.id, (const int32_t*)ws.gsr,
                   (const int32_t*)trl.start, (const int32_t*)trl.hits,
                   (const int32_t*)trl.nhits, (const int32_t*)trl.row_inner, lo, hi, count_cap,
                   trl.capacity, (unsigned long long*)ws.hitkey, ws.tspan);
        TPC_LAUNCH(k_sel_count_big, dim3(gx, nq), dim3(kBlock), 0, st, p->n_rows, p->params,
                   (const int32_t*)grid.id, (const int32_t*)trl.start,
                   (const int32_t*)trl.hits, (const int32_t*)trl.nhits, lo, hi, count_cap,
                   trl.capacity, (const unsigned long long*)ws.hitkey,
                   (const uint16_t*)ws.tspan, ws.ccnt);
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
               p->d_sectors, (const int32_t*)ws.gsr, trk.off, trk.hits, trk.tracklet, trk.side,
               trk.capacity, trk.hit_capacity);
    TPC_LAUNCH(k_sel_finish, dim3(1), dim3(1), 0, st, (const uint64_t*)(ws.toff + count_cap),
               ws.status, trk.off, trk.capacity, trk.hit_capacity);
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
