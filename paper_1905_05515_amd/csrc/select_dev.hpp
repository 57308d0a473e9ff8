// Device code of the tracklet selection, shared by the staged kernels and
// the persistent kernel.  Every tracklet's rows are read in chunks of
// kSelRows so that one item loads its chunk's hits at once.
#pragma once
#include "tpc_internal.hpp"

namespace tpc {

__device__ __forceinline__ uint64_t tracklet_key(int nh, int start_id, int min_hits)
{
    return nh >= min_hits ? (((uint64_t)nh << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)start_id)) : 0ull;
}

__device__ __forceinline__ uint64_t key_of(int64_t t, const tpc_params& prm,
                                           const int32_t* __restrict__ idg,
                                           const int32_t* __restrict__ t_start,
                                           const int32_t* __restrict__ t_nhits)
{
    return tracklet_key(t_nhits[t], idg[t_start[t]], prm.min_tracklet_hits);
}

// hits of rows [ra, ra + kSelRows) of tracklet t (-1 at and beyond n_rows)
__device__ __forceinline__ void load_chunk(int64_t t, int ra, int n_rows,
                                           const int32_t* __restrict__ t_hits, int64_t cap,
                                           int* c)
{
#pragma unroll
    for (int k = 0; k < kSelRows; ++k)
        c[k] = ra + k < n_rows ? t_hits[(int64_t)(ra + k) * cap + t] : -1;
}

// claim the hits of one row chunk with the tracklet's key (64-bit atomic max)
__device__ __forceinline__ void sel_keys_chunk(int64_t t, int ra, int n_rows, uint64_t key,
                                               const int32_t* __restrict__ t_hits, int64_t cap,
                                               unsigned long long* __restrict__ hitkey)
{
    int c[kSelRows];
    load_chunk(t, ra, n_rows, t_hits, cap, c);
#pragma unroll
    for (int k = 0; k < kSelRows; ++k)
        if (c[k] >= 0) atomicMax(&hitkey[c[k]], (unsigned long long)key);
}

// hits of one row chunk that the tracklet keeps (its key owns them)
__device__ __forceinline__ int sel_count_chunk(int64_t t, int ra, int n_rows, uint64_t key,
                                               const int32_t* __restrict__ t_hits, int64_t cap,
                                               const unsigned long long* __restrict__ hitkey)
{
    int c[kSelRows];
    load_chunk(t, ra, n_rows, t_hits, cap, c);
    int kept = 0;
#pragma unroll
    for (int k = 0; k < kSelRows; ++k) kept += c[k] >= 0 && hitkey[c[k]] == key;
    return kept;
}

// where the kept hits go: with pos set, their grid positions and (row set)
// their rows (a coalesced pass writes the rest, see k_trk_copy); else the
// cluster ids and
// (when y is set) the hits' rows and coordinates in the same order, read
// from the grid
struct TrkHitOut {
    int32_t* pos;
    int32_t* id;
    uint8_t* row;
    float* y;
    float* z;
    const float* yg;
    const float* zg;
};

// write the kept hits of one row chunk from hit offset o on; returns the
// offset after them
__device__ __forceinline__ int64_t sel_write_chunk(
    int64_t t, int ra, int n_rows, uint64_t key, int64_t o, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_hits, int64_t cap,
    const unsigned long long* __restrict__ hitkey, const TrkHitOut& out, int64_t hit_cap)
{
    int c[kSelRows];
    load_chunk(t, ra, n_rows, t_hits, cap, c);
    bool keep[kSelRows];
#pragma unroll
    for (int k = 0; k < kSelRows; ++k) keep[k] = c[k] >= 0 && hitkey[c[k]] == key;
#pragma unroll
    for (int k = 0; k < kSelRows; ++k)
        if (keep[k]) {
            if (o < hit_cap && out.pos) {
                out.pos[o] = c[k];
                if (out.row) out.row[o] = (uint8_t)(ra + k);
            } else if (o < hit_cap) {
                out.id[o] = idg[c[k]];
                if (out.y) {
                    out.row[o] = (uint8_t)(ra + k);
                    out.y[o] = out.yg[c[k]];
                    out.z[o] = out.zg[c[k]];
                }
            }
            ++o;
        }
    return o;
}

// track record of tracklet t as track k at hit offset o
__device__ __forceinline__ void sel_write_track(
    int64_t t, int64_t k, int64_t o, const int32_t* __restrict__ t_start,
    const tpc_sector* __restrict__ sec, const int32_t* __restrict__ gsr,
    int32_t* __restrict__ trk_off, int32_t* __restrict__ trk_tracklet,
    int8_t* __restrict__ trk_side, int64_t trk_cap)
{
    if (k < trk_cap) {
        trk_tracklet[k] = (int32_t)t;
        trk_off[k] = (int32_t)o;
        if (trk_side) trk_side[k] = sec[gsr[t_start[t]] >> 8].side < 0 ? -1 : 1;
    }
}

// Ownership keys by (sector, chunk of kSelRows pad rows): a tracklet's hits
// on those rows are grid positions of one contiguous range, so one block
// keeps the range's keys in LDS (kl[lds_cap], 64-bit LDS atomic max, no
// device-wide atomics), writes them out, and counts for every tracklet of
// the sector the hits of the chunk it keeps (ccnt[q * count_cap + t]).  A
// range larger than the LDS table uses the device-wide keys instead.
constexpr int kSelLds = 6144;   // LDS table of the staged kernel
constexpr int kSelKeep = 2;     // tracklets per thread kept in registers between passes

// tracklets [lo, hi) of the sector
__device__ __forceinline__ void sel_chunk_block(
    const tpc_sector& s, int q, int n_rows, const tpc_params& prm,
    const int32_t* __restrict__ bin_start, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_hits,
    const int32_t* __restrict__ t_nhits, int64_t lo, int64_t hi, int64_t count_cap,
    int64_t cap, unsigned long long* __restrict__ hitkey, uint8_t* __restrict__ ccnt,
    unsigned long long* kl, int lds_cap)
{
    const int ra = q * kSelRows, rb = ra + kSelRows < n_rows ? ra + kSelRows : n_rows;
    const int per_row = s.nbz * s.nby;
    const int p0 = bin_start[s.bin_base + ra * per_row];
    const int np = bin_start[s.bin_base + rb * per_row] - p0;
    if (hi > count_cap) hi = count_cap;
    if (lo < 0) lo = 0;
    if (lo > hi) lo = hi;
    const bool local = np <= lds_cap;
    for (int k = threadIdx.x; k < np; k += blockDim.x) {
        if (local) kl[k] = 0ull;
        else hitkey[p0 + k] = 0ull;
    }
    if (!local) __threadfence();
    __syncthreads();
    // the first kSelKeep tracklets of every thread keep their keys and
    // chunk hits in registers for the counting pass (one read of the
    // tracklet arrays instead of two for sectors of up to kSelKeep
    // tracklets per thread)
    uint64_t kkey[kSelKeep];
    int kc[kSelKeep][kSelRows];
#pragma unroll
    for (int u = 0; u < kSelKeep; ++u) {
        const int64_t t = lo + threadIdx.x + (int64_t)u * blockDim.x;
        kkey[u] = t < hi ? key_of(t, prm, idg, t_start, t_nhits) : 0ull;
        if (kkey[u]) load_chunk(t, ra, n_rows, t_hits, cap, kc[u]);
    }
#pragma unroll
    for (int u = 0; u < kSelKeep; ++u) {
        if (!kkey[u]) continue;
#pragma unroll
        for (int k = 0; k < kSelRows; ++k) {
            const unsigned o = (unsigned)(kc[u][k] - p0);
            if (kc[u][k] < 0 || o >= (unsigned)np) continue;
            if (local) atomicMax(&kl[o], (unsigned long long)kkey[u]);
            else atomicMax(&hitkey[kc[u][k]], (unsigned long long)kkey[u]);
        }
    }
    for (int64_t t = lo + threadIdx.x + (int64_t)kSelKeep * blockDim.x; t < hi;
         t += blockDim.x) {
        const uint64_t key = key_of(t, prm, idg, t_start, t_nhits);
        if (!key) continue;
        int c[kSelRows];
        load_chunk(t, ra, n_rows, t_hits, cap, c);
#pragma unroll
        for (int k = 0; k < kSelRows; ++k) {
            const unsigned o = (unsigned)(c[k] - p0);
            if (c[k] < 0 || o >= (unsigned)np) continue;
            if (local) atomicMax(&kl[o], (unsigned long long)key);
            else atomicMax(&hitkey[c[k]], (unsigned long long)key);
        }
    }
    if (!local) __threadfence();
    __syncthreads();
    if (local)
        for (int k = threadIdx.x; k < np; k += blockDim.x) hitkey[p0 + k] = kl[k];
#pragma unroll
    for (int u = 0; u < kSelKeep; ++u) {
        const int64_t t = lo + threadIdx.x + (int64_t)u * blockDim.x;
        if (t >= hi) continue;
        int kept = 0;
        if (kkey[u]) {
#pragma unroll
            for (int k = 0; k < kSelRows; ++k) {
                const unsigned o = (unsigned)(kc[u][k] - p0);
                if (kc[u][k] < 0 || o >= (unsigned)np) continue;
                const unsigned long long h = local ? kl[o] : hitkey[kc[u][k]];
                kept += h == kkey[u];
            }
        }
        ccnt[q * count_cap + t] = (uint8_t)kept;
    }
    for (int64_t t = lo + threadIdx.x + (int64_t)kSelKeep * blockDim.x; t < hi;
         t += blockDim.x) {
        const uint64_t key = key_of(t, prm, idg, t_start, t_nhits);
        int kept = 0;
        if (key) {
            int c[kSelRows];
            load_chunk(t, ra, n_rows, t_hits, cap, c);
#pragma unroll
            for (int k = 0; k < kSelRows; ++k) {
                const unsigned o = (unsigned)(c[k] - p0);
                if (c[k] < 0 || o >= (unsigned)np) continue;
                const unsigned long long h = local ? kl[o] : hitkey[c[k]];
                kept += h == key;
            }
        }
        ccnt[q * count_cap + t] = (uint8_t)kept;
    }
}

// the kept hits of tracklet t (cluster ids, row order) from hit offset o on;
// ccnt[q * count_cap + t]: kept hits of row chunk q (chunks without any are
// skipped)
__device__ __forceinline__ void sel_write_hits(
    int64_t t, int64_t o, int n_rows, const tpc_params& prm, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_hits,
    const int32_t* __restrict__ t_nhits, int64_t cap,
    const unsigned long long* __restrict__ hitkey, const uint8_t* __restrict__ ccnt,
    int64_t count_cap, const TrkHitOut& out, int64_t hit_cap)
{
    const uint64_t key = key_of(t, prm, idg, t_start, t_nhits);
    for (int ra = 0, q = 0; ra < n_rows; ra += kSelRows, ++q) {
        const int kept = ccnt[q * count_cap + t];
        if (kept) sel_write_chunk(t, ra, n_rows, key, o, idg, t_hits, cap, hitkey, out, hit_cap);
        o += kept;
    }
}

}  // namespace tpc
