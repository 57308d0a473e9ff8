// Device code of the tracklet selection, shared by the staged kernels and
// the persistent kernel.  Every tracklet's rows are read in chunks of
// kSelRows so that one item loads its chunk's hits at once; the staged
// kernels give each (sector, chunk) a block, the persistent kernel walks all
// chunks of a tracklet in one thread.
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

// write the kept hits (cluster ids) of one row chunk from hit offset o on;
// returns the offset after them
__device__ __forceinline__ int64_t sel_write_chunk(
    int64_t t, int ra, int n_rows, uint64_t key, int64_t o, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_hits, int64_t cap,
    const unsigned long long* __restrict__ hitkey, int32_t* __restrict__ trk_hits,
    int64_t hit_cap)
{
    int c[kSelRows];
    load_chunk(t, ra, n_rows, t_hits, cap, c);
    bool keep[kSelRows];
#pragma unroll
    for (int k = 0; k < kSelRows; ++k) keep[k] = c[k] >= 0 && hitkey[c[k]] == key;
#pragma unroll
    for (int k = 0; k < kSelRows; ++k)
        if (keep[k]) {
            if (o < hit_cap) trk_hits[o] = idg[c[k]];
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

// ---- whole tracklet in one thread (persistent kernel) -----------------------

__device__ __forceinline__ void sel_keys_one(
    int64_t t, int n_rows, const tpc_params& prm, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_hits,
    const int32_t* __restrict__ t_nhits, int64_t cap, unsigned long long* __restrict__ hitkey)
{
    const uint64_t key = key_of(t, prm, idg, t_start, t_nhits);
    if (!key) return;
    for (int ra = 0; ra < n_rows; ra += kSelRows)
        sel_keys_chunk(t, ra, n_rows, key, t_hits, cap, hitkey);
}

// 1 << 32 | kept hits if tracklet t becomes a track, else 0
__device__ __forceinline__ uint64_t sel_count_one(
    int64_t t, int n_rows, const tpc_params& prm, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_hits,
    const int32_t* __restrict__ t_nhits, int64_t cap,
    const unsigned long long* __restrict__ hitkey)
{
    const uint64_t key = key_of(t, prm, idg, t_start, t_nhits);
    if (!key) return 0ull;
    int kept = 0;
    for (int ra = 0; ra < n_rows; ra += kSelRows)
        kept += sel_count_chunk(t, ra, n_rows, key, t_hits, cap, hitkey);
    return kept >= prm.min_track_hits ? ((1ull << 32) | (uint64_t)kept) : 0ull;
}

// write track k = toff >> 32 of tracklet t at hit offset toff & (2^32 - 1)
__device__ __forceinline__ void sel_write_one(
    int64_t t, uint64_t toff, int n_rows, const tpc_params& prm,
    const int32_t* __restrict__ idg, const int32_t* __restrict__ t_start,
    const int32_t* __restrict__ t_hits, const int32_t* __restrict__ t_nhits, int64_t cap,
    const unsigned long long* __restrict__ hitkey, const tpc_sector* __restrict__ sec,
    const int32_t* __restrict__ gsr, int32_t* __restrict__ trk_off,
    int32_t* __restrict__ trk_hits, int32_t* __restrict__ trk_tracklet,
    int8_t* __restrict__ trk_side, int64_t trk_cap, int64_t hit_cap)
{
    int64_t o = (int64_t)(toff & 0xFFFFFFFFull);
    sel_write_track(t, (int64_t)(toff >> 32), o, t_start, sec, gsr, trk_off, trk_tracklet,
                    trk_side, trk_cap);
    const uint64_t key = key_of(t, prm, idg, t_start, t_nhits);
    for (int ra = 0; ra < n_rows; ra += kSelRows)
        o = sel_write_chunk(t, ra, n_rows, key, o, idg, t_hits, cap, hitkey, trk_hits, hit_cap);
}

}  // namespace tpc
