// Per-item device code of the tracklet selection, shared by the staged
// kernels and the persistent kernel.
#pragma once
#include "tpc_internal.hpp"

namespace tpc {

__device__ __forceinline__ uint64_t tracklet_key(int nh, int start_id, int min_hits)
{
    return nh >= min_hits ? (((uint64_t)nh << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)start_id)) : 0ull;
}

// claim the hits of tracklet t with its key (64-bit atomic max)
__device__ __forceinline__ void sel_keys_one(
    int64_t t, int n_rows, const tpc_params& prm, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_hits,
    const int32_t* __restrict__ t_nhits, int64_t cap, unsigned long long* __restrict__ hitkey)
{
    const uint64_t key = tracklet_key(t_nhits[t], idg[t_start[t]], prm.min_tracklet_hits);
    if (!key) return;
    for (int r = 0; r < n_rows; ++r) {
        const int c = t_hits[(int64_t)r * cap + t];
        if (c >= 0) atomicMax(&hitkey[c], (unsigned long long)key);
    }
}

// 1 << 32 | kept hits if tracklet t becomes a track, else 0
__device__ __forceinline__ uint64_t sel_count_one(
    int64_t t, int n_rows, const tpc_params& prm, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_hits,
    const int32_t* __restrict__ t_nhits, int64_t cap,
    const unsigned long long* __restrict__ hitkey)
{
    const uint64_t key = tracklet_key(t_nhits[t], idg[t_start[t]], prm.min_tracklet_hits);
    if (!key) return 0ull;
    int kept = 0;
    for (int r = 0; r < n_rows; ++r) {
        const int c = t_hits[(int64_t)r * cap + t];
        kept += c >= 0 && hitkey[c] == key;
    }
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
    const int64_t k = (int64_t)(toff >> 32);
    int64_t o = (int64_t)(toff & 0xFFFFFFFFull);
    if (k < trk_cap) {
        trk_tracklet[k] = (int32_t)t;
        trk_off[k] = (int32_t)o;
        if (trk_side) trk_side[k] = sec[gsr[t_start[t]] >> 8].side < 0 ? -1 : 1;
    }
    const uint64_t key = tracklet_key(t_nhits[t], idg[t_start[t]], prm.min_tracklet_hits);
    for (int r = 0; r < n_rows; ++r) {
        const int c = t_hits[(int64_t)r * cap + t];
        if (c >= 0 && hitkey[c] == key) {
            if (o < hit_cap) trk_hits[o] = idg[c];
            ++o;
        }
    }
}

}  // namespace tpc
