// Per-item device code of the grid build, shared by the staged kernels and
// the persistent kernel.
#pragma once
#include "tpc_internal.hpp"

namespace tpc {

__device__ __forceinline__ void grid_count_one(
    const tpc_sector* __restrict__ sec, int n_sec, int n_rows, const uint8_t* __restrict__ row,
    const float* __restrict__ y, const float* __restrict__ z, int64_t i,
    int32_t* __restrict__ cnt, tpc_status* status)
{
    const int r = row[i];
    if (r >= n_rows) atomicAdd((unsigned long long*)&status->n_bad_rows, 1ull);
    const tpc_sector& s = sec[find_sector(sec, n_sec, i)];
    atomicAdd(&cnt[global_bin(s, n_rows, r, y[i], z[i])], 1);
}

__device__ __forceinline__ void grid_scatter_one(
    const tpc_sector* __restrict__ sec, int n_sec, int n_rows, const uint8_t* __restrict__ row,
    const float* __restrict__ y, const float* __restrict__ z, int64_t i,
    const int32_t* __restrict__ bin_start, int32_t* __restrict__ fill, int32_t* __restrict__ tmp)
{
    const tpc_sector& s = sec[find_sector(sec, n_sec, i)];
    const int g = global_bin(s, n_rows, row[i], y[i], z[i]);
    const int slot = atomicAdd(&fill[g], 1);
    tmp[bin_start[g] + slot] = (int32_t)i;
}

// final place of the cluster at staging position p: its bin start plus the
// number of clusters of the bin with a smaller id
__device__ __forceinline__ void grid_rank_one(
    const tpc_sector* __restrict__ sec, int n_sec, int n_rows, const uint8_t* __restrict__ row,
    const float* __restrict__ y, const float* __restrict__ z,
    const int32_t* __restrict__ bin_start, int64_t p, const int32_t* __restrict__ tmp,
    float* __restrict__ yg, float* __restrict__ zg, int32_t* __restrict__ idg,
    int32_t* __restrict__ gsr)
{
    const int32_t id = tmp[p];
    const int si = find_sector(sec, n_sec, id);
    const tpc_sector& s = sec[si];
    const int r = row[id];
    const float yy = y[id], zz = z[id];
    const int g = global_bin(s, n_rows, r, yy, zz);
    const int32_t bs = bin_start[g], be = bin_start[g + 1];
    int rank = 0;
    for (int32_t q = bs; q < be; ++q) rank += tmp[q] < id;
    const int32_t o = bs + rank;
    yg[o] = yy;
    zg[o] = zz;
    idg[o] = id;
    gsr[o] = (si << 8) | r;
}

}  // namespace tpc
