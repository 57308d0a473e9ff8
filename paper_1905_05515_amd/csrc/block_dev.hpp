// Block-wide scans for 256-thread blocks (device code shared by several
// kernels).
#pragma once
#include "tpc_internal.hpp"

namespace tpc {

// ---- block scan ---------------------------------------------------------------
// Exclusive scan of one value per thread over a 256-thread block: wave-level
// inclusive scan with shuffles, wave totals through LDS.

template <typename T>
__device__ inline T wave_incl_scan(T x)
{
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    return x;
}

template <typename T>
__device__ inline T block_excl_scan(T v, T* lds, T* total)
{
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    T x = wave_incl_scan(v);
    if (lane == kWave - 1) lds[wid] = x;
    __syncthreads();
    T before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        T s = lds[w];
        before += (w < wid) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
}

template <typename T>
__device__ inline T block_sum(T v, T* lds)
{
    T tot;
    block_excl_scan(v, lds, &tot);
    return tot;
}

}  // namespace tpc
