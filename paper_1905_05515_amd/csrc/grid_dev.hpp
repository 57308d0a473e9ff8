// Device code of the grid build shared by the staged kernels (grid.hip) and
// the persistent kernel: the bucket of a cluster (a z slab of its pad row),
// the per-bucket bin sort of one block, and the final placement.
#pragma once
#include "block_dev.hpp"

namespace tpc {

// bucket of a cluster inside its sector
__device__ __forceinline__ int cluster_bucket(const tpc_sector& s, int n_rows, int S, int r,
                                              float z)
{
    if (r >= n_rows) return n_rows * S;
    const int iz = bin_of(z, s.z0, s.inv_bz, s.nbz);
    return r * S + iz / slab_zbins(s);
}

__device__ __forceinline__ int ctr_load(const int* c, bool local)
{
    return local ? c[0] : __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One block: bucket bk of sector si.  Counts the bucket's clusters per bin
// (in LDS, lds[kRowBinsLds]; in the device-wide counters cnt when the
// bucket has more bins), scans the counts into the bin starts and deals
// every cluster a slot of its bin (any order inside a bin).
__device__ __forceinline__ void grid_bins_bucket(
    const tpc_sector& s, int si, int bk, int n_rows, int S, const int32_t* __restrict__ rstart,
    const float* __restrict__ gy, const float* __restrict__ gz, const int32_t* __restrict__ gid,
    const uint8_t* __restrict__ row, int32_t* __restrict__ bin_start, int32_t* __restrict__ cnt,
    int32_t* __restrict__ gslot, int32_t* __restrict__ gbin, int32_t* __restrict__ gtag,
    int* lds, int* red, int lds_bins = kRowBinsLds)
{
    const int Rb = (n_rows + 1) * S;
    const int r = bk / S, slab = bk % S;
    const int zs = slab_zbins(s);
    if (slab >= (r < n_rows ? slab_count(s) : 1)) return;    // no such slab: no clusters
    const int a = rstart[(int64_t)si * Rb + bk], n = rstart[(int64_t)si * Rb + bk + 1] - a;
    const int per_row = s.nbz * s.nby;
    const int z_lo = slab * zs;
    const int z_hi = z_lo + zs < s.nbz ? z_lo + zs : s.nbz;
    const int nbr = r < n_rows ? (z_hi - z_lo) * s.nby : 1;
    const int g0 = s.bin_base + r * per_row + (r < n_rows ? z_lo * s.nby : 0);
    const bool local = nbr <= lds_bins;
    int* ctr = local ? lds : cnt + g0;
    for (int b = threadIdx.x; b < nbr; b += blockDim.x) ctr[b] = 0;
    if (!local) __threadfence();
    __syncthreads();
    for (int j = a + threadIdx.x; j < a + n; j += blockDim.x) {
        const int b = r < n_rows ? (bin_of(gz[j], s.z0, s.inv_bz, s.nbz) - z_lo) * s.nby +
                                       bin_of(gy[j], s.y0, s.inv_by, s.nby)
                                 : 0;
        atomicAdd(&ctr[b], 1);
    }
    if (!local) __threadfence();
    __syncthreads();
    // bin starts: exclusive scan of the counts from the bucket start
    int carry = a;
    for (int b0 = 0; b0 < nbr; b0 += kScanTile) {
        const int base = b0 + (int)threadIdx.x * kScanItems;
        int v[kScanItems];
        int sum = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = base + k < nbr ? ctr_load(ctr + base + k, local) : 0;
            sum += v[k];
        }
        int tot;
        int ex = block_excl_scan(sum, red, &tot) + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < nbr) {
                bin_start[g0 + base + k] = ex;
                ctr[base + k] = ex;
                ex += v[k];
            }
        carry += tot;
    }
    if (r == n_rows && threadIdx.x == 0) bin_start[g0 + 1] = a + n;
    if (!local) __threadfence();
    __syncthreads();
    for (int j = a + threadIdx.x; j < a + n; j += blockDim.x) {
        const int b = r < n_rows ? (bin_of(gz[j], s.z0, s.inv_bz, s.nbz) - z_lo) * s.nby +
                                       bin_of(gy[j], s.y0, s.inv_by, s.nby)
                                 : 0;
        const int slot = atomicAdd(&ctr[b], 1);
        gslot[slot] = j;
        gbin[slot] = g0 + b;
        // invalid rows keep their raw row value
        gtag[slot] = (si << 8) | (r < n_rows ? r : (int)row[gid[j]]);
    }
}

// Bucket sort and placement in one block, for buckets of at most
// kFuseMax clusters over at most fuse_bins bins: the cluster ids, their
// bins, the bin counters and the binned order stay in LDS; every cluster's
// place is its bin start plus the number of clusters of its bin with a
// smaller id (the stable order), as in the two-pass form.  The counters are
// 16-bit offsets from the bucket start (a bucket holds at most kFuseMax
// clusters), two to a 32-bit word, incremented by 32-bit LDS atomics on the
// word: a small LDS footprint lets more blocks share a compute unit, which
// is what this latency-bound step needs.  LDS use (ints): fused_lds_ints.
// Returns false, touching nothing, when the bucket is larger.
constexpr int kFuseBins = kRowBinsLds;   // every slab (16-bit counters, two a word)
constexpr int kFuseMax = 1024;

__host__ __device__ inline int fused_lds_ints(int fuse_bins)
{
    return (fuse_bins + 1) / 2 + 3 * kFuseMax;
}

__device__ __forceinline__ bool grid_bins_place_fused(
    const tpc_sector& s, int si, int bk, int n_rows, int S, const int32_t* __restrict__ rstart,
    const float* __restrict__ gy, const float* __restrict__ gz, const int32_t* __restrict__ gid,
    const uint8_t* __restrict__ row, int32_t* __restrict__ bin_start, float* __restrict__ yg,
    float* __restrict__ zg, int32_t* __restrict__ idg, int32_t* __restrict__ gsr, int* smem,
    int* red, int fuse_bins)
{
    const int Rb = (n_rows + 1) * S;
    const int r = bk / S, slab = bk % S;
    if (slab >= (r < n_rows ? slab_count(s) : 1)) return true;   // no such slab: nothing
    const int zs = slab_zbins(s);
    const int a = rstart[(int64_t)si * Rb + bk], n = rstart[(int64_t)si * Rb + bk + 1] - a;
    const int per_row = s.nbz * s.nby;
    const int z_lo = slab * zs;
    const int z_hi = z_lo + zs < s.nbz ? z_lo + zs : s.nbz;
    const int nbr = r < n_rows ? (z_hi - z_lo) * s.nby : 1;
    if (n > kFuseMax || nbr > fuse_bins) return false;
    const int g0 = s.bin_base + r * per_row + (r < n_rows ? z_lo * s.nby : 0);
    uint32_t* cw = reinterpret_cast<uint32_t*>(smem);   // [(fuse_bins + 1) / 2] counter pairs
    uint16_t* c16 = reinterpret_cast<uint16_t*>(smem);  // the same as 16-bit counters
    int* lid = smem + (fuse_bins + 1) / 2;              // [kFuseMax] cluster ids
    int* lb = lid + kFuseMax;                           // [kFuseMax] bins
    int* mem = lb + kFuseMax;                           // [kFuseMax] binned order
    for (int k = threadIdx.x; k < (nbr + 1) / 2; k += blockDim.x) cw[k] = 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float y = gy[a + i], z = gz[a + i];
        const int b = r < n_rows ? (bin_of(z, s.z0, s.inv_bz, s.nbz) - z_lo) * s.nby +
                                       bin_of(y, s.y0, s.inv_by, s.nby)
                                 : 0;
        lid[i] = gid[a + i];
        lb[i] = b;
        atomicAdd(&cw[b >> 1], 1u << ((b & 1) << 4));
    }
    __syncthreads();
    // bin starts: exclusive scan of the counts (16-bit offsets in LDS, the
    // absolute positions a + offset in the grid)
    int carry = 0;
    for (int b0 = 0; b0 < nbr; b0 += kScanTile) {
        const int base = b0 + (int)threadIdx.x * kScanItems;
        int v[kScanItems];
        int sum = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = base + k < nbr ? (int)c16[base + k] : 0;
            sum += v[k];
        }
        int tot;
        int ex = block_excl_scan(sum, red, &tot) + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < nbr) {
                bin_start[g0 + base + k] = a + ex;
                c16[base + k] = (uint16_t)ex;
                ex += v[k];
            }
        carry += tot;
    }
    if (r == n_rows && threadIdx.x == 0) bin_start[g0 + 1] = a + n;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int b = lb[i];
        const int sh = (b & 1) << 4;
        mem[(atomicAdd(&cw[b >> 1], 1u << sh) >> sh) & 0xFFFFu] = i;
    }
    __syncthreads();
    // c16[b] is now the end of bin b, i.e. the start of bin b + 1
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const int i = mem[q];
        const int b = lb[i];
        const int bs = b > 0 ? (int)c16[b - 1] : 0, be = (int)c16[b];
        const int id = lid[i];
        int rank = 0;
        for (int u = bs; u < be; ++u) rank += lid[mem[u]] < id;
        const int o = a + bs + rank;
        yg[o] = gy[a + i];
        zg[o] = gz[a + i];
        idg[o] = id;
        // invalid rows keep their raw row value
        gsr[o] = (si << 8) | (r < n_rows ? r : (int)row[id]);
    }
    return true;
}

// final place of the cluster at binned slot q: its bin start plus the number
// of clusters of the bin with a smaller id
__device__ __forceinline__ void grid_place_one(
    int64_t q, const int32_t* __restrict__ bin_start, const int32_t* __restrict__ gid,
    const float* __restrict__ gy, const float* __restrict__ gz,
    const int32_t* __restrict__ gslot, const int32_t* __restrict__ gbin,
    const int32_t* __restrict__ gtag, float* __restrict__ yg, float* __restrict__ zg,
    int32_t* __restrict__ idg, int32_t* __restrict__ gsr)
{
    const int j = gslot[q];
    const int g = gbin[q];
    const int32_t id = gid[j];
    const int32_t bs = bin_start[g], be = bin_start[g + 1];
    int rank = 0;
    for (int32_t u = bs; u < be; ++u) rank += gid[gslot[u]] < id;
    const int32_t o = bs + rank;
    yg[o] = gy[j];
    zg[o] = gz[j];
    idg[o] = id;
    gsr[o] = gtag[q];
}

}  // namespace tpc
