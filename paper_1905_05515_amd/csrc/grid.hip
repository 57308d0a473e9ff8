// Grid build: stable counting sort of each sector's clusters by
// (row, z bin, y bin), ties by cluster id; clusters with an invalid row go to
// the sector's last bin.  A sector's clusters occupy exactly its id range of
// grid positions, so sectors can be built independently.  The staged form
// partitions by row first (counts per tile in LDS), then sorts every row by
// bin in LDS, so that no cluster needs a device-wide atomic; the persistent
// kernel runs the same steps as tasks (grid_dev.hpp).
#include "block_dev.hpp"
#include "grid_dev.hpp"

namespace tpc {

// ---- staged grid build ------------------------------------------------------
// 1. rows:     tiles of kRowTile consecutive clusters count them per
//              (sector, row bucket) in LDS (a bucket is a z slab of a pad
//              row, or the invalid rows), one device atomic per non-empty
//              bucket and tile;
// 2. scan:     bucket starts (a sector's first bucket starts at its first id);
// 3. scatter:  tiles claim a range per bucket and copy (id, y, z) there, in
//              any order inside a bucket;
// 4. bins:     one block per (sector, bucket) counts its clusters per bin in
//              LDS and scans the counts into the bin starts; a bucket that
//              fits in LDS (grid_bins_place_fused) is also placed there: the
//              final place of a cluster is its bin start plus the number of
//              clusters of its bin with a smaller id; a larger one deals every
//              cluster a slot of its bin (any order inside a bin) and joins
//              the list of step 5;
// 5. place:    for the listed buckets, the same rule over the slots.
// No step depends on the order of atomics: the result is the stable sort.
constexpr int kRowTile = kBlock * 8;
constexpr int kTileCounters = 4096;  // LDS bucket counters of one tile

__device__ __forceinline__ int tile_sector(int64_t i, const int64_t* ends, int ns)
{
    for (int k = 0; k < ns; ++k)
        if (i < ends[k]) return k;
    return -1;
}

// LDS: the tile's first sector, the ends of its first ts sectors, and zeroed
// bucket counters; returns the number of sectors with counters
__device__ __forceinline__ int tile_setup(const tpc_sector* __restrict__ sec, int n_sec, int Rb,
                                          int ts, int64_t i0, int* hist, int64_t* ends,
                                          int* sf_sh)
{
    __syncthreads();
    if (threadIdx.x == 0) *sf_sh = find_sector(sec, n_sec, i0);
    for (int k = threadIdx.x; k < ts * Rb; k += blockDim.x) hist[k] = 0;
    __syncthreads();
    const int sf = *sf_sh;
    const int ns = n_sec - sf < ts ? n_sec - sf : ts;
    if ((int)threadIdx.x < ns) ends[threadIdx.x] = sec[sf + threadIdx.x].end;
    __syncthreads();
    return ns;
}

constexpr int kTileSecMax = 8;

// ts: sectors of a tile with LDS counters (Rb * ts <= kTileCounters)
__global__ __launch_bounds__(kBlock) void k_grid_rows(
    const tpc_sector* __restrict__ sec, int n_sec, int n_rows, int S, int ts,
    const uint8_t* __restrict__ row, const float* __restrict__ z, int64_t c0, int64_t c1,
    int32_t* __restrict__ rcnt, tpc_status* status, int32_t* __restrict__ bigq)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) bigq[0] = 0;   // the list of step 5
    __shared__ int hist[kTileCounters];
    __shared__ int64_t ends[kTileSecMax];
    __shared__ int sf_sh;
    __shared__ int64_t red[kBlock / kWave];
    const int Rb = (n_rows + 1) * S;
    const int64_t n_tiles = (c1 - c0 + kRowTile - 1) / kRowTile;
    int64_t bad = 0;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t i0 = c0 + tile * kRowTile;
        const int64_t i1 = i0 + kRowTile < c1 ? i0 + kRowTile : c1;
        const int ns = tile_setup(sec, n_sec, Rb, ts, i0, hist, ends, &sf_sh);
        const int sf = sf_sh;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
            const int r = row[i];
            if (r >= n_rows) ++bad;
            const int k = tile_sector(i, ends, ns);
            const int si = k >= 0 ? sf + k : find_sector(sec, n_sec, i);
            const int bk = cluster_bucket(sec[si], n_rows, S, r, z[i]);
            if (k >= 0) atomicAdd(&hist[k * Rb + bk], 1);
            else atomicAdd(&rcnt[(int64_t)si * Rb + bk], 1);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < ns * Rb; k += blockDim.x)
            if (hist[k]) atomicAdd(&rcnt[(int64_t)(sf + k / Rb) * Rb + k % Rb], hist[k]);
    }
    const int64_t tot = block_sum(bad, red);
    if (threadIdx.x == 0 && tot) atomicAdd((unsigned long long*)&status->n_bad_rows,
                                           (unsigned long long)tot);
}

__global__ __launch_bounds__(kBlock) void k_grid_rows_scatter(
    const tpc_sector* __restrict__ sec, int n_sec, int n_rows, int S, int ts,
    const uint8_t* __restrict__ row, const float* __restrict__ y, const float* __restrict__ z,
    int64_t c0, int64_t c1, const int32_t* __restrict__ rstart, int32_t* __restrict__ rfill,
    int32_t* __restrict__ gid, float* __restrict__ gy, float* __restrict__ gz)
{
    constexpr int kItems = kRowTile / kBlock;
    __shared__ int hist[kTileCounters];
    __shared__ int64_t ends[kTileSecMax];
    __shared__ int sf_sh;
    const int Rb = (n_rows + 1) * S;
    const int64_t n_tiles = (c1 - c0 + kRowTile - 1) / kRowTile;
    // each pass over gridDim.x tiles deals them to the XCDs in contiguous
    // ranges (block b runs on XCD b mod 8), so that the short runs that
    // neighbouring tiles write into one bucket meet in one L2 and leave it
    // as whole lines
    for (int64_t b0 = 0; b0 < n_tiles; b0 += gridDim.x) {
        const int64_t chunk = n_tiles - b0 < (int64_t)gridDim.x ? n_tiles - b0 : (int64_t)gridDim.x;
        if ((int64_t)blockIdx.x >= chunk) break;
        const int64_t tile = b0 + xcd_remap(blockIdx.x, (int)chunk);
        const int64_t i0 = c0 + tile * kRowTile;
        const int64_t i1 = i0 + kRowTile < c1 ? i0 + kRowTile : c1;
        const int ns = tile_setup(sec, n_sec, Rb, ts, i0, hist, ends, &sf_sh);
        const int sf = sf_sh;
        int bucket[kItems], rank[kItems];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int64_t i = i0 + threadIdx.x + (int64_t)j * kBlock;
            bucket[j] = -1;
            rank[j] = 0;
            if (i >= i1) continue;
            const int k = tile_sector(i, ends, ns);
            const int si = k >= 0 ? sf + k : find_sector(sec, n_sec, i);
            const int bk = cluster_bucket(sec[si], n_rows, S, row[i], z[i]);
            if (k >= 0) {
                bucket[j] = k * Rb + bk;
                rank[j] = atomicAdd(&hist[bucket[j]], 1);
            } else {   // a sector beyond the tile's LDS counters: claim one slot
                const int64_t gb = (int64_t)si * Rb + bk;
                rank[j] = rstart[gb] + atomicAdd(&rfill[gb], 1);
            }
        }
        __syncthreads();
        // one range per non-empty bucket; the counter becomes the range start
        for (int k = threadIdx.x; k < ns * Rb; k += blockDim.x) {
            const int c = hist[k];
            if (c) {
                const int64_t gb = (int64_t)(sf + k / Rb) * Rb + k % Rb;
                hist[k] = rstart[gb] + atomicAdd(&rfill[gb], c);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int64_t i = i0 + threadIdx.x + (int64_t)j * kBlock;
            if (i >= i1) continue;
            const int slot = bucket[j] >= 0 ? hist[bucket[j]] + rank[j] : rank[j];
            gid[slot] = (int32_t)i;
            gy[slot] = y[i];
            gz[slot] = z[i];
        }
    }
}

// one block per (sector, bucket) of sectors [sec_lo, ...)
__global__ __launch_bounds__(kBlock) void k_grid_bins(
    const tpc_sector* __restrict__ sec, int sec_lo, int n_rows, int S,
    const int32_t* __restrict__ rstart, const float* __restrict__ gy,
    const float* __restrict__ gz, const int32_t* __restrict__ gid,
    const uint8_t* __restrict__ row, int32_t* __restrict__ bin_start,
    int32_t* __restrict__ cnt, int32_t* __restrict__ gslot, int32_t* __restrict__ gbin,
    int32_t* __restrict__ gtag, float* __restrict__ yg, float* __restrict__ zg,
    int32_t* __restrict__ idg, int32_t* __restrict__ gsr, int32_t* __restrict__ bigq,
    int fuse_bins, int lds_ints)
{
    extern __shared__ int lds[];           // lds_ints, sized on the host for the problem
    __shared__ int red[kBlock / kWave];
    const int Rb = (n_rows + 1) * S;
    const int si = sec_lo + (int)(blockIdx.x / Rb);
    const int bk = (int)(blockIdx.x % Rb);
    const tpc_sector s = sec[si];
    if (grid_bins_place_fused(s, si, bk, n_rows, S, rstart, gy, gz, gid, row, bin_start, yg, zg,
                              idg, gsr, lds, red, fuse_bins))
        return;
    grid_bins_bucket(s, si, bk, n_rows, S, rstart, gy, gz, gid, row, bin_start, cnt, gslot, gbin,
                     gtag, lds, red, lds_ints);
    if (threadIdx.x == 0) bigq[1 + atomicAdd(&bigq[0], 1)] = si * Rb + bk;
}

// the listed buckets (one block each, any order)
__global__ __launch_bounds__(kBlock) void k_grid_place(
    const int32_t* __restrict__ bigq, const int32_t* __restrict__ rstart,
    const int32_t* __restrict__ bin_start, const int32_t* __restrict__ gid,
    const float* __restrict__ gy, const float* __restrict__ gz,
    const int32_t* __restrict__ gslot, const int32_t* __restrict__ gbin,
    const int32_t* __restrict__ gtag, float* __restrict__ yg, float* __restrict__ zg,
    int32_t* __restrict__ idg, int32_t* __restrict__ gsr)
{
    const int nq = bigq[0];
    for (int e = blockIdx.x; e < nq; e += gridDim.x) {
        const int gb = bigq[1 + e];
        const int a = rstart[gb], b = rstart[gb + 1];
        for (int q = a + threadIdx.x; q < b; q += blockDim.x)
            grid_place_one(q, bin_start, gid, gy, gz, gslot, gbin, gtag, yg, zg, idg, gsr);
    }
}

__global__ void k_set_grid_status(tpc_status* status, int64_t n_grid)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) status->n_grid = n_grid;
}

// Build the grid of sectors [sec_lo, sec_hi).  The first call of an event
// (sec_lo == 0) clears the status block.
int run_build_grid(const tpc_problem* p, int sec_lo, int sec_hi, tpc_clusters in,
                   tpc_grid out, const Workspace& ws, hipStream_t st)
{
    const tpc_sector& a = p->h_sectors[sec_lo];
    const tpc_sector& b = p->h_sectors[sec_hi - 1];
    const int64_t c0 = a.begin, c1 = b.end;
    const int S = grid_slabs(p);
    const int Rb = (p->n_rows + 1) * S;
    int ts = kTileCounters / Rb;
    if (ts > kTileSecMax) ts = kTileSecMax;
    if (ts < 1) ts = 1;
    if (Rb > kTileCounters) return TPC_ERR_UNSUPPORTED;
    const int64_t nbk = (int64_t)(sec_hi - sec_lo) * Rb;
    if (sec_lo == 0) launch_fill<int64_t>((int64_t*)ws.status, 0, sizeof(tpc_status) / 8, st);
    launch_fill<int32_t>(ws.rcnt + (int64_t)sec_lo * Rb, 0, nbk, st);
    launch_fill<int32_t>(ws.rfill + (int64_t)sec_lo * Rb, 0, nbk, st);
    const unsigned gt = grid_for_block(ceil_div(c1 - c0, kRowTile), 1, 4096);
    TPC_LAUNCH(k_grid_rows, dim3(gt), dim3(kBlock), 0, st, p->d_sectors, p->n_sectors,
               p->n_rows, S, ts, in.row, in.z, c0, c1, ws.rcnt, ws.status, ws.bigq);
    launch_scan<int32_t>(ws.rcnt + (int64_t)sec_lo * Rb, ws.rstart + (int64_t)sec_lo * Rb, nbk,
                         true, nullptr, nullptr, ws.partials, st, c0);
    TPC_LAUNCH(k_grid_rows_scatter, dim3(gt), dim3(kBlock), 0, st, p->d_sectors, p->n_sectors,
               p->n_rows, S, ts, in.row, in.y, in.z, c0, c1, (const int32_t*)ws.rstart,
               ws.rfill, ws.tmp, ws.gy, ws.gz);
    // LDS of the bin-sort blocks: the largest slab of these sectors decides
    // (bin counters of the fused form, or of a larger bucket; fewer bytes,
    // more resident blocks)
    int max_nbr = 1;
    for (int i = sec_lo; i < sec_hi; ++i) {
        const tpc_sector& s = p->h_sectors[i];
        const int zs = slab_zbins(s);
        const int nbr = (zs < s.nbz ? zs : s.nbz) * s.nby;
        if (nbr > max_nbr) max_nbr = nbr;
    }
    const int fuse_bins = max_nbr < kFuseBins ? max_nbr : kFuseBins;
    const int unfused = max_nbr < kRowBinsLds ? max_nbr : kRowBinsLds;
    const int lds_ints = fused_lds_ints(fuse_bins) > unfused ? fused_lds_ints(fuse_bins) : unfused;
    TPC_LAUNCH(k_grid_bins, dim3((unsigned)nbk), dim3(kBlock), sizeof(int) * lds_ints, st,
               p->d_sectors, sec_lo,
               p->n_rows, S, (const int32_t*)ws.rstart, (const float*)ws.gy, (const float*)ws.gz,
               (const int32_t*)ws.tmp, in.row, out.bin_start, ws.cnt, ws.gslot, ws.gbin,
               ws.gtag, out.y, out.z, out.id, ws.gsr, ws.bigq, fuse_bins, lds_ints);
    TPC_LAUNCH(k_grid_place, dim3(grid_for_block(nbk, 1, 2048)), dim3(kBlock), 0, st,
               (const int32_t*)ws.bigq, (const int32_t*)ws.rstart,
               (const int32_t*)out.bin_start, (const int32_t*)ws.tmp, (const float*)ws.gy,
               (const float*)ws.gz, (const int32_t*)ws.gslot, (const int32_t*)ws.gbin,
               (const int32_t*)ws.gtag, out.y, out.z, out.id, ws.gsr);
    TPC_LAUNCH(k_set_grid_status, dim3(1), dim3(1), 0, st, ws.status, c1);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // namespace tpc
