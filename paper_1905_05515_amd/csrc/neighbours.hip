// Cellular-automaton seeding: best up/down pair per hit, mutual-link
// cleaning, chain starts.
#include "seed_dev.hpp"

namespace tpc {

__global__ __launch_bounds__(kBlock) void k_neighbours(
    const tpc_sector* __restrict__ sec, int n_rows, const float* __restrict__ row_x,
    tpc_params prm, const int32_t* __restrict__ bin_start, const float* __restrict__ yg,
    const float* __restrict__ zg, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ gsr, int64_t begin, int64_t end,
    int32_t* __restrict__ up0, int32_t* __restrict__ down0)
{
    __shared__ float nb_l[3 * kNbList * kBlock];
    __shared__ float xs[256];
    const NbList L{nb_l, nb_l + kNbList * kBlock,
                   reinterpret_cast<int*>(nb_l + 2 * kNbList * kBlock)};
    for (int i = threadIdx.x; i < n_rows; i += blockDim.x) xs[i] = row_x[i];
    __syncthreads();
    // work blocks dealt to the XCDs in contiguous ranges (one sector's rows
    // share an L2)
    const int64_t nblk = (end - begin + blockDim.x - 1) / blockDim.x;
    for (int64_t b0 = 0; b0 < nblk; b0 += gridDim.x) {
        const int64_t chunk = nblk - b0 < (int64_t)gridDim.x ? nblk - b0 : (int64_t)gridDim.x;
        if ((int64_t)blockIdx.x >= chunk) break;
        const int64_t p = begin + (b0 + xcd_remap(blockIdx.x, (int)chunk)) * blockDim.x +
                          threadIdx.x;
        if (p < end)
            neighbours_one(p, sec, n_rows, xs, prm, bin_start, yg, zg, idg, gsr, up0, down0, L);
    }
}

__global__ __launch_bounds__(kBlock) void k_clean(
    const int32_t* __restrict__ up0, const int32_t* __restrict__ down0,
    const int32_t* __restrict__ idg, int64_t begin, int64_t end,
    int32_t* __restrict__ up, int32_t* __restrict__ down, int32_t* __restrict__ start_by_id)
{
    for (int64_t p = begin + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < end;
         p += (int64_t)gridDim.x * blockDim.x)
        clean_one(p, up0, down0, idg, up, down, start_by_id);
}

// Deterministic compaction of the flagged starts in id order: count per
// tile, scan of the tile counts, write.
__global__ __launch_bounds__(kBlock) void k_start_tile_counts(const int32_t* __restrict__ flag,
                                                              int64_t n,
                                                              int64_t* __restrict__ partials)
{
    __shared__ int lds[kBlock / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int c = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) c += (base + k < n) && flag[base + k] >= 0;
    // block sum
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
    if (lane == 0) lds[wid] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += lds[w];
        partials[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_start_write(const int32_t* __restrict__ flag,
                                                        int64_t n,
                                                        const int64_t* __restrict__ partials,
                                                        int32_t* __restrict__ out, int64_t cap)
{
    __shared__ int lds[kBlock / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int c = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? flag[base + k] : -1;
        c += v[k] >= 0;
    }
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    int x = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) lds[wid] = x;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wid; ++w) before += lds[w];
    int64_t o = partials[blockIdx.x] + before + x - c;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (v[k] >= 0) {
            if (o < cap) out[o] = v[k];
            ++o;
        }
}

// running start count before a range of sectors (first range: reset)
__global__ void k_start_mark(tpc_status* status, int64_t* sec_start, int sec_lo)
{
    if (blockIdx.x || threadIdx.x) return;
    if (sec_lo == 0) status->n_starts = 0;
    sec_start[sec_lo] = status->n_starts;
}

__global__ void k_start_status(tpc_status* status, int64_t* sec_start, int sec_hi, int64_t cap)
{
    if (blockIdx.x || threadIdx.x) return;
    sec_start[sec_hi] = status->n_starts;
    if (status->n_starts > cap) status->overflow |= 1;
}

// First start of every sector strictly inside (sec_lo, sec_hi): starts are
// stored in cluster-id order and a sector's starts are grid positions of its
// own id range, so the sector of starts[t] grows with t and a binary search
// for the first position at or beyond the sector's first id finds it.
__global__ void k_sector_starts(const tpc_sector* __restrict__ sec, int sec_lo, int sec_hi,
                                const int32_t* __restrict__ starts, int64_t cap,
                                int64_t* __restrict__ sec_start)
{
    const int s = sec_lo + 1 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= sec_hi) return;
    int64_t lo = sec_start[sec_lo], hi = sec_start[sec_hi];
    if (hi > cap) hi = cap;
    if (lo > hi) lo = hi;
    const int64_t first = sec[s].begin;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (starts[mid] < first) lo = mid + 1;
        else hi = mid;
    }
    sec_start[s] = lo;
}

// Seeding for sectors [sec_lo, sec_hi): their grid positions and cluster ids
// are the same range.  Starts are appended in id order after those of the
// earlier sectors.
int run_find_neighbours(const tpc_problem* p, int sec_lo, int sec_hi, tpc_grid grid,
                        tpc_links links, tpc_starts starts, const Workspace& ws, hipStream_t st,
                        const tpc_tuning* tune)
{
    const int64_t c0 = p->h_sectors[sec_lo].begin, c1 = p->h_sectors[sec_hi - 1].end;
    const int64_t n = c1 - c0;
    const unsigned gn = grid_for(n);
    const int nbk = tune && tune->neighbour_block ? tune->neighbour_block : kBlock;
    TPC_LAUNCH(k_neighbours, dim3(grid_for_block(n, nbk, 65536)), dim3(nbk), 0, st, p->d_sectors,
               p->n_rows, p->d_row_x, p->params, (const int32_t*)grid.bin_start,
               (const float*)grid.y, (const float*)grid.z, (const int32_t*)grid.id,
               (const int32_t*)ws.gsr, c0, c1, links.up0, links.down0);
    launch_fill<int32_t>(ws.tmp + c0, -1, n, st);
    TPC_LAUNCH(k_clean, dim3(gn), dim3(kBlock), 0, st, (const int32_t*)links.up0,
               (const int32_t*)links.down0, (const int32_t*)grid.id, c0, c1, links.up, links.down,
               ws.tmp);
    TPC_LAUNCH(k_start_mark, dim3(1), dim3(1), 0, st, ws.status, ws.sec_start, sec_lo);
    const int64_t nt = ceil_div(n > 0 ? n : 1, kScanTile);
    TPC_LAUNCH(k_start_tile_counts, dim3((unsigned)nt), dim3(kBlock), 0, st,
               (const int32_t*)(ws.tmp + c0), n, ws.partials);
    launch_scan_partials(ws.partials, nt, &ws.status->n_starts, &ws.status->n_starts, st);
    TPC_LAUNCH(k_start_write, dim3((unsigned)nt), dim3(kBlock), 0, st,
               (const int32_t*)(ws.tmp + c0), n, (const int64_t*)ws.partials, starts.pos,
               starts.capacity);
    TPC_LAUNCH(k_start_status, dim3(1), dim3(1), 0, st, ws.status, ws.sec_start, sec_hi,
               starts.capacity);
    if (sec_hi - sec_lo > 1)
        TPC_LAUNCH(k_sector_starts, dim3((unsigned)ceil_div(sec_hi - sec_lo - 1, kBlock)),
                   dim3(kBlock), 0, st, p->d_sectors, sec_lo, sec_hi,
                   (const int32_t*)starts.pos, starts.capacity, ws.sec_start);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // namespace tpc
