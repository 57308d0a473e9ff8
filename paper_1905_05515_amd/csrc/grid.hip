// Grid build: stable counting sort of each sector's clusters by
// (row, z bin, y bin), ties by cluster id; clusters with an invalid row go to
// the sector's last bin.  A sector's clusters occupy exactly its id range of
// grid positions, so sectors can be built independently.
//
// count   one thread per cluster: bin histogram (atomics on the bin counts)
// scan    exclusive scan of the counts -> bin_start
// scatter one thread per cluster: claim a slot in its bin (any order)
// rank    one thread per grid position: the final place of a cluster is its
//         bin start plus the number of clusters in the bin with a smaller id,
//         which restores id order inside every bin deterministically.
#include "grid_dev.hpp"

namespace tpc {

__global__ __launch_bounds__(kBlock) void k_grid_count(
    const tpc_sector* __restrict__ sec, int n_sec, int n_rows, const uint8_t* __restrict__ row,
    const float* __restrict__ y, const float* __restrict__ z, int64_t begin, int64_t end,
    int32_t* __restrict__ cnt, tpc_status* status)
{
    for (int64_t i = begin + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < end;
         i += (int64_t)gridDim.x * blockDim.x)
        grid_count_one(sec, n_sec, n_rows, row, y, z, i, cnt, status);
}

__global__ __launch_bounds__(kBlock) void k_grid_scatter(
    const tpc_sector* __restrict__ sec, int n_sec, int n_rows, const uint8_t* __restrict__ row,
    const float* __restrict__ y, const float* __restrict__ z, int64_t begin, int64_t end,
    const int32_t* __restrict__ bin_start, int32_t* __restrict__ fill, int32_t* __restrict__ tmp)
{
    for (int64_t i = begin + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < end;
         i += (int64_t)gridDim.x * blockDim.x)
        grid_scatter_one(sec, n_sec, n_rows, row, y, z, i, bin_start, fill, tmp);
}

// grid positions [begin, end) (= the cluster ids of the sectors handled)
__global__ __launch_bounds__(kBlock) void k_grid_rank(
    const tpc_sector* __restrict__ sec, int n_sec, int n_rows, const uint8_t* __restrict__ row,
    const float* __restrict__ y, const float* __restrict__ z,
    const int32_t* __restrict__ bin_start, int64_t begin, int64_t end,
    const int32_t* __restrict__ tmp, float* __restrict__ yg, float* __restrict__ zg,
    int32_t* __restrict__ idg, int32_t* __restrict__ gsr)
{
    for (int64_t p = begin + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < end;
         p += (int64_t)gridDim.x * blockDim.x)
        grid_rank_one(sec, n_sec, n_rows, row, y, z, bin_start, p, tmp, yg, zg, idg, gsr);
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
    const int64_t g0 = a.bin_base;
    const int64_t g1 = (int64_t)b.bin_base + (int64_t)p->n_rows * b.nby * b.nbz + 1;
    if (sec_lo == 0) launch_fill<int64_t>((int64_t*)ws.status, 0, sizeof(tpc_status) / 8, st);
    launch_fill<int32_t>(ws.cnt + g0, 0, g1 - g0, st);
    const unsigned gc = grid_for(c1 - c0);
    TPC_LAUNCH(k_grid_count, dim3(gc), dim3(kBlock), 0, st, p->d_sectors, p->n_sectors,
               p->n_rows, in.row, in.y, in.z, c0, c1, ws.cnt, ws.status);
    // the sectors' first bin starts at their first cluster id
    launch_scan<int32_t>(ws.cnt + g0, out.bin_start + g0, g1 - g0, true, nullptr, nullptr,
                         ws.partials, st, c0);
    launch_fill<int32_t>(ws.cnt + g0, 0, g1 - g0, st);
    TPC_LAUNCH(k_grid_scatter, dim3(gc), dim3(kBlock), 0, st, p->d_sectors, p->n_sectors,
               p->n_rows, in.row, in.y, in.z, c0, c1, (const int32_t*)out.bin_start, ws.cnt,
               ws.tmp);
    TPC_LAUNCH(k_grid_rank, dim3(gc), dim3(kBlock), 0, st, p->d_sectors, p->n_sectors, p->n_rows,
               in.row, in.y, in.z, (const int32_t*)out.bin_start, c0, c1,
               (const int32_t*)ws.tmp, out.y, out.z, out.id, ws.gsr);
    TPC_LAUNCH(k_set_grid_status, dim3(1), dim3(1), 0, st, ws.status, c1);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // namespace tpc
