// Cellular-automaton seeding: best up/down pair per hit, mutual-link
// cleaning, chain starts.
#include "tpc_internal.hpp"

namespace tpc {

// One thread per grid position (the centre hit).  Candidates on rows r+1 and
// r-1 come from the bins covering the windows around the straight line from
// the origin through the hit; the exact window test and the pair deviation
// decide, ties go to the lower (up id, down id).
__global__ __launch_bounds__(kBlock) void k_neighbours(
    const tpc_sector* __restrict__ sec, int n_rows, const float* __restrict__ row_x,
    tpc_params prm, const int32_t* __restrict__ bin_start, const float* __restrict__ yg,
    const float* __restrict__ zg, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ gsr, int64_t begin, int64_t end,
    int32_t* __restrict__ up0, int32_t* __restrict__ down0)
{
    const float Wy = prm.nb_win_y, Wz = prm.nb_win_z, D2max = prm.nb_d2max;
    for (int64_t p = begin + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < end;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int v = gsr[p];
        const int r = v & 255;
        int bu = -1, bd = -1;
        if (r > 0 && r + 1 < n_rows) {
            const tpc_sector s = sec[v >> 8];
            const float y = yg[p], z = zg[p];
            const float slope = y / row_x[r];
            const float yu_c = slope * row_x[r + 1];
            const float yd_c = slope * row_x[r - 1];
            const int iyu0 = bin_of(yu_c - Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
            const int iyu1 = bin_of(yu_c + Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
            const int iyd0 = bin_of(yd_c - Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
            const int iyd1 = bin_of(yd_c + Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
            const int iz0 = bin_of(z - Wz * TPC_WIDEN, s.z0, s.inv_bz, s.nbz);
            const int iz1 = bin_of(z + Wz * TPC_WIDEN, s.z0, s.inv_bz, s.nbz);
            float best = 0.0f;
            int bidu = -1, bidd = -1;
            for (int izu = iz0; izu <= iz1; ++izu) {
                const int gu = s.bin_base + ((r + 1) * s.nbz + izu) * s.nby;
                const int pu1 = bin_start[gu + iyu1 + 1];
                for (int pu = bin_start[gu + iyu0]; pu < pu1; ++pu) {
                    const float yu = yg[pu], zu = zg[pu];
                    if (!(fabsf(yu - yu_c) <= Wy && fabsf(zu - z) <= Wz)) continue;
                    const int idu = idg[pu];
                    for (int izd = iz0; izd <= iz1; ++izd) {
                        const int gd = s.bin_base + ((r - 1) * s.nbz + izd) * s.nby;
                        const int pd1 = bin_start[gd + iyd1 + 1];
                        for (int pd = bin_start[gd + iyd0]; pd < pd1; ++pd) {
                            const float yd = yg[pd], zd = zg[pd];
                            if (!(fabsf(yd - yd_c) <= Wy && fabsf(zd - z) <= Wz)) continue;
                            const float dy = (yu + yd) - (y + y);
                            const float dz = (zu + zd) - (z + z);
                            const float d2 = dy * dy + dz * dz;
                            if (!(d2 <= D2max)) continue;
                            const int idd = idg[pd];
                            if (bu < 0 || d2 < best ||
                                (d2 == best && (idu < bidu || (idu == bidu && idd < bidd)))) {
                                best = d2;
                                bu = pu;
                                bd = pd;
                                bidu = idu;
                                bidd = idd;
                            }
                        }
                    }
                }
            }
        }
        up0[p] = bu;
        down0[p] = bd;
    }
}

// Mutual links; a chain start (up link, no down link, and its up neighbour
// has an up link) is flagged in the id-indexed array `start_by_id`.
__global__ __launch_bounds__(kBlock) void k_clean(
    const int32_t* __restrict__ up0, const int32_t* __restrict__ down0,
    const int32_t* __restrict__ idg, int64_t begin, int64_t end,
    int32_t* __restrict__ up, int32_t* __restrict__ down, int32_t* __restrict__ start_by_id)
{
    for (int64_t p = begin + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < end;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int u = up0[p], d = down0[p];
        const int uc = (u >= 0 && down0[u] == p) ? u : -1;
        const int dc = (d >= 0 && up0[d] == p) ? d : -1;
        up[p] = uc;
        down[p] = dc;
        if (uc >= 0 && dc < 0) {
            const int uu = up0[uc];
            if (uu >= 0 && down0[uu] == uc) start_by_id[idg[p]] = (int32_t)p;
        }
    }
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

// Seeding for sectors [sec_lo, sec_hi): their grid positions and cluster ids
// are the same range.  Starts are appended in id order after those of the
// earlier sectors.
int run_find_neighbours(const tpc_problem* p, int sec_lo, int sec_hi, tpc_grid grid,
                        tpc_links links, tpc_starts starts, const Workspace& ws, hipStream_t st)
{
    const int64_t c0 = p->h_sectors[sec_lo].begin, c1 = p->h_sectors[sec_hi - 1].end;
    const int64_t n = c1 - c0;
    const unsigned gn = grid_for(n);
    TPC_LAUNCH(k_neighbours, dim3(gn), dim3(kBlock), 0, st, p->d_sectors, p->n_rows, p->d_row_x,
               p->params, (const int32_t*)grid.bin_start, (const float*)grid.y,
               (const float*)grid.z, (const int32_t*)grid.id, (const int32_t*)ws.gsr, c0, c1,
               links.up0, links.down0);
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
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // namespace tpc
