// Kalman-filter tracklet construction, one thread per chain start (the
// arithmetic is in tracklet_dev.hpp).
#include "tracklet_dev.hpp"

namespace tpc {

// One wave per 64 consecutive starts.  Two forms of one kernel: with the
// hit lists built in LDS (one column per lane, written out row by row,
// coalesced), or written straight into the [row][tracklet] output.  The LDS
// lists (4 B per row and lane) allow few waves per CU: they win while all
// waves fit on the chip at once, the direct form wins beyond (more waves in
// flight hide the latency).  Both are launched; the count of starts on the
// device decides which one works.  Work blocks are dealt to the XCDs in
// contiguous ranges, so that the starts of one sector, and the grid rows
// they search, share an L2.
template <bool kLds>
__global__ __launch_bounds__(kWave) void k_tracklets(
    const tpc_sector* __restrict__ sec, int n_rows, const float* __restrict__ row_x,
    tpc_params prm, const int32_t* __restrict__ bin_start, const float* __restrict__ yg,
    const float* __restrict__ zg, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ gsr, const int32_t* __restrict__ up,
    const int32_t* __restrict__ starts, tpc_status* __restrict__ status,
    const int64_t* __restrict__ t_lo, const int64_t* __restrict__ t_hi, int64_t count_cap,
    int64_t cap, int64_t lds_blocks,
    int32_t* __restrict__ t_start, int32_t* __restrict__ t_hits, int32_t* __restrict__ t_nhits,
    int32_t* __restrict__ t_rin, float* __restrict__ t_par, float* __restrict__ t_cov,
    float* __restrict__ t_chi2)
{
    extern __shared__ int32_t smem[];      // n_rows row positions, then [row][lane] hits
    const int64_t lo = *t_lo < count_cap ? *t_lo : count_cap;
    const int64_t m = *t_hi < count_cap ? *t_hi : count_cap;
    const int64_t nb = m > lo ? (m - lo + kWave - 1) / kWave : 0;
    if ((nb <= lds_blocks) != kLds) return;          // the other form works
    float* xs = reinterpret_cast<float*>(smem);
    int32_t* hl = smem + n_rows;
    for (int i = threadIdx.x; i < n_rows; i += blockDim.x) xs[i] = row_x[i];
    __syncthreads();
    int n_prop = 0, n_upd = 0, n_cand = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += gridDim.x) {
        const int64_t chunk = nb - b0 < (int64_t)gridDim.x ? nb - b0 : (int64_t)gridDim.x;
        if ((int64_t)blockIdx.x >= chunk) break;
        const int64_t tb = lo + (b0 + xcd_remap(blockIdx.x, (int)chunk)) * kWave;
        const int64_t t = tb + threadIdx.x;
        if (t < m) {
            if (kLds) {
                int32_t* th = hl + threadIdx.x;
                build_tracklet(t, sec, n_rows, xs, prm, bin_start, yg, zg, idg, gsr, up, starts,
                               th, kWave, t_start, t_nhits, t_rin, t_par, t_cov, t_chi2, n_prop,
                               n_upd, n_cand);
                // each lane copies its own column: no barrier needed
                for (int r = 0; r < n_rows; ++r) t_hits[(int64_t)r * cap + t] = th[r * kWave];
            } else {
                build_tracklet(t, sec, n_rows, xs, prm, bin_start, yg, zg, idg, gsr, up, starts,
                               t_hits + t, cap, t_start, t_nhits, t_rin, t_par, t_cov, t_chi2,
                               n_prop, n_upd, n_cand);
            }
        }
    }
    add_work(status, n_prop, n_upd, n_cand);
}

// LDS bytes of one k_tracklets block
inline size_t tracklet_lds_bytes(int n_rows, bool lds)
{
    return (size_t)n_rows * 4 * (lds ? kWave + 1 : 1);
}

// work blocks of the LDS form that are resident on the whole device at once
// (kept per device and row count: the query is not free and the per-sector
// form asks once per sector)
static int64_t tracklet_lds_capacity(int n_rows)
{
    constexpr int kDevs = 16;
    static int64_t cache[kDevs][256];
    int dev = 0, n_cu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev >= 0 && dev < kDevs && cache[dev][n_rows] > 0) return cache[dev][n_rows];
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tracklets<true>, kWave,
                                                     tracklet_lds_bytes(n_rows, true)) !=
            hipSuccess)
        return 0;
    const int64_t v = (int64_t)n_cu * per_cu;
    if (dev >= 0 && dev < kDevs) cache[dev][n_rows] = v;
    return v;
}

// Tracklets of the starts of sectors [sec_lo, sec_hi) (the start range that
// run_find_neighbours recorded for them).
int run_construct_tracklets(const tpc_problem* p, int sec_lo, int sec_hi, tpc_grid grid_,
                            tpc_links links, tpc_starts starts, tpc_tracklets trl,
                            const Workspace& ws, hipStream_t st)
{
    // tracklets processed: bounded by both capacities; the hit array's row
    // stride is the tracklet capacity
    const int64_t count_cap = starts.capacity < trl.capacity ? starts.capacity : trl.capacity;
    const int64_t bound = (p->h_sectors[sec_hi - 1].end - p->h_sectors[sec_lo].begin) / 3 + 1;
    const int64_t n_launch = bound < count_cap ? bound : count_cap;
    const int64_t cap_lds = tracklet_lds_capacity(p->n_rows);
    const dim3 grid(grid_for_block(n_launch, kWave, 65536));
    TPC_LAUNCH(k_tracklets<true>, grid, dim3(kWave), tracklet_lds_bytes(p->n_rows, true), st,
               p->d_sectors, p->n_rows, p->d_row_x, p->params, (const int32_t*)grid_.bin_start,
               (const float*)grid_.y, (const float*)grid_.z, (const int32_t*)grid_.id,
               (const int32_t*)ws.gsr, (const int32_t*)links.up, (const int32_t*)starts.pos,
               ws.status, (const int64_t*)(ws.sec_start + sec_lo),
               (const int64_t*)(ws.sec_start + sec_hi), count_cap, trl.capacity, cap_lds,
               trl.start, trl.hits, trl.nhits, trl.row_inner, trl.par, trl.cov, trl.chi2);
    TPC_LAUNCH(k_tracklets<false>, grid, dim3(kWave), tracklet_lds_bytes(p->n_rows, false), st,
               p->d_sectors, p->n_rows, p->d_row_x, p->params, (const int32_t*)grid_.bin_start,
               (const float*)grid_.y, (const float*)grid_.z, (const int32_t*)grid_.id,
               (const int32_t*)ws.gsr, (const int32_t*)links.up, (const int32_t*)starts.pos,
               ws.status, (const int64_t*)(ws.sec_start + sec_lo),
               (const int64_t*)(ws.sec_start + sec_hi), count_cap, trl.capacity, cap_lds,
               trl.start, trl.hits, trl.nhits, trl.row_inner, trl.par, trl.cov, trl.chi2);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // namespace tpc
