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
    int64_t cap, int64_t lds_blocks, int64_t q_blocks,
    int32_t* __restrict__ t_start, int32_t* __restrict__ t_hits, int32_t* __restrict__ t_nhits,
    int32_t* __restrict__ t_rin, float* __restrict__ t_par, float* __restrict__ t_cov,
    float* __restrict__ t_chi2)
{
    extern __shared__ int32_t smem[];      // n_rows row positions, then [row][lane] hits
    const int64_t lo = *t_lo < count_cap ? *t_lo : count_cap;
    const int64_t m = *t_hi < count_cap ? *t_hi : count_cap;
    const int64_t nb = m > lo ? (m - lo + kWave - 1) / kWave : 0;
    // the LDS form up to lds_blocks waves of starts, this form up to
    // q_blocks, the queue form beyond
    if (kLds ? nb > lds_blocks : (nb <= lds_blocks || nb > q_blocks)) return;
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

// Queue form: as many waves as are resident; the starts [lo, m) are split
// into eight ranges, one per XCD (block b runs on XCD b mod 8), each with a
// counter in `queue` (zero at launch).  A wave refills its idle lanes from
// its XCD's range and, when that is exhausted, from the others in turn, so
// the waves of one XCD mostly work on the starts of the same sectors (the
// grid rows they search stay in that XCD's L2) and every wave runs until no
// work is left.  It works when the start count needs more than
// `min_blocks` waves (the other forms exit then).
__global__ __launch_bounds__(kWave) void k_tracklets_queue(
    const tpc_sector* __restrict__ sec, int n_rows, const float* __restrict__ row_x,
    tpc_params prm, const int32_t* __restrict__ bin_start, const float* __restrict__ yg,
    const float* __restrict__ zg, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ gsr, const int32_t* __restrict__ up,
    const int32_t* __restrict__ starts, tpc_status* __restrict__ status,
    const int64_t* __restrict__ t_lo, const int64_t* __restrict__ t_hi, int64_t count_cap,
    int64_t cap, int64_t min_blocks, unsigned long long* __restrict__ queue,
    int32_t* __restrict__ t_start, int32_t* __restrict__ t_hits, int32_t* __restrict__ t_nhits,
    int32_t* __restrict__ t_rin, float* __restrict__ t_par, float* __restrict__ t_cov,
    float* __restrict__ t_chi2)
{
    extern __shared__ int32_t smem[];      // n_rows row positions
    const int64_t lo = *t_lo < count_cap ? *t_lo : count_cap;
    const int64_t m = *t_hi < count_cap ? *t_hi : count_cap;
    const int64_t nb = m > lo ? (m - lo + kWave - 1) / kWave : 0;
    if (nb <= min_blocks) return;          // another form works
    float* xs = reinterpret_cast<float*>(smem);
    for (int i = threadIdx.x; i < n_rows; i += blockDim.x) xs[i] = row_x[i];
    __syncthreads();
    const int lane = threadIdx.x;
    const int x = blockIdx.x & 7;
    const int64_t n = m - lo;
    int n_prop = 0, n_upd = 0, n_cand = 0;
    int qi = 0;                            // queues tried and found empty
    LaneTracklet L;
    L.ph = kLaneIdle;
    L.t = -1;
    for (;;) {
        const uint64_t idle = __ballot(L.ph == kLaneIdle || L.ph == kLaneDone);
        const uint64_t busy = __ballot(L.ph == kLaneUp || L.ph == kLaneDown);
        if (idle && (__popcll(idle) >= kRefill || !busy)) {
            if (L.ph == kLaneDone) {
                const int64_t t = L.t;
                t_start[t] = L.h0;
                t_nhits[t] = L.nh;
                t_rin[t] = L.rin;
#pragma unroll
                for (int i = 0; i < 5; ++i) t_par[t * 5 + i] = L.in.p[i];
#pragma unroll
                for (int i = 0; i < 15; ++i) t_cov[t * 15 + i] = L.in.C[i];
                t_chi2[t] = L.csum;
                L.ph = kLaneIdle;
            }
            // new starts for the idle lanes, in lane order
            const int need = __popcll(idle);
            const int rank = __popcll(idle & ((1ull << lane) - 1ull));
            int64_t mine = -1;
            int given = 0;
            while (given < need && qi < 8) {
                const int k = (x + qi) & 7;
                const int req = need - given;
                unsigned long long old = 0;
                if (lane == 0) old = atomicAdd(&queue[k], (unsigned long long)req);
                const int64_t o = (int64_t)(((uint64_t)(uint32_t)__shfl((int)(old >> 32), 0) << 32) |
                                            (uint32_t)__shfl((int)(old & 0xFFFFFFFFull), 0));
                const int64_t beg = lo + n * k / 8, len = lo + n * (k + 1) / 8 - beg;
                const int64_t avail = len - o > 0 ? len - o : 0;
                const int got = avail < req ? (int)avail : req;
                if (L.ph == kLaneIdle && rank >= given && rank < given + got)
                    mine = beg + o + (rank - given);
                given += got;
                if (got < req) ++qi;
            }
            if (L.ph == kLaneIdle) {
                if (mine >= 0) {
                    L.t = mine;
                    L.th = t_hits + mine;
                    for (int r = 0; r < n_rows; ++r) L.th[(int64_t)r * cap] = -1;
                    lane_init(L, mine, sec, n_rows, xs, prm, yg, zg, gsr, up, starts, cap);
                } else {
                    L.ph = kLaneOut;
                }
            }
        }
        if (!__ballot(L.ph == kLaneUp || L.ph == kLaneDown)) {
            // nothing left to do unless results are pending (a lane that
            // finished at its first step): write them on the next round
            if (!__ballot(L.ph == kLaneDone)) break;
            continue;
        }
        if (L.ph == kLaneUp || L.ph == kLaneDown)
            lane_step(L, n_rows, xs, prm, bin_start, yg, zg, idg, up, cap, n_prop, n_upd, n_cand);
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

// resident waves of the queue form on the current device
static int64_t tracklet_queue_waves(int n_rows)
{
    constexpr int kDevs = 16;
    static int64_t cache[kDevs][256];
    int dev = 0, n_cu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev >= 0 && dev < kDevs && cache[dev][n_rows] > 0) return cache[dev][n_rows];
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tracklets_queue, kWave,
                                                     tracklet_lds_bytes(n_rows, false)) !=
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
                            const Workspace& ws, hipStream_t st, const tpc_tuning* tune)
{
    // tracklets processed: bounded by both capacities; the hit array's row
    // stride is the tracklet capacity
    const int64_t count_cap = starts.capacity < trl.capacity ? starts.capacity : trl.capacity;
    const int64_t bound = (p->h_sectors[sec_hi - 1].end - p->h_sectors[sec_lo].begin) / 3 + 1;
    const int64_t n_launch = bound < count_cap ? bound : count_cap;
    // waves of starts up to which the LDS form works, then the direct form
    // up to cap_q, the queue form beyond.  Automatically the LDS form while
    // all its waves are resident, else the direct form: on the continuous
    // read-out slice (3.4M starts, lanes of a wave 47% busy in lockstep) the
    // queue form took 32.4 ms against 28.9 ms, its lanes at different rows
    // sharing less of the grid in the caches than lockstep lanes do
    const int form = tune ? tune->tracklet_form : TPC_TRACKLETS_AUTO;
    const int64_t q_waves = tracklet_queue_waves(p->n_rows);
    int64_t cap_lds = tracklet_lds_capacity(p->n_rows), cap_q = INT64_MAX;
    if (form == TPC_TRACKLETS_LDS) cap_lds = cap_q = INT64_MAX;
    if (form == TPC_TRACKLETS_DIRECT) cap_lds = -1, cap_q = INT64_MAX;
    if (form == TPC_TRACKLETS_QUEUE) cap_lds = -1, cap_q = 0;
    const dim3 grid(grid_for_block(n_launch, kWave, 65536));
    // the queue form: at most the resident waves, a multiple of 8 (one
    // share per XCD)
    int64_t qb = ceil_div(n_launch, kWave);
    if (qb > q_waves) qb = q_waves;
    qb = qb < 8 ? (qb < 1 ? 1 : qb) : qb / 8 * 8;
    launch_fill<uint64_t>(ws.tq, 0ull, 8, st);
    TPC_LAUNCH(k_tracklets_queue, dim3((unsigned)qb), dim3(kWave),
               tracklet_lds_bytes(p->n_rows, false), st, p->d_sectors, p->n_rows, p->d_row_x,
               p->params, (const int32_t*)grid_.bin_start, (const float*)grid_.y,
               (const float*)grid_.z, (const int32_t*)grid_.id, (const int32_t*)ws.gsr,
               (const int32_t*)links.up, (const int32_t*)starts.pos, ws.status,
               (const int64_t*)(ws.sec_start + sec_lo), (const int64_t*)(ws.sec_start + sec_hi),
               count_cap, trl.capacity, cap_q, (unsigned long long*)ws.tq, trl.start, trl.hits,
               trl.nhits, trl.row_inner, trl.par, trl.cov, trl.chi2);
    TPC_LAUNCH(k_tracklets<true>, grid, dim3(kWave), tracklet_lds_bytes(p->n_rows, true), st,
               p->d_sectors, p->n_rows, p->d_row_x, p->params, (const int32_t*)grid_.bin_start,
               (const float*)grid_.y, (const float*)grid_.z, (const int32_t*)grid_.id,
               (const int32_t*)ws.gsr, (const int32_t*)links.up, (const int32_t*)starts.pos,
               ws.status, (const int64_t*)(ws.sec_start + sec_lo),
               (const int64_t*)(ws.sec_start + sec_hi), count_cap, trl.capacity, cap_lds, cap_q,
               trl.start, trl.hits, trl.nhits, trl.row_inner, trl.par, trl.cov, trl.chi2);
    TPC_LAUNCH(k_tracklets<false>, grid, dim3(kWave), tracklet_lds_bytes(p->n_rows, false), st,
               p->d_sectors, p->n_rows, p->d_row_x, p->params, (const int32_t*)grid_.bin_start,
               (const float*)grid_.y, (const float*)grid_.z, (const int32_t*)grid_.id,
               (const int32_t*)ws.gsr, (const int32_t*)links.up, (const int32_t*)starts.pos,
               ws.status, (const int64_t*)(ws.sec_start + sec_lo),
               (const int64_t*)(ws.sec_start + sec_hi), count_cap, trl.capacity, cap_lds, cap_q,
               trl.start, trl.hits, trl.nhits, trl.row_inner, trl.par, trl.cov, trl.chi2);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // namespace tpc
