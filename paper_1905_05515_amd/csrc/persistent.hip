// Persistent batched form: the whole tracking chain of all sectors (or
// independent sector instances) in one launch over a device work queue.
//
// The queue holds tasks (phase, sector, tile) in phase-major order: every
// tile of phase P of every sector comes before any task of phase P+1.  A
// block pops the next task with one atomic, waits until the tasks it depends
// on have completed, runs it, and counts it done.  A task only ever waits on
// tasks of earlier phases, which sit earlier in the queue and were therefore
// popped by blocks that are already running, so the queue always drains,
// whatever the number of resident blocks.  Sectors of very different sizes
// interleave freely: a small sector's tracklets start while a large one is
// still being binned.
//
// Phases per sector s (clusters = grid positions [begin, end)):
//   0 zero the bin counts, the selection keys        tiles over bins/clusters
//   1 bin histogram                                  tiles over clusters
//   2 scan of the sector's bins (+ reset cursors)    one task
//   3 scatter to staging slots                       tiles over clusters
//   4 rank within bins                               tiles over positions
//   5 best up/down pairs (+ reset start flags)       tiles over positions
//   6 mutual links, start flags                      tiles over positions
//   7 count the sector's starts                      one task
//   8 write them after the earlier sectors' starts   one task (waits on 7 of all s' < s)
//   9 tracklets                                      tiles over the start bound
//  10 selection keys                                 tiles over the start bound
//  11 kept-hit counts                                tiles over the start bound
//  12 the sector's track and hit totals              one task
//  13 write its tracks after the earlier sectors'    one task (waits on 12 of all s' < s)
// The outputs are those of the staged and per-sector forms, bit for bit.
#include "block_dev.hpp"
#include "grid_dev.hpp"
#include "seed_dev.hpp"
#include "select_dev.hpp"
#include "tracklet_dev.hpp"

#include <vector>

namespace tpc {

namespace {

enum Phase {
    P_ZERO, P_COUNT, P_SCAN, P_SCATTER, P_RANK, P_NEIGH, P_CLEAN, P_SCOUNT, P_SWRITE,
    P_TRACKLET, P_KEYS, P_TCOUNT, P_TSUM, P_TWRITE
};
static_assert(P_TWRITE + 1 == kPhases, "phase count");

// items per task of the tiled phases (output invariant)
constexpr int kItems[kPhases] = {4096, 2048, 0, 2048, 1024, 256, 2048, 0, 0, 256, 256, 256, 0, 0};

// a dependency wait gives up after this many polls (an internal error, flagged
// in the status block): every wave reaches the end of the kernel
constexpr int kMaxPolls = 1 << 24;

struct PArgs {
    const tpc_sector* sec;
    int n_sec, n_rows;
    const float* row_x;
    tpc_params prm;
    tpc_clusters in;
    tpc_grid grid;
    tpc_links links;
    int32_t* starts;
    int64_t start_cap;
    tpc_tracklets trl;
    tpc_tracks trk;
    Workspace ws;
    const int32_t* tasks;   // [kPhases + 1] phase offsets, then [kPhases][n_sec + 1] tile prefixes
    int64_t n_tasks;
};

__host__ __device__ inline int64_t start_bound(const tpc_sector& s)
{
    return (s.end - s.begin) / 3 + 1;
}

// wait (thread 0) until *cnt >= need; false on timeout
__device__ __forceinline__ bool wait_count(const int32_t* cnt, int need)
{
    for (int k = 0; k < kMaxPolls; ++k) {
        if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) {
            __threadfence();
            return true;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    return false;
}

__global__ void k_persist_setup(Workspace ws, int n_sec)
{
    const int n = 1 + kPhases * n_sec;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        ws.pq[i] = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < (int)(sizeof(tpc_status) / 8);
         i += gridDim.x * blockDim.x)
        ((int64_t*)ws.status)[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_persistent(PArgs a)
{
    __shared__ float xs[256];
    __shared__ int64_t sh_task;
    __shared__ int sh_ok;
    __shared__ int64_t lds64[kBlock / kWave];
    __shared__ uint64_t ldsu[kBlock / kWave];
    for (int i = threadIdx.x; i < a.n_rows; i += blockDim.x) xs[i] = a.row_x[i];
    const int n_sec = a.n_sec;
    const int32_t* ph_off = a.tasks;
    int32_t* head = a.ws.pq;
    int32_t* done = a.ws.pq + 1;
    tpc_status* status = a.ws.status;
    const int64_t count_cap = a.start_cap < a.trl.capacity ? a.start_cap : a.trl.capacity;

    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) sh_task = atomicAdd(head, 1);
        __syncthreads();
        const int64_t task = sh_task;
        if (task >= a.n_tasks) break;
        // decode phase, sector, tile
        int ph = 0;
        while (ph + 1 < kPhases && task >= ph_off[ph + 1]) ++ph;
        const int32_t* pre = a.tasks + (kPhases + 1) + ph * (n_sec + 1);
        const int32_t local = (int32_t)(task - ph_off[ph]);
        int lo = 0, hi = n_sec - 1;
        while (lo < hi) {   // last sector whose prefix is <= local
            const int mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= local) lo = mid; else hi = mid - 1;
        }
        const int si = lo;
        const int tile = local - pre[si];
        const tpc_sector s = a.sec[si];

        // dependencies
        if (threadIdx.x == 0) {
            bool ok = true;
            if (ph > 0) {
                const int32_t* pp = a.tasks + (kPhases + 1) + (ph - 1) * (n_sec + 1);
                ok = wait_count(done + (ph - 1) * n_sec + si, pp[si + 1] - pp[si]);
            }
            if (ok && (ph == P_SWRITE || ph == P_TWRITE))
                for (int q = 0; q < si && ok; ++q)   // one task per sector in phases 7, 12
                    ok = wait_count(done + (ph - 1) * n_sec + q, 1);
            if (!ok) atomicOr(&status->overflow, 8);
            // after a timed-out wait every later task skips its work: its
            // inputs may be incomplete
            sh_ok = ok && !(__hip_atomic_load(&status->overflow, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT) & 8);
        }
        __syncthreads();

        const int64_t c0 = s.begin, c1 = s.end;
        const int64_t nb = (int64_t)a.n_rows * s.nby * s.nbz + 1;
        const int items = kItems[ph];
        const int64_t i0 = (int64_t)tile * items;
        switch (sh_ok ? ph : -1) {
        case P_ZERO:
            for (int64_t k = i0 + threadIdx.x; k < i0 + items; k += kBlock) {
                if (k < nb) a.ws.cnt[s.bin_base + k] = 0;
                if (k < c1 - c0) a.ws.hitkey[c0 + k] = 0ull;
            }
            break;
        case P_COUNT:
            for (int64_t k = c0 + i0 + threadIdx.x; k < c1 && k < c0 + i0 + items; k += kBlock)
                grid_count_one(a.sec, n_sec, a.n_rows, a.in.row, a.in.y, a.in.z, k, a.ws.cnt,
                               status);
            break;
        case P_SCAN: {
            int32_t* cnt = a.ws.cnt + s.bin_base;
            int32_t* out = a.grid.bin_start + s.bin_base;
            int64_t carry = c0;
            for (int64_t b = 0; b < nb; b += kScanTile) {
                const int64_t base = b + (int64_t)threadIdx.x * kScanItems;
                int64_t v[kScanItems];
                int64_t sum = 0;
#pragma unroll
                for (int k = 0; k < kScanItems; ++k) {
                    v[k] = base + k < nb ? cnt[base + k] : 0;
                    sum += v[k];
                }
                int64_t tot;
                int64_t ex = block_excl_scan(sum, lds64, &tot) + carry;
#pragma unroll
                for (int k = 0; k < kScanItems; ++k) {
                    if (base + k < nb) out[base + k] = (int32_t)ex;
                    ex += v[k];
                }
                carry += tot;
            }
            if (threadIdx.x == 0) out[nb] = (int32_t)carry;
            __syncthreads();
            for (int64_t k = threadIdx.x; k < nb; k += kBlock) cnt[k] = 0;   // fill cursors
            break;
        }
        case P_SCATTER:
            for (int64_t k = c0 + i0 + threadIdx.x; k < c1 && k < c0 + i0 + items; k += kBlock)
                grid_scatter_one(a.sec, n_sec, a.n_rows, a.in.row, a.in.y, a.in.z, k,
                                 a.grid.bin_start, a.ws.cnt, a.ws.tmp);
            break;
        case P_RANK:
            for (int64_t k = c0 + i0 + threadIdx.x; k < c1 && k < c0 + i0 + items; k += kBlock)
                grid_rank_one(a.sec, n_sec, a.n_rows, a.in.row, a.in.y, a.in.z, a.grid.bin_start, k,
                              a.ws.tmp, a.grid.y, a.grid.z, a.grid.id, a.ws.gsr);
            break;
        case P_NEIGH:
            for (int64_t k = c0 + i0 + threadIdx.x; k < c1 && k < c0 + i0 + items; k += kBlock) {
                neighbours_one(k, a.sec, a.n_rows, a.row_x, a.prm, a.grid.bin_start, a.grid.y,
                               a.grid.z, a.grid.id, a.ws.gsr, a.links.up0, a.links.down0);
                a.ws.tmp[k] = -1;   // start flags (the staging array is free again)
            }
            break;
        case P_CLEAN:
            for (int64_t k = c0 + i0 + threadIdx.x; k < c1 && k < c0 + i0 + items; k += kBlock)
                clean_one(k, a.links.up0, a.links.down0, a.grid.id, a.links.up, a.links.down,
                          a.ws.tmp);
            break;
        case P_SCOUNT: {
            int64_t c = 0;
            for (int64_t k = c0 + threadIdx.x; k < c1; k += kBlock) c += a.ws.tmp[k] >= 0;
            const int64_t tot = block_sum(c, lds64);
            if (threadIdx.x == 0) a.ws.scnt[si] = tot;
            break;
        }
        case P_SWRITE: {
            int64_t off = 0;
            for (int q = 0; q < si; ++q) off += a.ws.scnt[q];
            if (threadIdx.x == 0) {
                a.ws.sec_start[si] = off;
                if (si == n_sec - 1) {
                    const int64_t total = off + a.ws.scnt[si];
                    a.ws.sec_start[n_sec] = total;
                    status->n_starts = total;
                    if (total > a.start_cap) atomicOr(&status->overflow, 1);
                }
            }
            int64_t o = off;
            for (int64_t b = c0; b < c1; b += kBlock) {
                const int64_t k = b + threadIdx.x;
                const int32_t v = k < c1 ? a.ws.tmp[k] : -1;
                int64_t tot;
                const int64_t ex = block_excl_scan((int64_t)(v >= 0), lds64, &tot);
                if (v >= 0 && o + ex < a.start_cap) a.starts[o + ex] = v;
                o += tot;
            }
            break;
        }
        case P_TRACKLET: {
            int n_prop = 0, n_upd = 0, n_cand = 0;
            const int64_t lo_t = a.ws.sec_start[si];
            int64_t hi_t = lo_t + a.ws.scnt[si];
            if (hi_t > count_cap) hi_t = count_cap;
            const int64_t t = lo_t + i0 + threadIdx.x;
            if (threadIdx.x < items && t < hi_t)
                build_tracklet(t, a.sec, a.n_rows, xs, a.prm, a.grid.bin_start, a.grid.y,
                               a.grid.z, a.grid.id, a.ws.gsr, a.links.up, a.starts,
                               a.trl.hits + t, a.trl.capacity, a.trl.start, a.trl.nhits,
                               a.trl.row_inner, a.trl.par, a.trl.cov, a.trl.chi2, n_prop, n_upd,
                               n_cand);
            add_work(status, n_prop, n_upd, n_cand);
            break;
        }
        case P_KEYS:
        case P_TCOUNT: {
            const int64_t lo_t = a.ws.sec_start[si];
            int64_t hi_t = lo_t + a.ws.scnt[si];
            if (hi_t > count_cap) hi_t = count_cap;
            const int64_t t = lo_t + i0 + threadIdx.x;
            if (threadIdx.x < items && t < hi_t) {
                if (ph == P_KEYS)
                    sel_keys_one(t, a.n_rows, a.prm, a.grid.id, a.trl.start, a.trl.hits,
                                 a.trl.nhits, a.trl.capacity,
                                 (unsigned long long*)a.ws.hitkey);
                else
                    a.ws.tlen[t] = sel_count_one(t, a.n_rows, a.prm, a.grid.id, a.trl.start,
                                                 a.trl.hits, a.trl.nhits, a.trl.capacity,
                                                 (const unsigned long long*)a.ws.hitkey);
            }
            break;
        }
        case P_TSUM: {
            const int64_t lo_t = a.ws.sec_start[si];
            int64_t hi_t = lo_t + a.ws.scnt[si];
            if (hi_t > count_cap) hi_t = count_cap;
            uint64_t c = 0;
            for (int64_t t = lo_t + threadIdx.x; t < hi_t; t += kBlock) c += a.ws.tlen[t];
            const uint64_t tot = block_sum(c, ldsu);
            if (threadIdx.x == 0) a.ws.tsum[si] = tot;
            break;
        }
        case P_TWRITE: {
            uint64_t off = 0;
            for (int q = 0; q < si; ++q) off += a.ws.tsum[q];
            const int64_t lo_t = a.ws.sec_start[si];
            int64_t hi_t = lo_t + a.ws.scnt[si];
            if (hi_t > count_cap) hi_t = count_cap;
            uint64_t o = off;
            for (int64_t b = lo_t; b < hi_t; b += kBlock) {
                const int64_t t = b + threadIdx.x;
                const uint64_t v = t < hi_t ? a.ws.tlen[t] : 0ull;
                uint64_t tot;
                const uint64_t ex = block_excl_scan(v, ldsu, &tot);
                if (v)
                    sel_write_one(t, o + ex, a.n_rows, a.prm, a.grid.id, a.trl.start,
                                  a.trl.hits, a.trl.nhits, a.trl.capacity,
                                  (const unsigned long long*)a.ws.hitkey, a.sec, a.ws.gsr,
                                  a.trk.off, a.trk.hits, a.trk.tracklet, a.trk.side,
                                  a.trk.capacity, a.trk.hit_capacity);
                o += tot;
            }
            if (si == n_sec - 1 && threadIdx.x == 0) {
                const int64_t nt = (int64_t)(o >> 32), nh = (int64_t)(o & 0xFFFFFFFFull);
                status->n_tracks = nt;
                status->n_track_hits = nh;
                status->n_grid = c1;
                if (nt <= a.trk.capacity) a.trk.off[nt] = (int32_t)nh;
                if (nt > a.trk.capacity) atomicOr(&status->overflow, 2);
                if (nh > a.trk.hit_capacity) atomicOr(&status->overflow, 4);
            }
            break;
        }
        default:
            break;
        }
        // publish: every write of the task is visible before its count
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(done + ph * n_sec + si, 1);
        }
    }
}

// task table: tiles of every phase and sector
void build_tasks(const tpc_problem* p, std::vector<int32_t>& tab, int64_t& n_tasks)
{
    const int ns = p->n_sectors;
    tab.assign((size_t)(kPhases + 1) + (size_t)kPhases * (ns + 1), 0);
    int64_t total = 0;
    for (int ph = 0; ph < kPhases; ++ph) {
        tab[ph] = (int32_t)total;
        int32_t* pre = tab.data() + (kPhases + 1) + (size_t)ph * (ns + 1);
        int64_t acc = 0;
        for (int si = 0; si < ns; ++si) {
            const tpc_sector& s = p->h_sectors[si];
            const int64_t n = s.end - s.begin;
            const int64_t nb = (int64_t)p->n_rows * s.nby * s.nbz + 1;
            int64_t tiles = 1;
            switch (ph) {
            case P_ZERO: tiles = ceil_div(nb > n ? nb : n, kItems[ph]); break;
            case P_COUNT: case P_SCATTER: case P_RANK: case P_NEIGH: case P_CLEAN:
                tiles = ceil_div(n, kItems[ph]);
                break;
            case P_TRACKLET: case P_KEYS: case P_TCOUNT:
                tiles = ceil_div(start_bound(s), kItems[ph]);
                break;
            default: tiles = 1; break;
            }
            if (tiles < 1) tiles = 1;
            pre[si] = (int32_t)acc;
            acc += tiles;
        }
        pre[ns] = (int32_t)acc;
        total += acc;
    }
    tab[kPhases] = (int32_t)total;
    n_tasks = total;
}

uint64_t sectors_key(const tpc_problem* p)
{
    uint64_t h = 1469598103934665603ull;
    const unsigned char* b = (const unsigned char*)p->h_sectors;
    for (size_t i = 0; i < sizeof(tpc_sector) * (size_t)p->n_sectors; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    h ^= (uint64_t)p->n_rows * 0x9e3779b97f4a7c15ull;
    return h;
}

}  // namespace

int prepare_persistent(tpc_context* ctx, const tpc_problem* p)
{
    const uint64_t key = sectors_key(p);
    if (!ctx->d_tasks || ctx->tasks_key != key) {
        // the table depends on the sector table only: built once per problem
        // shape, outside any timed or captured sequence
        std::vector<int32_t> tab;
        int64_t n_tasks = 0;
        build_tasks(p, tab, n_tasks);
        if (n_tasks >= (int64_t(1) << 31) - 1) return TPC_ERR_INVALID_ARG;
        const size_t bytes = tab.size() * sizeof(int32_t);
        if (bytes > ctx->tasks_cap) {
            if (ctx->d_tasks) (void)hipFree(ctx->d_tasks);
            ctx->d_tasks = nullptr;
            ctx->tasks_cap = 0;
            if (hipMalloc(&ctx->d_tasks, bytes) != hipSuccess) return TPC_ERR_HIP;
            ctx->tasks_cap = bytes;
        }
        if (hipMemcpy(ctx->d_tasks, tab.data(), bytes, hipMemcpyHostToDevice) != hipSuccess)
            return TPC_ERR_HIP;
        ctx->tasks_key = key;
        ctx->n_tasks = n_tasks;
    }
    return TPC_OK;
}

int run_persistent(tpc_context* ctx, const tpc_problem* p, tpc_clusters in, tpc_grid grid,
                   tpc_links links, tpc_starts starts, tpc_tracklets trl, tpc_tracks trk,
                   const Workspace& ws, hipStream_t st)
{
    if (!ctx->d_tasks || ctx->tasks_key != sectors_key(p)) return TPC_ERR_INVALID_ARG;
    PArgs a;
    a.sec = p->d_sectors;
    a.n_sec = p->n_sectors;
    a.n_rows = p->n_rows;
    a.row_x = p->d_row_x;
    a.prm = p->params;
    a.in = in;
    a.grid = grid;
    a.links = links;
    a.starts = starts.pos;
    a.start_cap = starts.capacity;
    a.trl = trl;
    a.trk = trk;
    a.ws = ws;
    a.tasks = ctx->d_tasks;
    a.n_tasks = ctx->n_tasks;
    TPC_LAUNCH(k_persist_setup, dim3(64), dim3(kBlock), 0, st, ws, p->n_sectors);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent, kBlock, 0) !=
            hipSuccess || per_cu < 1)
        per_cu = 1;
    int64_t blocks = (int64_t)per_cu * ctx->n_cu;
    if (blocks > a.n_tasks) blocks = a.n_tasks;
    if (blocks < 1) blocks = 1;
    TPC_LAUNCH(k_persistent, dim3((unsigned)blocks), dim3(kBlock), 0, st, a);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // namespace tpc
