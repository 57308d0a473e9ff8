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
// Phases per sector s (clusters = grid positions [begin, end)); the steps
// are those of the staged kernels (grid_dev.hpp, seed_dev.hpp,
// tracklet_dev.hpp, select_dev.hpp):
//   0 zero the sector's bucket counters and totals     one task
//   1 count clusters per row bucket (LDS)              tiles over clusters
//   2 bucket starts                                    one task
//   3 copy clusters into their bucket                  tiles over clusters
//   4 bin sort of a bucket (LDS)                       one task per kBinsGroup buckets
//   5 final places                                     tiles over positions
//   6 best up/down pairs (+ reset start flags)         tiles over positions
//   7 mutual links, start flags                        tiles over positions
//   8 count starts per tile                            tiles over positions
//   9 write them after the earlier starts              tiles (wait on 8 of all s' < s)
//  10 tracklets                                        waves take chunks of the sector's starts
//  11 ownership keys and kept hits of a row chunk      one task per chunk
//  12 accepted / kept per tracklet                     tiles over the sector's tracklets
//  13 the sector's track and hit totals                one task
//  14 track offsets and records                        one task (waits on 13 of all s' < s)
//  15 track hits                                       tiles over the sector's tracklets
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
    P_ZERO, P_ROWS, P_RSCAN, P_RSCATTER, P_BINS, P_PLACE, P_NEIGH, P_CLEAN, P_SCOUNT,
    P_SWRITE, P_TRACKLET, P_SELCHUNK, P_SLEN, P_TSUM, P_TOFF, P_TWRITE
};
static_assert(P_TWRITE + 1 == kPhases, "phase count");

// Items per task of the tiled phases (clusters, grid positions or
// tracklets; the outputs do not depend on them), times the scale of the
// launch; 0: one task per sector, or one per row chunk.  Every task pays a
// few device-wide fences, so tasks are made large enough for that to be
// small beside their work, and the scale (1, 2 or 4) grows them with the
// clusters per resident block.
constexpr int kRowTile = kBlock * 8;   // clusters per bucket-count round
constexpr int kRowItems = 2 * kRowTile;
constexpr int kBinsGroup = 8;          // buckets per bin-sort task
constexpr int kItems[kPhases] = {0,    kRowItems, 0,   kRowItems, 0, 4096, 1024, 4096,
                                 4096, 4096,      512, 0,         4096, 0, 0, 1024};
// the start write reuses the tiles of the start count
static_assert(kItems[P_SCOUNT] == kItems[P_SWRITE], "start tiles");

// a dependency wait gives up after this many polls (an internal error, flagged
// in the status block): every wave reaches the end of the kernel
constexpr int kMaxPolls = 1 << 24;

// LDS scratch of a task, in 64-bit words: bucket counters (ROWS, RSCATTER),
// bin counters (BINS) and selection keys (SELCHUNK).  The registers of the
// tracklet code allow three 256-thread blocks per CU; three such tables fit.
constexpr int kPersistLds = 6144;
static_assert(kPersistLds * 2 >= kRowBinsLds, "bin counters of a slab");
constexpr int kFailed = 8;   // status overflow bit: a wait timed out

struct PArgs {
    const tpc_sector* sec;
    int n_sec, n_rows, S;
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
    int scale;              // tile size multiplier
    const int4* task;       // [n_tasks] {phase, sector, tile, tiles of the phase before}
    const int32_t* tiles;   // [kPhases][n_sec + 1] tile prefixes per phase
    int64_t n_tasks;
};

__host__ __device__ inline int64_t start_bound(const tpc_sector& s)
{
    return (s.end - s.begin) / 3 + 1;
}

// wait until *cnt >= need; false on timeout, or as soon as another task has
// failed (its outputs are missing, so nothing after it may run)
__device__ __forceinline__ bool wait_count(const int32_t* cnt, int need, const int32_t* flags)
{
    for (int k = 0; k < kMaxPolls; ++k) {
        const int c = __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int f = __hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (f & kFailed) return false;
        if (c >= need) {
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

// Tracklets [lo, hi) of a sector, in chunks of one wave taken from the
// sector's chunk counter: every wave of every tracklet task of the sector
// takes the next chunk as soon as it is done with its own (tracklet lengths
// vary a lot, and the static task count only bounds the sector's starts).
__device__ __forceinline__ void tracklet_task(const PArgs& a, const float* xs, int32_t* next,
                                              int64_t lo, int64_t hi)
{
    const int lane = threadIdx.x & (kWave - 1);
    int n_prop = 0, n_upd = 0, n_cand = 0;
    for (;;) {
        int c = 0;
        if (lane == 0) c = atomicAdd(next, 1);
        c = __shfl(c, 0, kWave);
        const int64_t tb = lo + (int64_t)c * kWave;
        if (tb >= hi) break;
        const int64_t t = tb + lane;
        if (t < hi)
            build_tracklet(t, a.sec, a.n_rows, xs, a.prm, a.grid.bin_start, a.grid.y, a.grid.z,
                           a.grid.id, a.ws.gsr, a.links.up, a.starts, a.trl.hits + t,
                           a.trl.capacity, a.trl.start, a.trl.nhits, a.trl.row_inner, a.trl.par,
                           a.trl.cov, a.trl.chi2, n_prop, n_upd, n_cand);
    }
    add_work(a.ws.status, n_prop, n_upd, n_cand);
}

// Kept out of line: with it inlined as well, the ROCm 7.2 code generator
// rejects the kernel at -O2 and above ("Operand has incorrect register
// class").
__device__ __noinline__ void write_track_hits(
    int64_t t, int64_t o, int n_rows, const tpc_params& prm, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ t_start, const int32_t* __restrict__ t_hits,
    const int32_t* __restrict__ t_nhits, int64_t cap,
    const unsigned long long* __restrict__ hitkey, const uint8_t* __restrict__ ccnt,
    int64_t count_cap, const TrkHitOut& out, int64_t hit_cap)
{
    sel_write_hits(t, o, n_rows, prm, idg, t_start, t_hits, t_nhits, cap, hitkey, ccnt,
                   count_cap, out, hit_cap);
}

// three waves per SIMD: the register budget of the fused code (168 VGPRs)
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
void k_persistent(PArgs a)
{
    __shared__ float xs[256];
    __shared__ int4 sh_task;
    __shared__ int64_t lds64[kBlock / kWave];
    __shared__ uint64_t ldsu[kBlock / kWave];
    __shared__ int red[kBlock / kWave];
    __shared__ unsigned long long pbuf[kPersistLds];
    int* ibuf = reinterpret_cast<int*>(pbuf);
    for (int i = threadIdx.x; i < a.n_rows; i += blockDim.x) xs[i] = a.row_x[i];
    const int n_sec = a.n_sec, n_rows = a.n_rows, S = a.S;
    const int Rb = (n_rows + 1) * S;
    int32_t* head = a.ws.pq;
    int32_t* done = a.ws.pq + 1;
    tpc_status* status = a.ws.status;
    const int32_t* flags = &status->overflow;
    const int64_t count_cap = a.start_cap < a.trl.capacity ? a.start_cap : a.trl.capacity;
    const int nq = (n_rows + kSelRows - 1) / kSelRows;

    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const int64_t task = atomicAdd(head, 1);
            sh_task = task < a.n_tasks ? a.task[task] : make_int4(-1, 0, 0, 0);
        }
        __syncthreads();
        const int ph = sh_task.x, si = sh_task.y, tile = sh_task.z, need = sh_task.w;
        if (ph < 0) break;
        const tpc_sector s = a.sec[si];

        // dependencies: all tasks of the previous phase of this sector; for
        // phases 9 and 14 also those of every earlier sector (one thread
        // per sector)
        bool ok = true;
        if (threadIdx.x == 0 && ph > 0) ok = wait_count(done + (ph - 1) * n_sec + si, need, flags);
        if (ph == P_SWRITE || ph == P_TOFF) {
            const int32_t* pp = a.tiles + (ph - 1) * (n_sec + 1);
            for (int q = threadIdx.x; q < si && ok; q += blockDim.x)
                ok = wait_count(done + (ph - 1) * n_sec + q, pp[q + 1] - pp[q], flags);
        }
        if (!ok) atomicOr(&status->overflow, kFailed);
        // a failed task skips its work and publishes nothing
        if (__syncthreads_or(!ok)) continue;

        const int64_t c0 = s.begin, c1 = s.end;
        const int items = kItems[ph] * a.scale;
        const int64_t i0 = (int64_t)tile * items;
        // the sector's tracklets (valid from phase 10 on)
        const int64_t t_lo = a.ws.sec_start[si];
        int64_t t_hi = t_lo + a.ws.scnt[si];
        if (ph < P_TRACKLET) t_hi = t_lo;
        if (t_hi > count_cap) t_hi = count_cap;
        switch (ph) {
        case P_ZERO:
            for (int k = threadIdx.x; k < Rb; k += blockDim.x) {
                a.ws.rcnt[(int64_t)si * Rb + k] = 0;
                a.ws.rfill[(int64_t)si * Rb + k] = 0;
            }
            if (threadIdx.x == 0) {
                a.ws.scnt[si] = 0;
                a.ws.tsum[si] = 0;
                a.ws.pchunk[si] = 0;
            }
            break;
        case P_ROWS:
        case P_RSCATTER: {
            // rounds of kRowTile clusters: per-bucket counts in LDS; ROWS adds
            // them to the sector's counters once, RSCATTER claims a range of
            // every bucket per round and copies the clusters there
            constexpr int kPer = kRowTile / kBlock;
            int64_t bad = 0;
            for (int k = threadIdx.x; k < Rb; k += blockDim.x) ibuf[k] = 0;
            for (int64_t r0 = c0 + i0; r0 < c1 && r0 < c0 + i0 + items; r0 += kRowTile) {
                __syncthreads();
                int bucket[kPer], rank[kPer];
#pragma unroll
                for (int j = 0; j < kPer; ++j) {
                    const int64_t i = r0 + threadIdx.x + (int64_t)j * kBlock;
                    bucket[j] = -1;
                    rank[j] = 0;
                    if (i >= c1) continue;
                    const int r = a.in.row[i];
                    bad += r >= n_rows;
                    bucket[j] = cluster_bucket(s, n_rows, S, r, a.in.z[i]);
                    rank[j] = atomicAdd(&ibuf[bucket[j]], 1);
                }
                if (ph == P_ROWS) continue;
                __syncthreads();
                for (int k = threadIdx.x; k < Rb; k += blockDim.x) {
                    const int c = ibuf[k];
                    if (c) {
                        const int64_t gb = (int64_t)si * Rb + k;
                        ibuf[k] = a.ws.rstart[gb] + atomicAdd(&a.ws.rfill[gb], c);
                    }
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < kPer; ++j) {
                    const int64_t i = r0 + threadIdx.x + (int64_t)j * kBlock;
                    if (i >= c1) continue;
                    const int slot = ibuf[bucket[j]] + rank[j];
                    a.ws.tmp[slot] = (int32_t)i;
                    a.ws.gy[slot] = a.in.y[i];
                    a.ws.gz[slot] = a.in.z[i];
                }
                __syncthreads();
                for (int k = threadIdx.x; k < Rb; k += blockDim.x) ibuf[k] = 0;
            }
            if (ph == P_ROWS) {
                __syncthreads();
                for (int k = threadIdx.x; k < Rb; k += blockDim.x)
                    if (ibuf[k]) atomicAdd(&a.ws.rcnt[(int64_t)si * Rb + k], ibuf[k]);
                const int64_t tot = block_sum(bad, lds64);
                if (threadIdx.x == 0 && tot)
                    atomicAdd((unsigned long long*)&status->n_bad_rows, (unsigned long long)tot);
            }
            break;
        }
        case P_RSCAN: {
            int32_t* out = a.ws.rstart + (int64_t)si * Rb;
            const int32_t* cnt = a.ws.rcnt + (int64_t)si * Rb;
            int64_t carry = c0;
            for (int64_t b = 0; b < Rb; b += kScanTile) {
                const int64_t base = b + (int64_t)threadIdx.x * kScanItems;
                int64_t v[kScanItems];
                int64_t sum = 0;
#pragma unroll
                for (int k = 0; k < kScanItems; ++k) {
                    v[k] = base + k < Rb ? cnt[base + k] : 0;
                    sum += v[k];
                }
                int64_t tot;
                int64_t ex = block_excl_scan(sum, lds64, &tot) + carry;
#pragma unroll
                for (int k = 0; k < kScanItems; ++k) {
                    if (base + k < Rb) out[base + k] = (int32_t)ex;
                    ex += v[k];
                }
                carry += tot;
            }
            // the end of the sector (the next sector writes the same value)
            if (threadIdx.x == 0) out[Rb] = (int32_t)c1;
            break;
        }
        case P_BINS: {
            const int group = kBinsGroup * a.scale;
            for (int bk = tile * group; bk < Rb && bk < (tile + 1) * group; ++bk) {
                grid_bins_bucket(s, si, bk, n_rows, S, a.ws.rstart, a.ws.gy, a.ws.gz, a.ws.tmp,
                                 a.in.row, a.grid.bin_start, a.ws.cnt, a.ws.gslot, a.ws.gbin,
                                 a.ws.gtag, ibuf, red);
                __syncthreads();   // the LDS counters are reused
            }
            break;
        }
        case P_PLACE:
            for (int64_t q = c0 + i0 + threadIdx.x; q < c1 && q < c0 + i0 + items; q += kBlock)
                grid_place_one(q, a.grid.bin_start, a.ws.tmp, a.ws.gy, a.ws.gz, a.ws.gslot,
                               a.ws.gbin, a.ws.gtag, a.grid.y, a.grid.z, a.grid.id, a.ws.gsr);
            break;
        case P_NEIGH: {
            // the down-candidate lists in the task scratch
            static_assert(3 * kNbList * kBlock <= 2 * kPersistLds, "neighbour lists");
            float* nbf = reinterpret_cast<float*>(pbuf);
            const NbList nbl{nbf, nbf + kNbList * kBlock,
                             reinterpret_cast<int*>(nbf + 2 * kNbList * kBlock)};
            for (int64_t k = c0 + i0 + threadIdx.x; k < c1 && k < c0 + i0 + items; k += kBlock) {
                neighbours_one(k, a.sec, n_rows, xs, a.prm, a.grid.bin_start, a.grid.y,
                               a.grid.z, a.grid.id, a.ws.gsr, a.links.up0, a.links.down0,
                               nbl);
                a.ws.tmp[k] = -1;   // start flags (the staging array is free again)
            }
            break;
        }
        case P_CLEAN:
            for (int64_t k = c0 + i0 + threadIdx.x; k < c1 && k < c0 + i0 + items; k += kBlock)
                clean_one(k, a.links.up0, a.links.down0, a.grid.id, a.links.up, a.links.down,
                          a.ws.tmp);
            break;
        case P_SCOUNT: {
            int64_t c = 0;
            for (int64_t k = c0 + i0 + threadIdx.x; k < c1 && k < c0 + i0 + items; k += kBlock)
                c += a.ws.tmp[k] >= 0;
            const int64_t tot = block_sum(c, lds64);
            if (threadIdx.x == 0) {
                a.ws.ptile[a.tiles[P_SCOUNT * (n_sec + 1) + si] + tile] = tot;
                if (tot) atomicAdd((unsigned long long*)&a.ws.scnt[si], (unsigned long long)tot);
            }
            break;
        }
        case P_SWRITE: {
            // starts before this tile: earlier sectors, then earlier tiles
            const int32_t* pc = a.tiles + P_SCOUNT * (n_sec + 1);
            int64_t part = 0, part_sec = 0;
            for (int q = threadIdx.x; q < si; q += blockDim.x) part_sec += a.ws.scnt[q];
            for (int k = threadIdx.x; k < tile; k += blockDim.x) part += a.ws.ptile[pc[si] + k];
            const int64_t sec_off = block_sum(part_sec, lds64);
            const int64_t off = sec_off + block_sum(part, lds64);
            if (threadIdx.x == 0) {
                if (tile == 0) a.ws.sec_start[si] = sec_off;
                if (si == n_sec - 1 && tile == pc[si + 1] - pc[si] - 1) {
                    const int64_t total = sec_off + a.ws.scnt[si];
                    a.ws.sec_start[n_sec] = total;
                    status->n_starts = total;
                    if (total > a.start_cap) atomicOr(&status->overflow, 1);
                }
                lds64[0] = off;
            }
            __syncthreads();
            int64_t o = lds64[0];
            __syncthreads();
            for (int64_t b = c0 + i0; b < c1 && b < c0 + i0 + items; b += kBlock) {
                const int64_t k = b + threadIdx.x;
                const int32_t v = k < c1 && k < c0 + i0 + items ? a.ws.tmp[k] : -1;
                int64_t tot;
                const int64_t ex = block_excl_scan((int64_t)(v >= 0), lds64, &tot);
                if (v >= 0 && o + ex < a.start_cap) a.starts[o + ex] = v;
                o += tot;
            }
            break;
        }
        case P_TRACKLET:
            tracklet_task(a, xs, a.ws.pchunk + si, t_lo, t_hi);
            break;
        case P_SELCHUNK:
            sel_chunk_block(s, tile, n_rows, a.prm, a.grid.bin_start, a.grid.id, a.trl.start,
                            a.trl.hits, a.trl.nhits, t_lo, t_hi, count_cap, a.trl.capacity,
                            (unsigned long long*)a.ws.hitkey, a.ws.ccnt, pbuf, kPersistLds);
            break;
        case P_SLEN:
            for (int64_t t = t_lo + i0 + threadIdx.x; t < t_hi && t < t_lo + i0 + items;
                 t += kBlock) {
                int kept = 0;
                for (int q = 0; q < nq; ++q) kept += a.ws.ccnt[q * count_cap + t];
                a.ws.tlen[t] =
                    kept >= a.prm.min_track_hits ? ((1ull << 32) | (uint64_t)kept) : 0ull;
            }
            break;
        case P_TSUM: {
            uint64_t c = 0;
            for (int64_t t = t_lo + threadIdx.x; t < t_hi; t += kBlock) c += a.ws.tlen[t];
            const uint64_t tot = block_sum(c, ldsu);
            if (threadIdx.x == 0) a.ws.tsum[si] = tot;
            break;
        }
        case P_TOFF: {
            uint64_t part = 0;
            for (int q = threadIdx.x; q < si; q += blockDim.x) part += a.ws.tsum[q];
            uint64_t o = block_sum(part, ldsu);
            for (int64_t b = t_lo; b < t_hi; b += kBlock) {
                const int64_t t = b + threadIdx.x;
                const uint64_t v = t < t_hi ? a.ws.tlen[t] : 0ull;
                uint64_t tot;
                const uint64_t ex = block_excl_scan(v, ldsu, &tot);
                if (v) {
                    a.ws.toff[t] = o + ex;
                    sel_write_track(t, (int64_t)((o + ex) >> 32),
                                    (int64_t)((o + ex) & 0xFFFFFFFFull), a.trl.start, a.sec,
                                    a.ws.gsr, a.trk.off, a.trk.tracklet, a.trk.side,
                                    a.trk.capacity);
                }
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
        case P_TWRITE: {
            const TrkHitOut out{nullptr, a.trk.hits, a.trk.hit_row, a.trk.hit_y, a.trk.hit_z,
                                (const float*)a.grid.y, (const float*)a.grid.z};
            for (int64_t t = t_lo + i0 + threadIdx.x; t < t_hi && t < t_lo + i0 + items;
                 t += kBlock)
                if (a.ws.tlen[t])
                    write_track_hits(t, (int64_t)(a.ws.toff[t] & 0xFFFFFFFFull), n_rows, a.prm,
                                     a.grid.id, a.trl.start, a.trl.hits, a.trl.nhits,
                                     a.trl.capacity, (const unsigned long long*)a.ws.hitkey,
                                     a.ws.ccnt, count_cap, out, a.trk.hit_capacity);
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

// tiles of phase ph of sector s
int64_t phase_tiles(const tpc_problem* p, int scale, int ph, const tpc_sector& s)
{
    const int64_t n = s.end - s.begin;
    int64_t tiles = 1;
    switch (ph) {
    case P_ROWS: case P_RSCATTER: case P_PLACE: case P_NEIGH: case P_CLEAN: case P_SCOUNT:
    case P_SWRITE:
        tiles = ceil_div(n, (int64_t)kItems[ph] * scale);
        break;
    case P_BINS:
        tiles = ceil_div((int64_t)(p->n_rows + 1) * grid_slabs(p), (int64_t)kBinsGroup * scale);
        break;
    case P_TRACKLET: case P_SLEN: case P_TWRITE:
        tiles = ceil_div(start_bound(s), (int64_t)kItems[ph] * scale);
        break;
    case P_SELCHUNK: tiles = sel_chunks(p->n_rows); break;
    default: break;
    }
    return tiles < 1 ? 1 : tiles;
}

// task table: the tasks in queue order (phase-major, then sector, then
// tile), then the tile prefixes [kPhases][n_sec + 1]
bool build_tasks(const tpc_problem* p, int scale, std::vector<int4>& task,
                 std::vector<int32_t>& pre)
{
    const int ns = p->n_sectors;
    pre.assign((size_t)kPhases * (ns + 1), 0);
    task.clear();
    for (int ph = 0; ph < kPhases; ++ph) {
        int32_t* pp = pre.data() + (size_t)ph * (ns + 1);
        int64_t acc = 0;
        for (int si = 0; si < ns; ++si) {
            const int64_t tiles = phase_tiles(p, scale, ph, p->h_sectors[si]);
            const int64_t need = ph > 0 ? phase_tiles(p, scale, ph - 1, p->h_sectors[si]) : 0;
            pp[si] = (int32_t)acc;
            acc += tiles;
            if (acc >= (int64_t(1) << 31) - 1 || (int64_t)task.size() + tiles >= (int64_t(1) << 31) - 1)
                return false;
            for (int64_t t = 0; t < tiles; ++t)
                task.push_back(make_int4(ph, si, (int)t, (int)need));
        }
        pp[ns] = (int32_t)acc;
    }
    return true;
}

// resident blocks of the persistent kernel on the context's device (the
// occupancy query is not free: kept per device)
int64_t persistent_blocks(const tpc_context* ctx)
{
    constexpr int kDevs = 16;
    static int cache[kDevs];
    const bool cached = ctx->device >= 0 && ctx->device < kDevs;
    int per_cu = cached ? cache[ctx->device] : 0;
    if (per_cu < 1) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent, kBlock, 0) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        if (cached) cache[ctx->device] = per_cu;
    }
    const int want = ctx->tune.persistent_blocks_per_cu;
    return (int64_t)(want > 0 && want < per_cu ? want : per_cu) * ctx->n_cu;
}

// tile scale: 1, 2 or 4, growing with the clusters per resident block,
// unless the context fixes it
int tile_scale(const tpc_context* ctx, const tpc_problem* p, int64_t blocks)
{
    if (ctx->tune.persistent_scale > 0) return ctx->tune.persistent_scale;
    const int64_t per_block = p->n_clusters / (blocks > 0 ? blocks : 1);
    return per_block >= 8192 ? 4 : per_block >= 4096 ? 2 : 1;
}

uint64_t sectors_key(const tpc_problem* p, int scale)
{
    uint64_t h = 1469598103934665603ull;
    const unsigned char* b = (const unsigned char*)p->h_sectors;
    for (size_t i = 0; i < sizeof(tpc_sector) * (size_t)p->n_sectors; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    h ^= (uint64_t)p->n_rows * 0x9e3779b97f4a7c15ull;
    h ^= (uint64_t)scale * 0xc2b2ae3d27d4eb4full;
    return h;
}

}  // namespace

namespace {

const tpc_context::TaskTable* find_table(const tpc_context* ctx, uint64_t key)
{
    for (int i = 0; i < ctx->n_tables; ++i)
        if (ctx->tables[i].key == key) return &ctx->tables[i];
    return nullptr;
}

}  // namespace

int prepare_persistent(tpc_context* ctx, const tpc_problem* p)
{
    const int scale = tile_scale(ctx, p, persistent_blocks(ctx));
    const uint64_t key = sectors_key(p, scale);
    if (find_table(ctx, key)) return TPC_OK;
    // the table depends on the sector table only: built once per problem
    // shape, outside any timed or captured sequence
    std::vector<int4> task;
    std::vector<int32_t> pre;
    if (!build_tasks(p, scale, task, pre)) return TPC_ERR_INVALID_ARG;
    const size_t tbytes = task.size() * sizeof(int4);
    const size_t bytes = tbytes + pre.size() * sizeof(int32_t);
    if (ctx->n_tables == tpc_context::kTaskTables) {
        // a launch on any stream may still read the oldest table
        if (hipDeviceSynchronize() != hipSuccess) return TPC_ERR_HIP;
        (void)hipFree(ctx->tables[0].d);
        for (int i = 1; i < ctx->n_tables; ++i) ctx->tables[i - 1] = ctx->tables[i];
        --ctx->n_tables;
    }
    int32_t* d = nullptr;
    if (hipMalloc(&d, bytes) != hipSuccess) return TPC_ERR_HIP;
    // a fresh allocation: no launch reads it yet
    if (hipMemcpy(d, task.data(), tbytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy((char*)d + tbytes, pre.data(), pre.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return TPC_ERR_HIP;
    }
    ctx->tables[ctx->n_tables++] = tpc_context::TaskTable{key, d, (int64_t)task.size()};
    return TPC_OK;
}

int run_persistent(tpc_context* ctx, const tpc_problem* p, tpc_clusters in, tpc_grid grid,
                   tpc_links links, tpc_starts starts, tpc_tracklets trl, tpc_tracks trk,
                   const Workspace& ws, hipStream_t st)
{
    const int64_t resident = persistent_blocks(ctx);
    const int scale = tile_scale(ctx, p, resident);
    const tpc_context::TaskTable* tab = find_table(ctx, sectors_key(p, scale));
    if (!tab) return TPC_ERR_INVALID_ARG;
    PArgs a;
    a.scale = scale;
    a.sec = p->d_sectors;
    a.n_sec = p->n_sectors;
    a.n_rows = p->n_rows;
    a.S = grid_slabs(p);
    if ((a.n_rows + 1) * a.S > kPersistLds * 2) return TPC_ERR_UNSUPPORTED;   // LDS bucket counters
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
    a.task = reinterpret_cast<const int4*>(tab->d);
    a.tiles = reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(tab->d) +
                                               tab->n_tasks * sizeof(int4));
    a.n_tasks = tab->n_tasks;
    TPC_LAUNCH(k_persist_setup, dim3(64), dim3(kBlock), 0, st, ws, p->n_sectors);
    int64_t blocks = resident;
    if (blocks > a.n_tasks) blocks = a.n_tasks;
    if (blocks < 1) blocks = 1;
    TPC_LAUNCH(k_persistent, dim3((unsigned)blocks), dim3(kBlock), 0, st, a);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // namespace tpc
