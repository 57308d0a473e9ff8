// Internal declarations shared by the HIP sources of libtpc.so.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/tpc.h"

// All decisions are taken in binary32 with the association order written in
// the source; contraction into FMA is off for the whole library (also passed
// on the command line), the refit included.
#pragma clang fp contract(off)

namespace tpc {

constexpr int kBlock = 256;          // threads per block of the streaming kernels
constexpr int kWave = 64;            // CDNA wavefront
constexpr int kScanItems = 8;        // items per thread in the scans
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kPhases = 16;          // phases of the persistent form

struct Workspace {
    tpc_status* status;
    int32_t* cnt;          // [n_bins + 1] bin counts, then fill cursors
    int32_t* tmp;          // [n] scatter staging, then start flags by id
    int32_t* gsr;          // [n] sector << 8 | row per grid position
    int64_t* partials;     // scan tile partials
    uint64_t* hitkey;      // [n] selection keys per grid position
    uint64_t* tlen;        // [start_cap + 1] per tracklet: accepted << 32 | kept
    uint64_t* toff;        // [start_cap + 1] exclusive scan of tlen
    uint8_t* ccnt;         // [row chunks * start_cap] kept hits per tracklet and row chunk
    uint64_t* tkey;        // [start_cap] selection, big sectors: key per tracklet
    uint64_t* kbits;       // [n_rows * sel_words(start_cap)] selection, big sectors: kept bits
    // grid build: clusters per (sector, row bucket), their running fill and
    // starts; the row-partitioned copy of the clusters; the binned order
    int32_t* rcnt;         // [n_sectors * (n_rows + 1) * S]
    int32_t* rfill;        // [n_sectors * (n_rows + 1) * S]
    int32_t* rstart;       // [n_sectors * (n_rows + 1) * S + 1]
    float* gy;             // [n]
    float* gz;             // [n]
    int32_t* gslot;        // [n] row-partitioned index of the cluster at a binned slot
    int32_t* gbin;         // [n] global bin of a binned slot
    int32_t* gtag;         // [n] sector << 8 | row of a binned slot
    int32_t* bigq;         // [n_sectors * (n_rows + 1) * S + 1] count, then the buckets
                           // the staged grid build places in a pass of their own
    int64_t* sec_start;    // [n_sectors + 1] first start of each sector
    int32_t* pq;           // persistent form: [1] queue head, [kPhases * n_sectors] done counts
    int64_t* scnt;         // persistent form: [n_sectors] starts per sector
    uint64_t* tsum;        // persistent form: [n_sectors] tracks << 32 | hits per sector
    int64_t* ptile;        // persistent form: starts per counting tile
    int32_t* pchunk;       // persistent form: [n_sectors] next tracklet chunk of each sector
    uint64_t* tq;          // [8] queue form of the tracklets: starts taken per XCD share
    int32_t* tpos;         // [n] selection: grid position of every track hit, in track order
    size_t bytes;
};

// Row buckets of the staged grid build.  Every pad row of a sector is cut
// into z slabs of at most kRowBinsLds bins (so that one block counts a
// slab's bins in LDS); bucket (row, slab) of a sector has index
// row * S + slab, S the largest slab count of the problem; the clusters of
// invalid rows form bucket (n_rows, 0).
constexpr int kRowBinsLds = 8192;
__host__ __device__ inline int slab_zbins(const tpc_sector& s)
{
    const int z = kRowBinsLds / (s.nby > 0 ? s.nby : 1);
    return z < 1 ? 1 : z;
}
__host__ __device__ inline int slab_count(const tpc_sector& s)
{
    const int zs = slab_zbins(s);
    return (s.nbz + zs - 1) / zs;
}
// S of a problem (host)
int grid_slabs(const tpc_problem* p);

// Rows of a tracklet handled by one selection work item.
constexpr int kSelRows = 8;
inline int sel_chunks(int n_rows) { return (n_rows + kSelRows - 1) / kSelRows; }
// 64-bit words of one row of the big-sector kept bits
inline int64_t sel_words(int64_t start_cap) { return (start_cap + 63) / 64 + 1; }

// Offsets of the workspace members for a problem; returns false on overflow.
bool layout_workspace(const tpc_problem* p, int64_t start_cap, void* base, Workspace* ws);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Grid size of a grid-stride launch over n items, capped.
inline unsigned grid_for(int64_t n, int64_t cap = 16384)
{
    int64_t g = ceil_div(n > 0 ? n : 1, kBlock);
    return (unsigned)(g < cap ? g : cap);
}

inline unsigned grid_for_block(int64_t n, int block, int64_t cap)
{
    int64_t g = ceil_div(n > 0 ? n : 1, block);
    return (unsigned)(g < cap ? g : cap);
}

// ---- device helpers ---------------------------------------------------------

__device__ inline int find_sector(const tpc_sector* sec, int n_sec, int64_t id)
{
    int lo = 0, hi = n_sec - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (sec[mid].begin <= id) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Bin of a coordinate: (v - v0) * inv clamped to [0, nb - 1] in float, then
// truncated.  Monotone in v.
__device__ inline int bin_of(float v, float v0, float inv, int nb)
{
    float f = (v - v0) * inv;
    if (!(f >= 0.0f)) f = 0.0f;
    float top = (float)(nb - 1);
    if (f > top) f = top;
    return (int)f;
}

// bin of a cluster; rows >= n_rows go to the sector's last (invalid-row) bin
__device__ inline int global_bin(const tpc_sector& s, int n_rows, int row, float y, float z)
{
    if (row >= n_rows) return s.bin_base + n_rows * s.nbz * s.nby;
    int iy = bin_of(y, s.y0, s.inv_by, s.nby);
    int iz = bin_of(z, s.z0, s.inv_bz, s.nbz);
    return s.bin_base + (row * s.nbz + iz) * s.nby + iy;
}

// Launch-order to work-order map that keeps consecutive work items on one
// XCD: workgroups are dealt to the 8 XCDs round robin, so workgroup b runs on
// XCD b % 8; XCD x is given the contiguous work range of its share, and the
// data of neighbouring work items (one sector's rows) stays in one L2.
__device__ __forceinline__ int xcd_remap(int b, int G)
{
    const int x = b & 7, i = b >> 3, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + i;
}

// Windows are widened by this factor before taking bins, so that a rounding
// difference at a window edge never drops a candidate; the exact predicate
// decides.
#define TPC_WIDEN (1.0f + 1.0f / 64.0f)

// ---- per-kernel timing (host) ----------------------------------------------
// When a context has timing enabled, every launch made on its behalf is
// bracketed by two HIP events on the launch stream (not while the stream is
// being captured into a graph).

struct KernelTimer;
KernelTimer* current_timer();
void set_current_timer(KernelTimer* t);
void timer_begin(const char* name, hipStream_t st);
void timer_end(hipStream_t st);

struct TimerScope {
    KernelTimer* saved;
    explicit TimerScope(KernelTimer* t) : saved(current_timer()) { set_current_timer(t); }
    ~TimerScope() { set_current_timer(saved); }
};

#define TPC_LAUNCH(k, g, b, sh, st, ...)                      \
    do {                                                      \
        ::tpc::timer_begin(#k, st);                           \
        hipLaunchKernelGGL(k, g, b, sh, st, __VA_ARGS__);     \
        ::tpc::timer_end(st);                                 \
    } while (0)

// ---- launch helpers (host) --------------------------------------------------

template <typename T>
void launch_fill(T* p, T v, int64_t n, hipStream_t st);

// Exclusive scan of in[0..n) into out[0..n), starting from carry0 +
// *carry_in (device, nullable: 0); out[n] = carry + total when write_total;
// *total_dst (device, nullable) = carry + total.  in may equal out.
template <typename T>
void launch_scan(const T* in, T* out, int64_t n, bool write_total, int64_t* total_dst,
                 const int64_t* carry_in, int64_t* partials, hipStream_t st,
                 int64_t carry0 = 0);

// Exclusive scan, in place, of nt int64 tile partials by one block.
void launch_scan_partials(int64_t* partials, int64_t nt, const int64_t* carry_in,
                          int64_t* total_dst, hipStream_t st);

}  // namespace tpc

struct tpc_context {
    int device;
    int n_cu;
    tpc::KernelTimer* timer;   // non-null while timing is enabled
    // cached graph of tpc_track_batch
    hipGraphExec_t graph_exec;
    uint64_t graph_key;
    bool graph_valid;
    // task tables of the persistent form (device copies), one per sector
    // table seen, keyed on it.  A table is never rewritten, so a launch still
    // running on any stream keeps reading its own; the oldest is freed (after
    // a device synchronisation) when a new one does not fit.
    struct TaskTable {
        uint64_t key;
        int32_t* d;
        int64_t n_tasks;
    };
    static constexpr int kTaskTables = 8;
    TaskTable tables[kTaskTables];
    int n_tables;
    tpc_tuning tune;           // launch shapes (0: automatic)
};

// stage launchers (stream-ordered, no host synchronisation); the sector
// range [sec_lo, sec_hi) selects the sectors a launch covers
namespace tpc {
int run_build_grid(const tpc_problem* p, int sec_lo, int sec_hi, tpc_clusters in,
                   tpc_grid out, const Workspace& ws, hipStream_t st);
// `tune` (may be null: automatic) picks launch shapes only
int run_find_neighbours(const tpc_problem* p, int sec_lo, int sec_hi, tpc_grid grid,
                        tpc_links links, tpc_starts starts, const Workspace& ws,
                        hipStream_t st, const tpc_tuning* tune = nullptr);
int run_construct_tracklets(const tpc_problem* p, int sec_lo, int sec_hi, tpc_grid grid,
                            tpc_links links, tpc_starts starts, tpc_tracklets trl,
                            const Workspace& ws, hipStream_t st,
                            const tpc_tuning* tune = nullptr);
int run_select_keys(const tpc_problem* p, int sec_lo, int sec_hi, tpc_grid grid,
                    int64_t count_cap, tpc_tracklets trl, const Workspace& ws, hipStream_t st);
int run_select_compact(const tpc_problem* p, tpc_grid grid, int64_t count_cap,
                       tpc_tracklets trl, tpc_tracks trk, const Workspace& ws, hipStream_t st);
// device address of the refit adjoint's static scratch on `device`, taken
// once per device (context creation)
int refit_scratch_setup(int device);
// task table of the persistent form (host work, no launch; call before
// any capture)
int prepare_persistent(tpc_context* ctx, const tpc_problem* p);
// all four stages in one persistent launch over a device work queue
int run_persistent(tpc_context* ctx, const tpc_problem* p, tpc_clusters in, tpc_grid grid,
                   tpc_links links, tpc_starts starts, tpc_tracklets trl, tpc_tracks trk,
                   const Workspace& ws, hipStream_t st);
// count_cap bounds the tracklets selected (<= the workspace's start capacity)
int run_select_tracks(const tpc_problem* p, tpc_grid grid, int64_t count_cap,
                      tpc_tracklets trl, tpc_tracks trk, const Workspace& ws,
                      hipStream_t st);
}  // namespace tpc
