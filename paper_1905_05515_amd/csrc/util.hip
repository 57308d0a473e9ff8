// Scans, fills, workspace layout, context and status calls.
#include "block_dev.hpp"

#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

namespace tpc {

// ---- fill -------------------------------------------------------------------

template <typename T>
__global__ void k_fill(T* __restrict__ p, T v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
void launch_fill(T* p, T v, int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    TPC_LAUNCH(k_fill<T>, dim3(grid_for(n, 8192)), dim3(kBlock), 0, st, p, v, n);
}
template void launch_fill<int32_t>(int32_t*, int32_t, int64_t, hipStream_t);
template void launch_fill<uint64_t>(uint64_t*, uint64_t, int64_t, hipStream_t);
template void launch_fill<int64_t>(int64_t*, int64_t, int64_t, hipStream_t);

// phase 1: sum of every tile
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_tile_sums(const T* __restrict__ in, int64_t n,
                                                           int64_t* __restrict__ partials)
{
    __shared__ T lds[kBlock / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    T tot = block_sum(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = (int64_t)tot;
}

// phase 2: exclusive scan of the tile sums by one block, starting from
// carry0 + *carry_in (device, nullable); *total_dst (nullable) = carry + total.
__global__ __launch_bounds__(kBlock) void k_scan_partials(int64_t* __restrict__ partials, int64_t nt,
                                                          const int64_t* carry_in, int64_t carry0,
                                                          int64_t* total_dst)
{
    __shared__ int64_t lds[kBlock / kWave];
    int64_t carry = carry0 + (carry_in ? *carry_in : 0);
    __syncthreads();
    for (int64_t b = 0; b < nt; b += kScanTile) {
        int64_t base = b + (int64_t)threadIdx.x * kScanItems;
        int64_t v[kScanItems];
        int64_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = (base + k < nt) ? partials[base + k] : 0;
            s += v[k];
        }
        int64_t tot;
        int64_t ex = block_excl_scan(s, lds, &tot) + carry;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (base + k < nt) partials[base + k] = ex;
            ex += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total_dst) *total_dst = carry;
}

// phase 3: scan inside every tile plus its offset
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const T* in, T* out, int64_t n,
                                                       const int64_t* __restrict__ partials,
                                                       int write_total)
{
    __shared__ T lds[kBlock / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : T(0);
        s += v[k];
    }
    T tot;
    T ex = block_excl_scan(s, lds, &tot) + (T)partials[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) out[n] = ex;
}

template <typename T>
void launch_scan(const T* in, T* out, int64_t n, bool write_total, int64_t* total_dst,
                 const int64_t* carry_in, int64_t* partials, hipStream_t st, int64_t carry0)
{
    int64_t nt = ceil_div(n > 0 ? n : 1, kScanTile);
    TPC_LAUNCH(k_scan_tile_sums<T>, dim3((unsigned)nt), dim3(kBlock), 0, st, in, n,
                       partials);
    TPC_LAUNCH(k_scan_partials, dim3(1), dim3(kBlock), 0, st, partials, nt, carry_in, carry0,
                       total_dst);
    TPC_LAUNCH(k_scan_tiles<T>, dim3((unsigned)nt), dim3(kBlock), 0, st, in, out, n,
                       (const int64_t*)partials, write_total ? 1 : 0);
}
void launch_scan_partials(int64_t* partials, int64_t nt, const int64_t* carry_in,
                          int64_t* total_dst, hipStream_t st)
{
    TPC_LAUNCH(k_scan_partials, dim3(1), dim3(kBlock), 0, st, partials, nt, carry_in,
               (int64_t)0, total_dst);
}

template void launch_scan<int32_t>(const int32_t*, int32_t*, int64_t, bool, int64_t*,
                                   const int64_t*, int64_t*, hipStream_t, int64_t);
template void launch_scan<uint64_t>(const uint64_t*, uint64_t*, int64_t, bool, int64_t*,
                                    const int64_t*, int64_t*, hipStream_t, int64_t);

// ---- workspace ----------------------------------------------------------------

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int grid_slabs(const tpc_problem* p)
{
    int S = 1;
    for (int i = 0; i < p->n_sectors; ++i) {
        const int c = slab_count(p->h_sectors[i]);
        if (c > S) S = c;
    }
    return S;
}

bool layout_workspace(const tpc_problem* p, int64_t start_cap, void* base, Workspace* ws)
{
    const int64_t n = p->n_clusters, nb = p->n_bins;
    int64_t scan_n = n > nb + 1 ? n : nb + 1;
    const int64_t nrb1 = (int64_t)p->n_sectors * (p->n_rows + 1) * grid_slabs(p) + 1;
    if (nrb1 > scan_n) scan_n = nrb1;
    if (start_cap + 1 > scan_n) scan_n = start_cap + 1;
    int64_t max_tiles = ceil_div(scan_n, kScanTile) + 1;
    char* b = (char*)base;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return b ? (void*)(b + at) : nullptr;
    };
    // members whose place depends on the problem only first: calls of one
    // problem with different start capacities agree on them
    ws->status = (tpc_status*)take(sizeof(tpc_status));
    ws->cnt = (int32_t*)take(sizeof(int32_t) * (size_t)(nb + 1));
    ws->tmp = (int32_t*)take(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    ws->gsr = (int32_t*)take(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    ws->hitkey = (uint64_t*)take(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    ws->sec_start = (int64_t*)take(sizeof(int64_t) * (size_t)(p->n_sectors + 1));
    ws->pq = (int32_t*)take(sizeof(int32_t) * (size_t)(1 + kPhases * p->n_sectors));
    ws->scnt = (int64_t*)take(sizeof(int64_t) * (size_t)p->n_sectors);
    ws->tsum = (uint64_t*)take(sizeof(uint64_t) * (size_t)p->n_sectors);
    ws->ptile = (int64_t*)take(sizeof(int64_t) * (size_t)(n / 1024 + p->n_sectors + 2));
    ws->pchunk = (int32_t*)take(sizeof(int32_t) * (size_t)p->n_sectors);
    ws->tq = (uint64_t*)take(sizeof(uint64_t) * 8);
    ws->tpos = (int32_t*)take(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    const size_t nrb = (size_t)p->n_sectors * (size_t)(p->n_rows + 1) * (size_t)grid_slabs(p);
    const size_t nn = (size_t)(n > 0 ? n : 1);
    ws->rcnt = (int32_t*)take(sizeof(int32_t) * nrb);
    ws->rfill = (int32_t*)take(sizeof(int32_t) * nrb);
    ws->rstart = (int32_t*)take(sizeof(int32_t) * (nrb + 1));
    ws->gy = (float*)take(sizeof(float) * nn);
    ws->gz = (float*)take(sizeof(float) * nn);
    ws->gslot = (int32_t*)take(sizeof(int32_t) * nn);
    ws->gbin = (int32_t*)take(sizeof(int32_t) * nn);
    ws->gtag = (int32_t*)take(sizeof(int32_t) * nn);
    ws->bigq = (int32_t*)take(sizeof(int32_t) * (nrb + 1));
    // scratch of single calls, sized by the start capacity
    ws->partials = (int64_t*)take(sizeof(int64_t) * (size_t)max_tiles);
    ws->tlen = (uint64_t*)take(sizeof(uint64_t) * (size_t)(start_cap + 1));
    ws->toff = (uint64_t*)take(sizeof(uint64_t) * (size_t)(start_cap + 2));
    ws->ccnt = (uint8_t*)take((size_t)sel_chunks(p->n_rows) * (size_t)(start_cap > 0 ? start_cap : 1));
    ws->tkey = (uint64_t*)take(sizeof(uint64_t) * (size_t)(start_cap > 0 ? start_cap : 1));
    ws->kbits = (uint64_t*)take(sizeof(uint64_t) * (size_t)p->n_rows *
                                (size_t)sel_words(start_cap));
    ws->bytes = o;
    return true;
}

// ---- per-kernel timing ---------------------------------------------------------

struct KernelTimer {
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<Rec> recs;
    const char* pending = nullptr;
    hipEvent_t pending_ev = nullptr;

    hipEvent_t take()
    {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    void reset()
    {
        used = 0;
        recs.clear();
        pending = nullptr;
    }
    ~KernelTimer()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

static thread_local KernelTimer* t_timer = nullptr;

KernelTimer* current_timer() { return t_timer; }
void set_current_timer(KernelTimer* t) { t_timer = t; }

static bool capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

void timer_begin(const char* name, hipStream_t st)
{
    KernelTimer* t = t_timer;
    if (!t || capturing(st)) return;
    for (const char* c = name; *c; ++c)      // drop namespace qualifiers
        if (c[0] == ':' && c[1] == ':') name = c + 2;
    hipEvent_t e = t->take();
    if (!e || hipEventRecord(e, st) != hipSuccess) return;
    t->pending = name;
    t->pending_ev = e;
}

void timer_end(hipStream_t st)
{
    KernelTimer* t = t_timer;
    if (!t || !t->pending) return;
    hipEvent_t e = t->take();
    if (e && hipEventRecord(e, st) == hipSuccess) t->recs.push_back({t->pending, t->pending_ev, e});
    t->pending = nullptr;
}

}  // namespace tpc

// ---- C ABI: context, status --------------------------------------------------

extern "C" {

int tpc_context_create(tpc_context** out, int device)
{
    if (!out) return TPC_ERR_INVALID_ARG;
    *out = nullptr;
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev)
        return TPC_ERR_INVALID_ARG;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return TPC_ERR_HIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TPC_ERR_UNSUPPORTED;
    const int se = tpc::refit_scratch_setup(device);
    if (se) return se;
    tpc_context* c = new (std::nothrow) tpc_context();
    if (!c) return TPC_ERR_HIP;
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    c->graph_exec = nullptr;
    c->graph_key = 0;
    c->graph_valid = false;
    c->timer = nullptr;
    c->n_tables = 0;
    c->tune = tpc_tuning{0, 0, 0, 0};
    *out = c;
    return TPC_OK;
}

int tpc_context_set_tuning(tpc_context* ctx, const tpc_tuning* t)
{
    if (!ctx || !t) return TPC_ERR_INVALID_ARG;
    const bool ok = t->tracklet_form >= TPC_TRACKLETS_AUTO &&
                    t->tracklet_form <= TPC_TRACKLETS_QUEUE &&
                    (t->neighbour_block == 0 || t->neighbour_block == 64 ||
                     t->neighbour_block == 128 || t->neighbour_block == 256) &&
                    (t->persistent_scale == 0 || t->persistent_scale == 1 ||
                     t->persistent_scale == 2 || t->persistent_scale == 4 ||
                     t->persistent_scale == 8) &&
                    t->persistent_blocks_per_cu >= 0 && t->persistent_blocks_per_cu <= 64;
    if (!ok) return TPC_ERR_INVALID_ARG;
    ctx->tune = *t;
    ctx->graph_valid = false;
    return TPC_OK;
}

int tpc_context_get_tuning(const tpc_context* ctx, tpc_tuning* t)
{
    if (!ctx || !t) return TPC_ERR_INVALID_ARG;
    *t = ctx->tune;
    return TPC_OK;
}

int tpc_context_destroy(tpc_context* ctx)
{
    if (!ctx) return TPC_ERR_INVALID_ARG;
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    for (int i = 0; i < ctx->n_tables; ++i) (void)hipFree(ctx->tables[i].d);
    delete ctx->timer;
    delete ctx;
    return TPC_OK;
}

int tpc_timing_enable(tpc_context* ctx, int enable)
{
    if (!ctx) return TPC_ERR_INVALID_ARG;
    if (enable) {
        if (!ctx->timer) ctx->timer = new (std::nothrow) tpc::KernelTimer();
        if (!ctx->timer) return TPC_ERR_HIP;
        ctx->timer->reset();
    } else {
        delete ctx->timer;
        ctx->timer = nullptr;
    }
    return TPC_OK;
}

int tpc_timing_report(tpc_context* ctx, int max_kernels, const char** h_names,
                      int64_t* h_launches, double* h_total_ms, int* h_count)
{
    if (!ctx || !ctx->timer || max_kernels < 0 || !h_count) return TPC_ERR_INVALID_ARG;
    tpc::KernelTimer* t = ctx->timer;
    std::vector<const char*> order;
    std::map<std::string, std::pair<int64_t, double>> agg;
    for (const auto& r : t->recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return TPC_ERR_HIP;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return TPC_ERR_HIP;
        auto it = agg.find(r.name);
        if (it == agg.end()) {
            order.push_back(r.name);
            agg[r.name] = {1, (double)ms};
        } else {
            it->second.first += 1;
            it->second.second += ms;
        }
    }
    int n = 0;
    for (const char* name : order) {
        if (n < max_kernels) {
            if (h_names) h_names[n] = name;
            if (h_launches) h_launches[n] = agg[name].first;
            if (h_total_ms) h_total_ms[n] = agg[name].second;
        }
        ++n;
    }
    *h_count = n;
    t->reset();
    return TPC_OK;
}

static int check_problem(const tpc_problem* p)
{
    if (!p || p->n_sectors <= 0 || p->n_rows < 3 || p->n_rows > 255 || p->n_clusters < 0 ||
        p->n_clusters >= (int64_t(1) << 31) - 1 || p->n_bins <= 0 ||
        p->n_bins >= (int64_t(1) << 31) - 1 || !p->h_sectors || !p->d_sectors || !p->d_row_x)
        return TPC_ERR_INVALID_ARG;
    int64_t prev_end = 0, bins = 0;
    for (int s = 0; s < p->n_sectors; ++s) {
        const tpc_sector& q = p->h_sectors[s];
        if (q.begin != prev_end || q.end < q.begin || q.nby <= 0 || q.nbz <= 0 ||
            q.bin_base != bins || !(q.inv_by > 0.0f) || !(q.inv_bz > 0.0f))
            return TPC_ERR_INVALID_ARG;
        bins += (int64_t)p->n_rows * q.nby * q.nbz + 1;
        prev_end = q.end;
    }
    if (prev_end != p->n_clusters || bins != p->n_bins) return TPC_ERR_INVALID_ARG;
    return TPC_OK;
}

int tpc_check_problem(const tpc_problem* p) { return check_problem(p); }

int tpc_workspace_size(const tpc_problem* h_prob, int64_t start_capacity, size_t* h_bytes)
{
    if (!h_bytes || start_capacity < 0) return TPC_ERR_INVALID_ARG;
    int e = check_problem(h_prob);
    if (e) return e;
    tpc::Workspace ws;
    tpc::layout_workspace(h_prob, start_capacity, nullptr, &ws);
    *h_bytes = ws.bytes;
    return TPC_OK;
}

int tpc_get_status(const void* d_ws, tpc_status* h_out, void* stream)
{
    if (!d_ws || !h_out) return TPC_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(h_out, d_ws, sizeof(tpc_status), hipMemcpyDeviceToHost, st) != hipSuccess)
        return TPC_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return TPC_ERR_HIP;
    return TPC_OK;
}

const char* tpc_status_string(int code)
{
    switch (code) {
    case TPC_OK: return "ok";
    case TPC_ERR_INVALID_ARG: return "invalid argument";
    case TPC_ERR_CAPACITY: return "output capacity exceeded";
    case TPC_ERR_HIP: return "HIP runtime error";
    case TPC_ERR_UNSUPPORTED: return "unsupported device or feature";
    default: return "unknown error";
    }
}

}  // extern "C"
