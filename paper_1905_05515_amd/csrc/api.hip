// C ABI entry points of the tracking chain: argument checks, workspace
// layout, stage launches, batched form with graph replay.
#include "tpc_internal.hpp"

#include <cstring>

extern "C" int tpc_check_problem(const tpc_problem* p);

namespace {

int prepare(tpc_context* ctx, const tpc_problem* p, void* d_ws, size_t ws_bytes,
            int64_t start_cap, tpc::Workspace* ws)
{
    if (!ctx || !d_ws) return TPC_ERR_INVALID_ARG;
    int e = tpc_check_problem(p);
    if (e) return e;
    tpc::layout_workspace(p, start_cap, d_ws, ws);
    if (ws->bytes > ws_bytes) return TPC_ERR_INVALID_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TPC_ERR_HIP;
    if (dev != ctx->device && hipSetDevice(ctx->device) != hipSuccess) return TPC_ERR_HIP;
    return TPC_OK;
}

bool grid_ok(const tpc_grid& g) { return g.bin_start && g.y && g.z && g.id; }
bool links_ok(const tpc_links& l) { return l.up0 && l.down0 && l.up && l.down; }
bool starts_ok(const tpc_starts& s) { return s.pos && s.capacity >= 0; }
bool trl_ok(const tpc_tracklets& t, const tpc_starts& s)
{
    return t.start && t.hits && t.nhits && t.row_inner && t.par && t.cov && t.chi2 &&
           t.capacity >= s.capacity;
}
bool trk_ok(const tpc_tracks& t)
{
    const bool copies = t.hit_row || t.hit_y || t.hit_z;
    return t.off && t.hits && t.tracklet && t.capacity >= 0 && t.hit_capacity >= 0 &&
           (!copies || (t.hit_row && t.hit_y && t.hit_z));
}

uint64_t mix(uint64_t h, uint64_t v)
{
    h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    return h;
}

}  // namespace

extern "C" {

int tpc_build_grid(tpc_context* ctx, const tpc_problem* h_prob, tpc_clusters in, tpc_grid out,
                   void* d_ws, size_t ws_bytes, void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    tpc::Workspace ws;
    int e = prepare(ctx, h_prob, d_ws, ws_bytes, 0, &ws);
    if (e) return e;
    if (!in.row || !in.y || !in.z || !grid_ok(out)) return TPC_ERR_INVALID_ARG;
    return tpc::run_build_grid(h_prob, 0, h_prob->n_sectors, in, out, ws, (hipStream_t)stream);
}

int tpc_find_neighbours(tpc_context* ctx, const tpc_problem* h_prob, tpc_grid grid,
                        tpc_links links, tpc_starts starts, void* d_ws, size_t ws_bytes,
                        void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    tpc::Workspace ws;
    int e = prepare(ctx, h_prob, d_ws, ws_bytes, starts.capacity, &ws);
    if (e) return e;
    if (!grid_ok(grid) || !links_ok(links) || !starts_ok(starts)) return TPC_ERR_INVALID_ARG;
    return tpc::run_find_neighbours(h_prob, 0, h_prob->n_sectors, grid, links, starts, ws,
                                    (hipStream_t)stream, ctx ? &ctx->tune : nullptr);
}

int tpc_construct_tracklets(tpc_context* ctx, const tpc_problem* h_prob, tpc_grid grid,
                            tpc_links links, tpc_starts starts, tpc_tracklets tracklets,
                            void* d_ws, size_t ws_bytes, void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    tpc::Workspace ws;
    int e = prepare(ctx, h_prob, d_ws, ws_bytes, starts.capacity, &ws);
    if (e) return e;
    if (!grid_ok(grid) || !links_ok(links) || !starts_ok(starts) || !trl_ok(tracklets, starts))
        return TPC_ERR_INVALID_ARG;
    return tpc::run_construct_tracklets(h_prob, 0, h_prob->n_sectors, grid, links, starts,
                                        tracklets, ws, (hipStream_t)stream,
                                        ctx ? &ctx->tune : nullptr);
}

int tpc_select_tracks(tpc_context* ctx, const tpc_problem* h_prob, tpc_grid grid,
                      tpc_tracklets tracklets, tpc_tracks tracks, void* d_ws, size_t ws_bytes,
                      void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    tpc::Workspace ws;
    int e = prepare(ctx, h_prob, d_ws, ws_bytes, tracklets.capacity, &ws);
    if (e) return e;
    tpc_starts dummy{nullptr, tracklets.capacity};
    if (!grid_ok(grid) || !trl_ok(tracklets, dummy) || !trk_ok(tracks)) return TPC_ERR_INVALID_ARG;
    return tpc::run_select_tracks(h_prob, grid, tracklets.capacity, tracklets, tracks, ws,
                                  (hipStream_t)stream);
}

int tpc_track_batch(tpc_context* ctx, const tpc_problem* h_prob, tpc_clusters in,
                    tpc_grid grid, tpc_links links, tpc_starts starts,
                    tpc_tracklets tracklets, tpc_tracks tracks, void* d_ws, size_t ws_bytes,
                    int mode, int use_graph, void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    tpc::Workspace ws;
    int e = prepare(ctx, h_prob, d_ws, ws_bytes, starts.capacity, &ws);
    if (e) return e;
    if (!in.row || !in.y || !in.z || !grid_ok(grid) || !links_ok(links) || !starts_ok(starts) ||
        !trl_ok(tracklets, starts) || !trk_ok(tracks))
        return TPC_ERR_INVALID_ARG;
    if (mode != TPC_MODE_STAGED && mode != TPC_MODE_PER_SECTOR && mode != TPC_MODE_PERSISTENT)
        return TPC_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int ns = h_prob->n_sectors;
    if (mode == TPC_MODE_PERSISTENT) {
        const int pe = tpc::prepare_persistent(ctx, h_prob);
        if (pe) return pe;
    }
    // never more tracklets than starts: the selection runs over the start
    // capacity the workspace was sized for
    const int64_t count_cap = starts.capacity;
    const tpc_tuning* tune = ctx ? &ctx->tune : nullptr;
    auto body = [&]() -> int {
        int r = TPC_OK;
        if (mode == TPC_MODE_STAGED) {
            r = tpc::run_build_grid(h_prob, 0, ns, in, grid, ws, st);
            if (!r)
                r = tpc::run_find_neighbours(h_prob, 0, ns, grid, links, starts, ws, st, tune);
            if (!r)
                r = tpc::run_construct_tracklets(h_prob, 0, ns, grid, links, starts, tracklets,
                                                 ws, st, tune);
            if (!r) r = tpc::run_select_tracks(h_prob, grid, count_cap, tracklets, tracks, ws, st);
        } else if (mode == TPC_MODE_PER_SECTOR) {
            // every stage sector by sector, then one dense compaction of the
            // track list over all tracklets
            tpc::launch_fill<uint64_t>(ws.tlen, 0ull, count_cap + 1, st);
            for (int s = 0; s < ns && !r; ++s) {
                r = tpc::run_build_grid(h_prob, s, s + 1, in, grid, ws, st);
                if (!r)
                    r = tpc::run_find_neighbours(h_prob, s, s + 1, grid, links, starts, ws, st,
                                                 tune);
                if (!r)
                    r = tpc::run_construct_tracklets(h_prob, s, s + 1, grid, links, starts,
                                                     tracklets, ws, st, tune);
                if (!r) r = tpc::run_select_keys(h_prob, s, s + 1, grid, count_cap, tracklets, ws, st);
            }
            if (!r) r = tpc::run_select_compact(h_prob, grid, count_cap, tracklets, tracks, ws, st);
        } else {
            r = tpc::run_persistent(ctx, h_prob, in, grid, links, starts, tracklets, tracks, ws, st);
        }
        return r;
    };
    if (!use_graph) return body();

    // graph keyed on every pointer and size the launches depend on
    uint64_t key = 1469598103934665603ull;
    const void* ptrs[] = {in.row, in.y, in.z, grid.bin_start, grid.y, grid.z, grid.id,
                          links.up0, links.down0, links.up, links.down, starts.pos,
                          tracklets.start, tracklets.hits, tracklets.nhits, tracklets.row_inner,
                          tracklets.par, tracklets.cov, tracklets.chi2, tracks.off, tracks.hits,
                          tracks.tracklet, tracks.side, tracks.hit_row, tracks.hit_y,
                          tracks.hit_z, d_ws, h_prob->d_sectors, h_prob->d_row_x, stream};
    for (const void* q : ptrs) key = mix(key, (uint64_t)(uintptr_t)q);
    key = mix(key, (uint64_t)starts.capacity);
    if (tune)
        key = mix(key, (uint64_t)(uint32_t)tune->tracklet_form |
                           (uint64_t)(uint32_t)tune->neighbour_block << 8 |
                           (uint64_t)(uint32_t)tune->persistent_scale << 24 |
                           (uint64_t)(uint32_t)tune->persistent_blocks_per_cu << 32);
    key = mix(key, (uint64_t)tracklets.capacity);
    key = mix(key, (uint64_t)tracks.capacity);
    key = mix(key, (uint64_t)tracks.hit_capacity);
    key = mix(key, (uint64_t)h_prob->n_clusters);
    key = mix(key, (uint64_t)h_prob->n_bins);
    key = mix(key, (uint64_t)mode);
    for (int s = 0; s < h_prob->n_sectors; ++s) {
        uint64_t w[5];
        std::memcpy(w, &h_prob->h_sectors[s], sizeof(w));
        for (uint64_t x : w) key = mix(key, x);
    }
    uint32_t pw[sizeof(tpc_params) / 4];
    std::memcpy(pw, &h_prob->params, sizeof(pw));
    for (uint32_t x : pw) key = mix(key, x);

    if (!(ctx->graph_valid && ctx->graph_key == key)) {
        if (ctx->graph_exec) {
            (void)hipGraphExecDestroy(ctx->graph_exec);
            ctx->graph_exec = nullptr;
        }
        ctx->graph_valid = false;
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return TPC_ERR_HIP;
        int r = body();
        hipError_t ce = hipStreamEndCapture(st, &g);
        if (r) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if (ce != hipSuccess) return TPC_ERR_HIP;
        hipGraphExec_t ex = nullptr;
        hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) return TPC_ERR_HIP;
        ctx->graph_exec = ex;
        ctx->graph_key = key;
        ctx->graph_valid = true;
    }
    return hipGraphLaunch(ctx->graph_exec, st) == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // extern "C"
