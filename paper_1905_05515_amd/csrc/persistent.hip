// Persistent batched form (placeholder until the work-queue kernel lands).
#include "tpc_internal.hpp"

namespace tpc {

int run_persistent(tpc_context* ctx, const tpc_problem* p, tpc_clusters in, tpc_grid grid,
                   tpc_links links, tpc_starts starts, tpc_tracklets trl, tpc_tracks trk,
                   const Workspace& ws, hipStream_t st)
{
    (void)ctx; (void)p; (void)in; (void)grid; (void)links; (void)starts; (void)trl; (void)trk;
    (void)ws; (void)st;
    return TPC_ERR_UNSUPPORTED;
}

}  // namespace tpc
