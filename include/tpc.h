/*
 * tpc.h -- C ABI of the MI355X TPC track-finding library (libtpc.so).
 *
 * Hot path of the online TPC tracking of arXiv:1905.05515, section 3: the
 * combinatorial seeding is a cellular automaton over adjacent pad rows, and
 * the track following after it is a single-hypothesis Kalman filter whose
 * run time is linear in the number of hits.  The calls below are the steps
 * of that path, in order:
 *
 *   tpc_build_grid           bin each sector's clusters into a pad-row grid
 *   tpc_find_neighbours      best up/down link per hit, mutual-link cleaning,
 *                            chain starts (cellular-automaton seeding)
 *   tpc_construct_tracklets  Kalman-filter following of each chain along the
 *                            rows, outwards then inwards
 *   tpc_select_tracks        resolve shared clusters, keep good tracklets
 *   tpc_refit                calibrated Kalman refit of found tracks (the
 *                            paper's refit once calibration is applied,
 *                            section 2, and online drift-velocity
 *                            calibration, section 3)
 *   tpc_refit_adjoint        gradient of the refit chi2 with respect to hit
 *                            coordinates and calibration parameters
 *   tpc_track_batch          the first four steps for many sectors or
 *                            collisions, in one persistent launch or as a
 *                            per-sector sequence, optionally graph-replayed
 *
 * Conventions
 *   - Pointers named d_* and all array members of the argument structs are
 *     device pointers (HIP device memory of the context's device); h_*
 *     pointers are host memory.  The caller owns every buffer; the library
 *     never allocates or frees caller memory.  tpc_context holds only a few
 *     KB of device memory of its own plus cached graphs.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL is the
 *     default stream) unless stated otherwise.  Argument errors are detected
 *     on the host before anything is launched and return
 *     TPC_ERR_INVALID_ARG.  Capacity overflows are detected on the device:
 *     the kernels stop writing past the capacity, set a flag and record the
 *     size that would have been needed in the workspace status block; the
 *     outputs are then incomplete and the caller re-sizes and calls again.
 *   - Nothing throws or aborts across this interface.
 *   - All decisions (bins, links, hit choices, selection) are taken in IEEE
 *     binary32 with a fixed association order and no contraction, and ties
 *     are broken on cluster ids: the outputs depend on the input values and
 *     ids only, not on launch shapes, bin sizes or launch form.
 *   - Cluster ids are indices into the caller's cluster arrays.  "Grid
 *     positions" index the grid arrays that tpc_build_grid writes.
 */
#ifndef TPC_H
#define TPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TPC_OK = 0,
    TPC_ERR_INVALID_ARG = 1,   /* bad argument, detected on the host */
    TPC_ERR_CAPACITY = 2,      /* an output was too small (see tpc_status) */
    TPC_ERR_HIP = 3,           /* a HIP runtime call failed */
    TPC_ERR_UNSUPPORTED = 4    /* device is not gfx950 or feature missing */
};

/* Physics constants and cuts.  They define the outputs; the values used by
 * this project are its readings of the paper, which states none. */
typedef struct tpc_params {
    float curv;            /* curvature [1/cm] per unit q/pT: -0.0029979*B[T] */
    float nb_win_y;        /* neighbour window half width in y [cm] */
    float nb_win_z;        /* neighbour window half width in z [cm] */
    float nb_d2max;        /* max straight-line deviation^2 of a link pair [cm^2] */
    float sigma_y2;        /* cluster variance in y [cm^2] */
    float sigma_z2;        /* cluster variance in z [cm^2] */
    float chi2_max;        /* hit-search gate on the predicted chi2 */
    float search_nsigma;   /* half width of the bins scanned, in sigma (speed only) */
    float s_max;           /* propagation stops where |sin(phi)| reaches this */
    float c_ss0, c_tt0, c_ww0;  /* initial variances of sin(phi), tan(lambda), q/pT */
    int32_t max_miss;      /* consecutive rows without a hit that end a search */
    int32_t min_tracklet_hits;  /* shorter tracklets take no part in selection */
    int32_t min_track_hits;     /* tracks keeping fewer hits are dropped */
} tpc_params;

/* One sector (or independent sector instance).  Its clusters are the ids
 * [begin, end), sector-local coordinates; its grid has n_rows * nbz * nby
 * bins starting at global bin index bin_base, bin (row, iz, iy) at
 * bin_base + (row * nbz + iz) * nby + iy, with
 * iy = clamp((y - y0) * inv_by, 0, nby - 1) truncated (likewise iz); one
 * more bin, bin_base + n_rows * nbz * nby, holds the clusters whose row is
 * >= n_rows (they take no part in tracking).  The sector thus owns
 * n_rows * nbz * nby + 1 bins and exactly the grid positions [begin, end).
 * side: -1 for a sector on the z < 0 side, otherwise +1 (used by the
 * refit's drift-length model only). */
typedef struct tpc_sector {
    float y0, z0;
    float inv_by, inv_bz;
    int32_t nby, nbz;
    int32_t bin_base;
    int32_t side;
    int64_t begin, end;
} tpc_sector;

typedef struct tpc_problem {
    int32_t n_sectors;
    int32_t n_rows;            /* pad rows, 3..255; row r sits at x = d_row_x[r] */
    int64_t n_clusters;        /* total, = last sector's end, < 2^31 */
    int64_t n_bins;            /* total bins over all sectors, < 2^31 */
    const tpc_sector* h_sectors;   /* host copy of the sector table */
    const tpc_sector* d_sectors;   /* device copy, same contents */
    const float* d_row_x;          /* device [n_rows], increasing */
    tpc_params params;
} tpc_problem;

/* Clusters, structure of arrays, grouped by sector (any order inside). */
typedef struct tpc_clusters {
    const uint8_t* row;    /* pad row; rows >= n_rows go to the invalid-row bin */
    const float* y;        /* sector-local y [cm] */
    const float* z;        /* z, or drift time scaled to z [cm] */
} tpc_clusters;

/* Grid: clusters ordered by (sector, row, z bin, y bin, cluster id).
 * bin_start[n_bins + 1]: first grid position of every bin; y, z, id
 * [n_clusters]: coordinates and cluster id at each grid position. */
typedef struct tpc_grid {
    int32_t* bin_start;
    float* y;
    float* z;
    int32_t* id;
} tpc_grid;

/* Links between hits on adjacent rows, indexed by grid position, values
 * are grid positions (-1 none).  up0/down0: best pair per hit before
 * cleaning; up/down: mutual links only. */
typedef struct tpc_links {
    int32_t* up0;
    int32_t* down0;
    int32_t* up;
    int32_t* down;
} tpc_links;

/* Chain starts: grid positions, ascending cluster id.  Count in tpc_status. */
typedef struct tpc_starts {
    int32_t* pos;
    int64_t capacity;
} tpc_starts;

/* Tracklets, one per chain start, in start order.
 * start[capacity]: grid position of the chain start;
 * hits[n_rows * capacity]: hits[r * capacity + t] is the grid position of
 * the hit of tracklet t on row r, -1 none;
 * par[capacity * 5] (y, z, sin(phi), tan(lambda), q/pT) and
 * cov[capacity * 15] (lower triangle, row by row) at the innermost hit,
 * row_inner its row; chi2 the sum of the inward pass. */
typedef struct tpc_tracklets {
    int32_t* start;
    int32_t* hits;
    int32_t* nhits;
    int32_t* row_inner;
    float* par;
    float* cov;
    float* chi2;
    int64_t capacity;
} tpc_tracklets;

/* Tracks (CSR): off[n_tracks + 1], hits[off[k]..off[k+1]) cluster ids in
 * ascending row, tracklet[k] the tracklet it came from (ascending), side[k]
 * (nullable) the z side of its sector.  hit_row, hit_y, hit_z (nullable,
 * all three or none, hit_capacity entries): the pad row and coordinates of
 * every hit in the order of hits, so that a refit reads the track hits as
 * contiguous runs instead of gathering them by cluster id. */
typedef struct tpc_tracks {
    int32_t* off;
    int32_t* hits;
    int32_t* tracklet;
    int8_t* side;
    int64_t capacity;      /* tracks; off needs capacity + 1 entries */
    int64_t hit_capacity;
    uint8_t* hit_row;
    float* hit_y;
    float* hit_z;
} tpc_tracks;

/* Device status block at the start of the workspace. */
typedef struct tpc_status {
    int64_t n_grid;        /* clusters placed in the grid (all of them) */
    int64_t n_bad_rows;    /* clusters with row >= n_rows (invalid-row bins) */
    int64_t n_starts;      /* chain starts found (may exceed capacity) */
    int64_t n_tracks;      /* tracks (may exceed capacity) */
    int64_t n_track_hits;  /* hits of all tracks (may exceed capacity) */
    int32_t overflow;      /* bit 0 starts, bit 1 tracks, bit 2 track hits */
    int32_t pad_;
    /* work of the tracklet construction: transports, Kalman updates and
     * predicted-chi2 evaluations of search candidates */
    int64_t n_propagations;
    int64_t n_updates;
    int64_t n_candidates;
} tpc_status;

typedef struct tpc_context tpc_context;

/* Context: binds a device, holds launch shapes and cached graphs.  One
 * context per stream at a time; distinct contexts are independent. */
int tpc_context_create(tpc_context** out, int device);
int tpc_context_destroy(tpc_context* ctx);

/* Launch shapes of a context (none changes any output; every field 0 is
 * the library's own choice).  tracklet_form: how tpc_construct_tracklets
 * holds the hit lists while it builds them and deals the starts to
 * waves: TPC_TRACKLETS_LDS (one LDS column per lane, written out at the
 * end), TPC_TRACKLETS_DIRECT (written into the output as found) or
 * TPC_TRACKLETS_QUEUE (written directly; resident waves whose lanes take a
 * new start from a device queue whenever theirs is done); automatic takes
 * the LDS form while all its waves are resident at once, else the direct
 * form.  neighbour_block: threads per block
 * of the neighbour kernel (64, 128 or 256).  persistent_scale: tile size
 * multiplier of the persistent form (1, 2, 4 or 8; automatic grows it with
 * the clusters per resident block).  persistent_blocks_per_cu: blocks of
 * the persistent launch per compute unit (at most the resident count;
 * automatic: all resident).  tpc_context_set_tuning returns
 * TPC_ERR_INVALID_ARG for any other value and drops the context's cached
 * graph. */
enum { TPC_TRACKLETS_AUTO = 0, TPC_TRACKLETS_LDS = 1, TPC_TRACKLETS_DIRECT = 2,
       TPC_TRACKLETS_QUEUE = 3 };
typedef struct tpc_tuning {
    int32_t tracklet_form;
    int32_t neighbour_block;
    int32_t persistent_scale;
    int32_t persistent_blocks_per_cu;
} tpc_tuning;
int tpc_context_set_tuning(tpc_context* ctx, const tpc_tuning* h_tuning);
int tpc_context_get_tuning(const tpc_context* ctx, tpc_tuning* h_tuning);

/* Bytes of device workspace needed by the tracking calls for this problem
 * and start capacity.  The same workspace must be passed, unchanged, to the
 * calls of one event in order; it holds the status block at offset 0. */
int tpc_workspace_size(const tpc_problem* h_prob, int64_t start_capacity, size_t* h_bytes);

/* Grid (section 3: the cellular automaton works on hits of adjacent pad
 * rows; the grid gives each hit its row neighbourhood).  Stable counting
 * sort per sector by (row, z bin, y bin), ties by cluster id. */
int tpc_build_grid(tpc_context* ctx, const tpc_problem* h_prob, tpc_clusters in,
                   tpc_grid out, void* d_ws, size_t ws_bytes, void* stream);

/* Cellular-automaton seeding (section 3).  For each hit on rows
 * 1..n_rows-2, among candidates on row r+1 within (nb_win_y, nb_win_z) of
 * the straight line from the origin through the hit (in y; the z vertex is
 * unknown in continuous read-out, section 2) and likewise on row r-1, the
 * pair of least straight-line deviation
 * ((y_u + y_d) - 2y)^2 + ((z_u + z_d) - 2z)^2 <= nb_d2max, ties by
 * (up id, down id).  Then only mutual links are kept; a chain start has an
 * up link, no down link, and a chain of at least three hits. */
int tpc_find_neighbours(tpc_context* ctx, const tpc_problem* h_prob, tpc_grid grid,
                        tpc_links links, tpc_starts starts, void* d_ws, size_t ws_bytes,
                        void* stream);

/* Kalman-filter track following (section 3).  Per start: state from the
 * first and third chain hits, filter along the chain, then row by row
 * outwards taking the hit of least predicted chi2 <= chi2_max (ties by id),
 * stopping after max_miss empty rows; then inwards from the outermost hit
 * with a reset covariance through the hits found, searching below the
 * start.  `tracklets.capacity` must be >= the start capacity. */
int tpc_construct_tracklets(tpc_context* ctx, const tpc_problem* h_prob, tpc_grid grid,
                            tpc_links links, tpc_starts starts, tpc_tracklets tracklets,
                            void* d_ws, size_t ws_bytes, void* stream);

/* Tracklet selection: one hypothesis per cluster (section 3).  A cluster
 * belongs to the tracklet of largest key (hits << 32 | ~start id) among
 * tracklets with >= min_tracklet_hits hits containing it; a tracklet keeping
 * >= min_track_hits of its clusters becomes a track. */
int tpc_select_tracks(tpc_context* ctx, const tpc_problem* h_prob, tpc_grid grid,
                      tpc_tracklets tracklets, tpc_tracks tracks, void* d_ws,
                      size_t ws_bytes, void* stream);

/* Synchronous: copies the status block of d_ws to *h_out. */
int tpc_get_status(const void* d_ws, tpc_status* h_out, void* stream);

/* The four tracking calls in one go.  mode: 0 one launch per stage over
 * all sectors, 1 one launch sequence per sector, 2 one persistent launch
 * over a device work queue.  use_graph != 0 captures the launch sequence
 * into a HIP graph on the first call and replays it on later calls with
 * the same arguments. */
enum { TPC_MODE_STAGED = 0, TPC_MODE_PER_SECTOR = 1, TPC_MODE_PERSISTENT = 2 };
int tpc_track_batch(tpc_context* ctx, const tpc_problem* h_prob, tpc_clusters in,
                    tpc_grid grid, tpc_links links, tpc_starts starts,
                    tpc_tracklets tracklets, tpc_tracks tracks, void* d_ws,
                    size_t ws_bytes, int mode, int use_graph, void* stream);

/* ---- track-based cluster attachment -------------------------------------- */

/* Cluster attachment and rejection marks (section 6, data compression).  Every track of the
 * selection gets a tube of `radius` cm over the pad rows from its first to
 * its last hit; its axis is the state of the track's tracklet (par, at the
 * plane of row row_inner) transported outwards row by row as in tracklet
 * construction, stopping where |sin(phi)| would reach s_max.  A cluster of
 * the track's sector on such a row lies in the tube when
 * dy*dy + dz*dz <= radius*radius (float32, in that order).  Per cluster id:
 *   track[c]: the track that owns c, else the track of least |q/pT| (ties to
 *             the lower index) whose tube holds c, else -1;
 *   state[c]: 1 attached (owned) | 2 adjacent (in a tube, not owned) |
 *             4 protected (in the tube of, or owned by, a track with
 *             |q/pT| <= 1/pt_good in float32) | 8 removed (attached or
 *             adjacent and not protected).
 * in, grid, tracklets and tracks are those of the tracking calls on the
 * same problem; d_n_tracks (device) holds the track count (the status
 * block's n_tracks; tracks beyond tracks.capacity do not exist).  track
 * and state are device arrays of n_clusters entries, owned by the caller.
 * d_ws: tpc_attach_workspace_size bytes of device scratch.  Returns
 * TPC_ERR_INVALID_ARG for a null pointer, radius or pt_good not > 0, or a
 * short workspace; asynchronous on stream. */
int tpc_attach_workspace_size(const tpc_problem* h_prob, size_t* h_bytes);
int tpc_attach_clusters(tpc_context* ctx, const tpc_problem* h_prob, tpc_clusters in,
                        tpc_grid grid, tpc_tracklets tracklets, tpc_tracks tracks,
                        const int64_t* d_n_tracks, float radius, float pt_good,
                        int32_t* track, uint8_t* state, void* d_ws, size_t ws_bytes,
                        void* stream);

/* ---- sector-track merging ------------------------------------------------ */

/* Cuts of the merging.  Sectors form sides of sectors_per_side (>= 3)
 * sectors; sector s lies on side s / sectors_per_side at index
 * i = s % sectors_per_side, its frame turned by (i + 1/2) times the sector
 * width, whose cosine and sine (float32) are cos_width and sin_width.
 * inv_window: inverse window widths of y, z [1/cm], sin(phi), tan(lambda)
 * and q/pT (finite, >= 0). */
typedef struct tpc_merge_cuts {
    int32_t sectors_per_side;
    float cos_width, sin_width;
    float inv_window[5];
} tpc_merge_cuts;

/* Sector-track merging (section 2: the first fit of the sector tracks serves
 * to find the whole track; section 3: sector boundaries).  The sector of a
 * track is that of its first hit; the up neighbour of index i is
 * (i + 1) % sectors_per_side on the same side, the down neighbour
 * (i + sectors_per_side - 1) % sectors_per_side.  For track k and a track j
 * of a neighbour sector, j's state (its tracklet's par at the plane of
 * row_inner, x_j) is turned into the frame of k's sector by D (cos D =
 * cos_width, sin D = +sin_width when j lies in the up neighbour, -sin_width
 * in the down one):
 *   x' = x c - y sd, y' = x sd + y c, sin' = sin c + cos sd,
 *   cos' = cos c - sin sd (cos = sqrt((1 - sin)(1 + sin))),
 * valid when cos' > 0 and |sin'| < s_max, and transported to x_k as in
 * tracklet construction (no candidate where that stops).  With
 * r_i = (p'_i - p_k,i) * inv_window[i], d2 = ((((r0^2 + r1^2) + r2^2) +
 * r3^2) + r4^2) in float32; a candidate needs d2 < 1.  In each direction the
 * best partner has the least d2, ties to the lower index; k and j are linked
 * when each is the other's best partner.  Per track k (device arrays of
 * tracks.capacity entries, owned by the caller; entries from the track
 * count on are not written):
 *   link_up[k]: the linked track in the up neighbour, else -1;
 *   link_dn[k]: the linked track in the down neighbour, else -1;
 *   group[k]:   the least track index on k's chain of links.
 * tracklets and tracks are those of the tracking calls on the same problem,
 * in any track order; d_n_tracks (device) holds the track count, tracks
 * beyond tracks.capacity do not exist.  d_ws: tpc_merge_workspace_size
 * bytes of device scratch for tracks.capacity tracks.  Returns
 * TPC_ERR_INVALID_ARG for a null pointer, a capacity outside [0, 2^31), a
 * sector count that is not a multiple of sectors_per_side, sectors_per_side
 * < 3, a non-finite cut or a short workspace; asynchronous on stream. */
int tpc_merge_workspace_size(const tpc_problem* h_prob, int64_t track_capacity, size_t* h_bytes);
int tpc_merge_sector_tracks(tpc_context* ctx, const tpc_problem* h_prob,
                            tpc_tracklets tracklets, tpc_tracks tracks,
                            const int64_t* d_n_tracks, tpc_merge_cuts cuts, int32_t* link_up,
                            int32_t* link_dn, int32_t* group, void* d_ws, size_t ws_bytes,
                            void* stream);

/* ---- full-track fit of merged sector tracks ------------------------------ */

/* Per-track outputs of tpc_fit_merged_tracks (device arrays of
 * tracks.capacity entries each, owned by the caller). */
typedef struct tpc_fit_out {
    float* par_in;         /* [5 per track] state at the first hit after the last inward pass */
    float* par_out;        /* [5 per track] state at the last hit after the last outward pass */
    float* cov_out;        /* [15 per track] its covariance (lower triangle, row by row) */
    float* chi2;           /* chi2 sum of the last pass */
    int32_t* n_hits;       /* hits of the merged track */
    int32_t* n_members;    /* sector tracks in it */
    int32_t* status;       /* 0 fitted, 1 fewer than 3 hits, 2 a transport or turn
                              stopped, -1 not a group leader (no output) */
} tpc_fit_out;

/* Full-track fit of the merged sector tracks (section 2: the first fit of
 * the sector tracks serves to find the whole track, which is then fitted;
 * section 3: several fit iterations, in and out, across sector
 * boundaries).  Inputs: the clusters, tracklets and tracks of the tracking
 * calls and link_up, link_dn, group of tpc_merge_sector_tracks (same
 * problem, sectors_per_side, cos_width, sin_width).  For every track g with
 * group[g] == g (the chain's least index): the chain is walked from its down
 * end (following link_dn from g, at most n_sectors steps, stopping before
 * g) along link_up, or from its up end along link_dn when the up end's first
 * hit lies on a lower row than the down end's first hit; the merged hit list
 * is the members' hits in that order, each member's row-ascending.  The fit
 * starts from the first member's tracklet state (par at the plane of
 * row_inner) and makes n_pass passes over all hits, alternately outwards
 * (first to last) and inwards, each from the previous pass's parameters and
 * a diagonal covariance: the variances of the first member's tracklet (cov)
 * for the first pass, of the previous pass's end for the others, times
 * cov_scale (params' initial variances stand in for any that is not
 * positive and finite); between hits of neighbouring sectors the
 * state is turned into the next sector's frame (D = alpha_now - alpha_next:
 * sin D = -sin_width towards the up neighbour, +sin_width towards the down
 * one; the point (x, y) goes to (x c - y sd, x sd + y c), the covariance by
 * the first-order map of moving onto the new plane; refused when cos' <= 0
 * or |sin'| >= s_max) and transported to the hit's row plane, then updated
 * with the hit.  par_in is zero with one pass.  Tracks from the track count
 * on are not written.  Float32.  Returns TPC_ERR_INVALID_ARG for a null
 * pointer, a capacity outside [0, 2^31), n_pass outside [1, 64],
 * sectors_per_side < 3 or not dividing the sector count, a non-finite width
 * or cov_scale not finite and > 0; asynchronous on stream. */
int tpc_fit_merged_tracks(tpc_context* ctx, const tpc_problem* h_prob, tpc_clusters clusters,
                          tpc_tracklets tracklets, tpc_tracks tracks, const int64_t* d_n_tracks,
                          const int32_t* link_up, const int32_t* link_dn, const int32_t* group,
                          int32_t sectors_per_side, float cos_width, float sin_width,
                          int32_t n_pass, float cov_scale, tpc_fit_out out, void* stream);

/* ---- cluster compression ------------------------------------------------ */

typedef struct tpc_compress_params {
    int32_t qbits;         /* y, z quantum 2^-qbits cm (0..12) */
    int32_t cbits;         /* leading significant bits kept of the charge (2..8) */
    int32_t chunk;         /* symbols per rANS chunk (64..2^20) */
} tpc_compress_params;

/* Bytes of device workspace of tpc_compress_clusters. */
int tpc_compress_workspace_size(const tpc_problem* h_prob, int64_t track_capacity,
                                int64_t hit_capacity, int32_t chunk, size_t* h_bytes);

/* Compression of the clusters of a tracked problem (section 6, TPC data
 * compression, steps 2-4: integer format with the resolution's precision
 * and a charge precision relative to its value; residuals to tracks for the
 * clusters on tracks, position differences otherwise; an entropy coder,
 * rANS).  Integer format: y, z -> rint(v 2^qbits); charge -> its count
 * rint(charge) in [0, 65535] keeping cbits leading significant bits
 * (code = v below 2^cbits, else 2^cbits + (e - 1) 2^(cbits-1) + (v >> e) -
 * 2^(cbits-1), e = bitlength(v) - cbits).  Nine byte streams, 255 escaping a
 * 32-bit value on the stream's escape list:
 *   tracks in track order: hit count; per hit the row step (from the
 *   header's row), the zigzag y and z residuals to the prediction, the
 *   charge code.  The prediction: the tracklet state (par at row_inner)
 *   rounded into a 16-byte header (row_inner, 0, sin, tan at 2^-14 and q/pT
 *   at 2^-10 as int16, y and z as int32 at 2^-qbits), the initial covariance
 *   of params, the tracklet transport to each hit's row and the tracklet
 *   update with the hit as decoded;
 *   the other clusters, sector by sector and row by row in grid order: the
 *   count per row, the zigzag z step to the previous one of the row (from 0),
 *   y + 2048 as a high byte (escaped outside [0, 4096)) and a low byte, the
 *   charge code after the tracks' codes.
 * Each stream: 12-bit frequencies normalised from its counts (floor of the
 * share, at least 1, then +-1 steps on the largest frequency above 1 or the
 * largest count, ties to the lower symbol), rANS (state in [2^23, 2^31),
 * byte output) in chunks of `chunk` symbols.  Blob (little-endian): magic
 * "TPCZ", version 1, cbits, qbits, chunk, n_sectors, n_rows (u32); n_clusters,
 * n_tracks, clusters on tracks, others (u64); per stream n_symbols,
 * n_escapes (u64), n_chunks (u32), 256 u16 frequencies (0xffff for 4096),
 * the chunks' byte counts (u32); then every stream's chunk bytes, every
 * stream's escapes (i32), the track headers.  Inputs: the clusters (with
 * charge), grid, tracklets and tracks of the tracking calls (the tracks'
 * hit copies hit_row, hit_y, hit_z, when given, are read in place of the
 * clusters' values: all three or none); d_n_tracks (device) the track
 * count.  *d_size (device) receives the blob size; when
 * it exceeds out_cap nothing is written to out (the caller re-sizes).
 * d_ws: tpc_compress_workspace_size bytes.  Returns TPC_ERR_INVALID_ARG for a
 * null pointer (one or two of the hit copies included), parameters out of
 * range or a short workspace; asynchronous
 * on stream. */
int tpc_compress_clusters(tpc_context* ctx, const tpc_problem* h_prob, tpc_clusters clusters,
                          const float* charge, tpc_grid grid, tpc_tracklets tracklets,
                          tpc_tracks tracks, const int64_t* d_n_tracks, tpc_compress_params cp,
                          uint8_t* out, int64_t out_cap, int64_t* d_size, void* d_ws,
                          size_t ws_bytes, void* stream);

/* ---- per-track interaction time ----------------------------------------- */

/* Interaction time of every track in continuous read-out (section 2: the z
 * of a hit depends on the unknown time of its collision).  A primary comes
 * from the beam axis at z = 0; a collision at time t shifts the z the
 * tracker sees by -side * vd * t (side of the track's sector: that of its
 * first hit; +1 for a track without hits).  The state of the track's
 * tracklet (par at the plane of row_inner, x_in) is transported to the
 * plane x = 0 of its sector frame with the tracklet transport in
 * n = ceil(x_in / 20 cm) (at least 1) equal steps of dx = (0 - x_in) / n.  Per track k (device arrays of tracks.capacity entries,
 * owned by the caller; entries from the track count on are not written):
 *   y0[k], z0[k]: the state's y and z at x = 0 (y0 is 0 for a primary);
 *   t0[k]: (side > 0 ? -z0 : z0) / vd, float32 [time unit of vd];
 *   ok[k]: 1, or 0 (and zeros) where |sin(phi)| would reach s_max.
 * d_n_tracks (device) holds the track count.  Returns TPC_ERR_INVALID_ARG
 * for a null pointer, vd not finite and > 0 or a negative capacity;
 * asynchronous on stream. */
int tpc_track_t0(tpc_context* ctx, const tpc_problem* h_prob, tpc_tracklets tracklets,
                 tpc_tracks tracks, const int64_t* d_n_tracks, float vd, float* z0, float* y0,
                 float* t0, int8_t* ok, void* stream);

/* ---- calibrated refit ---------------------------------------------------- */

/* Calibration model.  For a cluster of a sector on z side `side` (+1/-1) on
 * row plane x_r with raw (y, z): drift d = (1 + th[0]) (d_raw - vd th[1])
 * with d_raw = drift_len - side z; z' = side (drift_len - d); with
 * u = (x_r - u_centre)/u_scale, v = y / (x_r tan_half), w = d/drift_len and
 * basis b = (1, u, v, u^2, uv, v^2, w): plane x' = x_r + sum th[2+j] b_j,
 * y' = y + sum th[9+j] b_j. */
typedef struct tpc_calib_model {
    float drift_len, vd, tan_half, u_centre, u_scale;
} tpc_calib_model;

/* Found tracks' hits, CSR: the hits of track k are the entries
 * off[k]..off[k+1] (rows increasing).  Entry j is cluster idx[j] of the
 * arrays row/y/z, or cluster j when idx is NULL (so the output of
 * tpc_select_tracks refits directly).  side[k] = +1/-1 (NULL: all +1).
 * The number of tracks is n_tracks, or min(*d_count, n_tracks) when the
 * device pointer d_count is given (e.g. the status block's n_tracks), which
 * keeps the call free of host synchronisation.  Per-hit outputs are indexed
 * by entry j, n_hits entries. */
typedef struct tpc_track_hits {
    const int32_t* off;
    const int32_t* idx;
    const uint8_t* row;
    const float* y;
    const float* z;
    const int8_t* side;
    const int64_t* d_count;
    int64_t n_tracks;
    int64_t n_hits;
} tpc_track_hits;

/* Forward refit in float: calibrate with d_theta[16], state from hits 0
 * and 2, filter outwards through hits 1..n-1.  Outputs per track: par[5],
 * cov[15] at the last hit, chi2, status (0 ok, 1 fewer than 3 hits, 2
 * |sin(phi)| stop, 3 a hit row >= n_rows, 4 more hits than rows).  The CSR
 * must be well formed (off increasing, off[n_tracks] = n_hits).
 * checkpoints (nullable, ck_bytes long, at least tpc_refit_checkpoint_size
 * of the n_tracks member): the state and covariance after every update but
 * the last, for tpc_refit_adjoint, in a layout private to the library (tiles
 * of 64 tracks, 20 floats per hit slot; with a checkpoint buffer the tracks
 * are taken in order of decreasing hit count, equal counts in track order,
 * and that order is kept in the buffer too).  A shorter buffer is an
 * argument error, as are n_hits or n_tracks of 2^31 or more.  Outputs do not
 * depend on the order; the adjoint's theta reduction follows it. */
int tpc_refit(tpc_context* ctx, tpc_track_hits hits, int32_t n_rows, const float* d_row_x,
              const tpc_params* h_params, const tpc_calib_model* h_model,
              const float* d_theta, float* par, float* cov, float* chi2, int32_t* status,
              float* checkpoints, size_t ck_bytes, void* stream);

/* Bytes of the checkpoint buffer of tpc_refit / tpc_refit_adjoint for
 * n_tracks tracks (capacity) of at most n_rows hits. */
int tpc_refit_checkpoint_size(int64_t n_tracks, int32_t n_rows, size_t* h_bytes);

/* Bytes of workspace for tpc_refit_adjoint. */
int tpc_refit_workspace_size(int64_t n_tracks, size_t* h_bytes);

/* Adjoint of the refit: with L = sum_k grad_chi2[k] * chi2[k], writes
 * dL/dy and dL/dz of every raw hit (grad_y, grad_z [n_hits]) and
 * dL/dtheta (grad_theta[16], a deterministic reduction).  Needs the
 * checkpoints and status of tpc_refit with the same inputs; tracks with
 * status != 0 contribute zero. */
int tpc_refit_adjoint(tpc_context* ctx, tpc_track_hits hits, int32_t n_rows,
                      const float* d_row_x, const tpc_params* h_params,
                      const tpc_calib_model* h_model, const float* d_theta,
                      const float* checkpoints, size_t ck_bytes, const int32_t* status,
                      const float* grad_chi2, float* grad_y, float* grad_z,
                      float* grad_theta, void* d_ws, size_t ws_bytes, void* stream);

/* tpc_refit_adjoint for an objective that also depends on each track's
 * final state: L = sum_k grad_chi2[k] chi2[k] + sum_k grad_par[k] . par[k]
 * + sum_k grad_x[k] x[k], where par[k] is the refit state after the last
 * update and x[k] the calibrated plane of the track's last hit (the seeds
 * are the derivatives of the caller's terms, e.g. from
 * tpc_vertex_residual).  grad_par [5 per track] and grad_x [per track] are
 * device arrays, each nullable (zero).  Otherwise as tpc_refit_adjoint. */
int tpc_refit_adjoint_seeded(tpc_context* ctx, tpc_track_hits hits, int32_t n_rows,
                             const float* d_row_x, const tpc_params* h_params,
                             const tpc_calib_model* h_model, const float* d_theta,
                             const float* checkpoints, size_t ck_bytes, const int32_t* status,
                             const float* grad_chi2, const float* grad_par, const float* grad_x,
                             float* grad_y, float* grad_z, float* grad_theta, void* d_ws,
                             size_t ws_bytes, void* stream);

/* Beam-axis term of the calibration objective (section 3: online
 * calibration of drift velocity, t0 and distortions; section 2: primaries
 * from the origin).  For every track k with status[k] == 0 (of tpc_refit
 * with the same inputs) and at least 3 hits: x = the calibrated plane of its
 * last hit; its refit state and covariance (par[k], cov[k] at x) are
 * transported to the beam-axis plane x = 0 of its sector frame with the
 * tracklet transport in n = ceil(x / 20 cm) (at least 1) equal steps; with
 * r = (y0, z0) there and W = (w00, w01, w11) either w_in[k] (held by the
 * caller) or, when w_in is NULL, the inverse of the transported (y, z)
 * covariance plus sigma_v^2 on its diagonal (the chi2 increment of a vertex
 * measurement; written to w_out[k] when w_out is not NULL):
 *   loss[k] = r^T W r,
 *   grad_par[5 k .. 5 k + 4] = d loss / d par[k] (W held; product of the
 *     steps' transport Jacobians),
 *   grad_x[k] = d loss / d x = -2 ((W r)_0 s0 + (W r)_1 t) / c0 (moving the
 *     plane with the state held translates the track along x; s0, c0 sin
 *     and cos of phi at x = 0, t = tan(lambda)),
 *   ok[k] = 1 (nullable); all zero where the fit or the transport stopped.
 * Device arrays of hits.n_tracks entries (5 per track for grad_par, 3 for
 * the weights); the track count is read from hits.d_count when given.
 * Returns TPC_ERR_INVALID_ARG for a null pointer or sigma_v not finite and
 * >= 0; asynchronous on stream. */
int tpc_vertex_residual(tpc_context* ctx, tpc_track_hits hits, int32_t n_rows,
                        const float* d_row_x, const tpc_params* h_params,
                        const tpc_calib_model* h_model, const float* d_theta, const float* par,
                        const float* cov, const int32_t* status, float sigma_v,
                        const float* w_in, float* w_out, float* loss, float* grad_par,
                        float* grad_x, int8_t* ok, void* stream);

/* tpc_refit_adjoint for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the per-block partial sums
 * of the theta gradient in a static device array of the library (16384
 * blocks x 16 float64 = 2 MiB per GPU, held until the process ends) instead
 * of a workspace.
 * The adjoint never uses more than 16384 blocks, so every n_tracks fits;
 * TPC_ERR_CAPACITY would report one that did not.  The context's device must
 * be current (else TPC_ERR_INVALID_ARG).  Allocates nothing and calls no
 * allocating routine.  All calls on one GPU share that array: calls that
 * overlap in time on one GPU (two streams, two threads) race on it and
 * must be serialised by the caller.  Otherwise as tpc_refit_adjoint. */
int tpc_refit_adjoint_noalloc(tpc_context* ctx, tpc_track_hits hits, int32_t n_rows,
                              const float* d_row_x, const tpc_params* h_params,
                              const tpc_calib_model* h_model, const float* d_theta,
                              const float* checkpoints, size_t ck_bytes,
                              const int32_t* status, const float* grad_chi2, float* grad_y,
                              float* grad_z, float* grad_theta, void* stream);

/* Per-kernel timing.  While enabled, every kernel the context launches
 * (outside graph capture) is bracketed by two HIP events on its stream.
 * tpc_timing_report synchronises on them and returns, per kernel name in
 * first-launch order, the launch count and the summed duration in ms;
 * names are static strings of the library.  *h_count receives the number of
 * distinct kernels (only the first max_kernels are written); the records
 * are then cleared.  Enabling clears them too. */
int tpc_timing_enable(tpc_context* ctx, int enable);
int tpc_timing_report(tpc_context* ctx, int max_kernels, const char** h_names,
                      int64_t* h_launches, double* h_total_ms, int* h_count);

/* Static description of an error code. */
const char* tpc_status_string(int code);

#ifdef __cplusplus
}
#endif
#endif
