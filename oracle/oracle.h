/*
 * Oracle for the TPC track-finding hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded C implementation of what the GPU library
 * computes, used by the tests, the smoke check and the CPU-baseline leg of
 * the benchmark.  The product path never links or calls it.  It shares no
 * code, header, table or constant with the HIP library: all geometry and
 * cut values arrive as arguments.
 *
 * The paper (section 3) fixes only the method's shape: cellular-automaton
 * seeding followed by single-hypothesis Kalman-filter track following with
 * a linear-time tail.  Every concrete rule below (bins, windows, cuts, the
 * propagator, the tracklet and selection rules, the calibration model) is
 * this project's reading of that statement, written out step by step.
 *
 * Floating point: built with -ffp-contract=off; every decision is taken in
 * IEEE binary32 with the association order written in the source and fused
 * multiply-adds only where the source calls them (fmaf), so that an
 * implementation evaluating the same expressions in the same order
 * reproduces them bit for bit.
 *
 * Index spaces: cluster ids are indices into the caller's input arrays.
 * Links and tracks are returned in id space; the grid is returned as the
 * permutation (bin_start, yg, zg, idg).
 */
#ifndef TPC_ORACLE_H
#define TPC_ORACLE_H
#include <stdint.h>

typedef struct {
    float curv;            /* curvature [1/cm] per unit q/pT */
    float nb_win_y;        /* neighbour window half widths [cm] */
    float nb_win_z;
    float nb_d2max;        /* max straight-line deviation^2 [cm^2] */
    float sigma_y2;        /* measurement variances [cm^2] */
    float sigma_z2;
    float chi2_max;        /* hit-search gate */
    float search_nsigma;   /* search bin window (acceleration only) */
    float s_max;           /* |sin(phi)| stop */
    float c_ss0, c_tt0, c_ww0;  /* initial variances */
    int max_miss;          /* consecutive rows without a hit that stop a search */
    int min_tracklet_hits; /* tracklets shorter than this take no part in selection */
    int min_track_hits;    /* tracks keeping fewer hits are dropped */
} orc_params;

typedef struct {
    float y0, z0;          /* lower edge of the bin grid */
    float inv_by, inv_bz;  /* inverse bin widths */
    int nby, nbz;          /* bins per row in y and z */
    int bin_base;          /* index of the sector's first bin */
    int side;              /* z side, not used by the oracle's tracking */
    int64_t begin, end;    /* the sector's clusters: ids [begin, end) */
} orc_sector;

typedef struct {           /* calibration model of the refit */
    float drift_len;       /* cm */
    float vd;              /* cm/us */
    float tan_half;        /* tan of the sector half opening angle */
    float u_centre, u_scale;  /* radial coordinate u = (x - centre)/scale */
} orc_calib_model;

/* Grid (stable counting sort of each sector's clusters by pad row and
 * (z, y) bin).  Each sector has n_rows * nbz * nby bins for its rows and one
 * last bin for clusters with row >= n_rows.  Returns the number of
 * clusters placed (all). */
int orc_build_grid(int n_sec, const orc_sector* sec, int n_rows,
                   const uint8_t* row, const float* y, const float* z,
                   int n_bins, int* bin_start, float* yg, float* zg, int* idg);

/* Best up/down neighbour pair per cluster (id space, -1 if none). */
void orc_find_neighbours(int n_sec, const orc_sector* sec, int n_rows,
                         const float* row_x, const orc_params* prm,
                         const int* bin_start, const float* yg, const float* zg,
                         const int* idg, int64_t n_clusters,
                         int* up0, int* down0);

/* Mutual-link filter. */
void orc_clean_links(int64_t n, const int* up0, const int* down0, int* up, int* down);

/* Chain starts in ascending id; returns the count. */
int64_t orc_select_starts(int64_t n, const int* up, const int* down, int* starts);

/* Tracklet construction.  hits: [n_starts][n_rows] cluster ids (-1 none).
 * brute != 0 scans whole rows instead of grid bins (same result). */
void orc_construct_tracklets(int n_sec, const orc_sector* sec, int n_rows,
                             const float* row_x, const orc_params* prm,
                             const int* bin_start, const float* yg, const float* zg,
                             const int* idg,
                             const uint8_t* row, const float* y, const float* z,
                             const int* up, int64_t n_starts, const int* starts,
                             int brute, int* hits, int* nhits, int* row_inner,
                             float* par, float* cov, float* chi2);

/* Work of the last orc_construct_tracklets call: transports attempted,
 * Kalman updates, predicted-chi2 evaluations. */
void orc_tracklet_work(int64_t* out3);

/* FP64 replay of a tracklet's fit with its hit list fixed. */
int orc_tracklet_replay64(int n_rows, const float* row_x, const orc_params* prm,
                          const float* y, const float* z, int start_row,
                          const int* hits_by_row, double* par, double* cov,
                          double* chi2);

/* Selection; returns the number of tracks.  trk_off has n_tracklets+1
 * entries of room, trk_hits n_clusters. */
int64_t orc_select_tracks(int64_t n_clusters, int n_rows, const orc_params* prm,
                          int64_t n_tracklets, const int* hits, const int* nhits,
                          const int* starts, int* trk_off, int* trk_hits,
                          int* trk_tracklet);

/* Calibrated refit (forward).  side: +1/-1 per track or NULL (all +1).
 * status per track: 0 ok, 1 too few hits, 2 propagation stop. */
void orc_refit32(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                 const float* y, const float* z, const signed char* side,
                 const float* row_x, const orc_params* prm,
                 const orc_calib_model* cm, const float* theta,
                 float* par, float* cov, float* chi2, int* status);
void orc_refit64(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                 const double* y, const double* z, const signed char* side,
                 const float* row_x, const orc_params* prm,
                 const orc_calib_model* cm, const double* theta,
                 double* par, double* cov, double* chi2, int* status);

/* Central finite-difference gradient of L = sum_t g_t chi2_t (FP64):
 * w.r.t. the raw (y, z) of every hit of the listed tracks and w.r.t. the
 * 16 calibration parameters.  Steps: h_hit (absolute, cm) for hit
 * coordinates, h_theta * max(|theta_k|, 1) for the parameters. */
void orc_refit64_fd_grad(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                         const double* y, const double* z, const signed char* side,
                         const float* row_x, const orc_params* prm,
                         const orc_calib_model* cm, const double* theta,
                         const double* g, double h_hit, double h_theta,
                         double* grad_y, double* grad_z, double* grad_theta);

/* Gradient of sum_t g_t chi2_t of the double refit, by reverse-mode
 * differentiation of the same forward code on a recorded tape (adjoint.cc):
 * grad_y, grad_z per hit, grad_theta summed over tracks. */
void orc_refit64_adjoint(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                         const double* y, const double* z, const signed char* side,
                         const float* row_x, const orc_params* prm,
                         const orc_calib_model* cm, const double* theta, const double* g,
                         double* grad_y, double* grad_z, double* grad_theta);

/* Calibration objective (adjoint.cc): L = sum_t g_t (chi2_t + r_t^T W_t r_t),
 * r_t the refit state of the last hit transported to the beam-axis plane
 * x = 0 (20 cm steps), W_t given per track (w00, w01, w11; NULL: no vertex
 * term); returns L, writes dL/dtheta (nullable), the per-track terms and
 * whether the vertex term was taken (nullable). */
double orc_calib_objective64(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                             const double* y, const double* z, const signed char* side,
                             const float* row_x, const orc_params* prm,
                             const orc_calib_model* cm, const double* theta, const double* g,
                             const double* w, double* grad_theta, double* per_track,
                             int* vertex_ok);
/* Weights of the beam-axis term at theta (oracle.c). */
void orc_vertex_weights64(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                          const double* y, const double* z, const signed char* side,
                          const float* row_x, const orc_params* prm,
                          const orc_calib_model* cm, const double* theta, double sigma_v2,
                          double* w, int* ok);

/* ---- cluster compression (section 6, steps 2-4; compress.c) ------------
 * Integer format: y, z rounded to 2^-qbits cm; charge rounded to a count in
 * [0, 65535] keeping its leading cbits significant bits.  Clusters on tracks
 * (track by track, row-ascending): the number of hits, the row step, the
 * residuals of y and z to the track's prediction (its tracklet state rounded
 * into a 16-byte header and carried row by row with the tracker's float32
 * transport, updated with each decoded cluster), the charge.  The other
 * clusters sector by sector and row by row in grid order: their count per
 * row, the z step to the previous one of the row, y (offset 2048) as two
 * bytes, the charge.  Byte symbols, 255 escapes a 32-bit value; each stream
 * is rANS coded in chunks of `chunk` symbols with its own 12-bit table.
 * orc_compress returns the blob size (negative: the size needed when it
 * exceeds out_cap); orc_decompress the clusters in blob order. */
typedef struct {
    int32_t qbits;         /* position quantum 2^-qbits cm */
    int32_t cbits;         /* significant bits kept of the charge */
    int32_t chunk;         /* symbols per rANS chunk */
} orc_cmp_params;

int64_t orc_compress(int n_sec, const orc_sector* sec, int n_rows, const float* row_x,
                     const orc_params* prm, const uint8_t* row, const float* y, const float* z,
                     const float* charge, int64_t n_clusters, const int* bin_start,
                     const int* idg, int64_t n_tracks, const int* trk_off, const int* trk_hits,
                     const float* tpar, const int* trin, const orc_cmp_params* cp,
                     uint8_t* out, int64_t out_cap);
int64_t orc_decompress(const uint8_t* blob, int64_t size, const float* row_x,
                       const orc_params* prm, uint8_t* o_row, int32_t* o_yq, int32_t* o_zq,
                       int32_t* o_qcode, int32_t* o_track, int32_t* o_sector, int64_t cap);
int orc_charge_decode(int code, int cbits);
int64_t orc_rans_roundtrip(const uint8_t* sym, int64_t n, uint8_t* bytes, uint8_t* back);

/* Track-based cluster attachment (section 6): tube of `radius` around
 * every track over the rows of its hits, its axis the track state par[5k]
 * (at the plane of row rin[k]) transported outwards row by row; unowned
 * clusters in a tube are adjacent to the track of least |q/pT| (ties to the
 * lower index).  track[c]: owning or adjacent track, else -1; state[c]: 1
 * attached, 2 adjacent, |4 protected (tube or track of |q/pT| <= w_good),
 * |8 removed (attached or adjacent, not protected). */
void orc_attach_clusters(int n_sec, const int64_t* sector_offsets, int n_rows,
                         const float* row_x, const orc_params* prm, const uint8_t* row,
                         const float* y, const float* z, int64_t n_clusters, int64_t n_tracks,
                         const int* trk_off, const int* trk_hits, const float* par,
                         const int* rin, float radius, float w_good, int* track,
                         uint8_t* state);

/* Sector-track merging (sections 2 and 3): tracks in neighbouring sectors
 * of one side (n_sec = sides * sps, sps >= 3) are linked when each is the
 * other's best partner: track j's state (par[5j] at row rin[j]) rotated
 * into the frame of k's sector (cos_w, sin_w: the sector width) and
 * transported to k's plane must lie within d2 = sum ((p'_i - p_k,i) iw_i)^2
 * < 1, least d2 (ties to the lower index) in each direction.  link_up[k]:
 * the linked track in the next sector of the side (index + 1 mod sps),
 * link_dn[k]: in the previous one, -1 none; group[k]: least index on k's
 * chain of links. */
/* Full-track fit of the merged sector tracks (float64; see oracle.c): per
 * track index, defined for group leaders (group[k] == k). */
void orc_fit_merged64(int n_sec, const int64_t* sector_offsets, int sps, const float* row_x,
                      const orc_params* prm, const uint8_t* row, const float* y, const float* z,
                      int64_t n_tracks, const int* trk_off, const int* trk_hits,
                      const float* par, const float* cov, const int* rin,
                      const int* link_up, const int* link_dn, const int* group, float cos_w,
                      float sin_w, int n_pass, float cov_scale, double* par_in,
                      double* par_out, double* cov_out, double* chi2_out, int* n_hits,
                      int* n_members, int* status);
void orc_fit_merged32(int n_sec, const int64_t* sector_offsets, int sps, const float* row_x,
                      const orc_params* prm, const uint8_t* row, const float* y, const float* z,
                      int64_t n_tracks, const int* trk_off, const int* trk_hits,
                      const float* par, const float* cov, const int* rin,
                      const int* link_up, const int* link_dn, const int* group, float cos_w,
                      float sin_w, int n_pass, float cov_scale, float* par_in,
                      float* par_out, float* cov_out, float* chi2_out, int* n_hits,
                      int* n_members, int* status);
int orc_rotate64(double* x, double* p, double* C, double c, double sd, double curv,
                 double s_max);

void orc_merge_sector_tracks(int n_sec, const int64_t* sector_offsets, int sps,
                             const float* row_x, const orc_params* prm, int64_t n_tracks,
                             const int* trk_off, const int* trk_hits, const float* par,
                             const int* rin, float cos_w, float sin_w, const float* iw,
                             int* link_up, int* link_dn, int* group);
/* One state into a frame rotated by D (c = cos D, sd = sin D) and
 * transported to the plane x_to; 0 where the rotated state is invalid or the
 * transport stops. */
int orc_merge_transform(const float* pj, float xj, float c, float sd, float x_to, float curv,
                        float s_max, float* out5);

/* Interaction time of every track (section 2, continuous read-out): the
 * state (par[5k] at x_in[k]) transported to the plane x = 0 of its sector
 * frame; y0, z0 there and t0 = (side > 0 ? -z0 : z0) / vd; ok 0 (zeros)
 * where the transport stops. */
void orc_track_t0(int64_t n_tracks, const float* par, const float* x_in,
                  const signed char* side, float curv, float s_max, float vd, float* z0,
                  float* y0, float* t0, signed char* ok);

/* Single steps, exposed for the tests. */
int orc_propagate32(float* p, float* C, float dx, float curv, float s_max);
int orc_propagate64(double* p, double* C, double dx, double curv, double s_max);
float orc_update32(float* p, float* C, float my, float mz, float sy2, float sz2);
double orc_update64(double* p, double* C, double my, double mz, double sy2, double sz2);
float orc_chi2_pred32(const float* p, const float* C, float my, float mz, float sy2, float sz2);
void orc_calibrate64(const double* th, double xr, double yr, double zr, double side,
                     const orc_calib_model* cm, double* out3);

#endif
