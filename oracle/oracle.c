/*
 * Oracle of the TPC track-finding hot path -- TEST INFRASTRUCTURE ONLY.
 * Plain single-threaded C; see oracle.h for the conventions.  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg use it.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- Kalman primitives in float and double ----------------------------- */
#define REAL float
#define SUF _f
#define SQRT sqrtf
#define FABS fabsf
#define FMA fmaf
#define C_1_6 (1.0f / 6.0f)
#define C_3_40 (3.0f / 40.0f)
#define C_5_112 (5.0f / 112.0f)
#define C_3_8 (3.0f / 8.0f)
#define C_5_16 (5.0f / 16.0f)
#define C_3_20 (3.0f / 20.0f)
#define C_15_112 (15.0f / 112.0f)
#include "kalman_impl.h"
#undef REAL
#undef SUF
#undef SQRT
#undef FABS
#undef FMA
#undef C_1_6
#undef C_3_40
#undef C_5_112
#undef C_3_8
#undef C_5_16
#undef C_3_20
#undef C_15_112

#define REAL double
#define SUF _d
#define SQRT sqrt
#define FABS fabs
#define FMA fma
#define C_1_6 (1.0 / 6.0)
#define C_3_40 (3.0 / 40.0)
#define C_5_112 (5.0 / 112.0)
#define C_3_8 (3.0 / 8.0)
#define C_5_16 (5.0 / 16.0)
#define C_3_20 (3.0 / 20.0)
#define C_15_112 (15.0 / 112.0)
#include "kalman_impl.h"
#undef REAL
#undef SUF
#undef SQRT
#undef FABS
#undef FMA

/* ---- grid ----------------------------------------------------------------
 * Bin of a coordinate: f = (v - v0) * inv, clamped to [0, nb - 1] in float,
 * then truncated.  The map is monotone in v, so a window [lo, hi] is
 * covered by the bins bin(lo)..bin(hi). */
static int bin_of(float v, float v0, float inv, int nb)
{
    float f = (v - v0) * inv;
    if (!(f >= 0.0f)) f = 0.0f;
    float top = (float)(nb - 1);
    if (f > top) f = top;
    return (int)f;
}

/* Clusters with row >= n_rows go to the sector's last bin, after its rows. */
static int global_bin(const orc_sector* s, int n_rows, int row, float y, float z)
{
    if (row >= n_rows) return s->bin_base + n_rows * s->nbz * s->nby;
    int iy = bin_of(y, s->y0, s->inv_by, s->nby);
    int iz = bin_of(z, s->z0, s->inv_bz, s->nbz);
    return s->bin_base + (row * s->nbz + iz) * s->nby + iy;
}

int orc_build_grid(int n_sec, const orc_sector* sec, int n_rows,
                   const uint8_t* row, const float* y, const float* z,
                   int n_bins, int* bin_start, float* yg, float* zg, int* idg)
{
    int* count = calloc((size_t)n_bins + 1, sizeof(int));
    int* fill = malloc(((size_t)n_bins + 1) * sizeof(int));
    if (!count || !fill) {
        free(count);
        free(fill);
        return -1;
    }
    /* counting sort: histogram, exclusive prefix sum, stable placement in
     * ascending id order */
    for (int s = 0; s < n_sec; s++)
        for (int64_t i = sec[s].begin; i < sec[s].end; i++)
            count[global_bin(&sec[s], n_rows, row[i], y[i], z[i])]++;
    int acc = 0;
    for (int g = 0; g < n_bins; g++) {
        bin_start[g] = acc;
        fill[g] = acc;
        acc += count[g];
    }
    bin_start[n_bins] = acc;
    for (int s = 0; s < n_sec; s++)
        for (int64_t i = sec[s].begin; i < sec[s].end; i++) {
            int pos = fill[global_bin(&sec[s], n_rows, row[i], y[i], z[i])]++;
            yg[pos] = y[i];
            zg[pos] = z[i];
            idg[pos] = (int)i;
        }
    free(count);
    free(fill);
    return acc;
}

/* Positions of the grid bins of sector s, row r, covering [ylo, yhi] x
 * [zlo, zhi] are visited z-bin by z-bin. */
typedef struct {
    const orc_sector* s;
    const int* bin_start;
    int r, iy0, iy1, iz0, iz1;
} bin_window;

static bin_window make_window(const orc_sector* s, const int* bin_start, int r,
                              float ylo, float yhi, float zlo, float zhi)
{
    bin_window w;
    w.s = s;
    w.bin_start = bin_start;
    w.r = r;
    w.iy0 = bin_of(ylo, s->y0, s->inv_by, s->nby);
    w.iy1 = bin_of(yhi, s->y0, s->inv_by, s->nby);
    w.iz0 = bin_of(zlo, s->z0, s->inv_bz, s->nbz);
    w.iz1 = bin_of(zhi, s->z0, s->inv_bz, s->nbz);
    return w;
}

/* the window is widened by this factor before taking bins so that a
 * rounding difference at the window edge can never drop a candidate; the
 * exact predicate decides */
#define WIDEN (1.0f + 1.0f / 64.0f)

static int sector_of(int n_sec, const orc_sector* sec, int64_t id)
{
    int lo = 0, hi = n_sec - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (sec[mid].begin <= id) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* ---- neighbour finding ---------------------------------------------------
 * For a cluster h on row r (0 < r < n_rows - 1) at (y, z): candidates on
 * row r+1 lie within |y_u - y x_{r+1}/x_r| <= Wy, |z_u - z| <= Wz (the
 * straight line from the origin through h, in y only: the transverse
 * vertex is known, the z vertex is not); candidates on row r-1 likewise
 * around y x_{r-1}/x_r.  Among all pairs (u, d) with straight-line
 * deviation D2 = ((y_u + y_d) - (y + y))^2 + ((z_u + z_d) - (z + z))^2
 * <= D2max the lexicographic minimum of (D2, id_u, id_d) is chosen. */
void orc_find_neighbours(int n_sec, const orc_sector* sec, int n_rows,
                         const float* row_x, const orc_params* prm,
                         const int* bin_start, const float* yg, const float* zg,
                         const int* idg, int64_t n_clusters, int* up0, int* down0)
{
    for (int64_t i = 0; i < n_clusters; i++) {
        up0[i] = -1;
        down0[i] = -1;
    }
    const float Wy = prm->nb_win_y, Wz = prm->nb_win_z, D2max = prm->nb_d2max;
    for (int si = 0; si < n_sec; si++) {
        const orc_sector* s = &sec[si];
        int per_row = s->nby * s->nbz;
        for (int r = 1; r + 1 < n_rows; r++) {
            int p0 = bin_start[s->bin_base + r * per_row];
            int p1 = bin_start[s->bin_base + (r + 1) * per_row];
            for (int ph = p0; ph < p1; ph++) {
                float y = yg[ph], z = zg[ph];
                float slope = y / row_x[r];
                float yu_c = slope * row_x[r + 1];
                float yd_c = slope * row_x[r - 1];
                bin_window wu = make_window(s, bin_start, r + 1, yu_c - Wy * WIDEN,
                                            yu_c + Wy * WIDEN, z - Wz * WIDEN, z + Wz * WIDEN);
                bin_window wd = make_window(s, bin_start, r - 1, yd_c - Wy * WIDEN,
                                            yd_c + Wy * WIDEN, z - Wz * WIDEN, z + Wz * WIDEN);
                float best = 0.0f;
                int bu = -1, bd = -1;
                for (int izu = wu.iz0; izu <= wu.iz1; izu++) {
                    int gu = s->bin_base + ((r + 1) * s->nbz + izu) * s->nby;
                    for (int pu = bin_start[gu + wu.iy0]; pu < bin_start[gu + wu.iy1 + 1]; pu++) {
                        float yu = yg[pu], zu = zg[pu];
                        if (!(fabsf(yu - yu_c) <= Wy && fabsf(zu - z) <= Wz)) continue;
                        int idu = idg[pu];
                        for (int izd = wd.iz0; izd <= wd.iz1; izd++) {
                            int gd = s->bin_base + ((r - 1) * s->nbz + izd) * s->nby;
                            for (int pd = bin_start[gd + wd.iy0]; pd < bin_start[gd + wd.iy1 + 1]; pd++) {
                                float yd = yg[pd], zd = zg[pd];
                                if (!(fabsf(yd - yd_c) <= Wy && fabsf(zd - z) <= Wz)) continue;
                                float dy = (yu + yd) - (y + y);
                                float dz = (zu + zd) - (z + z);
                                float d2 = dy * dy + dz * dz;
                                if (!(d2 <= D2max)) continue;
                                int idd = idg[pd];
                                if (bu < 0 || d2 < best ||
                                    (d2 == best && (idu < bu || (idu == bu && idd < bd)))) {
                                    best = d2;
                                    bu = idu;
                                    bd = idd;
                                }
                            }
                        }
                    }
                }
                up0[idg[ph]] = bu;
                down0[idg[ph]] = bd;
            }
        }
    }
}

/* ---- link cleaning and chain starts --------------------------------------
 * A link survives only if it is mutual.  A chain start has an up link, no
 * down link, and its up neighbour has an up link (chain of >= 3 hits). */
void orc_clean_links(int64_t n, const int* up0, const int* down0, int* up, int* down)
{
    for (int64_t h = 0; h < n; h++) {
        int u = up0[h], d = down0[h];
        up[h] = (u >= 0 && down0[u] == h) ? u : -1;
        down[h] = (d >= 0 && up0[d] == h) ? d : -1;
    }
}

int64_t orc_select_starts(int64_t n, const int* up, const int* down, int* starts)
{
    int64_t m = 0;
    for (int64_t h = 0; h < n; h++)
        if (up[h] >= 0 && down[h] < 0 && up[up[h]] >= 0) starts[m++] = (int)h;
    return m;
}

/* ---- tracklet construction -----------------------------------------------
 * Per chain start h0 (row r0) with chain hits h1 = up[h0], h2 = up[h1]:
 *  init   position of h0, direction from h0 to h2, q/pT = 0, diagonal C;
 *  up     filter through the rest of the chain (unconditionally), then row
 *         by row outwards: propagate one row, take the hit of minimal
 *         predicted chi2 (<= chi2_max; ties to the lower id) and update,
 *         else count a miss; stop after max_miss consecutive misses, at the
 *         last row or when |sin(phi)| reaches s_max;
 *  down   restart from the state after the last update with the position
 *         of the last hit and the initial diagonal covariance; step row by
 *         row inwards, updating with the hits found on the way up (rows >=
 *         r0) and searching as above below r0.  A propagation stop ends the
 *         pass and drops the hits below it.
 * Output: hits of the down pass by row, the state after its last update,
 * and the sum of its update chi2. */
typedef struct {
    const orc_sector* s;
    const int* bin_start;
    const float *yg, *zg;
    const int* idg;
    int n_rows;
    const orc_params* prm;
    int brute;
} search_ctx;

/* work counters of the last orc_construct_tracklets call: transports
 * attempted, Kalman updates, predicted-chi2 evaluations */
static int64_t g_work[3];

void orc_tracklet_work(int64_t* out3)
{
    for (int i = 0; i < 3; i++) out3[i] = g_work[i];
}

static int prop_counted(float* p, float* C, float dx, float curv, float s_max)
{
    g_work[0]++;
    return propagate_f(p, C, dx, curv, s_max);
}

static float update_counted(float* p, float* C, float my, float mz, float sy2, float sz2)
{
    g_work[1]++;
    return update_f(p, C, my, mz, sy2, sz2);
}

static int search_row(const search_ctx* cx, int r, const float* p, const float* C)
{
    const orc_params* prm = cx->prm;
    const orc_sector* s = cx->s;
    int per_row = s->nby * s->nbz;
    float S00 = C[0] + prm->sigma_y2, S11 = C[2] + prm->sigma_z2;
    float hy = prm->search_nsigma * sqrtf(S00) * WIDEN + 0.01f;
    float hz = prm->search_nsigma * sqrtf(S11) * WIDEN + 0.01f;
    int iz0, iz1, iy0, iy1;
    if (cx->brute) {
        iz0 = 0; iz1 = s->nbz - 1; iy0 = 0; iy1 = s->nby - 1;
    } else {
        bin_window w = make_window(s, cx->bin_start, r, p[0] - hy, p[0] + hy, p[1] - hz, p[1] + hz);
        iz0 = w.iz0; iz1 = w.iz1; iy0 = w.iy0; iy1 = w.iy1;
    }
    (void)per_row;
    float best = 0.0f;
    int bid = -1;
    for (int iz = iz0; iz <= iz1; iz++) {
        int g = s->bin_base + (r * s->nbz + iz) * s->nby;
        for (int pc = cx->bin_start[g + iy0]; pc < cx->bin_start[g + iy1 + 1]; pc++) {
            g_work[2]++;
            float c2 = chi2_pred_f(p, C, cx->yg[pc], cx->zg[pc], prm->sigma_y2, prm->sigma_z2);
            if (!(c2 <= prm->chi2_max)) continue;
            int id = cx->idg[pc];
            if (bid < 0 || c2 < best || (c2 == best && id < bid)) {
                best = c2;
                bid = id;
            }
        }
    }
    return bid;
}

void orc_construct_tracklets(int n_sec, const orc_sector* sec, int n_rows,
                             const float* row_x, const orc_params* prm,
                             const int* bin_start, const float* yg, const float* zg,
                             const int* idg,
                             const uint8_t* row, const float* y, const float* z,
                             const int* up, int64_t n_starts, const int* starts,
                             int brute, int* hits, int* nhits, int* row_inner,
                             float* par, float* cov, float* chi2)
{
    const float sy2 = prm->sigma_y2, sz2 = prm->sigma_z2;
    g_work[0] = g_work[1] = g_work[2] = 0;
    for (int64_t t = 0; t < n_starts; t++) {
        int* th = hits + t * n_rows;
        for (int r = 0; r < n_rows; r++) th[r] = -1;
        int h0 = starts[t];
        search_ctx cx = {&sec[sector_of(n_sec, sec, h0)], bin_start, yg, zg, idg,
                         n_rows, prm, brute};
        int h1 = up[h0], h2 = up[h1];
        int r0 = row[h0];
        float p[5], C[15];
        init_state_f(p, C, row_x[r0], y[h0], z[h0], row_x[row[h2]], y[h2], z[h2], sy2,
                     sz2, prm->c_ss0, prm->c_tt0, prm->c_ww0);
        th[r0] = h0;
        int cur = r0, last = r0;
        float plast[5];
        memcpy(plast, p, sizeof plast);
        /* up: the chain */
        int ok = 1;
        for (int h = h1; h >= 0; h = up[h]) {
            int r = row[h];
            if (!prop_counted(p, C, row_x[r] - row_x[cur], prm->curv, prm->s_max)) {
                ok = 0;
                break;
            }
            update_counted(p, C, y[h], z[h], sy2, sz2);
            th[r] = h;
            cur = last = r;
            memcpy(plast, p, sizeof plast);
        }
        /* up: search outwards */
        if (ok) {
            int miss = 0;
            for (int r = cur + 1; r < n_rows; r++) {
                if (!prop_counted(p, C, row_x[r] - row_x[r - 1], prm->curv, prm->s_max)) break;
                int c = search_row(&cx, r, p, C);
                if (c >= 0) {
                    update_counted(p, C, y[c], z[c], sy2, sz2);
                    th[r] = c;
                    last = r;
                    memcpy(plast, p, sizeof plast);
                    miss = 0;
                } else if (++miss >= prm->max_miss) {
                    break;
                }
            }
        }
        /* down */
        memcpy(p, plast, sizeof plast);
        p[0] = y[th[last]];
        p[1] = z[th[last]];
        for (int i = 0; i < 15; i++) C[i] = 0.0f;
        C[0] = sy2;
        C[2] = sz2;
        C[5] = prm->c_ss0;
        C[9] = prm->c_tt0;
        C[14] = prm->c_ww0;
        float pin[5], Cin[15], csum = 0.0f;
        memcpy(pin, p, sizeof pin);
        memcpy(Cin, C, sizeof Cin);
        int rin = last, miss = 0;
        for (int r = last - 1; r >= 0; r--) {
            if (!prop_counted(p, C, row_x[r] - row_x[r + 1], prm->curv, prm->s_max)) {
                for (int q = r; q >= 0; q--) th[q] = -1;
                break;
            }
            int c = -1;
            if (r >= r0) {
                c = th[r];
            } else {
                c = search_row(&cx, r, p, C);
                if (c < 0) {
                    if (++miss >= prm->max_miss) break;
                    continue;
                }
                miss = 0;
            }
            if (c >= 0) {
                csum = csum + update_counted(p, C, y[c], z[c], sy2, sz2);
                th[r] = c;
                rin = r;
                memcpy(pin, p, sizeof pin);
                memcpy(Cin, C, sizeof Cin);
            }
        }
        int n = 0;
        for (int r = 0; r < n_rows; r++) n += th[r] >= 0;
        nhits[t] = n;
        row_inner[t] = rin;
        memcpy(par + t * 5, pin, sizeof pin);
        memcpy(cov + t * 15, Cin, sizeof Cin);
        chi2[t] = csum;
    }
}

/* FP64 replay: the same sequence of propagations and updates as the float
 * construction, with the hit list fixed (up pass over rows >= start_row
 * from the chain start, down pass from the outermost hit). */
int orc_tracklet_replay64(int n_rows, const float* row_x, const orc_params* prm,
                          const float* y, const float* z, int r0,
                          const int* th, double* p, double* C, double* chi2)
{
    const double sy2 = prm->sigma_y2, sz2 = prm->sigma_z2;
    int last = -1, rmin = n_rows;
    for (int r = 0; r < n_rows; r++)
        if (th[r] >= 0) {
            last = r;
            if (r < rmin) rmin = r;
        }
    if (last < 0 || th[r0] < 0) return 1;
    int r2 = -1, cnt = 0;
    for (int r = r0 + 1; r < n_rows; r++)
        if (th[r] >= 0 && ++cnt == 2) {
            r2 = r;
            break;
        }
    if (r2 < 0) return 1;
    int h0 = th[r0], h2 = th[r2];
    init_state_d(p, C, row_x[r0], y[h0], z[h0], row_x[r2], y[h2], z[h2], sy2, sz2,
                 prm->c_ss0, prm->c_tt0, prm->c_ww0);
    double plast[5];
    memcpy(plast, p, sizeof plast);
    for (int r = r0 + 1; r <= last; r++) {
        if (!propagate_d(p, C, (double)row_x[r] - (double)row_x[r - 1], prm->curv, prm->s_max))
            return 2;
        if (th[r] >= 0) {
            update_d(p, C, y[th[r]], z[th[r]], sy2, sz2);
            memcpy(plast, p, sizeof plast);
        }
    }
    memcpy(p, plast, sizeof plast);
    p[0] = y[th[last]];
    p[1] = z[th[last]];
    for (int i = 0; i < 15; i++) C[i] = 0.0;
    C[0] = sy2;
    C[2] = sz2;
    C[5] = prm->c_ss0;
    C[9] = prm->c_tt0;
    C[14] = prm->c_ww0;
    double csum = 0.0;
    for (int r = last - 1; r >= rmin; r--) {
        if (!propagate_d(p, C, (double)row_x[r] - (double)row_x[r + 1], prm->curv, prm->s_max))
            return 2;
        if (th[r] >= 0) csum += update_d(p, C, y[th[r]], z[th[r]], sy2, sz2);
    }
    *chi2 = csum;
    return 0;
}

/* ---- tracklet selection ---------------------------------------------------
 * key(t) = nhits << 32 | (2^32 - 1 - start id) for tracklets with at least
 * min_tracklet_hits hits, else 0.  Every cluster belongs to the tracklet of
 * largest key containing it; a tracklet becomes a track if it keeps at
 * least min_track_hits of its clusters.  Tracks come out in tracklet
 * order (ascending start id), hits by ascending row. */
int64_t orc_select_tracks(int64_t n_clusters, int n_rows, const orc_params* prm,
                          int64_t n_tracklets, const int* hits, const int* nhits,
                          const int* starts, int* trk_off, int* trk_hits,
                          int* trk_tracklet)
{
    uint64_t* owner = calloc((size_t)n_clusters, sizeof(uint64_t));
    uint64_t* key = malloc(((size_t)n_tracklets + 1) * sizeof(uint64_t));
    for (int64_t t = 0; t < n_tracklets; t++) {
        key[t] = nhits[t] >= prm->min_tracklet_hits
                     ? ((uint64_t)nhits[t] << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)starts[t])
                     : 0;
        if (!key[t]) continue;
        for (int r = 0; r < n_rows; r++) {
            int c = hits[t * n_rows + r];
            if (c >= 0 && key[t] > owner[c]) owner[c] = key[t];
        }
    }
    int64_t m = 0, nh = 0;
    trk_off[0] = 0;
    for (int64_t t = 0; t < n_tracklets; t++) {
        if (!key[t]) continue;
        int kept = 0;
        for (int r = 0; r < n_rows; r++) {
            int c = hits[t * n_rows + r];
            kept += c >= 0 && owner[c] == key[t];
        }
        if (kept < prm->min_track_hits) continue;
        for (int r = 0; r < n_rows; r++) {
            int c = hits[t * n_rows + r];
            if (c >= 0 && owner[c] == key[t]) trk_hits[nh++] = c;
        }
        trk_tracklet[m] = (int)t;
        trk_off[++m] = (int)nh;
    }
    free(owner);
    free(key);
    return m;
}

/* ---- calibrated refit ---------------------------------------------------- */
void orc_refit32(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                 const float* y, const float* z, const signed char* side,
                 const float* row_x, const orc_params* prm,
                 const orc_calib_model* cm, const float* theta,
                 float* par, float* cov, float* chi2, int* status)
{
    for (int64_t t = 0; t < n_tracks; t++) {
        int a = trk_off[t], n = trk_off[t + 1] - a;
        float sd = side ? (float)side[t] : 1.0f;
        status[t] = refit_track_f(n, row + a, y + a, z + a, sd, row_x, prm, cm, theta,
                                  par + 5 * t, cov + 15 * t, chi2 + t);
    }
}

void orc_refit64(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                 const double* y, const double* z, const signed char* side,
                 const float* row_x, const orc_params* prm,
                 const orc_calib_model* cm, const double* theta,
                 double* par, double* cov, double* chi2, int* status)
{
    for (int64_t t = 0; t < n_tracks; t++) {
        int a = trk_off[t], n = trk_off[t + 1] - a;
        double sd = side ? (double)side[t] : 1.0;
        status[t] = refit_track_d(n, row + a, y + a, z + a, sd, row_x, prm, cm, theta,
                                  par + 5 * t, cov + 15 * t, chi2 + t);
    }
}

static double track_chi2_d(int n, const uint8_t* row, const double* y, const double* z,
                           double sd, const float* row_x, const orc_params* prm,
                           const orc_calib_model* cm, const double* th)
{
    double p[5], C[15], c2;
    refit_track_d(n, row, y, z, sd, row_x, prm, cm, th, p, C, &c2);
    return c2;
}

void orc_refit64_fd_grad(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                         const double* y, const double* z, const signed char* side,
                         const float* row_x, const orc_params* prm,
                         const orc_calib_model* cm, const double* theta,
                         const double* g, double h_hit, double h_theta,
                         double* grad_y, double* grad_z, double* grad_theta)
{
    int nmax = 0;
    for (int64_t t = 0; t < n_tracks; t++)
        if (trk_off[t + 1] - trk_off[t] > nmax) nmax = trk_off[t + 1] - trk_off[t];
    double* wy = malloc(sizeof(double) * (size_t)(nmax > 0 ? nmax : 1));
    double* wz = malloc(sizeof(double) * (size_t)(nmax > 0 ? nmax : 1));
    double th[16];
    memcpy(th, theta, sizeof th);
    for (int k = 0; k < 16; k++) grad_theta[k] = 0.0;
    for (int64_t t = 0; t < n_tracks; t++) {
        int a = trk_off[t], n = trk_off[t + 1] - a;
        double sd = side ? (double)side[t] : 1.0;
        memcpy(wy, y + a, sizeof(double) * (size_t)n);
        memcpy(wz, z + a, sizeof(double) * (size_t)n);
        for (int i = 0; i < n; i++) {
            double* v[2] = {wy, wz};
            double* out[2] = {grad_y, grad_z};
            for (int c = 0; c < 2; c++) {
                double v0 = v[c][i];
                double h = h_hit;
                v[c][i] = v0 + h;
                double fp = track_chi2_d(n, row + a, wy, wz, sd, row_x, prm, cm, th);
                v[c][i] = v0 - h;
                double fm = track_chi2_d(n, row + a, wy, wz, sd, row_x, prm, cm, th);
                v[c][i] = v0;
                out[c][a + i] = g[t] * (fp - fm) / (2.0 * h);
            }
        }
        for (int k = 0; k < 16; k++) {
            double v0 = th[k];
            double h = h_theta * (fabs(v0) > 1.0 ? fabs(v0) : 1.0);
            th[k] = v0 + h;
            double fp = track_chi2_d(n, row + a, y + a, z + a, sd, row_x, prm, cm, th);
            th[k] = v0 - h;
            double fm = track_chi2_d(n, row + a, y + a, z + a, sd, row_x, prm, cm, th);
            th[k] = v0;
            grad_theta[k] += g[t] * (fp - fm) / (2.0 * h);
        }
    }
    free(wy);
    free(wz);
}

/* ---- single-step entry points for the tests ------------------------------ */
int orc_propagate32(float* p, float* C, float dx, float curv, float s_max)
{
    return propagate_f(p, C, dx, curv, s_max);
}

int orc_propagate64(double* p, double* C, double dx, double curv, double s_max)
{
    return propagate_d(p, C, dx, curv, s_max);
}

float orc_update32(float* p, float* C, float my, float mz, float sy2, float sz2)
{
    return update_f(p, C, my, mz, sy2, sz2);
}

double orc_update64(double* p, double* C, double my, double mz, double sy2, double sz2)
{
    return update_d(p, C, my, mz, sy2, sz2);
}

float orc_chi2_pred32(const float* p, const float* C, float my, float mz, float sy2, float sz2)
{
    return chi2_pred_f(p, C, my, mz, sy2, sz2);
}

void orc_calibrate64(const double* th, double xr, double yr, double zr, double side,
                     const orc_calib_model* cm, double* out3)
{
    calibrate_d(th, xr, yr, zr, side, cm->drift_len, cm->vd, cm->tan_half, cm->u_centre,
                cm->u_scale, out3, out3 + 1, out3 + 2);
}

/* ---- track-based cluster attachment (section 6, TPC data compression: cluster rejection) -------
 * The tracker lays a tube of fixed radius around every track and marks each
 * cluster that no track owns as adjacent to the track of highest transverse
 * momentum whose tube holds it.  Readings: the tube of track k covers the
 * pad rows from its first to its last hit; at row r its axis is the point
 * (y_r, z_r) of the track's state (at the plane of row rin[k], the output of
 * the inward pass) transported outwards row by row (the tracker's own
 * transport, stopping where |sin(phi)| reaches s_max); a cluster of the
 * track's sector on row r lies in the tube when dy*dy + dz*dz <= radius^2
 * (float32, in that order).  Highest pT = least |q/pT|, ties to the lower
 * track index.  Protected: in the tube of, or attached to, a track with
 * |q/pT| <= w_good; removed: attached or adjacent and not protected.
 * Brute force over the clusters of each row of the sector.
 * track[c]: owning track, else the adjacent track, else -1;
 * state[c]: 1 attached, 2 adjacent, | 4 protected, | 8 removed. */
void orc_attach_clusters(int n_sec, const int64_t* sector_offsets, int n_rows,
                         const float* row_x, const orc_params* prm, const uint8_t* row,
                         const float* y, const float* z, int64_t n_clusters, int64_t n_tracks,
                         const int* trk_off, const int* trk_hits, const float* par,
                         const int* rin, float radius, float w_good, int* track,
                         uint8_t* state)
{
    const float r2 = radius * radius;
    /* clusters of every (sector, row), in id order */
    int64_t n_lists = (int64_t)n_sec * n_rows;
    int64_t* first = (int64_t*)calloc((size_t)n_lists + 1, sizeof(int64_t));
    int64_t* members = (int64_t*)malloc((size_t)(n_clusters > 0 ? n_clusters : 1) * sizeof(int64_t));
    int64_t* fill = (int64_t*)calloc((size_t)n_lists + 1, sizeof(int64_t));
    float* best_w = (float*)malloc((size_t)(n_clusters > 0 ? n_clusters : 1) * sizeof(float));
    int s = 0;
    for (int64_t c = 0; c < n_clusters; c++) {
        while (s + 1 < n_sec && c >= sector_offsets[s + 1]) s++;
        if (row[c] < n_rows) first[(int64_t)s * n_rows + row[c] + 1]++;
    }
    for (int64_t k = 0; k < n_lists; k++) first[k + 1] += first[k];
    s = 0;
    for (int64_t c = 0; c < n_clusters; c++) {
        while (s + 1 < n_sec && c >= sector_offsets[s + 1]) s++;
        if (row[c] < n_rows) {
            int64_t l = (int64_t)s * n_rows + row[c];
            members[first[l] + fill[l]++] = c;
        }
    }
    for (int64_t c = 0; c < n_clusters; c++) {
        track[c] = -1;
        state[c] = 0;
        best_w[c] = 0.0f;
    }
    for (int64_t k = 0; k < n_tracks; k++)
        for (int i = trk_off[k]; i < trk_off[k + 1]; i++) {
            track[trk_hits[i]] = (int)k;
            state[trk_hits[i]] = 1;
        }
    for (int64_t k = 0; k < n_tracks; k++) {
        if (trk_off[k + 1] <= trk_off[k]) continue;
        int c0 = trk_hits[trk_off[k]];
        int sk = 0;
        while (sk + 1 < n_sec && c0 >= sector_offsets[sk + 1]) sk++;
        int r_first = row[c0], r_last = row[trk_hits[trk_off[k + 1] - 1]];
        float p[5], C[15];
        for (int i = 0; i < 5; i++) p[i] = par[5 * k + i];
        for (int i = 0; i < 15; i++) C[i] = 0.0f;
        float w = fabsf(p[4]);
        int good = w <= w_good;
        for (int r = rin[k]; r <= r_last; r++) {
            if (r > rin[k] && !propagate_f(p, C, row_x[r] - row_x[r - 1], prm->curv, prm->s_max))
                break;
            if (r < r_first) continue;
            int64_t l = (int64_t)sk * n_rows + r;
            for (int64_t m = first[l]; m < first[l + 1]; m++) {
                int64_t c = members[m];
                float dy = y[c] - p[0], dz = z[c] - p[1];
                if (!(dy * dy + dz * dz <= r2)) continue;
                if (good) state[c] |= 4;
                if (state[c] & 1) continue;
                if (track[c] < 0 || w < best_w[c] || (w == best_w[c] && (int)k < track[c])) {
                    track[c] = (int)k;
                    best_w[c] = w;
                }
            }
        }
    }
    for (int64_t c = 0; c < n_clusters; c++) {
        if (track[c] >= 0 && !(state[c] & 1)) state[c] |= 2;
        if ((state[c] & 1) && fabsf(par[5 * track[c] + 4]) <= w_good) state[c] |= 4;
        if ((state[c] & 3) && !(state[c] & 4)) state[c] |= 8;
    }
    free(first);
    free(members);
    free(fill);
    free(best_w);
}

/* ---- sector-track merging (section 2: the first fit of the sector tracks
 * serves to find the whole track; section 3: sector boundaries) -----------
 * Readings: the sector of a track is that of its first hit.  Sector s lies
 * on side s / sps at index i = s % sps; its frame is rotated by
 * (i + 1/2) * width; its up neighbour is index (i + 1) % sps on the same
 * side, its down neighbour (i + sps - 1) % sps.  The state of track j (par
 * at the plane x_j = row_x[rin[j]] of its sector's frame) is taken into the
 * frame of a sector rotated by D = alpha_j - alpha_k (cos D = c, sin D =
 * sd: +sin(width) when j's sector is the up neighbour of k's, -sin(width)
 * when it is the down neighbour):
 *   x' = x c - y sd,  y' = x sd + y c,  sin' = sin c + cos sd,
 *   cos' = cos c - sin sd  (cos = sqrt((1 - sin)(1 + sin))),
 * valid when cos' > 0 and |sin'| < s_max; z, tan(lambda) and q/pT do not
 * change.  It is then transported to x_k with the tracker's transport (no
 * candidate where that stops).  Distance: d2 = sum over the five
 * parameters, in order, of ((p'_i - p_k,i) * iw_i)^2; a candidate needs
 * d2 < 1.  Best partner per direction: least d2, ties to the lower index.
 * Tracks k and j (j in the up neighbour of k's sector) are linked when each
 * is the other's best partner in that direction.  group[k]: the least track
 * index over the chain of links through k. */
int orc_merge_transform(const float* pj, float xj, float c, float sd, float x_to, float curv,
                        float s_max, float* out5)
{
    float y = pj[0], s = pj[2];
    float cs = sqrtf((1.0f - s) * (1.0f + s));
    float xr = xj * c - y * sd;
    float p[5], C[15];
    p[0] = xj * sd + y * c;
    p[1] = pj[1];
    p[2] = s * c + cs * sd;
    p[3] = pj[3];
    p[4] = pj[4];
    float cr = cs * c - s * sd;
    if (!(cr > 0.0f) || !(fabsf(p[2]) < s_max)) return 0;
    for (int i = 0; i < 15; i++) C[i] = 0.0f;
    if (!propagate_f(p, C, x_to - xr, curv, s_max)) return 0;
    for (int i = 0; i < 5; i++) out5[i] = p[i];
    return 1;
}

void orc_merge_sector_tracks(int n_sec, const int64_t* sector_offsets, int sps,
                             const float* row_x, const orc_params* prm, int64_t n_tracks,
                             const int* trk_off, const int* trk_hits, const float* par,
                             const int* rin, float cos_w, float sin_w, const float* iw,
                             int* link_up, int* link_dn, int* group)
{
    int64_t nt1 = n_tracks > 0 ? n_tracks : 1;
    int* sec = (int*)malloc((size_t)nt1 * sizeof(int));
    int* best = (int*)malloc((size_t)nt1 * 2 * sizeof(int));
    int64_t* first = (int64_t*)calloc((size_t)n_sec + 1, sizeof(int64_t));
    int64_t* fill = (int64_t*)calloc((size_t)n_sec + 1, sizeof(int64_t));
    int64_t* members = (int64_t*)malloc((size_t)nt1 * sizeof(int64_t));
    for (int64_t k = 0; k < n_tracks; k++) {
        sec[k] = -1;
        if (trk_off[k + 1] > trk_off[k]) {
            int c0 = trk_hits[trk_off[k]];
            int s = 0;
            while (s + 1 < n_sec && c0 >= sector_offsets[s + 1]) s++;
            sec[k] = s;
            first[s + 1]++;
        }
    }
    for (int s = 0; s < n_sec; s++) first[s + 1] += first[s];
    for (int64_t k = 0; k < n_tracks; k++)
        if (sec[k] >= 0) members[first[sec[k]] + fill[sec[k]]++] = k;
    /* best partner of every track in its up (d = 0) and down (d = 1) neighbour */
    for (int64_t k = 0; k < n_tracks; k++)
        for (int d = 0; d < 2; d++) {
            best[2 * k + d] = -1;
            if (sec[k] < 0) continue;
            int side = sec[k] / sps, i = sec[k] % sps;
            int nb = side * sps + (d == 0 ? (i + 1) % sps : (i + sps - 1) % sps);
            float sd = d == 0 ? sin_w : -sin_w;
            float xk = row_x[rin[k]];
            float best_d2 = 0.0f;
            for (int64_t m = first[nb]; m < first[nb + 1]; m++) {
                int64_t j = members[m];
                float q[5];
                if (!orc_merge_transform(par + 5 * j, row_x[rin[j]], cos_w, sd, xk, prm->curv,
                                         prm->s_max, q))
                    continue;
                float d2 = 0.0f;
                for (int e = 0; e < 5; e++) {
                    float r = (q[e] - par[5 * k + e]) * iw[e];
                    d2 = d2 + r * r;
                }
                if (!(d2 < 1.0f)) continue;
                if (best[2 * k + d] < 0 || d2 < best_d2) {
                    best[2 * k + d] = (int)j;
                    best_d2 = d2;
                }
            }
        }
    for (int64_t k = 0; k < n_tracks; k++) {
        int j = best[2 * k];
        link_up[k] = (j >= 0 && best[2 * j + 1] == (int)k) ? j : -1;
        j = best[2 * k + 1];
        link_dn[k] = (j >= 0 && best[2 * j] == (int)k) ? j : -1;
    }
    for (int64_t k = 0; k < n_tracks; k++) {
        int g = (int)k;
        for (int d = 0; d < 2; d++) {
            const int* lk = d == 0 ? link_up : link_dn;
            int j = lk[k];
            for (int step = 0; j >= 0 && j != (int)k && step < n_sec; step++) {
                if (j < g) g = j;
                j = lk[j];
            }
        }
        group[k] = g;
    }
    free(sec);
    free(best);
    free(first);
    free(fill);
    free(members);
}

/* ---- full-track fit of merged sector tracks (section 2: the first fit of
 * the sector tracks finds the whole track, which is then fitted; section 3:
 * several fit iterations, inwards and outwards, across sector boundaries) --
 * Readings: the members of a merged track form a chain through the merging
 * links.  The chain is walked from its down end (link_dn) to its up end
 * (link_up), or the other way when the up end's first hit lies on a lower
 * row than the down end's first hit; the merged hit list is the members'
 * hits in that order, each member's row-ascending.  Between consecutive hits
 * of neighbouring sectors the state is turned into the next sector's frame
 * (D = alpha_now - alpha_next: sin D = -sin(width) towards the up
 * neighbour, +sin(width) towards the down neighbour) and transported to the
 * next hit's row plane.  The fit starts from the first member's tracklet
 * state (at the plane of its innermost fitted row) and makes n_pass passes
 * over all hits, alternately outwards (first to last hit) and inwards; every
 * pass starts from the previous pass's parameters and a diagonal covariance,
 * the variances of the first member's tracklet (first pass) or of the
 * previous pass's end, times cov_scale (a weak prior that keeps the float32
 * filter away from the cancellation a restart from the tracklet's initial
 * variances causes), and updates with every hit (the first at the plane
 * where the previous pass ended).  Outputs, for the chain's least track index
 * (its group) only: the state after the last outward pass at the last hit
 * (its sector's frame) and its covariance, the state after the last inward
 * pass at the first hit (zero with one pass), the chi2 sum of the last pass,
 * the hit count and the member count.  status: 0 fitted, 1 fewer than 3 hits, 2 a transport or a
 * frame turn stopped, -1 not a group's leader. */
#define REAL float
#define SUF _f
#include "fullfit_impl.h"
#undef REAL
#undef SUF
#define REAL double
#define SUF _d
#include "fullfit_impl.h"
#undef REAL
#undef SUF

void orc_fit_merged64(int n_sec, const int64_t* sector_offsets, int sps, const float* row_x,
                      const orc_params* prm, const uint8_t* row, const float* y, const float* z,
                      int64_t n_tracks, const int* trk_off, const int* trk_hits,
                      const float* par, const float* cov, const int* rin,
                      const int* link_up, const int* link_dn, const int* group, float cos_w,
                      float sin_w, int n_pass, float cov_scale, double* par_in,
                      double* par_out, double* cov_out, double* chi2_out, int* n_hits,
                      int* n_members, int* status)
{
    fit_merged_d(n_sec, sector_offsets, sps, row_x, prm, row, y, z, n_tracks, trk_off, trk_hits,
                 par, cov, rin, link_up, link_dn, group, cos_w, sin_w, n_pass, cov_scale,
                 par_in, par_out,
                 cov_out, chi2_out, n_hits, n_members, status);
}

void orc_fit_merged32(int n_sec, const int64_t* sector_offsets, int sps, const float* row_x,
                      const orc_params* prm, const uint8_t* row, const float* y, const float* z,
                      int64_t n_tracks, const int* trk_off, const int* trk_hits,
                      const float* par, const float* cov, const int* rin,
                      const int* link_up, const int* link_dn, const int* group, float cos_w,
                      float sin_w, int n_pass, float cov_scale, float* par_in,
                      float* par_out, float* cov_out, float* chi2_out, int* n_hits,
                      int* n_members, int* status)
{
    fit_merged_f(n_sec, sector_offsets, sps, row_x, prm, row, y, z, n_tracks, trk_off, trk_hits,
                 par, cov, rin, link_up, link_dn, group, cos_w, sin_w, n_pass, cov_scale,
                 par_in, par_out,
                 cov_out, chi2_out, n_hits, n_members, status);
}

/* ---- weights of the beam-axis term of the calibration objective ---------
 * Per track (refit at theta, float64): the state and covariance of the last
 * hit, at its calibrated plane, transported to x = 0 in ceil(x / 20 cm)
 * equal steps; S = the (y, z) block of the covariance there plus
 * sigma_v2 on the diagonal; W = S^-1 as (w00, w01, w11); zeros and ok = 0
 * where the refit or the transport stops. */
void orc_vertex_weights64(int64_t n_tracks, const int* trk_off, const uint8_t* row,
                          const double* y, const double* z, const signed char* side,
                          const float* row_x, const orc_params* prm,
                          const orc_calib_model* cm, const double* theta, double sigma_v2,
                          double* w, int* ok)
{
    for (int64_t t = 0; t < n_tracks; t++) {
        int a = trk_off[t], n = trk_off[t + 1] - a;
        double sd = side ? (double)side[t] : 1.0;
        double p[5], C[15], chi2;
        w[3 * t] = w[3 * t + 1] = w[3 * t + 2] = 0.0;
        ok[t] = 0;
        if (refit_track_d(n, row + a, y + a, z + a, sd, row_x, prm, cm, theta, p, C, &chi2))
            continue;
        double xl, yl, zl;
        calibrate_d(theta, (double)row_x[row[a + n - 1]], y[a + n - 1], z[a + n - 1], sd,
                    cm->drift_len, cm->vd, cm->tan_half, cm->u_centre, cm->u_scale, &xl, &yl,
                    &zl);
        int ns = (int)ceil(xl / 20.0);
        if (ns < 1) ns = 1;
        double dx = (0.0 - xl) / (double)ns;
        int good = 1;
        for (int i = 0; i < ns && good; i++) good = propagate_d(p, C, dx, prm->curv, prm->s_max);
        if (!good) continue;
        double s00 = C[0] + sigma_v2, s10 = C[1], s11 = C[2] + sigma_v2;
        double det = s00 * s11 - s10 * s10;
        w[3 * t] = s11 / det;
        w[3 * t + 1] = -s10 / det;
        w[3 * t + 2] = s00 / det;
        ok[t] = 1;
    }
}

/* One frame turn (float64) for the pins: x, p[5], C[15] in place. */
int orc_rotate64(double* x, double* p, double* C, double c, double sd, double curv,
                 double s_max)
{
    return rotate_d(x, p, C, c, sd, curv, s_max);
}

/* ---- per-track interaction time (section 2: continuous read-out; the z of
 * a hit depends on the unknown time of its collision) -----------------------
 * Readings: a primary track comes from the beam axis at z = 0; the tracker
 * sees z* = z - side * vd * t for a collision at time t (side +1 for z > 0,
 * -1 for z < 0).  The track's state (par at the plane x = row_x[rin]) is
 * transported to the plane x = 0 of its sector frame, which contains the
 * beam axis, with the tracker's transport in ceil(x_in / T0_STEP) equal
 * steps (float32: dx = (0 - x_in) / n): there y0 is the distance from
 * the axis (0 for a primary) and z0 = -side * vd * t, so the estimate is
 * t0 = (side > 0 ? -z0 : z0) / vd (float32).  ok = 0 (and z0, y0, t0 = 0)
 * where the transport stops. */
#define T0_STEP 20.0f

void orc_track_t0(int64_t n_tracks, const float* par, const float* x_in,
                  const signed char* side, float curv, float s_max, float vd, float* z0,
                  float* y0, float* t0, signed char* ok)
{
    for (int64_t k = 0; k < n_tracks; k++) {
        float p[5], C[15];
        for (int i = 0; i < 5; i++) p[i] = par[5 * k + i];
        for (int i = 0; i < 15; i++) C[i] = 0.0f;
        /* n equal steps of at most T0_STEP cm: over one such step the
         * arc-length series keeps its truncation error below 1e-5 of the
         * step down to pT = 0.05 GeV/c (|a| <= 0.3), where a single step
         * over the whole distance would not */
        int n = (int)ceilf(x_in[k] / T0_STEP);
        if (n < 1) n = 1;
        float dx = (0.0f - x_in[k]) / (float)n;
        int alive = 1;
        for (int i = 0; i < n && alive; i++) alive = propagate_f(p, C, dx, curv, s_max);
        if (!alive) {
            z0[k] = y0[k] = t0[k] = 0.0f;
            ok[k] = 0;
            continue;
        }
        y0[k] = p[0];
        z0[k] = p[1];
        t0[k] = (side[k] > 0 ? -p[1] : p[1]) / vd;
        ok[k] = 1;
    }
}
