/*
 * Full-track fit of merged sector tracks, written once for a generic real
 * type (oracle.c includes it for float, suffix _f, and double, _d).  TEST
 * INFRASTRUCTURE ONLY.  The reading is stated in oracle.c above the entry
 * points.
 */
#define CAT_(a, b) a##b
#define CAT(a, b) CAT_(a, b)
#define FN(name) CAT(name, SUF)

static int FN(sector_of_id)(int n_sec, const int64_t* sector_offsets, int c)
{
    int s = 0;
    while (s + 1 < n_sec && c >= sector_offsets[s + 1]) s++;
    return s;
}

static void FN(fit_merged)(int n_sec, const int64_t* sector_offsets, int sps, const float* row_x,
                      const orc_params* prm, const uint8_t* row, const float* y, const float* z,
                      int64_t n_tracks, const int* trk_off, const int* trk_hits,
                      const float* par, const float* cov, const int* rin,
                      const int* link_up, const int* link_dn, const int* group, float cos_w,
                      float sin_w, int n_pass, float cov_scale, REAL* par_in,
                      REAL* par_out, REAL* cov_out, REAL* chi2_out, int* n_hits,
                      int* n_members, int* status)
{
    int64_t nh_all = n_tracks > 0 ? trk_off[n_tracks] : 0;
    int* hits = malloc(sizeof(int) * (size_t)(nh_all > 0 ? nh_all : 1));
    int* hsec = malloc(sizeof(int) * (size_t)(nh_all > 0 ? nh_all : 1));
    int* chain = malloc(sizeof(int) * (size_t)(n_sec + 1));
    for (int64_t g = 0; g < n_tracks; g++) {
        for (int i = 0; i < 5; i++) par_in[5 * g + i] = par_out[5 * g + i] = 0;
        for (int i = 0; i < 15; i++) cov_out[15 * g + i] = 0;
        chi2_out[g] = 0;
        n_hits[g] = 0;
        n_members[g] = 0;
        if (group[g] != (int)g) {
            status[g] = -1;
            continue;
        }
        /* the chain: down end first, at most one member per sector */
        int j = (int)g;
        for (int step = 0; step < n_sec && link_dn[j] >= 0 && link_dn[j] != (int)g; step++)
            j = link_dn[j];
        int m = 0;
        while (j >= 0 && m < n_sec) {
            chain[m++] = j;
            j = link_up[j];
            if (j == chain[0]) break;
        }
        int r_dn = trk_off[chain[0] + 1] > trk_off[chain[0]] ? row[trk_hits[trk_off[chain[0]]]] : 0;
        int r_up = trk_off[chain[m - 1] + 1] > trk_off[chain[m - 1]]
                       ? row[trk_hits[trk_off[chain[m - 1]]]] : 0;
        if (r_up < r_dn)
            for (int a = 0, b = m - 1; a < b; a++, b--) {
                int t = chain[a];
                chain[a] = chain[b];
                chain[b] = t;
            }
        int n = 0;
        for (int a = 0; a < m; a++)
            for (int q = trk_off[chain[a]]; q < trk_off[chain[a] + 1]; q++) {
                hits[n] = trk_hits[q];
                hsec[n] = FN(sector_of_id)(n_sec, sector_offsets, trk_hits[q]);
                n++;
            }
        n_hits[g] = n;
        n_members[g] = m;
        if (n < 3) {
            status[g] = 1;
            continue;
        }
        REAL p[5], C[15], x = (REAL)row_x[rin[chain[0]]];
        REAL pout[5] = {0, 0, 0, 0, 0}, Cout[15], pin[5] = {0, 0, 0, 0, 0};
        for (int i = 0; i < 15; i++) Cout[i] = 0;
        for (int i = 0; i < 5; i++) p[i] = (REAL)par[5 * chain[0] + i];
        /* every pass starts from a diagonal covariance: the variances of the
         * first member's tracklet (first pass) or of the previous pass's end,
         * times cov_scale; the initial variances stand in for any that is
         * not positive and finite */
        const int di[5] = {0, 2, 5, 9, 14};
        const REAL v0[5] = {(REAL)prm->sigma_y2, (REAL)prm->sigma_z2, (REAL)prm->c_ss0,
                            (REAL)prm->c_tt0, (REAL)prm->c_ww0};
        REAL dg[5];
        for (int j = 0; j < 5; j++) {
            REAL v = (REAL)cov[15 * chain[0] + di[j]];
            dg[j] = v > 0 && v < (REAL)1e30 ? v : v0[j];
        }
        int cur = hsec[0], ok = 1;
        REAL chi2 = 0;
        for (int pass = 0; pass < n_pass && ok; pass++) {
            int out = pass % 2 == 0;
            for (int i = 0; i < 15; i++) C[i] = 0;
            for (int j = 0; j < 5; j++) C[di[j]] = dg[j] * (REAL)cov_scale;
            chi2 = 0;
            for (int k = 0; k < n && ok; k++) {
                int i = out ? k : n - 1 - k;
                if (hsec[i] != cur) {
                    /* neighbouring sectors of one side: up or down */
                    int side = cur / sps, ic = cur % sps;
                    int up = side * sps + (ic + 1) % sps;
                    REAL sd = hsec[i] == up ? -(REAL)sin_w : (REAL)sin_w;
                    if (!FN(rotate)(&x, p, C, (REAL)cos_w, sd, (REAL)prm->curv, (REAL)prm->s_max)) {
                        ok = 0;
                        break;
                    }
                    cur = hsec[i];
                }
                REAL xh = (REAL)row_x[row[hits[i]]];
                if (!FN(propagate)(p, C, xh - x, (REAL)prm->curv, (REAL)prm->s_max)) {
                    ok = 0;
                    break;
                }
                x = xh;
                chi2 = chi2 + FN(update)(p, C, (REAL)y[hits[i]], (REAL)z[hits[i]],
                                         (REAL)prm->sigma_y2, (REAL)prm->sigma_z2);
            }
            if (!ok) break;
            for (int j = 0; j < 5; j++) {
                REAL v = C[di[j]];
                dg[j] = v > 0 && v < (REAL)1e30 ? v : v0[j];
            }
            if (out) {
                for (int i = 0; i < 5; i++) pout[i] = p[i];
                for (int i = 0; i < 15; i++) Cout[i] = C[i];
            } else {
                for (int i = 0; i < 5; i++) pin[i] = p[i];
            }
        }
        if (!ok) {
            status[g] = 2;
            continue;
        }
        for (int i = 0; i < 5; i++) par_in[5 * g + i] = pin[i];
        for (int i = 0; i < 5; i++) par_out[5 * g + i] = pout[i];
        for (int i = 0; i < 15; i++) cov_out[15 * g + i] = Cout[i];
        chi2_out[g] = chi2;
        status[g] = 0;
    }
    free(hits);
    free(hsec);
    free(chain);
}

#undef FN
#undef CAT
#undef CAT_
