/*
 * Kalman-filter primitives of the oracle, written once for a generic real
 * type.  oracle.c includes this file twice: REAL=float (suffix _f) and
 * REAL=double (suffix _d).  TEST INFRASTRUCTURE ONLY.
 *
 * State at the sector-local plane x (reading of the paper's Kalman-filter
 * track following, section 3):  p = (y, z, s, t, w) with s = sin(phi),
 * t = tan(lambda), w = q/pT; covariance C stored as the lower triangle of
 * the symmetric 5x5 matrix, row by row: C(i,j), i >= j, at i*(i+1)/2 + j.
 *
 * Helix in a uniform field along z: the curvature k = curv * w is constant,
 * so sin(phi) grows linearly with x (ds/dx = k), the y step is
 * dx * (s1 + s2) / (c1 + c2) with c = sqrt(1 - s^2) (exact for a circle),
 * and the transverse arc length over the step is chord * asin(a)/a with
 * a = k * chord / 2, expanded to a^6 (the remainder is below 1e-10 for
 * single-row steps).
 *
 * FMA(a, b, c) is a * b + c with one rounding (fmaf / fma): the transport
 * and the update add their products that way, in the order written.
 */
#define CAT_(a, b) a##b
#define CAT(a, b) CAT_(a, b)
#define FN(name) CAT(name, SUF)

#define R0 ((REAL)0)
#define R1 ((REAL)1)
#define R2 ((REAL)2)
#define RH ((REAL)0.5)

static inline int FN(lt)(int i, int j)
{
    return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
}

/* Non-trivial entries of the transport Jacobian F = d(p2)/d(p1); the rest
 * is the identity.  F is upper triangular: y depends on s and w, z on s, t
 * and w, s on w. */
typedef struct {
    REAL ys, yw, zs, zt, zw, sw;
} FN(jac_t);

/* Propagate p, C from plane x1 to x2 = x1 + dx.  Returns 0 (and leaves
 * p, C untouched) when |sin(phi)| at either end of the step is not below
 * s_max: at the far end the track turns back before x2, at the near end an
 * update has pushed the state past the transport's domain (|s| >= 1 would
 * take the square root of a negative number). */
static int FN(propagate)(REAL* p, REAL* C, REAL dx, REAL curv, REAL s_max)
{
    REAL s = p[2], t = p[3], w = p[4];
    REAL k = curv * w;
    REAL s2 = FMA(k, dx, s);
    if (!(FABS(s) < s_max) || !(FABS(s2) < s_max)) return 0;
    REAL c1 = SQRT((R1 - s) * (R1 + s));
    REAL c2 = SQRT((R1 - s2) * (R1 + s2));
    REAL cc = c1 + c2;
    REAL icc = R1 / cc;                   /* one reciprocal for the three quotients by cc */
    REAL T = (s + s2) * icc;              /* dy/dx averaged over the step */
    REAL q = SQRT(FMA(T, T, R1));
    REAL L = dx * q;                      /* signed transverse chord */
    REAL a = RH * (k * L);
    REAL a2 = a * a;
    REAL g = FMA(a2, FMA(a2, FMA(a2, C_5_112, C_3_40), C_1_6), R1);   /* asin(a)/a */
    REAL S = L * g;                       /* transverse arc length */

    /* exact derivatives of (y2, z2, s2) */
    REAL Ts = FMA(T, s / c1 + s2 / c2, R2) * icc;
    REAL kdx = curv * dx;
    REAL Tw = (kdx * FMA(T, s2 / c2, R1)) * icc;
    REAL LT = dx * (T / q);               /* dL/dT */
    REAL G1 = FMA(a2, FMA(a2, FMA(a2, C_5_16, C_3_8), RH), R1);      /* dS/dL */
    REAL Sk = (L * (L * a)) * FMA(a2, FMA(a2, C_15_112, C_3_20), C_1_6);  /* dS/dk */
    FN(jac_t) F;
    F.ys = dx * Ts;
    F.yw = dx * Tw;
    F.zs = t * ((G1 * LT) * Ts);
    F.zt = S;
    F.zw = t * FMA(Sk, curv, (G1 * LT) * Tw);
    F.sw = kdx;

    /* B = F C (full 5x5), then C' = B F^T (lower triangle).  Each sum runs
     * over the non-zero F entries in increasing column order, every product
     * added by one fused multiply-add. */
    REAL B[5][5];
    for (int j = 0; j < 5; j++) {
        REAL cy = C[FN(lt)(0, j)], cz = C[FN(lt)(1, j)], cs = C[FN(lt)(2, j)];
        REAL ct = C[FN(lt)(3, j)], cw = C[FN(lt)(4, j)];
        B[0][j] = FMA(F.yw, cw, FMA(F.ys, cs, cy));
        B[1][j] = FMA(F.zw, cw, FMA(F.zt, ct, FMA(F.zs, cs, cz)));
        B[2][j] = FMA(F.sw, cw, cs);
        B[3][j] = ct;
        B[4][j] = cw;
    }
    for (int i = 0; i < 5; i++) {
        for (int j = 0; j <= i; j++) {
            REAL v;
            switch (j) {
            case 0: v = FMA(F.yw, B[i][4], FMA(F.ys, B[i][2], B[i][0])); break;
            case 1: v = FMA(F.zw, B[i][4], FMA(F.zt, B[i][3], FMA(F.zs, B[i][2], B[i][1]))); break;
            case 2: v = FMA(F.sw, B[i][4], B[i][2]); break;
            default: v = B[i][j]; break;
            }
            C[FN(lt)(i, j)] = v;
        }
    }
    p[0] = FMA(dx, T, p[0]);
    p[1] = FMA(t, S, p[1]);
    p[2] = s2;
    return 1;
}

/* Turn the frame: the state at plane *x of one sector frame is taken into
 * a frame turned by D (cos D = c, sin D = sd; a point (x, y) becomes
 * (x c - y sd, x sd + y c), the direction angle grows by D), at the plane
 * through the same point, which becomes *x.  Returns 0 (nothing changed)
 * when the direction would not point along +x in the new frame or
 * |sin(phi)| would reach s_max there.
 * Covariance: a change dy of y (at fixed plane) moves the point by
 * dy (-sd, c); sliding it back along the track onto the plane (transverse
 * arc dl = sd dy / cos') changes y by (c + sd sin'/cos') dy, z by
 * t sd / cos' dy and sin by k sd dy (k = curv w); a change ds of sin(phi)
 * turns the direction by ds / cos, so sin' changes by cos'/cos ds.
 * C' = J C J^T over those entries, the rest the identity. */
static int FN(rotate)(REAL* x, REAL* p, REAL* C, REAL c, REAL sd, REAL curv, REAL s_max)
{
    REAL y = p[0], s = p[2], t = p[3];
    REAL cs = SQRT((R1 - s) * (R1 + s));
    REAL s2 = s * c + cs * sd;
    REAL c2 = cs * c - s * sd;
    if (!(R0 < c2) || !(FABS(s2) < s_max)) return 0;
    REAL jyy = c + (sd * s2) / c2;
    REAL jzy = (t * sd) / c2;
    REAL jsy = (curv * p[4]) * sd;
    REAL jss = c2 / cs;
    /* B = J C (rows y, z, s change), then C' = B J^T */
    REAL B[5][5];
    for (int j = 0; j < 5; j++) {
        REAL cy = C[FN(lt)(0, j)], cz = C[FN(lt)(1, j)], cc = C[FN(lt)(2, j)];
        B[0][j] = jyy * cy;
        B[1][j] = cz + jzy * cy;
        B[2][j] = jsy * cy + jss * cc;
        B[3][j] = C[FN(lt)(3, j)];
        B[4][j] = C[FN(lt)(4, j)];
    }
    for (int i = 0; i < 5; i++) {
        for (int j = 0; j <= i; j++) {
            REAL v;
            switch (j) {
            case 0: v = jyy * B[i][0]; break;
            case 1: v = B[i][1] + jzy * B[i][0]; break;
            case 2: v = jsy * B[i][0] + jss * B[i][2]; break;
            default: v = B[i][j]; break;
            }
            C[FN(lt)(i, j)] = v;
        }
    }
    REAL x0 = *x;
    *x = x0 * c - y * sd;
    p[0] = x0 * sd + y * c;
    p[2] = s2;
    return 1;
}

/* chi2 of a measurement (my, mz) against the predicted state. */
static inline REAL FN(chi2_pred)(const REAL* p, const REAL* C, REAL my, REAL mz,
                          REAL sy2, REAL sz2)
{
    REAL r0 = my - p[0], r1 = mz - p[1];
    REAL S00 = C[0] + sy2, S10 = C[1], S11 = C[2] + sz2;
    REAL det = FMA(S00, S11, -(S10 * S10));
    REAL idet = R1 / det;
    REAL B00 = S11 * idet, B10 = -(S10 * idet), B11 = S00 * idet;
    return FMA(r1, FMA(B11, r1, B10 * r0), r0 * FMA(B10, r1, B00 * r0));
}

/* Kalman update with the measurement (my, mz); returns its chi2.  Every
 * sum of two products is one product and one fused multiply-add. */
static REAL FN(update)(REAL* p, REAL* C, REAL my, REAL mz, REAL sy2, REAL sz2)
{
    REAL r0 = my - p[0], r1 = mz - p[1];
    REAL S00 = C[0] + sy2, S10 = C[1], S11 = C[2] + sz2;
    REAL det = FMA(S00, S11, -(S10 * S10));
    REAL idet = R1 / det;
    REAL B00 = S11 * idet, B10 = -(S10 * idet), B11 = S00 * idet;
    REAL chi2 = FMA(r1, FMA(B11, r1, B10 * r0), r0 * FMA(B10, r1, B00 * r0));
    REAL A0[5], A1[5], K0[5], K1[5];
    for (int i = 0; i < 5; i++) {
        A0[i] = C[FN(lt)(i, 0)];
        A1[i] = C[FN(lt)(i, 1)];
    }
    for (int i = 0; i < 5; i++) {
        K0[i] = FMA(A1[i], B10, A0[i] * B00);
        K1[i] = FMA(A1[i], B11, A0[i] * B10);
    }
    for (int i = 0; i < 5; i++) {
        p[i] = p[i] + FMA(K1[i], r1, K0[i] * r0);
        for (int j = 0; j <= i; j++)
            C[FN(lt)(i, j)] = C[FN(lt)(i, j)] - FMA(K1[i], A1[j], K0[i] * A0[j]);
    }
    return chi2;
}

/* State from three points on consecutive-or-not planes: position of the
 * first, direction from the first to the third, q/pT = 0, diagonal
 * covariance. */
static void FN(init_state)(REAL* p, REAL* C, REAL x0, REAL y0, REAL z0,
                           REAL x2, REAL y2, REAL z2, REAL sy2, REAL sz2,
                           REAL css, REAL ctt, REAL cww)
{
    REAL dX = x2 - x0;
    REAL T0 = (y2 - y0) / dX;
    REAL q0 = SQRT(R1 + T0 * T0);
    p[0] = y0;
    p[1] = z0;
    p[2] = T0 / q0;
    p[3] = (z2 - z0) / (dX * q0);
    p[4] = 0;
    for (int i = 0; i < 15; i++) C[i] = 0;
    C[0] = sy2;
    C[2] = sz2;
    C[5] = css;
    C[9] = ctt;
    C[14] = cww;
}

/* Calibration of one raw cluster (refit).  side = +1 for z >= 0 sectors,
 * -1 otherwise.  th: vd scale, t0 [us], 7 radial and 7 azimuthal
 * coefficients over the basis (1, u, v, u^2, u v, v^2, w) with
 * u = (x - u_centre)/u_scale, v = y/(x tan_half), w = drift/drift_len. */
static void FN(calibrate)(const REAL* th, REAL xr, REAL yr, REAL zr, REAL sd,
                          REAL DL, REAL VD, REAL TH, REAL UC, REAL US,
                          REAL* xc, REAL* yc, REAL* zc)
{
    REAL d_raw = DL - sd * zr;
    REAL d = (R1 + th[0]) * (d_raw - VD * th[1]);
    *zc = sd * (DL - d);
    REAL u = (xr - UC) / US;
    REAL v = yr / (xr * TH);
    REAL w = d / DL;
    REAL b[7] = {R1, u, v, u * u, u * v, v * v, w};
    REAL dr = 0, drphi = 0;
    for (int j = 0; j < 7; j++) {
        dr = dr + th[2 + j] * b[j];
        drphi = drphi + th[9 + j] * b[j];
    }
    *xc = xr + dr;
    *yc = yr + drphi;
}

/* Forward refit of one track: calibrate, initialise from hits 0 and 2,
 * filter outwards through hits 1..n-1.  Returns 0 ok, 1 too few hits,
 * 2 propagation stop. */
static int FN(refit_track)(int n, const uint8_t* row, const REAL* y, const REAL* z,
                           REAL sd, const float* row_x, const orc_params* prm,
                           const orc_calib_model* cm, const REAL* th,
                           REAL* p, REAL* C, REAL* chi2_out)
{
    *chi2_out = 0;
    if (n < 3) return 1;
    REAL DL = (REAL)cm->drift_len, VD = (REAL)cm->vd, TH = (REAL)cm->tan_half;
    REAL UC = (REAL)cm->u_centre, US = (REAL)cm->u_scale;
    REAL sy2 = (REAL)prm->sigma_y2, sz2 = (REAL)prm->sigma_z2;
    REAL x0, y0, z0, x2, y2, z2, xp, xc, yc, zc;
    FN(calibrate)(th, (REAL)row_x[row[0]], y[0], z[0], sd, DL, VD, TH, UC, US, &x0, &y0, &z0);
    FN(calibrate)(th, (REAL)row_x[row[2]], y[2], z[2], sd, DL, VD, TH, UC, US, &x2, &y2, &z2);
    FN(init_state)(p, C, x0, y0, z0, x2, y2, z2, sy2, sz2, (REAL)prm->c_ss0,
                   (REAL)prm->c_tt0, (REAL)prm->c_ww0);
    REAL chi2 = 0;
    xp = x0;
    for (int i = 1; i < n; i++) {
        FN(calibrate)(th, (REAL)row_x[row[i]], y[i], z[i], sd, DL, VD, TH, UC, US, &xc, &yc, &zc);
        if (!FN(propagate)(p, C, xc - xp, (REAL)prm->curv, (REAL)prm->s_max)) {
            *chi2_out = chi2;
            return 2;
        }
        chi2 = chi2 + FN(update)(p, C, yc, zc, sy2, sz2);
        xp = xc;
    }
    *chi2_out = chi2;
    return 0;
}

#undef R0
#undef R1
#undef R2
#undef RH
#undef FN
#undef CAT
#undef CAT_
