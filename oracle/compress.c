/*
 * Oracle of the TPC cluster compression -- TEST INFRASTRUCTURE ONLY.
 *
 * Reading of the paper's section 6 (TPC data compression), steps 2 to 4:
 * clusters in an integer format with only the precision the detector
 * resolution needs (charge with a precision relative to its value), the
 * entropy of the cluster properties reduced by storing residuals to tracks
 * for clusters on tracks and position differences otherwise, and a standard
 * entropy coder (rANS here, one of the coders the paper names).  Everything
 * below is this project's reading, stated once in oracle.h.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* ---- float32 Kalman primitives (the tracker's transport and update) ---- */
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

/* ---- integer format ------------------------------------------------------ */

/* y or z in units of 2^-qbits cm, rounded to nearest, ties to even */
static int32_t quant(float v, float scale) { return (int32_t)rintf(v * scale); }

/* charge: rounded to an integer count in [0, 65535], then only its leading
 * cbits significant bits are kept: values below 2^cbits exactly, larger
 * ones as (exponent, mantissa) with the mantissa's leading one implied.
 * code = v for v < 2^cbits, else 2^cbits + (e - 1) 2^(cbits-1) + (m - 2^(cbits-1))
 * with e = bitlength(v) - cbits and m = v >> e. */
static int charge_code(float charge, int cbits)
{
    float r = rintf(charge);
    uint32_t v = r < 0.0f ? 0u : r > 65535.0f ? 65535u : (uint32_t)r;
    uint32_t top = 1u << cbits;
    if (v < top) return (int)v;
    int e = 0;
    while ((v >> e) >= top) e++;
    uint32_t half = top >> 1;
    return (int)(top + (uint32_t)(e - 1) * half + ((v >> e) - half));
}

int orc_charge_decode(int code, int cbits)
{
    int top = 1 << cbits, half = top >> 1;
    if (code < top) return code;
    int e = (code - top) / half + 1;
    int m = (code - top) % half + half;
    return (m << e) + (1 << (e - 1));
}

/* ---- symbol streams -------------------------------------------------------
 * Byte symbols; a value that does not fit goes out as the escape symbol 255
 * and its 32-bit value on the stream's escape list. */
enum { S_LEN, S_ROW, S_DY, S_DZ, S_Q, S_UN, S_UDZ, S_UYH, S_UYL, N_STREAMS };

typedef struct {
    uint8_t* sym;
    int64_t n, cap;
    int32_t* esc;
    int64_t n_esc;
} stream;

static void put(stream* s, uint32_t v, int32_t raw)
{
    if (v < 255u) {
        s->sym[s->n++] = (uint8_t)v;
    } else {
        s->sym[s->n++] = 255;
        s->esc[s->n_esc++] = raw;
    }
}

/* a byte symbol without escape (all 256 values are data) */
static void put_byte(stream* s, uint32_t v) { s->sym[s->n++] = (uint8_t)v; }

static uint32_t zigzag(int32_t d) { return ((uint32_t)d << 1) ^ (uint32_t)(d >> 31); }
static int32_t unzigzag(uint32_t u) { return (int32_t)(u >> 1) ^ -(int32_t)(u & 1u); }

/* ---- rANS (32-bit state, byte output, 12-bit probabilities) --------------
 * State x in [L, 256 L), L = 2^23.  Encoding a symbol of frequency f and
 * cumulative frequency c: while x >= (L / 2^12) * 256 * f emit the low byte
 * and shift; then x = (x / f) 2^12 + x mod f + c.  Symbols are encoded last
 * to first so that the decoder reads them first to last. */
#define RANS_L (1u << 23)
#define PROB_BITS 12
#define PROB_SCALE (1u << PROB_BITS)

/* counts -> frequencies summing to 2^12, every symbol present at least 1:
 * f = max(1, floor(count 2^12 / total)); then the sum is brought to 2^12 one
 * unit at a time, down on the largest frequency above 1 (ties to the lower
 * symbol), up on the largest count (ties to the lower symbol). */
static void normalise(const uint64_t* cnt, uint32_t* f)
{
    uint64_t total = 0;
    for (int i = 0; i < 256; i++) total += cnt[i];
    uint32_t sum = 0;
    for (int i = 0; i < 256; i++) {
        f[i] = 0;
        if (cnt[i]) {
            uint64_t v = cnt[i] * PROB_SCALE / total;
            f[i] = v ? (uint32_t)v : 1u;
            sum += f[i];
        }
    }
    if (!total) return;
    while (sum > PROB_SCALE) {
        int b = -1;
        for (int i = 0; i < 256; i++)
            if (f[i] > 1 && (b < 0 || f[i] > f[b])) b = i;
        f[b]--;
        sum--;
    }
    while (sum < PROB_SCALE) {
        int b = -1;
        for (int i = 0; i < 256; i++)
            if (cnt[i] && (b < 0 || cnt[i] > cnt[b])) b = i;
        f[b]++;
        sum++;
    }
}

/* encode n symbols; writes the bytes to out (first byte first) and returns
 * their count (at most 2 n + 4) */
static int64_t rans_encode(const uint8_t* s, int64_t n, const uint32_t* f, const uint32_t* c,
                           uint8_t* tmp, uint8_t* out)
{
    int64_t k = 0;            /* bytes emitted, last byte of the stream first */
    uint32_t x = RANS_L;
    for (int64_t i = n - 1; i >= 0; i--) {
        uint32_t fs = f[s[i]];
        uint32_t x_max = ((RANS_L >> PROB_BITS) << 8) * fs;
        while (x >= x_max) {
            tmp[k++] = (uint8_t)(x & 255u);
            x >>= 8;
        }
        x = ((x / fs) << PROB_BITS) + (x % fs) + c[s[i]];
    }
    for (int b = 0; b < 4; b++) {
        tmp[k++] = (uint8_t)(x & 255u);
        x >>= 8;
    }
    for (int64_t i = 0; i < k; i++) out[i] = tmp[k - 1 - i];
    return k;
}

static int64_t rans_decode(const uint8_t* in, int64_t n_bytes, int64_t n, const uint32_t* f,
                           const uint32_t* c, uint8_t* s)
{
    uint8_t slot2sym[PROB_SCALE];
    for (int i = 0; i < 256; i++)
        for (uint32_t j = 0; j < f[i]; j++) slot2sym[c[i] + j] = (uint8_t)i;
    int64_t k = 0;
    uint32_t x = 0;
    for (int b = 0; b < 4; b++) x = (x << 8) | in[k++];
    for (int64_t i = 0; i < n; i++) {
        uint32_t slot = x & (PROB_SCALE - 1u);
        uint8_t sy = slot2sym[slot];
        s[i] = sy;
        x = f[sy] * (x >> PROB_BITS) + slot - c[sy];
        while (x < RANS_L) {
            if (k >= n_bytes) return -1;
            x = (x << 8) | in[k++];
        }
    }
    return k;
}

int64_t orc_rans_roundtrip(const uint8_t* sym, int64_t n, uint8_t* bytes, uint8_t* back)
{
    uint64_t cnt[256] = {0};
    uint32_t f[256], c[256];
    for (int64_t i = 0; i < n; i++) cnt[sym[i]]++;
    normalise(cnt, f);
    c[0] = 0;
    for (int i = 1; i < 256; i++) c[i] = c[i - 1] + f[i - 1];
    uint8_t* tmp = malloc((size_t)(2 * n + 8));
    int64_t nb = rans_encode(sym, n, f, c, tmp, bytes);
    free(tmp);
    if (rans_decode(bytes, nb, n, f, c, back) < 0) return -1;
    return nb;
}

/* ---- blob ----------------------------------------------------------------
 * Little-endian.  Header: magic "TPCZ", version, cbits, qbits, chunk,
 * n_sectors, n_rows (u32), then n_clusters, n_tracks, n_attached,
 * n_unattached (u64) and per stream (track lengths, row steps, y and z
 * residuals, charges, row counts of the other clusters, their z steps, y
 * high and low bytes):
 * n_symbols, n_escapes (u64), n_chunks (u32), 256 u16 frequencies, the
 * chunks' byte counts (u32 each).  Payload: every stream's chunk bytes,
 * stream by stream; every stream's escapes (i32); the track headers (16 B:
 * row, 0, s, t, w as i16 at 2^-14, 2^-14, 2^-10, y, z as i32 at 2^-qbits). */
typedef struct {
    uint8_t* p;
    int64_t n, cap;
} wbuf;

static void wb(wbuf* b, const void* v, int64_t n)
{
    if (b->n + n <= b->cap) memcpy(b->p + b->n, v, (size_t)n);
    b->n += n;
}
static void w32(wbuf* b, uint32_t v) { wb(b, &v, 4); }
static void w64(wbuf* b, uint64_t v) { wb(b, &v, 8); }

static int16_t q16(float v, float scale)
{
    float r = rintf(v * scale);
    return (int16_t)(r < -32767.0f ? -32767.0f : r > 32767.0f ? 32767.0f : r);
}

/* the predictor of a track: its tracklet state rounded to the header's
 * precision at the plane of its innermost row, initial covariance */
static void track_state(const uint8_t* hdr, const float* row_x, const orc_params* prm,
                        float inv_q, float* p, float* C, float* x)
{
    int16_t s, t, w;
    int32_t yq, zq;
    memcpy(&s, hdr + 2, 2);
    memcpy(&t, hdr + 4, 2);
    memcpy(&w, hdr + 6, 2);
    memcpy(&yq, hdr + 8, 4);
    memcpy(&zq, hdr + 12, 4);
    p[0] = (float)yq / inv_q;
    p[1] = (float)zq / inv_q;
    p[2] = (float)s / 16384.0f;
    p[3] = (float)t / 16384.0f;
    p[4] = (float)w / 1024.0f;
    for (int i = 0; i < 15; i++) C[i] = 0.0f;
    C[0] = prm->sigma_y2;
    C[2] = prm->sigma_z2;
    C[5] = prm->c_ss0;
    C[9] = prm->c_tt0;
    C[14] = prm->c_ww0;
    *x = row_x[hdr[0]];
}

int64_t orc_compress(int n_sec, const orc_sector* sec, int n_rows, const float* row_x,
                     const orc_params* prm, const uint8_t* row, const float* y, const float* z,
                     const float* charge, int64_t n_clusters, const int* bin_start,
                     const int* idg, int64_t n_tracks, const int* trk_off, const int* trk_hits,
                     const float* tpar, const int* trin, const orc_cmp_params* cp,
                     uint8_t* out, int64_t out_cap)
{
    const float inv_q = ldexpf(1.0f, cp->qbits);
    const int64_t n_att = n_tracks > 0 ? trk_off[n_tracks] : 0;
    uint8_t* on = calloc((size_t)(n_clusters > 0 ? n_clusters : 1), 1);
    for (int64_t k = 0; k < n_att; k++) on[trk_hits[k]] = 1;
    int64_t n_un = 0;
    for (int64_t i = 0; i < n_clusters; i++) n_un += !on[i];
    int64_t n_rowseg = (int64_t)n_sec * n_rows;
    stream st[N_STREAMS];
    int64_t cap[N_STREAMS] = {n_tracks, n_att, n_att, n_att, n_att + n_un, n_rowseg,
                              n_un,     n_un,  n_un};
    for (int k = 0; k < N_STREAMS; k++) {
        st[k].cap = cap[k];
        st[k].n = st[k].n_esc = 0;
        st[k].sym = malloc((size_t)(cap[k] > 0 ? cap[k] : 1));
        st[k].esc = malloc(sizeof(int32_t) * (size_t)(cap[k] > 0 ? cap[k] : 1));
    }
    uint8_t* hdr = calloc((size_t)(n_tracks > 0 ? n_tracks : 1), 16);
    /* clusters on tracks: row step, residuals to the track's prediction,
     * charge; the prediction follows the decoded clusters (a Kalman filter
     * the decoder repeats) */
    for (int64_t k = 0; k < n_tracks; k++) {
        uint8_t* h = hdr + 16 * k;
        const float* q = tpar + 5 * k;
        h[0] = (uint8_t)trin[k];
        int16_t s = q16(q[2], 16384.0f), t = q16(q[3], 16384.0f), w = q16(q[4], 1024.0f);
        int32_t yq = quant(q[0], inv_q), zq = quant(q[1], inv_q);
        memcpy(h + 2, &s, 2);
        memcpy(h + 4, &t, 2);
        memcpy(h + 6, &w, 2);
        memcpy(h + 8, &yq, 4);
        memcpy(h + 12, &zq, 4);
        float p[5], C[15], x;
        track_state(h, row_x, prm, inv_q, p, C, &x);
        int nh = trk_off[k + 1] - trk_off[k];
        put(&st[S_LEN], (uint32_t)nh, nh);
        int alive = 1, prow = h[0];
        for (int j = trk_off[k]; j < trk_off[k + 1]; j++) {
            int c = trk_hits[j], r = row[c];
            put(&st[S_ROW], (uint32_t)(r - prow), r - prow);
            prow = r;
            int32_t cy = quant(y[c], inv_q), cz = quant(z[c], inv_q);
            if (alive && !propagate_f(p, C, row_x[r] - x, prm->curv, prm->s_max)) alive = 0;
            int32_t py = alive ? quant(p[0], inv_q) : 0, pz = alive ? quant(p[1], inv_q) : 0;
            put(&st[S_DY], zigzag(cy - py), cy - py);
            put(&st[S_DZ], zigzag(cz - pz), cz - pz);
            if (alive) {
                update_f(p, C, (float)cy / inv_q, (float)cz / inv_q, prm->sigma_y2,
                         prm->sigma_z2);
                x = row_x[r];
            }
            put(&st[S_Q], (uint32_t)charge_code(charge[c], cp->cbits), 0);
        }
    }
    /* the other clusters, row by row in grid order: count, z difference to
     * the previous one of the row, y (offset by 2048, high and low byte) */
    for (int s = 0; s < n_sec; s++) {
        const orc_sector* se = &sec[s];
        int per_row = se->nbz * se->nby;
        for (int r = 0; r < n_rows; r++) {
            int p0 = bin_start[se->bin_base + r * per_row];
            int p1 = bin_start[se->bin_base + (r + 1) * per_row];
            int cnt = 0;
            for (int g = p0; g < p1; g++) cnt += !on[idg[g]];
            put(&st[S_UN], (uint32_t)cnt, cnt);
            int32_t pz = 0;
            for (int g = p0; g < p1; g++) {
                int c = idg[g];
                if (on[c]) continue;
                int32_t cz = quant(z[c], inv_q), cy = quant(y[c], inv_q);
                put(&st[S_UDZ], zigzag(cz - pz), cz - pz);
                pz = cz;
                int32_t yo = cy + 2048;
                if (yo >= 0 && yo < 4096) {
                    put(&st[S_UYH], (uint32_t)(yo >> 8), 0);
                    put_byte(&st[S_UYL], (uint32_t)(yo & 255));
                } else {
                    put(&st[S_UYH], 255u, cy);
                    put_byte(&st[S_UYL], 0u);
                }
                put(&st[S_Q], (uint32_t)charge_code(charge[c], cp->cbits), 0);
            }
        }
    }
    /* tables and chunks */
    wbuf b = {out, 0, out_cap};
    w32(&b, 0x5a435054u);   /* "TPCZ" */
    w32(&b, 1u);
    w32(&b, (uint32_t)cp->cbits);
    w32(&b, (uint32_t)cp->qbits);
    w32(&b, (uint32_t)cp->chunk);
    w32(&b, (uint32_t)n_sec);
    w32(&b, (uint32_t)n_rows);
    w64(&b, (uint64_t)n_clusters);
    w64(&b, (uint64_t)n_tracks);
    w64(&b, (uint64_t)n_att);
    w64(&b, (uint64_t)n_un);
    uint32_t f[N_STREAMS][256], cum[N_STREAMS][256];
    int64_t nch[N_STREAMS];
    uint8_t** cbytes[N_STREAMS];
    int64_t* csize[N_STREAMS];
    uint8_t* tmp = malloc((size_t)(2 * cp->chunk + 8));
    for (int k = 0; k < N_STREAMS; k++) {
        uint64_t cnt[256] = {0};
        for (int64_t i = 0; i < st[k].n; i++) cnt[st[k].sym[i]]++;
        normalise(cnt, f[k]);
        cum[k][0] = 0;
        for (int i = 1; i < 256; i++) cum[k][i] = cum[k][i - 1] + f[k][i - 1];
        nch[k] = (st[k].n + cp->chunk - 1) / cp->chunk;
        cbytes[k] = malloc(sizeof(uint8_t*) * (size_t)(nch[k] > 0 ? nch[k] : 1));
        csize[k] = malloc(sizeof(int64_t) * (size_t)(nch[k] > 0 ? nch[k] : 1));
        for (int64_t j = 0; j < nch[k]; j++) {
            int64_t a = j * cp->chunk, e = a + cp->chunk < st[k].n ? a + cp->chunk : st[k].n;
            cbytes[k][j] = malloc((size_t)(2 * (e - a) + 8));
            csize[k][j] = rans_encode(st[k].sym + a, e - a, f[k], cum[k], tmp, cbytes[k][j]);
        }
        w64(&b, (uint64_t)st[k].n);
        w64(&b, (uint64_t)st[k].n_esc);
        w32(&b, (uint32_t)nch[k]);
        for (int i = 0; i < 256; i++) {
            uint16_t v = (uint16_t)(f[k][i] == PROB_SCALE ? 0xffffu : f[k][i]);
            wb(&b, &v, 2);
        }
        for (int64_t j = 0; j < nch[k]; j++) w32(&b, (uint32_t)csize[k][j]);
    }
    for (int k = 0; k < N_STREAMS; k++)
        for (int64_t j = 0; j < nch[k]; j++) wb(&b, cbytes[k][j], csize[k][j]);
    for (int k = 0; k < N_STREAMS; k++) wb(&b, st[k].esc, 4 * st[k].n_esc);
    wb(&b, hdr, 16 * n_tracks);
    for (int k = 0; k < N_STREAMS; k++) {
        for (int64_t j = 0; j < nch[k]; j++) free(cbytes[k][j]);
        free(cbytes[k]);
        free(csize[k]);
        free(st[k].sym);
        free(st[k].esc);
    }
    free(tmp);
    free(hdr);
    free(on);
    return b.n <= out_cap ? b.n : -b.n;
}

/* ---- decoder -------------------------------------------------------------
 * Clusters in blob order: those on tracks track by track (track index and
 * the row of every hit from the row steps), then the others sector by
 * sector and row by row (track -1).  Returns the cluster count, or -1 on a
 * malformed blob or too small a capacity. */
typedef struct {
    const uint8_t* p;
    int64_t n, k;
} rbuf;

static int rb(rbuf* b, void* v, int64_t n)
{
    if (n < 0 || b->k + n > b->n) return 0;
    memcpy(v, b->p + b->k, (size_t)n);
    b->k += n;
    return 1;
}

typedef struct {
    uint8_t* sym;
    int32_t* esc;
    int64_t n, n_esc, pos, epos;
} rstream;

static int get(rstream* s, int32_t* v)
{
    if (s->pos >= s->n) return 0;
    uint8_t c = s->sym[s->pos++];
    if (c < 255) {
        *v = c;
        return 1;
    }
    if (s->epos >= s->n_esc) return 0;
    *v = s->esc[s->epos++];
    return 1;
}

int64_t orc_decompress(const uint8_t* blob, int64_t size, const float* row_x,
                       const orc_params* prm, uint8_t* o_row, int32_t* o_yq, int32_t* o_zq,
                       int32_t* o_qcode, int32_t* o_track, int32_t* o_sector, int64_t cap)
{
    rbuf b = {blob, size, 0};
    uint32_t magic, ver, cbits, qbits, chunk, n_sec, n_rows;
    uint64_t n_cl, n_tr, n_att, n_un;
    if (!rb(&b, &magic, 4) || magic != 0x5a435054u || !rb(&b, &ver, 4) || !rb(&b, &cbits, 4) ||
        !rb(&b, &qbits, 4) || !rb(&b, &chunk, 4) || !rb(&b, &n_sec, 4) || !rb(&b, &n_rows, 4) ||
        !rb(&b, &n_cl, 8) || !rb(&b, &n_tr, 8) || !rb(&b, &n_att, 8) || !rb(&b, &n_un, 8))
        return -1;
    if ((int64_t)n_cl > cap || n_att + n_un != n_cl || chunk == 0) return -1;
    (void)cbits;
    (void)ver;
    const float inv_q = ldexpf(1.0f, (int)qbits);
    uint64_t nsym[N_STREAMS], nesc[N_STREAMS];
    uint32_t nch[N_STREAMS], f[N_STREAMS][256], cum[N_STREAMS][256];
    uint32_t* csz[N_STREAMS] = {0};
    rstream rs[N_STREAMS];
    memset(rs, 0, sizeof rs);
    int64_t ret = -1;
    for (int k = 0; k < N_STREAMS; k++) {
        if (!rb(&b, &nsym[k], 8) || !rb(&b, &nesc[k], 8) || !rb(&b, &nch[k], 4)) goto done;
        for (int i = 0; i < 256; i++) {
            uint16_t v;
            if (!rb(&b, &v, 2)) goto done;
            f[k][i] = v == 0xffffu ? PROB_SCALE : v;
        }
        cum[k][0] = 0;
        for (int i = 1; i < 256; i++) cum[k][i] = cum[k][i - 1] + f[k][i - 1];
        csz[k] = malloc(sizeof(uint32_t) * (nch[k] ? nch[k] : 1));
        for (uint32_t j = 0; j < nch[k]; j++)
            if (!rb(&b, &csz[k][j], 4)) goto done;
    }
    for (int k = 0; k < N_STREAMS; k++) {
        rs[k].n = (int64_t)nsym[k];
        rs[k].n_esc = (int64_t)nesc[k];
        rs[k].sym = malloc((size_t)(nsym[k] ? nsym[k] : 1));
        for (uint32_t j = 0; j < nch[k]; j++) {
            int64_t a = (int64_t)j * chunk;
            int64_t e = a + chunk < (int64_t)nsym[k] ? a + chunk : (int64_t)nsym[k];
            if (b.k + csz[k][j] > b.n ||
                rans_decode(b.p + b.k, csz[k][j], e - a, f[k], cum[k], rs[k].sym + a) < 0)
                goto done;
            b.k += csz[k][j];
        }
    }
    for (int k = 0; k < N_STREAMS; k++) {
        rs[k].esc = malloc(4 * (size_t)(nesc[k] ? nesc[k] : 1));
        if (!rb(&b, rs[k].esc, 4 * (int64_t)nesc[k])) goto done;
    }
    if (b.k + 16 * (int64_t)n_tr != b.n) goto done;
    const uint8_t* hdr = b.p + b.k;
    int64_t m = 0;
    for (uint64_t k = 0; k < n_tr; k++) {
        float p[5], C[15], x;
        track_state(hdr + 16 * k, row_x, prm, inv_q, p, C, &x);
        int32_t nh, r = hdr[16 * k];
        if (!get(&rs[S_LEN], &nh)) goto done;
        int alive = 1;
        for (int32_t j = 0; j < nh; j++) {
            int32_t dr, uy, uz, qc;
            if (!get(&rs[S_ROW], &dr) || !get(&rs[S_DY], &uy) || !get(&rs[S_DZ], &uz) ||
                !get(&rs[S_Q], &qc) || m >= (int64_t)n_att)
                goto done;
            r += dr;
            if (r < 0 || r >= 256) goto done;
            if (alive && !propagate_f(p, C, row_x[r] - x, prm->curv, prm->s_max)) alive = 0;
            int32_t py = alive ? quant(p[0], inv_q) : 0, pz = alive ? quant(p[1], inv_q) : 0;
            /* escaped residuals carry the value itself */
            int32_t dy = rs[S_DY].sym[rs[S_DY].pos - 1] == 255 ? uy : unzigzag((uint32_t)uy);
            int32_t dz = rs[S_DZ].sym[rs[S_DZ].pos - 1] == 255 ? uz : unzigzag((uint32_t)uz);
            int32_t cy = py + dy, cz = pz + dz;
            if (alive) {
                update_f(p, C, (float)cy / inv_q, (float)cz / inv_q, prm->sigma_y2,
                         prm->sigma_z2);
                x = row_x[r];
            }
            o_row[m] = (uint8_t)r;
            o_yq[m] = cy;
            o_zq[m] = cz;
            o_qcode[m] = qc;
            o_track[m] = (int32_t)k;
            o_sector[m] = -1;
            m++;
        }
    }
    for (uint32_t s = 0; s < n_sec; s++)
        for (uint32_t r = 0; r < n_rows; r++) {
            int32_t cnt, pz = 0;
            if (!get(&rs[S_UN], &cnt)) goto done;
            for (int32_t i = 0; i < cnt; i++) {
                int32_t uz, yh, yl, qc;
                if (!get(&rs[S_UDZ], &uz) || !get(&rs[S_UYH], &yh) ||
                    rs[S_UYL].pos >= rs[S_UYL].n || !get(&rs[S_Q], &qc) || m >= (int64_t)n_cl)
                    goto done;
                yl = rs[S_UYL].sym[rs[S_UYL].pos++];
                int32_t dz = rs[S_UDZ].sym[rs[S_UDZ].pos - 1] == 255 ? uz
                                                                     : unzigzag((uint32_t)uz);
                pz += dz;
                int32_t cy = rs[S_UYH].sym[rs[S_UYH].pos - 1] == 255 ? yh
                                                                     : ((yh << 8) | yl) - 2048;
                o_row[m] = (uint8_t)r;
                o_yq[m] = cy;
                o_zq[m] = pz;
                o_qcode[m] = qc;
                o_track[m] = -1;
                o_sector[m] = (int32_t)s;
                m++;
            }
        }
    ret = m == (int64_t)n_cl ? m : -1;
done:
    for (int k = 0; k < N_STREAMS; k++) {
        free(csz[k]);
        free(rs[k].sym);
        free(rs[k].esc);
    }
    return ret;
}
