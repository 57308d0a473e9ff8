// TPC cluster compression (section 6, steps 2 to 4): the clusters in an
// integer format with only the precision the resolution needs, the entropy
// of their properties reduced by residuals to tracks for clusters on tracks
// and position differences otherwise, and an entropy coder (rANS, one of the
// coders the paper names).
//
// Integer format: y, z rounded to 2^-qbits cm; the charge rounded to a count
// in [0, 65535] keeping its cbits leading significant bits.  Nine byte
// streams (255 escapes a 32-bit value on the stream's escape list):
//   clusters on tracks, track by track: the hit count, the row step, the y
//   and z residuals (zigzag) to the track's prediction -- its tracklet state
//   rounded into a 16-byte header, carried row by row with the tracklet
//   transport and updated with each cluster as decoded, so that a decoder
//   repeats it -- and the charge code;
//   the other clusters, sector by sector and row by row in grid order: the
//   count per row, the z step to the previous one of the row, y (offset
//   2048) as a high and a low byte, and the charge code after the tracks'.
// Each stream is rANS coded (32-bit state, byte output, 12-bit table of its
// own) in chunks of `chunk` symbols, one thread per chunk.
//
// Kernels: mark the clusters on tracks; one thread per track writes its
// header and symbols; one wave per (sector, row) counts, then (after a
// scan) writes the other clusters' symbols; per-stream histograms in LDS;
// one block per stream normalises its table; one thread per chunk encodes
// backwards into the end of its chunk slot; scans order the escapes; one
// block lays out the blob; copies place chunks, escapes and headers.
#include "block_dev.hpp"
#include "tracklet_dev.hpp"

namespace tpc {

namespace {

constexpr int kStreams = 9;
enum { S_LEN, S_ROW, S_DY, S_DZ, S_Q, S_UN, S_UDZ, S_UYH, S_UYL };
constexpr uint32_t kRansL = 1u << 23;
constexpr int kProbBits = 12;
constexpr uint32_t kProbScale = 1u << kProbBits;
constexpr int kHeaderFixed = 7 * 4 + 4 * 8;
constexpr int kStreamHeader = 8 + 8 + 4 + 256 * 2;

struct CmpWs {
    uint8_t* on;            // [n_clusters] cluster on a track
    uint8_t* sym[kStreams];  // [cap_k] symbols
    int32_t* esc[kStreams];  // [cap_k] escaped value at an escape's position
    int32_t* eflag;         // [max cap] escape flags of one stream, then positions
    int32_t* rowcnt;        // [n_rowseg + 1] other clusters per (sector, row), then offsets
    uint8_t* hdr;           // [track cap * 16]
    uint32_t* hist;         // [kStreams * 256]
    uint32_t* freq;         // [kStreams * 256]
    uint32_t* cum;          // [kStreams * 256]
    uint8_t* cbuf;          // [kStreams][chunk cap][slot] encoded chunks
    uint32_t* csize;        // [kStreams * chunk cap] encoded bytes per chunk
    int64_t* coff;          // [kStreams * chunk cap] blob offset of each chunk's bytes
    int64_t* counts;        // [16]: n_tracks, n_att, n_un, stream sizes, escape counts
    int64_t* eoff;          // [kStreams + 1] escape counts (scan totals)
    int64_t* lay;           // [kStreams * 3 + 4] blob offsets (chunk data, escapes, headers)
    int64_t* partials;      // scan partials
    int64_t cap[kStreams];
    int64_t chunk_cap;      // chunks per stream, at most
    int64_t slot;           // bytes per chunk slot
    int64_t n_rowseg;
};

__device__ __forceinline__ int32_t quant(float v, float scale) { return (int32_t)rintf(v * scale); }

__device__ __forceinline__ int16_t q16(float v, float scale)
{
    const float r = rintf(v * scale);
    return (int16_t)(r < -32767.0f ? -32767.0f : r > 32767.0f ? 32767.0f : r);
}

__device__ __forceinline__ uint32_t charge_code(float charge, int cbits)
{
    const float r = rintf(charge);
    const uint32_t v = r < 0.0f ? 0u : r > 65535.0f ? 65535u : (uint32_t)r;
    const uint32_t top = 1u << cbits;
    if (v < top) return v;
    int e = 0;
    while ((v >> e) >= top) ++e;
    const uint32_t half = top >> 1;
    return top + (uint32_t)(e - 1) * half + ((v >> e) - half);
}

__device__ __forceinline__ uint32_t zigzag(int32_t d)
{
    return ((uint32_t)d << 1) ^ (uint32_t)(d >> 31);
}

// symbol v at position i of stream k; 255 and the raw value when v >= 255
__device__ __forceinline__ void put(const CmpWs& w, int k, int64_t i, uint32_t v, int32_t raw)
{
    if (v < 255u) {
        w.sym[k][i] = (uint8_t)v;
    } else {
        w.sym[k][i] = 255;
        w.esc[k][i] = raw;
    }
}

__device__ __forceinline__ int64_t track_count(const int64_t* d_n_tracks, int64_t cap)
{
    const int64_t n = *d_n_tracks;
    return n < cap ? n : cap;
}

__global__ __launch_bounds__(kBlock) void k_cz_mark(const int32_t* __restrict__ off,
                                                    const int32_t* __restrict__ hits,
                                                    const int64_t* __restrict__ d_n_tracks,
                                                    int64_t cap, CmpWs w)
{
    const int64_t nt = track_count(d_n_tracks, cap);
    const int64_t na = nt > 0 ? off[nt] : 0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < na;
         j += (int64_t)gridDim.x * blockDim.x)
        w.on[hits[j]] = 1;
}

// one thread per track: header, hit count, row steps, residuals, charges.
// A hit's row, y and z come from the track-ordered copies where the tracks
// carry them (contiguous per track), else through the cluster index; the
// next hit's values are loaded while the current one is filtered.
__global__ __launch_bounds__(kBlock) void k_cz_tracks(
    const float* __restrict__ row_x, tpc_params prm, const uint8_t* __restrict__ row,
    const float* __restrict__ y, const float* __restrict__ z, const float* __restrict__ charge,
    const int32_t* __restrict__ off, const int32_t* __restrict__ hits,
    const uint8_t* __restrict__ h_row, const float* __restrict__ h_y,
    const float* __restrict__ h_z, const int32_t* __restrict__ trk_tracklet,
    const float* __restrict__ t_par, const int32_t* __restrict__ t_rin,
    const int64_t* __restrict__ d_n_tracks, int64_t cap, float inv_q, int cbits, CmpWs w)
{
    const bool copies = h_row != nullptr;
    const int64_t nt = track_count(d_n_tracks, cap);
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nt;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t tk = trk_tracklet[k];
        const float* q = t_par + (int64_t)tk * 5;
        const int rin = t_rin[tk];
        const int16_t s = q16(q[2], 16384.0f), t = q16(q[3], 16384.0f), wq = q16(q[4], 1024.0f);
        const int32_t yq = quant(q[0], inv_q), zq = quant(q[1], inv_q);
        uint8_t* h = w.hdr + k * 16;
        h[0] = (uint8_t)rin;
        h[1] = 0;
        memcpy(h + 2, &s, 2);
        memcpy(h + 4, &t, 2);
        memcpy(h + 6, &wq, 2);
        memcpy(h + 8, &yq, 4);
        memcpy(h + 12, &zq, 4);
        // the predictor, as the decoder builds it from the header
        KState st;
        st.p[0] = (float)yq / inv_q;
        st.p[1] = (float)zq / inv_q;
        st.p[2] = (float)s / 16384.0f;
        st.p[3] = (float)t / 16384.0f;
        st.p[4] = (float)wq / 1024.0f;
        reset_cov(st, prm);
        float x = row_x[(uint8_t)rin];
        const int a = off[k], b = off[k + 1];
        put(w, S_LEN, k, (uint32_t)(b - a), b - a);
        bool alive = true;
        int prow = (uint8_t)rin;
        int r_n = 0;
        float y_n = 0.0f, z_n = 0.0f, q_n = 0.0f, x_n = 0.0f;
        auto fetch = [&](int jj) {
            const int c = hits[jj];
            if (copies) {
                r_n = h_row[jj];
                y_n = h_y[jj];
                z_n = h_z[jj];
            } else {
                r_n = row[c];
                y_n = y[c];
                z_n = z[c];
            }
            q_n = charge[c];
            x_n = row_x[r_n];
        };
        if (a < b) fetch(a);
        for (int j = a; j < b; ++j) {
            const int r = r_n;
            const float yc = y_n, zc = z_n, qc = q_n, xr = x_n;
            if (j + 1 < b) fetch(j + 1);
            put(w, S_ROW, j, (uint32_t)(r - prow), r - prow);
            prow = r;
            const int32_t cy = quant(yc, inv_q), cz = quant(zc, inv_q);
            if (alive && !propagate(st, xr - x, prm.curv, prm.s_max)) alive = false;
            const int32_t py = alive ? quant(st.p[0], inv_q) : 0;
            const int32_t pz = alive ? quant(st.p[1], inv_q) : 0;
            put(w, S_DY, j, zigzag(cy - py), cy - py);
            put(w, S_DZ, j, zigzag(cz - pz), cz - pz);
            if (alive) {
                kupdate(st, (float)cy / inv_q, (float)cz / inv_q, prm.sigma_y2, prm.sigma_z2);
                x = xr;
            }
            w.sym[S_Q][j] = (uint8_t)charge_code(qc, cbits);
        }
    }
}

// One wave per (sector, row): the row's grid positions 64 at a time, the
// clusters on no track found by a ballot.  (One thread per row walking its
// positions took 0.13 + 0.35 ms on the central event.)
__global__ __launch_bounds__(kBlock) void k_cz_rowcount(const tpc_sector* __restrict__ sec,
                                                        int n_sec, int n_rows,
                                                        const int32_t* __restrict__ bin_start,
                                                        const int32_t* __restrict__ idg, CmpWs w)
{
    const int64_t n = (int64_t)n_sec * n_rows;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t i = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; i < n;
         i += waves) {
        const tpc_sector& s = sec[i / n_rows];
        const int r = (int)(i % n_rows);
        const int per_row = s.nbz * s.nby;
        const int p0 = bin_start[s.bin_base + r * per_row];
        const int p1 = bin_start[s.bin_base + (r + 1) * per_row];
        int cnt = 0;
        for (int g0 = p0; g0 < p1; g0 += kWave) {
            const int g = g0 + lane;
            cnt += __popcll(__ballot(g < p1 && !w.on[idg[g]]));
        }
        if (lane == 0) {
            w.rowcnt[i] = cnt;
            put(w, S_UN, i, (uint32_t)cnt, cnt);
        }
    }
}

// one wave per (sector, row): z steps, y bytes and charges of the row's
// clusters on no track, at the row's offset, in grid order (each one's z
// step is to the previous one of the row: a lane takes it from the lane of
// the previous such cluster, the first of a round from the round before)
__global__ __launch_bounds__(kBlock) void k_cz_rowemit(
    const tpc_sector* __restrict__ sec, int n_sec, int n_rows, const int32_t* __restrict__ bin_start,
    const int32_t* __restrict__ idg, const float* __restrict__ y, const float* __restrict__ z,
    const float* __restrict__ charge, const int32_t* __restrict__ off,
    const int64_t* __restrict__ d_n_tracks, int64_t cap, float inv_q, int cbits, CmpWs w)
{
    const int64_t nt = track_count(d_n_tracks, cap);
    const int64_t na = nt > 0 ? off[nt] : 0;
    const int64_t n = (int64_t)n_sec * n_rows;
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t i = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; i < n;
         i += waves) {
        const tpc_sector& s = sec[i / n_rows];
        const int r = (int)(i % n_rows);
        const int per_row = s.nbz * s.nby;
        const int p0 = bin_start[s.bin_base + r * per_row];
        const int p1 = bin_start[s.bin_base + (r + 1) * per_row];
        int64_t u0 = w.rowcnt[i];
        int32_t carry = 0;             // z of the last such cluster of the rounds before
        for (int g0 = p0; g0 < p1; g0 += kWave) {
            const int g = g0 + lane;
            int c = -1;
            if (g < p1) c = idg[g];
            const bool un = c >= 0 && !w.on[c];
            const uint64_t m = __ballot(un);
            int32_t cz = 0;
            if (un) cz = quant(z[c], inv_q);
            // the previous cluster of the row: the highest lane below with one
            const uint64_t prev = m & below;
            const int src = prev ? 63 - __clzll(prev) : 0;
            const int32_t zp = __shfl(cz, src, kWave);
            if (un) {
                const int32_t pz = prev ? zp : carry;
                const int64_t u = u0 + __popcll(prev);
                const int32_t cy = quant(y[c], inv_q);
                put(w, S_UDZ, u, zigzag(cz - pz), cz - pz);
                const int32_t yo = cy + 2048;
                if (yo >= 0 && yo < 4096) {
                    w.sym[S_UYH][u] = (uint8_t)(yo >> 8);
                    w.sym[S_UYL][u] = (uint8_t)(yo & 255);
                } else {
                    w.sym[S_UYH][u] = 255;
                    w.esc[S_UYH][u] = cy;
                    w.sym[S_UYL][u] = 0;
                }
                w.sym[S_Q][na + u] = (uint8_t)charge_code(charge[c], cbits);
            }
            if (m) carry = __shfl(cz, 63 - __clzll(m), kWave);
            u0 += __popcll(m);
        }
    }
}

// stream sizes (device): counts[0..2] n_tracks, n_att, n_un; counts[3 + k]
// symbols of stream k
__global__ void k_cz_counts(const int32_t* __restrict__ off, const int64_t* __restrict__ d_n_tracks,
                            int64_t cap, int64_t n_clusters, int64_t n_rowseg, CmpWs w)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int64_t nt = track_count(d_n_tracks, cap);
    const int64_t na = nt > 0 ? off[nt] : 0;
    const int64_t nu = n_clusters - na;
    w.counts[0] = nt;
    w.counts[1] = na;
    w.counts[2] = nu;
    const int64_t n[kStreams] = {nt, na, na, na, na + nu, n_rowseg, nu, nu, nu};
    for (int k = 0; k < kStreams; ++k) w.counts[3 + k] = n[k];
}

// histogram of stream blockIdx.y
__global__ __launch_bounds__(kBlock) void k_cz_hist(CmpWs w)
{
    __shared__ uint32_t h[256];
    const int k = blockIdx.y;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t n = w.counts[3 + k];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[w.sym[k][i]], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += blockDim.x)
        if (h[i]) atomicAdd(&w.hist[k * 256 + i], h[i]);
}

// counts -> 12-bit frequencies (the reading's normalisation: floor of the
// share, at least 1, then the sum is brought to 2^12 one unit at a time, down
// on the largest frequency above 1, up on the largest count, ties to the
// lower symbol); one thread per stream
__global__ __launch_bounds__(kBlock) void k_cz_norm(CmpWs w)
{
    // one thread per symbol.  The rule, decrementing the largest frequency
    // above 1 (lowest symbol on ties) one step at a time, is applied in
    // closed form: with E the excess and D(L) = sum_i max(0, f_i - L), the
    // steps bring every f_i above L + 1 down to L + 1, L the largest level
    // with D(L) >= E, and the remaining E - D(L + 1) steps take the lowest
    // symbols at L + 1 to L (the maximum is then L + 1 and ties go to the
    // lowest symbol first).  Incrementing the largest count (lowest symbol
    // on ties) always picks the same symbol: it takes the whole deficit.
    __shared__ uint64_t red[kBlock / kWave];
    const int k = blockIdx.x, i = threadIdx.x;
    const uint32_t ci = w.hist[k * 256 + i];
    const uint64_t total = block_sum<uint64_t>(ci, red);
    uint32_t fi = 0;
    if (ci) {
        const uint64_t v = (uint64_t)ci * kProbScale / total;
        fi = v ? (uint32_t)v : 1u;
    }
    const uint64_t sum = block_sum<uint64_t>(fi, red);
    if (total && sum > kProbScale) {
        const uint64_t E = sum - kProbScale;
        uint32_t lo = 1, hi = kProbScale;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) / 2;
            const uint64_t d = block_sum<uint64_t>(fi > mid ? fi - mid : 0u, red);
            if (d >= E) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t L = lo;
        const uint64_t d1 = block_sum<uint64_t>(fi > L + 1 ? fi - (L + 1) : 0u, red);
        const uint64_t r = E - d1;
        const bool at = fi >= L + 1;
        uint64_t n_at;
        const uint64_t rank = block_excl_scan<uint64_t>(at ? 1u : 0u, red, &n_at);
        if (fi > L + 1) fi = L + 1;
        if (at && rank < r) fi = L;
    } else if (total && sum < kProbScale) {
        // largest count, lowest symbol on ties: max of count << 8 | (255 - symbol)
        const uint64_t key = ((uint64_t)ci << 8) | (uint64_t)(255 - i);
        uint64_t m = key;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
            const uint64_t v = __shfl_xor(m, o, kWave);
            m = v > m ? v : m;
        }
        __shared__ uint64_t mx[kBlock / kWave];
        if ((i & (kWave - 1)) == 0) mx[i / kWave] = m;
        __syncthreads();
        uint64_t best = 0;
#pragma unroll
        for (int q = 0; q < kBlock / kWave; ++q) best = mx[q] > best ? mx[q] : best;
        if (key == best) fi += (uint32_t)(kProbScale - sum);
    }
    w.freq[k * 256 + i] = fi;
    uint64_t tot;
    const uint64_t c = block_excl_scan<uint64_t>(fi, red, &tot);
    w.cum[k * 256 + i] = (uint32_t)c;
}

// Symbols of chunk j, read backwards 16 at a time when the chunk starts on
// a multiple of 16, the next block loaded while the current one is coded;
// the tables in LDS.  Encoding is a serial chain per chunk: the chunk size
// sets the parallelism.
__device__ __forceinline__ uint4 load16(const uint8_t* p) { return *reinterpret_cast<const uint4*>(p); }

__device__ __forceinline__ uint32_t byte_of(const uint4& v, int b)
{
    const uint32_t word = b < 4 ? v.x : b < 8 ? v.y : b < 12 ? v.z : v.w;
    return (word >> (8 * (b & 3))) & 255u;
}

// one thread per (chunk, stream): rANS encode backwards; the bytes end at the
// end of the chunk's slot
__global__ __launch_bounds__(kBlock) void k_cz_encode(CmpWs w, int chunk)
{
    // Per symbol: the renormalisation bound, and the quotient by its
    // frequency f as a multiply and shift (exact division by an invariant
    // integer, Granlund and Montgomery 1994): after renormalisation the state
    // is below 2^31, and with l = ceil(log2 f), M = ceil(2^(31 + l) / f) < 2^32,
    // x / f = (x M) >> (31 + l) = hi32(2x M) >> l for every x < 2^31.  The new
    // state (x / f) 2^12 + x mod f + c equals x + c + (x / f) (2^12 - f).
    __shared__ uint32_t xm_l[256], m_l[256], pk_l[256], c_l[256];
    const int k = blockIdx.y;
    {
        const uint32_t f = w.freq[k * 256 + threadIdx.x];
        uint32_t l = 0, mm = 0;
        if (f > 0) {
            l = f > 1 ? 32u - (uint32_t)__clz(f - 1u) : 0u;
            mm = (uint32_t)((((uint64_t)1 << (31 + l)) + f - 1) / f);
        }
        xm_l[threadIdx.x] = ((kRansL >> kProbBits) << 8) * f;
        m_l[threadIdx.x] = mm;
        pk_l[threadIdx.x] = (kProbScale - f) | (l << 16);
        c_l[threadIdx.x] = w.cum[k * 256 + threadIdx.x];
    }
    __syncthreads();
    const int64_t n = w.counts[3 + k];
    const int64_t nch = (n + chunk - 1) / chunk;
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nch) return;
    const uint8_t* s = w.sym[k];
    const int64_t a = j * chunk, e = a + chunk < n ? a + chunk : n;
    // bytes go backwards from the end of the chunk's slot (256-byte aligned),
    // gathered into words (the first of four at the top, the highest address)
    uint8_t* end = w.cbuf + ((int64_t)k * w.chunk_cap + j) * w.slot + w.slot;
    uint32_t m = 0;
    uint64_t acc = 0;
    uint32_t x = kRansL;
    // nb (0, 1 or 2) bytes, the first in the higher byte of v
    auto emit = [&](uint32_t v, uint32_t nb) {
        acc = (acc << (8 * nb)) | (v & ((1u << (8 * nb)) - 1u));
        m += nb;
        if ((m & 3u) < nb) *reinterpret_cast<uint32_t*>(end - (m & ~3u)) = (uint32_t)(acc >> (8 * (m & 3u)));
    };
    // renormalise (x < 2^31 and the bound is at least 2^19: at most two
    // bytes, the low one first), then the state step
    auto code = [&](uint32_t xm, uint32_t mm, uint32_t pk, uint32_t c) {
        const uint32_t nb = (x >= xm ? 1u : 0u) + ((x >> 8) >= xm ? 1u : 0u);
        emit(nb == 2 ? ((x & 255u) << 8) | ((x >> 8) & 255u) : x & 255u, nb);
        x >>= 8 * nb;
        const uint32_t q = __umulhi(x << 1, mm) >> (pk >> 16);
        x += c + q * (pk & 0xFFFFu);
    };
    auto code_sym = [&](uint32_t sy) { code(xm_l[sy], m_l[sy], pk_l[sy], c_l[sy]); };
    int64_t i = e;
    if ((a & 15) == 0) {          // 16-byte blocks (chunk sizes that are multiples of 16)
        // the ragged tail first (symbols past the last multiple of 16)
        const int64_t e16 = a + (e - a) / 16 * 16;
        while (i > e16) code_sym(s[--i]);
        uint4 nxt = make_uint4(0, 0, 0, 0);
        if (i > a) nxt = load16(s + i - 16);
        while (i > a) {
            const uint4 cur = nxt;
            if (i - 16 > a) nxt = load16(s + i - 32);     // the next block, in flight meanwhile
            // the block's table entries first, then the dependent steps
            uint32_t txm[16], tm[16], tpk[16], tc[16];
#pragma unroll
            for (int b = 0; b < 16; ++b) {
                const uint32_t sy = byte_of(cur, b);
                txm[b] = xm_l[sy];
                tm[b] = m_l[sy];
                tpk[b] = pk_l[sy];
                tc[b] = c_l[sy];
            }
#pragma unroll
            for (int b = 15; b >= 0; --b) code(txm[b], tm[b], tpk[b], tc[b]);
            i -= 16;
        }
    }
    while (i > a) code_sym(s[--i]);
    // the final state, low byte first
    emit(((x & 255u) << 8) | ((x >> 8) & 255u), 2);
    emit(((x >> 16) & 255u) << 8 | (x >> 24), 2);
    // the bytes of a last, partial word
    const uint32_t p = m & 3u;
    for (uint32_t t = 0; t < p; ++t)
        *(end - 1 - (m - p) - t) = (uint8_t)(acc >> (8 * (p - 1 - t)));
    w.csize[(int64_t)k * w.chunk_cap + j] = m;
}

// escape flags of stream k over its capacity (zero past its size)
__global__ __launch_bounds__(kBlock) void k_cz_eflag(CmpWs w, int k)
{
    const int64_t n = w.counts[3 + k];
    const bool esc_ok = k != S_Q && k != S_UYL;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < w.cap[k];
         i += (int64_t)gridDim.x * blockDim.x)
        w.eflag[i] = (esc_ok && i < n && w.sym[k][i] == 255) ? 1 : 0;
}

__device__ __forceinline__ void put32(uint8_t* out, int64_t at, uint32_t v)
{
    out[at] = (uint8_t)v;
    out[at + 1] = (uint8_t)(v >> 8);
    out[at + 2] = (uint8_t)(v >> 16);
    out[at + 3] = (uint8_t)(v >> 24);
}

__device__ __forceinline__ void put64(uint8_t* out, int64_t at, uint64_t v)
{
    put32(out, at, (uint32_t)v);
    put32(out, at + 4, (uint32_t)(v >> 32));
}

// The blob's layout and header, one 256-thread block: per stream the chunk
// sizes are summed and scanned into every chunk's offset (block scans),
// the tables are written by all threads; lay[]: per stream the offset of
// its chunk data and of its escapes, then the headers' offset and whether
// the blob fits.  (One thread walking every chunk took 0.3 ms on the
// central event.)
__global__ __launch_bounds__(kBlock) void k_cz_layout(CmpWs w, int cbits, int qbits, int chunk,
                                                      int n_sec, int n_rows, int64_t n_clusters,
                                                      uint8_t* __restrict__ out, int64_t out_cap,
                                                      int64_t* __restrict__ d_size)
{
    __shared__ int64_t red[kBlock / kWave];
    __shared__ int64_t data_k[kStreams];
    __shared__ int fits;
    int64_t nch[kStreams];
#pragma unroll
    for (int k = 0; k < kStreams; ++k) nch[k] = (w.counts[3 + k] + chunk - 1) / chunk;
    int64_t hsize = kHeaderFixed;
#pragma unroll
    for (int k = 0; k < kStreams; ++k) hsize += kStreamHeader + 4 * nch[k];
    // chunk offsets relative to the stream's data start
    for (int k = 0; k < kStreams; ++k) {
        int64_t carry = 0;
        for (int64_t j0 = 0; j0 < nch[k]; j0 += blockDim.x) {
            const int64_t j = j0 + threadIdx.x;
            const int64_t v = j < nch[k] ? (int64_t)w.csize[k * w.chunk_cap + j] : 0;
            int64_t tot;
            const int64_t ex = block_excl_scan<int64_t>(v, red, &tot);
            if (j < nch[k]) w.coff[k * w.chunk_cap + j] = carry + ex;
            carry += tot;
        }
        if (threadIdx.x == 0) data_k[k] = carry;
    }
    __syncthreads();
    // stream starts: data of the earlier streams, then the escapes
    int64_t at = hsize, esc = 0;
    int64_t start[kStreams];
#pragma unroll
    for (int k = 0; k < kStreams; ++k) {
        start[k] = at;
        at += data_k[k];
        esc += 4 * w.eoff[k];
    }
    const int64_t size = at + esc + 16 * w.counts[0];
    if (threadIdx.x == 0) {
        *d_size = size;
        int64_t e = at;
        for (int k = 0; k < kStreams; ++k) {
            w.lay[3 * k] = start[k];
            w.lay[3 * k + 1] = e;
            e += 4 * w.eoff[k];
        }
        w.lay[3 * kStreams] = e;
        w.lay[3 * kStreams + 1] = size <= out_cap ? 1 : 0;
        fits = size <= out_cap;
    }
    __syncthreads();
    if (!fits) return;
    // chunk offsets become blob offsets
    for (int k = 0; k < kStreams; ++k)
        for (int64_t j = threadIdx.x; j < nch[k]; j += blockDim.x)
            w.coff[k * w.chunk_cap + j] += start[k];
    if (threadIdx.x == 0) {
        int64_t p = 0;
        const uint32_t head[7] = {0x5a435054u, 1u, (uint32_t)cbits, (uint32_t)qbits,
                                  (uint32_t)chunk, (uint32_t)n_sec, (uint32_t)n_rows};
        for (int i = 0; i < 7; ++i, p += 4) put32(out, p, head[i]);
        put64(out, p, (uint64_t)n_clusters);
        put64(out, p + 8, (uint64_t)w.counts[0]);
        put64(out, p + 16, (uint64_t)w.counts[1]);
        put64(out, p + 24, (uint64_t)w.counts[2]);
    }
    int64_t p = kHeaderFixed;
    for (int k = 0; k < kStreams; ++k) {
        if (threadIdx.x == 0) {
            put64(out, p, (uint64_t)w.counts[3 + k]);
            put64(out, p + 8, (uint64_t)w.eoff[k]);
            put32(out, p + 16, (uint32_t)nch[k]);
        }
        const int64_t pf = p + 20;
        for (int i = threadIdx.x; i < 256; i += blockDim.x) {
            const uint32_t f = w.freq[k * 256 + i];
            const uint16_t v = (uint16_t)(f == kProbScale ? 0xffffu : f);
            out[pf + 2 * i] = (uint8_t)v;
            out[pf + 2 * i + 1] = (uint8_t)(v >> 8);
        }
        const int64_t pc = pf + 512;
        for (int64_t j = threadIdx.x; j < nch[k]; j += blockDim.x)
            put32(out, pc + 4 * j, w.csize[k * w.chunk_cap + j]);
        p = pc + 4 * nch[k];
    }
}

// chunk bytes into the blob: block per (chunk, stream)
__global__ __launch_bounds__(kBlock) void k_cz_copy_chunks(CmpWs w, int chunk,
                                                           uint8_t* __restrict__ out)
{
    if (!w.lay[3 * kStreams + 1]) return;
    const int k = blockIdx.y;
    const int64_t nch = (w.counts[3 + k] + chunk - 1) / chunk;
    for (int64_t j = blockIdx.x; j < nch; j += gridDim.x) {
        const int64_t at = w.coff[k * w.chunk_cap + j];
        const uint32_t m = w.csize[k * w.chunk_cap + j];
        const uint8_t* src = w.cbuf + ((int64_t)k * w.chunk_cap + j) * w.slot + w.slot - m;
        for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) out[at + i] = src[i];
    }
}

// escapes of stream k in symbol order (eflag holds the exclusive scan of the
// flags)
__global__ __launch_bounds__(kBlock) void k_cz_copy_esc(CmpWs w, int k, uint8_t* __restrict__ out)
{
    if (!w.lay[3 * kStreams + 1]) return;
    const int64_t n = w.counts[3 + k];
    const int64_t base = w.lay[3 * k + 1];
    const bool esc_ok = k != S_Q && k != S_UYL;
    if (!esc_ok) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (w.sym[k][i] == 255) put32(out, base + 4 * (int64_t)w.eflag[i], (uint32_t)w.esc[k][i]);
}

__global__ __launch_bounds__(kBlock) void k_cz_copy_hdr(CmpWs w, uint8_t* __restrict__ out)
{
    if (!w.lay[3 * kStreams + 1]) return;
    const int64_t n = 16 * w.counts[0];
    const int64_t base = w.lay[3 * kStreams];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[base + i] = w.hdr[i];
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// carve the workspace; returns its size (nothing written when base is null)
size_t layout_cmp(const tpc_problem* p, int64_t track_cap, int64_t hit_cap, int chunk,
                  void* base, CmpWs* w)
{
    const int64_t n = p->n_clusters;
    const int64_t nrs = (int64_t)p->n_sectors * p->n_rows;
    const int64_t cap[kStreams] = {track_cap, hit_cap, hit_cap, hit_cap, n, nrs, n, n, n};
    int64_t maxcap = 1, ch = 1;
    for (int k = 0; k < kStreams; ++k) {
        w->cap[k] = cap[k];
        maxcap = cap[k] > maxcap ? cap[k] : maxcap;
        const int64_t c = (cap[k] + chunk - 1) / chunk;
        ch = c > ch ? c : ch;
    }
    w->chunk_cap = ch;
    w->slot = align256((size_t)(2 * (int64_t)chunk + 8));
    w->n_rowseg = nrs;
    size_t at = 0;
    char* b = (char*)base;
    auto take = [&](size_t bytes) -> char* {
        char* r = b ? b + at : nullptr;
        at += align256(bytes > 0 ? bytes : 1);
        return r;
    };
    w->on = (uint8_t*)take((size_t)n);
    for (int k = 0; k < kStreams; ++k) {
        w->sym[k] = (uint8_t*)take((size_t)cap[k]);
        w->esc[k] = (int32_t*)take(4 * (size_t)cap[k]);
    }
    w->eflag = (int32_t*)take(4 * (size_t)(maxcap + 1));
    w->rowcnt = (int32_t*)take(4 * (size_t)(nrs + 1));
    w->hdr = (uint8_t*)take(16 * (size_t)track_cap);
    w->hist = (uint32_t*)take(4 * kStreams * 256);
    w->freq = (uint32_t*)take(4 * kStreams * 256);
    w->cum = (uint32_t*)take(4 * kStreams * 256);
    w->cbuf = (uint8_t*)take((size_t)kStreams * ch * w->slot);
    w->csize = (uint32_t*)take(4 * (size_t)kStreams * ch);
    w->coff = (int64_t*)take(8 * (size_t)kStreams * ch);
    w->counts = (int64_t*)take(8 * 16);
    w->eoff = (int64_t*)take(8 * (kStreams + 1));
    w->lay = (int64_t*)take(8 * (3 * kStreams + 4));
    w->partials = (int64_t*)take(8 * (size_t)(ceil_div(maxcap + 1, kScanTile) + 1));
    return at;
}

}  // namespace

}  // namespace tpc

extern "C" int tpc_check_problem(const tpc_problem* p);

extern "C" {

int tpc_compress_workspace_size(const tpc_problem* h_prob, int64_t track_capacity,
                                int64_t hit_capacity, int32_t chunk, size_t* h_bytes)
{
    if (!h_bytes || track_capacity < 0 || hit_capacity < 0 || chunk < 64 || chunk > (1 << 20))
        return TPC_ERR_INVALID_ARG;
    const int e = tpc_check_problem(h_prob);
    if (e) return e;
    tpc::CmpWs w;
    *h_bytes = tpc::layout_cmp(h_prob, track_capacity, hit_capacity, chunk, nullptr, &w);
    return TPC_OK;
}

int tpc_compress_clusters(tpc_context* ctx, const tpc_problem* h_prob, tpc_clusters clusters,
                          const float* charge, tpc_grid grid, tpc_tracklets tracklets,
                          tpc_tracks tracks, const int64_t* d_n_tracks, tpc_compress_params cp,
                          uint8_t* out, int64_t out_cap, int64_t* d_size, void* d_ws,
                          size_t ws_bytes, void* stream)
{
    tpc::TimerScope timing(ctx ? ctx->timer : nullptr);
    if (!ctx || !clusters.row || !clusters.y || !clusters.z || !charge || !grid.bin_start ||
        !grid.id || !tracklets.par || !tracklets.row_inner || !tracks.off || !tracks.hits ||
        !tracks.tracklet || !d_n_tracks || !out || out_cap < 0 || !d_size || !d_ws ||
        tracks.capacity < 0 || tracks.hit_capacity < 0 || cp.qbits < 0 || cp.qbits > 12 ||
        cp.cbits < 2 || cp.cbits > 8 || cp.chunk < 64 || cp.chunk > (1 << 20))
        return TPC_ERR_INVALID_ARG;
    const int n_copies = !!tracks.hit_row + !!tracks.hit_y + !!tracks.hit_z;
    if (n_copies != 0 && n_copies != 3) return TPC_ERR_INVALID_ARG;
    const int e = tpc_check_problem(h_prob);
    if (e) return e;
    tpc::CmpWs w;
    const size_t need = tpc::layout_cmp(h_prob, tracks.capacity, tracks.hit_capacity, cp.chunk,
                                        d_ws, &w);
    if (need > ws_bytes) return TPC_ERR_INVALID_ARG;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TPC_ERR_HIP;
    if (dev != ctx->device && hipSetDevice(ctx->device) != hipSuccess) return TPC_ERR_HIP;
    hipStream_t st = (hipStream_t)stream;
    const float inv_q = std::ldexp(1.0f, cp.qbits);
    const int64_t n = h_prob->n_clusters;
    const int n_sec = h_prob->n_sectors, n_rows = h_prob->n_rows;
    const int64_t nrs = (int64_t)n_sec * n_rows;
    const int64_t tcap = tracks.capacity;
    // clear what is accumulated (fill kernels, no memset nodes in a graph);
    // the flag bytes are cleared as words (their slot is 256-byte aligned)
    tpc::launch_fill<int32_t>((int32_t*)w.on, 0, tpc::ceil_div(n > 0 ? n : 1, 4), st);
    tpc::launch_fill<int32_t>((int32_t*)w.hist, 0, tpc::kStreams * 256, st);
    TPC_LAUNCH(tpc::k_cz_counts, dim3(1), dim3(64), 0, st, (const int32_t*)tracks.off,
               d_n_tracks, tcap, n, nrs, w);
    if (tcap > 0) {
        TPC_LAUNCH(tpc::k_cz_mark, dim3(tpc::grid_for(tracks.hit_capacity)), dim3(tpc::kBlock), 0,
                   st, (const int32_t*)tracks.off, (const int32_t*)tracks.hits, d_n_tracks, tcap,
                   w);
        TPC_LAUNCH(tpc::k_cz_tracks, dim3(tpc::grid_for(tcap)), dim3(tpc::kBlock), 0, st,
                   h_prob->d_row_x, h_prob->params, clusters.row, clusters.y, clusters.z, charge,
                   (const int32_t*)tracks.off, (const int32_t*)tracks.hits,
                   (const uint8_t*)tracks.hit_row, (const float*)tracks.hit_y,
                   (const float*)tracks.hit_z, (const int32_t*)tracks.tracklet,
                   (const float*)tracklets.par, (const int32_t*)tracklets.row_inner, d_n_tracks,
                   tcap, inv_q, cp.cbits, w);
    }
    TPC_LAUNCH(tpc::k_cz_rowcount, dim3(tpc::grid_for(nrs * tpc::kWave)), dim3(tpc::kBlock), 0, st,
               h_prob->d_sectors, n_sec, n_rows, (const int32_t*)grid.bin_start,
               (const int32_t*)grid.id, w);
    tpc::launch_scan<int32_t>(w.rowcnt, w.rowcnt, nrs, false, nullptr, nullptr, w.partials, st);
    TPC_LAUNCH(tpc::k_cz_rowemit, dim3(tpc::grid_for(nrs * tpc::kWave)), dim3(tpc::kBlock), 0, st,
               h_prob->d_sectors, n_sec, n_rows, (const int32_t*)grid.bin_start,
               (const int32_t*)grid.id, clusters.y, clusters.z, charge,
               (const int32_t*)tracks.off, d_n_tracks, tcap, inv_q, cp.cbits, w);
    TPC_LAUNCH(tpc::k_cz_hist, dim3(256, tpc::kStreams), dim3(tpc::kBlock), 0, st, w);
    TPC_LAUNCH(tpc::k_cz_norm, dim3(tpc::kStreams), dim3(tpc::kBlock), 0, st, w);
    TPC_LAUNCH(tpc::k_cz_encode,
               dim3((unsigned)tpc::ceil_div(w.chunk_cap, tpc::kBlock), tpc::kStreams),
               dim3(tpc::kBlock), 0, st, w, (int)cp.chunk);
    // escape counts, the layout and header, then the chunk bytes, the
    // escapes in order (flags scanned again per stream) and the headers
    for (int k = 0; k < tpc::kStreams; ++k) {
        TPC_LAUNCH(tpc::k_cz_eflag, dim3(tpc::grid_for(w.cap[k])), dim3(tpc::kBlock), 0, st, w,
                   k);
        tpc::launch_scan<int32_t>(w.eflag, w.eflag, w.cap[k], false, w.eoff + k, nullptr,
                                  w.partials, st);
    }
    TPC_LAUNCH(tpc::k_cz_layout, dim3(1), dim3(tpc::kBlock), 0, st, w, (int)cp.cbits, (int)cp.qbits,
               (int)cp.chunk, n_sec, n_rows, n, out, out_cap, d_size);
    TPC_LAUNCH(tpc::k_cz_copy_chunks, dim3(1024, tpc::kStreams), dim3(tpc::kBlock), 0, st, w,
               (int)cp.chunk, out);
    for (int k = 0; k < tpc::kStreams; ++k) {
        TPC_LAUNCH(tpc::k_cz_eflag, dim3(tpc::grid_for(w.cap[k])), dim3(tpc::kBlock), 0, st, w,
                   k);
        tpc::launch_scan<int32_t>(w.eflag, w.eflag, w.cap[k], false, nullptr, nullptr,
                                  w.partials, st);
        TPC_LAUNCH(tpc::k_cz_copy_esc, dim3(tpc::grid_for(w.cap[k])), dim3(tpc::kBlock), 0, st,
                   w, k, out);
    }
    TPC_LAUNCH(tpc::k_cz_copy_hdr, dim3(tpc::grid_for(16 * (tcap > 0 ? tcap : 1))),
               dim3(tpc::kBlock), 0, st, w, out);
    return hipGetLastError() == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // extern "C"
