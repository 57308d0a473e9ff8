// Per-item device code of the cellular-automaton seeding, shared by the
// staged kernels and the persistent kernel.
#pragma once
#include "tpc_internal.hpp"

namespace tpc {

// Best up/down pair of the hit at grid position p.  Candidates on rows r+1
// and r-1 come from the bins covering the windows around the straight line
// from the origin through the hit; the exact window test and the pair
// deviation decide, ties go to the lower (up id, down id).
__device__ __forceinline__ void neighbours_one(
    int64_t p, const tpc_sector* __restrict__ sec, int n_rows, const float* __restrict__ row_x,
    const tpc_params& prm, const int32_t* __restrict__ bin_start, const float* __restrict__ yg,
    const float* __restrict__ zg, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ gsr, int32_t* __restrict__ up0, int32_t* __restrict__ down0)
{
    const float Wy = prm.nb_win_y, Wz = prm.nb_win_z, D2max = prm.nb_d2max;
    const int v = gsr[p];
    const int r = v & 255;
    int bu = -1, bd = -1;
    if (r > 0 && r + 1 < n_rows) {
        const tpc_sector s = sec[v >> 8];
        const float y = yg[p], z = zg[p];
        const float slope = y / row_x[r];
        const float yu_c = slope * row_x[r + 1];
        const float yd_c = slope * row_x[r - 1];
        const int iyu0 = bin_of(yu_c - Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
        const int iyu1 = bin_of(yu_c + Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
        const int iyd0 = bin_of(yd_c - Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
        const int iyd1 = bin_of(yd_c + Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
        const int iz0 = bin_of(z - Wz * TPC_WIDEN, s.z0, s.inv_bz, s.nbz);
        const int iz1 = bin_of(z + Wz * TPC_WIDEN, s.z0, s.inv_bz, s.nbz);
        float best = 0.0f;
        int bidu = -1, bidd = -1;
        for (int izu = iz0; izu <= iz1; ++izu) {
            const int gu = s.bin_base + ((r + 1) * s.nbz + izu) * s.nby;
            const int pu1 = bin_start[gu + iyu1 + 1];
            for (int pu = bin_start[gu + iyu0]; pu < pu1; ++pu) {
                const float yu = yg[pu], zu = zg[pu];
                if (!(fabsf(yu - yu_c) <= Wy && fabsf(zu - z) <= Wz)) continue;
                const int idu = idg[pu];
                for (int izd = iz0; izd <= iz1; ++izd) {
                    const int gd = s.bin_base + ((r - 1) * s.nbz + izd) * s.nby;
                    const int pd1 = bin_start[gd + iyd1 + 1];
                    for (int pd = bin_start[gd + iyd0]; pd < pd1; ++pd) {
                        const float yd = yg[pd], zd = zg[pd];
                        if (!(fabsf(yd - yd_c) <= Wy && fabsf(zd - z) <= Wz)) continue;
                        const float dy = (yu + yd) - (y + y);
                        const float dz = (zu + zd) - (z + z);
                        const float d2 = dy * dy + dz * dz;
                        if (!(d2 <= D2max)) continue;
                        const int idd = idg[pd];
                        if (bu < 0 || d2 < best ||
                            (d2 == best && (idu < bidu || (idu == bidu && idd < bidd)))) {
                            best = d2;
                            bu = pu;
                            bd = pd;
                            bidu = idu;
                            bidd = idd;
                        }
                    }
                }
            }
        }
    }
    up0[p] = bu;
    down0[p] = bd;
}

// Mutual links of the hit at p; a chain start (up link, no down link, and
// its up neighbour has an up link) is flagged in the id-indexed array
// start_by_id.
__device__ __forceinline__ void clean_one(
    int64_t p, const int32_t* __restrict__ up0, const int32_t* __restrict__ down0,
    const int32_t* __restrict__ idg, int32_t* __restrict__ up, int32_t* __restrict__ down,
    int32_t* __restrict__ start_by_id)
{
    const int u = up0[p], d = down0[p];
    const int uc = (u >= 0 && down0[u] == p) ? u : -1;
    const int dc = (d >= 0 && up0[d] == p) ? d : -1;
    up[p] = uc;
    down[p] = dc;
    if (uc >= 0 && dc < 0) {
        const int uu = up0[uc];
        if (uu >= 0 && down0[uu] == uc) start_by_id[idg[p]] = (int32_t)p;
    }
}

// ---- LDS-staged variant -------------------------------------------------------
// A block handles one pad row r of one sector, z-slab by z-slab.  For a slab
// of z bins [z0, z1) the candidates of rows r+1 and r-1 lie in z bins
// [z0 - m, z1 + m) of those rows: contiguous grid positions, copied to LDS
// with their bin starts.  A hit whose bin window leaves the staged bins, or a
// row whose staged range exceeds the LDS capacity, reads global memory; both
// paths evaluate the same predicates in the same order.

constexpr int kNbCap = 1024;     // staged candidates per neighbouring row
constexpr int kNbBinCap = 1024;  // staged bin starts per neighbouring row

struct NbRowStage {
    float y[kNbCap];
    float z[kNbCap];
    int32_t id[kNbCap];
    int32_t bs[kNbBinCap];   // bin starts relative to q0, bins [za, zb) x all y, plus the end
};

// candidate source: one neighbouring row, staged or global
struct NbSrc {
    const NbRowStage* st;    // null: global
    int za, zb;              // staged z bins
    int32_t q0;              // grid position of the first staged candidate
    int g_row;               // global bin of (row, z = 0, y = 0)
    int nby;
    const int32_t* bin_start;
    const float* yg;
    const float* zg;
    const int32_t* idg;
    __device__ __forceinline__ bool covers(int iz0, int iz1) const
    {
        return st && iz0 >= za && iz1 < zb;
    }
};

template <bool Staged>
__device__ __forceinline__ int nb_first(const NbSrc& S, int iz, int iy)
{
    if (Staged) return S.st->bs[(iz - S.za) * S.nby + iy];
    return S.bin_start[S.g_row + iz * S.nby + iy] - S.q0;
}
template <bool Staged>
__device__ __forceinline__ float nb_y(const NbSrc& S, int k) { return Staged ? S.st->y[k] : S.yg[S.q0 + k]; }
template <bool Staged>
__device__ __forceinline__ float nb_z(const NbSrc& S, int k) { return Staged ? S.st->z[k] : S.zg[S.q0 + k]; }
template <bool Staged>
__device__ __forceinline__ int nb_id(const NbSrc& S, int k) { return Staged ? S.st->id[k] : S.idg[S.q0 + k]; }

// best pair for one hit with its up candidates from U and down candidates
// from D (positions relative to U.q0 / D.q0); same expressions as
// neighbours_one.  The down candidates inside the window are gathered first
// (up to kNbList, in registers), so that each up candidate is paired with
// those only; a hit with more goes through the plain double scan.  The pair
// is the lexicographic minimum of (D2, up id, down id), whatever the order.
constexpr int kNbList = 8;

template <bool SU, bool SD>
__device__ __forceinline__ void nb_pairs(const NbSrc& U, const NbSrc& D, float y, float z,
                                         float yu_c, float yd_c, int iyu0, int iyu1, int iyd0,
                                         int iyd1, int iz0, int iz1, const tpc_params& prm,
                                         int& bu, int& bd)
{
    const float Wy = prm.nb_win_y, Wz = prm.nb_win_z, D2max = prm.nb_d2max;
    float best = 0.0f;
    int bidu = -1, bidd = -1;
    float ly[kNbList], lz[kNbList];
    int lid[kNbList], lpos[kNbList];
    int nd = 0;
    for (int izd = iz0; izd <= iz1; ++izd) {
        const int pd1 = nb_first<SD>(D, izd, iyd1 + 1);
        for (int pd = nb_first<SD>(D, izd, iyd0); pd < pd1; ++pd) {
            const float yd = nb_y<SD>(D, pd), zd = nb_z<SD>(D, pd);
            if (!(fabsf(yd - yd_c) <= Wy && fabsf(zd - z) <= Wz)) continue;
#pragma unroll
            for (int k = 0; k < kNbList; ++k)
                if (k == nd) {
                    ly[k] = yd;
                    lz[k] = zd;
                    lpos[k] = pd;
                }
            ++nd;
        }
    }
    if (nd == 0) return;
    const bool listed = nd <= kNbList;
    if (listed) {
#pragma unroll
        for (int k = 0; k < kNbList; ++k)
            if (k < nd) lid[k] = nb_id<SD>(D, lpos[k]);
    }
    for (int izu = iz0; izu <= iz1; ++izu) {
        const int pu1 = nb_first<SU>(U, izu, iyu1 + 1);
        for (int pu = nb_first<SU>(U, izu, iyu0); pu < pu1; ++pu) {
            const float yu = nb_y<SU>(U, pu), zu = nb_z<SU>(U, pu);
            if (!(fabsf(yu - yu_c) <= Wy && fabsf(zu - z) <= Wz)) continue;
            const int idu = nb_id<SU>(U, pu);
            if (listed) {
#pragma unroll
                for (int k = 0; k < kNbList; ++k) {
                    if (k >= nd) break;
                    const float dy = (yu + ly[k]) - (y + y);
                    const float dz = (zu + lz[k]) - (z + z);
                    const float d2 = dy * dy + dz * dz;
                    if (!(d2 <= D2max)) continue;
                    const int idd = lid[k];
                    if (bu < 0 || d2 < best ||
                        (d2 == best && (idu < bidu || (idu == bidu && idd < bidd)))) {
                        best = d2;
                        bu = U.q0 + pu;
                        bd = D.q0 + lpos[k];
                        bidu = idu;
                        bidd = idd;
                    }
                }
                continue;
            }
            for (int izd = iz0; izd <= iz1; ++izd) {
                const int pd1 = nb_first<SD>(D, izd, iyd1 + 1);
                for (int pd = nb_first<SD>(D, izd, iyd0); pd < pd1; ++pd) {
                    const float yd = nb_y<SD>(D, pd), zd = nb_z<SD>(D, pd);
                    if (!(fabsf(yd - yd_c) <= Wy && fabsf(zd - z) <= Wz)) continue;
                    const float dy = (yu + yd) - (y + y);
                    const float dz = (zu + zd) - (z + z);
                    const float d2 = dy * dy + dz * dz;
                    if (!(d2 <= D2max)) continue;
                    const int idd = nb_id<SD>(D, pd);
                    if (bu < 0 || d2 < best ||
                        (d2 == best && (idu < bidu || (idu == bidu && idd < bidd)))) {
                        best = d2;
                        bu = U.q0 + pu;
                        bd = D.q0 + pd;
                        bidu = idu;
                        bidd = idd;
                    }
                }
            }
        }
    }
}

// copy the candidates of row `row`, z bins [za, zb), to LDS; returns the
// source description (global when they do not fit)
__device__ __forceinline__ NbSrc nb_stage(NbRowStage* st, const tpc_sector& s, int row, int za,
                                          int zb, const int32_t* __restrict__ bin_start,
                                          const float* __restrict__ yg,
                                          const float* __restrict__ zg,
                                          const int32_t* __restrict__ idg)
{
    NbSrc S;
    S.za = za;
    S.zb = zb;
    S.nby = s.nby;
    S.g_row = s.bin_base + row * s.nbz * s.nby;
    S.bin_start = bin_start;
    S.yg = yg;
    S.zg = zg;
    S.idg = idg;
    const int gb0 = S.g_row + za * s.nby, gb1 = S.g_row + zb * s.nby;
    S.q0 = bin_start[gb0];
    const int n = bin_start[gb1] - S.q0;
    const int nbins = gb1 - gb0 + 1;
    const bool fit = n <= kNbCap && nbins <= kNbBinCap;
    S.st = fit ? st : nullptr;
    if (fit) {
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            st->y[k] = yg[S.q0 + k];
            st->z[k] = zg[S.q0 + k];
            st->id[k] = idg[S.q0 + k];
        }
        for (int k = threadIdx.x; k < nbins; k += blockDim.x) st->bs[k] = bin_start[gb0 + k] - S.q0;
    }
    return S;
}

// one hit (grid position p, row r) against the two sources
__device__ __forceinline__ void neighbours_staged_one(
    int64_t p, const tpc_sector& s, int r, const float* __restrict__ row_x,
    const tpc_params& prm, const NbSrc& U, const NbSrc& D, const float* __restrict__ yg,
    const float* __restrict__ zg, int32_t* __restrict__ up0, int32_t* __restrict__ down0)
{
    const float Wy = prm.nb_win_y, Wz = prm.nb_win_z;
    const float y = yg[p], z = zg[p];
    const float slope = y / row_x[r];
    const float yu_c = slope * row_x[r + 1];
    const float yd_c = slope * row_x[r - 1];
    const int iyu0 = bin_of(yu_c - Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
    const int iyu1 = bin_of(yu_c + Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
    const int iyd0 = bin_of(yd_c - Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
    const int iyd1 = bin_of(yd_c + Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
    const int iz0 = bin_of(z - Wz * TPC_WIDEN, s.z0, s.inv_bz, s.nbz);
    const int iz1 = bin_of(z + Wz * TPC_WIDEN, s.z0, s.inv_bz, s.nbz);
    int bu = -1, bd = -1;
    // the global sources describe the same positions (q0 relative)
    NbSrc Ug = U, Dg = D;
    if (!U.covers(iz0, iz1)) Ug.st = nullptr;
    if (!D.covers(iz0, iz1)) Dg.st = nullptr;
    if (Ug.st && Dg.st)
        nb_pairs<true, true>(Ug, Dg, y, z, yu_c, yd_c, iyu0, iyu1, iyd0, iyd1, iz0, iz1, prm, bu, bd);
    else if (Ug.st)
        nb_pairs<true, false>(Ug, Dg, y, z, yu_c, yd_c, iyu0, iyu1, iyd0, iyd1, iz0, iz1, prm, bu, bd);
    else if (Dg.st)
        nb_pairs<false, true>(Ug, Dg, y, z, yu_c, yd_c, iyu0, iyu1, iyd0, iyd1, iz0, iz1, prm, bu, bd);
    else
        nb_pairs<false, false>(Ug, Dg, y, z, yu_c, yd_c, iyu0, iyu1, iyd0, iyd1, iz0, iz1, prm, bu, bd);
    up0[p] = bu;
    down0[p] = bd;
}

// z-bin margin of the candidate windows
__device__ __forceinline__ int nb_margin(const tpc_sector& s, const tpc_params& prm)
{
    return (int)(prm.nb_win_z * TPC_WIDEN * s.inv_bz) + 2;
}

// z bins per slab: as many as the stage holds (bins, and the expected
// candidates of a neighbouring row with room to spare), balanced over the
// slabs of the row
__device__ __forceinline__ int nb_slab(const tpc_sector& s, int n_rows, int m)
{
    const int64_t n = s.end - s.begin;
    const int64_t per_row_zbin = n / ((int64_t)n_rows * s.nbz) + 1;
    if ((int64_t)s.nby * s.nbz + 1 <= kNbBinCap && 2 * per_row_zbin * s.nbz <= kNbCap)
        return s.nbz;                              // whole rows
    int64_t zs = (kNbBinCap - 1) / s.nby - 2 * m;
    const int64_t zc = kNbCap / (2 * per_row_zbin) - 2 * m;
    if (zc < zs) zs = zc;
    if (zs < 1) zs = 1;
    if (zs >= s.nbz) return s.nbz;
    const int64_t slabs = (s.nbz + zs - 1) / zs;
    return (int)((s.nbz + slabs - 1) / slabs);
}

// all hits of row r (1 <= r <= n_rows - 2) of sector s, by one block
__device__ __forceinline__ void neighbours_row(
    NbRowStage* stu, NbRowStage* std_, const tpc_sector& s, int r, int n_rows,
    const float* __restrict__ row_x, const tpc_params& prm,
    const int32_t* __restrict__ bin_start, const float* __restrict__ yg,
    const float* __restrict__ zg, const int32_t* __restrict__ idg, int32_t* __restrict__ up0,
    int32_t* __restrict__ down0)
{
    const int m = nb_margin(s, prm), zs = nb_slab(s, n_rows, m);
    const int g_r = s.bin_base + r * s.nbz * s.nby;
    for (int z0 = 0; z0 < s.nbz; z0 += zs) {
        const int z1 = z0 + zs < s.nbz ? z0 + zs : s.nbz;
        const int za = z0 - m > 0 ? z0 - m : 0, zb = z1 + m < s.nbz ? z1 + m : s.nbz;
        const int32_t p0 = bin_start[g_r + z0 * s.nby], p1 = bin_start[g_r + z1 * s.nby];
        __syncthreads();   // the previous slab's stage is consumed
        const NbSrc U = nb_stage(stu, s, r + 1, za, zb, bin_start, yg, zg, idg);
        const NbSrc D = nb_stage(std_, s, r - 1, za, zb, bin_start, yg, zg, idg);
        __syncthreads();
        for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x)
            neighbours_staged_one(p, s, r, row_x, prm, U, D, yg, zg, up0, down0);
    }
}

}  // namespace tpc
