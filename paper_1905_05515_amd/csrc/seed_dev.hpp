// Per-item device code of the cellular-automaton seeding, shared by the
// staged kernels and the persistent kernel.
#pragma once
#include "tpc_internal.hpp"

namespace tpc {

// candidate source: the grid of one neighbouring row
struct NbSrc {
    int g_row;               // global bin of (row, z = 0, y = 0)
    int nby;
    const int32_t* bin_start;
    const float* yg;
    const float* zg;
    const int32_t* idg;
    __device__ __forceinline__ int first(int iz, int iy) const { return bin_start[g_row + iz * nby + iy]; }
};

// best pair for one hit with its up candidates from U and down candidates
// from D.  The down candidates inside the window are gathered first (up to
// kNbList, in the lane's column of an LDS list), so that each up candidate
// is paired with those only; a hit with more goes through the plain double
// scan.  The pair is the lexicographic minimum of (D2, up id, down id),
// whatever the order; the ids are read only to break an exact tie of D2.
constexpr int kNbList = 8;

// down-candidate list of one lane: entry k at [k * blockDim.x + lane]
struct NbList {
    float* y;
    float* z;
    int* pos;
    __device__ __forceinline__ int at(int k) const
    {
        return k * (int)blockDim.x + (int)threadIdx.x;
    }
};

// does pair (pu, pd) at deviation d2 improve on the best (bu, bd) at best?
__device__ __forceinline__ bool nb_better(float d2, int pu, int pd, float best, int bu, int bd,
                                          const NbSrc& U, const NbSrc& D)
{
    if (bu < 0 || d2 < best) return true;
    if (!(d2 == best)) return false;
    const int idu = U.idg[pu], bidu = U.idg[bu];
    if (idu != bidu) return idu < bidu;
    return D.idg[pd] < D.idg[bd];
}

__device__ __forceinline__ void nb_pairs(const NbSrc& U, const NbSrc& D, float y, float z,
                                         float yu_c, float yd_c, int iyu0, int iyu1, int iyd0,
                                         int iyd1, int iz0, int iz1, const tpc_params& prm,
                                         const NbList& L, int& bu, int& bd)
{
    const float Wy = prm.nb_win_y, Wz = prm.nb_win_z, D2max = prm.nb_d2max;
    float best = 0.0f;
    int nd = 0;
    for (int izd = iz0; izd <= iz1; ++izd) {
        const int pd1 = D.first(izd, iyd1 + 1);
        for (int pd = D.first(izd, iyd0); pd < pd1; ++pd) {
            const float yd = D.yg[pd], zd = D.zg[pd];
            if (!(fabsf(yd - yd_c) <= Wy && fabsf(zd - z) <= Wz)) continue;
            if (nd < kNbList) {
                const int e = L.at(nd);
                L.y[e] = yd;
                L.z[e] = zd;
                L.pos[e] = pd;
            }
            ++nd;
        }
    }
    if (nd == 0) return;
    const bool listed = nd <= kNbList;
    for (int izu = iz0; izu <= iz1; ++izu) {
        const int pu1 = U.first(izu, iyu1 + 1);
        for (int pu = U.first(izu, iyu0); pu < pu1; ++pu) {
            const float yu = U.yg[pu], zu = U.zg[pu];
            if (!(fabsf(yu - yu_c) <= Wy && fabsf(zu - z) <= Wz)) continue;
            if (listed) {
                for (int k = 0; k < nd; ++k) {
                    const int e = L.at(k);
                    const float dy = (yu + L.y[e]) - (y + y);
                    const float dz = (zu + L.z[e]) - (z + z);
                    const float d2 = dy * dy + dz * dz;
                    if (!(d2 <= D2max)) continue;
                    const int pd = L.pos[e];
                    if (nb_better(d2, pu, pd, best, bu, bd, U, D)) {
                        best = d2;
                        bu = pu;
                        bd = pd;
                    }
                }
                continue;
            }
            for (int izd = iz0; izd <= iz1; ++izd) {
                const int pd1 = D.first(izd, iyd1 + 1);
                for (int pd = D.first(izd, iyd0); pd < pd1; ++pd) {
                    const float yd = D.yg[pd], zd = D.zg[pd];
                    if (!(fabsf(yd - yd_c) <= Wy && fabsf(zd - z) <= Wz)) continue;
                    const float dy = (yu + yd) - (y + y);
                    const float dz = (zu + zd) - (z + z);
                    const float d2 = dy * dy + dz * dz;
                    if (!(d2 <= D2max)) continue;
                    if (nb_better(d2, pu, pd, best, bu, bd, U, D)) {
                        best = d2;
                        bu = pu;
                        bd = pd;
                    }
                }
            }
        }
    }
}

// The same pair for windows that span at most kNbRows z rows of bins (the
// usual case), with fewer dependent memory round trips: the bin bounds of
// both neighbouring rows load together, then the first kNbBatch candidates
// of both rows, and only then are they compared.  A window with more rows,
// or more than kNbList down candidates, takes nb_pairs; the result is the
// same lexicographic minimum either way.
constexpr int kNbRows = 4;
constexpr int kNbBatch = 4;

// candidate e of a window whose z rows hold [lo[k], lo[k] + n[k])
__device__ __forceinline__ int nb_cand(int e, const int* lo, const int* n)
{
    int p = lo[0] + e;
#pragma unroll
    for (int k = 1; k < kNbRows; ++k) {
        e -= n[k - 1];
        if (e >= 0) p = lo[k] + e;
    }
    return p;
}

__device__ __forceinline__ void nb_pairs_near(const NbSrc& U, const NbSrc& D, float y, float z,
                                              float yu_c, float yd_c, int iyu0, int iyu1,
                                              int iyd0, int iyd1, int iz0, int iz1,
                                              const tpc_params& prm, const NbList& L, int& bu,
                                              int& bd)
{
    if (iz1 - iz0 >= kNbRows) {
        nb_pairs(U, D, y, z, yu_c, yd_c, iyu0, iyu1, iyd0, iyd1, iz0, iz1, prm, L, bu, bd);
        return;
    }
    const float Wy = prm.nb_win_y, Wz = prm.nb_win_z, D2max = prm.nb_d2max;
    int dlo[kNbRows], dn[kNbRows], ulo[kNbRows], un[kNbRows];
#pragma unroll
    for (int k = 0; k < kNbRows; ++k) {
        dlo[k] = ulo[k] = 0;
        dn[k] = un[k] = 0;
        if (iz0 + k <= iz1) {
            dlo[k] = D.first(iz0 + k, iyd0);
            dn[k] = D.first(iz0 + k, iyd1 + 1);
            ulo[k] = U.first(iz0 + k, iyu0);
            un[k] = U.first(iz0 + k, iyu1 + 1);
        }
    }
    int ndc = 0, nuc = 0;
#pragma unroll
    for (int k = 0; k < kNbRows; ++k) {
        dn[k] = dn[k] > dlo[k] ? dn[k] - dlo[k] : 0;
        un[k] = un[k] > ulo[k] ? un[k] - ulo[k] : 0;
        ndc += dn[k];
        nuc += un[k];
    }
    if (ndc == 0 || nuc == 0) return;
    float yb[kNbBatch], zb[kNbBatch], yu[kNbBatch], zu[kNbBatch];
    int pdb[kNbBatch], pub[kNbBatch];
#pragma unroll
    for (int j = 0; j < kNbBatch; ++j) {
        pdb[j] = nb_cand(j, dlo, dn);
        pub[j] = nb_cand(j, ulo, un);
        if (j < ndc) {
            yb[j] = D.yg[pdb[j]];
            zb[j] = D.zg[pdb[j]];
        }
        if (j < nuc) {
            yu[j] = U.yg[pub[j]];
            zu[j] = U.zg[pub[j]];
        }
    }
    // down candidates inside the window -> the lane's list
    int nd = 0;
    for (int b = 0; b < ndc; b += kNbBatch) {
        if (b > 0) {
#pragma unroll
            for (int j = 0; j < kNbBatch; ++j) {
                pdb[j] = nb_cand(b + j, dlo, dn);
                if (b + j < ndc) {
                    yb[j] = D.yg[pdb[j]];
                    zb[j] = D.zg[pdb[j]];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kNbBatch; ++j) {
            if (b + j >= ndc) break;
            if (!(fabsf(yb[j] - yd_c) <= Wy && fabsf(zb[j] - z) <= Wz)) continue;
            if (nd < kNbList) {
                const int e = L.at(nd);
                L.y[e] = yb[j];
                L.z[e] = zb[j];
                L.pos[e] = pdb[j];
            }
            ++nd;
        }
    }
    if (nd == 0) return;
    if (nd > kNbList) {
        nb_pairs(U, D, y, z, yu_c, yd_c, iyu0, iyu1, iyd0, iyd1, iz0, iz1, prm, L, bu, bd);
        return;
    }
    float best = 0.0f;
    for (int b = 0; b < nuc; b += kNbBatch) {
        if (b > 0) {
#pragma unroll
            for (int j = 0; j < kNbBatch; ++j) {
                pub[j] = nb_cand(b + j, ulo, un);
                if (b + j < nuc) {
                    yu[j] = U.yg[pub[j]];
                    zu[j] = U.zg[pub[j]];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kNbBatch; ++j) {
            if (b + j >= nuc) break;
            if (!(fabsf(yu[j] - yu_c) <= Wy && fabsf(zu[j] - z) <= Wz)) continue;
            for (int k = 0; k < nd; ++k) {
                const int e = L.at(k);
                const float dy = (yu[j] + L.y[e]) - (y + y);
                const float dz = (zu[j] + L.z[e]) - (z + z);
                const float d2 = dy * dy + dz * dz;
                if (!(d2 <= D2max)) continue;
                const int pd = L.pos[e];
                if (nb_better(d2, pub[j], pd, best, bu, bd, U, D)) {
                    best = d2;
                    bu = pub[j];
                    bd = pd;
                }
            }
        }
    }
}

// Best up/down pair of the hit at grid position p, candidates read from
// global memory (xs: the row positions, in LDS).  Candidates on rows r+1 and r-1 come from the bins
// covering the windows around the straight line from the origin through the
// hit; the exact window test and the pair deviation decide, ties go to the
// lower (up id, down id).
__device__ __forceinline__ void neighbours_one(
    int64_t p, const tpc_sector* __restrict__ sec, int n_rows, const float* xs,
    const tpc_params& prm, const int32_t* __restrict__ bin_start, const float* __restrict__ yg,
    const float* __restrict__ zg, const int32_t* __restrict__ idg,
    const int32_t* __restrict__ gsr, int32_t* __restrict__ up0, int32_t* __restrict__ down0,
    const NbList& L)
{
    const float Wy = prm.nb_win_y, Wz = prm.nb_win_z;
    const int v = gsr[p];
    const float y = yg[p], z = zg[p];
    // the hit's coordinates load with its row tag (one round trip): held
    // here, the compiler would otherwise sink their loads below the branch
    asm volatile("" ::"v"(y), "v"(z));
    const int r = v & 255;
    // The lanes of a wave hold consecutive grid positions, nearly always of
    // one sector: its record is then loaded at the wave-uniform address
    // (the scalar cache, a much shorter round trip than a vector load), and
    // per lane only when the wave spans two sectors.
    const int vf = __builtin_amdgcn_readfirstlane(v);
    const tpc_sector su = sec[vf >> 8];
    const bool mixed = __ballot((v >> 8) != (vf >> 8)) != 0ull;
    int bu = -1, bd = -1;
    if (r > 0 && r + 1 < n_rows) {
        tpc_sector s = su;
        if (mixed) s = sec[v >> 8];
        const float slope = y / xs[r];
        const float yu_c = slope * xs[r + 1];
        const float yd_c = slope * xs[r - 1];
        const int iyu0 = bin_of(yu_c - Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
        const int iyu1 = bin_of(yu_c + Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
        const int iyd0 = bin_of(yd_c - Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
        const int iyd1 = bin_of(yd_c + Wy * TPC_WIDEN, s.y0, s.inv_by, s.nby);
        const int iz0 = bin_of(z - Wz * TPC_WIDEN, s.z0, s.inv_bz, s.nbz);
        const int iz1 = bin_of(z + Wz * TPC_WIDEN, s.z0, s.inv_bz, s.nbz);
        const int per_row = s.nbz * s.nby;
        const NbSrc U{s.bin_base + (r + 1) * per_row, s.nby, bin_start, yg, zg, idg};
        const NbSrc D{s.bin_base + (r - 1) * per_row, s.nby, bin_start, yg, zg, idg};
        nb_pairs_near(U, D, y, z, yu_c, yd_c, iyu0, iyu1, iyd0, iyd1, iz0, iz1, prm, L, bu,
                      bd);
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

}  // namespace tpc
