// Nuclear cell items with Newton's third law (variant 4): every unordered
// pair inside r_nuc is evaluated once.  An item (a chunk of 32 targets of
// cell c, 8 lanes per target, as variant 3) stages the half stencil -- cell
// c itself and the 13 neighbours with a lexicographically positive offset
// -- screens and lists pairs as the compacting items do, and evaluates each
// listed pair once: the force on the target goes to the lane's accumulator,
// the reaction on the source (and the source's half of the pair energy) is
// added into a per-tile LDS accumulator of that source.  Pairs inside cell c
// are kept only when the source's sorted slot is above the target's, so
// each of them is evaluated by exactly one item.  When a tile's pairs are
// done, its sources' reactions go to a per-particle accumulator in global
// memory.
//
// Determinism without floating-point atomics: reactions are accumulated as
// 64-bit integers in units of 2^-43 MeV/fm (and MeV; react_fixed), whose
// sums do not depend on the order the lanes and items add them in.  One pair's reaction
// is rounded to 2^-44 (1e-13 MeV/fm); a particle's total stays below 2^20
// MeV/fm by a wide margin (a nuclear pair force is at most about 90 MeV/fm).
// The combine kernel adds the accumulated reactions to the target-side sums
// and clears the accumulators for the next launch.
#pragma once

#include "pair_items.hpp"

namespace pasta {

constexpr int HALF_TPT = 8;     // lanes per target
constexpr int HALF_TILE = 256;  // sources per LDS tile

// One pair's force on the target (MeV/fm, in the policy's units before
// f_scale) and energy V, zero outside the cutoff or when !valid.
__device__ __forceinline__ void pair_terms(const Fp64Policy::Src& me, const Fp64Policy::Lds& s,
                                           double B_L, double B, const NucConsts& k, bool valid,
                                           double& fx, double& fy, double& fz, double& v,
                                           bool& in)
{
    const double dx = nearest_image(me.x - s.x, k.L, k.hL);
    const double dy = nearest_image(me.y - s.y, k.L, k.hL);
    const double dz = nearest_image(me.z - s.z, k.L, k.hL);
    const double r2 = dx * dx + dy * dy + dz * dz;
    in = valid && r2 < k.rc2;
    const double g = in ? exp_nonpos(r2 * k.cg) : 0.0;
    const double fs = g * fma(k.A2, g, B_L);
    fx = fs * dx;
    fy = fs * dy;
    fz = fs * dz;
    v = g * fma(k.a, g, B);
}
__device__ __forceinline__ void pair_terms(const MixedPolicy::Src& me, const MixedPolicy::Lds& s,
                                           float B_L, float B, const NucConsts& k, bool valid,
                                           float& fx, float& fy, float& fz, float& v, bool& in)
{
    const float dx = (float)(int32_t)(me.x - s.x);
    const float dy = (float)(int32_t)(me.y - s.y);
    const float dz = (float)(int32_t)(me.z - s.z);
    float r2 = dx * dx + dy * dy + dz * dz;
    in = valid && r2 < k.thr_q;
    r2 = in ? r2 : 3.0e38f;  // exp2 underflows to exactly 0 outside the cutoff
    const float g = __builtin_amdgcn_exp2f(r2 * k.cgq);
    const float fs = g * fmaf(k.A2f, g, B_L);
    fx = fs * dx;
    fy = fs * dy;
    fz = fs * dz;
    v = g * fmaf(k.af, g, B);
}

template <class P>
constexpr int nuclear_half_lds_bytes()
{
    return HALF_TILE * ((int)sizeof(typename P::Lds) + 8 + 4 + 32) + NUC_CAP * WG * 2 +
           ITEM_LDS_BYTES;
}

// react: [4][A.react_stride] int64 accumulators per sorted slot (fx, fy, fz,
// V), zero on entry to the launch.  Requires at least 3 cells per side.
template <class P, int MODE>
__device__ void nuclear_item_half(const typename P::Src* __restrict__ stg, const NucArgs& A,
                                  const NucConsts& k, int item, char* lds,
                                  unsigned long long* __restrict__ react)
{
    using Lds = typename P::Lds;
    using F = typename P::CAcc;
    constexpr int T = HALF_TILE;
    constexpr int TPT = HALF_TPT;
    unsigned long long* racc = reinterpret_cast<unsigned long long*>(lds);  // [T][4]
    Lds* src = reinterpret_cast<Lds*>(racc + 4 * T);
    uint2* tst = reinterpret_cast<uint2*>(src + T);
    int* tslot = reinterpret_cast<int*>(tst + T);
    uint16_t* lists = reinterpret_cast<uint16_t*>(tslot + T);
    const ItemLds L = item_lds(reinterpret_cast<char*>(lists + NUC_CAP * WG));
    const int tid = threadIdx.x;

    const ItemTarget t = item_target<TPT>(A, item);
    const typename P::Src me = stg[t.slot];
    const uint3 mef = P::fixed(me, k);
    const uint32_t me_xy16 = (mef.x >> 16) | (mef.y & 0xffff0000u);
    item_setup<14>(A, L, t.c, true, t.active && t.q == 0, mef);
    // the target cell's own slot ranges (pairs inside it: source slot above)
    const int pb = t.c * A.sub, nbn = (A.C + t.c) * A.sub;
    const int own_p0 = A.start[pb], own_p1 = A.start[pb + A.sub];
    const int own_n0 = A.start[nbn], own_n1 = A.start[nbn + A.sub];
    for (int i = tid; i < 4 * T; i += WG)
        racc[i] = 0ull;

    const double fsc = P::f_scale(k);  // fm per coordinate unit (mixed) or 1
    typename P::Acc acc;
    {
        const auto BLp = P::bl(k, t.tprot), Bp = P::bv(k, t.tprot);    // proton sources
        const auto BLn = P::bl(k, !t.tprot), Bn = P::bv(k, !t.tprot);  // neutron sources
        typename P::Part part;
        const int q = t.q;
        constexpr int DU = P::DRAIN_U;
        auto drain = [&](int cnt, int kb) {
            for (int kk = 0; __ballot(kk < cnt); kk += DU) {
                int j[DU];
                bool v[DU];
                Lds sv[DU];
#pragma unroll
                for (int u = 0; u < DU; ++u) {
                    const int raw = lists[min(kk + u, NUC_CAP - 1) * WG + tid];
                    v[u] = kk + u < cnt;
                    j[u] = v[u] ? raw : 0;
                    sv[u] = src[j[u]];
                }
#pragma unroll
                for (int u = 0; u < DU; ++u) {
                    const int ss = tslot[j[u]];
                    const bool own = (ss >= own_p0 && ss < own_p1) || (ss >= own_n0 && ss < own_n1);
                    const bool ok = v[u] && !(own && ss <= t.slot);
                    const bool pu = j[u] < kb;  // protons first in the tile
                    F fx, fy, fz, e;
                    bool in;
                    pair_terms(me, sv[u], pu ? BLp : BLn, pu ? Bp : Bn, k, ok, fx, fy, fz, e, in);
                    part.fx += fx;
                    part.fy += fy;
                    part.fz += fz;
                    if (MODE != MODE_FORCE)
                        part.e += e;
                    if (MODE == MODE_COUNT)
                        part.np += in ? 2u : 0u;  // the pair counts for both members
                    if (in) {
                        unsigned long long* r = racc + 4 * j[u];
                        atomicAdd(r + 0, react_fixed(-(double)fx * fsc));
                        atomicAdd(r + 1, react_fixed(-(double)fy * fsc));
                        atomicAdd(r + 2, react_fixed(-(double)fz * fsc));
                        if (MODE != MODE_FORCE)
                            atomicAdd(r + 3, react_fixed((double)e));
                    }
                }
            }
        };
        const int thr = t.active ? k.thr16 : INT_MIN;
        const bool wave_live = __ballot(t.active) != 0ull;
        auto process = [&](int n, int kb) {
            if (wave_live) {
                int cnt = 0;
                constexpr int STEP = TPT * NUC_U;
                const int nfull = (n / STEP) * STEP;
                for (int j0 = 0; j0 < nfull; j0 += STEP) {
                    uint2 tv[NUC_U];
#pragma unroll
                    for (int u = 0; u < NUC_U; ++u)
                        tv[u] = tst[j0 + u * TPT + q];
#pragma unroll
                    for (int u = 0; u < NUC_U; ++u) {
                        const int j = j0 + u * TPT + q;
                        lists[cnt * WG + tid] = (uint16_t)j;
                        cnt += screen16(me_xy16, mef.z, tv[u]) < thr ? 1 : 0;
                    }
                    if (__ballot(cnt > NUC_CAP - NUC_U)) {
                        drain(cnt, kb);
                        cnt = 0;
                    }
                }
#pragma unroll
                for (int u = 0; u < NUC_U; ++u) {
                    const int j = nfull + u * TPT + q;
                    if (j < n) {
                        lists[cnt * WG + tid] = (uint16_t)j;
                        cnt += screen16(me_xy16, mef.z, tst[j]) < thr ? 1 : 0;
                    }
                }
                drain(cnt, kb);
                P::fold(acc, part);
            }
            // every pair of this tile is in: its sources' reactions go out
            __syncthreads();
            for (int p = tid; p < n; p += WG) {
                unsigned long long* r = racc + 4 * p;
                unsigned long long* g = react + tslot[p];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (r[c] != 0ull)
                        atomicAdd(g + c * A.react_stride, r[c]);
                    r[c] = 0ull;
                }
            }
            __syncthreads();
        };
        stage_neighbourhood<P, T, 14>(
            stg, k, L, k.thr_stage16,
            [&](int pos, const Lds& e, const uint3& f, int slot) {
                src[pos] = e;
                tst[pos] = make_uint2((f.x >> 16) | (f.y & 0xffff0000u), f.z);
                tslot[pos] = slot;
            },
            process);
    }
    nuclear_finish<P, TPT, true, MODE>(A, k, acc, t, item, false, L);
}

}  // namespace pasta
