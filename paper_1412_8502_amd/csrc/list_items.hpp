// Neighbour lists with a halo for the nuclear force (Sec. II.B.1: each
// target lists the sources within r_nuc + delta_r; forces use only those
// within r_nuc; the lists are rebuilt, all at once, only when particles may
// have moved far enough for a source outside a list to be in range).
//
// Work items are the cell items of the cell list built with r_cut = r_nuc +
// delta_r, with LIST_TPT lanes per target.  A target's list is split over
// its lanes: lane q keeps the qualifying candidates it screened (every
// LIST_TPT-th staged source), in staging order.
//
// Memory: one pool of rows of WG entries (int32 sorted slots).  Item i owns
// rows [hdr[i].x, hdr[i].x + hdr[i].y); entry k of lane tid is at row
// hdr.x + k, column tid, so the lanes of a wavefront read consecutive words.
// cnt[i * WG + tid] is the lane's entry count.  A build makes two passes over
// the staged neighbourhood: the first counts, the workgroup takes
// max(count) rows from the pool with one atomic, the second writes.  If the
// pool runs out the build sets ctl->overflow and the force items fall back
// to the screened cell sweep over the same (stale but still sufficient)
// cells until the next build.
//
// Why stale cells and lists stay sufficient: with u_i the nearest-image
// displacement of particle i since the build and L_b the box side then, a
// pair's nearest-image separation at the build was at most its separation
// now + |u_i| + |u_j| + sqrt(3) |L - L_b| (the image vector has components
// in {-1, 0, 1}).  So while 2 max|u| + sqrt(3) |L - L_b| < delta_r every
// pair inside r_nuc now was inside r_nuc + delta_r then: it is in the lists
// and its cells were neighbours (cells are at least r_nuc + delta_r wide).
#pragma once

#include "pair_items.hpp"

namespace pasta {

constexpr int LIST_TPT = 8;                // lanes per target
constexpr int LIST_CHUNK = WG / LIST_TPT;  // targets per work item
constexpr int LIST_TILE = 1024;            // staged candidates per LDS tile
constexpr int LIST_U = 4;                  // list entries per lane in flight

struct ListArgs {
    ListCtl* ctl;
    int2* hdr;        // [item_max] (first row, rows)
    int32_t* cnt;     // [item_max * WG]
    int32_t* pool;    // [pool_rows * WG]
    int64_t pool_rows;
};

constexpr int list_build_lds_bytes() { return LIST_TILE * 16 + ITEM_LDS_BYTES + 16; }

// Builds item `item`'s lists: sources s != target with nearest-image
// |d|^2 < r_list^2 (kl = the constants for r_list, with its rounding
// margin) from the fixed-point coordinates of the staging array.
template <class P>
__device__ void list_build_item(const typename P::Src* __restrict__ stg, const NucArgs& A,
                                const NucConsts& kl, const ListArgs& LA, int item, char* lds)
{
    uint4* cand = reinterpret_cast<uint4*>(lds);  // fixed x, y, z, sorted slot
    const ItemLds L = item_lds(lds + LIST_TILE * 16);
    int* bcast = L.misc + 22;
    const int tid = threadIdx.x;
    const ItemTarget t = item_target<LIST_TPT>(A, item);
    const uint3 mef = P::fixed(stg[t.slot], kl);
    item_setup(A, L, t.c, true, t.active && t.q == 0, mef);

    const float thr = t.active ? kl.thr_q : -1.0f;
    const int me_slot = t.active ? t.slot : -1;
    int cnt = 0, row0 = 0;
    for (int pass = 0; pass < 2; ++pass) {
        cnt = 0;
        int32_t* out = LA.pool + ((int64_t)row0 * WG + tid);
        stage_neighbourhood<P, LIST_TILE>(
            stg, kl, L, kl.thr_stage16,
            [&](int pos, const typename P::Lds&, const uint3& f, int slot) {
                cand[pos] = make_uint4(f.x, f.y, f.z, (uint32_t)slot);
            },
            [&](int n, int) {
                for (int j = t.q; j < n; j += LIST_TPT) {
                    const uint4 s = cand[j];
                    const float dx = (float)(int32_t)(mef.x - s.x);
                    const float dy = (float)(int32_t)(mef.y - s.y);
                    const float dz = (float)(int32_t)(mef.z - s.z);
                    const float r2 = dx * dx + dy * dy + dz * dz;
                    const bool in = r2 < thr && (int)s.w != me_slot;
                    if (pass == 1 && in)
                        out[(int64_t)cnt * WG] = (int32_t)s.w;
                    cnt += in ? 1 : 0;
                }
            });
        if (pass == 0) {
            // rows = the largest lane count of the item
            int m = cnt;
            for (int o = 32; o >= 1; o >>= 1)
                m = max(m, __shfl_xor(m, o, 64));
            if ((tid & 63) == 0)
                L.misc[6 + (tid >> 6)] = m;
            __syncthreads();
            if (tid == 0) {
                int rows = 0;
                for (int w = 0; w < WG / 64; ++w)
                    rows = max(rows, L.misc[6 + w]);
                unsigned long long r0 =
                    atomicAdd(&LA.ctl->pool_used, (unsigned long long)rows);
                atomicMax(&LA.ctl->max_rows, (unsigned)rows);
                const bool ok = r0 + (unsigned long long)rows <= (unsigned long long)LA.pool_rows;
                if (!ok)
                    atomicOr(&LA.ctl->overflow, 1);
                bcast[0] = ok ? (int)r0 : -1;
                bcast[1] = rows;
                LA.hdr[item] = make_int2(ok ? (int)r0 : 0, ok ? rows : 0);
            }
            __syncthreads();
            row0 = bcast[0];
            if (row0 < 0)
                return;  // out of list memory: the force items fall back to cells
        }
    }
    LA.cnt[(int64_t)item * WG + tid] = cnt;
}

// Nuclear force on the item's targets from their lists (the same contract
// as nuclear_item_compact; the target itself is not in its list).
template <class P, int MODE>
__device__ void list_force_item(const typename P::Src* __restrict__ stg, const NucArgs& A,
                                const NucConsts& k, const ListArgs& LA, int item, char* lds)
{
    using Lds = typename P::Lds;
    const ItemLds L = item_lds(lds);
    const ItemTarget t = item_target<LIST_TPT>(A, item);
    const int tid = threadIdx.x;
    const typename P::Src me = stg[t.slot];
    const int m = t.active ? LA.cnt[(int64_t)item * WG + tid] : 0;
    const int2 h = LA.hdr[item];
    const int32_t* lp = LA.pool + ((int64_t)h.x * WG + tid);
    const bool mp = P::is_proton(me);
    const auto BLlike = P::bl(k, true), Blike = P::bv(k, true);
    const auto BLun = P::bl(k, false), Bun = P::bv(k, false);

    typename P::Acc acc;
    typename P::Part part;
    int nxt[LIST_U];
#pragma unroll
    for (int u = 0; u < LIST_U; ++u)
        nxt[u] = u < m ? lp[(int64_t)u * WG] : t.slot;
    for (int j0 = 0; j0 < m; j0 += LIST_U) {
        Lds s[LIST_U];
#pragma unroll
        for (int u = 0; u < LIST_U; ++u)
            s[u] = P::load(stg, nxt[u]);
#pragma unroll
        for (int u = 0; u < LIST_U; ++u) {
            const int j = j0 + LIST_U + u;
            nxt[u] = j < m ? lp[(int64_t)j * WG] : t.slot;
        }
#pragma unroll
        for (int u = 0; u < LIST_U; ++u) {
            const bool like = P::is_proton(s[u]) == mp;
            P::template pair<MODE>(me, s[u], like ? BLlike : BLun, like ? Blike : Bun, k, part,
                                    j0 + u < m);
        }
        if ((j0 & 127) == 128 - LIST_U)  // FP32 partial sums over at most 128 pairs
            P::fold(acc, part);
    }
    P::fold(acc, part);
    nuclear_finish<P, LIST_TPT, true, MODE>(A, k, acc, t, item, false, L);
}

}  // namespace pasta
