// Pair-force kernels (a2 nuclear, a3 Coulomb) for one system.  The work
// items themselves live in pair_items.hpp and list_items.hpp, shared with
// the batched kernels.
//
// Coulomb: all proton pairs; protons occupy sorted slots [0, Z).  Gather
// form: a workgroup owns 256 targets (one per thread) and one of S source
// ranges, the sources streaming through an LDS tile as wave-wide broadcasts.
// Pairwise form: a workgroup owns a pair of 256-proton super-blocks and
// evaluates each proton pair once, moving sources and their reactions along
// the lanes.  Either way every proton gets S partial sums, added in fixed
// order afterwards; or, in the fused launch in mixed precision, the pairwise
// items add each proton's sum over the item into a 64-bit fixed-point
// accumulator with integer atomics (order-independent totals, no partials).
//
// Nuclear: cell items.  A workgroup owns a chunk of the targets of one cell
// (taken octant by octant); the neighbour cells' particles within range of
// the chunk are staged in LDS; 4 or 8 adjacent lanes share one target
// (dense sweep, or screen + per-lane pair lists + drain), and combine by
// shuffles.  The list form reads per-target neighbour lists instead.
//
// Fused form (default): one launch holds every nuclear item and then every
// Coulomb item; the nuclear items write raw (F, V) per sorted slot and
// k_combine adds the partials, writes F (and E) at the slot or the caller
// index, applies the second half kick and, in a simulation, the next step's
// drift and binning.  Unfused form: k_coulomb / k_coulomb_pair, then the
// nuclear kernel whose epilogue does the combine.
#include <type_traits>

#include "half_items.hpp"
#include "list_items.hpp"

namespace pasta {

namespace {

template <class P, bool E, bool CUT>
__global__ __launch_bounds__(WG) void k_coulomb(const typename P::Src* __restrict__ stg, int Z,
                                                int per_split, CoulConsts k, void* part,
                                                CoulCut cc)
{
    __shared__ __align__(16) char lds[coulomb_lds_bytes<P>()];
    using PT = typename P::CPart;
    coulomb_item<P, E, PT, CUT>(stg, Z, per_split, k, static_cast<PT*>(part), blockIdx.x,
                                blockIdx.y, lds, cc);
}

template <class P, bool E>
__global__ __launch_bounds__(WG) void k_coulomb_pair(const typename P::Src* __restrict__ stg,
                                                     int Z, CoulConsts k, void* part)
{
    __shared__ __align__(16) char lds[coulomb_pair_lds_bytes<P>()];
    using PT = typename P::CPart;
    coulomb_pair_item<P, E>(stg, Z, k, static_cast<PT*>(part), blockIdx.x, lds);
}

template <class P, bool NUC, int MODE>
__global__ __launch_bounds__(WG) void k_nuclear(const typename P::Src* __restrict__ stg,
                                                NucArgs A, const int32_t* __restrict__ n_items,
                                                NucConsts k)
{
    __shared__ __align__(16) char lds[nuclear_lds_bytes<P>()];
    if ((int)blockIdx.x >= *n_items)
        return;
    nuclear_item<P, NUC, MODE>(stg, A, k, blockIdx.x, lds);
}

template <class P, int TPT, bool NUC, int MODE>
__global__ __launch_bounds__(WG) void k_nuclear_compact(const typename P::Src* __restrict__ stg,
                                                        NucArgs A,
                                                        const int32_t* __restrict__ n_items,
                                                        NucConsts k)
{
    __shared__ __align__(16) char lds[nuclear_compact_lds_bytes<P>()];
    if ((int)blockIdx.x >= *n_items)
        return;
    nuclear_item_compact_t<P, TPT, NUC, MODE>(stg, A, k, blockIdx.x, lds);
}

// List form of a nuclear item: the lists of the last build, or, when that
// build ran out of list memory, the screened cell sweep over its cells (the
// grid of the last build is read from the control block).
template <class P, int MODE>
__device__ void nuclear_item_listed(const typename P::Src* __restrict__ stg, const NucArgs& A,
                                    const NucConsts& k, const ListArgs& LA, int item, char* lds)
{
    NucArgs B = A;
    B.nc = LA.ctl->nc;
    B.C = LA.ctl->C;
    if (LA.ctl->overflow)
        nuclear_item_compact_t<P, LIST_TPT, true, MODE>(stg, B, k, item, lds);
    else
        list_force_item<P, MODE>(stg, B, k, LA, item, lds);
}

template <class P, int MODE>
__global__ __launch_bounds__(WG) void k_nuclear_list(const typename P::Src* __restrict__ stg,
                                                     NucArgs A,
                                                     const int32_t* __restrict__ n_items,
                                                     NucConsts k, ListArgs LA)
{
    __shared__ __align__(16) char lds[nuclear_compact_lds_bytes<P>()];
    if ((int)blockIdx.x >= *n_items)
        return;
    nuclear_item_listed<P, MODE>(stg, A, k, LA, blockIdx.x, lds);
}

// Gated on the rebuild decision of this step.
template <class P>
__global__ __launch_bounds__(WG) void k_list_build(const typename P::Src* __restrict__ stg,
                                                   NucArgs A, const int32_t* __restrict__ n_items,
                                                   NucConsts kl, ListArgs LA)
{
    __shared__ __align__(16) char lds[list_build_lds_bytes()];
    if ((int)blockIdx.x >= *n_items || LA.ctl->rebuild == 0)
        return;
    list_build_item<P>(stg, A, kl, LA, blockIdx.x, lds);
}

// Fused form: blocks [0, item_max) are nuclear cell tiles (raw nuclear
// force and energy per sorted slot), blocks after them Coulomb tiles.
// One instantiation per nuclear variant (V), so each kernel carries only
// its own item code (registers and LDS sized for it).
template <class P, int V>
constexpr int fused_lds_bytes()
{
    static_assert(coulomb_pair_lds_bytes<P>() <= coulomb_lds_bytes<P>(), "LDS of the pair form");
    constexpr int a = coulomb_lds_bytes<P>();
    constexpr int b = V == 0   ? nuclear_lds_bytes<P>()
                      : V == 4 ? nuclear_half_lds_bytes<P>()
                      : V == 5 ? nuclear_compact_lds_bytes<P, NUC_TILE_SHORT>()
                      : V == 6 ? nuclear_compact_lds_bytes<P, NUC_TILE_LONG>()
                               : nuclear_compact_lds_bytes<P>();
    return a > b ? a : b;
}

// CF: Coulomb form, 0 = gather tiles (coul_blocks x splits items), 1 =
// pairwise super-block items, 2 = gather tiles with a finite cutoff, 3 =
// pairwise items that add into the per-proton fixed-point accumulators
// (A.react) instead of writing partials.
template <class P, int MODE, int V, int CF>
__global__ __launch_bounds__(WG) void k_forces_fused(const typename P::Src* __restrict__ stg,
                                                     NucArgs A, const int32_t* __restrict__ n_items,
                                                     int item_max, NucConsts k, int Z,
                                                     int per_split, int coul_blocks,
                                                     CoulConsts kc, void* part_raw, ListArgs LA,
                                                     CoulCut cc)
{
    __shared__ __align__(16) char lds[fused_lds_bytes<P, V>()];
    using PT = typename P::CPart;
    PT* part = static_cast<PT*>(part_raw);
    const int g = blockIdx.x;
    if (g < item_max) {
        if (g >= *n_items)
            return;
        if constexpr (V == 2)
            nuclear_item_listed<P, MODE>(stg, A, k, LA, g, lds);
        else if constexpr (V == 3)
            nuclear_item_compact_t<P, 8, true, MODE>(stg, A, k, g, lds);
        else if constexpr (V == 4)
            nuclear_item_half<P, MODE>(stg, A, k, g, lds, A.react);
        else if constexpr (V == 5)
            nuclear_item_compact_t<P, 8, true, MODE, NUC_TILE_SHORT>(stg, A, k, g, lds);
        else if constexpr (V == 6)
            nuclear_item_compact_t<P, 8, true, MODE, NUC_TILE_LONG>(stg, A, k, g, lds);
        else if constexpr (V == 1)
            nuclear_item_compact<P, true, MODE>(stg, A, k, g, lds);
        else
            nuclear_item<P, true, MODE>(stg, A, k, g, lds);
    } else {
        const int h = g - item_max;
        if constexpr (CF == 1)
            coulomb_pair_item<P, MODE != MODE_FORCE>(stg, Z, kc, part, h, lds);
        else if constexpr (CF == 3)
            coulomb_pair_item<P, MODE != MODE_FORCE>(
                stg, Z, kc, FixedPart{A.react, A.err, A.react_stride}, h, lds);
        else
            coulomb_item<P, MODE != MODE_FORCE, PT, CF == 2>(stg, Z, per_split, kc, part,
                                                             h % coul_blocks, h / coul_blocks, lds,
                                                             cc);
    }
}

// F = nuclear + Coulomb partials per sorted slot, written at perm[slot] (or
// the slot), with the optional second half kick and per-block kinetic
// energy.  With has_next (sorted order): then also the next step's half
// kick, drift and binning of the slot (nd), which the drift kernel would
// otherwise do at the start of the next step.
// Blocks [0, zb) take the protons, COMB_LANES lanes per proton: lane q adds
// the partials s = q, q + COMB_LANES, ... in order, the lanes then combine
// by a fixed shuffle tree and the first lane does the per-slot work (so a
// proton's S partial loads are spread over several lanes, all in flight).
// Blocks [zb, ...) take the neutrons, one lane each.  The slot's own loads
// (nuclear part, velocity, position, species, reactions) are issued before
// the partials, so the two latencies overlap.  react (optional): the
// fixed-point accumulators of slots [0, react_n) (Newton-3 reactions of
// every slot, and/or the Coulomb sums of the protons), added and cleared
// for the next launch; with the Coulomb sums there the caller passes no
// partials (S = 0, Z = zb = 0: one lane per slot).
constexpr int COMB_LANES = 8;
constexpr int COMB_UNROLL = 8;
__host__ __device__ inline int64_t combine_proton_blocks(int64_t Z)
{
    return (Z * COMB_LANES + WG - 1) / WG;
}

template <class PT>
__global__ __launch_bounds__(WG) void k_combine(const double4* __restrict__ fnuc,
                                                const PT* __restrict__ part, int S, int Z,
                                                int zb, const int32_t* __restrict__ perm,
                                                int64_t n, double* __restrict__ force,
                                                double* __restrict__ epot, double* vel, double hdtm,
                                                double mass, double* __restrict__ ke_part,
                                                int32_t* __restrict__ n_ke, uint32_t* err,
                                                NextDrift nd, int has_next,
                                                unsigned long long* __restrict__ react,
                                                int64_t react_n)
{
    __shared__ double red[WG / 64];
    const bool prot = (int)blockIdx.x < zb;
    int64_t sl;
    int q = 0;
    if (prot) {
        const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
        sl = t / COMB_LANES;
        q = (int)(t % COMB_LANES);
    } else {
        sl = (int64_t)Z + (int64_t)(blockIdx.x - zb) * WG + threadIdx.x;
    }
    const bool lead = q == 0 && sl < (prot ? (int64_t)Z : n);
    const bool has_r = react && sl < react_n;

    double4 fn = make_double4(0.0, 0.0, 0.0, 0.0);
    double v0[3] = {0.0, 0.0, 0.0}, x[3] = {0.0, 0.0, 0.0};
    unsigned long long rq[4] = {0ull, 0ull, 0ull, 0ull};
    int64_t id = sl;
    int spc = 0;
    if (lead) {
        fn = fnuc[sl];
        if (has_r) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
                rq[c] = react[c * n + sl];
        }
        id = perm ? perm[sl] : sl;
        if (vel) {
#pragma unroll
            for (int d = 0; d < 3; ++d)
                v0[d] = vel[3 * id + d];
            if (has_next) {
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    x[d] = nd.pos[3 * sl + d];
                spc = nd.species[sl];
            }
        }
    }

    double cx = 0.0, cy = 0.0, cz = 0.0, cw = 0.0;
    if (prot) {
        if (sl < Z) {
            for (int s = q; s < S; s += COMB_UNROLL * COMB_LANES) {
                PT v[COMB_UNROLL];
#pragma unroll
                for (int u = 0; u < COMB_UNROLL; ++u) {
                    const int k = s + u * COMB_LANES;
                    if (k < S)
                        v[u] = part[(int64_t)k * Z + sl];
                    else
                        v[u] = PT{0, 0, 0, 0};
                }
#pragma unroll
                for (int u = 0; u < COMB_UNROLL; ++u) {
                    cx += (double)v[u].x;
                    cy += (double)v[u].y;
                    cz += (double)v[u].z;
                    cw += (double)v[u].w;
                }
            }
        }
#pragma unroll
        for (int m = 1; m < COMB_LANES; m <<= 1) {
            cx += __shfl_xor(cx, m, COMB_LANES);
            cy += __shfl_xor(cy, m, COMB_LANES);
            cz += __shfl_xor(cz, m, COMB_LANES);
            cw += __shfl_xor(cw, m, COMB_LANES);
        }
    }
    double ke = 0.0;
    if (lead) {
        double rx = 0.0, ry = 0.0, rz = 0.0, rw = 0.0;
        if (has_r) {
            // accumulated reactions and sums (fixed point), cleared for the next launch
            rx = (double)(long long)rq[0] * REACT_UNIT;
            ry = (double)(long long)rq[1] * REACT_UNIT;
            rz = (double)(long long)rq[2] * REACT_UNIT;
            rw = (double)(long long)rq[3] * REACT_UNIT;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                react[c * n + sl] = 0ull;
        }
        const double Fx = (fn.x + rx) + cx, Fy = (fn.y + ry) + cy, Fz = (fn.z + rz) + cz,
                     V = (fn.w + rw) + cw;
        force[3 * id + 0] = Fx;
        force[3 * id + 1] = Fy;
        force[3 * id + 2] = Fz;
        if (epot)
            epot[id] = 0.5 * V;
        if (!(isfinite(Fx) && isfinite(Fy) && isfinite(Fz)))
            atomicOr(err, ERR_NONFINITE_FORCE);
        if (vel) {
            const double vx = v0[0] + hdtm * Fx, vy = v0[1] + hdtm * Fy, vz = v0[2] + hdtm * Fz;
            ke = 0.5 * mass * (vx * vx + vy * vy + vz * vz);
            if (has_next) {
                double v[3] = {vx, vy, vz};
                const double f[3] = {Fx, Fy, Fz};
                const uint32_t bad = drift_update(x, v, f, nd.step);
                if (bad)
                    atomicOr(err, bad);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    vel[3 * sl + d] = v[d];
                    nd.pos[3 * sl + d] = x[d];
                }
                const int bin = particle_bin(x[0], x[1], x[2], spc == 1, nd.inv_w, nd.nc, nd.C,
                                             nd.sub);
                nd.key[sl] = bin;
                wave_aggregated_add(nd.count, bin);
            } else {
                vel[3 * id + 0] = vx;
                vel[3 * id + 1] = vy;
                vel[3 * id + 2] = vz;
            }
        }
    }
    if (ke_part) {
        for (int m = 32; m >= 1; m >>= 1)
            ke += __shfl_xor(ke, m, 64);
        if ((threadIdx.x & 63) == 0)
            red[threadIdx.x >> 6] = ke;
        __syncthreads();
        if (threadIdx.x == 0) {
            ke_part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
            if (blockIdx.x == 0)
                *n_ke = (int32_t)gridDim.x;
        }
    }
}

template <class F>
void with_mode(int mode, F f)
{
    if (mode == MODE_COUNT)
        f(std::integral_constant<int, MODE_COUNT>());
    else if (mode == MODE_ENERGY)
        f(std::integral_constant<int, MODE_ENERGY>());
    else
        f(std::integral_constant<int, MODE_FORCE>());
}

template <class P>
void nuclear_dispatch(const typename P::Src* stg, const NucArgs& a, const int32_t* n_items,
                      const NucConsts& k, bool nuc, int mode, int variant, unsigned grid,
                      hipStream_t s)
{
    if (!nuc) {
        k_nuclear<P, false, MODE_ENERGY><<<grid, WG, 0, s>>>(stg, a, n_items, k);
        return;
    }
    with_mode(mode, [&](auto mt) {
        constexpr int M = decltype(mt)::value;
        if (variant == 3)
            k_nuclear_compact<P, 8, true, M><<<grid, WG, 0, s>>>(stg, a, n_items, k);
        else if (variant == 1)
            k_nuclear_compact<P, NUC_TPT, true, M><<<grid, WG, 0, s>>>(stg, a, n_items, k);
        else
            k_nuclear<P, true, M><<<grid, WG, 0, s>>>(stg, a, n_items, k);
    });
}

}  // namespace

int nuclear_chunk_for(int variant)
{
    return (variant >= 2) ? LIST_CHUNK : NUC_CHUNK;
}

static ListArgs list_args(const ListBuf* lb)
{
    ListArgs la{};
    if (lb) {
        la.ctl = lb->ctl;
        la.hdr = lb->hdr;
        la.cnt = lb->cnt;
        la.pool = lb->pool;
        la.pool_rows = lb->pool_rows;
    }
    return la;
}

int64_t list_pool_rows(int64_t n, double L_min, double r_list, int64_t item_max, double scale)
{
    // expected list entries per lane at the densest box, plus a Poisson
    // margin for the largest lane of an item, times the safety scale
    const double rho = (double)n / (L_min * L_min * L_min);
    const double per_lane = rho * (4.0 / 3.0) * M_PI * r_list * r_list * r_list / LIST_TPT;
    const double rows_item = 1.5 * per_lane + 4.0 * std::sqrt(per_lane) + 8.0;
    double rows = std::ceil((double)item_max * rows_item * (scale > 0.0 ? scale : 1.0));
    return rows < 1.0 ? 1 : (int64_t)rows;
}

size_t listbuf_carve(Carver& cv, ListBuf* out, int64_t n, int64_t item_max, int64_t pool_rows)
{
    ListBuf lb{};
    lb.ctl = cv.take<ListCtl>(1);
    lb.xb = cv.take<double>(3 * (size_t)n);
    lb.hdr = cv.take<int2>((size_t)item_max);
    lb.cnt = cv.take<int32_t>((size_t)item_max * WG);
    lb.pool = cv.take<int32_t>((size_t)pool_rows * WG);
    lb.pool_rows = pool_rows;
    if (out)
        *out = lb;
    return cv.size();
}

void launch_list_build(int precision, const ForceBuf& fb, const CellBuf& cb, const Grid& g,
                       const ListBuf& lb, const PairParams& pp, hipStream_t s, Timer* t)
{
    PairParams pl = pp;
    pl.r_nuc = (pp.r_nuc + lb.skin) * (1.0 + 1e-5);  // a superset: rounding margin
    const NucConsts kl = make_nuc_consts(pl);
    NucArgs a{};
    a.start = cb.start;
    a.items = cb.items;
    a.perm = cb.perm;
    a.nc = g.nc;
    a.C = g.C;
    a.sub = g.sub;
    const ListArgs la = list_args(&lb);
    timer_begin(t, KC_LIST, s);
    if (precision == PASTA_FP64)
        k_list_build<Fp64Policy><<<(unsigned)cb.item_max, WG, 0, s>>>(fb.stg64, a, cb.n_items,
                                                                       kl, la);
    else
        k_list_build<MixedPolicy><<<(unsigned)cb.item_max, WG, 0, s>>>(fb.stgq, a, cb.n_items,
                                                                       kl, la);
    timer_end(t, KC_LIST, s);
}

int coulomb_splits(int64_t Z, int64_t cap)
{
    if (Z <= 0)
        return 0;
    const int req = g_tuning.coulomb_splits;
    int64_t s = req > 0 ? req : 524288 / Z;
    s = s < 1 ? 1 : (s > 32 ? 32 : s);
    // the partial-sum buffer holds cap >= n >= Z entries
    while (s > 1 && s * Z > cap)
        --s;
    return (int)s;
}

int coulomb_pair_plan_supers(int64_t Z) { return coulomb_pair_supers(Z); }

CoulPlan coulomb_plan(int64_t Z, int64_t coul_max, bool cut, bool fixed_ok)
{
    CoulPlan p{0, 0};
    if (Z <= 0)
        return p;
    const int form = g_tuning.coulomb_form;
    if (cut) {
        p.form = 2;
        p.S = coulomb_splits(Z, coul_max);
    } else if (form == 2 && fixed_ok) {
        p.form = 3;
        p.S = coulomb_pair_supers(Z);
    } else if (form >= 1 && (int64_t)coulomb_pair_supers(Z) * Z <= coul_max) {
        p.form = 1;
        p.S = coulomb_pair_supers(Z);
    } else {
        p.S = coulomb_splits(Z, coul_max);
    }
    return p;
}

int64_t coulomb_partial_capacity(int64_t n)
{
    // the gather form's default splits (about 2^19 partials), and the
    // pairwise form's ceil(Z / 256) partials per proton for Z up to 0.4 n
    // (the largest proton fraction of the paper's runs)
    const int64_t zd = (int64_t)std::ceil(0.4 * (double)n);
    int64_t cap = 32 * n < 524288 ? 32 * n : 524288;
    const int64_t pair = (int64_t)coulomb_pair_supers(zd) * zd;
    cap = pair > cap ? pair : cap;
    return cap > n ? cap : n;
}

pasta_tuning g_tuning = {1, 0, 1, 0, 2.0, 1.0, 0, 0};  // coulomb_form 0: gather

void launch_forces_fused(int precision, const ForceBuf& fb, const CellBuf& cb, const Grid& g,
                         int64_t n, int64_t Z, const PairParams& pp, bool with_nuclear_terms,
                         bool with_coulomb, double* force, double* epot, const KickArgs& kick,
                         uint64_t* pair_counter, uint32_t* err, hipStream_t s, Timer* t,
                         int variant, const ListBuf* lb)
{
    const NucConsts k = make_nuc_consts(pp);
    const CoulConsts kc = make_coul_consts(pp);
    const bool cut = std::isfinite(pp.r_coul);
    const CoulPlan plan = (with_coulomb && Z > 0)
                              ? coulomb_plan(Z, fb.coul_max, cut, precision == PASTA_MIXED)
                              : CoulPlan{0, 0};
    // fixed-point form: no partials; the combine reads the accumulators
    const bool fixed = plan.form == 3;
    const CoulCut cc{fb.cut_pos, fb.cut_perm,
                     pair_counter ? reinterpret_cast<unsigned long long*>(pair_counter + 1)
                                  : nullptr};
    const int S = plan.S;
    const int per = S ? (int)((Z + S - 1) / S) : 0;
    const int coul_blocks = S ? (int)((Z + WG - 1) / WG) : 0;
    const int64_t coul_items = S == 0 ? 0 : (plan.form == 1 || fixed ? coulomb_pair_items(Z)
                                                                     : (int64_t)coul_blocks * S);
    NucArgs a{};
    a.start = cb.start;
    a.items = cb.items;
    a.perm = kick.slot_order ? nullptr : cb.perm;
    a.nc = g.nc;
    a.C = g.C;
    a.sub = g.sub;
    a.Z = (int)Z;
    a.pairs = reinterpret_cast<unsigned long long*>(pair_counter);
    a.err = err;
    a.fnuc = fb.fnuc;
    a.react = fb.react;
    a.react_stride = n;
    (void)with_nuclear_terms;  // the fused form always carries the nuclear terms
    const int item_max = (int)cb.item_max;
    const unsigned grid = (unsigned)(item_max + coul_items);
    const int mode = pair_counter ? MODE_COUNT : (epot ? MODE_ENERGY : MODE_FORCE);
    if (variant == 2 && !lb)
        variant = 1;
    // the half stencil needs three cells per side (its 14 cells distinct)
    if (variant == 4 && g.nc < 3)
        variant = 3;
    const ListArgs la = list_args(lb);
    timer_begin(t, KC_NUCLEAR, s);
    if (grid > 0) {
        auto go = [&](auto vtag, auto mtag) {
            constexpr int V = decltype(vtag)::value;
            constexpr int M = decltype(mtag)::value;
            auto launch = [&](auto ctag) {
                constexpr int CF = decltype(ctag)::value;
                if (precision == PASTA_FP64) {
                    if constexpr (CF != 3)  // the fixed-point form is mixed precision only
                        k_forces_fused<Fp64Policy, M, V, CF><<<grid, WG, 0, s>>>(
                            fb.stg64, a, cb.n_items, item_max, k, (int)Z, per, coul_blocks, kc,
                            fb.coul_part, la, cc);
                } else
                    k_forces_fused<MixedPolicy, M, V, CF><<<grid, WG, 0, s>>>(
                        fb.stgq, a, cb.n_items, item_max, k, (int)Z, per, coul_blocks, kc,
                        fb.coul_part, la, cc);
            };
            if (plan.form == 1)
                launch(std::integral_constant<int, 1>());
            else if (fixed)
                launch(std::integral_constant<int, 3>());
            else if (plan.form == 2)
                launch(std::integral_constant<int, 2>());
            else
                launch(std::integral_constant<int, 0>());
        };
        with_mode(mode, [&](auto mt) {
            switch (variant) {
            case 0: go(std::integral_constant<int, 0>(), mt); break;
            case 2: go(std::integral_constant<int, 2>(), mt); break;
            case 3: go(std::integral_constant<int, 3>(), mt); break;
            case 4: go(std::integral_constant<int, 4>(), mt); break;
            case 5: go(std::integral_constant<int, 5>(), mt); break;
            case 6: go(std::integral_constant<int, 6>(), mt); break;
            default: go(std::integral_constant<int, 1>(), mt); break;
            }
        });
    }
    timer_end(t, KC_NUCLEAR, s);
    timer_begin(t, KC_COMBINE, s);
    {
        // protons (COMB_LANES lanes each) then neutrons (one lane each); with
        // the fixed-point form every slot takes one lane (no partials)
        const int64_t Zc = fixed ? 0 : Z;
        const int zb = (int)combine_proton_blocks(Zc);
        const unsigned cgrid = (unsigned)(zb + (n - Zc + WG - 1) / WG);
        const NextDrift nd = kick.next ? *kick.next : NextDrift{};
        auto comb = [&](auto* part) {
            k_combine<<<cgrid, WG, 0, s>>>(fb.fnuc, part, fixed ? 0 : S, (int)Zc, zb,
                                           kick.slot_order ? nullptr : cb.perm, n, force, epot,
                                           kick.vel, kick.hdtm, kick.mass, kick.ke_part, fb.n_ke,
                                           err, nd, kick.next ? 1 : 0,
                                           variant == 4 || fixed ? fb.react : nullptr,
                                           variant == 4 ? n : Z);
        };
        if (precision == PASTA_FP64)
            comb(static_cast<const double4*>(fb.coul_part));
        else
            comb(static_cast<const float4*>(fb.coul_part));
    }
    timer_end(t, KC_COMBINE, s);
}

size_t forcebuf_carve(Carver& cv, ForceBuf* out, int64_t n, int64_t item_max, int precision)
{
    ForceBuf fb;
    fb.stg64 = precision == PASTA_FP64 ? cv.take<double4>(n) : nullptr;
    fb.stgq = precision == PASTA_MIXED ? cv.take<Q4>(n) : nullptr;
    fb.coul_max = coulomb_partial_capacity(n);
    if (precision == PASTA_FP64)
        fb.coul_part = cv.take<double4>(fb.coul_max);
    else
        fb.coul_part = cv.take<float4>(fb.coul_max);

    // per-block kinetic energies: one per nuclear item (unfused kick) or per
    // combine block (at most n * COMB_LANES / WG + 2)
    const int64_t comb_blocks = (n * COMB_LANES + WG - 1) / WG + 2;
    fb.ke_part = cv.take<double>(item_max > comb_blocks ? item_max : comb_blocks);
    fb.n_ke = cv.take<int32_t>(1);
    fb.fnuc = cv.take<double4>(n);
    fb.react = cv.take<unsigned long long>(4 * (size_t)n);
    fb.pairs = cv.take<uint64_t>(2);
    if (out)
        *out = fb;
    return cv.size();
}

int launch_coulomb(int precision, const ForceBuf& fb, int64_t Z, const PairParams& pp,
                   bool energy, hipStream_t s, Timer* t, uint64_t* count)
{
    if (Z <= 0)
        return 0;
    const bool cut = std::isfinite(pp.r_coul);
    const CoulPlan plan = coulomb_plan(Z, fb.coul_max, cut);
    const int S = plan.S;
    const int per = (int)((Z + S - 1) / S);
    const CoulCut cc{fb.cut_pos, fb.cut_perm,
                     count ? reinterpret_cast<unsigned long long*>(count) : nullptr};
    const CoulConsts k = make_coul_consts(pp);
    void* co = fb.coul_part;
    timer_begin(t, KC_COULOMB, s);
    if (plan.form == 1) {
        const unsigned g1 = (unsigned)coulomb_pair_items(Z);
        if (precision == PASTA_FP64) {
            if (energy)
                k_coulomb_pair<Fp64Policy, true><<<g1, WG, 0, s>>>(fb.stg64, (int)Z, k, co);
            else
                k_coulomb_pair<Fp64Policy, false><<<g1, WG, 0, s>>>(fb.stg64, (int)Z, k, co);
        } else {
            if (energy)
                k_coulomb_pair<MixedPolicy, true><<<g1, WG, 0, s>>>(fb.stgq, (int)Z, k, co);
            else
                k_coulomb_pair<MixedPolicy, false><<<g1, WG, 0, s>>>(fb.stgq, (int)Z, k, co);
        }
        timer_end(t, KC_COULOMB, s);
        return S;
    }
    dim3 grid((unsigned)((Z + WG - 1) / WG), (unsigned)S);
    auto go = [&](auto etag, auto ctag) {
        constexpr bool E = decltype(etag)::value, C = decltype(ctag)::value;
        if (precision == PASTA_FP64)
            k_coulomb<Fp64Policy, E, C><<<grid, WG, 0, s>>>(fb.stg64, (int)Z, per, k, co, cc);
        else
            k_coulomb<MixedPolicy, E, C><<<grid, WG, 0, s>>>(fb.stgq, (int)Z, per, k, co, cc);
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    if (energy)
        cut ? go(T_(), T_()) : go(T_(), F_());
    else
        cut ? go(F_(), T_()) : go(F_(), F_());
    timer_end(t, KC_COULOMB, s);
    return S;
}

void launch_nuclear(int precision, const ForceBuf& fb, const CellBuf& cb, const Grid& g,
                    int64_t n, int64_t Z, const PairParams& pp, bool with_nuclear_terms,
                    int coul_S, double* force, double* epot, const KickArgs& kick,
                    uint64_t* pair_counter, uint32_t* err, hipStream_t s, Timer* t,
                    int variant, const ListBuf* lb)
{
    (void)n;
    const NucConsts k = make_nuc_consts(pp);
    NucArgs a{};
    a.start = cb.start;
    a.items = cb.items;
    a.perm = kick.slot_order ? nullptr : cb.perm;
    a.nc = g.nc;
    a.C = g.C;
    a.sub = g.sub;
    a.Z = (int)Z;
    a.coul_part = fb.coul_part;
    a.S = coul_S;
    a.force = force;
    a.epot = epot;
    a.vel = kick.vel;
    a.hdtm = kick.hdtm;
    a.mass = kick.mass;
    a.ke_part = kick.ke_part;
    a.pairs = reinterpret_cast<unsigned long long*>(pair_counter);
    a.err = err;
    a.fnuc = nullptr;
    const unsigned grid = (unsigned)cb.item_max;
    const int mode = pair_counter ? MODE_COUNT : (epot ? MODE_ENERGY : MODE_FORCE);
    timer_begin(t, KC_NUCLEAR, s);
    if (variant == 2 && lb && with_nuclear_terms) {
        const ListArgs la = list_args(lb);
        with_mode(mode, [&](auto mt) {
            constexpr int M = decltype(mt)::value;
            if (precision == PASTA_FP64)
                k_nuclear_list<Fp64Policy, M><<<grid, WG, 0, s>>>(fb.stg64, a, cb.n_items, k, la);
            else
                k_nuclear_list<MixedPolicy, M><<<grid, WG, 0, s>>>(fb.stgq, a, cb.n_items, k, la);
        });
    } else if (precision == PASTA_FP64) {
        nuclear_dispatch<Fp64Policy>(fb.stg64, a, cb.n_items, k, with_nuclear_terms, mode,
                                     variant, grid, s);
    } else {
        nuclear_dispatch<MixedPolicy>(fb.stgq, a, cb.n_items, k, with_nuclear_terms, mode,
                                      variant, grid, s);
    }
    timer_end(t, KC_NUCLEAR, s);
}

}  // namespace pasta
