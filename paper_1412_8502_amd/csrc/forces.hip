// Pair-force kernels (a2 nuclear, a3 Coulomb) for one system.  The work
// items themselves live in pair_items.hpp, shared with the batched
// persistent kernel.
//
// Coulomb: all proton pairs.  Protons occupy sorted slots [0, Z).  A
// workgroup owns 256 targets (one per thread) and one of S source ranges;
// sources stream through an LDS tile and are read as wave-wide broadcasts.
// The S partial sums per target are added in fixed order by the nuclear
// kernel's epilogue.
//
// Nuclear: cell tiles.  A workgroup owns a chunk of the targets of one cell;
// the neighbour cells' particles (protons first, then neutrons) are staged
// into an LDS tile; NUC_TPT adjacent lanes share one target and split its
// sources, then combine by wavefront shuffles.  The epilogue adds the Coulomb
// partials, writes F and E in the caller's particle order and can apply the
// velocity-Verlet second half kick (fused integrate).
#include "pair_items.hpp"

namespace pasta {

namespace {

template <class P>
__global__ __launch_bounds__(WG) void k_coulomb(const typename P::Src* __restrict__ stg, int Z,
                                                int per_split, CoulConsts k,
                                                double4* __restrict__ part)
{
    __shared__ __align__(16) char lds[coulomb_lds_bytes<P>()];
    coulomb_item<P>(stg, Z, per_split, k, part, blockIdx.x, blockIdx.y, lds);
}

template <class P, bool NUC, bool COUNT>
__global__ __launch_bounds__(WG) void k_nuclear(const typename P::Src* __restrict__ stg,
                                                NucArgs A, const int32_t* __restrict__ n_items,
                                                NucConsts k)
{
    __shared__ __align__(16) char lds[nuclear_lds_bytes<P>()];
    if ((int)blockIdx.x >= *n_items)
        return;
    nuclear_item<P, NUC, COUNT>(stg, A, k, blockIdx.x, lds);
}

template <class P, bool NUC, bool COUNT>
__global__ __launch_bounds__(WG) void k_nuclear_compact(const typename P::Src* __restrict__ stg,
                                                        NucArgs A,
                                                        const int32_t* __restrict__ n_items,
                                                        NucConsts k)
{
    __shared__ __align__(16) char lds[nuclear_compact_lds_bytes<P>()];
    if ((int)blockIdx.x >= *n_items)
        return;
    nuclear_item_compact<P, NUC, COUNT>(stg, A, k, blockIdx.x, lds);
}

template <class P>
void nuclear_dispatch(const typename P::Src* stg, const NucArgs& a, const int32_t* n_items,
                      const NucConsts& k, bool nuc, bool count, int variant, unsigned grid,
                      hipStream_t s)
{
    if (!nuc)
        k_nuclear<P, false, false><<<grid, WG, 0, s>>>(stg, a, n_items, k);
    else if (variant == 1 && count)
        k_nuclear_compact<P, true, true><<<grid, WG, 0, s>>>(stg, a, n_items, k);
    else if (variant == 1)
        k_nuclear_compact<P, true, false><<<grid, WG, 0, s>>>(stg, a, n_items, k);
    else if (count)
        k_nuclear<P, true, true><<<grid, WG, 0, s>>>(stg, a, n_items, k);
    else
        k_nuclear<P, true, false><<<grid, WG, 0, s>>>(stg, a, n_items, k);
}

}  // namespace

int nuclear_chunk(int /*precision*/) { return NUC_CHUNK; }

int coulomb_splits(int64_t Z)
{
    if (Z <= 0)
        return 0;
    const int req = g_tuning.coulomb_splits;
    int64_t s = req > 0 ? req : 524288 / Z;
    s = s < 1 ? 1 : (s > 32 ? 32 : s);
    // the partial-sum buffer holds max(min(32 n, 2^19), n) entries, n >= Z
    while (s > 1 && s * Z > 524288)
        --s;
    return (int)s;
}

pasta_tuning g_tuning = {1, 0};

size_t forcebuf_carve(Carver& cv, ForceBuf* out, int64_t n, int64_t item_max, int precision)
{
    ForceBuf fb;
    fb.stg64 = precision == PASTA_FP64 ? cv.take<double4>(n) : nullptr;
    fb.stgq = precision == PASTA_MIXED ? cv.take<Q4>(n) : nullptr;
    int64_t cm = 32 * n < 524288 ? 32 * n : 524288;
    fb.coul_max = cm > n ? cm : n;
    fb.coul_part = cv.take<double4>(fb.coul_max);
    fb.ke_part = cv.take<double>(item_max);
    fb.pairs = cv.take<uint64_t>(2);
    if (out)
        *out = fb;
    return cv.size();
}

void launch_coulomb(int precision, const ForceBuf& fb, int64_t Z, const PairParams& pp,
                    uint64_t* /*pair_counter*/, hipStream_t s, Timer* t)
{
    if (Z <= 0)
        return;
    const int S = coulomb_splits(Z);
    const int per = (int)((Z + S - 1) / S);
    const CoulConsts k = make_coul_consts(pp);
    dim3 grid((unsigned)((Z + WG - 1) / WG), (unsigned)S);
    timer_begin(t, KC_COULOMB, s);
    if (precision == PASTA_FP64)
        k_coulomb<Fp64Policy><<<grid, WG, 0, s>>>(fb.stg64, (int)Z, per, k, fb.coul_part);
    else
        k_coulomb<MixedPolicy><<<grid, WG, 0, s>>>(fb.stgq, (int)Z, per, k, fb.coul_part);
    timer_end(t, KC_COULOMB, s);
}

void launch_nuclear(int precision, const ForceBuf& fb, const CellBuf& cb, const Grid& g,
                    int64_t n, int64_t Z, const PairParams& pp, bool with_nuclear_terms,
                    int coul_S, double* force, double* epot, const KickArgs& kick,
                    uint64_t* pair_counter, uint32_t* err, hipStream_t s, Timer* t)
{
    (void)n;
    const NucConsts k = make_nuc_consts(pp);
    NucArgs a{};
    a.start = cb.start;
    a.items = cb.items;
    a.perm = cb.perm;
    a.nc = g.nc;
    a.C = g.C;
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
    const bool count = pair_counter != nullptr;
    const int variant = g_tuning.nuclear_variant;
    timer_begin(t, KC_NUCLEAR, s);
    if (precision == PASTA_FP64)
        nuclear_dispatch<Fp64Policy>(fb.stg64, a, cb.n_items, k, with_nuclear_terms, count,
                                     variant, grid, s);
    else
        nuclear_dispatch<MixedPolicy>(fb.stgq, a, cb.n_items, k, with_nuclear_terms, count,
                                      variant, grid, s);
    timer_end(t, KC_NUCLEAR, s);
}

}  // namespace pasta
