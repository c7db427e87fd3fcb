// Internal declarations shared by the libpasta translation units: device
// helpers, the launch-parameter structs of every kernel, and the host-side
// error and workspace utilities.  Nothing here is part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/pasta.h"

namespace pasta {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);
#define PASTA_HIP(call)                                                              \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::pasta::fail(PASTA_EHIP, "%s failed: %s (%s:%d)", #call,         \
                                 hipGetErrorString(e_), __FILE__, __LINE__);         \
    } while (0)
#define PASTA_TRY(expr)             \
    do {                            \
        int rc_ = (expr);           \
        if (rc_ != PASTA_OK)        \
            return rc_;             \
    } while (0)

// Device error word bits.
enum : uint32_t {
    ERR_NONFINITE_FORCE = 1u << 0,
    ERR_NONFINITE_POS = 1u << 1,
    ERR_WRAP = 1u << 2,       // a particle crossed more than one box length
    ERR_UF_LIMIT = 1u << 3,   // union-find retry bound reached
    ERR_NONFINITE_VEL = 1u << 4,
    ERR_RANGE = 1u << 5,      // an input position outside [0, L)
    ERR_SPECIES = 1u << 6,    // an input species other than 0 or 1
};
std::string describe_device_error(uint32_t bits);

// ------------------------------------------------------------- workspace
// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.  Every block is 256-byte aligned.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += sizeof(T) * (count ? count : 1);
        return p;
    }
    size_t size() const { return (off + 255) & ~size_t(255); }
};

// ------------------------------------------------------------- cell grid
// ncell = the largest integer with L/ncell >= r_cut (at least 1).
inline int cell_dims(double L, double r_cut)
{
    int nc = (int)std::floor(L / r_cut);
    while (nc > 1 && L / (double)nc < r_cut)
        nc--;
    return nc < 1 ? 1 : nc;
}

// sub = bins per cell and species: 1, or 8 (the cell's octants, so that a
// run of consecutive slots inside a cell is spatially compact).  Bin of a
// particle = (proton ? 0 : C*sub) + cell*sub + octant rank; a cell's protons are
// the bins [cell*sub, cell*sub + sub), its neutrons the same range + C*sub.
struct Grid {
    int nc;        // cells per side
    int C;         // nc^3
    int sub;       // bins per cell and species (1 or 8)
    double inv_w;  // nc / L  (cell coordinate = floor(x * inv_w))
    double L;
    __host__ __device__ int64_t nbins() const { return 2 * (int64_t)C * sub; }
};
inline Grid make_grid(double L, double r_cut, int sub = 1)
{
    Grid g;
    g.nc = cell_dims(L, r_cut);
    g.C = g.nc * g.nc * g.nc;
    g.sub = sub;
    g.inv_w = (double)g.nc / L;
    g.L = L;
    return g;
}

// Sparse states: the force paths' grids have at most k cells per side, k
// the largest with k^3 * CELL_MIN_OCC <= n, so that a cell holds about
// CELL_MIN_OCC particles or more (a full 32-target work item).  Larger cells
// keep the 27-cell stencil complete (their side only grows past r_cut);
// they trade the per-item overhead of near-empty cells against more
// candidates screened per target.  Dense states (the paper's 0.08 fm^-3:
// about 150 per cell) never reach the cap.
constexpr int64_t CELL_MIN_OCC = 32;
__host__ __device__ inline int cap_cells(int nc, int64_t n)
{
    int k = 1;
    while ((int64_t)(k + 1) * (k + 1) * (k + 1) * CELL_MIN_OCC <= n)
        ++k;
    return nc < k ? nc : k;
}
inline Grid make_force_grid(double L, double r_cut, int64_t n, int sub)
{
    Grid g = make_grid(L, r_cut, sub);
    g.nc = cap_cells(g.nc, n);
    g.C = g.nc * g.nc * g.nc;
    g.inv_w = (double)g.nc / L;
    return g;
}

// Neighbour-cell offsets along one axis without duplicates: {-1,0,1} when
// there are at least 3 cells per side, {0,1} for 2, {0} for 1.
__host__ __device__ inline int axis_lo(int nc) { return nc >= 3 ? -1 : 0; }
__host__ __device__ inline int axis_hi(int nc) { return nc >= 2 ? 1 : 0; }

__device__ inline int cell_coord(double x, double inv_w, int nc)
{
    int k = (int)(x * inv_w);
    k = k > nc - 1 ? nc - 1 : k;
    return k < 0 ? 0 : k;
}

// Bin of a particle (see Grid).  The octant bit along an axis is whether
// the fractional cell coordinate a = x * inv_w is at least 1/2; floor(2a)
// is exact in binary, so the cell is floor(2a) / 2 and agrees with
// cell_coord.
__device__ inline int particle_bin(double x, double y, double z, bool proton, double inv_w,
                                   int nc, int C, int sub)
{
    const double a[3] = {x * inv_w, y * inv_w, z * inv_w};
    int k[3], o = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int h = (int)(2.0 * a[d]);
        int c = h >> 1;
        h &= 1;
        if (c > nc - 1) {
            c = nc - 1;
            h = 1;
        }
        if (c < 0) {
            c = 0;
            h = 0;
        }
        k[d] = c;
        o |= h << d;
    }
    const int cell = (k[2] * nc + k[1]) * nc + k[0];
    // octants in reflected-Gray-code order (o = x | y << 1 | z << 2 at rank
    // r = o ^ (o >> 1) ^ (o >> 2)): consecutive octants share a face, so a
    // run of consecutive slots spanning two or three octants stays within a
    // 2 x 1 x 1 or 2 x 2 x 1 block of them
    const int r = o ^ (o >> 1) ^ (o >> 2);
    return (proton ? 0 : C * sub) + cell * sub + (sub == 8 ? r : 0);
}

// One particle's share of a step's first part (Sec. II.A, Eq. 3): the half
// kick v += (dt/2M) F, the drift x += dt v, the optional affine scaling by
// L_new / L_old and the wrap into [0, L_new).  x and v are updated in place;
// returns ERR_* bits.  Every kernel that drifts uses this one function, so
// the arithmetic is the same code wherever the drift runs.
struct DriftStep {
    double hdtm, dt;
    double L_new, ratio;
    int scale_positions;
};
__device__ inline uint32_t drift_update(double (&x)[3], double (&v)[3], const double (&f)[3],
                                        const DriftStep& c)
{
    uint32_t bad = 0;
    const double L = c.L_new;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double vd = v[d] + c.hdtm * f[d];
        double xd = x[d] + c.dt * vd;
        if (c.scale_positions)
            xd *= c.ratio;
        if (xd < 0.0)
            xd += L;
        if (xd >= L)
            xd -= L;
        if (!(xd >= 0.0 && xd < L)) {
            bad |= isfinite(xd) ? ERR_WRAP : ERR_NONFINITE_POS;
            xd = isfinite(xd) ? xd - L * floor(xd / L) : 0.0;
            if (!(xd >= 0.0 && xd < L))
                xd = 0.0;
        }
        if (!isfinite(vd))
            bad |= ERR_NONFINITE_VEL;
        v[d] = vd;
        x[d] = xd;
    }
    return bad;
}

// Wave-aggregated atomic add of 1 per lane on counters[bin]: the lanes of a
// wavefront that share a bin are grouped (ballots only), then every group's
// leader lane adds its group size in one vector atomic instruction, so the
// wave makes a single round trip to memory however many bins it touches.
// Returns the counter value seen by this lane's share (old value + rank
// among the wave's lanes with the same bin, in lane order).  Must be called
// by every active lane of the wave (the loop below is wave-uniform).
__device__ inline int wave_aggregated_add(int32_t* counters, int bin)
{
    unsigned long long todo = __ballot(1);
    const int lane = __lane_id();
    int leader = lane, rank = 0, size = 0;
    while (todo) {
        const int l = __ffsll((unsigned long long)todo) - 1;
        const int b = __shfl(bin, l);
        const unsigned long long mask = __ballot(bin == b) & todo;
        if (bin == b) {
            leader = l;
            rank = __popcll(mask & ((1ull << lane) - 1ull));
            size = __popcll(mask);
        }
        todo &= ~mask;
    }
    int base = 0;
    if (lane == leader)
        base = atomicAdd(&counters[bin], size);
    return __shfl(base, leader) + rank;
}

// Exclusive prefix of one int64 per thread over the workgroup: a shuffle
// scan inside each wavefront, the wavefront totals scanned by the first
// wavefront through LDS (three barriers).  lds needs 64 entries.  Returns
// the prefix; *total gets the workgroup sum.
__device__ inline int64_t block_exclusive_scan(int64_t x, int64_t* lds, int64_t* total)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    int64_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(inc, off, 64);
        if (lane >= off)
            inc += y;
    }
    if (lane == 63)
        lds[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        int64_t t = lane < nw ? lds[lane] : 0;
        int64_t ti = t;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t y = __shfl_up(ti, off, 64);
            if (lane >= off)
                ti += y;
        }
        if (lane < nw)
            lds[lane] = ti - t;  // exclusive prefix of the wave totals
        if (lane == nw - 1)
            lds[63] = ti;
    }
    __syncthreads();
    const int64_t pre = lds[wave] + inc - x;
    *total = lds[63];
    __syncthreads();
    return pre;
}

// ------------------------------------------------------ staging formats
// FP64 staging: x, y, z in fm, w unused.
// MIXED staging: x, y, z as 32-bit fixed point (x/L * 2^32), w = species.
struct alignas(16) Q4 {
    uint32_t x, y, z, w;
};

// ------------------------------------------------- kernel classes (timing)
enum KernelClass : int {
    KC_DRIFT = 0,
    KC_SCAN = 1,
    KC_SCATTER = 2,
    KC_RANK = 3,
    KC_COULOMB = 4,
    KC_NUCLEAR = 5,
    KC_THERMO = 6,
    KC_COMBINE = 7,
    KC_LIST = 8,
};

// Launch timing hook: when non-null, brackets a launch with HIP events.
struct Timer;
void timer_begin(Timer* t, int kc, hipStream_t s);
void timer_end(Timer* t, int kc, hipStream_t s);

// -------------------------------------------------------- neighbour lists
// Device control block of the neighbour lists of one system.  The drift
// kernel's last workgroup decides, once per step, whether this step
// rebuilds (rebuild), and the gated build kernels read that word.
struct ListCtl {
    double L_build;                  // box side at the last build
    unsigned long long pool_used;    // pool rows taken by the last build
    unsigned long long n_builds;     // builds so far
    unsigned long long n_overflow;   // builds that ran out of list memory
    uint32_t maxd2[2];               // FP32 bits of max |u|^2, by step parity
    uint32_t done;                   // drift workgroups finished this step
    int32_t rebuild;                 // 1: this step rebuilds cells + lists
    int32_t overflow;                // 1: the last build ran out of memory
    int32_t nc, C;                   // cell grid of the last build
    uint32_t max_rows;               // largest item row count of the last build
    double max_disp;                 // max |u| seen at the last decision (fm)
};
struct ListBuf {
    ListCtl* ctl;
    double* xb;        // [3n] positions at the last build, sorted-slot order
    int2* hdr;         // [item_max]
    int32_t* cnt;      // [item_max * 256]
    int32_t* pool;     // [pool_rows * 256]
    int64_t pool_rows;
    double skin;       // delta_r (fm)
};
constexpr size_t LIST_ROW_BYTES = 256 * sizeof(int32_t);  // one pool row (a workgroup's entries)
int64_t list_pool_rows(int64_t n, double L_min, double r_list, int64_t item_max, double scale);
size_t listbuf_carve(Carver& cv, ListBuf* out, int64_t n, int64_t item_max, int64_t pool_rows);

// -------------------------------------------------------- cell-list build
struct CellBuf {
    int32_t* key;     // [n] bin of each particle (indexed like the build's positions)
    int32_t* count;   // [2 C_max sub] per-bin counts (zero between builds)
    int32_t* fill;    // [2 C_max sub] per-bin scatter cursors (zero between builds)
    int32_t* start;   // [2 C_max sub + 1]
    int32_t* tmp;     // [n] unsorted slots: particle index
    int32_t* src;     // [n] unsorted slots: source index (state moves)
    int32_t* perm;    // [n] slot -> source index (the particle index unless the
                      //     build moves a state kept in sorted order)
    int32_t* items;   // [2 * item_max] nuclear work items (cell, chunk)
    int32_t* n_items; // [1]
    int64_t item_max;
};
// C_max: the largest cell count; sub: bins per cell and species.
size_t cellbuf_carve(Carver& cv, CellBuf* out, int64_t n, int C_max, int chunk, int sub = 1);
void cellbuf_zero(const CellBuf& cb, int C_max, hipStream_t s, int sub = 1);
// Zero nwords 32-bit words at p with a fill kernel (no memset node, so the
// call may sit in a captured stream).
void launch_zero_words(void* p, int64_t nwords, hipStream_t s);

// Bins + counts from positions (caller order); the drift kernel does the
// same inside the integrator.
// gate (optional, device): when non-null the kernels of the build return at
// once unless *gate is non-zero (the neighbour-list rebuild decision).
void launch_bin_count(const double* pos, const uint8_t* species, int64_t n, const Grid& g,
                      const CellBuf& cb, uint32_t* err, hipStream_t s, Timer* t,
                      const int32_t* gate = nullptr);
// Exclusive scan of the 2C counts into start[]; zeroes count and fill; when
// chunk > 0, also writes the nuclear work list.
void launch_scan(const CellBuf& cb, const Grid& g, int chunk, hipStream_t s, Timer* t,
                 const int32_t* gate = nullptr);
// Particle state carried into sorted order by the rank kernel (all or
// nothing): destination slot d receives the position, velocity, species and
// particle index of source index perm[d].  Sources are indexed like the pos
// and species arrays of the build; id_src gives their particle indices (null:
// the source index is the particle index).  The sorted order is (bin,
// particle index) either way.
struct StateMove {
    const double* vel_src;  // [n][3]
    const int32_t* id_src;  // [n] or null
    double* pos_dst;        // [n][3]
    double* vel_dst;        // [n][3]
    int32_t* id_dst;        // [n]
    uint8_t* sp_dst;        // [n]
};
// Stable scatter: slot order = (bin, particle index); the source index is
// the position in pos/species.  Writes perm (slot -> source index) and, when
// given, the sorted staging coordinates, the build positions xb and the
// moved state.  prev_order: visit particles in the order of the previous
// build (cb.perm must hold it).
void launch_scatter_rank(const double* pos, const uint8_t* species, int64_t n, const Grid& g,
                         const CellBuf& cb, double4* stg64, Q4* stgq, hipStream_t s, Timer* t,
                         bool prev_order = false, const int32_t* gate = nullptr,
                         double* xb = nullptr, const StateMove* mv = nullptr);
// Gated copy of a moved state back into the primary arrays (list form: a
// rebuild moves the state to the spare arrays, this brings it back).
void launch_state_copy(const StateMove& from_spare, double* pos, double* vel, int32_t* id,
                       uint8_t* sp, int64_t n, const int32_t* gate, hipStream_t s);
// Caller-order copies of sorted-slot arrays: dst3[id[k]] = src3[k] (3
// doubles) and dst1[id[k]] = src1[k]; any pair may be null.
void launch_export(const int32_t* id, int64_t n, const double* src3a, double* dst3a,
                   const double* src3b, double* dst3b, const double* src1, double* dst1,
                   hipStream_t s);

// ----------------------------------------------------------------- forces
struct PairParams {
    // nuclear (Eq. 1a,b)
    double a, b_like, b_unlike, Lambda, r_nuc;
    // Coulomb (Eq. 1c); r_coul = +inf: uncut
    double alpha_hbarc, lambda_s, r_coul;
    double L;
};
// A finite Coulomb cutoff is decided on the FP64 r^2 of the positions the
// staging was built from: pos [n][3], row perm[slot] (perm null: row slot).
struct CoulCut {
    const double* pos;
    const int32_t* perm;
    unsigned long long* count;  // ordered pairs kept (counting calls), or null
};
struct KickArgs {
    double* vel;       // [n][3] or nullptr (no kick)
    double hdtm;       // dt / (2 M)
    double mass;
    double* ke_part;   // [item_max] per-work-item kinetic energy, or nullptr
    // Where F, E and the kicked velocity of sorted slot k live: index k
    // (true: the arrays are in sorted order) or perm[k] (false: caller order).
    bool slot_order;
    // Optional (fused form, sorted order, no kinetic energy): after the
    // second half kick of this step, the first part of the next step (half
    // kick, drift, wrap) and its cell binning, as the drift kernel does it.
    const struct NextDrift* next = nullptr;
};
struct NextDrift {
    double* pos;             // [n][3] sorted order
    const uint8_t* species;  // [n] sorted order
    int32_t* key;            // [n] bin of each slot
    int32_t* count;          // [2 C sub] bin counters (zero on entry)
    DriftStep step;          // hdtm, dt, L_{n+2}, L_{n+2} / L_{n+1}
    int nc, C, sub;          // the cell grid at L_{n+2}
    double inv_w;
};
struct ForceBuf {
    double4* stg64;     // [n] FP64 staging (sorted)
    Q4* stgq;           // [n] fixed-point staging (sorted)
    void* coul_part;    // [coul_max] partial Coulomb sums (fx, fy, fz, V): double4
                        // (FP64) or float4 (mixed)
    int64_t coul_max;   // capacity in partials
    double* ke_part;    // [item_max] kinetic-energy partials of the last kick
    int32_t* n_ke;      // [1] number of valid ke_part entries (fused form)
    double4* fnuc;      // [n] nuclear (F, V) per sorted slot (fused form)
    unsigned long long* react;  // [4][n] fixed point: Newton-3 reactions, Coulomb sums
                                // (zero between launches)
    uint64_t* pairs;    // [2] diagnostic pair counters (nuclear, Coulomb; ordered)
    // FP64 positions the staging was built from, for a finite Coulomb
    // cutoff (set per evaluation; see CoulCut)
    const double* cut_pos = nullptr;
    const int32_t* cut_perm = nullptr;
};
// Automatic source splits of the gather form (about 2^19 / Z, at most 32,
// at most cap / Z); the tuning's coulomb_splits overrides.
int coulomb_splits(int64_t Z, int64_t cap = 524288);
// How the Coulomb sums of Z protons are produced: form 0 = gather tiles
// with S source splits, 1 = pairwise super-block items (S = super-blocks of
// 256 protons; used when S Z partials fit coul_max); every proton then gets
// S partials.  Form 3 (only where fixed_ok: the fused launch in mixed
// precision) = pairwise items that add into per-proton fixed-point
// accumulators, no partials (S = super-blocks).
struct CoulPlan {
    int form;  // 0 gather, 1 pairwise, 2 gather with a finite cutoff, 3 pairwise fixed point
    int S;
};
CoulPlan coulomb_plan(int64_t Z, int64_t coul_max, bool cut = false, bool fixed_ok = false);
// Partials a force workspace holds for n particles: enough for the gather
// form's default splits and for the pairwise form up to Z = 0.4 n.
int64_t coulomb_partial_capacity(int64_t n);
// Super-blocks (partials per proton) of the pairwise form for Z protons.
int coulomb_pair_plan_supers(int64_t Z);
// Process-wide kernel choices (set through pasta_set_tuning).
extern pasta_tuning g_tuning;
// Source-tile lengths of the compacting nuclear items besides the default
// 512 (pasta_tuning.nuclear_tile; variant 3, fused form).
constexpr int NUC_TILE_SHORT = 256;
constexpr int NUC_TILE_LONG = 1024;
// The kernel variant a tuning runs: the public variant, except variant 3
// with a non-default tile length, which runs as 5 (256 sources) or 6
// (1024 sources).
inline int internal_variant(const pasta_tuning& t)
{
    if (t.nuclear_variant == 3 && t.nuclear_tile == NUC_TILE_SHORT)
        return 5;
    if (t.nuclear_variant == 3 && t.nuclear_tile == NUC_TILE_LONG)
        return 6;
    return t.nuclear_variant;
}
size_t forcebuf_carve(Carver& cv, ForceBuf* out, int64_t n, int64_t item_max, int precision);

// Coulomb all-pairs over protons (sorted slots [0, Z)).
// energy: also accumulate the energy shares (else the partials' w is 0).
// Returns the number of partials per proton written (the S to add).
// count (optional): ordered Coulomb pairs kept by a finite cutoff.
int launch_coulomb(int precision, const ForceBuf& fb, int64_t Z, const PairParams& pp,
                   bool energy, hipStream_t s, Timer* t, uint64_t* count = nullptr);
// Nuclear cell-tile kernel; adds the coul_S Coulomb partials of proton
// targets (coul_S = 0: none),
// writes F and E at the caller index (perm[slot]) or at the sorted slot
// (kick.slot_order), optionally applies the second half kick.
void launch_nuclear(int precision, const ForceBuf& fb, const CellBuf& cb, const Grid& g,
                    int64_t n, int64_t Z, const PairParams& pp, bool with_nuclear_terms,
                    int coul_S, double* force, double* epot, const KickArgs& kick,
                    uint64_t* pair_counter, uint32_t* err, hipStream_t s, Timer* t,
                    int variant, const ListBuf* lb = nullptr);
// Targets per nuclear work item (the scan's chunk) for a kernel variant:
// 64 for variants 0 and 1 (4 lanes per target), 32 for 2 to 6 (8 lanes).
int nuclear_chunk_for(int variant);
// Neighbour-list build (gated on lb.ctl->rebuild) for the cells of grid g.
void launch_list_build(int precision, const ForceBuf& fb, const CellBuf& cb, const Grid& g,
                       const ListBuf& lb, const PairParams& pp, hipStream_t s, Timer* t);

// ------------------------------------------------------------- integrate
struct DriftArgs {
    double* pos;
    double* vel;
    const double* force;
    const uint8_t* species;
    int64_t n;
    double hdtm, dt;
    double L_new, ratio;  // ratio = L_new / L_old (affine variant only)
    int scale_positions;
};
// The state arrays of DriftArgs are in the sorted order of the last build:
// thread k updates slot k and bins it (key[k]), so the lanes of a wave
// mostly fall in one bin and the count atomics aggregate.
void launch_drift(const DriftArgs& a, const Grid& g, const CellBuf& cb, uint32_t* err,
                  hipStream_t s, Timer* t);
// Neighbour-list form of the drift: the same update of the sorted slots of
// the last build; writes the slot's staging coordinates for the new
// box, reduces max |u|^2 (nearest-image displacement since the build) and,
// in its last workgroup, decides whether this step rebuilds (ListCtl).
// g is the cell grid a rebuild at this step would use.
void launch_drift_list(const DriftArgs& a, const Grid& g, const CellBuf& cb, const ListBuf& lb,
                       double4* stg64, Q4* stgq, int64_t step, uint32_t* err, hipStream_t s,
                       Timer* t);
// Marks the next build as due (initial state, set_state) for grid g.
void launch_list_force_rebuild(const ListBuf& lb, const Grid& g, hipStream_t s);
// Fused form: one launch with every Coulomb tile and nuclear cell tile (the
// nuclear items write fb.fnuc), then the combine kernel: F = nuclear +
// Coulomb partials, E, the optional half kick and kinetic-energy partials
// (count in *fb.n_ke).
void launch_forces_fused(int precision, const ForceBuf& fb, const CellBuf& cb, const Grid& g,
                         int64_t n, int64_t Z, const PairParams& pp, bool with_nuclear_terms,
                         bool with_coulomb, double* force, double* epot, const KickArgs& kick,
                         uint64_t* pair_counter, uint32_t* err, hipStream_t s, Timer* t,
                         int variant, const ListBuf* lb = nullptr);
// Thermostat: reduce ke_part[0 .. *n_items) and scale velocities to
// KE = 1.5 N T.  scale_out receives the factor.
void launch_thermostat(double* vel, int64_t n, const double* ke_part, const int32_t* n_items,
                       double target_ke, double* scale_out, hipStream_t s, Timer* t);
// Deterministic partial sums: out[b] for b < nblk over x[i] (kind 0) or over
// (1/2) M |v_i|^2 (kind 1).
void launch_partial_sums(const double* x, int64_t n, int kind, double mass, double* out,
                         int nblk, hipStream_t s);

}  // namespace pasta
