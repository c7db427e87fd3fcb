// Batched systems: several independent boxes (the paper's grid of runs over
// proton fraction and temperature, Sec. III.B) advanced together, one
// velocity-Verlet step per launch of a persistent kernel whose phases are
// separated by device-wide barriers, replayed from a captured hipGraph.
//
// Phases of one step (every system at once):
//   P1 drift      first half kick, drift, wrap, box growth from the device step
//                 counter, cell binning with wave-aggregated counts
//   P2 scan       one workgroup per system: bin starts, nuclear work list
//   P3 scatter    bin cursors, visiting particles in the previous cell order
//   P4 rank       stable order (bin, index) and fixed-point staging
//   P5 forces     one dynamic work queue holding every system's Coulomb tiles
//                 and nuclear cell tiles (uneven systems balance on it)
//   P6 combine    nuclear + Coulomb partials, second half kick, kinetic energy
//   P7 thermostat one workgroup per system on rescale steps (multi-kernel
//                 form: the combine's last workgroup, every system)
// The same phase functions also run as one kernel per phase ("multi-kernel"
// form) for comparison.  Barrier waits are bounded: a grid that is not fully
// resident sets an error bit and every workgroup leaves.
#include <type_traits>

#include "pair_items.hpp"

namespace pasta {

namespace {

constexpr int BW = WG;  // threads per workgroup in every phase
constexpr uint32_t ERR_BARRIER = 1u << 7;
constexpr long BARRIER_SPIN_LIMIT = 1L << 22;

struct SysDev {
    int64_t off;          // first particle of the system in the concatenated arrays
    int32_t n, Z;
    double L0, xi_dot, dt, T, hdtm;
    int32_t rescale_every, scale_positions;
    int64_t bin_off;      // count/fill: 2*C_max*BSUB entries
    int64_t start_off;    // start: 2*C_max*BSUB + 1 entries
    int64_t item_off;     // nuclear items: item_max pairs
    int32_t item_max;
    int64_t coul_off;     // Coulomb partials: S*Z entries
    // Coulomb form: 0 = gather tiles (coul_blocks x S splits of per_split
    // sources), 1 = pairwise super-block items (S = super-blocks)
    int32_t S, per_split, coul_blocks, coul_form;
    int64_t chunk_off;    // particle chunks of BW
    int32_t nchunks;
    int64_t coul_item_off;
    int64_t nuc_item_off;
};

struct BatchDev {
    const SysDev* sys;
    int nsys;
    int64_t total_chunks, coul_items, nuc_items;
    PairParams pp;        // L filled per system per step
    double mass;
    // the caller's concatenated particle arrays (caller order within each
    // system): read at creation, written after every step call
    double* cpos;
    double* cvel;
    const uint8_t* species;
    // the state, kept in the sorted order of the last cell build: slot k of
    // system s holds the particle ids[k] (caller index within the system)
    double* pos;          // [3N]
    double* vel;          // [3N]
    double* force;        // [3N] F of the state's positions
    double* epot;         // [N] energy shares (when evaluated)
    int32_t* ids;
    // the rank phase's copy of the state in the new order (the combine
    // updates it into pos/vel/ids)
    double* pos_t;
    double* vel_t;
    int32_t* perm;        // new slot -> caller index
    // work arrays
    int32_t* key;         // bin of each slot's next position
    int32_t* tmp;         // scatter: new slot -> caller index (the rank key)
    int32_t* srcix;       // scatter: new slot -> current slot (where the data is)
    int32_t* count;
    int32_t* fill;
    int32_t* start;
    int32_t* items;
    int32_t* n_items;
    void* stg;            // Q4 or double4 per sorted slot
    void* coul_part;      // Coulomb partials, typename P::CPart per entry
    unsigned long long* react;  // [4][n_total] fixed-point Coulomb sums per slot (the
                                // fixed-point form; zero between force phases)
    int64_t n_total;
    double4* fnuc;
    double* ke_chunk;
    double* pending;      // per-system velocity scale pending from the thermostat
    int64_t* step;
    unsigned* barrier;    // BAR_WORDS words: generation, root count, group counts
    unsigned* queue;      // QUEUE_WORDS words: [0] force-phase work counter, then the
                          // combine's arrival counters (root, groups; multi-kernel form)
    uint32_t* err;
    unsigned long long* pairs;  // [nsys] diagnostic nuclear pair counts
    double* red;          // [256] host-read reduction partials
    int nuc_variant;      // 0 dense, 1 screened + compacted, 3 the same with 8 lanes/target
    int chunk;            // targets per nuclear work item (64, or 32 for variant 3)
    // per-system pair constants and cell grid of the current box, written
    // once per step by the drift phase (read as uniform loads by the items)
    NucConsts* nk;
    CoulConsts* ck;
    int2* grid_nc;        // (nc, C)
    long spin_limit;      // bound of a barrier wait (polls)
};

__device__ __forceinline__ int find_sys_chunk(const BatchDev& B, int64_t g)
{
    int lo = 0, hi = B.nsys;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (B.sys[mid].chunk_off <= g)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ double box_at(const SysDev& S, int64_t step)
{
    return S.L0 * (1.0 + S.xi_dot * ((double)step * S.dt));
}

// octant bins inside each cell, as in the single-system path
constexpr int BSUB = 8;
constexpr int SCAN_WG = 1024;  // threads of the per-phase scan's workgroups

// The cell grid of a system of n particles in a box of side L, as the
// single-system path builds it (cells of side at least r_cut, at most
// cap_cells per side in sparse states).
__device__ __forceinline__ Grid grid_at(double L, double r_cut, int64_t n)
{
    Grid g;
    g.sub = BSUB;
    int nc = (int)floor(L / r_cut);
    while (nc > 1 && L / (double)nc < r_cut)
        nc--;
    g.nc = cap_cells(nc < 1 ? 1 : nc, n);
    g.C = g.nc * g.nc * g.nc;
    g.inv_w = (double)g.nc / L;
    g.L = L;
    return g;
}

// Bounded grid-wide barrier, two levels: workgroup g arrives at group
// counter g % BAR_GROUPS; the last arrival of a group resets that counter
// and arrives at the root counter; the last root arrival resets the root and
// publishes a new generation, which the waiting workgroups poll.  Every word
// has a 256-byte line of its own, so the arrivals of one group, the root and
// the polling do not contend for one line, and the polls back off (up to
// about a microsecond apart) so that waiting workgroups leave the memory
// system to the ones still working.  Returns false (and every later barrier
// returns false at once) when the wait limit is hit.  Memory ordering: an
// agent-scope release fence before each arrival, an acquire + release fence
// by each last arrival before it resets its counter (the reset is ordered
// before its next arrival or the release store of the generation), and an
// agent-scope acquire fence after the generation changed.
constexpr int BAR_GROUPS = 32;
constexpr int BAR_STRIDE = 64;  // words between counters (256 bytes)
constexpr int BAR_WORDS = (2 + BAR_GROUPS) * BAR_STRIDE;
constexpr int QUEUE_WORDS = (2 + BAR_GROUPS) * BAR_STRIDE;
__device__ bool grid_sync(const BatchDev& B, int* s_flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        if (__hip_atomic_load(B.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_BARRIER) {
            ok = 0;
        } else {
            unsigned* gen_w = B.barrier;
            unsigned* root_w = B.barrier + BAR_STRIDE;
            const unsigned nb = gridDim.x;
            const unsigned grp = blockIdx.x % BAR_GROUPS;
            const unsigned ngrp = nb < BAR_GROUPS ? nb : BAR_GROUPS;
            // members of this group: the workgroups with this residue
            const unsigned gsize = nb / BAR_GROUPS + (grp < nb % BAR_GROUPS ? 1u : 0u);
            unsigned* grp_w = B.barrier + (2 + grp) * BAR_STRIDE;
            const unsigned gen = __hip_atomic_load(gen_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            bool last = false;
            if (__hip_atomic_fetch_add(grp_w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u ==
                gsize) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                __hip_atomic_store(grp_w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                last = __hip_atomic_fetch_add(root_w, 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT) + 1u == ngrp;
            }
            if (last) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
                // the reset must be visible before the new generation: a
                // released group's next arrival then counts from zero
                __hip_atomic_store(root_w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(gen_w, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                long spins = 0;
                int nap = 1;
                while (__hip_atomic_load(gen_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                       gen) {
                    if (nap >= 32)
                        __builtin_amdgcn_s_sleep(32);
                    else if (nap >= 8)
                        __builtin_amdgcn_s_sleep(8);
                    else
                        __builtin_amdgcn_s_sleep(1);
                    nap = nap < 32 ? 2 * nap : 32;
                    if (++spins > B.spin_limit) {
                        atomicOr(B.err, ERR_BARRIER);
                        ok = 0;
                        break;
                    }
                    if ((spins & 255) == 0 &&
                        (__hip_atomic_load(B.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                         ERR_BARRIER)) {
                        ok = 0;
                        break;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
        }
        *s_flag = ok;
    }
    __syncthreads();
    return *s_flag != 0;
}

// ------------------------------------------------------------- phases
// mode: 0 = initial evaluation (bin the given positions, no kick),
//       1 = a full step.
// A step's first part (half kick, drift, binning) normally runs at the end
// of the previous step's combine, over the same sorted slots; the drift
// phase runs it only for the first step of a launch sequence (`first`) and
// for systems whose thermostat rescaled the velocities at the end of the
// previous step (the factor is known only after that step's reduction).

// Whether system S's drift for step `step` is left to the drift phase.
__device__ __forceinline__ bool drift_in_phase(const SysDev& S, int64_t step, int first)
{
    return first || (S.rescale_every > 0 && step % S.rescale_every == 0);
}

// One slot's first part of step `step` (positions move to step + 1): the
// pending velocity scale sc (1 when none), then the half kick with F and
// the drift (the single-system path's drift_update), and the bin of the new
// position.  Updates x and v; returns the bin.
__device__ __forceinline__ int drift_slot(const BatchDev& B, const SysDev& S, int64_t step,
                                          double sc, double (&x)[3], double (&v)[3],
                                          const double (&f)[3], bool proton)
{
    const double L_old = box_at(S, step), L_new = box_at(S, step + 1);
    const Grid gr = grid_at(L_new, B.pp.r_nuc, S.n);
    if (sc != 1.0) {
        v[0] *= sc;
        v[1] *= sc;
        v[2] *= sc;
    }
    DriftStep c;
    c.hdtm = S.hdtm;
    c.dt = S.dt;
    c.L_new = L_new;
    c.ratio = L_new / L_old;
    c.scale_positions = S.scale_positions;
    const uint32_t bad = drift_update(x, v, f, c);
    if (bad)
        atomicOr(B.err, bad);
    return particle_bin(x[0], x[1], x[2], proton, gr.inv_w, gr.nc, gr.C, gr.sub);
}

__device__ void phase_drift(const BatchDev& B, int64_t step, int mode, int first)
{
    if (blockIdx.x == 0 && threadIdx.x == 0)
        B.queue[0] = 0u;  // work counter of this step's force phase
    // the pair constants of every system's new box
    if (blockIdx.x == 0) {
        for (int s = threadIdx.x; s < B.nsys; s += blockDim.x) {
            const SysDev& S = B.sys[s];
            PairParams pp = B.pp;
            pp.L = box_at(S, mode ? step + 1 : step);
            B.nk[s] = make_nuc_consts(pp);
            B.ck[s] = make_coul_consts(pp);
            const Grid gr = grid_at(pp.L, pp.r_nuc, S.n);
            B.grid_nc[s] = make_int2(gr.nc, gr.C);
        }
    }
    for (int64_t g = blockIdx.x; g < B.total_chunks; g += gridDim.x) {
        const int s = find_sys_chunk(B, g);
        const SysDev& S = B.sys[s];
        if (mode && !drift_in_phase(S, step, first))
            continue;  // the previous combine drifted this system
        const int64_t sl = (g - S.chunk_off) * BW + threadIdx.x;
        if (sl >= S.n)
            continue;
        const int64_t k = S.off + sl;
        const bool proton = B.species[S.off + B.ids[k]] == 1;
        double x[3] = {B.pos[3 * k], B.pos[3 * k + 1], B.pos[3 * k + 2]};
        int bin;
        if (mode) {
            double v[3] = {B.vel[3 * k], B.vel[3 * k + 1], B.vel[3 * k + 2]};
            const double f[3] = {B.force[3 * k], B.force[3 * k + 1], B.force[3 * k + 2]};
            // a thermostat at the end of the previous step left its factor
            const double sc =
                (S.rescale_every > 0 && step % S.rescale_every == 0) ? B.pending[s] : 1.0;
            bin = drift_slot(B, S, step, sc, x, v, f, proton);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                B.pos[3 * k + d] = x[d];
                B.vel[3 * k + d] = v[d];
            }
        } else {
            const double L = box_at(S, step);
            const Grid gr = grid_at(L, B.pp.r_nuc, S.n);
            if (!(x[0] >= 0.0 && x[0] < L && x[1] >= 0.0 && x[1] < L && x[2] >= 0.0 && x[2] < L))
                atomicOr(B.err, ERR_RANGE);
            bin = particle_bin(x[0], x[1], x[2], proton, gr.inv_w, gr.nc, gr.C, gr.sub);
        }
        B.key[k] = bin;
        wave_aggregated_add(B.count + S.bin_off, bin);
    }
}

static_assert(BSUB == 8, "the scan phase reads a cell's bins as two 16-byte words per species");

// Starts, nuclear work list and counter reset of each system in one
// workgroup.  Thread t owns a contiguous range of cells: their 8 proton and
// 8 neutron octant bins, read as 16-byte loads (a system's count and fill
// start 64-byte aligned, a cell's 8 counters at 32 bytes).  One workgroup
// scan of the per-thread sums (proton and neutron totals packed in one
// 64-bit word: both are below 2^31, so the low half never carries) gives the
// bin starts, a second one the items' offsets; nothing is read back that
// this phase wrote, and each thread clears the counters it alone read.
__device__ void phase_scan(const BatchDev& B, int64_t step, int mode, char* lds_raw)
{
    int64_t* lds = reinterpret_cast<int64_t*>(lds_raw);
    for (int s = blockIdx.x; s < B.nsys; s += gridDim.x) {
        const SysDev& S = B.sys[s];
        const double L = box_at(S, mode ? step + 1 : step);
        const Grid gr = grid_at(L, B.pp.r_nuc, S.n);
        int32_t* count = B.count + S.bin_off;
        int32_t* fill = B.fill + S.bin_off;
        int32_t* start = B.start + S.start_off;
        const int64_t C = gr.C, CS = C * BSUB;
        const int64_t per = (C + blockDim.x - 1) / blockDim.x;
        const int64_t c0 = min((int64_t)threadIdx.x * per, C), c1 = min(c0 + per, C);
        int64_t sp = 0, sn = 0, sq = 0;
        for (int64_t c = c0; c < c1; ++c) {
            const int4* cp = reinterpret_cast<const int4*>(count + BSUB * c);
            const int4* cn = reinterpret_cast<const int4*>(count + CS + BSUB * c);
            const int4 p0 = cp[0], p1 = cp[1], n0 = cn[0], n1 = cn[1];
            const int32_t mp = p0.x + p0.y + p0.z + p0.w + p1.x + p1.y + p1.z + p1.w;
            const int32_t mn = n0.x + n0.y + n0.z + n0.w + n1.x + n1.y + n1.z + n1.w;
            sp += mp;
            sn += mn;
            sq += (mp + mn + B.chunk - 1) / B.chunk;
        }
        int64_t tot = 0, tq = 0;
        const int64_t pre = block_exclusive_scan(sp | (sn << 32), lds, &tot);
        int64_t bq = block_exclusive_scan(sq, lds, &tq);
        const int64_t Zt = tot & 0xffffffffll;  // all protons of the system
        int32_t bp = (int32_t)(pre & 0xffffffffll), bn = (int32_t)(Zt + (pre >> 32));
        int32_t* items = B.items + 2 * S.item_off;
        const int4 z{0, 0, 0, 0};
        for (int64_t c = c0; c < c1; ++c) {
            int4* cp = reinterpret_cast<int4*>(count + BSUB * c);
            int4* cn = reinterpret_cast<int4*>(count + CS + BSUB * c);
            const int4 p0 = cp[0], p1 = cp[1], n0 = cn[0], n1 = cn[1];
            const int32_t kp[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
            const int32_t kn[8] = {n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, n1.z, n1.w};
            int32_t m = 0;
#pragma unroll
            for (int o = 0; o < BSUB; ++o) {
                start[BSUB * c + o] = bp;
                start[CS + BSUB * c + o] = bn;
                bp += kp[o];
                bn += kn[o];
                m += kp[o] + kn[o];
            }
            const int32_t k = (m + B.chunk - 1) / B.chunk;
            for (int32_t q = 0; q < k; ++q) {
                items[2 * (bq + q) + 0] = (int32_t)c;
                items[2 * (bq + q) + 1] = q;
            }
            bq += k;
            int4* fp = reinterpret_cast<int4*>(fill + BSUB * c);
            int4* fn = reinterpret_cast<int4*>(fill + CS + BSUB * c);
            cp[0] = z;
            cp[1] = z;
            cn[0] = z;
            cn[1] = z;
            fp[0] = z;
            fp[1] = z;
            fn[0] = z;
            fn[1] = z;
        }
        if (threadIdx.x == 0) {
            start[2 * CS] = (int32_t)(Zt + (tot >> 32));
            B.n_items[s] = (int32_t)tq;
        }
        __syncthreads();
    }
}

// The slots of each bin in the new order, visiting the current (sorted)
// slots: tmp[new slot] = caller index, srcix[new slot] = current slot, in
// an order the rank phase then makes stable.
__device__ void phase_scatter(const BatchDev& B)
{
    for (int64_t g = blockIdx.x; g < B.total_chunks; g += gridDim.x) {
        const int s = find_sys_chunk(B, g);
        const SysDev& S = B.sys[s];
        const int64_t sl = (g - S.chunk_off) * BW + threadIdx.x;
        if (sl >= S.n)
            continue;
        const int b = B.key[S.off + sl];
        const int slot = B.start[S.start_off + b] + wave_aggregated_add(B.fill + S.bin_off, b);
        B.tmp[S.off + slot] = B.ids[S.off + sl];
        B.srcix[S.off + slot] = (int32_t)sl;
    }
}

template <class P>
__device__ void phase_rank(const BatchDev& B, int64_t step, int mode)
{
    auto* stg = reinterpret_cast<typename P::Src*>(B.stg);
    for (int64_t g = blockIdx.x; g < B.total_chunks; g += gridDim.x) {
        const int s = find_sys_chunk(B, g);
        const SysDev& S = B.sys[s];
        const int64_t sl = (g - S.chunk_off) * BW + threadIdx.x;
        if (sl >= S.n)
            continue;
        const int32_t* tmp = B.tmp + S.off;
        const int32_t id = tmp[sl];               // caller index: the rank key
        const int32_t src = B.srcix[S.off + sl];  // current slot: where its data is
        const int b = B.key[S.off + src];
        const int beg = B.start[S.start_off + b], end = B.start[S.start_off + b + 1];
        int r = 0, k = beg;
        for (; k + 8 <= end; k += 8) {
            int32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = tmp[k + u];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                r += v[u] < id;
        }
        for (; k < end; ++k)
            r += tmp[k] < id;
        // new slot: the bin's start plus the rank of the caller index among
        // the bin's members, the single-system path's order
        const int dst = beg + r;
        const int64_t i = S.off + src, o = S.off + dst;
        B.perm[o] = id;
        const uint8_t sp = B.species[S.off + id];
        const double x = B.pos[3 * i], y = B.pos[3 * i + 1], z = B.pos[3 * i + 2];
        const double vx = B.vel[3 * i], vy = B.vel[3 * i + 1], vz = B.vel[3 * i + 2];
        B.pos_t[3 * o] = x;
        B.pos_t[3 * o + 1] = y;
        B.pos_t[3 * o + 2] = z;
        B.vel_t[3 * o] = vx;
        B.vel_t[3 * o + 1] = vy;
        B.vel_t[3 * o + 2] = vz;
        if constexpr (sizeof(typename P::Src) == sizeof(Q4)) {
            const double L = box_at(S, mode ? step + 1 : step);
            const double qs = 4294967296.0 / L;
            Q4 q;
            q.x = (uint32_t)(uint64_t)(x * qs);
            q.y = (uint32_t)(uint64_t)(y * qs);
            q.z = (uint32_t)(uint64_t)(z * qs);
            q.w = sp;
            reinterpret_cast<Q4*>(stg)[o] = q;
        } else {
            reinterpret_cast<double4*>(stg)[o] = make_double4(x, y, z, (double)sp);
        }
    }
}

// M: what the pair items accumulate (MODE_FORCE in steps, MODE_ENERGY when
// the energies are asked for, MODE_COUNT for the pair counts).
template <class P, int M, int V>
// only < 0: the workgroups take items from the device work counter until
// it passes the last (persistent form); only >= 0: this workgroup runs item
// `only` alone (one workgroup per item, balanced by the dispatcher).
__device__ void phase_forces(const BatchDev& B, int64_t step, int mode, char* lds, int* s_item,
                             int64_t only)
{
    const auto* stg = reinterpret_cast<const typename P::Src*>(B.stg);
    const int64_t total = B.coul_items + B.nuc_items;
    unsigned* ctr = B.queue;
    auto run = [&](const int64_t it) {
        if (it < B.coul_items) {
            if (M == MODE_COUNT)
                return;
            int s = 0;
            while (s + 1 < B.nsys && B.sys[s + 1].coul_item_off <= it)
                ++s;
            s = __builtin_amdgcn_readfirstlane(s);  // uniform: the constants load as scalars
            const SysDev& S = B.sys[s];
            const int64_t local = it - S.coul_item_off;
            const CoulConsts k = B.ck[s];
            using PT = typename P::CPart;
            PT* part = static_cast<PT*>(B.coul_part) + S.coul_off;
            if (S.coul_form == 1) {
                coulomb_pair_item<P, M != MODE_FORCE>(stg + S.off, S.Z, k, part, (int)local, lds);
            } else if (S.coul_form == 3) {
                coulomb_pair_item<P, M != MODE_FORCE>(
                    stg + S.off, S.Z, k, FixedPart{B.react + S.off, B.err, B.n_total},
                    (int)local, lds);
            } else {
                const int tblock = (int)(local % S.coul_blocks),
                          split = (int)(local / S.coul_blocks);
                coulomb_item<P, M != MODE_FORCE, PT>(stg + S.off, S.Z, S.per_split, k, part,
                                                     tblock, split, lds);
            }
        } else {
            const int64_t jt = it - B.coul_items;
            int s = 0;
            while (s + 1 < B.nsys && B.sys[s + 1].nuc_item_off <= jt)
                ++s;
            s = __builtin_amdgcn_readfirstlane(s);
            const SysDev& S = B.sys[s];
            const int local = (int)(jt - S.nuc_item_off);
            if (local >= B.n_items[s])
                return;
            const NucConsts k = B.nk[s];
            const int2 gnc = B.grid_nc[s];
            NucArgs A{};
            A.start = B.start + S.start_off;
            A.items = B.items + 2 * S.item_off;
            A.perm = B.perm + S.off;
            A.nc = gnc.x;
            A.C = gnc.y;
            A.sub = BSUB;
            A.Z = S.Z;
            A.fnuc = B.fnuc + S.off;  // raw nuclear part; combine adds the rest
            A.pairs = B.pairs + s;
            A.err = B.err;
            if constexpr (V == 3)
                nuclear_item_compact_t<P, 8, true, M>(stg + S.off, A, k, local, lds);
            else if constexpr (V == 1)
                nuclear_item_compact<P, true, M>(stg + S.off, A, k, local, lds);
            else
                nuclear_item<P, true, M>(stg + S.off, A, k, local, lds);
        }
    };
    if (only >= 0) {
        if (only < total)
            run(only);
        return;
    }
    // the first item of workgroup b is item b; later ones come from the
    // counter (which starts at zero in every step), fetched when an item
    // starts so that the fetch overlaps the item's first loads
    int64_t it = blockIdx.x;
    while (it < total) {
        if (threadIdx.x == 0)
            s_item[0] = (int)(gridDim.x + atomicAdd(ctr, 1u));
        run(it);
        __syncthreads();
        it = __builtin_amdgcn_readfirstlane(s_item[0]);  // uniform: the next item
        __syncthreads();
    }
}

// Whether system S rescales its velocities at the end of step `step`.
__device__ __forceinline__ bool rescales_at(const SysDev& S, int64_t step, int mode)
{
    return mode && S.rescale_every > 0 && (step + 1) % S.rescale_every == 0;
}

// energy: the pair phase accumulated energies; write the shares.
// The Coulomb partials of a proton are summed in partial order from zero
// and the sum is added to the nuclear part, as in the single-system
// combine.  That combine spreads a proton's partials over lanes and adds the
// lane sums by a fixed tree; in mixed precision the partials are FP32 values
// summed in FP64, which is exact unless their exponents span more than 29
// bits, so the two orders give the same bits in practice (FP64 partials
// can differ in the last bit).
//
// The combine walks the new slots: F (written per slot), and with `state`
// the state moves from the rank phase's copy into pos/vel/ids, in a step
// (mode 1) with the second half kick (the kinetic-energy partials are of
// these velocities).  With `drift_next`, a system that does not rescale at
// the end of this step then takes the first part of step + 1 here (half
// kick with the same F, drift, bin); the velocities kept are then the
// half-step ones, which the next combine completes.  Without `state`
// (energies of the current state) only F and the energy shares are written.
template <class P>
__device__ void phase_combine(const BatchDev& B, int64_t step, int mode, bool energy, bool state,
                              bool drift_next, char* lds_raw)
{
    using PT = typename P::CPart;
    const PT* part = static_cast<const PT*>(B.coul_part);
    double* red = reinterpret_cast<double*>(lds_raw);
    for (int64_t g = blockIdx.x; g < B.total_chunks; g += gridDim.x) {
        const int s = find_sys_chunk(B, g);
        const SysDev& S = B.sys[s];
        const int64_t sl = (g - S.chunk_off) * BW + threadIdx.x;
        const bool drift = state && drift_next && mode && !rescales_at(S, step, mode);
        double ke = 0.0;
        if (sl < S.n) {
            const int64_t k = S.off + sl;
            const double4 fn = B.fnuc[k];
            double Fx = fn.x, Fy = fn.y, Fz = fn.z, V = fn.w;
            if (sl < S.Z && S.coul_form == 3) {
                // fixed-point sums, cleared for the next force phase
                unsigned long long* r = B.react + k;
                const int64_t N = B.n_total;
                Fx += (double)(long long)r[0] * REACT_UNIT;
                Fy += (double)(long long)r[N] * REACT_UNIT;
                Fz += (double)(long long)r[2 * N] * REACT_UNIT;
                V += (double)(long long)r[3 * N] * REACT_UNIT;
                r[0] = 0ull;
                r[N] = 0ull;
                r[2 * N] = 0ull;
                r[3 * N] = 0ull;
            } else if (sl < S.Z) {
                // partials in order k = 0, 1, ..., loaded eight at a time so
                // that the loads are in flight together
                constexpr int U = 8;
                const PT* pp = part + S.coul_off + sl;
                double cx = 0.0, cy = 0.0, cz = 0.0, cw = 0.0;
                for (int k0 = 0; k0 < S.S; k0 += U) {
                    PT cp[U];
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        cp[u] = k0 + u < S.S ? pp[(int64_t)(k0 + u) * S.Z] : PT{};
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        cx += (double)cp[u].x;
                        cy += (double)cp[u].y;
                        cz += (double)cp[u].z;
                        cw += (double)cp[u].w;
                    }
                }
                Fx += cx;
                Fy += cy;
                Fz += cz;
                V += cw;
            }
            B.force[3 * k + 0] = Fx;
            B.force[3 * k + 1] = Fy;
            B.force[3 * k + 2] = Fz;
            if (energy)
                B.epot[k] = 0.5 * V;
            if (!(isfinite(Fx) && isfinite(Fy) && isfinite(Fz)))
                atomicOr(B.err, ERR_NONFINITE_FORCE);
            if (state) {
                const int32_t cid = B.perm[k];
                B.ids[k] = cid;
                double x[3] = {B.pos_t[3 * k], B.pos_t[3 * k + 1], B.pos_t[3 * k + 2]};
                double v[3] = {B.vel_t[3 * k], B.vel_t[3 * k + 1], B.vel_t[3 * k + 2]};
                if (mode) {
                    v[0] = v[0] + S.hdtm * Fx;
                    v[1] = v[1] + S.hdtm * Fy;
                    v[2] = v[2] + S.hdtm * Fz;
                    ke = 0.5 * B.mass * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                }
                if (drift) {
                    const double f[3] = {Fx, Fy, Fz};
                    const bool proton = B.species[S.off + cid] == 1;
                    const int bin = drift_slot(B, S, step + 1, 1.0, x, v, f, proton);
                    B.key[k] = bin;
                    wave_aggregated_add(B.count + S.bin_off, bin);
                }
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    B.pos[3 * k + d] = x[d];
                    B.vel[3 * k + d] = v[d];
                }
            }
        }
        // fixed-order block reduction of the chunk's kinetic energy
        for (int m = 32; m >= 1; m >>= 1)
            ke += __shfl_xor(ke, m, 64);
        if ((threadIdx.x & 63) == 0)
            red[threadIdx.x >> 6] = ke;
        __syncthreads();
        if (threadIdx.x == 0)
            B.ke_chunk[g] = ((red[0] + red[1]) + red[2]) + red[3];
        __syncthreads();
    }
}

// Systems first, first + stride, ... (one workgroup each).
__device__ void phase_thermostat(const BatchDev& B, int64_t step, int mode, char* lds_raw,
                                 int first, int stride)
{
    double* red = reinterpret_cast<double*>(lds_raw);
    for (int s = first; s < B.nsys; s += stride) {
        const SysDev& S = B.sys[s];
        if (!rescales_at(S, step, mode)) {
            if (threadIdx.x == 0)
                B.pending[s] = 1.0;
            continue;
        }
        double acc = 0.0;
        for (int k = threadIdx.x; k < S.nchunks; k += BW)
            acc += B.ke_chunk[S.chunk_off + k];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int off = BW / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off)
                red[threadIdx.x] += red[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double ke = red[0];
            B.pending[s] = ke > 0.0 ? sqrt(1.5 * (double)S.n * S.T / ke) : 1.0;
        }
        __syncthreads();
    }
}

// One instantiation per nuclear variant V (registers and LDS sized for it).
template <class P, int V>
constexpr int batch_lds()
{
    constexpr int a = coulomb_lds_bytes<P>();
    constexpr int b = V == 0 ? nuclear_lds_bytes<P>() : nuclear_compact_lds_bytes<P>();
    return (a > b ? a : b) + 64;
}

// Waves per SIMD the persistent kernel is compiled for: five in mixed
// precision (96 VGPRs, no spills, five workgroups per CU), the compiler's
// choice in FP64.
template <class P>
constexpr int persist_waves() { return std::is_same<P, MixedPolicy>::value ? 5 : 1; }

template <class P, int M, int V>
__global__ __launch_bounds__(BW) __attribute__((amdgpu_waves_per_eu(persist_waves<P>())))
void k_batch_step(BatchDev B, int mode, int first, int last)
{
    __shared__ __align__(16) char lds[batch_lds<P, V>()];
    __shared__ int s_flag, s_item;
    if (__hip_atomic_load(B.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_BARRIER)
        return;
    const int64_t step = *B.step;
    phase_drift(B, step, mode, first);
    // the barrier after the drift phase only when it moved particles (what
    // else it writes is read after later barriers)
    bool moved = !mode || first;
    for (int s = 0; s < B.nsys && !moved; ++s)
        moved = drift_in_phase(B.sys[s], step, first);
    if (moved && !grid_sync(B, &s_flag))
        return;
    phase_scan(B, step, mode, lds);
    if (!grid_sync(B, &s_flag))
        return;
    phase_scatter(B);
    if (!grid_sync(B, &s_flag))
        return;
    phase_rank<P>(B, step, mode);
    if (!grid_sync(B, &s_flag))
        return;
    phase_forces<P, M, V>(B, step, mode, lds, &s_item, -1);
    if (!grid_sync(B, &s_flag))
        return;
    phase_combine<P>(B, step, mode, M != MODE_FORCE, true, !last, lds);
    // the thermostat (and the barrier before it) only in steps where some
    // system rescales; the next step's drift reads the factor only then
    bool thermo = false;
    for (int s = 0; s < B.nsys && mode; ++s)
        thermo |= B.sys[s].rescale_every > 0 && (step + 1) % B.sys[s].rescale_every == 0;
    if (thermo) {
        if (!grid_sync(B, &s_flag))
            return;
        phase_thermostat(B, step, mode, lds, blockIdx.x, gridDim.x);
    }
    if (mode && blockIdx.x == 0 && threadIdx.x == 0)
        *B.step = step + 1;
}

// ---- the same phases as separate kernels (multi-kernel form) -----------
template <class P>
__global__ __launch_bounds__(BW) void k_ph_drift(BatchDev B, int mode, int first)
{
    phase_drift(B, *B.step, mode, first);
}
// one workgroup of SCAN_WG threads per system (the persistent kernel runs the
// same phase with its BW threads)
__global__ __launch_bounds__(SCAN_WG) void k_ph_scan(BatchDev B, int mode)
{
    __shared__ __align__(16) char lds[BW * 8];
    phase_scan(B, *B.step, mode, lds);
}
__global__ __launch_bounds__(BW) void k_ph_scatter(BatchDev B) { phase_scatter(B); }
template <class P>
__global__ __launch_bounds__(BW) void k_ph_rank(BatchDev B, int mode)
{
    phase_rank<P>(B, *B.step, mode);
}
// Waves per SIMD the force phase is compiled for.  Without a bound the
// compiler takes up to 138 VGPRs for the compacting items (three waves).
// Five keeps it within 96 VGPRs without spills; six (80 VGPRs) spills a few
// registers but ran the mixed-precision variant-3 steps 4 % faster on the
// 15-system grid, while it slowed variant 1, which stays at five.
template <class P, int M, int V>
constexpr int ph_force_waves()
{
    return (std::is_same<P, MixedPolicy>::value && M == MODE_FORCE && V == 3) ? 6 : 5;
}
template <class P, int M, int V>
__global__ __launch_bounds__(BW) __attribute__((amdgpu_waves_per_eu(ph_force_waves<P, M, V>()))) void k_ph_forces(BatchDev B, int mode)
{
    __shared__ __align__(16) char lds[batch_lds<P, V>()];
    __shared__ int s_item;
    phase_forces<P, M, V>(B, *B.step, mode, lds, &s_item, (int64_t)blockIdx.x);
}

template <class F>
void with_batch_variant(int v, F f)
{
    if (v == 0)
        f(std::integral_constant<int, 0>());
    else if (v == 3)
        f(std::integral_constant<int, 3>());
    else
        f(std::integral_constant<int, 1>());
}

// The pair phase alone (mode 0: the state in place, no kick).
// Per-phase force launches: one workgroup per work item (every system's
// Coulomb items, then its nuclear item slots; empty slots exit at once).
inline unsigned item_grid(const BatchDev& dev)
{
    const int64_t t = dev.coul_items + dev.nuc_items;
    return (unsigned)(t > 0 ? t : 1);
}

template <int M>
void launch_pair_phase(const BatchDev& dev, int precision, hipStream_t s)
{
    const unsigned g = item_grid(dev);
    with_batch_variant(dev.nuc_variant, [&](auto vt) {
        constexpr int V = decltype(vt)::value;
        if (precision == PASTA_FP64)
            k_ph_forces<Fp64Policy, M, V><<<g, BW, 0, s>>>(dev, 0);
        else
            k_ph_forces<MixedPolicy, M, V><<<g, BW, 0, s>>>(dev, 0);
    });
}
// Two-level arrival count (thread 0 of each workgroup; no waiting): workgroup
// b arrives on the counter of group b mod BAR_GROUPS, the last member of a
// group on the root.  True in the one workgroup that arrives last.  Every
// counter is back at zero afterwards.  With `ordered`, each arrival is a
// release and the last one an acquire at agent scope, so the last workgroup
// sees every workgroup's earlier writes.
__device__ bool last_arrival(unsigned* ctr, bool ordered)
{
    const unsigned nb = gridDim.x;
    const unsigned grp = blockIdx.x % BAR_GROUPS;
    const unsigned ngrp = nb < BAR_GROUPS ? nb : BAR_GROUPS;
    const unsigned gsize = nb / BAR_GROUPS + (grp < nb % BAR_GROUPS ? 1u : 0u);
    unsigned* grp_w = ctr + (2 + grp) * BAR_STRIDE;
    unsigned* root_w = ctr + BAR_STRIDE;
    if (ordered)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (__hip_atomic_fetch_add(grp_w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u != gsize)
        return false;
    __hip_atomic_store(grp_w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ordered)
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
    if (__hip_atomic_fetch_add(root_w, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u != ngrp)
        return false;
    __hip_atomic_store(root_w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ordered)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return true;
}

// The combine phase.  With `tail`, the last workgroup to finish then runs
// the thermostat phase for every system and, in a step, advances the step
// counter, so a step needs no launches after the combine.  Every workgroup
// reads the step counter before it arrives, so the last one may advance it.
// Only on a step where some system rescales does the last workgroup read the
// others' kinetic-energy partials, and only then are the arrivals ordered by
// agent-scope fences: on this multi-XCD GPU those write back and invalidate
// L2, which costs tens of microseconds per launch when every workgroup
// issues them.
template <class P>
__global__ __launch_bounds__(BW) void k_ph_combine(BatchDev B, int mode, int energy, int tail,
                                                  int state, int drift_next)
{
    __shared__ __align__(16) char lds[BW * 8];
    __shared__ int s_last, s_rescale;
    __shared__ int64_t s_step;
    if (threadIdx.x == 0) {
        const int64_t step = *B.step;
        bool any = false;
        for (int s = 0; s < B.nsys; ++s)
            any |= rescales_at(B.sys[s], step, mode);
        s_step = step;
        s_rescale = any;
    }
    __syncthreads();
    phase_combine<P>(B, s_step, mode, energy != 0, state != 0, drift_next != 0, lds);
    if (!tail)
        return;
    __syncthreads();
    if (threadIdx.x == 0)
        s_last = last_arrival(B.queue, s_rescale != 0);
    __syncthreads();
    if (!s_last)
        return;
    const int64_t step = s_step;
    phase_thermostat(B, step, mode, lds, 0, 1);
    if (mode && threadIdx.x == 0)
        *B.step = step + 1;
}

// Apply the pending thermostat scale to the velocities (end of a step call;
// the velocities are then full-step ones: the last step does not drift).
__global__ __launch_bounds__(BW) void k_apply_pending(BatchDev B)
{
    for (int64_t g = blockIdx.x; g < B.total_chunks; g += gridDim.x) {
        const int s = find_sys_chunk(B, g);
        const SysDev& S = B.sys[s];
        const int64_t sl = (g - S.chunk_off) * BW + threadIdx.x;
        // only a thermostat in the last step left a factor to apply
        const int64_t st = *B.step;
        if (sl < S.n && S.rescale_every > 0 && st % S.rescale_every == 0) {
            const double sc = B.pending[s];
            double* v = B.vel + 3 * (S.off + sl);
            v[0] *= sc;
            v[1] *= sc;
            v[2] *= sc;
        }
    }
}
__global__ void k_reset_pending(BatchDev B)
{
    if (threadIdx.x < (unsigned)B.nsys)
        B.pending[threadIdx.x] = 1.0;
}

// The caller's state into the slots, in caller order (ids = identity).
__global__ __launch_bounds__(BW) void k_batch_load(BatchDev B, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * BW + threadIdx.x; k < n; k += (int64_t)gridDim.x * BW) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            B.pos[3 * k + d] = B.cpos[3 * k + d];
            B.vel[3 * k + d] = B.cvel[3 * k + d];
        }
    }
    for (int s = 0; s < B.nsys; ++s) {
        const SysDev& S = B.sys[s];
        for (int64_t k = (int64_t)blockIdx.x * BW + threadIdx.x; k < S.n;
             k += (int64_t)gridDim.x * BW)
            B.ids[S.off + k] = (int32_t)k;
    }
}

// Slot-ordered arrays of `width` doubles per particle back into caller
// order: dst[ids[k]] = src[k] within each system.
__global__ __launch_bounds__(BW) void k_batch_unsort(BatchDev B, const double* __restrict__ src,
                                                     double* __restrict__ dst, int width)
{
    for (int64_t g = blockIdx.x; g < B.total_chunks; g += gridDim.x) {
        const int s = find_sys_chunk(B, g);
        const SysDev& S = B.sys[s];
        const int64_t sl = (g - S.chunk_off) * BW + threadIdx.x;
        if (sl >= S.n)
            continue;
        const int64_t k = S.off + sl, i = S.off + B.ids[k];
        for (int d = 0; d < width; ++d)
            dst[width * i + d] = src[width * k + d];
    }
}

__global__ __launch_bounds__(BW) void k_batch_zero(int32_t* a, int32_t* b, int64_t m)
{
    for (int64_t k = (int64_t)blockIdx.x * BW + threadIdx.x; k < m; k += (int64_t)gridDim.x * BW) {
        a[k] = 0;
        b[k] = 0;
    }
}

__global__ void k_batch_init_scalars(BatchDev B, int64_t step0)
{
    for (int k = threadIdx.x; k < BAR_WORDS; k += blockDim.x)
        B.barrier[k] = 0u;
    if (threadIdx.x == 0) {
        *B.step = step0;
        *B.err = 0u;
    }
    for (int k = threadIdx.x; k < QUEUE_WORDS; k += blockDim.x)
        B.queue[k] = 0u;
    if (threadIdx.x < (unsigned)B.nsys) {
        B.pending[threadIdx.x] = 1.0;
        B.pairs[threadIdx.x] = 0ull;
    }
}

__global__ void k_batch_zero_pairs(BatchDev B)
{
    if (threadIdx.x < (unsigned)B.nsys)
        B.pairs[threadIdx.x] = 0ull;
    for (int k = threadIdx.x; k < QUEUE_WORDS; k += blockDim.x)
        B.queue[k] = 0u;
}

__global__ __launch_bounds__(BW) void k_batch_partial(const double* x, int64_t n, int kind,
                                                      double mass, double* out)
{
    __shared__ double lds[BW];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BW + threadIdx.x; i < n; i += (int64_t)gridDim.x * BW) {
        if (kind == 0) {
            s += x[i];
        } else {
            const double vx = x[3 * i], vy = x[3 * i + 1], vz = x[3 * i + 2];
            s += 0.5 * mass * (vx * vx + vy * vy + vz * vz);
        }
    }
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int off = BW / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            lds[threadIdx.x] += lds[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[blockIdx.x] = lds[0];
}

}  // namespace
}  // namespace pasta

// ===================================================================== host
#include <vector>

using namespace pasta;

struct pasta_batch {
    pasta_potential pot;
    int precision;
    int mode;            // 0 persistent, 1 multi-kernel
    int nsys;
    int64_t n_total;
    int64_t step;
    int steps_per_graph;
    std::vector<SysDev> sys;
    std::vector<pasta_integrator> integ;
    BatchDev dev;
    hipStream_t user;    // the caller's stream
    hipStream_t stream;  // the batch's own stream (graphs cannot be captured on
                         // the null stream); joined to the caller's by events
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    unsigned grid;       // persistent grid size
    unsigned phase_grid; // multi-kernel grid size
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double* red;         // [256]
    bool epot_valid = false;  // steps compute forces only
    ~pasta_batch()
    {
        if (stream)
            (void)hipStreamSynchronize(stream);
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (graph)
            (void)hipGraphDestroy(graph);
        if (ev_in)
            (void)hipEventDestroy(ev_in);
        if (ev_out)
            (void)hipEventDestroy(ev_out);
        if (stream)
            (void)hipStreamDestroy(stream);
    }
};

namespace {
// The batch's stream waits for the work already queued on the caller's
// stream, and the caller's stream for the batch's work.
int join_in(pasta_batch* bt)
{
    PASTA_HIP(hipEventRecord(bt->ev_in, bt->user));
    PASTA_HIP(hipStreamWaitEvent(bt->stream, bt->ev_in, 0));
    return PASTA_OK;
}
int join_out(pasta_batch* bt)
{
    PASTA_HIP(hipEventRecord(bt->ev_out, bt->stream));
    PASTA_HIP(hipStreamWaitEvent(bt->user, bt->ev_out, 0));
    return PASTA_OK;
}
}  // namespace

namespace {

struct BatchLayout {
    std::vector<SysDev> sys;
    int64_t n_total = 0, total_chunks = 0, coul_items = 0, nuc_items = 0;
    int64_t bins = 0, starts = 0, items = 0, coul = 0;
};

// Nuclear variant of the batch (the lists run as 3: the batch rebuilds its
// cells every step) and its work-item size.
int batch_variant()
{
    const int v = g_tuning.nuclear_variant;
    return v == 0 ? 0 : (v == 1 ? 1 : 3);  // lists (2) and Newton-3 (4) run as 3
}
int batch_chunk() { return nuclear_chunk_for(batch_variant()); }

int batch_layout(const pasta_potential* pot, int precision, int nsys, const int64_t* n,
                 const int64_t* Z,
                 const double* L_max, BatchLayout* out)
{
    if (!(pot->r_coul > 0) || std::isfinite(pot->r_coul))
        return fail(PASTA_EINVAL, "pasta_batch: the batched path takes the uncut Coulomb term "
                                  "only (r_coul = INFINITY)");
    BatchLayout lay;
    lay.sys.resize(nsys);
    for (int s = 0; s < nsys; ++s) {
        SysDev& S = lay.sys[s];
        S = SysDev{};
        if (n[s] <= 0 || n[s] > INT32_MAX / 2 || !(L_max[s] >= 2.0 * pot->r_nuc))
            return fail(PASTA_EINVAL, "pasta_batch: system %d: bad n or box", s);
        const int C_max = make_grid(L_max[s], pot->r_nuc).C;
        S.off = lay.n_total;
        S.n = (int32_t)n[s];
        S.Z = Z ? (int32_t)Z[s] : (int32_t)n[s];
        S.bin_off = lay.bins;
        S.start_off = lay.starts;
        S.item_max = (int32_t)(n[s] / batch_chunk() + C_max + 1);
        S.item_off = lay.items;
        // the partial capacity depends on n only (the single-system path's
        // rule), and the plan keeps S * Z within it for the system's Z
        const int64_t cap = coulomb_partial_capacity(n[s]);
        const CoulPlan cp = coulomb_plan(S.Z, cap, false, precision == PASTA_MIXED);
        S.coul_form = cp.form;
        S.S = cp.S;
        S.per_split = (S.S && cp.form == 0) ? (int32_t)((S.Z + S.S - 1) / S.S) : 0;
        S.coul_blocks = (int32_t)((S.Z + WG - 1) / WG);
        S.coul_off = lay.coul;
        S.nchunks = (int32_t)((n[s] + BW - 1) / BW);
        S.chunk_off = lay.total_chunks;
        S.coul_item_off = lay.coul_items;
        S.nuc_item_off = lay.nuc_items;
        lay.n_total += n[s];
        lay.bins += 2 * (int64_t)C_max * BSUB;
        lay.starts += 2 * (int64_t)C_max * BSUB + 1;
        lay.items += S.item_max;
        lay.coul += cap;
        lay.total_chunks += S.nchunks;
        lay.coul_items += (cp.form == 1 || cp.form == 3) ? coulomb_pair_items(S.Z)
                                                         : (int64_t)S.coul_blocks * S.S;
        lay.nuc_items += S.item_max;
    }
    *out = lay;
    return PASTA_OK;
}

size_t batch_carve(Carver& cv, const BatchLayout& lay, int nsys, int precision, BatchDev* d)
{
    BatchDev b{};
    const int64_t N = lay.n_total;
    b.sys = cv.take<SysDev>(nsys);
    b.pos = cv.take<double>(3 * N);
    b.vel = cv.take<double>(3 * N);
    b.force = cv.take<double>(3 * N);
    b.epot = cv.take<double>(N);
    b.ids = cv.take<int32_t>(N);
    b.pos_t = cv.take<double>(3 * N);
    b.vel_t = cv.take<double>(3 * N);
    b.perm = cv.take<int32_t>(N);
    b.key = cv.take<int32_t>(N);
    b.tmp = cv.take<int32_t>(N);
    b.srcix = cv.take<int32_t>(N);
    b.count = cv.take<int32_t>(lay.bins);
    b.fill = cv.take<int32_t>(lay.bins);
    b.start = cv.take<int32_t>(lay.starts);
    b.items = cv.take<int32_t>(2 * lay.items);
    b.n_items = cv.take<int32_t>(nsys);
    b.stg = precision == PASTA_FP64 ? (void*)cv.take<double4>(N) : (void*)cv.take<Q4>(N);
    if (precision == PASTA_FP64)
        b.coul_part = cv.take<double4>(lay.coul);
    else
        b.coul_part = cv.take<float4>(lay.coul);
    b.react = cv.take<unsigned long long>(4 * N);
    b.n_total = N;
    b.fnuc = cv.take<double4>(N);
    b.ke_chunk = cv.take<double>(lay.total_chunks);
    b.pending = cv.take<double>(nsys);
    b.step = cv.take<int64_t>(1);
    b.barrier = cv.take<unsigned>(BAR_WORDS);
    b.queue = cv.take<unsigned>(QUEUE_WORDS);
    b.err = cv.take<uint32_t>(1);
    b.pairs = cv.take<unsigned long long>(nsys);
    b.red = cv.take<double>(256);
    b.nk = cv.take<NucConsts>(nsys);
    b.ck = cv.take<CoulConsts>(nsys);
    b.grid_nc = cv.take<int2>(nsys);
    if (d)
        *d = b;
    return cv.size();
}

// Grid of the kernels that walk the 256-particle chunks: one workgroup per
// chunk, at most the multi-kernel grid.
static unsigned chunk_grid(const pasta_batch* bt)
{
    const int64_t c = bt->dev.total_chunks;
    return (unsigned)(c < (int64_t)bt->phase_grid ? (c > 0 ? c : 1) : bt->phase_grid);
}

// Steps (mode 1) accumulate forces only; the initial evaluation (mode 0)
// also the energies.  A run of steps launched back to back marks its first
// step (the drift phase moves every system) and its last (no drift after the
// combine, so the state ends at a full step).
template <class P>
int launch_step(pasta_batch* bt, int mode, int first, int last)
{
    hipStream_t s = bt->stream;
    if (bt->mode == 0) {
        with_batch_variant(bt->dev.nuc_variant, [&](auto vt) {
            constexpr int V = decltype(vt)::value;
            if (mode)
                k_batch_step<P, MODE_FORCE, V><<<bt->grid, BW, 0, s>>>(bt->dev, mode, first, last);
            else
                k_batch_step<P, MODE_ENERGY, V><<<bt->grid, BW, 0, s>>>(bt->dev, mode, 1, 1);
        });
    } else {
        const unsigned gc = chunk_grid(bt);
        k_ph_drift<P><<<gc, BW, 0, s>>>(bt->dev, mode, mode ? first : 1);
        k_ph_scan<<<(unsigned)bt->nsys, SCAN_WG, 0, s>>>(bt->dev, mode);
        k_ph_scatter<<<gc, BW, 0, s>>>(bt->dev);
        k_ph_rank<P><<<gc, BW, 0, s>>>(bt->dev, mode);
        const unsigned gi = item_grid(bt->dev);  // one workgroup per work item
        with_batch_variant(bt->dev.nuc_variant, [&](auto vt) {
            constexpr int V = decltype(vt)::value;
            if (mode)
                k_ph_forces<P, MODE_FORCE, V><<<gi, BW, 0, s>>>(bt->dev, mode);
            else
                k_ph_forces<P, MODE_ENERGY, V><<<gi, BW, 0, s>>>(bt->dev, mode);
        });
        // the combine's last workgroup also runs the thermostat and the advance
        k_ph_combine<P><<<gc, BW, 0, s>>>(bt->dev, mode, mode ? 0 : 1, 1, 1,
                                          mode && !last ? 1 : 0);
    }
    PASTA_HIP(hipGetLastError());
    return PASTA_OK;
}

int launch_one(pasta_batch* bt, int mode, int first = 1, int last = 1)
{
    return bt->precision == PASTA_FP64 ? launch_step<Fp64Policy>(bt, mode, first, last)
                                       : launch_step<MixedPolicy>(bt, mode, first, last);
}

int check_batch_err(pasta_batch* bt, const char* who)
{
    uint32_t e = 0;
    PASTA_HIP(hipMemcpyAsync(&e, bt->dev.err, sizeof(e), hipMemcpyDeviceToHost, bt->stream));
    PASTA_HIP(hipStreamSynchronize(bt->stream));
    if (e & ERR_BARRIER)
        return fail(PASTA_EDEVICE, "%s: a device-wide barrier timed out (grid not resident)", who);
    if (e & (ERR_RANGE | ERR_SPECIES))
        return fail(PASTA_EINVAL, "%s: %s", who, describe_device_error(e).c_str());
    if (e)
        return fail(PASTA_EDEVICE, "%s: %s", who, describe_device_error(e).c_str());
    return PASTA_OK;
}

template <class P>
int persistent_grid(int variant, unsigned* out)
{
    int dev = 0, ncu = 0, occ = 0;
    PASTA_HIP(hipGetDevice(&dev));
    PASTA_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // both instantiations run on the same grid
    int occ2 = 0;
    hipError_t e1 = hipSuccess, e2 = hipSuccess;
    with_batch_variant(variant, [&](auto vt) {
        constexpr int V = decltype(vt)::value;
        e1 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_batch_step<P, MODE_FORCE, V>,
                                                          BW, 0);
        e2 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ2, k_batch_step<P, MODE_ENERGY, V>,
                                                          BW, 0);
    });
    PASTA_HIP(e1);
    PASTA_HIP(e2);
    occ = occ < occ2 ? occ : occ2;
    if (occ < 1)
        return fail(PASTA_EHIP, "persistent batch kernel cannot be resident");
    // every workgroup must be resident at once: the occupancy the runtime
    // reports (at most eight per CU), or fewer when the tuning asks
    int per = occ < 8 ? occ : 8;
    if (g_tuning.batch_wgs_per_cu > 0 && g_tuning.batch_wgs_per_cu < per)
        per = g_tuning.batch_wgs_per_cu;
    *out = (unsigned)ncu * (unsigned)per;
    return PASTA_OK;
}

}  // namespace

extern "C" int pasta_batch_workspace(const pasta_potential* pot, int32_t precision, int32_t nsys,
                                     const int64_t* h_n, const double* h_L_max, size_t* h_bytes)
{
    if (!pot || !h_n || !h_L_max || !h_bytes || nsys <= 0 || nsys > 1024 ||
        (precision != PASTA_FP64 && precision != PASTA_MIXED))
        return fail(PASTA_EINVAL, "pasta_batch_workspace: bad argument");
    BatchLayout lay;
    PASTA_TRY(batch_layout(pot, precision, nsys, h_n, nullptr, h_L_max, &lay));
    Carver cv(nullptr);
    *h_bytes = batch_carve(cv, lay, nsys, precision, nullptr);
    return PASTA_OK;
}

extern "C" int pasta_batch_create(const pasta_potential* pot, int32_t precision, int32_t nsys,
                                  const int64_t* h_n, const double* h_L0,
                                  const pasta_integrator* h_integ, int64_t step0,
                                  const double* h_L_max, double* d_pos, double* d_vel,
                                  const uint8_t* d_species, void* d_work, size_t work_bytes,
                                  int32_t mode, int32_t steps_per_graph, void* stream,
                                  pasta_batch** out)
{
    if (!pot || !h_n || !h_L0 || !h_integ || !h_L_max || !d_pos || !d_vel || !d_species ||
        !out || nsys <= 0 || nsys > 1024 || step0 < 0 || (mode != 0 && mode != 1) ||
        steps_per_graph < 1 || (precision != PASTA_FP64 && precision != PASTA_MIXED))
        return fail(PASTA_EINVAL, "pasta_batch_create: bad argument");
    *out = nullptr;
    for (int s = 0; s < nsys; ++s) {
        const pasta_integrator& g = h_integ[s];
        if (!(g.dt > 0.0) || !std::isfinite(g.xi_dot) || !(g.T >= 0.0) || g.rescale_every < 0 ||
            !(h_L0[s] > 0.0))
            return fail(PASTA_EINVAL, "pasta_batch_create: system %d: bad integrator or L0", s);
        const double Ls = h_L0[s] * (1.0 + g.xi_dot * ((double)step0 * g.dt));
        if (Ls < 2.0 * pot->r_nuc || Ls > h_L_max[s] * (1.0 + 1e-12))
            return fail(PASTA_EBOX, "pasta_batch_create: system %d: L = %g outside "
                        "[2 r_nuc, L_max]", s, Ls);
    }
    BatchLayout lay;
    PASTA_TRY(batch_layout(pot, precision, nsys, h_n, nullptr, h_L_max, &lay));
    Carver cv0(nullptr);
    const size_t need = batch_carve(cv0, lay, nsys, precision, nullptr);
    if (!d_work || work_bytes < need || (reinterpret_cast<uintptr_t>(d_work) & 255))
        return fail(PASTA_EWORKSPACE, "pasta_batch_create: workspace needs %zu bytes", need);

    pasta_batch* bt = new (std::nothrow) pasta_batch();
    if (!bt)
        return fail(PASTA_ENOMEM, "pasta_batch_create: out of host memory");
    bt->pot = *pot;
    bt->precision = precision;
    bt->mode = mode;
    bt->nsys = nsys;
    bt->n_total = lay.n_total;
    bt->step = step0;
    bt->steps_per_graph = steps_per_graph;
    bt->integ.assign(h_integ, h_integ + nsys);
    bt->user = static_cast<hipStream_t>(stream);
    if (hipStreamCreateWithFlags(&bt->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&bt->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&bt->ev_out, hipEventDisableTiming) != hipSuccess) {
        delete bt;
        return fail(PASTA_EHIP, "pasta_batch_create: stream/event creation failed");
    }
    if (join_in(bt) != PASTA_OK) {
        delete bt;
        return PASTA_EHIP;
    }
    Carver cv(d_work);
    batch_carve(cv, lay, nsys, precision, &bt->dev);
    bt->red = bt->dev.red;
    auto fail_free = [&](int rc) {
        delete bt;
        return rc;
    };
    // Z per system: count protons on the host side of a first pass
    std::vector<int64_t> Z(nsys, 0);
    {
        std::vector<uint8_t> sp(lay.n_total);
        if (hipMemcpyAsync(sp.data(), d_species, lay.n_total, hipMemcpyDeviceToHost,
                           bt->stream) != hipSuccess ||
            hipStreamSynchronize(bt->stream) != hipSuccess)
            return fail_free(fail(PASTA_EHIP, "pasta_batch_create: species copy failed"));
        for (int s = 0; s < nsys; ++s)
            for (int64_t i = lay.sys[s].off; i < lay.sys[s].off + h_n[s]; ++i) {
                if (sp[i] > 1)
                    return fail_free(fail(PASTA_EINVAL, "pasta_batch_create: species not 0/1"));
                Z[s] += sp[i];
            }
    }
    BatchLayout lay2;
    int rc = batch_layout(pot, precision, nsys, h_n, Z.data(), h_L_max, &lay2);
    if (rc != PASTA_OK)
        return fail_free(rc);
    // the Z-dependent layout fits the carve made with Z = n: the partial
    // capacity per system depends on n only
    for (int s = 0; s < nsys; ++s) {
        SysDev& S = lay2.sys[s];
        S.coul_off = lay.sys[s].coul_off;
        const pasta_integrator& g = h_integ[s];
        S.L0 = h_L0[s];
        S.xi_dot = g.xi_dot;
        S.dt = g.dt;
        S.T = g.T;
        S.hdtm = g.dt / (2.0 * pot->mass);
        S.rescale_every = g.rescale_every;
        S.scale_positions = g.scale_positions;
    }
    bt->sys = lay2.sys;
    BatchDev& B = bt->dev;
    B.nsys = nsys;
    B.spin_limit = BARRIER_SPIN_LIMIT;
    B.total_chunks = lay2.total_chunks;
    B.coul_items = lay2.coul_items;
    B.nuc_items = lay2.nuc_items;
    B.pp.a = pot->a;
    B.pp.b_like = pot->b + pot->c;
    B.pp.b_unlike = pot->b - pot->c;
    B.pp.Lambda = pot->Lambda;
    B.pp.r_nuc = pot->r_nuc;
    B.pp.r_coul = INFINITY;
    B.pp.alpha_hbarc = pot->alpha_hbarc;
    B.pp.lambda_s = pot->lambda_s;
    B.pp.L = 0.0;
    B.mass = pot->mass;
    B.nuc_variant = batch_variant();
    B.chunk = batch_chunk();
    B.cpos = d_pos;
    B.cvel = d_vel;
    B.species = d_species;
    hipStream_t s = bt->stream;
    if (hipMemcpyAsync((void*)B.sys, bt->sys.data(), sizeof(SysDev) * nsys,
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return fail_free(fail(PASTA_EHIP, "pasta_batch_create: descriptor copy failed"));
    k_batch_init_scalars<<<1, 1024, 0, s>>>(B, step0);
    k_batch_zero<<<256, BW, 0, s>>>(B.count, B.fill, lay.bins);
    k_batch_zero<<<256, BW, 0, s>>>(reinterpret_cast<int32_t*>(B.react),
                                    reinterpret_cast<int32_t*>(B.react) + 4 * lay.n_total,
                                    4 * lay.n_total);
    k_batch_load<<<256, BW, 0, s>>>(B, lay.n_total);
    rc = precision == PASTA_FP64 ? persistent_grid<Fp64Policy>(B.nuc_variant, &bt->grid)
                                 : persistent_grid<MixedPolicy>(B.nuc_variant, &bt->grid);
    if (rc != PASTA_OK)
        return fail_free(rc);
    bt->phase_grid = bt->grid * 2;
    // initial forces at the starting state (mode 0: no drift, no kick)
    rc = launch_one(bt, 0);
    if (rc == PASTA_OK)
        rc = check_batch_err(bt, "pasta_batch_create");
    if (rc != PASTA_OK)
        return fail_free(rc);
    bt->epot_valid = true;
    rc = join_out(bt);
    if (rc != PASTA_OK)
        return fail_free(rc);
    *out = bt;
    return PASTA_OK;
}

static int batch_capture(pasta_batch* bt)
{
    if (bt->exec)
        return PASTA_OK;
    hipStream_t s = bt->stream;
    PASTA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = PASTA_OK;
    for (int k = 0; k < bt->steps_per_graph && rc == PASTA_OK; ++k)
        rc = launch_one(bt, 1, k == 0, k == bt->steps_per_graph - 1);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc != PASTA_OK)
        return rc;
    if (e != hipSuccess)
        return fail(PASTA_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    bt->graph = g;
    PASTA_HIP(hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0));
    return PASTA_OK;
}

extern "C" int pasta_batch_step(pasta_batch* bt, int64_t nsteps)
{
    if (!bt || nsteps < 0)
        return fail(PASTA_EINVAL, "pasta_batch_step: bad argument");
    for (int s = 0; s < bt->nsys; ++s) {
        const pasta_integrator& g = bt->integ[s];
        const double L = bt->sys[s].L0 * (1.0 + g.xi_dot * ((double)(bt->step + nsteps) * g.dt));
        const Grid gr = make_grid(L, bt->pot.r_nuc);
        const double Lm = bt->sys[s].L0 * (1.0 + g.xi_dot * ((double)bt->step * g.dt));
        const Grid g0 = make_grid(Lm, bt->pot.r_nuc);
        const int64_t cap = (int64_t)bt->sys[s].item_max - bt->sys[s].n / bt->dev.chunk - 1;
        if (L < 2.0 * bt->pot.r_nuc || gr.C > cap || g0.C > cap)
            return fail(PASTA_EBOX, "pasta_batch_step: system %d leaves [2 r_nuc, L_max]", s);
    }
    hipStream_t st = bt->stream;
    PASTA_TRY(join_in(bt));
    PASTA_TRY(batch_capture(bt));
    int64_t left = nsteps;
    while (left >= bt->steps_per_graph) {
        PASTA_HIP(hipGraphLaunch(bt->exec, st));
        left -= bt->steps_per_graph;
    }
    for (int64_t k = 0; k < left; ++k)
        PASTA_TRY(launch_one(bt, 1, k == 0, k == left - 1));
    k_apply_pending<<<bt->grid, BW, 0, st>>>(bt->dev);
    k_reset_pending<<<1, 1024, 0, st>>>(bt->dev);
    if (nsteps > 0) {  // the state into the caller's arrays
        k_batch_unsort<<<chunk_grid(bt), BW, 0, st>>>(bt->dev, bt->dev.pos, bt->dev.cpos, 3);
        k_batch_unsort<<<chunk_grid(bt), BW, 0, st>>>(bt->dev, bt->dev.vel, bt->dev.cvel, 3);
    }
    PASTA_HIP(hipGetLastError());
    bt->step += nsteps;
    if (nsteps > 0)
        bt->epot_valid = false;
    PASTA_TRY(join_out(bt));
    // a failed device check (a barrier wait that timed out stops every later
    // step on the device) is reported here and by every later call
    return check_batch_err(bt, "pasta_batch_step");
}

extern "C" int pasta_batch_set_wait_limit(pasta_batch* bt, int64_t polls)
{
    if (!bt || polls < 0)
        return fail(PASTA_EINVAL, "pasta_batch_set_wait_limit: bad argument");
    PASTA_HIP(hipStreamSynchronize(bt->stream));
    bt->dev.spin_limit = (long)polls;
    // the captured steps carry the old limit as a kernel argument
    if (bt->exec) {
        PASTA_HIP(hipGraphExecDestroy(bt->exec));
        bt->exec = nullptr;
    }
    if (bt->graph) {
        PASTA_HIP(hipGraphDestroy(bt->graph));
        bt->graph = nullptr;
    }
    return PASTA_OK;
}

// Energy shares of the current state, evaluated when asked for (the steps
// skip them): the pair phase with energies and the combine without a kick,
// on the cell lists and staging already in place; the forces are rewritten
// with the same bits.
static int batch_refresh_energies(pasta_batch* bt)
{
    if (bt->epot_valid)
        return PASTA_OK;
    hipStream_t s = bt->stream;
    k_batch_zero_pairs<<<1, 1024, 0, s>>>(bt->dev);
    const unsigned gc = chunk_grid(bt);
    launch_pair_phase<MODE_ENERGY>(bt->dev, bt->precision, s);
    if (bt->precision == PASTA_FP64)
        k_ph_combine<Fp64Policy><<<gc, BW, 0, s>>>(bt->dev, 0, 1, 0, 0, 0);
    else
        k_ph_combine<MixedPolicy><<<gc, BW, 0, s>>>(bt->dev, 0, 1, 0, 0, 0);
    PASTA_HIP(hipGetLastError());
    bt->epot_valid = true;
    return PASTA_OK;
}

extern "C" int pasta_batch_energies(pasta_batch* bt, double* h_ekin, double* h_epot, double* h_L,
                                    int64_t* h_step)
{
    if (!bt)
        return fail(PASTA_EINVAL, "pasta_batch_energies: null batch");
    PASTA_TRY(join_in(bt));
    if (h_epot)
        PASTA_TRY(batch_refresh_energies(bt));
    PASTA_TRY(check_batch_err(bt, "pasta_batch"));
    hipStream_t s = bt->stream;
    std::vector<double> h(256);
    for (int k = 0; k < bt->nsys; ++k) {
        const SysDev& S = bt->sys[k];
        for (int kind = 1; kind >= 0; --kind) {
            double* dst = kind ? h_ekin : h_epot;
            if (!dst)
                continue;
            const double* src = kind ? bt->dev.vel + 3 * S.off : bt->dev.epot + S.off;
            k_batch_partial<<<256, BW, 0, s>>>(src, S.n, kind, bt->pot.mass, bt->red);
            PASTA_HIP(hipMemcpyAsync(h.data(), bt->red, 256 * sizeof(double),
                                     hipMemcpyDeviceToHost, s));
            PASTA_HIP(hipStreamSynchronize(s));
            double acc = 0.0;
            for (double v : h)
                acc += v;
            dst[k] = acc;
        }
        if (h_L) {
            const pasta_integrator& g = bt->integ[k];
            h_L[k] = S.L0 * (1.0 + g.xi_dot * ((double)bt->step * g.dt));
        }
    }
    if (h_step)
        *h_step = bt->step;
    return PASTA_OK;
}

extern "C" int pasta_batch_forces(pasta_batch* bt, double* d_force, double* d_epot)
{
    if (!bt)
        return fail(PASTA_EINVAL, "pasta_batch_forces: null batch");
    PASTA_TRY(join_in(bt));
    if (d_epot)
        PASTA_TRY(batch_refresh_energies(bt));
    // slot order to caller order
    if (d_force)
        k_batch_unsort<<<chunk_grid(bt), BW, 0, bt->stream>>>(bt->dev, bt->dev.force, d_force, 3);
    if (d_epot)
        k_batch_unsort<<<chunk_grid(bt), BW, 0, bt->stream>>>(bt->dev, bt->dev.epot, d_epot, 1);
    PASTA_HIP(hipGetLastError());
    PASTA_TRY(join_out(bt));
    return check_batch_err(bt, "pasta_batch_forces");
}

extern "C" int pasta_batch_pair_counts(pasta_batch* bt, int64_t* h_nuclear, int64_t* h_coulomb)
{
    if (!bt || !h_nuclear || !h_coulomb)
        return fail(PASTA_EINVAL, "pasta_batch_pair_counts: bad argument");
    hipStream_t s = bt->stream;
    PASTA_TRY(join_in(bt));
    k_batch_zero_pairs<<<1, 1024, 0, s>>>(bt->dev);
    // the cell lists and staging of the current state are in place; the
    // count pass rewrites F (same values) without a kick
    launch_pair_phase<MODE_COUNT>(bt->dev, bt->precision, s);
    // no combine follows: clear the fixed-point Coulomb sums the count pass
    // added, so the next combine reads only its own force phase's
    k_batch_zero<<<256, BW, 0, s>>>(reinterpret_cast<int32_t*>(bt->dev.react),
                                    reinterpret_cast<int32_t*>(bt->dev.react) +
                                        4 * bt->dev.n_total,
                                    4 * bt->dev.n_total);
    PASTA_HIP(hipGetLastError());
    std::vector<unsigned long long> h(bt->nsys);
    PASTA_HIP(hipMemcpyAsync(h.data(), bt->dev.pairs, sizeof(unsigned long long) * bt->nsys,
                             hipMemcpyDeviceToHost, s));
    PASTA_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < bt->nsys; ++k) {
        h_nuclear[k] = (int64_t)(h[k] / 2);
        const int64_t Z = bt->sys[k].Z;
        h_coulomb[k] = Z * (Z - 1) / 2;
    }
    return check_batch_err(bt, "pasta_batch_pair_counts");
}

extern "C" int pasta_batch_info(pasta_batch* bt, int32_t* h_grid, int32_t* h_mode)
{
    if (!bt)
        return fail(PASTA_EINVAL, "pasta_batch_info: null batch");
    if (h_grid)
        *h_grid = (int32_t)(bt->mode == 0 ? bt->grid : bt->phase_grid);
    if (h_mode)
        *h_mode = bt->mode;
    return PASTA_OK;
}

extern "C" void pasta_batch_destroy(pasta_batch* bt)
{
    if (!bt)
        return;
    delete bt;
}
