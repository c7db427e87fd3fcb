// Cell-list build: a stable counting sort of particles into cubic cells no
// narrower than the interaction range (the binning of Sec. II.B.2), rebuilt
// from scratch every step (cell sweeps) or whenever the neighbour lists are
// rebuilt (the kernels then take a device gate word).  Memory-bound; four
// launches:
//   bin/count   one thread per particle: bin = (proton ? 0 : C) + cell,
//               integer atomic count per bin (order-independent);
//   scan        exclusive scan of the 2C counts, the nuclear work list (cell,
//               target chunk), and the reset of the counters: one workgroup
//               for grids of up to 2048 cells (one or two rows of 1024; a
//               third row would spill registers), else two launches of one
//               thread per cell;
//   scatter     one thread per particle: slot = start[bin] + atomic cursor
//               (arrival order, not yet stable);
//   rank        one thread per slot: the stable rank inside the bin is the
//               number of bin members with a smaller particle index, so the
//               final order is (bin, particle index) whatever order the
//               atomics took; the same thread gathers the particle's staging
//               coordinates and, for a simulation, moves its state.
// The source index is the particle's position in the arrays the build reads:
// the caller's order for a standalone build (source index = particle index),
// the previous sorted order for a simulation step (whose state is kept in
// sorted order, with the particle index of every slot beside it).
#include "internal.hpp"

namespace pasta {

namespace {

__global__ __launch_bounds__(256) void k_bin_count(const double* __restrict__ pos,
                                                   const uint8_t* __restrict__ species,
                                                   int64_t n, int nc, int C, int sub,
                                                   double inv_w, double L,
                                                   int32_t* __restrict__ key,
                                                   int32_t* __restrict__ count,
                                                   uint32_t* __restrict__ err,
                                                   const int32_t* __restrict__ gate)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (gate && *gate == 0))
        return;
    double x = pos[3 * i + 0], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const uint8_t sp = species[i];
    if (!(x >= 0.0 && x < L && y >= 0.0 && y < L && z >= 0.0 && z < L))
        atomicOr(err, (isfinite(x) && isfinite(y) && isfinite(z)) ? ERR_RANGE : ERR_NONFINITE_POS);
    if (sp > 1)
        atomicOr(err, ERR_SPECIES);
    const int bin = particle_bin(x, y, z, sp == 1, inv_w, nc, C, sub);
    key[i] = bin;
    wave_aggregated_add(count, bin);
}

constexpr int SCAN_THREADS = 1024;
static_assert(SCAN_THREADS <= 64 * 63, "wave totals must fit the LDS scratch");

// Exclusive scan of v[0..m) (per-thread contiguous runs + the workgroup scan
// of the run totals).  Returns the grand total to every thread.
// Runs of up to RUN_CACHE values are held in registers (loaded with
// independent loads), longer runs are re-read.
constexpr int RUN_CACHE = 8;
__device__ int64_t block_scan_runs(const int32_t* v, int32_t* out, int64_t m,
                                   int64_t* lds)
{
    const int tid = threadIdx.x;
    const int64_t per = (m + SCAN_THREADS - 1) / SCAN_THREADS;
    const int64_t b = tid * per, e = b + per < m ? b + per : m;
    int32_t c[RUN_CACHE];
    int64_t s = 0;
#pragma unroll
    for (int u = 0; u < RUN_CACHE; ++u) {
        c[u] = b + u < e ? v[b + u] : 0;
        s += c[u];
    }
    for (int64_t k = b + RUN_CACHE; k < e; ++k)
        s += v[k];
    int64_t total = 0;
    int64_t run = block_exclusive_scan(s, lds, &total);
#pragma unroll
    for (int u = 0; u < RUN_CACHE; ++u) {
        if (b + u < e)
            out[b + u] = (int32_t)run;
        run += c[u];
    }
    for (int64_t k = b + RUN_CACHE; k < e; ++k) {
        const int32_t x = v[k];
        out[k] = (int32_t)run;
        run += x;
    }
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan(int32_t* __restrict__ count,
                                                       int32_t* __restrict__ fill,
                                                       int32_t* __restrict__ start, int C,
                                                       int sub, int chunk,
                                                       int32_t* __restrict__ items,
                                                       int32_t* __restrict__ n_items,
                                                       int32_t* __restrict__ tmpc,
                                                       const int32_t* __restrict__ gate)
{
    __shared__ int64_t lds[SCAN_THREADS];
    if (gate && *gate == 0)
        return;
    const int tid = threadIdx.x;
    const int64_t nb = 2 * (int64_t)C * sub;
    int64_t total = block_scan_runs(count, start, nb, lds);
    if (tid == 0)
        start[nb] = (int32_t)total;
    __syncthreads();
    if (chunk > 0) {
        // chunks per cell (protons + neutrons of the cell)
        // members of cell c from the starts just written (four loads)
        const int64_t CS = (int64_t)C * sub;
        for (int64_t c = tid; c < C; c += SCAN_THREADS) {
            const int32_t m = (start[(c + 1) * sub] - start[c * sub]) +
                              (start[CS + (c + 1) * sub] - start[CS + c * sub]);
            tmpc[c] = (m + chunk - 1) / chunk;
        }
        __syncthreads();
        int64_t nit = block_scan_runs(tmpc, tmpc + C, C, lds);
        for (int64_t c = tid; c < C; c += SCAN_THREADS) {
            int32_t base = tmpc[C + c], k = tmpc[c];
            for (int32_t q = 0; q < k; ++q) {
                items[2 * (base + q) + 0] = (int32_t)c;
                items[2 * (base + q) + 1] = q;
            }
        }
        if (tid == 0)
            *n_items = (int32_t)nit;
        __syncthreads();
    }
    for (int64_t k = tid; k < nb; k += SCAN_THREADS) {
        count[k] = 0;
        fill[k] = 0;
    }
}

// The same for octant bins (sub = 8) and at most SCAN_THREADS cells, the
// simulation's case: thread c owns cell c, holds its 8 proton and 8 neutron
// counts in registers (four 16-byte loads, all in flight at once) and the
// workgroup scans their sums (proton and neutron totals packed in one 64-bit
// word: both are at most n < 2^31, so the low half never carries) and the
// cell's item count, so nothing is read back that the kernel wrote.  The
// buffers are 256-byte aligned and 8 c ints sit at a 32-byte boundary.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_oct(int32_t* __restrict__ count,
                                                           int32_t* __restrict__ fill,
                                                           int32_t* __restrict__ start, int C,
                                                           int chunk,
                                                           int32_t* __restrict__ items,
                                                           int32_t* __restrict__ n_items,
                                                           const int32_t* __restrict__ gate)
{
    __shared__ int64_t lds[64];
    if (gate && *gate == 0)
        return;
    const int c = threadIdx.x;
    const int64_t CS = (int64_t)C * 8;
    int4 p0{0, 0, 0, 0}, p1{0, 0, 0, 0}, n0{0, 0, 0, 0}, n1{0, 0, 0, 0};
    if (c < C) {
        const int4* cp = reinterpret_cast<const int4*>(count + 8 * (int64_t)c);
        const int4* cn = reinterpret_cast<const int4*>(count + CS + 8 * (int64_t)c);
        p0 = cp[0];
        p1 = cp[1];
        n0 = cn[0];
        n1 = cn[1];
    }
    const int64_t sp = (int64_t)p0.x + p0.y + p0.z + p0.w + p1.x + p1.y + p1.z + p1.w;
    const int64_t sn = (int64_t)n0.x + n0.y + n0.z + n0.w + n1.x + n1.y + n1.z + n1.w;
    const int64_t k = chunk > 0 ? (sp + sn + chunk - 1) / chunk : 0;
    int64_t tot = 0, tq = 0;
    const int64_t pre = block_exclusive_scan(sp | (sn << 32), lds, &tot);
    const int64_t bq = chunk > 0 ? block_exclusive_scan(k, lds, &tq) : 0;
    const int64_t Zt = tot & 0xffffffffll;  // all protons
    if (c < C) {
        int32_t b = (int32_t)(pre & 0xffffffffll);
        int4 s0, s1;
        s0.x = b; b += p0.x; s0.y = b; b += p0.y; s0.z = b; b += p0.z; s0.w = b; b += p0.w;
        s1.x = b; b += p1.x; s1.y = b; b += p1.y; s1.z = b; b += p1.z; s1.w = b;
        int4* sp4 = reinterpret_cast<int4*>(start + 8 * (int64_t)c);
        sp4[0] = s0;
        sp4[1] = s1;
        b = (int32_t)(Zt + (pre >> 32));
        s0.x = b; b += n0.x; s0.y = b; b += n0.y; s0.z = b; b += n0.z; s0.w = b; b += n0.w;
        s1.x = b; b += n1.x; s1.y = b; b += n1.y; s1.z = b; b += n1.z; s1.w = b;
        int4* sn4 = reinterpret_cast<int4*>(start + CS + 8 * (int64_t)c);
        sn4[0] = s0;
        sn4[1] = s1;
        for (int64_t q = 0; q < k; ++q) {
            items[2 * (bq + q) + 0] = c;
            items[2 * (bq + q) + 1] = (int32_t)q;
        }
        // this thread alone read these counters
        const int4 z{0, 0, 0, 0};
        int4* zc = reinterpret_cast<int4*>(count + 8 * (int64_t)c);
        int4* zn = reinterpret_cast<int4*>(count + CS + 8 * (int64_t)c);
        int4* fc = reinterpret_cast<int4*>(fill + 8 * (int64_t)c);
        int4* fn = reinterpret_cast<int4*>(fill + CS + 8 * (int64_t)c);
        zc[0] = z; zc[1] = z; zn[0] = z; zn[1] = z;
        fc[0] = z; fc[1] = z; fn[0] = z; fn[1] = z;
    }
    if (c == 0) {
        start[2 * CS] = (int32_t)(Zt + (tot >> 32));
        if (chunk > 0)
            *n_items = (int32_t)tq;
    }
}

// The same for grids of up to ROWS * SCAN_THREADS cells in one workgroup:
// cell r * SCAN_THREADS + t belongs to thread t (row r), so every load and
// store of a row is coalesced.  Each row is scanned on its own and offset by
// the totals of the rows before it; the neutron starts need the proton total
// of every row, so all rows are scanned before any start is written.
template <int ROWS>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_oct_rows(
    int32_t* __restrict__ count, int32_t* __restrict__ fill, int32_t* __restrict__ start, int C,
    int chunk, int32_t* __restrict__ items, int32_t* __restrict__ n_items,
    const int32_t* __restrict__ gate)
{
    __shared__ int64_t lds[64];
    if (gate && *gate == 0)
        return;
    const int64_t CS = (int64_t)C * 8;
    int4 p0[ROWS], p1[ROWS], n0[ROWS], n1[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int c = r * SCAN_THREADS + (int)threadIdx.x;
        p0[r] = p1[r] = n0[r] = n1[r] = int4{0, 0, 0, 0};
        if (c < C) {
            const int4* cp = reinterpret_cast<const int4*>(count + 8 * (int64_t)c);
            const int4* cn = reinterpret_cast<const int4*>(count + CS + 8 * (int64_t)c);
            p0[r] = cp[0];
            p1[r] = cp[1];
            n0[r] = cn[0];
            n1[r] = cn[1];
        }
    }
    int64_t pre[ROWS], bq[ROWS], kq[ROWS];
    int64_t run = 0, runq = 0;  // totals of the rows before (uniform)
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int64_t sp = (int64_t)p0[r].x + p0[r].y + p0[r].z + p0[r].w + p1[r].x + p1[r].y +
                           p1[r].z + p1[r].w;
        const int64_t sn = (int64_t)n0[r].x + n0[r].y + n0[r].z + n0[r].w + n1[r].x + n1[r].y +
                           n1[r].z + n1[r].w;
        kq[r] = chunk > 0 ? (sp + sn + chunk - 1) / chunk : 0;
        int64_t tot = 0, tq = 0;
        pre[r] = run + block_exclusive_scan(sp | (sn << 32), lds, &tot);
        bq[r] = chunk > 0 ? runq + block_exclusive_scan(kq[r], lds, &tq) : 0;
        run += tot;
        runq += tq;
    }
    const int64_t Zt = run & 0xffffffffll;  // all protons
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int c = r * SCAN_THREADS + (int)threadIdx.x;
        if (c >= C)
            continue;
        int32_t b = (int32_t)(pre[r] & 0xffffffffll);
        int4 s0, s1;
        s0.x = b; b += p0[r].x; s0.y = b; b += p0[r].y; s0.z = b; b += p0[r].z; s0.w = b;
        b += p0[r].w;
        s1.x = b; b += p1[r].x; s1.y = b; b += p1[r].y; s1.z = b; b += p1[r].z; s1.w = b;
        int4* sp4 = reinterpret_cast<int4*>(start + 8 * (int64_t)c);
        sp4[0] = s0;
        sp4[1] = s1;
        b = (int32_t)(Zt + (pre[r] >> 32));
        s0.x = b; b += n0[r].x; s0.y = b; b += n0[r].y; s0.z = b; b += n0[r].z; s0.w = b;
        b += n0[r].w;
        s1.x = b; b += n1[r].x; s1.y = b; b += n1[r].y; s1.z = b; b += n1[r].z; s1.w = b;
        int4* sn4 = reinterpret_cast<int4*>(start + CS + 8 * (int64_t)c);
        sn4[0] = s0;
        sn4[1] = s1;
        for (int64_t q = 0; q < kq[r]; ++q) {
            items[2 * (bq[r] + q) + 0] = c;
            items[2 * (bq[r] + q) + 1] = (int32_t)q;
        }
        // this thread alone read these counters
        const int4 z{0, 0, 0, 0};
        int4* zc = reinterpret_cast<int4*>(count + 8 * (int64_t)c);
        int4* zn = reinterpret_cast<int4*>(count + CS + 8 * (int64_t)c);
        int4* fc = reinterpret_cast<int4*>(fill + 8 * (int64_t)c);
        int4* fn = reinterpret_cast<int4*>(fill + CS + 8 * (int64_t)c);
        zc[0] = z; zc[1] = z; zn[0] = z; zn[1] = z;
        fc[0] = z; fc[1] = z; fn[0] = z; fn[1] = z;
    }
    if (threadIdx.x == 0) {
        start[2 * CS] = (int32_t)(Zt + (run >> 32));
        if (chunk > 0)
            *n_items = (int32_t)runq;
    }
}

// Grids of more than SCAN_THREADS cells (large systems, a decompressed box,
// the cluster grid): the same scan over all cells in two launches of one
// thread per cell.  k_mscan_sums: each workgroup's totals (protons and
// neutrons packed in one 64-bit word, and work items) into blk; then
// k_mscan_apply: every workgroup takes the exclusive prefix of the totals
// of the workgroups before it (at most MSCAN_MAX_BLOCKS of them), scans its
// own cells as k_scan_oct does, writes the starts and items and clears the
// counters.  SUB = bins per cell and species (1 or 8).
constexpr int MSCAN_THREADS = 1024;
constexpr int MSCAN_MAX_BLOCKS = MSCAN_THREADS;

template <int SUB>
__device__ inline void load_cell_counts(const int32_t* __restrict__ count, int64_t CS, int64_t c,
                                        int32_t (&p)[SUB], int32_t (&q)[SUB])
{
    if constexpr (SUB == 8) {
        const int4* cp = reinterpret_cast<const int4*>(count + 8 * c);
        const int4* cn = reinterpret_cast<const int4*>(count + CS + 8 * c);
        const int4 a = cp[0], b = cp[1], d = cn[0], e = cn[1];
        p[0] = a.x; p[1] = a.y; p[2] = a.z; p[3] = a.w;
        p[4] = b.x; p[5] = b.y; p[6] = b.z; p[7] = b.w;
        q[0] = d.x; q[1] = d.y; q[2] = d.z; q[3] = d.w;
        q[4] = e.x; q[5] = e.y; q[6] = e.z; q[7] = e.w;
    } else {
#pragma unroll
        for (int u = 0; u < SUB; ++u) {
            p[u] = count[SUB * c + u];
            q[u] = count[CS + SUB * c + u];
        }
    }
}

template <int SUB>
__global__ __launch_bounds__(MSCAN_THREADS) void k_mscan_sums(const int32_t* __restrict__ count,
                                                              int C, int chunk,
                                                              int64_t* __restrict__ blk,
                                                              const int32_t* __restrict__ gate)
{
    __shared__ int64_t lds[64];
    if (gate && *gate == 0)
        return;
    const int64_t c = (int64_t)blockIdx.x * MSCAN_THREADS + threadIdx.x;
    const int64_t CS = (int64_t)C * SUB;
    int64_t sp = 0, sn = 0;
    if (c < C) {
        int32_t p[SUB], q[SUB];
        load_cell_counts<SUB>(count, CS, c, p, q);
#pragma unroll
        for (int u = 0; u < SUB; ++u) {
            sp += p[u];
            sn += q[u];
        }
    }
    const int64_t k = chunk > 0 ? (sp + sn + chunk - 1) / chunk : 0;
    int64_t tot = 0, tq = 0;
    block_exclusive_scan(sp | (sn << 32), lds, &tot);
    block_exclusive_scan(k, lds, &tq);
    if (threadIdx.x == 0) {
        blk[2 * blockIdx.x + 0] = tot;
        blk[2 * blockIdx.x + 1] = tq;
    }
}

template <int SUB>
__global__ __launch_bounds__(MSCAN_THREADS) void k_mscan_apply(
    int32_t* __restrict__ count, int32_t* __restrict__ fill, int32_t* __restrict__ start, int C,
    int chunk, int32_t* __restrict__ items, int32_t* __restrict__ n_items,
    const int64_t* __restrict__ blk, int nblk, const int32_t* __restrict__ gate)
{
    __shared__ int64_t lds[64];
    __shared__ int64_t s_off[2];
    if (gate && *gate == 0)
        return;
    const int t = threadIdx.x;
    // exclusive prefix of the workgroup totals, and the grand totals
    const int64_t bt = t < nblk ? blk[2 * t + 0] : 0, bq = t < nblk ? blk[2 * t + 1] : 0;
    int64_t all_t = 0, all_q = 0;
    const int64_t pt = block_exclusive_scan(bt, lds, &all_t);
    const int64_t pq = block_exclusive_scan(bq, lds, &all_q);
    if (t == (int)blockIdx.x) {
        s_off[0] = pt;
        s_off[1] = pq;
    }
    __syncthreads();
    const int64_t off_t = s_off[0], off_q = s_off[1];
    const int64_t Zt = all_t & 0xffffffffll;  // all protons
    const int64_t c = (int64_t)blockIdx.x * MSCAN_THREADS + t;
    const int64_t CS = (int64_t)C * SUB;
    int32_t p[SUB], q[SUB];
    int64_t sp = 0, sn = 0;
    if (c < C) {
        load_cell_counts<SUB>(count, CS, c, p, q);
#pragma unroll
        for (int u = 0; u < SUB; ++u) {
            sp += p[u];
            sn += q[u];
        }
    }
    const int64_t k = chunk > 0 ? (sp + sn + chunk - 1) / chunk : 0;
    int64_t tot = 0, tq = 0;
    const int64_t pre = off_t + block_exclusive_scan(sp | (sn << 32), lds, &tot);
    const int64_t bqi = off_q + block_exclusive_scan(k, lds, &tq);
    if (c < C) {
        int32_t b = (int32_t)(pre & 0xffffffffll);
#pragma unroll
        for (int u = 0; u < SUB; ++u) {
            start[SUB * c + u] = b;
            b += p[u];
        }
        b = (int32_t)(Zt + (pre >> 32));
#pragma unroll
        for (int u = 0; u < SUB; ++u) {
            start[CS + SUB * c + u] = b;
            b += q[u];
        }
        for (int64_t r = 0; r < k; ++r) {
            items[2 * (bqi + r) + 0] = (int32_t)c;
            items[2 * (bqi + r) + 1] = (int32_t)r;
        }
        // this thread alone read these counters (in both launches)
#pragma unroll
        for (int u = 0; u < SUB; ++u) {
            count[SUB * c + u] = 0;
            count[CS + SUB * c + u] = 0;
            fill[SUB * c + u] = 0;
            fill[CS + SUB * c + u] = 0;
        }
    }
    if (blockIdx.x == 0 && t == 0) {
        start[2 * CS] = (int32_t)(Zt + (all_t >> 32));
        if (chunk > 0)
            *n_items = (int32_t)all_q;
    }
}

// order: the previous sorted order (perm of the last build) or null for the
// caller's order.  Visiting particles in the previous cell order keeps the
// lanes of a wave in one or two bins, so the cursor atomics aggregate.
// ids (optional): particle index of each source; then tmp receives the
// particle index and src the source index of each unsorted slot.
__global__ __launch_bounds__(256) void k_scatter(const int32_t* __restrict__ key, int64_t n,
                                                 const int32_t* __restrict__ order,
                                                 const int32_t* __restrict__ start,
                                                 int32_t* __restrict__ fill,
                                                 int32_t* __restrict__ tmp,
                                                 const int32_t* __restrict__ gate,
                                                 const int32_t* __restrict__ ids,
                                                 int32_t* __restrict__ src)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n || (gate && *gate == 0))
        return;
    const int32_t i = order ? order[s] : (int32_t)s;
    const int b = key[i];
    const int slot = start[b] + wave_aggregated_add(fill, b);
    if (ids) {
        tmp[slot] = ids[i];
        src[slot] = i;
    } else {
        tmp[slot] = i;
    }
}

__global__ __launch_bounds__(256) void k_rank(const int32_t* __restrict__ key,
                                              const int32_t* __restrict__ tmp, int64_t n,
                                              const int32_t* __restrict__ start,
                                              int32_t* __restrict__ perm,
                                              const double* __restrict__ pos,
                                              const uint8_t* __restrict__ species,
                                              double4* __restrict__ stg64,
                                              Q4* __restrict__ stgq, double qscale,
                                              const int32_t* __restrict__ gate,
                                              double* __restrict__ xb,
                                              const int32_t* __restrict__ srcix, StateMove mv)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n || (gate && *gate == 0))
        return;
    const int32_t id = tmp[s];                  // particle index: the rank key
    const int32_t src = srcix ? srcix[s] : id;  // where its data is
    const int b = key[src];
    const int beg = start[b], end = start[b + 1];
    // rank = members of the bin with a smaller index; eight independent
    // loads per iteration keep the loop from being latency-bound
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
    const int dst = beg + r;
    perm[dst] = src;
    double x = pos[3 * (int64_t)src + 0], y = pos[3 * (int64_t)src + 1],
           z = pos[3 * (int64_t)src + 2];
    if (xb) {
        xb[3 * (int64_t)dst + 0] = x;
        xb[3 * (int64_t)dst + 1] = y;
        xb[3 * (int64_t)dst + 2] = z;
    }
    const uint8_t sp = species[src];
    if (stg64)
        stg64[dst] = make_double4(x, y, z, (double)sp);
    if (stgq) {
        Q4 q;
        q.x = (uint32_t)(uint64_t)(x * qscale);
        q.y = (uint32_t)(uint64_t)(y * qscale);
        q.z = (uint32_t)(uint64_t)(z * qscale);
        q.w = sp;
        stgq[dst] = q;
    }
    if (mv.pos_dst) {
        const double* v = mv.vel_src + 3 * (int64_t)src;
        const double vx = v[0], vy = v[1], vz = v[2];
        mv.pos_dst[3 * (int64_t)dst + 0] = x;
        mv.pos_dst[3 * (int64_t)dst + 1] = y;
        mv.pos_dst[3 * (int64_t)dst + 2] = z;
        mv.vel_dst[3 * (int64_t)dst + 0] = vx;
        mv.vel_dst[3 * (int64_t)dst + 1] = vy;
        mv.vel_dst[3 * (int64_t)dst + 2] = vz;
        mv.id_dst[dst] = id;
        mv.sp_dst[dst] = sp;
    }
}

__global__ __launch_bounds__(256) void k_state_copy(StateMove m, double* __restrict__ pos,
                                                    double* __restrict__ vel,
                                                    int32_t* __restrict__ id,
                                                    uint8_t* __restrict__ sp, int64_t n,
                                                    const int32_t* __restrict__ gate)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || (gate && *gate == 0))
        return;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        pos[3 * k + d] = m.pos_dst[3 * k + d];
        vel[3 * k + d] = m.vel_dst[3 * k + d];
    }
    id[k] = m.id_dst[k];
    sp[k] = m.sp_dst[k];
}

__global__ __launch_bounds__(256) void k_export(const int32_t* __restrict__ id, int64_t n,
                                                const double* __restrict__ src3a,
                                                double* __restrict__ dst3a,
                                                const double* __restrict__ src3b,
                                                double* __restrict__ dst3b,
                                                const double* __restrict__ src1,
                                                double* __restrict__ dst1)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    const int64_t i = id[k];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (dst3a)
            dst3a[3 * i + d] = src3a[3 * k + d];
        if (dst3b)
            dst3b[3 * i + d] = src3b[3 * k + d];
    }
    if (dst1)
        dst1[i] = src1[k];
}

__global__ void k_zero_words(uint32_t* a, int64_t m)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m)
        a[k] = 0u;
}

__global__ void k_zero2(int32_t* a, int32_t* b, int64_t m)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) {
        a[k] = 0;
        b[k] = 0;
    }
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

size_t cellbuf_carve(Carver& cv, CellBuf* out, int64_t n, int C_max, int chunk, int sub)
{
    CellBuf cb;
    const int64_t nb = 2 * (int64_t)C_max * sub;
    cb.key = cv.take<int32_t>(n);
    cb.count = cv.take<int32_t>((size_t)nb);
    cb.fill = cv.take<int32_t>((size_t)nb);
    cb.start = cv.take<int32_t>((size_t)nb + 1);
    cb.tmp = cv.take<int32_t>(n > nb ? n : nb);
    cb.perm = cv.take<int32_t>(n);
    cb.src = cv.take<int32_t>(n);
    cb.item_max = chunk > 0 ? n / chunk + C_max + 1 : 1;
    cb.items = cv.take<int32_t>(2 * (size_t)cb.item_max);
    cb.n_items = cv.take<int32_t>(1);
    if (out)
        *out = cb;
    return cv.size();
}

void launch_zero_words(void* p, int64_t nwords, hipStream_t s)
{
    if (nwords > 0)
        k_zero_words<<<blocks_for(nwords, 256), 256, 0, s>>>(static_cast<uint32_t*>(p), nwords);
}

void cellbuf_zero(const CellBuf& cb, int C_max, hipStream_t s, int sub)
{
    int64_t m = 2 * (int64_t)C_max * sub;
    k_zero2<<<blocks_for(m, 256), 256, 0, s>>>(cb.count, cb.fill, m);
}

void launch_bin_count(const double* pos, const uint8_t* species, int64_t n, const Grid& g,
                      const CellBuf& cb, uint32_t* err, hipStream_t s, Timer* t,
                      const int32_t* gate)
{
    timer_begin(t, KC_DRIFT, s);
    if (n > 0)
        k_bin_count<<<blocks_for(n, 256), 256, 0, s>>>(pos, species, n, g.nc, g.C, g.sub,
                                                       g.inv_w, g.L, cb.key, cb.count, err,
                                                       gate);
    timer_end(t, KC_DRIFT, s);
}

void launch_scan(const CellBuf& cb, const Grid& g, int chunk, hipStream_t s, Timer* t,
                 const int32_t* gate)
{
    timer_begin(t, KC_SCAN, s);
    // cb.tmp doubles as scratch: the per-cell chunk counts of k_scan (2C
    // entries), the workgroup totals of k_mscan_* (4 per workgroup); the
    // scatter only writes it after the scan
    const int64_t nblk = ((int64_t)g.C + MSCAN_THREADS - 1) / MSCAN_THREADS;
    if (g.sub == 8 && g.C <= SCAN_THREADS) {
        k_scan_oct<<<1, SCAN_THREADS, 0, s>>>(cb.count, cb.fill, cb.start, g.C, chunk, cb.items,
                                              cb.n_items, gate);
    } else if (g.sub == 8 && g.C <= 2 * SCAN_THREADS) {
        k_scan_oct_rows<2><<<1, SCAN_THREADS, 0, s>>>(cb.count, cb.fill, cb.start, g.C, chunk,
                                                      cb.items, cb.n_items, gate);
    } else if (g.C > SCAN_THREADS && nblk <= MSCAN_MAX_BLOCKS && (g.sub == 8 || g.sub == 1)) {
        int64_t* blk = reinterpret_cast<int64_t*>(cb.tmp);
        if (g.sub == 8) {
            k_mscan_sums<8><<<(unsigned)nblk, MSCAN_THREADS, 0, s>>>(cb.count, g.C, chunk, blk,
                                                                     gate);
            k_mscan_apply<8><<<(unsigned)nblk, MSCAN_THREADS, 0, s>>>(
                cb.count, cb.fill, cb.start, g.C, chunk, cb.items, cb.n_items, blk, (int)nblk,
                gate);
        } else {
            k_mscan_sums<1><<<(unsigned)nblk, MSCAN_THREADS, 0, s>>>(cb.count, g.C, chunk, blk,
                                                                     gate);
            k_mscan_apply<1><<<(unsigned)nblk, MSCAN_THREADS, 0, s>>>(
                cb.count, cb.fill, cb.start, g.C, chunk, cb.items, cb.n_items, blk, (int)nblk,
                gate);
        }
    } else {
        k_scan<<<1, SCAN_THREADS, 0, s>>>(cb.count, cb.fill, cb.start, g.C, g.sub, chunk,
                                          cb.items, cb.n_items, cb.tmp, gate);
    }
    timer_end(t, KC_SCAN, s);
}

void launch_scatter_rank(const double* pos, const uint8_t* species, int64_t n, const Grid& g,
                         const CellBuf& cb, double4* stg64, Q4* stgq, hipStream_t s, Timer* t,
                         bool prev_order, const int32_t* gate, double* xb,
                         const StateMove* mv)
{
    if (n <= 0)
        return;
    const StateMove none{};
    timer_begin(t, KC_SCATTER, s);
    // a state move ranks by particle index: the scatter records it (the
    // source's id, or the source index itself when there are no ids)
    const bool ids = mv && mv->id_src;
    k_scatter<<<blocks_for(n, 256), 256, 0, s>>>(cb.key, n, prev_order ? cb.perm : nullptr,
                                                 cb.start, cb.fill, cb.tmp, gate,
                                                 ids ? mv->id_src : nullptr, cb.src);
    timer_end(t, KC_SCATTER, s);
    timer_begin(t, KC_RANK, s);
    k_rank<<<blocks_for(n, 256), 256, 0, s>>>(cb.key, cb.tmp, n, cb.start, cb.perm, pos,
                                              species, stg64, stgq, 4294967296.0 / g.L, gate,
                                              xb, ids ? cb.src : nullptr, mv ? *mv : none);
    timer_end(t, KC_RANK, s);
}

void launch_state_copy(const StateMove& m, double* pos, double* vel, int32_t* id, uint8_t* sp,
                       int64_t n, const int32_t* gate, hipStream_t s)
{
    if (n > 0)
        k_state_copy<<<blocks_for(n, 256), 256, 0, s>>>(m, pos, vel, id, sp, n, gate);
}

void launch_export(const int32_t* id, int64_t n, const double* src3a, double* dst3a,
                   const double* src3b, double* dst3b, const double* src1, double* dst1,
                   hipStream_t s)
{
    if (n > 0)
        k_export<<<blocks_for(n, 256), 256, 0, s>>>(id, n, src3a, dst3a, src3b, dst3b, src1,
                                                    dst1);
}

}  // namespace pasta
