// Cluster algorithm of Sec. II.C on the device.
//
//   1. cell list with cells no narrower than r_pp (protons first);
//   2. union-find over proton pairs within r_pp: each proton links to the
//      protons of higher index in its neighbour cells; a union always hooks
//      the larger root under the smaller one, so every component ends with
//      its smallest proton index as root, whatever order the atomics took;
//   3. compression (root of every proton), a flag per root and a scan over
//      particle indices: clusters are numbered in increasing root index;
//   4. neutron attachment: nearest proton within r_np, ties to the lower
//      proton index;
//   5. per-cluster A and Z with integer atomics, then the A and Z histograms.
// Every result is an integer that does not depend on scheduling, so it can be
// compared bit for bit.  Distances are FP64 without contraction into FMA so
// that the <= tests see the same numbers as a plain CPU evaluation.
#pragma clang fp contract(off)
#include "internal.hpp"

namespace pasta {

namespace {

constexpr int UF_RETRY_LIMIT = 1 << 22;

__device__ __forceinline__ double min_image_exact(double d, double L)
{
    if (d > 0.5 * L)
        d -= L;
    else if (d < -0.5 * L)
        d += L;
    return d;
}

__device__ __forceinline__ double dist2_exact(const double* pos, int64_t i, int64_t j, double L)
{
    const double dx = min_image_exact(pos[3 * i + 0] - pos[3 * j + 0], L);
    const double dy = min_image_exact(pos[3 * i + 1] - pos[3 * j + 1], L);
    const double dz = min_image_exact(pos[3 * i + 2] - pos[3 * j + 2], L);
    // this file is compiled with -ffp-contract=off: no fused multiply-add
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ int32_t load_parent(int32_t* parent, int32_t x)
{
    return __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving.  Invariant: parent[x] <= x, and a parent only
// ever decreases, so every loop below terminates.
__device__ int32_t uf_find(int32_t* parent, int32_t x)
{
    int32_t p = load_parent(parent, x);
    while (p != x) {
        const int32_t gp = load_parent(parent, p);
        if (gp != p)
            __hip_atomic_fetch_min(&parent[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = p;
        p = gp;
    }
    return x;
}

__device__ bool uf_union(int32_t* parent, int32_t a, int32_t b)
{
    for (int it = 0; it < UF_RETRY_LIMIT; ++it) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b)
            return true;
        if (a > b) {
            const int32_t t = a;
            a = b;
            b = t;
        }
        // hook root b under the smaller root a, if b is still a root
        int32_t expected = b;
        if (__hip_atomic_compare_exchange_strong(&parent[b], &expected, a, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return true;
    }
    return false;
}

__global__ __launch_bounds__(256) void k_uf_init(int32_t* parent, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        parent[i] = (int32_t)i;
}

struct ClusterArgs {
    const double* pos;
    const uint8_t* species;
    const int32_t* start;
    const int32_t* perm;
    int64_t n;
    int nc, C;
    double inv_w, L, rpp2, rnp2;
    int32_t* parent;
    int32_t* label;
    int32_t* flag;     // [n] root flags, then (in place) their exclusive scan
    int32_t* cnt_a;    // [n] per-cluster mass number
    int32_t* cnt_z;    // [n] per-cluster charge
    int32_t* scalars;  // [0] K, [1] free neutrons
    uint32_t* err;
};

__device__ __forceinline__ void cell_of_particle(const ClusterArgs& a, int64_t i, int& cx, int& cy,
                                                 int& cz)
{
    cx = cell_coord(a.pos[3 * i + 0], a.inv_w, a.nc);
    cy = cell_coord(a.pos[3 * i + 1], a.inv_w, a.nc);
    cz = cell_coord(a.pos[3 * i + 2], a.inv_w, a.nc);
}

// One thread per proton slot: link to protons of higher index in range.
__global__ __launch_bounds__(256) void k_uf_link(ClusterArgs a, int32_t Z)
{
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= Z)
        return;
    const int32_t i = a.perm[s];
    int cx, cy, cz;
    cell_of_particle(a, i, cx, cy, cz);
    const int lo = axis_lo(a.nc), hi = axis_hi(a.nc), nc = a.nc;
    bool ok = true;
    for (int oz = lo; oz <= hi; ++oz)
        for (int oy = lo; oy <= hi; ++oy)
            for (int ox = lo; ox <= hi; ++ox) {
                const int c = (((cz + oz + nc) % nc) * nc + (cy + oy + nc) % nc) * nc +
                              (cx + ox + nc) % nc;
                for (int t = a.start[c]; t < a.start[c + 1]; ++t) {
                    const int32_t j = a.perm[t];
                    if (j > i && dist2_exact(a.pos, i, j, a.L) <= a.rpp2)
                        ok &= uf_union(a.parent, i, j);
                }
            }
    if (!ok)
        atomicOr(a.err, ERR_UF_LIMIT);
}

// Final roots and root flags (over particle indices, caller order).
__global__ __launch_bounds__(256) void k_uf_flags(ClusterArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n)
        return;
    int32_t f = 0;
    if (a.species[i] == 1) {
        const int32_t r = uf_find(a.parent, (int32_t)i);
        a.parent[i] = r;
        f = (r == (int32_t)i);
    }
    a.flag[i] = f;
}

constexpr int SCAN_T = 1024;

// In-place exclusive scan of flag[0..n) in one workgroup; K = total.
__global__ __launch_bounds__(SCAN_T) void k_flag_scan(int32_t* flag, int64_t n, int32_t* scalars)
{
    __shared__ int64_t lds[SCAN_T];
    const int tid = threadIdx.x;
    const int64_t per = (n + SCAN_T - 1) / SCAN_T;
    const int64_t b = tid * per, e = b + per < n ? b + per : n;
    int64_t s = 0;
    for (int64_t k = b; k < e; ++k)
        s += flag[k];
    lds[tid] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        const int64_t t = tid >= off ? lds[tid - off] : 0;
        __syncthreads();
        lds[tid] += t;
        __syncthreads();
    }
    int64_t run = lds[tid] - s;
    for (int64_t k = b; k < e; ++k) {
        const int32_t v = flag[k];
        flag[k] = (int32_t)run;
        run += v;
    }
    if (tid == SCAN_T - 1) {
        scalars[0] = (int32_t)lds[SCAN_T - 1];
        scalars[1] = 0;
    }
}

__global__ __launch_bounds__(256) void k_label_protons(ClusterArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n)
        return;
    if (a.species[i] == 1)
        a.label[i] = a.flag[a.parent[i]];
    a.cnt_a[i] = 0;
    a.cnt_z[i] = 0;
}

// One thread per neutron slot: nearest proton within r_np (lower index on ties).
__global__ __launch_bounds__(256) void k_attach(ClusterArgs a, int32_t Z)
{
    const int64_t s = (int64_t)Z + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n)
        return;
    const int32_t k = a.perm[s];
    int cx, cy, cz;
    cell_of_particle(a, k, cx, cy, cz);
    const int lo = axis_lo(a.nc), hi = axis_hi(a.nc), nc = a.nc;
    int32_t best = -1;
    double bd = 0.0;
    for (int oz = lo; oz <= hi; ++oz)
        for (int oy = lo; oy <= hi; ++oy)
            for (int ox = lo; ox <= hi; ++ox) {
                const int c = (((cz + oz + nc) % nc) * nc + (cy + oy + nc) % nc) * nc +
                              (cx + ox + nc) % nc;
                for (int t = a.start[c]; t < a.start[c + 1]; ++t) {
                    const int32_t j = a.perm[t];
                    const double d2 = dist2_exact(a.pos, k, j, a.L);
                    if (d2 <= a.rnp2 && (best < 0 || d2 < bd || (d2 == bd && j < best))) {
                        best = j;
                        bd = d2;
                    }
                }
            }
    if (best >= 0) {
        a.label[k] = a.label[best];
    } else {
        a.label[k] = -1;
        atomicAdd(&a.scalars[1], 1);
    }
}

__global__ __launch_bounds__(256) void k_members(ClusterArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n)
        return;
    const int32_t l = a.label[i];
    if (l >= 0) {
        atomicAdd(&a.cnt_a[l], 1);
        if (a.species[i] == 1)
            atomicAdd(&a.cnt_z[l], 1);
    }
}

__global__ __launch_bounds__(256) void k_hist_clear(int32_t* ha, int32_t* hz, int64_t m)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) {
        ha[i] = 0;
        hz[i] = 0;
    }
}

__global__ __launch_bounds__(256) void k_hist(ClusterArgs a, int32_t* ha, int32_t* hz)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.scalars[0])
        return;
    atomicAdd(&ha[a.cnt_a[k]], 1);
    atomicAdd(&hz[a.cnt_z[k]], 1);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

}  // namespace

struct ClusterBuf {
    CellBuf cb;
    int32_t* parent;
    int32_t* flag;
    int32_t* cnt_a;
    int32_t* cnt_z;
    int32_t* scalars;
    uint32_t* err;
};

static size_t cluster_carve(Carver& cv, ClusterBuf* out, int64_t n, int C)
{
    ClusterBuf b;
    cellbuf_carve(cv, &b.cb, n, C, 0);
    b.parent = cv.take<int32_t>(n);
    b.flag = cv.take<int32_t>(n);
    b.cnt_a = cv.take<int32_t>(n);
    b.cnt_z = cv.take<int32_t>(n);
    b.scalars = cv.take<int32_t>(4);
    b.err = cv.take<uint32_t>(1);
    if (out)
        *out = b;
    return cv.size();
}

}  // namespace pasta

using namespace pasta;

extern "C" int pasta_cluster_workspace(int64_t n, double L, double r_pp, double r_np,
                                       size_t* h_bytes)
{
    if (!h_bytes || n < 0 || !(L > 0.0) || !(r_pp > 0.0) || !(r_np > 0.0))
        return fail(PASTA_EINVAL, "pasta_cluster_workspace: bad argument");
    const double rc = r_pp > r_np ? r_pp : r_np;
    const Grid g = make_grid(L, rc);
    Carver cv(nullptr);
    *h_bytes = cluster_carve(cv, nullptr, n, g.C);
    return PASTA_OK;
}

extern "C" int pasta_cluster(int64_t n, double L, const double* d_pos, const uint8_t* d_species,
                             double r_pp, double r_np, int32_t* d_label, int32_t* d_hist_A,
                             int32_t* d_hist_Z, int32_t* h_nclusters, int32_t* h_nfree,
                             void* d_work, size_t work_bytes, void* stream)
{
    if (n < 0 || (n > 0 && (!d_pos || !d_species || !d_label)) || !d_hist_A || !d_hist_Z ||
        !h_nclusters || !(r_pp > 0.0) || !(r_np > 0.0) || !(L > 0.0) || !std::isfinite(L))
        return fail(PASTA_EINVAL, "pasta_cluster: bad argument");
    if (n > INT32_MAX - 1)
        return fail(PASTA_EINVAL, "pasta_cluster: n too large");
    const double rc = r_pp > r_np ? r_pp : r_np;
    if (L < 2.0 * rc)
        return fail(PASTA_EBOX, "pasta_cluster: L = %g < 2 * %g", L, rc);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid g = make_grid(L, rc);
    Carver cv(nullptr);
    const size_t need = cluster_carve(cv, nullptr, n, g.C);
    if (!d_work || work_bytes < need || (reinterpret_cast<uintptr_t>(d_work) & 255))
        return fail(PASTA_EWORKSPACE, "pasta_cluster: workspace needs %zu bytes (256-aligned)",
                    need);
    ClusterBuf b;
    Carver cw(d_work);
    cluster_carve(cw, &b, n, g.C);
    if (n == 0) {
        k_hist_clear<<<1, 256, 0, s>>>(d_hist_A, d_hist_Z, 1);
        PASTA_HIP(hipStreamSynchronize(s));
        *h_nclusters = 0;
        if (h_nfree)
            *h_nfree = 0;
        return PASTA_OK;
    }
    PASTA_HIP(hipMemsetAsync(b.err, 0, sizeof(uint32_t), s));
    cellbuf_zero(b.cb, g.C, s);
    launch_bin_count(d_pos, d_species, n, g, b.cb, b.err, s, nullptr);
    launch_scan(b.cb, g, 0, s, nullptr);
    launch_scatter_rank(d_pos, d_species, n, g, b.cb, nullptr, nullptr, s, nullptr);

    ClusterArgs a{};
    a.pos = d_pos;
    a.species = d_species;
    a.start = b.cb.start;
    a.perm = b.cb.perm;
    a.n = n;
    a.nc = g.nc;
    a.C = g.C;
    a.inv_w = g.inv_w;
    a.L = L;
    a.rpp2 = r_pp * r_pp;
    a.rnp2 = r_np * r_np;
    a.parent = b.parent;
    a.label = d_label;
    a.flag = b.flag;
    a.cnt_a = b.cnt_a;
    a.cnt_z = b.cnt_z;
    a.scalars = b.scalars;
    a.err = b.err;

    // Z = number of protons = start of the neutron bins
    int32_t Z = 0;
    PASTA_HIP(hipMemcpyAsync(&Z, b.cb.start + g.C, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PASTA_HIP(hipStreamSynchronize(s));
    k_uf_init<<<nblk(n), 256, 0, s>>>(b.parent, n);
    if (Z > 0)
        k_uf_link<<<nblk(Z), 256, 0, s>>>(a, Z);
    k_uf_flags<<<nblk(n), 256, 0, s>>>(a);
    k_flag_scan<<<1, SCAN_T, 0, s>>>(b.flag, n, b.scalars);
    k_label_protons<<<nblk(n), 256, 0, s>>>(a);
    if (n - Z > 0)
        k_attach<<<nblk(n - Z), 256, 0, s>>>(a, Z);
    k_members<<<nblk(n), 256, 0, s>>>(a);
    k_hist_clear<<<nblk(n + 1), 256, 0, s>>>(d_hist_A, d_hist_Z, n + 1);
    k_hist<<<nblk(Z > 0 ? Z : 1), 256, 0, s>>>(a, d_hist_A, d_hist_Z);
    int32_t sc[2] = {0, 0};
    uint32_t err = 0;
    PASTA_HIP(hipMemcpyAsync(sc, b.scalars, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PASTA_HIP(hipMemcpyAsync(&err, b.err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    PASTA_HIP(hipStreamSynchronize(s));
    PASTA_HIP(hipGetLastError());
    if (err)
        return fail(PASTA_EDEVICE, "pasta_cluster: %s", describe_device_error(err).c_str());
    *h_nclusters = sc[0];
    if (h_nfree)
        *h_nfree = sc[1];
    return PASTA_OK;
}
