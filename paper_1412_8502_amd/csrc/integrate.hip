// Velocity-Verlet integration in the expanding periodic box (Sec. II.A and
// Eq. 3).  FP64 throughout.
//
// The drift kernel fuses, per particle (sorted slot): the first half kick
// v += (dt/2M) F_n, the drift x += dt v, the optional affine scaling of the
// variant, the wrap into [0, L_{n+1}), and the cell binning of the new
// position with its integer atomic count (the first pass of the cell-list
// build).  The second half kick is fused into the force combine (k_combine,
// or the nuclear kernel's epilogue in the unfused form), which in a run of
// several steps also performs the next step's drift and binning.
//
// The thermostat (every rescale_every steps) reduces the per-work-item
// kinetic energies in fixed order in one workgroup and scales v by
// sqrt(1.5 N T / KE).
#include "internal.hpp"

namespace pasta {

namespace {

__device__ inline DriftStep drift_step(const DriftArgs& a)
{
    return DriftStep{a.hdtm, a.dt, a.L_new, a.ratio, a.scale_positions};
}

// The state is in the sorted order of the previous cell build, so the lanes
// of a wave mostly fall in one bin and the count atomics aggregate.
__global__ __launch_bounds__(256) void k_drift(DriftArgs a, int nc, int C, int sub, double inv_w,
                                               int32_t* __restrict__ key,
                                               int32_t* __restrict__ count,
                                               uint32_t* __restrict__ err)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n)
        return;
    double x[3], v[3], f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        x[d] = a.pos[3 * s + d];
        v[d] = a.vel[3 * s + d];
        f[d] = a.force[3 * s + d];
    }
    const uint32_t bad = drift_update(x, v, f, drift_step(a));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        a.vel[3 * s + d] = v[d];
        a.pos[3 * s + d] = x[d];
    }
    if (bad)
        atomicOr(err, bad);
    const int bin = particle_bin(x[0], x[1], x[2], a.species[s] == 1, inv_w, nc, C, sub);
    key[s] = bin;
    wave_aggregated_add(count, bin);
}

// List form.  Thread s owns sorted slot s of the last build.  The rebuild
// decision is taken by the last workgroup to finish (a device-scope counter
// after a release fence), so it sees every workgroup's maximum; the other
// workgroups never wait.
__global__ __launch_bounds__(256) void k_drift_list(DriftArgs a, ListCtl* __restrict__ ctl,
                                                    const double* __restrict__ xb,
                                                    double4* __restrict__ stg64,
                                                    Q4* __restrict__ stgq, double qscale,
                                                    int parity, double skin, int nc_new,
                                                    int C_new, uint32_t* __restrict__ err)
{
    __shared__ float wmax[4];
    __shared__ int last;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double L = a.L_new;
    float d2 = 0.f;
    if (s < a.n) {
        double xn[3], v[3], f[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            xn[d] = a.pos[3 * s + d];
            v[d] = a.vel[3 * s + d];
            f[d] = a.force[3 * s + d];
        }
        const uint32_t bad = drift_update(xn, v, f, drift_step(a));
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            a.vel[3 * s + d] = v[d];
            a.pos[3 * s + d] = xn[d];
        }
        if (bad)
            atomicOr(err, bad);
        double u2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double u = xn[d] - xb[3 * s + d];
            u -= L * rint(u / L);
            u2 += u * u;
        }
        d2 = (float)u2 * 1.000001f;  // rounded up: the test stays conservative
        const uint8_t sp = a.species[s];
        if (stg64)
            stg64[s] = make_double4(xn[0], xn[1], xn[2], (double)sp);
        if (stgq) {
            Q4 q;
            q.x = (uint32_t)(uint64_t)(xn[0] * qscale);
            q.y = (uint32_t)(uint64_t)(xn[1] * qscale);
            q.z = (uint32_t)(uint64_t)(xn[2] * qscale);
            q.w = sp;
            stgq[s] = q;
        }
    }
    for (int m = 32; m >= 1; m >>= 1)
        d2 = fmaxf(d2, __shfl_xor(d2, m, 64));
    if ((threadIdx.x & 63) == 0)
        wmax[threadIdx.x >> 6] = d2;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float bm = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
        // non-negative floats order like their bit patterns
        atomicMax(&ctl->maxd2[parity], __float_as_uint(bm));
        __threadfence();
        last = atomicAdd(&ctl->done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        __threadfence();
        const float m2 = __uint_as_float(atomicAdd(&ctl->maxd2[parity], 0u));
        const double dmax = sqrt((double)m2);
        const double growth = 1.7320508075688772 * fabs(L - ctl->L_build);
        const int need = !(2.0 * dmax + growth < skin);
        ctl->max_disp = dmax;
        if (need) {
            ctl->n_overflow += ctl->overflow ? 1u : 0u;
            ctl->L_build = L;
            ctl->nc = nc_new;
            ctl->C = C_new;
            ctl->pool_used = 0;
            ctl->max_rows = 0;
            ctl->overflow = 0;
            ctl->n_builds += 1;
        }
        ctl->rebuild = need;
        ctl->maxd2[parity ^ 1] = 0u;
        ctl->done = 0u;
    }
}

// Forces a build at the next gated launch sequence (rebuild = 1) for grid
// nc/C at box side L.
__global__ void k_list_force_rebuild(ListCtl* ctl, double L, int nc, int C)
{
    ctl->n_overflow += ctl->overflow ? 1u : 0u;
    ctl->L_build = L;
    ctl->nc = nc;
    ctl->C = C;
    ctl->pool_used = 0;
    ctl->max_rows = 0;
    ctl->overflow = 0;
    ctl->n_builds += 1;
    ctl->rebuild = 1;
    ctl->maxd2[0] = 0u;
    ctl->maxd2[1] = 0u;
    ctl->done = 0u;
}

constexpr int RED = 1024;

__global__ __launch_bounds__(RED) void k_thermostat_reduce(const double* __restrict__ ke_part,
                                                           const int32_t* __restrict__ n_items,
                                                           double target_ke,
                                                           double* __restrict__ scale_out)
{
    __shared__ double lds[RED];
    const int tid = threadIdx.x;
    const int m = *n_items;
    // each thread sums a contiguous run, then a fixed-shape tree: deterministic
    const int per = (m + RED - 1) / RED;
    double s = 0.0;
    for (int k = tid * per; k < min(m, (tid + 1) * per); ++k)
        s += ke_part[k];
    lds[tid] = s;
    __syncthreads();
    for (int off = RED / 2; off > 0; off >>= 1) {
        if (tid < off)
            lds[tid] += lds[tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        const double ke = lds[0];
        scale_out[0] = ke > 0.0 ? sqrt(target_ke / ke) : 1.0;
        scale_out[1] = ke;
    }
}

__global__ __launch_bounds__(256) void k_scale(double* __restrict__ vel, int64_t m,
                                               const double* __restrict__ scale)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m)
        vel[k] *= scale[0];
}

__global__ __launch_bounds__(256) void k_partial(const double* __restrict__ x, int64_t n,
                                                 int kind, double mass,
                                                 double* __restrict__ out)
{
    __shared__ double lds[256];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
        if (kind == 0) {
            s += x[i];
        } else {
            const double vx = x[3 * i], vy = x[3 * i + 1], vz = x[3 * i + 2];
            s += 0.5 * mass * (vx * vx + vy * vy + vz * vz);
        }
    }
    lds[tid] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off)
            lds[tid] += lds[tid + off];
        __syncthreads();
    }
    if (tid == 0)
        out[blockIdx.x] = lds[0];
}

}  // namespace

void launch_drift(const DriftArgs& a, const Grid& g, const CellBuf& cb, uint32_t* err,
                  hipStream_t s, Timer* t)
{
    if (a.n <= 0)
        return;
    timer_begin(t, KC_DRIFT, s);
    k_drift<<<(unsigned)((a.n + 255) / 256), 256, 0, s>>>(a, g.nc, g.C, g.sub, g.inv_w, cb.key,
                                                          cb.count, err);
    timer_end(t, KC_DRIFT, s);
}

void launch_drift_list(const DriftArgs& a, const Grid& g, const CellBuf& cb, const ListBuf& lb,
                       double4* stg64, Q4* stgq, int64_t step, uint32_t* err, hipStream_t s,
                       Timer* t)
{
    if (a.n <= 0)
        return;
    timer_begin(t, KC_DRIFT, s);
    k_drift_list<<<(unsigned)((a.n + 255) / 256), 256, 0, s>>>(
        a, lb.ctl, lb.xb, stg64, stgq, 4294967296.0 / a.L_new, (int)(step & 1),
        lb.skin, g.nc, g.C, err);
    timer_end(t, KC_DRIFT, s);
}

void launch_list_force_rebuild(const ListBuf& lb, const Grid& g, hipStream_t s)
{
    k_list_force_rebuild<<<1, 1, 0, s>>>(lb.ctl, g.L, g.nc, g.C);
}

void launch_thermostat(double* vel, int64_t n, const double* ke_part, const int32_t* n_items,
                       double target_ke, double* scale_out, hipStream_t s, Timer* t)
{
    timer_begin(t, KC_THERMO, s);
    k_thermostat_reduce<<<1, RED, 0, s>>>(ke_part, n_items, target_ke, scale_out);
    k_scale<<<(unsigned)((3 * n + 255) / 256), 256, 0, s>>>(vel, 3 * n, scale_out);
    timer_end(t, KC_THERMO, s);
}

void launch_partial_sums(const double* x, int64_t n, int kind, double mass, double* out,
                         int nblk, hipStream_t s)
{
    k_partial<<<nblk, 256, 0, s>>>(x, n, kind, mass, out);
}

}  // namespace pasta
