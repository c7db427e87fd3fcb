// Pair-force kernels for the potentials of Eq. (1a-c) (Table I constants,
// nuclear cut at r_nuc, screened Coulomb between protons uncut, nearest
// periodic image only).
//
// Both kernels are gather-form (every target sums all of its own sources, no
// third-law scatter), so no floating-point atomics are used and the result
// does not depend on scheduling.
//
// Coulomb (a3): all proton pairs.  Protons occupy sorted slots [0, Z).  A
// workgroup owns 256 targets (one per thread) and one of S source ranges;
// sources stream through an LDS tile and are read as wave-wide broadcasts.
// The S partial sums per target are added in fixed order by the nuclear
// kernel's epilogue.
//
// Nuclear (a2): cell tiles.  A workgroup owns a chunk of the targets of one
// cell; the neighbour cells' particles (protons first, then neutrons) are
// staged into an LDS tile; TPT adjacent lanes share one target and split its
// sources, then combine by wavefront shuffles.  The epilogue adds the Coulomb
// partials, writes F and E in the caller's particle order and can apply the
// velocity-Verlet second half kick (fused integrate).
//
// Precision policies:
//   FP64  -- double coordinates, nearest image d - L*rint(d/L), double exp.
//   MIXED -- 32-bit fixed-point coordinates (q = L/2^32 fm per unit): the
//            int32 difference of two coordinates is the nearest-image
//            separation in units of q, exactly; the pair arithmetic is FP32
//            with the hardware exp2 and rsqrt; each lane sums at most one
//            tile of sources in FP32 and adds that into FP64 accumulators.
#include "internal.hpp"

namespace pasta {

namespace {

constexpr int WG = 256;
constexpr int NUC_TPT = 4;                // lanes per target (nuclear)
constexpr int NUC_CHUNK = WG / NUC_TPT;   // targets per workgroup
constexpr int TILE64 = 1024;              // FP64 sources per LDS tile (32 KB)
constexpr int TILEQ = 2048;               // fixed-point sources per tile (32 KB)

// ----------------------------------------------------------- constants
struct NucConsts {
    // FP64 form: g = exp(r2 * cg); fs = g (A2 g + B/Lambda); V = g (a g + B)
    double cg, A2, a, Bl_L, Bu_L, Bl, Bu, rc2;
    double L, invL;
    // MIXED form (r2 in units of q^2)
    float cgq, A2f, af, Blf_L, Buf_L, Blf, Buf, thr_q;
    double q;        // fm per fixed-point unit
    double self_v;   // V(0) of a like pair = a + b + c, removed from E
};
struct CoulConsts {
    // FP64: V = ahc e^{-r/lambda}/r; fs = V (1/r + 1/lambda)/r
    double ahc, inv_lambda, L, invL;
    // MIXED: w = exp2(ru * c_exp) * ir; fs_u = w ir (ir cA + cB)
    float c_exp, cA, cB;
    double v_scale;  // alpha_hbarc / q  (V = v_scale * w)
    double f_scale;  // alpha_hbarc      (F = f_scale * fs_u * du)
};

// ============================================================ Coulomb ==
__device__ __forceinline__ void coul_pair64(const double4 me, const double4 s, int self,
                                            const CoulConsts& k, double& fx, double& fy,
                                            double& fz, double& e)
{
    double dx = me.x - s.x, dy = me.y - s.y, dz = me.z - s.z;
    dx = fma(-k.L, rint(dx * k.invL), dx);
    dy = fma(-k.L, rint(dy * k.invL), dy);
    dz = fma(-k.L, rint(dz * k.invL), dz);
    double r2 = dx * dx + dy * dy + dz * dz;
    r2 = self ? 1e300 : r2;
    double ir = rsqrt(r2);
    double r = r2 * ir;
    double v = k.ahc * exp(-r * k.inv_lambda) * ir;
    double fs = v * (ir + k.inv_lambda) * ir;
    fx = fma(fs, dx, fx);
    fy = fma(fs, dy, fy);
    fz = fma(fs, dz, fz);
    e += v;
}

__device__ __forceinline__ void coul_pairq(const Q4 me, const uint4 s, int self,
                                           const CoulConsts& k, float& fx, float& fy,
                                           float& fz, float& e)
{
    float dx = (float)(int32_t)(me.x - s.x);
    float dy = (float)(int32_t)(me.y - s.y);
    float dz = (float)(int32_t)(me.z - s.z);
    float r2 = dx * dx + dy * dy + dz * dz;
    r2 = self ? 3.0e38f : r2;
    float ir = __builtin_amdgcn_rsqf(r2);
    float ru = r2 * ir;
    float w = __builtin_amdgcn_exp2f(ru * k.c_exp) * ir;
    float fs = w * ir * fmaf(ir, k.cA, k.cB);
    fx = fmaf(fs, dx, fx);
    fy = fmaf(fs, dy, fy);
    fz = fmaf(fs, dz, fz);
    e += w;
}

__global__ __launch_bounds__(WG) void k_coulomb64(const double4* __restrict__ stg, int Z,
                                                  int per_split, CoulConsts k,
                                                  double4* __restrict__ part)
{
    __shared__ double4 tile[TILE64];
    const int t = blockIdx.x * WG + threadIdx.x;
    const int split = blockIdx.y;
    const int j0 = split * per_split;
    const int j1 = min(Z, j0 + per_split);
    const int tb0 = blockIdx.x * WG, tb1 = min(Z, tb0 + WG);
    const double4 me = stg[t < Z ? t : 0];
    double fx = 0, fy = 0, fz = 0, e = 0;
    for (int base = j0; base < j1; base += TILE64) {
        const int cnt = min(TILE64, j1 - base);
        for (int q = threadIdx.x; q < cnt; q += WG)
            tile[q] = stg[base + q];
        __syncthreads();
        if (base < tb1 && base + cnt > tb0) {
            for (int q = 0; q < cnt; ++q)
                coul_pair64(me, tile[q], base + q == t, k, fx, fy, fz, e);
        } else {
#pragma unroll 4
            for (int q = 0; q < cnt; ++q)
                coul_pair64(me, tile[q], 0, k, fx, fy, fz, e);
        }
        __syncthreads();
    }
    if (t < Z)
        part[(int64_t)split * Z + t] = make_double4(fx, fy, fz, e);
}

__global__ __launch_bounds__(WG) void k_coulombq(const Q4* __restrict__ stg, int Z,
                                                 int per_split, CoulConsts k,
                                                 double4* __restrict__ part)
{
    __shared__ uint4 tile[TILEQ];
    const int t = blockIdx.x * WG + threadIdx.x;
    const int split = blockIdx.y;
    const int j0 = split * per_split;
    const int j1 = min(Z, j0 + per_split);
    const int tb0 = blockIdx.x * WG, tb1 = min(Z, tb0 + WG);
    const Q4 me = stg[t < Z ? t : 0];
    const uint4* src = reinterpret_cast<const uint4*>(stg);
    double fx = 0, fy = 0, fz = 0, e = 0;
    for (int base = j0; base < j1; base += TILEQ) {
        const int cnt = min(TILEQ, j1 - base);
        for (int q = threadIdx.x; q < cnt; q += WG)
            tile[q] = src[base + q];
        __syncthreads();
        float ax = 0.f, ay = 0.f, az = 0.f, ae = 0.f;
        if (base < tb1 && base + cnt > tb0) {
            for (int q = 0; q < cnt; ++q)
                coul_pairq(me, tile[q], base + q == t, k, ax, ay, az, ae);
        } else {
#pragma unroll 4
            for (int q = 0; q < cnt; ++q)
                coul_pairq(me, tile[q], 0, k, ax, ay, az, ae);
        }
        fx += ax;
        fy += ay;
        fz += az;
        e += ae;
        __syncthreads();
    }
    if (t < Z)
        part[(int64_t)split * Z + t] =
            make_double4(fx * k.f_scale, fy * k.f_scale, fz * k.f_scale, e * k.v_scale);
}

// ============================================================ nuclear ==
struct Fp64Policy {
    using Src = double4;
    using Lds = double4;
    static constexpr int TILE = TILE64;
    struct Acc {
        double fx = 0, fy = 0, fz = 0, e = 0;
        uint32_t np = 0;
    };
    struct Part {
        double fx = 0, fy = 0, fz = 0, e = 0;
        uint32_t np = 0;
    };
    __device__ static Lds load(const Src* s, int j) { return s[j]; }
    template <bool COUNT>
    __device__ static void pair(const Src& me, const Lds& s, double B_L, double B,
                                const NucConsts& k, Part& p)
    {
        double dx = me.x - s.x, dy = me.y - s.y, dz = me.z - s.z;
        dx = fma(-k.L, rint(dx * k.invL), dx);
        dy = fma(-k.L, rint(dy * k.invL), dy);
        dz = fma(-k.L, rint(dz * k.invL), dz);
        double r2 = dx * dx + dy * dy + dz * dz;
        const bool in = r2 < k.rc2;
        if (COUNT)
            p.np += in ? 1u : 0u;
        double g = in ? exp(r2 * k.cg) : 0.0;
        double fs = g * fma(k.A2, g, B_L);
        p.fx = fma(fs, dx, p.fx);
        p.fy = fma(fs, dy, p.fy);
        p.fz = fma(fs, dz, p.fz);
        p.e = fma(g, fma(k.a, g, B), p.e);
    }
    __device__ static void fold(Acc& a, Part& p)
    {
        a.fx += p.fx;
        a.fy += p.fy;
        a.fz += p.fz;
        a.e += p.e;
        a.np += p.np;
        p = Part();
    }
    __device__ static double f_scale(const NucConsts&) { return 1.0; }
    __device__ static double bl(const NucConsts& k, bool like) { return like ? k.Bl_L : k.Bu_L; }
    __device__ static double bv(const NucConsts& k, bool like) { return like ? k.Bl : k.Bu; }
};

struct MixedPolicy {
    using Src = Q4;
    using Lds = uint4;
    static constexpr int TILE = TILEQ;
    struct Acc {
        double fx = 0, fy = 0, fz = 0, e = 0;
        uint32_t np = 0;
    };
    struct Part {
        float fx = 0.f, fy = 0.f, fz = 0.f, e = 0.f;
        uint32_t np = 0;
    };
    __device__ static Lds load(const Src* s, int j)
    {
        return reinterpret_cast<const uint4*>(s)[j];
    }
    template <bool COUNT>
    __device__ static void pair(const Src& me, const Lds& s, float B_L, float B,
                                const NucConsts& k, Part& p)
    {
        float dx = (float)(int32_t)(me.x - s.x);
        float dy = (float)(int32_t)(me.y - s.y);
        float dz = (float)(int32_t)(me.z - s.z);
        float r2 = dx * dx + dy * dy + dz * dz;
        const bool in = r2 < k.thr_q;
        if (COUNT)
            p.np += in ? 1u : 0u;
        r2 = in ? r2 : 3.0e38f;  // exp2 underflows to exactly 0 outside the cutoff
        float g = __builtin_amdgcn_exp2f(r2 * k.cgq);
        float fs = g * fmaf(k.A2f, g, B_L);
        p.fx = fmaf(fs, dx, p.fx);
        p.fy = fmaf(fs, dy, p.fy);
        p.fz = fmaf(fs, dz, p.fz);
        p.e = fmaf(g, fmaf(k.af, g, B), p.e);
    }
    __device__ static void fold(Acc& a, Part& p)
    {
        a.fx += (double)p.fx;
        a.fy += (double)p.fy;
        a.fz += (double)p.fz;
        a.e += (double)p.e;
        a.np += p.np;
        p = Part();
    }
    __device__ static double f_scale(const NucConsts& k) { return k.q; }
    __device__ static float bl(const NucConsts& k, bool like) { return like ? k.Blf_L : k.Buf_L; }
    __device__ static float bv(const NucConsts& k, bool like) { return like ? k.Blf : k.Buf; }
};

struct NucArgs {
    const int32_t* start;   // [2C+1]
    const int32_t* items;   // [2*item_max]
    const int32_t* n_items; // [1]
    const int32_t* perm;    // [n]
    int nc, C;
    int Z;
    const double4* coul_part;
    int S;                  // Coulomb splits (0 = no Coulomb)
    double* force;          // [n][3] caller order
    double* epot;           // [n] or null
    double* vel;            // [n][3] or null: apply the half kick
    double hdtm, mass;
    double* ke_part;        // [item_max] or null
    unsigned long long* pairs;
    uint32_t* err;
};

template <class P, bool NUC, bool COUNT>
__global__ __launch_bounds__(WG) void k_nuclear(const typename P::Src* __restrict__ stg,
                                                NucArgs A, NucConsts k)
{
    using Lds = typename P::Lds;
    __shared__ Lds tile[P::TILE];
    __shared__ int seg_beg[54];
    __shared__ int seg_off[55];
    __shared__ double ke_red[WG / 64];
    __shared__ unsigned long long np_red[WG / 64];

    const int item = blockIdx.x;
    if (item >= *A.n_items)
        return;
    const int c = A.items[2 * item + 0];
    const int chunk = A.items[2 * item + 1];
    const int tid = threadIdx.x;
    const int nc = A.nc, C = A.C;
    const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);

    if (NUC && tid < 54) {
        const int kk = tid % 27, sp = tid / 27;  // sp 0: protons, 1: neutrons
        const int ox = kk % 3 - 1, oy = (kk / 3) % 3 - 1, oz = kk / 9 - 1;
        const int lo = axis_lo(nc), hi = axis_hi(nc);
        int beg = 0, len = 0;
        if (ox >= lo && ox <= hi && oy >= lo && oy <= hi && oz >= lo && oz <= hi) {
            const int nx = (cx + ox + nc) % nc, ny = (cy + oy + nc) % nc,
                      nz = (cz + oz + nc) % nc;
            const int b = sp * C + (nz * nc + ny) * nc + nx;
            beg = A.start[b];
            len = A.start[b + 1] - beg;
        }
        seg_beg[tid] = beg;
        seg_off[tid + 1] = len;
    }
    __syncthreads();
    if (NUC && tid == 0) {
        seg_off[0] = 0;
        for (int s = 1; s <= 54; ++s)
            seg_off[s] += seg_off[s - 1];
    }
    __syncthreads();

    const int ps = A.start[c], npc = A.start[c + 1] - ps;
    const int ns = A.start[C + c], mc = npc + (A.start[C + c + 1] - ns);
    const int tl = tid / NUC_TPT, q = tid % NUC_TPT;
    const int tidx = chunk * NUC_CHUNK + tl;
    const bool active = tidx < mc;
    const int slot = active ? (tidx < npc ? ps + tidx : ns + (tidx - npc)) : 0;
    const bool tprot = tidx < npc;
    const typename P::Src me = stg[slot];

    typename P::Acc acc;
    if (NUC) {
        const int total = seg_off[54], np_tot = seg_off[27];
        const auto BLp = P::bl(k, tprot), Bp = P::bv(k, tprot);     // proton sources
        const auto BLn = P::bl(k, !tprot), Bn = P::bv(k, !tprot);   // neutron sources
        typename P::Part part;
        for (int w0 = 0; w0 < total; w0 += P::TILE) {
            const int cnt = min(P::TILE, total - w0);
            for (int kq = tid; kq < cnt; kq += WG) {
                const int gidx = w0 + kq;
                int lo = 0, hi = 54;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (seg_off[mid] <= gidx)
                        lo = mid;
                    else
                        hi = mid;
                }
                tile[kq] = P::load(stg, seg_beg[lo] + (gidx - seg_off[lo]));
            }
            __syncthreads();
            const int kb = min(max(np_tot - w0, 0), cnt);
            for (int j = q; j < kb; j += NUC_TPT)
                P::template pair<COUNT>(me, tile[j], BLp, Bp, k, part);
            for (int j = kb + q; j < cnt; j += NUC_TPT)
                P::template pair<COUNT>(me, tile[j], BLn, Bn, k, part);
            P::fold(acc, part);
            __syncthreads();
        }
#pragma unroll
        for (int m = 1; m < NUC_TPT; m <<= 1) {
            acc.fx += __shfl_xor(acc.fx, m, NUC_TPT);
            acc.fy += __shfl_xor(acc.fy, m, NUC_TPT);
            acc.fz += __shfl_xor(acc.fz, m, NUC_TPT);
            acc.e += __shfl_xor(acc.e, m, NUC_TPT);
            if (COUNT)
                acc.np += __shfl_xor(acc.np, m, NUC_TPT);
        }
    }

    double ke = 0.0;
    unsigned long long npairs = 0;
    if (active && q == 0) {
        const double fsc = P::f_scale(k);
        double Fx = acc.fx * fsc, Fy = acc.fy * fsc, Fz = acc.fz * fsc;
        // the self pair (r = 0) entered the sum with V(0) = a + b + c
        double V = NUC ? acc.e - k.self_v : 0.0;
        if (COUNT)
            npairs = acc.np - 1u;  // minus the self pair
        if (A.S > 0 && tprot) {
            for (int s = 0; s < A.S; ++s) {
                const double4 cp = A.coul_part[(int64_t)s * A.Z + slot];
                Fx += cp.x;
                Fy += cp.y;
                Fz += cp.z;
                V += cp.w;
            }
        }
        const int64_t id = A.perm[slot];
        A.force[3 * id + 0] = Fx;
        A.force[3 * id + 1] = Fy;
        A.force[3 * id + 2] = Fz;
        if (A.epot)
            A.epot[id] = 0.5 * V;
        if (!(isfinite(Fx) && isfinite(Fy) && isfinite(Fz)))
            atomicOr(A.err, ERR_NONFINITE_FORCE);
        if (A.vel) {
            double vx = A.vel[3 * id + 0] + A.hdtm * Fx;
            double vy = A.vel[3 * id + 1] + A.hdtm * Fy;
            double vz = A.vel[3 * id + 2] + A.hdtm * Fz;
            A.vel[3 * id + 0] = vx;
            A.vel[3 * id + 1] = vy;
            A.vel[3 * id + 2] = vz;
            ke = 0.5 * A.mass * (vx * vx + vy * vy + vz * vz);
        }
    }
    if (A.ke_part || COUNT) {
        // fixed-order block reduction (deterministic)
        for (int m = 32; m >= 1; m >>= 1) {
            ke += __shfl_xor(ke, m, 64);
            if (COUNT)
                npairs += __shfl_xor(npairs, m, 64);
        }
        if ((tid & 63) == 0) {
            ke_red[tid >> 6] = ke;
            np_red[tid >> 6] = npairs;
        }
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            unsigned long long sn = 0;
            for (int w = 0; w < WG / 64; ++w) {
                s += ke_red[w];
                sn += np_red[w];
            }
            if (A.ke_part)
                A.ke_part[item] = s;
            if (COUNT)
                atomicAdd(A.pairs, sn);
        }
    }
}

template <class P>
void nuclear_dispatch(const typename P::Src* stg, const NucArgs& a, const NucConsts& k,
                      bool nuc, bool count, unsigned grid, hipStream_t s)
{
    if (nuc && count)
        k_nuclear<P, true, true><<<grid, WG, 0, s>>>(stg, a, k);
    else if (nuc)
        k_nuclear<P, true, false><<<grid, WG, 0, s>>>(stg, a, k);
    else
        k_nuclear<P, false, false><<<grid, WG, 0, s>>>(stg, a, k);
}

}  // namespace

int nuclear_chunk(int /*precision*/) { return NUC_CHUNK; }

int coulomb_splits(int64_t Z)
{
    if (Z <= 0)
        return 0;
    int64_t s = 524288 / Z;
    return (int)(s < 1 ? 1 : (s > 32 ? 32 : s));
}

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
    CoulConsts k{};
    k.ahc = pp.alpha_hbarc;
    k.inv_lambda = 1.0 / pp.lambda_s;
    k.L = pp.L;
    k.invL = 1.0 / pp.L;
    const double q = pp.L / 4294967296.0;
    k.c_exp = (float)(-q / pp.lambda_s * 1.4426950408889634);
    k.cA = (float)(1.0 / (q * q));
    k.cB = (float)(1.0 / (pp.lambda_s * q));
    k.v_scale = pp.alpha_hbarc / q;
    k.f_scale = pp.alpha_hbarc;
    dim3 grid((unsigned)((Z + WG - 1) / WG), (unsigned)S);
    timer_begin(t, KC_COULOMB, s);
    if (precision == PASTA_FP64)
        k_coulomb64<<<grid, WG, 0, s>>>(fb.stg64, (int)Z, per, k, fb.coul_part);
    else
        k_coulombq<<<grid, WG, 0, s>>>(fb.stgq, (int)Z, per, k, fb.coul_part);
    timer_end(t, KC_COULOMB, s);
}

void launch_nuclear(int precision, const ForceBuf& fb, const CellBuf& cb, const Grid& g,
                    int64_t n, int64_t Z, const PairParams& pp, bool with_nuclear_terms,
                    int coul_S, double* force, double* epot, const KickArgs& kick,
                    uint64_t* pair_counter, uint32_t* err, hipStream_t s, Timer* t)
{
    (void)n;
    NucConsts k{};
    const double Lam = pp.Lambda;
    k.cg = -1.0 / (2.0 * Lam);
    k.A2 = 2.0 * pp.a / Lam;
    k.a = pp.a;
    k.Bl = pp.b_like;
    k.Bu = pp.b_unlike;
    k.Bl_L = pp.b_like / Lam;
    k.Bu_L = pp.b_unlike / Lam;
    k.rc2 = pp.r_nuc * pp.r_nuc;
    k.L = pp.L;
    k.invL = 1.0 / pp.L;
    k.q = pp.L / 4294967296.0;
    k.cgq = (float)(-(k.q * k.q) / (2.0 * Lam) * 1.4426950408889634);
    k.A2f = (float)k.A2;
    k.af = (float)pp.a;
    k.Blf = (float)pp.b_like;
    k.Buf = (float)pp.b_unlike;
    k.Blf_L = (float)k.Bl_L;
    k.Buf_L = (float)k.Bu_L;
    k.thr_q = (float)(k.rc2 / (k.q * k.q));
    k.self_v = pp.a + pp.b_like;

    NucArgs a{};
    a.start = cb.start;
    a.items = cb.items;
    a.n_items = cb.n_items;
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
    unsigned grid = (unsigned)cb.item_max;
    timer_begin(t, KC_NUCLEAR, s);
    const bool count = pair_counter != nullptr;
    if (precision == PASTA_FP64)
        nuclear_dispatch<Fp64Policy>(fb.stg64, a, k, with_nuclear_terms, count, grid, s);
    else
        nuclear_dispatch<MixedPolicy>(fb.stgq, a, k, with_nuclear_terms, count, grid, s);
    timer_end(t, KC_NUCLEAR, s);
}

}  // namespace pasta
