// Device-side work items of the pair-force kernels, shared by the
// single-system kernels (forces.hip) and the batched persistent kernel
// (batch.hip).  Potentials: Eq. (1a-c) with the Table I constants, nuclear
// part cut at r_nuc, screened Coulomb between protons uncut, nearest
// periodic image only.
//
// Both forms are gather-form (every target sums all of its own sources), so no
// floating-point atomics are used and the results do not depend on
// scheduling.
//
// Precision policies:
//   Fp64Policy  -- double coordinates, nearest image by the strict L/2 test, the
//                  FP64 exp and rsqrt of fp64math.hpp, double accumulation.
//   MixedPolicy -- 32-bit fixed-point coordinates (q = L/2^32 fm per unit):
//                  the int32 difference of two coordinates is the
//                  nearest-image separation in units of q, exactly; FP32 pair
//                  arithmetic with the hardware exp2 and rsqrt; each lane's
//                  FP32 sum over at most one source tile is added into FP64
//                  accumulators.
#pragma once

#include <climits>

#include "fp64math.hpp"
#include "internal.hpp"

namespace pasta {

// Nearest periodic image of an FP64 coordinate difference, positions held
// in [0, L): subtract L when d > L/2, add L when d < -L/2 (strict, so the
// difference stays antisymmetric and |d| = L/2 keeps its sign).  hL = L/2.
__device__ __forceinline__ double nearest_image(double d, double L, double hL)
{
    return d > hL ? d - L : (d < -hL ? d + L : d);
}

// r^2 = (dx dx + dy dy) + dz dz with every product and sum rounded on its
// own (no fused multiply-add), the order of the definition.
__device__ __forceinline__ double r2_exact(double dx, double dy, double dz)
{
    return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

// What a pair kernel accumulates: forces only, forces and energy shares,
// or forces, energies and the count of pairs inside the cutoff.
constexpr int MODE_FORCE = 0;
constexpr int MODE_ENERGY = 1;
constexpr int MODE_COUNT = 2;

constexpr int WG = 256;
constexpr int NUC_TPT = 4;               // lanes per target (nuclear)
constexpr int NUC_CHUNK = WG / NUC_TPT;  // targets per work item
constexpr int TILE64 = 1024;             // FP64 sources per LDS tile (32 KB)
constexpr int TILEQ = 1024;              // fixed-point sources per tile (16 KB)

// ----------------------------------------------------------- constants
struct NucConsts {
    // FP64 form: g = exp(r2 * cg); fs = g (A2 g + B/Lambda); V = g (a g + B)
    double cg, A2, a, Bl_L, Bu_L, Bl, Bu, rc2;
    double L, hL;
    // MIXED form (r2 in units of q^2)
    float cgq, A2f, af, Blf_L, Buf_L, Blf, Buf, thr_q;
    double q;       // fm per fixed-point unit
    double self_v;  // V(0) of a like pair = a + b + c, removed from E
    // screening pass of the compacting kernel
    double qscale;  // 2^32 / L (fixed-point units per fm)
    int thr16;      // (r_nuc / (L/2^16) + 2)^2: conservative 16-bit test
    uint32_t thr_stage16;  // (r_nuc / (L/2^16))^2 + 1: the staging gap test
};

__host__ __device__ inline NucConsts make_nuc_consts(const PairParams& pp)
{
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
    k.hL = 0.5 * pp.L;
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
    k.qscale = 4294967296.0 / pp.L;
    const double r16 = pp.r_nuc * 65536.0 / pp.L + 2.0;
    k.thr16 = (int)(r16 * r16) + 1;
    const double rs = pp.r_nuc * 65536.0 / pp.L;
    k.thr_stage16 = (uint32_t)(rs * rs) + 1u;
    return k;
}

struct CoulConsts {
    // FP64: V = ahc e^{-r/lambda}/r; fs = V (1/r + 1/lambda)/r
    double ahc, inv_lambda, L, hL;
    // MIXED: w = exp2(ru * c_exp) * ir; fs_u = w ir (1 + ir cAB), the
    // physical factor ir (ir/q^2 + 1/(lambda q)) divided by 1/(lambda q),
    // which f_scale carries (so the FMA takes the inline constant 1)
    float c_exp, cAB;
    double v_scale;  // alpha_hbarc / q              (V = v_scale * w)
    double f_scale;  // alpha_hbarc / (lambda q)     (F = f_scale * fs_u * du)
    // finite cutoff: keep r^2 < rc2 (FP64, fm^2); the mixed form decides on
    // its FP32 r^2 (q^2 units) below thr_lo or at/above thr_hi and on the
    // FP64 r^2 of the positions in between
    double rc2;
    float thr_lo, thr_hi;
};

__host__ __device__ inline CoulConsts make_coul_consts(const PairParams& pp)
{
    CoulConsts k{};
    k.ahc = pp.alpha_hbarc;
    k.inv_lambda = 1.0 / pp.lambda_s;
    k.L = pp.L;
    k.hL = 0.5 * pp.L;
    const double q = pp.L / 4294967296.0;
    k.c_exp = (float)(-q / pp.lambda_s * 1.4426950408889634);
    k.cAB = (float)(pp.lambda_s / q);
    k.v_scale = pp.alpha_hbarc / q;
    k.f_scale = pp.alpha_hbarc / (pp.lambda_s * q);
    k.rc2 = pp.r_coul * pp.r_coul;  // +inf when uncut
    // the FP32 r^2 of the fixed-point difference is within 2e-7 (rounding)
    // + 4 q / r (quantisation) of the FP64 one; the band is far wider
    const double rc2q = k.rc2 / (q * q);
    k.thr_lo = (float)(rc2q * (1.0 - 4e-6));
    k.thr_hi = (float)(rc2q * (1.0 + 4e-6));
    return k;
}

// ============================================================ policies ==
struct Fp64Policy {
    using Src = double4;
    using Lds = double4;
    static constexpr int TILE = TILE64;
    struct Acc {
        double fx = 0, fy = 0, fz = 0, e = 0;
        uint32_t np = 0;
    };
    using Part = Acc;
    using CAcc = double;  // Coulomb per-tile accumulator
    using CPart = double4;  // stored Coulomb partial sum
    __device__ static Lds load(const Src* s, int j) { return s[j]; }

    template <int MODE>
    __device__ static void pair(const Src& me, const Lds& s, double B_L, double B,
                                const NucConsts& k, Part& p, bool valid = true)
    {
        double dx = me.x - s.x, dy = me.y - s.y, dz = me.z - s.z;
        dx = nearest_image(dx, k.L, k.hL);
        dy = nearest_image(dy, k.L, k.hL);
        dz = nearest_image(dz, k.L, k.hL);
        double r2 = dx * dx + dy * dy + dz * dz;
        const bool in = valid && r2 < k.rc2;
        if (MODE == MODE_COUNT)
            p.np += in ? 1u : 0u;
        double g = in ? exp_nonpos(r2 * k.cg) : 0.0;
        double fs = g * fma(k.A2, g, B_L);
        p.fx = fma(fs, dx, p.fx);
        p.fy = fma(fs, dy, p.fy);
        p.fz = fma(fs, dz, p.fz);
        if (MODE != MODE_FORCE)
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
    __device__ static bool is_proton(const double4& s) { return s.w != 0.0; }
    __device__ static double f_scale(const NucConsts&) { return 1.0; }
    __device__ static double bl(const NucConsts& k, bool like) { return like ? k.Bl_L : k.Bu_L; }
    __device__ static double bv(const NucConsts& k, bool like) { return like ? k.Bl : k.Bu; }
    // Pair coefficients of one target in the compacting items: by the
    // source's species (sources of a tile are protons first, pu).
    struct Coefs {
        double BLp, BLn, Bp, Bn;
    };
    __device__ static Coefs coefs(const NucConsts& k, bool tprot)
    {
        return Coefs{bl(k, tprot), bl(k, !tprot), bv(k, tprot), bv(k, !tprot)};
    }
    __device__ static Lds tile_entry(const Lds& e) { return e; }
    template <int MODE>
    __device__ static void pair_c(const Src& me, const Lds& s, const Coefs& c, bool pu,
                                  const NucConsts& k, Part& p, bool valid)
    {
        pair<MODE>(me, s, pu ? c.BLp : c.BLn, pu ? c.Bp : c.Bn, k, p, valid);
    }

    template <bool E>
    __device__ static void coul(const Src& me, const Lds& s, bool self, const CoulConsts& k,
                                CAcc& fx, CAcc& fy, CAcc& fz, CAcc& e)
    {
        double dx = me.x - s.x, dy = me.y - s.y, dz = me.z - s.z;
        dx = nearest_image(dx, k.L, k.hL);
        dy = nearest_image(dy, k.L, k.hL);
        dz = nearest_image(dz, k.L, k.hL);
        double r2 = dx * dx + dy * dy + dz * dz;
        r2 = self ? 1e300 : r2;
        double ir = rsqrt_fast(r2);
        double r = r2 * ir;
        double v = k.ahc * exp_nonpos(-r * k.inv_lambda) * ir;
        double fs = v * (ir + k.inv_lambda) * ir;
        fx = fma(fs, dx, fx);
        fy = fma(fs, dy, fy);
        fz = fma(fs, dz, fz);
        if (E)
            e += v;
    }
    // Pairwise form: the difference vector, the force factor fs (force on
    // the first particle = fs d, on the second -fs d) and the pair energy w.
    __device__ static void coul_pair(const Src& me, const Src& s, const CoulConsts& k, CAcc& dx,
                                     CAcc& dy, CAcc& dz, CAcc& fs, CAcc& w)
    {
        dx = me.x - s.x;
        dy = me.y - s.y;
        dz = me.z - s.z;
        dx = nearest_image(dx, k.L, k.hL);
        dy = nearest_image(dy, k.L, k.hL);
        dz = nearest_image(dz, k.L, k.hL);
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double ir = rsqrt_fast(r2);
        const double r = r2 * ir;
        w = k.ahc * exp_nonpos(-r * k.inv_lambda) * ir;
        fs = w * (ir + k.inv_lambda) * ir;
    }
    __device__ static double coul_fscale(const CoulConsts&) { return 1.0; }
    __device__ static double coul_vscale(const CoulConsts&) { return 1.0; }
    // Finite Coulomb cutoff: r^2 as the definition forms it (strict nearest
    // image, (dx dx + dy dy) + dz dz, no fused multiply-add), compared with
    // rc2; never undecided.
    __device__ static bool coul_cut_in(const Src& me, const Lds& s, const CoulConsts& k,
                                       bool& undecided)
    {
        const double dx = nearest_image(me.x - s.x, k.L, k.hL);
        const double dy = nearest_image(me.y - s.y, k.L, k.hL);
        const double dz = nearest_image(me.z - s.z, k.L, k.hL);
        undecided = false;
        return r2_exact(dx, dy, dz) < k.rc2;
    }
    // 32-bit fixed-point coordinates (x/L * 2^32) for the screening pass
    __device__ static uint3 fixed(const Src& s, const NucConsts& k)
    {
        return make_uint3((uint32_t)(uint64_t)(s.x * k.qscale), (uint32_t)(uint64_t)(s.y * k.qscale),
                          (uint32_t)(uint64_t)(s.z * k.qscale));
    }
    static constexpr int CTILE = 512;  // sources per tile in the compacting kernel
    static constexpr int DRAIN_U = 2;  // listed pairs per drain round
    // targets per lane of the off-diagonal pairwise Coulomb items (four
    // would take the kernel past 128 VGPRs)
    static constexpr int COUL_NT = 2;
    static constexpr int STAGE_PER_THREAD = 1;  // candidates per thread per staging round
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
    using CAcc = float;
    // stored Coulomb partial sum: an item's sums are FP32 accumulators (or
    // at most a few tiles of them), so FP32 storage keeps their precision
    using CPart = float4;
    __device__ static Lds load(const Src* s, int j)
    {
        return reinterpret_cast<const uint4*>(s)[j];
    }

    template <int MODE>
    __device__ static void pair(const Src& me, const Lds& s, float B_L, float B,
                                const NucConsts& k, Part& p, bool valid = true)
    {
        float dx = (float)(int32_t)(me.x - s.x);
        float dy = (float)(int32_t)(me.y - s.y);
        float dz = (float)(int32_t)(me.z - s.z);
        float r2 = dx * dx + dy * dy + dz * dz;
        const bool in = valid && r2 < k.thr_q;
        if (MODE == MODE_COUNT)
            p.np += in ? 1u : 0u;
        r2 = in ? r2 : 3.0e38f;  // exp2 underflows to exactly 0 outside the cutoff
        float g = __builtin_amdgcn_exp2f(r2 * k.cgq);
        float fs = g * fmaf(k.A2f, g, B_L);
        p.fx = fmaf(fs, dx, p.fx);
        p.fy = fmaf(fs, dy, p.fy);
        p.fz = fmaf(fs, dz, p.fz);
        if (MODE != MODE_FORCE)
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
    __device__ static bool is_proton(const Q4& s) { return s.w != 0u; }
    __device__ static bool is_proton(const uint4& s) { return s.w != 0u; }
    __device__ static double f_scale(const NucConsts& k) { return k.q; }
    __device__ static float bl(const NucConsts& k, bool like) { return like ? k.Blf_L : k.Buf_L; }
    __device__ static float bv(const NucConsts& k, bool like) { return like ? k.Blf : k.Buf; }
    // Pair coefficients of one target in the compacting items, as one FMA
    // per pair: a tile entry carries its species as s_j = +1 (proton) or -1
    // (neutron) in FP32, and with s_i the target's, the like/unlike
    // coefficient is m + (h s_i) s_j, m and h the mean and half-difference
    // of the like and unlike values (rounded once to FP32 each).
    struct Coefs {
        float hL, mL, h, m;
    };
    __device__ static Coefs coefs(const NucConsts& k, bool tprot)
    {
        const double s = tprot ? 1.0 : -1.0;
        return Coefs{(float)(0.5 * ((double)k.Blf_L - (double)k.Buf_L) * s),
                     (float)(0.5 * ((double)k.Blf_L + (double)k.Buf_L)),
                     (float)(0.5 * ((double)k.Blf - (double)k.Buf) * s),
                     (float)(0.5 * ((double)k.Blf + (double)k.Buf))};
    }
    __device__ static Lds tile_entry(const Lds& e)
    {
        return make_uint4(e.x, e.y, e.z, __float_as_uint(e.w != 0u ? 1.0f : -1.0f));
    }
    template <int MODE>
    __device__ static void pair_c(const Src& me, const Lds& s, const Coefs& c, bool,
                                  const NucConsts& k, Part& p, bool valid)
    {
        const float sj = __uint_as_float(s.w);
        pair<MODE>(me, s, fmaf(sj, c.hL, c.mL), fmaf(sj, c.h, c.m), k, p, valid);
    }

    template <bool E>
    __device__ static void coul(const Src& me, const Lds& s, bool self, const CoulConsts& k,
                                CAcc& fx, CAcc& fy, CAcc& fz, CAcc& e)
    {
        float dx = (float)(int32_t)(me.x - s.x);
        float dy = (float)(int32_t)(me.y - s.y);
        float dz = (float)(int32_t)(me.z - s.z);
        float r2 = dx * dx + dy * dy + dz * dz;
        r2 = self ? 3.0e38f : r2;
        float ir = __builtin_amdgcn_rsqf(r2);
        float ru = r2 * ir;
        float w = __builtin_amdgcn_exp2f(ru * k.c_exp) * ir;
        float fs = w * ir * fmaf(ir, k.cAB, 1.0f);
        fx = fmaf(fs, dx, fx);
        fy = fmaf(fs, dy, fy);
        fz = fmaf(fs, dz, fz);
        if (E)
            e += w;
    }
    __device__ static void coul_pair(const Src& me, const Src& s, const CoulConsts& k, CAcc& dx,
                                     CAcc& dy, CAcc& dz, CAcc& fs, CAcc& w)
    {
        dx = (float)(int32_t)(me.x - s.x);
        dy = (float)(int32_t)(me.y - s.y);
        dz = (float)(int32_t)(me.z - s.z);
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float ir = __builtin_amdgcn_rsqf(r2);
        const float ru = r2 * ir;
        w = __builtin_amdgcn_exp2f(ru * k.c_exp) * ir;
        fs = w * ir * fmaf(ir, k.cAB, 1.0f);
    }
    __device__ static double coul_fscale(const CoulConsts& k) { return k.f_scale; }
    __device__ static double coul_vscale(const CoulConsts& k) { return k.v_scale; }
    // Finite Coulomb cutoff on the FP32 r^2 of the exact fixed-point
    // difference; pairs in the narrow band around the cutoff are left to the
    // FP64 test on the positions (coul_cut_exact).
    __device__ static bool coul_cut_in(const Src& me, const Lds& s, const CoulConsts& k,
                                       bool& undecided)
    {
        const float dx = (float)(int32_t)(me.x - s.x);
        const float dy = (float)(int32_t)(me.y - s.y);
        const float dz = (float)(int32_t)(me.z - s.z);
        const float r2 = dx * dx + dy * dy + dz * dz;
        undecided = r2 >= k.thr_lo && r2 < k.thr_hi;
        return r2 < k.thr_lo;
    }
    __device__ static uint3 fixed(const Src& s, const NucConsts&)
    {
        return make_uint3(s.x, s.y, s.z);
    }
    // 512 sources per tile keep the compacting item's LDS (tile, screen
    // coordinates, pair lists, scratch) under 160 KB / 6: with <= 80 VGPRs,
    // six workgroups per CU
    static constexpr int CTILE = 512;
    static constexpr int DRAIN_U = 4;
    static constexpr int STAGE_PER_THREAD = 2;
    // targets per lane of the off-diagonal pairwise Coulomb items
    static constexpr int COUL_NT = 4;
};

// LDS bytes a work item needs (the caller provides at least this much,
// 16-byte aligned).
template <class P>
constexpr int coulomb_lds_bytes() { return P::TILE * (int)sizeof(typename P::Lds); }
template <class P>
constexpr int nuclear_lds_bytes()
{
    return P::TILE * (int)sizeof(typename P::Lds) + 54 * 4 + 55 * 4 + 4 + 4 * 8 + 4 * 8;
}
// Per-lane pair-list capacity of the compacting kernel.  Entry c of thread
// t is the 16-bit word c * WG + t: whatever the lanes' counts, a wavefront's
// appends then fall in one bank per pair of lanes, and a drain round reads
// one row.
constexpr int NUC_CAP = 26;
constexpr int NUC_U = 4;     // candidates per lane between list-fill checks

// A Coulomb partial sum (Fx, Fy, Fz, sum V), already scaled to MeV/fm and
// MeV, stored as double4 or float4.
__device__ __forceinline__ void store_part(double4* p, double x, double y, double z, double w)
{
    *p = make_double4(x, y, z, w);
}
__device__ __forceinline__ void store_part(float4* p, double x, double y, double z, double w)
{
    *p = make_float4((float)x, (float)y, (float)z, (float)w);
}

// Per-particle fixed-point accumulators: 64-bit integers in units of 2^-43
// MeV/fm (and MeV), added with integer atomics, so a particle's total does
// not depend on the order in which work items add to it.  One added value is
// rounded to 2^-44 (1e-13 MeV/fm); the representable total is +-2^20.
constexpr double REACT_PER_UNIT = 8796093022208.0;    // 2^43 units per MeV/fm
constexpr double REACT_UNIT = 1.0 / 8796093022208.0;  // MeV/fm per unit

__device__ __forceinline__ unsigned long long react_fixed(double x)
{
    return (unsigned long long)(long long)llrint(x * REACT_PER_UNIT);
}

// Where a pairwise Coulomb item puts one proton's sum over the item (MeV/fm
// and MeV).  A partial array: part[X * Z + p], X the other super-block of the
// item, summed by the combine in super-block order.  FixedPart: the proton's
// fixed-point accumulators acc[c * stride + p], c = x, y, z, V (the energy
// only when E), so no partials exist; a sum that is not finite or not below
// 2^19 in magnitude is not added and sets the error word instead.  The
// component-major layout puts a wavefront's 64 consecutive protons of one
// component in 512 contiguous bytes.
struct FixedPart {
    unsigned long long* acc;
    uint32_t* err;
    int64_t stride;
};
template <bool E, class PT>
__device__ __forceinline__ void put_part(PT* __restrict__ part, int X, int Z, int p, double x,
                                         double y, double z, double w)
{
    store_part(&part[(int64_t)X * Z + p], x, y, z, w);
}
template <bool E>
__device__ __forceinline__ void put_part(const FixedPart& fp, int, int, int p, double x,
                                         double y, double z, double w)
{
    constexpr double lim = 524288.0;  // 2^19
    if (!(fabs(x) < lim && fabs(y) < lim && fabs(z) < lim && (!E || fabs(w) < lim))) {
        atomicOr(fp.err, ERR_NONFINITE_FORCE);
        return;
    }
    unsigned long long* a = fp.acc + p;
    atomicAdd(a, react_fixed(x));
    atomicAdd(a + fp.stride, react_fixed(y));
    atomicAdd(a + 2 * fp.stride, react_fixed(z));
    if (E)
        atomicAdd(a + 3 * fp.stride, react_fixed(w));
}

// ============================================================ Coulomb ==
// Targets are the proton slots [tb, tb + WG) ∩ [0, Z); sources the slots
// [split * per_split, ...).  Writes part[split * Z + t] = (Fx, Fy, Fz, sum V).
// The FP64 cutoff test of the definition on the positions of proton slots
// a and b (the undecided band of the mixed form's test).
__device__ inline bool coul_cut_exact(const CoulCut& cc, const CoulConsts& k, int a, int b)
{
    const int64_t ia = cc.perm ? cc.perm[a] : a, ib = cc.perm ? cc.perm[b] : b;
    const double dx = nearest_image(cc.pos[3 * ia + 0] - cc.pos[3 * ib + 0], k.L, k.hL);
    const double dy = nearest_image(cc.pos[3 * ia + 1] - cc.pos[3 * ib + 1], k.L, k.hL);
    const double dz = nearest_image(cc.pos[3 * ia + 2] - cc.pos[3 * ib + 2], k.L, k.hL);
    return r2_exact(dx, dy, dz) < k.rc2;
}

// CUT: a finite Coulomb cutoff (k.rc2): a pair outside enters as the self
// pair does (exactly zero); cc.count, when set, counts the ordered pairs
// kept.
template <class P, bool E = true, class PT = double4, bool CUT = false>
__device__ void coulomb_item(const typename P::Src* __restrict__ stg, int Z, int per_split,
                             const CoulConsts& k, PT* __restrict__ part, int tblock,
                             int split, char* lds, const CoulCut& cc = CoulCut{})
{
    using Lds = typename P::Lds;
    Lds* tile = reinterpret_cast<Lds*>(lds);
    const int t = tblock * WG + threadIdx.x;
    const int j0 = split * per_split;
    const int j1 = min(Z, j0 + per_split);
    const int tb0 = tblock * WG, tb1 = min(Z, tb0 + WG);
    const typename P::Src me = stg[t < Z ? t : 0];
    double fx = 0, fy = 0, fz = 0, e = 0;
    unsigned long long kept = 0;
    for (int base = j0; base < j1; base += P::TILE) {
        const int cnt = min(P::TILE, j1 - base);
        for (int q = threadIdx.x; q < cnt; q += WG)
            tile[q] = P::load(stg, base + q);
        __syncthreads();
        typename P::CAcc ax = 0, ay = 0, az = 0, ae = 0;
        if constexpr (CUT) {
            for (int q = 0; q < cnt; ++q) {
                bool undecided;
                bool in = P::coul_cut_in(me, tile[q], k, undecided);
                if (undecided && t < Z)
                    in = coul_cut_exact(cc, k, t, base + q);
                const bool skip = base + q == t || !in;
                kept += (!skip && t < Z) ? 1ull : 0ull;
                P::template coul<E>(me, tile[q], skip, k, ax, ay, az, ae);
            }
        } else if (base < tb1 && base + cnt > tb0) {
            for (int q = 0; q < cnt; ++q)
                P::template coul<E>(me, tile[q], base + q == t, k, ax, ay, az, ae);
        } else {
#pragma unroll 4
            for (int q = 0; q < cnt; ++q)
                P::template coul<E>(me, tile[q], false, k, ax, ay, az, ae);
        }
        fx += (double)ax;
        fy += (double)ay;
        fz += (double)az;
        e += (double)ae;
        __syncthreads();
    }
    if (t < Z) {
        const double fs = P::coul_fscale(k), vs = P::coul_vscale(k);
        store_part(&part[(int64_t)split * Z + t], fx * fs, fy * fs, fz * fs, e * vs);
    }
    if constexpr (CUT) {
        if (cc.count) {
            for (int m = 32; m >= 1; m >>= 1)
                kept += __shfl_xor(kept, m, 64);
            if ((threadIdx.x & 63) == 0)
                atomicAdd(cc.count, kept);
        }
    }
}

// ============================================== Coulomb, pairwise form ==
// Each unordered proton pair is evaluated once (Newton's third law).
// Protons (sorted slots [0, Z)) are taken in blocks of 64, one per lane of
// a wavefront, and super-blocks of CP_SUPER blocks.  A work item is a
// super-block pair (A, B), A <= B, and one workgroup: wavefront w owns the
// target block I = CP_SUPER A + w and visits every source block J of B
// (J >= I when A == B).  Each lane holds its target and one source; it
// evaluates the pair, adds the force to its target and the reaction to the
// source's accumulator, then the sources and their accumulators move: one
// column along the lane's row of 16 (a row rotation), and after every 16
// rotations one row down (a 16-lane shift), so an off-diagonal block pair
// takes 4 x 16 steps and leaves every source accumulator at its own lane.
// Write a held source's offset from its lane as (row, column) offsets
// (rho, c).  For a diagonal block (J = I) each unordered pair appears at
// two opposite offsets, so one of each is visited: (0, 1..8), (1, all 16),
// (2, 8..15 and 0), where the self-opposite offsets (0, 8), (2, 8) and
// (2, 0) are evaluated by half of the lanes; the accumulators then sit two
// rows away from home and move back with one 32-lane shift.  The schedule
// does not depend on which way the hardware rotates.
// Partials: proton p of super-block X receives from item (A, B) the sum of
// its contributions as part[Y][p], Y the other super-block of the item
// (Y = X when A == B), i.e. exactly one partial per super-block, which the
// combine adds in super-block order; or every item adds that sum into the
// proton's fixed-point accumulator (FixedPart).
constexpr int CP_SUPER = 4;  // blocks per super-block (= wavefronts per workgroup)
static_assert(CP_SUPER * 64 == WG, "one wavefront per block of a super-block");

__host__ __device__ inline int coulomb_pair_supers(int64_t Z) { return (int)((Z + 255) / 256); }
__host__ __device__ inline int64_t coulomb_pair_items(int64_t Z)
{
    const int64_t S = coulomb_pair_supers(Z);
    return S * (S + 1) / 2;
}

// Row rotation: DPP row_ror:1 (each row of 16 lanes rotates by one; every
// lane has a source lane, so no old value is needed).
__device__ __forceinline__ uint32_t row_rotate(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x121, 0xF, 0xF, true);
}
__device__ __forceinline__ float row_rotate(float v)
{
    return __builtin_bit_cast(float, row_rotate(__builtin_bit_cast(uint32_t, v)));
}
__device__ __forceinline__ double row_rotate(double v)
{
    uint2 u = __builtin_bit_cast(uint2, v);
    u.x = row_rotate(u.x);
    u.y = row_rotate(u.y);
    return __builtin_bit_cast(double, u);
}
// Row shift: lane l takes the value of lane l + 16 (mod 64).
__device__ __forceinline__ uint32_t row_shift(uint32_t v)
{
    return (uint32_t)__shfl((int)v, (__lane_id() + 16) & 63);
}
__device__ __forceinline__ float row_shift(float v) { return __shfl(v, (__lane_id() + 16) & 63); }
__device__ __forceinline__ double row_shift(double v)
{
    return __shfl(v, (__lane_id() + 16) & 63);
}
template <class T>
__device__ __forceinline__ Q4 move_src(const Q4& s, T op)
{
    Q4 r;
    r.x = op(s.x);
    r.y = op(s.y);
    r.z = op(s.z);
    r.w = s.w;
    return r;
}
template <class T>
__device__ __forceinline__ double4 move_src(const double4& s, T op)
{
    return make_double4(op(s.x), op(s.y), op(s.z), s.w);
}

template <class P>
constexpr int coulomb_pair_lds_bytes()
{
    return CP_SUPER * CP_SUPER * 64 * 4 * (int)sizeof(typename P::CAcc);
}

// Item index -> super-block pair (A, B), A <= B, row-major over A.
__host__ __device__ inline void coulomb_pair_ab(int item, int S, int* A_out, int* B_out)
{
    int A = 0, r = item;
    while (r >= S - A) {
        r -= S - A;
        ++A;
    }
    *A_out = A;
    *B_out = A + r;
}

// Off-diagonal item (A < B) whose eight blocks are all full: NT targets per
// lane (NT = 2 or 4).  The four target blocks of A form 4 / NT groups of NT
// blocks; wave w holds group w % (4 / NT) (one target of each of its blocks
// per lane) and meets its share of B's source blocks, 4 / NT of them, one
// after the other.  Each source and its reaction accumulator meet all of the
// lane's targets before they move, so one set of row rotations serves NT
// pairs.  A target block is covered by NT wavefronts, a source block by
// 4 / NT; where a block has more than one, their FP32 sums meet in LDS and
// are added in FP64 in wavefront order.  The pairs evaluated and the
// partials written are those of the one-target schedule.
template <class P, bool E, class PH, int NT = P::COUL_NT>
__device__ void coulomb_pair_item_mt(const typename P::Src* __restrict__ stg, int Z,
                                     const CoulConsts& k, PH part, int A, int Bs, char* lds)
{
    static_assert(NT == 2 || NT == 4, "two or four targets per lane");
    constexpr int TG = CP_SUPER / NT;   // target groups = source blocks per wave
    using Src = typename P::Src;
    using CA = typename P::CAcc;
    // [wave][NT target blocks][lane][4], then (TG > 1) [wave][TG source blocks][lane][4]
    CA* acc_t = reinterpret_cast<CA*>(lds);
    CA* acc_s = acc_t + CP_SUPER * NT * 64 * 4;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int I0 = CP_SUPER * A + NT * (w % TG), J0 = CP_SUPER * Bs + TG * (w / TG);
    Src me[NT];
    CA tx[NT], ty[NT], tz[NT], te[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        me[i] = stg[(I0 + i) * 64 + lane];
        tx[i] = ty[i] = tz[i] = te[i] = CA(0);
    }
    const double fsc = P::coul_fscale(k), vsc = P::coul_vscale(k);
#pragma unroll 1
    for (int jj = 0; jj < TG; ++jj) {
        Src src = stg[(J0 + jj) * 64 + lane];
        CA sx = 0, sy = 0, sz = 0, se = 0;
#pragma unroll 1
        for (int rho = 0; rho < 4; ++rho) {
            // a short loop body: the fused kernel's item code shares the
            // instruction cache
#pragma unroll 8 / NT
            for (int c = 0; c < 16; ++c) {
#pragma unroll
                for (int i = 0; i < NT; ++i) {
                    CA dx, dy, dz, fs, wv;
                    P::coul_pair(me[i], src, k, dx, dy, dz, fs, wv);
                    tx[i] += fs * dx;
                    ty[i] += fs * dy;
                    tz[i] += fs * dz;
                    sx -= fs * dx;
                    sy -= fs * dy;
                    sz -= fs * dz;
                    if (E) {
                        te[i] += wv;
                        se += wv;
                    }
                }
                src = move_src(src, [](auto v) { return row_rotate(v); });
                sx = row_rotate(sx);
                sy = row_rotate(sy);
                sz = row_rotate(sz);
                if (E)
                    se = row_rotate(se);
            }
            src = move_src(src, [](auto v) { return row_shift(v); });
            sx = row_shift(sx);
            sy = row_shift(sy);
            sz = row_shift(sz);
            if (E)
                se = row_shift(se);
        }
        if (TG == 1) {
            // this wave alone covers the source block: its partial from A
            const int p = (J0 + jj) * 64 + lane;
            put_part<E>(part, A, Z, p, (double)sx * fsc, (double)sy * fsc,
                        (double)sz * fsc, (double)se * vsc);
        } else {
            CA* a = acc_s + ((w * TG + jj) * 64 + lane) * 4;
            a[0] = sx;
            a[1] = sy;
            a[2] = sz;
            a[3] = se;
        }
    }
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        CA* a = acc_t + ((w * NT + i) * 64 + lane) * 4;
        a[0] = tx[i];
        a[1] = ty[i];
        a[2] = tz[i];
        a[3] = te[i];
    }
    __syncthreads();
    // wavefront b writes block b of A (targets; its partial from B) and, when
    // a source block has several wavefronts, block b of B (its partial from A)
    {
        const int b = w, g = b / NT, slot = b % NT;  // waves g + TG m hold target block b
        double fx = 0, fy = 0, fz = 0, fe = 0;
        for (int m = 0; m < NT; ++m) {
            const CA* a = acc_t + (((g + TG * m) * NT + slot) * 64 + lane) * 4;
            fx += (double)a[0];
            fy += (double)a[1];
            fz += (double)a[2];
            fe += (double)a[3];
        }
        const int t = (CP_SUPER * A + b) * 64 + lane;
        put_part<E>(part, Bs, Z, t, fx * fsc, fy * fsc, fz * fsc, fe * vsc);
    }
    if (TG > 1) {
        const int b = w, s0 = (b / TG) * TG, slot = b % TG;  // waves s0 .. s0 + TG - 1
        double fx = 0, fy = 0, fz = 0, fe = 0;
        for (int i = 0; i < TG; ++i) {
            const CA* a = acc_s + (((s0 + i) * TG + slot) * 64 + lane) * 4;
            fx += (double)a[0];
            fy += (double)a[1];
            fz += (double)a[2];
            fe += (double)a[3];
        }
        const int p = (CP_SUPER * Bs + b) * 64 + lane;
        put_part<E>(part, A, Z, p, fx * fsc, fy * fsc, fz * fsc, fe * vsc);
    }
    __syncthreads();
}

// part: a partial array (float4* / double4*) or a FixedPart (put_part).
template <class P, bool E, class PH>
__device__ void coulomb_pair_item(const typename P::Src* __restrict__ stg, int Z,
                                  const CoulConsts& k, PH part, int item, char* lds)
{
    using Src = typename P::Src;
    using CA = typename P::CAcc;
    CA* acc = reinterpret_cast<CA*>(lds);  // [wave][block of B][lane][4]
    const int S = coulomb_pair_supers(Z);
    int A, Bs;
    coulomb_pair_ab(item, S, &A, &Bs);
    if (A != Bs && CP_SUPER * Bs + CP_SUPER <= Z / 64) {  // A < B, every block full
        coulomb_pair_item_mt<P, E, PH>(stg, Z, k, part, A, Bs, lds);
        return;
    }
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int nb = (Z + 63) / 64;
    for (int i = tid; i < CP_SUPER * CP_SUPER * 64 * 4; i += WG)
        acc[i] = CA(0);
    __syncthreads();
    const int I = CP_SUPER * A + w;  // wave-uniform
    if (I < nb) {
        const int t = I * 64 + lane;
        const bool tv = t < Z;
        const Src me = stg[tv ? t : Z - 1];
        CA tx = 0, ty = 0, tz = 0, te = 0;
        const int J0 = A == Bs ? I : CP_SUPER * Bs;
        const int J1 = min(CP_SUPER * Bs + CP_SUPER, nb);
        const bool low_col = (lane & 15) < 8, low_row = lane < 32;
        for (int J = J0; J < J1; ++J) {
            const int s0 = J * 64 + lane;
            Src src = stg[s0 < Z ? s0 : Z - 1];
            int sidx = s0;  // travels with the source (validity of partial blocks)
            CA sx = 0, sy = 0, sz = 0, se = 0;
            const bool full = I * 64 + 64 <= Z && J * 64 + 64 <= Z;  // wave-uniform
            auto one = [&](bool valid) {
                CA dx, dy, dz, fs, wv;
                P::coul_pair(me, src, k, dx, dy, dz, fs, wv);
                fs = valid ? fs : CA(0);
                tx += fs * dx;
                ty += fs * dy;
                tz += fs * dz;
                sx -= fs * dx;
                sy -= fs * dy;
                sz -= fs * dz;
                if (E) {
                    wv = valid ? wv : CA(0);
                    te += wv;
                    se += wv;
                }
            };
            auto rot = [&]() {
                src = move_src(src, [](auto v) { return row_rotate(v); });
                sx = row_rotate(sx);
                sy = row_rotate(sy);
                sz = row_rotate(sz);
                if (E)
                    se = row_rotate(se);
                if (!full)
                    sidx = (int)row_rotate((uint32_t)sidx);
            };
            auto down = [&]() {
                src = move_src(src, [](auto v) { return row_shift(v); });
                sx = row_shift(sx);
                sy = row_shift(sy);
                sz = row_shift(sz);
                if (E)
                    se = row_shift(se);
                if (!full)
                    sidx = (int)row_shift((uint32_t)sidx);
            };
            auto ok = [&](bool half_ok) { return full ? half_ok : (tv && sidx < Z && half_ok); };
            if (J != I) {
                for (int rho = 0; rho < 4; ++rho) {
                    if (full) {
                        for (int c = 0; c < 16; ++c) {
                            one(true);
                            rot();
                        }
                    } else {
                        for (int c = 0; c < 16; ++c) {
                            one(tv && sidx < Z);
                            rot();
                        }
                    }
                    down();
                }
            } else {
                // (0, 1..8)
                for (int c = 1; c <= 8; ++c) {
                    rot();
                    one(ok(c < 8 || low_col));
                }
                // (1, 8..15, 0..7)
                down();
                one(ok(true));
                for (int c = 1; c < 16; ++c) {
                    rot();
                    one(ok(true));
                }
                // (2, 8), (2, 9..15), (2, 0)
                rot();
                down();
                one(ok(low_col));
                for (int c = 1; c < 8; ++c) {
                    rot();
                    one(ok(true));
                }
                rot();
                one(ok(low_row));
                // two rows from home: one 32-lane shift brings them back
                sx = __shfl(sx, (lane + 32) & 63);
                sy = __shfl(sy, (lane + 32) & 63);
                sz = __shfl(sz, (lane + 32) & 63);
                if (E)
                    se = __shfl(se, (lane + 32) & 63);
            }
            CA* a = acc + ((w * CP_SUPER + (J - CP_SUPER * Bs)) * 64 + lane) * 4;
            a[0] += sx;
            a[1] += sy;
            a[2] += sz;
            a[3] += se;
        }
        const double fsc = P::coul_fscale(k), vsc = P::coul_vscale(k);
        if (A != Bs) {
            if (tv)
                put_part<E>(part, Bs, Z, t, (double)tx * fsc, (double)ty * fsc,
                            (double)tz * fsc, (double)te * vsc);
        } else {
            CA* a = acc + ((w * CP_SUPER + (I - CP_SUPER * A)) * 64 + lane) * 4;
            a[0] += tx;
            a[1] += ty;
            a[2] += tz;
            a[3] += te;
        }
    }
    __syncthreads();
    // the source side (and, for A == B, everything) of block b of B, summed
    // over the wavefronts in fixed order
    {
        const int b = tid >> 6;
        const int p = (CP_SUPER * Bs + b) * 64 + lane;
        if (p < Z) {
            double fx = 0, fy = 0, fz = 0, e = 0;
            for (int v = 0; v < CP_SUPER; ++v) {
                const CA* a = acc + ((v * CP_SUPER + b) * 64 + lane) * 4;
                fx += (double)a[0];
                fy += (double)a[1];
                fz += (double)a[2];
                e += (double)a[3];
            }
            const double fsc = P::coul_fscale(k), vsc = P::coul_vscale(k);
            put_part<E>(part, A, Z, p, fx * fsc, fy * fsc, fz * fsc, e * vsc);
        }
    }
    __syncthreads();
}

// ------------------------------------------------- Coulomb partial sums --
// Every proton p receives S partial sums part[s * Z + p] (s = 0..S-1).
// Sequential sum from zero in s order (the nuclear epilogue of the unfused
// form and the batched combine use it).
template <class PT>
__device__ inline double4 coul_sum_seq(const PT* __restrict__ part, int S, int Z, int p)
{
    double x = 0.0, y = 0.0, z = 0.0, w = 0.0;
    for (int s = 0; s < S; ++s) {
        const PT v = part[(int64_t)s * Z + p];
        x += (double)v.x;
        y += (double)v.y;
        z += (double)v.z;
        w += (double)v.w;
    }
    return make_double4(x, y, z, w);
}

// ============================================================ nuclear ==
struct NucArgs {
    const int32_t* start;    // [2 C sub + 1]
    const int32_t* items;    // [2*item_max]
    const int32_t* perm;     // [n] slot -> output index of F and E, or null (slot)
    int nc, C;
    int sub;                 // bins per cell and species (1 or 8)
    int Z;
    const void* coul_part;   // typename P::CPart [S * Z]: Coulomb partials
    int S;                   // Coulomb partials per proton to add (0 = none)
    double* force;           // [n][3] at perm[slot] (caller order) or the slot
    double* epot;            // [n] or null
    double* vel;             // [n][3] or null: apply the half kick
    double hdtm, mass;
    double* ke_part;         // [item_max] or null
    unsigned long long* pairs;
    uint32_t* err;
    double4* fnuc;           // batch form: raw nuclear (F, V) per sorted slot, no epilogue
    unsigned long long* react;  // [4][react_stride] fixed-point accumulators per sorted
                                // slot (x, y, z, V): Newton-3 reactions (variant 4) and
                                // the fixed-point form's Coulomb sums
    int64_t react_stride;
};

template <class P, bool NUC, int MODE>
__device__ void nuclear_item(const typename P::Src* __restrict__ stg, const NucArgs& A,
                             const NucConsts& k, int item, char* lds)
{
    using Lds = typename P::Lds;
    Lds* tile = reinterpret_cast<Lds*>(lds);
    int* seg_beg = reinterpret_cast<int*>(lds + P::TILE * sizeof(Lds));
    int* seg_off = seg_beg + 54;
    double* ke_red = reinterpret_cast<double*>(
        (reinterpret_cast<uintptr_t>(seg_off + 55) + 7) & ~uintptr_t(7));
    unsigned long long* np_red = reinterpret_cast<unsigned long long*>(ke_red + WG / 64);

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
            const int b = (sp * C + (nz * nc + ny) * nc + nx) * A.sub;
            beg = A.start[b];
            len = A.start[b + A.sub] - beg;
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

    const int ps = A.start[c * A.sub], npc = A.start[(c + 1) * A.sub] - ps;
    const int ns = A.start[(C + c) * A.sub], mc = npc + (A.start[(C + c + 1) * A.sub] - ns);
    const int tl = tid / NUC_TPT, q = tid % NUC_TPT;
    const int tidx = chunk * NUC_CHUNK + tl;
    const bool active = tidx < mc;
    const int slot = active ? (tidx < npc ? ps + tidx : ns + (tidx - npc)) : 0;
    const bool tprot = tidx < npc;
    const typename P::Src me = stg[slot];

    typename P::Acc acc;
    if (NUC) {
        const int total = seg_off[54], np_tot = seg_off[27];
        const auto BLp = P::bl(k, tprot), Bp = P::bv(k, tprot);    // proton sources
        const auto BLn = P::bl(k, !tprot), Bn = P::bv(k, !tprot);  // neutron sources
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
                P::template pair<MODE>(me, tile[j], BLp, Bp, k, part);
            for (int j = kb + q; j < cnt; j += NUC_TPT)
                P::template pair<MODE>(me, tile[j], BLn, Bn, k, part);
            P::fold(acc, part);
            __syncthreads();
        }
#pragma unroll
        for (int m = 1; m < NUC_TPT; m <<= 1) {
            acc.fx += __shfl_xor(acc.fx, m, NUC_TPT);
            acc.fy += __shfl_xor(acc.fy, m, NUC_TPT);
            acc.fz += __shfl_xor(acc.fz, m, NUC_TPT);
            acc.e += __shfl_xor(acc.e, m, NUC_TPT);
            if (MODE == MODE_COUNT)
                acc.np += __shfl_xor(acc.np, m, NUC_TPT);
        }
    }

    const double fsc = P::f_scale(k);
    double ke = 0.0;
    unsigned long long npairs = 0;
    if (active && q == 0) {
        if (MODE == MODE_COUNT)
            npairs = acc.np - 1u;  // minus the self pair
        // the self pair (r = 0) entered the sum with V(0) = a + b + c
        double V = NUC ? acc.e - k.self_v : 0.0;
        double Fx = acc.fx * fsc, Fy = acc.fy * fsc, Fz = acc.fz * fsc;
        if (A.fnuc) {
            // batch form: the combine pass adds the Coulomb partials and kicks
            A.fnuc[slot] = make_double4(Fx, Fy, Fz, V);
        } else {
            if (A.S > 0 && tprot) {
                const double4 cp = coul_sum_seq(
                    static_cast<const typename P::CPart*>(A.coul_part), A.S, A.Z, slot);
                Fx += cp.x;
                Fy += cp.y;
                Fz += cp.z;
                V += cp.w;
            }
            const int64_t id = A.perm ? A.perm[slot] : slot;
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
    }
    if (A.ke_part || MODE == MODE_COUNT) {
        // fixed-order block reduction (deterministic)
        for (int m = 32; m >= 1; m >>= 1) {
            ke += __shfl_xor(ke, m, 64);
            if (MODE == MODE_COUNT)
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
            if (A.ke_part && !A.fnuc)
                A.ke_part[item] = s;
            if (MODE == MODE_COUNT)
                atomicAdd(A.pairs, sn);
        }
        __syncthreads();
    }
}


// ================================================ nuclear, compacting ==
// Same contract as nuclear_item, with a two-pass inner loop.  The
// neighbourhood is staged tile by tile, keeping only sources that can reach
// the bounding box of the chunk's targets.  Each lane then screens its share
// of the tile with a cheap conservative test on 16-bit truncated coordinates
// (packed 16-bit subtraction, which wraps to the nearest image, and a 2-wide
// integer dot product), appends the survivors to a private list in LDS, and
// evaluates the exact pair arithmetic only on listed pairs.  The screen never
// drops a pair inside the cutoff (|d_true| < |d_16| + 1 per axis), and the
// exact cutoff test of the pair arithmetic removes the false positives.
__device__ __forceinline__ int screen16(uint32_t me_xy16, uint32_t me_z, uint2 t)
{
    typedef short v2s __attribute__((ext_vector_type(2)));
    const v2s a = __builtin_bit_cast(v2s, me_xy16);
    const v2s b = __builtin_bit_cast(v2s, t.x);
    const v2s d = a - b;
    const int dz = ((int32_t)(me_z - t.y)) >> 16;
    return __builtin_amdgcn_sdot2(d, d, dz * dz, false);
}

// LDS scratch shared by the cell-item helpers below (after the tiles).
// Candidate-index buckets: bucket[b] is the neighbour bin holding candidate
// b * SEG_BUCKET (for the first SEG_BUCKETS * SEG_BUCKET candidates), so a
// candidate's bin is found from its bucket's bin by a short forward walk.
constexpr int SEG_BUCKET = 32;
constexpr int SEG_BUCKETS = WG;
struct ItemLds {
    int* seg_beg;   // [54] first sorted slot of each neighbour bin
    int* seg_off;   // [55] exclusive prefix of the bin lengths
    int* misc;      // [24] box lo/hi, per-wave kept counts
    double* ke_red;  // [WG/64]
    unsigned long long* np_red;  // [WG/64]
    uint8_t* bucket;  // [SEG_BUCKETS]
};
constexpr int ITEM_LDS_BYTES = 54 * 4 + 55 * 4 + 24 * 4 + 4 * 8 + 4 * 8 + 16 + SEG_BUCKETS;
__device__ inline ItemLds item_lds(char* p)
{
    ItemLds s;
    s.seg_beg = reinterpret_cast<int*>(p);
    s.seg_off = s.seg_beg + 54;
    s.misc = s.seg_off + 55;
    // the buckets right after misc (a plain offset, so the compiler keeps
    // them in LDS), then the 8-byte aligned reductions
    s.bucket = reinterpret_cast<uint8_t*>(s.misc + 24);
    s.ke_red = reinterpret_cast<double*>(
        (reinterpret_cast<uintptr_t>(s.bucket + SEG_BUCKETS) + 7) & ~uintptr_t(7));
    s.np_red = reinterpret_cast<unsigned long long*>(s.ke_red + WG / 64);
    return s;
}

// The neighbour bin of candidate g (seg_off ascending, g < seg_off[2 NCELL]):
// binary search.
template <int NCELL>
__device__ inline int seg_search(const ItemLds& L, int g)
{
    int seg = 0, hi = 2 * NCELL;
    while (hi - seg > 1) {
        const int mid = (seg + hi) >> 1;
        if (L.seg_off[mid] <= g)
            seg = mid;
        else
            hi = mid;
    }
    return seg;
}

// The bins are at most 54 and the buckets one byte each.
static_assert(2 * 27 <= 256, "bucket entries are bytes");

// Conservative staging test on 16-bit truncated coordinates, one packed
// pair of axes: with d = s - c (the wrapped 16-bit difference of source and
// box centre) and hh = ceil(half extent) + 1 (16-bit units), adds
// max(|d| - hh, 0)^2 for both halves to acc.  |d| - 1 bounds the true
// offset from below, so the sum bounds the squared gap to the box from
// below (in (L / 2^16)^2 units).
__device__ __forceinline__ uint32_t gap2_16(uint32_t s, uint32_t c, uint32_t hh, uint32_t acc)
{
    typedef short v2s __attribute__((ext_vector_type(2)));
    typedef unsigned short v2u __attribute__((ext_vector_type(2)));
    const v2s d = __builtin_bit_cast(v2s, s) - __builtin_bit_cast(v2s, c);
    const v2s nd = (v2s)0 - d;
    const v2s a = __builtin_elementwise_max(d, nd);  // |d|; -32768 stays 0x8000
    const v2u au = __builtin_bit_cast(v2u, a), h = __builtin_bit_cast(v2u, hh);
    const v2u g = __builtin_elementwise_sub_sat(au, h);
    return __builtin_amdgcn_udot2(g, g, acc, false);
}

// The item's target: chunk `chunk` of cell c holds targets chunk*(WG/TPT) +
// tid/TPT of the cell's members taken octant by octant (within an octant the
// protons, then the neutrons); TPT lanes share a target.  Octant order keeps
// a chunk's targets close together, so the sources within range of their
// bounding box are fewer than for a chunk that spans the whole cell.
struct ItemTarget {
    int c, tl, q, slot;
    bool active, tprot;
};
template <int TPT>
__device__ inline ItemTarget item_target(const NucArgs& A, int item)
{
    ItemTarget t;
    t.c = A.items[2 * item + 0];
    const int chunk = A.items[2 * item + 1];
    const int S = A.sub;
    const int pb = t.c * S, nb = (A.C + t.c) * S;  // the cell's first proton / neutron bin
    t.tl = threadIdx.x / TPT;
    t.q = threadIdx.x % TPT;
    const int tidx = chunk * (WG / TPT) + t.tl;
    int before = 0, slot = -1;
    bool prot = false;
    for (int o = 0; o < S; ++o) {
        const int p0 = A.start[pb + o], np = A.start[pb + o + 1] - p0;
        const int n0 = A.start[nb + o], nn = A.start[nb + o + 1] - n0;
        const int r = tidx - before;
        if (slot < 0 && r >= 0 && r < np) {
            slot = p0 + r;
            prot = true;
        } else if (slot < 0 && r >= np && r < np + nn) {
            slot = n0 + (r - np);
        }
        before += np + nn;
    }
    t.active = slot >= 0;
    t.slot = t.active ? slot : 0;
    t.tprot = prot;
    return t;
}

// Neighbour bins of cell c (protons of the NCELL cells, then their
// neutrons) and the bounding box of the item's targets (fixed-point; a
// chunk lies inside one cell, so no wrap).  NCELL = 27: the full stencil,
// duplicates removed for small grids; NCELL = 14: the cell itself and the
// 13 neighbours whose offset (oz, oy, ox) is lexicographically positive (the
// half stencil of Newton's third law; needs at least 3 cells per side).
// Ends with a barrier; afterwards seg_off[2 NCELL] is the candidate count.
template <int NCELL = 27>
__device__ inline void item_setup(const NucArgs& A, const ItemLds& L, int c, bool nuc,
                                  bool in_box, uint3 mef)
{
    constexpr int NS = 2 * NCELL;
    const int tid = threadIdx.x, nc = A.nc, C = A.C;
    const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
    if (tid < NS) {
        const int kc = tid % NCELL, sp = tid / NCELL;  // sp 0: protons, 1: neutrons
        const int kk = NCELL == 27 ? kc : (kc == 0 ? 13 : 13 + kc);
        const int ox = kk % 3 - 1, oy = (kk / 3) % 3 - 1, oz = kk / 9 - 1;
        const int lo = axis_lo(nc), hi = axis_hi(nc);
        int beg = 0, len = 0;
        if (nuc && ox >= lo && ox <= hi && oy >= lo && oy <= hi && oz >= lo && oz <= hi) {
            const int nx = (cx + ox + nc) % nc, ny = (cy + oy + nc) % nc,
                      nz = (cz + oz + nc) % nc;
            const int b = (sp * C + (nz * nc + ny) * nc + nx) * A.sub;
            beg = A.start[b];
            len = A.start[b + A.sub] - beg;
        }
        L.seg_beg[tid] = beg;
        L.seg_off[tid + 1] = len;
    }
    if (tid < 6)
        L.misc[tid] = tid < 3 ? -1 : 0;  // lo = UINT_MAX, hi = 0 (as unsigned)
    __syncthreads();
    if (tid < 64) {
        // exclusive prefix of the bin lengths by a shuffle scan in the first
        // wavefront (lane l holds the length of bin l - 1)
        int v = (tid >= 1 && tid <= NS) ? L.seg_off[tid] : 0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(v, off, 64);
            if (tid >= off)
                v += y;
        }
        if (tid <= NS)
            L.seg_off[tid] = v;
    }
    if (in_box) {
        atomicMin(reinterpret_cast<unsigned*>(&L.misc[0]), mef.x);
        atomicMin(reinterpret_cast<unsigned*>(&L.misc[1]), mef.y);
        atomicMin(reinterpret_cast<unsigned*>(&L.misc[2]), mef.z);
        atomicMax(reinterpret_cast<unsigned*>(&L.misc[3]), mef.x);
        atomicMax(reinterpret_cast<unsigned*>(&L.misc[4]), mef.y);
        atomicMax(reinterpret_cast<unsigned*>(&L.misc[5]), mef.z);
    }
    __syncthreads();
    // the bin of every SEG_BUCKET-th candidate
    if (tid < SEG_BUCKETS && tid * SEG_BUCKET < L.seg_off[NS])
        L.bucket[tid] = (uint8_t)seg_search<NCELL>(L, tid * SEG_BUCKET);
    __syncthreads();
}

// Stages the neighbourhood in rounds of SP candidates per thread (SP * WG
// at most the tile size T, so a round fits the tile after a flush): locate
// (the candidate's bucket, then a short forward walk; a binary search past
// the buckets), load, keep the sources whose periodic gap to the targets'
// box may be below r (a conservative test on 16-bit truncated coordinates,
// gap2_16, against thr_stage16 = (r / (L/2^16))^2 + 1), and compact them in
// candidate order (so protons stay first).  put(pos, src,
// fixed, slot) stores a kept source at tile position pos; flush(n, np) is
// called, by the whole workgroup, when the next round might not fit in a
// tile of T entries and at the end (np = protons among the n).
template <class P, int T, int NCELL = 27, class Put, class Flush>
__device__ __forceinline__ void stage_neighbourhood(const typename P::Src* __restrict__ stg,
                                                    const NucConsts& k, const ItemLds& L,
                                                    uint32_t thr_stage16, Put put, Flush flush)
{
    using Lds = typename P::Lds;
    // a round keeps at most SP * WG candidates, which must fit an empty tile
    constexpr int SP = P::STAGE_PER_THREAD * WG <= T ? P::STAGE_PER_THREAD : T / WG;
    static_assert(SP >= 1 && SP * WG <= T, "a staging round must fit one tile");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int total = L.seg_off[2 * NCELL], np_tot = L.seg_off[NCELL];
    // box centre (16-bit truncated) and half extent, rounded up, plus the
    // one unit of truncation (16-bit units)
    uint32_t bc[3], hh[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint32_t lo = (uint32_t)L.misc[a], ext = (uint32_t)L.misc[3 + a] - lo;
        bc[a] = (lo + (ext >> 1)) >> 16;
        hh[a] = (uint32_t)(((uint64_t)(ext - (ext >> 1)) + 65535u) >> 16) + 1u;
    }
    const uint32_t cxy = bc[0] | (bc[1] << 16), hxy = hh[0] | (hh[1] << 16);
    int tile_n = 0, tile_np = 0;  // workgroup-uniform tile fill
    for (int base = 0; base < total; base += SP * WG) {
        bool keep[SP];
        uint3 f[SP];
        int gidx[SP], src_idx[SP];
#pragma unroll
        for (int u = 0; u < SP; ++u) {
            gidx[u] = base + u * WG + tid;
            src_idx[u] = -1;
            if (gidx[u] < total) {
                const int b = gidx[u] / SEG_BUCKET;
                int seg = b < SEG_BUCKETS ? (int)L.bucket[b] : seg_search<NCELL>(L, gidx[u]);
                while (L.seg_off[seg + 1] <= gidx[u])
                    ++seg;
                src_idx[u] = L.seg_beg[seg] + (gidx[u] - L.seg_off[seg]);
            }
        }
        typename P::Src sv[SP];
#pragma unroll
        for (int u = 0; u < SP; ++u)
            sv[u] = stg[src_idx[u] >= 0 ? src_idx[u] : 0];
#pragma unroll
        for (int u = 0; u < SP; ++u) {
            f[u] = P::fixed(sv[u], k);
            const uint32_t sxy = (f[u].x >> 16) | (f[u].y & 0xffff0000u);
            const uint32_t g2 = gap2_16(f[u].z >> 16, bc[2], hh[2], gap2_16(sxy, cxy, hxy, 0u));
            keep[u] = src_idx[u] >= 0 && g2 < thr_stage16;
        }
        // block compaction in candidate order (u, thread)
        unsigned long long m[SP];
#pragma unroll
        for (int u = 0; u < SP; ++u) {
            m[u] = __ballot(keep[u]);
            const unsigned long long mp = __ballot(keep[u] && gidx[u] < np_tot);
            if (lane == 0) {
                L.misc[6 + u * 4 + wave] = __popcll(m[u]);
                L.misc[14 + u * 4 + wave] = __popcll(mp);
            }
        }
        __syncthreads();
        int blk = 0, blkp = 0;
        int off[SP];
#pragma unroll
        for (int u = 0; u < SP; ++u) {
            off[u] = blk;
            for (int w = 0; w < WG / 64; ++w)
                off[u] += w < wave ? L.misc[6 + u * 4 + w] : 0;
            for (int w = 0; w < WG / 64; ++w) {
                blk += L.misc[6 + u * 4 + w];
                blkp += L.misc[14 + u * 4 + w];
            }
        }
        if (tile_n + blk > T) {  // no room: use the tile as it is first
            flush(tile_n, tile_np);
            tile_n = 0;
            tile_np = 0;
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < SP; ++u) {
            if (keep[u]) {
                const int pos = tile_n + off[u] + __popcll(m[u] & ((1ull << lane) - 1ull));
                put(pos, *reinterpret_cast<const Lds*>(&sv[u]), f[u], src_idx[u]);
            }
        }
        tile_n += blk;
        tile_np += blkp;
        __syncthreads();
    }
    if (tile_n > 0)
        flush(tile_n, tile_np);
}

// Epilogue of a nuclear cell item: combine the TPT lanes of each target,
// then either store the raw nuclear (F, V) per sorted slot (fnuc form) or
// add the Coulomb partials, write F and E (at perm[slot], or at the slot when
// perm is null) and apply the
// optional half kick; finally the fixed-order per-item kinetic-energy and
// pair-count reductions.  self_in_sum: the target's own r = 0 term (a like
// pair, V(0) = a + b + c) was summed and is removed here.
template <class P, int TPT, bool NUC, int MODE>
__device__ void nuclear_finish(const NucArgs& A, const NucConsts& k, typename P::Acc acc,
                               const ItemTarget& t, int item, bool self_in_sum,
                               const ItemLds& L)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (NUC) {
#pragma unroll
        for (int m = 1; m < TPT; m <<= 1) {
            acc.fx += __shfl_xor(acc.fx, m, TPT);
            acc.fy += __shfl_xor(acc.fy, m, TPT);
            acc.fz += __shfl_xor(acc.fz, m, TPT);
            acc.e += __shfl_xor(acc.e, m, TPT);
            if (MODE == MODE_COUNT)
                acc.np += __shfl_xor(acc.np, m, TPT);
        }
    }
    const double fsc = P::f_scale(k);
    double ke = 0.0;
    unsigned long long npairs = 0;
    if (t.active && t.q == 0) {
        if (MODE == MODE_COUNT)
            npairs = acc.np - (self_in_sum ? 1u : 0u);
        double V = NUC ? acc.e - (self_in_sum ? k.self_v : 0.0) : 0.0;
        double Fx = acc.fx * fsc, Fy = acc.fy * fsc, Fz = acc.fz * fsc;
        if (A.fnuc) {
            A.fnuc[t.slot] = make_double4(Fx, Fy, Fz, V);
        } else {
            if (A.S > 0 && t.tprot) {
                const double4 cp = coul_sum_seq(
                    static_cast<const typename P::CPart*>(A.coul_part), A.S, A.Z, t.slot);
                Fx += cp.x;
                Fy += cp.y;
                Fz += cp.z;
                V += cp.w;
            }
            const int64_t id = A.perm ? A.perm[t.slot] : t.slot;
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
    }
    if (A.ke_part || MODE == MODE_COUNT) {
        for (int m = 32; m >= 1; m >>= 1) {
            ke += __shfl_xor(ke, m, 64);
            if (MODE == MODE_COUNT)
                npairs += __shfl_xor(npairs, m, 64);
        }
        if (lane == 0) {
            L.ke_red[wave] = ke;
            L.np_red[wave] = npairs;
        }
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            unsigned long long sn = 0;
            for (int w = 0; w < WG / 64; ++w) {
                s += L.ke_red[w];
                sn += L.np_red[w];
            }
            if (A.ke_part && !A.fnuc)
                A.ke_part[item] = s;
            if (MODE == MODE_COUNT)
                atomicAdd(A.pairs, sn);
        }
        __syncthreads();
    }
}

// T: sources per LDS tile (the policy's default, or a tuned length)
template <class P, int T = P::CTILE>
constexpr int nuclear_compact_lds_bytes()
{
    return T * ((int)sizeof(typename P::Lds) + 8) + NUC_CAP * WG * 2 + ITEM_LDS_BYTES;
}

static_assert(nuclear_compact_lds_bytes<MixedPolicy>() <= 26 * 1024 + 512,
              "mixed compacting item: six workgroups per CU");

template <class P, int TPT, bool NUC, int MODE, int T = P::CTILE>
__device__ void nuclear_item_compact_t(const typename P::Src* __restrict__ stg,
                                       const NucArgs& A, const NucConsts& k, int item, char* lds)
{
    using Lds = typename P::Lds;
    Lds* src = reinterpret_cast<Lds*>(lds);
    uint2* tst = reinterpret_cast<uint2*>(src + T);
    uint16_t* lists = reinterpret_cast<uint16_t*>(tst + T);
    const ItemLds L = item_lds(reinterpret_cast<char*>(lists + NUC_CAP * WG));
    const int tid = threadIdx.x;

    const ItemTarget t = item_target<TPT>(A, item);
    const typename P::Src me = stg[t.slot];
    const uint3 mef = P::fixed(me, k);
    const uint32_t me_xy16 = (mef.x >> 16) | (mef.y & 0xffff0000u);
    item_setup(A, L, t.c, NUC, t.active && t.q == 0, mef);

    typename P::Acc acc;
    if (NUC) {
        const typename P::Coefs cf = P::coefs(k, t.tprot);
        typename P::Part part;
        const int q = t.q;
        // list entries are byte offsets of the sources in the tile
        constexpr int ES = (int)sizeof(Lds);
        static_assert(T * ES <= 65536, "tile offsets must fit 16 bits");
        const char* src_b = reinterpret_cast<const char*>(src);

        // Every entry of this lane's list column holds a tile offset from
        // here on (rows past the count keep older offsets of this item), so
        // a drain may read any row.
#pragma unroll
        for (int c = 0; c < NUC_CAP; ++c)
            lists[c * WG + tid] = 0;

        // evaluate the listed pairs of every lane, DU per round, then empty
        // the lists.  Every lane reads DU entries per round (rows clamped to
        // the capacity) and masks those at or past its count.
        constexpr int DU = P::DRAIN_U;
        auto drain = [&](int cnt, int kb) {
            const int kbb = kb * ES;
            for (int kk = 0; __ballot(kk < cnt); kk += DU) {
                int o[DU];
                bool v[DU];
                Lds sv[DU];
#pragma unroll
                for (int u = 0; u < DU; ++u) {
                    o[u] = lists[min(kk + u, NUC_CAP - 1) * WG + tid];
                    v[u] = kk + u < cnt;
                    sv[u] = *reinterpret_cast<const Lds*>(src_b + o[u]);
                }
#pragma unroll
                for (int u = 0; u < DU; ++u)  // protons first in the tile
                    P::template pair_c<MODE>(me, sv[u], cf, o[u] < kbb, k, part, v[u]);
            }
        };
        // Screen the tile's sources against this lane's target.  The append
        // is branch-free: every candidate is written at position cnt and cnt
        // advances only for survivors (slot cnt < NUC_CAP always exists).
        // Lanes without a target get a threshold nothing passes.
        const int thr = t.active ? k.thr16 : INT_MIN;
        const bool wave_live = __ballot(t.active) != 0ull;
        auto process = [&](int n, int kb) {
            if (!wave_live)
                return;
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
                    lists[cnt * WG + tid] = (uint16_t)(j * ES);
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
                    lists[cnt * WG + tid] = (uint16_t)(j * ES);
                    cnt += screen16(me_xy16, mef.z, tst[j]) < thr ? 1 : 0;
                }
            }
            drain(cnt, kb);
            P::fold(acc, part);
        };
        stage_neighbourhood<P, T>(
            stg, k, L, k.thr_stage16,
            [&](int pos, const Lds& e, const uint3& f, int) {
                src[pos] = P::tile_entry(e);
                tst[pos] = make_uint2((f.x >> 16) | (f.y & 0xffff0000u), f.z);
            },
            process);
    }
    nuclear_finish<P, TPT, NUC, MODE>(A, k, acc, t, item, true, L);
}

template <class P, bool NUC, int MODE>
__device__ void nuclear_item_compact(const typename P::Src* __restrict__ stg, const NucArgs& A,
                                     const NucConsts& k, int item, char* lds)
{
    nuclear_item_compact_t<P, NUC_TPT, NUC, MODE>(stg, A, k, item, lds);
}

}  // namespace pasta
