// Host side of the C ABI declared in include/pasta.h: argument checks,
// workspace layout, launch sequences, the simulation handle and the
// per-kernel event timing.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.hpp"

namespace pasta {

// ------------------------------------------------------------------ errors
static thread_local char g_err[1024] = "no error";

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

std::string describe_device_error(uint32_t bits)
{
    std::string s;
    auto add = [&](uint32_t b, const char* m) {
        if (bits & b) {
            if (!s.empty())
                s += "; ";
            s += m;
        }
    };
    add(ERR_NONFINITE_FORCE, "non-finite force (or a Coulomb sum beyond the fixed-point range)");
    add(ERR_NONFINITE_POS, "non-finite position");
    add(ERR_WRAP, "a particle moved more than one box length in a step");
    add(ERR_UF_LIMIT, "union-find retry bound reached");
    add(ERR_NONFINITE_VEL, "non-finite velocity");
    add(ERR_RANGE, "a position lies outside [0, L)");
    add(ERR_SPECIES, "a species value is not 0 or 1");
    if (s.empty())
        s = "unknown device error";
    return s;
}

// ------------------------------------------------------------------ timing
struct Timer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    int open[PASTA_KERNEL_CLASSES];
    struct Rec {
        int kc;
        size_t b, e;
    };
    std::vector<Rec> recs;
    double ms[PASTA_KERNEL_CLASSES] = {};
    int64_t launches[PASTA_KERNEL_CLASSES] = {};
    hipEvent_t take()
    {
        if (used == pool.size()) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess)
                return nullptr;
            pool.push_back(ev);
        }
        return pool[used++];
    }
    ~Timer()
    {
        for (auto ev : pool)
            (void)hipEventDestroy(ev);
    }
};

void timer_begin(Timer* t, int kc, hipStream_t s)
{
    if (!t || !t->on)
        return;
    hipEvent_t ev = t->take();
    if (!ev)
        return;
    t->open[kc] = (int)(t->used - 1);
    (void)hipEventRecord(ev, s);
}

void timer_end(Timer* t, int kc, hipStream_t s)
{
    if (!t || !t->on || t->open[kc] < 0)
        return;
    hipEvent_t ev = t->take();
    if (!ev)
        return;
    (void)hipEventRecord(ev, s);
    t->recs.push_back({kc, (size_t)t->open[kc], t->used - 1});
    t->open[kc] = -1;
}

static int timer_collect(Timer* t, hipStream_t s)
{
    PASTA_HIP(hipStreamSynchronize(s));
    for (const auto& r : t->recs) {
        float ms = 0.f;
        PASTA_HIP(hipEventElapsedTime(&ms, t->pool[r.b], t->pool[r.e]));
        t->ms[r.kc] += ms;
        t->launches[r.kc] += 1;
    }
    t->recs.clear();
    t->used = 0;
    return PASTA_OK;
}

// A finite Coulomb cutoff (r_coul = +inf: uncut).
static bool coulomb_cut_finite(const pasta_potential* p) { return std::isfinite(p->r_coul); }

// Largest interaction range: r_nuc, or a finite r_coul beyond it.
static double max_range(const pasta_potential* p)
{
    return coulomb_cut_finite(p) && p->r_coul > p->r_nuc ? p->r_coul : p->r_nuc;
}

static int check_pot(const pasta_potential* p)
{
    if (!p)
        return fail(PASTA_EINVAL, "null potential");
    const double v[] = {p->a, p->b, p->c, p->Lambda, p->lambda_s, p->alpha_hbarc, p->mass,
                        p->r_nuc};
    for (double x : v)
        if (!std::isfinite(x))
            return fail(PASTA_EINVAL, "non-finite potential parameter");
    if (!(p->Lambda > 0) || !(p->lambda_s > 0) || !(p->mass > 0) || !(p->r_nuc > 0))
        return fail(PASTA_EINVAL, "Lambda, lambda_s, mass and r_nuc must be positive");
    if (!(p->r_coul > 0))  // also NaN; +inf is the uncut model
        return fail(PASTA_EINVAL, "r_coul must be positive (INFINITY: uncut)");
    return PASTA_OK;
}

static PairParams pair_params(const pasta_potential* p, double L)
{
    PairParams pp;
    pp.a = p->a;
    pp.b_like = p->b + p->c;
    pp.b_unlike = p->b - p->c;
    pp.Lambda = p->Lambda;
    pp.r_nuc = p->r_nuc;
    pp.alpha_hbarc = p->alpha_hbarc;
    pp.r_coul = coulomb_cut_finite(p) ? p->r_coul : INFINITY;
    pp.lambda_s = p->lambda_s;
    pp.L = L;
    return pp;
}

// Nuclear-kernel settings of a workspace: the variant (0 dense, 1 compact,
// 2 lists, 3 compact with 8 lanes per target), and for the list form the
// halo and the pool sized for box sides down to L_min.  Calls without the
// nuclear terms use variant 1's layout.
constexpr int CELL_SUB = 8;  // octant bins inside each cell (compact chunks)
struct ListCfg {
    int variant = 1;
    bool on = false;
    double skin = 0.0;
    double L_min = 0.0;
    double pool_scale = 1.0;
};
static ListCfg list_cfg(int terms, double L_min)
{
    ListCfg c;
    c.variant = (terms & PASTA_TERM_NUCLEAR) ? internal_variant(g_tuning) : 1;
    c.on = c.variant == 2;
    c.skin = g_tuning.list_skin;
    c.L_min = L_min;
    c.pool_scale = g_tuning.list_pool_scale;
    return c;
}
static ListCfg cfg_variant(int v)
{
    ListCfg c;
    c.variant = v;
    return c;
}
// cell width of the grid: r_nuc, or r_nuc + skin for the list form
static double cell_cut(const pasta_potential* p, const ListCfg& lc)
{
    return lc.on ? p->r_nuc + lc.skin : p->r_nuc;
}

// Shared layout of the force workspace (a1 + a2 + a3 [+ lists]).
struct ForceWork {
    CellBuf cb;
    ForceBuf fb;
    ListBuf lb;
    bool lists;
    int variant;
    int chunk;
    uint32_t* err;
    double* red;  // [256] reduction partials
    double* scale;  // [2]
};
static size_t force_carve(Carver& cv, ForceWork* w, int64_t n, int C_max, int precision,
                          const pasta_potential* pot, const ListCfg& lc, int64_t pool_rows = -1)
{
    ForceWork fw;
    fw.variant = lc.variant;
    fw.chunk = nuclear_chunk_for(lc.variant);
    cellbuf_carve(cv, &fw.cb, n, C_max, fw.chunk, CELL_SUB);
    forcebuf_carve(cv, &fw.fb, n, fw.cb.item_max, precision);
    fw.err = cv.take<uint32_t>(1);
    fw.red = cv.take<double>(256);
    fw.scale = cv.take<double>(2);
    fw.lists = lc.on;
    fw.lb = ListBuf{};
    if (lc.on) {
        const int64_t rows =
            pool_rows > 0 ? pool_rows
                          : list_pool_rows(n, lc.L_min, pot->r_nuc + lc.skin, fw.cb.item_max,
                                           lc.pool_scale);
        listbuf_carve(cv, &fw.lb, n, fw.cb.item_max, rows);
        fw.lb.skin = lc.skin;
    }
    if (w)
        *w = fw;
    return cv.size();
}

static int check_work(void* d_work, size_t work_bytes, size_t need, const char* who)
{
    if (!d_work || work_bytes < need || (reinterpret_cast<uintptr_t>(d_work) & 255))
        return fail(PASTA_EWORKSPACE, "%s: workspace needs %zu bytes, 256-byte aligned (got %zu)",
                    who, need, work_bytes);
    return PASTA_OK;
}

static int read_err(uint32_t* d_err, hipStream_t s, const char* who)
{
    uint32_t e = 0;
    PASTA_HIP(hipMemcpyAsync(&e, d_err, sizeof(e), hipMemcpyDeviceToHost, s));
    PASTA_HIP(hipStreamSynchronize(s));
    if (e & (ERR_RANGE | ERR_SPECIES))
        return fail(PASTA_EINVAL, "%s: %s", who, describe_device_error(e).c_str());
    if (e)
        return fail(PASTA_EDEVICE, "%s: %s", who, describe_device_error(e).c_str());
    return PASTA_OK;
}

// Build the cell list (+ staging) for positions at box side L (grid g); in
// the list form also the lists (a forced build: positions recorded in xb).
// mv (optional): also move the particle state into sorted order.
static int build_cells(const double* pos, const uint8_t* species, int64_t n, const Grid& g,
                       ForceWork& w, int precision, const PairParams& pp, hipStream_t s,
                       Timer* t, const StateMove* mv = nullptr)
{
    launch_bin_count(pos, species, n, g, w.cb, w.err, s, t);
    launch_scan(w.cb, g, w.chunk, s, t);
    launch_scatter_rank(pos, species, n, g, w.cb, w.fb.stg64, w.fb.stgq, s, t, false, nullptr,
                        w.lists ? w.lb.xb : nullptr, mv);
    if (w.lists) {
        launch_list_force_rebuild(w.lb, g, s);
        launch_list_build(precision, w.fb, w.cb, g, w.lb, pp, s, t);
    }
    return PASTA_OK;
}

// pos / pos_perm: the FP64 positions the staging was built from (row
// pos_perm[slot], or the slot when pos_perm is null), read only by the
// finite-cutoff Coulomb test.
static void eval_forces(int precision, int terms, const ForceWork& w, const Grid& g, int64_t n,
                        int64_t Z, const PairParams& pp, double* force, double* epot,
                        const KickArgs& kick, uint64_t* pair_counter, hipStream_t s, Timer* t,
                        const double* pos, const int32_t* pos_perm)
{
    const ListBuf* lb = (w.lists && (terms & PASTA_TERM_NUCLEAR)) ? &w.lb : nullptr;
    ForceBuf fb = w.fb;
    fb.cut_pos = pos;
    fb.cut_perm = pos_perm;
    // the Newton-3 variant needs the combine kernel (reactions from every
    // item), so it always takes the fused form, as do the non-default tile
    // lengths (kernel variants 5 and 6)
    if ((g_tuning.fused_forces || w.variant >= 4) && (terms & PASTA_TERM_NUCLEAR)) {
        launch_forces_fused(precision, fb, w.cb, g, n, Z, pp, true,
                            (terms & PASTA_TERM_COULOMB) != 0, force, epot, kick, pair_counter,
                            w.err, s, t, w.variant, lb);
        return;
    }
    int S = 0;
    if ((terms & PASTA_TERM_COULOMB) && Z > 0)
        S = launch_coulomb(precision, fb, Z, pp, epot != nullptr || pair_counter != nullptr, s,
                           t, pair_counter ? pair_counter + 1 : nullptr);
    launch_nuclear(precision, fb, w.cb, g, n, Z, pp, (terms & PASTA_TERM_NUCLEAR) != 0, S,
                   force, epot, kick, pair_counter, w.err, s, t, w.variant, lb);
}

}  // namespace pasta

using namespace pasta;

// ===================================================================== ABI

extern "C" const char* pasta_last_error(void) { return g_err; }

extern "C" const char* pasta_version(void) { return "libpasta 0.1 (gfx950)"; }

extern "C" void pasta_potential_paper(pasta_potential* out)
{
    if (!out)
        return;
    out->a = 110.0;
    out->b = -26.0;
    out->c = 24.0;
    out->Lambda = 1.25;
    out->lambda_s = 10.0;
    out->alpha_hbarc = 7.2973525693e-3 * 197.3269804;
    out->mass = 939.0;
    out->r_nuc = 11.5;
    out->r_coul = INFINITY;
}

extern "C" int pasta_set_tuning(const pasta_tuning* t)
{
    if (!t || t->nuclear_variant < 0 || t->nuclear_variant > 4 || t->coulomb_splits < 0 ||
        t->coulomb_splits > 32 || (t->fused_forces != 0 && t->fused_forces != 1) ||
        t->coulomb_form < 0 || t->coulomb_form > 2 || !(t->list_skin > 0.0 && t->list_skin <= 64.0) ||
        !(t->list_pool_scale > 0.0 && t->list_pool_scale <= 1e3) || t->batch_wgs_per_cu < 0 ||
        t->batch_wgs_per_cu > 8 ||
        (t->nuclear_tile != 0 && t->nuclear_tile != NUC_TILE_SHORT && t->nuclear_tile != 512 &&
         t->nuclear_tile != NUC_TILE_LONG))
        return fail(PASTA_EINVAL, "pasta_set_tuning: bad argument");
    g_tuning = *t;
    return PASTA_OK;
}

extern "C" int pasta_get_tuning(pasta_tuning* out)
{
    if (!out)
        return fail(PASTA_EINVAL, "pasta_get_tuning: null");
    *out = g_tuning;
    return PASTA_OK;
}

extern "C" const char* pasta_kernel_class_name(int32_t k)
{
    static const char* names[PASTA_KERNEL_CLASSES] = {
        "drift+bin", "scan", "scatter", "rank+stage", "coulomb", "nuclear+kick", "thermostat",
        "combine+kick", "list build"};
    return (k >= 0 && k < PASTA_KERNEL_CLASSES) ? names[k] : "?";
}

// ------------------------------------------------------------------- a1
extern "C" int pasta_cell_dims(double L, double r_cut, int32_t* h_ncell)
{
    if (!h_ncell || !(L > 0.0) || !std::isfinite(L) || !(r_cut > 0.0))
        return fail(PASTA_EINVAL, "pasta_cell_dims: bad argument");
    *h_ncell = cell_dims(L, r_cut);
    return PASTA_OK;
}

extern "C" int pasta_cell_list_workspace(int64_t n, double L, double r_cut, size_t* h_bytes)
{
    if (!h_bytes || n < 0 || !(L > 0.0) || !(r_cut > 0.0) || !std::isfinite(L))
        return fail(PASTA_EINVAL, "pasta_cell_list_workspace: bad argument");
    const Grid g = make_grid(L, r_cut);
    Carver cv(nullptr);
    CellBuf cb;
    cellbuf_carve(cv, &cb, n, g.C, 0);
    cv.take<uint32_t>(1);
    *h_bytes = cv.size();
    return PASTA_OK;
}

extern "C" int pasta_cell_list(int64_t n, double L, double r_cut, const double* d_pos,
                               const uint8_t* d_species, int32_t* d_cell_start, int32_t* d_perm,
                               int32_t* h_ncell, void* d_work, size_t work_bytes, void* stream)
{
    if (n < 0 || n > INT32_MAX - 1 || (n > 0 && (!d_pos || !d_species || !d_perm)) ||
        !d_cell_start || !(L > 0.0) || !std::isfinite(L) || !(r_cut > 0.0))
        return fail(PASTA_EINVAL, "pasta_cell_list: bad argument");
    if (L < 2.0 * r_cut)
        return fail(PASTA_EBOX, "pasta_cell_list: L = %g < 2 r_cut = %g", L, 2.0 * r_cut);
    size_t need = 0;
    PASTA_TRY(pasta_cell_list_workspace(n, L, r_cut, &need));
    PASTA_TRY(check_work(d_work, work_bytes, need, "pasta_cell_list"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid g = make_grid(L, r_cut);
    Carver cv(d_work);
    CellBuf cb;
    cellbuf_carve(cv, &cb, n, g.C, 0);
    uint32_t* err = cv.take<uint32_t>(1);
    PASTA_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), s));
    cellbuf_zero(cb, g.C, s);
    launch_bin_count(d_pos, d_species, n, g, cb, err, s, nullptr);
    launch_scan(cb, g, 0, s, nullptr);
    launch_scatter_rank(d_pos, d_species, n, g, cb, nullptr, nullptr, s, nullptr);
    PASTA_HIP(hipMemcpyAsync(d_cell_start, cb.start, sizeof(int32_t) * (2 * (size_t)g.C + 1),
                             hipMemcpyDeviceToDevice, s));
    if (n > 0)
        PASTA_HIP(hipMemcpyAsync(d_perm, cb.perm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    PASTA_HIP(hipGetLastError());
    if (h_ncell)
        *h_ncell = g.nc;
    return read_err(err, s, "pasta_cell_list");
}

// -------------------------------------------------------------- a2 + a3
extern "C" int pasta_forces_workspace(const pasta_potential* pot, int32_t precision, int64_t n,
                                      double L, size_t* h_bytes)
{
    PASTA_TRY(check_pot(pot));
    if (!h_bytes || n < 0 || !(L > 0.0) || !std::isfinite(L) ||
        (precision != PASTA_FP64 && precision != PASTA_MIXED))
        return fail(PASTA_EINVAL, "pasta_forces_workspace: bad argument");
    const ListCfg lc = list_cfg(PASTA_TERM_ALL, L);
    const Grid g = make_force_grid(L, cell_cut(pot, lc), n, CELL_SUB);
    Carver cv(nullptr);
    *h_bytes = force_carve(cv, nullptr, n, g.C, precision, pot, lc);
    return PASTA_OK;
}

namespace pasta {

// Argument checks shared by pasta_forces and pasta_forces_noalloc.
static int check_force_args(const char* who, const pasta_potential* pot, int32_t precision,
                            int32_t terms, int64_t n, double L, const double* d_pos,
                            const uint8_t* d_species, const double* d_force)
{
    PASTA_TRY(check_pot(pot));
    if (n < 0 || n > INT32_MAX - 1 || (n > 0 && (!d_pos || !d_species || !d_force)) ||
        !(L > 0.0) || !std::isfinite(L) || (terms & ~PASTA_TERM_ALL) ||
        (precision != PASTA_FP64 && precision != PASTA_MIXED))
        return fail(PASTA_EINVAL, "%s: bad argument", who);
    if (L < 2.0 * max_range(pot))
        return fail(PASTA_EBOX, "%s: L = %g < 2 max(r_nuc, r_coul) = %g", who, L,
                    2.0 * max_range(pot));
    return PASTA_OK;
}

// One force evaluation on a checked workspace: cell list, pair kernels,
// device error word.  Clears what must start at zero with fill kernels.
static int forces_run(const char* who, const pasta_potential* pot, int32_t precision,
                      int32_t terms, int64_t n, double L, const double* d_pos,
                      const uint8_t* d_species, double* d_force, double* d_epot, void* d_work,
                      size_t work_bytes, hipStream_t s)
{
    if (n == 0)
        return PASTA_OK;
    // a call without the nuclear terms uses the cell-sweep layout, which is
    // smaller than the list layout the workspace query may have sized
    const ListCfg lc = list_cfg(terms, L);
    const Grid g = make_force_grid(L, cell_cut(pot, lc), n, CELL_SUB);
    Carver cv0(nullptr);
    PASTA_TRY(check_work(d_work, work_bytes, force_carve(cv0, nullptr, n, g.C, precision, pot, lc),
                         who));
    ForceWork w;
    Carver cv(d_work);
    force_carve(cv, &w, n, g.C, precision, pot, lc);
    const PairParams pp = pair_params(pot, L);
    launch_zero_words(w.err, 1, s);
    if (w.lists)
        launch_zero_words(w.lb.ctl, (int64_t)(sizeof(ListCtl) / sizeof(uint32_t)), s);
    cellbuf_zero(w.cb, g.C, s, g.sub);
    launch_zero_words(w.fb.react, 8 * n, s);
    build_cells(d_pos, d_species, n, g, w, precision, pp, s, nullptr);
    int32_t Z = 0;
    PASTA_HIP(hipMemcpyAsync(&Z, w.cb.start + (int64_t)g.C * g.sub, sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
    PASTA_HIP(hipStreamSynchronize(s));
    KickArgs kick{nullptr, 0.0, pot->mass, nullptr, false};
    eval_forces(precision, terms, w, g, n, Z, pp, d_force, d_epot, kick, nullptr, s, nullptr,
                d_pos, w.cb.perm);
    PASTA_HIP(hipGetLastError());
    return read_err(w.err, s, who);
}

}  // namespace pasta

extern "C" int pasta_forces(const pasta_potential* pot, int32_t precision, int32_t terms,
                            int64_t n, double L, const double* d_pos, const uint8_t* d_species,
                            double* d_force, double* d_epot, void* d_work, size_t work_bytes,
                            void* stream)
{
    PASTA_TRY(check_force_args("pasta_forces", pot, precision, terms, n, L, d_pos, d_species,
                               d_force));
    size_t need = 0;
    PASTA_TRY(pasta_forces_workspace(pot, precision, n, L, &need));
    PASTA_TRY(check_work(d_work, work_bytes, need, "pasta_forces"));
    return forces_run("pasta_forces", pot, precision, terms, n, L, d_pos, d_species, d_force,
                      d_epot, d_work, work_bytes, static_cast<hipStream_t>(stream));
}

// -------------------------------------------------- forces without allocation
// The scratch memory of pasta_forces_noalloc: one static device array, which
// every device the library runs on holds until the process ends.  In host
// code `scratch` names a host-side stand-in, never the device memory: its
// device address is taken once per device with hipGetSymbolAddress (with
// that device current) and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[PASTA_NOALLOC_SCRATCH_BYTES];

namespace pasta {
namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[SCRATCH_MAX_DEVICES] = {};

int scratch_address(void** out)
{
    int dev = 0;
    PASTA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES)
        return fail(PASTA_EINVAL, "pasta_forces_noalloc: device %d beyond %d", dev,
                    SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PASTA_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return PASTA_OK;
}
}  // namespace
}  // namespace pasta

extern "C" int pasta_forces_noalloc(const pasta_potential* pot, int32_t precision,
                                    int32_t terms, int64_t n, double L, const double* d_pos,
                                    const uint8_t* d_species, double* d_force, double* d_epot,
                                    void* stream)
{
    PASTA_TRY(check_force_args("pasta_forces_noalloc", pot, precision, terms, n, L, d_pos,
                               d_species, d_force));
    size_t need = 0;
    PASTA_TRY(pasta_forces_workspace(pot, precision, n, L, &need));
    if (need > PASTA_NOALLOC_SCRATCH_BYTES)
        return fail(PASTA_EWORKSPACE,
                    "pasta_forces_noalloc: n = %lld at L = %g needs %zu bytes of scratch, "
                    "more than the static %zu",
                    (long long)n, L, need, (size_t)PASTA_NOALLOC_SCRATCH_BYTES);
    void* work = nullptr;
    PASTA_TRY(scratch_address(&work));
    return forces_run("pasta_forces_noalloc", pot, precision, terms, n, L, d_pos, d_species,
                      d_force, d_epot, work, PASTA_NOALLOC_SCRATCH_BYTES,
                      static_cast<hipStream_t>(stream));
}

// -------------------------------------------------------------- tuning
// Times the two pair kernels (Coulomb + nuclear with its epilogue, forces
// only) on the given state for every candidate setting and keeps the
// fastest.  Candidates: nuclear variant {dense, compacted, compacted with 8
// lanes per target, Newton-3 half stencil (fused only)} x Coulomb {gather
// with source splits S/2, S, 2S around the automatic S (clamped to 1..32),
// pairwise, pairwise into fixed-point accumulators (fused, mixed precision)}
// x fused {0, 1}.  The cell list is built once per item size.  Each
// candidate is timed twice, in two passes over the list, and keeps the
// faster time.
extern "C" int pasta_autotune(const pasta_potential* pot, int32_t precision, int64_t n, double L,
                              const double* d_pos, const uint8_t* d_species, void* d_work,
                              size_t work_bytes, void* stream, int32_t reps, pasta_tuning* h_best,
                              double* h_ms, pasta_tuning* h_cands, int32_t* h_ncand)
{
    PASTA_TRY(check_pot(pot));
    if (n <= 0 || n > INT32_MAX - 1 || !d_pos || !d_species || !h_best || reps < 1 ||
        !(L > 0.0) || !std::isfinite(L) || (precision != PASTA_FP64 && precision != PASTA_MIXED))
        return fail(PASTA_EINVAL, "pasta_autotune: bad argument");
    if (L < 2.0 * max_range(pot))
        return fail(PASTA_EBOX, "pasta_autotune: L < 2 max(r_nuc, r_coul)");
    // laid out for the 32-target items (the larger item list); 64-target
    // candidates use a prefix of it
    const ListCfg lay = cfg_variant(3);
    Carver cvn(nullptr);
    const Grid g = make_force_grid(L, pot->r_nuc, n, CELL_SUB);
    force_carve(cvn, nullptr, n, g.C, precision, pot, lay);
    cvn.take<double>(3 * (size_t)n);  // scratch force output
    PASTA_TRY(check_work(d_work, work_bytes, cvn.size(), "pasta_autotune"));
    hipStream_t s = static_cast<hipStream_t>(stream);
    ForceWork w;
    Carver cv(d_work);
    force_carve(cv, &w, n, g.C, precision, pot, lay);
    const int64_t items32 = w.cb.item_max;
    const int64_t items64 = n / nuclear_chunk_for(1) + g.C + 1;
    double* f = cv.take<double>(3 * (size_t)n);
    const PairParams pp = pair_params(pot, L);
    PASTA_HIP(hipMemsetAsync(w.err, 0, sizeof(uint32_t), s));
    cellbuf_zero(w.cb, g.C, s, g.sub);
    launch_zero_words(w.fb.react, 8 * n, s);
    int32_t Z = 0;
    int built_chunk = 0;
    // (re)builds the cell list for a candidate's item size
    auto cells_for = [&](int variant) {
        w.variant = variant;
        w.chunk = nuclear_chunk_for(variant);
        w.cb.item_max = w.chunk == nuclear_chunk_for(1) ? items64 : items32;
        if (w.chunk != built_chunk) {
            build_cells(d_pos, d_species, n, g, w, precision, pp, s, nullptr);
            built_chunk = w.chunk;
        }
    };
    cells_for(1);
    PASTA_HIP(hipMemcpyAsync(&Z, w.cb.start + (int64_t)g.C * g.sub, sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
    PASTA_HIP(hipStreamSynchronize(s));

    const pasta_tuning saved = g_tuning;
    pasta_tuning auto_t = saved;
    auto_t.nuclear_variant = 1;
    auto_t.coulomb_splits = 0;
    auto_t.fused_forces = 0;
    auto_t.coulomb_form = 0;
    g_tuning = auto_t;
    const int S0 = Z > 0 ? coulomb_splits(Z) : 1;
    std::vector<pasta_tuning> cands;
    const bool pair_fits = Z > 0 && (int64_t)coulomb_pair_plan_supers(Z) * Z <= w.fb.coul_max;
    // (public variant, tile length) pairs; 4 and the non-default tiles run
    // in the fused form only
    const int vt[][2] = {{0, 0}, {1, 0}, {3, 0}, {4, 0}, {3, NUC_TILE_SHORT}, {3, NUC_TILE_LONG}};
    for (int fused = 0; fused <= 1; ++fused)
        for (const auto& p : vt) {
            const int v = p[0], tile = p[1];
            if ((v == 4 || tile) && !fused)
                continue;
            int last = -1;
            for (int sc : {S0 / 2, S0, 2 * S0}) {
                int sv = sc < 1 ? 1 : (sc > 32 ? 32 : sc);
                if (sv == last)
                    continue;
                last = sv;
                pasta_tuning c = saved;
                c.nuclear_variant = v;
                c.nuclear_tile = tile;
                c.coulomb_splits = sv;
                c.fused_forces = fused;
                c.coulomb_form = 0;
                cands.push_back(c);
            }
            if (pair_fits) {
                pasta_tuning c = saved;
                c.nuclear_variant = v;
                c.nuclear_tile = tile;
                c.coulomb_splits = 0;
                c.fused_forces = fused;
                c.coulomb_form = 1;
                cands.push_back(c);
            }
            // pairwise into fixed-point accumulators: fused, mixed precision
            if (Z > 0 && fused && precision == PASTA_MIXED) {
                pasta_tuning c = saved;
                c.nuclear_variant = v;
                c.nuclear_tile = tile;
                c.coulomb_splits = 0;
                c.fused_forces = 1;
                c.coulomb_form = 2;
                cands.push_back(c);
            }
        }
    hipEvent_t e0, e1;
    PASTA_HIP(hipEventCreate(&e0));
    PASTA_HIP(hipEventCreate(&e1));
    KickArgs kick{nullptr, 0.0, pot->mass, nullptr, true};  // sorted order, as in a simulation
    // two rounds over the candidate list; each candidate keeps its faster
    // round, so one slow moment of the GPU does not decide between settings
    // that differ by a few percent
    constexpr int ROUNDS = 2;
    std::vector<double> per_c(cands.size(), 1e300);
    int rc = PASTA_OK;
    for (int round = 0; round < ROUNDS && rc == PASTA_OK; ++round)
        for (size_t c = 0; c < cands.size() && rc == PASTA_OK; ++c) {
            g_tuning = cands[c];
            cells_for(internal_variant(cands[c]));
            // one untimed warm-up, then reps timed evaluations; forces only,
            // as a simulation step evaluates them (energies are rarely asked)
            eval_forces(precision, PASTA_TERM_ALL, w, g, n, Z, pp, f, nullptr, kick, nullptr, s,
                        nullptr, d_pos, w.cb.perm);
            if (hipEventRecord(e0, s) != hipSuccess) {
                rc = fail(PASTA_EHIP, "hipEventRecord failed");
                break;
            }
            for (int r = 0; r < reps; ++r)
                eval_forces(precision, PASTA_TERM_ALL, w, g, n, Z, pp, f, nullptr, kick,
                            nullptr, s, nullptr, d_pos, w.cb.perm);
            float ms = 0.f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = fail(PASTA_EHIP, "event timing failed");
                break;
            }
            per_c[c] = std::min(per_c[c], (double)ms / reps);
        }
    double best = 1e300;
    int best_k = 0;
    for (size_t c = 0; c < cands.size() && rc == PASTA_OK; ++c) {
        if (h_ms && h_ncand && (int)c < *h_ncand)
            h_ms[c] = per_c[c];
        if (h_cands && h_ncand && (int)c < *h_ncand)
            h_cands[c] = cands[c];
        if (per_c[c] < best) {
            best = per_c[c];
            best_k = (int)c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    g_tuning = saved;
    if (rc != PASTA_OK)
        return rc;
    if (h_ncand)
        *h_ncand = (int32_t)cands.size();
    *h_best = cands[best_k];
    PASTA_HIP(hipGetLastError());
    return read_err(w.err, s, "pasta_autotune");
}

extern "C" int pasta_autotune_workspace(const pasta_potential* pot, int32_t precision, int64_t n,
                                        double L, size_t* h_bytes)
{
    PASTA_TRY(check_pot(pot));
    if (!h_bytes || n < 0 || !(L > 0.0) || !std::isfinite(L) ||
        (precision != PASTA_FP64 && precision != PASTA_MIXED))
        return fail(PASTA_EINVAL, "pasta_autotune_workspace: bad argument");
    const Grid g = make_force_grid(L, pot->r_nuc, n, CELL_SUB);
    Carver cv(nullptr);
    force_carve(cv, nullptr, n, g.C, precision, pot, cfg_variant(3));
    cv.take<double>(3 * (size_t)n);
    *h_bytes = cv.size();
    return PASTA_OK;
}

// ------------------------------------------------------------------- a4
struct pasta_sim {
    pasta_potential pot;
    pasta_integrator integ;
    int precision;
    int64_t n, Z;
    double L0, L_max;
    int64_t step;
    double* pos;  // caller's arrays (caller order): read on import, written on export
    double* vel;
    const uint8_t* species;
    hipStream_t stream;
    int C_max;
    double r_cell;  // cell width: r_nuc, or r_nuc + list halo
    ForceWork w;
    // The state lives in the sorted order of the last cell build, so every
    // per-particle kernel of a step reads and writes contiguous memory.  Two
    // copies: the rank kernel of a build moves the state from one into the
    // other (cur names the live one).  ids[k] is the caller index of slot k.
    double* xs[2];
    double* vs[2];
    int32_t* ids[2];
    uint8_t* sps[2];
    int cur;
    double* force;  // [n][3] F of the current state, sorted order
    double* epot;   // [n] energy shares, sorted order
    bool epot_valid;  // steps compute forces only; energies are evaluated on demand
    Timer timer;
};

static double box_side(const pasta_sim* sim, int64_t step)
{
    // Eq. (3a): l(t) = l(0) (1 + xi_dot t), t = step dt, from the index
    return sim->L0 * (1.0 + sim->integ.xi_dot * ((double)step * sim->integ.dt));
}

static size_t sim_carve(Carver& cv, pasta_sim* sim, int64_t n, int C_max, int precision,
                        const pasta_potential* pot, const ListCfg& lc, int64_t pool_rows = -1)
{
    force_carve(cv, sim ? &sim->w : nullptr, n, C_max, precision, pot, lc, pool_rows);
    double* f = cv.take<double>(3 * (size_t)n);
    double* e = cv.take<double>((size_t)n);
    double* xs[2];
    double* vs[2];
    int32_t* ids[2];
    uint8_t* sps[2];
    for (int b = 0; b < 2; ++b) {
        xs[b] = cv.take<double>(3 * (size_t)n);
        vs[b] = cv.take<double>(3 * (size_t)n);
        ids[b] = cv.take<int32_t>((size_t)n);
        sps[b] = cv.take<uint8_t>((size_t)n);
    }
    if (sim) {
        sim->force = f;
        sim->epot = e;
        for (int b = 0; b < 2; ++b) {
            sim->xs[b] = xs[b];
            sim->vs[b] = vs[b];
            sim->ids[b] = ids[b];
            sim->sps[b] = sps[b];
        }
    }
    return cv.size();
}

// The spare copy of the sorted state as the destination of a state move
// from the live one.
static StateMove sim_move(const pasta_sim* sim)
{
    const int a = sim->cur, b = 1 - sim->cur;
    return StateMove{sim->vs[a], sim->ids[a], sim->xs[b], sim->vs[b], sim->ids[b], sim->sps[b]};
}

// Writes the live sorted state to the caller's arrays (caller order).
static void sim_export(pasta_sim* sim)
{
    launch_export(sim->ids[sim->cur], sim->n, sim->xs[sim->cur], sim->pos, sim->vs[sim->cur],
                  sim->vel, nullptr, nullptr, sim->stream);
}

static int check_integ(const pasta_integrator* g)
{
    if (!g)
        return fail(PASTA_EINVAL, "null integrator");
    if (!(g->dt > 0.0) || !std::isfinite(g->dt) || !std::isfinite(g->xi_dot) ||
        !(g->T >= 0.0) || g->rescale_every < 0)
        return fail(PASTA_EINVAL, "bad integrator parameters");
    return PASTA_OK;
}

extern "C" int pasta_sim_workspace(const pasta_potential* pot, const pasta_integrator* integ,
                                   int32_t precision, int64_t n, double L_start, double L_max,
                                   size_t* h_bytes)
{
    PASTA_TRY(check_pot(pot));
    PASTA_TRY(check_integ(integ));
    if (!h_bytes || n < 0 || !(L_max > 0.0) || !std::isfinite(L_max) || !(L_start > 0.0) ||
        !std::isfinite(L_start) || (precision != PASTA_FP64 && precision != PASTA_MIXED))
        return fail(PASTA_EINVAL, "pasta_sim_workspace: bad argument");
    const ListCfg lc = list_cfg(PASTA_TERM_ALL, L_start);
    const Grid g = make_force_grid(L_max > L_start ? L_max : L_start, cell_cut(pot, lc), n, CELL_SUB);
    Carver cv(nullptr);
    *h_bytes = sim_carve(cv, nullptr, n, g.C, precision, pot, lc);
    return PASTA_OK;
}

// Imports the caller's state: the cell build sorts it into the live copy.
static int sim_eval_initial(pasta_sim* sim)
{
    hipStream_t s = sim->stream;
    const double L = box_side(sim, sim->step);
    const Grid g = make_force_grid(L, sim->r_cell, sim->n, CELL_SUB);
    const PairParams pp = pair_params(&sim->pot, L);
    sim->cur = 0;
    const StateMove mv{sim->vel, nullptr, sim->xs[0], sim->vs[0], sim->ids[0], sim->sps[0]};
    build_cells(sim->pos, sim->species, sim->n, g, sim->w, sim->precision, pp, s, &sim->timer,
                &mv);
    int32_t Z = 0;
    PASTA_HIP(hipMemcpyAsync(&Z, sim->w.cb.start + (int64_t)g.C * g.sub, sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
    PASTA_HIP(hipStreamSynchronize(s));
    sim->Z = Z;
    KickArgs kick{nullptr, 0.0, sim->pot.mass, nullptr, true};
    eval_forces(sim->precision, PASTA_TERM_ALL, sim->w, g, sim->n, sim->Z, pp, sim->force,
                sim->epot, kick, nullptr, s, &sim->timer, sim->xs[sim->cur], nullptr);
    sim->epot_valid = true;
    PASTA_HIP(hipGetLastError());
    return read_err(sim->w.err, s, "pasta_sim");
}

// Energy shares of the current state (the steps skip them): one force
// evaluation with energies on the cell list / neighbour lists in place.
// The forces it writes are the same bits the step wrote.
static int sim_refresh_energies(pasta_sim* sim)
{
    if (sim->epot_valid)
        return PASTA_OK;
    const double L = box_side(sim, sim->step);
    const Grid g = make_force_grid(L, sim->r_cell, sim->n, CELL_SUB);
    KickArgs kick{nullptr, 0.0, sim->pot.mass, nullptr, true};
    eval_forces(sim->precision, PASTA_TERM_ALL, sim->w, g, sim->n, sim->Z,
                pair_params(&sim->pot, L), sim->force, sim->epot, kick, nullptr, sim->stream,
                nullptr, sim->xs[sim->cur], nullptr);
    PASTA_HIP(hipGetLastError());
    sim->epot_valid = true;
    return PASTA_OK;
}

extern "C" int pasta_sim_create(const pasta_potential* pot, const pasta_integrator* integ,
                                int32_t precision, int64_t n, double L0, int64_t step0,
                                double L_max, double* d_pos, double* d_vel,
                                const uint8_t* d_species, void* d_work, size_t work_bytes,
                                void* stream, pasta_sim** out)
{
    PASTA_TRY(check_pot(pot));
    PASTA_TRY(check_integ(integ));
    if (!out || n <= 0 || n > INT32_MAX - 1 || !d_pos || !d_vel || !d_species ||
        !(L0 > 0.0) || !std::isfinite(L0) || step0 < 0 ||
        (precision != PASTA_FP64 && precision != PASTA_MIXED))
        return fail(PASTA_EINVAL, "pasta_sim_create: bad argument");
    *out = nullptr;
    pasta_sim* sim = new (std::nothrow) pasta_sim();
    if (!sim)
        return fail(PASTA_ENOMEM, "pasta_sim_create: out of host memory");
    sim->pot = *pot;
    sim->integ = *integ;
    sim->precision = precision;
    sim->n = n;
    sim->L0 = L0;
    sim->step = step0;
    sim->pos = d_pos;
    sim->vel = d_vel;
    sim->species = d_species;
    sim->stream = static_cast<hipStream_t>(stream);
    const double Lstart = box_side(sim, step0);
    sim->L_max = L_max > Lstart ? L_max : Lstart;
    if (Lstart < 2.0 * max_range(pot)) {
        delete sim;
        return fail(PASTA_EBOX, "pasta_sim_create: L = %g < 2 max(r_nuc, r_coul)", Lstart);
    }
    // the nuclear variant (and the list settings) in force when the
    // simulation is created stay with it; the list memory takes the rest of
    // the workspace
    const ListCfg lc = list_cfg(PASTA_TERM_ALL, Lstart);
    sim->r_cell = cell_cut(pot, lc);
    sim->C_max = make_force_grid(sim->L_max, sim->r_cell, sim->n, CELL_SUB).C;
    Carver cv0(nullptr);
    const size_t need = sim_carve(cv0, nullptr, n, sim->C_max, precision, pot, lc, 1);
    int rc = check_work(d_work, work_bytes, need, "pasta_sim_create");
    if (rc != PASTA_OK) {
        delete sim;
        return rc;
    }
    int64_t rows = -1;
    if (lc.on) {
        rows = 1 + (int64_t)((work_bytes - need) / LIST_ROW_BYTES);
        for (;;) {
            Carver cvr(nullptr);
            if (sim_carve(cvr, nullptr, n, sim->C_max, precision, pot, lc, rows) <= work_bytes ||
                rows == 1)
                break;
            --rows;
        }
    }
    Carver cv(d_work);
    sim_carve(cv, sim, n, sim->C_max, precision, pot, lc, rows);
    for (int k = 0; k < PASTA_KERNEL_CLASSES; ++k)
        sim->timer.open[k] = -1;
    hipStream_t s = sim->stream;
    if (hipMemsetAsync(sim->w.err, 0, sizeof(uint32_t), s) != hipSuccess) {
        delete sim;
        return fail(PASTA_EHIP, "hipMemsetAsync failed");
    }
    cellbuf_zero(sim->w.cb, sim->C_max, s, CELL_SUB);
    launch_zero_words(sim->w.fb.react, 8 * n, s);
    if (sim->w.lists && hipMemsetAsync(sim->w.lb.ctl, 0, sizeof(ListCtl), s) != hipSuccess) {
        delete sim;
        return fail(PASTA_EHIP, "hipMemsetAsync failed");
    }
    rc = sim_eval_initial(sim);
    if (rc != PASTA_OK) {
        delete sim;
        return rc;
    }
    *out = sim;
    return PASTA_OK;
}

extern "C" int pasta_sim_step(pasta_sim* sim, int64_t nsteps)
{
    if (!sim || nsteps < 0)
        return fail(PASTA_EINVAL, "pasta_sim_step: bad argument");
    hipStream_t s = sim->stream;
    const pasta_integrator& gi = sim->integ;
    const double hdtm = gi.dt / (2.0 * sim->pot.mass);
    auto box_ok = [&](double L) {
        return !(L > sim->L_max * (1.0 + 1e-12) || L < 2.0 * max_range(&sim->pot));
    };
    // drifted: this step's first part (half kick, drift, binning) was done by
    // the previous step's combine kernel (cell form, fused forces: every step
    // but the last of the call and the thermostat steps)
    bool drifted = false;
    for (int64_t k = 0; k < nsteps; ++k) {
        const int64_t n0 = sim->step;
        const double L_old = box_side(sim, n0), L_new = box_side(sim, n0 + 1);
        if (!box_ok(L_new))
            return fail(PASTA_EBOX, "pasta_sim_step: box side %g at step %lld is outside "
                        "[2 r_nuc, L_max = %g]", L_new, (long long)(n0 + 1), sim->L_max);
        const Grid g = make_force_grid(L_new, sim->r_cell, sim->n, CELL_SUB);
        const int c = sim->cur;
        DriftArgs da;
        da.pos = sim->xs[c];
        da.vel = sim->vs[c];
        da.force = sim->force;
        da.species = sim->sps[c];
        da.n = sim->n;
        da.hdtm = hdtm;
        da.dt = gi.dt;
        da.L_new = L_new;
        da.ratio = L_new / L_old;
        da.scale_positions = gi.scale_positions;
        const PairParams pp = pair_params(&sim->pot, L_new);
        if (sim->w.lists) {
            // drift + staging + rebuild decision, then the build kernels,
            // each of which returns at once unless this step rebuilds
            // (a rebuild sorts the state into the spare copy and copies it
            // back, so the live copy stays the same on the host side)
            const ListBuf& lb = sim->w.lb;
            const int32_t* gate = &lb.ctl->rebuild;
            const StateMove mv = sim_move(sim);
            launch_drift_list(da, g, sim->w.cb, lb, sim->w.fb.stg64, sim->w.fb.stgq, n0,
                              sim->w.err, s, &sim->timer);
            launch_bin_count(sim->xs[c], sim->sps[c], sim->n, g, sim->w.cb, sim->w.err, s,
                             &sim->timer, gate);
            launch_scan(sim->w.cb, g, sim->w.chunk, s, &sim->timer, gate);
            launch_scatter_rank(sim->xs[c], sim->sps[c], sim->n, g, sim->w.cb, sim->w.fb.stg64,
                                sim->w.fb.stgq, s, &sim->timer, false, gate, lb.xb, &mv);
            launch_state_copy(mv, sim->xs[c], sim->vs[c], sim->ids[c], sim->sps[c], sim->n, gate,
                              s);
            launch_list_build(sim->precision, sim->w.fb, sim->w.cb, g, lb, pp, s, &sim->timer);
        } else {
            const StateMove mv = sim_move(sim);
            if (!drifted)
                launch_drift(da, g, sim->w.cb, sim->w.err, s, &sim->timer);
            launch_scan(sim->w.cb, g, sim->w.chunk, s, &sim->timer);
            launch_scatter_rank(sim->xs[c], sim->sps[c], sim->n, g, sim->w.cb, sim->w.fb.stg64,
                                sim->w.fb.stgq, s, &sim->timer, false, nullptr, nullptr, &mv);
            sim->cur = 1 - c;
        }
        const bool thermo = gi.rescale_every > 0 && (n0 + 1) % gi.rescale_every == 0;
        double* v = sim->vs[sim->cur];
        KickArgs kick{v, hdtm, sim->pot.mass, thermo ? sim->w.fb.ke_part : nullptr, true};
        const double L_next = box_side(sim, n0 + 2);
        const bool fuse = !sim->w.lists && g_tuning.fused_forces && !thermo && k + 1 < nsteps &&
                          box_ok(L_next);
        NextDrift nd{};
        if (fuse) {
            const Grid g2 = make_force_grid(L_next, sim->r_cell, sim->n, CELL_SUB);
            nd.pos = sim->xs[sim->cur];
            nd.species = sim->sps[sim->cur];
            nd.key = sim->w.cb.key;
            nd.count = sim->w.cb.count;
            nd.step = DriftStep{hdtm, gi.dt, L_next, L_next / L_new, gi.scale_positions};
            nd.nc = g2.nc;
            nd.C = g2.C;
            nd.sub = g2.sub;
            nd.inv_w = g2.inv_w;
            kick.next = &nd;
        }
        eval_forces(sim->precision, PASTA_TERM_ALL, sim->w, g, sim->n, sim->Z, pp, sim->force,
                    nullptr, kick, nullptr, s, &sim->timer, sim->xs[sim->cur], nullptr);
        drifted = fuse;
        sim->epot_valid = false;
        if (thermo)
            launch_thermostat(v, sim->n, sim->w.fb.ke_part,
                              g_tuning.fused_forces ? sim->w.fb.n_ke : sim->w.cb.n_items,
                              1.5 * (double)sim->n * gi.T, sim->w.scale, s, &sim->timer);
        sim->step = n0 + 1;
    }
    if (nsteps > 0)
        sim_export(sim);
    PASTA_HIP(hipGetLastError());
    return PASTA_OK;
}

static int sum_on_device(pasta_sim* sim, const double* x, int64_t n, int kind, double* out)
{
    hipStream_t s = sim->stream;
    launch_partial_sums(x, n, kind, sim->pot.mass, sim->w.red, 256, s);
    double h[256];
    PASTA_HIP(hipMemcpyAsync(h, sim->w.red, sizeof(h), hipMemcpyDeviceToHost, s));
    PASTA_HIP(hipStreamSynchronize(s));
    double acc = 0.0;
    for (double v : h)
        acc += v;
    *out = acc;
    return PASTA_OK;
}

extern "C" int pasta_sim_energies(pasta_sim* sim, double* h_ekin, double* h_epot, double* h_L,
                                  int64_t* h_step)
{
    if (!sim)
        return fail(PASTA_EINVAL, "pasta_sim_energies: null sim");
    PASTA_TRY(read_err(sim->w.err, sim->stream, "pasta_sim"));
    if (h_ekin)
        PASTA_TRY(sum_on_device(sim, sim->vel, sim->n, 1, h_ekin));
    if (h_epot) {
        PASTA_TRY(sim_refresh_energies(sim));
        PASTA_TRY(sum_on_device(sim, sim->epot, sim->n, 0, h_epot));
    }
    if (h_L)
        *h_L = box_side(sim, sim->step);
    if (h_step)
        *h_step = sim->step;
    return PASTA_OK;
}

extern "C" int pasta_sim_forces(pasta_sim* sim, double* d_force, double* d_epot)
{
    if (!sim)
        return fail(PASTA_EINVAL, "pasta_sim_forces: null sim");
    if (d_epot)
        PASTA_TRY(sim_refresh_energies(sim));
    launch_export(sim->ids[sim->cur], sim->n, sim->force, d_force, nullptr, nullptr, sim->epot,
                  d_epot, sim->stream);
    PASTA_HIP(hipGetLastError());
    return PASTA_OK;
}

extern "C" int pasta_sim_pair_counts(pasta_sim* sim, int64_t* h_nuclear, int64_t* h_coulomb)
{
    if (!sim)
        return fail(PASTA_EINVAL, "pasta_sim_pair_counts: null sim");
    hipStream_t s = sim->stream;
    const double L = box_side(sim, sim->step);
    const Grid g = make_force_grid(L, sim->r_cell, sim->n, CELL_SUB);
    uint64_t* ctr = sim->w.fb.pairs;
    PASTA_HIP(hipMemsetAsync(ctr, 0, 2 * sizeof(uint64_t), s));
    KickArgs kick{nullptr, 0.0, sim->pot.mass, nullptr, true};
    // the cell list and staging of the current state are in place
    eval_forces(sim->precision, PASTA_TERM_ALL, sim->w, g, sim->n, sim->Z,
                pair_params(&sim->pot, L), sim->force, sim->epot, kick, ctr, s, nullptr,
                sim->xs[sim->cur], nullptr);
    sim->epot_valid = true;
    uint64_t h[2] = {0, 0};
    PASTA_HIP(hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, s));
    PASTA_HIP(hipStreamSynchronize(s));
    if (h_nuclear)
        *h_nuclear = (int64_t)(h[0] / 2);  // ordered -> unordered
    if (h_coulomb)
        *h_coulomb = coulomb_cut_finite(&sim->pot) ? (int64_t)(h[1] / 2)  // ordered -> unordered
                                                   : sim->Z * (sim->Z - 1) / 2;
    return PASTA_OK;
}

extern "C" int pasta_sim_list_stats(pasta_sim* sim, int64_t* h_builds, int64_t* h_overflows,
                                    double* h_max_disp, int64_t* h_rows_used,
                                    int64_t* h_rows_capacity)
{
    if (!sim)
        return fail(PASTA_EINVAL, "pasta_sim_list_stats: null sim");
    ListCtl c{};
    if (sim->w.lists) {
        PASTA_HIP(hipMemcpyAsync(&c, sim->w.lb.ctl, sizeof(c), hipMemcpyDeviceToHost,
                                 sim->stream));
        PASTA_HIP(hipStreamSynchronize(sim->stream));
    }
    if (h_builds)
        *h_builds = (int64_t)c.n_builds;
    if (h_overflows)
        *h_overflows = (int64_t)c.n_overflow + (c.overflow ? 1 : 0);
    if (h_max_disp)
        *h_max_disp = c.max_disp;
    if (h_rows_used)
        *h_rows_used = (int64_t)c.pool_used;
    if (h_rows_capacity)
        *h_rows_capacity = sim->w.lists ? sim->w.lb.pool_rows : 0;
    return PASTA_OK;
}

extern "C" int pasta_sim_get_step(pasta_sim* sim, int64_t* h_step)
{
    if (!sim || !h_step)
        return fail(PASTA_EINVAL, "pasta_sim_get_step: bad argument");
    *h_step = sim->step;
    return PASTA_OK;
}

extern "C" int pasta_sim_get_state(pasta_sim* sim, double* d_pos, double* d_vel, int64_t* h_step)
{
    if (!sim)
        return fail(PASTA_EINVAL, "pasta_sim_get_state: null sim");
    if (d_pos || d_vel)
        launch_export(sim->ids[sim->cur], sim->n, sim->xs[sim->cur], d_pos, sim->vs[sim->cur],
                      d_vel, nullptr, nullptr, sim->stream);
    PASTA_HIP(hipGetLastError());
    if (h_step)
        *h_step = sim->step;
    return PASTA_OK;
}

extern "C" int pasta_sim_set_state(pasta_sim* sim, const double* d_pos, const double* d_vel,
                                   int64_t step)
{
    if (!sim || step < 0)
        return fail(PASTA_EINVAL, "pasta_sim_set_state: bad argument");
    const double L = box_side(sim, step);
    if (L > sim->L_max * (1.0 + 1e-12) || L < 2.0 * max_range(&sim->pot))
        return fail(PASTA_EBOX, "pasta_sim_set_state: box side %g out of range", L);
    hipStream_t s = sim->stream;
    if (d_pos && d_pos != sim->pos)
        PASTA_HIP(hipMemcpyAsync(sim->pos, d_pos, sizeof(double) * 3 * sim->n,
                                 hipMemcpyDeviceToDevice, s));
    if (d_vel && d_vel != sim->vel)
        PASTA_HIP(hipMemcpyAsync(sim->vel, d_vel, sizeof(double) * 3 * sim->n,
                                 hipMemcpyDeviceToDevice, s));
    sim->step = step;
    return sim_eval_initial(sim);
}

extern "C" int pasta_sim_set_timing(pasta_sim* sim, int32_t on)
{
    if (!sim)
        return fail(PASTA_EINVAL, "pasta_sim_set_timing: null sim");
    if (on) {
        PASTA_TRY(timer_collect(&sim->timer, sim->stream));
        for (int k = 0; k < PASTA_KERNEL_CLASSES; ++k) {
            sim->timer.ms[k] = 0.0;
            sim->timer.launches[k] = 0;
            sim->timer.open[k] = -1;
        }
    }
    sim->timer.on = on != 0;
    return PASTA_OK;
}

extern "C" int pasta_sim_kernel_times(pasta_sim* sim, double* h_ms, int64_t* h_launches)
{
    if (!sim)
        return fail(PASTA_EINVAL, "pasta_sim_kernel_times: null sim");
    PASTA_TRY(timer_collect(&sim->timer, sim->stream));
    for (int k = 0; k < PASTA_KERNEL_CLASSES; ++k) {
        if (h_ms)
            h_ms[k] = sim->timer.ms[k];
        if (h_launches)
            h_launches[k] = sim->timer.launches[k];
    }
    return PASTA_OK;
}

extern "C" void pasta_sim_destroy(pasta_sim* sim)
{
    if (!sim)
        return;
    (void)hipStreamSynchronize(sim->stream);
    delete sim;
}
