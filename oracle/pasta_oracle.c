/*
 * FP64 CPU oracle for the nuclear-pasta molecular-dynamics hot path
 * (Caplan, Schneider, Horowitz, Berry, "Pasta Nucleosynthesis: Molecular
 * dynamics simulations of nuclear statistical equilibrium", arXiv:1412.8502).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * path never does.  It shares no code, header, table or constant with the HIP
 * library: every constant below is restated from the paper.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 *        (no FMA contraction, so distance arithmetic is the literal
 *        expression written here).
 *
 * Functions and the passages they follow:
 *   oracle_forces      Sec. II.A, Eq. (1a-c), Table I, the cutoff paragraph
 *                      after Eq. (2) (nuclear cut at r_nuc, Coulomb uncut,
 *                      nearest periodic image only).  Brute force over all
 *                      pairs, per-target Neumaier-compensated sums, sources
 *                      visited in ascending index order.
 *   oracle_pair_counts the same pair loop, counting pairs inside the
 *                      nuclear cutoff and proton-proton pairs evaluated.
 *   oracle_run         Sec. II.A, Eq. (3a,b) and the two paragraphs after
 *                      it: velocity Verlet, box growth after the step,
 *                      positions and velocities not rescaled, velocity
 *                      rescale to <KE> = (3/2)kT every `rescale_every` steps.
 *   oracle_cluster     Sec. II.C (cluster algorithm): protons linked when
 *                      within r_pp (transitively); a neutron belongs to the
 *                      cluster of a proton within r_np; nearest image.
 *   oracle_cell_list   the cell binning of Sec. II.B.2 (cells of width at
 *                      least the cutoff), as a plain definition: the order of
 *                      particles by (species, cell, index).
 * Readings of points the paper leaves open are listed at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double a;           /* MeV, Table I                              */
    double b;           /* MeV, Table I                              */
    double c;           /* MeV, Table I                              */
    double Lambda;      /* fm^2, Table I                             */
    double lambda_s;    /* screening length, fm (fixed to 10 fm)     */
    double alpha_hbarc; /* MeV fm (alpha times hbar c)               */
    double mass;        /* nucleon mass, MeV                         */
    double r_nuc;       /* nuclear cutoff, fm (11.5)                 */
    double r_coul;      /* Coulomb cutoff, fm; <= 0 or inf = uncut   */
} oracle_potential;

typedef struct {
    double dt;            /* fm/c                                    */
    double xi_dot;        /* box expansion rate, c/fm                */
    double T;             /* thermostat temperature, MeV (k_B = 1)   */
    int32_t rescale_every;   /* velocity-rescale period; 0 = none    */
    int32_t scale_positions; /* 1: x scaled with the box (variant)   */
} oracle_integrator;

/* ---- nearest periodic image (reading: positions held in [0, L); the strict
 *      comparisons make the difference antisymmetric, d(i,j) = -d(j,i)) ---- */
static double min_image(double d, double L)
{
    if (d > 0.5 * L)
        d -= L;
    else if (d < -0.5 * L)
        d += L;
    return d;
}

/* Neumaier (improved Kahan) compensated accumulator. */
typedef struct { double s, comp; } nsum;
static void nsum_add(nsum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->comp += (a->s - t) + x;
    else
        a->comp += (x - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum* a) { return a->s + a->comp; }

static int coulomb_uncut(const oracle_potential* p)
{
    return !(p->r_coul > 0.0) || isinf(p->r_coul);
}

/*
 * Force and potential-energy share on one target i from all sources j != i.
 * Eq. (1a,b): V = a exp(-r^2/Lambda) + [b -/+ c] exp(-r^2/(2 Lambda)),
 *   minus for a neutron-proton pair, plus for like pairs; zero and not
 *   computed for r >= r_nuc (reading: strict r < r_nuc is inside).
 * Eq. (1c): proton-proton pairs add (alpha/r) exp(-r/lambda), with alpha
 *   carrying hbar c, i.e. alpha_hbarc / r * exp(-r/lambda); no cutoff.
 * Force on i: F_i = sum_j -dV/dr * (x_i - x_j)/r, with
 *   -dV/dr / r = (2a/Lambda) e^{-r^2/Lambda} + ([b-/+c]/Lambda) e^{-r^2/2Lambda}
 *              + V_C (1/r + 1/lambda) / r.
 * Each pair's energy is split evenly between its two members, so the sum of
 * the per-particle shares is the total potential energy.
 * terms: bit 0 = nuclear, bit 1 = Coulomb.
 */
static void force_on(int64_t i, int64_t n, double L, const double* pos,
                     const uint8_t* species, const oracle_potential* p,
                     int terms, double* f_out, double* e_out)
{
    nsum fx = {0, 0}, fy = {0, 0}, fz = {0, 0}, e = {0, 0};
    const double rn2 = p->r_nuc * p->r_nuc;
    const int uncut = coulomb_uncut(p);
    const double rc2 = uncut ? 0.0 : p->r_coul * p->r_coul;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i)
            continue;
        double dx = min_image(pos[3 * i + 0] - pos[3 * j + 0], L);
        double dy = min_image(pos[3 * i + 1] - pos[3 * j + 1], L);
        double dz = min_image(pos[3 * i + 2] - pos[3 * j + 2], L);
        double r2 = (dx * dx + dy * dy) + dz * dz;
        double fs = 0.0, v = 0.0;
        int any = 0;
        if ((terms & 1) && r2 < rn2) {
            double bb = (species[i] == species[j]) ? (p->b + p->c) : (p->b - p->c);
            double e1 = exp(-r2 / p->Lambda);
            double e2 = exp(-r2 / (2.0 * p->Lambda));
            v += p->a * e1 + bb * e2;
            fs += (2.0 * p->a / p->Lambda) * e1 + (bb / p->Lambda) * e2;
            any = 1;
        }
        if ((terms & 2) && species[i] == 1 && species[j] == 1 && (uncut || r2 < rc2)) {
            double r = sqrt(r2);
            double vc = p->alpha_hbarc * exp(-r / p->lambda_s) / r;
            v += vc;
            fs += vc * (1.0 / r + 1.0 / p->lambda_s) / r;
            any = 1;
        }
        if (any) {
            nsum_add(&fx, fs * dx);
            nsum_add(&fy, fs * dy);
            nsum_add(&fz, fs * dz);
            nsum_add(&e, 0.5 * v);
        }
    }
    f_out[0] = nsum_get(&fx);
    f_out[1] = nsum_get(&fy);
    f_out[2] = nsum_get(&fz);
    *e_out = nsum_get(&e);
}

/*
 * Forces [ntargets][3] (MeV/fm) and per-particle energy shares [ntargets]
 * (MeV) on the listed targets (all particles when targets == NULL).
 * pos is [n][3] in fm, each coordinate in [0, L); species 0 = n, 1 = p.
 */
void oracle_forces(int64_t n, double L, const double* pos, const uint8_t* species,
                   const oracle_potential* p, int terms, const int64_t* targets,
                   int64_t ntargets, double* force, double* epot, int nthreads)
{
    if (targets == NULL)
        ntargets = n;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t t = 0; t < ntargets; ++t) {
        int64_t i = targets ? targets[t] : t;
        double e;
        force_on(i, n, L, pos, species, p, terms, force + 3 * t, &e);
        if (epot)
            epot[t] = e;
    }
}

/* Unordered pair counts: pairs with r < r_nuc, and proton-proton pairs whose
 * Coulomb term is evaluated (all of them when uncut). */
void oracle_pair_counts(int64_t n, double L, const double* pos, const uint8_t* species,
                        const oracle_potential* p, int64_t* n_nuc, int64_t* n_coul,
                        int nthreads)
{
    const double rn2 = p->r_nuc * p->r_nuc;
    const int uncut = coulomb_uncut(p);
    const double rc2 = uncut ? 0.0 : p->r_coul * p->r_coul;
    int64_t cn = 0, cc = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : cn, cc) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
            double dx = min_image(pos[3 * i + 0] - pos[3 * j + 0], L);
            double dy = min_image(pos[3 * i + 1] - pos[3 * j + 1], L);
            double dz = min_image(pos[3 * i + 2] - pos[3 * j + 2], L);
            double r2 = (dx * dx + dy * dy) + dz * dz;
            if (r2 < rn2)
                cn++;
            if (species[i] == 1 && species[j] == 1 && (uncut || r2 < rc2))
                cc++;
        }
    }
    *n_nuc = cn;
    *n_coul = cc;
}

static double kinetic(int64_t n, const double* vel, double mass)
{
    nsum k = {0, 0};
    for (int64_t i = 0; i < 3 * n; ++i)
        nsum_add(&k, 0.5 * mass * vel[i] * vel[i]);
    return nsum_get(&k);
}

/* Box side after `step` steps, Eq. (3a): l(t) = l(0) (1 + xi_dot t), t = step dt.
 * Computed directly from the step index, never accumulated. */
double oracle_box_length(double L0, double xi_dot, double dt, int64_t step)
{
    return L0 * (1.0 + xi_dot * ((double)step * dt));
}

/*
 * Advance (pos, vel) from global step `step0` by `nsteps` velocity-Verlet
 * steps, in place.  Readings:
 *   - the box side used for the force after step n -> n+1 is L_{n+1}: the box
 *     grows once the step's drift is complete (the paper: "after the timestep
 *     is completed"), and forces are always evaluated in the current box;
 *   - positions are not scaled with the box (the paper's statement) unless
 *     scale_positions = 1, which multiplies x by L_{n+1}/L_n;
 *   - a particle that leaves through a face re-enters through the opposite
 *     one with unchanged velocity (two-branch wrap into [0, L));
 *   - the velocity rescale acts after the second half kick of every step
 *     whose new global index is a multiple of rescale_every, to
 *     KE = (3/2) N T exactly (N, not N - 1; no centre-of-mass removal);
 *   - kinetic energy is non-relativistic, (1/2) M v^2.
 * Outputs: final L, KE and potential energy at the final state, and the
 * final forces (optional, [n][3]).
 */
int oracle_run(int64_t n, double* pos, double* vel, const uint8_t* species,
               const oracle_potential* p, const oracle_integrator* g, double L0,
               int64_t step0, int64_t nsteps, double* L_out, double* ekin_out,
               double* epot_out, double* force_out, int nthreads)
{
    double* F = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* E = (double*)malloc(sizeof(double) * (size_t)n);
    if (!F || !E) {
        free(F);
        free(E);
        return -1;
    }
    const double M = p->mass;
    double L = oracle_box_length(L0, g->xi_dot, g->dt, step0);
    oracle_forces(n, L, pos, species, p, 3, NULL, n, F, E, nthreads);
    for (int64_t s = 0; s < nsteps; ++s) {
        int64_t step = step0 + s;
        for (int64_t k = 0; k < 3 * n; ++k) {
            vel[k] += (g->dt / (2.0 * M)) * F[k];
            pos[k] += g->dt * vel[k];
        }
        double Lnew = oracle_box_length(L0, g->xi_dot, g->dt, step + 1);
        if (g->scale_positions) {
            for (int64_t k = 0; k < 3 * n; ++k)
                pos[k] *= Lnew / L;
        }
        L = Lnew;
        for (int64_t k = 0; k < 3 * n; ++k) {
            if (pos[k] < 0.0)
                pos[k] += L;
            if (pos[k] >= L)
                pos[k] -= L;
        }
        oracle_forces(n, L, pos, species, p, 3, NULL, n, F, E, nthreads);
        for (int64_t k = 0; k < 3 * n; ++k)
            vel[k] += (g->dt / (2.0 * M)) * F[k];
        if (g->rescale_every > 0 && (step + 1) % g->rescale_every == 0) {
            double ke = kinetic(n, vel, M);
            double scale = sqrt(1.5 * (double)n * g->T / ke);
            for (int64_t k = 0; k < 3 * n; ++k)
                vel[k] *= scale;
        }
    }
    if (L_out)
        *L_out = L;
    if (ekin_out)
        *ekin_out = kinetic(n, vel, M);
    if (epot_out) {
        nsum e = {0, 0};
        for (int64_t i = 0; i < n; ++i)
            nsum_add(&e, E[i]);
        *epot_out = nsum_get(&e);
    }
    if (force_out)
        memcpy(force_out, F, sizeof(double) * 3 * (size_t)n);
    free(F);
    free(E);
    return 0;
}

double oracle_kinetic(int64_t n, const double* vel, double mass) { return kinetic(n, vel, mass); }

/* ---------------------------------------------------------------- clusters */

static double dist2(const double* pos, int64_t i, int64_t j, double L)
{
    double dx = min_image(pos[3 * i + 0] - pos[3 * j + 0], L);
    double dy = min_image(pos[3 * i + 1] - pos[3 * j + 1], L);
    double dz = min_image(pos[3 * i + 2] - pos[3 * j + 2], L);
    return (dx * dx + dy * dy) + dz * dz;
}

static int64_t uf_find(int64_t* parent, int64_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]]; /* path halving: roots are unchanged */
        x = parent[x];
    }
    return x;
}

/*
 * Cluster algorithm of Sec. II.C.  Readings:
 *   - "within" is inclusive: |d|^2 <= r_pp^2 (r_pp^2 = 20.25 fm^2 and
 *     r_np^2 = 9 fm^2 are exact in binary);
 *   - proton clusters are the connected components of the graph joining
 *     protons within r_pp (transitive membership); an isolated proton is a
 *     cluster of its own;
 *   - a neutron within r_np of protons of two clusters joins the cluster of
 *     its nearest such proton, ties going to the lower proton index;
 *   - clusters are numbered 0..K-1 in increasing order of their smallest
 *     proton index (canonical labels); free neutrons get label -1.
 * Outputs: label[n], *nclusters, hist_A[A] = number of clusters with mass
 * number A (size n+1), hist_Z[Z] = number with charge Z (size n+1), *nfree.
 */
int oracle_cluster(int64_t n, double L, const double* pos, const uint8_t* species,
                   double r_pp, double r_np, int32_t* label, int32_t* nclusters,
                   int32_t* hist_A, int32_t* hist_Z, int32_t* nfree, int nthreads)
{
    const double rpp2 = r_pp * r_pp, rnp2 = r_np * r_np;
    int64_t* parent = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* canon = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t* zc = (int32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int32_t* ac = (int32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    if (!parent || !canon || !zc || !ac) {
        free(parent); free(canon); free(zc); free(ac);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i)
        parent[i] = i;
    /* the protons in increasing index: the pair loops below visit only
     * protons, in the order a loop over every particle would reach them */
    int64_t Z = 0;
    for (int64_t i = 0; i < n; ++i)
        if (species[i] == 1)
            canon[Z++] = i;
    int64_t* prot = (int64_t*)malloc(sizeof(int64_t) * (size_t)(Z > 0 ? Z : 1));
    int64_t* row = (int64_t*)calloc((size_t)Z + 1, sizeof(int64_t));
    if (!prot || !row) {
        free(parent); free(canon); free(zc); free(ac); free(prot); free(row);
        return -1;
    }
    memcpy(prot, canon, sizeof(int64_t) * (size_t)Z);
    /* union over every proton pair within r_pp; the smaller root becomes the
     * root, so each component's root is its smallest proton index.  The
     * distance tests run in parallel, one row (proton a, partners b > a) per
     * iteration, counted and then listed; the unions then take the linked
     * pairs serially in increasing (a, b), the order of a double loop. */
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t a = 0; a < Z; ++a) {
        int64_t c = 0;
        for (int64_t b = a + 1; b < Z; ++b)
            if (dist2(pos, prot[a], prot[b], L) <= rpp2)
                c++;
        row[a + 1] = c;
    }
    for (int64_t a = 0; a < Z; ++a)
        row[a + 1] += row[a];
    int64_t* link = (int64_t*)malloc(sizeof(int64_t) * (size_t)(row[Z] > 0 ? row[Z] : 1));
    if (!link) {
        free(parent); free(canon); free(zc); free(ac); free(prot); free(row);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t a = 0; a < Z; ++a) {
        int64_t c = row[a];
        for (int64_t b = a + 1; b < Z; ++b)
            if (dist2(pos, prot[a], prot[b], L) <= rpp2)
                link[c++] = prot[b];
    }
    for (int64_t a = 0; a < Z; ++a) {
        for (int64_t e = row[a]; e < row[a + 1]; ++e) {
            int64_t ri = uf_find(parent, prot[a]), rj = uf_find(parent, link[e]);
            if (ri < rj)
                parent[rj] = ri;
            else if (rj < ri)
                parent[ri] = rj;
        }
    }
    free(link);
    free(row);
    /* canonical numbering in increasing root index */
    int32_t K = 0;
    for (int64_t i = 0; i < n; ++i)
        canon[i] = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (species[i] == 1 && uf_find(parent, i) == i)
            canon[i] = K++;
    }
    for (int64_t i = 0; i < n; ++i)
        label[i] = (species[i] == 1) ? (int32_t)canon[uf_find(parent, i)] : -1;
    /* neutrons: nearest proton within r_np, lower index on ties */
    int32_t free_count = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : free_count) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t k = 0; k < n; ++k) {
        if (species[k] == 1)
            continue;
        int64_t best = -1;
        double bd = 0.0;
        for (int64_t b = 0; b < Z; ++b) {
            const int64_t j = prot[b];
            double d2 = dist2(pos, k, j, L);
            if (d2 <= rnp2 && (best < 0 || d2 < bd)) {
                best = j;
                bd = d2;
            }
        }
        if (best >= 0)
            label[k] = label[best];
        else {
            label[k] = -1;
            free_count++;
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        if (label[i] < 0)
            continue;
        ac[label[i]]++;
        if (species[i] == 1)
            zc[label[i]]++;
    }
    if (hist_A)
        memset(hist_A, 0, sizeof(int32_t) * (size_t)(n + 1));
    if (hist_Z)
        memset(hist_Z, 0, sizeof(int32_t) * (size_t)(n + 1));
    for (int32_t c = 0; c < K; ++c) {
        if (hist_A)
            hist_A[ac[c]]++;
        if (hist_Z)
            hist_Z[zc[c]]++;
    }
    *nclusters = K;
    if (nfree)
        *nfree = free_count;
    free(parent); free(canon); free(zc); free(ac); free(prot);
    return 0;
}

/* ---------------------------------------------------------------- cell list */

/*
 * Cell binning as a definition (Sec. II.B.2 bins the volume into cubic cells
 * no narrower than the interaction range).  ncell = the largest integer with
 * L / ncell >= rcut (at least 1).  A particle's cell along one axis is
 * floor(x * (ncell / L)), clamped to ncell - 1; the linear cell index is
 * (cz * ncell + cy) * ncell + cx.  Protons are listed before neutrons: bin =
 * cell for a proton, ncell^3 + cell for a neutron.  perm lists particle
 * indices in increasing (bin, index); cell_start[b] is the first position of
 * bin b in perm, b = 0..2 ncell^3 (the last entry is n).
 */
int oracle_cell_dims(double L, double rcut)
{
    int nc = (int)floor(L / rcut);
    while (nc > 1 && L / (double)nc < rcut)
        nc--;
    return nc < 1 ? 1 : nc;
}

static int64_t g_bins_for_sort_n;
static const int64_t* g_bins_for_sort;
static int cmp_by_bin(const void* pa, const void* pb)
{
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    int64_t ba = g_bins_for_sort[a], bb = g_bins_for_sort[b];
    if (ba != bb)
        return ba < bb ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

int oracle_cell_list(int64_t n, double L, double rcut, const double* pos,
                     const uint8_t* species, int32_t* ncell_out, int32_t* cell_start,
                     int32_t* perm)
{
    int nc = oracle_cell_dims(L, rcut);
    int64_t C = (int64_t)nc * nc * nc;
    int64_t* bin = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!bin || !idx) {
        free(bin); free(idx);
        return -1;
    }
    const double inv_w = (double)nc / L;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c3[3];
        for (int a = 0; a < 3; ++a) {
            int64_t k = (int64_t)(pos[3 * i + a] * inv_w);
            if (k > nc - 1)
                k = nc - 1;
            if (k < 0)
                k = 0;
            c3[a] = k;
        }
        int64_t cell = (c3[2] * nc + c3[1]) * nc + c3[0];
        bin[i] = (species[i] == 1 ? 0 : C) + cell;
        idx[i] = i;
    }
    g_bins_for_sort = bin;
    g_bins_for_sort_n = n;
    qsort(idx, (size_t)n, sizeof(int64_t), cmp_by_bin);
    for (int64_t i = 0; i < n; ++i)
        perm[i] = (int32_t)idx[i];
    int64_t pos_i = 0;
    for (int64_t b = 0; b <= 2 * C; ++b) {
        while (pos_i < n && bin[idx[pos_i]] < b)
            pos_i++;
        cell_start[b] = (int32_t)pos_i;
    }
    *ncell_out = nc;
    free(bin);
    free(idx);
    return 0;
}
