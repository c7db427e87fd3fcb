/*
 * Host driver of the oracle for the sanitizer build (gcc with
 * AddressSanitizer and UndefinedBehaviorSanitizer): every entry point of
 * pasta_oracle.c on small systems, including the degenerate ones (no
 * particle, one particle, no proton, a finite Coulomb cutoff), with the
 * invariants that need no reference (Newton's third law, labels in range,
 * histogram totals).  Test infrastructure, like the oracle itself.
 */
#include "pasta_oracle.c"

#include <stdio.h>

static uint64_t lcg = 88172645463325252ull;
static double urand(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static int check_system(int64_t n, double L, double yp, double r_coul)
{
    oracle_potential p = {110.0, -26.0, 24.0, 1.25, 10.0, 1.4399645, 939.0, 11.5, r_coul};
    oracle_integrator g = {2.0, 1e-3, 1.0, 3, 0};
    double* pos = calloc((size_t)(3 * n + 3), sizeof(double));
    double* vel = calloc((size_t)(3 * n + 3), sizeof(double));
    double* f = calloc((size_t)(3 * n + 3), sizeof(double));
    double* e = calloc((size_t)(n + 1), sizeof(double));
    uint8_t* sp = calloc((size_t)(n + 1), 1);
    int32_t* label = calloc((size_t)(n + 1), sizeof(int32_t));
    int32_t* hA = calloc((size_t)(n + 2), sizeof(int32_t));
    int32_t* hZ = calloc((size_t)(n + 2), sizeof(int32_t));
    int bad = 0;
    for (int64_t i = 0; i < 3 * n; ++i) {
        pos[i] = urand() * L;
        vel[i] = (urand() - 0.5) * 0.05;
    }
    for (int64_t i = 0; i < n; ++i)
        sp[i] = (double)i < yp * (double)n;
    oracle_forces(n, L, pos, sp, &p, 3, NULL, n, f, e, 4);
    double sx = 0, sm = 0;
    for (int64_t i = 0; i < 3 * n; ++i) {
        sx += f[i];
        sm += fabs(f[i]);
    }
    if (fabs(sx) > 1e-9 * (sm + 1.0))
        bad |= 1;
    int64_t tg[2] = {0, n > 1 ? n - 1 : 0};
    if (n > 0)
        oracle_forces(n, L, pos, sp, &p, 2, tg, 2, f, e, 2);
    int64_t cn = 0, cc = 0;
    oracle_pair_counts(n, L, pos, sp, &p, &cn, &cc, 3);
    double Lr = 0, ek = 0, ep = 0;
    if (oracle_run(n, pos, vel, sp, &p, &g, L, 0, 4, &Lr, &ek, &ep, f, 2) != 0)
        bad |= 2;
    int32_t K = 0, nf = 0;
    if (oracle_cluster(n, Lr, pos, sp, 4.5, 3.0, label, &K, hA, hZ, &nf, 3) != 0)
        bad |= 4;
    int64_t sumA = 0;
    for (int64_t a = 0; a <= n; ++a)
        sumA += a * hA[a];
    if (sumA + nf != n)
        bad |= 8;
    for (int64_t i = 0; i < n; ++i)
        if (label[i] < -1 || label[i] >= K)
            bad |= 16;
    if (n > 0) {
        int nc = oracle_cell_dims(Lr, 11.5);
        int32_t* start = calloc((size_t)(2 * nc * nc * nc + 1), sizeof(int32_t));
        int32_t* perm = calloc((size_t)n, sizeof(int32_t));
        int32_t ncell = 0;
        if (oracle_cell_list(n, Lr, 11.5, pos, sp, &ncell, start, perm) != 0 || ncell != nc ||
            start[2 * nc * nc * nc] != n)
            bad |= 32;
        free(start);
        free(perm);
    }
    printf("n %lld L %.2f yp %.2f r_coul %g: K %d free %d pairs %lld/%lld flags %d\n",
           (long long)n, L, yp, r_coul, K, nf, (long long)cn, (long long)cc, bad);
    free(pos); free(vel); free(f); free(e); free(sp); free(label); free(hA); free(hZ);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= check_system(0, 30.0, 0.4, INFINITY);
    bad |= check_system(1, 30.0, 1.0, INFINITY);
    bad |= check_system(2, 25.0, 0.5, INFINITY);
    bad |= check_system(300, 30.0, 0.0, INFINITY);
    bad |= check_system(500, 40.0, 0.4, INFINITY);
    bad |= check_system(400, 45.0, 0.4, 20.0);
    bad |= check_system(200, 24.0, 1.0, INFINITY);
    printf(bad ? "oracle sanitizer run FAILED\n" : "oracle sanitizer run ok\n");
    return bad ? 1 : 0;
}
