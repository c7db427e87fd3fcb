// Host driver for the sanitizer build (AddressSanitizer + UndefinedBehavior
// Sanitizer on the host code of libpasta): every entry point's argument
// checks, each of which must refuse before touching a device, so this runs
// without a GPU.  Prints one line per check and "abi checks ok" at the end;
// exits non-zero on the first unexpected return code.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>

#include "../../include/pasta.h"

static int failures = 0;

static void expect(const char* what, int got, int want)
{
    std::printf("%-46s rc %3d (want %3d)  %s\n", what, got, want,
                got == want ? "" : pasta_last_error());
    if (got != want)
        ++failures;
}

int main()
{
    pasta_potential p;
    pasta_potential_paper(&p);
    if (!std::isinf(p.r_coul) || p.r_nuc != 11.5) {
        std::printf("paper potential wrong\n");
        return 1;
    }
    // a device-looking pointer that is never dereferenced: every call below
    // fails its argument checks first
    void* fake = reinterpret_cast<void*>(uintptr_t(1) << 20);
    double* fd = static_cast<double*>(fake);
    uint8_t* fs = static_cast<uint8_t*>(fake);
    int32_t nc = 0;
    size_t nb = 0;

    expect("cell_dims", pasta_cell_dims(86.18, 11.5, &nc), PASTA_OK);
    expect("cell_dims value", nc, 7);
    expect("cell_dims bad L", pasta_cell_dims(-1.0, 11.5, &nc), PASTA_EINVAL);
    expect("cell_dims null", pasta_cell_dims(86.18, 11.5, nullptr), PASTA_EINVAL);
    expect("cell_list_workspace", pasta_cell_list_workspace(3200, 43.09, 11.5, &nb), PASTA_OK);
    expect("cell_list box", pasta_cell_list(10, 20.0, 11.5, fd, fs, static_cast<int32_t*>(fake),
                                            static_cast<int32_t*>(fake), &nc, fake, 1u << 30,
                                            nullptr), PASTA_EBOX);
    for (int prec : {PASTA_FP64, PASTA_MIXED})
        expect("forces_workspace", pasta_forces_workspace(&p, prec, 51200, 86.18, &nb), PASTA_OK);
    expect("forces n < 0", pasta_forces(&p, 0, 3, -1, 86.0, fd, fs, fd, nullptr, fake, 1u << 30,
                                        nullptr), PASTA_EINVAL);
    expect("forces precision", pasta_forces(&p, 7, 3, 10, 86.0, fd, fs, fd, nullptr, fake,
                                            1u << 30, nullptr), PASTA_EINVAL);
    expect("forces terms", pasta_forces(&p, 0, 8, 10, 86.0, fd, fs, fd, nullptr, fake, 1u << 30,
                                        nullptr), PASTA_EINVAL);
    expect("forces null pos", pasta_forces(&p, 0, 3, 10, 86.0, nullptr, fs, fd, nullptr, fake,
                                           1u << 30, nullptr), PASTA_EINVAL);
    expect("forces box", pasta_forces(&p, 0, 3, 10, 22.9, fd, fs, fd, nullptr, fake, 1u << 30,
                                      nullptr), PASTA_EBOX);
    expect("forces workspace small", pasta_forces(&p, 0, 3, 10, 30.0, fd, fs, fd, nullptr, fake,
                                                  16, nullptr), PASTA_EWORKSPACE);
    expect("forces workspace misaligned",
           pasta_forces(&p, 0, 3, 10, 30.0, fd, fs, fd, nullptr,
                        reinterpret_cast<void*>((uintptr_t(1) << 20) + 8), 1u << 30, nullptr),
           PASTA_EWORKSPACE);
    expect("noalloc beyond scratch", pasta_forces_noalloc(&p, 0, 3, 4000000, 400.0, fd, fs, fd,
                                                          nullptr, nullptr), PASTA_EWORKSPACE);
    pasta_potential bad = p;
    bad.Lambda = NAN;
    expect("forces NaN Lambda", pasta_forces(&bad, 0, 3, 10, 30.0, fd, fs, fd, nullptr, fake,
                                             1u << 30, nullptr), PASTA_EINVAL);
    bad = p;
    bad.r_coul = NAN;
    expect("forces NaN r_coul", pasta_forces(&bad, 0, 3, 10, 30.0, fd, fs, fd, nullptr, fake,
                                             1u << 30, nullptr), PASTA_EINVAL);
    bad.r_coul = 20.0;
    expect("forces box below 2 r_coul", pasta_forces(&bad, 0, 3, 10, 39.0, fd, fs, fd, nullptr,
                                                     fake, 1u << 30, nullptr), PASTA_EBOX);
    expect("forces null potential", pasta_forces(nullptr, 0, 3, 10, 30.0, fd, fs, fd, nullptr,
                                                 fake, 1u << 30, nullptr), PASTA_EINVAL);

    pasta_integrator g{2.0, 0.0, 1.0, 100, 0};
    expect("sim_workspace", pasta_sim_workspace(&p, &g, 1, 51200, 86.18, 344.71, &nb), PASTA_OK);
    pasta_integrator gb{-1.0, 0.0, 1.0, 0, 0};
    expect("sim_workspace bad dt", pasta_sim_workspace(&p, &gb, 0, 10, 30.0, 30.0, &nb),
           PASTA_EINVAL);
    pasta_sim* sim = nullptr;
    expect("sim_create box", pasta_sim_create(&p, &g, 0, 10, 20.0, 0, 20.0, fd, fd, fs, fake,
                                              1u << 30, nullptr, &sim), PASTA_EBOX);
    expect("sim_step null", pasta_sim_step(nullptr, 1), PASTA_EINVAL);
    expect("sim_energies null", pasta_sim_energies(nullptr, nullptr, nullptr, nullptr, nullptr),
           PASTA_EINVAL);
    expect("sim_get_state null", pasta_sim_get_state(nullptr, nullptr, nullptr, nullptr),
           PASTA_EINVAL);
    expect("sim_set_state null", pasta_sim_set_state(nullptr, fd, fd, 0), PASTA_EINVAL);
    pasta_sim_destroy(nullptr);

    expect("cluster_workspace", pasta_cluster_workspace(3200, 43.09, 4.5, 3.0, &nb), PASTA_OK);
    int32_t K = 0;
    expect("cluster box", pasta_cluster(10, 8.0, fd, fs, 4.5, 3.0, static_cast<int32_t*>(fake),
                                        static_cast<int32_t*>(fake), static_cast<int32_t*>(fake),
                                        &K, nullptr, fake, 1u << 30, nullptr), PASTA_EBOX);

    const int64_t ns[2] = {1000, 2000};
    const double lm[2] = {40.0, 50.0};
    expect("batch_workspace", pasta_batch_workspace(&p, 1, 2, ns, lm, &nb), PASTA_OK);
    expect("batch_workspace cut", pasta_batch_workspace(&bad, 1, 2, ns, lm, &nb), PASTA_EINVAL);
    expect("batch_step null", pasta_batch_step(nullptr, 1), PASTA_EINVAL);
    expect("batch_wait_limit null", pasta_batch_set_wait_limit(nullptr, 0), PASTA_EINVAL);
    pasta_batch_destroy(nullptr);

    pasta_tuning t{};
    expect("get_tuning", pasta_get_tuning(&t), PASTA_OK);
    pasta_tuning tb = t;
    tb.nuclear_variant = 9;
    expect("set_tuning bad variant", pasta_set_tuning(&tb), PASTA_EINVAL);
    tb = t;
    tb.list_skin = NAN;
    expect("set_tuning NaN halo", pasta_set_tuning(&tb), PASTA_EINVAL);
    expect("set_tuning null", pasta_set_tuning(nullptr), PASTA_EINVAL);
    expect("autotune bad reps", pasta_autotune(&p, 1, 100, 30.0, fd, fs, fake, 1u << 30, nullptr,
                                               0, &t, nullptr, nullptr, nullptr), PASTA_EINVAL);
    if (std::strlen(pasta_last_error()) == 0 || std::strlen(pasta_version()) == 0)
        ++failures;
    for (int k = -1; k <= PASTA_KERNEL_CLASSES; ++k)
        if (!pasta_kernel_class_name(k))
            ++failures;
    if (failures) {
        std::printf("%d unexpected results\n", failures);
        return 1;
    }
    std::printf("abi checks ok\n");
    return 0;
}
