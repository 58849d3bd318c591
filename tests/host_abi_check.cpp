// Sanitizer run of the C ABI's host-side argument validation (built by
// tests/test_sanitizers.py from the library sources, host code only, with
// -fsanitize=address,undefined; no GPU is touched).  Every call below must be
// rejected with the documented status before any HIP call, and leave a
// message in gsn_last_error().
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "gsn.h"

static int fails = 0;

static void expect(const char *what, gsn_status got, gsn_status want)
{
    const char *msg = gsn_last_error();
    if (got != want || (want != GSN_OK && (!msg || !*msg))) {
        std::printf("FAIL %s: status %d, expected %d (%s)\n", what, (int)got, (int)want, msg ? msg : "");
        ++fails;
    }
}

int main()
{
    size_t bytes = 0;
    const int32_t n2[2] = {64, 128}, n3[3] = {16, 32, 64}, bad[2] = {48, 64}, tiny[2] = {4, 64},
                  huge[2] = {4096, 64};
    expect("workspace 2-D", gsn_workspace_bytes(2, n2, &bytes), GSN_OK);
    if (bytes < 64 * 128 * 24) { std::printf("FAIL workspace size %zu\n", bytes); ++fails; }
    expect("workspace 3-D", gsn_workspace_bytes(3, n3, &bytes), GSN_OK);
    expect("workspace ndim 1", gsn_workspace_bytes(1, n2, &bytes), GSN_EUNSUPPORTED);
    expect("workspace ndim 4", gsn_workspace_bytes(4, n3, &bytes), GSN_EUNSUPPORTED);
    expect("workspace not pow2", gsn_workspace_bytes(2, bad, &bytes), GSN_EUNSUPPORTED);
    expect("workspace too short", gsn_workspace_bytes(2, tiny, &bytes), GSN_EUNSUPPORTED);
    expect("workspace too long", gsn_workspace_bytes(2, huge, &bytes), GSN_EUNSUPPORTED);
    expect("workspace null n", gsn_workspace_bytes(2, nullptr, &bytes), GSN_EINVAL);
    expect("workspace null out", gsn_workspace_bytes(2, n2, nullptr), GSN_EINVAL);
    expect("workspace_ex dtype", gsn_workspace_bytes_ex(2, n2, 7, &bytes), GSN_EINVAL);

    gsn_grid g = nullptr;
    const double L2[2] = {64.0, 128.0}, Lneg[2] = {64.0, -1.0}, Lnan[2] = {NAN, 1.0};
    std::vector<unsigned char> host(1 << 16);
    void *ws = (void *)(((uintptr_t)host.data() + 255) & ~(uintptr_t)255);
    expect("create null out", gsn_create(nullptr, 2, n2, L2, ws, bytes, nullptr), GSN_EINVAL);
    expect("create bad shape", gsn_create(&g, 2, bad, L2, ws, bytes, nullptr), GSN_EUNSUPPORTED);
    expect("create negative L", gsn_create(&g, 2, n2, Lneg, ws, bytes, nullptr), GSN_EINVAL);
    expect("create NaN L", gsn_create(&g, 2, n2, Lnan, ws, bytes, nullptr), GSN_EINVAL);
    expect("create null L", gsn_create(&g, 2, n2, nullptr, ws, bytes, nullptr), GSN_EINVAL);
    expect("create null workspace", gsn_create(&g, 2, n2, L2, nullptr, bytes, nullptr), GSN_EINVAL);
    expect("create misaligned", gsn_create(&g, 2, n2, L2, (char *)ws + 8, bytes, nullptr), GSN_EWORKSPACE);
    expect("create small workspace", gsn_create(&g, 2, n2, L2, ws, 1024, nullptr), GSN_EWORKSPACE);
    expect("create_ex storage", gsn_create_ex(&g, 2, n2, L2, 9, ws, bytes, nullptr), GSN_EINVAL);
    if (g) { std::printf("FAIL grid handle set on error\n"); ++fails; }

    // calls on a NULL handle
    gsn_kernel k{1.0, 0.3, 0.1, 0.0};
    double d4[4];
    int64_t st = 0;
    int v[32];
    expect("destroy null", gsn_destroy(nullptr), GSN_EINVAL);
    expect("kernel null", gsn_set_kernel(nullptr, &k), GSN_EINVAL);
    expect("coefficients null", gsn_set_coefficients(nullptr, 0.5, 0.0, 1e-3), GSN_EINVAL);
    expect("step null", gsn_step(nullptr, 1), GSN_EINVAL);
    expect("mass null", gsn_mass(nullptr, d4), GSN_EINVAL);
    expect("energy null", gsn_energy(nullptr, d4), GSN_EINVAL);
    expect("phase null", gsn_phase(nullptr, d4, &st), GSN_EINVAL);
    expect("schedule null", gsn_get_schedule(nullptr, v, 32), GSN_EINVAL);
    expect("autotune null", gsn_autotune(nullptr, 3), GSN_EINVAL);
    expect("psi null", gsn_set_psi(nullptr, host.data(), 0, GSN_C64), GSN_EINVAL);
    if (gsn_variant_count() < 1 || std::strlen(gsn_variant_name(0)) == 0 || std::strlen(gsn_variant_name(-1)) != 0 ||
        std::strlen(gsn_variant_name(gsn_variant_count())) != 0) {
        std::printf("FAIL variant names\n");
        ++fails;
    }

    // batches
    const int32_t bn[6] = {64, 64, 128, 64, 32, 32}, bbad[4] = {64, 64, 64, 40};
    const double bL[6] = {64, 64, 128, 64, 32, 32};
    expect("batch workspace", gsn_batch_workspace_bytes(3, 2, bn, &bytes), GSN_OK);
    expect("batch workspace count 0", gsn_batch_workspace_bytes(0, 2, bn, &bytes), GSN_EINVAL);
    expect("batch workspace 3-D", gsn_batch_workspace_bytes(3, 3, bn, &bytes), GSN_EUNSUPPORTED);
    expect("batch workspace bad extent", gsn_batch_workspace_bytes(2, 2, bbad, &bytes), GSN_EUNSUPPORTED);
    gsn_batch b = nullptr;
    expect("batch create null ws", gsn_batch_create(&b, 3, 2, bn, bL, nullptr, bytes, nullptr), GSN_EINVAL);
    expect("batch create small ws", gsn_batch_create(&b, 3, 2, bn, bL, ws, 256, nullptr), GSN_EWORKSPACE);
    expect("batch set null", gsn_batch_set(nullptr, 0, &k, 0.5, 0.0, 1e-3, host.data(), 0, GSN_C64), GSN_EINVAL);
    expect("batch step null", gsn_batch_step(nullptr, 1), GSN_EINVAL);
    expect("batch autotune null", gsn_batch_autotune(nullptr, 2), GSN_EINVAL);
    expect("batch schedule null", gsn_batch_get_schedule(nullptr, 0, v, 5, v), GSN_EINVAL);

    // corrector
    expect("corrector workspace", gsn_corrector_workspace_bytes(64, 64, 2, &bytes), GSN_OK);
    expect("corrector workspace W", gsn_corrector_workspace_bytes(64, 7, 2, &bytes), GSN_EINVAL);
    expect("corrector workspace H*W", gsn_corrector_workspace_bytes(8, 12, 2, &bytes), GSN_EUNSUPPORTED);
    expect("corrector workspace B", gsn_corrector_workspace_bytes(64, 64, 0, &bytes), GSN_EINVAL);
    gsn_corrector c = nullptr;
    expect("corrector create null ws", gsn_corrector_create(&c, 64, 64, 2, nullptr, bytes, nullptr), GSN_EINVAL);
    std::vector<float> w(19970, 0.0f);
    expect("corrector weights null", gsn_corrector_set_weights(nullptr, w.data(), w.size()), GSN_EINVAL);
    expect("corrected step null", gsn_step_corrected(nullptr, nullptr, 1, 0, 0.0, &st, d4), GSN_EINVAL);

    std::printf("fails %d\n", fails);
    return fails != 0;
}
