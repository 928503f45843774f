// Host-only exercise of the C ABI (include/tc.h) for the sanitizer build:
// geometry validation, host-only (TC_FLAG_DRYRUN) contexts of several shapes
// and instance counts, every query that works on them, the device calls that
// must refuse them, and tc_destroy.  Built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (host_setup.cpp, tc_api.cpp and
// this driver); no call here reaches the GPU.  Prints one line per check and
// exits non-zero on the first failure.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/tc.h"

static int failures = 0;

#define CHECK(cond)                                                     \
    do {                                                                \
        if (!(cond)) {                                                  \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

static tc_geometry base(int nr, int nt, int nz, double stretch) {
    tc_geometry g;
    std::memset(&g, 0, sizeof(g));
    g.radius_ratio = 0.883;
    g.gap = 1.0;
    g.re = 2000.0;
    g.re_outer = 0.0;
    g.nr = nr;
    g.ntheta = nt;
    g.nz = nz;
    g.stretch = stretch;
    g.dt = 1e-3;
    g.precision = TC_PREC_FP64;
    g.flags = TC_FLAG_DRYRUN;
    return g;
}

static void check_context(tc_ctx* c, int inst, const tc_geometry& g) {
    int nr = 0, nj = 0, nl = 0;
    CHECK(tc_mode_shape(c, inst, &nr, &nj, &nl) == TC_OK);
    CHECK(nr == g.nr && nj == (g.ntheta - 1) / 3 + 1 && nl == 2 * ((g.nz - 1) / 3) + 1);
    std::vector<double> r(nr);
    CHECK(tc_grid(c, inst, r.data()) == TC_OK);
    for (int n = 1; n < nr; ++n) CHECK(r[n] > r[n - 1]);
    std::vector<double> coef((size_t)5 * nr * 5);
    std::vector<int> sigma(nr);
    CHECK(tc_coefficients(c, inst, coef.data(), sigma.data()) == TC_OK);
    CHECK(tc_coefficients(c, inst, nullptr, nullptr) == TC_OK);
    for (int n = 0; n < nr; ++n) {
        CHECK(sigma[n] >= 0 && sigma[n] <= nr - 5);
        double s0 = 0.0;
        for (int j = 0; j < 5; ++j) s0 += coef[(size_t)n * 5 + j];
        CHECK(std::fabs(s0 - 1.0) < 1e-12);  // the d0 rows sum to one
        for (size_t q = 0; q < 5; ++q) CHECK(std::isfinite(coef[(q * nr + n) * 5]));
    }
    int rr = 0, sh = 0;
    CHECK(tc_tuning(c, inst, &rr, &sh) == TC_OK);
    for (int id = -1; id <= tc_kernel_count(); ++id) {
        const double b = tc_kernel_bytes(c, inst, id);
        CHECK(b >= 0.0 && std::isfinite(b));
        CHECK(tc_kernel_name(id) != nullptr);
    }
    // out-of-range instance and null pointers
    CHECK(tc_mode_shape(c, inst + 1000, &nr, &nj, &nl) == TC_EINVAL);
    CHECK(tc_grid(c, inst, nullptr) == TC_EINVAL);
    CHECK(tc_grid(c, -1, r.data()) == TC_EINVAL);
    CHECK(std::strlen(tc_last_error(c)) > 0);
}

int main() {
    CHECK(tc_abi_version() == TC_ABI_VERSION);
    CHECK(tc_kernel_count() > 0);
    CHECK(tc_destroy(nullptr) == TC_OK);

    // invalid geometries: error code, message, *out untouched
    {
        tc_ctx* c = reinterpret_cast<tc_ctx*>(0x1);
        const tc_geometry good = base(33, 32, 32, 0.0);
        tc_geometry bad[] = {good, good, good, good, good, good, good, good, good};
        bad[0].radius_ratio = 1.0;
        bad[1].nr = 6;
        bad[2].ntheta = 40;
        bad[3].nz = 25;
        bad[4].re = -1.0;
        bad[5].dt = 0.0;
        bad[6].stretch = -1.0;
        bad[7].precision = 7;
        bad[8].gap = std::nan("");
        for (const auto& g : bad) {
            CHECK(tc_create(&g, 1, &c) == TC_EINVAL);
            CHECK(c == reinterpret_cast<tc_ctx*>(0x1));
            CHECK(std::strlen(tc_last_error(nullptr)) > 0);
        }
        CHECK(tc_create(nullptr, 1, &c) == TC_EINVAL);
        CHECK(tc_create(&good, 1, nullptr) == TC_EINVAL);
        CHECK(tc_create(&good, 0, &c) == TC_EINVAL);
        tc_geometry mixed[2] = {good, good};
        mixed[1].precision = TC_PREC_MIXED;
        CHECK(tc_create(mixed, 2, &c) == TC_EINVAL);
        std::printf("validation checks done\n");
    }

    // host-only contexts of several shapes, single and batched
    const tc_geometry shapes[] = {base(7, 4, 4, 0.0),      base(33, 32, 32, 0.0), base(129, 768, 384, 1.5),
                                  base(140, 12, 24, 1.2),  base(300, 48, 96, 2.0), base(65, 96, 64, 0.0)};
    for (const auto& g : shapes) {
        tc_ctx* c = nullptr;
        CHECK(tc_create(&g, 1, &c) == TC_OK && c != nullptr);
        if (!c) continue;
        check_context(c, 0, g);
        // device calls refuse a host-only context
        std::vector<double> buf((size_t)2 * g.nr * ((g.ntheta - 1) / 3 + 1) * (2 * ((g.nz - 1) / 3) + 1), 0.0);
        std::vector<double> prof((size_t)6 * g.nr, 0.0);
        tc_stats_t st;
        CHECK(tc_step(c, 1) == TC_EINVAL);
        CHECK(tc_substep(c, 1) == TC_EINVAL);
        CHECK(tc_stats(c, 0, &st) == TC_EINVAL);
        CHECK(tc_stats_noalloc(c, 0, &st) == TC_EINVAL);
        CHECK(tc_get_fields(c, 0, buf.data(), buf.data(), prof.data(), prof.data()) == TC_EINVAL);
        CHECK(tc_profiles(c, 0, prof.data()) == TC_EINVAL);
        CHECK(tc_use_graphs(c, 0) == TC_EINVAL);
        CHECK(tc_set_rhs_elimination(c, 0) == TC_EINVAL);
        CHECK(tc_timing(c, 1) == TC_EINVAL);
        CHECK(tc_autotune(c, 1) == TC_EINVAL);
        CHECK(tc_set_stream(c, nullptr) == TC_EINVAL);
        CHECK(tc_set_solve_shape(c, 0, 804) == TC_EINVAL);
        CHECK(tc_set_tiles(c, 0, 0, 0, 0) == TC_EINVAL);
        int zi = -1, th = -1, zf = -1;
        CHECK(tc_tiles(c, 0, &zi, &th, &zf) == TC_OK && zi == 0 && th == 0 && zf == 0);
        CHECK(tc_destroy(c) == TC_OK);
        std::printf("dry-run context nr=%d ntheta=%d nz=%d ok\n", g.nr, g.ntheta, g.nz);
    }
    {
        const int n = (int)(sizeof(shapes) / sizeof(shapes[0]));
        tc_ctx* c = nullptr;
        CHECK(tc_create(shapes, n, &c) == TC_OK && c != nullptr);
        if (c) {
            for (int i = 0; i < n; ++i) check_context(c, i, shapes[i]);
            CHECK(tc_destroy(c) == TC_OK);
        }
        std::printf("batched dry-run context of %d instances ok\n", n);
    }
    std::printf(failures ? "FAILED %d\n" : "ALL OK\n", failures);
    return failures ? 1 : 0;
}
