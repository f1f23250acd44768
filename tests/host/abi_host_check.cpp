// Host-only checks of libfem, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side (device code unchanged) and run
// on a machine without a GPU: the argument checks of the C ABI, the parsing of
// the batch tuner's cache file, the quadrature-rule builder and the function
// catalogue's parameter checks. Exit status 0 when every check holds; a
// sanitizer report aborts the run.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>

#include "../../paper_1409_4618_amd/csrc/fem_internal.h"
#include "../../paper_1409_4618_amd/csrc/tune_cache.h"
#include "fem.h"

static int g_fail = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++g_fail;                                                      \
        }                                                                  \
    } while (0)

static void write_file(const std::string& path, const std::string& text) {
    std::ofstream f(path, std::ios::trunc | std::ios::binary);
    f << text;
}

static void check_cache(const std::string& dir) {
    const std::string p = dir + "/cache.jsonl";
    int R = -7, S = -7, N = -7;
    CHECK(!fem::cache_lookup(nullptr, "dev", "sig", &R, &S, &N));
    CHECK(!fem::cache_lookup((dir + "/missing.jsonl").c_str(), "dev", "sig", &R, &S, &N));
    std::string junk;
    junk += "\n";                                              // empty line
    junk += "{\"device\": \"dev\", \"signature\": \"sig\", \"rows_per_tile\": ";  // truncated
    junk += "\n{\"device\": \"dev\", \"signature\": \"sig\", \"rows_per_tile\": 64, \"schedule\": 1, \"ms\": 1.0}\n";
    junk += "{\"device\": \"dev\", \"signature\": \"sig\", \"rows_per_tile\": 99999999999999999999, \"schedule\": 0}\n";
    junk += "{\"device\": \"dev\", \"signature\": \"sig\", \"rows_per_tile\": -128, \"schedule\": 0}\n";
    junk += "{\"device\": \"dev\", \"signature\": \"sig\", \"rows_per_tile\": 128, \"schedule\": 7}\n";
    junk += "{\"device\": \"dev\", \"signature\": \"sig\", \"rows_per_tile\": x, \"schedule\": 0}\n";
    junk += "{\"device\": \"other\", \"signature\": \"sig\", \"rows_per_tile\": 256, \"schedule\": 2}\n";
    junk += "{\"device\": \"dev\", \"signature\": \"sig2\", \"rows_per_tile\": 256, \"schedule\": 2}\n";
    junk += "{\"device\": \"dev\", \"signature\": \"sig3\", \"rows_per_tile\": 0, \"schedule\": 1, \"threads\": 128}\n";
    junk += "{\"device\": \"dev\", \"signature\": \"sig3\", \"rows_per_tile\": 64, \"schedule\": 1, \"threads\": 128}\n";
    junk += "{\"device\": \"dev\", \"signature\": \"sig3\", \"rows_per_tile\": 0, \"schedule\": 0, \"threads\": 512}\n";
    junk += "{\"device\": \"dev\", \"signature\": \"sig3\", \"rows_per_tile\": 0, \"schedule\": 0, \"threads\": }\n";
    // per-kind launches (schedules 3-4) are valid with element-major tiles only
    junk += "{\"device\": \"dev\", \"signature\": \"sig4\", \"rows_per_tile\": 0, \"schedule\": 4, \"threads\": 256}\n";
    junk += "{\"device\": \"dev\", \"signature\": \"sig4\", \"rows_per_tile\": 64, \"schedule\": 3, \"threads\": 256}\n";
    junk += "{\"device\": \"dev\", \"signature\": \"sig4\", \"rows_per_tile\": 0, \"schedule\": 5, \"threads\": 256}\n";
    junk += std::string(200000, 'z') + "\n";                  // a long line
    junk += std::string("\0\x01\xff", 3) + "\n";              // binary bytes
    junk += "{\"device\": \"dev\", \"signature\": \"sig\", \"rows_per_tile\": 0, \"schedule\": 2, \"ms\": 0.5}";  // no newline
    write_file(p, junk);
    CHECK(fem::cache_lookup(p.c_str(), "dev", "sig", &R, &S, &N));
    CHECK(R == 0 && S == 2 && N == 256);  // the last valid matching line wins; no threads field: 256
    CHECK(fem::cache_lookup(p.c_str(), "dev", "sig2", &R, &S, &N) && R == 256 && S == 2);
    CHECK(fem::cache_lookup(p.c_str(), "dev", "sig3", &R, &S, &N) && R == 0 && S == 1 && N == 128);
    CHECK(fem::cache_lookup(p.c_str(), "dev", "sig4", &R, &S, &N) && R == 0 && S == 4 && N == 256);
    CHECK(!fem::cache_lookup(p.c_str(), "dev", "nosuch", &R, &S, &N));
    // store, then read back
    const std::string q = dir + "/store.jsonl";
    write_file(q, "");
    const std::string longsig(5000, 'a');
    fem::cache_store(q.c_str(), "gfx950-cu256", longsig, 128, 1, 256, 0.123456);
    fem::cache_store(q.c_str(), "gfx950-cu256", "s", 64, 0, 256, 1e300);
    fem::cache_store(q.c_str(), "gfx950-cu256", "t", 0, 2, 128, 0.5);
    fem::cache_store(nullptr, "d", "s", 64, 0, 256, 1.0);
    R = S = -1;
    CHECK(fem::cache_lookup(q.c_str(), "gfx950-cu256", longsig, &R, &S, &N) && R == 128 && S == 1);
    CHECK(fem::cache_lookup(q.c_str(), "gfx950-cu256", "s", &R, &S, &N) && R == 64 && S == 0 && N == 256);
    CHECK(fem::cache_lookup(q.c_str(), "gfx950-cu256", "t", &R, &S, &N) && R == 0 && S == 2 && N == 128);
    int v = 0;
    CHECK(!fem::cache_field("\"k\": ", "\"k\": ", &v));
    CHECK(fem::cache_field("\"k\": 12x", "\"k\": ", &v) && v == 12);
    CHECK(fem::cache_field("\"k\": -3", "\"k\": ", &v) && v == -3);
}

static void check_quadrature() {
    fem::QuadRule q;
    CHECK(fem::gauss_legendre01(0, &q) == FEM_EINVAL);
    CHECK(fem::gauss_legendre01(fem::FEM_QUAD_MAX + 1, &q) == FEM_EINVAL);
    CHECK(fem::gauss_legendre01(-5, &q) == FEM_EINVAL);
    for (int m = 1; m <= fem::FEM_QUAD_MAX; ++m) {
        CHECK(fem::gauss_legendre01(m, &q) == FEM_OK);
        double sw = 0.0, sx3 = 0.0;
        for (int i = 0; i < m; ++i) {
            CHECK(q.x[i] > 0.0 && q.x[i] < 1.0 && q.w[i] > 0.0);
            sw += q.w[i];
            sx3 += q.w[i] * q.x[i] * q.x[i] * q.x[i];
        }
        CHECK(std::fabs(sw - 1.0) < 1e-14);
        if (m >= 2) CHECK(std::fabs(sx3 - 0.25) < 1e-14);  // exact for degree 2m - 1 >= 3
    }
}

static void check_functions() {
    fem::FnArgs F;
    double p[fem::FEM_POLY_MAX_TERMS * 5 + 5];
    for (int t = 0; t < fem::FEM_POLY_MAX_TERMS + 1; ++t) {
        p[t * 5 + 0] = 1.0;
        p[t * 5 + 1] = (double)(t % 3);
        p[t * 5 + 2] = 1.0;
        p[t * 5 + 3] = 2.0;
        p[t * 5 + 4] = 0.0;
    }
    CHECK(fem::make_fn_args(FEM_FN_POLYNOMIAL, 3, p, fem::FEM_POLY_MAX_TERMS * 5, &F) == FEM_OK);
    CHECK(F.n_terms == fem::FEM_POLY_MAX_TERMS && F.n_comp == 3);
    CHECK(fem::make_fn_args(FEM_FN_POLYNOMIAL, 3, p, (fem::FEM_POLY_MAX_TERMS + 1) * 5, &F) == FEM_EINVAL);
    CHECK(fem::make_fn_args(FEM_FN_POLYNOMIAL, 3, nullptr, 5, &F) == FEM_EINVAL);
    CHECK(fem::make_fn_args(FEM_FN_POLYNOMIAL, 3, p, 7, &F) == FEM_EINVAL);
    CHECK(fem::make_fn_args(FEM_FN_POLYNOMIAL, 3, p, 0, &F) == FEM_EINVAL);
    const double p2[12] = {1.0, 0.0, 1.0, 2.0, -2.0, 1.0, 0.0, 3.0, 0.5, 2.0, 1.0, 1.0};
    CHECK(fem::make_fn_args(FEM_FN_POLYNOMIAL, 2, p2, 8, &F) == FEM_OK && F.n_comp == 2);  // components 0, 1
    CHECK(fem::make_fn_args(FEM_FN_POLYNOMIAL, 2, p2, 12, &F) == FEM_EINVAL);  // component 2 in 2D
    double bad[5] = {1.0, 0.0, 31.0, 0.0, 0.0};
    CHECK(fem::make_fn_args(FEM_FN_POLYNOMIAL, 3, bad, 5, &F) == FEM_EINVAL);
    bad[2] = NAN;
    CHECK(fem::make_fn_args(FEM_FN_POLYNOMIAL, 3, bad, 5, &F) == FEM_EINVAL);
    bad[2] = 1.5;
    CHECK(fem::make_fn_args(FEM_FN_POLYNOMIAL, 3, bad, 5, &F) == FEM_EINVAL);
    CHECK(fem::make_fn_args((fem_function)99, 3, nullptr, 0, &F) == FEM_EINVAL);
    CHECK(fem::make_fn_args((fem_function)-1, 3, nullptr, 0, &F) == FEM_EINVAL);
    CHECK(fem::make_fn_args(FEM_FN_BUBBLE_U, 3, nullptr, 0, &F) == FEM_OK);
    CHECK(fem::make_fn_args(FEM_FN_EDDY_E, 3, nullptr, 0, &F) != FEM_OK);  // the eddy example is 2D
}

static void check_abi() {
    fem_mesh out = reinterpret_cast<fem_mesh>(0x1);
    CHECK(fem_topology(nullptr, 10, 3, nullptr, 10, nullptr, nullptr) == FEM_EINVAL);
    CHECK(fem_topology(nullptr, 10, 5, nullptr, 10, nullptr, &out) == FEM_EINVAL);
    CHECK(out == nullptr);
    CHECK(std::string(fem_last_error()).find("dim") != std::string::npos);
    const double* fake = reinterpret_cast<const double*>(16);
    const int32_t* fakei = reinterpret_cast<const int32_t*>(16);
    CHECK(fem_topology(fake, int64_t(1) << 31, 3, fakei, 10, nullptr, &out) == FEM_EOVERFLOW);
    CHECK(fem_topology(fake, 10, 3, fakei, int64_t(1) << 29, nullptr, &out) == FEM_EOVERFLOW);
    int64_t a = 0;
    CHECK(fem_mesh_counts(nullptr, &a, &a, &a, &a, nullptr) == FEM_EINVAL);
    CHECK(fem_pattern(nullptr, FEM_NEDELEC, nullptr, nullptr, nullptr, nullptr, nullptr) == FEM_EINVAL);
    CHECK(fem_assemble(nullptr, (fem_kind)7, fake, nullptr, nullptr, nullptr, nullptr, nullptr) == FEM_EINVAL);
    CHECK(fem_assemble(nullptr, FEM_NEDELEC, fake, nullptr, nullptr, nullptr, nullptr, nullptr) == FEM_EINVAL);
    CHECK(fem_assemble_backward(nullptr, FEM_NEDELEC, fake, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                nullptr, nullptr) == FEM_EINVAL);
    CHECK(fem_quadratic_value(nullptr, FEM_NEDELEC, fake, nullptr, nullptr, fake, nullptr, nullptr) == FEM_EINVAL);
    CHECK(fem_quadratic_value_noalloc(nullptr, FEM_NEDELEC, fake, nullptr, nullptr, fake, nullptr, nullptr) ==
          FEM_EINVAL);
    CHECK(fem_norm_L2(nullptr, fake, FEM_FN_BUBBLE_U, nullptr, 0, 4, nullptr, nullptr, nullptr) == FEM_EINVAL);
    CHECK(fem_load_vector(nullptr, FEM_NEDELEC, fake, FEM_FN_EDDY_F, nullptr, 0, 4, nullptr, nullptr) == FEM_EINVAL);
    CHECK(fem_p1_assemble(nullptr, fake, nullptr, nullptr, nullptr) == FEM_EINVAL);
    CHECK(fem_majorant_terms(nullptr, fake, fake, fake, FEM_FN_BUBBLE_F, nullptr, 0, 4, nullptr, nullptr) ==
          FEM_EINVAL);
    int64_t it = 0;
    double rr = 0.0;
    const int64_t* rp = reinterpret_cast<const int64_t*>(16);
    double* x = reinterpret_cast<double*>(32);
    CHECK(fem_cg_solve(0, rp, fakei, fake, nullptr, 1, 0, fake, x, 1e-12, 10, nullptr, &it, &rr) == FEM_EINVAL);
    CHECK(fem_cg_solve(5, nullptr, fakei, fake, nullptr, 1, 0, fake, x, 1e-12, 10, nullptr, &it, &rr) == FEM_EINVAL);
    CHECK(fem_cg_solve(5, rp, fakei, fake, nullptr, 1, 0, fake, x, -1.0, 10, nullptr, &it, &rr) == FEM_EINVAL);
    CHECK(fem_cg_solve(5, rp, fakei, fake, nullptr, 1, 0, fake, x, NAN, 10, nullptr, &it, &rr) == FEM_EINVAL);
    CHECK(fem_cg_solve(5, rp, fakei, fake, nullptr, 1, 0, x, x, 1e-12, 10, nullptr, &it, &rr) == FEM_EINVAL);
    CHECK(fem_csr_matvec(-1, rp, fakei, fake, nullptr, 1, 0, fake, x, nullptr) == FEM_EINVAL);
    fem_batch b = reinterpret_cast<fem_batch>(0x1);
    CHECK(fem_batch_create(nullptr, nullptr, 3, &b) == FEM_EINVAL && b == nullptr);
    CHECK(fem_batch_create(nullptr, nullptr, 0, nullptr) == FEM_EINVAL);
    CHECK(fem_batch_tune(nullptr, nullptr, nullptr) == FEM_EINVAL);
    CHECK(fem_batch_set_config(nullptr, 64, 0, 256) == FEM_EINVAL);
    CHECK(fem_status_query(nullptr) == FEM_EINVAL);
    fem_mesh_destroy(nullptr);
    fem_batch_destroy(nullptr);
    CHECK(fem_version() != nullptr && fem_version()[0] != '\0');
}

int main(int argc, char** argv) {
    const std::string dir = argc > 1 ? argv[1] : ".";
    check_cache(dir);
    check_quadrature();
    check_functions();
    check_abi();
    if (g_fail) {
        std::fprintf(stderr, "%d check(s) failed\n", g_fail);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
