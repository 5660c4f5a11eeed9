// Exercises the host-side logic of the C ABI (tests/test_abi_sanitized.py
// links it with the library's host code built under AddressSanitizer and
// UndefinedBehaviorSanitizer): handle creation for every system and lattice,
// parameters, storage, references, buffer sizes, the checks of unbound or
// invalid calls and every error path that needs no device.  Prints "ok" and
// exits 0 on completion.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lbm.h"

static int fails = 0;
#define EXPECT(c)                                                  \
    do {                                                           \
        if (!(c)) {                                                \
            std::fprintf(stderr, "line %d: %s\n", __LINE__, #c);   \
            ++fails;                                               \
        }                                                          \
    } while (0)

int main()
{
    struct Case {
        const char *sys, *lat;
        int nz;
    };
    const Case cases[] = {
        {"advdiff_trk2d", "D2Q5", 1}, {"advdiff_trk2d", "D2Q9", 1}, {"swe2d", "D2Q9", 1}, {"swe2d", "D2Q5", 1},
        {"neohooke2d", "D2Q9", 1},    {"neohooke2d", "D2Q5", 1},    {"nsf3d_trk17", "D3Q7", 5},
        {"burgers2d", "D2Q5", 1},     {"euler2d", "D2Q5", 1},       {"euler2d", "D2Q9", 1},
        {"maxwell2d", "D2Q5", 1},     {"allencahn_trk2d", "D2Q5", 1}, {"relhydro2d", "D2Q5", 1},
        {"nse_trk2d", "D2Q5", 1},     {"cnsf_trk2d", "D2Q5", 1},    {"mhd_trk2d", "D2Q5", 1},
        {"hcnsf3d_trk14", "D3Q7", 3}, {"gen_euler2d", "D2Q5", 1},   {"gen_advdiff_trk2d", "D2Q5", 1},
        {"gen_cnsf_trk2d", "D2Q5", 1},
    };
    int n = 0;
    for (const Case &c : cases) {
        lbm_state *h = lbm_create(c.sys, c.lat, 37, 11, c.nz, 0.6, 1e-3, 1e-2);
        EXPECT(h != nullptr);
        if (!h) continue;
        const int K = lbm_num_fields(h), Q = lbm_num_velocities(h);
        EXPECT(K > 0 && K <= 18 && Q >= 5 && Q <= 9);
        double v = 0.0;
        EXPECT(lbm_get_param(h, "dt", &v) == LBM_OK && v > 0.0);
        EXPECT(lbm_get_param(h, "no_such_parameter", &v) == LBM_EINVAL);
        EXPECT(lbm_set_param(h, "no_such_parameter", 1.0) == LBM_EINVAL);
        EXPECT(lbm_last_error(h) != nullptr && std::strlen(lbm_last_error(h)) > 0);
        lbm_set_param(h, "g_tau", 3.0);
        EXPECT(lbm_set_param(h, "check_every", -1.0) == LBM_EINVAL);
        EXPECT(lbm_set_param(h, "check_every", 4.0) == LBM_OK);
        for (int s = LBM_F64; s <= LBM_F16NE; ++s) {
            lbm_set_storage(h, s);
            EXPECT(lbm_required_bytes(h, 0) > 0);
            EXPECT(lbm_required_bytes(h, 1) > 0);
        }
        EXPECT(lbm_set_storage(h, 99) == LBM_EINVAL);
        lbm_set_storage(h, LBM_F32);
        std::vector<double> q0((size_t)K, 0.0);
        EXPECT(lbm_get_reference(h, q0.data()) == LBM_OK);
        for (double &x : q0) x += 0.25;
        lbm_set_reference(h, q0.data());
        EXPECT(lbm_step(h, 1) == LBM_ENOTBOUND);
        EXPECT(lbm_init_moments(h, nullptr) != LBM_OK);
        EXPECT(lbm_moments(h, nullptr, 1, 0) != LBM_OK);
        double out[64];
        EXPECT(lbm_reduce(h, 0, nullptr, out) != LBM_OK);
        EXPECT(lbm_reduce_static(h, 0, nullptr, out) != LBM_OK);
        EXPECT(lbm_set_field(h, "no_such_field", nullptr) == LBM_EINVAL);
        EXPECT(lbm_step_count(h) == 0 && lbm_time(h) == 0.0);
        size_t nbytes = 0;
        EXPECT(lbm_save(h, nullptr, &nbytes) != LBM_OK || nbytes > 0);
        EXPECT(lbm_load(h, "x", 1) != LBM_OK);
        EXPECT(lbm_adjoint_step(h, 1, nullptr, nullptr, nullptr, nullptr) != LBM_OK);
        lbm_destroy(h);
        ++n;
    }
    // invalid creation: unknown names, lattice of the wrong dimension, empty grids
    EXPECT(lbm_create("no_such_system", "D2Q9", 8, 8, 1, 0.6, 1e-3, 1e-2) == nullptr);
    EXPECT(lbm_last_error(nullptr) != nullptr);
    EXPECT(lbm_create("swe2d", "D3Q7", 8, 8, 1, 0.6, 1e-3, 1e-2) == nullptr);
    EXPECT(lbm_create("swe2d", "D2Q9", 0, 8, 1, 0.6, 1e-3, 1e-2) == nullptr);
    EXPECT(lbm_create("nsf3d_trk17", "D3Q7", 8, 8, 0, 0.6, 1e-3, 1e-2) == nullptr);
    EXPECT(lbm_create("swe2d", "D2Q9", 8, 8, 1, 0.4, 1e-3, 1e-2) == nullptr);   // tau below 1/2
    EXPECT(lbm_create("swe2d", "D2Q9", 8, 8, 1, std::nan(""), 1e-3, 1e-2) == nullptr);
    EXPECT(lbm_bw_copy(nullptr, nullptr, 16, nullptr) == LBM_EINVAL);
    EXPECT(lbm_bw_streams(nullptr, nullptr, 8, 8, 3, nullptr) == LBM_EINVAL);
    EXPECT(lbm_bw_streams3(nullptr, nullptr, 8, 8, 8, 17, nullptr) == LBM_EINVAL);
    lbm_destroy(nullptr);
    if (fails) return 1;
    std::printf("ok %d handles\n", n);
    return 0;
}
