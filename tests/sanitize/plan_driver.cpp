// Host-sanitizer driver for the library's host-only plan code (plan.cpp):
// plan creation over a grid of valid and invalid arguments, every option,
// the size helpers, the Eq. 2 limit and the DM-list checks, including
// non-finite and extreme values, so that AddressSanitizer and UBSan see any
// overflow or undefined operation.  Exit status 0 when every call returned
// what it documents.
#include <cmath>
#include <cstdio>
#include <initializer_list>
#include <limits>

#include "../../paper_1607_00909_amd/csrc/plan.hpp"

static int failures = 0;
#define EXPECT(cond)                                                             \
    do {                                                                         \
        if (!(cond)) {                                                           \
            std::fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                          \
        }                                                                        \
    } while (0)

int main() {
    const double inf = std::numeric_limits<double>::infinity();
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const int ints[] = {-2147483647 - 1, -1, 0, 1, 2, 3, 7, 8, 16, 64, 256, 1000, 1024, 2048,
                        4096, 15360, 65536, 131072, 262144, 1 << 30, 2147483647};
    const double freqs[] = {-1.0, 0.0, 1e-300, 0.195, 120.0, 1e300, inf, nan};
    long made = 0;
    for (int nfft : ints)
        for (int nov : ints)
            for (int nchan : ints)
                for (int ndec : {1, 2, 3, 8, 0, -1, 2147483647})
                    for (double fc : freqs) {
                        cdmt_plan_t p = nullptr;
                        const int st = cdmt_plan(&p, 3, fc, 0.1953125, nfft, nov, nchan, ndec);
                        EXPECT((st == CDMT_OK) == (p != nullptr));
                        if (p) {
                            ++made;
                            long long a, b;
                            int c;
                            EXPECT(cdmt_output_shape(p, 39, &a, &b, &c) == CDMT_OK);
                            size_t z;
                            EXPECT(cdmt_workspace_size(p, 39, &z) == CDMT_OK);
                            double lim = 0;
                            EXPECT(cdmt_dm_limit(p, &lim) == CDMT_OK && lim >= 0);
                            cdmt_destroy(p);
                        }
                    }
    EXPECT(made > 0);
    EXPECT(cdmt_plan(nullptr, 1, 120.0, 0.2, 4096, 0, 8, 1) == CDMT_E_ARG);
    EXPECT(cdmt_plan_set(nullptr, 0, 0) == CDMT_E_ARG);

    cdmt_plan_t p = nullptr;
    EXPECT(cdmt_plan(&p, 288, 138.0, 0.1953125, 65536, 15360, 16, 8) == CDMT_OK);
    for (int opt = -3; opt < 14; ++opt)
        for (int v : ints) {
            const int st = cdmt_plan_set(p, opt, v);
            int back = -12345;
            if (st == CDMT_OK) {
                EXPECT(cdmt_plan_get(p, opt, &back) == CDMT_OK);
                EXPECT(back == v);
            }
        }
    // restore the defaults the checks below assume
    EXPECT(cdmt_plan_set(p, CDMT_OPT_CHIRP_REF, 1) == CDMT_OK);
    EXPECT(cdmt_plan_set(p, CDMT_OPT_DM_CHECK, 1) == CDMT_OK);
    EXPECT(cdmt_plan_set(p, CDMT_OPT_FWD_N2, 256) == CDMT_OK);
    int iv = 0;
    EXPECT(cdmt_plan_get(p, CDMT_OPT_INPUT, nullptr) == CDMT_E_ARG);
    EXPECT(cdmt_plan_get(p, 99, &iv) == CDMT_E_ARG);

    double lim = 0;
    EXPECT(cdmt_dm_limit(p, &lim) == CDMT_OK);
    EXPECT(lim > 63.5 && lim < 65.0);
    const double good[] = {0.0, 63.5, -63.5, lim};
    EXPECT(cdmt::check_dms(p, good, 4) == CDMT_OK);
    const double past[] = {lim * (1 + 1e-9)};
    EXPECT(cdmt::check_dms(p, past, 1) == CDMT_E_SHAPE);
    for (double bad : {inf, -inf, nan, 1e300, -1e300})
        EXPECT(cdmt::check_dms(p, &bad, 1) == CDMT_E_ARG);
    EXPECT(cdmt_plan_set(p, CDMT_OPT_DM_CHECK, 0) == CDMT_OK);
    EXPECT(cdmt::check_dms(p, past, 1) == CDMT_OK);
    const double prog[] = {0.0, 0.5, 1.0, 1.5000001};
    EXPECT(cdmt::arithmetic(prog, 3, 1e-9));
    EXPECT(!cdmt::arithmetic(prog, 4, 1e-9));
    const double flat[] = {2.0, 2.0};
    EXPECT(!cdmt::arithmetic(flat, 2, 1e-9));

    size_t z = 0;
    EXPECT(cdmt::workspace_bytes(p, -1, &z) == CDMT_E_ARG);
    EXPECT(cdmt::workspace_bytes(p, 2147483647, &z) == CDMT_OK);
    EXPECT(cdmt::check_call(p, nullptr, 0, 0) == CDMT_OK);
    EXPECT(cdmt::check_call(p, nullptr, 0, 1) == CDMT_E_ARG);
    EXPECT(cdmt::check_call(p, &z, 8, 1) == CDMT_E_WORKSPACE);
    EXPECT(cdmt::check_call(p, &z, ~(size_t)0, 2147483647) == CDMT_E_SHAPE);
    EXPECT(cdmt_gradient_workspace_size(p, 39, 64, &z) == CDMT_OK);
    EXPECT(cdmt_voltage_gradient_workspace_size(p, 39, &z) == CDMT_OK);
    cdmt_destroy(p);

    int nov = 0;
    EXPECT(cdmt_noverlap_for(109.875, 0.1953125, 63.5, 16, 8, 1, &nov) == CDMT_OK && nov == 15360);
    EXPECT(cdmt_noverlap_for(1e-300, 1e300, 1e300, 16, 8, 1, &nov) == CDMT_E_SHAPE);
    EXPECT(cdmt_noverlap_for(nan, 0.2, 1.0, 16, 8, 0, &nov) == CDMT_E_ARG);
    EXPECT(cdmt_noverlap_for(110.0, 0.2, 1.0, 16, 8, 0, nullptr) == CDMT_E_ARG);
    for (int s = -6; s <= 1; ++s)
        EXPECT(cdmt_status_string(s) != nullptr);
    cdmt_destroy(nullptr);
    if (failures)
        std::fprintf(stderr, "%d failures\n", failures);
    else
        std::printf("plan sanitizer run: ok (%ld plans made)\n", made);
    return failures ? 1 : 0;
}
