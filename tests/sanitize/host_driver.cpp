// Runs the library's host-only code under AddressSanitizer and UBSan: the
// self-tests of the index arithmetic and of the tile builder, and argument
// checks that return before any device call.  Built and run by
// tests/test_sanitizers.py; exits 0 when every check holds.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "lbm.h"

int main()
{
    const int rc = lbm_selftest_host();
    std::printf("lbm_selftest_host: %d %s\n", rc, lbm_last_error());
    if (rc != LBM_OK)
        return 1;
    std::vector<uint8_t> fl(3 * 4 * 5, LBM_FLUID);
    fl[1 * 5 + 2] = LBM_OUTLET; // an outlet cell off the last x plane
    lbm_domain *d = nullptr;
    if (lbm_create_domain(fl.data(), 5, 4, 3, 0, LBM_FP32, nullptr, &d) != LBM_ERR_ARG || d)
        return 2;
    if (lbm_create_domain(nullptr, 5, 4, 3, 0, LBM_FP32, nullptr, &d) != LBM_ERR_ARG)
        return 3;
    fl[1 * 5 + 2] = 7; // an unknown flag
    if (lbm_create_domain(fl.data(), 5, 4, 3, 0, LBM_FP32, nullptr, &d) != LBM_ERR_ARG)
        return 4;
    if (lbm_set_params(nullptr, 0.6, 1.0, 1.0) != LBM_ERR_ARG || lbm_step(nullptr, 1) != LBM_ERR_ARG)
        return 5;
    if (lbm_array_bytes(0, 4, 3, LBM_FP32) != 0 || lbm_array_bytes(5, 4, 3, 9) != 0)
        return 6;
    if (lbm_array_bytes(64, 1, 1, LBM_FP16S) != 3584 || lbm_debug_fail_after(-1) != LBM_ERR_ARG)
        return 7;
    std::printf("argument checks: ok\n");
    return 0;
}
