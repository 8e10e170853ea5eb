// Exercises the host side of libcos (state tables, plan counts, Pade,
// argument validation, failure injection, the no-device path) in a build
// whose host code carries the address and undefined-behaviour sanitizers
// (test infrastructure; runs without a GPU).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "libcos.h"

#define CHECK(x)                                                             \
    do {                                                                     \
        if (!(x)) {                                                          \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); \
            return 1;                                                        \
        }                                                                    \
    } while (0)

int main() {
    int64_t st = 0, ex = 0, cl = 0, sh = 0, ma = 0, ro = 0;
    for (int n = 1; n <= COS_NMAX; ++n) {
        CHECK(cos_plan_counts(n, &st, &ex, &cl, &sh, &ma, &ro) == COS_OK);
        CHECK(cos_plan_counts_mask_only(n, 0, &st, &ex, &cl) == COS_OK);
        std::printf("n=%d states=%lld ext=%lld rows=%lld\n", n, (long long)st, (long long)ex, (long long)ro);
    }
    for (int n = 1; n <= COS_NMAX_SUBLATTICE; ++n) {
        CHECK(cos_plan_counts_sublattice(n, &st, &ex, &cl, &ma, &ro) == COS_OK);
        CHECK(cos_plan_counts_mask_only(n, COS_F_SUBLATTICE, &st, &ex, &cl) == COS_OK);
    }
    CHECK(cos_plan_counts(0, &st, 0, 0, 0, 0, 0) == COS_ERANGE);
    CHECK(cos_plan_counts(13, &st, 0, 0, 0, 0, 0) == COS_ERANGE);
    std::vector<double> a{1.0, 1.0, 0.5, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720};
    std::vector<double> g(a.size());
    double v = 0;
    for (int m = 0; m <= 3; ++m)
        for (int k = 0; k <= 3; ++k) CHECK(cos_pade(m, k, a.data(), 0.5, &v, g.data()) == COS_OK);
    CHECK(cos_pade(0, 1, a.data(), 1.0, &v, g.data()) == COS_ERANGE);   // 1 / (1 - x) at x = 1
    CHECK(cos_pade(-1, 0, a.data(), 1.0, &v, nullptr) == COS_ERANGE);
    // argument validation of the device entry points (before any device work)
    cos_batch_t b = nullptr;
    int32_t n[3] = {4, 5, 13};
    CHECK(cos_batch_create(3, n, 2, COS_UNIFORM, 0, &b) == COS_ERANGE);
    CHECK(cos_batch_create(2, n, 2, 7, 0, &b) == COS_EINVAL);
    CHECK(cos_batch_create(2, n, 0, COS_UNIFORM, 0, &b) == COS_ERANGE);
    CHECK(cos_connected_sum_batched(nullptr, nullptr, nullptr, nullptr, -1.0, nullptr, nullptr) == COS_EINVAL);
    CHECK(cos_connected_sum_static(4, 9, 2, COS_UNIFORM, 0, a.data(), nullptr, -1.0, g.data(), nullptr) == COS_ERANGE);
    CHECK(cos_inject_failures(2, 0, 1) == COS_EINVAL);
    CHECK(cos_set_workspace_limit(-1) == COS_EINVAL);
    CHECK(cos_set_workspace_limit(0) == COS_OK);
    // without a usable device every device call says so
    double G[16] = {0}, out = 0;
    const cos_status s = cos_connected_sum(4, 2, COS_UNIFORM, 0, G, nullptr, -1.0, &out);
    CHECK(s == COS_EUNSUPPORTED || s == COS_EDEVICE);
    CHECK(cos_last_error()[0] != 0);
    CHECK(cos_release() == COS_OK);
    std::printf("host checks passed\n");
    return 0;
}
