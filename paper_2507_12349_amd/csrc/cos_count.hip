// Integer counting mode (cos_connected_count in include/libcos.h): the
// forward rules of the level kernels with every propagator equal to 1 and an
// integer weight x per closed cycle, in unsigned 64-bit arithmetic (exact
// modulo 2^64).  With G = 1 the product f . G is the same sum for every
// output, and every configuration is alike, so a thread takes one mask of a
// level (its rows in turn) instead of a lane per configuration.  Each child
// slot has exactly one parent mask, so threads never write the same word.
#include <cstring>
#include <vector>

#include "cos_internal.hpp"

namespace libcos {
namespace {

__global__ void count_level_kernel(const int32_t *__restrict__ mrec, const int4 *__restrict__ levels, int n,
                                   int level, const uint64_t *__restrict__ cur, uint64_t *__restrict__ nxt,
                                   uint64_t x, uint64_t *__restrict__ out) {
    const int4 L = levels[level];
    const int mi = blockIdx.x * blockDim.x + threadIdx.x;
    if (mi >= L.w) return;
    const int32_t *r = mrec + (int64_t)(L.z + mi) * kRecInts;
    const uint32_t info = (uint32_t)r[1], ones = info & 0xffffu, twos = info >> 16;
    const int rb = r[2];
    const bool start = level == 1, last = level == 2 * n;
    uint32_t hs = (twos & 1u) ? (twos & ~1u) : 0u;   // heads >= 1, ascending
    int u = 0, slot = 0;
    uint64_t cp = 0, dext = 0;
    while (true) {
        const uint32_t cm = current_set(u, ones, twos);
        uint64_t acc = 0;
        if (start) {
            acc = 1;   // the start state (e_0, 0, 0)
        } else {
            for (int v = 0; v < n; ++v)
                if ((cm >> v) & 1u) acc += cur[(int64_t)(rb + slot) * n + v];
        }
        cp += acc;   // this row's close
        for (int w = 0; w < n; ++w) {
            const uint32_t bit = 1u << w;
            if (twos & bit) continue;
            const bool first = !(ones & bit);
            const uint64_t val = first ? 2 * acc : acc;
            if (w == 0 && u == 0 && !(twos & 1u)) {
                dext = val;   // m_0 = 1: the next cycle opens on this same slot
                continue;
            }
            const uint32_t ctw = first ? twos : (twos | bit);
            nxt[(int64_t)(r[3 + w] + head_slot(u, ctw)) * n + w] = val;
        }
        if (!hs) break;
        u = __builtin_ctz(hs);
        hs &= hs - 1u;
        ++slot;
    }
    const uint64_t t = x * cp;
    if (last) {
        *out = t;
    } else if (ones) {
        const int h = __builtin_ctz(ones);
        nxt[(int64_t)(r[3 + h] + head_slot(h, twos | (1u << h))) * n + h] = t + (h == 0 ? dext : 0);
    }
}

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace libcos

using namespace libcos;

extern "C" cos_status cos_connected_count(int32_t n, int64_t cycle_weight, int64_t *count) {
    if (!count) return report(COS_EINVAL, "count is NULL");
    if (n < 1 || n > COS_NMAX) return report(COS_ERANGE, "n must be in [1, %d], got %d", COS_NMAX, n);
    int dev = 0, ncu = 0;
    if (cos_status st = current_device(&dev, &ncu)) return st;
    PlanTables t;
    if (cos_status st = plan_tables(n, &t)) return st;
    // one allocation: the state tables, two level windows and the result
    const size_t mb = up256(t.mrec_ints * 4), lb = up256(t.nlevels * sizeof(int4));
    const size_t win = (size_t)t.max_rows * n;
    char *d = nullptr;
    if (hipMalloc((void **)&d, mb + lb + sizeof(uint64_t) * (2 * win + 1)) != hipSuccess) {
        (void)hipGetLastError();
        return report(COS_ENOMEM, "device allocation for counting at n = %d failed", n);
    }
    const int32_t *mrec = (const int32_t *)d;
    const int4 *levels = (const int4 *)(d + mb);
    uint64_t *w0 = (uint64_t *)(d + mb + lb), *w1 = w0 + win, *res = w1 + win;
    hipError_t e = hipMemcpy(d, t.mrec, t.mrec_ints * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d + mb, t.levels, t.nlevels * sizeof(int4), hipMemcpyHostToDevice);
    std::vector<int4> lv(t.levels, t.levels + t.nlevels);
    for (int l = 1; l <= 2 * n && e == hipSuccess; ++l) {
        const int nm = lv[l].w;
        if (nm <= 0) continue;
        hipLaunchKernelGGL(count_level_kernel, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, 0, mrec, levels, n,
                           l, (l & 1) ? w1 : w0, (l & 1) ? w0 : w1, (uint64_t)cycle_weight, res);
        e = hipGetLastError();
    }
    uint64_t c = 0;
    if (e == hipSuccess) e = hipMemcpy(&c, res, sizeof(uint64_t), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return report(COS_EDEVICE, "counting failed: %s", hipGetErrorString(e));
    *count = (int64_t)c;
    return COS_OK;
}
