// libcos host side: argument validation, state tables (plans), batch handles,
// workspace and kernel launches behind the C ABI of include/libcos.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <complex>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "cos_internal.hpp"

using namespace libcos;

namespace {

thread_local std::string g_err;

cos_status fail(cos_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
cos_status fail(cos_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(COS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));           \
    } while (0)

// failures injected by cos_inject_failures: after `skip` successes, `count`
// device allocations (kind 0) or kernel launches (kind 1) fail
std::atomic<int> g_inj_skip[2], g_inj_count[2];

bool injected(int kind) {
    if (g_inj_count[kind].load() <= 0) return false;
    if (g_inj_skip[kind].load() > 0) {
        --g_inj_skip[kind];
        return false;
    }
    --g_inj_count[kind];
    return true;
}

// every device allocation of the library goes through here
hipError_t dev_malloc(void **p, size_t bytes) {
    if (injected(0)) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

// a kernel launch of the library; an injected failure skips the launch
#define LAUNCH_TRY(expr)                                                                       \
    do {                                                                                       \
        if (injected(1)) return fail(COS_EDEVICE, "%s failed: injected launch failure", #expr); \
        HIP_TRY(expr);                                                                         \
    } while (0)

// ---------------------------------------------------------------------------
// Host plan: the state tables for one order n (identical for every
// configuration and flavour).  Rows are ordered by level, then mask code,
// then head slot; masks by level then code.
// ---------------------------------------------------------------------------
struct HostPlan {
    int n = 0;
    std::vector<int32_t> rowbase;   // [3^n]
    std::vector<uint32_t> minfo;    // [3^n]
    std::vector<int2> rows;
    std::vector<int32_t> masks;
    std::vector<int4> levels;       // [2n + 2]
    std::vector<int32_t> mrec;      // [masks][rec_ints]
    bool sub = false;               // sublattice-labelled state space
    int rec_ints = kRecInts;
    int32_t max_rows = 0, max_masks = 0;
    int64_t states = 0, ext = 0, closes = 0, shift_edges = 0;
};

void build_host_plan(int n, HostPlan &P) {
    const int N3 = pow3(n);
    P.n = n;
    P.rowbase.assign(N3, -1);
    P.minfo.assign(N3, 0);
    std::vector<std::vector<int32_t>> bylevel(2 * n + 2);
    for (int code = 0; code < N3; ++code) {
        uint32_t ones = 0, twos = 0;
        int c = code, lvl = 0;
        for (int k = 0; k < n; ++k) {
            int d = c % 3;
            c /= 3;
            if (d == 1) ones |= 1u << k;
            if (d == 2) twos |= 1u << k;
            lvl += d;
        }
        P.minfo[code] = ones | (twos << 16);
        if (!((ones | twos) & 1u)) continue;   // vertex 0 is always visited
        bylevel[lvl].push_back(code);
    }
    P.levels.assign(2 * n + 2, make_int4(0, 0, 0, 0));
    for (int l = 1; l <= 2 * n; ++l) {
        int4 L;
        L.x = (int)P.rows.size();
        L.z = (int)P.masks.size();
        int r = 0, mi = 0;
        for (int code : bylevel[l]) {
            const uint32_t ones = P.minfo[code] & 0xffffu, twos = P.minfo[code] >> 16;
            P.rowbase[code] = r;
            P.masks.push_back(code);
            int nopen = 0, nzero = 0;
            for (int k = 0; k < n; ++k) {
                if (!((twos >> k) & 1u)) ++nopen;
                if (!(((ones | twos) >> k) & 1u)) ++nzero;
            }
            // heads in slot order: 0, then h >= 1 with m_h = 2 (only when m_0 = 2)
            std::vector<int> heads{0};
            if (twos & 1u)
                for (int h = 1; h < n; ++h)
                    if ((twos >> h) & 1u) heads.push_back(h);
            for (int u : heads) {
                P.rows.push_back(make_int2((code << 4) | u, mi));
                const int cnt = __builtin_popcount(current_set(u, ones, twos));
                P.states += cnt;
                P.ext += (int64_t)cnt * nopen;
                P.shift_edges += (int64_t)cnt * nzero;
                ++r;
            }
            ++mi;
        }
        L.y = r;
        L.w = mi;
        P.levels[l] = L;
        P.max_rows = std::max(P.max_rows, r);
        P.max_masks = std::max(P.max_masks, mi);
    }
    P.closes = P.states;
    P.levels[2 * n + 1] = make_int4((int)P.rows.size(), 0, (int)P.masks.size(), 0);
    P.mrec.assign(P.masks.size() * kRecInts, -1);
    for (size_t i = 0; i < P.masks.size(); ++i) {
        const int code = P.masks[i];
        const uint32_t ones = P.minfo[code] & 0xffffu, twos = P.minfo[code] >> 16;
        int32_t *r = &P.mrec[i * kRecInts];
        r[0] = code;
        r[1] = (int32_t)P.minfo[code];
        r[2] = P.rowbase[code];
        for (int w = 0; w < n; ++w)
            if (!((twos >> w) & 1u)) r[3 + w] = P.rowbase[code + pow3(w)];
        (void)ones;
    }
}

// The sublattice-labelled plan (mask digits base 4; see cos_internal.hpp).
void build_host_plan_sub(int n, HostPlan &P) {
    P.n = n;
    P.sub = true;
    P.rec_ints = kSubRecInts;
    int N4 = 1;
    for (int k = 0; k < n; ++k) N4 *= 4;
    P.rowbase.assign(N4, -1);
    P.minfo.assign(N4, 0);
    std::vector<uint32_t> subb(N4, 0);
    std::vector<std::vector<int32_t>> bylevel(2 * n + 2);
    for (int code = 0; code < N4; ++code) {
        uint32_t ones = 0, twos = 0, sb = 0;
        int c = code, lvl = 0;
        for (int k = 0; k < n; ++k) {
            const int d = c & 3;
            c >>= 2;
            if (d == 1 || d == 2) ones |= 1u << k, lvl += 1;
            if (d == 2) sb |= 1u << k;
            if (d == 3) twos |= 1u << k, lvl += 2;
        }
        P.minfo[code] = ones | (twos << 16);
        subb[code] = sb;
        if (!((ones | twos) & 1u)) continue;   // vertex 0 is always visited
        bylevel[lvl].push_back(code);
    }
    P.levels.assign(2 * n + 2, make_int4(0, 0, 0, 0));
    for (int l = 1; l <= 2 * n; ++l) {
        int4 L;
        L.x = (int)P.rows.size();
        L.z = (int)P.masks.size();
        int r = 0, mi = 0;
        for (int code : bylevel[l]) {
            const uint32_t ones = P.minfo[code] & 0xffffu, twos = P.minfo[code] >> 16;
            P.rowbase[code] = r;
            P.masks.push_back(code);
            // rows: (0, s_0) alone, or label pairs for head 0 and every h >= 1 visited twice
            std::vector<std::pair<int, int>> heads;
            if (!(twos & 1u)) {
                heads.push_back({0, (int)(subb[code] & 1u)});
            } else {
                heads.push_back({0, 0});
                heads.push_back({0, 1});
                for (int h = 1; h < n; ++h)
                    if ((twos >> h) & 1u) heads.push_back({h, 0}), heads.push_back({h, 1});
            }
            for (auto [u, su] : heads) {
                P.rows.push_back(make_int2(code, 2 * u + su));
                const uint32_t cs = sub_current(n, u, su, ones, twos, subb[code]);
                int edges = 0;   // per state: one child per open vertex and admissible label
                for (int w = 0; w < n; ++w) {
                    if ((twos >> w) & 1u) continue;
                    edges += ((ones >> w) & 1u) ? 1 : 2;
                }
                const int cnt = __builtin_popcount(cs);
                P.states += cnt;
                P.ext += (int64_t)cnt * edges;
                ++r;
            }
            ++mi;
        }
        L.y = r;
        L.w = mi;
        P.levels[l] = L;
        P.max_rows = std::max(P.max_rows, r);
        P.max_masks = std::max(P.max_masks, mi);
    }
    P.closes = P.states;
    P.levels[2 * n + 1] = make_int4((int)P.rows.size(), 0, (int)P.masks.size(), 0);
    P.mrec.assign(P.masks.size() * kSubRecInts, -1);
    int p4[kSubNmax + 1];
    p4[0] = 1;
    for (int k = 1; k <= kSubNmax; ++k) p4[k] = 4 * p4[k - 1];
    for (size_t i = 0; i < P.masks.size(); ++i) {
        const int code = P.masks[i];
        int32_t *r = &P.mrec[i * kSubRecInts];
        r[0] = code;
        r[1] = (int32_t)P.minfo[code];
        r[2] = P.rowbase[code];
        r[3] = (int32_t)subb[code];
        for (int w = 0; w < n; ++w) {
            const int d = (code / p4[w]) & 3;
            if (d == 0) {
                r[4 + 2 * w] = P.rowbase[code + p4[w]];          // -> once on A
                r[4 + 2 * w + 1] = P.rowbase[code + 2 * p4[w]];  // -> once on B
            } else if (d != 3) {
                r[4 + 2 * w + (d - 1)] = P.rowbase[code + (3 - d) * p4[w]];   // -> twice, label kept
            }
        }
    }
}

struct DevTables {
    DevPlan dp{};
    void *mem = nullptr;
};

std::mutex g_mu;
std::map<std::pair<int, int>, std::shared_ptr<HostPlan>> g_host;   // (n, sublattice)
std::map<std::tuple<int, int, int>, DevTables> g_dev;              // (device, n, sublattice)
int64_t g_live = 0;   // batch handles alive: they hold pointers into g_dev's tables

std::shared_ptr<HostPlan> host_plan(int n, bool sub = false) {
    auto key = std::make_pair(n, sub ? 1 : 0);
    auto it = g_host.find(key);
    if (it != g_host.end()) return it->second;
    auto p = std::make_shared<HostPlan>();
    if (sub) build_host_plan_sub(n, *p);
    else build_host_plan(n, *p);
    g_host[key] = p;
    return p;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// upper bound on each of a batch's two level workspaces (bytes):
// cos_set_workspace_limit, or by default a share of the device memory free
// when the workspace is made.  A batch whose groups do not fit runs them in
// chunks.
std::atomic<int64_t> g_ws_limit{0};

int64_t workspace_cap(int64_t lim, double share_of_free) {
    if (lim > 0) return lim;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return 0;
    return (int64_t)(share_of_free * (double)fr);
}

// allocates `doubles_of()` doubles after fitting the chunks under `cap`
// bytes; while the allocation fails, halves every chunk of more than one
// group and tries again
template <class Chunk, class Size>
cos_status alloc_chunked(double **out, std::vector<int> &chunks, const std::vector<int> &ngroups, int64_t cap,
                         Chunk per_group_doubles, Size doubles_of, const char *what) {
    for (size_t i = 0; i < chunks.size(); ++i)
        chunks[i] = (int)std::max<int64_t>(1, std::min<int64_t>(ngroups[i], cap / (8 * per_group_doubles(i))));
    while (true) {
        const int64_t n = doubles_of();
        if (dev_malloc((void **)out, sizeof(double) * (size_t)std::max<int64_t>(n, 1)) == hipSuccess) return COS_OK;
        (void)hipGetLastError();
        *out = nullptr;
        bool halved = false;
        for (int &c : chunks)
            if (c > 1) c = (c + 1) / 2, halved = true;
        if (!halved) return fail(COS_ENOMEM, "%s allocation failed (%.1f MB, one group per chunk)", what, 8.0 * n / 1e6);
    }
}

cos_status device_plan(int dev, int n, bool sub, DevPlan *out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_tuple(dev, n, sub ? 1 : 0);
    auto it = g_dev.find(key);
    if (it != g_dev.end()) {
        *out = it->second.dp;
        return COS_OK;
    }
    auto hp = host_plan(n, sub);
    const size_t s1 = align_up(hp->mrec.size() * 4), s2 = align_up(hp->levels.size() * sizeof(int4));
    char *mem = nullptr;
    if (dev_malloc((void **)&mem, s1 + s2) != hipSuccess)
        return fail(COS_ENOMEM, "device allocation of the state tables for n=%d failed", n);
    hipError_t e = hipMemcpy(mem, hp->mrec.data(), hp->mrec.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mem + s1, hp->levels.data(), hp->levels.size() * sizeof(int4), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return fail(COS_EDEVICE, "upload of the state tables failed: %s", hipGetErrorString(e));
    }
    DevTables t;
    t.mem = mem;
    t.dp.mrec = (const int32_t *)mem;
    t.dp.levels = (const int4 *)(mem + s1);
    t.dp.n = n;
    t.dp.max_rows = hp->max_rows;
    t.dp.max_masks = hp->max_masks;
    t.dp.total_rows = (int64_t)hp->rows.size();
    g_dev[key] = t;
    *out = t.dp;
    return COS_OK;
}

cos_status check_device(int *dev, int *ncu, int64_t *mem = nullptr) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
        return fail(COS_EUNSUPPORTED, "no HIP device available");
    HIP_TRY(hipGetDevice(dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, *dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(COS_EUNSUPPORTED, "device %d is %s; this library is built for gfx950", *dev, prop.gcnArchName);
    *ncu = prop.multiProcessorCount;
    if (mem) *mem = (int64_t)prop.totalGlobalMem;
    return COS_OK;
}

cos_status check_common(int32_t nflav, int32_t variant, int32_t flags) {
    if (variant != COS_UNIFORM && variant != COS_FLAVOUR)
        return fail(COS_EINVAL, "variant must be COS_UNIFORM (0) or COS_FLAVOUR (1), got %d", variant);
    const int32_t known = COS_F_STUBS | COS_F_SUBLATTICE | COS_F_MASK_ONLY | COS_F_DETERMINISTIC;
    if (flags & ~known) return fail(COS_EINVAL, "unknown flag bits 0x%x", flags & ~known);
    if ((flags & COS_F_STUBS) && (flags & COS_F_SUBLATTICE))
        return fail(COS_EINVAL, "COS_F_STUBS cannot be combined with COS_F_SUBLATTICE");
    if ((flags & COS_F_DETERMINISTIC) && (flags & COS_F_SUBLATTICE))
        return fail(COS_EINVAL, "COS_F_DETERMINISTIC cannot be combined with COS_F_SUBLATTICE");
    if (nflav < 1 || nflav > COS_FMAX) return fail(COS_ERANGE, "nflav must be in [1, %d], got %d", COS_FMAX, nflav);
    if (flags & COS_F_MASK_ONLY) {
        if (variant != COS_FLAVOUR || nflav != 2)
            return fail(COS_EINVAL, "COS_F_MASK_ONLY needs COS_FLAVOUR with nflav = 2 (the two spin blocks)");
        if (flags & COS_F_STUBS) return fail(COS_EINVAL, "COS_F_MASK_ONLY cannot be combined with COS_F_STUBS");
    }
    return COS_OK;
}

// the mask-only variant keeps non-physical clows, which cancel only through
// the fermion sign of a cycle
cos_status check_weight(int32_t flags, double cycle_weight) {
    if ((flags & COS_F_MASK_ONLY) && cycle_weight != -1.0)
        return fail(COS_EINVAL, "COS_F_MASK_ONLY needs cycle_weight = -1, got %g", cycle_weight);
    return COS_OK;
}

}  // namespace

// launch shape of the level kernels of one order
struct LaunchShape {
    int fwd_wpb = 8;    // forward: wavefronts per workgroup (<= 8; sublattice: <= 16, default 16)
    int fwd_cap = 0;    // forward: most masks per wavefront (0: by flavour count)
    int adj_cap = 8;    // reverse: most masks per wavefront
};

// all configurations of one order inside a batch
struct OrderGroup {
    int n = 0, first = 0, count = 0;   // configurations d_order[first .. first + count)
    int ngroups = 0;                   // 64 configurations per group (one per lane)
    int64_t gt_off = 0, sig_off = 0, lane_off = 0;   // offsets into the packed buffers
    int chunk_fwd = 1, chunk_adj = 1;  // groups per chunk (bounded workspace)
    int adj_split = 0;                 // reverse sweep: 0 = every forward level stored; h > 0 = levels
                                       // h+1..2n stored by the forward, levels 1..h recomputed later
    int64_t gb_off = 0, sb_off = 0;    // offsets into the packed gradient accumulators
    int64_t sp_off = 0;                // deterministic reverse: offset into the shift partial sums
    LaunchShape shape;                 // launch shape of the level kernels (autotuned)
    bool sub = false;                  // sublattice-labelled states (2n slots per row)
    bool side = false;                 // forward on the batch's side stream, in the side windows
    std::shared_ptr<HostPlan> hp;
    int slots() const { return sub ? 2 * n : n; }
};

struct cos_batch_s {
    int dev = 0, ncu = 0;
    int64_t ws_cap = 0;                // bytes of the forward's level windows (chunking of the groups)
    int64_t ws_limit = 0;              // cos_set_workspace_limit when planned (0: share of free memory)
    int32_t nconf = 0, nflav = 0, variant = 0, flags = 0;
    int nfs = 1, nmat = 1, nstub = 1;
    bool uniform_n = true;
    DevPlan plans[COS_NMAX + 1]{};
    std::vector<OrderGroup> orders;    // largest order first
    int32_t *d_order = nullptr;        // configurations grouped by order
    double *d_GT = nullptr, *d_sigT = nullptr;
    int32_t *d_lane = nullptr;
    double *d_win = nullptr;           // forward level windows
    int64_t win_doubles = 0;
    // with two or more orders the batched forward runs the orders after the
    // largest (or after the two largest, when the windows of the others would
    // not fit) on a second stream (default priority), in level windows of
    // their own, while the rest run on the caller's stream: the side orders'
    // launches fill the chip while the large ones are in their small first
    // and last levels
    size_t side_first = 0;             // first order on the side stream (0: none)
    double *d_win2 = nullptr;          // the side orders' level windows (each order in one chunk)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // reverse sweep (allocated on first use)
    double *d_Fall = nullptr, *d_GbT = nullptr, *d_sbT = nullptr;
    double *d_Gpart = nullptr, *d_Spart = nullptr;   // deterministic reverse: per-part partial sums
    int64_t fall_doubles = 0;
    // phase timing: events recorded at phase boundaries since the last read,
    // each labelled with the phase that starts there (-1: end of a call)
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_phase;
    bool counted = false;              // included in g_live
    int adj_segments = 0;              // 0 automatic, 1 store every forward level, 2 two segments
};

namespace {

// start of `phase` (or, with -1, the end of a call) on stream s
hipError_t tmark(cos_batch_s *b, int phase, hipStream_t s) {
    if (!b->timing) return hipSuccess;
    const size_t k = b->ev_phase.size();
    if (k == b->ev.size()) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        b->ev.push_back(e);
    }
    b->ev_phase.push_back(phase);
    return hipEventRecord(b->ev[k], s);
}

}  // namespace

extern "C" {

const char *cos_status_string(cos_status s) {
    switch (s) {
        case COS_OK: return "ok";
        case COS_EINVAL: return "invalid argument";
        case COS_ERANGE: return "argument out of range";
        case COS_ENOMEM: return "out of memory";
        case COS_EDEVICE: return "device error";
        case COS_EUNSUPPORTED: return "unsupported device";
    }
    return "unknown status";
}

const char *cos_last_error(void) { return g_err.c_str(); }

cos_status cos_plan_counts(int32_t n, int64_t *states, int64_t *extensions, int64_t *closes,
                           int64_t *shift_edges, int64_t *masks, int64_t *rows) {
    if (n < 1 || n > COS_NMAX) return fail(COS_ERANGE, "n must be in [1, %d], got %d", COS_NMAX, n);
    std::shared_ptr<HostPlan> p;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        p = host_plan(n);
    }
    if (states) *states = p->states;
    if (extensions) *extensions = p->ext;
    if (closes) *closes = p->closes;
    if (shift_edges) *shift_edges = p->shift_edges;
    if (masks) *masks = (int64_t)p->masks.size();
    if (rows) *rows = (int64_t)p->rows.size();
    return COS_OK;
}

cos_status cos_plan_counts_sublattice(int32_t n, int64_t *states, int64_t *extensions, int64_t *closes,
                                      int64_t *masks, int64_t *rows) {
    if (n < 1 || n > COS_NMAX_SUBLATTICE)
        return fail(COS_ERANGE, "n must be in [1, %d], got %d", COS_NMAX_SUBLATTICE, n);
    std::shared_ptr<HostPlan> p;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        p = host_plan(n, true);
    }
    if (states) *states = p->states;
    if (extensions) *extensions = p->ext;
    if (closes) *closes = p->closes;
    if (masks) *masks = (int64_t)p->masks.size();
    if (rows) *rows = (int64_t)p->rows.size();
    return COS_OK;
}

cos_status cos_plan_counts_mask_only(int32_t n, int32_t flags, int64_t *states, int64_t *extensions,
                                     int64_t *closes) {
    if (flags & ~COS_F_SUBLATTICE) return fail(COS_EINVAL, "flags may only hold COS_F_SUBLATTICE, got 0x%x", flags);
    const bool sub = (flags & COS_F_SUBLATTICE) != 0;
    const int nmax = sub ? COS_NMAX_SUBLATTICE : COS_NMAX;
    if (n < 1 || n > nmax) return fail(COS_ERANGE, "n must be in [1, %d], got %d", nmax, n);
    // the slots the level kernels visit in mask-only mode: rows (m, u[, s_u])
    // with the plane of head vertex 0 fixed by m_0, current slots from the
    // closed-form tables
    const int base = sub ? 4 : 3;
    int64_t ncodes = 1;
    for (int k = 0; k < n; ++k) ncodes *= base;
    int64_t st = 0, ex = 0, cl = 0;
    for (int64_t code = 0; code < ncodes; ++code) {
        uint32_t ones = 0, twos = 0, subb = 0;
        int64_t c = code;
        for (int k = 0; k < n; ++k) {
            const int d = (int)(c % base);
            c /= base;
            if (d == base - 1) {
                twos |= 1u << k;   // visited twice
            } else if (d != 0) {
                ones |= 1u << k;   // visited once (labelled: digit 1 on A, 2 on B)
                if (d == 2) subb |= 1u << k;
            }
        }
        if (!((ones | twos) & 1u)) continue;   // vertex 0 is visited first
        const bool full = twos == (1u << n) - 1u;
        int open_pts = 0;   // extension targets of one slot (points, with their labels)
        for (int w = 0; w < n; ++w)
            if (!((twos >> w) & 1u)) open_pts += (sub && !((ones >> w) & 1u)) ? 2 : 1;
        for (int u = 0; u < n; ++u) {
            if (u > 0 && !((twos & 1u) && ((twos >> u) & 1u))) continue;
            const int nlab = sub ? ((u == 0 && (ones & 1u)) ? 1 : 2) : 1;
            for (int li = 0; li < nlab; ++li) {
                const int su = (sub && u == 0 && (ones & 1u)) ? (int)(subb & 1u) : li;
                for (int b = 0; b < 2; ++b) {
                    if (u == 0 && ((b == 0) == ((twos & 1u) != 0u))) continue;   // empty plane
                    const uint32_t cs = sub ? sub_current(n, u, su, ones, twos, subb) : current_set(u, ones, twos);
                    const int nc = __builtin_popcount(cs);
                    // no extension onto the head point of the first cycle
                    const int e = open_pts - ((u == 0 && (ones & 1u)) ? 1 : 0);
                    st += nc;
                    ex += (int64_t)nc * e;
                    if (ones || full) cl += nc;
                }
            }
        }
    }
    if (states) *states = st;
    if (extensions) *extensions = ex;
    if (closes) *closes = cl;
    return COS_OK;
}

cos_status cos_batch_create(int32_t nconf, const int32_t *n, int32_t nflav, int32_t variant,
                            int32_t flags, cos_batch_t *out) {
    if (!out) return fail(COS_EINVAL, "out is NULL");
    *out = nullptr;
    if (nconf < 1) return fail(COS_EINVAL, "nconf must be >= 1, got %d", nconf);
    if (!n) return fail(COS_EINVAL, "n is NULL");
    cos_status st = check_common(nflav, variant, flags);
    if (st) return st;
    const bool sub = (flags & COS_F_SUBLATTICE) != 0;
    const int nmax = sub ? COS_NMAX_SUBLATTICE : COS_NMAX;
    for (int32_t c = 0; c < nconf; ++c)
        if (n[c] < 1 || n[c] > nmax)
            return fail(COS_ERANGE, "n[%d] = %d outside [1, %d]", c, n[c], nmax);
    int dev = 0, ncu = 0;
    int64_t mem = 0;
    if ((st = check_device(&dev, &ncu, &mem))) return st;

    struct Del { void operator()(cos_batch_s *p) const { cos_batch_destroy(p); } };
    std::unique_ptr<cos_batch_s, Del> b(new cos_batch_s());
    b->dev = dev;
    b->ncu = ncu;
    // the forward's level windows take up to 45% of the free memory; the
    // reverse sweep's stored levels (made at its first call) up to 90% of what
    // is free then
    b->ws_limit = g_ws_limit.load();
    b->ws_cap = workspace_cap(b->ws_limit, 0.45);
    if (b->ws_cap <= 0) b->ws_cap = mem / 3;
    b->nconf = nconf;
    b->nflav = nflav;
    b->variant = variant;
    b->flags = flags;
    b->nfs = variant == COS_FLAVOUR ? nflav : 1;
    b->nmat = b->nfs;
    b->nstub = b->nfs;
    bool seen[COS_NMAX + 1] = {false};
    for (int c = 0; c < nconf; ++c) seen[n[c]] = true;
    for (int k = 1; k <= COS_NMAX; ++k)
        if (seen[k]) {
            if ((st = device_plan(dev, k, sub, &b->plans[k]))) return st;
        }
    b->uniform_n = std::all_of(n, n + nconf, [&](int32_t x) { return x == n[0]; });

    // configurations grouped by order, largest order first; 64 per group
    std::vector<int32_t> order(nconf);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return n[a] > n[c]; });
    int64_t gt = 0, sg = 0, ln = 0;
    for (int i = 0; i < nconf;) {
        int j = i;
        while (j < nconf && n[order[j]] == n[order[i]]) ++j;
        OrderGroup o;
        o.n = n[order[i]];
        o.first = i;
        o.count = j - i;
        o.ngroups = (o.count + 63) / 64;
        o.gt_off = gt;
        o.sig_off = sg;
        o.lane_off = ln;
        o.sub = sub;
        if (sub) o.shape.fwd_wpb = 16;   // (2n)^2 matrices in LDS: one workgroup per CU, make it wide
        {
            std::lock_guard<std::mutex> lk(g_mu);
            o.hp = host_plan(o.n, sub);
        }
        gt += (int64_t)o.ngroups * b->nfs * o.slots() * o.slots() * 64;
        sg += (int64_t)o.ngroups * b->nfs * 64;
        ln += (int64_t)o.ngroups * 64;
        b->orders.push_back(o);
        i = j;
    }
    if (dev_malloc((void **)&b->d_order, sizeof(int32_t) * nconf) != hipSuccess ||
        dev_malloc((void **)&b->d_GT, sizeof(double) * gt) != hipSuccess ||
        dev_malloc((void **)&b->d_sigT, sizeof(double) * sg) != hipSuccess ||
        dev_malloc((void **)&b->d_lane, sizeof(int32_t) * ln) != hipSuccess)
        return fail(COS_ENOMEM, "workspace allocation failed (%.1f MB)", 8.0 * (gt + sg) / 1e6);
    {
        // two level windows per group of the chunk
        std::vector<int> chunks(b->orders.size()), ng(b->orders.size());
        for (size_t i = 0; i < b->orders.size(); ++i) ng[i] = b->orders[i].ngroups;
        auto per_group = [&](size_t i) {
            const OrderGroup &o = b->orders[i];
            return 2 * (int64_t)o.hp->max_rows * b->nfs * o.slots() * 64;
        };
        auto total = [&]() {
            int64_t w = 0;
            for (size_t i = 0; i < chunks.size(); ++i) w = std::max(w, per_group(i) * chunks[i]);
            return w;
        };
        if ((st = alloc_chunked(&b->d_win, chunks, ng, b->ws_cap, per_group, total, "level window"))) return st;
        for (size_t i = 0; i < chunks.size(); ++i) b->orders[i].chunk_fwd = chunks[i];
        b->win_doubles = total();
        // side stream for the orders after the largest (else after the two
        // largest) when their windows, each order whole, take at most half of
        // the workspace bound; otherwise, or if any of it cannot be had, every
        // order runs on the caller's stream
        size_t first = 0;
        int64_t w2 = 0;
        for (size_t f = 1; f <= 2 && !first && f < b->orders.size(); ++f) {
            int64_t w = 0;
            for (size_t i = f; i < b->orders.size(); ++i) w = std::max(w, per_group(i) * b->orders[i].ngroups);
            if (8 * w <= b->ws_cap / 2) first = f, w2 = w;
        }
        if (first) {
            bool ok = dev_malloc((void **)&b->d_win2, sizeof(double) * w2) == hipSuccess;
            ok = ok && hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) == hipSuccess;
            if (ok) {
                b->side_first = first;
                for (size_t i = first; i < b->orders.size(); ++i) {
                    b->orders[i].side = true;
                    b->orders[i].chunk_fwd = b->orders[i].ngroups;
                }
            } else {
                (void)hipGetLastError();
                (void)hipFree(b->d_win2);
                b->d_win2 = nullptr;
                if (b->side) (void)hipStreamDestroy(b->side);
                if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
                b->side = nullptr;
                b->ev_fork = nullptr;
            }
        }
    }
    HIP_TRY(hipMemcpy(b->d_order, order.data(), sizeof(int32_t) * nconf, hipMemcpyHostToDevice));
    {
        std::lock_guard<std::mutex> lk(g_mu);
        ++g_live;
        b->counted = true;
    }
    *out = b.release();
    return COS_OK;
}

cos_status cos_batch_destroy(cos_batch_t b) {
    if (!b) return COS_OK;
    (void)hipFree(b->d_order);
    (void)hipFree(b->d_GT);
    (void)hipFree(b->d_sigT);
    (void)hipFree(b->d_lane);
    (void)hipFree(b->d_win);
    (void)hipFree(b->d_win2);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    (void)hipFree(b->d_Fall);
    (void)hipFree(b->d_GbT);
    (void)hipFree(b->d_sbT);
    (void)hipFree(b->d_Gpart);
    (void)hipFree(b->d_Spart);
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    if (b->counted) {
        std::lock_guard<std::mutex> lk(g_mu);
        --g_live;
    }
    delete b;
    return COS_OK;
}

// a handle's buffers and tables live on the device it was planned on
static cos_status check_batch_device(cos_batch_t b) {
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != b->dev)
        return fail(COS_EINVAL, "the batch was planned on device %d but device %d is current", b->dev, cur);
    return COS_OK;
}

static cos_status check_batch_ptrs(cos_batch_t b, const double *d_G, const int64_t *d_Goff,
                                   const double *d_stub) {
    if (!b) return fail(COS_EINVAL, "batch handle is NULL");
    if (cos_status st = check_batch_device(b)) return st;
    if (!d_G) return fail(COS_EINVAL, "d_G is NULL");
    if (!d_Goff && !b->uniform_n) return fail(COS_EINVAL, "d_Goff is required when the orders differ");
    if ((b->flags & COS_F_STUBS) && !d_stub) return fail(COS_EINVAL, "COS_F_STUBS set but d_stub is NULL");
    return COS_OK;
}

static PackArgs pack_args(cos_batch_t b, const OrderGroup &o, const double *d_G, const int64_t *d_Goff,
                          const double *d_stub) {
    PackArgs p;
    std::memset(&p, 0, sizeof(p));
    p.G = d_G;
    p.Goff = d_Goff;
    p.stub = (b->flags & COS_F_STUBS) ? d_stub : nullptr;
    p.order = b->d_order + o.first;
    p.GT = b->d_GT + o.gt_off;
    p.sigT = b->d_sigT + o.sig_off;
    p.lane_cfg = b->d_lane + o.lane_off;
    p.n = o.slots();   // matrix side: n, or 2n with sublattice labels
    p.nfs = b->nfs;
    p.nmat = b->nmat;
    p.nstub = b->nstub;
    p.variant = b->variant;
    p.ngroups = o.ngroups;
    p.count = o.count;
    return p;
}

static LvlArgs level_args(cos_batch_t b, const OrderGroup &o, double cycle_weight) {
    LvlArgs a;
    std::memset(&a, 0, sizeof(a));
    a.plan = b->plans[o.n];
    a.GT = b->d_GT + o.gt_off;
    a.sigT = b->d_sigT + o.sig_off;
    a.lane_cfg = b->d_lane + o.lane_off;
    a.nfs = b->nfs;
    a.stubs = (b->flags & COS_F_STUBS) ? 1 : 0;
    a.W = cycle_weight * (b->variant == COS_UNIFORM ? (double)b->nflav : 1.0);
    a.mask_only = (b->flags & COS_F_MASK_ONLY) ? 1 : 0;
    return a;
}

// masks per wavefront of a forward level launch with `nm` masks and `ng`
// groups: up to the shape's cap (to amortise loading G into LDS), fewer when
// the level is small so that its rows spread over enough wavefronts
static int fwd_masks(const LaunchShape &sh, int nfs, int nm, int ng, int ncu) {
    int cap = sh.fwd_cap ? sh.fwd_cap : (nfs <= 1 ? 8 : kMultiMasks);
    if (nfs > 1) cap = std::min(cap, kMultiMasks);   // close sums of several flavours in registers
    const int64_t per = ((int64_t)nm * ng) / std::max<int64_t>(1, (int64_t)ncu * 16);
    return (int)std::max<int64_t>(1, std::min<int64_t>(cap, per));
}

// masks per wavefront of a reverse level launch: one workgroup (16
// wavefronts, one per CU by its LDS footprint) loads G and flushes its dS/dG
// accumulator once per flavour, so blocks should be large; its wavefronts
// share the block's masks dynamically, so workgroups take equal time, and the
// level is cut into as few rounds of one workgroup per CU as the cap allows,
// with the masks spread evenly over them
static int adj_masks(const LaunchShape &sh, int nm, int ng, int ncu) {
    const int64_t slots = (int64_t)std::max(1, ncu) * 16;                 // wavefronts of one round (16 per CU)
    const int64_t work = (int64_t)nm * ng;
    const int64_t rounds = std::max<int64_t>(1, (work + slots * sh.adj_cap - 1) / (slots * sh.adj_cap));
    return (int)std::max<int64_t>(1, std::min<int64_t>(sh.adj_cap, (work + slots * rounds - 1) / (slots * rounds)));
}

// forward levels of one order, all groups, chunk by chunk (two level windows:
// the side windows for a side order); `mark`: record the phase marks on s
static cos_status forward_order(cos_batch_t b, const OrderGroup &o, const double *d_G, const int64_t *d_Goff,
                                const double *d_stub, double cycle_weight, double *d_out, hipStream_t s,
                                bool mark = true) {
    if (mark) HIP_TRY(tmark(b, COS_PHASE_PACK, s));
    LAUNCH_TRY(launch_pack(pack_args(b, o, d_G, d_Goff, d_stub), s));
    if (mark) HIP_TRY(tmark(b, COS_PHASE_FORWARD, s));
    const int64_t rs = (int64_t)b->nfs * o.slots() * 64;
    const int64_t gstride = (int64_t)o.hp->max_rows * rs;
    double *const base = o.side ? b->d_win2 : b->d_win;
    for (int c0 = 0; c0 < o.ngroups; c0 += o.chunk_fwd) {
        const int cg = std::min(o.chunk_fwd, o.ngroups - c0);
        double *win0 = base, *win1 = base + gstride * cg;
        for (int l = 1; l <= 2 * o.n; ++l) {
            LvlArgs a = level_args(b, o, cycle_weight);
            a.level = l;
            a.group0 = c0;
            a.cur = (l & 1) ? win1 : win0;
            a.nxt = (l & 1) ? win0 : win1;
            a.cur_gstride = a.nxt_gstride = gstride;
            a.cur_frows = a.nxt_frows = o.hp->max_rows;
            const int nm = o.hp->levels[l].w;
            a.mpb = fwd_masks(o.shape, b->nfs, nm, cg, b->ncu);
            a.out = d_out;
            if (o.sub) LAUNCH_TRY(launch_sub_level(a, (nm + a.mpb - 1) / a.mpb, cg, o.shape.fwd_wpb, s));
            else LAUNCH_TRY(launch_level(a, false, (nm + a.mpb - 1) / a.mpb, cg, o.shape.fwd_wpb, s));
        }
    }
    return COS_OK;
}

cos_status cos_connected_sum_batched(cos_batch_t b, const double *d_G, const int64_t *d_Goff,
                                     const double *d_stub, double cycle_weight, double *d_out,
                                     void *stream) {
    cos_status st = check_batch_ptrs(b, d_G, d_Goff, d_stub);
    if (st) return st;
    if ((st = check_weight(b->flags, cycle_weight))) return st;
    if (!d_out) return fail(COS_EINVAL, "d_out is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (!b->side_first) {
        for (const OrderGroup &o : b->orders)
            if ((st = forward_order(b, o, d_G, d_Goff, d_stub, cycle_weight, d_out, s))) return st;
        HIP_TRY(tmark(b, -1, s));
        return COS_OK;
    }
    // fork: the side orders start after what s holds so far; join: s waits
    // for them (also after a failure, so that no side work outlives the call's
    // place on s); the phase marks stay on s
    HIP_TRY(hipEventRecord(b->ev_fork, s));
    HIP_TRY(hipStreamWaitEvent(b->side, b->ev_fork, 0));
    cos_status st_side = COS_OK, st_main = COS_OK;
    for (size_t i = b->side_first; i < b->orders.size() && !st_side; ++i)
        st_side = forward_order(b, b->orders[i], d_G, d_Goff, d_stub, cycle_weight, d_out, b->side, false);
    for (size_t i = 0; i < b->side_first && !st_main; ++i)
        st_main = forward_order(b, b->orders[i], d_G, d_Goff, d_stub, cycle_weight, d_out, s);
    HIP_TRY(hipEventRecord(b->ev_join, b->side));
    HIP_TRY(hipStreamWaitEvent(s, b->ev_join, 0));
    if (st_side) return st_side;
    if (st_main) return st_main;
    HIP_TRY(tmark(b, -1, s));
    return COS_OK;
}

// rows of levels a..c (inclusive) of a plan
static int64_t level_rows(const HostPlan &p, int a, int c) { return (int64_t)p.levels[c + 1].x - p.levels[a].x; }

// the split level h of a two-segment reverse sweep that minimises the larger
// segment (levels 1..h, recomputed, or h+1..2n, stored by the first forward)
static int best_split(const HostPlan &p, int n) {
    int best = 0;
    int64_t bv = INT64_MAX;
    for (int h = 1; h < 2 * n; ++h) {
        const int64_t v = std::max(level_rows(p, 1, h), level_rows(p, h + 1, 2 * n));
        if (v < bv) bv = v, best = h;
    }
    return best;
}

// forward-state rows the reverse sweep of one group keeps
static int64_t adj_store_rows(const HostPlan &p, int n, int h) {
    return h ? std::max(level_rows(p, 1, h), level_rows(p, h + 1, 2 * n)) : (int64_t)p.rows.size();
}

static cos_status prepare_adjoint(cos_batch_t b) {
    if (b->d_Fall) return COS_OK;
    int64_t gb = 0, sb = 0, sp = 0;
    for (OrderGroup &o : b->orders) {
        o.gb_off = gb;
        o.sb_off = sb;
        o.sp_off = sp;
        gb += (int64_t)o.ngroups * b->nfs * o.slots() * o.slots() * 64;
        sb += (int64_t)o.ngroups * b->nfs * 64;
        sp += (int64_t)kDetParts * o.ngroups * b->nfs * o.slots() * 64;
    }
    const bool det = (b->flags & COS_F_DETERMINISTIC) != 0;
    if (dev_malloc((void **)&b->d_GbT, sizeof(double) * gb) != hipSuccess ||
        dev_malloc((void **)&b->d_sbT, sizeof(double) * sb) != hipSuccess ||
        (det && (dev_malloc((void **)&b->d_Gpart, sizeof(double) * kDetParts * gb) != hipSuccess ||
                 dev_malloc((void **)&b->d_Spart, sizeof(double) * sp) != hipSuccess))) {
        (void)hipFree(b->d_GbT);
        (void)hipFree(b->d_sbT);
        (void)hipFree(b->d_Gpart);
        b->d_GbT = b->d_sbT = b->d_Gpart = b->d_Spart = nullptr;
        return fail(COS_ENOMEM, "gradient accumulator allocation failed");
    }
    // all forward levels and two adjoint windows per group of the chunk, in
    // at most 90% of the memory free now (or the caller's bound)
    int64_t cap = workspace_cap(b->ws_limit, 0.9);
    if (cap <= 0) cap = b->ws_cap;
    // two segments (about 40% less memory, the lower levels computed twice)
    // when asked for, or when storing every level would split the groups
    for (OrderGroup &o : b->orders) {
        const int64_t rs = (int64_t)b->nfs * o.slots() * 64;
        const int64_t all = ((int64_t)o.hp->rows.size() + 2 * (int64_t)o.hp->max_rows) * rs;
        const bool seg = o.n >= 3 && (b->adj_segments == 2 ||
                                      (b->adj_segments == 0 && cap / (8 * all) < o.ngroups));
        o.adj_split = seg ? best_split(*o.hp, o.n) : 0;
    }
    std::vector<int> chunks(b->orders.size()), ng(b->orders.size());
    for (size_t i = 0; i < b->orders.size(); ++i) ng[i] = b->orders[i].ngroups;
    auto per_group = [&](size_t i) {
        const OrderGroup &o = b->orders[i];
        return (adj_store_rows(*o.hp, o.n, o.adj_split) + 2 * (int64_t)o.hp->max_rows) * b->nfs * o.slots() * 64;
    };
    auto total = [&]() {
        int64_t w = 0;
        for (size_t i = 0; i < chunks.size(); ++i) w = std::max(w, per_group(i) * chunks[i]);
        return w;
    };
    if (cos_status st = alloc_chunked(&b->d_Fall, chunks, ng, cap, per_group, total, "reverse-sweep workspace")) {
        (void)hipFree(b->d_GbT);
        (void)hipFree(b->d_sbT);
        (void)hipFree(b->d_Gpart);
        (void)hipFree(b->d_Spart);
        b->d_GbT = b->d_sbT = b->d_Gpart = b->d_Spart = nullptr;
        return st;
    }
    for (size_t i = 0; i < chunks.size(); ++i) b->orders[i].chunk_adj = chunks[i];
    b->fall_doubles = total();
    return COS_OK;
}

// forward (every level kept) and reverse levels of one order
// forward (levels kept) and reverse levels of one order.  Every forward level
// is stored, or with a split level h only levels h+1..2n: their reverse runs
// first, then levels 1..h are computed again into the same store and
// reversed (the adjoint windows keep B(h+1) meanwhile)
static cos_status adjoint_order(cos_batch_t b, const OrderGroup &o, const double *d_G, const int64_t *d_Goff,
                                const double *d_stub, double cycle_weight, const double *d_out_bar,
                                double *d_out, double *d_G_bar, double *d_stub_bar, hipStream_t s) {
    const PackArgs pa = pack_args(b, o, d_G, d_Goff, d_stub);
    HIP_TRY(tmark(b, COS_PHASE_PACK, s));
    LAUNCH_TRY(launch_pack(pa, s));
    double *GbT = b->d_GbT + o.gb_off, *sbT = b->d_sbT + o.sb_off;
    const int64_t ngb = (int64_t)o.ngroups * b->nfs * o.slots() * o.slots() * 64;
    const int64_t nsb = (int64_t)o.ngroups * b->nfs * 64;
    const bool det = (b->flags & COS_F_DETERMINISTIC) != 0;
    double *Gp = det ? b->d_Gpart + (int64_t)kDetParts * o.gb_off : nullptr;
    double *Sp = det ? b->d_Spart + o.sp_off : nullptr;
    const int64_t nsp = (int64_t)kDetParts * o.ngroups * b->nfs * o.slots() * 64;
    if (det) {
        LAUNCH_TRY(launch_zero(Gp, (int64_t)kDetParts * ngb, s));
        LAUNCH_TRY(launch_zero(Sp, nsp, s));
    } else {
        LAUNCH_TRY(launch_zero(GbT, ngb, s));
        LAUNCH_TRY(launch_zero(sbT, nsb, s));
    }
    const int n2 = 2 * o.n, h = o.adj_split;
    const int64_t rs = (int64_t)b->nfs * o.slots() * 64;
    const int64_t srows = adj_store_rows(*o.hp, o.n, h), mrows = o.hp->max_rows;
    const int64_t fstride = srows * rs, bstride = mrows * rs;
    // store row of level l: levels are stored from level 1 (all, or the lower
    // segment) or from level h + 1 (the upper segment)
    auto srow = [&](int l, bool upper) { return o.hp->levels[l].x - (upper ? o.hp->levels[h + 1].x : 0); };
    for (int c0 = 0; c0 < o.ngroups; c0 += o.chunk_adj) {
        const int cg = std::min(o.chunk_adj, o.ngroups - c0);
        double *Fs = b->d_Fall;
        double *B0 = Fs + fstride * cg, *B1 = B0 + bstride * cg;
        // forward from level `from` to `to`: reads level l, writes level l + 1;
        // stored levels in Fs, the others (below the upper segment, first
        // pass only) in the adjoint windows, which are free until the reverse
        auto forward = [&](int from, int to, bool first_pass) -> cos_status {
            for (int l = from; l <= to; ++l) {
                LvlArgs a = level_args(b, o, cycle_weight);
                a.level = l;
                a.group0 = c0;
                const bool in_store = !first_pass || !h || l > h;      // level l
                const bool out_store = !first_pass || !h || l + 1 > h; // level l + 1
                const bool up = first_pass && h;
                a.cur = in_store ? Fs : ((l & 1) ? B1 : B0);
                a.cur_gstride = in_store ? fstride : bstride;
                a.cur_frows = in_store ? srows : mrows;
                a.cur_row0 = in_store ? (int32_t)srow(l, up) : 0;
                a.nxt = out_store ? Fs : (((l + 1) & 1) ? B1 : B0);
                a.nxt_gstride = out_store ? fstride : bstride;
                a.nxt_frows = out_store ? srows : mrows;
                a.nxt_row0 = out_store ? (int32_t)srow(std::min(l + 1, n2 + 1), up) : 0;
                const int nm = o.hp->levels[l].w;
                a.mpb = fwd_masks(o.shape, b->nfs, nm, cg, b->ncu);
                a.out = d_out;
                if (o.sub) LAUNCH_TRY(launch_sub_level(a, (nm + a.mpb - 1) / a.mpb, cg, o.shape.fwd_wpb, s));
                else LAUNCH_TRY(launch_level(a, false, (nm + a.mpb - 1) / a.mpb, cg, o.shape.fwd_wpb, s));
            }
            return COS_OK;
        };
        auto reverse = [&](int from, int to, bool upper) -> cos_status {
            for (int l = from; l >= to; --l) {
                LvlArgs a = level_args(b, o, cycle_weight);
                a.level = l;
                a.group0 = c0;
                a.cur = (l & 1) ? B0 : B1;     // adjoints of level + 1
                a.nxt = (l & 1) ? B1 : B0;     // adjoints of level
                a.cur_gstride = a.nxt_gstride = bstride;
                a.cur_frows = a.nxt_frows = mrows;
                a.F = Fs;
                a.F_gstride = fstride;
                a.F_frows = srows;
                a.F_row0 = (int32_t)srow(l, upper);
                const int nm = o.hp->levels[l].w;
                // a level whose masks fill at most half the wavefronts of one
                // round (labelled: an eighth; its rows are split over two
                // workgroups at n = 7, 8 and each row reloads its mask's close
                // adjoints in every flavour), and whose masks hold at least
                // half the most rows a mask can have (n, labelled 2n) on
                // average (the upper levels), gives every row a wavefront of its own
                const int64_t fill = o.sub ? 8 : 2;
                a.row_items = ((int64_t)nm * cg * fill <= (int64_t)b->ncu * 16 &&
                               2 * level_rows(*o.hp, l, l) >= (int64_t)nm * o.slots()) ? 1 : 0;
                const int items = a.row_items ? nm * o.slots() : nm;
                a.mpb = adj_masks(o.shape, items, cg, b->ncu);
                a.out_bar = d_out_bar;
                a.Gbar_T = GbT;
                a.sbar_T = sbT;
                if (det) {
                    a.Gbar_T = Gp;
                    a.sbar_T = Sp;
                    a.det_groups = o.ngroups;
                    LAUNCH_TRY(launch_level_det(a, cg, s));
                    continue;
                }
                if (o.sub) LAUNCH_TRY(launch_sub_adj_level(a, (items + a.mpb - 1) / a.mpb, cg, s));
                else LAUNCH_TRY(launch_level(a, true, (items + a.mpb - 1) / a.mpb, cg, adj_waves_per_block(), s));
            }
            return COS_OK;
        };
        HIP_TRY(tmark(b, COS_PHASE_FORWARD, s));
        if (cos_status st = forward(1, n2, true)) return st;
        HIP_TRY(tmark(b, COS_PHASE_REVERSE, s));
        if (cos_status st = reverse(n2, h + 1, h != 0)) return st;
        if (h) {
            // level 1 is the start state, which the kernels form themselves
            HIP_TRY(tmark(b, COS_PHASE_FORWARD, s));
            if (cos_status st = forward(1, h - 1, false)) return st;
            HIP_TRY(tmark(b, COS_PHASE_REVERSE, s));
            if (cos_status st = reverse(h, 1, false)) return st;
        }
    }
    HIP_TRY(tmark(b, COS_PHASE_UNPACK, s));
    if (det)
        LAUNCH_TRY(launch_det_reduce(Gp, (b->flags & COS_F_STUBS) ? Sp : nullptr, ngb, nsb, o.slots(), GbT, sbT, s));
    LAUNCH_TRY(launch_unpack(pa, GbT, sbT, d_G_bar, (b->flags & COS_F_STUBS) ? d_stub_bar : nullptr, s));
    return COS_OK;
}

cos_status cos_connected_sum_adjoint(cos_batch_t b, const double *d_G, const int64_t *d_Goff,
                                     const double *d_stub, double cycle_weight,
                                     const double *d_out_bar, double *d_out, double *d_G_bar,
                                     double *d_stub_bar, void *stream) {
    cos_status st = check_batch_ptrs(b, d_G, d_Goff, d_stub);
    if (st) return st;
    if ((st = check_weight(b->flags, cycle_weight))) return st;
    if (!d_out_bar || !d_G_bar) return fail(COS_EINVAL, "d_out_bar and d_G_bar are required");
    if ((b->flags & COS_F_STUBS) && !d_stub_bar) return fail(COS_EINVAL, "COS_F_STUBS set but d_stub_bar is NULL");
    if ((st = prepare_adjoint(b))) return st;
    hipStream_t s = (hipStream_t)stream;
    for (const OrderGroup &o : b->orders)
        if ((st = adjoint_order(b, o, d_G, d_Goff, d_stub, cycle_weight, d_out_bar, d_out, d_G_bar, d_stub_bar, s)))
            return st;
    HIP_TRY(tmark(b, -1, s));
    return COS_OK;
}

// device time of fn() on stream s: one warm-up, then the best of `reps`
// windows; a window repeats fn() back to back until it spans about half a
// millisecond, so that short calls are not timed at the events' resolution
static cos_status time_best(hipStream_t s, int reps, const std::function<cos_status()> &fn, float *best) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(COS_EDEVICE, "hipEventCreate failed");
    }
    cos_status st = fn();
    *best = 1e30f;
    int inner = 1;
    for (int r = 0; r < reps + 1 && st == COS_OK; ++r) {
        float t = 0.0f;
        if (hipEventRecord(e0, s) != hipSuccess) { st = fail(COS_EDEVICE, "hipEventRecord failed"); break; }
        for (int i = 0; i < inner && st == COS_OK; ++i) st = fn();
        if (st) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
            st = fail(COS_EDEVICE, "timing events failed");
            break;
        }
        if (r == 0) {   // sizing window, not counted
            inner = std::max(1, std::min(64, (int)(0.5f / std::max(t, 1e-3f))));
            continue;
        }
        *best = std::min(*best, t / (float)inner);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

cos_status cos_batch_autotune(cos_batch_t b, const double *d_G, const int64_t *d_Goff, const double *d_stub,
                              double cycle_weight, const double *d_out_bar, double *d_out, double *d_G_bar,
                              double *d_stub_bar, void *stream) {
    cos_status st = check_batch_ptrs(b, d_G, d_Goff, d_stub);
    if (st) return st;
    if ((st = check_weight(b->flags, cycle_weight))) return st;
    if (!d_out) return fail(COS_EINVAL, "d_out is NULL");
    if (d_out_bar) {
        if (!d_G_bar) return fail(COS_EINVAL, "d_G_bar is required to tune the reverse sweep");
        if ((b->flags & COS_F_STUBS) && !d_stub_bar) return fail(COS_EINVAL, "COS_F_STUBS set but d_stub_bar is NULL");
        if ((st = prepare_adjoint(b))) return st;
    }
    hipStream_t s = (hipStream_t)stream;
    const bool was_timing = b->timing;
    b->timing = false;
    static const int kWaves[] = {4, 8, 16}, kSubWaves[] = {8, 16, 16};   // (16 twice: arrays of one size)
    static const int kCaps[] = {1, 2, 4, 8, 16};
    static const int kAdjCaps[] = {2, 4, 6, 8, 12, 16, 24, 32, 48, 64};
    for (OrderGroup &o : b->orders) {
        // forward: waves per workgroup x masks per wavefront
        LaunchShape best = o.shape;
        float tbest = 1e30f;
        for (int wv : (o.sub ? kSubWaves : kWaves))
            for (int cap : kCaps) {
                o.shape.fwd_wpb = wv;
                o.shape.fwd_cap = cap;
                float t;
                st = time_best(s, 3, [&] { return forward_order(b, o, d_G, d_Goff, d_stub, cycle_weight, d_out, s); }, &t);
                if (st) break;
                if (t < tbest) { tbest = t; best = o.shape; }
            }
        o.shape = best;
        if (st) break;
        if (!d_out_bar || (b->flags & COS_F_DETERMINISTIC)) continue;   // the deterministic reverse has one shape
        // reverse: masks per wavefront (the forward part is the same for every candidate)
        tbest = 1e30f;
        for (int cap : kAdjCaps) {
            o.shape.adj_cap = cap;
            float t;
            st = time_best(s, 3, [&] {
                return adjoint_order(b, o, d_G, d_Goff, d_stub, cycle_weight, d_out_bar, d_out, d_G_bar, d_stub_bar, s);
            }, &t);
            if (st) break;
            if (t < tbest) { tbest = t; best.adj_cap = cap; }
        }
        o.shape = best;
        if (st) break;
    }
    b->timing = was_timing;
    if (st) return st;
    // leave the outputs as a call with the chosen shapes writes them
    if (d_out_bar) return cos_connected_sum_adjoint(b, d_G, d_Goff, d_stub, cycle_weight, d_out_bar, d_out, d_G_bar,
                                                    d_stub_bar, stream);
    return cos_connected_sum_batched(b, d_G, d_Goff, d_stub, cycle_weight, d_out, stream);
}

cos_status cos_batch_launch_shape(cos_batch_t b, int32_t n, int32_t *fwd_waves, int32_t *fwd_masks_cap,
                                  int32_t *adj_masks_cap) {
    if (!b || !fwd_waves || !fwd_masks_cap || !adj_masks_cap) return fail(COS_EINVAL, "null argument");
    for (const OrderGroup &o : b->orders)
        if (o.n == n) {
            *fwd_waves = o.shape.fwd_wpb;
            int cap = o.shape.fwd_cap ? o.shape.fwd_cap : (b->nfs <= 1 ? 8 : kMultiMasks);
            if (b->nfs > 1) cap = std::min(cap, kMultiMasks);
            *fwd_masks_cap = cap;
            *adj_masks_cap = o.shape.adj_cap;
            return COS_OK;
        }
    return fail(COS_EINVAL, "the batch has no configuration of order %d", n);
}

cos_status cos_batch_set_launch_shape(cos_batch_t b, int32_t n, int32_t fwd_waves, int32_t fwd_masks,
                                      int32_t adj_masks) {
    if (!b) return fail(COS_EINVAL, "batch handle is NULL");
    for (OrderGroup &o : b->orders)
        if (o.n == n) {
            if (fwd_waves < 1 || fwd_waves > 16) return fail(COS_EINVAL, "fwd_waves must be in [1, 16]");
            if (fwd_masks < 1 || fwd_masks > 16 || adj_masks < 1 || adj_masks > 64)
                return fail(COS_EINVAL, "fwd_masks must be in [1, 16] and adj_masks in [1, 64]");
            o.shape.fwd_wpb = fwd_waves;
            o.shape.fwd_cap = fwd_masks;
            o.shape.adj_cap = adj_masks;
            return COS_OK;
        }
    return fail(COS_EINVAL, "the batch has no configuration of order %d", n);
}

cos_status cos_batch_timing_enable(cos_batch_t b, int32_t enable) {
    if (!b) return fail(COS_EINVAL, "batch handle is NULL");
    b->timing = enable != 0;
    b->ev_phase.clear();
    return COS_OK;
}

cos_status cos_batch_timing_read(cos_batch_t b, double *ms, int32_t *ncalls) {
    if (!b || !ms) return fail(COS_EINVAL, "batch handle and ms are required");
    for (int p = 0; p < COS_NPHASES; ++p) ms[p] = 0.0;
    int32_t calls = 0;
    const size_t k = b->ev_phase.size();
    if (k) HIP_TRY(hipEventSynchronize(b->ev[k - 1]));
    for (size_t i = 0; i < k; ++i) {
        if (b->ev_phase[i] < 0 || i + 1 == k) {
            ++calls;
            continue;
        }
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, b->ev[i], b->ev[i + 1]));
        ms[b->ev_phase[i]] += t;
    }
    b->ev_phase.clear();
    if (ncalls) *ncalls = calls;
    return COS_OK;
}

cos_status cos_connected_sum(int32_t n, int32_t nflav, int32_t variant, int32_t flags, const double *G,
                             const double *stub, double cycle_weight, double *out) {
    if (!G || !out) return fail(COS_EINVAL, "G and out are required");
    cos_status st = check_common(nflav, variant, flags);
    if (st) return st;
    if (n < 1 || n > COS_NMAX) return fail(COS_ERANGE, "n must be in [1, %d], got %d", COS_NMAX, n);
    if ((flags & COS_F_STUBS) && !stub) return fail(COS_EINVAL, "COS_F_STUBS set but stub is NULL");
    cos_batch_t b = nullptr;
    if ((st = cos_batch_create(1, &n, nflav, variant, flags, &b))) return st;
    const size_t side = (flags & COS_F_SUBLATTICE) ? 2 * (size_t)n : (size_t)n;
    const size_t ng = (size_t)b->nmat * side * side;
    double *d = nullptr;
    if (dev_malloc((void **)&d, sizeof(double) * (ng + COS_FMAX + 1)) != hipSuccess) {
        cos_batch_destroy(b);
        return fail(COS_ENOMEM, "device allocation failed");
    }
    hipError_t e = hipMemcpy(d, G, sizeof(double) * ng, hipMemcpyHostToDevice);
    if (!e && (flags & COS_F_STUBS)) e = hipMemcpy(d + ng, stub, sizeof(double) * b->nstub, hipMemcpyHostToDevice);
    if (!e) {
        st = cos_connected_sum_batched(b, d, nullptr, d + ng, cycle_weight, d + ng + COS_FMAX, nullptr);
        if (!st) e = hipMemcpy(out, d + ng + COS_FMAX, sizeof(double), hipMemcpyDeviceToHost);
    }
    (void)hipFree(d);
    cos_batch_destroy(b);
    if (e) return fail(COS_EDEVICE, "HIP error: %s", hipGetErrorString(e));
    return st;
}

cos_status cos_build_g0(int32_t nconf, const int32_t *d_n, const int64_t *d_voff, const int32_t *d_sites,
                        const double *d_tau, int32_t L, double t, double beta, int32_t nmat, const double *mu,
                        const double *alpha, const int64_t *d_Goff, double *d_G, double *d_dG, void *stream) {
    if (nconf < 1) return fail(COS_EINVAL, "nconf must be >= 1");
    if (!d_n || !d_voff || !d_sites || !d_tau || !d_Goff || !d_G || !mu || !alpha)
        return fail(COS_EINVAL, "null pointer argument");
    if (L < 1 || L > 32) return fail(COS_ERANGE, "L must be in [1, 32], got %d", L);
    if (nmat < 1 || nmat > COS_FMAX) return fail(COS_ERANGE, "nmat must be in [1, %d]", COS_FMAX);
    if (!(beta > 0.0)) return fail(COS_ERANGE, "beta must be positive");
    LAUNCH_TRY(launch_g0(nconf, d_n, d_voff, d_sites, d_tau, L, t, beta, nmat, mu, alpha, d_Goff, d_G, d_dG,
                      (hipStream_t)stream));
    return COS_OK;
}

cos_status cos_build_g0_honeycomb(int32_t nconf, const int32_t *d_n, const int64_t *d_voff,
                                  const int32_t *d_cells, const double *d_tau, int32_t L, double t, double beta,
                                  int32_t nmat, const double *mu, const double *alpha, const double *delta,
                                  const int64_t *d_Goff, double *d_G, double *d_dG, void *stream) {
    if (nconf < 1) return fail(COS_EINVAL, "nconf must be >= 1");
    if (!d_n || !d_voff || !d_cells || !d_tau || !d_Goff || !d_G || !mu || !alpha || !delta)
        return fail(COS_EINVAL, "null pointer argument");
    if (L < 1 || L > 32) return fail(COS_ERANGE, "L must be in [1, 32], got %d", L);
    if (nmat < 1 || nmat > COS_FMAX) return fail(COS_ERANGE, "nmat must be in [1, %d]", COS_FMAX);
    if (!(beta > 0.0)) return fail(COS_ERANGE, "beta must be positive");
    LAUNCH_TRY(launch_g0_honeycomb(nconf, d_n, d_voff, d_cells, d_tau, L, t, beta, nmat, mu, alpha, delta, d_Goff,
                                d_G, d_dG, (hipStream_t)stream));
    return COS_OK;
}

cos_status cos_chain_mu_shift(int32_t nconf, const int32_t *d_n, int32_t nmat, const int64_t *d_Goff,
                              const double *d_G_bar, const double *d_dG, const double *d_stub_bar,
                              int32_t nstub, double U, double *d_mu_bar, double *d_alpha_bar, void *stream) {
    if (nconf < 1) return fail(COS_EINVAL, "nconf must be >= 1");
    if (!d_n || !d_Goff || !d_G_bar || !d_dG || !d_mu_bar || !d_alpha_bar)
        return fail(COS_EINVAL, "null pointer argument");
    if (nmat < 1 || nmat > COS_FMAX) return fail(COS_ERANGE, "nmat must be in [1, %d]", COS_FMAX);
    if (d_stub_bar && nstub != 1 && nstub != nmat) return fail(COS_EINVAL, "nstub must be 1 or nmat");
    if (d_stub_bar && U == 0.0) return fail(COS_EINVAL, "U must be nonzero");
    LAUNCH_TRY(launch_chain(nconf, d_n, nmat, d_Goff, d_G_bar, d_dG, d_stub_bar, nstub, U, d_mu_bar, d_alpha_bar,
                         (hipStream_t)stream));
    return COS_OK;
}

cos_status cos_mc_sample(int32_t nconf, int32_t n, int32_t L, double beta, uint64_t seed, int64_t first,
                         int32_t *d_sites, double *d_tau, void *stream) {
    if (nconf < 1 || !d_sites || !d_tau) return fail(COS_EINVAL, "nconf >= 1 and output buffers are required");
    if (n < 1 || n > COS_NMAX) return fail(COS_ERANGE, "n must be in [1, %d], got %d", COS_NMAX, n);
    if (L < 1 || L > 32) return fail(COS_ERANGE, "L must be in [1, 32], got %d", L);
    if (!(beta > 0.0)) return fail(COS_ERANGE, "beta must be positive");
    if (first < 0) return fail(COS_EINVAL, "first must be >= 0");
    LAUNCH_TRY(launch_mc_sample(nconf, n, L, beta, seed, first, d_sites, d_tau, (hipStream_t)stream));
    return COS_OK;
}

cos_status cos_cdet_workspace(int32_t n, int32_t nconf, int32_t precision, uint64_t *bytes) {
    if (!bytes) return fail(COS_EINVAL, "bytes is NULL");
    if (n < 1 || n > COS_NMAX_SUBLATTICE) return fail(COS_ERANGE, "n must be in [1, %d], got %d", COS_NMAX_SUBLATTICE, n);
    if (nconf < 1) return fail(COS_EINVAL, "nconf must be >= 1");
    if (precision != 0 && precision != 1) return fail(COS_EINVAL, "precision must be 0 (FP64) or 1 (double-double)");
    *bytes = (uint64_t)cdet_elems_per_config(n) * (uint64_t)nconf * (precision ? 16u : 8u);
    return COS_OK;
}

cos_status cos_cdet_su2(int32_t nconf, int32_t n, const double *d_A, int32_t precision, double eps, void *d_work,
                        uint64_t work_bytes, double *d_out, void *stream) {
    uint64_t need = 0;
    cos_status st = cos_cdet_workspace(n, nconf, precision, &need);
    if (st) return st;
    if (!d_A || !d_work || !d_out) return fail(COS_EINVAL, "null pointer argument");
    if (work_bytes < need) return fail(COS_EINVAL, "workspace too small: %llu bytes, need %llu",
                                       (unsigned long long)work_bytes, (unsigned long long)need);
    if (!(eps >= 0.0)) return fail(COS_EINVAL, "eps must be >= 0");
    LAUNCH_TRY(launch_cdet(nconf, n, d_A, precision, eps, d_work, d_out, (hipStream_t)stream));
    return COS_OK;
}

cos_status cos_accumulate_moments(int32_t count, const double *d_x, double *d_acc, void *stream) {
    if (count < 1 || !d_x || !d_acc) return fail(COS_EINVAL, "count >= 1 and device buffers are required");
    LAUNCH_TRY(launch_moments(count, d_x, d_acc, (hipStream_t)stream));
    return COS_OK;
}

}  // extern "C"

namespace {

// value of the [m/k] Pade approximant of sum_i a_i x^i at x (T = double, or
// complex for the complex-step derivative); false when the denominator system
// is singular
template <class T>
bool pade_eval(int m, int k, const T *a, double x, T *value) {
    // denominator q_0 = 1, q_1..q_k: sum_{j=0..k} q_j a_{i-j} = 0 for i = m+1..m+k
    std::vector<T> A((size_t)k * k), rhs(k), q(k + 1);
    for (int r = 0; r < k; ++r) {
        const int i = m + 1 + r;
        for (int j = 1; j <= k; ++j) A[(size_t)r * k + (j - 1)] = (i - j >= 0) ? a[i - j] : T(0.0);
        rhs[r] = -a[i];
    }
    // Gaussian elimination with partial pivoting
    for (int c = 0; c < k; ++c) {
        int piv = c;
        for (int r = c + 1; r < k; ++r)
            if (std::abs(A[(size_t)r * k + c]) > std::abs(A[(size_t)piv * k + c])) piv = r;
        if (std::abs(A[(size_t)piv * k + c]) == 0.0) return false;
        if (piv != c) {
            for (int j = 0; j < k; ++j) std::swap(A[(size_t)c * k + j], A[(size_t)piv * k + j]);
            std::swap(rhs[c], rhs[piv]);
        }
        for (int r = c + 1; r < k; ++r) {
            const T f = A[(size_t)r * k + c] / A[(size_t)c * k + c];
            for (int j = c; j < k; ++j) A[(size_t)r * k + j] -= f * A[(size_t)c * k + j];
            rhs[r] -= f * rhs[c];
        }
    }
    q[0] = T(1.0);
    for (int c = k - 1; c >= 0; --c) {
        T v = rhs[c];
        for (int j = c + 1; j < k; ++j) v -= A[(size_t)c * k + j] * q[j + 1];
        q[c + 1] = v / A[(size_t)c * k + c];
    }
    // numerator p_i = sum_{j<=min(i,k)} q_j a_{i-j}; Horner in x
    T P(0.0), Q(0.0);
    for (int i = m; i >= 0; --i) {
        T pi(0.0);
        for (int j = 0; j <= std::min(i, k); ++j) pi += q[j] * a[i - j];
        P = P * x + pi;
    }
    for (int j = k; j >= 0; --j) Q = Q * x + q[j];
    if (std::abs(Q) == 0.0) return false;
    *value = P / Q;
    return true;
}

}  // namespace

extern "C" {

cos_status cos_pade(int32_t m, int32_t k, const double *a, double x, double *value, double *grad) {
    if (!a || !value) return fail(COS_EINVAL, "a and value are required");
    if (m < 0 || k < 0 || m + k > 64) return fail(COS_ERANGE, "need 0 <= m, k and m + k <= 64");
    const int na = m + k + 1;
    double v = 0.0;
    if (!pade_eval<double>(m, k, a, x, &v)) return fail(COS_ERANGE, "the [%d/%d] approximant does not exist", m, k);
    *value = v;
    if (grad) {
        // complex-step derivative: d value / d a_j = Im value(a + i h e_j) / h, exact to rounding
        const double h = 1e-30;
        std::vector<std::complex<double>> ac(a, a + na);
        for (int j = 0; j < na; ++j) {
            ac[j] += std::complex<double>(0.0, h);
            std::complex<double> vc;
            if (!pade_eval<std::complex<double>>(m, k, ac.data(), x, &vc))
                return fail(COS_ERANGE, "the [%d/%d] approximant does not exist", m, k);
            grad[j] = vc.imag() / h;
            ac[j] = a[j];
        }
    }
    return COS_OK;
}

cos_status cos_batch_set_adjoint_segments(cos_batch_t b, int32_t segments) {
    if (!b) return fail(COS_EINVAL, "batch handle is NULL");
    if (segments < 0 || segments > 2) return fail(COS_EINVAL, "segments must be 0, 1 or 2, got %d", segments);
    if (cos_status st = check_batch_device(b)) return st;
    b->adj_segments = segments;
    // the reverse-sweep workspace is planned again at the next reverse call
    if (b->d_Fall) {
        HIP_TRY(hipDeviceSynchronize());
        (void)hipFree(b->d_Fall);
        (void)hipFree(b->d_GbT);
        (void)hipFree(b->d_sbT);
        (void)hipFree(b->d_Gpart);
        (void)hipFree(b->d_Spart);
        b->d_Fall = b->d_GbT = b->d_sbT = b->d_Gpart = b->d_Spart = nullptr;
    }
    return COS_OK;
}

cos_status cos_batch_adjoint_plan(cos_batch_t b, int32_t n, int32_t *split_level, int32_t *groups_per_chunk,
                                  int64_t *bytes_per_group) {
    if (!b) return fail(COS_EINVAL, "batch handle is NULL");
    if (!b->d_Fall) return fail(COS_EINVAL, "no reverse call has planned the reverse-sweep workspace yet");
    for (const OrderGroup &o : b->orders)
        if (o.n == n) {
            if (split_level) *split_level = o.adj_split;
            if (groups_per_chunk) *groups_per_chunk = o.chunk_adj;
            if (bytes_per_group)
                *bytes_per_group = 8 * (adj_store_rows(*o.hp, o.n, o.adj_split) + 2 * (int64_t)o.hp->max_rows) *
                                   b->nfs * o.slots() * 64;
            return COS_OK;
        }
    return fail(COS_EINVAL, "the batch has no configuration of order %d", n);
}

cos_status cos_inject_failures(int32_t kind, int32_t skip, int32_t count) {
    if (kind != 0 && kind != 1) return fail(COS_EINVAL, "kind must be 0 (device allocation) or 1 (kernel launch)");
    if (skip < 0 || count < 0) return fail(COS_EINVAL, "skip and count must be >= 0");
    g_inj_skip[kind].store(skip);
    g_inj_count[kind].store(count);
    return COS_OK;
}

cos_status cos_set_workspace_limit(int64_t bytes) {
    if (bytes < 0) return fail(COS_EINVAL, "bytes must be >= 0, got %lld", (long long)bytes);
    g_ws_limit.store(bytes);
    return COS_OK;
}

cos_status cos_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_live > 0)
        return fail(COS_EINVAL, "%lld batch handle(s) still alive: destroy them before releasing the state tables",
                    (long long)g_live);
    for (auto &kv : g_dev) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(std::get<0>(kv.first));
        (void)hipFree(kv.second.mem);
        (void)hipSetDevice(cur);
    }
    g_dev.clear();
    g_host.clear();
    return COS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Forward sums on workspace the caller places (the allocation-free entry
// point in cos_static.hip builds on these).
// ---------------------------------------------------------------------------
cos_status libcos::report(cos_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

cos_status libcos::current_device(int *dev, int *ncu) { return check_device(dev, ncu); }

cos_status libcos::plan_tables(int n, PlanTables *out) {
    if (n < 1 || n > COS_NMAX) return fail(COS_ERANGE, "n must be in [1, %d], got %d", COS_NMAX, n);
    std::shared_ptr<HostPlan> p;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        p = host_plan(n);
    }
    // the plan stays in the process-wide cache, which only cos_release clears
    out->mrec = p->mrec.data();
    out->mrec_ints = p->mrec.size();
    out->levels = p->levels.data();
    out->nlevels = p->levels.size();
    out->max_rows = p->max_rows;
    out->max_masks = p->max_masks;
    out->total_rows = (int64_t)p->rows.size();
    return COS_OK;
}

FixedSizes libcos::fixed_sizes(int nconf, int n, int nfs, int32_t max_rows) {
    const int64_t ngroups = (nconf + 63) / 64;
    FixedSizes z;
    z.order_ints = nconf;
    z.gt_doubles = ngroups * nfs * n * n * 64;
    z.sig_doubles = ngroups * nfs * 64;
    z.lane_ints = ngroups * 64;
    z.win_doubles_per_group = 2 * (int64_t)max_rows * nfs * n * 64;
    return z;
}

cos_status libcos::forward_fixed(int dev, int ncu, const FixedWorkspace &ws, int32_t nconf, int32_t n,
                                 int32_t nflav, int32_t variant, int32_t flags, const double *d_G,
                                 const double *d_stub, double cycle_weight, double *d_out, hipStream_t s) {
    // a batch description on the stack: every device pointer is the caller's
    cos_batch_s b;
    b.dev = dev;
    b.ncu = ncu;
    b.nconf = nconf;
    b.nflav = nflav;
    b.variant = variant;
    b.flags = flags;
    b.nfs = b.nmat = b.nstub = variant == COS_FLAVOUR ? nflav : 1;
    b.uniform_n = true;
    b.plans[n] = ws.plan;
    b.d_order = ws.order;
    b.d_GT = ws.GT;
    b.d_sigT = ws.sigT;
    b.d_lane = ws.lane;
    b.d_win = ws.win;
    OrderGroup o;
    o.n = n;
    o.count = nconf;
    o.ngroups = (nconf + 63) / 64;
    o.chunk_fwd = std::max(1, std::min(ws.chunk, o.ngroups));
    {
        std::lock_guard<std::mutex> lk(g_mu);
        o.hp = host_plan(n);
    }
    LAUNCH_TRY(launch_iota(ws.order, nconf, s));
    return forward_order(&b, o, d_G, nullptr, d_stub, cycle_weight, d_out, s);
}
