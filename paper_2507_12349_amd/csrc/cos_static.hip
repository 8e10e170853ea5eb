// The forward entry point that allocates no device memory
// (cos_connected_sum_static in include/libcos.h).
//
// Its workspace is one file-scope device array, `scratch`, of
// COS_STATIC_SCRATCH_BYTES: the state tables of every order up to
// COS_STATIC_NMAX (uploaded once per device) followed by the per-call region
// (schedule, packed propagators and shift weights, lane map, two level
// windows).  Host code never passes the array's name to a kernel or a copy:
// the name is a host-side stand-in.  At the first call on a device the
// array's device address is taken with hipGetSymbolAddress and kept per
// device, and every later use goes through that address.  Each device holds
// its own copy of the array until the process ends; calls on one device share
// it, so calls that overlap on one device race.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "cos_internal.hpp"

namespace libcos {
namespace {

static_assert(COS_STATIC_SCRATCH_BYTES % 256 == 0, "scratch size must be a multiple of 256 bytes");

static __device__ __align__(256) double scratch[COS_STATIC_SCRATCH_BYTES / sizeof(double)];

constexpr int kMaxDevices = 64;

struct StaticDevice {
    bool ready = false;
    int ncu = 0;
    char *base = nullptr;         // device address of `scratch` on this device
    DevPlan plans[COS_STATIC_NMAX + 1]{};
    size_t call_offset = 0;       // first byte of the per-call region
};

std::mutex g_static_mu;
StaticDevice g_static[kMaxDevices];

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// once per device, with that device current: the array's device address and
// the state tables of orders 1..COS_STATIC_NMAX copied into its head
cos_status setup_device(int dev, StaticDevice *sd) {
    int cur = -1, ncu = 0;
    if (cos_status st = current_device(&cur, &ncu)) return st;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return report(COS_EDEVICE, "hipGetSymbolAddress of the static scratch failed on device %d: %s", dev,
                      hipGetErrorString(e));
    char *base = (char *)ptr;
    size_t off = 0;
    for (int n = 1; n <= COS_STATIC_NMAX; ++n) {
        PlanTables t;
        if (cos_status st = plan_tables(n, &t)) return st;
        const size_t mb = t.mrec_ints * sizeof(int32_t), lb = t.nlevels * sizeof(int4);
        if (off + up256(mb) + up256(lb) > (size_t)COS_STATIC_SCRATCH_BYTES)
            return report(COS_ENOMEM, "the state tables do not fit the static scratch");
        e = hipMemcpy(base + off, t.mrec, mb, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(base + off + up256(mb), t.levels, lb, hipMemcpyHostToDevice);
        if (e != hipSuccess)
            return report(COS_EDEVICE, "upload of the state tables into the static scratch failed: %s",
                          hipGetErrorString(e));
        DevPlan &p = sd->plans[n];
        p.mrec = (const int32_t *)(base + off);
        p.levels = (const int4 *)(base + off + up256(mb));
        p.n = n;
        p.max_rows = t.max_rows;
        p.max_masks = t.max_masks;
        p.total_rows = t.total_rows;
        off += up256(mb) + up256(lb);
    }
    sd->base = base;
    sd->ncu = ncu;
    sd->call_offset = off;
    sd->ready = true;
    return COS_OK;
}

}  // namespace
}  // namespace libcos

using namespace libcos;

extern "C" cos_status cos_connected_sum_static(int32_t nconf, int32_t n, int32_t nflav, int32_t variant,
                                               int32_t flags, const double *d_G, const double *d_stub,
                                               double cycle_weight, double *d_out, void *stream) {
    if (nconf < 1) return report(COS_EINVAL, "nconf must be >= 1, got %d", nconf);
    if (variant != COS_UNIFORM && variant != COS_FLAVOUR)
        return report(COS_EINVAL, "variant must be COS_UNIFORM (0) or COS_FLAVOUR (1), got %d", variant);
    if (flags & ~COS_F_STUBS)
        return report(COS_EINVAL, "cos_connected_sum_static takes only COS_F_STUBS, got flags 0x%x", flags);
    if (nflav < 1 || nflav > COS_FMAX) return report(COS_ERANGE, "nflav must be in [1, %d], got %d", COS_FMAX, nflav);
    if (n < 1 || n > COS_STATIC_NMAX)
        return report(COS_ERANGE, "cos_connected_sum_static takes orders 1..%d, got %d", COS_STATIC_NMAX, n);
    if (!d_G || !d_out) return report(COS_EINVAL, "d_G and d_out are required");
    if ((flags & COS_F_STUBS) && !d_stub) return report(COS_EINVAL, "COS_F_STUBS set but d_stub is NULL");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return report(COS_EUNSUPPORTED, "no current HIP device: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return report(COS_EUNSUPPORTED, "device index %d not supported", dev);
    StaticDevice *sd = &g_static[dev];
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (!sd->ready)
            if (cos_status st = setup_device(dev, sd)) return st;
    }
    // carve the per-call region: schedule, packed inputs, lane map, windows
    const int nfs = variant == COS_FLAVOUR ? nflav : 1;
    const FixedSizes z = fixed_sizes(nconf, n, nfs, sd->plans[n].max_rows);
    size_t off = sd->call_offset;
    FixedWorkspace ws;
    ws.plan = sd->plans[n];
    ws.order = (int32_t *)(sd->base + off);
    off += up256((size_t)z.order_ints * 4);
    ws.GT = (double *)(sd->base + off);
    off += up256((size_t)z.gt_doubles * 8);
    ws.sigT = (double *)(sd->base + off);
    off += up256((size_t)z.sig_doubles * 8);
    ws.lane = (int32_t *)(sd->base + off);
    off += up256((size_t)z.lane_ints * 4);
    const size_t per_group = (size_t)z.win_doubles_per_group * 8;
    const size_t room = off < (size_t)COS_STATIC_SCRATCH_BYTES ? (size_t)COS_STATIC_SCRATCH_BYTES - off : 0;
    if (room < per_group)
        return report(COS_ERANGE,
                      "cos_connected_sum_static: %d configurations of order %d with %d flavour slot(s) need %zu "
                      "bytes of workspace, more than the %d-byte static scratch holds",
                      nconf, n, nfs, off + per_group, (int)COS_STATIC_SCRATCH_BYTES);
    ws.win = (double *)(sd->base + off);
    ws.chunk = (int)std::min<size_t>(room / per_group, (size_t)((nconf + 63) / 64));
    return forward_fixed(dev, sd->ncu, ws, nconf, n, nflav, variant, flags, d_G, d_stub, cycle_weight, d_out,
                         (hipStream_t)stream);
}
