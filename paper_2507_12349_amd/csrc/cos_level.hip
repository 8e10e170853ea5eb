// Level-synchronous kernels: one configuration per lane, 64 configurations
// per wavefront.
//
// The state tables (which rows, heads and currents exist at each level) are
// the same for every configuration of an order n, so a wavefront walks them
// with wave-uniform control flow: mask codes, row bases and current sets sit
// in SGPRs, and every DP state access reads or writes 64 consecutive doubles
// (one per lane), a single 512-byte transaction.  Each lane holds its own
// configuration's propagator matrix in VGPRs.  One launch per level (the
// level = number of visited points, the layer of Alg. 1-3); the launches of
// a batch run back to back on one stream (and can be captured in a graph).
//
// Packed layouts (lane fastest):
//   GT   [group][flavour][v][w][64]      propagators
//   sigT [group][flavour][64]            shift weights
//   state buffers [group][row][flavour][v][64]
//
// Forward rules per row (m, u) and flavour l (Results; Alg. 2/3):
//   acc = f . G_l;  extension to w (m_w < 2): child (m + e_w, u)[w] = c_w acc[w]
//   (c_w = 2 on a first visit); shift head on the partner of a vertex just
//   reached for the first time: + (-sigma_l) f[w] (doubled on the start row);
//   close: t_m = W sum_{u,l} acc[u]; the next cycle opens at
//   h = min{k : m_k = 1} with value t_m in every flavour, or S = t_m at the
//   full mask.
//
// Mask-only rules (SU(2), w = -1; Results, the variant without cycle factors;
// Alg. 1): the states are (head point, current point, mask) with points, not
// vertices.  They fill the same rows with the two spin blocks as the two
// planes: row (m, 0) holds the head on the up point of vertex 0 (plane 0)
// while m_0 = 1, and on its down point (plane 1) once m_0 = 2; rows (m, h),
// h >= 1, hold both.  The other plane of a row (m, 0) stays empty and is
// skipped.  A point is reached with weight 1 (no factor 2), never onto the
// head point; after the first cycle the next one can open only on the down
// point of vertex 0 (the head is not repeated), later cycles on either end.
#include "cos_device.hpp"

namespace libcos {

// one mask of a level: its code bits, row base and child row bases
template <int N>
struct MaskRec {
    int code, rb;
    uint32_t ones, twos;
    int crb[N];   // level-relative row of (m + e_w, 0); valid where m_w < 2
};

template <int N>
__device__ __forceinline__ MaskRec<N> load_rec(const DevPlan &P, int gi) {
    const cint32 *r = (const cint32 *)(P.mrec + (int64_t)gi * kRecInts);
    MaskRec<N> m;
    m.code = r[0];
    const uint32_t info = (uint32_t)r[1];
    m.ones = info & 0xffffu;
    m.twos = info >> 16;
    m.rb = r[2];
#pragma unroll
    for (int w = 0; w < N; ++w) m.crb[w] = r[3 + w];
    return m;
}

// child row base for the vertex h that opens the next cycle (h is wave-uniform;
// a select chain keeps the record in scalar registers)
template <int N>
__device__ __forceinline__ int close_row_base(const MaskRec<N> &M, int h) {
    int rb = 0;
#pragma unroll
    for (int w = 0; w < N; ++w) rb = (w == h) ? M.crb[w] : rb;
    return rb;
}

// ---------------------------------------------------------------------------
// packing: caller layout -> per-lane layout (zeros in padding lanes)
// ---------------------------------------------------------------------------
__global__ void pack_kernel(const PackArgs A) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int N = A.n, nfs = A.nfs;
    const int64_t per_group = (int64_t)nfs * N * N * 64;
    if (i >= per_group * A.ngroups) return;
    const int lane = (int)(i & 63);
    int64_t rest = i >> 6;
    const int w = (int)(rest % N); rest /= N;
    const int v = (int)(rest % N); rest /= N;
    const int l = (int)(rest % nfs); rest /= nfs;
    const int g = (int)rest;
    const int slot = g * 64 + lane;
    const int c = slot < A.count ? A.order[slot] : -1;
    double x = 0.0;
    if (c >= 0) {
        const int64_t off = A.Goff ? A.Goff[c] : (int64_t)c * A.nmat * N * N;
        x = A.G[off + ((int64_t)(A.variant ? l : 0) * N + v) * N + w];
    }
    A.GT[i] = x;
    if (v == 0 && w == 0) {
        const int64_t si = ((int64_t)g * nfs + l) * 64 + lane;
        if (A.sigT) A.sigT[si] = (c >= 0 && A.stub) ? A.stub[(int64_t)c * A.nstub + (A.variant ? l : 0)] : 0.0;
        if (l == 0) A.lane_cfg[slot] = c;
    }
}

// ---------------------------------------------------------------------------
// forward: level -> level + 1
//
// A workgroup of WPB wavefronts serves one group of 64 configurations and
// WPB consecutive blocks of `mpb` masks.  G_l of the 64 lanes sits in LDS
// ([v][w][lane], conflict-free: the lanes read consecutive words), loaded
// once per flavour by the whole workgroup.  With one flavour the close sums
// stay in registers; with several, the flavour loop is outermost and the
// per-mask sums wait in LDS until every flavour is done.
// ---------------------------------------------------------------------------
template <int N, bool MASK>
__device__ __forceinline__ void fwd_row(const MaskRec<N> &M, uint32_t gaddr, const double *__restrict__ cur,
                                        double *__restrict__ nxt, uint32_t lane8, int64_t cpl, int64_t npl, int lam,
                                        int u, int r, bool start, double sgx, double &cp, double &dext) {
    const uint32_t ones = M.ones, twos = M.twos;
    const uint32_t cm = current_set(u, ones, twos);
    const double *__restrict__ src = cur + lam * cpl + (int64_t)r * N * 64;
    // G comes from LDS for every row: an opaque base keeps the N^2 reads inside
    // the row instead of hoisted into N^2 registers for the whole loop
    asm volatile("" : "+v"(gaddr));
    const lds_double *Gs = (const lds_double *)(uintptr_t)gaddr;
    // only current slots are loaded; the product f . G is formed output by
    // output, and only for the outputs the row uses (open vertices and the
    // head's close): each is consumed at once, no array crosses a branch
    double f[N];
#pragma unroll
    for (int v = 0; v < N; ++v) {
        const bool c = (cm >> v) & 1u;
        f[v] = c ? lane_ld_nt(src + v * 64, lane8) : 0.0;
    }
    if (start) {
#pragma unroll
        for (int v = 0; v < N; ++v) f[v] = v == 0 ? 1.0 : 0.0;   // mask-only: plane 0 only (plane 1 skipped)
    }
#pragma unroll
    for (int w = 0; w < N; ++w) {
        const uint32_t bit = 1u << w;
        if ((twos & bit) && w != u) continue;   // wave-uniform: output not needed
        double a = 0.0;
#pragma unroll
        for (int v = 0; v < N; ++v) a = __builtin_fma(f[v], Gs[(v * N + w) * 64], a);
        if (w == u) cp += a;
        if (twos & bit) continue;
        const bool first = !(ones & bit);
        if (MASK && w == 0 && u == 0) continue;   // the head point itself: not an extension
        double val = first ? (MASK ? a : 2.0 * a) : a;
        if (!first && (cm & bit)) val = __builtin_fma(-sgx, f[w], val);
        if (w == 0 && u == 0 && !(twos & 1u)) {
            dext = val;   // m_0 = 1: the next cycle opens on this same slot
            continue;
        }
        const uint32_t ctw = first ? twos : (twos | bit);
        const int crow = M.crb[w] + head_slot(u, ctw);
        lane_st_nt(nxt + lam * npl + (int64_t)crow * N * 64 + w * 64, lane8, val);
    }
}

template <int N>
__device__ __forceinline__ void fwd_close(const MaskRec<N> &M, double *__restrict__ nxt, uint32_t lane8,
                                          int64_t npl, int lam, double t, double dext) {
    const int h = __builtin_ctz(M.ones);
    const int crow = close_row_base<N>(M, h) + head_slot(h, M.twos | (1u << h));
    lane_st(nxt + lam * npl + (int64_t)crow * N * 64 + h * 64, lane8, t + (h == 0 ? dext : 0.0));
}

// with several flavours (kMultiMasks masks per wavefront at most) the close
// sums of the wave's masks stay in registers across the flavour loop
// mask-only: the plane of row (m, 0) that holds no head point
__device__ __forceinline__ bool empty_plane(int u, int lam, uint32_t twos) {
    return u == 0 && ((lam == 0) == ((twos & 1u) != 0u));
}

template <int N, bool MULTI, bool MASK>
__global__ void __launch_bounds__(1024) level_fwd_kernel(const LvlArgs A) {
    extern __shared__ double lds[];
    double *Gs_all = lds;                      // [N * N][64]
    const int lane = threadIdx.x & 63, wave = COS_RF(threadIdx.x >> 6);   // wave index: uniform
    const int wpb = blockDim.x >> 6;
    const DevPlan &P = A.plan;
    const int4 L = load_level(P, A.level);
    const int mb0 = (blockIdx.x * wpb + wave) * A.mpb;
    const int mb1 = min(mb0 + A.mpb, L.w);     // may be empty: the wave still joins the barriers
    const int gl = blockIdx.y, g = A.group0 + gl;
    const int nfs = A.nfs;
    // wave-uniform bases; the lane's word is added at each access.  States are
    // stored by flavour plane: [flavour][row][v][lane], planes of *_frows rows
    const double *__restrict__ cur = A.cur + gl * A.cur_gstride + (int64_t)A.cur_row0 * N * 64;
    double *__restrict__ nxt = A.nxt + gl * A.nxt_gstride + (int64_t)A.nxt_row0 * N * 64;
    const int64_t cpl = A.cur_frows * N * 64, npl = A.nxt_frows * N * 64;
    const uint32_t lane8 = (uint32_t)lane * 8u;
    const uint32_t gaddr = lds_addr(Gs_all) + lane * 8u;
    const int cfg = A.lane_cfg[g * 64 + lane];
    const bool last = A.level == 2 * N, start = A.level == 1;
    constexpr int K = MULTI ? kMultiMasks : 1;
    double cpk[K];   // MULTI: close sum of each of the wave's masks, over heads and flavours
#pragma unroll
    for (int k = 0; k < K; ++k) cpk[k] = 0.0;

    for (int lam = 0; lam < nfs; ++lam) {
        __syncthreads();
        const double *__restrict__ gsrc = A.GT + (int64_t)(g * nfs + lam) * N * N * 64;
        for (int i = threadIdx.x; i < N * N * 64; i += blockDim.x) Gs_all[i] = gsrc[i];
        __syncthreads();
        const double sg = A.stubs ? A.sigT[(int64_t)(g * nfs + lam) * 64 + lane] : 0.0;
        // MULTI: at most K masks, unrolled so that cpk stays in registers
        const int mend = MULTI ? min(mb1, mb0 + K) : mb1;
#pragma unroll
        for (int k = 0; k < (MULTI ? K : 1); ++k) {
            for (int mi = mb0 + k; mi < mend; mi += (MULTI ? K : 1)) {
                const MaskRec<N> M = load_rec<N>(P, L.z + mi);
                const uint32_t ones = M.ones, twos = M.twos;
                const double sgx = sg * (M.code == 1 ? 2.0 : 1.0);
                uint32_t hs = (twos & 1u) ? (twos & ~1u) : 0u;   // heads >= 1, ascending
                int u = 0, slot = 0;
                double cp = 0.0, dext = 0.0;
                while (true) {
                    if (!(MASK && empty_plane(u, lam, twos)))
                        fwd_row<N, MASK>(M, gaddr, cur, nxt, lane8, cpl, npl, lam, u, M.rb + slot, start, sgx, cp,
                                         dext);
                    if (!hs) break;
                    u = __builtin_ctz(hs);
                    hs &= hs - 1u;
                    ++slot;
                }
                if (MULTI) {
                    cpk[k] += cp;
                    // m_0 = 1 (so h = 0): this flavour's extension into the slot
                    // the next cycle opens on; the close adds to it at the end
                    if (!MASK && !last && (ones & 1u)) fwd_close<N>(M, nxt, lane8, npl, lam, 0.0, dext);
                } else {
                    const double t = A.W * cp;
                    if (last) {
                        if (cfg >= 0 && A.out) A.out[cfg] = t;
                    } else if (ones) {
                        fwd_close<N>(M, nxt, lane8, npl, 0, t, dext);
                    }
                }
            }
        }
    }
    if (MULTI) {
        // t_m = W sum over heads and flavours; the next cycle opens in every flavour
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int mi = mb0 + k;
            if (mi >= mb1) continue;
            const MaskRec<N> M = load_rec<N>(P, L.z + mi);
            const double t = A.W * cpk[k];
            if (last) {
                if (cfg >= 0 && A.out) A.out[cfg] = t;
            } else if (M.ones) {
                const int h = __builtin_ctz(M.ones);
                const int crow = close_row_base<N>(M, h) + head_slot(h, M.twos | (1u << h));
                double *dst = nxt + (int64_t)crow * N * 64 + h * 64;
                if (MASK) {
                    // the first cycle's successor opens on the down point of
                    // vertex 0 only; later ones on both ends of vertex h
                    for (int lam = (h == 0 ? 1 : 0); lam < nfs; ++lam) lane_st(dst + lam * npl, lane8, t);
                } else {
                    for (int lam = 0; lam < nfs; ++lam) {
                        // h = 0: the slot holds this wave's own extension value (written above)
                        const double x = h == 0 ? lane_ld(dst + lam * npl, lane8) : 0.0;
                        lane_st(dst + lam * npl, lane8, t + x);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// reverse: B = dS/dF at level `level` from B at level + 1.
//   a[w] = c_w B(m + e_w, u)[w] (open w) + [w == u] W tbar_m,
//   tbar_m = sum_l B(m + e_h, h, l)[h] (1 at the full mask, 0 when dropped),
//   B(m, u)[v] = sum_w G[v][w] a[w] + [m_v = 1, v current] (-sigma) a'[v]
//   (a' = a without the close term), Gbar[v][w] += f[v] a[w],
//   sigmabar += -f[w] B(m + e_w, u)[w] on the shift edges.
//
// Every wavefront owns whole rows.  The dS/dG accumulator of the 64
// configurations of the workgroup lives in LDS next to G ([v][w][lane], the
// lanes add to consecutive words) and is added to the packed gradient once per
// workgroup and flavour; only the (v, w) pairs a row can touch (v current,
// w open or the head) are accumulated.
// ---------------------------------------------------------------------------
template <int N, bool MASK>
__device__ __forceinline__ void adj_row(const MaskRec<N> &M, uint32_t gaddr, uint32_t gbaddr,
                                        const double *__restrict__ F, const double *__restrict__ Bn,
                                        double *__restrict__ Bc, uint32_t lane8, int64_t fpl, int64_t cpl,
                                        int64_t npl, int lam, int u, int r, bool start, double tb, double sgx,
                                        double sc, double &sacc) {
    const uint32_t ones = M.ones, twos = M.twos;
    const uint32_t cm = current_set(u, ones, twos);
    const double *__restrict__ src = F + lam * fpl + (int64_t)r * N * 64;
    // only the current slots' forward states and the open slots' child
    // adjoints are loaded (wave-uniform branches around the loads; the values
    // are consumed after all of them are issued).  Measured against loading
    // every slot with selected addresses: reverse 7.06 -> 6.79 ms (forward
    // states) and 7.06 -> 6.87 ms (child adjoints) on the adjoint workload.
    double f[N], a[N];
#pragma unroll
    for (int v = 0; v < N; ++v) {
        double x = 0.0;
        if (((cm >> v) & 1u) && !start) x = lane_ld_nt(src + v * 64, lane8);
        f[v] = start ? (v == 0 ? 1.0 : 0.0) : x;   // start: (e_0, 0, 0) = 1
    }
#pragma unroll
    for (int w = 0; w < N; ++w) {
        const uint32_t bit = 1u << w;
        const bool open = !(twos & bit), first = !(ones & bit);
        double bc = 0.0;
        if (open) {
            const int crow = M.crb[w] + head_slot(u, first ? twos : (twos | bit));
            bc = lane_ld(Bn + lam * cpl + (int64_t)crow * N * 64 + w * 64, lane8);
        }
        a[w] = open ? (first ? (MASK ? bc : 2.0 * bc) : bc) : 0.0;
        if (MASK && w == 0 && u == 0) a[w] = 0.0;   // no extension onto the head point
        const bool shift = open && !first && (cm & bit);
        sacc = shift ? __builtin_fma(-sc * f[w], bc, sacc) : sacc;
    }
    // the close of this row feeds t_m: dS/dacc[u] gains W tbar
#pragma unroll
    for (int w = 0; w < N; ++w) a[w] = (w == u) ? a[w] + tb : a[w];
    const uint32_t need = (~twos | (1u << u)) & ((1u << N) - 1u);   // w with a[w] != 0 possible
    asm volatile("" : "+v"(gaddr));
    asm volatile("" : "+v"(gbaddr));
    const lds_double *Gs = (const lds_double *)(uintptr_t)gaddr;
    lds_double *Gb = (lds_double *)(uintptr_t)gbaddr;
    double *__restrict__ dst = Bc + lam * npl + (int64_t)r * N * 64;
#pragma unroll
    for (int v = 0; v < N; ++v) {
        const uint32_t bit = 1u << v;
        if (!(cm & bit)) continue;   // wave-uniform
        double b = 0.0;
#pragma unroll
        for (int w = 0; w < N; ++w) b = __builtin_fma(Gs[(v * N + w) * 64], a[w], b);
        if (ones & bit) {
            // shift edge out of this slot: child adjoint, without the close term
            const double bcv = (v == u) ? a[v] - tb : a[v];
            b = __builtin_fma(-sgx, bcv, b);
        }
        lane_st_nt(dst + v * 64, lane8, b);
#pragma unroll
        for (int w = 0; w < N; ++w)
            if (need & (1u << w))   // wave-uniform
                __hip_atomic_fetch_add(Gb + (v * N + w) * 64, f[v] * a[w], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

template <int N, bool MASK>
__global__ void __launch_bounds__(1024) level_adj_kernel(const LvlArgs A) {
    extern __shared__ double lds[];
    double *Gs_all = lds;                     // [N * N][64]  G of the flavour
    double *Gb_all = lds + N * N * 64;        // [N * N][64]  dS/dG of the flavour, this workgroup
    const int lane = threadIdx.x & 63, wave = COS_RF(threadIdx.x >> 6);   // wave index: uniform
    const int wpb = blockDim.x >> 6;
    const DevPlan &P = A.plan;
    const int4 L = load_level(P, A.level);
    // the workgroup's block of masks; its wavefronts claim masks one at a time
    // from an LDS counter, so that a wavefront that drew short rows takes more.
    // On levels of few masks the items are (mask, row) pairs instead, item
    // i = N m + k standing for row k of mask m, so that the rows of a mask run
    // side by side rather than one after another in one wavefront.
    const int nitems = A.row_items ? L.w * N : L.w;
    const int blk0 = blockIdx.x * wpb * A.mpb;
    const int blk1 = min(blk0 + wpb * A.mpb, nitems);   // may hold fewer items than waves: they still join the barriers
    __shared__ int next_mask;
    const int gl = blockIdx.y, g = A.group0 + gl;
    const int nfs = A.nfs;
    // wave-uniform bases; the lane's word is added at each access; flavour planes
    const double *__restrict__ F = A.F + gl * A.F_gstride + (int64_t)A.F_row0 * N * 64;
    const int64_t fpl = A.F_frows * N * 64, cpl = A.cur_frows * N * 64, npl = A.nxt_frows * N * 64;
    const double *__restrict__ Bn = A.cur + gl * A.cur_gstride;   // level + 1
    double *__restrict__ Bc = A.nxt + gl * A.nxt_gstride;         // level
    const uint32_t lane8 = (uint32_t)lane * 8u;
    const int cfg = A.lane_cfg[g * 64 + lane];
    const double obar = cfg >= 0 ? A.out_bar[cfg] : 0.0;
    const uint32_t gaddr = lds_addr(Gs_all) + lane * 8u, gbaddr = lds_addr(Gb_all) + lane * 8u;
    const bool top = A.level == 2 * N, start = A.level == 1;

    for (int lam = 0; lam < nfs; ++lam) {
        __syncthreads();   // the previous flavour's accumulator has been flushed
        const double *__restrict__ gsrc = A.GT + (int64_t)(g * nfs + lam) * N * N * 64;
        for (int i = threadIdx.x; i < N * N * 64; i += blockDim.x) {
            Gs_all[i] = gsrc[i];
            Gb_all[i] = 0.0;
        }
        if (threadIdx.x == 0) next_mask = blk0 + wpb;   // masks blk0 .. blk0 + wpb - 1 go to the waves in order
        __syncthreads();
        const double sg = A.stubs ? A.sigT[(int64_t)(g * nfs + lam) * 64 + lane] : 0.0;
        double sacc = 0.0;
        bool any = false;
        for (int it = blk0 + wave; it < blk1;) {
            any = true;
            const int mi = A.row_items ? it / N : it;
            const MaskRec<N> M = load_rec<N>(P, L.z + mi);
            const uint32_t ones = M.ones, twos = M.twos;
            uint32_t hs = (twos & 1u) ? (twos & ~1u) : 0u;   // heads >= 1, ascending
            int u = 0, slot = 0;
            bool go = true;
            if (A.row_items) {
                // this item's row alone: slot k = 0 (head 0) or the k-th head >= 1
                const int k = it - mi * N;
                for (int j = 1; j < k; ++j) hs &= hs - 1u;
                if (k > 0) {
                    go = hs != 0;   // the mask has fewer rows
                    u = go ? __builtin_ctz(hs) : 0;
                    slot = k;
                }
                hs = 0;
            }
            if (go) {
                double tb = 0.0;
                if (top) {
                    tb = obar;
                } else if (ones) {
                    const int h = __builtin_ctz(ones);
                    const int crow = close_row_base<N>(M, h) + head_slot(h, twos | (1u << h));
                    for (int k = (MASK && h == 0 ? 1 : 0); k < nfs; ++k)
                        tb += lane_ld(Bn + k * cpl + (int64_t)crow * N * 64 + h * 64, lane8);
                }
                tb *= A.W;
                const double sc = (M.code == 1 ? 2.0 : 1.0);
                while (true) {
                    if (!(MASK && empty_plane(u, lam, twos)))
                        adj_row<N, MASK>(M, gaddr, gbaddr, F, Bn, Bc, lane8, fpl, cpl, npl, lam, u, M.rb + slot, start,
                                         tb, sg * sc, sc, sacc);
                    if (!hs) break;
                    u = __builtin_ctz(hs);
                    hs &= hs - 1u;
                    ++slot;
                }
            }
            int nx = 0;
            if (lane == 0) nx = atomicAdd(&next_mask, 1);
            it = COS_RF(nx);   // lane 0's claim (every lane is active here)
        }
        if (A.stubs && any) atomicAdd(A.sbar_T + (int64_t)(g * nfs + lam) * 64 + lane, sacc);
        __syncthreads();
        double *__restrict__ gb = A.Gbar_T + (int64_t)(g * nfs + lam) * N * N * 64;
        for (int i = threadIdx.x; i < N * N * 64; i += blockDim.x) {
            const double x = Gb_all[i];
            if (x != 0.0) atomicAdd(gb + i, x);
        }
    }
}

// ---------------------------------------------------------------------------
// reverse, deterministic: the same rules as level_adj_kernel, with an order of
// summation that depends on nothing but the order n.  A level's masks are cut
// into kDetParts fixed parts; a workgroup of N wavefronts takes one part of
// one group, wavefront v owns slot v: it forms B(m, u)[v], keeps row v of G
// and the partial sums dS/dG[v][*] (and its shift term) in registers over the
// part's rows in order, and adds them to the part's own slot of a partial
// buffer (no atomics: one wavefront per slot and level, the levels follow one
// another on the stream).  det_reduce_kernel then sums the parts in order.
// The child adjoints of a row are read by each of its current wavefronts;
// those reads hit the caches after the first.
// ---------------------------------------------------------------------------
template <int N, bool MASK>
__global__ void __launch_bounds__(64 * COS_NMAX) level_adj_det_kernel(const LvlArgs A) {
    const int lane = threadIdx.x & 63, v = COS_RF(threadIdx.x >> 6);   // the wave's slot: uniform
    const DevPlan &P = A.plan;
    const int4 L = load_level(P, A.level);
    const int part = blockIdx.x;
    const int lo = (int)(((int64_t)part * L.w) / kDetParts), hi = (int)(((int64_t)(part + 1) * L.w) / kDetParts);
    const int gl = blockIdx.y, g = A.group0 + gl;
    const int nfs = A.nfs;
    const double *__restrict__ F = A.F + gl * A.F_gstride + (int64_t)A.F_row0 * N * 64;
    const int64_t fpl = A.F_frows * N * 64, cpl = A.cur_frows * N * 64, npl = A.nxt_frows * N * 64;
    const double *__restrict__ Bn = A.cur + gl * A.cur_gstride;   // level + 1
    double *__restrict__ Bc = A.nxt + gl * A.nxt_gstride;         // level
    const uint32_t lane8 = (uint32_t)lane * 8u, vbit = 1u << v;
    const int cfg = A.lane_cfg[g * 64 + lane];
    const double obar = cfg >= 0 ? A.out_bar[cfg] : 0.0;
    const bool top = A.level == 2 * N, start = A.level == 1;
    if (lo >= hi) return;

    for (int lam = 0; lam < nfs; ++lam) {
        const double *__restrict__ grow = A.GT + ((int64_t)(g * nfs + lam) * N + v) * N * 64;
        double gv[N], gb[N];
#pragma unroll
        for (int w = 0; w < N; ++w) {
            gv[w] = lane_ld(grow + w * 64, lane8);
            gb[w] = 0.0;
        }
        const double sg = A.stubs ? A.sigT[(int64_t)(g * nfs + lam) * 64 + lane] : 0.0;
        double sacc = 0.0;
        for (int mi = lo; mi < hi; ++mi) {
            const MaskRec<N> M = load_rec<N>(P, L.z + mi);
            const uint32_t ones = M.ones, twos = M.twos;
            double tb = 0.0;
            if (top) {
                tb = obar;
            } else if (ones) {
                const int h = __builtin_ctz(ones);
                const int crow = close_row_base<N>(M, h) + head_slot(h, twos | (1u << h));
                for (int k = (MASK && h == 0 ? 1 : 0); k < nfs; ++k)
                    tb += lane_ld(Bn + k * cpl + (int64_t)crow * N * 64 + h * 64, lane8);
            }
            tb *= A.W;
            const double sc = (M.code == 1 ? 2.0 : 1.0);
            uint32_t hs = (twos & 1u) ? (twos & ~1u) : 0u;   // heads >= 1, ascending
            int u = 0, slot = 0;
            while (true) {
                const uint32_t cm = current_set(u, ones, twos);
                if ((cm & vbit) && !(MASK && empty_plane(u, lam, twos))) {
                    const int r = M.rb + slot;
                    const double fv = start ? (v == 0 ? 1.0 : 0.0)
                                            : lane_ld_nt(F + lam * fpl + (int64_t)r * N * 64 + v * 64, lane8);
                    double a[N];
                    double bcv = 0.0;
#pragma unroll
                    for (int w = 0; w < N; ++w) {
                        const uint32_t bit = 1u << w;
                        const bool open = !(twos & bit), first = !(ones & bit);
                        double bc = 0.0;
                        if (open) {   // wave-uniform: the open slots' child adjoints only
                            const int crow = M.crb[w] + head_slot(u, first ? twos : (twos | bit));
                            bc = lane_ld(Bn + lam * cpl + (int64_t)crow * N * 64 + w * 64, lane8);
                        }
                        a[w] = open ? (first ? (MASK ? bc : 2.0 * bc) : bc) : 0.0;
                        if (MASK && w == 0 && u == 0) a[w] = 0.0;   // no extension onto the head point
                        if (w == v) bcv = bc;
                    }
                    // the shift edge out of slot v (child adjoint without the close term)
                    const bool vopen = !(twos & vbit), vfirst = !(ones & vbit);
                    if (vopen && !vfirst) sacc = __builtin_fma(-sc * fv, bcv, sacc);
#pragma unroll
                    for (int w = 0; w < N; ++w) a[w] = (w == u) ? a[w] + tb : a[w];
                    const uint32_t need = (~twos | (1u << u)) & ((1u << N) - 1u);
                    double b = 0.0;
#pragma unroll
                    for (int w = 0; w < N; ++w) b = __builtin_fma(gv[w], a[w], b);
                    if (ones & vbit) b = __builtin_fma(-sg * sc, (v == u) ? a[v] - tb : a[v], b);
                    lane_st_nt(Bc + lam * npl + (int64_t)r * N * 64 + v * 64, lane8, b);
#pragma unroll
                    for (int w = 0; w < N; ++w)
                        if (need & (1u << w)) gb[w] = __builtin_fma(fv, a[w], gb[w]);   // wave-uniform test
                }
                if (!hs) break;
                u = __builtin_ctz(hs);
                hs &= hs - 1u;
                ++slot;
            }
        }
        // this part's slot of the partial sums (one wavefront per slot and level)
        double *gp = A.Gbar_T + (((int64_t)part * A.det_groups + g) * nfs + lam) * N * N * 64 + (int64_t)v * N * 64;
#pragma unroll
        for (int w = 0; w < N; ++w) lane_st(gp + w * 64, lane8, lane_ld(gp + w * 64, lane8) + gb[w]);
        if (A.stubs) {
            double *sp = A.sbar_T + ((((int64_t)part * A.det_groups + g) * nfs + lam) * N + v) * 64;
            lane_st(sp, lane8, lane_ld(sp, lane8) + sacc);
        }
    }
}

// sums the parts in order: GbT[i] = sum_p Gpart[p][i], sbT[g][l] = sum_p sum_v Spart[p][g][l][v]
__global__ void det_reduce_kernel(const double *__restrict__ Gpart, const double *__restrict__ Spart, int64_t gsize,
                                  int64_t ssize, int n, double *__restrict__ GbT, double *__restrict__ sbT) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < gsize) {
        double x = 0.0;
        for (int p = 0; p < kDetParts; ++p) x += Gpart[(int64_t)p * gsize + i];
        GbT[i] = x;
    }
    if (Spart && i < ssize) {   // i = (g * nfs + l) * 64 + lane
        const int64_t gl = i >> 6, lane = i & 63;
        double x = 0.0;
        for (int p = 0; p < kDetParts; ++p)
            for (int v = 0; v < n; ++v) x += Spart[(((int64_t)p * (ssize >> 6) + gl) * n + v) * 64 + lane];
        sbT[i] = x;
    }
}

__global__ void zero_kernel(double *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void iota_kernel(int32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = i;
}

// packed gradients -> caller layout
__global__ void unpack_kernel(const PackArgs A, const double *__restrict__ GbT, const double *__restrict__ sbT,
                              double *__restrict__ Gb, double *__restrict__ sb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int N = A.n, nfs = A.nfs;
    const int64_t per_group = (int64_t)nfs * N * N * 64;
    if (i >= per_group * A.ngroups) return;
    const int lane = (int)(i & 63);
    int64_t rest = i >> 6;
    const int w = (int)(rest % N); rest /= N;
    const int v = (int)(rest % N); rest /= N;
    const int l = (int)(rest % nfs); rest /= nfs;
    const int g = (int)rest;
    const int slot = g * 64 + lane;
    if (slot >= A.count) return;
    const int c = A.order[slot];
    const int64_t off = A.Goff ? A.Goff[c] : (int64_t)c * A.nmat * N * N;
    Gb[off + ((int64_t)(A.variant ? l : 0) * N + v) * N + w] = GbT[i];
    if (v == 0 && w == 0 && sb) sb[(int64_t)c * A.nstub + (A.variant ? l : 0)] = sbT[((int64_t)g * nfs + l) * 64 + lane];
}

hipError_t launch_pack(const PackArgs &a, hipStream_t s) {
    const int64_t tot = (int64_t)a.ngroups * a.nfs * a.n * a.n * 64;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_unpack(const PackArgs &a, const double *GbT, const double *sbT, double *Gb, double *sb,
                         hipStream_t s) {
    const int64_t tot = (int64_t)a.ngroups * a.nfs * a.n * a.n * 64;
    hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a, GbT, sbT, Gb, sb);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t *p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_level_det(const LvlArgs &a, int ngroups, hipStream_t s) {
    const int n = a.plan.n;
    const dim3 grid((unsigned)kDetParts, (unsigned)ngroups);
    switch (n) {
#define COS_DET_CASE(K)                                                                              \
    case K:                                                                                          \
        if (a.mask_only) hipLaunchKernelGGL((level_adj_det_kernel<K, true>), grid, dim3(64 * K), 0, s, a); \
        else hipLaunchKernelGGL((level_adj_det_kernel<K, false>), grid, dim3(64 * K), 0, s, a);         \
        break;
        COS_DET_CASE(1) COS_DET_CASE(2) COS_DET_CASE(3) COS_DET_CASE(4)
        COS_DET_CASE(5) COS_DET_CASE(6) COS_DET_CASE(7) COS_DET_CASE(8)
        COS_DET_CASE(9) COS_DET_CASE(10) COS_DET_CASE(11) COS_DET_CASE(12)
#undef COS_DET_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_det_reduce(const double *Gpart, const double *Spart, int64_t gsize, int64_t ssize, int n,
                             double *GbT, double *sbT, hipStream_t s) {
    const int64_t tot = (Spart && ssize > gsize) ? ssize : gsize;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(det_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Gpart, Spart, gsize,
                       ssize, n, GbT, sbT);
    return hipGetLastError();
}

// the reverse sweep shares one LDS accumulator among the wavefronts of a
// workgroup: large workgroups
int adj_waves_per_block() { return 16; }

// raise a kernel's dynamic-LDS limit when a launch needs more than 64 KB
static hipError_t allow_lds(const void *fn, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_level(const LvlArgs &a, bool reverse, int nblocks, int ngroups, int wpb, hipStream_t s) {
    const int n = a.plan.n;
    if (!reverse && (wpb < 1 || wpb > 16)) return hipErrorInvalidValue;
    if (reverse) {
        const int wpa = adj_waves_per_block();
        if (wpb != wpa) return hipErrorInvalidValue;
        const size_t shm = 2 * (size_t)n * n * 64 * sizeof(double);
        const dim3 grid((unsigned)((nblocks + wpa - 1) / wpa), (unsigned)ngroups);
        switch (n) {
#define COS_ADJ_CASE(K)                                                                           \
    case K: {                                                                                     \
        const void *fn = a.mask_only ? (const void *)level_adj_kernel<K, true>                    \
                                     : (const void *)level_adj_kernel<K, false>;                  \
        hipError_t e = allow_lds(fn, shm);                                                        \
        if (e != hipSuccess) return e;                                                            \
        if (a.mask_only) hipLaunchKernelGGL((level_adj_kernel<K, true>), grid, dim3(64 * wpa), shm, s, a);  \
        else hipLaunchKernelGGL((level_adj_kernel<K, false>), grid, dim3(64 * wpa), shm, s, a);             \
        break;                                                                                    \
    }
            COS_ADJ_CASE(1) COS_ADJ_CASE(2) COS_ADJ_CASE(3) COS_ADJ_CASE(4)
            COS_ADJ_CASE(5) COS_ADJ_CASE(6) COS_ADJ_CASE(7) COS_ADJ_CASE(8)
            COS_ADJ_CASE(9) COS_ADJ_CASE(10) COS_ADJ_CASE(11) COS_ADJ_CASE(12)
#undef COS_ADJ_CASE
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    const bool multi = a.nfs > 1;
    if (multi && a.mpb > kMultiMasks) return hipErrorInvalidValue;
    const size_t shm = (size_t)n * n * 64 * sizeof(double);
    const dim3 grid((unsigned)((nblocks + wpb - 1) / wpb), (unsigned)ngroups);
    switch (n) {
#define COS_FWD_CASE(K)                                                                                    \
    case K: {                                                                                              \
        const void *fn = a.mask_only ? (const void *)level_fwd_kernel<K, true, true>                       \
                         : multi     ? (const void *)level_fwd_kernel<K, true, false>                      \
                                     : (const void *)level_fwd_kernel<K, false, false>;                    \
        hipError_t e = allow_lds(fn, shm);                                                                 \
        if (e != hipSuccess) return e;                                                                     \
        if (a.mask_only) hipLaunchKernelGGL((level_fwd_kernel<K, true, true>), grid, dim3(64 * wpb), shm, s, a); \
        else if (multi) hipLaunchKernelGGL((level_fwd_kernel<K, true, false>), grid, dim3(64 * wpb), shm, s, a); \
        else hipLaunchKernelGGL((level_fwd_kernel<K, false, false>), grid, dim3(64 * wpb), shm, s, a);           \
        break;                                                                                             \
    }
        COS_FWD_CASE(1) COS_FWD_CASE(2) COS_FWD_CASE(3) COS_FWD_CASE(4)
        COS_FWD_CASE(5) COS_FWD_CASE(6) COS_FWD_CASE(7) COS_FWD_CASE(8)
        COS_FWD_CASE(9) COS_FWD_CASE(10) COS_FWD_CASE(11) COS_FWD_CASE(12)
#undef COS_FWD_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace libcos
