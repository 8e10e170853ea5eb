// Sublattice-summed forward levels (bipartite lattices): the connected sum over
// every assignment of a sublattice label to each vertex, in one pass over the
// labelled state space (Results, four-state interaction mask; Alg. 1/2).
//
// Same organisation as the unlabelled level kernels: one configuration per
// lane, wave-uniform control flow from scalar mask records, one launch per
// level.  A row (m, u, s_u) holds 2n slots (v, s_v); the 2n x 2n matrix of the
// current flavour sits in LDS as [2n][2n][lane] ((2n)^2 x 512 B, 128 KB at
// n = 8), shared by the 16 wavefronts of a workgroup.
//
// Rules per row (m, u, s_u), current slots f[(v, s_v)], acc = f . G (formed
// output by output, only for the outputs the row uses):
//   a once-unvisited w is reached on either label: child (m + (w, s)), slot
//   (w, s) = 2 acc[(w, s)] (first visit: either point of w);
//   a once-visited w keeps its label s: child (m with w twice), slot (w, s) =
//   acc[(w, s)];
//   close: t_m = W sum_rows acc[(u, s_u)]; the next cycle opens at the lowest
//   once-visited vertex h with its label s_h (slot (h, s_h) of row (m', h, s_h)),
//   or S = t_m at the full mask.
// Mask-only rules (SU(2), Alg. 1 with its labels): the two planes are the spin
// blocks, as in the unlabelled level kernels: a first visit has weight 1, the
// head point is never reached by an extension, rows (m, 0, s) use plane 0
// while m_0 is once-visited and plane 1 afterwards (the other plane is
// skipped), and the first cycle's successor opens on plane 1 only.
#include "cos_device.hpp"

namespace libcos {

template <int N>
struct SubRec {
    int code, rb;
    uint32_t ones, twos, subb;
    int crb[2 * N];
};

template <int N>
__device__ __forceinline__ SubRec<N> load_sub_rec(const DevPlan &P, int gi) {
    const cint32 *r = (const cint32 *)(P.mrec + (int64_t)gi * kSubRecInts);
    SubRec<N> m;
    m.code = r[0];
    const uint32_t info = (uint32_t)r[1];
    m.ones = info & 0xffffu;
    m.twos = info >> 16;
    m.rb = r[2];
    m.subb = (uint32_t)r[3];
#pragma unroll
    for (int i = 0; i < 2 * N; ++i) m.crb[i] = r[4 + i];
    return m;
}

// child row base for visiting slot i = 2w + s (i wave-uniform; select chain
// keeps the record in scalar registers)
template <int N>
__device__ __forceinline__ int sub_child_base(const SubRec<N> &M, int i) {
    int rb = 0;
#pragma unroll
    for (int k = 0; k < 2 * N; ++k) rb = (k == i) ? M.crb[k] : rb;
    return rb;
}

template <int N, bool MASK>
__device__ __forceinline__ void sub_fwd_row(const SubRec<N> &M, uint32_t gaddr, const double *__restrict__ curL,
                                            double *__restrict__ nxtL, uint32_t lane8, int u, int su, int r,
                                            bool start, double &cp, double &dext) {
    constexpr int D = 2 * N;
    const uint32_t ones = M.ones, twos = M.twos, subb = M.subb;
    const uint32_t cs = sub_current(N, u, su, ones, twos, subb);
    // curL, nxtL: this flavour's planes; row offsets in 32-bit (a level's rows
    // times (2n)^2 x 64 stay far below 2^31)
    const double *__restrict__ src = curL + r * D * 64;
    asm volatile("" : "+v"(gaddr));
    const lds_double *Gs = (const lds_double *)(uintptr_t)gaddr;
    double f[D];
#pragma unroll
    for (int i = 0; i < D; ++i) f[i] = ((cs >> i) & 1u) ? lane_ld_nt(src + i * 64, lane8) : 0.0;
    if (start) {
#pragma unroll
        for (int i = 0; i < D; ++i) f[i] = i == su ? 1.0 : 0.0;   // start: vertex 0 on label s_u
    }
#pragma unroll
    for (int w = 0; w < N; ++w) {
        const uint32_t bit = 1u << w;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int j = 2 * w + s;
            const bool close = (w == u) && (s == su);
            // outputs used: both labels of an unvisited w, the kept label of a
            // once-visited w, and the close slot (wave-uniform tests)
            const bool ext = !(twos & bit) && (!(ones & bit) || (int)((subb >> w) & 1u) == s);
            if (!ext && !close) continue;
            double a = 0.0;
#pragma unroll
            for (int i = 0; i < D; ++i) a = __builtin_fma(f[i], Gs[(i * D + j) * 64], a);
            if (close) cp += a;
            if (!ext) continue;
            if (!(ones & bit)) {
                const int crow = M.crb[j] + sub_head_slot(u, su, twos);
                lane_st_nt(nxtL + (crow * D + j) * 64, lane8, MASK ? a : 2.0 * a);
                continue;
            }
            const double val = a;
            if (w == 0 && u == 0) {
                // vertex 0 once visited: the next cycle opens on this same slot
                // (mask-only: the head point itself, not an extension)
                if (!MASK) dext = val;
                continue;
            }
            const int crow = (s ? M.crb[2 * w + 1] : M.crb[2 * w]) + sub_head_slot(u, su, twos | bit);
            lane_st_nt(nxtL + (crow * D + 2 * w + s) * 64, lane8, val);
        }
    }
}

template <int N>
__device__ __forceinline__ void sub_fwd_close(const SubRec<N> &M, double *__restrict__ nxtL, uint32_t lane8,
                                              double t, double dext) {
    constexpr int D = 2 * N;
    const int h = __builtin_ctz(M.ones);
    const int sh = (M.subb >> h) & 1u;
    const int crow = sub_child_base<N>(M, 2 * h + sh) + sub_head_slot(h, sh, M.twos | (1u << h));
    lane_st(nxtL + (crow * D + 2 * h + sh) * 64, lane8, t + (h == 0 ? dext : 0.0));
}

template <int N, bool MULTI, bool MASK>
__global__ void __launch_bounds__(1024) sub_fwd_kernel(const LvlArgs A) {
    constexpr int D = 2 * N;
    extern __shared__ double lds[];
    double *Gs_all = lds;                      // [D * D][64]
    const int lane = threadIdx.x & 63, wave = COS_RF(threadIdx.x >> 6);   // wave index: uniform
    const int wpb = blockDim.x >> 6;
    const DevPlan &P = A.plan;
    const int4 L = load_level(P, A.level);
    const int mb0 = (blockIdx.x * wpb + wave) * A.mpb;
    const int mb1 = min(mb0 + A.mpb, L.w);     // may be empty: the wave still joins the barriers
    const int gl = blockIdx.y, g = A.group0 + gl;
    const int nfs = A.nfs;
    const double *__restrict__ cur = A.cur + gl * A.cur_gstride + (int64_t)A.cur_row0 * D * 64;
    double *__restrict__ nxt = A.nxt + gl * A.nxt_gstride + (int64_t)A.nxt_row0 * D * 64;
    const int64_t cpl = A.cur_frows * D * 64, npl = A.nxt_frows * D * 64;
    const uint32_t lane8 = (uint32_t)lane * 8u;
    const uint32_t gaddr = lds_addr(Gs_all) + lane * 8u;
    const int cfg = A.lane_cfg[g * 64 + lane];
    const bool last = A.level == 2 * N, start = A.level == 1;
    constexpr int K = MULTI ? kMultiMasks : 1;
    double cpk[K];   // MULTI: close sum of each of the wave's masks, over rows and flavours
#pragma unroll
    for (int k = 0; k < K; ++k) cpk[k] = 0.0;

    for (int lam = 0; lam < nfs; ++lam) {
        __syncthreads();
        const double *__restrict__ gsrc = A.GT + (int64_t)(g * nfs + lam) * D * D * 64;
        for (int i = threadIdx.x; i < D * D * 64; i += blockDim.x) Gs_all[i] = gsrc[i];
        __syncthreads();
        const double *__restrict__ curL = cur + lam * cpl;
        double *__restrict__ nxtL = nxt + lam * npl;
        const int mend = MULTI ? min(mb1, mb0 + K) : mb1;
        // one copy of the mask body (the close sums of MULTI are picked by a
        // select chain on the wave-uniform k, so that they stay in registers
        // without unrolling the body K times)
        for (int mi = mb0; mi < mend; ++mi) {
            const int k = mi - mb0;
            const SubRec<N> M = load_sub_rec<N>(P, L.z + mi);
            const uint32_t ones = M.ones, twos = M.twos;
            const bool full0 = twos & 1u;            // vertex 0 visited twice: rows come in label pairs
            uint32_t hs = full0 ? (twos & ~1u) : 0u;  // heads >= 1, ascending
            int u = 0, su = full0 ? 0 : (int)(M.subb & 1u), slot = 0;
            double cp = 0.0, dext = 0.0;
            while (true) {
                // mask-only: rows of head vertex 0 use one plane (plane 0 while m_0 is once-visited)
                if (!(MASK && u == 0 && ((lam == 0) == full0)))
                    sub_fwd_row<N, MASK>(M, gaddr, curL, nxtL, lane8, u, su, M.rb + slot, start, cp, dext);
                ++slot;
                if (full0 && su == 0) {
                    su = 1;
                    continue;
                }
                if (!hs) break;
                u = __builtin_ctz(hs);
                hs &= hs - 1u;
                su = 0;
            }
            if (MULTI) {
#pragma unroll
                for (int kk = 0; kk < K; ++kk) cpk[kk] = (kk == k) ? cpk[kk] + cp : cpk[kk];
                if (!MASK && !last && (ones & 1u)) sub_fwd_close<N>(M, nxtL, lane8, 0.0, dext);
            } else {
                const double t = A.W * cp;
                if (last) {
                    if (cfg >= 0 && A.out) A.out[cfg] = t;
                } else if (ones) {
                    sub_fwd_close<N>(M, nxt, lane8, t, dext);
                }
            }
        }
    }
    if (MULTI) {
        // t_m = W sum over rows and flavours; the next cycle opens in every flavour
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int mi = mb0 + k;
            if (mi >= mb1) continue;
            const SubRec<N> M = load_sub_rec<N>(P, L.z + mi);
            const double t = A.W * cpk[k];
            if (last) {
                if (cfg >= 0 && A.out) A.out[cfg] = t;
            } else if (M.ones) {
                const int h = __builtin_ctz(M.ones);
                const int sh = (M.subb >> h) & 1u;
                const int crow = sub_child_base<N>(M, 2 * h + sh) + sub_head_slot(h, sh, M.twos | (1u << h));
                double *dst = nxt + (int64_t)crow * D * 64 + (2 * h + sh) * 64;
                if (MASK) {
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
// reverse: B = dS/dF of the labelled states at `level` from B at level + 1,
// the transpose of the forward rules above:
//   a[(w, s)] = c B(child)[(w, s)] for every output the row extends to
//   (c = 2 on a first visit, 1 otherwise and in mask-only mode), plus
//   W tbar_m on the row's close slot (u, s_u);
//   tbar_m = sum_l B(m', h, s_h, l)[(h, s_h)] of the slot the next cycle opens
//   on (1 at the full mask), B(m, u, s_u)[i] = sum_j G[i][j] a[j] over the
//   current slots i, and dS/dG[i][j] += f[i] a[j].
// A wavefront owns whole rows.  The workgroup keeps the rows i of G it needs
// and their dS/dG accumulator for its 64 configurations in LDS ([i][j][lane]),
// adding the accumulator to the packed gradient once per flavour.  Up to
// n = 6 one workgroup owns every row i (2 x 72 KB at n = 6); at n = 7, 8 the
// two matrices would not fit (2 x 128 KB at n = 8), so two workgroups share
// a block of masks, each owning half of the rows i (grid z): both read the
// child adjoints a, each reads its half of the states and writes its half of
// B.
// ---------------------------------------------------------------------------
template <int N>
struct SubAdjShape {
    static constexpr int D = 2 * N;
    static constexpr bool SPLIT = 2 * D * D * 64 * 8 > 160 * 1024;
    static constexpr int RI = SPLIT ? N : D;   // rows i owned by one workgroup
};

template <int N, bool MASK>
__device__ __forceinline__ void sub_adj_row(const SubRec<N> &M, uint32_t gaddr, uint32_t gbaddr,
                                            const double *__restrict__ FL, const double *__restrict__ BnL,
                                            double *__restrict__ BcL, uint32_t lane8, int u, int su, int r,
                                            bool start, double tb, int i0) {
    constexpr int D = 2 * N, RI = SubAdjShape<N>::RI;
    const uint32_t ones = M.ones, twos = M.twos, subb = M.subb;
    const uint32_t cs = sub_current(N, u, su, ones, twos, subb) >> i0;   // owned rows, from bit 0
    if (!(cs & ((1u << RI) - 1u))) return;   // wave-uniform: nothing of this row is owned here
    // FL, BnL, BcL: this flavour's planes; row offsets in 32-bit (a level's
    // rows times (2n)^2 x 64 stay far below 2^31)
    const double *__restrict__ src = FL + (r * D + i0) * 64;
    // only the owned current slots' states are loaded (wave-uniform branches:
    // 16.3 -> 15.7 ms on the honeycomb workload against loading every owned
    // slot with selected addresses); the child adjoints below keep the
    // selected addresses (loading only the extended outputs' ones measured
    // 21.8 ms)
    double f[RI], a[D];
#pragma unroll
    for (int k = 0; k < RI; ++k) {
        double x = 0.0;
        if (((cs >> k) & 1u) && !start) x = lane_ld_nt(src + k * 64, lane8);
        f[k] = start ? (i0 + k == su ? 1.0 : 0.0) : x;   // start: vertex 0 on label s_u
    }
    uint32_t need = 0;   // outputs j with a[j] possibly nonzero (wave-uniform)
#pragma unroll
    for (int w = 0; w < N; ++w) {
        const uint32_t bit = 1u << w;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int j = 2 * w + s;
            const bool once = ones & bit;
            bool ext = !(twos & bit) && (!once || (int)((subb >> w) & 1u) == s);
            if (MASK && once && w == 0 && u == 0) ext = false;   // the head point itself
            const int crow = ext ? M.crb[j] + sub_head_slot(u, su, once ? (twos | bit) : twos) : 0;
            const double bc = lane_ld(BnL + (ext ? (crow * D + j) * 64 : 0), lane8);
            a[j] = ext ? ((!once && !MASK) ? 2.0 * bc : bc) : 0.0;
            if (ext) need |= 1u << j;
        }
    }
    const int jc = 2 * u + su;   // the row's close slot
#pragma unroll
    for (int j = 0; j < D; ++j) a[j] = (j == jc) ? a[j] + tb : a[j];
    need |= 1u << jc;
    asm volatile("" : "+v"(gaddr));
    asm volatile("" : "+v"(gbaddr));
    const lds_double *Gs = (const lds_double *)(uintptr_t)gaddr;
    lds_double *Gb = (lds_double *)(uintptr_t)gbaddr;
    double *__restrict__ dst = BcL + (r * D + i0) * 64;
#pragma unroll
    for (int k = 0; k < RI; ++k) {
        if (!((cs >> k) & 1u)) continue;   // wave-uniform
        // every output j, a[j] = 0 where nothing is needed: straight-line LDS
        // reads that issue together and are waited for once, rather than one
        // read-and-wait per needed output behind a branch
        double b = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) b = __builtin_fma((double)Gs[(k * D + j) * 64], a[j], b);
        lane_st_nt(dst + k * 64, lane8, b);
#pragma unroll
        for (int j = 0; j < D; ++j)
            if ((need >> j) & 1u)   // wave-uniform
                __hip_atomic_fetch_add(Gb + (k * D + j) * 64, f[k] * a[j], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

template <int N, bool MASK>
__global__ void __launch_bounds__(1024) sub_adj_kernel(const LvlArgs A) {
    constexpr int D = 2 * N, RI = SubAdjShape<N>::RI;
    extern __shared__ double lds[];
    double *Gs_all = lds;                      // [RI][D][64]  the owned rows of G
    double *Gb_all = lds + RI * D * 64;        // [RI][D][64]  dS/dG of the owned rows, this workgroup
    const int lane = threadIdx.x & 63, wave = COS_RF(threadIdx.x >> 6);   // wave index: uniform
    const int wpb = blockDim.x >> 6;
    const int i0 = SubAdjShape<N>::SPLIT ? (int)blockIdx.z * RI : 0;   // first owned row i
    const DevPlan &P = A.plan;
    const int4 L = load_level(P, A.level);
    // the workgroup's block of masks, claimed one at a time by its wavefronts;
    // on levels of few masks the items are (mask, row) pairs instead, item
    // i = 2n m + k standing for row k of mask m (a mask has at most 2n rows),
    // so that the rows of a mask run side by side
    constexpr int RPM = D;
    const int nitems = A.row_items ? L.w * RPM : L.w;
    const int blk0 = blockIdx.x * wpb * A.mpb;
    const int blk1 = min(blk0 + wpb * A.mpb, nitems);   // may hold fewer items than waves: they still join the barriers
    __shared__ int next_mask;
    const int gl = blockIdx.y, g = A.group0 + gl;
    const int nfs = A.nfs;
    const double *__restrict__ F = A.F + gl * A.F_gstride + (int64_t)A.F_row0 * D * 64;
    const int64_t fpl = A.F_frows * D * 64, cpl = A.cur_frows * D * 64, npl = A.nxt_frows * D * 64;
    const double *__restrict__ Bn = A.cur + gl * A.cur_gstride;   // level + 1
    double *__restrict__ Bc = A.nxt + gl * A.nxt_gstride;         // level
    const uint32_t lane8 = (uint32_t)lane * 8u;
    const int cfg = A.lane_cfg[g * 64 + lane];
    const double obar = cfg >= 0 ? A.out_bar[cfg] : 0.0;
    const uint32_t gaddr = lds_addr(Gs_all) + lane * 8u, gbaddr = lds_addr(Gb_all) + lane * 8u;
    const bool top = A.level == 2 * N, start = A.level == 1;

    for (int lam = 0; lam < nfs; ++lam) {
        __syncthreads();   // the previous flavour's accumulator has been flushed
        const double *__restrict__ gsrc = A.GT + (int64_t)(g * nfs + lam) * D * D * 64 + (int64_t)i0 * D * 64;
        for (int i = threadIdx.x; i < RI * D * 64; i += blockDim.x) {
            Gs_all[i] = gsrc[i];
            Gb_all[i] = 0.0;
        }
        if (threadIdx.x == 0) next_mask = blk0 + wpb;   // masks blk0 .. blk0 + wpb - 1 go to the waves in order
        __syncthreads();
        const double *__restrict__ FL = F + lam * fpl;
        const double *__restrict__ BnL = Bn + lam * cpl;
        double *__restrict__ BcL = Bc + lam * npl;
        for (int it = blk0 + wave; it < blk1;) {
            const int mi = A.row_items ? it / RPM : it;
            const SubRec<N> M = load_sub_rec<N>(P, L.z + mi);
            const uint32_t ones = M.ones, twos = M.twos;
            const bool full0 = twos & 1u;
            uint32_t hs = full0 ? (twos & ~1u) : 0u;   // heads >= 1, ascending
            int u = 0, su = full0 ? 0 : (int)(M.subb & 1u), slot = 0;
            bool go = true, one = false;
            if (A.row_items) {
                // this item's row alone.  The rows of a mask: (0, s_0) alone
                // while vertex 0 is once visited; once it is full, (0, 0),
                // (0, 1), then (h, 0), (h, 1) for the heads h >= 1 in order
                const int k = it - mi * RPM;
                one = true;
                if (k > 0) {
                    go = full0;
                    if (full0) {
                        const int j = k >> 1;   // 0: vertex 0; j >= 1: the j-th head >= 1
                        for (int q = 1; q < j; ++q) hs &= hs - 1u;
                        if (j > 0) {
                            go = hs != 0;   // the mask has fewer rows
                            u = go ? __builtin_ctz(hs) : 0;
                        }
                        su = k & 1;
                    }
                    slot = k;
                }
            }
            if (go) {
                double tb = 0.0;
                if (top) {
                    tb = obar;
                } else if (ones) {
                    const int h = __builtin_ctz(ones);
                    const int sh = (M.subb >> h) & 1u;
                    const int crow = sub_child_base<N>(M, 2 * h + sh) + sub_head_slot(h, sh, twos | (1u << h));
                    // mask-only: the first cycle's successor lives on plane 1 only
                    for (int k = (MASK && h == 0 ? 1 : 0); k < nfs; ++k)
                        tb += lane_ld(Bn + k * cpl + (int64_t)crow * D * 64 + (2 * h + sh) * 64, lane8);
                }
                tb *= A.W;
                while (true) {
                    if (!(MASK && u == 0 && ((lam == 0) == full0)))
                        sub_adj_row<N, MASK>(M, gaddr, gbaddr, FL, BnL, BcL, lane8, u, su, M.rb + slot, start, tb, i0);
                    if (one) break;
                    ++slot;
                    if (full0 && su == 0) {
                        su = 1;
                        continue;
                    }
                    if (!hs) break;
                    u = __builtin_ctz(hs);
                    hs &= hs - 1u;
                    su = 0;
                }
            }
            int nx = 0;
            if (lane == 0) nx = atomicAdd(&next_mask, 1);
            it = COS_RF(nx);   // lane 0's claim (every lane is active here)
        }
        __syncthreads();
        double *__restrict__ gb = A.Gbar_T + (int64_t)(g * nfs + lam) * D * D * 64 + (int64_t)i0 * D * 64;
        for (int i = threadIdx.x; i < RI * D * 64; i += blockDim.x) {
            const double x = Gb_all[i];
            if (x != 0.0) atomicAdd(gb + i, x);
        }
    }
}

static hipError_t allow_sub_lds(const void *fn, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_sub_level(const LvlArgs &a, int nblocks, int ngroups, int wpb, hipStream_t s) {
    const int n = a.plan.n;
    if (wpb < 1 || wpb > 16) return hipErrorInvalidValue;
    const bool multi = a.nfs > 1;
    if (multi && a.mpb > kMultiMasks) return hipErrorInvalidValue;
    const size_t shm = (size_t)(2 * n) * (2 * n) * 64 * sizeof(double);
    const dim3 grid((unsigned)((nblocks + wpb - 1) / wpb), (unsigned)ngroups);
    switch (n) {
#define COS_SUB_CASE(K)                                                                                  \
    case K: {                                                                                            \
        const void *fn = a.mask_only ? (const void *)sub_fwd_kernel<K, true, true>                       \
                         : multi     ? (const void *)sub_fwd_kernel<K, true, false>                      \
                                     : (const void *)sub_fwd_kernel<K, false, false>;                    \
        hipError_t e = allow_sub_lds(fn, shm);                                                           \
        if (e != hipSuccess) return e;                                                                   \
        if (a.mask_only) hipLaunchKernelGGL((sub_fwd_kernel<K, true, true>), grid, dim3(64 * wpb), shm, s, a); \
        else if (multi) hipLaunchKernelGGL((sub_fwd_kernel<K, true, false>), grid, dim3(64 * wpb), shm, s, a); \
        else hipLaunchKernelGGL((sub_fwd_kernel<K, false, false>), grid, dim3(64 * wpb), shm, s, a);           \
        break;                                                                                           \
    }
        COS_SUB_CASE(1) COS_SUB_CASE(2) COS_SUB_CASE(3) COS_SUB_CASE(4)
        COS_SUB_CASE(5) COS_SUB_CASE(6) COS_SUB_CASE(7) COS_SUB_CASE(8)
#undef COS_SUB_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_sub_adj_level(const LvlArgs &a, int nblocks, int ngroups, hipStream_t s) {
    const int n = a.plan.n;
    const int wpa = adj_waves_per_block();
    const size_t side = 2 * (size_t)n, mat = side * side * 64 * sizeof(double);
    const bool split = 2 * mat > 160 * 1024;   // as SubAdjShape: two workgroups per block of masks
    const size_t shm = split ? mat : 2 * mat;   // owned rows of G and of the accumulator
    const dim3 grid((unsigned)((nblocks + wpa - 1) / wpa), (unsigned)ngroups, split ? 2u : 1u);
    switch (n) {
#define COS_SUBADJ_CASE(K)                                                                               \
    case K: {                                                                                            \
        const void *fn = a.mask_only ? (const void *)sub_adj_kernel<K, true>                             \
                                     : (const void *)sub_adj_kernel<K, false>;                           \
        hipError_t e = allow_sub_lds(fn, shm);                                                           \
        if (e != hipSuccess) return e;                                                                   \
        if (a.mask_only) hipLaunchKernelGGL((sub_adj_kernel<K, true>), grid, dim3(64 * wpa), shm, s, a); \
        else hipLaunchKernelGGL((sub_adj_kernel<K, false>), grid, dim3(64 * wpa), shm, s, a);            \
        break;                                                                                           \
    }
        COS_SUBADJ_CASE(1) COS_SUBADJ_CASE(2) COS_SUBADJ_CASE(3) COS_SUBADJ_CASE(4)
        COS_SUBADJ_CASE(5) COS_SUBADJ_CASE(6) COS_SUBADJ_CASE(7) COS_SUBADJ_CASE(8)
#undef COS_SUBADJ_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace libcos
