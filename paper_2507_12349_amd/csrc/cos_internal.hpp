// Internal declarations shared by the host side (libcos.cpp) and the HIP
// kernels (cos_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/libcos.h"

namespace libcos {

// ---------------------------------------------------------------------------
// State space of the vertex-level dynamic programme.
//
// A state is (m, u, v[, l]): m in {0,1,2}^n counts the visited points of each
// vertex (the per-interaction status of the Results section: unvisited,
// visited once, visited twice), u is the head vertex of the open cycle, v the
// current vertex, l the cycle's flavour.  Level = sum_k m_k (the number of
// visited points, the layer index of Alg. 1-3).  States are grouped in rows
// (m, u); a row holds one dense slot per vertex v (slots outside the row's
// current set are never read).  Buffers hold one plane of rows per flavour.
//
// Which rows and currents exist (reachable from the start (e_0, 0, 0)):
//   row (m, 0) for every m with m_0 >= 1 (the first cycle is still open);
//   row (m, h), h >= 1, iff m_0 = m_h = 2 (later heads are opened on the
//   second point of the lowest half-visited vertex, so vertex 0 is full).
//   currents of (m, 0): visited vertices, except 0 when m_0 = 1 and m != e_0;
//   currents of (m, h): visited vertices other than 0 and h, plus h itself
//   when no vertex below h is half visited (the cycle is still at its head).
// ---------------------------------------------------------------------------

// Per-level mask records (one 64-byte record per mask, level by level): what a
// wavefront needs to process a mask, fetched with one scalar load.
//   [0] mask code (base 3)     [1] ones | (twos << 16)
//   [2] level-relative row of (m, 0)
//   [3 + w] level-relative row of (m + e_w, 0) for each vertex w with m_w < 2
//           (-1 otherwise)
constexpr int kRecInts = 16;
static_assert(3 + COS_NMAX <= kRecInts, "mask record too small");

struct DevPlan {
    const int32_t *mrec;      // [total_masks][kRecInts]
    const int4 *levels;       // [2n + 2] .x = first row, .y = #rows, .z = first mask, .w = #masks
    int32_t n;
    int32_t max_rows;         // largest #rows of a level
    int32_t max_masks;        // largest #masks of a level
    int32_t pad;
    int64_t total_rows;
};

__host__ __device__ inline constexpr int pow3(int k) { return k <= 0 ? 1 : 3 * pow3(k - 1); }

// slot of head u inside the rows of a mask with twos-set `twos`
__host__ __device__ inline int head_slot(int u, uint32_t twos) {
    return u == 0 ? 0 : 1 + __builtin_popcount(twos & ((1u << u) - 1u) & ~1u);
}

// current set of row (m, u)
__host__ __device__ inline uint32_t current_set(int u, uint32_t ones, uint32_t twos) {
    uint32_t vis = ones | twos;
    if (u == 0) {
        // vertex 0 half visited and something else visited: the walk left vertex 0
        if ((ones & 1u) && vis != 1u) return vis & ~1u;
        return vis;
    }
    uint32_t c = vis & ~1u & ~(1u << u);
    if ((ones & ((1u << u) - 1u)) == 0u) c |= 1u << u;
    return c;
}

// ---------------------------------------------------------------------------
// Sublattice-labelled state space (bipartite lattices; Results, four-state
// interaction mask {0, (1,A), (1,B), 2}; Alg. 1/2).  Every vertex k carries a
// label s_k in {A = 0, B = 1} shared by its two points; matrices are 2n x 2n,
// index 2k + s.  Mask digit (base 4): 0 unvisited, 1 once on A, 2 once on B,
// 3 twice (the label is forgotten).  ones / twos as above, subb = vertices
// visited once on B.  A row is (m, u, s_u); a slot is (v, s_v), index 2v + s_v.
//   rows of m: (0, s_0) only, when m_0 is once-visited (s_0 from the mask);
//   otherwise (0, A), (0, B), then (h, A), (h, B) for each h >= 1 with m_h = 2;
//   current slots of (m, u, s_u): for v in current_set(u, ...): (v, label from
//   the mask) if v is once-visited, (u, s_u) if v = u, both labels otherwise.
// Mask records (kSubRecInts ints): [0] code (base 4), [1] ones | (twos << 16),
// [2] level-relative row of the mask's first row, [3] subb,
// [4 + 2w + s] first row of the child mask reached by visiting (w, s) (-1 when
// not allowed: w visited twice, or once with the other label).
// ---------------------------------------------------------------------------
constexpr int kSubNmax = 8;       // G of 64 lanes, (2n)^2 doubles each, must fit LDS
constexpr int kSubRecInts = 24;
static_assert(4 + 2 * kSubNmax <= kSubRecInts, "sublattice mask record too small");

__host__ __device__ inline int sub_head_slot(int u, int su, uint32_t twos) {
    if (u == 0) return (twos & 1u) ? su : 0;
    return 2 + 2 * __builtin_popcount(twos & ((1u << u) - 1u) & ~1u) + su;
}

__host__ __device__ inline uint32_t sub_current(int n, int u, int su, uint32_t ones, uint32_t twos, uint32_t subb) {
    const uint32_t cm = current_set(u, ones, twos);
    uint32_t out = 0;
    for (int v = 0; v < n; ++v) {
        if (!((cm >> v) & 1u)) continue;
        if ((ones >> v) & 1u) out |= 1u << (2 * v + ((subb >> v) & 1u));
        else if (v == u) out |= 1u << (2 * v + su);
        else out |= 3u << (2 * v);
    }
    return out;
}

// packing between the caller's layout and the per-lane layout of one order
struct PackArgs {
    const double *G;          // caller matrices
    const int64_t *Goff;      // may be null: back-to-back layout
    const double *stub;       // caller shift weights or null
    const int32_t *order;     // configurations of this order, in lane order
    double *GT;               // [ngroups][nfs][n][n][64]
    double *sigT;             // [ngroups][nfs][64] or null
    int32_t *lane_cfg;        // [ngroups][64], -1 = padding lane
    int32_t n, nfs, nmat, nstub, variant, ngroups, count;
};

// one level launch (forward or reverse)
struct LvlArgs {
    DevPlan plan;
    const double *GT, *sigT;
    const int32_t *lane_cfg;
    const double *cur;        // forward: states of `level`; reverse: adjoints of level + 1
    double *nxt;              // forward: states of level + 1; reverse: adjoints of `level`
    int64_t cur_gstride, nxt_gstride;   // doubles per group
    int64_t cur_frows, nxt_frows;       // rows per flavour plane ([flavour][row][v][lane])
    int32_t cur_row0, nxt_row0;         // first row of the level inside its plane
    const double *F;          // reverse: forward states of all levels
    int64_t F_gstride, F_frows;
    int32_t F_row0;
    int32_t level, group0, nfs, stubs, mpb;
    int32_t mask_only;        // SU(2) mask-only rules (two spin blocks as the two planes)
    int32_t det_groups;       // deterministic reverse: groups of the order (stride of the partial sums)
    int32_t row_items;        // reverse: the work items are (mask, row) pairs, not masks (levels of few masks)
    double W;                 // factor of one closed cycle: w * nflav (uniform) or w
    double *out;              // forward, last level: S per configuration (may be null)
    const double *out_bar;    // reverse: dL/dS per configuration
    double *Gbar_T, *sbar_T;  // reverse: packed gradient accumulators
};

// launchers (cos_level.hip)
hipError_t launch_pack(const PackArgs &a, hipStream_t s);
hipError_t launch_unpack(const PackArgs &a, const double *GbT, const double *sbT, double *Gb, double *sb,
                         hipStream_t s);
hipError_t launch_zero(double *p, int64_t n, hipStream_t s);
// sublattice forward level (cos_sub.hip): `a.plan` is a sublattice plan, rows
// hold 2n slots, GT holds 2n x 2n matrices; wpb <= 16
hipError_t launch_sub_level(const LvlArgs &a, int nblocks, int ngroups, int wpb, hipStream_t s);
// sublattice reverse level: adj_waves_per_block() wavefronts per workgroup
hipError_t launch_sub_adj_level(const LvlArgs &a, int nblocks, int ngroups, hipStream_t s);
// nblocks = blocks of `a.mpb` masks (reverse with row_items: of (mask, row)
// items); `wpb` wavefronts per workgroup (forward: at most 16; reverse:
// adj_waves_per_block())
hipError_t launch_level(const LvlArgs &a, bool reverse, int nblocks, int ngroups, int wpb, hipStream_t s);
int adj_waves_per_block();
// deterministic reverse sweep: every level's masks in kDetParts fixed parts;
// Gbar_T / sbar_T of the LvlArgs point to the partial sums
// [part][group][flavour][v][w][64] and [part][group][flavour][v][64]
constexpr int kDetParts = 32;
hipError_t launch_level_det(const LvlArgs &a, int ngroups, hipStream_t s);
// GbT = sum of the gsize-element parts in order; sbT (ssize elements,
// [group][flavour][64]) = sum over parts and slots v < n
hipError_t launch_det_reduce(const double *Gpart, const double *Spart, int64_t gsize, int64_t ssize, int n,
                             double *GbT, double *sbT, hipStream_t s);
// most masks per wavefront of the forward kernel when there are several flavours
constexpr int kMultiMasks = 4;
// launchers (cos_kernels.hip)
hipError_t launch_g0(int nconf, const int32_t *n, const int64_t *voff, const int32_t *sites,
                     const double *tau, int L, double t, double beta, int nmat, const double *mu,
                     const double *alpha, const int64_t *Goff, double *G, double *dG, hipStream_t s);
hipError_t launch_g0_honeycomb(int nconf, const int32_t *n, const int64_t *voff, const int32_t *cells,
                               const double *tau, int L, double t, double beta, int nmat, const double *mu,
                               const double *alpha, const double *delta, const int64_t *Goff, double *G,
                               double *dG, hipStream_t s);
// CDet comparison path (cos_cdet.hip): workspace elements per configuration
// (doubles for precision 0, double-double pairs for 1) and the launcher
int64_t cdet_elems_per_config(int n);
hipError_t launch_cdet(int nconf, int n, const double *A, int precision, double eps, void *work, double *out,
                       hipStream_t s);
// Monte Carlo support (cos_mc.hip)
hipError_t launch_mc_sample(int nconf, int n, int L, double beta, uint64_t seed, int64_t first, int32_t *sites,
                            double *tau, hipStream_t s);
hipError_t launch_moments(int count, const double *x, double *acc, hipStream_t s);
hipError_t launch_chain(int nconf, const int32_t *n, int nmat, const int64_t *Goff, const double *Gb,
                        const double *dG, const double *sb, int nstub, double U, double *mub,
                        double *alb, hipStream_t s);
// p[i] = i for i < n (the identity schedule of a one-order batch)
hipError_t launch_iota(int32_t *p, int n, hipStream_t s);

// ---------------------------------------------------------------------------
// Forward sums on device memory the caller places (libcos.cpp), for the entry
// point that allocates nothing (cos_static.hip).
// ---------------------------------------------------------------------------
// records the error text of the calling thread (cos_last_error) and returns s
cos_status report(cos_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
// gfx950 check and compute-unit count of the current device
cos_status current_device(int *dev, int *ncu);
// host state tables of order n (built once, cached for the process)
struct PlanTables {
    const int32_t *mrec;      // [masks][kRecInts]
    size_t mrec_ints;
    const int4 *levels;       // [2n + 2]
    size_t nlevels;
    int32_t max_rows, max_masks;
    int64_t total_rows;
};
cos_status plan_tables(int n, PlanTables *out);
// workspace of one forward call: every pointer inside device memory the
// caller owns; the level windows hold `chunk` groups of 64 configurations
struct FixedWorkspace {
    DevPlan plan;             // state tables of the order, already on the device
    int32_t *order;           // [nconf]
    double *GT, *sigT;        // packed propagators and shift weights of every group
    int32_t *lane;            // [ngroups * 64]
    double *win;              // two level windows of `chunk` groups
    int32_t chunk;
};
// sizes (doubles, or int32 for order / lane) of the pieces of a FixedWorkspace
struct FixedSizes {
    int64_t order_ints, gt_doubles, sig_doubles, lane_ints, win_doubles_per_group;
};
FixedSizes fixed_sizes(int nconf, int n, int nfs, int32_t max_rows);
// forward sums of nconf configurations of order n stored back to back (layout
// of cos_connected_sum_batched with d_Goff = NULL), asynchronous on s
cos_status forward_fixed(int dev, int ncu, const FixedWorkspace &ws, int32_t nconf, int32_t n, int32_t nflav,
                         int32_t variant, int32_t flags, const double *d_G, const double *d_stub,
                         double cycle_weight, double *d_out, hipStream_t s);

}  // namespace libcos
