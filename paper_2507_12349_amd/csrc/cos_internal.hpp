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
// current set are never read).
//
// Which rows and currents exist (reachable from the start (e_0, 0, 0)):
//   row (m, 0) for every m with m_0 >= 1 (the first cycle is still open);
//   row (m, h), h >= 1, iff m_0 = m_h = 2 (later heads are opened on the
//   second point of the lowest half-visited vertex, so vertex 0 is full).
//   currents of (m, 0): visited vertices, except 0 when m_0 = 1 and m != e_0;
//   currents of (m, h): visited vertices other than 0 and h, plus h itself
//   when no vertex below h is half visited (the cycle is still at its head).
// ---------------------------------------------------------------------------

struct DevPlan {
    const int32_t *rowbase;   // [3^n] level-relative index of row (m, 0); -1 if m_0 = 0
    const uint32_t *minfo;    // [3^n] ones | (twos << 16): vertices with m_k = 1, m_k = 2
    const int2 *rows;         // [total_rows] .x = code << 4 | u, .y = mask index in its level
    const int32_t *masks;     // [total_masks] mask codes, level by level
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

struct FwdArgs {
    DevPlan plan;             // one order per launch
    const int32_t *order;     // configurations of this order
    const double *G;
    const int64_t *Goff;      // may be null: back-to-back layout (uniform n only)
    const double *stub;
    double *out;
    double *ws;               // workspace, ws_per_wg doubles per workgroup
    int32_t *counter;         // work queue head
    int64_t ws_per_wg;
    double W;                 // factor of one closed cycle: w * nflav (uniform) or w
    int32_t nconf, nfs, nmat, nstub, variant, stubs;
};

struct AdjArgs {
    DevPlan plan;             // one order per launch
    const int32_t *order;     // configurations of this order
    const double *G;
    const int64_t *Goff;
    const double *stub;
    const double *out_bar;
    double *out;              // may be null
    double *G_bar;
    double *stub_bar;         // may be null
    double *ws;
    int32_t *counter;
    int64_t ws_per_wg;
    double W;
    int32_t nconf, nfs, nmat, nstub, variant, stubs;
};

// workspace sizes (doubles) per workgroup
inline int64_t fwd_ws_doubles(const DevPlan &p, int nfs) {
    int64_t rs = (int64_t)nfs * p.n;
    return 2 * (int64_t)p.max_rows * rs + (int64_t)p.max_rows * nfs + 8;
}
inline int64_t adj_ws_doubles(const DevPlan &p, int nfs) {
    int64_t rs = (int64_t)nfs * p.n;
    return p.total_rows * rs + 2 * (int64_t)p.max_rows * rs + (int64_t)p.max_rows * nfs +
           (int64_t)p.max_masks + 8;
}

// launchers (cos_kernels.hip)
hipError_t launch_forward(const FwdArgs &a, int grid, int block, hipStream_t s);
hipError_t launch_adjoint(const AdjArgs &a, int grid, int block, hipStream_t s);
hipError_t launch_g0(int nconf, const int32_t *n, const int64_t *voff, const int32_t *sites,
                     const double *tau, int L, double t, double beta, int nmat, const double *mu,
                     const double *alpha, const int64_t *Goff, double *G, double *dG, hipStream_t s);
hipError_t launch_chain(int nconf, const int32_t *n, int nmat, const int64_t *Goff, const double *Gb,
                        const double *dG, const double *sb, int nstub, double U, double *mub,
                        double *alb, hipStream_t s);

}  // namespace libcos
