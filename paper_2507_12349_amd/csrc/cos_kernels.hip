// HIP kernels for gfx950 (CDNA4): forward and reverse sweeps of the
// connected-diagram dynamic programme, the free-propagator builder and the
// chain rule to (mu, shift).
//
// Forward (Results: Mahajan-Vinay clow DP with CoS-2 connected head ordering,
// merged contact states and SB-CoS shift heads; Alg. 2/3).  One workgroup owns
// one configuration at a time and sweeps the levels (number of visited
// points) in order.  Within a level every (row, flavour) pair is independent:
// a thread loads the row's currents f[v], forms acc = f . G_l (N^2 FMAs, G_l
// read through the scalar cache into SGPRs since it is uniform over the
// workgroup) and writes
//   extension to w (m_w < 2): child (m + e_w, u)[w] = c_w acc[w]
//     (c_w = 2 for the first visit of w: either of its two points),
//   shift head (m_w = 1, current w just reached w for the first time):
//     + (-sigma_l) f[w]  (the other point of w becomes a shift head of the
//     cycle's colour; doubled for the start row, whose head point may be
//     either point of vertex 0),
//   close partial acc[u].
// Every child slot has exactly one parent mask, so no write conflicts.  A
// second pass per mask sums the close partials over heads and flavours
// (t = W sum), and opens the next cycle at h = min{k : m_k = 1} with value t
// for every flavour (the new head hangs on an interaction line of the visited
// part, so only connected diagrams are produced), or stores S at the full
// mask.
//
// Reverse: the same sweep backwards with B = dS/dF, recomputing the forward
// layers first; dS/dG accumulates per thread in registers (outer products
// f x a) and is reduced over the workgroup at the end.
#include "cos_internal.hpp"

namespace libcos {

#define COS_RF(x) __builtin_amdgcn_readfirstlane(x)

// read-only data that every lane of the workgroup reads at the same address:
// in the constant address space the loads go through the scalar cache
typedef const __attribute__((address_space(4))) double cdouble;

// a pointer the caller knows to be equal on every lane, moved to SGPRs
template <class T>
__device__ __forceinline__ T *uniform_ptr(T *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T *>(((uint64_t)hi << 32) | lo);
}

__global__ void reset_counter_kernel(int32_t *c) {
    if (threadIdx.x == 0) c[0] = 0;
}

// ---------------------------------------------------------------------------
// forward sweep of one configuration
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void fwd_config(const FwdArgs &A, const DevPlan &P, int c,
                                           double *__restrict__ ws) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    const int nfs = A.nfs;
    const int lam = COS_RF(wave % nfs);
    const int r0 = (wave / nfs) * 64 + lane;
    const int rstride = (nwaves / nfs) * 64;
    const int RS = nfs * N;
    double *__restrict__ F0 = ws;
    double *__restrict__ F1 = ws + (size_t)P.max_rows * RS;
    double *__restrict__ cb = F1 + (size_t)P.max_rows * RS;

    const int64_t goff = A.Goff ? A.Goff[c] : (int64_t)c * A.nmat * N * N;
    const double *__restrict__ G = uniform_ptr(A.G + goff + (A.variant ? (int64_t)lam * N * N : 0));
    double sig = 0.0;
    if (A.stubs) sig = A.stub[(int64_t)c * A.nstub + (A.variant ? lam : 0)];

    // level 1: the single row (e_0, 0), current 0, value 1 for every flavour
    if (tid < nfs) F1[tid * N] = 1.0;
    __syncthreads();

    for (int l = 1; l <= 2 * N; ++l) {
        const int4 L = P.levels[l];
        double *__restrict__ Fc = (l & 1) ? F1 : F0;
        double *__restrict__ Fn = (l & 1) ? F0 : F1;
        for (int r = r0; r < L.y; r += rstride) {
            const int2 ri = P.rows[L.x + r];
            const int code = ri.x >> 4, u = ri.x & 15;
            const uint32_t mi = P.minfo[code];
            const uint32_t ones = mi & 0xffffu, twos = mi >> 16;
            const uint32_t cm = current_set(u, ones, twos);
            const double *__restrict__ src = Fc + (size_t)r * RS + lam * N;
            // keep the N^2 loads of G inside the row loop: they come from the
            // scalar cache each time instead of pinning N^2 registers
            cdouble *Gr = (cdouble *)G;
            asm volatile("" : "+s"(Gr));
            double f[N], acc[N];
#pragma unroll
            for (int v = 0; v < N; ++v) {
                const double x = src[v];   // every slot of a row is in bounds
                f[v] = ((cm >> v) & 1u) ? x : 0.0;
            }
#pragma unroll
            for (int w = 0; w < N; ++w) acc[w] = 0.0;
#pragma unroll
            for (int v = 0; v < N; ++v) {
#pragma unroll
                for (int w = 0; w < N; ++w) acc[w] = __builtin_fma(f[v], Gr[v * N + w], acc[w]);
                // one row of G live in SGPRs at a time
                __builtin_amdgcn_sched_barrier(0);
            }
            double cp = 0.0;
#pragma unroll
            for (int w = 0; w < N; ++w) cp = (w == u) ? acc[w] : cp;
            cb[r * nfs + lam] = cp;
            const double sg = sig * (code == 1 ? 2.0 : 1.0);
#pragma unroll
            for (int w = 0; w < N; ++w) {
                const uint32_t bit = 1u << w;
                if (twos & bit) continue;
                const bool first = !(ones & bit);
                double val = first ? 2.0 * acc[w] : acc[w];
                if (!first && (cm & bit)) val = __builtin_fma(-sg, f[w], val);
                const uint32_t ctw = first ? twos : (twos | bit);
                const int crow = P.rowbase[code + pow3(w)] + head_slot(u, ctw);
                Fn[(size_t)crow * RS + lam * N + w] = val;
            }
        }
        __syncthreads();
        for (int i = tid; i < L.w; i += blockDim.x) {
            const int code = P.masks[L.z + i];
            const uint32_t mi = P.minfo[code];
            const uint32_t ones = mi & 0xffffu, twos = mi >> 16;
            const int rb = P.rowbase[code];
            const int nh = 1 + ((twos & 1u) ? __builtin_popcount(twos & ~1u) : 0);
            double s = 0.0;
            for (int j = 0; j < nh; ++j)
                for (int k = 0; k < nfs; ++k) s += cb[(rb + j) * nfs + k];
            const double t = A.W * s;
            if (l == 2 * N) {
                A.out[c] = t;
            } else if (ones) {
                const int h = __builtin_ctz(ones);
                const int crow = P.rowbase[code + pow3(h)] + head_slot(h, twos | (1u << h));
                double *dst = Fn + (size_t)crow * RS + h;
                for (int k = 0; k < nfs; ++k) {
                    if (h == 0) dst[k * N] += t;   // the first cycle's own extension landed here
                    else dst[k * N] = t;
                }
            }
        }
        __syncthreads();
    }
}

template <int N, int MAXT>
__global__ void __launch_bounds__(MAXT) forward_kernel(const FwdArgs A) {
    __shared__ int s_item;
    double *ws = A.ws + (size_t)blockIdx.x * A.ws_per_wg;
    while (true) {
        if (threadIdx.x == 0) s_item = atomicAdd(A.counter, 1);
        __syncthreads();
        const int item = COS_RF(s_item);
        __syncthreads();
        if (item >= A.nconf) break;   // every workgroup reaches this once the queue is empty
        const int c = COS_RF(A.order[item]);
        fwd_config<N>(A, A.plan, c, ws);
    }
}

hipError_t launch_forward(const FwdArgs &a, int grid, int block, hipStream_t s) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, a.counter);
    switch (a.plan.n) {
#define COS_FWD_CASE(K)                                                                                   \
    case K:                                                                                               \
        if (block <= 256) hipLaunchKernelGGL((forward_kernel<K, 256>), dim3(grid), dim3(block), 0, s, a); \
        else hipLaunchKernelGGL((forward_kernel<K, 1024>), dim3(grid), dim3(block), 0, s, a);             \
        break;
        COS_FWD_CASE(1) COS_FWD_CASE(2) COS_FWD_CASE(3) COS_FWD_CASE(4)
        COS_FWD_CASE(5) COS_FWD_CASE(6) COS_FWD_CASE(7) COS_FWD_CASE(8)
        COS_FWD_CASE(9) COS_FWD_CASE(10) COS_FWD_CASE(11) COS_FWD_CASE(12)
#undef COS_FWD_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reverse sweep of one configuration (forward layers recomputed first)
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void adj_config(const AdjArgs &A, int c, double *__restrict__ ws,
                                           double *__restrict__ red) {
    const DevPlan &P = A.plan;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    const int nfs = A.nfs;
    const int lam = COS_RF(wave % nfs);
    const int r0 = (wave / nfs) * 64 + lane;
    const int rstride = (nwaves / nfs) * 64;
    const int RS = nfs * N;
    double *__restrict__ Fall = ws;
    double *__restrict__ B0 = Fall + (size_t)P.total_rows * RS;
    double *__restrict__ B1 = B0 + (size_t)P.max_rows * RS;
    double *__restrict__ cb = B1 + (size_t)P.max_rows * RS;
    double *__restrict__ tbar = cb + (size_t)P.max_rows * nfs;

    const int64_t goff = A.Goff ? A.Goff[c] : (int64_t)c * A.nmat * N * N;
    const double *__restrict__ G = uniform_ptr(A.G + goff + (A.variant ? (int64_t)lam * N * N : 0));
    double sig = 0.0;
    if (A.stubs) sig = A.stub[(int64_t)c * A.nstub + (A.variant ? lam : 0)];

    // ---- forward, all layers kept ----
    if (tid < nfs) Fall[(size_t)P.levels[1].x * RS + tid * N] = 1.0;
    __syncthreads();
    for (int l = 1; l <= 2 * N; ++l) {
        const int4 L = P.levels[l];
        const int4 Ln = P.levels[l < 2 * N ? l + 1 : l];
        double *__restrict__ Fc = Fall + (size_t)L.x * RS;
        double *__restrict__ Fn = Fall + (size_t)Ln.x * RS;
        for (int r = r0; r < L.y; r += rstride) {
            const int2 ri = P.rows[L.x + r];
            const int code = ri.x >> 4, u = ri.x & 15;
            const uint32_t mi = P.minfo[code];
            const uint32_t ones = mi & 0xffffu, twos = mi >> 16;
            const uint32_t cm = current_set(u, ones, twos);
            const double *__restrict__ src = Fc + (size_t)r * RS + lam * N;
            // keep the N^2 loads of G inside the row loop: they come from the
            // scalar cache each time instead of pinning N^2 registers
            cdouble *Gr = (cdouble *)G;
            asm volatile("" : "+s"(Gr));
            double f[N], acc[N];
#pragma unroll
            for (int v = 0; v < N; ++v) {
                const double x = src[v];   // every slot of a row is in bounds
                f[v] = ((cm >> v) & 1u) ? x : 0.0;
            }
#pragma unroll
            for (int w = 0; w < N; ++w) acc[w] = 0.0;
#pragma unroll
            for (int v = 0; v < N; ++v) {
#pragma unroll
                for (int w = 0; w < N; ++w) acc[w] = __builtin_fma(f[v], Gr[v * N + w], acc[w]);
                // one row of G live in SGPRs at a time
                __builtin_amdgcn_sched_barrier(0);
            }
            double cp = 0.0;
#pragma unroll
            for (int w = 0; w < N; ++w) cp = (w == u) ? acc[w] : cp;
            cb[r * nfs + lam] = cp;
            const double sg = sig * (code == 1 ? 2.0 : 1.0);
#pragma unroll
            for (int w = 0; w < N; ++w) {
                const uint32_t bit = 1u << w;
                if (twos & bit) continue;
                const bool first = !(ones & bit);
                double val = first ? 2.0 * acc[w] : acc[w];
                if (!first && (cm & bit)) val = __builtin_fma(-sg, f[w], val);
                const uint32_t ctw = first ? twos : (twos | bit);
                const int crow = P.rowbase[code + pow3(w)] + head_slot(u, ctw);
                Fn[(size_t)crow * RS + lam * N + w] = val;
            }
        }
        __syncthreads();
        for (int i = tid; i < L.w; i += blockDim.x) {
            const int code = P.masks[L.z + i];
            const uint32_t mi = P.minfo[code];
            const uint32_t ones = mi & 0xffffu, twos = mi >> 16;
            const int rb = P.rowbase[code];
            const int nh = 1 + ((twos & 1u) ? __builtin_popcount(twos & ~1u) : 0);
            double s = 0.0;
            for (int j = 0; j < nh; ++j)
                for (int k = 0; k < nfs; ++k) s += cb[(rb + j) * nfs + k];
            const double t = A.W * s;
            if (l == 2 * N) {
                if (A.out) A.out[c] = t;
            } else if (ones) {
                const int h = __builtin_ctz(ones);
                const int crow = P.rowbase[code + pow3(h)] + head_slot(h, twos | (1u << h));
                double *dst = Fn + (size_t)crow * RS + h;
                for (int k = 0; k < nfs; ++k) {
                    if (h == 0) dst[k * N] += t;
                    else dst[k * N] = t;
                }
            }
        }
        __syncthreads();
    }

    // ---- reverse sweep ----
    double gacc[N][N];
#pragma unroll
    for (int v = 0; v < N; ++v)
#pragma unroll
        for (int w = 0; w < N; ++w) gacc[v][w] = 0.0;
    double sacc = 0.0;
    const double obar = A.out_bar[c];
    for (int l = 2 * N; l >= 1; --l) {
        const int4 L = P.levels[l];
        double *__restrict__ Bc = (l & 1) ? B1 : B0;
        double *__restrict__ Bn = (l & 1) ? B0 : B1;
        const double *__restrict__ Fc = Fall + (size_t)L.x * RS;
        // per mask: W * (adjoint of the close value)
        for (int i = tid; i < L.w; i += blockDim.x) {
            const int code = P.masks[L.z + i];
            const uint32_t mi = P.minfo[code];
            const uint32_t ones = mi & 0xffffu, twos = mi >> 16;
            double tb = 0.0;
            if (l == 2 * N) {
                tb = obar;
            } else if (ones) {
                const int h = __builtin_ctz(ones);
                const int crow = P.rowbase[code + pow3(h)] + head_slot(h, twos | (1u << h));
                for (int k = 0; k < nfs; ++k) tb += Bn[(size_t)crow * RS + k * N + h];
            }
            tbar[i] = A.W * tb;
        }
        __syncthreads();
        for (int r = r0; r < L.y; r += rstride) {
            const int2 ri = P.rows[L.x + r];
            const int code = ri.x >> 4, u = ri.x & 15;
            const uint32_t mi = P.minfo[code];
            const uint32_t ones = mi & 0xffffu, twos = mi >> 16;
            const uint32_t cm = current_set(u, ones, twos);
            const double *__restrict__ src = Fc + (size_t)r * RS + lam * N;
            cdouble *Gr = (cdouble *)G;
            asm volatile("" : "+s"(Gr));
            double f[N], a[N], bc[N];
#pragma unroll
            for (int v = 0; v < N; ++v) {
                const double x = src[v];   // every slot of a row is in bounds
                f[v] = ((cm >> v) & 1u) ? x : 0.0;
            }
#pragma unroll
            for (int w = 0; w < N; ++w) {
                const uint32_t bit = 1u << w;
                a[w] = 0.0;
                bc[w] = 0.0;
                if (twos & bit) continue;
                const bool first = !(ones & bit);
                const uint32_t ctw = first ? twos : (twos | bit);
                const int crow = P.rowbase[code + pow3(w)] + head_slot(u, ctw);
                bc[w] = Bn[(size_t)crow * RS + lam * N + w];
                a[w] = first ? 2.0 * bc[w] : bc[w];
            }
            const double tb = tbar[ri.y];
#pragma unroll
            for (int w = 0; w < N; ++w) a[w] = (w == u) ? a[w] + tb : a[w];
            const double sg = sig * (code == 1 ? 2.0 : 1.0);
            const double sc = (code == 1 ? 2.0 : 1.0);
            double b[N];
#pragma unroll
            for (int v = 0; v < N; ++v) {
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < N; ++w) s = __builtin_fma(Gr[v * N + w], a[w], s);
                b[v] = s;
                __builtin_amdgcn_sched_barrier(0);
            }
            if (A.stubs) {
#pragma unroll
                for (int w = 0; w < N; ++w) {
                    const uint32_t bit = 1u << w;
                    if ((ones & bit) && (cm & bit)) {
                        b[w] = __builtin_fma(-sg, bc[w], b[w]);
                        sacc = __builtin_fma(-sc * f[w], bc[w], sacc);
                    }
                }
            }
#pragma unroll
            for (int v = 0; v < N; ++v)
#pragma unroll
                for (int w = 0; w < N; ++w) gacc[v][w] = __builtin_fma(f[v], a[w], gacc[v][w]);
            double *__restrict__ dstb = Bc + (size_t)r * RS + lam * N;
#pragma unroll
            for (int v = 0; v < N; ++v)
                if ((cm >> v) & 1u) dstb[v] = b[v];
        }
        __syncthreads();
    }

    // ---- reduce dS/dG and dS/dsigma over the workgroup (fixed order) ----
#pragma unroll
    for (int v = 0; v < N; ++v)
#pragma unroll
        for (int w = 0; w < N; ++w) {
            double x = gacc[v][w];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
            gacc[v][w] = x;
        }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) sacc += __shfl_xor(sacc, off, 64);
    if (lane == 0) {
#pragma unroll
        for (int v = 0; v < N; ++v)
#pragma unroll
            for (int w = 0; w < N; ++w) red[wave * (N * N + 1) + v * N + w] = gacc[v][w];
        red[wave * (N * N + 1) + N * N] = sacc;
    }
    __syncthreads();
    for (int e = tid; e < nfs * (N * N + 1); e += blockDim.x) {
        const int lf = e / (N * N + 1), k = e % (N * N + 1);
        double s = 0.0;
        for (int wv = lf; wv < nwaves; wv += nfs) s += red[wv * (N * N + 1) + k];
        if (k < N * N) {
            A.G_bar[goff + (A.variant ? (int64_t)lf * N * N : 0) + k] = s;
        } else if (A.stubs && A.stub_bar) {
            A.stub_bar[(int64_t)c * A.nstub + (A.variant ? lf : 0)] = s;
        }
    }
    __syncthreads();
}

template <int N, int MAXT>
__global__ void __launch_bounds__(MAXT) adjoint_kernel(const AdjArgs A) {
    __shared__ int s_item;
    __shared__ double red[16 * (COS_NMAX * COS_NMAX + 1)];
    double *ws = A.ws + (size_t)blockIdx.x * A.ws_per_wg;
    while (true) {
        if (threadIdx.x == 0) s_item = atomicAdd(A.counter, 1);
        __syncthreads();
        const int item = COS_RF(s_item);
        __syncthreads();
        if (item >= A.nconf) break;
        const int c = COS_RF(A.order[item]);
        adj_config<N>(A, c, ws, red);
    }
}

hipError_t launch_adjoint(const AdjArgs &a, int grid, int block, hipStream_t s) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, a.counter);
    switch (a.plan.n) {
#define COS_ADJ_CASE(K)                                                                            \
    case K:                                                                                        \
        if (block <= 256) hipLaunchKernelGGL((adjoint_kernel<K, 256>), dim3(grid), dim3(block), 0, s, a); \
        else hipLaunchKernelGGL((adjoint_kernel<K, 1024>), dim3(grid), dim3(block), 0, s, a);       \
        break;
        COS_ADJ_CASE(1) COS_ADJ_CASE(2) COS_ADJ_CASE(3) COS_ADJ_CASE(4)
        COS_ADJ_CASE(5) COS_ADJ_CASE(6) COS_ADJ_CASE(7) COS_ADJ_CASE(8)
        COS_ADJ_CASE(9) COS_ADJ_CASE(10) COS_ADJ_CASE(11) COS_ADJ_CASE(12)
#undef COS_ADJ_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// free propagator (Methods, square-lattice dispersion; imaginary-time
// propagator with tau = 0 read as 0^-), one workgroup per configuration
// ---------------------------------------------------------------------------
struct G0Params {
    double mu[COS_FMAX], alpha[COS_FMAX];
    double t, beta;
    int L, nmat;
};

__global__ void __launch_bounds__(256) g0_kernel(const int32_t *__restrict__ nvec,
                                                 const int64_t *__restrict__ voff,
                                                 const int32_t *__restrict__ sites,
                                                 const double *__restrict__ tau,
                                                 const int64_t *__restrict__ Goff,
                                                 double *__restrict__ Gout, double *__restrict__ dGout,
                                                 const G0Params p) {
    extern __shared__ double sm[];
    const int L = p.L, L2 = L * L;
    double *xi = sm;            // [L2]
    double *nf = sm + L2;       // [L2]
    double *cs = sm + 2 * L2;   // [L] cos(2 pi j / L)
    const int c = blockIdx.x;
    const int n = nvec[c];
    const int64_t v0 = voff[c];
    const int64_t goff = Goff[c];
    for (int j = threadIdx.x; j < L; j += blockDim.x) cs[j] = cospi(2.0 * (double)j / (double)L);
    for (int g = 0; g < p.nmat; ++g) {
        __syncthreads();
        for (int k = threadIdx.x; k < L2; k += blockDim.x) {
            const int mx = k % L, my = k / L;
            const double e = -2.0 * p.t * (cospi(2.0 * mx / (double)L) + cospi(2.0 * my / (double)L)) -
                             p.mu[g] + p.alpha[g];
            xi[k] = e;
            // Fermi function without overflow
            nf[k] = (e >= 0.0) ? exp(-p.beta * e) / (1.0 + exp(-p.beta * e)) : 1.0 / (exp(p.beta * e) + 1.0);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
            const int a = e / n, b = e % n;
            const int dx = sites[2 * (v0 + a)] - sites[2 * (v0 + b)];
            const int dy = sites[2 * (v0 + a) + 1] - sites[2 * (v0 + b) + 1];
            const double d = tau[v0 + a] - tau[v0 + b];
            double sg = 0.0, sd = 0.0;
            for (int k = 0; k < L2; ++k) {
                const int mx = k % L, my = k / L;
                int ph = (mx * dx + my * dy) % L;
                if (ph < 0) ph += L;
                const double x = xi[k], nF = nf[k];
                double gk, dk;
                if (d > 0.0) {
                    // -exp(-x d)(1 - nF), every exponent kept non-positive
                    gk = (x >= 0.0) ? -exp(-x * d) / (1.0 + exp(-p.beta * x))
                                    : -exp(x * (p.beta - d)) / (exp(p.beta * x) + 1.0);
                    dk = gk * (p.beta * nF - d);
                } else {
                    const double s = -d;   // exp(x s) nF
                    gk = (x <= 0.0) ? exp(x * s) / (exp(p.beta * x) + 1.0)
                                    : exp(-x * (p.beta - s)) / (1.0 + exp(-p.beta * x));
                    dk = gk * (p.beta * nF - p.beta - d);
                }
                sg = __builtin_fma(cs[ph], gk, sg);
                sd = __builtin_fma(cs[ph], dk, sd);
            }
            const double inv = 1.0 / (double)L2;
            Gout[goff + (int64_t)g * n * n + e] = sg * inv;
            if (dGout) dGout[goff + (int64_t)g * n * n + e] = sd * inv;
        }
    }
}

hipError_t launch_g0(int nconf, const int32_t *n, const int64_t *voff, const int32_t *sites,
                     const double *tau, int L, double t, double beta, int nmat, const double *mu,
                     const double *alpha, const int64_t *Goff, double *G, double *dG, hipStream_t s) {
    G0Params p;
    for (int g = 0; g < COS_FMAX; ++g) {
        p.mu[g] = g < nmat ? mu[g] : 0.0;
        p.alpha[g] = g < nmat ? alpha[g] : 0.0;
    }
    p.t = t; p.beta = beta; p.L = L; p.nmat = nmat;
    const size_t shm = (size_t)(2 * L * L + L) * sizeof(double);
    hipLaunchKernelGGL(g0_kernel, dim3(nconf), dim3(256), shm, s, n, voff, sites, tau, Goff, G, dG, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// chain rule to mu and the shift, one thread per (configuration, matrix)
// ---------------------------------------------------------------------------
__global__ void chain_kernel(int nconf, const int32_t *__restrict__ nvec, int nmat,
                             const int64_t *__restrict__ Goff, const double *__restrict__ Gb,
                             const double *__restrict__ dG, const double *__restrict__ sb, int nstub,
                             double U, double *__restrict__ mub, double *__restrict__ alb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nconf * nmat) return;
    const int c = i / nmat, g = i % nmat;
    const int n = nvec[c];
    const int64_t base = Goff[c] + (int64_t)g * n * n;
    double x = 0.0;
    for (int e = 0; e < n * n; ++e) x = __builtin_fma(Gb[base + e], dG[base + e], x);
    mub[i] = -x;
    alb[i] = x + (sb ? sb[(int64_t)c * nstub + (nstub == 1 ? 0 : g)] / U : 0.0);
}

hipError_t launch_chain(int nconf, const int32_t *n, int nmat, const int64_t *Goff, const double *Gb,
                        const double *dG, const double *sb, int nstub, double U, double *mub,
                        double *alb, hipStream_t s) {
    const int tot = nconf * nmat;
    hipLaunchKernelGGL(chain_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, nconf, n, nmat, Goff, Gb,
                       dG, sb, nstub, U, mub, alb);
    return hipGetLastError();
}

}  // namespace libcos
