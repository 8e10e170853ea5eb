// Connected-determinant comparison path (Methods: fast generation of the 3^n
// principal minors by Schur complements with pseudo-pivots; connected part by
// the subset recursion) for the SU(2) bipartite model, in FP64 or in
// double-double arithmetic (two doubles per number, ~32 significant digits).
//
// One workgroup per configuration.  The 3^n labelled subsets (each vertex
// absent, on A or on B) are the leaves of a ternary tree over the vertices;
// level d holds the Schur complements of the 3^d prefixes (2(n-d) x 2(n-d)
// matrices), built breadth-first in the caller's workspace; a leaf's minor is
// the product of the pivots on its path.  A pivot below eps in magnitude is
// replaced by C = sum|A| / (2n)^2; by multilinearity the minors below it are
// then corrected by -(C - p) times the minors of the sibling subtree without
// that vertex, deepest first.  a(T) = det A_up[T] det A_dn[T];
// c(T) = a(T) - sum_{T' subset T holding T's first vertex} c(T') a(T \ T');
// out = sum of c over the 2^n full labellings.
//
// Leaf order inside the tree: vertex 0 is the most significant base-3 digit
// (digit 0 absent, 1 on A, 2 on B).
#include "cos_internal.hpp"

// The error-free transformations below require every sum and product to be
// rounded exactly as written: a product contracted into a following
// addition (FMA) breaks them once they are inlined into each other.
#pragma STDC FP_CONTRACT OFF

namespace libcos {

// ---- double-double arithmetic (Dekker / Knuth error-free transformations) ----
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
    const double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
    const double s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ dd dd_add(dd x, dd y) {
    dd s = two_sum(x.hi, y.hi);
    const dd t = two_sum(x.lo, y.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd x) { return {-x.hi, -x.lo}; }
__device__ __forceinline__ dd dd_mul(dd x, dd y) {
    const double p = x.hi * y.hi;
    double e = __builtin_fma(x.hi, y.hi, -p);   // exact low part of the product
    e += x.hi * y.lo + x.lo * y.hi;
    return quick_two_sum(p, e);
}
__device__ __forceinline__ dd dd_div(dd x, dd y) {
    // long division with three double quotient digits
    const double q1 = x.hi / y.hi;
    dd r = dd_add(x, dd_neg(dd_mul({q1, 0.0}, y)));
    const double q2 = r.hi / y.hi;
    r = dd_add(r, dd_neg(dd_mul({q2, 0.0}, y)));
    const double q3 = r.hi / y.hi;
    const dd q = quick_two_sum(q1, q2);
    return dd_add(q, {q3, 0.0});
}

// one number type interface for the kernel
template <class T>
struct Num;
template <>
struct Num<double> {
    static __device__ __forceinline__ double from(double x) { return x; }
    static __device__ __forceinline__ double add(double a, double b) { return a + b; }
    static __device__ __forceinline__ double sub(double a, double b) { return a - b; }
    static __device__ __forceinline__ double mul(double a, double b) { return a * b; }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double mag(double a) { return fabs(a); }
    static __device__ __forceinline__ double to(double a) { return a; }
};
template <>
struct Num<dd> {
    static __device__ __forceinline__ dd from(double x) { return {x, 0.0}; }
    static __device__ __forceinline__ dd add(dd a, dd b) { return dd_add(a, b); }
    static __device__ __forceinline__ dd sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
    static __device__ __forceinline__ dd mul(dd a, dd b) { return dd_mul(a, b); }
    static __device__ __forceinline__ dd div(dd a, dd b) { return dd_div(a, b); }
    static __device__ __forceinline__ double mag(dd a) { return fabs(a.hi); }
    static __device__ __forceinline__ double to(dd a) { return a.hi + a.lo; }
};

// per-configuration workspace layout (elements of T)
struct CdetLayout {
    int64_t lvl, prod, delta, minor, conn, total;
};

__host__ __device__ inline int64_t ipow3(int k) {
    int64_t r = 1;
    for (int i = 0; i < k; ++i) r *= 3;
    return r;
}

__host__ __device__ inline CdetLayout cdet_layout(int n) {
    int64_t lvl = 0;
    for (int d = 0; d <= n; ++d) {
        const int64_t m = 2 * (n - d);
        lvl = lvl > ipow3(d) * m * m ? lvl : ipow3(d) * m * m;
    }
    const int64_t N3 = ipow3(n);
    int64_t dsum = 0;
    for (int d = 1; d <= n; ++d) dsum += ipow3(d);
    CdetLayout L;
    L.lvl = 0;                     // two level buffers
    L.prod = 2 * lvl;              // two product buffers of up to 3^n
    L.delta = L.prod + 2 * N3;     // pivot shift of every node at depths 1..n (0: none)
    L.minor = L.delta + dsum;      // minors of both spins
    L.conn = L.minor + 2 * N3;     // c(T)
    L.total = L.conn + N3;
    return L;
}

template <class T>
__global__ void __launch_bounds__(256) cdet_kernel(int n, const double *__restrict__ Aall, double eps,
                                                   T *__restrict__ work, int64_t per_config,
                                                   double *__restrict__ out) {
    using X = Num<T>;
    __shared__ double red[256];
    const int c = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int D = 2 * n;
    const int64_t N3 = ipow3(n);
    const CdetLayout LY = cdet_layout(n);
    T *__restrict__ W = work + (int64_t)c * per_config;
    int64_t lvl_size = 0;
    for (int d = 0; d <= n; ++d) {
        const int64_t m = 2 * (n - d);
        lvl_size = lvl_size > ipow3(d) * m * m ? lvl_size : ipow3(d) * m * m;
    }
    T *lv[2] = {W + LY.lvl, W + LY.lvl + lvl_size};
    T *pr[2] = {W + LY.prod, W + LY.prod + N3};
    T *delta = W + LY.delta;
    T *minor[2] = {W + LY.minor, W + LY.minor + N3};
    T *conn = W + LY.conn;

    for (int sp = 0; sp < 2; ++sp) {
        const double *__restrict__ A = Aall + ((int64_t)c * 2 + sp) * D * D;
        // pseudo-pivot value: mean absolute entry
        double s = 0.0;
        for (int i = tid; i < D * D; i += nt) s += fabs(A[i]);
        red[tid] = s;
        __syncthreads();
        for (int h = nt / 2; h > 0; h >>= 1) {
            if (tid < h) red[tid] += red[tid + h];
            __syncthreads();
        }
        const double C = red[0] / (double)(D * D);
        __syncthreads();
        // depth 0: the whole matrix
        for (int i = tid; i < D * D; i += nt) lv[0][i] = X::from(A[i]);
        if (tid == 0) pr[0][0] = X::from(1.0);
        __syncthreads();
        int64_t doff = 0;   // offset of depth d + 1 inside delta
        for (int d = 0; d < n; ++d) {
            const int m = 2 * (n - d), mc = m - 2;
            const int64_t nodes = ipow3(d);
            T *cur = lv[d & 1], *nxt = lv[(d + 1) & 1];
            T *pc = pr[d & 1], *pn = pr[(d + 1) & 1];
            for (int64_t e = tid; e < nodes * 3; e += nt) {
                const int64_t node = e / 3;
                const int ch = (int)(e % 3);
                const T *M = cur + node * m * m;
                T *Mc = nxt + e * mc * mc;
                if (ch == 0) {
                    for (int i = 0; i < mc; ++i)
                        for (int j = 0; j < mc; ++j) Mc[i * mc + j] = M[(i + 2) * m + (j + 2)];
                    pn[e] = pc[node];
                    delta[doff + e] = X::from(0.0);
                } else {
                    const int q = ch - 1;   // pivot row / column 0 (A) or 1 (B)
                    T p = M[q * m + q];
                    T sh = X::from(0.0);
                    if (X::mag(p) < eps) {
                        sh = X::sub(X::from(C), p);
                        p = X::from(C);
                    }
                    for (int i = 0; i < mc; ++i) {
                        const T f = X::div(M[(i + 2) * m + q], p);
                        for (int j = 0; j < mc; ++j)
                            Mc[i * mc + j] = X::sub(M[(i + 2) * m + (j + 2)], X::mul(f, M[q * m + (j + 2)]));
                    }
                    pn[e] = X::mul(pc[node], p);
                    delta[doff + e] = sh;
                }
            }
            doff += nodes * 3;
            __syncthreads();
        }
        T *mn = minor[sp];
        T *leaf = pr[n & 1];
        for (int64_t i = tid; i < N3; i += nt) mn[i] = leaf[i];
        __syncthreads();
        // multilinearity corrections of pseudo-pivots, deepest first
        int64_t off = doff;
        for (int d = n - 1; d >= 0; --d) {
            const int64_t nodes = ipow3(d + 1);
            off -= nodes;
            const int64_t sub = ipow3(n - d - 1);
            for (int64_t e = tid; e < nodes * sub; e += nt) {
                const int64_t child = e / sub, sfx = e % sub;
                if (child % 3 == 0) continue;
                const T sh = delta[off + child];
                if (X::to(sh) == 0.0) continue;
                const int64_t sib = child - child % 3;
                mn[child * sub + sfx] = X::sub(mn[child * sub + sfx], X::mul(sh, mn[sib * sub + sfx]));
            }
            __syncthreads();
        }
    }
    // connected parts, by number of present vertices
    for (int k = 1; k <= n; ++k) {
        for (int64_t code = tid; code < N3; code += nt) {
            int dg[kSubNmax], pres[kSubNmax], np = 0;
            int64_t x = code;
            for (int v = n - 1; v >= 0; --v) {   // vertex v has weight 3^(n-1-v)
                dg[v] = (int)(x % 3);
                x /= 3;
            }
            for (int v = 0; v < n; ++v)
                if (dg[v]) pres[np++] = v;
            if (np != k) continue;
            T a = X::mul(minor[0][code], minor[1][code]);
            // proper subsets holding the first present vertex
            const int rest = np - 1;
            for (int mask = 0; mask < (1 << rest) - 1; ++mask) {
                int64_t sub = 0;
                for (int i = 0; i < np; ++i) {
                    const int v = pres[i];
                    const bool keep = i == 0 || ((mask >> (i - 1)) & 1);
                    if (keep) sub += dg[v] * ipow3(n - 1 - v);
                }
                const T ar = X::mul(minor[0][code - sub], minor[1][code - sub]);
                a = X::sub(a, X::mul(conn[sub], ar));
            }
            conn[code] = a;
        }
        __syncthreads();
    }
    if (tid == 0) {
        // sum over the 2^n full labellings, fixed order
        T tot = X::from(0.0);
        for (int lab = 0; lab < (1 << n); ++lab) {
            int64_t code = 0;
            for (int v = 0; v < n; ++v) code = code * 3 + 1 + ((lab >> v) & 1);
            tot = X::add(tot, conn[code]);
        }
        out[c] = X::to(tot);
    }
}

int64_t cdet_elems_per_config(int n) { return cdet_layout(n).total; }

hipError_t launch_cdet(int nconf, int n, const double *A, int precision, double eps, void *work,
                       double *out, hipStream_t s) {
    const int64_t per = cdet_layout(n).total;
    if (precision == 0)
        hipLaunchKernelGGL(cdet_kernel<double>, dim3(nconf), dim3(256), 0, s, n, A, eps, (double *)work, per, out);
    else
        hipLaunchKernelGGL(cdet_kernel<dd>, dim3(nconf), dim3(256), 0, s, n, A, eps, (dd *)work, per, out);
    return hipGetLastError();
}

}  // namespace libcos
