// Monte Carlo support around the batched connected sum: device sampling of
// vertex configurations and moment accumulation of the sampled sums (the
// series coefficients are integrals over vertex positions and times of the
// connected sums; Methods, diagrammatic expansion; Results, Padé analysis).
#include "cos_internal.hpp"

namespace libcos {

// counter-based generator: the splitmix64 output function (Steele, Lea and
// Flood, "Fast splittable pseudorandom number generators", 2014) applied to
// seed + golden * (counter + 1)
__device__ __forceinline__ uint64_t mix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (counter + 1ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// vertex 0 of every configuration at cell/site (0, 0), time 0; vertices
// 1..n-1 uniform over the L x L sites and [0, beta).  Counter of component q
// (0: site, 1: time) of vertex k of configuration (first + c): ((first + c) *
// n + k) * 2 + q.  Site = high 32 bits * L^2 >> 32 (multiply-shift, exact
// range), time = beta * (53 high bits) / 2^53.
__global__ void mc_sample_kernel(int nconf, int n, int L, double beta, uint64_t seed, int64_t first,
                                 int32_t *__restrict__ sites, double *__restrict__ tau) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nconf * n) return;
    const int64_t c = i / n;
    const int k = (int)(i % n);
    if (k == 0) {
        sites[2 * i] = 0;
        sites[2 * i + 1] = 0;
        tau[i] = 0.0;
        return;
    }
    const uint64_t ctr = ((uint64_t)(first + c) * (uint64_t)n + (uint64_t)k) * 2ull;
    const uint64_t zs = mix64(seed, ctr), zt = mix64(seed, ctr + 1ull);
    const uint64_t L2 = (uint64_t)L * (uint64_t)L;
    const uint32_t site = (uint32_t)(((zs >> 32) * L2) >> 32);
    sites[2 * i] = (int32_t)(site % (uint32_t)L);
    sites[2 * i + 1] = (int32_t)(site / (uint32_t)L);
    tau[i] = beta * ((double)(zt >> 11) * 0x1.0p-53);
}

// acc[0] += sum x, acc[1] += sum x^2 over count values, one workgroup, fixed
// summation order (deterministic)
__global__ void __launch_bounds__(1024) moments_kernel(int count, const double *__restrict__ x,
                                                       double *__restrict__ acc) {
    __shared__ double s1[1024], s2[1024];
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) {
        const double v = x[i];
        a += v;
        b = __builtin_fma(v, v, b);
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s1[threadIdx.x] += s1[threadIdx.x + h];
            s2[threadIdx.x] += s2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        acc[0] += s1[0];
        acc[1] += s2[0];
    }
}

hipError_t launch_mc_sample(int nconf, int n, int L, double beta, uint64_t seed, int64_t first, int32_t *sites,
                            double *tau, hipStream_t s) {
    const int64_t tot = (int64_t)nconf * n;
    hipLaunchKernelGGL(mc_sample_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, nconf, n, L, beta,
                       seed, first, sites, tau);
    return hipGetLastError();
}

hipError_t launch_moments(int count, const double *x, double *acc, hipStream_t s) {
    hipLaunchKernelGGL(moments_kernel, dim3(1), dim3(1024), 0, s, count, x, acc);
    return hipGetLastError();
}

}  // namespace libcos
