// HIP kernels for gfx950 (CDNA4): the free-propagator builder and the chain
// rule to (mu, shift).  The dynamic-programme kernels are in cos_level.hip.
#include "cos_internal.hpp"

namespace libcos {

// ---------------------------------------------------------------------------
// free propagator (Methods, square-lattice dispersion; imaginary-time
// propagator with tau = 0 read as 0^-), one workgroup per configuration
// ---------------------------------------------------------------------------
// 128 threads: the n^2 <= 144 entries of a configuration in one or two passes
constexpr int kG0Threads = 128;

struct G0Params {
    double mu[COS_FMAX], alpha[COS_FMAX];
    double t, beta;
    int L, nmat;
};

// Per momentum k the propagator term is -e^{-xi d} (1 - n_F) for d > 0 and
// e^{xi s} n_F for d = -s <= 0.  Written with every exponent non-positive,
// each case is +-exp(E) R_k with R_k = 1 / (1 + e^{-beta |xi_k|}) (the same
// factor for both signs of xi) and E one of -xi d, xi (beta - d), xi s or
// -xi (beta - s): one exponential per term, R_k shared by the entries.
// dG/dxi follows from the same term: g (beta n_F - d), resp. g (beta n_F -
// beta - d).  The phase index (k . dx) mod L advances by dx mod L per step.
__global__ void __launch_bounds__(kG0Threads) g0_kernel(const int32_t *__restrict__ nvec,
                                                        const int64_t *__restrict__ voff,
                                                        const int32_t *__restrict__ sites,
                                                        const double *__restrict__ tau,
                                                        const int64_t *__restrict__ Goff,
                                                        double *__restrict__ Gout, double *__restrict__ dGout,
                                                        const G0Params p) {
    extern __shared__ double sm[];
    const int L = p.L, L2 = L * L;
    double *xi = sm;            // [L2]
    double *nf = sm + L2;       // [L2] n_F(xi)
    double *rk = sm + 2 * L2;   // [L2] 1 / (1 + e^{-beta |xi|})
    double *cs = sm + 3 * L2;   // [L] cos(2 pi j / L)
    const int c = blockIdx.x;
    const int n = nvec[c];
    const int64_t v0 = voff[c];
    const int64_t goff = Goff[c];
    const double beta = p.beta;
    for (int j = threadIdx.x; j < L; j += blockDim.x) cs[j] = cospi(2.0 * (double)j / (double)L);
    for (int g = 0; g < p.nmat; ++g) {
        __syncthreads();
        for (int k = threadIdx.x; k < L2; k += blockDim.x) {
            const int mx = k % L, my = k / L;
            const double e = -2.0 * p.t * (cospi(2.0 * mx / (double)L) + cospi(2.0 * my / (double)L)) -
                             p.mu[g] + p.alpha[g];
            const double q = exp(-beta * fabs(e)), r = 1.0 / (1.0 + q);
            xi[k] = e;
            rk[k] = r;
            nf[k] = (e >= 0.0) ? q * r : r;   // Fermi function without overflow
        }
        __syncthreads();
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
            const int a = e / n, b = e % n;
            int dx = (sites[2 * (v0 + a)] - sites[2 * (v0 + b)]) % L;
            int dy = (sites[2 * (v0 + a) + 1] - sites[2 * (v0 + b) + 1]) % L;
            dx += dx < 0 ? L : 0;
            dy += dy < 0 ? L : 0;
            const double d = tau[v0 + a] - tau[v0 + b];
            const bool fwd = d > 0.0;
            // exponent coefficients for xi >= 0 and xi < 0, sign, dG offset
            const double cpos = fwd ? -d : -(beta + d), cneg = fwd ? beta - d : -d;
            const double sgn = fwd ? -1.0 : 1.0, doff = fwd ? -d : -beta - d;
            double sg = 0.0, sd = 0.0;
            int phy = 0;
            for (int my = 0, k = 0; my < L; ++my) {
                int ph = phy;
                for (int mx = 0; mx < L; ++mx, ++k) {
                    const double x = xi[k];
                    const double gk = sgn * exp(x * (x >= 0.0 ? cpos : cneg)) * rk[k];
                    const double dk = gk * __builtin_fma(beta, nf[k], doff);
                    sg = __builtin_fma(cs[ph], gk, sg);
                    sd = __builtin_fma(cs[ph], dk, sd);
                    ph += dx;
                    ph -= ph >= L ? L : 0;
                }
                phy += dy;
                phy -= phy >= L ? L : 0;
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
    const size_t shm = (size_t)(3 * L * L + L) * sizeof(double);
    hipLaunchKernelGGL(g0_kernel, dim3(nconf), dim3(kG0Threads), shm, s, n, voff, sites, tau, Goff, G, dG, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// free propagator of the honeycomb lattice (Methods, honeycomb Bloch
// Hamiltonian): per flavour H(k) = [[Delta - (mu - alpha), eps], [eps*,
// -Delta - (mu - alpha)]], eps(k) = -t (1 + e^{i k.b1} + e^{i k.b2}).  With
// H = d0 + d.sigma, |d| = r: f(H) = (f(d0 + r) + f(d0 - r)) / 2 + (f(d0 + r) -
// f(d0 - r)) / 2 * d.sigma / r, so per k two eigenvalues and the unit vector
// d / r (in LDS) give every sublattice entry.  One workgroup per
// configuration; thread per vertex pair, four sublattice entries each.
// dG/dxi for a uniform move H -> H + xi (xi = -(mu - alpha)) shifts both
// eigenvalues and keeps d / r, so it is the same sum with f replaced by f'.
// ---------------------------------------------------------------------------
struct HcParams {
    double mu[COS_FMAX], alpha[COS_FMAX], delta[COS_FMAX];
    double t, beta;
    int L, nmat;
};

// Fermi function without overflow
__device__ __forceinline__ double fermi(double x, double beta) {
    return (x >= 0.0) ? exp(-beta * x) / (1.0 + exp(-beta * x)) : 1.0 / (exp(beta * x) + 1.0);
}

// imaginary-time factor of one eigenvalue x with Fermi factor nF for the time
// difference d, as in g0_kernel: +-exp(E) R with every exponent E non-positive
// and R = 1 / (1 + e^{-beta |x|}) = (x >= 0 ? 1 - nF : nF); cpos, cneg and sgn
// are the entry's exponent coefficients and sign.
__device__ __forceinline__ double g0_branch(double x, double nF, double cpos, double cneg, double sgn) {
    const bool pos = x >= 0.0;
    return sgn * exp(x * (pos ? cpos : cneg)) * (pos ? 1.0 - nF : nF);
}

__global__ void __launch_bounds__(kG0Threads) g0_honeycomb_kernel(const int32_t *__restrict__ nvec,
                                                                  const int64_t *__restrict__ voff,
                                                                  const int32_t *__restrict__ cells,
                                                                  const double *__restrict__ tau,
                                                                  const int64_t *__restrict__ Goff,
                                                                  double *__restrict__ Gout,
                                                                  double *__restrict__ dGout, const HcParams p) {
    extern __shared__ double sm[];
    const int L = p.L, L2 = L * L;
    double *ep = sm, *em = sm + L2, *rz = sm + 2 * L2, *ex = sm + 3 * L2, *ey = sm + 4 * L2;
    double *np_ = sm + 5 * L2, *nm_ = sm + 6 * L2;   // Fermi factors of the two eigenvalues
    double *cs = sm + 7 * L2, *sn = cs + L;   // cos / sin (2 pi j / L)
    const int c = blockIdx.x;
    const int n = nvec[c];
    const int64_t v0 = voff[c];
    const int64_t goff = Goff[c];
    const int D = 2 * n;
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        cs[j] = cospi(2.0 * (double)j / (double)L);
        sn[j] = sinpi(2.0 * (double)j / (double)L);
    }
    for (int g = 0; g < p.nmat; ++g) {
        __syncthreads();
        for (int k = threadIdx.x; k < L2; k += blockDim.x) {
            const int m1 = k % L, m2 = k / L;
            const double er = -p.t * (1.0 + cospi(2.0 * m1 / (double)L) + cospi(2.0 * m2 / (double)L));
            const double ei = -p.t * (sinpi(2.0 * m1 / (double)L) + sinpi(2.0 * m2 / (double)L));
            const double d0 = -(p.mu[g] - p.alpha[g]), dz = p.delta[g];
            const double r = sqrt(er * er + ei * ei + dz * dz);
            ep[k] = d0 + r;
            em[k] = d0 - r;
            np_[k] = fermi(d0 + r, p.beta);
            nm_[k] = fermi(d0 - r, p.beta);
            const double inv = r > 0.0 ? 1.0 / r : 0.0;   // r = 0: both eigenvalues equal, f(H) = f(d0)
            rz[k] = dz * inv;
            ex[k] = er * inv;
            ey[k] = ei * inv;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
            const int a = e / n, b = e % n;
            int r1 = (cells[2 * (v0 + a)] - cells[2 * (v0 + b)]) % L;
            int r2 = (cells[2 * (v0 + a) + 1] - cells[2 * (v0 + b) + 1]) % L;
            r1 += r1 < 0 ? L : 0;
            r2 += r2 < 0 ? L : 0;
            const double d = tau[v0 + a] - tau[v0 + b], beta = p.beta;
            const bool fwd = d > 0.0;
            const double cpos = fwd ? -d : -(beta + d), cneg = fwd ? beta - d : -d, sgn = fwd ? -1.0 : 1.0;
            // d/dx of the branch factor: d > 0: f (beta nF - d); d <= 0: f (beta nF - beta - d)
            const double dsh = fwd ? -d : -beta - d;
            double acc[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};   // [G, dG/dxi][aa, bb, ab, ba]
            int ph2 = 0;   // (m1 r1 + m2 r2) mod L, advanced step by step
            for (int m2 = 0, k = 0; m2 < L; ++m2) {
                int ph = ph2;
                for (int m1 = 0; m1 < L; ++m1, ++k) {
                    const double c0 = cs[ph], s0 = sn[ph];
                    ph += r1;
                    ph -= ph >= L ? L : 0;
                    const double gp = g0_branch(ep[k], np_[k], cpos, cneg, sgn);
                    const double gm = g0_branch(em[k], nm_[k], cpos, cneg, sgn);
                    const double fpv[2] = {gp, gp * __builtin_fma(beta, np_[k], dsh)};
                    const double fmv[2] = {gm, gm * __builtin_fma(beta, nm_[k], dsh)};
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        if (q == 1 && !dGout) break;
                        const double S = 0.5 * (fpv[q] + fmv[q]), Dd = 0.5 * (fpv[q] - fmv[q]);
                        acc[q][0] = __builtin_fma(c0, __builtin_fma(Dd, rz[k], S), acc[q][0]);
                        acc[q][1] = __builtin_fma(c0, __builtin_fma(-Dd, rz[k], S), acc[q][1]);
                        // Re[e^{i phi} Dd (ex + i ey)] and Re[e^{i phi} Dd (ex - i ey)]
                        const double xr = Dd * ex[k], xi = Dd * ey[k];
                        acc[q][2] = __builtin_fma(c0, xr, __builtin_fma(-s0, xi, acc[q][2]));
                        acc[q][3] = __builtin_fma(c0, xr, __builtin_fma(s0, xi, acc[q][3]));
                    }
                }
                ph2 += r2;
                ph2 -= ph2 >= L ? L : 0;
            }
            const double inv = 1.0 / (double)L2;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                double *base = q == 0 ? Gout : dGout;
                if (!base) continue;
                double *out = base + goff + (int64_t)g * D * D;
                out[(2 * a) * D + 2 * b] = acc[q][0] * inv;
                out[(2 * a) * D + 2 * b + 1] = acc[q][2] * inv;
                out[(2 * a + 1) * D + 2 * b] = acc[q][3] * inv;
                out[(2 * a + 1) * D + 2 * b + 1] = acc[q][1] * inv;
            }
        }
    }
}

hipError_t launch_g0_honeycomb(int nconf, const int32_t *n, const int64_t *voff, const int32_t *cells,
                               const double *tau, int L, double t, double beta, int nmat, const double *mu,
                               const double *alpha, const double *delta, const int64_t *Goff, double *G,
                               double *dG, hipStream_t s) {
    HcParams p;
    for (int g = 0; g < COS_FMAX; ++g) {
        p.mu[g] = g < nmat ? mu[g] : 0.0;
        p.alpha[g] = g < nmat ? alpha[g] : 0.0;
        p.delta[g] = g < nmat ? delta[g] : 0.0;
    }
    p.t = t; p.beta = beta; p.L = L; p.nmat = nmat;
    const size_t shm = (size_t)(7 * L * L + 2 * L) * sizeof(double);
    hipLaunchKernelGGL(g0_honeycomb_kernel, dim3(nconf), dim3(kG0Threads), shm, s, n, voff, cells, tau, Goff, G, dG, p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// chain rule to mu and the shift: x = sum_jk dS/dG[j][k] dG/dxi[j][k] per
// (configuration, matrix), mu_bar = -x, alpha_bar = x + sigma_bar / U.  One
// wavefront per (configuration, matrix): the lanes read the n^2 entries
// coalesced and a butterfly over the 64 lanes sums their partial products
// (a fixed order, so repeated calls agree bit for bit).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) chain_kernel(int nconf, const int32_t *__restrict__ nvec, int nmat,
                                                    const int64_t *__restrict__ Goff, const double *__restrict__ Gb,
                                                    const double *__restrict__ dG, const double *__restrict__ sb,
                                                    int nstub, double U, double *__restrict__ mub,
                                                    double *__restrict__ alb) {
    const int lane = threadIdx.x & 63;
    const int64_t nw = (int64_t)nconf * nmat, stride = (int64_t)gridDim.x * (blockDim.x >> 6);
    // wid is uniform in a wavefront: whole wavefronts leave the loop together
    for (int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; wid < nw; wid += stride) {
        const int c = (int)(wid / nmat), g = (int)(wid % nmat);
        const int n = nvec[c];
        const int64_t base = Goff[c] + (int64_t)g * n * n;
        double x = 0.0;
        for (int e = lane; e < n * n; e += 64) x = __builtin_fma(Gb[base + e], dG[base + e], x);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) {
            mub[wid] = -x;
            alb[wid] = x + (sb ? sb[(int64_t)c * nstub + (nstub == 1 ? 0 : g)] / U : 0.0);
        }
    }
}

hipError_t launch_chain(int nconf, const int32_t *n, int nmat, const int64_t *Goff, const double *Gb,
                        const double *dG, const double *sb, int nstub, double U, double *mub,
                        double *alb, hipStream_t s) {
    const int64_t blocks = ((int64_t)nconf * nmat + 3) / 4;   // four wavefronts per workgroup
    hipLaunchKernelGGL(chain_kernel, dim3((unsigned)std::min<int64_t>(blocks, 1 << 20)), dim3(256), 0, s, nconf, n,
                       nmat, Goff, Gb, dG, sb, nstub, U, mub, alb);
    return hipGetLastError();
}

}  // namespace libcos
