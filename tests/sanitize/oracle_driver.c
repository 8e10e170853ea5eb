/* Runs every routine of the C oracle on small seeded inputs, for a build with
 * the address and undefined-behaviour sanitizers (test infrastructure). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

long double cos_oracle_brute_ld(int, int, int, int, const double *, const double *, double, int);
long double cos_oracle_dp_ld(int, int, int, int, const double *, const double *, double, int64_t *);
long double cos_oracle_dp_adjoint_ld(int, int, int, int, const double *, const double *, double, long double *,
                                     long double *);
void cos_oracle_dp_subsets_ld(int, int, int, int, const double *, const double *, double, long double *);
long double cos_oracle_alg3_ld(int, int, int, int, const double *, const double *, double);
double cos_oracle_dp_d(int, int, int, int, const double *, const double *, double, int64_t *);
double cos_oracle_dp_adjoint_d(int, int, int, int, const double *, const double *, double, double *, double *);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static double uniform(void) {
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

int main(void) {
    double G[3 * 8 * 8], stub[3];
    long double gb[3 * 8 * 8], sb[3], sub[1 << 8];
    double gbd[3 * 8 * 8], sbd[3];
    int64_t counts[5];
    for (int n = 1; n <= 7; ++n) {
        for (int variant = 0; variant <= 1; ++variant) {
            const int nf = variant ? 3 : 2, nm = variant ? nf : 1;
            for (int i = 0; i < nm * n * n; ++i) G[i] = uniform();
            for (int i = 0; i < nm; ++i) stub[i] = uniform();
            for (int st = 0; st <= 1; ++st) {
                long double a = cos_oracle_dp_ld(n, nf, variant, st, G, stub, -1.0, counts);
                long double b = cos_oracle_dp_adjoint_ld(n, nf, variant, st, G, stub, -1.0, gb, sb);
                double c = cos_oracle_dp_d(n, nf, variant, st, G, stub, -1.0, NULL);
                double d = cos_oracle_dp_adjoint_d(n, nf, variant, st, G, stub, -1.0, gbd, sbd);
                cos_oracle_dp_subsets_ld(n, nf, variant, st, G, stub, -1.0, sub);
                long double e = n <= 4 ? cos_oracle_brute_ld(n, nf, variant, st, G, stub, -1.0, 1) : a;
                long double f = n <= 3 ? cos_oracle_alg3_ld(n, nf, variant, st, G, stub, -1.0) : a;
                printf("n=%d variant=%d stubs=%d dp=%.12Le adj=%.12Le d=%.12e %.12e brute=%.12Le alg3=%.12Le\n", n,
                       variant, st, a, b, c, d, e, f);
            }
        }
    }
    return 0;
}
