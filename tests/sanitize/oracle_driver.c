/* Host sanitizer driver for the oracle (test infrastructure).  Built with
 * AddressSanitizer and UndefinedBehaviorSanitizer together with
 * oracle/mfm_oracle.c by tests/test_host_sanitizers.py; runs every exported
 * stage of the oracle on small sets (periodic and open boxes, bucket grid and
 * brute-force search, both schemes, the optional limiters, the levelled
 * fluxes) and the argument errors, and prints one checksum line. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double gamma;
    double n_ngb;
    double box[3];
    int32_t periodic[3];
    double beta;
    double cond_max;
    double cell;
    int32_t scheme;
    int32_t limiter;
    double beta_min;
    double cond_lo, cond_hi;
} or_params;

int or_solve_h(const or_params *p, int64_t n, const double *x, const double *y, const double *z,
               const uint8_t *mask, double *H, double *nk, double *V, int64_t *iters);
int or_gradients(const or_params *p, int64_t n, const double *x, const double *y, const double *z,
                 const double *m, const double *vx, const double *vy, const double *vz, const double *u,
                 const double *H, const double *nk, const double *V, const uint8_t *mask, double *B,
                 double *rho, double *P, double *grad, double *grad_raw, double *alpha, double *cond,
                 int64_t *n_illcond);
int or_fluxes_levels(const or_params *p, int64_t n, const double *x, const double *y, const double *z,
                     const double *vx, const double *vy, const double *vz, const double *H, const double *V,
                     const double *B, const double *rho, const double *P, const double *grad,
                     const uint8_t *mask, double hmax, double *dp, double *dE, double *vsig, int64_t *counts,
                     double *dm, const int64_t *bins, int64_t lmin, int64_t nlev, double *lev);
int or_fluxes(const or_params *p, int64_t n, const double *x, const double *y, const double *z,
              const double *vx, const double *vy, const double *vz, const double *H, const double *V,
              const double *B, const double *rho, const double *P, const double *grad, const uint8_t *mask,
              double hmax, double *dp, double *dE, double *vsig, int64_t *counts, double *dm);
double or_pair_limit(double f, double pk, double po);
double or_limiter_beta(const or_params *p, double kappa);
double or_kernel_W(double r, double H);

/* a plain 64-bit LCG for the jitter: input generation only */
static uint64_t lcg_state = 88172645463325252ull;
static double uniform(void)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

static double checksum = 0.0;

static int run_set(const char *name, int64_t n, const double *x, const double *y, const double *z,
                   or_params p)
{
    double *m = calloc(n, 8), *vx = calloc(n, 8), *vy = calloc(n, 8), *vz = calloc(n, 8), *u = calloc(n, 8);
    double *H = calloc(n, 8), *nk = calloc(n, 8), *V = calloc(n, 8), *B = calloc(6 * n, 8);
    double *rho = calloc(n, 8), *P = calloc(n, 8), *grad = calloc(15 * n, 8), *graw = calloc(15 * n, 8);
    double *alpha = calloc(5 * n, 8), *cond = calloc(n, 8), *dp = calloc(3 * n, 8), *dE = calloc(n, 8);
    double *vsig = calloc(n, 8), *dm = calloc(n, 8);
    int64_t *bins = calloc(n, 8);
    double *lev = calloc(3 * 5 * n, 8);
    uint8_t *mask = calloc(n, 1);
    int64_t *iters = calloc(n, 8), ill = 0, counts[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; i++) {
        m[i] = 1.0 / (double)n;
        vx[i] = 0.3 * sin(6.28318530717958648 * y[i]);
        vy[i] = 0.2 * cos(6.28318530717958648 * z[i]);
        vz[i] = 0.1 * (uniform() - 0.5);
        u[i] = 1.0 + 0.5 * uniform();
        bins[i] = i % 3;
        mask[i] = (uint8_t)(i % 2);
    }
    int rc = or_solve_h(&p, n, x, y, z, NULL, H, nk, V, iters);
    if (rc == 0) rc = or_gradients(&p, n, x, y, z, m, vx, vy, vz, u, H, nk, V, NULL, B, rho, P, grad, graw,
                                   alpha, cond, &ill);
    double hmax = 0.0;
    for (int64_t i = 0; rc == 0 && i < n; i++) hmax = H[i] > hmax ? H[i] : hmax;
    for (int scheme = 0; rc == 0 && scheme < 2; scheme++) {
        for (int lim = 0; rc == 0 && lim < 2; lim++) {
            or_params q = p;
            q.scheme = scheme;
            q.limiter = lim;
            rc = or_gradients(&q, n, x, y, z, m, vx, vy, vz, u, H, nk, V, NULL, B, rho, P, grad, NULL, NULL,
                              NULL, &ill);
            if (rc == 0) rc = or_fluxes(&q, n, x, y, z, vx, vy, vz, H, V, B, rho, P, grad, NULL, hmax, dp, dE,
                                        vsig, counts, scheme ? dm : NULL);
            for (int64_t i = 0; rc == 0 && i < n; i++) checksum += dp[i] + dE[i] + vsig[i];
        }
    }
    /* masked passes and the levelled fluxes over three levels, lmin 1 */
    if (rc == 0) rc = or_solve_h(&p, n, x, y, z, mask, H, nk, V, iters);
    if (rc == 0) rc = or_fluxes_levels(&p, n, x, y, z, vx, vy, vz, H, V, B, rho, P, grad, mask, hmax, dp, dE,
                                       vsig, counts, NULL, bins, 1, 3, lev);
    for (int64_t i = 0; rc == 0 && i < 15 * n; i++) checksum += lev[i];
    printf("%s: n=%lld rc=%d pairs=%lld\n", name, (long long)n, rc, (long long)counts[0]);
    free(m); free(vx); free(vy); free(vz); free(u); free(H); free(nk); free(V); free(B); free(rho); free(P);
    free(grad); free(graw); free(alpha); free(cond); free(dp); free(dE); free(vsig); free(dm); free(bins);
    free(lev); free(mask); free(iters);
    return rc;
}

int main(void)
{
    or_params p;
    memset(&p, 0, sizeof p);
    p.gamma = 5.0 / 3.0;
    p.n_ngb = 32.0;
    p.box[0] = p.box[1] = p.box[2] = 1.0;
    p.periodic[0] = p.periodic[1] = p.periodic[2] = 1;
    p.beta = 1.0;
    p.cond_max = 1e6;
    p.beta_min = 0.5;
    p.cond_lo = 10.0;
    p.cond_hi = 1000.0;
    const int side = 7;
    const int64_t n = (int64_t)side * side * side;
    double *x = malloc(n * 8), *y = malloc(n * 8), *z = malloc(n * 8);
    int64_t k = 0;
    for (int a = 0; a < side; a++)
        for (int b = 0; b < side; b++)
            for (int c = 0; c < side; c++, k++) {
                x[k] = (a + 0.5 + 0.4 * (uniform() - 0.5)) / side;
                y[k] = (b + 0.5 + 0.4 * (uniform() - 0.5)) / side;
                z[k] = (c + 0.5 + 0.4 * (uniform() - 0.5)) / side;
            }
    int bad = 0;
    or_params q = p;
    q.cell = 0.0;
    bad |= run_set("periodic, brute force", n, x, y, z, q) != 0;
    q.cell = 0.3;
    bad |= run_set("periodic, bucket grid", n, x, y, z, q) != 0;
    q.periodic[0] = q.periodic[1] = q.periodic[2] = 0;
    bad |= run_set("open box, bucket grid", n, x, y, z, q) != 0;
    /* a lone particle in a periodic box: the minimum-image error, no crash */
    double one[1] = {0.5}, H1[1] = {0.0}, nk1[1], V1[1];
    int64_t it1[1];
    const int rc1 = or_solve_h(&p, 1, one, one, one, NULL, H1, nk1, V1, it1);
    printf("lone particle: rc=%d\n", rc1);
    bad |= rc1 == 0;
    /* an empty set */
    bad |= or_solve_h(&p, 0, x, y, z, NULL, H1, nk1, V1, it1) != 0;
    for (int i = 0; i < 64; i++) {
        checksum += or_pair_limit(4.0 * uniform() - 2.0, uniform(), 2.0 * uniform() - 0.5);
        checksum += or_limiter_beta(&p, pow(10.0, 4.0 * uniform()));
        checksum += or_kernel_W(uniform(), 0.7);
    }
    printf("checksum %.17g\n", checksum);
    free(x); free(y); free(z);
    return bad ? 1 : 0;
}
