/*
 * Plain single-threaded FP64 oracle of the MFM (meshless finite-mass) hydro pass.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP path; the two meet only at the seeded
 * input generators.
 *
 * The release paper (Hopkins 2017, "A New Public Release of the GIZMO Code")
 * names the method only: a Lagrangian mesh-free finite-volume Godunov scheme
 * whose mesh moves with the fluid (abstract; section "Arbitrary (Moving)
 * Meshes"; the Hydrodynamics item of section 2).  The formulas below are the
 * standard meshless finite-mass discretisation that sentence points to, taken
 * as the numbered readings R1..R16 below (the GPU library's header marks its
 * calls with the same labels):
 *
 *   R1  cubic-spline kernel with support radius H
 *   R2  gather set r < H_i (self included), flux set r < max(H_i, H_j)
 *   R3/R4  neighbour-number equation (4 pi / 3) H^3 n(H) = N_ngb, unique root
 *   R5  V = 1/n, rho = m n, P = (gamma-1) rho u
 *   R6/R7  partition weights psi = W V, gradient matrix E, B = E^-1
 *   R8  least-squares gradients, R10 per-particle Barth-Jespersen limiter
 *   R9  effective faces A_ij, R11 midpoint face, R12 linear reconstruction
 *   R13 face frame moving with the mean particle velocity
 *   R14 HLLC star state with Davis wave speeds, R15 zero-mass-flux MFM flux
 *   R16 antisymmetric accumulation, each unordered pair in canonical order
 *   MFV (the other mesh-free Godunov form that section 2 lists, with the
 *   moving faces of section 4): faces move with the frame of R13 and the
 *   full HLLC flux of mass, momentum and energy crosses them
 *
 * Everything is written as plain loops over an explicit neighbour search
 * (brute force, or a uniform bucket grid that the tests pin against brute
 * force).  Compiled with -O2 -ffp-contract=off and no fast-math, single-
 * threaded; a second build with -fopenmp shares the per-particle loops out
 * over threads (each particle's arithmetic is the same, so are the results).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_E_INVALID (-1)
#define OR_E_NOCONV (-3)
#define OR_E_ILLCOND (-4)
#define OR_E_MINIMAGE (-5)
#define OR_E_NOMEM (-8)

typedef struct {
    double gamma;
    double n_ngb;
    double box[3];
    int32_t periodic[3];
    double beta;      /* limiter constant (R10) */
    double cond_max;  /* flag threshold on ||E||_F ||B||_F (R7) */
    double cell;      /* bucket grid cell size; <= 0 selects brute force */
    int32_t scheme;   /* 0: meshless finite mass (R15), 1: meshless finite volume */
    int32_t limiter;  /* 0: per-particle limiter only (R10); 1: + pairwise face limiter (R23)
                         and a condition-adaptive beta (R24) */
    double beta_min;  /* R24: beta at cond(E) >= cond_hi (beta itself applies at <= cond_lo) */
    double cond_lo, cond_hi;
} or_params;

/* threads a pass uses: 1, or the OpenMP team size of an OpenMP build */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* R1: cubic spline, support radius H.  W = 8/(pi H^3) w(r/H).          */
/* ------------------------------------------------------------------ */
static double spline_w(double q)
{
    if (q <= 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    if (q <= 1.0) { double t = 1.0 - q; return 2.0 * t * t * t; }
    return 0.0;
}

static double spline_dw(double q)
{
    if (q <= 0.5) return -12.0 * q + 18.0 * q * q;
    if (q <= 1.0) { double t = 1.0 - q; return -6.0 * t * t; }
    return 0.0;
}

double or_kernel_W(double r, double H)
{
    return 8.0 / (M_PI * H * H * H) * spline_w(r / H);
}

/* d W(r,H) / d H at fixed r */
double or_kernel_dWdH(double r, double H)
{
    double q = r / H;
    double W = 8.0 / (M_PI * H * H * H) * spline_w(q);
    return -(3.0 * W + q * 8.0 / (M_PI * H * H * H) * spline_dw(q)) / H;
}

/* ------------------------------------------------------------------ */
/* Neighbour search: minimum image on periodic axes; brute force or a   */
/* bucket grid.  Membership is always the strict test r < R.           */
/* ------------------------------------------------------------------ */
typedef struct { int64_t j; double d[3]; double r; } nbr_t;
typedef struct { nbr_t *a; int64_t n, cap; } nbr_list;

static int list_push(nbr_list *L, int64_t j, const double d[3], double r)
{
    if (L->n == L->cap) {
        int64_t c = L->cap ? 2 * L->cap : 256;
        nbr_t *p = (nbr_t *)realloc(L->a, (size_t)c * sizeof(nbr_t));
        if (!p) return OR_E_NOMEM;
        L->a = p;
        L->cap = c;
    }
    L->a[L->n].j = j;
    L->a[L->n].d[0] = d[0];
    L->a[L->n].d[1] = d[1];
    L->a[L->n].d[2] = d[2];
    L->a[L->n].r = r;
    L->n++;
    return OR_OK;
}

typedef struct {
    const or_params *p;
    int64_t n;
    const double *x, *y, *z;
    int brute;
    int32_t nc[3];
    double cs[3];
    int64_t *head;   /* first particle of each bucket, -1 if empty */
    int64_t *next;   /* next particle in the same bucket */
} grid_t;

/* displacement x_j - x_i along one axis, wrapped to the nearest image */
static double min_image(double dx, double L, int periodic)
{
    if (periodic) {
        if (dx > 0.5 * L) dx -= L;
        else if (dx < -0.5 * L) dx += L;
    }
    return dx;
}

static int bucket_of(const grid_t *g, int a, double xa)
{
    int c = (int)floor(xa / g->cs[a]);
    if (c < 0) c = 0;
    if (c >= g->nc[a]) c = g->nc[a] - 1;
    return c;
}

static int grid_build(grid_t *g, const or_params *p, int64_t n,
                      const double *x, const double *y, const double *z)
{
    memset(g, 0, sizeof(*g));
    g->p = p;
    g->n = n;
    g->x = x;
    g->y = y;
    g->z = z;
    g->brute = !(p->cell > 0.0);
    if (g->brute) return OR_OK;
    int64_t tot = 1;
    for (int a = 0; a < 3; a++) {
        int64_t k = (int64_t)floor(p->box[a] / p->cell);
        if (k < 1) k = 1;
        if (k > 1024) k = 1024;
        g->nc[a] = (int32_t)k;
        g->cs[a] = p->box[a] / (double)k;
        tot *= k;
    }
    g->head = (int64_t *)malloc((size_t)tot * sizeof(int64_t));
    g->next = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!g->head || !g->next) return OR_E_NOMEM;
    for (int64_t c = 0; c < tot; c++) g->head[c] = -1;
    /* insert in decreasing index so that every bucket lists increasing indices */
    for (int64_t i = n - 1; i >= 0; i--) {
        int64_t c = ((int64_t)bucket_of(g, 0, x[i]) * g->nc[1] + bucket_of(g, 1, y[i])) * g->nc[2]
                    + bucket_of(g, 2, z[i]);
        g->next[i] = g->head[c];
        g->head[c] = i;
    }
    return OR_OK;
}

static void grid_free(grid_t *g)
{
    free(g->head);
    free(g->next);
    g->head = g->next = NULL;
}

static int try_pair(const grid_t *g, int64_t i, int64_t j, double R, nbr_list *out)
{
    const or_params *p = g->p;
    double d[3];
    d[0] = min_image(g->x[j] - g->x[i], p->box[0], p->periodic[0]);
    d[1] = min_image(g->y[j] - g->y[i], p->box[1], p->periodic[1]);
    d[2] = min_image(g->z[j] - g->z[i], p->box[2], p->periodic[2]);
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (r < R) return list_push(out, j, d, r);
    return OR_OK;
}

/* all j (self included) with r_ij < R; R must stay below half of every periodic side */
static int grid_find(const grid_t *g, int64_t i, double R, nbr_list *out)
{
    const or_params *p = g->p;
    out->n = 0;
    for (int a = 0; a < 3; a++)
        if (p->periodic[a] && !(R < 0.5 * p->box[a])) return OR_E_MINIMAGE;
    if (g->brute) {
        for (int64_t j = 0; j < g->n; j++) {
            int rc = try_pair(g, i, j, R, out);
            if (rc) return rc;
        }
        return OR_OK;
    }
    double xi[3] = {g->x[i], g->y[i], g->z[i]};
    int lo[3], cnt[3];
    for (int a = 0; a < 3; a++) {
        int l = (int)floor((xi[a] - R) / g->cs[a]);
        int h = (int)floor((xi[a] + R) / g->cs[a]);
        if (p->periodic[a]) {
            if (h - l + 1 >= g->nc[a]) { l = 0; h = g->nc[a] - 1; }
        } else {
            if (l < 0) l = 0;
            if (h > g->nc[a] - 1) h = g->nc[a] - 1;
        }
        lo[a] = l;
        cnt[a] = h - l + 1;
    }
    for (int a0 = 0; a0 < cnt[0]; a0++)
        for (int a1 = 0; a1 < cnt[1]; a1++)
            for (int a2 = 0; a2 < cnt[2]; a2++) {
                int c[3] = {lo[0] + a0, lo[1] + a1, lo[2] + a2};
                for (int a = 0; a < 3; a++) {
                    c[a] %= g->nc[a];
                    if (c[a] < 0) c[a] += g->nc[a];
                }
                int64_t cell = ((int64_t)c[0] * g->nc[1] + c[1]) * g->nc[2] + c[2];
                for (int64_t j = g->head[cell]; j >= 0; j = g->next[j]) {
                    int rc = try_pair(g, i, j, R, out);
                    if (rc) return rc;
                }
            }
    return OR_OK;
}

static int cmp_nbr(const void *a, const void *b)
{
    int64_t x = ((const nbr_t *)a)->j, y = ((const nbr_t *)b)->j;
    return (x > y) - (x < y);
}

/* Exported for the tests: the neighbour set of i within R, sorted by index. */
int or_find_neighbours(const or_params *p, int64_t n, const double *x, const double *y,
                       const double *z, int64_t i, double R, int64_t cap, int64_t *js,
                       int64_t *count)
{
    grid_t g;
    nbr_list L = {0};
    int rc = grid_build(&g, p, n, x, y, z);
    if (!rc) rc = grid_find(&g, i, R, &L);
    if (!rc) {
        qsort(L.a, (size_t)L.n, sizeof(nbr_t), cmp_nbr);
        *count = L.n;
        for (int64_t k = 0; k < L.n && k < cap; k++) js[k] = L.a[k].j;
    }
    free(L.a);
    grid_free(&g);
    return rc;
}

/* Exported for the tests: mark[j] = 1 for every j within R of any seed i (mark[i] != 0 on input
 * selects the seeds; seeds stay marked).  One bucket grid for all seeds. */
int or_mark_within(const or_params *p, int64_t n, const double *x, const double *y, const double *z,
                   const uint8_t *seeds, double R, uint8_t *mark)
{
    grid_t g;
    nbr_list L = {0};
    int rc = grid_build(&g, p, n, x, y, z);
    for (int64_t i = 0; i < n && !rc; i++) {
        if (!seeds[i]) continue;
        mark[i] = 1;
        rc = grid_find(&g, i, R, &L);
        for (int64_t k = 0; k < L.n && !rc; k++) mark[L.a[k].j] = 1;
    }
    free(L.a);
    grid_free(&g);
    return rc;
}

/* ------------------------------------------------------------------ */
/* R3/R4: kernel length.  f(H) = (4 pi/3) H^3 n(H) - N_ngb, n(H) the   */
/* kernel-weighted number density at H; f is non-decreasing in H, so   */
/* bisection on a sign-change bracket finds its unique root.           */
/* ------------------------------------------------------------------ */
static double number_density(const nbr_list *L, double H)
{
    double s = 0.0;
    for (int64_t k = 0; k < L->n; k++) s += or_kernel_W(L->a[k].r, H);
    return s;
}

static double h_residual(const nbr_list *L, double H, double n_ngb)
{
    return 4.0 * M_PI / 3.0 * H * H * H * number_density(L, H) - n_ngb;
}

/*
 * For every i with mask[i] != 0 (mask may be NULL): H[i] in = guess (<= 0:
 * from the mean density), out = root; nk = n(H), V = 1/nk.  iters[i] counts
 * the bisection steps.
 */
/* the root for one particle i; L is the caller's scratch list */
static int solve_one(const grid_t *g, const or_params *p, int64_t i, double cold, double half,
                     nbr_list *L, double *H, double *nk, double *V, int64_t *iters)
{
    double hi = H[i] > 0.0 ? H[i] : cold;
    double lo = 0.0;
    /* grow the bracket until f(hi) >= 0 */
    for (;;) {
        int rc = grid_find(g, i, hi, L);
        if (rc) return rc;
        if (h_residual(L, hi, p->n_ngb) >= 0.0) break;
        lo = hi;
        hi *= 1.5;
        if (!(hi < half)) {
            /* halve the remaining distance to the limit instead; once that
             * no longer moves, no admissible radius reaches the root */
            double h2 = 0.5 * (lo + half);
            if (!(h2 > lo && h2 < half)) return OR_E_MINIMAGE;
            hi = h2;
        }
    }
    int64_t it = 0;
    for (; it < 400; it++) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        if (h_residual(L, mid, p->n_ngb) < 0.0) lo = mid;
        else hi = mid;
    }
    if (it == 400) return OR_E_NOCONV;
    H[i] = hi;
    nk[i] = number_density(L, hi);
    V[i] = 1.0 / nk[i];
    if (iters) iters[i] = it;
    return OR_OK;
}

/*
 * For every i with mask[i] != 0 (mask may be NULL): H[i] in = guess (<= 0:
 * from the mean density), out = root; nk = n(H), V = 1/nk.  iters[i] counts
 * the bisection steps.  Particles are independent: an OpenMP build of this
 * file shares them out over threads (the result is the same, bit for bit).
 */
int or_solve_h(const or_params *p, int64_t n, const double *x, const double *y,
               const double *z, const uint8_t *mask, double *H, double *nk, double *V,
               int64_t *iters)
{
    grid_t g;
    int rc = grid_build(&g, p, n, x, y, z);
    double vol = p->box[0] * p->box[1] * p->box[2];
    double cold = cbrt(3.0 * p->n_ngb * vol / (4.0 * M_PI * (double)n));
    /* the root must stay below half of every periodic side (R2); the bracket
     * may approach that limit but never reach it */
    double half = INFINITY;
    for (int a = 0; a < 3; a++)
        if (p->periodic[a] && 0.5 * p->box[a] < half) half = 0.5 * p->box[a];
    if (!rc) {
#pragma omp parallel
        {
            nbr_list L = {0};
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < n; i++) {
                if (mask && !mask[i]) continue;
                int e;
#pragma omp atomic read
                e = rc;
                if (e) continue;
                e = solve_one(&g, p, i, cold, half, &L, H, nk, V, iters);
                if (e) {
#pragma omp atomic write
                    rc = e;
                }
            }
            free(L.a);
        }
    }
    grid_free(&g);
    return rc;
}

/* ------------------------------------------------------------------ */
/* R6-R8, R10: gradient matrix, its inverse, limited gradients.        */
/* Field order: rho, vx, vy, vz, P.                                    */
/* B is stored as xx, xy, xz, yy, yz, zz (6 x n, field-major).         */
/* grad is 15 x n: component c of field f at row 3 f + c.             */
/* ------------------------------------------------------------------ */
static void invert_sym3(const double E[3][3], double B[3][3], double *det_out)
{
    /* adjugate over determinant */
    double c00 = E[1][1] * E[2][2] - E[1][2] * E[2][1];
    double c01 = E[1][2] * E[2][0] - E[1][0] * E[2][2];
    double c02 = E[1][0] * E[2][1] - E[1][1] * E[2][0];
    double det = E[0][0] * c00 + E[0][1] * c01 + E[0][2] * c02;
    double id = 1.0 / det;
    B[0][0] = c00 * id;
    B[1][0] = c01 * id;
    B[2][0] = c02 * id;
    B[0][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) * id;
    B[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) * id;
    B[2][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) * id;
    B[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) * id;
    B[1][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) * id;
    B[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) * id;
    *det_out = det;
}

/*
 * rho = m nk, P = (gamma-1) rho u for masked i and every gather neighbour it
 * uses (so nk must be valid there).  Outputs per masked i: B, rho, P, grad
 * (limited), and optionally grad_raw (unlimited), alpha (5 x n limiter
 * factors), cond (||E||_F ||B||_F).  *n_illcond counts flagged particles.
 */
/*
 * R24: the per-particle limiter constant.  With the pairwise limiter on, a
 * particle whose gradient matrix is well conditioned (cond <= cond_lo) keeps
 * beta, one that is badly conditioned (cond >= cond_hi, or singular) takes
 * beta_min, and in between beta moves linearly in log10(cond).  Without it,
 * beta for every particle (R10).
 */
static double limiter_beta(const or_params *p, double kappa)
{
    if (!p->limiter) return p->beta;
    double t;
    if (kappa <= p->cond_lo) t = 0.0;
    else if (kappa < p->cond_hi) t = (log10(kappa) - log10(p->cond_lo)) / (log10(p->cond_hi) - log10(p->cond_lo));
    else t = 1.0;   /* at or above cond_hi, and a NaN condition number */
    return p->beta + (p->beta_min - p->beta) * t;
}

/* R6-R8, R10 for one particle i; *ill = 1 when its E is flagged (R7) */
static int gradients_one(const grid_t *g, const or_params *p, int64_t n, int64_t i, const double *m,
                         const double *vx, const double *vy, const double *vz, const double *u,
                         const double *H, const double *nk, const double *V, nbr_list *L, double *B,
                         double *rho, double *P, double *grad, double *grad_raw, double *alpha,
                         double *cond, int *ill)
{
    int rc = grid_find(g, i, H[i], L);
    if (rc) return rc;
    double phi_i[5];
    double rho_i = m[i] * nk[i];
    phi_i[0] = rho_i;
    phi_i[1] = vx[i];
    phi_i[2] = vy[i];
    phi_i[3] = vz[i];
    phi_i[4] = (p->gamma - 1.0) * rho_i * u[i];
    double E[3][3] = {{0}}, S[5][3] = {{0}};
    double pmax[5], pmin[5], rmax = 0.0;
    for (int f = 0; f < 5; f++) pmax[f] = pmin[f] = phi_i[f];
    for (int64_t k = 0; k < L->n; k++) {
        int64_t j = L->a[k].j;
        const double *d = L->a[k].d;
        double psi = or_kernel_W(L->a[k].r, H[i]) * V[i];
        double rho_j = m[j] * nk[j];
        double phi_j[5] = {rho_j, vx[j], vy[j], vz[j], (p->gamma - 1.0) * rho_j * u[j]};
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) E[a][b] += d[a] * d[b] * psi;
        for (int f = 0; f < 5; f++) {
            for (int a = 0; a < 3; a++) S[f][a] += (phi_j[f] - phi_i[f]) * d[a] * psi;
            if (phi_j[f] > pmax[f]) pmax[f] = phi_j[f];
            if (phi_j[f] < pmin[f]) pmin[f] = phi_j[f];
        }
        if (L->a[k].r > rmax) rmax = L->a[k].r;
    }
    double Bm[3][3], det;
    invert_sym3(E, Bm, &det);
    double fe = 0.0, fb = 0.0;
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            fe += E[a][b] * E[a][b];
            fb += Bm[a][b] * Bm[a][b];
        }
    double kappa = sqrt(fe) * sqrt(fb);
    if (!(det > 0.0) || !(kappa <= p->cond_max)) *ill = 1;
    double beta_i = limiter_beta(p, kappa);
    if (cond) cond[i] = kappa;
    B[0 * n + i] = Bm[0][0];
    B[1 * n + i] = Bm[0][1];
    B[2 * n + i] = Bm[0][2];
    B[3 * n + i] = Bm[1][1];
    B[4 * n + i] = Bm[1][2];
    B[5 * n + i] = Bm[2][2];
    rho[i] = phi_i[0];
    P[i] = phi_i[4];
    double half_span = 0.5 * rmax;
    for (int f = 0; f < 5; f++) {
        double gr[3];
        for (int a = 0; a < 3; a++)
            gr[a] = Bm[a][0] * S[f][0] + Bm[a][1] * S[f][1] + Bm[a][2] * S[f][2];
        double gn = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
        double al = 1.0;
        if (gn > 0.0) {
            double up = (pmax[f] - phi_i[f]) / (gn * half_span);
            double dn = (phi_i[f] - pmin[f]) / (gn * half_span);
            double lim = beta_i * (up < dn ? up : dn);
            al = lim < 1.0 ? lim : 1.0;
        }
        for (int a = 0; a < 3; a++) {
            if (grad_raw) grad_raw[(3 * f + a) * n + i] = gr[a];
            grad[(3 * f + a) * n + i] = al * gr[a];
        }
        if (alpha) alpha[f * n + i] = al;
    }
    return OR_OK;
}

int or_gradients(const or_params *p, int64_t n, const double *x, const double *y,
                 const double *z, const double *m, const double *vx, const double *vy,
                 const double *vz, const double *u, const double *H, const double *nk,
                 const double *V, const uint8_t *mask, double *B, double *rho, double *P,
                 double *grad, double *grad_raw, double *alpha, double *cond,
                 int64_t *n_illcond)
{
    grid_t g;
    int rc = grid_build(&g, p, n, x, y, z);
    int64_t nill = 0;
    if (!rc) {
#pragma omp parallel reduction(+ : nill)
        {
            nbr_list L = {0};
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < n; i++) {
                if (mask && !mask[i]) continue;
                int e;
#pragma omp atomic read
                e = rc;
                if (e) continue;
                int ill = 0;
                e = gradients_one(&g, p, n, i, m, vx, vy, vz, u, H, nk, V, &L, B, rho, P, grad, grad_raw,
                                  alpha, cond, &ill);
                nill += ill;
                if (e) {
#pragma omp atomic write
                    rc = e;
                }
            }
            free(L.a);
        }
    }
    if (n_illcond) *n_illcond = nill;
    grid_free(&g);
    return rc;
}

/* ------------------------------------------------------------------ */
/* R9, R11-R15: one unordered pair in canonical order (a = lower index, */
/* b = higher).  d = x_b - x_a.  Returns the momentum flux P* A_ab and  */
/* the energy flux P* (S* + w.n)|A_ab| that a sends to b.              */
/* ------------------------------------------------------------------ */
typedef struct {
    double H, V, B[3][3];
    double phi[5];     /* rho, vx, vy, vz, P */
    double g[5][3];    /* limited gradients */
} side_t;

static void load_side(side_t *s, int64_t i, int64_t n, const double *H, const double *V,
                      const double *B, const double *rho, const double *vx, const double *vy,
                      const double *vz, const double *P, const double *grad)
{
    s->H = H[i];
    s->V = V[i];
    s->B[0][0] = B[0 * n + i];
    s->B[0][1] = s->B[1][0] = B[1 * n + i];
    s->B[0][2] = s->B[2][0] = B[2 * n + i];
    s->B[1][1] = B[3 * n + i];
    s->B[1][2] = s->B[2][1] = B[4 * n + i];
    s->B[2][2] = B[5 * n + i];
    s->phi[0] = rho[i];
    s->phi[1] = vx[i];
    s->phi[2] = vy[i];
    s->phi[3] = vz[i];
    s->phi[4] = P[i];
    for (int f = 0; f < 5; f++)
        for (int a = 0; a < 3; a++) s->g[f][a] = grad[(3 * f + a) * n + i];
}

typedef struct { double Fm, Fp[3], FE, Pstar, Sstar; int fallback, clamp, skipped; } pairflux_t;

/*
 * MFV: the HLLC flux through a face moving with w (R13), per unit area, in the
 * face frame, then back in the lab frame.  With primes for face-frame
 * velocities, U = (rho, rho v', E) with E = P/(gamma-1) + rho |v'|^2 / 2 and
 * physical flux F = (rho u, rho v' u + P n, (E + P) u), u = v'.n.  The star
 * state of side K keeps the tangential velocity and takes the normal speed S*:
 *   U*_K = rho_K (S_K - u_K)/(S_K - S*) (1, v'_K + (S* - u_K) n,
 *          E_K/rho_K + (S* - u_K)(S* + P_K/(rho_K (S_K - u_K)))),
 * and the flux is F_L (0 <= S_L), F_L + S_L (U*_L - U_L) (S_L < 0 <= S*),
 * F_R + S_R (U*_R - U_R) (S* < 0 <= S_R), F_R (S_R < 0).  In the lab frame the
 * mass flux is unchanged, the momentum flux gains w times it and the energy
 * flux gains w.F_mom' + |w|^2/2 times the mass flux.
 */
static void mfv_face_flux(const double qL[5], const double qR[5], const double w[3],
                          const double nh[3], double uL, double uR, double SL, double SR,
                          double Ss, double gamma, double F[5])
{
    const double *q[2] = {qL, qR};
    double Us[2][5], U[2][5], Fk[2][5];
    double u[2] = {uL, uR}, S[2] = {SL, SR};
    for (int k = 0; k < 2; k++) {
        double rho = q[k][0], P = q[k][4];
        double v[3] = {q[k][1] - w[0], q[k][2] - w[1], q[k][3] - w[2]};
        double E = P / (gamma - 1.0) + 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        U[k][0] = rho;
        for (int c = 0; c < 3; c++) U[k][1 + c] = rho * v[c];
        U[k][4] = E;
        Fk[k][0] = rho * u[k];
        for (int c = 0; c < 3; c++) Fk[k][1 + c] = rho * v[c] * u[k] + P * nh[c];
        Fk[k][4] = (E + P) * u[k];
        double fac = rho * (S[k] - u[k]) / (S[k] - Ss);
        Us[k][0] = fac;
        for (int c = 0; c < 3; c++) Us[k][1 + c] = fac * (v[c] + (Ss - u[k]) * nh[c]);
        Us[k][4] = fac * (E / rho + (Ss - u[k]) * (Ss + P / (rho * (S[k] - u[k]))));
    }
    double Ff[5];
    for (int e = 0; e < 5; e++) {
        if (SL >= 0.0) Ff[e] = Fk[0][e];
        else if (Ss >= 0.0) Ff[e] = Fk[0][e] + SL * (Us[0][e] - U[0][e]);
        else if (SR >= 0.0) Ff[e] = Fk[1][e] + SR * (Us[1][e] - U[1][e]);
        else Ff[e] = Fk[1][e];
    }
    double ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    F[0] = Ff[0];
    for (int c = 0; c < 3; c++) F[1 + c] = Ff[1 + c] + w[c] * Ff[0];
    F[4] = Ff[4] + w[0] * Ff[1] + w[1] * Ff[2] + w[2] * Ff[3] + 0.5 * ww * Ff[0];
}

/*
 * R23: the pairwise limiter on one face value.  f is the value side K
 * extrapolated to the midpoint face, pk and po the centre values of K and of
 * the other particle.  With lo/hi their min/max and D = hi - lo, the face
 * value may not pass the midpoint interpolant (pk + po)/2 by more than psi2 D
 * on the far side, nor leave [lo, hi] by more than psi1 D on the near side;
 * an expanded bound that would change the sign of lo (hi) is replaced by
 * lo / (1 + psi1 D / |lo|) (likewise for hi), so a positive field keeps
 * positive face values.  Equal centre values give the centre value.
 */
#define OR_PSI1 0.5
#define OR_PSI2 0.25

static double pair_limit(double f, double pk, double po)
{
    if (pk == po) return pk;
    double lo = pk < po ? pk : po, hi = pk < po ? po : pk;
    double D = hi - lo;
    double mid = 0.5 * (pk + po);
    if (pk < po) {
        double lb = lo - OR_PSI1 * D;
        if (!(lb * lo > 0.0)) lb = lo / (1.0 + OR_PSI1 * D / fabs(lo));
        double ub = mid + OR_PSI2 * D;
        double v = f < ub ? f : ub;
        return v > lb ? v : lb;
    }
    double ub = hi + OR_PSI1 * D;
    if (!(ub * hi > 0.0)) ub = hi / (1.0 + OR_PSI1 * D / fabs(hi));
    double lb = mid - OR_PSI2 * D;
    double v = f > lb ? f : lb;
    return v < ub ? v : ub;
}

static void pair_flux(const side_t *a, const side_t *b, const double d[3], double r,
                      double gamma, int mfv, int limiter, pairflux_t *out)
{
    memset(out, 0, sizeof(*out));
    double Wa = or_kernel_W(r, a->H), Wb = or_kernel_W(r, b->H);
    double A[3];
    for (int c = 0; c < 3; c++) {
        double ta = a->B[c][0] * d[0] + a->B[c][1] * d[1] + a->B[c][2] * d[2];
        double tb = b->B[c][0] * d[0] + b->B[c][1] * d[1] + b->B[c][2] * d[2];
        A[c] = a->V * a->V * Wa * ta + b->V * b->V * Wb * tb;
    }
    double Amag = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
    if (!(Amag > 0.0)) { out->skipped = 1; return; }
    double nh[3] = {A[0] / Amag, A[1] / Amag, A[2] / Amag};

    /* R12: linear reconstruction to the midpoint face, first order if not positive */
    double qL[5], qR[5];
    for (int f = 0; f < 5; f++) {
        qL[f] = a->phi[f] + 0.5 * (a->g[f][0] * d[0] + a->g[f][1] * d[1] + a->g[f][2] * d[2]);
        qR[f] = b->phi[f] - 0.5 * (b->g[f][0] * d[0] + b->g[f][1] * d[1] + b->g[f][2] * d[2]);
        if (limiter) {
            /* R23 on each side's face value */
            qL[f] = pair_limit(qL[f], a->phi[f], b->phi[f]);
            qR[f] = pair_limit(qR[f], b->phi[f], a->phi[f]);
        }
    }
    if (!(qL[0] > 0.0) || !(qL[4] > 0.0) || !(qR[0] > 0.0) || !(qR[4] > 0.0)) {
        for (int f = 0; f < 5; f++) { qL[f] = a->phi[f]; qR[f] = b->phi[f]; }
        out->fallback = 1;
    }

    /* R13: face frame moves with the mean particle velocity */
    double w[3] = {0.5 * (a->phi[1] + b->phi[1]), 0.5 * (a->phi[2] + b->phi[2]),
                   0.5 * (a->phi[3] + b->phi[3])};
    double uL = (qL[1] - w[0]) * nh[0] + (qL[2] - w[1]) * nh[1] + (qL[3] - w[2]) * nh[2];
    double uR = (qR[1] - w[0]) * nh[0] + (qR[2] - w[1]) * nh[1] + (qR[3] - w[2]) * nh[2];
    double rL = qL[0], pL = qL[4], rR = qR[0], pR = qR[4];

    /* R14: HLLC with Davis wave speeds */
    double cL = sqrt(gamma * pL / rL), cR = sqrt(gamma * pR / rR);
    double SL = uL - cL < uR - cR ? uL - cL : uR - cR;
    double SR = uL + cL > uR + cR ? uL + cL : uR + cR;
    double mL = rL * (SL - uL), mR = rR * (SR - uR);
    double Ss = (pR - pL + mL * uL - mR * uR) / (mL - mR);
    double Ps = 0.5 * (pL + pR + mL * (Ss - uL) + mR * (Ss - uR));
    if (mfv) {
        double F[5];
        mfv_face_flux(qL, qR, w, nh, uL, uR, SL, SR, Ss, gamma, F);
        out->Fm = F[0] * Amag;
        for (int c = 0; c < 3; c++) out->Fp[c] = F[1 + c] * Amag;
        out->FE = F[4] * Amag;
        out->Pstar = Ps;
        out->Sstar = Ss;
        return;
    }
    if (Ps < 0.0) { Ps = 0.0; out->clamp = 1; }

    /* R15: zero mass flux; momentum P* A, energy P* (S* + w.n)|A| */
    double wn = w[0] * nh[0] + w[1] * nh[1] + w[2] * nh[2];
    for (int c = 0; c < 3; c++) out->Fp[c] = Ps * A[c];
    out->FE = Ps * (Ss + wn) * Amag;
    out->Pstar = Ps;
    out->Sstar = Ss;
}

/* Exported for the tests: the HLLC star state of two 1D states. */
void or_hllc_star(double gamma, double rL, double uL, double pL, double rR, double uR,
                  double pR, double *Sstar, double *Pstar)
{
    side_t a, b;
    memset(&a, 0, sizeof(a));
    memset(&b, 0, sizeof(b));
    /* unit separation along x, identity B and V, equal H: A = (c, 0, 0), n = +x */
    a.H = b.H = 2.0;
    a.V = b.V = 1.0;
    for (int c = 0; c < 3; c++) a.B[c][c] = b.B[c][c] = 1.0;
    a.phi[0] = rL; a.phi[1] = uL; a.phi[4] = pL;
    b.phi[0] = rR; b.phi[1] = uR; b.phi[4] = pR;
    /* shift both velocities by the face velocity so that u is measured in the face frame */
    double w = 0.5 * (uL + uR);
    double d[3] = {1.0, 0.0, 0.0};
    pairflux_t o;
    pair_flux(&a, &b, d, 1.0, gamma, 0, 0, &o);
    *Sstar = o.Sstar + w;
    *Pstar = o.Pstar;
}

/* Exported for the tests: the MFV flux (mass, momentum, energy per unit face
 * area, lab frame) between two 1D face states (rho, u, P) along +x, when the
 * particles themselves move with vL and vR, so that the face moves with
 * (vL + vR)/2.  The face states are made by the reconstruction of R12: each
 * side's velocity gradient along x is set so that its midpoint value is the
 * given face velocity (d = 1, so half a unit of gradient per unit offset). */
void or_mfv_flux_moving(double gamma, double vL, double vR, double rL, double uL, double pL,
                        double rR, double uR, double pR, double F[3])
{
    side_t a, b;
    memset(&a, 0, sizeof(a));
    memset(&b, 0, sizeof(b));
    /* identity B and V, equal H: A = W(1, 2) (1, 0, 0); the flux is divided by |A| */
    a.H = b.H = 2.0;
    a.V = b.V = 1.0;
    for (int c = 0; c < 3; c++) a.B[c][c] = b.B[c][c] = 1.0;
    a.phi[0] = rL; a.phi[1] = vL; a.phi[4] = pL;
    b.phi[0] = rR; b.phi[1] = vR; b.phi[4] = pR;
    a.g[1][0] = 2.0 * (uL - vL);     /* qL = vL + g/2 = uL */
    b.g[1][0] = 2.0 * (vR - uR);     /* qR = vR - g/2 = uR */
    double d[3] = {1.0, 0.0, 0.0};
    pairflux_t o;
    pair_flux(&a, &b, d, 1.0, gamma, 1, 0, &o);
    double Amag = 2.0 * or_kernel_W(1.0, 2.0);
    F[0] = o.Fm / Amag;
    F[1] = o.Fp[0] / Amag;
    F[2] = o.FE / Amag;
}

/* The same with the particles moving at the face states' own velocities, so
 * that the face moves with (uL + uR)/2. */
void or_mfv_flux(double gamma, double rL, double uL, double pL, double rR, double uR, double pR,
                 double F[3])
{
    or_mfv_flux_moving(gamma, uL, uR, rL, uL, pL, rR, uR, pR, F);
}

/*
 * R2, R16: for every masked i, sum over its flux set j (r_ij < max(H_i, H_j),
 * j != i) of -s F_p and -s F_E, where each pair is evaluated with the lower
 * index as the left state and s = +1 if i is that state, -1 otherwise.
 * vsig_i = max_j [c_i + c_j - min(0, (v_i - v_j).(x_i - x_j)/r_ij)] (R18).
 * hmax must bound H over all particles.  Counts: pair entries (directed),
 * first-order fallbacks and P* clamps (directed).  With scheme 1 (MFV) the
 * pair flux is the full HLLC one and dm (nullable) receives -s F_m summed.
 */
/* R2, R9, R11-R16, R18 for one particle i: its flux sums and signal speed */
static int fluxes_one(const grid_t *g, const or_params *p, int64_t n, int64_t i, const double *vx,
                      const double *vy, const double *vz, const double *H, const double *V,
                      const double *B, const double *rho, const double *P, const double *grad,
                      double hmax, nbr_list *L, double *dp, double *dE, double *vsig, double *dm,
                      const int64_t *bins, int64_t lmin, int64_t nlev, double *lev,
                      int64_t *npair, int64_t *nfall, int64_t *nclamp)
{
    double R = H[i] > hmax ? H[i] : hmax;
    int rc = grid_find(g, i, R, L);
    if (rc) return rc;
    /* R25: the sums of the due levels start again; the others keep their values */
    if (bins)
        for (int64_t l = lmin; l < nlev; l++)
            for (int c = 0; c < 5; c++) lev[(l * 5 + c) * n + i] = 0.0;
    double acc[4] = {0, 0, 0, 0}, accm = 0.0;
    double ci = sqrt(p->gamma * P[i] / rho[i]);
    double vs = 0.0;
    side_t si, sj;
    load_side(&si, i, n, H, V, B, rho, vx, vy, vz, P, grad);
    for (int64_t k = 0; k < L->n; k++) {
        int64_t j = L->a[k].j;
        double r = L->a[k].r;
        if (j == i) continue;
        if (!(r < H[i] || r < H[j])) continue;
        double cj = sqrt(p->gamma * P[j] / rho[j]);
        const double *d = L->a[k].d; /* x_j - x_i */
        double proj = ((vx[i] - vx[j]) * (-d[0]) + (vy[i] - vy[j]) * (-d[1]) +
                       (vz[i] - vz[j]) * (-d[2])) / r;
        double sig = ci + cj - (proj < 0.0 ? proj : 0.0);
        if (sig > vs) vs = sig;
        /* R25: a pair's level is the finer bin of its two particles; only due levels */
        int64_t lev_ij = 0;
        if (bins) {
            lev_ij = bins[i] > bins[j] ? bins[i] : bins[j];
            if (lev_ij < lmin) continue;
        }
        (*npair)++;
        load_side(&sj, j, n, H, V, B, rho, vx, vy, vz, P, grad);
        pairflux_t o;
        double s;
        if (i < j) {
            pair_flux(&si, &sj, L->a[k].d, r, p->gamma, p->scheme == 1, p->limiter, &o);
            s = 1.0;
        } else {
            double dn[3] = {-L->a[k].d[0], -L->a[k].d[1], -L->a[k].d[2]};
            pair_flux(&sj, &si, dn, r, p->gamma, p->scheme == 1, p->limiter, &o);
            s = -1.0;
        }
        *nfall += o.fallback;
        *nclamp += o.clamp;
        for (int c = 0; c < 3; c++) acc[c] -= s * o.Fp[c];
        acc[3] -= s * o.FE;
        accm -= s * o.Fm;
        if (bins) {
            for (int c = 0; c < 3; c++) lev[(lev_ij * 5 + c) * n + i] -= s * o.Fp[c];
            lev[(lev_ij * 5 + 3) * n + i] -= s * o.FE;
            lev[(lev_ij * 5 + 4) * n + i] -= s * o.Fm;
        }
    }
    dp[0 * n + i] = acc[0];
    dp[1 * n + i] = acc[1];
    dp[2 * n + i] = acc[2];
    dE[i] = acc[3];
    vsig[i] = vs;
    if (dm) dm[i] = accm;
    return OR_OK;
}

/*
 * As or_fluxes, with R25's levels when bins is not NULL: pair {i, j} has level
 * max(bins[i], bins[j]); only pairs of level >= lmin are evaluated (and
 * counted), dp, dE, dm summing those; lev (5 x nlev x n, [(l * 5 + c) * n + i],
 * c = dp x, y, z, dE, dm) receives each particle's sums per level for the
 * levels >= lmin and keeps its values for the others.  vsig covers every
 * flux neighbour.
 */
int or_fluxes_levels(const or_params *p, int64_t n, const double *x, const double *y,
                     const double *z, const double *vx, const double *vy, const double *vz,
                     const double *H, const double *V, const double *B, const double *rho,
                     const double *P, const double *grad, const uint8_t *mask, double hmax,
                     double *dp, double *dE, double *vsig, int64_t *counts, double *dm,
                     const int64_t *bins, int64_t lmin, int64_t nlev, double *lev)
{
    grid_t g;
    int rc = grid_build(&g, p, n, x, y, z);
    int64_t npair = 0, nfall = 0, nclamp = 0;
    if (!rc) {
#pragma omp parallel reduction(+ : npair, nfall, nclamp)
        {
            nbr_list L = {0};
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < n; i++) {
                if (mask && !mask[i]) continue;
                int e;
#pragma omp atomic read
                e = rc;
                if (e) continue;
                e = fluxes_one(&g, p, n, i, vx, vy, vz, H, V, B, rho, P, grad, hmax, &L, dp, dE, vsig, dm,
                               bins, lmin, nlev, lev, &npair, &nfall, &nclamp);
                if (e) {
#pragma omp atomic write
                    rc = e;
                }
            }
            free(L.a);
        }
    }
    if (counts) {
        counts[0] = npair;
        counts[1] = nfall;
        counts[2] = nclamp;
    }
    grid_free(&g);
    return rc;
}

int or_fluxes(const or_params *p, int64_t n, const double *x, const double *y,
              const double *z, const double *vx, const double *vy, const double *vz,
              const double *H, const double *V, const double *B, const double *rho,
              const double *P, const double *grad, const uint8_t *mask, double hmax,
              double *dp, double *dE, double *vsig, int64_t *counts, double *dm)
{
    return or_fluxes_levels(p, n, x, y, z, vx, vy, vz, H, V, B, rho, P, grad, mask, hmax, dp, dE, vsig,
                            counts, dm, NULL, 0, 0, NULL);
}

/* Exported for the tests: R23 on one face value (see pair_limit). */
double or_pair_limit(double f, double pk, double po) { return pair_limit(f, pk, po); }

/* Exported for the tests: R24's limiter constant at a condition number. */
double or_limiter_beta(const or_params *p, double kappa) { return limiter_beta(p, kappa); }

/* Exported for the tests: the face vector A_ab of one pair from given sides. */
void or_face(double Ha, double Va, const double *Ba6, double Hb, double Vb, const double *Bb6,
             const double *d, double *A)
{
    double Ba[3][3] = {{Ba6[0], Ba6[1], Ba6[2]}, {Ba6[1], Ba6[3], Ba6[4]}, {Ba6[2], Ba6[4], Ba6[5]}};
    double Bb[3][3] = {{Bb6[0], Bb6[1], Bb6[2]}, {Bb6[1], Bb6[3], Bb6[4]}, {Bb6[2], Bb6[4], Bb6[5]}};
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double Wa = or_kernel_W(r, Ha), Wb = or_kernel_W(r, Hb);
    for (int c = 0; c < 3; c++) {
        double ta = Ba[c][0] * d[0] + Ba[c][1] * d[1] + Ba[c][2] * d[2];
        double tb = Bb[c][0] * d[0] + Bb[c][1] * d[1] + Bb[c][2] * d[2];
        A[c] = Va * Va * Wa * ta + Vb * Vb * Wb * tb;
    }
}
