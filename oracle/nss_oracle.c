/*
 * Plain FP64 CPU oracle for Nested Slice Sampling (NSS).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header, table or constant with the GPU
 * library (paper_2601_23252_amd/csrc); the only thing both sides share is the seeded problem
 * generator, which holds none of the method's arithmetic.
 *
 * What it computes (paper references are section / equation / algorithm / table):
 *   - the batched NS outer kernel: delete the k worst, resample parents uniformly among the
 *     survivors, mutate each parent with a constrained kernel, replace
 *     (Sec. 3.1 "Parallel Nested Sampling"; Alg. "Nested Sampling outer kernel");
 *   - the constrained kernel, Hit-and-Run Slice Sampling: random direction in the Mahalanobis
 *     metric of the live-set covariance, randomised initial bracket of width w, linear
 *     stepping-out capped at 10 expansions per side, shrinkage capped at 100 proposals with a
 *     null move on the cap (Sec. 3.2; App. A.6 "Hit-and-Run Slice Sampling Implementation");
 *   - evidence by the rectangle rule Z = sum L_i dX_i (Sec. 2.1, eq. marginal) with each batch
 *     of k deaths unrolled into single deaths at live counts m, m-1, ..., m-k+1
 *     (Sec. 2.1; App. D.2.1), using the deterministic log-volume decrement -1/n per death
 *     (the expectation of log t for t ~ Beta(n,1), App. D.2.2);
 *   - termination when an upper bound on the live set's remaining contribution is below a
 *     tolerance (Sec. 2.1), and the final live-set contribution.
 *
 * Readings where the paper is silent are listed in the design notes: Mahalanobis-normalised
 * direction; survivors' covariance with 1e-12 trace jitter; parents drawn from survivors with
 * logL strictly above L* in ascending (logL, index) order; literal 10-per-side step-out cap;
 * shrink side chosen by the sign of t'; normalised likelihood densities.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11), written here from that definition.  Counter = (purpose<<24 | index,
 * iteration, step, draw), key = (seed_lo, seed_hi ^ run_id).  A 64-bit word x gives the uniform
 * (2*(x>>12)+1) * 2^-53 in (0,1); normals by the Box-Muller transform.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

enum { P_INIT = 1, P_RESAMPLE = 2, P_DIR = 3, P_STEP = 4, P_SHRINK = 5, P_GEOM = 6, P_POST = 7 };
enum { PRIOR_BOX = 0, PRIOR_GAUSS = 1 };
enum { LIK_MIXTURE = 1, LIK_FUNNEL = 2, LIK_GP = 3, LIK_RG = 4 };

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10                                                                               */
/* ------------------------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double u53(uint32_t lo, uint32_t hi)
{
    uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
    return (double)(2u * (x >> 12) + 1u) * 0x1p-53;
}

typedef struct { uint32_t k[2]; } okey;

/* Two FP64 uniforms from one Philox call at counter (purpose<<24|index, c1, c2, c3). */
static void draw2(okey key, uint32_t purpose, uint32_t index, uint32_t c1, uint32_t c2,
                  uint32_t c3, double *ua, double *ub)
{
    uint32_t ctr[4] = { (purpose << 24) | (index & 0xFFFFFFu), c1, c2, c3 }, r[4];
    or_philox4x32_10(ctr, key.k, r);
    *ua = u53(r[0], r[1]);
    *ub = u53(r[2], r[3]);
}

void or_uniform_pair(uint64_t seed, uint32_t run_id, uint32_t purpose, uint32_t index,
                     uint32_t c1, uint32_t c2, uint32_t c3, double out[2])
{
    okey key = { { (uint32_t)seed, (uint32_t)(seed >> 32) ^ run_id } };
    draw2(key, purpose, index, c1, c2, c3, &out[0], &out[1]);
}

/* Box-Muller: one pair of uniforms -> two independent standard normals. */
static void box_muller(double ua, double ub, double *z0, double *z1)
{
    double rad = sqrt(-2.0 * log(ua));
    double th = 2.0 * OR_PI * ub;
    *z0 = rad * cos(th);
    *z1 = rad * sin(th);
}

/* ------------------------------------------------------------------------------------------ */
/* Problem: prior Pi and energy E = -log L                                                     */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int d;
    int prior_kind;
    double *pa, *pb;          /* box: lower, upper; gauss: mean, std (per coordinate) */
    int lik_kind;
    int K;                    /* mixture components */
    double *logw;             /* K log weights */
    double *mu;               /* K x d means */
    double *chol;             /* K x d x d lower Cholesky factors of the covariances */
    double *logdet_half;      /* K: sum log diag(chol) = 0.5 log det C */
    int gp_n;                 /* GP regression: n observations */
    double *gp_x;             /* n x 2 inputs */
    double *gp_y;             /* n targets */
    double rg_alpha, rg_amp;  /* Gaussian-Rastrigin mixture weight alpha and amplitude A */
} oprob;

static int cholesky_lower(const double *A, double *L, int n)
{
    memset(L, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[i * n + j];
            for (int t = 0; t < j; ++t) s -= L[i * n + t] * L[j * n + t];
            if (i == j) {
                if (!(s > 0.0)) return -1;
                L[i * n + i] = sqrt(s);
            } else {
                L[i * n + j] = s / L[j * n + j];
            }
        }
    }
    return 0;
}

void or_problem_free(void *pp)
{
    oprob *p = (oprob *)pp;
    if (!p) return;
    free(p->pa); free(p->pb); free(p->logw); free(p->mu); free(p->chol); free(p->logdet_half);
    free(p->gp_x); free(p->gp_y);
    free(p);
}

/* Returns NULL on invalid input (non-positive-definite covariance, bad sizes). */
void *or_problem_new(int d, int prior_kind, const double *pa, const double *pb, int lik_kind,
                     int K, const double *logw, const double *mu, const double *cov)
{
    if (d < 1) return NULL;
    oprob *p = (oprob *)calloc(1, sizeof(oprob));
    p->d = d;
    p->prior_kind = prior_kind;
    p->pa = (double *)malloc(sizeof(double) * d);
    p->pb = (double *)malloc(sizeof(double) * d);
    memcpy(p->pa, pa, sizeof(double) * d);
    memcpy(p->pb, pb, sizeof(double) * d);
    p->lik_kind = lik_kind;
    if (lik_kind == LIK_MIXTURE) {
        if (K < 1) { or_problem_free(p); return NULL; }
        p->K = K;
        p->logw = (double *)malloc(sizeof(double) * K);
        p->mu = (double *)malloc(sizeof(double) * (size_t)K * d);
        p->chol = (double *)malloc(sizeof(double) * (size_t)K * d * d);
        p->logdet_half = (double *)malloc(sizeof(double) * K);
        memcpy(p->logw, logw, sizeof(double) * K);
        memcpy(p->mu, mu, sizeof(double) * (size_t)K * d);
        for (int i = 0; i < K; ++i) {
            double *L = p->chol + (size_t)i * d * d;
            if (cholesky_lower(cov + (size_t)i * d * d, L, d) != 0) { or_problem_free(p); return NULL; }
            double s = 0.0;
            for (int j = 0; j < d; ++j) s += log(L[j * d + j]);
            p->logdet_half[i] = s;
        }
    } else if (lik_kind != LIK_FUNNEL) {
        or_problem_free(p);
        return NULL;
    }
    return p;
}

/* GP hyperparameter marginalisation: d = 6 coordinates u = log theta with
 * theta = (sigma_f, l_1, l_2, l_p, P, sigma_n), a box prior on u (log-uniform theta), data
 * (X[n][2], y[n]).  Returns NULL on invalid input. */
void *or_problem_new_gp(int n, const double *X, const double *y, const double *pa,
                        const double *pb)
{
    if (n < 1) return NULL;
    const int d = 6;
    oprob *p = (oprob *)calloc(1, sizeof(oprob));
    p->d = d;
    p->prior_kind = PRIOR_BOX;
    p->pa = (double *)malloc(sizeof(double) * d);
    p->pb = (double *)malloc(sizeof(double) * d);
    memcpy(p->pa, pa, sizeof(double) * d);
    memcpy(p->pb, pb, sizeof(double) * d);
    p->lik_kind = LIK_GP;
    p->gp_n = n;
    p->gp_x = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    p->gp_y = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(p->gp_x, X, sizeof(double) * 2 * (size_t)n);
    memcpy(p->gp_y, y, sizeof(double) * (size_t)n);
    return p;
}

/* Gaussian-Rastrigin test likelihood (the evidence comparison of the constrained samplers):
 * L = alpha f + (1 - alpha) g with f = exp(-|x|^2 / 2) and
 * g = exp(-A d + A sum_i cos(2 pi x_i)), any prior.  Returns NULL on invalid input. */
void *or_problem_new_rg(int d, int prior_kind, const double *pa, const double *pb, double alpha,
                        double amp)
{
    if (d < 1 || !(alpha >= 0.0 && alpha <= 1.0) || !(amp >= 0.0)) return NULL;
    oprob *p = (oprob *)calloc(1, sizeof(oprob));
    p->d = d;
    p->prior_kind = prior_kind;
    p->pa = (double *)malloc(sizeof(double) * d);
    p->pb = (double *)malloc(sizeof(double) * d);
    memcpy(p->pa, pa, sizeof(double) * d);
    memcpy(p->pb, pb, sizeof(double) * d);
    p->lik_kind = LIK_RG;
    p->rg_alpha = alpha;
    p->rg_amp = amp;
    return p;
}

/* log L of the Gaussian-Rastrigin likelihood: log(alpha e^{-|x|^2/2} + (1-alpha) e^{-A d +
 * A sum cos(2 pi x_i)}) as a log-sum-exp of the two terms; cos(2 pi x) is taken at the
 * distance of x to the nearest integer (the same value; the argument stays below pi, so its
 * rounding does not grow with |x|). */
static double rg_loglik(const oprob *p, const double *x)
{
    double s2 = 0.0, sc = 0.0;
    for (int j = 0; j < p->d; ++j) {
        s2 += x[j] * x[j];
        sc += cos(2.0 * OR_PI * (x[j] - nearbyint(x[j])));
    }
    const double tf = p->rg_alpha > 0.0 ? log(p->rg_alpha) - 0.5 * s2 : -INFINITY;
    const double tg = p->rg_alpha < 1.0 ? log1p(-p->rg_alpha) - p->rg_amp * p->d + p->rg_amp * sc
                                        : -INFINITY;
    const double mx = tf > tg ? tf : tg;
    return mx + log(exp(tf - mx) + exp(tg - mx));
}

/* Prior support test. */
static int prior_in_support(const oprob *p, const double *x)
{
    if (p->prior_kind == PRIOR_BOX) {
        for (int j = 0; j < p->d; ++j)
            if (!(x[j] >= p->pa[j] && x[j] <= p->pb[j])) return 0;
    }
    return 1;
}

/* log Pi(x): normalised density; -inf outside the support. */
double or_logprior(const void *pp, const double *x)
{
    const oprob *p = (const oprob *)pp;
    if (!prior_in_support(p, x)) return -INFINITY;
    double s = 0.0;
    if (p->prior_kind == PRIOR_BOX) {
        for (int j = 0; j < p->d; ++j) s -= log(p->pb[j] - p->pa[j]);
    } else {
        for (int j = 0; j < p->d; ++j) {
            double z = (x[j] - p->pa[j]) / p->pb[j];
            s += -0.5 * z * z - log(p->pb[j]) - 0.5 * log(2.0 * OR_PI);
        }
    }
    return s;
}

/* log N(x; mu, C) with C = L L^T: solve L z = x - mu by forward substitution. */
static double log_gauss_chol(const double *x, const double *mu, const double *L,
                             double logdet_half, int d)
{
    double z[512];
    double q = 0.0;
    for (int a = 0; a < d; ++a) {
        double s = x[a] - mu[a];
        for (int b = 0; b < a; ++b) s -= L[a * d + b] * z[b];
        z[a] = s / L[a * d + a];
        q += z[a] * z[a];
    }
    return -0.5 * q - logdet_half - 0.5 * d * log(2.0 * OR_PI);
}

/* GP log marginal likelihood log N(y; 0, K + sigma_n^2 I) with the product kernel
 *   k(a, b) = sigma_f^2 exp(-1/2 sum_j (a_j - b_j)^2 / l_j^2)
 *                       exp(-2 sum_j sin^2(pi (a_j - b_j) / P) / l_p^2),   j = 1, 2,
 * (a squared-exponential times a periodic kernel, each a product over the input dimensions),
 * by a Cholesky factorisation K_y = L L^T: log L = -1/2 |L^{-1} y|^2 - sum log L_ii
 * - n/2 log(2 pi).  A factorisation that breaks down gives -inf. */
static double gp_loglik(const oprob *p, const double *u)
{
    const int n = p->gp_n;
    const double sf2 = exp(2.0 * u[0]), l1 = exp(u[1]), l2 = exp(u[2]), lp = exp(u[3]);
    const double per = exp(u[4]), sn2 = exp(2.0 * u[5]);
    double *K = (double *)malloc(sizeof(double) * (size_t)n * n);
    double *L = (double *)malloc(sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            const double d1 = p->gp_x[2 * i] - p->gp_x[2 * j];
            const double d2 = p->gp_x[2 * i + 1] - p->gp_x[2 * j + 1];
            const double s1 = sin(OR_PI * d1 / per), s2 = sin(OR_PI * d2 / per);
            double k = sf2 * exp(-0.5 * (d1 * d1 / (l1 * l1) + d2 * d2 / (l2 * l2))) *
                       exp(-2.0 * (s1 * s1 + s2 * s2) / (lp * lp));
            if (i == j) k += sn2;
            K[(size_t)i * n + j] = k;
            K[(size_t)j * n + i] = k;
        }
    double r;
    if (cholesky_lower(K, L, n) != 0) {
        r = -INFINITY;
    } else {
        double q = 0.0, ld = 0.0;
        double *z = K;  /* reuse: forward substitution L z = y */
        for (int i = 0; i < n; ++i) {
            double s = p->gp_y[i];
            for (int t = 0; t < i; ++t) s -= L[(size_t)i * n + t] * z[t];
            z[i] = s / L[(size_t)i * n + i];
            q += z[i] * z[i];
            ld += log(L[(size_t)i * n + i]);
        }
        r = -0.5 * q - ld - 0.5 * n * log(2.0 * OR_PI);
    }
    free(K);
    free(L);
    return r;
}

/* log L(x) = -E(x).  Mixture: log sum_i w_i N(x; mu_i, C_i).  Funnel: v = x_0 ~ N(0, 9),
 * x_j | v ~ N(0, e^v) for j >= 1.  GP: log marginal likelihood of the regression data. */
double or_loglik(const void *pp, const double *x)
{
    const oprob *p = (const oprob *)pp;
    int d = p->d;
    if (p->lik_kind == LIK_GP) return gp_loglik(p, x);
    if (p->lik_kind == LIK_RG) return rg_loglik(p, x);
    if (p->lik_kind == LIK_MIXTURE) {
        double terms[256];
        double mx = -INFINITY;
        for (int i = 0; i < p->K; ++i) {
            terms[i] = p->logw[i] + log_gauss_chol(x, p->mu + (size_t)i * d,
                                                   p->chol + (size_t)i * d * d,
                                                   p->logdet_half[i], d);
            if (terms[i] > mx) mx = terms[i];
        }
        if (mx == -INFINITY) return -INFINITY;
        double s = 0.0;
        for (int i = 0; i < p->K; ++i) s += exp(terms[i] - mx);
        return mx + log(s);
    } else {
        double v = x[0];
        double r = -0.5 * v * v / 9.0 - 0.5 * log(2.0 * OR_PI * 9.0);
        for (int j = 1; j < d; ++j)
            r += -0.5 * x[j] * x[j] * exp(-v) - 0.5 * v - 0.5 * log(2.0 * OR_PI);
        return r;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Hit-and-Run Slice Sampling chain                                                            */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int64_t evals;          /* likelihood computations (candidate passed the prior checks) */
    int64_t tests;          /* all inside-tests, including prior rejections */
    int64_t prior_rejects;  /* candidates outside the prior support or below the height */
    int64_t stepout_caps;   /* sides that stopped at the expansion cap */
    int64_t shrink_caps;    /* null moves from the shrink cap */
    int64_t nonfinite;      /* NaN / +inf log-likelihoods, treated as -inf */
} octr;

typedef struct {
    const oprob *p;
    const double *x0, *v;
    double Lstar, logy;
    double beta;            /* < 0: nested-sampling slice; >= 0: tempered slice at beta */
    int uniform_prior;
    double *y;              /* scratch, d */
    octr *c;
    double last_logL;
} inside_ctx;

/* The slice predicate along the line.  Nested sampling: x0 + t v inside the prior support,
 * above the prior height (non-uniform priors only) and strictly above the likelihood
 * threshold.  Tempered (the SMC mutation, no hard constraint): inside the prior support and
 * log Pi(y) + beta log L(y) above the slice height, log Pi taken as 0 for a box prior. */
static int inside(inside_ctx *s, double t)
{
    const int d = s->p->d;
    for (int a = 0; a < d; ++a) s->y[a] = s->x0[a] + t * s->v[a];
    s->c->tests++;
    if (!prior_in_support(s->p, s->y)) { s->c->prior_rejects++; return 0; }
    if (s->beta < 0.0 && !s->uniform_prior && !(or_logprior(s->p, s->y) > s->logy)) {
        s->c->prior_rejects++;
        return 0;
    }
    double L = or_loglik(s->p, s->y);
    s->c->evals++;
    if (isnan(L) || L == INFINITY) { s->c->nonfinite++; L = -INFINITY; }
    s->last_logL = L;
    if (s->beta >= 0.0) {
        const double lp = s->uniform_prior ? 0.0 : or_logprior(s->p, s->y);
        return lp + s->beta * L > s->logy;
    }
    return L > s->Lstar;
}

/*
 * One chain of p HRSS steps from (x, logL) under the hard constraint logL > Lstar.
 * Lsig: d x d lower-triangular factor of the direction covariance (row-major).
 * trace (optional, 4 ints per step): left expansions, right expansions, shrink proposals,
 * accepted (1) or null move (0).
 * x and *logL are updated in place.
 */
static void hrss_chain(const oprob *p, double *x, double *logL, double Lstar, double beta,
                       const double *Lsig, double w, int p_steps, int stepout_cap,
                       int shrink_cap, uint64_t seed, uint32_t run_id, uint32_t iter,
                       uint32_t chain, int64_t *counters, int32_t *trace)
{
    const int d = p->d;
    okey key = { { (uint32_t)seed, (uint32_t)(seed >> 32) ^ run_id } };
    double *z = (double *)malloc(sizeof(double) * d * 3);
    double *v = z + d, *y = z + 2 * d;
    octr c; memset(&c, 0, sizeof c);
    inside_ctx s;
    s.p = p; s.x0 = x; s.v = v; s.Lstar = Lstar; s.y = y; s.c = &c; s.beta = beta;
    s.uniform_prior = (p->prior_kind == PRIOR_BOX);
    for (int st = 0; st < p_steps; ++st) {
        /* direction: z ~ N(0, I), v = Lsig z / |z| (unit length in the Mahalanobis metric) */
        for (int q = 0; 2 * q < d; ++q) {
            double ua, ub, z0, z1;
            draw2(key, P_DIR, chain, iter, (uint32_t)st, (uint32_t)q, &ua, &ub);
            box_muller(ua, ub, &z0, &z1);
            z[2 * q] = z0;
            if (2 * q + 1 < d) z[2 * q + 1] = z1;
        }
        double nz = 0.0;
        for (int a = 0; a < d; ++a) nz += z[a] * z[a];
        nz = sqrt(nz);
        for (int a = 0; a < d; ++a) {
            double s2 = 0.0;
            for (int b = 0; b <= a; ++b) s2 += Lsig[a * d + b] * z[b];
            v[a] = s2 / nz;
        }
        /* initial bracket position and slice height */
        double U, uh;
        draw2(key, P_STEP, chain, iter, (uint32_t)st, 0u, &U, &uh);
        if (beta >= 0.0)   /* tempered slice height: log Pi(x) + beta log L(x) + log uh */
            s.logy = (s.uniform_prior ? 0.0 : or_logprior(p, x)) + beta * (*logL) + log(uh);
        else
            s.logy = s.uniform_prior ? -INFINITY : or_logprior(p, x) + log(uh);
        double tL = -w * U, tR = tL + w;
        /* linear stepping-out, at most stepout_cap expansions per side */
        int nl = 0, nr = 0;
        while (nl < stepout_cap && inside(&s, tL)) { tL -= w; ++nl; }
        if (nl == stepout_cap) c.stepout_caps++;
        while (nr < stepout_cap && inside(&s, tR)) { tR += w; ++nr; }
        if (nr == stepout_cap) c.stepout_caps++;
        /* shrinkage */
        int ns = 0, acc = 0;
        for (; ns < shrink_cap; ++ns) {
            double us, unused;
            draw2(key, P_SHRINK, chain, iter, (uint32_t)st, (uint32_t)ns, &us, &unused);
            double t = tL + us * (tR - tL);
            if (inside(&s, t)) {
                for (int a = 0; a < d; ++a) x[a] = x[a] + t * v[a];
                *logL = s.last_logL;
                acc = 1;
                ++ns;
                break;
            }
            if (t < 0.0) tL = t; else tR = t;
        }
        if (!acc) c.shrink_caps++;
        if (trace) {
            trace[4 * st + 0] = nl; trace[4 * st + 1] = nr;
            trace[4 * st + 2] = ns; trace[4 * st + 3] = acc;
        }
    }
    free(z);
    if (counters) {
        counters[0] += c.evals; counters[1] += c.tests; counters[2] += c.prior_rejects;
        counters[3] += c.stepout_caps; counters[4] += c.shrink_caps; counters[5] += c.nonfinite;
    }
}

void or_hrss_chain(const void *pp, double *x, double *logL, double Lstar, const double *Lsig,
                   double w, int p_steps, int stepout_cap, int shrink_cap, uint64_t seed,
                   uint32_t run_id, uint32_t iter, uint32_t chain, int64_t *counters,
                   int32_t *trace)
{
    hrss_chain((const oprob *)pp, x, logL, Lstar, -1.0, Lsig, w, p_steps, stepout_cap,
               shrink_cap, seed, run_id, iter, chain, counters, trace);
}

/* The same chain on the tempered density Pi(x) L(x)^beta, beta >= 0, without a hard
 * constraint (the slice-sampling mutation of adaptive tempered SMC, App. "Adaptive
 * non-equilibrium samplers", SMC-SS): slice height log Pi(x0) + beta log L(x0) - Exp(1). */
void or_hrss_chain_tempered(const void *pp, double *x, double *logL, double beta,
                            const double *Lsig, double w, int p_steps, int stepout_cap,
                            int shrink_cap, uint64_t seed, uint32_t run_id, uint32_t iter,
                            uint32_t chain, int64_t *counters, int32_t *trace)
{
    hrss_chain((const oprob *)pp, x, logL, 0.0, beta < 0.0 ? 0.0 : beta, Lsig, w, p_steps,
               stepout_cap, shrink_cap, seed, run_id, iter, chain, counters, trace);
}

/*
 * One chain of p constrained Gaussian random-walk Metropolis steps, the alternative replacement
 * kernel (Sec. 3.1 "Replacement strategies"; App. "Slice Sampling vs Random Walk"): the
 * proposal is x' = x + s Lsig z with z ~ N(0, I), i.e. Gaussian with the live-set covariance
 * scaled by s^2; it is accepted if x' lies in the prior support, passes the Metropolis test of
 * the prior ratio (non-uniform priors: log Pi(x') > log Pi(x) + log uh) and has
 * logL(x') > Lstar; otherwise the chain stays where it is.  z uses the draws of an HRSS
 * direction (purpose DIR) and uh the second uniform of the step draw (purpose STEP).
 * trace (optional, 4 ints per step): 0, 0, 1 if the proposal was evaluated, accepted (1 / 0).
 * x and *logL are updated in place.
 */
void or_rw_chain(const void *pp, double *x, double *logL, double Lstar, const double *Lsig,
                 double scale, int p_steps, uint64_t seed, uint32_t run_id, uint32_t iter,
                 uint32_t chain, int64_t *counters, int32_t *trace)
{
    const oprob *p = (const oprob *)pp;
    const int d = p->d;
    okey key = { { (uint32_t)seed, (uint32_t)(seed >> 32) ^ run_id } };
    double *z = (double *)malloc(sizeof(double) * d * 2);
    double *y = z + d;
    octr c; memset(&c, 0, sizeof c);
    const int uniform_prior = (p->prior_kind == PRIOR_BOX);
    for (int st = 0; st < p_steps; ++st) {
        for (int q = 0; 2 * q < d; ++q) {
            double ua, ub, z0, z1;
            draw2(key, P_DIR, chain, iter, (uint32_t)st, (uint32_t)q, &ua, &ub);
            box_muller(ua, ub, &z0, &z1);
            z[2 * q] = z0;
            if (2 * q + 1 < d) z[2 * q + 1] = z1;
        }
        for (int a = 0; a < d; ++a) {
            double s2 = 0.0;
            for (int b = 0; b <= a; ++b) s2 += Lsig[a * d + b] * z[b];
            y[a] = x[a] + s2 * scale;
        }
        double U, uh;
        draw2(key, P_STEP, chain, iter, (uint32_t)st, 0u, &U, &uh);
        (void)U;
        int evald = 0, acc = 0;
        c.tests++;
        if (!prior_in_support(p, y) ||
            (!uniform_prior && !(or_logprior(p, y) > or_logprior(p, x) + log(uh)))) {
            c.prior_rejects++;
        } else {
            double L = or_loglik(p, y);
            c.evals++;
            evald = 1;
            if (isnan(L) || L == INFINITY) { c.nonfinite++; L = -INFINITY; }
            if (L > Lstar) {
                memcpy(x, y, sizeof(double) * d);
                *logL = L;
                acc = 1;
            }
        }
        if (trace) {
            trace[4 * st + 0] = 0; trace[4 * st + 1] = 0;
            trace[4 * st + 2] = evald; trace[4 * st + 3] = acc;
        }
    }
    free(z);
    if (counters) {
        counters[0] += c.evals; counters[1] += c.tests; counters[2] += c.prior_rejects;
        counters[5] += c.nonfinite;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* NS outer loop                                                                               */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    const oprob *p;
    int m, k, p_steps, stepout_cap, shrink_cap;
    double width, term_frac;
    uint64_t seed;
    uint32_t run_id;
    /* state */
    double *x;        /* m x d, row per particle */
    double *logL;     /* m */
    int *perm;        /* m: ascending (logL, index) */
    double Lstar;
    double logZ, logX, M;   /* M = posterior mean of logL so far, H = M - logZ */
    int64_t iter;
    int64_t counters[6];
    double *Lsig;     /* d x d, last whitening factor */
    int *parents;     /* k, last resample */
    double *dead;     /* dead logL record */
    double *dead_x;   /* the dead points' coordinates, [cap_dead][d] */
    int64_t n_dead, cap_dead;
    int whiten_fallbacks;
    int replacement;  /* 0: HRSS (width = slice width); 1: random walk (width = step scale) */
    int freeze;       /* 1: the whitening factor of the first iteration is kept for the run */
    int held;         /* 1: a caller-supplied factor is kept (freeze only; no whitening at all) */
    int diag;         /* 1: the metric keeps only the survivors' variances (diagonal M) */
    /* adaptive tempered SMC (or_smc_*): all m particles move each step */
    int smc;
    double beta, ess_frac;
} orun;

void or_run_free(void *rr)
{
    orun *r = (orun *)rr;
    if (!r) return;
    free(r->x); free(r->logL); free(r->perm); free(r->Lsig); free(r->parents); free(r->dead);
    free(r->dead_x);
    free(r);
}

void *or_run_new(const void *pp, int m, int k, int p_steps, double width, int stepout_cap,
                 int shrink_cap, double term_frac, uint64_t seed, uint32_t run_id)
{
    const oprob *p = (const oprob *)pp;
    if (!p || m < 2 || k < 1 || k > m - 1 || p_steps < 1 || !(width > 0.0)) return NULL;
    orun *r = (orun *)calloc(1, sizeof(orun));
    int d = p->d;
    r->p = p; r->m = m; r->k = k; r->p_steps = p_steps; r->width = width;
    r->stepout_cap = stepout_cap; r->shrink_cap = shrink_cap; r->term_frac = term_frac;
    r->seed = seed; r->run_id = run_id;
    r->x = (double *)malloc(sizeof(double) * (size_t)m * d);
    r->logL = (double *)malloc(sizeof(double) * m);
    r->perm = (int *)malloc(sizeof(int) * m);
    r->Lsig = (double *)calloc((size_t)d * d, sizeof(double));
    r->parents = (int *)calloc(k, sizeof(int));
    r->cap_dead = 1 << 16;
    r->dead = (double *)malloc(sizeof(double) * r->cap_dead);
    r->dead_x = (double *)malloc(sizeof(double) * (size_t)r->cap_dead * d);
    return r;
}

static const double *g_sort_logL;
static int cmp_logL_index(const void *a, const void *b)
{
    int i = *(const int *)a, j = *(const int *)b;
    double li = g_sort_logL[i], lj = g_sort_logL[j];
    if (li < lj) return -1;
    if (li > lj) return 1;
    return (i > j) - (i < j);
}

static double lse2(double a, double b)
{
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    double mx = a > b ? a : b;
    return mx + log(exp(a - mx) + exp(b - mx));
}

/* Delete-k: sort by (logL, index); the first k are the deaths; L* is the k-th worst.  Then
 * account the k deaths one at a time at live counts m, m-1, ..., m-k+1. */
static void select_and_account(orun *r)
{
    const int m = r->m, k = r->k;
    for (int i = 0; i < m; ++i) r->perm[i] = i;
    g_sort_logL = r->logL;
    qsort(r->perm, (size_t)m, sizeof(int), cmp_logL_index);
    r->Lstar = r->logL[r->perm[k - 1]];
    for (int j = 1; j <= k; ++j) {
        double n = (double)(m - j + 1);
        double L = r->logL[r->perm[j - 1]];
        double logdX = r->logX + log(-expm1(-1.0 / n));   /* log(X_{j-1} - X_j) */
        r->logX -= 1.0 / n;
        double lw = L + logdX;
        double zn = lse2(r->logZ, lw);
        double Mn = (r->logZ == -INFINITY ? 0.0 : exp(r->logZ - zn) * r->M);
        if (lw != -INFINITY) Mn += exp(lw - zn) * L;
        r->M = Mn;
        r->logZ = zn;
        if (r->n_dead == r->cap_dead) {
            r->cap_dead *= 2;
            r->dead = (double *)realloc(r->dead, sizeof(double) * r->cap_dead);
            r->dead_x = (double *)realloc(r->dead_x,
                                          sizeof(double) * (size_t)r->cap_dead * r->p->d);
        }
        memcpy(r->dead_x + (size_t)r->n_dead * r->p->d, r->x + (size_t)r->perm[j - 1] * r->p->d,
               sizeof(double) * r->p->d);
        r->dead[r->n_dead++] = L;
    }
}

static int termination_reached(const orun *r)
{
    if (!(r->term_frac > 0.0)) return 0;
    double maxL = r->logL[r->perm[r->m - 1]];
    return (r->logX + maxL - r->logZ) < log(r->term_frac);
}

/* Draw m points from the prior, evaluate them, then the first delete-k.  Returns 1 if the
 * termination test already holds, 0 otherwise. */
static void draw_initial(orun *r)
{
    const oprob *p = r->p;
    const int d = p->d, m = r->m;
    okey key = { { (uint32_t)r->seed, (uint32_t)(r->seed >> 32) ^ r->run_id } };
    for (int i = 0; i < m; ++i) {
        double *xi = r->x + (size_t)i * d;
        for (int q = 0; 2 * q < d; ++q) {
            double ua, ub, a0, a1;
            draw2(key, P_INIT, (uint32_t)i, 0u, 0u, (uint32_t)q, &ua, &ub);
            if (p->prior_kind == PRIOR_BOX) {
                a0 = ua; a1 = ub;
                xi[2 * q] = p->pa[2 * q] + (p->pb[2 * q] - p->pa[2 * q]) * a0;
                if (2 * q + 1 < d)
                    xi[2 * q + 1] = p->pa[2 * q + 1] + (p->pb[2 * q + 1] - p->pa[2 * q + 1]) * a1;
            } else {
                box_muller(ua, ub, &a0, &a1);
                xi[2 * q] = p->pa[2 * q] + p->pb[2 * q] * a0;
                if (2 * q + 1 < d) xi[2 * q + 1] = p->pa[2 * q + 1] + p->pb[2 * q + 1] * a1;
            }
        }
        double L = or_loglik(p, xi);
        if (isnan(L) || L == INFINITY) { r->counters[5]++; L = -INFINITY; }
        r->logL[i] = L;
    }
}

int or_init(void *rr)
{
    orun *r = (orun *)rr;
    draw_initial(r);
    r->logZ = -INFINITY; r->logX = 0.0; r->M = 0.0; r->iter = 0; r->n_dead = 0;
    select_and_account(r);
    return termination_reached(r);
}

/* Whitening: covariance (divided by n) of the m-k survivors (SMC: of all m particles) plus
 * 1e-12 tr/d jitter, and its lower Cholesky factor; diagonal fallback if the factorisation
 * fails.  The two passes work on the points minus the first of them (the covariance does not
 * change under a shift), so survivors that coincide give an exactly zero covariance. */
static void whiten(orun *r)
{
    const int d = r->p->d, m = r->m, k = r->smc ? 0 : r->k, n = m - k;
    double *mean = (double *)calloc(d, sizeof(double));
    double *C = (double *)calloc((size_t)d * d, sizeof(double));
    const double *x0 = r->x + (size_t)r->perm[k] * d;
    for (int t = k; t < m; ++t) {
        const double *xi = r->x + (size_t)r->perm[t] * d;
        for (int a = 0; a < d; ++a) mean[a] += xi[a] - x0[a];
    }
    for (int a = 0; a < d; ++a) mean[a] /= n;
    for (int t = k; t < m; ++t) {
        const double *xi = r->x + (size_t)r->perm[t] * d;
        for (int a = 0; a < d; ++a)
            for (int b = 0; b <= a; ++b)
                C[a * d + b] += (xi[a] - x0[a] - mean[a]) * (xi[b] - x0[b] - mean[b]);
    }
    double tr = 0.0;
    for (int a = 0; a < d; ++a) {
        for (int b = 0; b <= a; ++b) { C[a * d + b] /= n; C[b * d + a] = C[a * d + b]; }
        tr += C[a * d + a];
    }
    for (int a = 0; a < d; ++a) C[a * d + a] += 1e-12 * tr / d;
    if (r->diag)   /* a diagonal conditioning matrix: the variances alone */
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b)
                if (a != b) C[a * d + b] = 0.0;
    if (cholesky_lower(C, r->Lsig, d) != 0) {
        r->whiten_fallbacks++;
        memset(r->Lsig, 0, sizeof(double) * (size_t)d * d);
        for (int a = 0; a < d; ++a) r->Lsig[a * d + a] = sqrt(C[a * d + a] > 0 ? C[a * d + a] : 1.0);
    }
    free(mean); free(C);
}

/* One outer iteration: whiten, resample, mutate, replace, delete-k, account, terminate?
 * Returns 1 when terminated, 0 otherwise, -4 if no survivor lies strictly above L*. */
int or_step(void *rr, int n_threads)
{
    orun *r = (orun *)rr;
    const oprob *p = r->p;
    const int d = p->d, m = r->m, k = r->k;
    const uint32_t it = (uint32_t)(r->iter + 1);
    okey key = { { (uint32_t)r->seed, (uint32_t)(r->seed >> 32) ^ r->run_id } };
    if (!r->freeze || (r->iter == 0 && !r->held)) whiten(r);
    /* resample: uniform over survivors with logL > L*, in ascending (logL, index) order */
    int t0 = k;
    while (t0 < m && !(r->logL[r->perm[t0]] > r->Lstar)) ++t0;
    const int ns = m - t0;
    if (ns == 0) return -4;
    for (int j = 0; j < k; ++j) {
        double u, unused;
        draw2(key, P_RESAMPLE, (uint32_t)j, it, 0u, 0u, &u, &unused);
        int q = (int)floor(u * ns);
        if (q > ns - 1) q = ns - 1;
        r->parents[j] = r->perm[t0 + q];
    }
    /* mutate: k independent chains */
    double *xn = (double *)malloc(sizeof(double) * (size_t)k * d);
    double *ln = (double *)malloc(sizeof(double) * k);
    int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0;
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads) reduction(+:c0,c1,c2,c3,c4,c5)
#endif
    for (int j = 0; j < k; ++j) {
        int64_t cc[6] = { 0, 0, 0, 0, 0, 0 };
        memcpy(xn + (size_t)j * d, r->x + (size_t)r->parents[j] * d, sizeof(double) * d);
        ln[j] = r->logL[r->parents[j]];
        if (r->replacement == 1)
            or_rw_chain(p, xn + (size_t)j * d, &ln[j], r->Lstar, r->Lsig, r->width, r->p_steps,
                        r->seed, r->run_id, it, (uint32_t)j, cc, NULL);
        else
            or_hrss_chain(p, xn + (size_t)j * d, &ln[j], r->Lstar, r->Lsig, r->width, r->p_steps,
                          r->stepout_cap, r->shrink_cap, r->seed, r->run_id, it, (uint32_t)j, cc,
                          NULL);
        c0 += cc[0]; c1 += cc[1]; c2 += cc[2]; c3 += cc[3]; c4 += cc[4]; c5 += cc[5];
    }
    (void)n_threads;
    r->counters[0] += c0; r->counters[1] += c1; r->counters[2] += c2;
    r->counters[3] += c3; r->counters[4] += c4; r->counters[5] += c5;
    /* replace: the j-th new point takes the slot of the j-th deleted point */
    for (int j = 0; j < k; ++j) {
        int slot = r->perm[j];
        memcpy(r->x + (size_t)slot * d, xn + (size_t)j * d, sizeof(double) * d);
        r->logL[slot] = ln[j];
    }
    free(xn); free(ln);
    r->iter = it;
    select_and_account(r);
    return termination_reached(r);
}

/* ------------------------------------------------------------------------------------------ */
/* Adaptive tempered SMC with the slice-sampling mutation (App. "Adaptive Tempered SMC";       */
/* SMC-SS in App. "Adaptive non-equilibrium samplers")                                        */
/* ------------------------------------------------------------------------------------------ */
/* m particles; each step: the next inverse temperature by bisection on the ESS of the
 * incremental weights, the log-mean-weight evidence increment, systematic resampling, then p
 * tempered HRSS steps per particle with directions whitened by the particle covariance.
 * ess_frac is the ESS target rho in (0, 1).  Returns NULL on invalid input. */
void *or_smc_new(const void *pp, int m, int p_steps, double width, int stepout_cap,
                 int shrink_cap, double ess_frac, uint64_t seed, uint32_t run_id)
{
    const oprob *p = (const oprob *)pp;
    if (!p || m < 2 || p_steps < 1 || !(width > 0.0) || !(ess_frac > 0.0 && ess_frac < 1.0))
        return NULL;
    orun *r = (orun *)calloc(1, sizeof(orun));
    const int d = p->d;
    r->p = p; r->m = m; r->k = m; r->p_steps = p_steps; r->width = width;
    r->stepout_cap = stepout_cap; r->shrink_cap = shrink_cap; r->term_frac = 0.0;
    r->seed = seed; r->run_id = run_id;
    r->smc = 1; r->ess_frac = ess_frac;
    r->x = (double *)malloc(sizeof(double) * (size_t)m * d);
    r->logL = (double *)malloc(sizeof(double) * m);
    r->perm = (int *)malloc(sizeof(int) * m);
    r->Lsig = (double *)calloc((size_t)d * d, sizeof(double));
    r->parents = (int *)calloc(m, sizeof(int));
    r->cap_dead = 1;
    r->dead = (double *)malloc(sizeof(double));
    r->dead_x = (double *)malloc(sizeof(double) * d);
    return r;
}

/* Prior draws (the same stream as nested sampling's) at beta = 0, log Z = 0. */
void or_smc_init(void *rr)
{
    orun *r = (orun *)rr;
    draw_initial(r);
    for (int i = 0; i < r->m; ++i) r->perm[i] = i;
    r->beta = 0.0; r->logZ = 0.0; r->logX = 0.0; r->M = 0.0; r->iter = 0; r->Lstar = 0.0;
}

/* ESS of the incremental weights exp((b - beta) (L_i - Lmax)), L = -inf weighing 0. */
static double smc_ess(const orun *r, double b, double Lmax)
{
    double s1 = 0.0, s2 = 0.0;
    for (int i = 0; i < r->m; ++i) {
        if (r->logL[i] == -INFINITY) continue;
        const double e = exp((b - r->beta) * (r->logL[i] - Lmax));
        s1 += e;
        s2 += e * e;
    }
    return s1 * s1 / s2;
}

/* One SMC step.  Returns 1 once beta has reached 1 (after that step's mutation), 0 otherwise,
 * -4 if every particle has log L = -inf. */
int or_smc_step(void *rr, int n_threads)
{
    orun *r = (orun *)rr;
    const oprob *p = r->p;
    const int d = p->d, m = r->m;
    const uint32_t it = (uint32_t)(r->iter + 1);
    okey key = { { (uint32_t)r->seed, (uint32_t)(r->seed >> 32) ^ r->run_id } };
    double Lmax = -INFINITY;
    for (int i = 0; i < m; ++i) if (r->logL[i] > Lmax) Lmax = r->logL[i];
    if (Lmax == -INFINITY) return -4;
    /* next temperature: ESS(b) = rho m by 50 bisection steps on (beta, 1] */
    const double target = r->ess_frac * m;
    double nb = 1.0;
    if (smc_ess(r, 1.0, Lmax) < target) {
        double lo = r->beta, hi = 1.0;
        for (int t = 0; t < 50; ++t) {
            const double mid = 0.5 * (lo + hi);
            if (smc_ess(r, mid, Lmax) >= target) lo = mid; else hi = mid;
        }
        nb = lo > r->beta ? lo : hi;
    }
    /* evidence increment: log of the mean incremental weight */
    const double db = nb - r->beta;
    double *w = (double *)malloc(sizeof(double) * m);
    double sw = 0.0;
    for (int i = 0; i < m; ++i) {
        w[i] = r->logL[i] == -INFINITY ? 0.0 : exp(db * (r->logL[i] - Lmax));
        sw += w[i];
    }
    r->logZ += db * Lmax + log(sw) - log((double)m);
    /* systematic resampling: positions (u + j) / m against the cumulative normalised weights */
    double u, unused;
    draw2(key, P_RESAMPLE, 0u, it, 0u, 0u, &u, &unused);
    int i = 0;
    double cum = w[0] / sw;
    for (int j = 0; j < m; ++j) {
        const double pos = (u + j) / m;
        while (cum < pos && i < m - 1) { ++i; cum += w[i] / sw; }
        r->parents[j] = i;
    }
    double *xn = (double *)malloc(sizeof(double) * (size_t)m * d);
    double *ln = (double *)malloc(sizeof(double) * m);
    for (int j = 0; j < m; ++j) {
        memcpy(xn + (size_t)j * d, r->x + (size_t)r->parents[j] * d, sizeof(double) * d);
        ln[j] = r->logL[r->parents[j]];
    }
    memcpy(r->x, xn, sizeof(double) * (size_t)m * d);
    memcpy(r->logL, ln, sizeof(double) * m);
    r->beta = nb;
    r->Lstar = nb;
    r->iter = it;
    /* mutation at the new temperature, particle j by chain j */
    whiten(r);
    int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0;
#ifdef _OPENMP
    if (n_threads < 1) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads) reduction(+:c0,c1,c2,c3,c4,c5)
#endif
    for (int j = 0; j < m; ++j) {
        int64_t cc[6] = { 0, 0, 0, 0, 0, 0 };
        hrss_chain(p, r->x + (size_t)j * d, &r->logL[j], 0.0, nb, r->Lsig, r->width,
                   r->p_steps, r->stepout_cap, r->shrink_cap, r->seed, r->run_id, it,
                   (uint32_t)j, cc, NULL);
        c0 += cc[0]; c1 += cc[1]; c2 += cc[2]; c3 += cc[3]; c4 += cc[4]; c5 += cc[5];
    }
    (void)n_threads;
    r->counters[0] += c0; r->counters[1] += c1; r->counters[2] += c2;
    r->counters[3] += c3; r->counters[4] += c4; r->counters[5] += c5;
    free(w); free(xn); free(ln);
    return nb == 1.0;
}

/* Replacement kernel of the run: 0 HRSS (the default), 1 constrained random walk with the
 * run's width as the proposal scale.  Returns 0, or -1 for an unknown kind. */
int or_run_set_replacement(void *rr, int kind)
{
    orun *r = (orun *)rr;
    if (!r || (kind != 0 && kind != 1)) return -1;
    r->replacement = kind;
    return 0;
}

/* Whitening kept from the first iteration on (1) or recomputed every iteration (0, the
 * default): the fixed-scale proposal variant of the random-walk comparison. */
int or_run_set_freeze(void *rr, int on)
{
    orun *r = (orun *)rr;
    if (!r || (on != 0 && on != 1)) return -1;
    r->freeze = on;
    return 0;
}

/* Direction metric from the survivors' full covariance (0, the default) or from their
 * variances alone (1): the diagonal restriction the paper suggests for high dimensions. */
int or_run_set_diag(void *rr, int on)
{
    orun *r = (orun *)rr;
    if (!r || (on != 0 && on != 1)) return -1;
    r->diag = on;
    return 0;
}

/* With the whitening frozen: keep the caller's lower-triangular factor L (d x d, row-major;
 * entries above the diagonal are ignored) for the whole run instead of computing one, e.g. the
 * Cholesky factor of the target's covariance for a proposal matched to the target. */
int or_run_set_factor(void *rr, const double *L)
{
    orun *r = (orun *)rr;
    if (!r || !L || !r->freeze) return -1;
    const int d = r->p->d;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) r->Lsig[a * d + b] = b <= a ? L[a * d + b] : 0.0;
    r->held = 1;
    return 0;
}

/* Evidence with the live set's remaining contribution added (non-destructive):
 * out = {logZ, sqrt(H/m), H}. */
void or_logz(const void *rr, double out[3])
{
    const orun *r = (const orun *)rr;
    const int m = r->m, k = r->k, n = m - k;
    double mx = -INFINITY;
    for (int t = k; t < m; ++t) if (r->logL[r->perm[t]] > mx) mx = r->logL[r->perm[t]];
    double s = 0.0;
    for (int t = k; t < m; ++t) s += exp(r->logL[r->perm[t]] - mx);
    double lme = mx + log(s) - log((double)n);
    double zf = lse2(r->logZ, r->logX + lme);
    double Mf = (r->logZ == -INFINITY ? 0.0 : exp(r->logZ - zf) * r->M);
    for (int t = k; t < m; ++t) {
        double L = r->logL[r->perm[t]];
        double lw = r->logX - log((double)n) + L;
        if (lw != -INFINITY) Mf += exp(lw - zf) * L;
    }
    double H = Mf - zf;
    out[0] = zf;
    out[1] = sqrt(H > 0 ? H / m : 0.0);
    out[2] = H;
}

/* State access for parity tests. */
void or_get_state(const void *rr, double *x, double *logL, int *perm, double scalars[4],
                  int64_t *iter, int64_t counters[6])
{
    const orun *r = (const orun *)rr;
    const int d = r->p->d, m = r->m;
    if (x) memcpy(x, r->x, sizeof(double) * (size_t)m * d);
    if (logL) memcpy(logL, r->logL, sizeof(double) * m);
    if (perm) memcpy(perm, r->perm, sizeof(int) * m);
    if (scalars) { scalars[0] = r->Lstar; scalars[1] = r->logZ; scalars[2] = r->logX; scalars[3] = r->M; }
    if (iter) *iter = r->iter;
    if (counters) memcpy(counters, r->counters, sizeof(int64_t) * 6);
}

/* Overwrite the live set and evidence scalars, then recompute the delete-k order (without
 * re-accounting the deaths). */
void or_set_state(void *rr, const double *x, const double *logL, const double scalars3[3],
                  int64_t iter)
{
    orun *r = (orun *)rr;
    const int d = r->p->d, m = r->m;
    memcpy(r->x, x, sizeof(double) * (size_t)m * d);
    memcpy(r->logL, logL, sizeof(double) * m);
    /* a NaN or +inf log L is a rejected point (-inf), counted like a computed one */
    for (int i = 0; i < m; ++i)
        if (isnan(r->logL[i]) || r->logL[i] == INFINITY) { r->logL[i] = -INFINITY; r->counters[5]++; }
    r->logZ = scalars3[0]; r->logX = scalars3[1]; r->M = scalars3[2];
    r->iter = iter;
    for (int i = 0; i < m; ++i) r->perm[i] = i;
    g_sort_logL = r->logL;
    qsort(r->perm, (size_t)m, sizeof(int), cmp_logL_index);
    r->Lstar = r->logL[r->perm[r->k - 1]];
}

void or_get_aux(const void *rr, double *Lsig, int *parents)
{
    const orun *r = (const orun *)rr;
    const int d = r->p->d;
    if (Lsig) memcpy(Lsig, r->Lsig, sizeof(double) * (size_t)d * d);
    if (parents) memcpy(parents, r->parents, sizeof(int) * r->k);
}

/* The dead points' coordinates, [n][d] row by row; returns the number of dead points. */
int64_t or_get_dead_x(const void *rr, double *out, int64_t cap)
{
    const orun *r = (const orun *)rr;
    const int64_t n = r->n_dead < cap ? r->n_dead : cap;
    if (out && n > 0) memcpy(out, r->dead_x, sizeof(double) * (size_t)n * r->p->d);
    return r->n_dead;
}

int64_t or_get_dead(const void *rr, double *out, int64_t cap)
{
    const orun *r = (const orun *)rr;
    int64_t n = r->n_dead < cap ? r->n_dead : cap;
    if (out && n > 0) memcpy(out, r->dead, sizeof(double) * n);
    return r->n_dead;
}

/* ------------------------------------------------------------------------------------------ */
/* Post-hoc geometric uncertainty (App. "Estimation of prior volumes and propagation of         */
/* geometric uncertainty")                                                                     */
/* ------------------------------------------------------------------------------------------ */
/*
 * Deaths i = 1..N in likelihood order: the dead record (batch after batch; the j-th death of a
 * batch has n = m - (j-1) live points) followed by the final survivors in ascending logL with
 * n = nf, nf-1, ..., 1.  Replica r draws shrinkages t_i = u_i^(1/n_i), u_i uniform: deaths
 * 2h+1 and 2h+2 take the two uniforms of Philox (purpose GEOM, index r, counter word h), so
 * log t_i = log(u_i)/n_i and
 * log X_i = log X_{i-1} + log t_i, X_0 = 1.  Trapezoid elements dX_i = (X_{i-1} - X_{i+1})/2
 * with X_{N+1} = 0, i.e. dX_i = X_{i-1} (1 - t_i t_{i+1}) / 2 with t_{N+1} = 0, evaluated as
 * log dX_i = log X_{i-1} + log1p(-exp(log t_i + log t_{i+1})) - log 2.
 * Weights log w_i = beta logL_i + log dX_i, where the tempered term is 0 at beta = 0 (prior
 * volumes, also for logL = -inf); log Z_r = log sum_i w_i.  Geometric-mean weights
 * log w~_i = (1/R) sum_r log w_i; Kish ESS = (sum w~)^2 / sum w~^2.
 * Outputs: logz[R]; logw_mean[N] and *ess unless NULL.
 */
static double tempered(double beta, double lL) { return beta == 0.0 ? 0.0 : beta * lL; }

void or_geom(const double *dead, int64_t n_dead, const double *final_sorted, int64_t nf,
             int m, int k, int R, double beta, uint64_t seed, uint32_t run_id, double *logz,
             double *logw_mean, double *ess)
{
    const int64_t N = n_dead + nf;
    okey key = { { (uint32_t)seed, (uint32_t)(seed >> 32) ^ run_id } };
    double *lt = (double *)malloc(sizeof(double) * (size_t)(N + 1));     /* log t_1..t_{N+1} */
    double *lw = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *acc = (double *)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    for (int r = 0; r < R; ++r) {
        for (int64_t i = 1; i <= N; ++i) {
            const int64_t g = i - 1;
            const double n = (g < n_dead) ? (double)(m - (int)(g % k)) : (double)(nf - (g - n_dead));
            double ua, ub;
            draw2(key, P_GEOM, (uint32_t)r, (uint32_t)(g >> 1), 0u, 0u, &ua, &ub);
            lt[i - 1] = log((g & 1) ? ub : ua) / n;
        }
        lt[N] = -INFINITY;
        double lx = 0.0, mx = -INFINITY;       /* lx = log X_{i-1} */
        for (int64_t i = 1; i <= N; ++i) {
            const double lL = (i - 1 < n_dead) ? dead[i - 1] : final_sorted[i - 1 - n_dead];
            const double ldx = lx + log1p(-exp(lt[i - 1] + lt[i])) - log(2.0);
            lw[i - 1] = tempered(beta, lL) + ldx;
            acc[i - 1] += lw[i - 1];
            if (lw[i - 1] > mx) mx = lw[i - 1];
            lx += lt[i - 1];
        }
        double sum = 0.0;
        if (mx > -INFINITY)
            for (int64_t i = 0; i < N; ++i) sum += exp(lw[i] - mx);
        logz[r] = mx > -INFINITY ? mx + log(sum) : -INFINITY;
    }
    double m1 = -INFINITY;
    for (int64_t i = 0; i < N; ++i) {
        acc[i] /= R;
        if (logw_mean) logw_mean[i] = acc[i];
        if (acc[i] > m1) m1 = acc[i];
    }
    if (ess) {
        double s1 = 0.0, s2 = 0.0;
        if (m1 > -INFINITY)
            for (int64_t i = 0; i < N; ++i) {
                const double e = exp(acc[i] - m1);
                s1 += e;
                s2 += e * e;
            }
        *ess = s2 > 0.0 ? s1 * s1 / s2 : 0.0;
    }
    free(lt);
    free(lw);
    free(acc);
}

/* Weighted posterior samples: the geometric-mean weights w~_i of or_geom (R replicas, beta),
 * then n draws by systematic resampling: positions (u + j) / n, u uniform (Philox purpose
 * POST, counter 0), against the cumulative normalised weights in death order; sample j is the
 * first death whose cumulative weight reaches its position (the last if rounding leaves none).
 * dead_x[n_dead][d] and final_x[nf][d] hold the coordinates in the order of dead and
 * final_sorted.  Outputs x[n][d] and idx[n] (death indices). */
void or_posterior_samples(const double *dead, const double *dead_x, int64_t n_dead,
                          const double *final_sorted, const double *final_x, int64_t nf, int d,
                          int m, int k, int R, double beta, uint64_t seed, uint32_t run_id,
                          int n, double *x, int64_t *idx)
{
    const int64_t N = n_dead + nf;
    double *lw = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *lz = (double *)malloc(sizeof(double) * (size_t)R);
    or_geom(dead, n_dead, final_sorted, nf, m, k, R, beta, seed, run_id, lz, lw, NULL);
    double mx = -INFINITY;
    for (int64_t i = 0; i < N; ++i) if (lw[i] > mx) mx = lw[i];
    double *cum = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        s += lw[i] > -INFINITY ? exp(lw[i] - mx) : 0.0;
        cum[i] = s;
    }
    for (int64_t i = 0; i < N; ++i) cum[i] /= s;
    okey key = { { (uint32_t)seed, (uint32_t)(seed >> 32) ^ run_id } };
    double u, unused;
    draw2(key, P_POST, 0u, 0u, 0u, 0u, &u, &unused);
    int64_t i = 0;
    for (int j = 0; j < n; ++j) {
        const double pos = (u + j) / n;
        while (i < N - 1 && cum[i] < pos) ++i;
        idx[j] = i;
        const double *src = i < n_dead ? dead_x + (size_t)i * d : final_x + (size_t)(i - n_dead) * d;
        memcpy(x + (size_t)j * d, src, sizeof(double) * d);
    }
    free(lw); free(lz); free(cum);
}
