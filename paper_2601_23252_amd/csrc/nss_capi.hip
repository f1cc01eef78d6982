// C ABI of the gfx950 Nested Slice Sampling library: argument validation, problem preparation
// (host FP64), device allocation and the per-iteration launch sequence.
#include "../../include/nss.h"
#include "nss_internal.hpp"

#include <math.h>
#include <string.h>

#include <string>
#include <utility>
#include <vector>

using namespace nss;

struct ns_ctx {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    ns_config cfg;
    int d = 0, D = 0, m = 0, m_pad = 0, k = 0, p = 0, mode = 0;
    DevProblem P;
    DevRun R;
    double *part1 = nullptr, *part2 = nullptr;
    // 16-bit W fragments per format, and the rounded remainders for the split modes
    const uint4 *wf_bf16 = nullptr, *wf_fp16 = nullptr, *wf_bf16_lo = nullptr, *wf_fp16_lo = nullptr;
    int covG = 1;
    int *h_iscal = nullptr;   // pinned mirror of iscal[0..7]
    int done = 0;
    std::vector<void *> allocs;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    double hrss_ms = 0.0;
    long long hrss_launches = 0;
    std::string err;
};

static std::string g_init_err = "";

#define CK(expr)                                                                           \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                  \
            return NS_EDEVICE;                                                             \
        }                                                                                  \
    } while (0)

static ns_status fail(ns_ctx *ctx, ns_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg; else g_init_err = msg;
    return st;
}

template <typename T>
static ns_status dalloc(ns_ctx *ctx, T **ptr, size_t count)
{
    void *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
        ctx->err = "hipMalloc failed";
        return NS_ENOMEM;
    }
    ctx->allocs.push_back(p);
    *ptr = (T *)p;
    return NS_OK;
}

extern "C" void ns_config_default(ns_config *c)
{
    if (!c) return;
    memset(c, 0, sizeof(*c));
    c->n_live = 1000;
    c->k = 100;
    c->chain_len = 0;
    c->width = 0.0;
    c->stepout_cap = 10;
    c->shrink_cap = 100;
    c->term_frac = 1e-3;
    c->seed = 0;
    c->run_id = 0;
    c->precision = NS_FP64;
    c->max_iter = 100000;
    c->flags = 0;
}

// ---- host-side problem preparation (FP64) ----
static int chol_lower(const double *A, double *L, int n)
{
    for (int i = 0; i < n * n; ++i) L[i] = 0.0;
    for (int i = 0; i < n; ++i)
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
    return 0;
}
// inverse of a lower-triangular matrix by forward substitution on the identity
static void tri_inv_lower(const double *L, double *W, int n)
{
    for (int i = 0; i < n * n; ++i) W[i] = 0.0;
    for (int c = 0; c < n; ++c)
        for (int i = c; i < n; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int t = c; t < i; ++t) s -= L[i * n + t] * W[t * n + c];
            W[i * n + c] = s / L[i * n + i];
        }
}
static uint16_t to_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
static float from_bf16(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}
static float from_fp16(uint16_t u)
{
    _Float16 h;
    memcpy(&h, &u, 2);
    return (float)h;
}
static uint16_t to_fp16(float f)
{
    _Float16 h = (_Float16)f;
    uint16_t u;
    memcpy(&u, &h, 2);
    return u;
}

static ns_status prepare_problem(ns_ctx *ctx, const ns_prior *prior, const ns_energy *en)
{
    const int d = ctx->d, D = ctx->D;
    DevProblem &P = ctx->P;
    memset(&P, 0, sizeof(P));
    P.d = d;
    P.D = D;
    P.prior_kind = prior->kind == NS_PRIOR_BOX ? PRIOR_BOX : PRIOR_GAUSS;
    std::vector<double> pa(D, 0.0), pb(D, 1.0);
    double norm = 0.0;
    for (int j = 0; j < d; ++j) {
        pa[j] = prior->a[j];
        pb[j] = prior->b[j];
        if (P.prior_kind == PRIOR_BOX) {
            if (!(pb[j] > pa[j])) return fail(ctx, NS_EINVAL, "box prior needs b > a");
            norm -= log(pb[j] - pa[j]);
        } else {
            if (!(pb[j] > 0.0)) return fail(ctx, NS_EINVAL, "Gaussian prior needs std > 0");
            norm -= log(pb[j]);
        }
    }
    if (P.prior_kind == PRIOR_GAUSS) norm -= 0.5 * d * log(2.0 * M_PI);
    P.logprior_norm = norm;
    double *dpa, *dpb;
    ns_status st;
    if ((st = dalloc(ctx, &dpa, D)) || (st = dalloc(ctx, &dpb, D))) return st;
    CK(hipMemcpy(dpa, pa.data(), D * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(dpb, pb.data(), D * 8, hipMemcpyHostToDevice));
    P.pa = dpa;
    P.pb = dpb;
    P.lik_kind = en->kind == NS_LIK_MIXTURE ? LIK_MIXTURE : LIK_FUNNEL;
    P.guard_rel = 0.f;
    P.guard_abs = 0.f;
    if (P.lik_kind == LIK_FUNNEL) {
        P.K = 0;
        return NS_OK;
    }
    const int K = en->n_comp;
    P.K = K;
    const int NJB = D / 16, NKS = D / 4, NKS32 = D / 32;
    std::vector<double> mu((size_t)K * D, 0.0), cst(K), wf64((size_t)K * NJB * NKS * 64, 0.0);
    std::vector<float> mu32((size_t)K * D, 0.f), cst32(K);
    const size_t nf16 = (size_t)K * NJB * NKS32 * 64 * 8;
    std::vector<uint16_t> wbf(nf16, 0), wh(nf16, 0), wbf_lo(nf16, 0), wh_lo(nf16, 0);
    std::vector<double> L((size_t)d * d), W((size_t)D * D);
    std::vector<double> Wd((size_t)d * d);
    float cmax = -INFINITY;
    for (int c = 0; c < K; ++c) {
        if (chol_lower(en->cov + (size_t)c * d * d, L.data(), d) != 0)
            return fail(ctx, NS_EINVAL, "mixture covariance is not positive definite");
        tri_inv_lower(L.data(), Wd.data(), d);
        double logdetW = 0.0;
        for (int j = 0; j < d; ++j) logdetW -= log(L[j * d + j]);
        std::fill(W.begin(), W.end(), 0.0);
        for (int r = 0; r < d; ++r)
            for (int s = 0; s < d; ++s) W[r * D + s] = Wd[r * d + s];
        for (int j = 0; j < d; ++j) {
            mu[(size_t)c * D + j] = en->mean[(size_t)c * d + j];
            mu32[(size_t)c * D + j] = (float)mu[(size_t)c * D + j];
        }
        cst[c] = en->logw[c] - 0.5 * d * log(2.0 * M_PI) + logdetW;
        cst32[c] = (float)cst[c];
        if (cst32[c] > cmax) cmax = cst32[c];
        for (int jb = 0; jb < NJB; ++jb) {
            for (int ks = 0; ks < NKS; ++ks)
                for (int l = 0; l < 64; ++l) {
                    const int jj = 16 * jb + (l & 15), kk = 4 * ks + (l >> 4);
                    wf64[(((size_t)c * NJB + jb) * NKS + ks) * 64 + l] = W[jj * D + kk];
                }
            for (int ks = 0; ks < NKS32; ++ks)
                for (int l = 0; l < 64; ++l)
                    for (int e = 0; e < 8; ++e) {
                        const int jj = 16 * jb + (l & 15), kk = 32 * ks + 8 * (l >> 4) + e;
                        const size_t o = ((((size_t)c * NJB + jb) * NKS32 + ks) * 64 + l) * 8 + e;
                        const float wv = (float)W[jj * D + kk];
                        wbf[o] = to_bf16(wv);
                        wh[o] = to_fp16(wv);
                        wbf_lo[o] = to_bf16(wv - from_bf16(wbf[o]));
                        wh_lo[o] = to_fp16(wv - from_fp16(wh[o]));
                    }
        }
    }
    double *dmu, *dcst, *dwf64;
    float *dmu32, *dcst32;
    uint4 *dwf16;
    if ((st = dalloc(ctx, &dmu, mu.size())) || (st = dalloc(ctx, &dcst, K)) ||
        (st = dalloc(ctx, &dwf64, wf64.size())) || (st = dalloc(ctx, &dmu32, mu32.size())) ||
        (st = dalloc(ctx, &dcst32, K)) || (st = dalloc(ctx, &dwf16, wbf.size() / 8)))
        return st;
    CK(hipMemcpy(dmu, mu.data(), mu.size() * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(dcst, cst.data(), K * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(dwf64, wf64.data(), wf64.size() * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(dmu32, mu32.data(), mu32.size() * 4, hipMemcpyHostToDevice));
    CK(hipMemcpy(dcst32, cst32.data(), K * 4, hipMemcpyHostToDevice));
    P.mu = dmu; P.cst = dcst; P.wf64 = dwf64; P.mu32 = dmu32; P.cst32 = dcst32;
    P.cmax32 = cmax;
    // both 16-bit formats are kept so that any precision can be evaluated (ns_eval_loglik)
    uint4 *dwfh, *dwfbl, *dwfhl;
    if ((st = dalloc(ctx, &dwfh, nf16 / 8)) || (st = dalloc(ctx, &dwfbl, nf16 / 8)) ||
        (st = dalloc(ctx, &dwfhl, nf16 / 8)))
        return st;
    CK(hipMemcpy(dwf16, wbf.data(), nf16 * 2, hipMemcpyHostToDevice));
    CK(hipMemcpy(dwfh, wh.data(), nf16 * 2, hipMemcpyHostToDevice));
    CK(hipMemcpy(dwfbl, wbf_lo.data(), nf16 * 2, hipMemcpyHostToDevice));
    CK(hipMemcpy(dwfhl, wh_lo.data(), nf16 * 2, hipMemcpyHostToDevice));
    ctx->wf_bf16 = dwf16;
    ctx->wf_fp16 = dwfh;
    ctx->wf_bf16_lo = dwfbl;
    ctx->wf_fp16_lo = dwfhl;
    P.wf16 = dwf16;
    return NS_OK;
}

static int pad_dim(int d) { return d <= 32 ? 32 : (d <= 64 ? 64 : 128); }

// Problem descriptor for one precision.  Guard band of the mixed modes (a candidate whose
// FP32 estimate L satisfies |L - L*| <= rel * max(0, cmax - L) + abs is re-evaluated in FP64):
// the mixture's error is at most (relative error of |W r|^2) x (cmax - L + ln K), so rel is
// ~4.5x the worst relative error of the quadratic forms measured on the synthetic mixtures
// (bf16 5.5e-3, fp16 7e-4, split bf16 8.9e-6, split fp16 6.4e-7 with FP32 accumulation) and
// abs covers FP32 rounding of the log-sum-exp.
static void run_dev_mode(const ns_ctx *ctx, int mode, DevProblem &P)
{
    P = ctx->P;
    float rel = 0.f, ab = 0.f;
    switch (mode) {
    case NS_MIXED_BF16: P.wf16 = ctx->wf_bf16; rel = 0.025f; ab = 2e-3f; break;
    case NS_MIXED_FP16: P.wf16 = ctx->wf_fp16; rel = 0.0032f; ab = 2e-3f; break;
    case NS_MIXED_BF16X3:
        P.wf16 = ctx->wf_bf16; P.wf16lo = ctx->wf_bf16_lo; rel = 4e-5f; ab = 2e-4f; break;
    case NS_MIXED_FP16X3:
        P.wf16 = ctx->wf_fp16; P.wf16lo = ctx->wf_fp16_lo; rel = 6e-6f; ab = 2e-4f; break;
    default: break;
    }
    P.guard_rel = rel;
    P.guard_abs = ab + rel * (P.K > 1 ? logf((float)P.K) : 0.f);
}

static int kmode(int precision) { return precision; }  // ns_precision values equal nss::Mode
static bool precision_valid(int p) { return p >= NS_FP64 && p <= NS_MIXED_FP16X3; }

static ns_status sync_flags(ns_ctx *ctx)
{
    CK(hipMemcpyAsync(ctx->h_iscal, ctx->R.iscal, 8 * sizeof(int), hipMemcpyDeviceToHost,
                      ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    ctx->done = ctx->h_iscal[0];
    return NS_OK;
}

static ns_status enqueue_iteration(ns_ctx *ctx)
{
    DevProblem P;
    run_dev_mode(ctx, ctx->mode, P);
    CK(launch_cov(P, ctx->R, ctx->part1, ctx->part2, ctx->covG, ctx->stream));
    CK(launch_dirs(P, ctx->R, ctx->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->cfg.flags & NS_FLAG_TIMING) {
        CK(hipEventCreate(&e0));
        CK(hipEventCreate(&e1));
        CK(hipEventRecord(e0, ctx->stream));
    }
    hipError_t e = launch_hrss(P, ctx->R, kmode(ctx->mode), ctx->stream);
    if (e != hipSuccess) {
        ctx->err = std::string("HRSS launch: ") + hipGetErrorString(e);
        return e == hipErrorNotSupported ? NS_EUNSUPPORTED : NS_EDEVICE;
    }
    if (e1) {
        CK(hipEventRecord(e1, ctx->stream));
        ctx->events.emplace_back(e0, e1);
    }
    CK(launch_select(P, ctx->R, 1, ctx->stream));
    return NS_OK;
}

static ns_status collect_events(ns_ctx *ctx)
{
    if (ctx->events.empty()) return NS_OK;
    CK(hipStreamSynchronize(ctx->stream));
    for (auto &pr : ctx->events) {
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, pr.first, pr.second));
        ctx->hrss_ms += ms;
        ctx->hrss_launches += 1;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    ctx->events.clear();
    return NS_OK;
}

// Prior draws, FP64 evaluation, first delete-k; resets every run counter.
static ns_status start_run(ns_ctx *ctx)
{
    DevRun &R = ctx->R;
    const int D = ctx->D, k = ctx->k, p = ctx->p;
    CK(hipMemsetAsync(R.X, 0, (size_t)D * ctx->m_pad * 8, ctx->stream));
    CK(hipMemsetAsync(R.iscal, 0, 8 * sizeof(int), ctx->stream));
    CK(hipMemsetAsync(R.ctr, 0, 16 * 8, ctx->stream));
    CK(hipMemsetAsync(R.Lsig, 0, (size_t)D * D * 8, ctx->stream));
    CK(hipMemsetAsync(R.Lpk, 0, (size_t)D * (D + 1) / 2 * 8, ctx->stream));
    if (R.trace) CK(hipMemsetAsync(R.trace, 0, (size_t)k * p * 16, ctx->stream));
    if (R.prof) CK(hipMemsetAsync(R.prof, 0, 16 * 8, ctx->stream));
    static const double sc0[8] = {0.0, -INFINITY, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    CK(hipMemcpyAsync(R.scal, sc0, sizeof(sc0), hipMemcpyHostToDevice, ctx->stream));
    CK(launch_init_draw(ctx->P, R, ctx->stream));
    hipError_t e = launch_eval_points(ctx->P, R.X, ctx->m_pad, ctx->m, R.logL, R.ctr + 5,
                                      MODE_FP64, ctx->stream);
    if (e != hipSuccess) {
        ctx->err = std::string("init evaluation: ") + hipGetErrorString(e);
        return NS_EDEVICE;
    }
    CK(launch_select(ctx->P, R, 0, ctx->stream));
    for (auto &pr : ctx->events) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    ctx->events.clear();
    ctx->hrss_ms = 0.0;
    ctx->hrss_launches = 0;
    return sync_flags(ctx);
}

extern "C" const char *ns_last_error(const ns_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_init_err.c_str();
}

extern "C" void ns_free(ns_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto &pr : ctx->events) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (void *p : ctx->allocs) if (p) (void)hipFree(p);
    if (ctx->h_iscal) (void)hipHostFree(ctx->h_iscal);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

extern "C" ns_status ns_init(const ns_prior *prior, const ns_energy *energy, const ns_config *cfg,
                             void *hip_stream, ns_ctx **out)
{
    g_init_err.clear();
    if (!out) return fail(nullptr, NS_EINVAL, "out is NULL");
    *out = nullptr;
    if (!prior || !energy || !cfg || !prior->a || !prior->b)
        return fail(nullptr, NS_EINVAL, "NULL argument");
    const int d = prior->d;
    if (d < 1 || energy->d != d) return fail(nullptr, NS_EINVAL, "dimension mismatch or d < 1");
    if (d > 128) return fail(nullptr, NS_EUNSUPPORTED, "d > 128");
    if (prior->kind != NS_PRIOR_BOX && prior->kind != NS_PRIOR_GAUSS_DIAG)
        return fail(nullptr, NS_EINVAL, "unknown prior kind");
    if (energy->kind == NS_LIK_MIXTURE) {
        if (energy->n_comp < 1 || !energy->logw || !energy->mean || !energy->cov)
            return fail(nullptr, NS_EINVAL, "mixture needs n_comp >= 1, logw, mean, cov");
        if (energy->n_comp > 64) return fail(nullptr, NS_EUNSUPPORTED, "n_comp > 64");
    } else if (energy->kind != NS_LIK_FUNNEL) {
        return fail(nullptr, NS_EINVAL, "unknown likelihood kind");
    } else if (d < 2) {
        return fail(nullptr, NS_EINVAL, "funnel needs d >= 2");
    }
    const int m = cfg->n_live, k = cfg->k, p = cfg->chain_len;
    if (m < 2 || k < 1 || k > m - 1 || p < 1)
        return fail(nullptr, NS_EINVAL, "need 2 <= n_live, 1 <= k <= n_live-1, chain_len >= 1");
    if (m > kMaxLive) return fail(nullptr, NS_EUNSUPPORTED, "n_live > 8192");
    if (cfg->stepout_cap < 0 || cfg->shrink_cap < 0 || cfg->max_iter < 1)
        return fail(nullptr, NS_EINVAL, "negative cap or max_iter < 1");
    if (!precision_valid(cfg->precision)) return fail(nullptr, NS_EINVAL, "unknown precision");
    if (cfg->precision != NS_FP64 && energy->kind != NS_LIK_MIXTURE)
        return fail(nullptr, NS_EUNSUPPORTED, "mixed precision is implemented for mixtures only");

    ns_ctx *ctx = new ns_ctx();
    ctx->cfg = *cfg;
    ctx->d = d;
    ctx->D = pad_dim(d);
    ctx->m = m;
    ctx->m_pad = (m + 63) & ~63;
    ctx->k = k;
    ctx->p = p;
    ctx->mode = cfg->precision;
    ns_status st;
    auto bail = [&](ns_status s) {
        g_init_err = ctx->err;
        ns_free(ctx);
        return s;
    };
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&ctx->stream) != hipSuccess) {
            ctx->err = "hipStreamCreate failed";
            return bail(NS_EDEVICE);
        }
        ctx->own_stream = true;
    }
    if ((st = prepare_problem(ctx, prior, energy)) != NS_OK) return bail(st);
    if (!mode_supported(ctx->P, kmode(ctx->mode))) {
        ctx->err = "mixed precision: n_comp too large for this dimension";
        return bail(NS_EUNSUPPORTED);
    }
    DevRun &R = ctx->R;
    memset(&R, 0, sizeof(R));
    R.m = m; R.m_pad = ctx->m_pad; R.k = k; R.p = p;
    const double kappa = 1.3035;
    R.width = cfg->width > 0.0 ? cfg->width
                               : 4.0 * kappa * sqrt((double)d + 2.0) * sqrt(2.0 / (M_PI * d));
    R.stepout_cap = cfg->stepout_cap;
    R.shrink_cap = cfg->shrink_cap;
    R.term_on = cfg->term_frac > 0.0;
    R.log_term = cfg->term_frac > 0.0 ? log(cfg->term_frac) : 0.0;
    R.key0 = (uint32_t)cfg->seed;
    R.key1 = (uint32_t)(cfg->seed >> 32) ^ cfg->run_id;
    const int D = ctx->D;
    R.dead_cap = (long long)(cfg->max_iter + 1) * k;
    if ((st = dalloc(ctx, &R.X, (size_t)D * ctx->m_pad)) || (st = dalloc(ctx, &R.logL, m)) ||
        (st = dalloc(ctx, &R.perm, m)) || (st = dalloc(ctx, &R.scal, 8)) ||
        (st = dalloc(ctx, &R.iscal, 8)) || (st = dalloc(ctx, &R.ctr, 16)) ||
        (st = dalloc(ctx, &R.Lsig, (size_t)D * D)) ||
        (st = dalloc(ctx, &R.Lpk, (size_t)D * (D + 1) / 2)) || (st = dalloc(ctx, &R.parents, k)) ||
        (st = dalloc(ctx, &R.dead, (size_t)R.dead_cap)))
        return bail(st);
    if (cfg->flags & NS_FLAG_TRACE)
        if ((st = dalloc(ctx, &R.trace, (size_t)k * p * 4))) return bail(st);
#ifdef NSS_PHASE_TIMING
    if ((st = dalloc(ctx, &R.prof, 16))) return bail(st);
#endif
    // per-iteration direction buffer (k p D doubles) unless it would exceed 4 GiB; without it
    // the chains generate their directions inline
    {
        const size_t bytes = (size_t)k * p * D * 8;
        if (bytes <= ((size_t)4 << 30) && !(cfg->flags & NS_FLAG_INLINE_DIRECTIONS))
            if ((st = dalloc(ctx, &R.dirbuf, (size_t)k * p * D))) return bail(st);
    }
    const int n = m - k;
    ctx->covG = n / 64 < 1 ? 1 : (n / 64 > 32 ? 32 : n / 64);
    const int nt = D / 16, ntile = nt * (nt + 1) / 2;
    if ((st = dalloc(ctx, &ctx->part1, (size_t)ctx->covG * D)) ||
        (st = dalloc(ctx, &ctx->part2, (size_t)ctx->covG * ntile * 256)))
        return bail(st);
    if (hipHostMalloc((void **)&ctx->h_iscal, 8 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
        ctx->err = "hipHostMalloc failed";
        return bail(NS_ENOMEM);
    }
    if ((st = start_run(ctx)) != NS_OK) return bail(st);
    if (ctx->h_iscal[4]) {
        ctx->err = "no live point lies strictly above L* after the first deletion";
        return bail(NS_ESTATE);
    }
    *out = ctx;
    return NS_OK;
}

extern "C" ns_status ns_reset(ns_ctx *ctx, uint64_t seed, uint32_t run_id)
{
    if (!ctx) return NS_EINVAL;
    CK(hipStreamSynchronize(ctx->stream));
    ctx->R.key0 = (uint32_t)seed;
    ctx->R.key1 = (uint32_t)(seed >> 32) ^ run_id;
    ctx->cfg.seed = seed;
    ctx->cfg.run_id = run_id;
    ns_status st = start_run(ctx);
    if (st != NS_OK) return st;
    if (ctx->h_iscal[4]) return fail(ctx, NS_ESTATE, "no live point lies strictly above L*");
    return NS_OK;
}

extern "C" ns_status ns_step(ns_ctx *ctx, int32_t *done)
{
    if (!ctx) return NS_EINVAL;
    if (ctx->done) {
        if (done) *done = 1;
        return NS_DONE;
    }
    ns_status st = enqueue_iteration(ctx);
    if (st != NS_OK) return st;
    if ((st = sync_flags(ctx)) != NS_OK) return st;
    if ((st = collect_events(ctx)) != NS_OK) return st;
    if (done) *done = ctx->done;
    if (ctx->h_iscal[4]) return fail(ctx, NS_ESTATE, "no live point lies strictly above L*");
    return NS_OK;
}

extern "C" ns_status ns_run(ns_ctx *ctx, int32_t max_iter, int32_t *iters)
{
    if (!ctx || max_iter < 0) return NS_EINVAL;
    ns_status st;
    if ((st = sync_flags(ctx)) != NS_OK) return st;
    const int start = ctx->h_iscal[3];
    int issued = 0;
    while (!ctx->done && issued < max_iter) {
        const int batch = (max_iter - issued) < 16 ? (max_iter - issued) : 16;
        for (int b = 0; b < batch; ++b)
            if ((st = enqueue_iteration(ctx)) != NS_OK) return st;
        issued += batch;
        if ((st = sync_flags(ctx)) != NS_OK) return st;
        if (ctx->h_iscal[4]) break;
    }
    if ((st = collect_events(ctx)) != NS_OK) return st;
    if (iters) *iters = ctx->h_iscal[3] - start;
    if (ctx->h_iscal[4]) return fail(ctx, NS_ESTATE, "no live point lies strictly above L*");
    return NS_OK;
}

extern "C" ns_status ns_logz(ns_ctx *ctx, double *logz, double *logz_err, double *H)
{
    if (!ctx) return NS_EINVAL;
    CK(launch_logz(ctx->P, ctx->R, ctx->stream));
    double out[3];
    CK(hipMemcpyAsync(out, ctx->R.scal + 4, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    if (logz) *logz = out[0];
    if (logz_err) *logz_err = out[1];
    if (H) *H = out[2];
    return NS_OK;
}

extern "C" ns_status ns_stats(ns_ctx *ctx, ns_stats_t *o)
{
    if (!ctx || !o) return NS_EINVAL;
    ns_status st;
    if ((st = collect_events(ctx)) != NS_OK) return st;
    unsigned long long c[16];
    CK(hipMemcpyAsync(c, ctx->R.ctr, sizeof(c), hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync_flags(ctx)) != NS_OK) return st;
    memset(o, 0, sizeof(*o));
    o->iterations = ctx->h_iscal[3];
    o->evals = (int64_t)c[0];
    o->tests = (int64_t)c[1];
    o->prior_rejects = (int64_t)c[2];
    o->stepout_caps = (int64_t)c[3];
    o->shrink_caps = (int64_t)c[4];
    o->nonfinite = (int64_t)c[5];
    o->rechecks = (int64_t)c[6];
    o->band_violations = (int64_t)c[7];
    o->whiten_fallbacks = (int64_t)c[8];
    o->n_dead = (int64_t)c[9];
    o->hrss_ms = ctx->hrss_ms;
    o->hrss_launches = ctx->hrss_launches;
    o->width = ctx->R.width;
    return NS_OK;
}

extern "C" ns_status ns_get_state(ns_ctx *ctx, ns_state_view *v)
{
    if (!ctx || !v) return NS_EINVAL;
    const int d = ctx->d, D = ctx->D, m = ctx->m, mp = ctx->m_pad;
    CK(hipStreamSynchronize(ctx->stream));
    if (v->x) {
        std::vector<double> t((size_t)D * mp);
        CK(hipMemcpy(t.data(), ctx->R.X, t.size() * 8, hipMemcpyDeviceToHost));
        for (int i = 0; i < m; ++i)
            for (int a = 0; a < d; ++a) v->x[(size_t)i * d + a] = t[(size_t)a * mp + i];
    }
    if (v->logL) CK(hipMemcpy(v->logL, ctx->R.logL, m * 8, hipMemcpyDeviceToHost));
    if (v->perm) CK(hipMemcpy(v->perm, ctx->R.perm, m * 4, hipMemcpyDeviceToHost));
    if (v->Lsig) {
        std::vector<double> t((size_t)D * D);
        CK(hipMemcpy(t.data(), ctx->R.Lsig, t.size() * 8, hipMemcpyDeviceToHost));
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) v->Lsig[a * d + b] = t[a * D + b];
    }
    if (v->parents) CK(hipMemcpy(v->parents, ctx->R.parents, ctx->k * 4, hipMemcpyDeviceToHost));
    double sc[4];
    int is[8];
    CK(hipMemcpy(sc, ctx->R.scal, sizeof(sc), hipMemcpyDeviceToHost));
    CK(hipMemcpy(is, ctx->R.iscal, sizeof(is), hipMemcpyDeviceToHost));
    v->Lstar = sc[0]; v->logZ = sc[1]; v->logX = sc[2]; v->M = sc[3];
    v->iter = is[3];
    v->done = is[0];
    return NS_OK;
}

extern "C" ns_status ns_set_state(ns_ctx *ctx, const ns_state_view *v)
{
    if (!ctx || !v || !v->x || !v->logL) return NS_EINVAL;
    const int d = ctx->d, D = ctx->D, m = ctx->m, mp = ctx->m_pad;
    std::vector<double> t((size_t)D * mp, 0.0);
    for (int i = 0; i < m; ++i)
        for (int a = 0; a < d; ++a) t[(size_t)a * mp + i] = v->x[(size_t)i * d + a];
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(ctx->R.X, t.data(), t.size() * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(ctx->R.logL, v->logL, m * 8, hipMemcpyHostToDevice));
    double sc[4] = {0.0, v->logZ, v->logX, v->M};
    CK(hipMemcpy(ctx->R.scal, sc, sizeof(sc), hipMemcpyHostToDevice));
    int is[8];
    CK(hipMemcpy(is, ctx->R.iscal, sizeof(is), hipMemcpyDeviceToHost));
    is[0] = 0; is[3] = (int)v->iter; is[4] = 0;
    CK(hipMemcpy(ctx->R.iscal, is, sizeof(is), hipMemcpyHostToDevice));
    CK(launch_select(ctx->P, ctx->R, 2, ctx->stream));
    ns_status st;
    if ((st = sync_flags(ctx)) != NS_OK) return st;
    is[0] = v->done ? 1 : 0;
    CK(hipMemcpy(ctx->R.iscal, is, sizeof(int), hipMemcpyHostToDevice));
    ctx->done = is[0];
    return NS_OK;
}

extern "C" ns_status ns_get_dead(ns_ctx *ctx, double *out, int64_t cap, int64_t *n)
{
    if (!ctx) return NS_EINVAL;
    unsigned long long nd = 0;
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(&nd, ctx->R.ctr + 9, 8, hipMemcpyDeviceToHost));
    long long stored = (long long)nd < ctx->R.dead_cap ? (long long)nd : ctx->R.dead_cap;
    if (n) *n = (int64_t)nd;
    if (out && cap > 0) {
        const long long c = stored < cap ? stored : cap;
        if (c > 0) CK(hipMemcpy(out, ctx->R.dead, c * 8, hipMemcpyDeviceToHost));
    }
    return NS_OK;
}

extern "C" ns_status ns_get_trace(ns_ctx *ctx, int32_t *out)
{
    if (!ctx || !out) return NS_EINVAL;
    if (!ctx->R.trace) return fail(ctx, NS_EINVAL, "context was created without NS_FLAG_TRACE");
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(out, ctx->R.trace, (size_t)ctx->k * ctx->p * 16, hipMemcpyDeviceToHost));
    return NS_OK;
}

extern "C" ns_status ns_eval_loglik(ns_ctx *ctx, const double *x, int32_t n, int32_t precision,
                                    double *out)
{
    if (!ctx || (!x && n > 0) || (!out && n > 0) || n < 0) return NS_EINVAL;
    if (n == 0) return NS_OK;
    if (!precision_valid(precision)) return fail(ctx, NS_EINVAL, "unknown precision");
    DevProblem P;
    run_dev_mode(ctx, precision, P);
    if (!mode_supported(P, kmode(precision)))
        return fail(ctx, NS_EUNSUPPORTED, "precision not supported for this problem");
    const int d = ctx->d, D = ctx->D;
    const int np = (n + 63) & ~63;
    std::vector<double> t((size_t)D * np, 0.0);
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < d; ++a) t[(size_t)a * np + i] = x[(size_t)i * d + a];
    double *dx = nullptr, *dout = nullptr;
    CK(hipMalloc(&dx, t.size() * 8));
    hipError_t e = hipMalloc(&dout, (size_t)n * 8);
    if (e != hipSuccess) { (void)hipFree(dx); return fail(ctx, NS_ENOMEM, "hipMalloc failed"); }
    ns_status st = NS_OK;
    e = hipMemcpyAsync(dx, t.data(), t.size() * 8, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = launch_eval_points(P, dx, np, n, dout, nullptr, kmode(precision), ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, dout, (size_t)n * 8, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        ctx->err = std::string("ns_eval_loglik: ") + hipGetErrorString(e);
        st = NS_EDEVICE;
    }
    (void)hipFree(dx);
    (void)hipFree(dout);
    return st;
}

#ifdef NSS_PHASE_TIMING
// Timing builds only: per-phase shader-clock cycles of one lane per HRSS workgroup, summed
// over workgroups and launches (0 direction, 1 candidates, 2 barrier, 3 tile, 4 re-check vote,
// 5 FP64 re-check, 6 round top, 7 state update, 8 rounds, 9 steps, 10 re-check rounds).
extern "C" ns_status nss_debug_phase_times(ns_ctx *ctx, unsigned long long *out)
{
    if (!ctx || !out || !ctx->R.prof) return NS_EINVAL;
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(out, ctx->R.prof, 12 * 8, hipMemcpyDeviceToHost));
    return NS_OK;
}
#endif
