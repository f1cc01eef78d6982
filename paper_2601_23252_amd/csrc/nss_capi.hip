// C ABI of the gfx950 Nested Slice Sampling library: argument validation, problem preparation
// (host FP64), device allocation and the per-iteration launch sequence.
#include "../../include/nss.h"
#include "nss_internal.hpp"

#include <math.h>
#include <cmath>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

using namespace nss;

// One run of a context: its configuration, the device descriptors (host copies holding device
// pointers) and the run's launch shape.
struct RunHost {
    ns_config cfg;
    int d = 0, D = 0, m = 0, m_pad = 0, k = 0, p = 0, mode = 0, lik = 0, K = 0, upw = 1;
    DevProblem P;   // descriptor in the run's own precision
    DevRun R;
    // 16-bit W fragments per format, and the rounded remainders for the split modes
    const uint4 *wf_bf16 = nullptr, *wf_fp16 = nullptr, *wf_bf16_lo = nullptr,
                *wf_fp16_lo = nullptr;
    int done = 0;
    long long deaths_bound = 0;   // upper bound of the deaths recorded once the issued work ends
};

// Runs that share one compiled HRSS kernel: (padded dimension, likelihood, precision, fragment
// capacity).
struct Group {
    int D, lik, mode, upwT, rw;
    bool plan_ok;   // 16-bit mixture chains that may use the hypothesis-plan kernel
    int plan;       // tests a chain plans per round: 0 = the k_hrss kernel (up to 4), or 8 / 16
    std::vector<int> runs;
};

// A launch shape of a group's HRSS kernel: chains per workgroup and planned tests per round.
struct Shape {
    int C, plan;
};

// Autotuning state of one group: the candidate shapes, and whether the group still has to be
// tuned (at its next iteration).
struct GroupTune {
    std::vector<Shape> cand;
    std::vector<double> sum;   // per candidate: its best times summed over the points taken
    int points = 0;            // tuning points taken
    long long next_at = 0;     // context iteration of the next tuning point
    bool done = true;
};

struct ns_ctx {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n = 0;                       // runs
    int timing = 0;
    int smc = 0;                     // every run uses the adaptive tempered SMC outer loop
    std::vector<RunHost> runs;
    std::vector<Group> groups;
    DevProblem *dP = nullptr;        // [n + 1] device descriptors; slot n is ns_eval_loglik's
    DevRun *dR = nullptr;            // [n + 1]
    int *d_iscal = nullptr;          // [n][8] run flags, contiguous so one copy reads them all
    double *d_scal = nullptr;        // [n][8]
    unsigned long long *d_ctr = nullptr;  // [n][16]
    int *h_iscal = nullptr;          // pinned mirror of d_iscal
    int2 *d_map1 = nullptr;          // [n + 1]: (r, 0), a one-block launch of run r
    int2 *d_map = nullptr;           // block maps of the current launches
    size_t map_cap = 0;
    std::vector<int2> h_map;
    // launches over the unfinished runs (rebuilt when the set changes)
    Launch L_init, L_one, L_cov, L_dirs[4];   // directions per padded dimension 32/64/128/320
    std::vector<Launch> L_eval;      // per group (FP64 initial evaluation)
    std::vector<Launch> L_hrss;      // per group
    int Dmax = 32;
    std::vector<char> mapped_active;
    std::vector<void *> allocs;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    double hrss_ms = 0.0;
    long long hrss_launches = 0;
    // NS_FLAG_GRAPH: a captured batch of kGraphIters iterations, valid for one block-map epoch
    int use_graph = 0;
    long long map_epoch = 0, graph_epoch = -1;
    hipGraphExec_t gexec = nullptr;
    // groups after the first launch their chains on side streams (default priority), forked
    // from and joined back into `stream` around the chain phase of each iteration
    std::vector<hipStream_t> side;   // [groups - 1]
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;   // [groups - 1]
    bool capturing = false;            // a graph capture is recording the iterations
    bool forked = false;               // the chain launches being issued run concurrently
    // NS_FLAG_AUTOTUNE: the launch shape of each group chosen by timing its candidates on saved
    // iterations (see tune_iteration)
    int autotune = 0;
    std::vector<GroupTune> tune;     // per group
    long long tune_launches = 0;     // HRSS launches timed by the tuner
    long long iters_issued = 0;      // outer iterations issued since the runs started
    // per run: the state an HRSS launch changes (live points, logL, counters), saved before the
    // tuner's candidate launches and restored after each (allocated on first use)
    std::vector<double *> snap_x, snap_l;
    std::vector<unsigned long long *> snap_c;
    // ns_geom_uncertainty's device buffer (outputs and partial results), grown on demand
    void *geom_buf = nullptr;
    size_t geom_bytes = 0;
    // this device's copy of the fixed workspace (ns_geom_uncertainty_noalloc), or null with
    // the reason in scratch_err
    void *scratch = nullptr;
    std::string scratch_err;
    std::string err;
};

constexpr int kGraphIters = 16;   // iterations per host synchronisation in ns_run
constexpr int kDefaultPlan = 16;  // tests per round of the 16-bit mixture chains without tuning

// Workspace of ns_geom_uncertainty_noalloc: a fixed device array, one copy per GPU, held until
// the process ends.  Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in symbol); it uses the device address that hipGetSymbolAddress returns,
// looked up once per device by ns_init_batch with that device current.
static __device__ __align__(256) unsigned char scratch[NS_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_addr;   // device ordinal -> its copy of scratch

static void *scratch_for_current_device(std::string &err)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        err = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(dev);
    if (it != g_scratch_addr.end()) return it->second;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return nullptr;
    }
    g_scratch_addr[dev] = ptr;
    return ptr;
}

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
    c->replacement = NS_REPLACE_HRSS;
    c->outer = NS_OUTER_NESTED;
    c->ess_frac = 0.5;
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


static ns_status prepare_problem(ns_ctx *ctx, RunHost &rh, const ns_prior *prior,
                                 const ns_energy *en)
{
    const int d = rh.d, D = rh.D;
    DevProblem &P = rh.P;
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
    P.lik_kind = en->kind == NS_LIK_MIXTURE ? LIK_MIXTURE
                 : en->kind == NS_LIK_GP      ? LIK_GP
                 : en->kind == NS_LIK_GAUSS_RASTRIGIN ? LIK_RG
                                              : LIK_FUNNEL;
    if (P.lik_kind == LIK_FUNNEL) {
        P.K = 0;
        return NS_OK;
    }
    if (P.lik_kind == LIK_RG) {
        P.K = 0;
        P.rg_la = en->alpha > 0.0 ? log(en->alpha) : -INFINITY;
        P.rg_l1a = en->alpha < 1.0 ? log1p(-en->alpha) : -INFINITY;
        P.rg_amp = en->amp;
        return NS_OK;
    }
    if (P.lik_kind == LIK_GP) {
        P.K = 0;
        P.gp_n = en->n_obs;
        double *gx, *gy;
        if ((st = dalloc(ctx, &gx, (size_t)2 * en->n_obs)) || (st = dalloc(ctx, &gy, en->n_obs)))
            return st;
        CK(hipMemcpy(gx, en->x_obs, (size_t)2 * en->n_obs * 8, hipMemcpyHostToDevice));
        CK(hipMemcpy(gy, en->y_obs, (size_t)en->n_obs * 8, hipMemcpyHostToDevice));
        P.gp_x = gx;
        P.gp_y = gy;
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
    if ((st = dalloc(ctx, &dmu, mu.size())) || (st = dalloc(ctx, &dcst, K)) ||
        (st = dalloc(ctx, &dwf64, wf64.size())) || (st = dalloc(ctx, &dmu32, mu32.size())) ||
        (st = dalloc(ctx, &dcst32, K)))
        return st;
    CK(hipMemcpy(dmu, mu.data(), mu.size() * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(dcst, cst.data(), K * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(dwf64, wf64.data(), wf64.size() * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(dmu32, mu32.data(), mu32.size() * 4, hipMemcpyHostToDevice));
    CK(hipMemcpy(dcst32, cst32.data(), K * 4, hipMemcpyHostToDevice));
    P.mu = dmu; P.cst = dcst; P.wf64 = dwf64; P.mu32 = dmu32; P.cst32 = dcst32;
    P.cmax32 = cmax;
    // both 16-bit formats are kept so that any precision can be evaluated (ns_eval_loglik)
    uint4 *dwfb, *dwfh, *dwfbl, *dwfhl;
    if ((st = dalloc(ctx, &dwfb, nf16 / 8)) || (st = dalloc(ctx, &dwfh, nf16 / 8)) ||
        (st = dalloc(ctx, &dwfbl, nf16 / 8)) || (st = dalloc(ctx, &dwfhl, nf16 / 8)))
        return st;
    CK(hipMemcpy(dwfb, wbf.data(), nf16 * 2, hipMemcpyHostToDevice));
    CK(hipMemcpy(dwfh, wh.data(), nf16 * 2, hipMemcpyHostToDevice));
    CK(hipMemcpy(dwfbl, wbf_lo.data(), nf16 * 2, hipMemcpyHostToDevice));
    CK(hipMemcpy(dwfhl, wh_lo.data(), nf16 * 2, hipMemcpyHostToDevice));
    rh.wf_bf16 = dwfb;
    rh.wf_fp16 = dwfh;
    rh.wf_bf16_lo = dwfbl;
    rh.wf_fp16_lo = dwfhl;
    return NS_OK;
}

static int pad_dim(int d) { return d <= 32 ? 32 : (d <= 64 ? 64 : (d <= 128 ? 128 : 320)); }
static constexpr int kDims[4] = {32, 64, 128, 320};

// Problem descriptor for one precision.  Guard band of the mixed modes (a candidate whose
// FP32 estimate L satisfies |L - L*| <= rel * max(0, cmax - L) + abs is re-evaluated in FP64):
// the mixture's error is at most (relative error of |W r|^2) x (cmax - L + ln K), so rel is
// ~4.5x the worst relative error of the quadratic forms measured on the synthetic mixtures
// (bf16 5.5e-3, fp16 7e-4, split bf16 8.9e-6, split fp16 6.4e-7 with FP32 accumulation) and
// abs covers FP32 rounding of the log-sum-exp.
static DevProblem problem_for_mode(const RunHost &rh, int mode)
{
    DevProblem P = rh.P;
    P.wf16 = nullptr;
    P.wf16lo = nullptr;
    float rel = 0.f, ab = 0.f;
    switch (mode) {
    case NS_MIXED_BF16: P.wf16 = rh.wf_bf16; rel = 0.025f; ab = 2e-3f; break;
    case NS_MIXED_FP16: P.wf16 = rh.wf_fp16; rel = 0.0032f; ab = 2e-3f; break;
    case NS_MIXED_BF16X3:
        P.wf16 = rh.wf_bf16; P.wf16lo = rh.wf_bf16_lo; rel = 4e-5f; ab = 2e-4f; break;
    case NS_MIXED_FP16X3:
        P.wf16 = rh.wf_fp16; P.wf16lo = rh.wf_fp16_lo; rel = 6e-6f; ab = 2e-4f; break;
    case NS_MIXED_FP32:
        // GP: FP32 factorisation of the rounded FP64 kernel matrix, the quadratic form refined
        // in FP64, the log-determinant summed in FP64.  Band = rel |L| + abs + c n s with
        // s = (sigma_f^2 + sigma_n^2) / sigma_n^2, and FP64 decides outright beyond n s = 1e5:
        // on 12,000 prior and posterior draws (n = 23..256) the error stayed below
        // 2.7e-7 n s + 1e-5 there (the FP32 log-determinant), and grew without bound beyond;
        // c is about four times that (the tests check a 2x margin).
        P.guard_rel = 1e-6f;
        P.guard_abs = 4e-3f;
        P.guard_kappa = 1e-6f;
        return P;
    default: break;
    }
    P.guard_rel = rel;
    P.guard_abs = ab + rel * (P.K > 1 ? logf((float)P.K) : 0.f);
    return P;
}

static bool precision_valid(int p) { return p >= NS_FP64 && p <= NS_MIXED_FP32; }

// ---- block maps of the launches over the unfinished runs ----
static int init_blocks(const RunHost &r) { return (r.m * ((r.d + 1) / 2) + 255) / 256; }
static int eval_blocks(const RunHost &r)
{
    return r.lik == LIK_GP ? r.m : (r.m + kRows - 1) / kRows;  // GP: one point per workgroup
}
static int cov_blocks(const RunHost &r)
{
    const int nt = r.D / 16;
    return nt * (nt + 1) / 2 * r.R.covG;
}
static int dirs_blocks(const RunHost &r)
{
    if (!r.R.dirbuf) return 0;
    const long long t = (long long)r.k * r.p;
    return (int)((t + dirs_rows(r.D) - 1) / dirs_rows(r.D));
}
static int hrss_blocks(const RunHost &r) { return (r.k + r.R.C - 1) / r.R.C; }  // GP: C = 1

struct MapBuilder {
    std::vector<int2> &h;
    std::vector<std::pair<Launch *, size_t>> fix;
    template <typename F>
    void add(ns_ctx *ctx, Launch &L, const std::vector<int> &rs, const std::vector<char> &act,
             F blocks)
    {
        const size_t off = h.size();
        L = Launch{ctx->dP, ctx->dR, nullptr, 0, 0, 0};
        for (int r : rs) {
            if (!act[r]) continue;
            const RunHost &rh = ctx->runs[r];
            const int nb = blocks(rh);
            for (int b = 0; b < nb; ++b) h.push_back(make_int2(r, b));
            if (nb > 0) {
                if (rh.m > L.max_m) L.max_m = rh.m;
                if (rh.K > L.max_K) L.max_K = rh.K;
            }
        }
        L.nblocks = (int)(h.size() - off);
        fix.emplace_back(&L, off);
    }
};

// (Re)build every launch for the runs in act; uploads the maps (synchronously).
static ns_status build_maps(ns_ctx *ctx, const std::vector<char> &act)
{
    ctx->h_map.clear();
    MapBuilder mb{ctx->h_map, {}};
    std::vector<int> all(ctx->n);
    for (int r = 0; r < ctx->n; ++r) all[r] = r;
    mb.add(ctx, ctx->L_init, all, act, init_blocks);
    mb.add(ctx, ctx->L_one, all, act, [](const RunHost &) { return 1; });
    mb.add(ctx, ctx->L_cov, all, act, cov_blocks);
    for (int di = 0; di < 4; ++di) {
        const int D = kDims[di];
        std::vector<int> rs;
        for (int r = 0; r < ctx->n; ++r)
            if (ctx->runs[r].D == D) rs.push_back(r);
        mb.add(ctx, ctx->L_dirs[di], rs, act, dirs_blocks);
    }
    ctx->L_eval.resize(ctx->groups.size());
    ctx->L_hrss.resize(ctx->groups.size());
    for (size_t g = 0; g < ctx->groups.size(); ++g) {
        mb.add(ctx, ctx->L_eval[g], ctx->groups[g].runs, act, eval_blocks);
        mb.add(ctx, ctx->L_hrss[g], ctx->groups[g].runs, act, hrss_blocks);
    }
    ctx->Dmax = 32;
    for (int r = 0; r < ctx->n; ++r)
        if (act[r] && ctx->runs[r].D > ctx->Dmax) ctx->Dmax = ctx->runs[r].D;
    if (ctx->h_map.size() > ctx->map_cap) {
        ctx->err = "internal: block map larger than its allocation";
        return NS_EDEVICE;
    }
    for (auto &f : mb.fix) f.first->map = ctx->d_map + f.second;
    if (!ctx->h_map.empty()) {
        CK(hipStreamSynchronize(ctx->stream));
        CK(hipMemcpy(ctx->d_map, ctx->h_map.data(), ctx->h_map.size() * sizeof(int2),
                     hipMemcpyHostToDevice));
    }
    ctx->mapped_active = act;
    ++ctx->map_epoch;
    return NS_OK;
}

static Launch launch_one(const ns_ctx *ctx, int slot)
{
    const RunHost &rh = ctx->runs[slot < ctx->n ? slot : 0];
    return Launch{ctx->dP, ctx->dR, ctx->d_map1 + slot, 1, rh.m, rh.K};
}

static ns_status sync_flags(ns_ctx *ctx)
{
    CK(hipMemcpyAsync(ctx->h_iscal, ctx->d_iscal, (size_t)ctx->n * 8 * sizeof(int),
                      hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    for (int r = 0; r < ctx->n; ++r) ctx->runs[r].done = ctx->h_iscal[8 * r];
    return NS_OK;
}

static bool all_done(const ns_ctx *ctx)
{
    for (const RunHost &r : ctx->runs)
        if (!r.done) return false;
    return true;
}

static bool any_error(const ns_ctx *ctx)
{
    for (int r = 0; r < ctx->n; ++r)
        if (ctx->h_iscal[8 * r + 4]) return true;
    return false;
}

static const char *state_error_text(const ns_ctx *ctx)
{
    return ctx->smc ? "every particle has log L = -inf" : "no live point lies strictly above L*";
}

// drop finished runs from the launches once they are known to be finished
static ns_status refresh_maps(ns_ctx *ctx)
{
    std::vector<char> act(ctx->n);
    bool changed = false;
    for (int r = 0; r < ctx->n; ++r) {
        act[r] = !ctx->runs[r].done;
        if (act[r] != ctx->mapped_active[r]) changed = true;
    }
    return changed ? build_maps(ctx, act) : NS_OK;
}

static ns_status device_error(ns_ctx *ctx, const char *what, hipError_t e)
{
    ctx->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorNotSupported ? NS_EUNSUPPORTED : NS_EDEVICE;
}

// The part of an iteration before the chains: SMC reweighting, whitening, directions.
static ns_status enqueue_pre(ns_ctx *ctx)
{
    hipError_t e;
    if (ctx->smc) {   // next temperature, evidence increment, resampling
        e = launch_smc(ctx->L_one, 1, ctx->stream);
        if (e != hipSuccess) return device_error(ctx, "SMC reweighting launch", e);
    }
    e = launch_cov(ctx->L_cov, ctx->L_one, ctx->Dmax, ctx->stream);
    if (e != hipSuccess) return device_error(ctx, "whitening launch", e);
    for (int di = 0; di < 4; ++di) {
        e = launch_dirs(ctx->L_dirs[di], kDims[di], ctx->stream);
        if (e != hipSuccess) return device_error(ctx, "direction launch", e);
    }
    return NS_OK;
}

// The chains of group g.
// Workgroups per CU the hypothesis-plan kernel is compiled for: two when the launch has more
// workgroups than the chip has CUs, or runs beside other groups' chains on side streams (two
// resident workgroups then hide each other's latency, at the cost of spilled registers), else
// one.
constexpr int kChipCUs = 256;
static int plan_occupancy(const ns_ctx *ctx, const Launch &L)
{
    return (L.nblocks > kChipCUs || ctx->forked) ? 2 : 1;
}

static ns_status enqueue_hrss_group(ns_ctx *ctx, size_t g, hipStream_t s)
{
    const Group &G = ctx->groups[g];
    const hipError_t e =
        G.lik == LIK_GP ? launch_hrss_gp(ctx->L_hrss[g], G.mode, s)
        : G.rw          ? launch_rw(ctx->L_hrss[g], G.D, G.lik, G.mode, G.upwT, s)
        : G.plan        ? launch_hrss_plan(ctx->L_hrss[g], G.D, G.mode, G.upwT, G.plan,
                                           plan_occupancy(ctx, ctx->L_hrss[g]), s)
                        : launch_hrss(ctx->L_hrss[g], G.D, G.lik, G.mode, G.upwT, s);
    if (e != hipSuccess) return device_error(ctx, "HRSS launch", e);
    return NS_OK;
}
static ns_status enqueue_hrss_group(ns_ctx *ctx, size_t g)
{
    return enqueue_hrss_group(ctx, g, ctx->stream);
}

// The chains of every group with unfinished runs: the first such group on the context's
// stream, the others concurrently on side streams (their runs are disjoint, and a run's
// arithmetic does not depend on the order), forked after the directions and joined before
// delete-k.  Inside a graph capture the groups go one after the other on the context's stream:
// a graph whose iterations branched over the side streams stalled once in a batch test (no
// cause found; the runtime then schedules the branches itself), so graphs stay linear.
static ns_status enqueue_chains(ns_ctx *ctx)
{
    std::vector<size_t> live;
    for (size_t g = 0; g < ctx->groups.size(); ++g)
        if (ctx->L_hrss[g].nblocks > 0) live.push_back(g);
    ns_status st;
    if (live.size() <= 1 || ctx->side.empty() || ctx->capturing) {
        for (size_t g : live)
            if ((st = enqueue_hrss_group(ctx, g)) != NS_OK) return st;
        return NS_OK;
    }
    CK(hipEventRecord(ctx->ev_fork, ctx->stream));
    struct Forked {   // the launches below run concurrently (read by plan_occupancy)
        ns_ctx *c;
        explicit Forked(ns_ctx *x) : c(x) { c->forked = true; }
        ~Forked() { c->forked = false; }
    } forked(ctx);
    for (size_t i = 1; i < live.size(); ++i) {
        hipStream_t s = ctx->side[i - 1];
        CK(hipStreamWaitEvent(s, ctx->ev_fork, 0));
        if ((st = enqueue_hrss_group(ctx, live[i], s)) != NS_OK) return st;
        CK(hipEventRecord(ctx->ev_join[i - 1], s));
    }
    if ((st = enqueue_hrss_group(ctx, live[0])) != NS_OK) return st;
    for (size_t i = 1; i < live.size(); ++i)
        CK(hipStreamWaitEvent(ctx->stream, ctx->ev_join[i - 1], 0));
    return NS_OK;
}

// The chains of every group (timed under NS_FLAG_TIMING), then delete-k and evidence.
static ns_status enqueue_rest(ns_ctx *ctx)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->timing) {
        CK(hipEventCreate(&e0));
        CK(hipEventCreate(&e1));
        CK(hipEventRecord(e0, ctx->stream));
    }
    ns_status st;
    if ((st = enqueue_chains(ctx)) != NS_OK) return st;
    if (e1) {
        CK(hipEventRecord(e1, ctx->stream));
        ctx->events.emplace_back(e0, e1);
    }
    hipError_t e = ctx->smc ? launch_smc(ctx->L_one, 2, ctx->stream)
                            : launch_select(ctx->L_one, 1, ctx->stream);
    if (e != hipSuccess) return device_error(ctx, "select launch", e);
    return NS_OK;
}

static ns_status enqueue_iteration(ns_ctx *ctx)
{
    ns_status st = enqueue_pre(ctx);
    return st != NS_OK ? st : enqueue_rest(ctx);
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

// ------------------------------------------------------------------------------------------
// NS_FLAG_AUTOTUNE: the launch shape of each group's HRSS kernel (chains per workgroup, and for
// the 16-bit mixture chains the tests planned per round).  A chain's decisions and arithmetic
// do not depend on the shape, so every candidate is timed on the same iteration: after the
// whitening and directions, the state the chains change is saved, each candidate's HRSS
// launch is timed and the state restored, kTuneReps times over (the minimum counts), and the
// iteration then runs with the shape of least summed time so far.  The chains' behaviour
// changes over a run (early contours are wide and brackets expand often, later ones rarely),
// so this is done at up to kTunePoints iterations spread over the run's start (kTuneAt) and
// the candidates are ranked by their summed times; a leader 25% ahead of every other candidate
// after the first point, or 5% ahead after two, ends the tuning early.  The current choice is cached per group shape
// in this process after every point; a context whose shape is cached does not tune.
// ------------------------------------------------------------------------------------------
constexpr int kTuneReps = 2;   // timed launches per candidate and point
constexpr int kTunePoints = 3;
constexpr long long kTuneAt[kTunePoints] = {0, 32, 96};   // context iterations of the points
constexpr double kTuneClear1 = 1.25;   // a lead that ends tuning after the first point
constexpr double kTuneClear2 = 1.05;   // ... after the second point

static std::mutex g_tune_mu;
// group shape -> (chains per workgroup, planned tests per round)
static std::map<std::vector<long long>, Shape> g_tuned;

static std::vector<long long> tune_key(const ns_ctx *ctx, const Group &G)
{
    long long chains = 0;
    for (int r : G.runs) chains += ctx->runs[r].k;
    return {G.D, G.lik, G.mode, G.upwT, G.rw, chains, G.plan_ok ? 1 : 0};
}

// Launch shape of group g's runs, on the host and in the device descriptors (slot n mirrors
// run 0).  The caller rebuilds the launches.
static ns_status set_group_shape(ns_ctx *ctx, size_t g, Shape sh)
{
    CK(hipStreamSynchronize(ctx->stream));
    ctx->groups[g].plan = sh.plan;
    for (int r : ctx->groups[g].runs) {
        ctx->runs[r].R.C = sh.C;
        CK(hipMemcpy(ctx->dR + r, &ctx->runs[r].R, sizeof(DevRun), hipMemcpyHostToDevice));
        if (r == 0)
            CK(hipMemcpy(ctx->dR + ctx->n, &ctx->runs[0].R, sizeof(DevRun), hipMemcpyHostToDevice));
    }
    return NS_OK;
}

// Group g still has tuning points to take and unfinished runs to take them on.
static bool tune_waiting(const ns_ctx *ctx, size_t g)
{
    if (ctx->tune[g].done) return false;
    for (int r : ctx->groups[g].runs)
        if (!ctx->runs[r].done) return true;
    return false;
}

// A tuning point is due at this iteration for some group.
static bool tuning_due(const ns_ctx *ctx)
{
    for (size_t g = 0; g < ctx->tune.size(); ++g)
        if (tune_waiting(ctx, g) && ctx->iters_issued >= ctx->tune[g].next_at) return true;
    return false;
}

// save (dir = 0) or restore (dir = 1) the state group g's chains change
static ns_status group_state(ns_ctx *ctx, size_t g, int dir)
{
    for (int r : ctx->groups[g].runs) {
        const RunHost &rh = ctx->runs[r];
        const size_t nx = (size_t)rh.D * rh.m_pad, nl = (size_t)rh.m;
        ns_status st;
        if (!ctx->snap_x[r]) {
            if ((st = dalloc(ctx, &ctx->snap_x[r], nx)) || (st = dalloc(ctx, &ctx->snap_l[r], nl)) ||
                (st = dalloc(ctx, &ctx->snap_c[r], 16)))
                return st;
        }
        double *x = rh.R.X, *lg = rh.R.logL;
        unsigned long long *c = rh.R.ctr;
        if (dir == 0) {
            CK(hipMemcpyAsync(ctx->snap_x[r], x, nx * 8, hipMemcpyDeviceToDevice, ctx->stream));
            CK(hipMemcpyAsync(ctx->snap_l[r], lg, nl * 8, hipMemcpyDeviceToDevice, ctx->stream));
            CK(hipMemcpyAsync(ctx->snap_c[r], c, 16 * 8, hipMemcpyDeviceToDevice, ctx->stream));
        } else {
            CK(hipMemcpyAsync(x, ctx->snap_x[r], nx * 8, hipMemcpyDeviceToDevice, ctx->stream));
            CK(hipMemcpyAsync(lg, ctx->snap_l[r], nl * 8, hipMemcpyDeviceToDevice, ctx->stream));
            CK(hipMemcpyAsync(c, ctx->snap_c[r], 16 * 8, hipMemcpyDeviceToDevice, ctx->stream));
        }
    }
    return NS_OK;
}

// One iteration in which every group still to be tuned times its candidates on the same
// state, keeps the fastest, and the iteration completes with the chosen shapes.
static ns_status tune_iteration(ns_ctx *ctx)
{
    ns_status st = enqueue_pre(ctx);
    if (st != NS_OK) return st;
    for (size_t g = 0; g < ctx->groups.size(); ++g) {
        GroupTune &t = ctx->tune[g];
        if (!tune_waiting(ctx, g) || ctx->iters_issued < t.next_at) continue;
        if ((st = group_state(ctx, g, 0)) != NS_OK) return st;
        const size_t nc = t.cand.size();
        std::vector<double> best(nc, 1e300);
        for (int rep = 0; rep < kTuneReps; ++rep) {
            for (size_t ci = 0; ci < nc; ++ci) {
                if ((st = set_group_shape(ctx, g, t.cand[ci])) != NS_OK) return st;
                if ((st = build_maps(ctx, ctx->mapped_active)) != NS_OK) return st;
                if ((st = group_state(ctx, g, 1)) != NS_OK) return st;
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
                    if (e0) (void)hipEventDestroy(e0);
                    return fail(ctx, NS_EDEVICE, "autotune: event creation failed");
                }
                float ms = 0.f;
                const bool ok = hipEventRecord(e0, ctx->stream) == hipSuccess &&
                                (st = enqueue_hrss_group(ctx, g)) == NS_OK &&
                                hipEventRecord(e1, ctx->stream) == hipSuccess &&
                                hipEventSynchronize(e1) == hipSuccess &&
                                hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                if (st != NS_OK) return st;
                if (!ok) return fail(ctx, NS_EDEVICE, "autotune: event timing failed");
                ctx->tune_launches += 1;
                if (ms < best[ci]) best[ci] = ms;
            }
        }
        t.sum.resize(nc, 0.0);
        size_t bi = 0;
        for (size_t ci = 0; ci < nc; ++ci) {
            t.sum[ci] += best[ci];
            if (t.sum[ci] < t.sum[bi]) bi = ci;
        }
        if ((st = set_group_shape(ctx, g, t.cand[bi])) != NS_OK) return st;
        if ((st = group_state(ctx, g, 1)) != NS_OK) return st;
        t.points += 1;
        // done after the last point, or earlier when the leader is clearly ahead of every
        // other candidate: by kTuneClear1 after one point, by kTuneClear2 after two
        double second = 1e300;
        for (size_t ci = 0; ci < nc; ++ci)
            if (ci != bi && t.sum[ci] < second) second = t.sum[ci];
        t.done = t.points >= kTunePoints ||
                 second > (t.points == 1 ? kTuneClear1 : kTuneClear2) * t.sum[bi];
        if (!t.done) t.next_at = kTuneAt[t.points];
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[tune_key(ctx, ctx->groups[g])] = t.cand[bi];
    }
    if ((st = build_maps(ctx, ctx->mapped_active)) != NS_OK) return st;
    return enqueue_rest(ctx);
}

// Prior draws, FP64 evaluation and first delete-k of every run; resets every run counter.
// Replaces the allocation `old` (owned by the context) with `nw`, freeing `old`.
static void swap_alloc(ns_ctx *ctx, void *old, void *nw)
{
    for (void *&p : ctx->allocs)
        if (p == old) { p = nw; break; }
    (void)hipFree(old);
}

// Makes room in every unfinished run's dead record for the deaths of `iters` more iterations:
// a record that could overflow is reallocated at twice its size (or what is needed, up to
// max_iter + 1 iterations), its contents copied, and the run's device descriptor updated.
// The kernels read the record's address from the descriptor, so captured graphs stay valid.
static ns_status reserve_dead(ns_ctx *ctx, int iters)
{
    bool synced = false;
    for (int r = 0; r < ctx->n; ++r) {
        RunHost &rh = ctx->runs[r];
        DevRun &R = rh.R;
        if (rh.done || R.smc) continue;
        rh.deaths_bound += (long long)iters * rh.k;
        const long long maxcap = (long long)(rh.cfg.max_iter + 1) * rh.k;
        if (rh.deaths_bound <= R.dead_cap || R.dead_cap >= maxcap) continue;
        long long cap = rh.deaths_bound > 2 * R.dead_cap ? rh.deaths_bound : 2 * R.dead_cap;
        if (cap > maxcap) cap = maxcap;
        if (!synced) {
            CK(hipStreamSynchronize(ctx->stream));
            synced = true;
        }
        double *nd = nullptr, *nx = nullptr;
        if (hipMalloc((void **)&nd, (size_t)cap * 8) != hipSuccess)
            return fail(ctx, NS_ENOMEM, "growing the dead record failed");
        if (R.deadx && hipMalloc((void **)&nx, (size_t)cap * rh.d * 8) != hipSuccess) {
            (void)hipFree(nd);
            return fail(ctx, NS_ENOMEM, "growing the dead points' record failed");
        }
        CK(hipMemcpy(nd, R.dead, (size_t)R.dead_cap * 8, hipMemcpyDeviceToDevice));
        swap_alloc(ctx, R.dead, nd);
        R.dead = nd;
        if (R.deadx) {
            CK(hipMemcpy(nx, R.deadx, (size_t)R.dead_cap * rh.d * 8, hipMemcpyDeviceToDevice));
            swap_alloc(ctx, R.deadx, nx);
            R.deadx = nx;
        }
        R.dead_cap = cap;
        CK(hipMemcpy(ctx->dR + r, &R, sizeof(DevRun), hipMemcpyHostToDevice));
        if (r == 0) CK(hipMemcpy(ctx->dR + ctx->n, &R, sizeof(DevRun), hipMemcpyHostToDevice));
    }
    return NS_OK;
}

static ns_status start_runs(ns_ctx *ctx)
{
    const int n = ctx->n;
    for (RunHost &rh : ctx->runs) {
        DevRun &R = rh.R;
        CK(hipMemsetAsync(R.X, 0, (size_t)rh.D * rh.m_pad * 8, ctx->stream));
        CK(hipMemsetAsync(R.Lsig, 0, (size_t)rh.D * rh.D * 8, ctx->stream));
        CK(hipMemsetAsync(R.Lpk, 0, (size_t)rh.D * (rh.D + 1) / 2 * 8, ctx->stream));
        if (R.trace) CK(hipMemsetAsync(R.trace, 0, (size_t)rh.k * rh.p * 16, ctx->stream));
        if (R.prof) CK(hipMemsetAsync(R.prof, 0, 16 * 8, ctx->stream));
        rh.done = 0;
        rh.deaths_bound = rh.k;   // the first deletion
    }
    ctx->iters_issued = 0;
    for (GroupTune &t : ctx->tune)   // pending tuning points count from the new start
        if (!t.done) t.next_at = kTuneAt[t.points];
    CK(hipMemsetAsync(ctx->d_iscal, 0, (size_t)n * 8 * sizeof(int), ctx->stream));
    CK(hipMemsetAsync(ctx->d_ctr, 0, (size_t)n * 16 * 8, ctx->stream));
    std::vector<double> sc((size_t)n * 8, 0.0);
    for (int r = 0; r < n; ++r) sc[(size_t)8 * r + 1] = -INFINITY;  // logZ
    CK(hipMemcpyAsync(ctx->d_scal, sc.data(), sc.size() * 8, hipMemcpyHostToDevice, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));  // sc is pageable host memory
    ns_status st = build_maps(ctx, std::vector<char>(n, 1));
    if (st != NS_OK) return st;
    hipError_t e = launch_init_draw(ctx->L_init, ctx->stream);
    if (e != hipSuccess) return device_error(ctx, "prior draw launch", e);
    for (size_t g = 0; g < ctx->groups.size(); ++g) {
        const Group &G = ctx->groups[g];
        e = G.lik == LIK_GP
                ? launch_eval_gp(ctx->L_eval[g], MODE_FP64, nullptr, 0, 0, nullptr, 1, ctx->stream)
                : launch_eval_init(ctx->L_eval[g], G.D, G.lik, ctx->stream);
        if (e != hipSuccess) return device_error(ctx, "initial evaluation", e);
    }
    e = ctx->smc ? launch_smc(ctx->L_one, 0, ctx->stream) : launch_select(ctx->L_one, 0, ctx->stream);
    if (e != hipSuccess) return device_error(ctx, "select launch", e);
    for (auto &pr : ctx->events) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    ctx->events.clear();
    ctx->hrss_ms = 0.0;
    ctx->hrss_launches = 0;
    if ((st = sync_flags(ctx)) != NS_OK) return st;
    return refresh_maps(ctx);
}

extern "C" const char *ns_last_error(const ns_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_init_err.c_str();
}

extern "C" void ns_free(ns_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    for (hipStream_t st : ctx->side) if (st) { (void)hipStreamSynchronize(st); (void)hipStreamDestroy(st); }
    for (hipEvent_t ev : ctx->ev_join) if (ev) (void)hipEventDestroy(ev);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    for (auto &pr : ctx->events) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
    for (void *p : ctx->allocs) if (p) (void)hipFree(p);
    if (ctx->geom_buf) (void)hipFree(ctx->geom_buf);
    if (ctx->h_iscal) (void)hipHostFree(ctx->h_iscal);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

// Argument checks of one run (no allocation).
static ns_status validate_run(const ns_prior *prior, const ns_energy *energy, const ns_config *cfg,
                              std::string &msg)
{
    if (!prior || !energy || !cfg || !prior->a || !prior->b) { msg = "NULL argument"; return NS_EINVAL; }
    const int d = prior->d;
    if (d < 1 || energy->d != d) { msg = "dimension mismatch or d < 1"; return NS_EINVAL; }
    if (d > 320) { msg = "d > 320"; return NS_EUNSUPPORTED; }
    if (d > 128 && ((energy->kind != NS_LIK_FUNNEL && energy->kind != NS_LIK_GAUSS_RASTRIGIN) ||
                    cfg->precision != NS_FP64 || (cfg->flags & NS_FLAG_INLINE_DIRECTIONS))) {
        msg = "d > 128 is implemented for the funnel and Gaussian-Rastrigin likelihoods in FP64 "
              "with the direction buffer";
        return NS_EUNSUPPORTED;
    }
    if (prior->kind != NS_PRIOR_BOX && prior->kind != NS_PRIOR_GAUSS_DIAG) {
        msg = "unknown prior kind";
        return NS_EINVAL;
    }
    if (energy->kind == NS_LIK_MIXTURE) {
        if (energy->n_comp < 1 || !energy->logw || !energy->mean || !energy->cov) {
            msg = "mixture needs n_comp >= 1, logw, mean, cov";
            return NS_EINVAL;
        }
        if (energy->n_comp > 64) { msg = "n_comp > 64"; return NS_EUNSUPPORTED; }
    } else if (energy->kind == NS_LIK_GP) {
        if (d != 6) { msg = "GP likelihood needs d = 6 (log hyperparameters)"; return NS_EINVAL; }
        if (energy->n_obs < 1 || !energy->x_obs || !energy->y_obs) {
            msg = "GP likelihood needs n_obs >= 1, x_obs, y_obs";
            return NS_EINVAL;
        }
        if (energy->n_obs > kGpMaxObs) { msg = "GP n_obs > 256"; return NS_EUNSUPPORTED; }
    } else if (energy->kind == NS_LIK_GAUSS_RASTRIGIN) {
        if (!(energy->alpha >= 0.0 && energy->alpha <= 1.0) || !(energy->amp >= 0.0) ||
            energy->amp == INFINITY) {
            msg = "Gaussian-Rastrigin likelihood needs 0 <= alpha <= 1 and finite amp >= 0";
            return NS_EINVAL;
        }
    } else if (energy->kind != NS_LIK_FUNNEL) {
        msg = "unknown likelihood kind";
        return NS_EINVAL;
    } else if (d < 2) {
        msg = "funnel needs d >= 2";
        return NS_EINVAL;
    }
    const int m = cfg->n_live, p = cfg->chain_len;
    const bool smc = cfg->outer == NS_OUTER_SMC;
    const int k = smc ? 1 : cfg->k;   // SMC moves every particle; k is unused
    if (cfg->outer != NS_OUTER_NESTED && !smc) { msg = "unknown outer loop"; return NS_EINVAL; }
    if (m < 2 || k < 1 || k > m - 1 || p < 1) {
        msg = "need 2 <= n_live, 1 <= k <= n_live-1, chain_len >= 1";
        return NS_EINVAL;
    }
    if (smc) {
        if (!(cfg->ess_frac > 0.0 && cfg->ess_frac < 1.0)) {
            msg = "SMC needs 0 < ess_frac < 1";
            return NS_EINVAL;
        }
        if (energy->kind == NS_LIK_GP || cfg->precision != NS_FP64 ||
            cfg->replacement != NS_REPLACE_HRSS) {
            msg = "SMC is implemented for FP64 slice mutation of the non-GP likelihoods";
            return NS_EUNSUPPORTED;
        }
    }
    if (m > kMaxLive) { msg = "n_live > 8192"; return NS_EUNSUPPORTED; }
    if (cfg->stepout_cap < 0 || cfg->shrink_cap < 0 || cfg->max_iter < 1) {
        msg = "negative cap or max_iter < 1";
        return NS_EINVAL;
    }
    if (!precision_valid(cfg->precision)) { msg = "unknown precision"; return NS_EINVAL; }
    if (cfg->replacement != NS_REPLACE_HRSS && cfg->replacement != NS_REPLACE_RW) {
        msg = "unknown replacement kernel";
        return NS_EINVAL;
    }
    if (cfg->replacement == NS_REPLACE_RW && energy->kind == NS_LIK_GP) {
        msg = "random-walk replacement is not implemented for the GP likelihood";
        return NS_EUNSUPPORTED;
    }
    if (energy->kind == NS_LIK_GP) {
        if (cfg->precision != NS_FP64 && cfg->precision != NS_MIXED_FP32) {
            msg = "GP likelihood: precision NS_FP64 or NS_MIXED_FP32";
            return NS_EUNSUPPORTED;
        }
    } else if (cfg->precision == NS_MIXED_FP32) {
        msg = "NS_MIXED_FP32 is implemented for the GP likelihood only";
        return NS_EUNSUPPORTED;
    } else if (cfg->precision != NS_FP64 && energy->kind != NS_LIK_MIXTURE) {
        msg = "mixed precision is implemented for mixtures only";
        return NS_EUNSUPPORTED;
    }
    return NS_OK;
}

static void set_key(DevRun &R, uint64_t seed, uint32_t run_id)
{
    R.key0 = (uint32_t)seed;
    R.key1 = (uint32_t)(seed >> 32) ^ run_id;
}

// Device buffers of one run (the scalar blocks come from the context's contiguous arrays).
static ns_status alloc_run(ns_ctx *ctx, int r)
{
    RunHost &rh = ctx->runs[r];
    const ns_config *cfg = &rh.cfg;
    DevRun &R = rh.R;
    memset(&R, 0, sizeof(R));
    const int d = rh.d, D = rh.D, m = rh.m, k = rh.k, p = rh.p;
    R.m = m; R.m_pad = rh.m_pad; R.k = k; R.p = p;
    const double kappa = 1.3035;
    R.rw = cfg->replacement == NS_REPLACE_RW;
    R.width = cfg->width > 0.0 ? cfg->width
              : R.rw           ? 2.38 / sqrt((double)d)
                               : 4.0 * kappa * sqrt((double)d + 2.0) * sqrt(2.0 / (M_PI * d));
    R.stepout_cap = cfg->stepout_cap;
    R.shrink_cap = cfg->shrink_cap;
    R.term_on = cfg->term_frac > 0.0;
    R.log_term = cfg->term_frac > 0.0 ? log(cfg->term_frac) : 0.0;
    set_key(R, cfg->seed, cfg->run_id);
    R.smc = cfg->outer == NS_OUTER_SMC;
    R.freeze = (cfg->flags & NS_FLAG_FREEZE_WHITENING) && !R.smc;
    R.diag = (cfg->flags & NS_FLAG_DIAGONAL_METRIC) ? 1 : 0;
    R.ess_frac = cfg->ess_frac;
    // the dead record starts at kDeadInitIters iterations and grows between launches
    // (reserve_dead), up to max_iter + 1 iterations
    R.dead_cap = R.smc ? 1
                       : (long long)(cfg->max_iter + 1 < kDeadInitIters ? cfg->max_iter + 1
                                                                         : kDeadInitIters) * k;
    R.iscal = ctx->d_iscal + 8 * r;
    R.scal = ctx->d_scal + 8 * r;
    R.ctr = ctx->d_ctr + 16 * r;
    ns_status st;
    if ((st = dalloc(ctx, &R.X, (size_t)D * rh.m_pad)) || (st = dalloc(ctx, &R.logL, m)) ||
        (st = dalloc(ctx, &R.perm, m)) || (st = dalloc(ctx, &R.Lsig, (size_t)D * D)) ||
        (st = dalloc(ctx, &R.Lpk, (size_t)D * (D + 1) / 2)) || (st = dalloc(ctx, &R.parents, k)) ||
        (st = dalloc(ctx, &R.dead, (size_t)R.dead_cap)))
        return st;
    if (cfg->flags & NS_FLAG_TRACE)
        if ((st = dalloc(ctx, &R.trace, (size_t)k * p * 4))) return st;
    if ((cfg->flags & NS_FLAG_RECORD_POINTS) && !R.smc)
        if ((st = dalloc(ctx, &R.deadx, (size_t)R.dead_cap * d))) return st;
#ifdef NSS_PHASE_TIMING
    if ((st = dalloc(ctx, &R.prof, 16))) return st;
#endif
    // per-iteration direction buffer (k p D doubles) unless it would exceed 32 GiB; without it
    // the chains generate their directions inline (D <= 128 only)
    const size_t bytes = (size_t)k * p * (D + 8) * 8;
    if (bytes <= ((size_t)32 << 30) && !(cfg->flags & NS_FLAG_INLINE_DIRECTIONS) &&
        rh.lik != LIK_GP) {  // GP chains draw their directions themselves
        if ((st = dalloc(ctx, &R.dirbuf, (size_t)k * p * D))) return st;
        if ((st = dalloc(ctx, &R.ubuf, (size_t)k * p * 8))) return st;
    } else if (R.rw || D > 128) {
        return fail(ctx, NS_EUNSUPPORTED,
                    "random-walk replacement and d > 128 need the direction buffer "
                    "(k p (d+8) doubles <= 32 GiB, no NS_FLAG_INLINE_DIRECTIONS)");
    }
    const int n = R.smc ? m : m - k;   // points of the whitening covariance
    R.covG = n / 64 < 1 ? 1 : (n / 64 > 32 ? 32 : n / 64);
    if (R.smc)
        if ((st = dalloc(ctx, &R.Xtmp, (size_t)D * rh.m_pad)) || (st = dalloc(ctx, &R.Ltmp, m)))
            return st;
    const int nt = D / 16, ntile = nt * (nt + 1) / 2;
    if ((st = dalloc(ctx, &R.part1, (size_t)R.covG * D)) ||
        (st = dalloc(ctx, &R.part2, (size_t)R.covG * ntile * 256)))
        return st;
    return NS_OK;
}

extern "C" ns_status ns_init_batch(int32_t n_runs, const ns_prior *priors,
                                   const ns_energy *energies, const ns_config *cfgs,
                                   void *hip_stream, ns_ctx **out)
{
    g_init_err.clear();
    if (!out) return fail(nullptr, NS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_runs < 1 || !priors || !energies || !cfgs)
        return fail(nullptr, NS_EINVAL, "need n_runs >= 1 and non-NULL arrays");
    if (n_runs > 65536) return fail(nullptr, NS_EUNSUPPORTED, "n_runs > 65536");
    for (int r = 0; r < n_runs; ++r) {
        std::string msg;
        const ns_status s = validate_run(priors + r, energies + r, cfgs + r, msg);
        if (s != NS_OK)
            return fail(nullptr, s, n_runs > 1 ? "run " + std::to_string(r) + ": " + msg : msg);
    }
    ns_ctx *ctx = new ns_ctx();
    ctx->n = n_runs;
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
    ctx->scratch = scratch_for_current_device(ctx->scratch_err);
    const int n = n_runs;
    if ((st = dalloc(ctx, &ctx->d_iscal, (size_t)n * 8)) ||
        (st = dalloc(ctx, &ctx->d_scal, (size_t)n * 8)) ||
        (st = dalloc(ctx, &ctx->d_ctr, (size_t)n * 16)) ||
        (st = dalloc(ctx, &ctx->dP, (size_t)n + 1)) || (st = dalloc(ctx, &ctx->dR, (size_t)n + 1)) ||
        (st = dalloc(ctx, &ctx->d_map1, (size_t)n + 1)))
        return bail(st);
    if (hipHostMalloc((void **)&ctx->h_iscal, (size_t)n * 8 * sizeof(int), hipHostMallocDefault) !=
        hipSuccess) {
        ctx->err = "hipHostMalloc failed";
        return bail(NS_ENOMEM);
    }
    ctx->runs.resize(n);
    for (int r = 0; r < n; ++r) {
        RunHost &rh = ctx->runs[r];
        rh.cfg = cfgs[r];
        rh.d = priors[r].d;
        rh.D = pad_dim(rh.d);
        rh.m = cfgs[r].n_live;
        rh.m_pad = (rh.m + 63) & ~63;
        rh.k = cfgs[r].outer == NS_OUTER_SMC ? cfgs[r].n_live : cfgs[r].k;   // SMC: every particle
        rh.p = cfgs[r].chain_len;
        rh.mode = cfgs[r].precision;
        if (cfgs[r].flags & NS_FLAG_TIMING) ctx->timing = 1;
        if (cfgs[r].flags & NS_FLAG_GRAPH) ctx->use_graph = 1;
        if (cfgs[r].flags & NS_FLAG_AUTOTUNE) ctx->autotune = 1;
        if (r == 0) ctx->smc = cfgs[r].outer == NS_OUTER_SMC;
        if ((cfgs[r].outer == NS_OUTER_SMC) != (ctx->smc != 0)) {
            ctx->err = "run " + std::to_string(r) + ": all runs of a context share the outer loop";
            return bail(NS_EINVAL);
        }
        if ((st = prepare_problem(ctx, rh, priors + r, energies + r)) != NS_OK) return bail(st);
        rh.lik = rh.P.lik_kind;
        rh.K = rh.P.K;
        if (rh.lik != LIK_GP && !mode_supported(rh.P, rh.mode)) {
            ctx->err = "mixed precision: n_comp too large for this dimension";
            if (n > 1) ctx->err = "run " + std::to_string(r) + ": " + ctx->err;
            return bail(NS_EUNSUPPORTED);
        }
        rh.upw = (rh.mode == NS_FP64 || rh.lik == LIK_GP) ? 1 : upw_template(rh.D, upw_for(rh.P));
        rh.P = problem_for_mode(rh, rh.mode);
        rh.P.gp_spin_max = (rh.cfg.flags & NS_FLAG_GP_NO_WAIT) ? -1 : (1 << 22);
        if ((st = alloc_run(ctx, r)) != NS_OK) return bail(st);
        // group by compiled HRSS kernel; the 16-bit mixture chains may plan 8 or 16 tests per
        // round unless NS_FLAG_SHALLOW_PLAN keeps them on the 4-test kernel
        const bool m16 = rh.mode == NS_MIXED_BF16 || rh.mode == NS_MIXED_FP16 ||
                         rh.mode == NS_MIXED_BF16X3 || rh.mode == NS_MIXED_FP16X3;
        const bool plan_ok = m16 && rh.lik == LIK_MIXTURE && !rh.R.rw && !rh.R.smc &&
                             rh.D <= 128 && rh.R.dirbuf &&
                             !(rh.cfg.flags & NS_FLAG_SHALLOW_PLAN);
        const int plan0 = !plan_ok ? 0 : (rh.cfg.flags & NS_FLAG_PLAN8) ? 8 : kDefaultPlan;
        int g = -1;
        for (size_t i = 0; i < ctx->groups.size(); ++i) {
            const Group &G = ctx->groups[i];
            if (G.D == rh.D && G.lik == rh.lik && G.mode == rh.mode && G.upwT == rh.upw &&
                G.rw == rh.R.rw && G.plan_ok == plan_ok && G.plan == plan0)
                g = (int)i;
        }
        if (g < 0) {
            ctx->groups.push_back(Group{rh.D, rh.lik, rh.mode, rh.upw, rh.R.rw, plan_ok, plan0,
                                        {}});
            g = (int)ctx->groups.size() - 1;
        }
        ctx->groups[g].runs.push_back(r);
    }
    ctx->snap_x.assign(n, nullptr);
    ctx->snap_l.assign(n, nullptr);
    ctx->snap_c.assign(n, nullptr);
    // chains per HRSS workgroup: enough workgroups to cover the CUs, full 16-row tiles beyond
    for (const Group &G : ctx->groups) {
        long long chains = 0;
        for (int r : G.runs) chains += ctx->runs[r].k;
        int C = (int)((chains + 255) / 256);
        C = C < 1 ? 1 : (C > kMaxChainsPerWG ? kMaxChainsPerWG : C);
        if (G.lik == LIK_GP) C = 1;   // one chain per workgroup
        for (int r : G.runs) ctx->runs[r].R.C = C;
    }
    // side streams and fork / join events for the concurrent chain launches of the groups
    if (ctx->groups.size() > 1 && !(cfgs[0].flags & NS_FLAG_SERIAL_GROUPS)) {
        ctx->side.assign(ctx->groups.size() - 1, nullptr);
        ctx->ev_join.assign(ctx->groups.size() - 1, nullptr);
        bool ok = hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) == hipSuccess;
        for (size_t i = 0; ok && i + 1 < ctx->groups.size(); ++i)
            ok = hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&ctx->ev_join[i], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            ctx->err = "side stream or event creation failed";
            return bail(NS_EDEVICE);
        }
    }
    // NS_FLAG_AUTOTUNE: a shape tuned before in this process takes its cached value; the others
    // time every candidate on their first iterations
    ctx->tune.assign(ctx->groups.size(), GroupTune{});
    for (size_t g = 0; g < ctx->groups.size() && ctx->autotune; ++g) {
        const Group &G = ctx->groups[g];
        if (G.lik == LIK_GP) continue;
        Shape cached{0, 0};
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tuned.find(tune_key(ctx, G));
            if (it != g_tuned.end()) cached = it->second;
        }
        if (cached.C > 0) {
            for (int r : G.runs) ctx->runs[r].R.C = cached.C;
            ctx->groups[g].plan = cached.plan;
            continue;
        }
        GroupTune &t = ctx->tune[g];
        for (int plan : {0, 8, 16}) {
            if (plan && !G.plan_ok) continue;
            for (int c = 1; c <= kMaxChainsPerWG; ++c) t.cand.push_back(Shape{c, plan});
        }
        t.done = false;
    }
    std::vector<DevProblem> hp(n + 1);
    std::vector<DevRun> hr(n + 1);
    std::vector<int2> m1(n + 1);
    size_t cap = 0;
    for (int r = 0; r < n; ++r) {
        const RunHost &rh = ctx->runs[r];
        hp[r] = rh.P;
        hr[r] = rh.R;
        m1[r] = make_int2(r, 0);
        // HRSS blocks at one chain per workgroup, the most any chains-per-workgroup value needs
        cap += (size_t)init_blocks(rh) + 1 + cov_blocks(rh) + dirs_blocks(rh) + eval_blocks(rh) +
               (size_t)rh.k;
    }
    hp[n] = hp[0];
    hr[n] = hr[0];
    m1[n] = make_int2(n, 0);
    if ((st = dalloc(ctx, &ctx->d_map, cap))) return bail(st);
    ctx->map_cap = cap;
    if (hipMemcpy(ctx->dP, hp.data(), hp.size() * sizeof(DevProblem), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(ctx->dR, hr.data(), hr.size() * sizeof(DevRun), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(ctx->d_map1, m1.data(), m1.size() * sizeof(int2), hipMemcpyHostToDevice) !=
            hipSuccess) {
        ctx->err = "descriptor upload failed";
        return bail(NS_EDEVICE);
    }
    if ((st = start_runs(ctx)) != NS_OK) return bail(st);
    if (any_error(ctx)) {
        ctx->err = "no live point lies strictly above L* after the first deletion";
        return bail(NS_ESTATE);
    }
    *out = ctx;
    return NS_OK;
}

extern "C" ns_status ns_init(const ns_prior *prior, const ns_energy *energy, const ns_config *cfg,
                             void *hip_stream, ns_ctx **out)
{
    if (!prior || !energy || !cfg) {
        g_init_err = "NULL argument";
        if (out) *out = nullptr;
        return NS_EINVAL;
    }
    return ns_init_batch(1, prior, energy, cfg, hip_stream, out);
}

extern "C" int32_t ns_num_runs(const ns_ctx *ctx) { return ctx ? ctx->n : 0; }

extern "C" ns_status ns_reset(ns_ctx *ctx, uint64_t seed, uint32_t run_id)
{
    if (!ctx) return NS_EINVAL;
    CK(hipStreamSynchronize(ctx->stream));
    std::vector<DevRun> hr(ctx->n + 1);
    for (int r = 0; r < ctx->n; ++r) {
        RunHost &rh = ctx->runs[r];
        rh.cfg.seed = seed;
        rh.cfg.run_id = run_id + (uint32_t)r;
        set_key(rh.R, seed, rh.cfg.run_id);
        hr[r] = rh.R;
    }
    hr[ctx->n] = hr[0];
    CK(hipMemcpy(ctx->dR, hr.data(), hr.size() * sizeof(DevRun), hipMemcpyHostToDevice));
    ns_status st = start_runs(ctx);
    if (st != NS_OK) return st;
    if (any_error(ctx)) return fail(ctx, NS_ESTATE, state_error_text(ctx));
    return NS_OK;
}

extern "C" ns_status ns_step(ns_ctx *ctx, int32_t *done)
{
    if (!ctx) return NS_EINVAL;
    if (all_done(ctx)) {
        if (done) *done = 1;
        return NS_DONE;
    }
    ns_status st = reserve_dead(ctx, 1);
    if (st != NS_OK) return st;
    st = tuning_due(ctx) ? tune_iteration(ctx) : enqueue_iteration(ctx);
    if (st != NS_OK) return st;
    ctx->iters_issued += 1;
    if ((st = sync_flags(ctx)) != NS_OK) return st;
    if ((st = collect_events(ctx)) != NS_OK) return st;
    if ((st = refresh_maps(ctx)) != NS_OK) return st;
    if (done) *done = all_done(ctx) ? 1 : 0;
    if (any_error(ctx)) return fail(ctx, NS_ESTATE, state_error_text(ctx));
    return NS_OK;
}

// kGraphIters iterations as one HIP graph: captured from the stream once per block-map epoch
// (the launch grids change when runs finish), replayed otherwise.  The iterations contain
// kernel launches only (no memset or copy nodes).
static ns_status launch_graph_batch(ns_ctx *ctx)
{
    if (!ctx->gexec || ctx->graph_epoch != ctx->map_epoch) {
        if (ctx->gexec) {
            CK(hipGraphExecDestroy(ctx->gexec));
            ctx->gexec = nullptr;
        }
        CK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        ns_status st = NS_OK;
        ctx->capturing = true;
        for (int b = 0; b < kGraphIters && st == NS_OK; ++b) st = enqueue_iteration(ctx);
        ctx->capturing = false;
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->stream, &g);
        if (st != NS_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return device_error(ctx, "graph capture", e);
        const hipError_t e2 = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) {
            ctx->gexec = nullptr;
            return device_error(ctx, "graph instantiation", e2);
        }
        ctx->graph_epoch = ctx->map_epoch;
    }
    CK(hipGraphLaunch(ctx->gexec, ctx->stream));
    return NS_OK;
}

extern "C" ns_status ns_run(ns_ctx *ctx, int32_t max_iter, int32_t *iters)
{
    if (!ctx || max_iter < 0) return NS_EINVAL;
    ns_status st;
    if ((st = sync_flags(ctx)) != NS_OK) return st;
    std::vector<int> start(ctx->n);
    for (int r = 0; r < ctx->n; ++r) start[r] = ctx->h_iscal[8 * r + 3];
    int issued = 0;
    while (!all_done(ctx) && issued < max_iter) {
        if ((st = refresh_maps(ctx)) != NS_OK) return st;
        if (tuning_due(ctx)) {   // a tuning iteration, alone
            if ((st = reserve_dead(ctx, 1)) != NS_OK) return st;
            if ((st = tune_iteration(ctx)) != NS_OK) return st;
            issued += 1;
            ctx->iters_issued += 1;
            if ((st = sync_flags(ctx)) != NS_OK) return st;
            continue;
        }
        int batch = (max_iter - issued) < kGraphIters ? (max_iter - issued) : kGraphIters;
        for (size_t g = 0; g < ctx->tune.size(); ++g)   // stop at the next tuning point
            if (tune_waiting(ctx, g) && ctx->tune[g].next_at - ctx->iters_issued < batch)
                batch = (int)(ctx->tune[g].next_at - ctx->iters_issued);
        if ((st = reserve_dead(ctx, batch)) != NS_OK) return st;
        if (ctx->use_graph && !ctx->timing && batch == kGraphIters) {
            if ((st = launch_graph_batch(ctx)) != NS_OK) return st;
        } else {
            for (int b = 0; b < batch; ++b)
                if ((st = enqueue_iteration(ctx)) != NS_OK) return st;
        }
        issued += batch;
        ctx->iters_issued += batch;
        if ((st = sync_flags(ctx)) != NS_OK) return st;
    }
    if ((st = collect_events(ctx)) != NS_OK) return st;
    int adv = 0;
    for (int r = 0; r < ctx->n; ++r) {
        const int a = ctx->h_iscal[8 * r + 3] - start[r];
        if (a > adv) adv = a;
    }
    if (iters) *iters = adv;
    if (any_error(ctx)) return fail(ctx, NS_ESTATE, state_error_text(ctx));
    return NS_OK;
}

// The tuning cache as JSON: {"nss_tune": 2, "entries": [{"D": .., "lik": .., "mode": ..,
// "upw": .., "rw": .., "chains": .., "planned": .., "C": .., "plan": ..}, ...]}, one entry per
// line ("planned": whether the group may use the hypothesis-plan kernel).
extern "C" ns_status ns_tune_save(const char *path, int32_t *n)
{
    if (!path) return NS_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = fopen(path, "w");
    if (!f) return fail(nullptr, NS_EINVAL, std::string("cannot write ") + path);
    fprintf(f, "{\"nss_tune\": 2, \"entries\": [");
    size_t i = 0;
    for (const auto &kv : g_tuned) {
        const std::vector<long long> &k = kv.first;
        fprintf(f, "%s\n  {\"D\": %lld, \"lik\": %lld, \"mode\": %lld, \"upw\": %lld, "
                   "\"rw\": %lld, \"chains\": %lld, \"planned\": %lld, \"C\": %d, \"plan\": %d}",
                i++ ? "," : "", k[0], k[1], k[2], k[3], k[4], k[5], k[6], kv.second.C,
                kv.second.plan);
    }
    fprintf(f, "\n]}\n");
    const bool ok = fclose(f) == 0;
    if (n) *n = (int32_t)g_tuned.size();
    return ok ? NS_OK : fail(nullptr, NS_EINVAL, std::string("cannot write ") + path);
}

extern "C" ns_status ns_tune_load(const char *path, int32_t *n)
{
    if (!path) return NS_EINVAL;
    FILE *f = fopen(path, "r");
    if (!f) return fail(nullptr, NS_EINVAL, std::string("cannot open ") + path);
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, got);
    fclose(f);
    if (txt.find("\"nss_tune\": 2") == std::string::npos)
        return fail(nullptr, NS_EINVAL, std::string(path) + ": not a tuning cache");
    std::map<std::vector<long long>, Shape> add;
    size_t pos = txt.find("\"entries\"");
    if (pos == std::string::npos)
        return fail(nullptr, NS_EINVAL, std::string(path) + ": not a tuning cache");
    for (; (pos = txt.find('{', pos)) != std::string::npos; ++pos) {
        long long D, lik, mode, upw, rw, chains, planned;
        int C, plan, end = -1;
        if (sscanf(txt.c_str() + pos,
                   "{\"D\": %lld, \"lik\": %lld, \"mode\": %lld, \"upw\": %lld, \"rw\": %lld, "
                   "\"chains\": %lld, \"planned\": %lld, \"C\": %d, \"plan\": %d}%n",
                   &D, &lik, &mode, &upw, &rw, &chains, &planned, &C, &plan, &end) != 9 ||
            end < 0 || C < 1 || C > kMaxChainsPerWG || chains < 1 || (rw != 0 && rw != 1) ||
            (D != 32 && D != 64 && D != 128 && D != 320) || lik < LIK_MIXTURE || lik > LIK_RG ||
            mode < NS_FP64 || mode > NS_MIXED_FP32 ||
            ((mode == NS_FP64 || lik == LIK_GP) ? upw != 1
                                                : upw_template((int)D, (int)upw) != upw) ||
            (planned != 0 && planned != 1) || (plan != 0 && plan != 8 && plan != 16) ||
            (plan != 0 && !planned))
            return fail(nullptr, NS_EINVAL, std::string(path) + ": malformed entry");
        add[{D, lik, mode, upw, rw, chains, planned}] = Shape{C, plan};
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : add) g_tuned[kv.first] = kv.second;
    if (n) *n = (int32_t)g_tuned.size();
    return NS_OK;
}

extern "C" ns_status ns_tune_clear(int32_t *n)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (n) *n = (int32_t)g_tuned.size();
    g_tuned.clear();
    return NS_OK;
}

extern "C" ns_status ns_launch_shape(const ns_ctx *ctx, int32_t run, int32_t *chains_per_wg,
                                     int32_t *plan_tests)
{
    if (!ctx || run < 0 || run >= ctx->n) return NS_EINVAL;
    int plan = 0;
    for (const Group &G : ctx->groups)
        for (int r : G.runs)
            if (r == run) plan = G.plan;
    if (chains_per_wg) *chains_per_wg = ctx->runs[run].R.C;
    if (plan_tests) *plan_tests = plan ? plan : (ctx->runs[run].lik == LIK_GP ? 1 : kSlots);
    return NS_OK;
}

extern "C" int32_t ns_chains_per_workgroup(const ns_ctx *ctx, int32_t run)
{
    if (!ctx || run < 0 || run >= ctx->n) return 0;
    return ctx->runs[run].R.C;
}

extern "C" ns_status ns_logz_batch(ns_ctx *ctx, double *logz, double *logz_err, double *H)
{
    if (!ctx) return NS_EINVAL;
    // every run, finished or not (the finalisation does not change the run's state)
    if (!ctx->smc) {
        Launch L{ctx->dP, ctx->dR, ctx->d_map1, ctx->n, 0, 0};
        hipError_t e = launch_logz(L, ctx->stream);
        if (e != hipSuccess) return device_error(ctx, "ns_logz", e);
    }
    std::vector<double> sc((size_t)ctx->n * 8);
    CK(hipMemcpyAsync(sc.data(), ctx->d_scal, sc.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    for (int r = 0; r < ctx->n; ++r) {
        if (logz) logz[r] = sc[(size_t)8 * r + (ctx->smc ? 1 : 4)];
        if (logz_err) logz_err[r] = ctx->smc ? NAN : sc[(size_t)8 * r + 5];
        if (H) H[r] = ctx->smc ? NAN : sc[(size_t)8 * r + 6];
    }
    return NS_OK;
}

extern "C" ns_status ns_logz(ns_ctx *ctx, double *logz, double *logz_err, double *H)
{
    if (!ctx) return NS_EINVAL;
    if (ctx->smc) {   // the accumulated estimate; a single SMC run gives no error estimate
        double z = 0.0;
        CK(hipMemcpyAsync(&z, ctx->d_scal + 1, sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
        CK(hipStreamSynchronize(ctx->stream));
        if (logz) *logz = z;
        if (logz_err) *logz_err = NAN;
        if (H) *H = NAN;
        return NS_OK;
    }
    const Launch L = launch_one(ctx, 0);
    hipError_t e = launch_logz(L, ctx->stream);
    if (e != hipSuccess) return device_error(ctx, "ns_logz", e);
    double out[3];
    CK(hipMemcpyAsync(out, ctx->d_scal + 4, 3 * sizeof(double), hipMemcpyDeviceToHost,
                      ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    if (logz) *logz = out[0];
    if (logz_err) *logz_err = out[1];
    if (H) *H = out[2];
    return NS_OK;
}

static bool run_ok(const ns_ctx *ctx, int r) { return ctx && r >= 0 && r < ctx->n; }

extern "C" ns_status ns_stats_run(ns_ctx *ctx, int32_t run, ns_stats_t *o)
{
    if (!run_ok(ctx, run) || !o) return NS_EINVAL;
    ns_status st;
    if ((st = collect_events(ctx)) != NS_OK) return st;
    unsigned long long c[16];
    CK(hipMemcpyAsync(c, ctx->d_ctr + 16 * run, sizeof(c), hipMemcpyDeviceToHost, ctx->stream));
    if ((st = sync_flags(ctx)) != NS_OK) return st;
    memset(o, 0, sizeof(*o));
    o->iterations = ctx->h_iscal[8 * run + 3];
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
    o->width = ctx->runs[run].R.width;
    o->tune_launches = ctx->tune_launches;
    o->gp_wait_timeouts = (int64_t)c[10];
    return NS_OK;
}

extern "C" ns_status ns_stats(ns_ctx *ctx, ns_stats_t *o) { return ns_stats_run(ctx, 0, o); }

extern "C" ns_status ns_get_state_run(ns_ctx *ctx, int32_t run, ns_state_view *v)
{
    if (!run_ok(ctx, run) || !v) return NS_EINVAL;
    const RunHost &rh = ctx->runs[run];
    const DevRun &R = rh.R;
    const int d = rh.d, D = rh.D, m = rh.m, mp = rh.m_pad;
    CK(hipStreamSynchronize(ctx->stream));
    if (v->x) {
        std::vector<double> t((size_t)D * mp);
        CK(hipMemcpy(t.data(), R.X, t.size() * 8, hipMemcpyDeviceToHost));
        for (int i = 0; i < m; ++i)
            for (int a = 0; a < d; ++a) v->x[(size_t)i * d + a] = t[(size_t)a * mp + i];
    }
    if (v->logL) CK(hipMemcpy(v->logL, R.logL, m * 8, hipMemcpyDeviceToHost));
    if (v->perm) CK(hipMemcpy(v->perm, R.perm, m * 4, hipMemcpyDeviceToHost));
    if (v->Lsig) {
        std::vector<double> t((size_t)D * D);
        CK(hipMemcpy(t.data(), R.Lsig, t.size() * 8, hipMemcpyDeviceToHost));
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) v->Lsig[a * d + b] = t[a * D + b];
    }
    if (v->parents) CK(hipMemcpy(v->parents, R.parents, rh.k * 4, hipMemcpyDeviceToHost));
    double sc[4];
    int is[8];
    CK(hipMemcpy(sc, R.scal, sizeof(sc), hipMemcpyDeviceToHost));
    CK(hipMemcpy(is, R.iscal, sizeof(is), hipMemcpyDeviceToHost));
    v->Lstar = sc[0]; v->logZ = sc[1]; v->logX = sc[2]; v->M = sc[3];
    v->iter = is[3];
    v->done = is[0];
    return NS_OK;
}

extern "C" ns_status ns_get_state(ns_ctx *ctx, ns_state_view *v)
{
    return ns_get_state_run(ctx, 0, v);
}

extern "C" ns_status ns_set_state(ns_ctx *ctx, const ns_state_view *v)
{
    if (!ctx || !v || !v->x || !v->logL) return NS_EINVAL;
    if (ctx->smc) return fail(ctx, NS_EUNSUPPORTED, "ns_set_state is for nested-sampling runs");
    RunHost &rh = ctx->runs[0];
    const DevRun &R = rh.R;
    const int d = rh.d, D = rh.D, m = rh.m, mp = rh.m_pad;
    std::vector<double> t((size_t)D * mp, 0.0);
    for (int i = 0; i < m; ++i)
        for (int a = 0; a < d; ++a) t[(size_t)a * mp + i] = v->x[(size_t)i * d + a];
    // a stored log L that is NaN or +inf is taken as -inf (rejected) and counted, as for a
    // computed one
    std::vector<double> lg(v->logL, v->logL + m);
    unsigned long long nf = 0;
    for (double &l : lg)
        if (l != l || l == INFINITY) { l = -INFINITY; ++nf; }
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(R.X, t.data(), t.size() * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(R.logL, lg.data(), m * 8, hipMemcpyHostToDevice));
    if (nf) {
        unsigned long long c5 = 0;
        CK(hipMemcpy(&c5, R.ctr + 5, sizeof(c5), hipMemcpyDeviceToHost));
        c5 += nf;
        CK(hipMemcpy(R.ctr + 5, &c5, sizeof(c5), hipMemcpyHostToDevice));
    }
    double sc[4] = {0.0, v->logZ, v->logX, v->M};
    CK(hipMemcpy(R.scal, sc, sizeof(sc), hipMemcpyHostToDevice));
    int is[8];
    CK(hipMemcpy(is, R.iscal, sizeof(is), hipMemcpyDeviceToHost));
    is[0] = 0; is[3] = (int)v->iter; is[4] = 0;
    if (R.freeze && v->Lsig) {
        // the caller's factor is kept for the run: both the row-major and the packed copy
        std::vector<double> Ls((size_t)D * D, 0.0), pk((size_t)D * (D + 1) / 2, 0.0);
        for (int a = 0; a < d; ++a)
            for (int b = 0; b <= a; ++b) {
                const double e = v->Lsig[(size_t)a * d + b];
                if (!std::isfinite(e)) return fail(ctx, NS_EINVAL, "non-finite factor entry");
                Ls[(size_t)a * D + b] = e;
                pk[(size_t)a * (a + 1) / 2 + b] = e;
            }
        CK(hipMemcpy(R.Lsig, Ls.data(), Ls.size() * 8, hipMemcpyHostToDevice));
        CK(hipMemcpy(R.Lpk, pk.data(), pk.size() * 8, hipMemcpyHostToDevice));
        is[6] = 1;
    }
    CK(hipMemcpy(R.iscal, is, sizeof(is), hipMemcpyHostToDevice));
    hipError_t e = launch_select(launch_one(ctx, 0), 2, ctx->stream);
    if (e != hipSuccess) return device_error(ctx, "select launch", e);
    ns_status st;
    if ((st = sync_flags(ctx)) != NS_OK) return st;
    is[0] = v->done ? 1 : 0;
    CK(hipMemcpy(R.iscal, is, sizeof(int), hipMemcpyHostToDevice));
    rh.done = is[0];
    return refresh_maps(ctx);
}

extern "C" ns_status ns_get_dead(ns_ctx *ctx, double *out, int64_t cap, int64_t *n)
{
    if (!ctx) return NS_EINVAL;
    const DevRun &R = ctx->runs[0].R;
    unsigned long long nd = 0;
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(&nd, R.ctr + 9, 8, hipMemcpyDeviceToHost));
    long long stored = (long long)nd < R.dead_cap ? (long long)nd : R.dead_cap;
    if (n) *n = (int64_t)nd;
    if (out && cap > 0) {
        const long long c = stored < cap ? stored : cap;
        if (c > 0) CK(hipMemcpy(out, R.dead, c * 8, hipMemcpyDeviceToHost));
    }
    return NS_OK;
}

// Checks the arguments of a geometric-uncertainty call on run `run` and fills G (sizes, keys
// and run buffers; no output or workspace pointers).  Reads the run's death count (a copy and
// a wait on the context's stream).
static ns_status plan_geom(ns_ctx *ctx, int run, int R, double beta, uint64_t seed,
                           uint32_t run_id, GeomLaunch &G)
{
    if (ctx->smc) return fail(ctx, NS_EUNSUPPORTED, "an SMC run has no dead record");
    if (R < 1 || R > 65535) return fail(ctx, NS_EINVAL, "replicas must be in [1, 65535]");
    if (!(beta >= 0.0) || beta == INFINITY) return fail(ctx, NS_EINVAL, "beta must be finite and >= 0");
    const RunHost &rh = ctx->runs[run];
    const DevRun &D = rh.R;
    unsigned long long nd = 0;
    CK(hipMemcpyAsync(&nd, D.ctr + 9, 8, hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    if ((long long)nd > D.dead_cap)
        return fail(ctx, NS_ESTATE, "dead record truncated: more deaths than max_iter + 1 iterations hold");
    const long long N = (long long)nd + (rh.m - rh.k);
    if (N >= (1ll << 31)) return fail(ctx, NS_EUNSUPPORTED, "more than 2^31 - 1 deaths");
    G = GeomLaunch{};
    G.dead = D.dead;
    G.n_dead = (long long)nd;
    G.N = N;
    G.logL = D.logL;
    G.perm = D.perm;
    G.m = rh.m;
    G.k = rh.k;
    G.R = R;
    G.groups = geom_groups(N, R);
    G.beta = beta;
    G.key0 = (uint32_t)seed;
    G.key1 = (uint32_t)(seed >> 32) ^ run_id;
    return NS_OK;
}

// The geometric-uncertainty computation of run `run` on the context's stream, outputs left in
// the context's buffer (extra = further bytes reserved after them, at *extra_ptr).
static ns_status enqueue_geom(ns_ctx *ctx, int run, int R, double beta, uint64_t seed,
                              uint32_t run_id, size_t extra, GeomLaunch &G, char **extra_ptr)
{
    ns_status st = plan_geom(ctx, run, R, beta, seed, run_id, G);
    if (st != NS_OK) return st;
    const long long N = G.N;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t out_bytes = up((size_t)R * 8) + up((size_t)N * 8) + up(8);
    const size_t wsb = up(geom_workspace_bytes(N, R, G.groups));
    const size_t need = out_bytes + wsb + extra;
    if (need > ctx->geom_bytes) {
        if (ctx->geom_buf) CK(hipFree(ctx->geom_buf));
        ctx->geom_buf = nullptr;
        ctx->geom_bytes = 0;
        CK(hipMalloc(&ctx->geom_buf, need));
        ctx->geom_bytes = need;
    }
    char *b = (char *)ctx->geom_buf;
    G.logz = (double *)b;
    G.logw_mean = (double *)(b + up((size_t)R * 8));
    G.ess = (double *)(b + up((size_t)R * 8) + up((size_t)N * 8));
    G.ws = b + out_bytes;
    if (extra_ptr) *extra_ptr = b + out_bytes + wsb;
    hipError_t e = launch_geom(G, ctx->stream);
    if (e != hipSuccess) return device_error(ctx, "geometric-uncertainty launch", e);
    return NS_OK;
}

extern "C" ns_status ns_geom_uncertainty(ns_ctx *ctx, int32_t run, int32_t R, double beta,
                                         uint64_t seed, uint32_t run_id, double *logz,
                                         double *logw_mean, int64_t cap, double *ess,
                                         int64_t *n_deaths, double *device_ms)
{
    if (!run_ok(ctx, run) || !logz) return NS_EINVAL;
    if (cap < 0) return fail(ctx, NS_EINVAL, "cap < 0");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (device_ms) {
        CK(hipEventCreate(&e0));
        CK(hipEventCreate(&e1));
    }
    GeomLaunch G;
    ns_status st;
    if (device_ms) CK(hipEventRecord(e0, ctx->stream));
    if ((st = enqueue_geom(ctx, run, R, beta, seed, run_id, 0, G, nullptr)) != NS_OK) {
        if (e0) { (void)hipEventDestroy(e0); (void)hipEventDestroy(e1); }
        return st;
    }
    if (device_ms) CK(hipEventRecord(e1, ctx->stream));
    if (n_deaths) *n_deaths = G.N;
    CK(hipMemcpyAsync(logz, G.logz, (size_t)R * 8, hipMemcpyDeviceToHost, ctx->stream));
    const long long nc = cap < G.N ? (long long)cap : G.N;
    if (logw_mean && nc > 0)
        CK(hipMemcpyAsync(logw_mean, G.logw_mean, (size_t)nc * 8, hipMemcpyDeviceToHost,
                          ctx->stream));
    if (ess) CK(hipMemcpyAsync(ess, G.ess, 8, hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    if (device_ms) {
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, e0, e1));
        *device_ms = ms;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return NS_OK;
}

extern "C" ns_status ns_geom_uncertainty_noalloc(ns_ctx *ctx, int32_t run, int32_t R,
                                                 double beta, uint64_t seed, uint32_t run_id,
                                                 double *logz, double *logw_mean, int64_t cap,
                                                 double *ess, int64_t *n_deaths)
{
    if (!run_ok(ctx, run) || !logz || !logw_mean || !ess) return NS_EINVAL;
    if (!ctx->scratch)
        return fail(ctx, NS_EDEVICE, "no fixed workspace on this device: " + ctx->scratch_err);
    GeomLaunch G;
    ns_status st = plan_geom(ctx, run, R, beta, seed, run_id, G);
    if (st != NS_OK) return st;
    if (n_deaths) *n_deaths = G.N;
    if (cap < G.N)
        return fail(ctx, NS_EINVAL, "logw_mean holds " + std::to_string(cap) + " values, " +
                                        std::to_string(G.N) + " deaths");
    const size_t wsb = geom_workspace_bytes(G.N, R, G.groups);
    if (wsb > (size_t)NS_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, NS_EINVAL, "workspace of " + std::to_string(wsb) + " bytes exceeds the " +
                                        std::to_string((size_t)NS_NOALLOC_SCRATCH_BYTES) +
                                        "-byte fixed workspace (fewer replicas or deaths)");
    G.logz = logz;
    G.logw_mean = logw_mean;
    G.ess = ess;
    G.ws = ctx->scratch;
    hipError_t e = launch_geom(G, ctx->stream);
    if (e != hipSuccess) return device_error(ctx, "geometric-uncertainty launch", e);
    return NS_OK;
}

extern "C" ns_status ns_posterior_samples(ns_ctx *ctx, int32_t run, int32_t R, double beta,
                                          uint64_t seed, uint32_t run_id, int32_t n, double *x,
                                          int64_t *idx)
{
    if (!run_ok(ctx, run) || !x || n < 1) return NS_EINVAL;
    const RunHost &rh = ctx->runs[run];
    if (!rh.R.deadx)
        return fail(ctx, NS_ESTATE, "the dead points' coordinates were not recorded "
                                    "(NS_FLAG_RECORD_POINTS)");
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const long long nd_cap = rh.R.dead_cap + (rh.m - rh.k);   // bound on N for the scratch
    const size_t b_cum = up((size_t)nd_cap * 8), b_x = up((size_t)n * rh.d * 8),
                 b_i = up((size_t)n * 8), b_ws = up((size_t)(2 + 2 * post_cum_blocks(nd_cap)) * 8);
    GeomLaunch G;
    char *xb = nullptr;
    ns_status st;
    if ((st = enqueue_geom(ctx, run, R, beta, seed, run_id, b_cum + b_x + b_i + b_ws, G, &xb)) !=
        NS_OK)
        return st;
    double *cum = (double *)xb;
    double *xo = (double *)(xb + b_cum);
    long long *io = (long long *)(xb + b_cum + b_x);
    double *cws = (double *)(xb + b_cum + b_x + b_i);
    hipError_t e = launch_post_samples(G, rh.R.deadx, rh.R.X, rh.m_pad, rh.d, n, cum, cws, xo, io,
                                       ctx->stream);
    if (e != hipSuccess) return device_error(ctx, "posterior-sample launch", e);
    CK(hipMemcpyAsync(x, xo, (size_t)n * rh.d * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (idx) CK(hipMemcpyAsync(idx, io, (size_t)n * 8, hipMemcpyDeviceToHost, ctx->stream));
    CK(hipStreamSynchronize(ctx->stream));
    return NS_OK;
}

extern "C" ns_status ns_get_trace(ns_ctx *ctx, int32_t *out)
{
    if (!ctx || !out) return NS_EINVAL;
    const RunHost &rh = ctx->runs[0];
    if (!rh.R.trace) return fail(ctx, NS_EINVAL, "context was created without NS_FLAG_TRACE");
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(out, rh.R.trace, (size_t)rh.k * rh.p * 16, hipMemcpyDeviceToHost));
    return NS_OK;
}

extern "C" ns_status ns_eval_loglik(ns_ctx *ctx, const double *x, int32_t n, int32_t precision,
                                    double *out)
{
    if (!ctx || (!x && n > 0) || (!out && n > 0) || n < 0) return NS_EINVAL;
    if (n == 0) return NS_OK;
    if (!precision_valid(precision)) return fail(ctx, NS_EINVAL, "unknown precision");
    const RunHost &rh = ctx->runs[0];
    const bool gp = rh.lik == LIK_GP;
    if (gp ? (precision != NS_FP64 && precision != NS_MIXED_FP32)
           : (precision == NS_MIXED_FP32 || !mode_supported(rh.P, precision)))
        return fail(ctx, NS_EUNSUPPORTED, "precision not supported for this problem");
    const DevProblem P = problem_for_mode(rh, precision);
    const int upw = (precision == NS_FP64 || gp) ? 1 : upw_template(rh.D, upw_for(P));
    const int d = rh.d, D = rh.D;
    const int np = (n + 63) & ~63;
    const int nb = gp ? n : (n + kRows - 1) / kRows;
    std::vector<double> t((size_t)D * np, 0.0);
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < d; ++a) t[(size_t)a * np + i] = x[(size_t)i * d + a];
    std::vector<int2> mp(nb);
    for (int b = 0; b < nb; ++b) mp[b] = make_int2(ctx->n, b);  // the scratch descriptor slot
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(ctx->dP + ctx->n, &P, sizeof(P), hipMemcpyHostToDevice));
    double *dx = nullptr, *dout = nullptr;
    int2 *dmap = nullptr;
    hipError_t e = hipMalloc(&dx, t.size() * 8);
    if (e == hipSuccess) e = hipMalloc(&dout, (size_t)n * 8);
    if (e == hipSuccess) e = hipMalloc(&dmap, (size_t)nb * sizeof(int2));
    if (e != hipSuccess) {
        (void)hipFree(dx);
        (void)hipFree(dout);
        return fail(ctx, NS_ENOMEM, "hipMalloc failed");
    }
    ns_status st = NS_OK;
    e = hipMemcpy(dx, t.data(), t.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dmap, mp.data(), mp.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        const Launch L{ctx->dP, ctx->dR, dmap, nb, rh.m, rh.K};
        e = gp ? launch_eval_gp(L, precision, dx, np, n, dout, 0, ctx->stream)
               : launch_eval_points(L, D, rh.lik, precision, upw, dx, np, n, dout, ctx->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, dout, (size_t)n * 8, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        ctx->err = std::string("ns_eval_loglik: ") + hipGetErrorString(e);
        st = e == hipErrorNotSupported ? NS_EUNSUPPORTED : NS_EDEVICE;
    }
    (void)hipFree(dx);
    (void)hipFree(dout);
    (void)hipFree(dmap);
    return st;
}

#ifdef NSS_PHASE_TIMING
// Timing builds only: per-phase shader-clock cycles of one lane per HRSS workgroup, summed
// over workgroups and launches (0 direction, 1 candidates, 2 barrier, 3 tile, 4 re-check vote,
// 5 FP64 re-check, 6 round top, 7 state update, 8 rounds, 9 steps, 10 re-check rounds).
extern "C" ns_status nss_debug_phase_times(ns_ctx *ctx, unsigned long long *out)
{
    if (!ctx || !out || !ctx->runs[0].R.prof) return NS_EINVAL;
    CK(hipStreamSynchronize(ctx->stream));
    CK(hipMemcpy(out, ctx->runs[0].R.prof, 12 * 8, hipMemcpyDeviceToHost));
    return NS_OK;
}
#endif
