// Internal shared declarations of the gfx950 NSS library: device-side problem and run
// descriptors and the kernel launchers called by the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nss {

constexpr int kWG = 256;         // threads per chain workgroup (4 waves of 64)
constexpr int kRows = 16;        // candidate rows per evaluation tile (one 16-row MFMA block)
constexpr int kSlots = 4;        // candidate rows per chain per round (4 chains x 4 = 16 rows)
constexpr int kMaxChainsPerWG = 4;
constexpr int kStepU = 8;        // per chain step in the uniform buffer: tL0, uh, shrink uniforms
constexpr int kStepShrinkU = kStepU - 2;
constexpr int kSelectThreads = 1024;
constexpr int kMaxLive = 8192;
constexpr long long kDeadInitIters = 512;   // initial dead record, in iterations (then grown)

// likelihood arithmetic inside the chains (values equal the C ABI's ns_precision)
enum Mode { MODE_FP64 = 0, MODE_BF16 = 1, MODE_FP16 = 2, MODE_BF16X3 = 3, MODE_FP16X3 = 4,
            MODE_FP32 = 5 };
enum PriorKind { PRIOR_BOX = 0, PRIOR_GAUSS = 1 };
enum LikKind { LIK_MIXTURE = 1, LIK_FUNNEL = 2, LIK_GP = 3, LIK_RG = 4 };
constexpr int kGpMaxObs = 256;   // GP observations per problem

// Problem, resident on the device for the lifetime of a context.
struct DevProblem {
    int d;                 // dimension
    int D;                 // padded dimension: 32, 64 or 128
    int prior_kind;
    const double *pa;      // [D] box lower | Gaussian mean
    const double *pb;      // [D] box upper | Gaussian std
    double logprior_norm;  // box: -sum log(b-a); Gaussian: -sum log b - d/2 log(2 pi)
    int lik_kind;
    int K;                 // mixture components
    const double *mu;      // [K][D]
    const float *mu32;     // [K][D]
    const double *wf64;    // FP64 W fragments, [K][D/16][D/4][64]
    const uint4 *wf16;     // 16-bit W fragments, [K][D/16][D/32][64], 8 halves each
    const uint4 *wf16lo;   // rounded remainders W - wf16 (split-precision modes)
    const double *cst;     // [K] log w_c - d/2 log(2 pi) + log det W_c
    const float *cst32;
    float cmax32;          // max_c cst32[c]
    float guard_rel;       // mixed precision guard band: rel * max(0, cmax - L) + abs
    float guard_abs;       //   (GP: rel |L| + abs + kappa_coef kappa n / 256)
    float guard_kappa;
    int gp_n;              // GP: observations
    int gp_spin_max;       // GP: bound on the pivot wave's wait per diagonal tile (< 0: give
                           //     up at once, a test mode)
    const double *gp_x;    // GP: [n][2] inputs
    const double *gp_y;    // GP: [n] targets
    double rg_la, rg_l1a;  // Gaussian-Rastrigin: log alpha, log(1 - alpha) (-inf at 0 / 1)
    double rg_amp;         // Gaussian-Rastrigin: A
};

// Run state on the device.
struct DevRun {
    int m, m_pad, k, p;
    double width;
    int stepout_cap, shrink_cap;
    double log_term;       // ln(term_frac), or +inf-like flag when disabled (use term_on)
    int term_on;
    uint32_t key0, key1;   // Philox key
    double *X;             // [D][m_pad] live points, coordinate-major (particle index fastest)
    double *logL;          // [m]
    int *perm;             // [m] ascending (logL, index)
    double *scal;          // [0] L*, [1] logZ, [2] logX, [3] M = H + logZ, [4..6] logz output
    int *iscal;            // [0] done, [1] t0, [2] n_s, [3] iter, [4] state error
    unsigned long long *ctr;  // [0] evals [1] tests [2] prior_rejects [3] stepout_caps
                              // [4] shrink_caps [5] nonfinite [6] rechecks [7] band_violations
                              // [8] whiten_fallbacks [9] n_dead [10] GP wait time-outs
    double *Lsig;          // [D][D] lower factor (row-major, zero above the diagonal)
    double *Lpk;           // packed lower factor, D(D+1)/2
    int *parents;          // [k]
    double *dead;          // dead logL record
    double *deadx;         // NS_FLAG_RECORD_POINTS: dead coordinates [dead_cap][d], or null
    long long dead_cap;
    int *trace;            // [k][p][4] or null
    unsigned long long *prof;  // per-phase cycle counters of the HRSS kernel (timing builds)
    double *dirbuf;        // [k][p][D] directions of the current iteration, or null (inline)
    double *ubuf;          // [k][p][8] per-step default plan (tL0, uh, 6 shrink), with dirbuf
    int rw;                // replacement by constrained random walk (width = its scale)
    int freeze;            // whitening factor of the first iteration kept for the run
    int diag;              // metric from the survivors' variances alone (diagonal)
    int smc;               // adaptive tempered SMC outer loop (k = m chains, no hard constraint)
    double ess_frac;       // SMC: ESS target rho of the next temperature
    double *Xtmp, *Ltmp;   // SMC: gather buffers [D][m_pad], [m]
    int C;                 // chains per HRSS workgroup
    int covG;              // survivor groups of the covariance partial sums
    double *part1, *part2; // covariance partials [covG][D], [covG][ntile][256]
};

// One kernel launch over a group of runs: block b works on run map[b].x, local block map[b].y.
// P and R are device arrays of the batch's runs.
struct Launch {
    const DevProblem *P;
    const DevRun *R;
    const int2 *map;
    int nblocks;
    int max_m;   // largest n_live among the launch's runs (select workspace)
    int max_K;   // largest component count among the launch's runs (HRSS workspace)
};

// ---- launchers (nss_kernels.hip); D, likelihood and mode are the group's template values ----
hipError_t launch_init_draw(const Launch &L, hipStream_t s);
// FP64 evaluation of each run's live set into its logL (after launch_init_draw)
hipError_t launch_eval_init(const Launch &L, int D, int lik, hipStream_t s);
// evaluation of n points X[a * ld + i] of the map's run(s) into out (tests)
hipError_t launch_eval_points(const Launch &L, int D, int lik, int mode, int upw, const double *X,
                              int ld, int n, double *out, hipStream_t s);
// op: 0 = initial delete-k (accounted), 1 = delete-k of an iteration (accounted, iter + 1),
//     2 = re-sort only (no accounting; after an external state overwrite); one block per run
hipError_t launch_select(const Launch &L, int op, hipStream_t s);
// adaptive tempered SMC: op 0 start, 1 next temperature + resampling, 2 end of step
hipError_t launch_smc(const Launch &L, int op, hipStream_t s);
// survivors' covariance (cov map: (run, tile + ntile * group)) and factorisation (one per run)
hipError_t launch_cov(const Launch &cov, const Launch &one, int D, hipStream_t s);
hipError_t launch_dirs(const Launch &L, int D, hipStream_t s);
hipError_t launch_hrss(const Launch &L, int D, int lik, int mode, int upw, hipStream_t s);
// the mixture chains in a 16-bit mode with S-test hypothesis plans (nss_hrss_plan.hip),
// S = 8 or 16; needs the direction buffer
hipError_t launch_hrss_plan(const Launch &L, int D, int mode, int upw, int S, int occ,
                            hipStream_t s);
size_t hrss_plan_lds_bytes(int D, int K, int S);
// the random-walk replacement kernel (same grid and tile evaluators as the HRSS kernel)
hipError_t launch_rw(const Launch &L, int D, int lik, int mode, int upw, hipStream_t s);
hipError_t launch_logz(const Launch &L, hipStream_t s);
// GP likelihood (nss_gp.hip): chains one per workgroup (map: (run, chain)); evaluation one
// point per workgroup (map: (run, point)), from_run = 1 evaluates the run's live set
hipError_t launch_hrss_gp(const Launch &L, int mode, hipStream_t s);
hipError_t launch_eval_gp(const Launch &L, int mode, const double *X, int ld, int n, double *out,
                          int from_run, hipStream_t s);
int mode_supported(const DevProblem &P, int mode);
int upw_for(const DevProblem &P);
int upw_template(int D, int upw);         // the compiled UPW that covers upw (0 if none)
size_t hrss_lds_bytes(int D, int K);
int dirs_rows(int D);                     // directions per k_dirs block

// Post-hoc geometric uncertainty (nss_post.hip).  Deaths: the dead record, then the final
// survivors logL[perm[k..m-1]]; outputs logz[R], logw_mean[N], ess[1] on the device; ws holds
// geom_workspace_bytes(N, R, groups) bytes of partial results.
struct GeomLaunch {
    const double *dead;
    long long n_dead, N;
    const double *logL;
    const int *perm;
    int m, k, R, groups;
    double beta;
    uint32_t key0, key1;
    double *logz, *logw_mean, *ess;
    void *ws;
};
size_t geom_workspace_bytes(long long N, int R, int groups);
int geom_groups(long long N, int R);
hipError_t launch_geom(const GeomLaunch &G, hipStream_t s);
// Posterior samples from the geometric-mean weights left in G.logw_mean: systematic resampling
// of n deaths (one uniform, purpose 7), coordinates from deadx (point-major, stride d) or the
// survivors' columns of X.  cum: [N] scratch; cws: [2 + 2 post_cum_blocks(N)] scratch;
// xo: [n][d]; io: [n] death indices.
long long post_cum_blocks(long long N);
hipError_t launch_post_samples(const GeomLaunch &G, const double *deadx, const double *X,
                               int m_pad, int d, int n, double *cum, double *cws, double *xo,
                               long long *io, hipStream_t s);

}  // namespace nss
