// Internal shared declarations of the gfx950 NSS library: device-side problem and run
// descriptors and the kernel launchers called by the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nss {

constexpr int kWG = 256;         // threads per chain workgroup (4 waves of 64)
constexpr int kRows = 16;        // candidate rows per evaluation tile (one 16-row MFMA block)
constexpr int kSlots = 2;        // candidate slots per chain per round (left / right end)
constexpr int kMaxChainsPerWG = 4;
constexpr int kSelectThreads = 1024;
constexpr int kMaxLive = 8192;

// likelihood arithmetic inside the chains (values equal the C ABI's ns_precision)
enum Mode { MODE_FP64 = 0, MODE_BF16 = 1, MODE_FP16 = 2, MODE_BF16X3 = 3, MODE_FP16X3 = 4 };
enum PriorKind { PRIOR_BOX = 0, PRIOR_GAUSS = 1 };
enum LikKind { LIK_MIXTURE = 1, LIK_FUNNEL = 2 };

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
    float guard_abs;
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
                              // [8] whiten_fallbacks [9] n_dead
    double *Lsig;          // [D][D] lower factor (row-major, zero above the diagonal)
    double *Lpk;           // packed lower factor, D(D+1)/2
    int *parents;          // [k]
    double *dead;          // dead logL record
    long long dead_cap;
    int *trace;            // [k][p][4] or null
    unsigned long long *prof;  // per-phase cycle counters of the HRSS kernel (timing builds)
    double *dirbuf;        // [k][p][D] directions of the current iteration, or null (inline)
};

// ---- launchers (nss_kernels.hip) ----
hipError_t launch_init_draw(const DevProblem &P, const DevRun &R, hipStream_t s);
hipError_t launch_eval_points(const DevProblem &P, const double *X, int ld, int n, double *out,
                              unsigned long long *nonfinite, int mode, hipStream_t s);
// op: 0 = initial delete-k (accounted), 1 = delete-k of an iteration (accounted, iter + 1),
//     2 = re-sort only (no accounting; after an external state overwrite)
hipError_t launch_select(const DevProblem &P, const DevRun &R, int op, hipStream_t s);
hipError_t launch_cov(const DevProblem &P, const DevRun &R, double *part1, double *part2, int G,
                      hipStream_t s);
hipError_t launch_dirs(const DevProblem &P, const DevRun &R, hipStream_t s);
hipError_t launch_hrss(const DevProblem &P, const DevRun &R, int mode, hipStream_t s);
hipError_t launch_logz(const DevProblem &P, const DevRun &R, hipStream_t s);
int mode_supported(const DevProblem &P, int mode);

}  // namespace nss
