// gfx950 kernels of the Nested Slice Sampling hot path.
//
//  k_init_draw   prior draws of the m initial live points (Philox purpose INIT)
//  k_eval        batched likelihood of n points, 16 rows per workgroup (init, tests)
//  k_select      delete-k: sort (logL, index), threshold L*, unrolled evidence update of the
//                k deaths, dead record, termination flag (Sec. 2.1; App. D.2.1)
//  k_cov/k_chol  whitening: survivors' covariance + jitter, lower Cholesky factor (Sec. 3.2)
//  k_hrss        the k HRSS chains (App. A.6): one wave runs one chain's finite-state machine
//                (direction, bracket, step-out, shrink), the four waves of a workgroup
//                evaluate the tile of up to 16 candidate rows together on MFMA
//  k_logz        final live-set contribution to the evidence (Sec. 2.1)
#include "nss_internal.hpp"
#include "nss_rng.hpp"
#include "nss_tiles.hpp"
#include "nss_wave.hpp"

#include <math.h>

namespace nss {


// ------------------------------------------------------------------------------------------
// init: m prior draws
// ------------------------------------------------------------------------------------------
__global__ void k_init_draw(Launch Lc)
{
    const int2 bm = Lc.map[blockIdx.x];
    const DevProblem P = Lc.P[bm.x];
    const DevRun R = Lc.R[bm.x];
    const int nq = (P.d + 1) >> 1;
    const long long gid = (long long)bm.y * blockDim.x + threadIdx.x;
    if (gid >= (long long)R.m * nq) return;
    const int i = (int)(gid / nq), q = (int)(gid - (long long)i * nq);
    double ua, ub;
    draw2(R.key0, R.key1, PUR_INIT, (uint32_t)i, 0u, 0u, (uint32_t)q, ua, ub);
    const int a0 = 2 * q, a1 = 2 * q + 1;
    double x0, x1;
    if (P.prior_kind == PRIOR_BOX) {
        x0 = P.pa[a0] + (P.pb[a0] - P.pa[a0]) * ua;
        x1 = (a1 < P.d) ? P.pa[a1] + (P.pb[a1] - P.pa[a1]) * ub : 0.0;
    } else {
        double z0, z1;
        box_muller(ua, ub, z0, z1);
        x0 = P.pa[a0] + P.pb[a0] * z0;
        x1 = (a1 < P.d) ? P.pa[a1] + P.pb[a1] * z1 : 0.0;
    }
    R.X[(size_t)a0 * R.m_pad + i] = x0;
    if (a1 < P.d) R.X[(size_t)a1 * R.m_pad + i] = x1;
}

// ------------------------------------------------------------------------------------------
// batched evaluation of n points stored coordinate-major X[a*ld + i]
// ------------------------------------------------------------------------------------------
// from_run: evaluate the run's own live set X -> logL (init); else the given points
template <int D, int MODE, int LIK, int UPW>
__global__ __launch_bounds__(256) void k_eval(Launch Lc, const double *X, int ld, int n,
                                              double *out, int from_run)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bm = Lc.map[blockIdx.x];
    const DevProblem P = Lc.P[bm.x];
    const DevRun R = Lc.R[bm.x];
    unsigned long long *nonfinite = nullptr;
    if (from_run) { X = R.X; ld = R.m_pad; n = R.m; out = R.logL; nonfinite = R.ctr + 5; }
    const HLayout lay = hrss_layout(D, P.K);
    const Tile T = tile_of(smem, lay);
    const int tid = threadIdx.x;
    const int p0 = bm.y * kRows;
    for (int i = tid; i < kRows * D; i += 256) {
        const int r = i / D, a = i - r * D;
        const int p = p0 + r;
        const double x = (p < n && a < P.d) ? X[(size_t)a * ld + p] : 0.0;
        T.cand[r * (D + 1) + a] = x;
        T.cand32[r * (D + 4) + a] = (float)x;
    }
    if (tid < kRows) T.mask[tid] = (p0 + tid < n);
    stage_problem<D>(P, T);
    __syncthreads();
    WFrag<D, UPW, NPOf<MODE>::v> wr;
    if constexpr (MODE != MODE_FP64) load_wfrag<D, UPW, NPOf<MODE>::v>(P, wr);
    const Guard g = {0.0, 0.f, 0.f, 0.f};
    eval_tile<D, MODE, LIK, UPW, NPOf<MODE>::v>(P, wr, T, T.mask, g);
    if (tid < kRows && p0 + tid < n) {
        unsigned long long nf = 0;
        const double L = (MODE == MODE_FP64) ? T.L[tid] : (double)T.L32[tid];
        out[p0 + tid] = sanitize(L, nf);
        if (nf && nonfinite) atomicAdd(nonfinite, nf);
    }
}

// ------------------------------------------------------------------------------------------
// delete-k, threshold, unrolled evidence, termination (one workgroup of 1024 threads)
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long key_of(double x)
{
    if (x == 0.0) x = 0.0;  // -0 -> +0
    const unsigned long long b = __double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double val_of(unsigned long long k)
{
    const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return __longlong_as_double(b);
}

// Block reductions over 1024 threads (16 waves); red has >= 16 doubles.
__device__ __forceinline__ double block_sum(double v, double *red)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    v = wave_sum(v);
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    return s;
}
__device__ __forceinline__ double block_max(double v, double *red)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    v = wave_max(v);
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = -INFINITY;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = fmax(s, red[i]);
    return s;
}
// Exclusive prefix sum over the block.
__device__ __forceinline__ double block_exscan(double v, double *red)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    double inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double t = __shfl_up(inc, o, 64);
        if (l >= o) inc += t;
    }
    __syncthreads();
    if (l == 63) red[w] = inc;
    __syncthreads();
    double pre = 0.0;
    for (int i = 0; i < w; ++i) pre += red[i];
    return pre + inc - v;
}

// packed lower-triangular index e = a(a+1)/2 + b  ->  (a, b)
__device__ __forceinline__ void unpack_tri(int e, int &a, int &b)
{
    a = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (a * (a + 1) / 2 > e) --a;
    while ((a + 1) * (a + 2) / 2 <= e) ++a;
    b = e - a * (a + 1) / 2;
}

__device__ __forceinline__ double lse2(double a, double b)
{
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    const double mx = fmax(a, b);
    return mx + log(exp(a - mx) + exp(b - mx));
}

__global__ __launch_bounds__(1024) void k_select(Launch Lc, int op)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const DevRun R = Lc.R[Lc.map[blockIdx.x].x];
    if (R.iscal[0]) return;
    const int m = R.m, k = R.k, tid = threadIdx.x;
    int NP = 1;
    while (NP < m) NP <<= 1;
    unsigned long long *key = (unsigned long long *)smem;
    int *idx = (int *)(key + NP);
    double *red = (double *)(idx + NP + (NP & 1));
    int *st0 = (int *)(red + 32);
    for (int t = tid; t < NP; t += blockDim.x) {
        if (t < m) { key[t] = key_of(R.logL[t]); idx[t] = t; }
        else { key[t] = ~0ull; idx[t] = 0x7FFFFFFF; }
    }
    if (tid == 0) *st0 = m;
    __syncthreads();
    // bitonic sort of (key, idx) ascending
    for (int size = 2; size <= NP; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = tid; t < (NP >> 1); t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1));
                const int j = i + stride;
                const bool asc = ((i & size) == 0);
                const unsigned long long ki = key[i], kj = key[j];
                const int ii = idx[i], ij = idx[j];
                const bool gt = (ki > kj) || (ki == kj && ii > ij);
                if (gt == asc) { key[i] = kj; key[j] = ki; idx[i] = ij; idx[j] = ii; }
            }
            __syncthreads();
        }
    }
    for (int t = tid; t < m; t += blockDim.x) R.perm[t] = idx[t];
    const double Lstar = val_of(key[k - 1]);
    for (int t = k + tid; t < m; t += blockDim.x)
        if (val_of(key[t]) > Lstar) atomicMin(st0, t);
    if (op == 2) {
        __syncthreads();
        if (tid == 0) {
            R.scal[0] = Lstar;
            R.iscal[1] = *st0;
            R.iscal[2] = m - *st0;
        }
        return;
    }
    // unrolled deaths j = 1..k at live counts n_j = m - j + 1
    const double logZ0 = R.scal[1], logX0 = R.scal[2], M0 = R.scal[3];
    const int E = (k + (int)blockDim.x - 1) / (int)blockDim.x;
    const int j0 = tid * E;
    double ssum = 0.0;
    for (int e = 0; e < E; ++e) {
        const int jj = j0 + e + 1;
        if (jj <= k) ssum += 1.0 / (double)(m - jj + 1);
    }
    const double pre = block_exscan(ssum, red);
    double lwv[8], Lv[8];
    double lmax = -INFINITY, run = pre;
    for (int e = 0; e < E; ++e) {
        const int jj = j0 + e + 1;
        lwv[e] = -INFINITY; Lv[e] = 0.0;
        if (jj <= k) {
            const double inv = 1.0 / (double)(m - jj + 1);
            const double L = val_of(key[jj - 1]);
            const double lw = L + (logX0 - run) + log(-expm1(-inv));
            run += inv;
            lwv[e] = lw; Lv[e] = L;
            lmax = fmax(lmax, lw);
        }
    }
    const double S_k = block_sum(ssum, red);
    const double mx = block_max(lmax, red);
    double es = 0.0;
    for (int e = 0; e < E; ++e) if (lwv[e] != -INFINITY) es += exp(lwv[e] - mx);
    const double esum = block_sum(es, red);
    const double lse_new = (mx == -INFINITY) ? -INFINITY : mx + log(esum);
    const double logZ1 = lse2(logZ0, lse_new);
    double mt = 0.0;
    for (int e = 0; e < E; ++e) if (lwv[e] != -INFINITY) mt += exp(lwv[e] - logZ1) * Lv[e];
    const double msum = block_sum(mt, red);
    const double M1 = (logZ0 == -INFINITY ? 0.0 : exp(logZ0 - logZ1) * M0) + msum;
    const double logX1 = logX0 - S_k;
    // dead record
    const long long nd0 = (long long)R.ctr[9];
    for (int t = tid; t < k; t += blockDim.x)
        if (nd0 + t < R.dead_cap) R.dead[nd0 + t] = val_of(key[t]);
    if (R.deadx) {   // NS_FLAG_RECORD_POINTS: the dead points' coordinates, point-major [n][d]
        const int d = Lc.P[Lc.map[blockIdx.x].x].d;
        for (long long e = tid; e < (long long)k * d; e += blockDim.x) {
            const int t = (int)(e / d), a = (int)(e - (long long)t * d);
            if (nd0 + t < R.dead_cap)
                R.deadx[(nd0 + t) * d + a] = R.X[(size_t)a * R.m_pad + idx[t]];
        }
    }
    __syncthreads();
    if (tid == 0) {
        const int t0 = *st0;
        const double maxL = val_of(key[m - 1]);
        int done = (R.term_on && (logX1 + maxL - logZ1 < R.log_term)) ? 1 : 0;
        R.scal[0] = Lstar; R.scal[1] = logZ1; R.scal[2] = logX1; R.scal[3] = M1;
        R.iscal[1] = t0;
        R.iscal[2] = m - t0;
        if (!done && m - t0 <= 0) { R.iscal[4] = 1; done = 1; }
        R.iscal[0] = done;
        if (op == 1) R.iscal[3] += 1;
        R.ctr[9] = (unsigned long long)(nd0 + k);
    }
}

// ------------------------------------------------------------------------------------------
// whitening: survivors' covariance (one-pass about a fixed shift c = the best live point),
// partial sums over groups of survivors, then a single-workgroup reduction + Cholesky
// ------------------------------------------------------------------------------------------
// grid (tile, group); tile = lower 16x16 block (ta >= tb).  part2[g][tile][256], part1[g][D]
__global__ __launch_bounds__(256) void k_cov(Launch Lc)
{
    const int2 bm = Lc.map[blockIdx.x];
    const DevProblem P = Lc.P[bm.x];
    const DevRun R = Lc.R[bm.x];
    if (R.iscal[0]) return;
    // frozen whitening: the first iteration's factor, or one the caller supplied, is kept
    if (R.freeze && (R.iscal[3] > 0 || R.iscal[6])) return;
    const int d = P.d;
    const int nt = P.D / 16, ntile = nt * (nt + 1) / 2;
    const int G = R.covG;
    double *part1 = R.part1, *part2 = R.part2;
    const int tile = bm.y % ntile, g = bm.y / ntile, tid = threadIdx.x;
    int ta, tb;
    unpack_tri(tile, ta, tb);
    const int off = R.smc ? 0 : R.k;   // SMC: every particle
    const int n = R.m - off;
    const int s0 = (int)((long long)n * g / G), s1 = (int)((long long)n * (g + 1) / G);
    const int cidx = R.perm[R.m - 1];
    __shared__ double ca[32][17], cb[32][17];
    __shared__ double shift[32];
    if (tid < 16) {
        const int aa = ta * 16 + tid, bb = tb * 16 + tid;
        shift[tid] = (aa < d) ? R.X[(size_t)aa * R.m_pad + cidx] : 0.0;
        shift[16 + tid] = (bb < d) ? R.X[(size_t)bb * R.m_pad + cidx] : 0.0;
    }
    __syncthreads();
    double acc = 0.0, acc1 = 0.0;
    for (int sb = s0; sb < s1; sb += 32) {
        // stage up to 32 survivors: columns of tile a and tile b
        for (int i = tid; i < 32 * 32; i += 256) {
            const int s = i >> 5, c = i & 31;
            const int ss = sb + s;
            double v = 0.0;
            if (ss < s1) {
                const int pi = R.perm[off + ss];
                const int coord = (c < 16) ? ta * 16 + c : tb * 16 + (c - 16);
                if (coord < d) v = R.X[(size_t)coord * R.m_pad + pi] - shift[c];
            }
            if (c < 16) ca[s][c] = v; else cb[s][c - 16] = v;
        }
        __syncthreads();
        const int ns = (s1 - sb < 32) ? s1 - sb : 32;
        for (int s = 0; s < ns; ++s) acc += ca[s][tid & 15] * cb[s][tid >> 4];
        if (ta == tb && tid < 16)
            for (int s = 0; s < ns; ++s) acc1 += ca[s][tid];
        __syncthreads();
    }
    part2[((size_t)g * ntile + tile) * 256 + tid] = acc;
    if (ta == tb && tid < 16) part1[(size_t)g * P.D + ta * 16 + tid] = acc1;
}

__global__ __launch_bounds__(1024) void k_chol(Launch Lc)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bm = Lc.map[blockIdx.x];
    const DevProblem P = Lc.P[bm.x];
    const DevRun R = Lc.R[bm.x];
    if (R.iscal[0]) return;
    if (R.freeze && (R.iscal[3] > 0 || R.iscal[6])) return;
    const int G = R.covG, ntile = (P.D / 16) * (P.D / 16 + 1) / 2;
    const double *part1 = R.part1, *part2 = R.part2;
    const int D = P.D, d = P.d, tid = threadIdx.x;
    // packed lower triangle, D(D+1)/2: in LDS up to D = 128, else worked in place in the run's
    // packed factor (global memory, coherent within the workgroup across its barriers)
    double *A = D <= 128 ? (double *)smem : R.Lpk;
    double *mc = (double *)smem + (D <= 128 ? D * (D + 1) / 2 : 0);   // mean - shift, [D]
    double *red = mc + D;                    // [32]
    int *fail = (int *)(red + 32);
    const int n = R.smc ? R.m : R.m - R.k;
    for (int a = tid; a < D; a += blockDim.x) {
        double s = 0.0;
        if (a < d) for (int g = 0; g < G; ++g) s += part1[(size_t)g * D + a];
        mc[a] = s / n;
    }
    if (tid == 0) *fail = 0;
    __syncthreads();
    const int np = D * (D + 1) / 2;
    for (int e = tid; e < np; e += blockDim.x) {
        int a, b;  // a >= b
        unpack_tri(e, a, b);
        double v = 0.0;
        if (a < d && b < d && (a == b || !R.diag)) {   // the diagonal metric needs variances only
            const int ta = a >> 4, tb = b >> 4;
            const int tile = ta * (ta + 1) / 2 + tb;
            const int off = (b & 15) * 16 + (a & 15);
            double s = 0.0;
            for (int g = 0; g < G; ++g) s += part2[((size_t)g * ntile + tile) * 256 + off];
            v = s / n - mc[a] * mc[b];
        } else if (a == b) {
            v = 1.0;  // padded coordinates: identity (never used, keeps the factor regular)
        }
        A[e] = v;
    }
    __syncthreads();
    // jitter: 1e-12 * tr / d on the diagonal
    double tr = 0.0;
    for (int a = tid; a < d; a += blockDim.x) tr += A[a * (a + 1) / 2 + a];
    tr = block_sum(tr, red);
    for (int a = tid; a < d; a += blockDim.x) A[a * (a + 1) / 2 + a] += 1e-12 * tr / d;
    __syncthreads();
    // right-looking Cholesky on the packed lower triangle; for the diagonal metric it reduces
    // to the square roots of the (jittered) variances, taken directly
    if (R.diag) {
        for (int a = tid; a < d; a += blockDim.x) {
            const double v = A[a * (a + 1) / 2 + a];
            if (!(v > 0.0)) *fail = 1;
            else A[a * (a + 1) / 2 + a] = sqrt(v);
        }
        __syncthreads();
    } else
    for (int j = 0; j < d; ++j) {
        const double ajj = A[j * (j + 1) / 2 + j];
        if (!(ajj > 0.0)) { if (tid == 0) *fail = 1; break; }
        const double ljj = sqrt(ajj);
        __syncthreads();
        for (int i = j + 1 + tid; i < d; i += blockDim.x) A[i * (i + 1) / 2 + j] /= ljj;
        __syncthreads();
        if (tid == 0) A[j * (j + 1) / 2 + j] = ljj;
        const int rem = d - j - 1;
        for (int e = tid; e < rem * rem; e += blockDim.x) {
            const int ii = e / rem, r2 = e - ii * rem;
            if (r2 > ii) continue;
            const int i = j + 1 + ii, l2 = j + 1 + r2;
            A[i * (i + 1) / 2 + l2] -= A[i * (i + 1) / 2 + j] * A[l2 * (l2 + 1) / 2 + j];
        }
        __syncthreads();
    }
    __syncthreads();
    const int failed = *fail;
    if (failed) {
        // diagonal fallback: sqrt of the (jittered) variances, recomputed from the partials
        for (int e = tid; e < np; e += blockDim.x) A[e] = 0.0;
        __syncthreads();
        for (int a = tid; a < d; a += blockDim.x) {
            const int ta = a >> 4;
            const int tile = ta * (ta + 1) / 2 + ta;
            const int off = (a & 15) * 16 + (a & 15);
            double s = 0.0;
            for (int g = 0; g < G; ++g) s += part2[((size_t)g * ntile + tile) * 256 + off];
            const double v = s / n - mc[a] * mc[a];
            A[a * (a + 1) / 2 + a] = (v > 0.0) ? sqrt(v) : 1.0;
        }
        if (tid == 0) atomicAdd(&R.ctr[8], 1ull);
    }
    __syncthreads();
    for (int a = d; a < D; ++a)
        if (tid == 0) A[a * (a + 1) / 2 + a] = 0.0;  // padded coordinates never move
    for (int e = tid; e < np; e += blockDim.x) {
        int a, b;
        unpack_tri(e, a, b);
        R.Lpk[e] = (a < d && b < d) ? A[e] : 0.0;
    }
    for (int e = tid; e < D * D; e += blockDim.x) {
        const int a = e / D, b = e - a * D;
        R.Lsig[e] = (b <= a && a < d) ? A[a * (a + 1) / 2 + b] : 0.0;
    }
}

// ------------------------------------------------------------------------------------------
// directions of every chain and step of the iteration (they do not depend on the chains'
// outcomes): z ~ N(0, I_d) from Philox purpose DIR, v = L z / |z| (unit Mahalanobis length;
// random-walk runs: the proposal step v = s L z), dirbuf[(j p + s) D + a], zero for a >= d.
// 64 directions per workgroup.
// ------------------------------------------------------------------------------------------
// directions per k_dirs workgroup: 64, or 32 at D = 320 (their normals fill the LDS)
__host__ __device__ constexpr int dir_rows(int D) { return D > 128 ? 32 : 64; }
__host__ __device__ inline int dirs_lds_bytes(int D)
{
    const int rows = dir_rows(D);
    return al16(rows * (D + 1) * 8) + rows * 8 + rows * kStepU * 8 + 2 * rows * 4;
}

// The normals and uniforms are drawn by all threads; v = L z is one small FP64 MFMA product per
// workgroup: wave w takes directions 16w..16w+15 as the B operand (lane l: direction
// 16w + (l & 15), coordinate 4ks + (l >> 4)) against L as the A operand (read from the run's
// row-major factor, cached; only the normals occupy LDS), and gets
// V[16w + (l & 15)][16t + (l >> 4) + 4i] in register i of tile t; the lower-triangular L skips
// k-steps above each tile.  The results go back through the wave's own rows of the normals
// buffer so that the stores to the direction buffer are whole rows.
template <int D>
__global__ __launch_bounds__(256) void k_dirs(Launch Lc)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bm = Lc.map[blockIdx.x];
    const DevProblem P = Lc.P[bm.x];
    const DevRun R = Lc.R[bm.x];
    if (R.iscal[0] || R.iscal[2] <= 0) return;
    constexpr int LDZ = D + 1, ROWS = dir_rows(D);
    double *zs = (double *)smem;
    double *nz = zs + ROWS * LDZ;
    double *udraw = nz + ROWS;              // [ROWS][kStepU] raw uniforms
    int *rj = (int *)(udraw + ROWS * kStepU);   // chain of each row (-1 past the end)
    int *rs = rj + ROWS;                    // step of each row
    const int tid = threadIdx.x, d = P.d, p = R.p;
    const long long total = (long long)R.k * p;
    const long long base = (long long)bm.y * ROWS;
    const uint32_t it = (uint32_t)R.iscal[3] + 1u;
    if (tid < ROWS) {
        const long long idx = base + tid;
        int j = -1, st = 0;
        if (idx < total) { j = (int)(idx / p); st = (int)(idx - (long long)j * p); }
        rj[tid] = j;
        rs[tid] = st;
    }
    __syncthreads();
    const int nq = (d + 1) >> 1;
    for (int i = tid; i < ROWS * nq; i += 256) {
        const int r = i / nq, q = i - r * nq;
        const int j = rj[r];
        if (j < 0) continue;
        double ua, ub, z0, z1;
        draw2(R.key0, R.key1, PUR_DIR, (uint32_t)j, it, (uint32_t)rs[r], (uint32_t)q, ua, ub);
        box_muller(ua, ub, z0, z1);
        zs[r * LDZ + 2 * q] = z0;
        if (2 * q + 1 < d) zs[r * LDZ + 2 * q + 1] = z1;
    }
    // The step's uniforms: ubuf[0] = tL0 = -w U, ubuf[1] = the height uniform uh (purpose
    // STEP), ubuf[2 + i] = the uniform of the i-th shrink proposal (purpose SHRINK, draw i).
    for (int i = tid; i < ROWS * kStepU; i += 256) {
        const int r = i / kStepU, q = i - r * kStepU;
        const int j = rj[r], st = rs[r];
        if (j < 0) continue;
        double ua, ub;
        if (q < 2) {
            draw2(R.key0, R.key1, PUR_STEP, (uint32_t)j, it, (uint32_t)st, 0u, ua, ub);
            udraw[r * kStepU + q] = (q == 0) ? ua : ub;
        } else {
            draw2(R.key0, R.key1, PUR_SHRINK, (uint32_t)j, it, (uint32_t)st, (uint32_t)(q - 2), ua, ub);
            udraw[r * kStepU + q] = ua;
        }
    }
    __syncthreads();
    if (tid < ROWS && rj[tid] >= 0) {
        const double *u = udraw + tid * kStepU;
        double *o = R.ubuf + (base + tid) * kStepU;
        o[0] = -R.width * u[0];
        for (int q = 1; q < kStepU; ++q) o[q] = u[q];
    }
    const int w = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
    if (16 * w >= ROWS) return;   // D = 320: two waves hold the 32 directions
    const int r = 16 * w + li;
    // |z| of the wave's 16 directions: four partial sums per direction, then lane exchanges
    double s2 = 0.0;
    for (int a = lk; a < d; a += 4) {
        const double z = zs[r * LDZ + a];
        s2 += z * z;
    }
    s2 += __shfl_xor(s2, 16, 64);
    s2 += __shfl_xor(s2, 32, 64);
    const double nrm = sqrt(s2);
    constexpr int NT = D / 16, NKS = D / 4;
    d4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
        const int b = 4 * ks + lk;
        const double bz = (b < d) ? zs[r * LDZ + b] : 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (ks < 4 * t + 4) {   // L is zero above its diagonal
                const double la = R.Lsig[(16 * t + li) * D + b];
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(la, bz, acc[t], 0, 0, 0);
            }
        }
    }
    // HRSS: unit Mahalanobis length; random walk: the proposal step s L z
    wave_sync();   // this wave's reads of its rows are done
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int a = 16 * t + lk + 4 * i;
            zs[r * LDZ + a] = (a < d) ? (R.rw ? acc[t][i] * R.width : acc[t][i] / nrm) : 0.0;
        }
    }
    wave_sync();
    for (int e = l; e < 16 * D; e += 64) {
        const int rr = e / D, a = e - rr * D;
        const int row = 16 * w + rr;
        if (rj[row] >= 0) R.dirbuf[(base + row) * D + a] = zs[row * LDZ + a];
    }
}

// ------------------------------------------------------------------------------------------
// the k HRSS chains
// ------------------------------------------------------------------------------------------
enum Phase { PH_NEWSTEP = 0, PH_STEPOUT = 1, PH_SHRINK = 2, PH_DONE = 3 };

// One workgroup = four waves = up to four chains (chain c <-> wave c).  Each wave runs its
// chain's finite-state machine with wave-uniform state; lane l owns coordinates l and l + 64 of
// the chain's point and direction in registers.  A round: every active chain emits up to two
// candidates (the two bracket ends while stepping out, one proposal while shrinking), the four
// waves evaluate the 16-row tile together, each chain consumes its results.  Mixed precision:
// a candidate whose FP32 estimate lies within the guard band of L* is re-evaluated in FP64
// before the decision, so decisions equal the FP64 ones; the stored logL is FP64.
template <int D, int MODE, int LIK, int UPW>
__global__ __launch_bounds__(256) void k_hrss(Launch Lc)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bm = Lc.map[blockIdx.x];
    const DevProblem P = Lc.P[bm.x];
    const DevRun R = Lc.R[bm.x];
    const int C = R.C;
    if (R.iscal[0]) return;
    if (R.iscal[2] <= 0) return;
    constexpr int LDC = D + 1, LDC32 = D + 4;
    constexpr int NA = (D + 63) / 64;        // coordinates per lane
    constexpr int NP = NPOf<MODE>::v;
    const HLayout lay = hrss_layout(D, P.K);
    const Tile T = tile_of(smem, lay);
    double *sz = (double *)(smem + lay.z);
    double *sLs = (double *)(smem + lay.lsig);
    double *scand = T.cand;
    float *scand32 = T.cand32;
    int *smask = T.mask;
    int *src = T.rc;

    const int tid = threadIdx.x, w = uniform_i(tid >> 6), l = tid & 63;
    const int d = P.d;
    const double Lstar = R.scal[0];
    // adaptive tempered SMC (FP64 only): no hard constraint; scal[0] holds the inverse
    // temperature
    const bool tempered = MODE == MODE_FP64 && R.smc != 0;
    const double beta = Lstar;
    const int t0 = R.iscal[1], nsurv = R.iscal[2];
    const uint32_t it = (uint32_t)R.iscal[3] + 1u;
    const double width = R.width;
    const int p = R.p, cap_out = R.stepout_cap, cap_sh = R.shrink_cap;
    const bool box = (P.prior_kind == PRIOR_BOX);
    const bool pre = D > 128 || R.dirbuf != nullptr;   // D = 320 always reads the buffer

    if (!pre) {
        if constexpr (D <= 64) {
            for (int i = tid; i < D * D; i += 256) {
                const int a = i / D, b = i - a * D;
                sLs[a * (D + 1) + b] = R.Lsig[i];
            }
        } else {
            for (int i = tid; i < D * (D + 1) / 2; i += 256) sLs[i] = R.Lpk[i];
        }
    }
    stage_problem<D>(P, T);
    if (tid < kRows) { smask[tid] = 0; src[tid] = 0; }
    for (int i = tid; i < kRows * LDC; i += 256) scand[i] = 0.0;
    for (int i = tid; i < kRows * LDC32; i += 256) scand32[i] = 0.f;
    WFrag<D, UPW, NP> wr;
    if constexpr (MODE != MODE_FP64) load_wfrag<D, UPW, NP>(P, wr);
#ifdef NSS_PHASE_TIMING
    unsigned long long pt[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long tmark = __builtin_amdgcn_s_memtime();
#define PT(slot)                                                                             \
    do {                                                                                     \
        const unsigned long long t_ = __builtin_amdgcn_s_memtime();                          \
        pt[slot] += t_ - tmark;                                                              \
        tmark = t_;                                                                          \
    } while (0)
#else
#define PT(slot) do {} while (0)
#endif

    const int j = bm.y * C + w;
    const bool has_chain = (w < C) && (j < R.k);
    double *zz = sz + w * D;

    // lane-owned coordinates a = l + 64 i of the point, direction and prior parameters
    double x0r[NA], vr[NA], par[NA], pbr[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int a = l + 64 * i;
        x0r[i] = 0.0; vr[i] = 0.0;
        par[i] = (a < D) ? P.pa[a] : 0.0;
        pbr[i] = (a < D) ? P.pb[a] : 1.0;
    }

    // per-chain state (wave-uniform, replicated in every lane of the chain's wave)
    int phase = PH_DONE, step = 0, nl = 0, nr = 0, ns = 0;
    bool la = false, ra = false;
    double tL = 0.0, tR = 0.0, logy = -INFINITY, logL0 = -INFINITY;
    unsigned long long c_evals = 0, c_tests = 0, c_prej = 0, c_outcap = 0, c_shcap = 0,
                       c_nonfin = 0, c_rc = 0, c_viol = 0;

    if (has_chain) {
        int parent = j;   // tempered SMC: the resampled particle j, gathered into slot j
        if (!tempered) {
            double u, unused;
            draw2(R.key0, R.key1, PUR_RESAMPLE, (uint32_t)j, it, 0u, 0u, u, unused);
            int qi = (int)floor(u * (double)nsurv);
            if (qi > nsurv - 1) qi = nsurv - 1;
            parent = R.perm[t0 + qi];
            if (l == 0) R.parents[j] = parent;
        }
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int a = l + 64 * i;
            if (a < d) x0r[i] = R.X[(size_t)a * R.m_pad + parent];
        }
        if (!pre)
            for (int a = l; a < D; a += 64) zz[a] = 0.0;
        logL0 = R.logL[parent];
        phase = (p > 0) ? PH_NEWSTEP : PH_DONE;
    }
    __syncthreads();

    // next step's direction and uniforms, prefetched into registers one step ahead (the
    // uniforms sit in lanes 0..7: U, uh, then shrink uniforms 0..5)
    double pv[NA], pu[kStepU], cu[kStepU];
#pragma unroll
    for (int i = 0; i < NA; ++i) pv[i] = 0.0;
#pragma unroll
    for (int q = 0; q < kStepU; ++q) { pu[q] = 0.0; cu[q] = 0.0; }
    auto prefetch_dir = [&](int st) {
        if (has_chain && st < p) {
            const double *srcv = R.dirbuf + ((size_t)j * p + st) * D;
#pragma unroll
            for (int i = 0; i < NA; ++i) if (l + 64 * i < D) pv[i] = srcv[l + 64 * i];
            const double *su = R.ubuf + ((size_t)j * p + st) * kStepU;
#pragma unroll
            for (int q = 0; q < kStepU; ++q) pu[q] = su[q];
        }
    };
    if (pre) prefetch_dir(0);
    // shrink uniform number sn of the current step
    auto shrink_u = [&](int sn) -> double {
        double us, unused;
        draw2(R.key0, R.key1, PUR_SHRINK, (uint32_t)j, it, (uint32_t)step, (uint32_t)sn, us, unused);
        return us;
    };

    // log prior density at the lane-owned point (Gaussian prior only)
    auto logprior_x0 = [&]() -> double {
        double lp = 0.0;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int a = l + 64 * i;
            if (a < d) { const double zt = (x0r[i] - par[i]) / pbr[i]; lp += -0.5 * zt * zt; }
        }
        return wave_sum_fast(lp) + P.logprior_norm;
    };

    auto finish_step = [&](int acc, int nsh) {
        if (R.trace && l == 0) {
            int *tr = R.trace + ((size_t)j * p + step) * 4;
            tr[0] = nl; tr[1] = nr; tr[2] = nsh; tr[3] = acc;
        }
        if (!acc) ++c_shcap;
        ++step;
        phase = (step >= p) ? PH_DONE : PH_NEWSTEP;
    };

    auto enter_shrink = [&]() {
        phase = PH_SHRINK;
        ns = 0;
        if (cap_sh <= 0) finish_step(0, 0);
    };

    const Guard guard = {Lstar, P.guard_rel, P.guard_abs, P.cmax32};

    // A round's plan: up to kSlots tests in the order the sequential algorithm would make them
    // if every stepping-out test fell outside and every shrink proposal were rejected.  Each
    // proposal after a rejection is fully determined (the bracket end that moves depends only
    // on the sign of t'), so the plan is exact up to its first surprise; the rest is discarded
    // and neither counted nor used.
    enum { S_NONE = 0, S_LEFT = 1, S_RIGHT = 2, S_SHRINK = 3 };
    for (;;) {
        const bool act = has_chain && phase != PH_DONE;
        int kind[kSlots], ok[kSlots];
        double tv[kSlots], bLa[kSlots], bRa[kSlots];   // t per slot; bracket after rejecting it
        double lps[kSlots];                             // log prior density (Gaussian prior)
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl) {
            kind[sl] = S_NONE; ok[sl] = 0; tv[sl] = 0.0; bLa[sl] = 0.0; bRa[sl] = 0.0;
            lps[sl] = 0.0;
        }
        if (act) {
            PT(6);
            if (phase == PH_NEWSTEP) {
                if (pre) {
#pragma unroll
                    for (int i = 0; i < NA; ++i) vr[i] = pv[i];
#pragma unroll
                    for (int q = 0; q < kStepU; ++q) cu[q] = pu[q];
                    prefetch_dir(step + 1);
                } else {
                    // direction z ~ N(0, I_d), v = L z / |z|, drawn by the chain itself
                    const int nq = (d + 1) >> 1;
                    for (int q = l; q < nq; q += 64) {
                        double ua, ub, z0, z1;
                        draw2(R.key0, R.key1, PUR_DIR, (uint32_t)j, it, (uint32_t)step,
                              (uint32_t)q, ua, ub);
                        box_muller(ua, ub, z0, z1);
                        zz[2 * q] = z0;
                        if (2 * q + 1 < d) zz[2 * q + 1] = z1;
                    }
                    wave_sync();
                    double s2 = 0.0;
                    for (int a = l; a < d; a += 64) s2 += zz[a] * zz[a];
                    const double nz = sqrt(wave_sum_fast(s2));
#pragma unroll
                    for (int i = 0; i < NA; ++i) {
                        const int a = l + 64 * i;
                        double v = 0.0;
                        if (a < d) {
                            const double *Lr = (D <= 64) ? sLs + a * (D + 1) : sLs + a * (a + 1) / 2;
                            double s0 = 0.0;
                            for (int b = 0; b <= a; ++b) s0 += Lr[b] * zz[b];
                            v = s0 / nz;
                        }
                        vr[i] = v;
                    }
                }
                double uh;
                if (pre) {
                    tL = cu[0];
                    uh = cu[1];
                } else {
                    double U;
                    draw2(R.key0, R.key1, PUR_STEP, (uint32_t)j, it, (uint32_t)step, 0u, U, uh);
                    tL = -width * U;
                }
                if (tempered)   // slice of Pi L^beta: log Pi(x0) + beta log L(x0) - Exp(1)
                    logy = (box ? 0.0 : logprior_x0()) + beta * logL0 + log(uh);
                else
                    logy = box ? -INFINITY : logprior_x0() + log(uh);
                tR = tL + width;
                nl = nr = 0;
                la = ra = (cap_out > 0);
                if (cap_out <= 0) c_outcap += 2;
                phase = PH_STEPOUT;
                if (!la && !ra) enter_shrink();
#ifdef NSS_PHASE_TIMING
                pt[9] += 1;
#endif
                PT(0);
            }
            // the plan
            int ns_plan = 0;
            double sL = tL, sR = tR;
            int sn = ns;
            if (phase == PH_STEPOUT) {
                if (la) { kind[ns_plan] = S_LEFT; tv[ns_plan] = tL; ++ns_plan; }
                if (ra) { kind[ns_plan] = S_RIGHT; tv[ns_plan] = tR; ++ns_plan; }
                sn = 0;
            }
            if (phase == PH_STEPOUT || phase == PH_SHRINK) {
#pragma unroll
                for (int sl = 0; sl < kSlots; ++sl) {
                    if (sl >= ns_plan && sn < cap_sh) {
                        double us;
                        if (pre && sn < kStepShrinkU) {
                            us = cu[2];
#pragma unroll
                            for (int q = 1; q < kStepShrinkU; ++q) if (sn == q) us = cu[2 + q];
                        } else {
                            us = shrink_u(sn);
                        }
                        const double t = sL + us * (sR - sL);
                        kind[sl] = S_SHRINK;
                        tv[sl] = t;
                        ++sn;
                        if (t < 0.0) sL = t; else sR = t;
                    }
                    bLa[sl] = sL;
                    bRa[sl] = sR;
                }
            }
            PT(4);
            {
                // all planned candidates in one pass over the lane's coordinates
                bool inb[kSlots];
                double lp[kSlots];
#pragma unroll
                for (int sl = 0; sl < kSlots; ++sl) { inb[sl] = true; lp[sl] = 0.0; }
#pragma unroll
                for (int i = 0; i < NA; ++i) {
                    const int a = l + 64 * i;
                    if (a < D) {
#pragma unroll
                        for (int sl = 0; sl < kSlots; ++sl) {
                            if (kind[sl] == S_NONE) continue;
                            const int r = w * kSlots + sl;
                            const double y = x0r[i] + tv[sl] * vr[i];
                            scand[r * LDC + a] = y;
                            if constexpr (MODE != MODE_FP64) scand32[r * LDC32 + a] = (float)y;
                            if (a < d) {
                                if (box) inb[sl] = inb[sl] && (y >= par[i] && y <= pbr[i]);
                                else { const double zt = (y - par[i]) / pbr[i]; lp[sl] += -0.5 * zt * zt; }
                            }
                        }
                    }
                }
                PT(1);
#pragma unroll
                for (int sl = 0; sl < kSlots; ++sl) {
                    if (kind[sl] == S_NONE) continue;
                    if (box) {
                        ok[sl] = __all(inb[sl]) != 0;
                    } else {
                        lps[sl] = wave_sum_fast(lp[sl]) + P.logprior_norm;
                        ok[sl] = tempered || lps[sl] > logy;   // tempered: no prior gate
                    }
                }
            }
            PT(11);
        }
        if (l == 0) {
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl) smask[w * kSlots + sl] = (kind[sl] != S_NONE) && ok[sl];
        }
        if (!__syncthreads_or(act)) break;
        PT(2);
#ifdef NSS_PHASE_TIMING
        pt[8] += 1;
#endif

        // ---- batched likelihood of the tile (+ FP64 re-check of near-threshold rows) ----
        const int any_rc = eval_tile<D, MODE, LIK, UPW, NP>(P, wr, T, smask, guard);
        PT(3);
        if constexpr (MODE != MODE_FP64) {
            if (any_rc) {
                eval64<D, LIK>(P, T, T.rc, T.L);
#ifdef NSS_PHASE_TIMING
                pt[10] += 1;
#endif
                PT(5);
            }
        }

        // ---- walk the plan ----
        if (act) {
            // every slot's outcome at once (FP64 where re-checked), as bit masks
            unsigned okm = 0, inm = 0, rcm = 0, nfm = 0, shm = 0;
            double Lv[kSlots];
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl) {
                Lv[sl] = -INFINITY;
                if (kind[sl] == S_SHRINK) shm |= 1u << sl;
                if (kind[sl] != S_NONE && ok[sl]) {
                    const int r = w * kSlots + sl;
                    int rc = 0;
                    double L;
                    if constexpr (MODE == MODE_FP64) L = T.L[r];
                    else { rc = T.rc[r]; L = rc ? T.L[r] : (double)T.L32[r]; }
                    const bool nf = (L != L) || L == INFINITY;
                    if (nf) L = -INFINITY;
                    Lv[sl] = L;
                    okm |= 1u << sl;
                    if (tempered ? (lps[sl] + beta * L > logy) : (L > Lstar)) inm |= 1u << sl;
                    if (rc) rcm |= 1u << sl;
                    if (nf) nfm |= 1u << sl;
                }
            }
            auto tally = [&](unsigned cons) {
                c_tests += __builtin_popcount(cons);
                c_evals += __builtin_popcount(cons & okm);
                c_prej += __builtin_popcount(cons & ~okm);
                c_rc += __builtin_popcount(cons & rcm);
                c_nonfin += __builtin_popcount(cons & nfm);
            };
            bool moved = false;   // a bracket end moved during stepping-out this round
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                if (kind[sl] == S_LEFT || kind[sl] == S_RIGHT) {
                    tally(1u << sl);
                    const bool in = (inm >> sl) & 1u;
                    if (kind[sl] == S_LEFT) {
                        if (in) { tL -= width; ++nl; moved = true; if (nl >= cap_out) { la = false; ++c_outcap; } }
                        else la = false;
                    } else {
                        if (in) { tR += width; ++nr; moved = true; if (nr >= cap_out) { ra = false; ++c_outcap; } }
                        else ra = false;
                    }
                }
            }
            if (phase == PH_STEPOUT && !la && !ra) enter_shrink();
            if (phase == PH_SHRINK && !moved && shm) {
                const int s0 = __builtin_ctz(shm);
                const unsigned acc = inm & shm;
                const int last = acc ? __builtin_ctz(acc) : 31 - __builtin_clz(shm);
                const unsigned cons = shm & ((2u << last) - 1u);
                tally(cons);
                const int nrej = __builtin_popcount(cons) - (acc ? 1 : 0);
                // bracket after the last rejected slot (slots are contiguous from s0)
                if (nrej > 0) {
                    const int lr = s0 + nrej - 1;
                    double bl = bLa[0], br = bRa[0];
#pragma unroll
                    for (int sl = 1; sl < kSlots; ++sl) if (sl == lr) { bl = bLa[sl]; br = bRa[sl]; }
                    tL = bl; tR = br;
                }
                ns += nrej;
                if (acc) {
                    // the accepted point is the evaluated candidate row, bit for bit
                    const int r = w * kSlots + last;
#pragma unroll
                    for (int i = 0; i < NA; ++i)
                        if (l + 64 * i < D) x0r[i] = scand[r * LDC + l + 64 * i];
                    double La = Lv[0];
#pragma unroll
                    for (int sl = 1; sl < kSlots; ++sl) if (sl == last) La = Lv[sl];
                    logL0 = La;
                    finish_step(1, ns + 1);
                } else if (ns >= cap_sh) {
                    finish_step(0, ns);
                }
            }
            PT(7);
        }
    }
#ifdef NSS_PHASE_TIMING
    if (tid == 0 && R.prof) for (int i = 0; i < 12; ++i) atomicAdd(&R.prof[i], pt[i]);
#endif
#undef PT

    if constexpr (MODE != MODE_FP64) {
        // stored log-likelihoods are FP64: re-evaluate each chain's final point
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NA; ++i)
            if (l + 64 * i < D) scand[w * LDC + l + 64 * i] = has_chain ? x0r[i] : 0.0;
        if (tid < kRows) smask[tid] = (tid < kMaxChainsPerWG) && (tid < C) &&
                                      (bm.y * C + tid < R.k);
        __syncthreads();
        eval64<D, LIK>(P, T, smask, T.L);
        if (has_chain) {
            unsigned long long dummy = 0;
            logL0 = sanitize(T.L[w], dummy);
            if (!(logL0 > Lstar)) ++c_viol;
        }
    }

    if (has_chain) {
        const int slot = tempered ? j : R.perm[j];
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int a = l + 64 * i;
            if (a < d) R.X[(size_t)a * R.m_pad + slot] = x0r[i];
        }
        if (l == 0) {
            R.logL[slot] = logL0;
            atomicAdd(&R.ctr[0], c_evals);
            atomicAdd(&R.ctr[1], c_tests);
            atomicAdd(&R.ctr[2], c_prej);
            atomicAdd(&R.ctr[3], c_outcap);
            atomicAdd(&R.ctr[4], c_shcap);
            atomicAdd(&R.ctr[5], c_nonfin);
            atomicAdd(&R.ctr[6], c_rc);
            atomicAdd(&R.ctr[7], c_viol);
        }
    }
}

// ------------------------------------------------------------------------------------------
// the k chains of the random-walk replacement
// ------------------------------------------------------------------------------------------
// Constrained Gaussian random-walk Metropolis: step st of chain j proposes x + u_{j,st} with
// u = s L z from the direction buffer; the proposal is accepted if it is in the prior support,
// passes the prior-ratio test (Gaussian prior: log Pi(x') > log Pi(x) + log uh, uh from the step
// plan) and has logL > L*.  Same grid, tile and evaluators as k_hrss: chain c <-> wave c.  While
// proposals are rejected the chain stays, so the proposals of steps st, st+1, ... all start
// from the current point and a round plans up to four of them; the plan is exact up to its
// first acceptance, the rest is discarded uncounted.  Mixed precision re-checks near-threshold
// rows in FP64 exactly as the HRSS kernel does.
template <int D, int MODE, int LIK, int UPW>
__global__ __launch_bounds__(256) void k_rw(Launch Lc)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bm = Lc.map[blockIdx.x];
    const DevProblem P = Lc.P[bm.x];
    const DevRun R = Lc.R[bm.x];
    const int C = R.C;
    if (R.iscal[0]) return;
    if (R.iscal[2] <= 0) return;
    constexpr int LDC = D + 1, LDC32 = D + 4;
    constexpr int NA = (D + 63) / 64;
    constexpr int NP = NPOf<MODE>::v;
    const HLayout lay = hrss_layout(D, P.K);
    const Tile T = tile_of(smem, lay);
    double *scand = T.cand;
    float *scand32 = T.cand32;
    int *smask = T.mask;

    const int tid = threadIdx.x, w = uniform_i(tid >> 6), l = tid & 63;
    const int d = P.d;
    const double Lstar = R.scal[0];
    const int t0 = R.iscal[1], nsurv = R.iscal[2];
    const uint32_t it = (uint32_t)R.iscal[3] + 1u;
    const int p = R.p;
    const bool box = (P.prior_kind == PRIOR_BOX);

    stage_problem<D>(P, T);
    if (tid < kRows) { smask[tid] = 0; T.rc[tid] = 0; }
    for (int i = tid; i < kRows * LDC; i += 256) scand[i] = 0.0;
    for (int i = tid; i < kRows * LDC32; i += 256) scand32[i] = 0.f;
    WFrag<D, UPW, NP> wr;
    if constexpr (MODE != MODE_FP64) load_wfrag<D, UPW, NP>(P, wr);

    const int j = bm.y * C + w;
    const bool has_chain = (w < C) && (j < R.k);
    double x0r[NA], par[NA], pbr[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int a = l + 64 * i;
        x0r[i] = 0.0;
        par[i] = (a < D) ? P.pa[a] : 0.0;
        pbr[i] = (a < D) ? P.pb[a] : 1.0;
    }
    int step = 0;
    double logL0 = -INFINITY, lp0 = 0.0;   // lp0: log prior density of the current point
    unsigned long long c_evals = 0, c_tests = 0, c_prej = 0, c_nonfin = 0, c_rc = 0, c_viol = 0;
    if (has_chain) {
        double u, unused;
        draw2(R.key0, R.key1, PUR_RESAMPLE, (uint32_t)j, it, 0u, 0u, u, unused);
        int qi = (int)floor(u * (double)nsurv);
        if (qi > nsurv - 1) qi = nsurv - 1;
        const int parent = R.perm[t0 + qi];
        if (l == 0) R.parents[j] = parent;
        double lp = 0.0;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int a = l + 64 * i;
            if (a < d) {
                x0r[i] = R.X[(size_t)a * R.m_pad + parent];
                const double zt = (x0r[i] - par[i]) / pbr[i];
                lp += -0.5 * zt * zt;
            }
        }
        if (!box) lp0 = wave_sum_fast(lp) + P.logprior_norm;
        logL0 = R.logL[parent];
    }
    __syncthreads();
    const Guard guard = {Lstar, P.guard_rel, P.guard_abs, P.cmax32};

    for (;;) {
        const bool act = has_chain && step < p;
        const int np = act ? min(kSlots, p - step) : 0;   // proposals planned this round
        int ok[kSlots];
        double lpv[kSlots];
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl) { ok[sl] = 0; lpv[sl] = 0.0; }
        if (act) {
            bool inb[kSlots];
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl) inb[sl] = true;
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int a = l + 64 * i;
                if (a < D) {
#pragma unroll
                    for (int sl = 0; sl < kSlots; ++sl) {
                        if (sl >= np) continue;
                        const int r = w * kSlots + sl;
                        const double y = x0r[i] + R.dirbuf[((size_t)j * p + step + sl) * D + a];
                        scand[r * LDC + a] = y;
                        if constexpr (MODE != MODE_FP64) scand32[r * LDC32 + a] = (float)y;
                        if (a < d) {
                            if (box) inb[sl] = inb[sl] && (y >= par[i] && y <= pbr[i]);
                            else { const double zt = (y - par[i]) / pbr[i]; lpv[sl] += -0.5 * zt * zt; }
                        }
                    }
                }
            }
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl) {
                if (sl >= np) continue;
                if (box) {
                    ok[sl] = __all(inb[sl]) != 0;
                } else {
                    const double uh = R.ubuf[((size_t)j * p + step + sl) * kStepU + 1];
                    lpv[sl] = wave_sum_fast(lpv[sl]) + P.logprior_norm;
                    ok[sl] = lpv[sl] > lp0 + log(uh);
                }
            }
        }
        if (l == 0) {
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl) smask[w * kSlots + sl] = (sl < np) && ok[sl];
        }
        if (!__syncthreads_or(act)) break;

        const int any_rc = eval_tile<D, MODE, LIK, UPW, NP>(P, wr, T, smask, guard);
        if constexpr (MODE != MODE_FP64) {
            if (any_rc) eval64<D, LIK>(P, T, T.rc, T.L);
        }

        if (act) {
            unsigned okm = 0, inm = 0, rcm = 0, nfm = 0;
            const unsigned planned = (1u << np) - 1u;
            double Lv[kSlots];
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl) {
                Lv[sl] = -INFINITY;
                if (sl < np && ok[sl]) {
                    const int r = w * kSlots + sl;
                    int rc = 0;
                    double L;
                    if constexpr (MODE == MODE_FP64) L = T.L[r];
                    else { rc = T.rc[r]; L = rc ? T.L[r] : (double)T.L32[r]; }
                    const bool nf = (L != L) || L == INFINITY;
                    if (nf) L = -INFINITY;
                    Lv[sl] = L;
                    okm |= 1u << sl;
                    if (L > Lstar) inm |= 1u << sl;
                    if (rc) rcm |= 1u << sl;
                    if (nf) nfm |= 1u << sl;
                }
            }
            const unsigned acc = inm & planned;
            const int last = acc ? __builtin_ctz(acc) : np - 1;
            const unsigned cons = planned & ((2u << last) - 1u);
            c_tests += __builtin_popcount(cons);
            c_evals += __builtin_popcount(cons & okm);
            c_prej += __builtin_popcount(cons & ~okm);
            c_rc += __builtin_popcount(cons & rcm);
            c_nonfin += __builtin_popcount(cons & nfm);
            if (R.trace && l == 0) {
#pragma unroll
                for (int sl = 0; sl < kSlots; ++sl) {
                    if (!((cons >> sl) & 1u)) continue;
                    int *tr = R.trace + ((size_t)j * p + step + sl) * 4;
                    tr[0] = 0; tr[1] = 0; tr[2] = (okm >> sl) & 1u; tr[3] = (acc && sl == last) ? 1 : 0;
                }
            }
            if (acc) {
                // the accepted point is the evaluated candidate row, bit for bit
                const int r = w * kSlots + last;
#pragma unroll
                for (int i = 0; i < NA; ++i)
                    if (l + 64 * i < D) x0r[i] = scand[r * LDC + l + 64 * i];
                double La = Lv[0], lpa = lpv[0];
#pragma unroll
                for (int sl = 1; sl < kSlots; ++sl)
                    if (sl == last) { La = Lv[sl]; lpa = lpv[sl]; }
                logL0 = La;
                lp0 = lpa;
            }
            step += last + 1;
        }
    }

    if constexpr (MODE != MODE_FP64) {
        // stored log-likelihoods are FP64: re-evaluate each chain's final point
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NA; ++i)
            if (l + 64 * i < D) scand[w * LDC + l + 64 * i] = has_chain ? x0r[i] : 0.0;
        if (tid < kRows) smask[tid] = (tid < kMaxChainsPerWG) && (tid < C) &&
                                      (bm.y * C + tid < R.k);
        __syncthreads();
        eval64<D, LIK>(P, T, smask, T.L);
        if (has_chain) {
            unsigned long long dummy = 0;
            logL0 = sanitize(T.L[w], dummy);
            if (!(logL0 > Lstar)) ++c_viol;
        }
    }

    if (has_chain) {
        const int slot = R.perm[j];
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int a = l + 64 * i;
            if (a < d) R.X[(size_t)a * R.m_pad + slot] = x0r[i];
        }
        if (l == 0) {
            R.logL[slot] = logL0;
            atomicAdd(&R.ctr[0], c_evals);
            atomicAdd(&R.ctr[1], c_tests);
            atomicAdd(&R.ctr[2], c_prej);
            atomicAdd(&R.ctr[5], c_nonfin);
            atomicAdd(&R.ctr[6], c_rc);
            atomicAdd(&R.ctr[7], c_viol);
        }
    }
}

// ------------------------------------------------------------------------------------------
// adaptive tempered SMC (the slice-sampling mutation runs in k_hrss with R.smc set)
// ------------------------------------------------------------------------------------------
// One workgroup per run.  op 0: start at beta = 0 (identity order, log Z = 0).  op 1 (the
// start of a step): the next inverse temperature by 50 bisection steps on the ESS of the
// incremental weights exp((b - beta) (logL - max logL)) (target rho m, or beta = 1), the log
// mean incremental weight added to log Z, systematic resampling with one uniform (purpose
// RESAMPLE, counter (0, step)) against the cumulative normalised weights, and the gather of
// the resampled particles into slots 0..m-1.  op 2 (the end of a step): the step count, and
// done once beta = 1.  scal[0] = beta, scal[1] = log Z; iscal[5] = this step reached beta = 1.
// The step's draws (resampling, directions, chains) use iteration number iscal[3] + 1.
constexpr int kSmcPer = kMaxLive / kSelectThreads;   // particles per thread, contiguous

__global__ __launch_bounds__(kSelectThreads) void k_smc(Launch Lc, int op)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[32];
    const int2 bm = Lc.map[blockIdx.x];
    const DevProblem P = Lc.P[bm.x];
    const DevRun R = Lc.R[bm.x];
    const int m = R.m, tid = threadIdx.x;
    if (op == 0) {
        for (int i = tid; i < m; i += blockDim.x) R.perm[i] = i;
        if (tid == 0) {
            R.scal[0] = 0.0; R.scal[1] = 0.0; R.scal[2] = 0.0; R.scal[3] = 0.0;
            R.iscal[1] = 0; R.iscal[2] = m; R.iscal[5] = 0;
        }
        return;
    }
    if (op == 2) {   // the step's draws used iteration number iscal[3] + 1
        if (tid == 0 && !R.iscal[0]) {
            R.iscal[3] += 1;
            if (R.iscal[5]) R.iscal[0] = 1;
        }
        return;
    }
    if (R.iscal[0]) return;
    double *cum = (double *)smem;                         // [m]
    int *par = (int *)(smem + (size_t)kMaxLive * 8);      // [m]
    const double beta = R.scal[0];
    const int i0 = tid * kSmcPer;
    double Lr[kSmcPer];
    double lmax = -INFINITY;
#pragma unroll
    for (int q = 0; q < kSmcPer; ++q) {
        Lr[q] = (i0 + q < m) ? R.logL[i0 + q] : -INFINITY;
        lmax = fmax(lmax, Lr[q]);
    }
    lmax = block_max(lmax, red);
    if (!(lmax > -INFINITY)) {   // every particle has log L = -inf: nothing to weigh
        if (tid == 0) { R.iscal[4] = 1; R.iscal[0] = 1; }
        return;
    }
    auto ess = [&](double b) -> double {
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int q = 0; q < kSmcPer; ++q) {
            if (Lr[q] > -INFINITY) {
                const double e = exp((b - beta) * (Lr[q] - lmax));
                s1 += e;
                s2 += e * e;
            }
        }
        s1 = block_sum(s1, red);
        s2 = block_sum(s2, red);
        return s1 * s1 / s2;
    };
    const double target = R.ess_frac * m;
    double nb = 1.0;
    if (ess(1.0) < target) {
        double lo = beta, hi = 1.0;
        for (int t = 0; t < 50; ++t) {
            const double mid = 0.5 * (lo + hi);
            if (ess(mid) >= target) lo = mid; else hi = mid;
        }
        nb = lo > beta ? lo : hi;
    }
    const double db = nb - beta;
    double w[kSmcPer], loc = 0.0;
#pragma unroll
    for (int q = 0; q < kSmcPer; ++q) {
        w[q] = (Lr[q] > -INFINITY) ? exp(db * (Lr[q] - lmax)) : 0.0;
        loc += w[q];
    }
    const double pre = block_exscan(loc, red);
    const double sw = block_sum(loc, red);
    double c = pre;
#pragma unroll
    for (int q = 0; q < kSmcPer; ++q) {
        c += w[q];
        if (i0 + q < m) cum[i0 + q] = c / sw;
    }
    const uint32_t it = (uint32_t)R.iscal[3] + 1u;
    double u, unused;
    draw2(R.key0, R.key1, PUR_RESAMPLE, 0u, it, 0u, 0u, u, unused);
    __syncthreads();
    // parent of slot j: the first particle whose cumulative weight reaches (u + j) / m
    for (int j = tid; j < m; j += blockDim.x) {
        const double pos = (u + j) / m;
        int lo = 0, hi = m - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cum[mid] >= pos) hi = mid; else lo = mid + 1;
        }
        par[j] = lo;
        R.parents[j] = lo;
    }
    __syncthreads();
    // gather through the scratch copy, then back into the live arrays
    const int d = P.d;
    for (long long e = tid; e < (long long)d * m; e += blockDim.x) {
        const int a = (int)(e / m), j = (int)(e - (long long)a * m);
        R.Xtmp[(size_t)a * R.m_pad + j] = R.X[(size_t)a * R.m_pad + par[j]];
    }
    for (int j = tid; j < m; j += blockDim.x) R.Ltmp[j] = R.logL[par[j]];
    __syncthreads();
    for (long long e = tid; e < (long long)d * m; e += blockDim.x) {
        const int a = (int)(e / m), j = (int)(e - (long long)a * m);
        R.X[(size_t)a * R.m_pad + j] = R.Xtmp[(size_t)a * R.m_pad + j];
    }
    for (int j = tid; j < m; j += blockDim.x) R.logL[j] = R.Ltmp[j];
    if (tid == 0) {
        R.scal[0] = nb;
        R.scal[1] += db * lmax + log(sw) - log((double)m);
        R.iscal[1] = 0;
        R.iscal[2] = m;
        R.iscal[5] = (nb == 1.0) ? 1 : 0;
    }
}

// ------------------------------------------------------------------------------------------
// final live-set contribution (non-destructive): scal[4..6] = ln Z, sqrt(H/m), H
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_logz(Launch Lc)
{
    const DevRun R = Lc.R[Lc.map[blockIdx.x].x];
    __shared__ double red[32];
    const int m = R.m, k = R.k, n = m - k, tid = threadIdx.x;
    double mx = -INFINITY;
    for (int t = k + tid; t < m; t += blockDim.x) mx = fmax(mx, R.logL[R.perm[t]]);
    mx = block_max(mx, red);
    double s = 0.0;
    for (int t = k + tid; t < m; t += blockDim.x) s += exp(R.logL[R.perm[t]] - mx);
    s = block_sum(s, red);
    const double logZ = R.scal[1], logX = R.scal[2], M = R.scal[3];
    const double lme = mx + log(s) - log((double)n);
    const double zf = lse2(logZ, logX + lme);
    double mt = 0.0;
    for (int t = k + tid; t < m; t += blockDim.x) {
        const double L = R.logL[R.perm[t]];
        const double lw = logX - log((double)n) + L;
        if (lw != -INFINITY) mt += exp(lw - zf) * L;
    }
    mt = block_sum(mt, red);
    if (tid == 0) {
        const double Mf = (logZ == -INFINITY ? 0.0 : exp(logZ - zf) * M) + mt;
        const double H = Mf - zf;
        R.scal[4] = zf;
        R.scal[5] = sqrt(H > 0.0 ? H / m : 0.0);
        R.scal[6] = H;
    }
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
// register fragment units per wave: whole components (K >= 4) or spread blocks (K < 4)
int upw_for(const DevProblem &P)
{
    const int NJB = P.D / 16;
    return P.K >= 4 ? (P.K + 3) / 4 * NJB : (P.K * NJB + 3) / 4;
}

// compiled fragment capacities per padded dimension
int upw_template(int D, int upw)
{
    if (D == 32) return upw <= 4 ? 4 : (upw <= 16 ? 16 : 0);
    if (D == 64) return upw <= 2 ? 2 : (upw <= 4 ? 4 : (upw <= 8 ? 8 : 0));
    if (D == 128) return upw <= 4 ? 4 : 0;
    return 0;
}

size_t hrss_lds_bytes(int D, int K) { return (size_t)hrss_layout(D, K).total; }
int dirs_rows(int D) { return dir_rows(D); }

int mode_supported(const DevProblem &P, int mode)
{
    if (hrss_lds_bytes(P.D, P.K) > 160 * 1024) return 0;  // one workgroup's LDS
    if (mode == MODE_FP64) return 1;
    if (P.lik_kind != LIK_MIXTURE) return 0;
    return upw_template(P.D, upw_for(P)) != 0;
}

template <typename F>
static hipError_t set_lds(F *f, size_t bytes)
{
    return hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

hipError_t launch_init_draw(const Launch &L, hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_draw, dim3(L.nblocks), dim3(256), 0, s, L);
    return hipGetLastError();
}

template <int D, int MODE, int LIK, int UPW>
static hipError_t eval_t(const Launch &L, const double *X, int ld, int n, double *out,
                         int from_run, hipStream_t s)
{
    const size_t lds = hrss_lds_bytes(D, L.max_K);
    auto f = k_eval<D, MODE, LIK, UPW>;
    hipError_t e = set_lds(f, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(f, dim3(L.nblocks), dim3(256), lds, s, L, X, ld, n, out, from_run);
    return hipGetLastError();
}

template <int D, int MODE, int LIK, int UPW>
static hipError_t hrss_t(const Launch &L, hipStream_t s)
{
    const size_t lds = hrss_lds_bytes(D, L.max_K);
    auto f = k_hrss<D, MODE, LIK, UPW>;
    hipError_t e = set_lds(f, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(f, dim3(L.nblocks), dim3(256), lds, s, L);
    return hipGetLastError();
}

template <int D, int MODE, int LIK, int UPW>
static hipError_t rw_t(const Launch &L, hipStream_t s)
{
    const size_t lds = hrss_lds_bytes(D, L.max_K);
    auto f = k_rw<D, MODE, LIK, UPW>;
    hipError_t e = set_lds(f, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(f, dim3(L.nblocks), dim3(256), lds, s, L);
    return hipGetLastError();
}

// dispatch over (D, mode, likelihood); UPW = register fragment units per wave (mixed only)
#define NSS_MIXED_D(FN, MODE_, ...)                                                           \
    do {                                                                                      \
        if (D == 32) {                                                                        \
            if (upw <= 4) return FN<32, MODE_, LIK_MIXTURE, 4>(__VA_ARGS__);                  \
            return FN<32, MODE_, LIK_MIXTURE, 16>(__VA_ARGS__);                               \
        }                                                                                     \
        if (D == 64) {                                                                        \
            if (upw <= 2) return FN<64, MODE_, LIK_MIXTURE, 2>(__VA_ARGS__);                  \
            if (upw <= 4) return FN<64, MODE_, LIK_MIXTURE, 4>(__VA_ARGS__);                  \
            return FN<64, MODE_, LIK_MIXTURE, 8>(__VA_ARGS__);                                \
        }                                                                                     \
        return FN<128, MODE_, LIK_MIXTURE, 4>(__VA_ARGS__);                                   \
    } while (0)
#define NSS_DISPATCH(FN, ...)                                                                 \
    do {                                                                                      \
        if (D != 32 && D != 64 && D != 128 && D != 320) return hipErrorInvalidValue;          \
        if (lik == LIK_FUNNEL) {                                                              \
            if (mode != MODE_FP64) return hipErrorNotSupported;                               \
            if (D == 32) return FN<32, MODE_FP64, LIK_FUNNEL, 1>(__VA_ARGS__);                \
            if (D == 64) return FN<64, MODE_FP64, LIK_FUNNEL, 1>(__VA_ARGS__);                \
            if (D == 128) return FN<128, MODE_FP64, LIK_FUNNEL, 1>(__VA_ARGS__);              \
            return FN<320, MODE_FP64, LIK_FUNNEL, 1>(__VA_ARGS__);                            \
        }                                                                                     \
        if (lik == LIK_RG) {                                                                  \
            if (mode != MODE_FP64) return hipErrorNotSupported;                               \
            if (D == 32) return FN<32, MODE_FP64, LIK_RG, 1>(__VA_ARGS__);                    \
            if (D == 64) return FN<64, MODE_FP64, LIK_RG, 1>(__VA_ARGS__);                    \
            if (D == 128) return FN<128, MODE_FP64, LIK_RG, 1>(__VA_ARGS__);                  \
            return FN<320, MODE_FP64, LIK_RG, 1>(__VA_ARGS__);                                \
        }                                                                                     \
        if (lik != LIK_MIXTURE || D == 320) return hipErrorInvalidValue;                      \
        if (mode == MODE_FP64) {                                                              \
            if (D == 32) return FN<32, MODE_FP64, LIK_MIXTURE, 1>(__VA_ARGS__);               \
            if (D == 64) return FN<64, MODE_FP64, LIK_MIXTURE, 1>(__VA_ARGS__);               \
            return FN<128, MODE_FP64, LIK_MIXTURE, 1>(__VA_ARGS__);                           \
        }                                                                                     \
        if (upw_template(D, upw) == 0) return hipErrorNotSupported;                           \
        if (mode == MODE_BF16) NSS_MIXED_D(FN, MODE_BF16, __VA_ARGS__);                       \
        if (mode == MODE_FP16) NSS_MIXED_D(FN, MODE_FP16, __VA_ARGS__);                       \
        if (mode == MODE_BF16X3) NSS_MIXED_D(FN, MODE_BF16X3, __VA_ARGS__);                   \
        if (mode == MODE_FP16X3) NSS_MIXED_D(FN, MODE_FP16X3, __VA_ARGS__);                   \
        return hipErrorInvalidValue;                                                          \
    } while (0)

hipError_t launch_eval_init(const Launch &L, int D, int lik, hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    const int mode = MODE_FP64, upw = 1;
    NSS_DISPATCH(eval_t, L, nullptr, 0, 0, nullptr, 1, s);
}

hipError_t launch_eval_points(const Launch &L, int D, int lik, int mode, int upw, const double *X,
                              int ld, int n, double *out, hipStream_t s)
{
    if (n <= 0 || L.nblocks <= 0) return hipSuccess;
    NSS_DISPATCH(eval_t, L, X, ld, n, out, 0, s);
}

hipError_t launch_hrss(const Launch &L, int D, int lik, int mode, int upw, hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    NSS_DISPATCH(hrss_t, L, s);
}

hipError_t launch_rw(const Launch &L, int D, int lik, int mode, int upw, hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    NSS_DISPATCH(rw_t, L, s);
}

hipError_t launch_smc(const Launch &L, int op, hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    const size_t lds = (size_t)kMaxLive * 12;
    hipError_t e = set_lds(k_smc, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_smc, dim3(L.nblocks), dim3(kSelectThreads), lds, s, L, op);
    return hipGetLastError();
}

hipError_t launch_select(const Launch &L, int op, hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    int NP = 1;
    while (NP < L.max_m) NP <<= 1;
    const size_t lds = (size_t)NP * 8 + (size_t)(NP + (NP & 1)) * 4 + 32 * 8 + 16;
    hipError_t e = set_lds(k_select, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_select, dim3(L.nblocks), dim3(kSelectThreads), lds, s, L, op);
    return hipGetLastError();
}

hipError_t launch_cov(const Launch &cov, const Launch &one, int D, hipStream_t s)
{
    if (one.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cov, dim3(cov.nblocks), dim3(256), 0, s, cov);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int Dl = D <= 128 ? D : 128;   // runs above 128 keep their factor in global memory
    const size_t lds = (size_t)(Dl * (Dl + 1) / 2 + D + 32) * 8 + 16;
    e = set_lds(k_chol, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_chol, dim3(one.nblocks), dim3(1024), lds, s, one);
    return hipGetLastError();
}

template <int D>
static hipError_t dirs_t(const Launch &L, hipStream_t s)
{
    const size_t lds = (size_t)dirs_lds_bytes(D);
    hipError_t e = set_lds(k_dirs<D>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dirs<D>, dim3(L.nblocks), dim3(256), lds, s, L);
    return hipGetLastError();
}

hipError_t launch_dirs(const Launch &L, int D, hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    if (D == 32) return dirs_t<32>(L, s);
    if (D == 64) return dirs_t<64>(L, s);
    if (D == 128) return dirs_t<128>(L, s);
    if (D == 320) return dirs_t<320>(L, s);
    return hipErrorInvalidValue;
}

hipError_t launch_logz(const Launch &L, hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_logz, dim3(L.nblocks), dim3(1024), 0, s, L);
    return hipGetLastError();
}
}  // namespace nss
