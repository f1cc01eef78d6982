// Post-hoc geometric uncertainty of a run (App. "Estimation of prior volumes and propagation
// of geometric uncertainty"): R replicas of the prior-volume trajectory with random shrinkages,
// trapezoid weights at inverse temperature beta, log Z per replica, the geometric-mean weights
// over the replicas and their Kish effective sample size.
//
// Deaths g = 0..N-1 in likelihood order: the dead record (the j-th death of a batch, j = 0..k-1,
// sees n = m - j live points) followed by the final survivors in ascending logL (n = nf - q).
// Replica r: log t_g = log(u_g) / n_g with u_g the first (g even) or second (g odd) uniform of
// Philox (purpose GEOM, index r, counter word g/2); log X_g = sum_{h<g} log t_h (X before death
// g); the trapezoid element X_g (1 - t_g t_{g+1}) / 2 with t_N = 0 (X after the last death is 0);
// log w = beta logL + log dX (the tempered term is 0 at beta = 0).
//
// Nothing of size R x N is stored: the shrinkages are counter-based, so they are drawn twice.
//  k_geom_sums     grid (chunk, replica group): sum of log t over each chunk of kGeomC deaths,
//                  per replica
//  k_geom_offsets  one workgroup per replica: exclusive scan of the chunk sums (log X at each
//                  chunk's first death)
//  k_geom_weights  grid (chunk, replica group): each workgroup keeps its chunk's logL and live
//                  counts in registers, loops over the group's replicas, rebuilds log X inside
//                  the chunk, forms the log weights, accumulates them per death for the mean and
//                  emits per-wave (max, sum) partials of each replica's evidence
//  k_geom_mean     per death: mean of the log weights over the replicas; per-wave ESS partials
//  k_geom_final    one workgroup per replica combines its evidence partials; one more combines
//                  the ESS partials
#include "nss_internal.hpp"
#include "nss_rng.hpp"
#include "nss_wave.hpp"

#include <math.h>

namespace nss {

namespace {

constexpr uint32_t PUR_GEOM = 6;
constexpr int kGeomT = 256;                 // threads per workgroup
constexpr int kGeomE = 4;                   // consecutive deaths per thread (even)
constexpr int kGeomC = kGeomT * kGeomE;     // deaths per chunk
constexpr int kGeomW = kGeomT / 64;         // waves per workgroup
constexpr double kLn2 = 0.69314718055994530942;

struct GeomArgs {
    const double *dead;   // [n_dead] dead-point logL in death order
    const double *logL;   // [m] live logL, ascending through perm
    const int *perm;      // [m]; the final survivors are perm[k..m-1]
    long long n_dead, N;
    int m, k, R, nchunk, rpg;  // rpg: replicas per group in k_geom_weights
    double beta;
    uint32_t key0, key1;
    double *csum;      // [R][nchunk] chunk sums of log t, scanned in place into offsets
    double2 *zpart;    // [R][nchunk * kGeomW] per-wave (max, sum) of the evidence terms
    double *accp;      // [groups][N] per-group sums of log w over replicas
    double *logw_mean; // [N]
    double4 *epart;    // [ceil(N / 64)] per-wave (max, sum, sum of squares) of mean weights
    double *logz;      // [R]
    double *ess;       // [1]
};

// (N < 2^31 deaths, checked by the caller, so death indices are 32-bit)
__device__ __forceinline__ double live_count(const GeomArgs &a, int g)
{
    return g < (int)a.n_dead ? (double)(a.m - (int)((unsigned)g % (unsigned)a.k))
                             : (double)((a.m - a.k) - (g - (int)a.n_dead));
}

__device__ __forceinline__ double death_logL(const GeomArgs &a, int g)
{
    return g < (int)a.n_dead ? a.dead[g] : a.logL[a.perm[a.k + (g - (int)a.n_dead)]];
}

// log t for the kGeomE consecutive deaths g0 .. g0+kGeomE-1 (g0 even) of replica r; rn holds the
// reciprocal live counts (0 past the last death, which makes those shrinkages exactly 1).
__device__ __forceinline__ void draw_logt(const GeomArgs &a, int r, int g0, const double *rn,
                                          double *s)
{
#pragma unroll
    for (int h = 0; h < kGeomE / 2; ++h) {
        double ua, ub;
        draw2(a.key0, a.key1, PUR_GEOM, (uint32_t)r, (uint32_t)((g0 >> 1) + h), 0u, 0u, ua, ub);
        s[2 * h] = log(ua) * rn[2 * h];
        s[2 * h + 1] = log(ub) * rn[2 * h + 1];
    }
}

// Combined (max, sum exp(x - max)) of per-thread pairs over the wave; an empty pair is
// (-inf, 0).
__device__ __forceinline__ double2 wave_lse(double ref, double sum)
{
    const double M = wave_max(ref);
    double c = 0.0;
    if (ref > -INFINITY) c = sum * exp(ref - M);
    return make_double2(M, wave_sum_fast(c));
}

}  // namespace

__global__ __launch_bounds__(kGeomT) void k_geom_sums(GeomArgs a)
{
    __shared__ double red[2][kGeomW];
    const int c = blockIdx.x, grp = blockIdx.y;
    const int g0 = c * kGeomC + (int)threadIdx.x * kGeomE;
    double rn[kGeomE];
#pragma unroll
    for (int q = 0; q < kGeomE; ++q) rn[q] = g0 + q < a.N ? 1.0 / live_count(a, g0 + q) : 0.0;
    const int r0 = grp * a.rpg, r1 = min(a.R, r0 + a.rpg);
    for (int r = r0; r < r1; ++r) {
        double s[kGeomE];
        draw_logt(a, r, g0, rn, s);
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kGeomE; ++q) t += s[q];
        // workgroup sum; the two LDS buffers alternate so one barrier per replica suffices
        t = wave_sum_fast(t);
        if ((threadIdx.x & 63) == 0) red[r & 1][threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double v = 0.0;
#pragma unroll
            for (int w = 0; w < kGeomW; ++w) v += red[r & 1][w];
            a.csum[(size_t)r * a.nchunk + c] = v;
        }
    }
}

__global__ __launch_bounds__(kGeomT) void k_geom_offsets(GeomArgs a)
{
    __shared__ double red[kGeomW];
    double *cs = a.csum + (size_t)blockIdx.x * a.nchunk;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    double carry = 0.0;
    for (int c0 = 0; c0 < a.nchunk; c0 += kGeomT) {
        const int c = c0 + (int)threadIdx.x;
        const double v = c < a.nchunk ? cs[c] : 0.0;
        double inc = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double u = __shfl_up(inc, o, 64);
            if (l >= o) inc += u;
        }
        double ex = __shfl_up(inc, 1, 64);
        if (l == 0) ex = 0.0;
        if (l == 63) red[w] = inc;
        __syncthreads();
        double pre = carry, all = carry;
#pragma unroll
        for (int i = 0; i < kGeomW; ++i) {
            if (i < w) pre += red[i];
            all += red[i];
        }
        if (c < a.nchunk) cs[c] = pre + ex;
        carry = all;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kGeomT) void k_geom_weights(GeomArgs a)
{
    __shared__ double tot[2][kGeomW];   // wave totals of log t, by replica parity
    __shared__ double first[2][kGeomW]; // each wave's first shrinkage t
    const int c = blockIdx.x, grp = blockIdx.y;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int g0 = c * kGeomC + (int)threadIdx.x * kGeomE;
    const int gnext = (c + 1) * kGeomC;   // first death of the next chunk
    double rn[kGeomE], tl[kGeomE], ew[kGeomE], acc[kGeomE];
    double tmax = -INFINITY;
#pragma unroll
    for (int q = 0; q < kGeomE; ++q) {
        const bool ok = g0 + q < a.N;
        rn[q] = ok ? 1.0 / live_count(a, g0 + q) : 0.0;
        const double L = ok ? death_logL(a, g0 + q) : -INFINITY;
        tl[q] = !ok ? -INFINITY : (a.beta == 0.0 ? 0.0 : a.beta * L);
        tmax = fmax(tmax, tl[q]);
        acc[q] = 0.0;
    }
    // likelihood factors relative to the thread's largest, taken once for all replicas
#pragma unroll
    for (int q = 0; q < kGeomE; ++q) ew[q] = tl[q] > -INFINITY ? exp(tl[q] - tmax) : 0.0;
    const bool chunk_end = threadIdx.x == kGeomT - 1 && gnext < a.N;
    const double rn_next = chunk_end ? 1.0 / live_count(a, gnext) : 0.0;
    const int r0 = grp * a.rpg, r1 = min(a.R, r0 + a.rpg);
    for (int r = r0; r < r1; ++r) {
        const int par = r & 1;
        double s[kGeomE], t[kGeomE];
        draw_logt(a, r, g0, rn, s);
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < kGeomE; ++q) {
            t[q] = exp(s[q]);
            sum += s[q];
        }
        // shrinkage of the death after this thread's last one
        double tn = __shfl_down(t[0], 1, 64);
        // wave scan of the thread totals
        double inc = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const double u = __shfl_up(inc, o, 64);
            if (l >= o) inc += u;
        }
        double ex = __shfl_up(inc, 1, 64);
        if (l == 0) ex = 0.0;
        if (l == 63) tot[par][w] = inc;
        if (l == 0) first[par][w] = t[0];
        if (chunk_end) {
            double ua, ub;
            draw2(a.key0, a.key1, PUR_GEOM, (uint32_t)r, (uint32_t)(gnext >> 1), 0u, 0u, ua, ub);
            tn = exp(log(ua) * rn_next);
        }
        __syncthreads();
        if (l == 63 && w + 1 < kGeomW) tn = first[par][w + 1];
        double P = a.csum[(size_t)r * a.nchunk + c];
#pragma unroll
        for (int i = 0; i < kGeomW; ++i)
            if (i < w) P += tot[par][i];
        P += ex;
        // weights: log dX = log X_g + log1p(-t_g t_{g+1}) - log 2
        double p = P, X = 1.0, z = 0.0;
#pragma unroll
        for (int q = 0; q < kGeomE; ++q) {
            const int g = g0 + q;
            const double tnext = q + 1 < kGeomE ? t[q + 1] : tn;
            const double y = g + 1 < a.N ? t[q] * tnext : 0.0;
            const double lw = tl[q] + p + log1p(-y) - kLn2;
            if (g < a.N) {
                acc[q] += lw;
                z += ew[q] * X * (1.0 - y);
            }
            p += s[q];
            X *= t[q];
        }
        // evidence terms of this thread: exp(tmax + P) * z / 2
        const double ref = (z > 0.0) ? tmax + P - kLn2 : -INFINITY;
        const double2 pr = wave_lse(ref, z);
        if (l == 0) a.zpart[((size_t)r * a.nchunk + c) * kGeomW + w] = pr;
    }
#pragma unroll
    for (int q = 0; q < kGeomE; ++q)
        if (g0 + q < a.N) a.accp[(size_t)grp * a.N + g0 + q] = acc[q];
}

__global__ __launch_bounds__(256) void k_geom_mean(GeomArgs a, int groups)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double v = -INFINITY;
    if (g < a.N) {
        double s = 0.0;
        for (int i = 0; i < groups; ++i) s += a.accp[(size_t)i * a.N + g];
        v = s / a.R;
        a.logw_mean[g] = v;
    }
    const double M = wave_max(v);
    const double e = v > -INFINITY ? exp(v - M) : 0.0;
    const double s1 = wave_sum_fast(e), s2 = wave_sum_fast(e * e);
    if ((threadIdx.x & 63) == 0 && g < a.N) a.epart[g >> 6] = make_double4(M, s1, s2, 0.0);
}

__global__ __launch_bounds__(256) void k_geom_final(GeomArgs a)
{
    __shared__ double red[4];
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < a.R) {
        const double2 *zp = a.zpart + (size_t)blockIdx.x * a.nchunk * kGeomW;
        const int n = a.nchunk * kGeomW;
        double M = -INFINITY;
        for (int i = tid; i < n; i += 256) M = fmax(M, zp[i].x);
        M = wave_max(M);
        if ((tid & 63) == 0) red[tid >> 6] = M;
        __syncthreads();
        M = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        __syncthreads();
        double s = 0.0;
        if (M > -INFINITY)
            for (int i = tid; i < n; i += 256)
                if (zp[i].x > -INFINITY) s += zp[i].y * exp(zp[i].x - M);
        s = wave_sum_fast(s);
        if ((tid & 63) == 0) red[tid >> 6] = s;
        __syncthreads();
        if (tid == 0) {
            s = (red[0] + red[1]) + (red[2] + red[3]);
            a.logz[blockIdx.x] = (M > -INFINITY && s > 0.0) ? M + log(s) : -INFINITY;
        }
        return;
    }
    const long long n = (a.N + 63) >> 6;
    double M = -INFINITY;
    for (long long i = tid; i < n; i += 256) M = fmax(M, a.epart[i].x);
    M = wave_max(M);
    if ((tid & 63) == 0) red[tid >> 6] = M;
    __syncthreads();
    M = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    double s1 = 0.0, s2 = 0.0;
    if (M > -INFINITY)
        for (long long i = tid; i < n; i += 256) {
            const double4 e = a.epart[i];
            if (e.x > -INFINITY) {
                const double f = exp(e.x - M);
                s1 += e.y * f;
                s2 += e.z * f * f;
            }
        }
    s1 = wave_sum_fast(s1);
    s2 = wave_sum_fast(s2);
    __shared__ double red2[4];
    if ((tid & 63) == 0) { red[tid >> 6] = s1; red2[tid >> 6] = s2; }
    __syncthreads();
    if (tid == 0) {
        s1 = (red[0] + red[1]) + (red[2] + red[3]);
        s2 = (red2[0] + red2[1]) + (red2[2] + red2[3]);
        *a.ess = s2 > 0.0 ? s1 * s1 / s2 : 0.0;
    }
}

// ------------------------------------------------------------------------------------------
// weighted posterior samples (resampling with the geometric-mean weights)
// ------------------------------------------------------------------------------------------
constexpr uint32_t PUR_POST = 7;

// Normalised cumulative weights cum[i] = sum_{l <= i} w_l / sum w, w = exp(logw_mean - max), in
// index order, over blocks of 8192 deaths (eight consecutive per thread).  The scratch ws holds
// [0] the maximum, [1] the total, [2, 2 + nb) the block maxima and then the blocks' exclusive
// offsets, [2 + nb, 2 + 2 nb) the block sums.
constexpr int kCumT = 1024, kCumPer = 8;
constexpr long long kCumChunk = (long long)kCumT * kCumPer;

long long post_cum_blocks(long long N) { return (N + kCumChunk - 1) / kCumChunk; }

__global__ __launch_bounds__(kCumT) void k_post_bmax(const double *lw, long long N, double *ws)
{
    __shared__ double red[16];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const long long base = (long long)blockIdx.x * kCumChunk;
    double mx = -INFINITY;
#pragma unroll
    for (int q = 0; q < kCumPer; ++q) {
        const long long i = base + (long long)q * kCumT + tid;
        if (i < N) mx = fmax(mx, lw[i]);
    }
    mx = wave_max(mx);
    if (l == 0) red[w] = mx;
    __syncthreads();
    if (tid == 0) {
        double m = red[0];
        for (int i = 1; i < 16; ++i) m = fmax(m, red[i]);
        ws[2 + blockIdx.x] = m;
    }
}

// One workgroup: the maximum of the nb block maxima into ws[0].
__global__ __launch_bounds__(kCumT) void k_post_gmax(double *ws, int nb)
{
    __shared__ double red[16];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    double mx = -INFINITY;
    for (int b = tid; b < nb; b += kCumT) mx = fmax(mx, ws[2 + b]);
    mx = wave_max(mx);
    if (l == 0) red[w] = mx;
    __syncthreads();
    if (tid == 0) {
        double m = red[0];
        for (int i = 1; i < 16; ++i) m = fmax(m, red[i]);
        ws[0] = m;
    }
}

// exp(lw - M) over this workgroup's block: thread t takes deaths i0 .. i0 + 7 (i0 = base + 8 t),
// v[q] its running sums, pre the sum of the block's earlier deaths; returns the block's total.
// The block sums and the final pass both use this, so their totals agree bit for bit.
__device__ __forceinline__ double block_cum(const double *lw, long long N, double M, long long i0,
                                            double (&v)[kCumPer], double &pre, double *red)
{
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kCumPer; ++q) {
        const long long i = i0 + q;
        const double x = i < N ? lw[i] : -INFINITY;
        s += x > -INFINITY ? exp(x - M) : 0.0;
        v[q] = s;
    }
    double inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double t = __shfl_up(inc, o, 64);
        if (l >= o) inc += t;
    }
    if (l == 63) red[w] = inc;
    __syncthreads();
    double p = 0.0, all = 0.0;
    for (int q = 0; q < 16; ++q) {
        if (q < w) p += red[q];
        all += red[q];
    }
    pre = p + (inc - s);
    return all;
}

__global__ __launch_bounds__(kCumT) void k_post_bsum(const double *lw, long long N, double *ws,
                                                     int nb)
{
    __shared__ double red[16];
    const long long i0 = (long long)blockIdx.x * kCumChunk + (long long)threadIdx.x * kCumPer;
    double v[kCumPer], pre;
    const double all = block_cum(lw, N, ws[0], i0, v, pre, red);
    if (threadIdx.x == 0) ws[2 + nb + blockIdx.x] = all;
}

// One thread, in block order: the exclusive offsets (over the block maxima, no longer needed)
// and the total, so that each offset plus its block's sum is exactly the next offset.
__global__ void k_post_offsets(double *ws, int nb)
{
    if (threadIdx.x != 0) return;
    double acc = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double sb = ws[2 + nb + b];
        ws[2 + b] = acc;
        acc += sb;
    }
    ws[1] = acc;
}

__global__ __launch_bounds__(kCumT) void k_post_cum(const double *lw, long long N,
                                                    const double *ws, double *cum)
{
    __shared__ double red[16];
    const long long i0 = (long long)blockIdx.x * kCumChunk + (long long)threadIdx.x * kCumPer;
    double v[kCumPer], pre;
    (void)block_cum(lw, N, ws[0], i0, v, pre, red);
    const double off = ws[2 + blockIdx.x] + pre, tot = ws[1];
#pragma unroll
    for (int q = 0; q < kCumPer; ++q)
        if (i0 + q < N) cum[i0 + q] = (off + v[q]) / tot;
}

// Sample j: the first death whose cumulative weight reaches (u + j) / n; its coordinates.
__global__ __launch_bounds__(256) void k_post_pick(const double *cum, long long N, long long n_dead,
                                                   const double *deadx, const double *X,
                                                   const int *perm, int k, int m_pad, int d,
                                                   int n, uint32_t key0, uint32_t key1,
                                                   double *xo, long long *io)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double u, unused;
    draw2(key0, key1, PUR_POST, 0u, 0u, 0u, 0u, u, unused);
    const double pos = (u + j) / n;
    long long lo = 0, hi = N - 1;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (cum[mid] >= pos) hi = mid; else lo = mid + 1;
    }
    io[j] = lo;
    for (int a = 0; a < d; ++a)
        xo[(size_t)j * d + a] = lo < n_dead ? deadx[lo * d + a]
                                            : X[(size_t)a * m_pad + perm[k + (int)(lo - n_dead)]];
}

hipError_t launch_post_samples(const GeomLaunch &G, const double *deadx, const double *X,
                               int m_pad, int d, int n, double *cum, double *cws, double *xo,
                               long long *io, hipStream_t s)
{
    const long long nbl = post_cum_blocks(G.N);
    const int nb = (int)nbl;
    hipLaunchKernelGGL(k_post_bmax, dim3((unsigned)nb), dim3(kCumT), 0, s, G.logw_mean, G.N, cws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_post_gmax, dim3(1), dim3(kCumT), 0, s, cws, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_post_bsum, dim3((unsigned)nb), dim3(kCumT), 0, s, G.logw_mean, G.N, cws,
                       nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_post_offsets, dim3(1), dim3(64), 0, s, cws, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_post_cum, dim3((unsigned)nb), dim3(kCumT), 0, s, G.logw_mean, G.N, cws,
                       cum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_post_pick, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cum, G.N,
                       G.n_dead, deadx, X, G.perm, G.k, m_pad, d, n, G.key0, G.key1, xo, io);
    return hipGetLastError();
}

size_t geom_workspace_bytes(long long N, int R, int groups)
{
    const long long nchunk = (N + kGeomC - 1) / kGeomC;
    size_t b = 0;
    auto add = [&](size_t n) { b += (n + 255) / 256 * 256; };
    add((size_t)R * nchunk * 8);                 // csum
    add((size_t)R * nchunk * kGeomW * 16);       // zpart
    add((size_t)groups * N * 8);                 // accp
    add((size_t)((N + 63) / 64) * 32);           // epart
    return b;
}

int geom_groups(long long N, int R)
{
    // enough workgroups to fill the chip several times over, at least 8 replicas per group
    const long long nchunk = (N + kGeomC - 1) / kGeomC;
    long long g = (2048 + nchunk - 1) / nchunk;
    if (g > (R + 7) / 8) g = (R + 7) / 8;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_geom(const GeomLaunch &G, hipStream_t s)
{
    const long long nchunk = (G.N + kGeomC - 1) / kGeomC;
    const int groups = G.groups;
    GeomArgs a{};
    a.dead = G.dead; a.logL = G.logL; a.perm = G.perm;
    a.n_dead = G.n_dead; a.N = G.N; a.m = G.m; a.k = G.k; a.R = G.R; a.nchunk = (int)nchunk;
    a.rpg = (G.R + groups - 1) / groups;
    a.beta = G.beta; a.key0 = G.key0; a.key1 = G.key1;
    char *p = (char *)G.ws;
    auto take = [&](size_t n) { char *q = p; p += (n + 255) / 256 * 256; return (void *)q; };
    a.csum = (double *)take((size_t)G.R * nchunk * 8);
    a.zpart = (double2 *)take((size_t)G.R * nchunk * kGeomW * 16);
    a.accp = (double *)take((size_t)groups * G.N * 8);
    a.epart = (double4 *)take((size_t)((G.N + 63) / 64) * 32);
    a.logz = G.logz;
    a.logw_mean = G.logw_mean;
    a.ess = G.ess;
    hipLaunchKernelGGL(k_geom_sums, dim3((unsigned)nchunk, groups), dim3(kGeomT), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_geom_offsets, dim3(G.R), dim3(kGeomT), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_geom_weights, dim3((unsigned)nchunk, groups), dim3(kGeomT), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_geom_mean, dim3((unsigned)((G.N + 255) / 256)), dim3(256), 0, s, a,
                       groups);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_geom_final, dim3(G.R + 1), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace nss
