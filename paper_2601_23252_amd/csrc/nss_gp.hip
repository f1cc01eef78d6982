// GP hyperparameter marginalisation on gfx950 (Sec. 5 "Gaussian process" experiments; App.
// "Gaussian Process Hyperparameter Marginalization"): the likelihood of a candidate
// u = log theta, theta = (sigma_f, l_1, l_2, l_p, P, sigma_n), is the log marginal likelihood
//   log N(y; 0, K + sigma_n^2 I),  K_ab = sigma_f^2 exp(-1/2 sum_j (a_j-b_j)^2 / l_j^2
//                                               - 2 sum_j sin^2(pi (a_j-b_j)/P) / l_p^2)
// over n <= 256 observations with 2-D inputs (a squared-exponential times a periodic kernel,
// each a product over the input dimensions).
//
// One workgroup of 8 waves evaluates one candidate at a time.  The kernel matrix is built as
// 16x16 tiles of the lower triangle in the accumulator layout of the 16x16x4 MFMA (tile t is
// owned by tile wave t mod 7; a wave's first seven tiles sit in its own LDS area, the others in
// its registers), and factorised by a right-looking blocked
// Cholesky: for each block column J one wave factors the diagonal tile and inverts the factor,
// the panel tiles are multiplied by that inverse on MFMA, and every trailing tile takes its
// rank-16 update on MFMA with operands from LDS.  The right-hand side y rides along, so the
// forward solve z = L^{-1} y and the log-determinant come out of the same sweep:
//   log L = -|z|^2 / 2 - sum_i log L_ii - n/2 log(2 pi).
// A pivot that is not positive makes the factorisation fail (FP64: log L = -inf).
//
//  k_hrss_gp   one HRSS chain per workgroup (App. A.6), candidates evaluated one at a time
//  k_eval_gp   one point per workgroup (initial live set, tests)
#include "nss_internal.hpp"
#include "nss_rng.hpp"
#include "nss_wave.hpp"

#include <math.h>

namespace nss {

namespace {

constexpr int kGpWaves = 8;                                           // per workgroup
constexpr int kGpThreads = 64 * kGpWaves;
constexpr int kGpTileWaves = 7;        // waves 0..6 hold the covariance tiles
constexpr int kGpPivot = 7;            // wave 7 factors the diagonal tiles
constexpr int kGpMaxTiles = 136;                                      // 16 * 17 / 2
constexpr int kGpSlots = (kGpMaxTiles + kGpTileWaves - 1) / kGpTileWaves;  // tiles per wave
// a wave's first kGpLdsSlots tiles (the upper block rows, final after few updates) live in its
// own LDS area, the rest in registers: 14 register tiles keep the wave inside its 256 VGPRs
constexpr int kGpLdsSlots = 7;
constexpr int kGpRegSlots = kGpSlots - kGpLdsSlots;
constexpr int kGpSpinMax = 1 << 22;    // bound on the pivot wave's wait for a diagonal tile
constexpr int kGpLd = 17;                                             // LDS tile row stride
constexpr int kTile = 16 * kGpLd;
constexpr int kGpD = 6;                                               // hyperparameters

// LDS: inputs and targets (FP64), reduction slots, then the factorisation's tiles in T
constexpr int kOffXs = 0;                                             // double [256][2]
constexpr int kOffYs = kOffXs + 2 * kGpMaxObs * 8;                    // double [256]
constexpr int kOffMisc = kOffYs + kGpMaxObs * 8;                      // double [16], int flag
constexpr int kOffChain = kOffMisc + 256;                             // chain point, direction
constexpr int kOffSc = kOffChain + 128;                               // double [256][4]
constexpr int kOffT = kOffSc + 4 * kGpMaxObs * 8;
template <typename T>
constexpr int gp_lds_bytes()
{
    // 16 panel tiles, diagonal tile, inverse tile, right-hand side, z block, reciprocal pivots,
    // then the tile waves' LDS-resident tiles; the FP32 refinement adds the inverse factors of
    // all diagonal tiles, z, alpha, the partial products of a block step and one 16-vector
    return kOffT + (int)sizeof(T) * (16 * kTile + 2 * kTile + kGpMaxObs + 32 +
                                     kGpLdsSlots * kGpTileWaves * kTile) +
           (sizeof(T) == 4 ? 4 * (16 * kTile + 2 * kGpMaxObs + 16 * 16 + 16) : 0);
}

template <typename T> struct Mf;
template <> struct Mf<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 mma(double a, double b, v4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // accumulator row of register r in lane l (column l & 15)
    __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <> struct Mf<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 mma(float a, float b, v4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};

__device__ __forceinline__ double readlane_t(double v, int lane) { return readlane_d(v, lane); }
__device__ __forceinline__ float readlane_t(float v, int lane)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// lower tile index t = I (I + 1) / 2 + K  ->  (I, K), K <= I
__device__ __forceinline__ void tile_ik(int t, int &I, int &K)
{
    int i = (int)((sqrtf(8.f * (float)t + 1.f) - 1.f) * 0.5f);
    while (i * (i + 1) / 2 > t) --i;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    I = i;
    K = t - i * (i + 1) / 2;
}

struct GpTheta {
    double sf2, il1, il2, ilp2, iper, sn2;
};

__device__ __forceinline__ GpTheta gp_theta(const double *u)
{
    GpTheta h;
    h.sf2 = exp(2.0 * u[0]);
    h.il1 = exp(-u[1]);
    h.il2 = exp(-u[2]);
    h.ilp2 = exp(-2.0 * u[3]);
    h.iper = exp(-u[4]);
    h.sn2 = exp(2.0 * u[5]);
    return h;
}

// Entry (row, col) of the padded covariance: identity outside the n observations, zero above
// the diagonal (never read as data).  sin(pi (a - b) / P) = s_a c_b - c_a s_b from the per-point
// sc[i] = (sin, cos)(pi x_i1 / P), (sin, cos)(pi x_i2 / P), so an entry costs one exponential.
template <typename T>
__device__ __forceinline__ T gp_entry(const double *xs, const double *sc, int n, int row, int col,
                                      const GpTheta &h)
{
    if (row >= n || col >= n) return (row == col) ? T(1) : T(0);
    if (col > row) return T(0);
    const double d1 = xs[2 * row] - xs[2 * col], d2 = xs[2 * row + 1] - xs[2 * col + 1];
    const double *pa = sc + 4 * row, *pb = sc + 4 * col;
    const double s1 = pa[0] * pb[1] - pa[1] * pb[0], s2 = pa[2] * pb[3] - pa[3] * pb[2];
    if constexpr (sizeof(T) == 8) {
        const double a1 = d1 * h.il1, a2 = d2 * h.il2;
        double v = h.sf2 * exp(-0.5 * (a1 * a1 + a2 * a2) - 2.0 * (s1 * s1 + s2 * s2) * h.ilp2);
        if (row == col) v += h.sn2;
        return v;
    } else {
        const float a1 = (float)(d1 * h.il1), a2 = (float)(d2 * h.il2);
        const float f1 = (float)s1, f2 = (float)s2;
        float v = (float)h.sf2 *
                  expf(-0.5f * (a1 * a1 + a2 * a2) - 2.0f * (f1 * f1 + f2 * f2) * (float)h.ilp2);
        if (row == col) v += (float)h.sn2;
        return v;
    }
}

template <typename T, typename V>
__device__ __forceinline__ void store_tile(const V &acc, T *p, int l)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) p[Mf<T>::row(l, r) * kGpLd + (l & 15)] = acc[r];
}
template <typename T, typename V>
__device__ __forceinline__ void load_tile(V &acc, const T *p, int l)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = p[Mf<T>::row(l, r) * kGpLd + (l & 15)];
}

// Factor the diagonal tile in dg (rows of stride kGpLd) in place, write the inverse of the
// factor to li and its reciprocal pivots to dv, z = L^{-1} y_J to zb, add log det and |z|^2 to
// this wave's (ldet, quad) (lane 0) and raise the flag on a pivot that is not positive.  Run by
// one whole wave; lane i (mod 16) holds row i, every DPP row a copy.
// 1/sqrt(x): the hardware estimate refined by Newton steps r <- r (3/2 - x r^2 / 2)
// (two in FP64, one in FP32), for a short dependent chain per pivot.
__device__ __forceinline__ double rsq_refined(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    r = r * (1.5 - h * r * r);
    r = r * (1.5 - h * r * r);
    return r;
}
__device__ __forceinline__ float rsq_refined(float x)
{
    float r = __builtin_amdgcn_rsqf(x);
    return r * (1.5f - 0.5f * x * r * r);
}

template <typename T>
__device__ __forceinline__ void diag_block(T *dg, T *li, T *zb, T *dv, const T *yJ, int *flag,
                                           int l, double &ldet, double &quad)
{
    const int i = l & 15;
    T a[16], iv[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) a[c] = dg[i * kGpLd + c];
    bool bad = false;
    double prod = 1.0;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
        const T piv = readlane_t(a[jj], jj);
        const bool ok = piv > T(0);
        bad = bad || !ok;
        const T r = ok ? rsq_refined(piv) : T(1);
        const T ljj = ok ? piv * r : T(1);
        iv[jj] = r;
        prod *= (double)ljj;
        // column jj scaled; rows above jj only touch their unused upper part
        a[jj] = (i == jj) ? ljj : a[jj] * r;
#pragma unroll
        for (int c = jj + 1; c < 16; ++c) a[c] -= a[jj] * readlane_t(a[jj], c);
    }
    ldet += log(prod);
    if (l == 0 && bad) *flag = 1;
    // inverse, one column per lane: x = L^{-1} e_c by forward substitution, L[r][t] taken from
    // lane r's registers (one row's operands in flight at a time)
    const int c = l & 15;
    T x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        T sacc = (r == c) ? T(1) : T(0);
#pragma unroll
        for (int t = 0; t < r; ++t) sacc -= readlane_t(a[t], r) * x[t];
        x[r] = sacc * iv[r];
        __builtin_amdgcn_sched_barrier(0);
    }
    // z_J = L_JJ^{-1} y_J: row sums over the 16 lanes of a DPP row
    const T yc = yJ[c];
    double q2 = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        if (l < 16) li[r * kGpLd + c] = x[r];
        const T zr = row_sum16(x[r] * yc);
        if (l == 0) zb[r] = zr;
        q2 += (double)zr * (double)zr;
    }
    if (l == 0) {
        quad += q2;
#pragma unroll
        for (int r = 0; r < 16; ++r) dv[r] = iv[r];
    }
}

// log N(y; 0, K_theta + sigma_n^2 I) at u = log theta with the factorisation in T.  Called by
// every thread of the workgroup with the same u (the result is uniform); the inputs and
// targets must be staged at kOffXs / kOffYs.  failed = a pivot was not positive.
//
// Waves 0..6 hold the covariance tiles and do the panel and trailing updates; wave 7 factors
// each diagonal tile as soon as its owner has applied the last update to it and published it
// (a one-block look-ahead: the factorisation of block J+1 overlaps the trailing update of
// step J).  The two roles run separate loops with the same barrier count, so the pivot wave's
// code holds none of the tile registers.
template <typename T>
__device__ __forceinline__ double gp_eval(const double *u, int n, unsigned char *smem, bool &failed,
                                          bool &timed_out, int spin_max = kGpSpinMax)
{
    typedef Mf<T> M;
    typedef typename M::v4 v4;
    const double *xs = (const double *)(smem + kOffXs);
    const double *ys = (const double *)(smem + kOffYs);
    double *red = (double *)(smem + kOffMisc);
    int *flag = (int *)(red + 16);
    int *dflag = flag + 1;           // index of the last diagonal tile published to dg
    int *tflag = flag + 2;           // the pivot wave's bounded wait gave up
    double *sc = (double *)(smem + kOffSc);
    T *pan = (T *)(smem + kOffT);
    T *dg = pan + 16 * kTile;
    T *li = dg + kTile;
    T *yb = li + kTile;
    T *zb = yb + kGpMaxObs;
    T *dv = zb + 16;                 // reciprocal pivots of the diagonal tile
    T *far = dv + 16;                // [kGpLdsSlots][kGpTileWaves] LDS-resident tiles
    constexpr bool refine = sizeof(T) == 4;
    // FP32 refinement: L_JJ^{-1} of every block (the factor's inverse diagonal tiles), z,
    // alpha = L^{-T} z, partial products of one block step, one 16-vector
    float *linv = (float *)(far + kGpLdsSlots * kGpTileWaves * kTile);
    float *zall = linv + 16 * kTile;
    float *alpha = zall + kGpMaxObs;
    float *part = alpha + kGpMaxObs;
    float *wv = part + 16 * 16;
    const int tid = threadIdx.x, lane0 = tid & 63, w = uniform_i(tid >> 6);
    const int NT = (n + 15) >> 4, NTT = NT * (NT + 1) / 2;
    const GpTheta h = gp_theta(u);

    for (int i = tid; i < 16 * NT; i += kGpThreads) yb[i] = (i < n) ? (T)ys[i] : T(0);
    for (int i = tid; i < n; i += kGpThreads) {
        double s0, c0, s1, c1;
        sincospi(xs[2 * i] * h.iper, &s0, &c0);
        sincospi(xs[2 * i + 1] * h.iper, &s1, &c1);
        sc[4 * i] = s0; sc[4 * i + 1] = c0; sc[4 * i + 2] = s1; sc[4 * i + 3] = c1;
    }
    if (tid == 0) { *flag = 0; *dflag = -1; *tflag = 0; }
    __syncthreads();

    if (w == kGpPivot) {
        double ldet = 0.0, quad = 0.0;   // lane 0
        for (int J = -1; J < NT; ++J) {
            int l = lane0;
            asm volatile("" : "+v"(l));
            if (J >= 0) __syncthreads();   // the panel step of the tile waves
            const int J1 = J + 1;
            if (J1 < NT) {
                // bounded wait for the diagonal tile; giving up fails this evaluation (log L =
                // -inf) and is reported (spin_max < 0: give up at once, a host-set test mode)
                int spins = 0;
                while (spin_max < 0 ||
                       __hip_atomic_load(dflag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != J1) {
                    if (++spins > spin_max) {
                        if (l == 0) { *flag = 1; *tflag = 1; }
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                diag_block<T>(dg, li, zb, dv, yb + 16 * J1, flag, l, ldet, quad);
                if constexpr (refine) {
                    for (int e = l; e < kTile; e += 64) linv[J1 * kTile + e] = (float)li[e];
                    if (l < 16) zall[16 * J1 + l] = (float)zb[l];
                }
            }
            __syncthreads();
        }
        if (lane0 == 0) {
            red[0] = ldet;
            red[1] = quad;
        }
        if constexpr (refine) {
            // alpha = L^{-T} z, block rows from the last: alpha_J = L_JJ^{-T} (z_J - sum_{I > J}
            // L_IJ^T alpha_I), the products L_IJ^T alpha_I from the tiles' owners
            for (int J = NT - 1; J >= 0; --J) {
                __syncthreads();   // the owners' partial products of step J
                const int l = lane0;
                if (l < 16) {
                    float w = zall[16 * J + l];
                    for (int I = J + 1; I < NT; ++I) w -= part[16 * I + l];
                    wv[l] = w;
                }
                wave_sync();
                if (l < 16) {
                    float a = 0.f;
                    for (int r = l; r < 16; ++r) a += linv[J * kTile + r * kGpLd + l] * wv[r];
                    alpha[16 * J + l] = a;
                }
                __syncthreads();
            }
        }
    } else {
        int tI[kGpSlots], tK[kGpSlots];
        v4 acc[kGpRegSlots];             // slot s >= kGpLdsSlots in acc[s - kGpLdsSlots]
        T *lt[kGpLdsSlots];              // slot s < kGpLdsSlots in LDS
#pragma unroll
        for (int s = 0; s < kGpSlots; ++s) {
            const int t = w + kGpTileWaves * s;
            int I = -1, K = 0;
            if (t < NTT) tile_ik(t, I, K);
            tI[s] = I;
            tK[s] = K;
        }
#pragma unroll
        for (int s = 0; s < kGpLdsSlots; ++s) lt[s] = far + (s * kGpTileWaves + w) * kTile;
#pragma unroll
        for (int s = 0; s < kGpRegSlots; ++s)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[s][r] = T(0);
        {
            // entries of the wave's tiles (a slot's four entries in a loop that is not unrolled,
            // so the exponential's code appears once per slot)
            const int l = lane0;
#pragma unroll
            for (int s = 0; s < kGpSlots; ++s) {
                const int t = w + kGpTileWaves * s;
                if (t < NTT) {
                    int I, K;
                    tile_ik(t, I, K);
                    const int col = 16 * K + (l & 15);
                    if (s < kGpLdsSlots) {
#pragma unroll 1
                        for (int r = 0; r < 4; ++r)
                            lt[s][M::row(l, r) * kGpLd + (l & 15)] =
                                gp_entry<T>(xs, sc, n, 16 * I + M::row(l, r), col, h);
                    } else {
#pragma unroll 1
                        for (int r = 0; r < 4; ++r)
                            acc[s - kGpLdsSlots][r] =
                                gp_entry<T>(xs, sc, n, 16 * I + M::row(l, r), col, h);
                    }
                }
            }
        }
        for (int J = -1; J < NT; ++J) {
            // the lane index, opaque to the compiler inside each iteration: keeps the many
            // lane-derived masks and LDS addresses of the unrolled code below from being
            // hoisted out of the loop, where they would hold registers across all of it
            int l = lane0;
            asm volatile("" : "+v"(l));
            if (J >= 0) {
                // panel: L_IJ = A_IJ L_JJ^{-T}, and y_I -= L_IJ z_J
#pragma unroll
                for (int s = 0; s < kGpSlots; ++s) {
                    if (tK[s] == J && tI[s] > J) {
                        T *pI = pan + tI[s] * kTile;
                        v4 a;
                        if (s < kGpLdsSlots) load_tile<T>(a, lt[s], l);
                        else a = acc[s - kGpLdsSlots];
                        store_tile<T>(a, pI, l);
                        wave_sync();
                        v4 o;
#pragma unroll
                        for (int r = 0; r < 4; ++r) o[r] = T(0);
#pragma unroll
                        for (int ks = 0; ks < 4; ++ks) {
                            const int ko = (l & 15) * kGpLd + 4 * ks + (l >> 4);
                            o = M::mma(pI[ko], li[ko], o);
                        }
                        wave_sync();
                        store_tile<T>(o, pI, l);
                        if constexpr (refine) {   // the factor's tile, kept for the solve
                            if (s < kGpLdsSlots) store_tile<T>(o, lt[s], l);
                            else acc[s - kGpLdsSlots] = o;
                        }
                        const T zc = zb[l & 15];
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const T sr = row_sum16(o[r] * zc);
                            if ((l & 15) == 0) yb[16 * tI[s] + M::row(l, r)] -= sr;
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                __syncthreads();
            }
            // trailing update A_IK -= L_IJ L_KJ^T for J < K <= I; the next diagonal tile first,
            // published to the pivot wave as soon as it is final
            const int J1 = J + 1;
            const int tD = J1 * (J1 + 1) / 2 + J1;
            if (J1 < NT && w == tD % kGpTileWaves) {
                const T *pD = pan + J1 * kTile;
#pragma unroll
                for (int s = 0; s < kGpSlots; ++s) {
                    if (w + kGpTileWaves * s == tD) {
                        v4 a;
                        if (s < kGpLdsSlots) load_tile<T>(a, lt[s], l);
                        else a = acc[s - kGpLdsSlots];
                        if (J >= 0) {
#pragma unroll
                            for (int ks = 0; ks < 4; ++ks) {
                                const int ko = (l & 15) * kGpLd + 4 * ks + (l >> 4);
                                a = M::mma(-pD[ko], pD[ko], a);
                            }
                        }
                        store_tile<T>(a, dg, l);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (l == 0) __hip_atomic_store(dflag, J1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            if (J >= 0) {
#pragma unroll
                for (int s = 0; s < kGpSlots; ++s) {
                    if (tK[s] > J && w + kGpTileWaves * s != tD) {
                        const T *pI = pan + tI[s] * kTile, *pK = pan + tK[s] * kTile;
                        v4 a;
                        if (s < kGpLdsSlots) load_tile<T>(a, lt[s], l);
                        else a = acc[s - kGpLdsSlots];
#pragma unroll
                        for (int ks = 0; ks < 4; ++ks) {
                            const int ko = (l & 15) * kGpLd + 4 * ks + (l >> 4);
                            a = M::mma(-pI[ko], pK[ko], a);
                        }
                        if (s < kGpLdsSlots) store_tile<T>(a, lt[s], l);
                        else acc[s - kGpLdsSlots] = a;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            __syncthreads();
        }
        if constexpr (refine) {
            for (int J = NT - 1; J >= 0; --J) {
                int l = lane0;
                asm volatile("" : "+v"(l));
                // the partial products L_IJ^T alpha_I of this wave's tiles (I, J), I > J
#pragma unroll
                for (int s = 0; s < kGpSlots; ++s) {
                    if (tK[s] == J && tI[s] > J) {
                        v4 a;
                        if (s < kGpLdsSlots) load_tile<T>(a, lt[s], l);
                        else a = acc[s - kGpLdsSlots];
                        float v = 0.f;
#pragma unroll
                        for (int r = 0; r < 4; ++r) v += (float)a[r] * alpha[16 * tI[s] + M::row(l, r)];
                        v += __shfl_xor(v, 16, 64);
                        v += __shfl_xor(v, 32, 64);
                        if (l < 16) part[16 * tI[s] + l] = v;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
                __syncthreads();
                __syncthreads();   // alpha_J from the pivot wave
            }
        }
    }
    __syncthreads();
    const double ld = red[0];
    double q = red[1];
    failed = (*flag != 0);
    timed_out = (*tflag != 0);
    if constexpr (refine) {
        // y^T K^{-1} y from the FP32 solve alpha, with the entries in FP64:
        // 2 y^T alpha - alpha^T K alpha = y^T K^{-1} y - |alpha - K^{-1} y|_K^2, exact up to a
        // term of second order in the solve's error
        double s2 = 0.0;
        const int ne = n * (n + 1) / 2;
        for (int e = tid; e < ne; e += kGpThreads) {
            int i = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
            while (i * (i + 1) / 2 > e) --i;
            while ((i + 1) * (i + 2) / 2 <= e) ++i;
            const int jj = e - i * (i + 1) / 2;
            const double kij = gp_entry<double>(xs, sc, n, i, jj, h);
            const double t = (double)alpha[i] * (double)alpha[jj] * kij;
            s2 += (i == jj) ? t : 2.0 * t;
        }
        for (int i = tid; i < n; i += kGpThreads) s2 -= 2.0 * ys[i] * (double)alpha[i];
        s2 = wave_sum(s2);
        __syncthreads();
        if ((tid & 63) == 0) red[2 + w] = s2;
        __syncthreads();
        double qv = 0.0;
#pragma unroll
        for (int v = 0; v < kGpWaves; ++v) qv -= red[2 + v];
        q = qv;
    }
    __syncthreads();   // the LDS slots are reused by the next evaluation
    return -0.5 * q - ld - 0.5 * (double)n * LOG_2PI;
}

__device__ __forceinline__ void gp_stage(const DevProblem &P, unsigned char *smem)
{
    double *xs = (double *)(smem + kOffXs);
    double *ys = (double *)(smem + kOffYs);
    for (int i = threadIdx.x; i < 2 * P.gp_n; i += blockDim.x) xs[i] = P.gp_x[i];
    for (int i = threadIdx.x; i < P.gp_n; i += blockDim.x) ys[i] = P.gp_y[i];
}

// Mixed precision: the FP32 estimate decides unless it lies within this band of L*; then (and
// when the FP32 factorisation breaks down) the FP64 value decides.  After the refinement the
// error is that of the FP32 log-determinant, which grows with the condition number, bounded
// by n s with s = (sigma_f^2 + sigma_n^2) / sigma_n^2 (the noise floor bounds the smallest
// eigenvalue of the covariance, its trace the largest).  Beyond n s = kGpMaxCond the FP32
// factor is not trusted and the FP64 value decides.
constexpr double kGpMaxCond = 1e5;
__device__ __forceinline__ double gp_cond(const DevProblem &P, const double *u)
{
    const double sf2 = exp(2.0 * u[0]), sn2 = exp(2.0 * u[5]);
    return (sf2 + sn2) / sn2 * (double)P.gp_n;
}
// beyond the bound the candidate is evaluated in FP64 only (no FP32 attempt)
__device__ __forceinline__ bool gp_illcond(const DevProblem &P, const double *u)
{
    return !(gp_cond(P, u) <= kGpMaxCond);
}
__device__ __forceinline__ bool gp_near(double L32, double Lstar, const DevProblem &P,
                                        const double *u)
{
    const double cond = gp_cond(P, u);
    if (!(cond <= kGpMaxCond)) return true;
    const double band = (double)P.guard_rel * fabs(L32) + (double)P.guard_abs +
                        (double)P.guard_kappa * cond;
    return !(fabs(L32 - Lstar) > band);
}

}  // namespace

template <int MODE>
__global__ __launch_bounds__(kGpThreads) void k_eval_gp(Launch Lc, const double *X, int ld, int n,
                                                        double *out, int from_run)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bm = Lc.map[blockIdx.x];
    const DevProblem P = Lc.P[bm.x];
    const DevRun R = Lc.R[bm.x];
    unsigned long long *nonfinite = nullptr;
    if (from_run) { X = R.X; ld = R.m_pad; n = R.m; out = R.logL; nonfinite = R.ctr + 5; }
    const int i = bm.y;
    if (i >= n) return;
    gp_stage(P, smem);
    double u[kGpD];
#pragma unroll
    for (int a = 0; a < kGpD; ++a) u[a] = X[(size_t)a * ld + i];
    __syncthreads();
    bool failed = false, timed_out = false;
    double L;
    if constexpr (MODE == MODE_FP64) L = gp_eval<double>(u, P.gp_n, smem, failed, timed_out);
    else L = gp_eval<float>(u, P.gp_n, smem, failed, timed_out);
    if (timed_out && from_run && threadIdx.x == 0) atomicAdd(&R.ctr[10], 1ull);
    if (threadIdx.x == 0) {
        unsigned long long nf = 0;
        out[i] = failed ? -INFINITY : sanitize(L, nf);
        if (nf && nonfinite) atomicAdd(nonfinite, nf);
    }
}

template <int MODE>
__global__ __launch_bounds__(kGpThreads) void k_hrss_gp(Launch Lc)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bm = Lc.map[blockIdx.x];
    const DevProblem P = Lc.P[bm.x];
    const DevRun R = Lc.R[bm.x];
    if (R.iscal[0] || R.iscal[2] <= 0) return;
    const int j = bm.y;
    if (j >= R.k) return;
    const int tid = threadIdx.x, n = P.gp_n;
    double *sx0 = (double *)(smem + kOffChain);   // current point of the chain
    double *sv = sx0 + 8;                         // direction of the current step
    gp_stage(P, smem);
    const double Lstar = R.scal[0];
    const int t0 = R.iscal[1], nsurv = R.iscal[2];
    const uint32_t it = (uint32_t)R.iscal[3] + 1u;
    const double width = R.width;
    const int p = R.p, cap_out = R.stepout_cap, cap_sh = R.shrink_cap;
    const bool box = (P.prior_kind == PRIOR_BOX);

    double ur, unused;
    draw2(R.key0, R.key1, PUR_RESAMPLE, (uint32_t)j, it, 0u, 0u, ur, unused);
    int qi = (int)floor(ur * (double)nsurv);
    if (qi > nsurv - 1) qi = nsurv - 1;
    const int parent = R.perm[t0 + qi];
    if (tid == 0) R.parents[j] = parent;
    if (tid < kGpD) sx0[tid] = R.X[(size_t)tid * R.m_pad + parent];
    double logL0 = R.logL[parent];
    bool exact0 = true;
    // counters (every thread keeps identical copies; thread 0 publishes them)
    unsigned long long c_evals = 0, c_tests = 0, c_prej = 0, c_outcap = 0, c_shcap = 0,
                       c_nonfin = 0, c_rc = 0, c_viol = 0, c_wait = 0;
    const int spin_max = P.gp_spin_max;
    __syncthreads();

    // log prior density (Gaussian prior; the box prior is uniform on its support)
    auto logprior = [&](const double *x) -> double {
        double lp = 0.0;
#pragma unroll
        for (int a = 0; a < kGpD; ++a) {
            const double zt = (x[a] - P.pa[a]) / P.pb[a];
            lp += -0.5 * zt * zt;
        }
        return lp + P.logprior_norm;
    };

    // The chain as one loop with a single evaluation site (the evaluator is large and fully
    // inlined): each pass picks the next test of the current phase, evaluates it and advances.
    enum { PH_NEW = 0, PH_LEFT = 1, PH_RIGHT = 2, PH_SHRINK = 3, PH_FINAL = 4 };
    int phase = PH_NEW, st = 0, nl = 0, nr = 0, ns = 0;
    double tL = 0.0, tR = 0.0, logy = -INFINITY;
    for (;;) {
        if (phase == PH_NEW) {
            if (st == p) {
                if (MODE == MODE_FP64 || exact0) break;
                phase = PH_FINAL;   // stored log-likelihoods are FP64
                __syncthreads();    // the last accepted point is in sx0 for every wave
            } else {
                __syncthreads();   // every thread is done with the previous direction
                if (tid == 0) {
                    // direction z ~ N(0, I), v = Lsig z / |z|
                    double z[kGpD];
#pragma unroll
                    for (int q = 0; q < kGpD / 2; ++q) {
                        double ua, ub;
                        draw2(R.key0, R.key1, PUR_DIR, (uint32_t)j, it, (uint32_t)st,
                              (uint32_t)q, ua, ub);
                        box_muller(ua, ub, z[2 * q], z[2 * q + 1]);
                    }
                    double nz = 0.0;
#pragma unroll
                    for (int a = 0; a < kGpD; ++a) nz += z[a] * z[a];
                    nz = sqrt(nz);
                    for (int a = 0; a < kGpD; ++a) {
                        double s2 = 0.0;
                        for (int b = 0; b <= a; ++b) s2 += R.Lsig[a * P.D + b] * z[b];
                        sv[a] = s2 / nz;
                    }
                }
                __syncthreads();
                double U, uh;
                draw2(R.key0, R.key1, PUR_STEP, (uint32_t)j, it, (uint32_t)st, 0u, U, uh);
                logy = box ? -INFINITY : logprior(sx0) + log(uh);
                tL = -width * U;
                tR = tL + width;
                nl = nr = ns = 0;
                phase = PH_LEFT;
                continue;
            }
        }
        double t = 0.0;
        if (phase == PH_LEFT) {
            if (nl >= cap_out) { ++c_outcap; phase = PH_RIGHT; continue; }
            t = tL;
        } else if (phase == PH_RIGHT) {
            if (nr >= cap_out) { ++c_outcap; phase = PH_SHRINK; continue; }
            t = tR;
        } else if (phase == PH_SHRINK) {
            if (ns >= cap_sh) {
                // null move
                ++c_shcap;
                if (R.trace && tid == 0) {
                    int *tr = R.trace + ((size_t)j * p + st) * 4;
                    tr[0] = nl; tr[1] = nr; tr[2] = ns; tr[3] = 0;
                }
                ++st;
                phase = PH_NEW;
                continue;
            }
            double us, un2;
            draw2(R.key0, R.key1, PUR_SHRINK, (uint32_t)j, it, (uint32_t)st, (uint32_t)ns, us, un2);
            t = tL + us * (tR - tL);
        }
        double y[kGpD];
#pragma unroll
        for (int a = 0; a < kGpD; ++a) y[a] = (phase == PH_FINAL) ? sx0[a] : sx0[a] + t * sv[a];
        bool in = true;
        if (phase != PH_FINAL) {
            ++c_tests;
            if (box) {
#pragma unroll
                for (int a = 0; a < kGpD; ++a) in = in && (y[a] >= P.pa[a] && y[a] <= P.pb[a]);
            } else {
                in = logprior(y) > logy;
            }
        }
        bool r = false, exact = true;
        double L = -INFINITY;
        if (!in) {
            ++c_prej;
        } else {
            // the single evaluation site
            bool failed = false, tout = false;
            if constexpr (MODE == MODE_FP64) {
                L = gp_eval<double>(y, n, smem, failed, tout, spin_max);
                c_wait += tout;
            } else {
                bool need64 = (phase == PH_FINAL);
                if (!need64 && gp_illcond(P, y)) {   // FP64 only, no FP32 attempt
                    need64 = true;
                    ++c_rc;
                } else if (!need64) {
                    L = gp_eval<float>(y, n, smem, failed, tout, spin_max);
                    c_wait += tout;
                    need64 = (failed && !tout) || !(L == L) || gp_near(L, Lstar, P, y);
                    if (need64) ++c_rc; else exact = false;
                }
                if (need64) {
                    L = gp_eval<double>(y, n, smem, failed, tout, spin_max);
                    c_wait += tout;
                }
            }
            if (failed) L = -INFINITY;
            if (phase == PH_FINAL) {
                logL0 = L;
                if (!(logL0 > Lstar)) ++c_viol;
                break;
            }
            ++c_evals;
            L = sanitize(L, c_nonfin);
            r = L > Lstar;
        }
        if (phase == PH_LEFT) {
            if (r) { tL -= width; ++nl; } else phase = PH_RIGHT;
        } else if (phase == PH_RIGHT) {
            if (r) { tR += width; ++nr; } else phase = PH_SHRINK;
        } else {
            ++ns;
            if (r) {
                // every thread has passed the evaluation's barriers: sx0 is free to update
                if (tid < kGpD) sx0[tid] = y[tid];
                logL0 = L;
                exact0 = exact;
                if (R.trace && tid == 0) {
                    int *tr = R.trace + ((size_t)j * p + st) * 4;
                    tr[0] = nl; tr[1] = nr; tr[2] = ns; tr[3] = 1;
                }
                ++st;
                phase = PH_NEW;
            } else if (t < 0.0) {
                tL = t;
            } else {
                tR = t;
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        const int slot = R.perm[j];
#pragma unroll
        for (int a = 0; a < kGpD; ++a) R.X[(size_t)a * R.m_pad + slot] = sx0[a];
        R.logL[slot] = logL0;
        atomicAdd(&R.ctr[0], c_evals);
        atomicAdd(&R.ctr[1], c_tests);
        atomicAdd(&R.ctr[2], c_prej);
        atomicAdd(&R.ctr[3], c_outcap);
        atomicAdd(&R.ctr[4], c_shcap);
        atomicAdd(&R.ctr[5], c_nonfin);
        atomicAdd(&R.ctr[6], c_rc);
        atomicAdd(&R.ctr[7], c_viol);
        if (c_wait) atomicAdd(&R.ctr[10], c_wait);
    }
}

template <typename F>
static hipError_t gp_lds(F *f, size_t bytes)
{
    return hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

hipError_t launch_hrss_gp(const Launch &L, int mode, hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    const size_t lds = (size_t)gp_lds_bytes<double>();
    if (mode == MODE_FP64) {
        hipError_t e = gp_lds(k_hrss_gp<MODE_FP64>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_hrss_gp<MODE_FP64>, dim3(L.nblocks), dim3(kGpThreads), lds, s, L);
    } else if (mode == MODE_FP32) {
        hipError_t e = gp_lds(k_hrss_gp<MODE_FP32>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_hrss_gp<MODE_FP32>, dim3(L.nblocks), dim3(kGpThreads), lds, s, L);
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

hipError_t launch_eval_gp(const Launch &L, int mode, const double *X, int ld, int n, double *out,
                          int from_run, hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    const size_t lds = (size_t)gp_lds_bytes<double>();
    if (mode == MODE_FP64) {
        hipError_t e = gp_lds(k_eval_gp<MODE_FP64>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_eval_gp<MODE_FP64>, dim3(L.nblocks), dim3(kGpThreads), lds, s, L, X,
                           ld, n, out, from_run);
    } else if (mode == MODE_FP32) {
        hipError_t e = gp_lds(k_eval_gp<MODE_FP32>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_eval_gp<MODE_FP32>, dim3(L.nblocks), dim3(kGpThreads), lds, s, L, X,
                           ld, n, out, from_run);
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

}  // namespace nss
