// Evaluation tiles shared by the gfx950 chain kernels: the LDS layout of a chain workgroup,
// the staged problem constants, and the batched likelihood tiles (FP64 mixture on FP64 MFMA,
// 16-bit mixture on BF16 / FP16 MFMA with the guard band, funnel, Gaussian-Rastrigin).
#pragma once
#include "nss_internal.hpp"
#include "nss_wave.hpp"

#include <math.h>

namespace nss {

// ------------------------------------------------------------------------------------------
// LDS layout of the chain / evaluation workgroups (byte offsets; identical on host)
// ------------------------------------------------------------------------------------------
struct HLayout {
    int z, cand, cand32, mu64, mu32, cst, cst32, pa, pb, L, L32, mask, rc, q, q32, lsig,
        total;
};
__host__ __device__ inline int al16(int b) { return (b + 15) & ~15; }
// direction factor in LDS: dense rows of stride D+1 (conflict-free column reads) up to D = 64,
// packed lower triangle for D = 128
__host__ __device__ inline int lsig_doubles(int D) { return D <= 64 ? D * (D + 1) : D * (D + 1) / 2; }
// partial quadratic forms of a tile: q[row * q_stride + (c * D/16 + jb) * 4 + g], one value per
// (candidate row, component, column block, lane group g); the row stride is padded by 4
__host__ __device__ inline int q_stride(int D, int K) { return (K > 0 ? K : 1) * (D / 16) * 4 + 4; }
__host__ __device__ inline HLayout hrss_layout(int D, int K)
{
    const int Kc = K > 0 ? K : 1;
    HLayout o;
    int off = 0;
    o.z = off; off += al16(4 * D * 8);
    o.cand = off; off += al16(kRows * (D + 1) * 8);
    o.cand32 = off; off += al16(kRows * (D + 4) * 4);
    o.mu64 = off; off += al16(Kc * D * 8);
    o.mu32 = off; off += al16(Kc * D * 4);
    o.cst = off; off += al16(Kc * 8);
    o.cst32 = off; off += al16(Kc * 4);
    o.pa = off; off += al16(D * 8);
    o.pb = off; off += al16(D * 8);
    o.L = off; off += al16(kRows * 8);
    o.L32 = off; off += al16(kRows * 4);
    o.mask = off; off += al16(kRows * 4);
    o.rc = off; off += al16(kRows * 4);
    o.q = off; off += al16(kRows * q_stride(D, K) * 8);
    o.q32 = off; off += al16(kRows * q_stride(D, K) * 4);
    // the factor is staged only for chains that draw their own directions (D <= 128)
    o.lsig = off; off += D <= 128 ? al16(lsig_doubles(D) * 8) : 0;
    o.total = off;
    return o;
}

// LDS views of one workgroup's evaluation tile and the problem constants it stages.
struct Tile {
    double *cand;        // [16][D+1] candidate rows, FP64
    float *cand32;       // [16][D+4] candidate rows, FP32 (mixed precision)
    double *mu64;        // [K][D]
    float *mu32;         // [K][D]
    double *cst;         // [K] log w_c - d/2 log(2 pi) + log det W_c
    float *cst32;
    double *pa, *pb;     // prior parameters, [D]
    double *L;           // [16] FP64 results
    float *L32;          // [16] FP32 results
    int *mask;           // [16] rows to evaluate
    int *rc;             // [16] rows to re-check in FP64
    double *q;           // [16][q_stride] partial quadratic forms
    float *q32;
};
__device__ __forceinline__ Tile tile_of(unsigned char *smem, const HLayout &lay)
{
    Tile t;
    t.cand = (double *)(smem + lay.cand);
    t.cand32 = (float *)(smem + lay.cand32);
    t.mu64 = (double *)(smem + lay.mu64);
    t.mu32 = (float *)(smem + lay.mu32);
    t.cst = (double *)(smem + lay.cst);
    t.cst32 = (float *)(smem + lay.cst32);
    t.pa = (double *)(smem + lay.pa);
    t.pb = (double *)(smem + lay.pb);
    t.L = (double *)(smem + lay.L);
    t.L32 = (float *)(smem + lay.L32);
    t.mask = (int *)(smem + lay.mask);
    t.rc = (int *)(smem + lay.rc);
    t.q = (double *)(smem + lay.q);
    t.q32 = (float *)(smem + lay.q32);
    return t;
}
// Copy the problem constants into LDS (caller synchronises).
template <int D>
__device__ __forceinline__ void stage_problem(const DevProblem &P, const Tile &T)
{
    const int tid = threadIdx.x;
    for (int i = tid; i < P.K * D; i += blockDim.x) { T.mu64[i] = P.mu[i]; T.mu32[i] = P.mu32[i]; }
    for (int i = tid; i < P.K; i += blockDim.x) { T.cst[i] = P.cst[i]; T.cst32[i] = P.cst32[i]; }
    for (int i = tid; i < D; i += blockDim.x) { T.pa[i] = P.pa[i]; T.pb[i] = P.pb[i]; }
}

// ------------------------------------------------------------------------------------------
// Likelihood tiles.  16 candidate rows live in LDS; mask[r] != 0 marks rows to evaluate.
// All 256 threads call these; they end with a barrier, after which out[r] holds log L of
// every masked row.
//
// Mixture work unit = (component c, 16-column block jb of W_c^T), W_c the inverse of the lower
// Cholesky factor of cov_c, so the quadratic form is |W_c (x - mu_c)|^2 and W_c is lower
// triangular: block jb needs k <= 16 jb + 15 only.  Units are dealt to the four waves so that
// each wave gets the same mix of short and long blocks: wave w's uu-th unit is
//   D/16 = 2: u = w + 4 uu (c = u/2, jb = u%2);
//   D/16 = 4: c = uu, jb = (w - uu) mod 4;
//   D/16 = 8: c = uu/2, jb = kk or 7 - kk with kk = (w - c) mod 4.
// ------------------------------------------------------------------------------------------
// With K >= 4 components, wave w instead takes whole components c = w, w+4, ... (all their
// column blocks): the residual of a component is then converted once per wave and shared by its
// blocks, and every wave still gets the same triangular work.  uu = (c - w)/4 * D/16 + jb.
__device__ __forceinline__ bool comp_major(int K) { return K >= 4; }
// The same for the register-fragment tiles of the mixed modes, decided at compile time where the
// fragment capacity is only used with K >= 4 (D = 64 with 8 units per wave holds K = 5..8,
// D = 32 with 16 units K = 9..32), so the fragments that the dealing never reads are dropped.
template <int D, int UPW>
__device__ __forceinline__ bool comp_major_t(int K)
{
    if constexpr ((D == 64 && UPW == 8) || (D == 32 && UPW == 16)) return true;
    else return K >= 4;
}

template <int NJB>
__device__ __forceinline__ void unit_of_cm(int w, int uu, int &c, int &jb)
{
    c = w + 4 * (uu / NJB);
    jb = uu % NJB;
}

template <int NJB>
__device__ __forceinline__ void unit_of(int w, int uu, int &c, int &jb)
{
    if constexpr (NJB == 2) {
        const int u = w + 4 * uu;
        c = u >> 1;
        jb = u & 1;
    } else if constexpr (NJB == 4) {
        c = uu;
        jb = (w - uu) & 3;
    } else {
        c = uu >> 1;
        const int kk = (w - c) & 3;
        jb = (uu & 1) ? 7 - kk : kk;
    }
}

// log L = LSE_c (cst_c - q_c / 2) from the partials.  Wave w handles rows 4w..4w+3: the lanes
// of DPP row rr take row 4w+rr, lane c of the row takes components c, c+16, ...
template <int D, typename F>
__device__ __forceinline__ F lse_rows(const DevProblem &P, const F *q, const F *cst, int r, int c)
{
    constexpr int NJB = D / 16;
    const int QS = q_stride(D, P.K);
    F mx = -INFINITY, se = 0;
    for (int c0 = 0; c0 < P.K; c0 += 16) {
        const int cc = c0 + c;
        F t = -INFINITY;
        if (cc < P.K) {
            const F *src = q + r * QS + cc * NJB * 4;
            F s = 0;
#pragma unroll
            for (int i = 0; i < NJB * 4; ++i) s += src[i];
            t = cst[cc] - (F)0.5 * s;
        }
        const F m = row_max16(t);
        F e;
        if constexpr (sizeof(F) == 8) e = (cc < P.K && m != -INFINITY) ? exp(t - m) : 0.0;
        else e = (cc < P.K && m != -INFINITY) ? __expf(t - m) : 0.f;
        e = row_sum16(e);
        if (m > mx) {
            if constexpr (sizeof(F) == 8) se = se * exp(mx - m) + e;
            else se = se * __expf(mx - m) + e;
            mx = m;
        } else if (m != -INFINITY) {
            if constexpr (sizeof(F) == 8) se += e * exp(m - mx);
            else se += e * __expf(m - mx);
        }
    }
    if (mx == -INFINITY) return -INFINITY;
    if constexpr (sizeof(F) == 8) return mx + log(se);
    else return mx + __logf(se);
}

// FP64 mixture tile on v_mfma_f64_16x16x4 with W as the A operand and the residuals as B:
// D[j][n] = sum_k W_c[16 jb + j][k] (x_n - mu_c)[k], so lane l, register i holds
// y[n = l & 15][16 jb + (l >> 4) + 4 i]; its four squares sum to one partial per lane group.
// The unit's B fragments (pre-swizzled, 512 contiguous bytes per k-step) are requested
// before the first product so their L2 latencies overlap.
template <int D>
__device__ void mix_eval64(const DevProblem &P, const Tile &T, const int *mask, double *out)
{
    constexpr int NJB = D / 16, NKS = D / 4, LDC = D + 1;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int row = l & 15, kq = l >> 4;
    const int QS = q_stride(D, P.K);
    const bool on = mask[row] != 0;
    const double *cr = T.cand + row * LDC;
    if constexpr (D <= 64) {
        if (comp_major(P.K)) {
            for (int c = w; c < P.K; c += 4) {
                const double *wf = P.wf64 + (size_t)c * NJB * NKS * 64 + l;
                const double *mu = T.mu64 + c * D;
                d4 acc[NJB];
#pragma unroll
                for (int jb = 0; jb < NJB; ++jb) acc[jb] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks) {
                    const int kk = 4 * ks + kq;
                    const double b = on ? cr[kk] - mu[kk] : 0.0;
#pragma unroll
                    for (int jb = 0; jb < NJB; ++jb)
                        if (ks < 4 * jb + 4)
                            acc[jb] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                wf[((size_t)jb * NKS + ks) * 64], b, acc[jb], 0, 0, 0);
                }
#pragma unroll
                for (int jb = 0; jb < NJB; ++jb)
                    T.q[row * QS + (c * NJB + jb) * 4 + kq] =
                        (acc[jb][0] * acc[jb][0] + acc[jb][1] * acc[jb][1]) +
                        (acc[jb][2] * acc[jb][2] + acc[jb][3] * acc[jb][3]);
            }
            __syncthreads();
            {
                const int r = 4 * w + (l >> 4), c = l & 15;
                const double L = lse_rows<D, double>(P, T.q, T.cst, r, c);
                if (c == 0) out[r] = L;
            }
            __syncthreads();
            return;
        }
    }
    for (int uu = 0;; ++uu) {
        int c, jb;
        unit_of<NJB>(w, uu, c, jb);
        if (c >= P.K) break;
        const int u = c * NJB + jb;
        const int ke = (4 * jb + 4 < NKS) ? 4 * jb + 4 : NKS;
        const double *wf = P.wf64 + (size_t)u * NKS * 64 + l;
        double bfr[NKS];
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) bfr[ks] = (ks < ke) ? wf[ks * 64] : 0.0;
        const double *mu = T.mu64 + c * D;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            if (ks < ke) {
                const int kk = 4 * ks + kq;
                const double b = on ? cr[kk] - mu[kk] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(bfr[ks], b, acc, 0, 0, 0);
            }
        }
        T.q[row * QS + u * 4 + kq] = (acc[0] * acc[0] + acc[1] * acc[1]) + (acc[2] * acc[2] + acc[3] * acc[3]);
    }
    __syncthreads();
    {
        const int r = 4 * w + (l >> 4), c = l & 15;
        const double L = lse_rows<D, double>(P, T.q, T.cst, r, c);
        if (c == 0) out[r] = L;
    }
    __syncthreads();
}

template <int MODE> struct MixTraits;
template <> struct MixTraits<MODE_BF16> { typedef __bf16 H; typedef bf8 V8; static constexpr int NP = 1; };
template <> struct MixTraits<MODE_FP16> { typedef _Float16 H; typedef h8 V8; static constexpr int NP = 1; };
template <> struct MixTraits<MODE_BF16X3> { typedef __bf16 H; typedef bf8 V8; static constexpr int NP = 2; };
template <> struct MixTraits<MODE_FP16X3> { typedef _Float16 H; typedef h8 V8; static constexpr int NP = 2; };

__device__ __forceinline__ f4 mfma16(bf8 a, bf8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(h8 a, h8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Register-resident 16-bit W fragments of one wave: v[0] = rounded W, v[1] = W - v[0] rounded
// (split-precision modes only).
template <int D, int UPW, int NP>
struct WFrag { uint4 v[NP][UPW][D / 32]; };

// Guard band of the mixed modes: a row whose FP32 estimate L has
// |L - L*| <= rel * max(0, cmax - L) + abs + 1e-6 |L| is re-evaluated in FP64.
struct Guard {
    double Lstar;
    float rel, abs, cmax;
};
__device__ __forceinline__ bool near_threshold(const Guard &g, float L)
{
    if (L != L) return true;
    const float band = g.rel * fmaxf(0.f, g.cmax - L) + g.abs + 1e-6f * fabsf(L);
    return fabs((double)L - g.Lstar) <= (double)band;
}

// Mixed-precision mixture tile: residuals x - mu_c in FP32 rounded to 16 bits (split into a
// rounded part and the rounded remainder in the split modes), times the 16-bit W_c fragments on
// v_mfma_f32_16x16x32_{bf16,f16} with FP32 accumulation (W as A, residuals as B, lane l,
// register i = y[n = l & 15][16 jb + 4 (l >> 4) + i]); the split modes form
// W_hi r_hi + W_hi r_lo + W_lo r_hi.  FP32 squares and log-sum-exp.  Every row is computed
// (rows outside the mask hold stale finite data and are never read).  Rows inside the mask
// whose estimate is near L* get rc[r] = 1; returns whether any row did (the vote is the
// tile's final barrier).
template <int D, int UPW, int MODE>
__device__ int mix_eval16(const DevProblem &P, const WFrag<D, UPW, MixTraits<MODE>::NP> &wr,
                          const Tile &T, const int *mask, float *out, const Guard &g)
{
    typedef typename MixTraits<MODE>::H H;
    typedef typename MixTraits<MODE>::V8 V8;
    constexpr int NP = MixTraits<MODE>::NP;
    constexpr int NJB = D / 16, NKS = D / 32, LDC = D + 4;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int row = l & 15, kq = l >> 4;
    const int QS = q_stride(D, P.K);
    // this lane's candidate coordinates, read once for all units
    float cx[NKS][8];
    {
        const float *cr = T.cand32 + row * LDC;
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            const float4 c0 = *(const float4 *)(cr + 32 * ks + 8 * kq);
            const float4 c1 = *(const float4 *)(cr + 32 * ks + 8 * kq + 4);
            cx[ks][0] = c0.x; cx[ks][1] = c0.y; cx[ks][2] = c0.z; cx[ks][3] = c0.w;
            cx[ks][4] = c1.x; cx[ks][5] = c1.y; cx[ks][6] = c1.z; cx[ks][7] = c1.w;
        }
    }
    if (comp_major_t<D, UPW>(P.K)) {
        constexpr int CW = (UPW + NJB - 1) / NJB;
#pragma unroll
        for (int cw = 0; cw < CW; ++cw) {
            const int c = w + 4 * cw;
            if (c < P.K) {
                const float *mu = T.mu32 + c * D + 8 * kq;
                f4 acc[NJB];
#pragma unroll
                for (int jb = 0; jb < NJB; ++jb) acc[jb] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks) {
                    const float4 m0 = *(const float4 *)(mu + 32 * ks);
                    const float4 m1 = *(const float4 *)(mu + 32 * ks + 4);
                    const float mm[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
                    float rr[8];
                    V8 hi, lo;
#pragma unroll
                    for (int e = 0; e < 8; ++e) { rr[e] = cx[ks][e] - mm[e]; hi[e] = (H)rr[e]; }
                    if constexpr (NP == 2) {
#pragma unroll
                        for (int e = 0; e < 8; ++e) lo[e] = (H)(rr[e] - (float)hi[e]);
                    }
#pragma unroll
                    for (int jb = 0; jb < NJB; ++jb) {
                        if (ks < (16 * jb + 16 + 31) / 32 && cw * NJB + jb < UPW) {
                            const V8 w0 = __builtin_bit_cast(V8, wr.v[0][cw * NJB + jb][ks]);
                            acc[jb] = mfma16(w0, hi, acc[jb]);
                            if constexpr (NP == 2) {
                                acc[jb] = mfma16(w0, lo, acc[jb]);
                                acc[jb] = mfma16(__builtin_bit_cast(V8, wr.v[1][cw * NJB + jb][ks]),
                                                 hi, acc[jb]);
                            }
                        }
                    }
                }
#pragma unroll
                for (int jb = 0; jb < NJB; ++jb)
                    T.q32[row * QS + (c * NJB + jb) * 4 + kq] =
                        (acc[jb][0] * acc[jb][0] + acc[jb][1] * acc[jb][1]) +
                        (acc[jb][2] * acc[jb][2] + acc[jb][3] * acc[jb][3]);
            }
        }
    } else {
#pragma unroll
    for (int uu = 0; uu < UPW; ++uu) {
        int c, jb;
        unit_of<NJB>(w, uu, c, jb);
        if (c < P.K) {
            const int u = c * NJB + jb;
            const int ke = (16 * jb + 16 + 31) / 32;
            const float *mu = T.mu32 + c * D + 8 * kq;
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
                if (ks < ke) {
                    const float4 m0 = *(const float4 *)(mu + 32 * ks);
                    const float4 m1 = *(const float4 *)(mu + 32 * ks + 4);
                    const float mm[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
                    float rr[8];
                    V8 hi;
#pragma unroll
                    for (int e = 0; e < 8; ++e) { rr[e] = cx[ks][e] - mm[e]; hi[e] = (H)rr[e]; }
                    const V8 w0 = __builtin_bit_cast(V8, wr.v[0][uu][ks]);
                    acc = mfma16(w0, hi, acc);
                    if constexpr (NP == 2) {
                        V8 lo;
#pragma unroll
                        for (int e = 0; e < 8; ++e) lo[e] = (H)(rr[e] - (float)hi[e]);
                        acc = mfma16(w0, lo, acc);
                        acc = mfma16(__builtin_bit_cast(V8, wr.v[1][uu][ks]), hi, acc);
                    }
                }
            }
            T.q32[row * QS + u * 4 + kq] = (acc[0] * acc[0] + acc[1] * acc[1]) + (acc[2] * acc[2] + acc[3] * acc[3]);
        }
    }
    }
    __syncthreads();
    int flag = 0;
    {
        const int r = 4 * w + (l >> 4), c = l & 15;
        const float L = lse_rows<D, float>(P, T.q32, T.cst32, r, c);
        if (c == 0) {
            out[r] = L;
            flag = (mask[r] != 0) && near_threshold(g, L);
            T.rc[r] = flag;
        }
    }
    return __syncthreads_or(flag);
}

// Neal's funnel, FP64: log N(v; 0, 9) + sum_{j>=1} log N(x_j; 0, e^v), v = x_0.
template <int D>
__device__ void funnel_eval64(const DevProblem &P, const Tile &T, const int *mask, double *out)
{
    constexpr int LDC = D + 1;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    for (int rr = 0; rr < 4; ++rr) {
        const int r = 4 * w + rr;
        if (!mask[r]) continue;
        const double v = T.cand[r * LDC];
        double s = 0.0;
        for (int a = l; a < P.d; a += 64)
            if (a >= 1) { const double x = T.cand[r * LDC + a]; s += x * x; }
        s = wave_sum_fast(s);
        if (l == 0)
            out[r] = -v * v / 18.0 - 0.5 * (LOG_2PI + log(9.0)) - 0.5 * exp(-v) * s
                     - (double)(P.d - 1) * 0.5 * (v + LOG_2PI);
    }
    __syncthreads();
}

// Gaussian-Rastrigin test likelihood, FP64: log(alpha e^{-|x|^2/2} + (1 - alpha)
// e^{-A d + A sum cos(2 pi x_i)}) as a log-sum-exp of the two terms; cos(2 pi x) = cospi(2x)
// (no rounding of the argument by pi).  Each wave takes 4 rows, lane l coordinates l, l+64.
template <int D>
__device__ void rg_eval64(const DevProblem &P, const Tile &T, const int *mask, double *out)
{
    constexpr int LDC = D + 1;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    for (int rr = 0; rr < 4; ++rr) {
        const int r = 4 * w + rr;
        if (!mask[r]) continue;
        double s2 = 0.0, sc = 0.0;
        for (int a = l; a < P.d; a += 64) {
            const double x = T.cand[r * LDC + a];
            s2 += x * x;
            sc += cospi(2.0 * x);
        }
        s2 = wave_sum_fast(s2);
        sc = wave_sum_fast(sc);
        if (l == 0) {
            const double tf = P.rg_la - 0.5 * s2;
            const double tg = P.rg_l1a - P.rg_amp * P.d + P.rg_amp * sc;
            const double mx = fmax(tf, tg);
            out[r] = mx + log(exp(tf - mx) + exp(tg - mx));
        }
    }
    __syncthreads();
}

template <int D, int LIK>
__device__ __forceinline__ void eval64(const DevProblem &P, const Tile &T, const int *mask,
                                       double *out)
{
    if constexpr (LIK == LIK_MIXTURE) mix_eval64<D>(P, T, mask, out);
    else if constexpr (LIK == LIK_RG) rg_eval64<D>(P, T, mask, out);
    else funnel_eval64<D>(P, T, mask, out);
}

// Loads this wave's register-resident 16-bit W fragments (same unit order as mix_eval16).
template <int D, int UPW, int NP>
__device__ __forceinline__ void load_wfrag(const DevProblem &P, WFrag<D, UPW, NP> &wr)
{
    constexpr int NJB = D / 16, NKS = D / 32;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int uu = 0; uu < UPW; ++uu) {
        int c, jb;
        if (comp_major_t<D, UPW>(P.K)) unit_of_cm<NJB>(w, uu, c, jb);
        else unit_of<NJB>(w, uu, c, jb);
        const int u = c * NJB + jb;
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
            const size_t o = ((size_t)u * NKS + ks) * 64 + l;
            wr.v[0][uu][ks] = (c < P.K) ? P.wf16[o] : make_uint4(0, 0, 0, 0);
            if constexpr (NP == 2) wr.v[1][uu][ks] = (c < P.K) ? P.wf16lo[o] : make_uint4(0, 0, 0, 0);
        }
    }
}

// Evaluates the masked rows of the tile in the kernel's precision: FP64 results in T.L, 16-bit
// mode results in T.L32 with the re-check flags in T.rc; returns whether any row needs an FP64
// re-check (always 0 in FP64 mode).
template <int D, int MODE, int LIK, int UPW, int NP>
__device__ __forceinline__ int eval_tile(const DevProblem &P, const WFrag<D, UPW, NP> &wr,
                                         const Tile &T, const int *mask, const Guard &g)
{
    if constexpr (MODE == MODE_FP64) {
        eval64<D, LIK>(P, T, mask, T.L);
        return 0;
    } else {
        return mix_eval16<D, UPW, MODE>(P, wr, T, mask, T.L32, g);
    }
}

template <int MODE> struct NPOf { static constexpr int v = 1; };
template <> struct NPOf<MODE_BF16X3> { static constexpr int v = 2; };
template <> struct NPOf<MODE_FP16X3> { static constexpr int v = 2; };

}  // namespace nss
