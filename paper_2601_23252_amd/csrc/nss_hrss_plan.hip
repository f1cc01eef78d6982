// gfx950 HRSS chains with hypothesis plans, for the mixture likelihood in the 16-bit modes.
//
// One workgroup = four waves = up to four chains (chain c <-> wave c), as in k_hrss, but each
// chain plans S tests per round (S = 8 or 16) and the workgroup evaluates one tile of 4 S
// candidate rows.  A round's plan covers the next stepping-out tests of every open bracket end
// (two per end) and, for the most likely outcomes of those tests (hypotheses: how many more
// times each end expands), the shrink proposals that the sequential algorithm would make if
// every one of them were rejected.  Each proposal is fully determined by the bracket and the
// step's shrink uniforms, so every planned row is exactly the test the sequential algorithm
// makes in that case.  After the tile the chain walks its plan in the sequential order: the
// stepping-out tests, then the shrink proposals of the hypothesis that came true, up to the
// first acceptance; the rest is discarded and neither counted nor used.
//
// Precision: rows are evaluated with 16-bit products and FP32 accumulation.  A consumed row
// whose estimate lies within the guard band of L* is not decided in FP32: the walk stops before
// it, and in the next round that row (the first test of the next plan) is evaluated in FP64
// and decided on that value.  Decisions therefore equal FP64 decisions, and so do the
// trajectory and the counters; the chain's final point is re-evaluated in FP64 for the stored
// logL.
#include "nss_internal.hpp"
#include "nss_rng.hpp"
#include "nss_tiles.hpp"
#include "nss_wave.hpp"

#include <math.h>

namespace nss {

constexpr int kPlanE = 2;   // stepping-out tests per open bracket end per round
constexpr int kPlanH = 3;   // at most this many hypotheses per round

// LDS of one workgroup (byte offsets; identical on host).  FP64 area: the staged constants and
// a 16-row FP64 tile (rows 0..3: each chain's row to decide in FP64, or its final point);
// 16-bit area: the constants in FP32, the 4 S candidate rows in FP32, their partial quadratic
// forms (one per k-quarter); per chain: the shrink uniforms of a round that needs more than the
// step's buffer holds.
struct PlanLayout {
    int cand, mu64, cst, q, L, mask, mu32, cst32, c32, qd, su, total;
};
__host__ __device__ constexpr int plan_rows(int S) { return 4 * S; }
__host__ __device__ inline int plan_qk(int D, int K) { return (K > 0 ? K : 1) * (D / 16) * 4; }
__host__ __device__ inline PlanLayout plan_layout(int D, int K, int S)
{
    const int Kc = K > 0 ? K : 1;
    PlanLayout o;
    int off = 0;
    o.cand = off; off += al16(kRows * (D + 1) * 8);
    o.mu64 = off; off += al16(Kc * D * 8);
    o.cst = off; off += al16(Kc * 8);
    o.q = off; off += al16(kRows * q_stride(D, K) * 8);
    o.L = off; off += al16(kRows * 8);
    o.mask = off; off += al16(kRows * 4);
    o.mu32 = off; off += al16(Kc * D * 4);
    o.cst32 = off; off += al16(Kc * 4);
    o.c32 = off; off += al16(plan_rows(S) * (D + 4) * 4);
    o.qd = off; off += al16(plan_rows(S) * plan_qk(D, K) * 4);
    o.su = off; off += al16(4 * S * 8);
    o.total = off;
    return o;
}

// Slot layout of a plan with S slots (fixed, so that every per-slot value lives in registers
// at a compile-time index): slots 0, 1 are the next two stepping-out tests of the left end,
// slots 2, 3 those of the right end, then three hypothesis blocks of shrink proposals; while
// shrinking, all S slots are the next S proposals.  Unused slots are not evaluated.
template <int S> struct PlanShape;
template <> struct PlanShape<16> {
    static constexpr int off[kPlanH] = {4, 8, 12}, len[kPlanH] = {4, 4, 4};
};
template <> struct PlanShape<8> {
    static constexpr int off[kPlanH] = {4, 6, 7}, len[kPlanH] = {2, 1, 1};
};

// Partial quadratic forms of the 16-bit tile over the NRB 16-row blocks of c32:
// qd[(row * K + c) * NJB * 4 + jb * 4 + kq] = the lane's share (k-quarter kq) of
// |(W_c (x_row - mu_c))_{16 jb .. 16 jb + 15}|^2; with whole components per wave
// (comp_major_t) the lane's share of the full form in slot jb = 0.  W as the A operand (register
// fragments), residuals as B.  Ends with a barrier.
template <int D, int UPW, int MODE, int NRB>
__device__ __forceinline__ void plan_tile(const DevProblem &P,
                                          const WFrag<D, UPW, MixTraits<MODE>::NP> &wr,
                                          const float *c32, const float *mu32, float *qd)
{
    typedef typename MixTraits<MODE>::H H;
    typedef typename MixTraits<MODE>::V8 V8;
    constexpr int NP = MixTraits<MODE>::NP;
    constexpr int NJB = D / 16, NKS = D / 32, LDC = D + 4;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int row = l & 15, kq = l >> 4;
    const int K = P.K;
    const bool cm = comp_major_t<D, UPW>(K);
    // comp-major: this wave's component means, read once for the four row blocks
    constexpr int CWM = (UPW + NJB - 1) / NJB;
    float mreg[CWM][NKS][8];
    if (cm) {
#pragma unroll
        for (int cw = 0; cw < CWM; ++cw) {
            const int c = w + 4 * cw;
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
                float4 m0 = {0.f, 0.f, 0.f, 0.f}, m1 = m0;
                if (c < K) {
                    const float *mu = mu32 + c * D + 8 * kq + 32 * ks;
                    m0 = *(const float4 *)mu;
                    m1 = *(const float4 *)(mu + 4);
                }
                mreg[cw][ks][0] = m0.x; mreg[cw][ks][1] = m0.y; mreg[cw][ks][2] = m0.z;
                mreg[cw][ks][3] = m0.w; mreg[cw][ks][4] = m1.x; mreg[cw][ks][5] = m1.y;
                mreg[cw][ks][6] = m1.z; mreg[cw][ks][7] = m1.w;
            }
        }
    }
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
        float cx[NKS][8];
        {
            const float *cr = c32 + (16 * rb + row) * LDC;
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
                const float4 a0 = *(const float4 *)(cr + 32 * ks + 8 * kq);
                const float4 a1 = *(const float4 *)(cr + 32 * ks + 8 * kq + 4);
                cx[ks][0] = a0.x; cx[ks][1] = a0.y; cx[ks][2] = a0.z; cx[ks][3] = a0.w;
                cx[ks][4] = a1.x; cx[ks][5] = a1.y; cx[ks][6] = a1.z; cx[ks][7] = a1.w;
            }
        }
        float *qrow = qd + (16 * rb + row) * K * NJB * 4 + kq;
        if (cm) {
            constexpr int CW = (UPW + NJB - 1) / NJB;
#pragma unroll
            for (int cw = 0; cw < CW; ++cw) {
                const int c = w + 4 * cw;
                if (c < K) {
                    f4 acc[NJB];
#pragma unroll
                    for (int jb = 0; jb < NJB; ++jb) acc[jb] = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < NKS; ++ks) {
                        float rr[8];
                        V8 hi, lo;
#pragma unroll
                        for (int e = 0; e < 8; ++e) { rr[e] = cx[ks][e] - mreg[cw][ks][e]; hi[e] = (H)rr[e]; }
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
                    float sq = 0.f;
#pragma unroll
                    for (int jb = 0; jb < NJB; ++jb)
                        sq += (acc[jb][0] * acc[jb][0] + acc[jb][1] * acc[jb][1]) +
                              (acc[jb][2] * acc[jb][2] + acc[jb][3] * acc[jb][3]);
                    qrow[c * NJB * 4] = sq;
                }
            }
        } else {
#pragma unroll
            for (int uu = 0; uu < UPW; ++uu) {
                int c, jb;
                unit_of<NJB>(w, uu, c, jb);
                if (c < K) {
                    const int ke = (16 * jb + 16 + 31) / 32;
                    const float *mu = mu32 + c * D + 8 * kq;
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
                    qrow[(c * NJB + jb) * 4] =
                        (acc[0] * acc[0] + acc[1] * acc[1]) + (acc[2] * acc[2] + acc[3] * acc[3]);
                }
            }
        }
    }
    __syncthreads();
}

// log L of the chain's S rows (rows row0 .. row0 + S - 1) from the partials: lane l takes row
// l / G of the chain (G = 64 / S lanes per row) and components sub, sub + G, ...
// (sub = l mod G); every lane of the row's group ends with the row's value.
template <int D, int UPW, int S>
__device__ __forceinline__ float plan_lse(const DevProblem &P, const float *qd, const float *cst32,
                                          int row0)
{
    constexpr int NJB = D / 16, G = 64 / S;
    const int l = threadIdx.x & 63, r = l / G, sub = l % G;
    const int K = P.K;
    const bool cm = comp_major_t<D, UPW>(K);
    const float *q = qd + (row0 + r) * K * NJB * 4;
    auto term = [&](int c) -> float {
        const float4 *qc = (const float4 *)(q + c * NJB * 4);
        float4 v = qc[0];
        float s = (v.x + v.y) + (v.z + v.w);
        if (!cm) {
            for (int jb = 1; jb < NJB; ++jb) {
                v = qc[jb];
                s += (v.x + v.y) + (v.z + v.w);
            }
        }
        return cst32[c] - 0.5f * s;
    };
    constexpr int NT = 4;            // components per lane held in registers
    float t[NT];
    float mx = -INFINITY;
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int c = sub + G * i;
        t[i] = (c < K) ? term(c) : -INFINITY;
        mx = fmaxf(mx, t[i]);
    }
    for (int c = sub + G * NT; c < K; c += G) mx = fmaxf(mx, term(c));
    mx = fmaxf(mx, dppf<DPP_XOR1>(mx));
    if constexpr (G >= 4) mx = fmaxf(mx, dppf<DPP_XOR2>(mx));
    if constexpr (G >= 8) mx = fmaxf(mx, dppf<DPP_HMIR>(mx));
    float e = 0.f;
    if (mx != -INFINITY) {
#pragma unroll
        for (int i = 0; i < NT; ++i)
            if (sub + G * i < K) e += __expf(t[i] - mx);
        for (int c = sub + G * NT; c < K; c += G) e += __expf(term(c) - mx);
    }
    e += dppf<DPP_XOR1>(e);
    if constexpr (G >= 4) e += dppf<DPP_XOR2>(e);
    if constexpr (G >= 8) e += dppf<DPP_HMIR>(e);
    return mx == -INFINITY ? -INFINITY : mx + __logf(e);
}

// Bits G * s of a ballot, compressed to bit s (s < S), by folding the kept bits together.
template <int S>
__device__ __forceinline__ unsigned compress_ballot(unsigned long long b)
{
    if constexpr (S == 16) {   // every 4th bit
        unsigned long long x = b & 0x1111111111111111ull;
        x = (x | (x >> 3)) & 0x0303030303030303ull;
        x = (x | (x >> 6)) & 0x000F000F000F000Full;
        x = (x | (x >> 12)) & 0x000000FF000000FFull;
        x = (x | (x >> 24)) & 0x000000000000FFFFull;
        return (unsigned)x;
    } else {                   // every 8th bit
        unsigned long long x = b & 0x0101010101010101ull;
        x = (x | (x >> 7)) & 0x0003000300030003ull;
        x = (x | (x >> 14)) & 0x0000000F0000000Full;
        x = (x | (x >> 28)) & 0x00000000000000FFull;
        return (unsigned)x;
    }
}

enum { PF_NONE = 0, PF_LEFT = 1, PF_RIGHT = 2, PF_SHRINK = 3 };

// OCC: workgroups per CU the register allocation targets (1, or 2 with the excess spilled):
// two resident workgroups hide each other's round latency when a launch has more workgroups
// than the chip has CUs; the arithmetic, and so every result, is the same.
template <int D, int MODE, int UPW, int S, int OCC>
__global__ __launch_bounds__(256, OCC) void k_hrss_plan(Launch Lc)
{
    static_assert(S == 8 || S == 16, "plan slots");
    typedef PlanShape<S> Shape;
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
    const PlanLayout lay = plan_layout(D, P.K, S);
    Tile T64;   // the FP64 tile (16 rows) for decisions and final points taken in FP64
    T64.cand = (double *)(smem + lay.cand);
    T64.cand32 = nullptr;
    T64.mu64 = (double *)(smem + lay.mu64);
    T64.mu32 = nullptr;
    T64.cst = (double *)(smem + lay.cst);
    T64.cst32 = nullptr;
    T64.pa = T64.pb = nullptr;
    T64.L = (double *)(smem + lay.L);
    T64.L32 = nullptr;
    T64.mask = (int *)(smem + lay.mask);
    T64.rc = nullptr;
    T64.q = (double *)(smem + lay.q);
    T64.q32 = nullptr;
    float *mu32 = (float *)(smem + lay.mu32);
    float *cst32 = (float *)(smem + lay.cst32);
    float *c32 = (float *)(smem + lay.c32);
    float *qd = (float *)(smem + lay.qd);
    double *shu = (double *)(smem + lay.su);   // [4][S] shrink uniforms of a SHRINK round

    const int tid = threadIdx.x, w = uniform_i(tid >> 6), l = tid & 63;
    const int d = P.d;
    const double Lstar = R.scal[0];
    const int t0 = R.iscal[1], nsurv = R.iscal[2];
    const uint32_t it = (uint32_t)R.iscal[3] + 1u;
    const double width = R.width;
    const int p = R.p, cap_out = R.stepout_cap, cap_sh = R.shrink_cap;
    const bool box = (P.prior_kind == PRIOR_BOX);

    for (int i = tid; i < P.K * D; i += 256) { T64.mu64[i] = P.mu[i]; mu32[i] = P.mu32[i]; }
    for (int i = tid; i < P.K; i += 256) { T64.cst[i] = P.cst[i]; cst32[i] = P.cst32[i]; }
    for (int i = tid; i < kRows * LDC; i += 256) T64.cand[i] = 0.0;
    for (int i = tid; i < plan_rows(S) * LDC32; i += 256) c32[i] = 0.f;
    if (tid < kRows) T64.mask[tid] = 0;
    WFrag<D, UPW, NP> wr;
    load_wfrag<D, UPW, NP>(P, wr);

    const int j = bm.y * C + w;
    const bool has_chain = (w < C) && (j < R.k);
    double *su = shu + w * S;
    float *crow = c32 + w * S * LDC32;
    double *frow = T64.cand + w * LDC;

    double x0r[NA], vr[NA], par[NA], pbr[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int a = l + 64 * i;
        x0r[i] = 0.0; vr[i] = 0.0;
        par[i] = (a < D) ? P.pa[a] : 0.0;
        pbr[i] = (a < D) ? P.pb[a] : 1.0;
    }

    // per-chain state (wave-uniform, replicated in every lane of the chain's wave)
    enum { NEWSTEP = 0, STEPOUT = 1, SHRINK = 2, DONE = 3 };
    int phase = DONE, step = 0, nl = 0, nr = 0, ns = 0, force = PF_NONE;
    bool la = false, ra = false;
    double tL = 0.0, tR = 0.0, logy = -INFINITY;
    unsigned long long c_evals = 0, c_tests = 0, c_prej = 0, c_outcap = 0, c_shcap = 0,
                       c_nonfin = 0, c_rc = 0, c_viol = 0;

    if (has_chain) {
        double u, unused;
        draw2(R.key0, R.key1, PUR_RESAMPLE, (uint32_t)j, it, 0u, 0u, u, unused);
        int qi = (int)floor(u * (double)nsurv);
        if (qi > nsurv - 1) qi = nsurv - 1;
        const int parent = R.perm[t0 + qi];
        if (l == 0) R.parents[j] = parent;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int a = l + 64 * i;
            if (a < d) x0r[i] = R.X[(size_t)a * R.m_pad + parent];
        }
        phase = (p > 0) ? NEWSTEP : DONE;
    }
    __syncthreads();

    // the step's direction and uniforms (tL0, uh, shrink uniforms 0..5), the next step's
    // prefetched into registers one step ahead
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
            const double *sp = R.ubuf + ((size_t)j * p + st) * kStepU;
#pragma unroll
            for (int q = 0; q < kStepU; ++q) pu[q] = sp[q];
        }
    };
    prefetch_dir(0);
    auto logprior_at = [&](const double *y) -> double {
        double lp = 0.0;
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const int a = l + 64 * i;
            if (a < d) { const double zt = (y[i] - par[i]) / pbr[i]; lp += -0.5 * zt * zt; }
        }
        return wave_sum_fast(lp) + P.logprior_norm;
    };
    auto finish_step = [&](int acc, int nsh) {
        if (R.trace && l == 0) {
            int *trc = R.trace + ((size_t)j * p + step) * 4;
            trc[0] = nl; trc[1] = nr; trc[2] = nsh; trc[3] = acc;
        }
        if (!acc) ++c_shcap;
        ++step;
        phase = (step >= p) ? DONE : NEWSTEP;
    };
    auto enter_shrink = [&]() {
        phase = SHRINK;
        ns = 0;
        if (cap_sh <= 0) finish_step(0, 0);
    };
    const Guard guard = {Lstar, P.guard_rel, P.guard_abs, P.cmax32};
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

    for (;;) {
        PT(11);
        // ---- a new step: direction, bracket offset, slice height ----
        if (has_chain && phase == NEWSTEP) {
#ifdef NSS_PHASE_TIMING
            pt[9] += 1;
#endif
#pragma unroll
            for (int i = 0; i < NA; ++i) vr[i] = pv[i];
#pragma unroll
            for (int q = 0; q < kStepU; ++q) cu[q] = pu[q];
            prefetch_dir(step + 1);
            tL = cu[0];
            logy = box ? -INFINITY : logprior_at(x0r) + log(cu[1]);
            tR = tL + width;
            nl = nr = 0;
            la = ra = (cap_out > 0);
            if (cap_out <= 0) c_outcap += 2;
            phase = STEPOUT;
            if (!la && !ra) enter_shrink();
        }
        PT(0);
        const bool act = has_chain && phase != DONE;
        const int phase0 = phase;

        // ---- the plan: t of every slot (registers, compile-time slot indices) ----
        double tv[S];
        unsigned vm = 0;   // planned slots
        int hA[kPlanH], hB[kPlanH];
        bool hV[kPlanH];
#pragma unroll
        for (int s = 0; s < S; ++s) tv[s] = 0.0;
#pragma unroll
        for (int h = 0; h < kPlanH; ++h) { hA[h] = 0; hB[h] = 0; hV[h] = false; }
        if (act && phase == STEPOUT) {
            const int nsl = la ? min(kPlanE, cap_out - nl) : 0;
            const int nsr = ra ? min(kPlanE, cap_out - nr) : 0;
            tv[0] = tL; tv[1] = tL - width;
            tv[2] = tR; tv[3] = tR + width;
            vm = (nsl >= 1 ? 1u : 0u) | (nsl >= 2 ? 2u : 0u) | (nsr >= 1 ? 4u : 0u) |
                 (nsr >= 2 ? 8u : 0u);
            // the end's outcomes that resolve it this round: its first test outside at
            // position a < n, or all n tests inside with the cap reached
            const unsigned va = la ? ((1u << nsl) - 1u) | (nl + nsl >= cap_out ? 1u << nsl : 0u) : 1u;
            const unsigned vb = ra ? ((1u << nsr) - 1u) | (nr + nsr >= cap_out ? 1u << nsr : 0u) : 1u;
            if (la && ra && va == 3u && vb == 3u) {
                // both ends open, two tests each, no cap in reach: (1,0), (0,1), (0,0)
                hA[0] = 1; hB[0] = 0; hA[1] = 0; hB[1] = 1; hA[2] = 0; hB[2] = 0;
                hV[0] = hV[1] = hV[2] = true;
            } else {
                // outcome pairs (a, b) in the order of preference (1,0), (0,1), (0,0), (1,1),
                // (2,0), (0,2), (2,1), (1,2), (2,2), four bits each: a | b << 2
                constexpr unsigned long long kPref = 1ull | 4ull << 4 | 0ull << 8 | 5ull << 12 |
                                                     2ull << 16 | 8ull << 20 | 6ull << 24 |
                                                     9ull << 28 | 10ull << 32;
                int nh = 0;
#pragma unroll
                for (int k2 = 0; k2 < 9; ++k2) {
                    const int a = (int)(kPref >> (4 * k2)) & 3, b = (int)(kPref >> (4 * k2 + 2)) & 3;
                    const bool ok = ((va >> a) & 1u) && ((vb >> b) & 1u);
#pragma unroll
                    for (int h = 0; h < kPlanH; ++h)
                        if (ok && nh == h) { hA[h] = a; hB[h] = b; hV[h] = true; }
                    nh += ok ? 1 : 0;
                }
            }
#pragma unroll
            for (int h = 0; h < kPlanH; ++h) {
                double sL = tL, sR = tR;
                if (hA[h] >= 1) sL -= width;
                if (hA[h] >= 2) sL -= width;
                if (hB[h] >= 1) sR += width;
                if (hB[h] >= 2) sR += width;
#pragma unroll
                for (int q = 0; q < Shape::len[h]; ++q) {
                    const double t = sL + cu[2 + q] * (sR - sL);
                    tv[Shape::off[h] + q] = t;
                    if (hV[h] && q < cap_sh) vm |= 1u << (Shape::off[h] + q);
                    if (t < 0.0) sL = t; else sR = t;
                }
            }
        } else if (act && phase == SHRINK) {
            // the next S proposals: their uniforms (numbers ns .. ns + S - 1) drawn one per
            // lane where the step's buffer does not hold them
            if (ns + S > kStepShrinkU) {
                double u = 0.0;
                if (l < S) {
                    const int q = ns + l;
                    if (q < kStepShrinkU) {
#pragma unroll
                        for (int i = 0; i < kStepShrinkU; ++i) if (q == i) u = cu[2 + i];
                    } else {
                        double unused;
                        draw2(R.key0, R.key1, PUR_SHRINK, (uint32_t)j, it, (uint32_t)step,
                              (uint32_t)q, u, unused);
                    }
                    su[l] = u;
                }
                wave_sync();
            }
            double sL = tL, sR = tR;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                double u;
                if (ns + S > kStepShrinkU) {
                    u = su[q];
                } else {
                    u = cu[2];
#pragma unroll
                    for (int i = 1; i < kStepShrinkU; ++i) if (ns + q == i) u = cu[2 + i];
                }
                const double t = sL + u * (sR - sL);
                tv[q] = t;
                if (ns + q < cap_sh) vm |= 1u << q;
                if (t < 0.0) sL = t; else sR = t;
            }
        }
        PT(1);

        // ---- candidate rows (FP32 for the tile), prior tests; the forced row in FP64 ----
        const int fslot = (force == PF_RIGHT) ? 2 : 0;
        unsigned okm = 0;
        if (act) {
            unsigned oob = 0;   // slots with a coordinate outside the box
#pragma unroll
            for (int s = 0; s < S; ++s) {   // every slot (unplanned ones are never consumed)
                double y[NA];
                bool inb = true;
#pragma unroll
                for (int i = 0; i < NA; ++i) {
                    const int a = l + 64 * i;
                    y[i] = fma(tv[s], vr[i], x0r[i]);
                    if (a < D) crow[s * LDC32 + a] = (float)y[i];
                    if (a < d) inb = inb && (y[i] >= par[i] && y[i] <= pbr[i]);
                }
                // a slot is in the box when every lane's coordinates are (a wave vote)
                if (box) oob |= (__all(inb) != 0 ? 0u : 1u) << s;
                else if ((vm >> s) & 1u) okm |= (logprior_at(y) > logy ? 1u : 0u) << s;
            }
            if (box) okm = vm & ~oob;
            if (force != PF_NONE) {
                const double tf = (force == PF_RIGHT) ? tv[2] : tv[0];
#pragma unroll
                for (int i = 0; i < NA; ++i)
                    if (l + 64 * i < D) frow[l + 64 * i] = fma(tf, vr[i], x0r[i]);
            }
        }
        const int want64 = act && force != PF_NONE && ((okm >> fslot) & 1u);
        if (l == 0) T64.mask[w] = want64;
        PT(2);
        if (!__syncthreads_or(act)) break;
        const int any64 = T64.mask[0] | T64.mask[1] | T64.mask[2] | T64.mask[3];
        PT(3);
#ifdef NSS_PHASE_TIMING
        pt[8] += 1;
#endif

        // ---- FP64 decision rows (rare), then the 16-bit tile of the 4 S rows ----
        if (any64) {
            mix_eval64<D>(P, T64, T64.mask, T64.L);
#ifdef NSS_PHASE_TIMING
            pt[10] += 1;
#endif
        }
        PT(4);
        plan_tile<D, UPW, MODE, plan_rows(S) / 16>(P, wr, c32, mu32, qd);
        PT(5);
        float Lr = -INFINITY;
        if (w < C) Lr = plan_lse<D, UPW, S>(P, qd, cst32, w * S);
        PT(6);

        // ---- walk the plan in the sequential algorithm's order ----
        if (act) {
            constexpr int G = 64 / S;
            const int rs = l / G;
            const bool okr = (okm >> rs) & 1u;
            unsigned inm = compress_ballot<S>(__ballot(okr && (double)Lr > Lstar));
            unsigned flm = compress_ballot<S>(__ballot(okr && near_threshold(guard, Lr)));
            unsigned rcm = 0, nfm = 0;
            if (want64) {
                double L64 = T64.L[w];
                const bool nf = (L64 != L64) || L64 == INFINITY;
                if (nf) L64 = -INFINITY;
                inm = (inm & ~(1u << fslot)) | ((L64 > Lstar ? 1u : 0u) << fslot);
                flm &= ~(1u << fslot);
                rcm = 1u << fslot;
                nfm = (nf ? 1u : 0u) << fslot;
            }
            force = PF_NONE;
            unsigned cons = 0;   // consumed slots
            // 0: outside, 1: inside, 2: near L* (decided in FP64 next round)
            auto consume = [&](int s) -> int {
                if ((flm >> s) & 1u) return 2;
                cons |= 1u << s;
                return (inm >> s) & 1u;
            };
            // shrink proposals at slots s0 .. s0 + n - 1 on [tL, tR]; stops at an acceptance, the
            // cap, a row to decide in FP64 or an unplanned slot
            auto shrink_walk = [&](int s0, int n) {
                bool go = true;
#pragma unroll
                for (int q = 0; q < S; ++q) {
                    if (go && q < n) {
                        const int s = s0 + q;
                        if (!((vm >> s) & 1u)) {
                            go = false;
                        } else {
                            const int r = consume(s);
                            double t = tv[0];
#pragma unroll
                            for (int i = 1; i < S; ++i) if (i == s) t = tv[i];
                            if (r == 2) {
                                force = PF_SHRINK;
                                go = false;
                            } else if (r == 1) {
#pragma unroll
                                for (int i = 0; i < NA; ++i) x0r[i] = fma(t, vr[i], x0r[i]);
                                finish_step(1, ns + 1);
                                go = false;
                            } else {
                                if (t < 0.0) tL = t; else tR = t;
                                ++ns;
                                if (ns >= cap_sh) { finish_step(0, ns); go = false; }
                            }
                        }
                    }
                }
            };
            if (phase0 == STEPOUT) {
                int a = 0, b = 0;
                bool paused = false;
#pragma unroll
                for (int i = 0; i < kPlanE; ++i) {
                    if (!paused && la && ((vm >> i) & 1u)) {
                        const int r = consume(i);
                        if (r == 2) { force = PF_LEFT; paused = true; }
                        else if (r == 1) {
                            tL -= width; ++nl; ++a;
                            if (nl >= cap_out) { la = false; ++c_outcap; }
                        } else {
                            la = false;
                        }
                    }
                }
#pragma unroll
                for (int i = 0; i < kPlanE; ++i) {
                    if (!paused && ra && ((vm >> (2 + i)) & 1u)) {
                        const int r = consume(2 + i);
                        if (r == 2) { force = PF_RIGHT; paused = true; }
                        else if (r == 1) {
                            tR += width; ++nr; ++b;
                            if (nr >= cap_out) { ra = false; ++c_outcap; }
                        } else {
                            ra = false;
                        }
                    }
                }
                if (!paused && !la && !ra) {
                    enter_shrink();
                    if (phase == SHRINK) {
#pragma unroll
                        for (int h = 0; h < kPlanH; ++h)
                            if (hV[h] && hA[h] == a && hB[h] == b)
                                shrink_walk(Shape::off[h], Shape::len[h]);
                    }
                }
            } else if (phase0 == SHRINK) {
                shrink_walk(0, S);
            }
            c_tests += __builtin_popcount(cons);
            c_evals += __builtin_popcount(cons & okm);
            c_prej += __builtin_popcount(cons & ~okm);
            c_rc += __builtin_popcount(cons & rcm);
            c_nonfin += __builtin_popcount(cons & nfm);
        }
        PT(7);
    }
#ifdef NSS_PHASE_TIMING
    if (tid == 0 && R.prof) for (int i = 0; i < 12; ++i) atomicAdd(&R.prof[i], pt[i]);
#endif
#undef PT

    // stored log-likelihoods are FP64: re-evaluate each chain's final point
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NA; ++i)
        if (l + 64 * i < D) frow[l + 64 * i] = has_chain ? x0r[i] : 0.0;
    if (tid < kRows) T64.mask[tid] = (tid < kMaxChainsPerWG) && (tid < C) && (bm.y * C + tid < R.k);
    __syncthreads();
    mix_eval64<D>(P, T64, T64.mask, T64.L);
    if (has_chain) {
        unsigned long long dummy = 0;
        const double logL0 = sanitize(T64.L[w], dummy);
        if (!(logL0 > Lstar)) ++c_viol;
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
            atomicAdd(&R.ctr[3], c_outcap);
            atomicAdd(&R.ctr[4], c_shcap);
            atomicAdd(&R.ctr[5], c_nonfin);
            atomicAdd(&R.ctr[6], c_rc);
            atomicAdd(&R.ctr[7], c_viol);
        }
    }
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
size_t hrss_plan_lds_bytes(int D, int K, int S) { return (size_t)plan_layout(D, K, S).total; }

template <int D, int MODE, int UPW, int S, int OCC>
static hipError_t plan_t(const Launch &L, hipStream_t s)
{
    const size_t lds = hrss_plan_lds_bytes(D, L.max_K, S);
    auto f = k_hrss_plan<D, MODE, UPW, S, OCC>;
    hipError_t e = hipFuncSetAttribute((const void *)f,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(f, dim3(L.nblocks), dim3(256), lds, s, L);
    return hipGetLastError();
}

template <int MODE, int S, int OCC>
static hipError_t plan_mode(const Launch &L, int D, int upw, hipStream_t s)
{
    if (D == 32)
        return upw <= 4 ? plan_t<32, MODE, 4, S, OCC>(L, s) : plan_t<32, MODE, 16, S, OCC>(L, s);
    if (D == 64) {
        if (upw <= 2) return plan_t<64, MODE, 2, S, OCC>(L, s);
        if (upw <= 4) return plan_t<64, MODE, 4, S, OCC>(L, s);
        return plan_t<64, MODE, 8, S, OCC>(L, s);
    }
    if (D == 128) return plan_t<128, MODE, 4, S, OCC>(L, s);
    return hipErrorInvalidValue;
}

template <int S, int OCC>
static hipError_t plan_s(const Launch &L, int D, int mode, int upw, hipStream_t s)
{
    switch (mode) {
    case MODE_BF16: return plan_mode<MODE_BF16, S, OCC>(L, D, upw, s);
    case MODE_FP16: return plan_mode<MODE_FP16, S, OCC>(L, D, upw, s);
    case MODE_BF16X3: return plan_mode<MODE_BF16X3, S, OCC>(L, D, upw, s);
    case MODE_FP16X3: return plan_mode<MODE_FP16X3, S, OCC>(L, D, upw, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hrss_plan(const Launch &L, int D, int mode, int upw, int S, int occ,
                            hipStream_t s)
{
    if (L.nblocks <= 0) return hipSuccess;
    if (upw_template(D, upw) == 0) return hipErrorNotSupported;
    if (occ != 1 && occ != 2) return hipErrorInvalidValue;
    if (S == 8) return occ == 2 ? plan_s<8, 2>(L, D, mode, upw, s) : plan_s<8, 1>(L, D, mode, upw, s);
    if (S == 16)
        return occ == 2 ? plan_s<16, 2>(L, D, mode, upw, s) : plan_s<16, 1>(L, D, mode, upw, s);
    return hipErrorInvalidValue;
}

}  // namespace nss
