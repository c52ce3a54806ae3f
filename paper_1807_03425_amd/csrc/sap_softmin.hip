// Soft-min surrogate of the minimum projected unit-secant norm, and its
// gradient in P (gfx950).  Not part of the paper's method: a differentiable
// stand-in for its min, for gradient-based optimisation of P.
//
//   L      = -tau log sum_{kept i<j} exp(-r_ij / tau),   r_ij = ||P^T s_ij||
//   dL/dP  = sum w_ij s_ij (P^T s_ij)^T / r_ij,          w_ij = exp(-(r_ij - L)/tau)
//
// With Y = (X - mu) P, y_i - y_j = P^T (x_i - x_j), and d_ij = ||x_i - x_j||,
// s (P^T s)^T / r = (x_i - x_j)(y_i - y_j)^T / (d^2 r), so the gradient is a
// weighted graph Laplacian contraction:
//   dL/dP = (X - mu)^T Z,   z_i = sum_{j != i} a_ij (y_i - y_j),
//   a_ij  = w_ij (1/d_ij^2) / r_ij   (0 when r_ij = 0).
// The weights a_ij are recomputed tile by tile from Y and the stored 1/d^2
// (never stored), in the same 64 x 64 tile order as the pair pass.  Pairs on
// the short-pair list (fused form) are evaluated from their FP64 difference
// vectors, as in the iteration.
//
// Launch sequence
//   forward:  k_sm_loadP   P (FP32, n x k) -> FP64 k x n
//             k_sm_prep    Y = (X - mu) P (FP64 MFMA, rounded to FP32) and the
//                          FP64 (min, sum) partials of the short pairs
//             k_sm_fwd     per-block (min, scaled sum) over the tiles
//             k_sm_fin     one block: merge in FP64, L, loss
//   backward: k_sm_prep    (short-pair blocks only) a_ij (y_i - y_j) per short pair
//             k_sm_bwd     per half-tile partial z sums, rows and columns
//                          (weights and column side on VALU, row-side
//                          contraction on FP64 MFMA)
//             k_sm_zred    z_i per point: tile partials + short pairs, FP64
//             k_sm_grad    (X - mu)^T Z per row chunk, FP64 MFMA
//             k_sm_dP      sum of the chunks times dL/dloss
#include "sap_common.h"

namespace sap {

// log-sum-exp state: reference m and s = sum exp(-(r - m)/tau); s == 0 means
// empty (m is then ignored)
struct SmPart {
    double m, s;
};

struct SmArgs {
    const float *Y;        // soft-min Y, Npad x kp
    int kp;
    const float4 *invd2;
    const int2 *tiles;
    int64_t nhalf;
    int npass;             // pass blocks; their partials come first in `part`
    int n;
    // short pairs
    const int2 *close;
    const double *cd;
    int64_t nclose;
    // parameters
    const double *P64t;    // soft-min P, k x n FP64
    int vx, vp;            // 16-byte loads: X rows aligned; n even
    int gemm;              // arithmetic of the Y GEMM (SAP_GEMM_*)
    double tau;
    float c2;              // log2(e) / tau
    SmPart *part;          // npass + nshort partials (forward)
    const double *Lp;      // L of the forward (backward)
    // backward partials
    float *Zr;             // per half-tile: 32 x K row-side partials, point-major
    float *Zc;             // per half-tile: 64 x K column-side partials, point-major
    double *zpair;         // per short pair: a (y_i - y_j), K values
};

// (m1, s1) <- (m1, s1) merged with (m2, s2), FP64.
__device__ __forceinline__ void lse_merge(double &m1, double &s1, double m2, double s2, double tau) {
    if (!(s2 > 0.0)) return;
    if (!(s1 > 0.0)) { m1 = m2; s1 = s2; return; }
    const double m = fmin(m1, m2);
    s1 = s1 * exp((m - m1) / tau) + s2 * exp((m - m2) / tau);
    m1 = m;
}

// Block-wide merge of per-thread (m, s) into *out (thread 0).  All threads call.
__device__ void block_lse(double m, double s, double tau, SmPart *out) {
    __shared__ SmPart sp[kPairBlock / kWave];
#pragma unroll 1
    for (int o = 32; o > 0; o >>= 1) {
        const double m2 = __shfl_xor(m, o, kWave);
        const double s2 = __shfl_xor(s, o, kWave);
        lse_merge(m, s, m2, s2, tau);
    }
    if ((threadIdx.x & 63) == 0) sp[threadIdx.x >> 6] = SmPart{m, s};
    __syncthreads();
    if (threadIdx.x == 0) {
        double mm = sp[0].m, ss = sp[0].s;
        for (int w = 1; w < kPairBlock / kWave; ++w) lse_merge(mm, ss, sp[w].m, sp[w].s, tau);
        *out = SmPart{mm, ss};
    }
}

#ifndef SAP_KINST
// P (n x k row-major FP32) -> k x n FP64.
__global__ void k_sm_loadP(const float *__restrict__ P, int n, int k, double *__restrict__ P64t) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int l = e / k, q = e % k;
    P64t[(int64_t)q * n + l] = (double)P[e];
}

#endif

// Short pairs in FP64 (c = P^T (x_i - x_j) on the matrix cores, 16 pairs per
// wavefront, grid-stride).  Forward: the block's (min, sum) partial.
// Backward: a (y_i - y_j) = exp(-(r - L)/tau) / (r d^2) c per pair into zpair
// (lane m writes component m).
template <int K, typename TX>
__device__ void sm_short_block(const SmArgs &a, const TX *__restrict__ X, int64_t ldx, int sb,
                               int nshort, int bwd) {
    const int lane = threadIdx.x & 63;
    const int m = lane & 15, kk = lane >> 4;
    const int64_t ngroups = (a.nclose + 15) / 16;
    const double tau = a.tau;
    const double L = bwd ? *a.Lp : 0.0;
    double mm = 0.0, ss = 0.0;
    for (int64_t g16 = (int64_t)sb * (kPairBlock / kWave) + (threadIdx.x >> 6); g16 < ngroups;
         g16 += (int64_t)nshort * (kPairBlock / kWave)) {
        const int64_t row = g16 * 16 + m;
        const bool rin = row < a.nclose;
        const int2 pr = a.close[rin ? row : a.nclose - 1];
        const double dlen = a.cd[rin ? row : a.nclose - 1];
        const double4_t acc = short_c16<K, TX>(X, ldx, pr, rin, a.n, a.P64t, a.vx, a.vp);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double q2 = row_sum16(acc[v] * acc[v]);
            const int src = kk + 4 * v;          // the lane (m = src) that loaded this pair
            const double d = __shfl(dlen, src, kWave);
            const int64_t e = g16 * 16 + src;
            if (e < a.nclose) {
                const double r = sqrt(q2) / d;
                if (!bwd) {
                    if (m == 0) lse_merge(mm, ss, r, 1.0, tau);
                } else if (m < K) {
                    const double coef = r > 0.0 ? exp(-(r - L) / tau) / (r * d * d) : 0.0;
                    a.zpair[e * K + m] = coef * acc[v];
                }
            }
        }
    }
    if (!bwd) block_lse(mm, ss, tau, a.part + a.npass + sb);
}

// Blocks below gemm_blocks: Y = (X - mu) P; the others: short pairs.
template <int K, typename TX>
__global__ __launch_bounds__(kPairBlock) void k_sm_prep(SmArgs a, const TX *__restrict__ X,
                                                        int64_t ldx, int64_t N,
                                                        const double *__restrict__ mu,
                                                        float *__restrict__ Y, int64_t Npad,
                                                        int gemm_blocks, int bwd) {
    if ((int)blockIdx.x < gemm_blocks)
    {
        const TX nx[16] = {};
        const double none[16] = {};
        gemm_block<TX>(X, ldx, N, a.n, K, mu, a.P64t, Y, nullptr, a.kp, Npad, a.vx, a.vp, nx, none, false,
                       a.gemm);
    }
    else
        sm_short_block<K, TX>(a, X, ldx, (int)blockIdx.x - gemm_blocks, (int)gridDim.x - gemm_blocks,
                              bwd);
}

__device__ __forceinline__ float comp4(const float4 &v, int r) {
    return r == 0 ? v.x : r == 1 ? v.y : r == 2 ? v.z : v.w;
}

// Forward pass: one wavefront per half-tile (as the pair pass).  Per lane,
// the 32 r of a half-tile are reduced to their min m_c and
// s_c = sum 2^((m_c - r) c2), then folded into the lane's running (m, s).
// Masked pairs take r = 2e30, beyond the 1e30 start of every min, so their
// terms underflow to 0.
template <int K>
__global__ __launch_bounds__(kPairBlock) void k_sm_fwd(SmArgs a) {
    __shared__ float4 s_y[kPairBlock / kWave][32 * kMaxK / 4];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wid = (int64_t)blockIdx.x * (kPairBlock / kWave) + wv;
    const int64_t nw = (int64_t)a.npass * (kPairBlock / kWave);
    const int kp = a.kp;
    const float c2 = a.c2;
    float4 *yl = s_y[wv];
    const int nf4 = 8 * kp;
    float m = 1e30f;
    double s = 0.0;
    for (int64_t h = wid; h < a.nhalf; h += nw) {
        const int64_t t = h >> 1;
        const int half = (int)(h & 1);
        const float4 *tp = a.invd2 + t * (kTileElems / 4) + half * 512 + lane;
        float4 w[8];
#pragma unroll
        for (int g = 0; g < 8; ++g) w[g] = tp[g * 64];
        const int2 b = a.tiles[t];
        const float4 *ysrc =
            reinterpret_cast<const float4 *>(a.Y + ((int64_t)b.x * kTile + 32 * half) * kp);
        __builtin_amdgcn_wave_barrier();
        for (int f = lane; f < nf4; f += kWave) yl[f] = ysrc[f];
        __builtin_amdgcn_wave_barrier();
        float yj[K];
        load_yj<K>(a.Y, kp, (int64_t)b.y * kTile + lane, yj);
        const float *yi0 = reinterpret_cast<const float *>(yl);
        float r[32];
        float mc = 1e30f;
#pragma unroll
        for (int g = 0; g < 8; ++g) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const float wt = comp4(w[g], rr);
                const float acc = pair_r2<K>(yi0 + (4 * g + rr) * kp, yj, 1.0f);
                const float rv = wt > 0.0f ? __builtin_amdgcn_sqrtf(acc * wt) : 2e30f;
                r[4 * g + rr] = rv;
                mc = fminf(mc, rv);
            }
        }
        float sc = 0.0f;
        const float mcc = mc * c2;
#pragma unroll
        for (int e = 0; e < 32; ++e) sc += __builtin_amdgcn_exp2f(__builtin_fmaf(-r[e], c2, mcc));
        const float mn = fminf(m, mc);
        s = s * (double)__builtin_amdgcn_exp2f((mn - m) * c2) +
            (double)(sc * __builtin_amdgcn_exp2f((mn - mc) * c2));
        m = mn;
    }
    block_lse((double)m, s, a.tau, a.part + blockIdx.x);
}

#ifndef SAP_KINST
// Final merge of the forward (one block): L = m - tau log s.
__global__ __launch_bounds__(kPairBlock) void k_sm_fin(const SmPart *__restrict__ part, int nparts,
                                                       double tau, float *__restrict__ loss,
                                                       DevState *st) {
    double m = 0.0, s = 0.0;
    for (int b = threadIdx.x; b < nparts; b += kPairBlock) lse_merge(m, s, part[b].m, part[b].s, tau);
    __shared__ SmPart out;
    block_lse(m, s, tau, &out);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double L = out.s > 0.0 ? out.m - tau * log(out.s) : __builtin_huge_val();
        st->sm_m = out.m;
        st->sm_s = out.s;
        st->sm_L = L;
        loss[0] = (float)L;
    }
}

#endif

// Row stride of a wavefront's 32 x 64 weight block in LDS.  66 = 2 mod 32
// words: the row contraction's reads (16 rows x 4 consecutive columns) meet
// every bank once per half-wavefront, and the phase-1 writes (one row, 64
// consecutive columns) too.
constexpr int kAStride = 66;

// Backward pass: one wavefront per half-tile (rows i = 64 bi + 32 half +
// 0..31, columns j = 64 bj + 0..63).
// Phase 1 (lane = column j): the weights a_ij of the lane's column, one
// float4 of 1/d^2 per four rows, and the column side
//   z_j += sum_i a_ij (y_j - y_i)
// accumulated in FP32 from the differences y_i - y_j that the weight needed
// anyway; a_ij goes to the wavefront's LDS block.
// Phase 2: the row side
//   z_i += sum_j a_ij (y_i - y_j) = (sum_j a_ij) y_i - (A Y_J)_i
// on the matrix cores in FP64 (v_mfma_f64_16x16x4f64, K padded to 16
// columns): lane (c16 = lane % 16, r4 = lane / 16) feeds A = a[16 mb + c16]
// [4 t + r4] from LDS and B = y_J[4 t + r4][c16].  The FP32 weights and
// coordinates are exact in FP64 and the products and sums FP64, so the
// difference of the two large terms keeps the accuracy of the direct sum of
// differences.  For K < 16 the padding column 15 of B is 1, which makes
// column 15 of the product the row sum; K = 16 sums the rows separately.
// Partials go to Zr (32 x K) and Zc (64 x K) per half-tile, point-major, in
// FP32.  LDS per block: 38 KB (K <= 4) to 56 KB (K >= 13): three blocks per
// compute unit for K <= 12 (at most 168 registers), two for K >= 13.
template <int K>
__global__ __launch_bounds__(kPairBlock, K <= 12 ? 3 : 2) void k_sm_bwd(SmArgs a) {
    constexpr int KP = K <= 4 ? 4 : (K <= 8 ? 8 : (K <= 12 ? 12 : 16));   // the Y row length kp
    __shared__ float4 s_y[kPairBlock / kWave][32 * KP / 4];
    __shared__ float4 s_yc[kPairBlock / kWave][64 * KP / 4];
    __shared__ float s_a[kPairBlock / kWave][32 * kAStride];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wid = (int64_t)blockIdx.x * (kPairBlock / kWave) + wv;
    const int64_t nw = (int64_t)a.npass * (kPairBlock / kWave);
    constexpr int kp = KP;                            // equals a.kp
    const float c2 = a.c2;
    const float Lc = (float)(*a.Lp) * c2;
    float4 *yl = s_y[wv];
    float4 *ycl = s_yc[wv];
    float *al = s_a[wv];
    const int c16 = lane & 15, r4 = lane >> 4;
    const bool qin = c16 < K;
    const int qc = qin ? c16 : K - 1;                 // clamped component: in-bounds LDS reads
    const double bpad = (K < 16 && c16 == 15) ? 1.0 : 0.0;
    const float *alr = al + c16 * kAStride + r4;      // row-side reads: + 16 mb kAStride + 4 tt
    for (int64_t h = wid; h < a.nhalf; h += nw) {
        const int64_t t = h >> 1;
        const int half = (int)(h & 1);
        const float4 *tp = a.invd2 + t * (kTileElems / 4) + half * 512 + lane;
        float4 wn = tp[0];
        const int2 b = a.tiles[t];
        const float4 *ysrc =
            reinterpret_cast<const float4 *>(a.Y + ((int64_t)b.x * kTile + 32 * half) * kp);
        const float4 *ycsrc = reinterpret_cast<const float4 *>(a.Y + (int64_t)b.y * kTile * kp);
        __builtin_amdgcn_wave_barrier();
        for (int f = lane; f < 8 * kp; f += kWave) yl[f] = ysrc[f];
        for (int f = lane; f < 16 * kp; f += kWave) ycl[f] = ycsrc[f];
        __builtin_amdgcn_wave_barrier();
        const float *yi0 = reinterpret_cast<const float *>(yl);
        const float *yc0 = reinterpret_cast<const float *>(ycl);
        float yj[K], zc[K];
#pragma unroll
        for (int q = 0; q < K; ++q) { yj[q] = yc0[lane * kp + q]; zc[q] = 0.0f; }
        // phase 1, four rows (one weight float4) per step; the next step's
        // weights are loaded ahead
#pragma unroll 1
        for (int g = 0; g < 8; ++g) {
            const float4 w4 = wn;
            if (g < 7) wn = tp[(g + 1) * 64];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int i = 4 * g + rr;
                const float wt = comp4(w4, rr);
                const float *yi = yi0 + i * kp;
                float d[K];
                float acc2 = 0.0f;
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    d[q] = yi[q] - yj[q];
                    acc2 = __builtin_fmaf(d[q], d[q], acc2);
                }
                // r2 > 0 also excludes the masked pairs (1/d^2 < 0)
                const float r2 = acc2 * wt;
                const float rinv = __builtin_amdgcn_rsqf(r2);
                const float rv = r2 * rinv;
                const float ex = __builtin_amdgcn_exp2f(__builtin_fmaf(-rv, c2, Lc));
                const float av = r2 > 0.0f ? ex * wt * rinv : 0.0f;
#pragma unroll
                for (int q = 0; q < K; ++q) zc[q] = __builtin_fmaf(-av, d[q], zc[q]);
                al[i * kAStride + lane] = av;
            }
        }
        float *zcol = a.Zc + h * (int64_t)(K * 64) + lane * K;
#pragma unroll
        for (int q = 0; q < K; ++q) zcol[q] = zc[q];
        __builtin_amdgcn_wave_barrier();
        // phase 2: A[16 mb + c16][4 tt + r4] from LDS, B = Y_J[4 tt + r4][c16]
        double4_t accr0 = {0.0, 0.0, 0.0, 0.0}, accr1 = {0.0, 0.0, 0.0, 0.0};
        double rs0 = 0.0, rs1 = 0.0;
#pragma unroll 4
        for (int tt = 0; tt < 16; ++tt) {
            const int jc = 4 * tt + r4;
            const float yv = yc0[jc * kp + qc];
            const double bq = qin ? (double)yv : bpad;
            const double a0 = (double)alr[4 * tt];
            const double a1 = (double)alr[16 * kAStride + 4 * tt];
            if constexpr (K == 16) {
                rs0 += a0;
                rs1 += a1;
            }
            accr0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bq, accr0, 0, 0, 0);
            accr1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bq, accr1, 0, 0, 0);
        }
        if constexpr (K == 16) {
            rs0 += __shfl_xor(rs0, 16, kWave);
            rs0 += __shfl_xor(rs0, 32, kWave);
            rs1 += __shfl_xor(rs1, 16, kWave);
            rs1 += __shfl_xor(rs1, 32, kWave);
        }
        float *zrow = a.Zr + h * (int64_t)(K * 32);
        // lane holds (A Y_J)[16 mb + r4 + 4 v][c16]; row (r4 + 4 v)'s sum sits
        // in the lanes with c16 = r4 + 4 v (K = 16), or in column 15 of the
        // product, lane (r4, 15) (K < 16)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i0 = r4 + 4 * v, i1 = 16 + r4 + 4 * v;
            double s0, s1;
            if constexpr (K == 16) {
                const int src = (lane & 48) | (r4 + 4 * v);
                s0 = __shfl(rs0, src, kWave);
                s1 = __shfl(rs1, src, kWave);
            } else {
                s0 = __shfl(accr0[v], (lane & 48) | 15, kWave);
                s1 = __shfl(accr1[v], (lane & 48) | 15, kWave);
            }
            const double z0 = s0 * (double)yi0[i0 * kp + qc] - accr0[v];
            const double z1 = s1 * (double)yi0[i1 * kp + qc] - accr1[v];
            if (qin) {
                zrow[i0 * K + c16] = (float)z0;
                zrow[i1 * K + c16] = (float)z1;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// z_p for the 64 points of point block b (one block per point block):
// row-side partials of tiles (b, bj >= b), column-side partials of tiles
// (bi <= b, b), then the short pairs through their CSR segments (pairs with
// i = p add, pairs with j = p subtract).  The four wavefronts split the terms;
// their sums are added in a fixed order.
template <int K>
__global__ __launch_bounds__(kPairBlock) void k_sm_zred(SmArgs a, int64_t nb, int64_t N,
                                                        const int32_t *__restrict__ rp_i,
                                                        const int32_t *__restrict__ rp_j,
                                                        const int32_t *__restrict__ permj,
                                                        double *__restrict__ Z) {
    __shared__ double sz[kPairBlock / kWave][64 * K];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t b = blockIdx.x;
    double z[K];
#pragma unroll
    for (int q = 0; q < K; ++q) z[q] = 0.0;
    const int64_t trow0 = b * nb - b * (b - 1) / 2;   // first tile of row b
    const int half = lane >> 5, rr = lane & 31;
    // two tiles per step, all their loads issued before the adds
    int64_t bj = b + wv;
    for (; bj + 4 < nb; bj += 8) {
        const float *z0 = a.Zr + (2 * (trow0 + bj - b) + half) * (int64_t)(K * 32) + rr * K;
        const float *z1 = z0 + 8 * (int64_t)(K * 32);   // tile bj + 4 of the same row
        float t0[K], t1[K];
#pragma unroll
        for (int q = 0; q < K; ++q) { t0[q] = z0[q]; t1[q] = z1[q]; }
#pragma unroll
        for (int q = 0; q < K; ++q) z[q] += (double)t0[q] + (double)t1[q];
    }
    for (; bj < nb; bj += 4) {
        const float *zp = a.Zr + (2 * (trow0 + bj - b) + half) * (int64_t)(K * 32) + rr * K;
#pragma unroll
        for (int q = 0; q < K; ++q) z[q] += (double)zp[q];
    }
    int64_t bi = wv;
    for (; bi + 4 <= b; bi += 8) {
        const int64_t t0 = bi * nb - bi * (bi - 1) / 2 + (b - bi);
        const int64_t bi1 = bi + 4;
        const int64_t t1 = bi1 * nb - bi1 * (bi1 - 1) / 2 + (b - bi1);
        const float *z0 = a.Zc + 2 * t0 * (int64_t)(K * 64) + lane * K;
        const float *z1 = a.Zc + 2 * t1 * (int64_t)(K * 64) + lane * K;
        float u0[K], u1[K], v0[K], v1[K];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            u0[q] = z0[q]; v0[q] = z0[K * 64 + q];
            u1[q] = z1[q]; v1[q] = z1[K * 64 + q];
        }
#pragma unroll
        for (int q = 0; q < K; ++q) z[q] += ((double)u0[q] + (double)v0[q]) + ((double)u1[q] + (double)v1[q]);
    }
    for (; bi <= b; bi += 4) {
        const int64_t t = bi * nb - bi * (bi - 1) / 2 + (b - bi);
        const float *zp = a.Zc + 2 * t * (int64_t)(K * 64) + lane * K;
#pragma unroll
        for (int q = 0; q < K; ++q) z[q] += (double)zp[q] + (double)zp[K * 64 + q];
    }
    const int64_t p = b * kTile + lane;
    if (a.nclose > 0 && p < N) {
        for (int32_t e = rp_i[p] + wv; e < rp_i[p + 1]; e += 4) {
#pragma unroll
            for (int q = 0; q < K; ++q) z[q] += a.zpair[(int64_t)e * K + q];
        }
        for (int32_t e = rp_j[p] + wv; e < rp_j[p + 1]; e += 4) {
            const int64_t ee = permj[e];
#pragma unroll
            for (int q = 0; q < K; ++q) z[q] -= a.zpair[ee * K + q];
        }
    }
#pragma unroll
    for (int q = 0; q < K; ++q) sz[wv][lane * K + q] = z[q];
    __syncthreads();
    if (wv == 0 && p < N) {
#pragma unroll
        for (int q = 0; q < K; ++q)
            Z[p * K + q] = ((sz[0][lane * K + q] + sz[1][lane * K + q]) + sz[2][lane * K + q]) +
                           sz[3][lane * K + q];
    }
}

#ifndef SAP_KINST
// G_c = sum_{p in chunk c} (x_p - mu) z_p^T (n x K, element e = q n + l) on
// the matrix cores in FP64 (v_mfma_f64_16x16x4f64): output rows are 16
// components l of x, the contraction runs over the chunk's points four at a
// time.  Lane (c16, r4) feeds A = x[p][16 mb + c16] - mu and B = z[p][c16]
// for p = p0 + 4 s + r4; wavefront w takes the component blocks mb = w,
// w + 4, ...  Rows past the chunk and columns past n or K contribute 0
// (selects, not multiplies, so no value of a masked element matters).
template <typename TX>
__global__ __launch_bounds__(256) void k_sm_grad(const TX *__restrict__ X, int64_t ldx, int64_t N,
                                                 int n, int K, const double *__restrict__ mu,
                                                 const double *__restrict__ Z, int64_t rows,
                                                 double *__restrict__ Gpart) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c16 = lane & 15, r4 = lane >> 4;
    const int64_t p0 = (int64_t)blockIdx.x * rows;
    const int64_t p1 = p0 + rows < N ? p0 + rows : N;
    const int64_t nsteps = (p1 - p0 + 3) / 4;
    const int nmb = (n + 15) / 16;
    const bool qin = c16 < K;
    const int qc = qin ? c16 : K - 1;
    double *out = Gpart + (int64_t)blockIdx.x * n * K;
    for (int mb = wv; mb < nmb; mb += 4) {
        const int l = 16 * mb + c16;
        const bool lin = l < n;
        const int lc = lin ? l : n - 1;
        const double ml = mu[lc];
        double4_t acc = {0.0, 0.0, 0.0, 0.0};
        for (int64_t s0 = 0; s0 < nsteps; s0 += 4) {
            double xa[4], zb[4];
            bool pin[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t p = p0 + 4 * (s0 + u) + r4;
                pin[u] = p < p1;
                const int64_t pc = pin[u] ? p : p0;
                xa[u] = (double)X[pc * ldx + lc];
                zb[u] = Z[pc * K + qc];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double av = (pin[u] && lin) ? xa[u] - ml : 0.0;
                const double bv = (pin[u] && qin) ? zb[u] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
        }
        // lane holds G[16 mb + r4 + 4 v][c16]
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int lo = 16 * mb + r4 + 4 * v;
            if (lo < n && qin) out[(int64_t)c16 * n + lo] = acc[v];
        }
    }
}

// dP (n x k row-major FP32) = dL/dloss * sum over the chunks: one block per
// 64 output elements; its four wavefronts take every fourth chunk, with
// eight loads in flight per lane, and their sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_sm_dP(const double *__restrict__ Gpart, int nchunks, int n,
                                               int K, const float *__restrict__ grad_loss,
                                               float *__restrict__ dP) {
    __shared__ double sp[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    const int nk = n * K;
    double acc = 0.0;
    if (e < nk) {
        int c = wv;
        for (; c + 28 < nchunks; c += 32) {
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = Gpart[(int64_t)(c + 4 * u) * nk + e];
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += t[u];
        }
        for (; c < nchunks; c += 4) acc += Gpart[(int64_t)c * nk + e];
    }
    sp[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && e < nk) {
        const int l = e % n, q = e / n;
        const double g = ((sp[0][lane] + sp[1][lane]) + sp[2][lane]) + sp[3][lane];
        dP[(int64_t)l * K + q] = (float)((double)grad_loss[0] * g);
    }
}

#endif

}  // namespace sap
