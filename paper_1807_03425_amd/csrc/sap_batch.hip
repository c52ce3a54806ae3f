// Batched SAP (gfx950): many independent small problems, one workgroup each,
// the whole run of Algorithm 1 (Sec. 4) inside one kernel launch.
//
// The paper applies Algorithm 1 to many small secant sets: for every target
// dimension of a sweep (Sec. 6.1), to random subsamples of a data set whose
// full secant matrix does not fit (Sec. 6.3), and with the length threshold
// of Sec. 7.  Each such problem here is one workgroup of 256 threads that
// loops over the iterations with block barriers only:
//   Y = (X_S - mean_S) P     FP64 on the matrix cores (v_mfma_f64_16x16x4f64),
//                            the set's rows gathered through its index list;
//   pass                     for every 16 x 64 quarter of the set's 64 x 64
//                            tiles: ||y_i - y_j||^2 (FP64 differences) times
//                            the stored FP32 1/d^2, rounded to an FP32 key;
//                            the candidate window of the block's running
//                            minimum, as in the single-problem pass;
//   rescoring                every window pair in FP64 from X (the same
//                            routine as the single-problem pass), lexicographic
//                            (r, i, j) minimum, certificate, trace entry;
//   update                   the FP64 argmax / modified Gram-Schmidt / shift
//                            of the single-problem handle, in LDS.
// Y stays FP64, so the coarse error is that of the FP64 product (no pair is
// too short for it and there is no short-pair list); keys round to FP32.
//
// Scratch (device): per-set index lists, tile tables and 1/d^2 tiles (FP32,
// the single-problem layout), per-set mean / radius / largest kept 1/d^2 /
// pair counts, per-problem P (kp x n FP64, rows >= k zero) and Y
// (Mpad x kp FP64).
#define SAP_KINST 1

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "sap_iter.hip"

namespace sap {

constexpr int kBatchMaxPoints = 32768;
constexpr int kBatchLdsDoubles = 16384;   // the update's (k + 2) n doubles: 128 KB beside the pass's 31 KB

struct BatchSet {        // per point set
    int64_t pt_off;      // first entry of its row-index list
    int64_t tile_off;    // first tile (tile table and 1/d^2 tiles)
    int32_t M, nb;       // points, 64-point blocks
    int32_t ntiles, pad;
};

struct BatchProb {       // per problem
    int32_t set, k, kp, rule;
    double alpha;
    int64_t P_off;       // its kp x n P in Pbuf (doubles)
    int64_t Y_off;       // its Mpad x kp Y in Ybuf (doubles)
    int64_t P0_off;      // its n x k block in the caller's P0 / P_out (doubles)
};

// per-set statistics written by the precomputation
struct BatchStat {
    uint64_t radius_bits;   // max ||x - mean|| (FP64 bits; non-negative)
    uint32_t wmax_bits;     // largest FP32 1/d^2 of a kept pair (bits)
    int32_t nonfinite;
    uint64_t kept, dropped;
};

struct BatchArgs {
    const void *X;
    int64_t ldx;
    int n, vx;
    const int32_t *pts;
    const BatchSet *sets;
    const BatchProb *probs;
    const int4 *tiles;       // (bi, bj, set, 0) per tile
    float4 *w;               // 1/d^2 tiles (kTileElems floats each)
    double *mu;              // n_sets x n
    BatchStat *stat;         // n_sets
    const double *set_min_len;
    double *Pbuf, *Ybuf;
    const double *P0;
    double *P_out;
    int iters, cap;
    double *tr_min;
    int64_t *tr_ij;
    int32_t *tr_cert;
};

// ---------------------------------------------------------------- precomputation

// zero the per-set statistics (a fill kernel, not a memset)
__global__ void k_batch_clear(BatchStat *stat, int n_sets) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_sets) stat[s] = BatchStat{0ull, 0u, 0, 0ull, 0ull};
}

// mean of each set's rows, column by column in point order; flags NaN / Inf
template <typename TX>
__global__ __launch_bounds__(256) void k_batch_mean(BatchArgs a) {
    const int s = blockIdx.y;
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.n) return;
    const BatchSet st = a.sets[s];
    const TX *X = static_cast<const TX *>(a.X);
    double acc = 0.0;
    int bad = 0;
    for (int p = 0; p < st.M; ++p) {
        const double v = (double)X[(int64_t)a.pts[st.pt_off + p] * a.ldx + l];
        if (!isfinite(v)) bad = 1;
        acc += v;
    }
    a.mu[(int64_t)s * a.n + l] = acc / (double)st.M;
    if (bad) atomicOr(&a.stat[s].nonfinite, 1);
}

// radius of each set: one wavefront per point
template <typename TX>
__global__ __launch_bounds__(256) void k_batch_radius(BatchArgs a) {
    const int s = blockIdx.y;
    const BatchSet st = a.sets[s];
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= st.M) return;
    const int lane = threadIdx.x & 63;
    const TX *x = static_cast<const TX *>(a.X) + (int64_t)a.pts[st.pt_off + p] * a.ldx;
    const double *mu = a.mu + (int64_t)s * a.n;
    double acc = 0.0;
    for (int l = lane; l < a.n; l += kWave) {
        const double t = (double)x[l] - mu[l];
        acc += t * t;
    }
    acc = wave_sum(acc);
    if (lane == 0) atomicMax(reinterpret_cast<unsigned long long *>(&a.stat[s].radius_bits),
                             (unsigned long long)__double_as_longlong(sqrt(acc)));
}

// 1/d^2 tiles of every set, by direct FP64 differences of the gathered rows
// (the single-problem layout: element (r, c) of a tile at float index
// (r/4)*256 + c*4 + r%4).  Dropped pairs (duplicates, d < the set's l) and
// padding / i >= j hold -1.  Counts kept and dropped pairs per set and folds
// the largest kept FP32 value into the set's statistics.
template <typename TX>
__global__ __launch_bounds__(256) void k_batch_invd2(BatchArgs a, int64_t ntiles_all) {
    __shared__ unsigned long long s_kept, s_drop;
    __shared__ unsigned s_wmax;
    const int c = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const TX *X = static_cast<const TX *>(a.X);
    for (int64_t t = blockIdx.x; t < ntiles_all; t += gridDim.x) {
        if (threadIdx.x == 0) { s_kept = 0; s_drop = 0; s_wmax = 0u; }
        __syncthreads();
        const int4 tb = a.tiles[t];
        const BatchSet st = a.sets[tb.z];
        const double ml = a.set_min_len ? a.set_min_len[tb.z] : 0.0;
        const int32_t *idx = a.pts + st.pt_off;
        const int64_t j = (int64_t)tb.y * kTile + c;
        const bool jin = j < st.M;
        const TX *xj = X + (int64_t)idx[jin ? j : st.M - 1] * a.ldx;
        unsigned mx = 0u;
        for (int m = 0; m < 4; ++m) {
            const int g = w + 4 * m;
            const int64_t i0 = (int64_t)tb.x * kTile + 4 * g;
            const TX *xi[4];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) xi[rr] = X + (int64_t)idx[i0 + rr < st.M ? i0 + rr : st.M - 1] * a.ldx;
            double d2[4] = {0.0, 0.0, 0.0, 0.0};
            if (jin) {
                for (int l = 0; l < a.n; ++l) {
                    const double xv = (double)xj[l];
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const double t2 = (double)xi[rr][l] - xv;
                        d2[rr] += t2 * t2;
                    }
                }
            }
            float out[4];
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int64_t i = i0 + rr;
                float v = kMaskDropped;
                if (jin && i < j) {
                    const double d = sqrt(d2[rr]);
                    if (d == 0.0 || d < ml) {
                        atomicAdd(&s_drop, 1ull);
                    } else {
                        v = (float)(1.0 / d2[rr]);
                        atomicAdd(&s_kept, 1ull);
                        mx = max(mx, __float_as_uint(v));
                    }
                }
                out[rr] = v;
            }
            a.w[t * (kTileElems / 4) + g * 64 + c] = make_float4(out[0], out[1], out[2], out[3]);
        }
        atomicMax(&s_wmax, mx);
        __syncthreads();
        if (threadIdx.x == 0) {
            BatchStat *so = a.stat + tb.z;
            if (s_kept) atomicAdd(reinterpret_cast<unsigned long long *>(&so->kept), s_kept);
            if (s_drop) atomicAdd(reinterpret_cast<unsigned long long *>(&so->dropped), s_drop);
            if (s_wmax) atomicMax(&so->wmax_bits, s_wmax);
        }
        __syncthreads();
    }
}

// P0 blocks (n x k row-major) -> per-problem P (kp x n, rows >= k zero)
__global__ void k_batch_loadP(BatchArgs a) {
    const BatchProb pr = a.probs[blockIdx.y];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = a.n;
    if (e >= pr.kp * n) return;
    const int q = e / n, l = e % n;
    a.Pbuf[pr.P_off + e] = q < pr.k ? a.P0[pr.P0_off + (int64_t)l * pr.k + q] : 0.0;
}

// per-problem P (kp x n) -> P_out blocks (n x k row-major)
__global__ void k_batch_storeP(BatchArgs a) {
    const BatchProb pr = a.probs[blockIdx.y];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= pr.k * a.n) return;
    const int l = e / pr.k, q = e % pr.k;
    a.P_out[pr.P0_off + e] = a.Pbuf[pr.P_off + (int64_t)q * a.n + l];
}

// ---------------------------------------------------------------- the run

// 16 rows of Y = (X_S - mean) P in FP64 (rows row0 .. row0 + 15 of the set;
// rows >= M are zero), KP columns (P rows >= k are zero).  The MFMA tiling of
// gemm_block, the rows gathered through the set's index list.
template <typename TX, int KP>
__device__ __forceinline__ void batch_gemm16(const TX *__restrict__ X, int64_t ldx, const int32_t *__restrict__ idx,
                                             int M, int n, const double *__restrict__ mu,
                                             const double *__restrict__ P, double *__restrict__ Y, int row0,
                                             bool vx, bool vp) {
    const int lane = threadIdx.x & 63;
    const int m = lane & 15, kk = lane >> 4;
    const int row = row0 + m;
    const bool rin = row < M;
    const double rmask = rin ? 1.0 : 0.0, pmask = m < KP ? 1.0 : 0.0;
    const TX *xr = X + (int64_t)idx[rin ? row : M - 1] * ldx;
    const double *pc = P + (int64_t)(m < KP ? m : KP - 1) * n;
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    int l0 = 0;
    for (; l0 + 64 <= n; l0 += 64) {
        double xa[16], ma[16], pb[16];
        const int lb = l0 + 16 * kk;
        load16(xr + lb, vx, xa);
        load16(mu + lb, true, ma);
        load16(pc + lb, vp, pb);
#pragma unroll
        for (int s = 0; s < 16; ++s)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64((xa[s] - ma[s]) * rmask, pb[s] * pmask, acc, 0, 0, 0);
    }
    for (; l0 < n; l0 += 4) {
        const int l = l0 + kk;
        double x = 0.0, p = 0.0;
        if (l < n) {
            if (rin) x = (double)xr[l] - mu[l];
            if (m < KP) p = pc[l];
        }
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, p, acc, 0, 0, 0);
    }
    if (m < KP) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = row0 + kk + 4 * v;
            Y[(int64_t)r * KP + m] = r < M ? acc[v] : 0.0;
        }
    }
}

// The FP64 update of Algorithm 1 for the exact k (K_LO <= k <= K_HI), with
// P (k x n) staged in LDS and written back to P (global, rows 0..k-1): the
// single-problem handle's routines -- one wavefront with the vectors in
// registers when n <= 64 and k <= 8, the whole block over LDS otherwise.
// Every thread of the block calls it.
template <typename TX, int K_LO, int K_HI>
__device__ __forceinline__ void batch_update(const TX *X, int64_t ldx, int n, int k, double *P, double alpha, int rule,
                                             int64_t gi, int64_t gj, double *sm) {
    if constexpr (K_LO <= K_HI) {
        if (k == K_LO) {
            if (K_LO <= 8 && n <= kWave) {
                if (threadIdx.x < kWave)
                    apply_update_reg<K_LO, 1, TX>(X, ldx, n, sm, P, nullptr, 0, alpha, rule, nullptr, gi, gj, false);
            } else {
                apply_update<K_LO, TX>(X, ldx, n, P, nullptr, 0, alpha, rule, nullptr, gi, gj, sm);
            }
        } else {
            batch_update<TX, K_LO + 1, K_HI>(X, ldx, n, k, P, alpha, rule, gi, gj, sm);
        }
    }
}

template <int KP> struct KRange;
template <> struct KRange<2> { static constexpr int lo = 1, hi = 2; };
template <> struct KRange<4> { static constexpr int lo = 3, hi = 4; };
template <> struct KRange<8> { static constexpr int lo = 5, hi = 8; };
template <> struct KRange<12> { static constexpr int lo = 9, hi = 12; };
template <> struct KRange<16> { static constexpr int lo = 13, hi = 16; };

// LDS of a problem's pass, declared once in the kernel (the five KP variants
// share it): every wavefront's staged y_i rows and candidate list, the
// block's running minimum and its result.
struct BatchLds {
    double y[kPairBlock / kWave][16 * kMaxK];
    int2 cij[kPairBlock / kWave][kCandCap];
    uint32_t ckey[kPairBlock / kWave][kCandCap];
    uint32_t run;
    Partial fin;
};

// Tile (bi, bj), bi <= bj, of index t in the row-major order of a set's
// nb x nb upper triangle (t = bi nb - bi (bi - 1) / 2 + bj - bi): bi from the
// quadratic, corrected by at most a step each way.  Wavefront-uniform.
__device__ __forceinline__ int2 tile_of_index(int64_t t, int nb) {
    auto start = [nb](int64_t b) { return b * nb - b * (b - 1) / 2; };
    const double q = 2.0 * nb + 1.0;
    int64_t bi = (int64_t)floor((q - sqrt(fmax(q * q - 8.0 * (double)t, 0.0))) * 0.5);
    bi = bi < 0 ? 0 : (bi > nb - 1 ? nb - 1 : bi);
    while (bi > 0 && start(bi) > t) --bi;
    while (bi + 1 < nb && start(bi + 1) <= t) ++bi;
    return make_int2((int)bi, (int)(bi + (t - start(bi))));
}

// One problem, the whole run.  Every thread of the block calls it.
template <int KP, typename TX>
__device__ void batch_problem(const BatchArgs &a, int b, double *sm, BatchLds &L) {
    constexpr int NY = (16 * KP + kWave - 1) / kWave;   // doubles of an item's y_i rows per lane
    auto &s_y = L.y;
    auto &s_cij = L.cij;
    auto &s_ckey = L.ckey;
    uint32_t &s_run = L.run;
    Partial &s_fin = L.fin;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const BatchProb pr = a.probs[b];
    const BatchSet st = a.sets[pr.set];
    const BatchStat bs = a.stat[pr.set];
    const int n = a.n, k = pr.k, M = st.M;
    const TX *X = static_cast<const TX *>(a.X);
    const int32_t *idx = a.pts + st.pt_off;
    double *P = a.Pbuf + pr.P_off;
    double *Y = a.Ybuf + pr.Y_off;
    const double *mu = a.mu + (int64_t)pr.set * n;
    const float4 *wt = a.w + st.tile_off * (kTileElems / 4);
    const bool vp = (n & 1) == 0;
    // coarse error bound |r~ - r| <= e_abs + e_rel r: the FP64 product's
    // error on y (norm over the k columns) and the FP32 rounding of 1/d^2
    // and of the key
    const double R = __longlong_as_double((long long)bs.radius_bits);
    const double delta = R * (double)(n + 2) * sqrt((double)k) * 1.1102230246251565e-16 * 4.0;
    const double wmax = (double)__uint_as_float(bs.wmax_bits);
    const double e_abs = bs.wmax_bits ? 2.0 * delta * sqrt(wmax * (1.0 + 2.384185791015625e-07)) : 0.0;
    const double e_rel = 2.0 * 5.9604644775390625e-08 + (KP + 4) * 1.1102230246251565e-16;
    float wa = (float)((1.0 + e_rel) / (1.0 - e_rel));
    wa = __uint_as_float(__float_as_uint(wa) + 1u);
    float wbb = (float)(2.0 * e_abs / (1.0 - e_rel));
    wbb = __uint_as_float(__float_as_uint(wbb) + 1u);
    const int64_t nitem = (int64_t)st.ntiles * 4;        // quarter tiles
    const int iters = a.iters;
    const int64_t tr0 = (int64_t)b * (iters + 1);
    for (int it = 0; it <= iters; ++it) {
        // Y = (X_S - mean) P
        for (int slab = wv; slab < st.nb * 4; slab += kPairBlock / kWave)
            batch_gemm16<TX, KP>(X, a.ldx, idx, M, n, mu, P, Y, slab * 16, a.vx, vp);
        if (threadIdx.x == 0) s_run = kKeyNone;
        __syncthreads();
        // pass: wavefront wv takes quarter tiles wv, wv + 4, ...; the loads of
        // the next item are issued before the current item's arithmetic, and
        // every load of an item is independent (tile coordinates computed,
        // not loaded)
        WaveBest wb{__builtin_huge_val(), __builtin_huge_val(), 0x7fffffff, 0x7fffffff, 0, 0, 0};
        CandList cl{s_cij[wv], s_ckey[wv], 0, a.cap, 0, kKeyNone};
        uint32_t kmin = kKeyNone;
        double *yl = s_y[wv];
        struct ItemLoads {
            float4 w4[4];
            double yr[NY];
            double yj[KP];
            int32_t row0, col;
        };
        auto fetch = [&](int64_t hh, ItemLoads &L) __attribute__((always_inline)) {
            const int64_t t = hh >> 2;
            const int q = (int)(hh & 3);
            const int2 tc = tile_of_index(t, st.nb);
            const float4 *tp = wt + t * (kTileElems / 4) + q * 256 + lane;
#pragma unroll
            for (int g = 0; g < 4; ++g) L.w4[g] = tp[g * 64];
            L.row0 = tc.x * kTile + 16 * q;
            L.col = tc.y * kTile + lane;
            const double *ysrc = Y + (int64_t)L.row0 * KP;
#pragma unroll
            for (int u = 0; u < NY; ++u) {
                const int f = lane + u * kWave;
                L.yr[u] = ysrc[f < 16 * KP ? f : 0];
            }
#pragma unroll
            for (int c = 0; c < KP; ++c) L.yj[c] = Y[(int64_t)L.col * KP + c];
        };
        ItemLoads cur, nxt;
        int64_t h = wv;
        if (h < nitem) fetch(h, cur);
        nxt = cur;
        for (; h < nitem; h += kPairBlock / kWave) {
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int u = 0; u < NY; ++u) {
                const int f = lane + u * kWave;
                if (f < 16 * KP) yl[f] = cur.yr[u];
            }
            __builtin_amdgcn_wave_barrier();
            if (h + kPairBlock / kWave < nitem) fetch(h + kPairBlock / kWave, nxt);
            uint32_t key[16];
            uint32_t lmin = kKeyNone;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const double *yi = yl + e * KP;
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < KP; ++c) {
                    const double d = yi[c] - cur.yj[c];
                    acc = __builtin_fma(d, d, acc);
                }
                const float4 &wg = cur.w4[e >> 2];
                const float wv4 = (e & 3) == 0 ? wg.x : (e & 3) == 1 ? wg.y : (e & 3) == 2 ? wg.z : wg.w;
                key[e] = __float_as_uint((float)(acc * (double)wv4));
                lmin = min(lmin, key[e]);
            }
            const uint32_t m = wave_min_u32_fast(lmin);
            kmin = min(kmin, m);
            const uint32_t T2 = item_window(block_run_min(&s_run, m), wa, wbb);
            const int32_t row0 = cur.row0, col = cur.col;
            if (m <= T2)
                emit_cands(cl, key, lmin, T2,
                           [=](int e, int32_t &i, int32_t &j) __attribute__((always_inline)) {
                               i = row0 + e;
                               j = col;
                           },
                           wb);
            __builtin_amdgcn_wave_barrier();
            cur = nxt;
        }
        // rescore the window pairs in FP64 from X
        {
            const uint32_t run = __builtin_amdgcn_readfirstlane(*(const volatile uint32_t *)&s_run);
            if (run < 0x7f800000u) {
                const uint32_t T2b = item_window(run, wa, wbb);
                __builtin_amdgcn_wave_barrier();
#pragma unroll 1
                for (int c = 0; c < cl.n; ++c) {
                    const uint32_t kv = cl.key[c];
                    if (kv > T2b) continue;
                    const int2 ij = cl.ij[c];
                    const double r = exact_r_wave<KP, TX>(X, a.ldx, n, P, idx[ij.x], idx[ij.y]);
                    ++wb.nwin;
                    wb.nviol += bound_broken(r, (double)__uint_as_float(kv), e_abs, e_rel);
                    if (lex_less(r, ij.x, ij.y, wb.r, wb.i, wb.j)) {
                        wb.r2 = wb.r;
                        wb.r = r; wb.i = ij.x; wb.j = ij.y;
                    } else {
                        wb.r2 = fmin(wb.r2, r);
                    }
                }
            }
            wb.nviol += cl.lost;
            block_reduce_partial(wb.r, wb.i, wb.j, wb.r2, lane == 0 ? wb.nwin : 0, lane == 0 ? wb.nunits : 0,
                                 lane == 0 ? wb.nviol : 0, kmin, cl.limit, &s_fin, true);
        }
        const Partial f = s_fin;
        const bool found = f.r < __builtin_huge_val();
        if (threadIdx.x == 0) {
            const uint32_t wkey = f.kmin < 0x7f800000u ? item_window(f.kmin, wa, wbb) : 0u;
            const int cert = (found && f.n_viol == 0 && f.limit >= wkey) ? 1 : 0;
            a.tr_min[tr0 + it] = f.r;
            if (a.tr_ij) {
                a.tr_ij[2 * (tr0 + it)] = found ? f.i : -1;
                a.tr_ij[2 * (tr0 + it) + 1] = found ? f.j : -1;
            }
            if (a.tr_cert) a.tr_cert[tr0 + it] = cert;
        }
        if (it == iters || !found) {
            if (it < iters) {
                // no kept pair: the remaining entries repeat this one
                if (threadIdx.x == 0)
                    for (int r = it + 1; r <= iters; ++r) {
                        a.tr_min[tr0 + r] = f.r;
                        if (a.tr_ij) { a.tr_ij[2 * (tr0 + r)] = -1; a.tr_ij[2 * (tr0 + r) + 1] = -1; }
                        if (a.tr_cert) a.tr_cert[tr0 + r] = 0;
                    }
            }
            break;
        }
        // the update, in LDS
        stage_P(P, k * n, sm);
        __syncthreads();
        batch_update<TX, KRange<KP>::lo, KRange<KP>::hi>(X, a.ldx, n, k, P, pr.alpha, pr.rule, idx[f.i], idx[f.j],
                                                         sm);
        __syncthreads();
    }
}

// One workgroup per problem.  Dynamic LDS: the update's (k + 2) n doubles.
template <typename TX>
__global__ __launch_bounds__(kPairBlock) void k_batch_run(BatchArgs a) {
    extern __shared__ __align__(16) double sm_batch[];
    __shared__ BatchLds L;
    const int b = blockIdx.x;
    switch (a.probs[b].kp) {
        case 2: batch_problem<2, TX>(a, b, sm_batch, L); break;
        case 4: batch_problem<4, TX>(a, b, sm_batch, L); break;
        case 8: batch_problem<8, TX>(a, b, sm_batch, L); break;
        case 12: batch_problem<12, TX>(a, b, sm_batch, L); break;
        default: batch_problem<16, TX>(a, b, sm_batch, L); break;
    }
}

}  // namespace sap

// ---------------------------------------------------------------- host

using namespace sap;

namespace {

thread_local std::string t_err;

sap_status bfail(sap_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    sap_internal_set_error(buf);
    return st;
}

#define B_HIP(expr)                                                                              \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            (void)hipGetLastError();                                                             \
            return bfail(e_ == hipErrorOutOfMemory ? SAP_ERR_OUT_OF_MEMORY : SAP_ERR_DEVICE,     \
                         "%s: %s", #expr, hipGetErrorString(e_));                                \
        }                                                                                        \
    } while (0)

int kp_of(int k) { return k <= 2 ? 2 : k <= 4 ? 4 : k <= 8 ? 8 : k <= 12 ? 12 : 16; }

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Host-side plan of one batch call: validated tables and the scratch layout.
struct BatchPlan {
    std::vector<BatchSet> sets;
    std::vector<BatchProb> probs;
    std::vector<int4> tiles;
    std::vector<int32_t> pts;
    std::vector<double> minlen;
    int64_t ntiles_all = 0, P_total = 0, Y_total = 0, P0_total = 0;
    size_t lds = 0;
    // scratch offsets (bytes)
    size_t o_pts, o_sets, o_probs, o_tiles, o_w, o_mu, o_stat, o_minlen, o_P, o_Y, total;
};

sap_status plan_batch(const void *X, int32_t dtype, int64_t N, int32_t n, int64_t ldx, int32_t n_sets,
                      const int64_t *set_offsets, const int32_t *set_points, const double *set_min_len,
                      int32_t n_problems, const sap_batch_problem *problems, const double *P0, int32_t iters,
                      int32_t cand_cap, double *P_out, double *min_trace, BatchPlan &pl) {
    if (!X || !set_offsets || !set_points || !problems || !P0 || !P_out || !min_trace)
        return bfail(SAP_ERR_INVALID_ARG, "sap_batch_run: null pointer argument");
    if (dtype != SAP_F64 && dtype != SAP_F32) return bfail(SAP_ERR_INVALID_ARG, "dtype must be SAP_F64 or SAP_F32");
    if (N < 2 || N >= (1ll << 31)) return bfail(SAP_ERR_INVALID_ARG, "N must lie in [2, 2^31)");
    if (n < 1) return bfail(SAP_ERR_INVALID_ARG, "n must be >= 1");
    if (ldx < n) return bfail(SAP_ERR_INVALID_ARG, "ldx must be >= n");
    if (n_sets < 1 || n_problems < 1) return bfail(SAP_ERR_INVALID_ARG, "n_sets and n_problems must be >= 1");
    if (n_problems > 65535) return bfail(SAP_ERR_UNSUPPORTED, "at most 65535 problems per call");
    if (iters < 0) return bfail(SAP_ERR_INVALID_ARG, "iters must be >= 0");
    if (cand_cap < 0 || cand_cap > kCandCap) return bfail(SAP_ERR_INVALID_ARG, "cand_cap must lie in [0, %d]", kCandCap);
    if (set_offsets[0] != 0) return bfail(SAP_ERR_INVALID_ARG, "set_offsets[0] must be 0");
    pl.sets.resize(n_sets);
    pl.minlen.resize(n_sets);
    for (int s = 0; s < n_sets; ++s) {
        const int64_t M = set_offsets[s + 1] - set_offsets[s];
        if (M < 2 || M > kBatchMaxPoints)
            return bfail(SAP_ERR_INVALID_ARG, "set %d has %lld points: need 2 .. %d", s, (long long)M, kBatchMaxPoints);
        const double ml = set_min_len ? set_min_len[s] : 0.0;
        if (!(ml >= 0.0) || !std::isfinite(ml)) return bfail(SAP_ERR_INVALID_ARG, "set_min_len[%d] must be finite, >= 0", s);
        pl.minlen[s] = ml;
        BatchSet &b = pl.sets[s];
        b.pt_off = set_offsets[s];
        b.M = (int32_t)M;
        b.nb = (int32_t)((M + kTile - 1) / kTile);
        b.ntiles = b.nb * (b.nb + 1) / 2;
        b.tile_off = pl.ntiles_all;
        b.pad = 0;
        for (int bi = 0; bi < b.nb; ++bi)
            for (int bj = bi; bj < b.nb; ++bj) pl.tiles.push_back(make_int4(bi, bj, s, 0));
        pl.ntiles_all += b.ntiles;
    }
    const int64_t npts = set_offsets[n_sets];
    pl.pts.assign(set_points, set_points + npts);
    for (int64_t e = 0; e < npts; ++e)
        if (pl.pts[e] < 0 || pl.pts[e] >= N)
            return bfail(SAP_ERR_INVALID_ARG, "set_points[%lld] = %d is not a row of X", (long long)e, pl.pts[e]);
    pl.probs.resize(n_problems);
    size_t lds = 0;
    for (int b = 0; b < n_problems; ++b) {
        const sap_batch_problem &q = problems[b];
        if (q.set < 0 || q.set >= n_sets) return bfail(SAP_ERR_INVALID_ARG, "problem %d: set %d out of range", b, q.set);
        if (q.k < 1 || q.k > n) return bfail(SAP_ERR_INVALID_ARG, "problem %d: k = %d outside [1, n]", b, q.k);
        if (q.k > kMaxK) return bfail(SAP_ERR_UNSUPPORTED, "problem %d: k > %d", b, kMaxK);
        if ((int64_t)n * (q.k + 2) > kBatchLdsDoubles)
            return bfail(SAP_ERR_UNSUPPORTED, "problem %d: n (k + 2) must be <= %d", b, kBatchLdsDoubles);
        if (!(q.alpha >= 0.0 && q.alpha <= 1.0)) return bfail(SAP_ERR_INVALID_ARG, "problem %d: alpha outside [0, 1]", b);
        if (q.rule != SAP_STEP_LITERAL && q.rule != SAP_STEP_NORMALIZED)
            return bfail(SAP_ERR_INVALID_ARG, "problem %d: bad rule", b);
        BatchProb &p = pl.probs[b];
        p.set = q.set;
        p.k = q.k;
        p.kp = kp_of(q.k);
        p.rule = q.rule;
        p.alpha = q.alpha;
        p.P_off = pl.P_total;
        p.Y_off = pl.Y_total;
        p.P0_off = pl.P0_total;
        pl.P_total += align_up((int64_t)p.kp * n, 32);
        pl.Y_total += (int64_t)pl.sets[q.set].nb * kTile * p.kp;
        pl.P0_total += (int64_t)n * q.k;
        lds = std::max(lds, sizeof(double) * (size_t)n * (q.k + 2));
    }
    pl.lds = lds;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off = (size_t)align_up((int64_t)(off + bytes), 256); return o; };
    pl.o_pts = take(sizeof(int32_t) * npts);
    pl.o_sets = take(sizeof(BatchSet) * n_sets);
    pl.o_probs = take(sizeof(BatchProb) * n_problems);
    pl.o_tiles = take(sizeof(int4) * pl.ntiles_all);
    pl.o_w = take(sizeof(float) * (size_t)pl.ntiles_all * kTileElems);
    pl.o_mu = take(sizeof(double) * (size_t)n_sets * n);
    pl.o_stat = take(sizeof(BatchStat) * n_sets);
    pl.o_minlen = take(sizeof(double) * n_sets);
    pl.o_P = take(sizeof(double) * (size_t)pl.P_total);
    pl.o_Y = take(sizeof(double) * (size_t)pl.Y_total);
    pl.total = off;
    (void)iters;
    return SAP_OK;
}

sap_status check_P0(const BatchPlan &pl, int n, const double *P0, hipStream_t stream) {
    std::vector<double> h((size_t)pl.P0_total);
    B_HIP(hipMemcpyAsync(h.data(), P0, sizeof(double) * h.size(), hipMemcpyDeviceToHost, stream));
    B_HIP(hipStreamSynchronize(stream));
    for (size_t b = 0; b < pl.probs.size(); ++b) {
        const BatchProb &p = pl.probs[b];
        const double *P = h.data() + p.P0_off;
        double e = 0.0;
        for (int l = 0; l < n * p.k; ++l)
            if (!std::isfinite(P[l])) return bfail(SAP_ERR_NONFINITE, "problem %zu: P0 holds NaN or Inf", b);
        for (int x = 0; x < p.k; ++x)
            for (int y = 0; y < p.k; ++y) {
                double acc = 0.0;
                for (int l = 0; l < n; ++l) acc += P[(size_t)l * p.k + x] * P[(size_t)l * p.k + y];
                e = std::max(e, std::fabs(acc - (x == y ? 1.0 : 0.0)));
            }
        if (e > 1e-6) return bfail(SAP_ERR_NOT_ORTHONORMAL, "problem %zu: max |P0^T P0 - I| = %.3g > 1e-6", b, e);
    }
    return SAP_OK;
}

// Enqueue the whole batch on `stream` with the scratch at `base` (pl.total
// bytes), and wait for it.
sap_status run_batch(const BatchPlan &pl, char *base, const void *X, int32_t dtype, int64_t ldx, int32_t n,
                     int32_t n_sets, int32_t n_problems, const double *P0, int32_t iters, int32_t cand_cap,
                     double *P_out, double *min_trace, int64_t *ij_trace, int32_t *cert_trace, hipStream_t stream,
                     sap_batch_stats *stats, bool timed) {
    BatchArgs a{};
    a.X = X;
    a.ldx = ldx;
    a.n = n;
    const size_t es = dtype == SAP_F64 ? 8 : 4;
    a.vx = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && ((size_t)ldx * es) % 16 == 0;
    a.pts = reinterpret_cast<const int32_t *>(base + pl.o_pts);
    a.sets = reinterpret_cast<const BatchSet *>(base + pl.o_sets);
    a.probs = reinterpret_cast<const BatchProb *>(base + pl.o_probs);
    a.tiles = reinterpret_cast<const int4 *>(base + pl.o_tiles);
    a.w = reinterpret_cast<float4 *>(base + pl.o_w);
    a.mu = reinterpret_cast<double *>(base + pl.o_mu);
    a.stat = reinterpret_cast<BatchStat *>(base + pl.o_stat);
    a.set_min_len = reinterpret_cast<const double *>(base + pl.o_minlen);
    a.Pbuf = reinterpret_cast<double *>(base + pl.o_P);
    a.Ybuf = reinterpret_cast<double *>(base + pl.o_Y);
    a.P0 = P0;
    a.P_out = P_out;
    a.iters = iters;
    a.cap = cand_cap > 0 ? cand_cap : kCandCap;
    a.tr_min = min_trace;
    a.tr_ij = ij_trace;
    a.tr_cert = cert_trace;
    B_HIP(hipMemcpyAsync(base + pl.o_pts, pl.pts.data(), sizeof(int32_t) * pl.pts.size(), hipMemcpyHostToDevice, stream));
    B_HIP(hipMemcpyAsync(base + pl.o_sets, pl.sets.data(), sizeof(BatchSet) * pl.sets.size(), hipMemcpyHostToDevice, stream));
    B_HIP(hipMemcpyAsync(base + pl.o_probs, pl.probs.data(), sizeof(BatchProb) * pl.probs.size(), hipMemcpyHostToDevice,
                         stream));
    B_HIP(hipMemcpyAsync(base + pl.o_tiles, pl.tiles.data(), sizeof(int4) * pl.tiles.size(), hipMemcpyHostToDevice, stream));
    B_HIP(hipMemcpyAsync(base + pl.o_minlen, pl.minlen.data(), sizeof(double) * pl.minlen.size(), hipMemcpyHostToDevice,
                         stream));
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
    if (timed) {
        B_HIP(hipEventCreate(&e0));
        B_HIP(hipEventCreate(&e1));
        B_HIP(hipEventCreate(&e2));
        B_HIP(hipEventRecord(e0, stream));
    }
    auto launched = [&](const char *what) -> sap_status {
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return bfail(SAP_ERR_DEVICE, "launch of %s: %s", what, hipGetErrorString(e));
        return SAP_OK;
    };
    sap_status st = SAP_OK;
    hipLaunchKernelGGL(k_batch_clear, dim3((n_sets + 255) / 256), dim3(256), 0, stream, a.stat, n_sets);
    if ((st = launched("k_batch_clear")) != SAP_OK) return st;
    int maxM = 0;
    for (const BatchSet &s : pl.sets) maxM = std::max(maxM, s.M);
    const dim3 gm((unsigned)((n + 255) / 256), (unsigned)n_sets), gr((unsigned)((maxM + 3) / 4), (unsigned)n_sets);
    const unsigned gt = (unsigned)std::min<int64_t>(pl.ntiles_all, 8192);
    if (dtype == SAP_F64) {
        hipLaunchKernelGGL(k_batch_mean<double>, gm, dim3(256), 0, stream, a);
        hipLaunchKernelGGL(k_batch_radius<double>, gr, dim3(256), 0, stream, a);
        hipLaunchKernelGGL(k_batch_invd2<double>, dim3(gt), dim3(256), 0, stream, a, pl.ntiles_all);
    } else {
        hipLaunchKernelGGL(k_batch_mean<float>, gm, dim3(256), 0, stream, a);
        hipLaunchKernelGGL(k_batch_radius<float>, gr, dim3(256), 0, stream, a);
        hipLaunchKernelGGL(k_batch_invd2<float>, dim3(gt), dim3(256), 0, stream, a, pl.ntiles_all);
    }
    if ((st = launched("batch precomputation")) != SAP_OK) return st;
    int kpmax = 0;
    for (const BatchProb &p : pl.probs) kpmax = std::max(kpmax, p.kp);
    hipLaunchKernelGGL(k_batch_loadP, dim3((unsigned)((kpmax * n + 255) / 256), (unsigned)n_problems), dim3(256), 0,
                       stream, a);
    if ((st = launched("k_batch_loadP")) != SAP_OK) return st;
    // inputs checked before the run: finite rows, kept pairs
    {
        std::vector<BatchStat> hs(n_sets);
        B_HIP(hipMemcpyAsync(hs.data(), a.stat, sizeof(BatchStat) * n_sets, hipMemcpyDeviceToHost, stream));
        B_HIP(hipStreamSynchronize(stream));
        int64_t kept = 0;
        for (int s = 0; s < n_sets; ++s) {
            if (hs[s].nonfinite) return bfail(SAP_ERR_NONFINITE, "set %d: X holds NaN or Inf", s);
        }
        for (const BatchProb &p : pl.probs) kept += (int64_t)hs[p.set].kept;
        if (stats) stats->n_pairs = kept;
    }
    if (timed) B_HIP(hipEventRecord(e1, stream));
    const void *fn = dtype == SAP_F64 ? reinterpret_cast<const void *>(&k_batch_run<double>)
                                      : reinterpret_cast<const void *>(&k_batch_run<float>);
    B_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds));
    if (dtype == SAP_F64)
        hipLaunchKernelGGL(k_batch_run<double>, dim3((unsigned)n_problems), dim3(kPairBlock), (uint32_t)pl.lds, stream, a);
    else
        hipLaunchKernelGGL(k_batch_run<float>, dim3((unsigned)n_problems), dim3(kPairBlock), (uint32_t)pl.lds, stream, a);
    if ((st = launched("k_batch_run")) != SAP_OK) return st;
    if (timed) B_HIP(hipEventRecord(e2, stream));
    hipLaunchKernelGGL(k_batch_storeP, dim3((unsigned)((kpmax * n + 255) / 256), (unsigned)n_problems), dim3(256), 0,
                       stream, a);
    if ((st = launched("k_batch_storeP")) != SAP_OK) return st;
    B_HIP(hipStreamSynchronize(stream));
    if (stats) {
        stats->init_ms = -1.0;
        stats->run_ms = -1.0;
        stats->scratch_bytes = (int64_t)pl.total;
    }
    if (timed) {
        float t1 = 0.0f, t2 = 0.0f;
        B_HIP(hipEventElapsedTime(&t1, e0, e1));
        B_HIP(hipEventElapsedTime(&t2, e1, e2));
        stats->init_ms = t1;
        stats->run_ms = t2;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipEventDestroy(e2);
    }
    (void)n;
    return SAP_OK;
}

}  // namespace

extern "C" sap_status sap_batch_run(const void *X, int32_t dtype, int64_t N, int32_t n, int64_t ldx, int32_t n_sets,
                                    const int64_t *set_offsets, const int32_t *set_points, const double *set_min_len,
                                    int32_t n_problems, const sap_batch_problem *problems, const double *P0,
                                    int32_t iters, int32_t cand_cap, double *P_out, double *min_trace,
                                    int64_t *ij_trace, int32_t *cert_trace, void *stream, sap_batch_stats *stats) {
    BatchPlan pl;
    sap_status st = plan_batch(X, dtype, N, n, ldx, n_sets, set_offsets, set_points, set_min_len, n_problems, problems,
                               P0, iters, cand_cap, P_out, min_trace, pl);
    if (st != SAP_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = check_P0(pl, n, P0, s)) != SAP_OK) return st;
    void *base = nullptr;
    hipError_t e = hipMalloc(&base, pl.total);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return bfail(e == hipErrorOutOfMemory ? SAP_ERR_OUT_OF_MEMORY : SAP_ERR_DEVICE, "hipMalloc(%zu bytes): %s",
                     pl.total, hipGetErrorString(e));
    }
    st = run_batch(pl, static_cast<char *>(base), X, dtype, ldx, n, n_sets, n_problems, P0, iters, cand_cap, P_out,
                   min_trace, ij_trace, cert_trace, s, stats, stats != nullptr);
    (void)hipStreamSynchronize(s);
    (void)hipFree(base);
    return st;
}

// ---------------------------------------------------------------- allocation-free variant

// The scratch of sap_batch_run_noalloc: a fixed array in device memory.  In
// host code its name only stands for the symbol; its address on a device is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and that address is what the kernels are given.  Each device holds its own
// copy until the process ends; every call on one device shares it.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<char *> g_scratch_ptr;   // per device id: the array's device address

sap_status static_scratch(char **out) {
    int dev = 0;
    B_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (!g_scratch_ptr[(size_t)dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return bfail(SAP_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        }
        g_scratch_ptr[(size_t)dev] = static_cast<char *>(p);
    }
    *out = g_scratch_ptr[(size_t)dev];
    return SAP_OK;
}
}  // namespace

extern "C" sap_status sap_batch_run_noalloc(const void *X, int32_t dtype, int64_t N, int32_t n, int64_t ldx,
                                            int32_t n_sets, const int64_t *set_offsets, const int32_t *set_points,
                                            const double *set_min_len, int32_t n_problems,
                                            const sap_batch_problem *problems, const double *P0, int32_t iters,
                                            int32_t cand_cap, double *P_out, double *min_trace, int64_t *ij_trace,
                                            int32_t *cert_trace, void *stream, sap_batch_stats *stats) {
    BatchPlan pl;
    sap_status st = plan_batch(X, dtype, N, n, ldx, n_sets, set_offsets, set_points, set_min_len, n_problems, problems,
                               P0, iters, cand_cap, P_out, min_trace, pl);
    if (st != SAP_OK) return st;
    if (pl.total > kStaticScratchBytes)
        return bfail(SAP_ERR_CAPACITY, "sap_batch_run_noalloc: the batch needs %zu bytes of scratch, above the fixed %zu",
                     pl.total, kStaticScratchBytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = nullptr;
    if ((st = static_scratch(&base)) != SAP_OK) return st;
    if ((st = check_P0(pl, n, P0, s)) != SAP_OK) return st;
    st = run_batch(pl, base, X, dtype, ldx, n, n_sets, n_problems, P0, iters, cand_cap, P_out, min_trace, ij_trace,
                   cert_trace, s, stats, false);
    (void)hipStreamSynchronize(s);
    return st;
}
