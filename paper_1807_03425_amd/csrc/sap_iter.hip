// Per-iteration kernels of the SAP library (gfx950).
//
// One iteration of the method (paper Sec. 4, Algorithm 1) is
//   evaluate  r_ij = ||P^T s_ij|| for every kept pair, min + argmin,
//   update    argmax basis vector, modified Gram-Schmidt, alpha shift.
// Here it runs as
//   [fused]  k_gemm_y        Y = (X - mu) P in FP64 on the matrix cores -> FP32
//            k_pair_fused    coarse r~^2 = ||y_i - y_j||^2 / d_ij^2 per 64x64 tile,
//                            per-tile minimum + global minimum
//   [plain]  k_pair_plain    coarse r~^2 = ||P^T s||^2 streaming the stored secants
//   [both]   k_rescore_*     FP64 evaluation, from X, of every pair whose coarse
//                            value falls in the proven window (and of the
//                            fused form's short pairs)
//            k_tail          FP64 min/argmin, record, and the update of P.
//
// The library is compiled with -ffp-contract=off: every FMA below is
// written explicitly, so a coarse value recomputed by the rescoring kernel
// is bit-identical to the one the pass reduced.
#include "sap_common.h"

namespace sap {

typedef double double4_t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ GEMM

// Y[r][c] = fl32( sum_l (x_rl - mu_l) P_lc ), rows >= N and columns >= k set
// to 0.  One wavefront per 16-row block; v_mfma_f64_16x16x4_f64 with
//   A (16 x 4):  lane = row + 16 * kk   (row = lane % 16, kk = lane / 16)
//   B (4 x 16):  lane = col + 16 * kk
//   D (16 x 16): lane holds rows lane/16 + 4 v, v = 0..3, column lane % 16
//                (measured on gfx950 with an in-bounds probe of the builtin).
__global__ __launch_bounds__(256) void k_gemm_y(const void *X, int dtype, int64_t ldx,
                                                int64_t N, int n, int k,
                                                const double *__restrict__ mu,
                                                const double *__restrict__ P64t,
                                                float *__restrict__ Y, int kp, int64_t Npad) {
    const int lane = threadIdx.x & 63;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (row0 >= Npad) return;
    const int m = lane & 15, kk = lane >> 4;
    const int64_t row = row0 + m;
    const bool rin = row < N;
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int l0 = 0; l0 < n; l0 += 4) {
        const int l = l0 + kk;
        double a = 0.0, b = 0.0;
        if (l < n) {
            if (rin) a = load_x(X, dtype, row * ldx + l) - mu[l];
            if (m < k) b = P64t[(int64_t)m * n + l];
        }
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    if (m < kp) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t r = row0 + kk + 4 * v;
            Y[r * kp + m] = (r < N && m < k) ? (float)acc[v] : 0.0f;
        }
    }
}

// ------------------------------------------------------------------ fused pass

// Coarse squared ratio of one pair: ||y_i - y_j||^2 * (1/d^2).  y_i is
// wavefront-uniform (scalar loads), y_j lives in the lane's registers.
template <int K>
__device__ __forceinline__ float pair_r2(const float *__restrict__ yi, const float (&yj)[K],
                                         float w) {
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const float d = yi[c] - yj[c];
        acc = __builtin_fmaf(d, d, acc);
    }
    return acc * w;
}

// One wavefront per tile (grid-stride).  Lane c owns column j = 64 bj + c and
// walks the 64 rows in 16 float4 groups.  Per pair: K subtractions, K FMAs,
// one multiply, one unsigned min.
template <int K>
__global__ __launch_bounds__(kPairBlock) void k_pair_fused(
    const float *__restrict__ Y, int kp, const float4 *__restrict__ invd2,
    const int2 *__restrict__ tiles, int64_t ntiles, uint32_t *__restrict__ tile_min,
    uint32_t *__restrict__ gmin) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (kPairBlock / kWave) +
                        __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (kPairBlock / kWave);
    uint32_t best = kKeyNone;
    for (int64_t t = wid; t < ntiles; t += nw) {
        const int2 b = tiles[t];
        float yj[K];
        const float *pj = Y + ((int64_t)b.y * kTile + lane) * kp;
#pragma unroll
        for (int c = 0; c < K; ++c) yj[c] = pj[c];
        const float *yi0 = Y + (int64_t)b.x * kTile * kp;
        const float4 *tp = invd2 + t * (kTileElems / 4) + lane;
        uint32_t m = kKeyNone;
#pragma unroll 2
        for (int g = 0; g < 16; ++g) {
            const float4 w = tp[g * 64];
            const float *yi = yi0 + (int64_t)(4 * g) * kp;
            m = min(m, __float_as_uint(pair_r2<K>(yi, yj, w.x)));
            m = min(m, __float_as_uint(pair_r2<K>(yi + kp, yj, w.y)));
            m = min(m, __float_as_uint(pair_r2<K>(yi + 2 * kp, yj, w.z)));
            m = min(m, __float_as_uint(pair_r2<K>(yi + 3 * kp, yj, w.w)));
        }
        m = wave_min_u32(m);
        if (lane == 0) tile_min[t] = m;
        best = min(best, m);
    }
    if (lane == 0 && best < 0x7f800000u) atomicMin(gmin, best);
}

// ------------------------------------------------------------------ plain pass

template <typename T> struct Vec4;
template <> struct Vec4<float> {
    static __device__ __forceinline__ void load(const float *p, float (&v)[4]) {
        const float4 t = *reinterpret_cast<const float4 *>(p);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    }
    static __device__ __forceinline__ float fma(float a, float b, float c) {
        return __builtin_fmaf(a, b, c);
    }
};
template <> struct Vec4<double> {
    static __device__ __forceinline__ void load(const double *p, double (&v)[4]) {
        const double2 a = reinterpret_cast<const double2 *>(p)[0];
        const double2 b = reinterpret_cast<const double2 *>(p)[1];
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
    static __device__ __forceinline__ double fma(double a, double b, double c) {
        return __builtin_fma(a, b, c);
    }
};

// Squared projected norms of the 4 consecutive pairs q0..q0+3:
// c = P^T s accumulated over the n components, then ||c||^2.
template <int K, typename T>
__device__ __forceinline__ void plain_r2(const T *__restrict__ S, int64_t pcols, int n,
                                         const T *__restrict__ Pr, int64_t q0, T (&r2)[4]) {
    T acc[4][K];
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int c = 0; c < K; ++c) acc[e][c] = (T)0;
    const T *sp = S + q0;
#pragma unroll 4
    for (int l = 0; l < n; ++l) {
        T s[4];
        Vec4<T>::load(sp + (int64_t)l * pcols, s);
        const T *pl = Pr + l * K;
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const T p = pl[c];
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e][c] = Vec4<T>::fma(s[e], p, acc[e][c]);
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        T a = (T)0;
#pragma unroll
        for (int c = 0; c < K; ++c) a = Vec4<T>::fma(acc[e][c], acc[e][c], a);
        r2[e] = a;
    }
}

template <typename T>
__device__ __forceinline__ uint32_t key_of(T r2) {
    // dropped pairs hold NaN secants; NaN compares false with itself
    return r2 == r2 ? __float_as_uint((float)r2) : kKeyNone;
}

template <int K, typename T>
__global__ __launch_bounds__(kPairBlock) void k_pair_plain(
    const T *__restrict__ S, int64_t pcols, int n, const T *__restrict__ Pr, int64_t nchunks,
    uint32_t *__restrict__ chunk_min, uint32_t *__restrict__ gmin) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (kPairBlock / kWave) +
                        __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (kPairBlock / kWave);
    uint32_t best = kKeyNone;
    for (int64_t ch = wid; ch < nchunks; ch += nw) {
        T r2[4];
        plain_r2<K, T>(S, pcols, n, Pr, ch * kChunk + lane * 4, r2);
        uint32_t m = kKeyNone;
#pragma unroll
        for (int e = 0; e < 4; ++e) m = min(m, key_of<T>(r2[e]));
        m = wave_min_u32(m);
        if (lane == 0) chunk_min[ch] = m;
        best = min(best, m);
    }
    if (lane == 0 && best < 0x7f800000u) atomicMin(gmin, best);
}

// ------------------------------------------------------------------ FP64 rescoring

// Exact-as-FP64 r of pair (i, j) from X: ||P^T (x_i - x_j)|| / ||x_i - x_j||.
// Wavefront-cooperative (lanes split the n components); every lane returns
// the same value.
template <int K, typename TX>
__device__ double exact_r_wave(const TX *__restrict__ X, int64_t ldx, int n,
                               const double *__restrict__ P64t, int64_t i, int64_t j) {
    const int lane = threadIdx.x & 63;
    double d2 = 0.0, c[K];
#pragma unroll
    for (int q = 0; q < K; ++q) c[q] = 0.0;
    for (int l = lane; l < n; l += kWave) {
        const double dl = (double)X[i * ldx + l] - (double)X[j * ldx + l];
        d2 = __builtin_fma(dl, dl, d2);
#pragma unroll
        for (int q = 0; q < K; ++q) c[q] = __builtin_fma(P64t[(int64_t)q * n + l], dl, c[q]);
    }
    d2 = wave_sum(d2);
    double r2 = 0.0;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double cq = wave_sum(c[q]);
        r2 = __builtin_fma(cq, cq, r2);
    }
    return sqrt(r2) / sqrt(d2);
}

// Same quantity, one lane per pair (sequential over the components).
template <int K, typename TX>
__device__ double exact_r_lane(const TX *__restrict__ X, int64_t ldx, int n,
                               const double *__restrict__ P64t, int64_t i, int64_t j) {
    double d2 = 0.0, c[K];
#pragma unroll
    for (int q = 0; q < K; ++q) c[q] = 0.0;
    for (int l = 0; l < n; ++l) {
        const double dl = (double)X[i * ldx + l] - (double)X[j * ldx + l];
        d2 = __builtin_fma(dl, dl, d2);
#pragma unroll
        for (int q = 0; q < K; ++q) c[q] = __builtin_fma(P64t[(int64_t)q * n + l], dl, c[q]);
    }
    double r2 = 0.0;
#pragma unroll
    for (int q = 0; q < K; ++q) r2 = __builtin_fma(c[q], c[q], r2);
    return sqrt(r2) / sqrt(d2);
}

// Squared-ratio threshold of the rescoring window.  With coarse values
// obeying |r~ - r| <= e_abs + e_rel r, any pair whose true r does not exceed
// the true r of the coarse argmin has r~ <= T; T^2 is rounded up to FP32.
__device__ __forceinline__ uint32_t window_key(uint32_t gmin, double e_abs, double e_rel,
                                               double *coarse, double *tr) {
    if (gmin >= 0x7f800000u) { *coarse = -1.0; *tr = 0.0; return 0u; }
    const double rc = sqrt((double)__uint_as_float(gmin));
    const double T = (rc * (1.0 + e_rel) + 2.0 * e_abs) / (1.0 - e_rel);
    const double T2 = T * T;
    float f = (float)T2;
    if ((double)f < T2) f = __uint_as_float(__float_as_uint(f) + 1u);  // next float up (f >= 0)
    *coarse = rc;
    *tr = T;
    return __float_as_uint(f);
}

// The proven bound |r~ - r| <= e_abs + e_rel r, checked on every rescored
// window pair: a violation means the coarse pass is not what the bound
// describes, and the result is then reported uncertified.
__device__ __forceinline__ int bound_broken(double r, double r2c, double e_abs, double e_rel) {
    const double rc = sqrt(r2c);
    return fabs(r - rc) > (e_abs + e_rel * fmax(r, rc)) * 1.0001 ? 1 : 0;
}

// Reduce (r, i, j) and the counters over the block; thread 0 writes the partial.
__device__ __forceinline__ void block_finish(double r, int32_t i, int32_t j, int32_t nres,
                                             int32_t ntl, int32_t nviol, Partial *out) {
    __shared__ Partial sb[kPairBlock / kWave];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    wave_min_lex(r, i, j);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        nres += __shfl_xor(nres, o, kWave);
        ntl += __shfl_xor(ntl, o, kWave);
        nviol += __shfl_xor(nviol, o, kWave);
    }
    if (lane == 0) sb[wv] = Partial{r, i, j, nres, ntl, nviol, 0};
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial b = sb[0];
        for (int w = 1; w < kPairBlock / kWave; ++w) {
            if (lex_less(sb[w].r, sb[w].i, sb[w].j, b.r, b.i, b.j)) {
                b.r = sb[w].r; b.i = sb[w].i; b.j = sb[w].j;
            }
            b.n_rescored += sb[w].n_rescored;
            b.n_tiles += sb[w].n_tiles;
            b.n_viol += sb[w].n_viol;
        }
        *out = b;
    }
}

// Fused form: (a) the short-pair list, one lane per pair; (b) every tile whose
// minimum is inside the window, revisited by one wavefront, each in-window
// pair rescored cooperatively.
template <int K, typename TX>
__global__ __launch_bounds__(kPairBlock) void k_rescore_fused(
    const float *__restrict__ Y, int kp, const float4 *__restrict__ invd2,
    const int2 *__restrict__ tiles, int64_t ntiles, const uint32_t *__restrict__ tile_min,
    const uint32_t *__restrict__ gmin, double e_abs, double e_rel, const TX *__restrict__ X,
    int64_t ldx, int n, const double *__restrict__ P64t, const int2 *__restrict__ close,
    int64_t nclose, Partial *__restrict__ partials) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (kPairBlock / kWave) +
                        __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (kPairBlock / kWave);
    double coarse, tr;
    const uint32_t T2 = window_key(*gmin, e_abs, e_rel, &coarse, &tr);
    double best = __builtin_huge_val();
    int32_t bi = 0x7fffffff, bj = 0x7fffffff, nres = 0, ntl = 0;

    for (int64_t e = (int64_t)blockIdx.x * kPairBlock + threadIdx.x; e < nclose;
         e += (int64_t)gridDim.x * kPairBlock) {
        const int2 pr = close[e];
        const double r = exact_r_lane<K, TX>(X, ldx, n, P64t, pr.x, pr.y);
        ++nres;
        if (lex_less(r, pr.x, pr.y, best, bi, bj)) { best = r; bi = pr.x; bj = pr.y; }
    }

    int32_t nwin = 0, nviol = 0;
    if (coarse >= 0.0) {
        for (int64_t t0 = wid * 64; t0 < ntiles; t0 += nw * 64) {
            const int64_t tl = t0 + lane;
            const uint32_t tm = tl < ntiles ? tile_min[tl] : kKeyNone;
            uint64_t hits = __ballot(tm <= T2);
            while (hits) {
                const int bit = __builtin_ctzll(hits);
                hits &= hits - 1;
                const int64_t t = t0 + bit;
                ++ntl;
                const int2 b = tiles[t];
                float yj[K];
                const float *pj = Y + ((int64_t)b.y * kTile + lane) * kp;
#pragma unroll
                for (int c = 0; c < K; ++c) yj[c] = pj[c];
                const float *yi0 = Y + (int64_t)b.x * kTile * kp;
                const float4 *tp = invd2 + t * (kTileElems / 4) + lane;
                for (int g = 0; g < 16; ++g) {
                    const float4 w4 = tp[g * 64];
                    const float wv[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const float r2 = pair_r2<K>(yi0 + (int64_t)(4 * g + rr) * kp, yj, wv[rr]);
                        uint64_t cm = __ballot(__float_as_uint(r2) <= T2);
                        while (cm) {
                            const int ln = __builtin_ctzll(cm);
                            cm &= cm - 1;
                            const int32_t i = b.x * kTile + 4 * g + rr;
                            const int32_t j = b.y * kTile + ln;
                            const double r = exact_r_wave<K, TX>(X, ldx, n, P64t, i, j);
                            const float r2c = __shfl(r2, ln, kWave);
                            ++nwin;
                            nviol += bound_broken(r, (double)r2c, e_abs, e_rel);
                            if (lex_less(r, i, j, best, bi, bj)) { best = r; bi = i; bj = j; }
                        }
                    }
                }
            }
        }
    }
    if (lane != 0) { nwin = 0; ntl = 0; nviol = 0; }
    block_finish(best, bi, bj, nres + nwin, ntl, nviol, partials + blockIdx.x);
}

__device__ __forceinline__ void decode_q(int64_t q, int64_t N, int64_t &i, int64_t &j) {
    const double b = 2.0 * (double)N - 1.0;
    const double disc = b * b - 8.0 * (double)q;
    int64_t ii = (int64_t)floor((b - sqrt(disc > 0.0 ? disc : 0.0)) * 0.5);
    if (ii < 0) ii = 0;
    if (ii > N - 2) ii = N - 2;
    while (ii > 0 && pair_index(N, ii, ii + 1) > q) --ii;
    while (ii < N - 2 && pair_index(N, ii + 1, ii + 2) <= q) ++ii;
    i = ii;
    j = q - pair_index(N, ii, ii + 1) + ii + 1;
}

// Plain form: every chunk whose minimum is inside the window is recomputed
// by one wavefront and its in-window pairs rescored cooperatively.
template <int K, typename T>
__global__ __launch_bounds__(kPairBlock) void k_rescore_plain(
    const T *__restrict__ S, int64_t pcols, int n, const T *__restrict__ Pr, int64_t nchunks,
    const uint32_t *__restrict__ chunk_min, const uint32_t *__restrict__ gmin, double e_abs,
    double e_rel, const T *__restrict__ X, int64_t ldx, int64_t N,
    const double *__restrict__ P64t, Partial *__restrict__ partials) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * (kPairBlock / kWave) +
                        __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (kPairBlock / kWave);
    double coarse, tr;
    const uint32_t T2 = window_key(*gmin, e_abs, e_rel, &coarse, &tr);
    double best = __builtin_huge_val();
    int32_t bi = 0x7fffffff, bj = 0x7fffffff, nwin = 0, ntl = 0, nviol = 0;
    if (coarse >= 0.0) {
        for (int64_t c0 = wid * 64; c0 < nchunks; c0 += nw * 64) {
            const int64_t cl = c0 + lane;
            const uint32_t cmin = cl < nchunks ? chunk_min[cl] : kKeyNone;
            uint64_t hits = __ballot(cmin <= T2);
            while (hits) {
                const int bit = __builtin_ctzll(hits);
                hits &= hits - 1;
                const int64_t ch = c0 + bit;
                ++ntl;
                T r2[4];
                plain_r2<K, T>(S, pcols, n, Pr, ch * kChunk + lane * 4, r2);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    uint64_t cm = __ballot(key_of<T>(r2[e]) <= T2);
                    while (cm) {
                        const int ln = __builtin_ctzll(cm);
                        cm &= cm - 1;
                        int64_t i, j;
                        decode_q(ch * kChunk + ln * 4 + e, N, i, j);
                        const double r = exact_r_wave<K, T>(X, ldx, n, P64t, i, j);
                        const T r2c = __shfl(r2[e], ln, kWave);
                        ++nwin;
                        nviol += bound_broken(r, (double)r2c, e_abs, e_rel);
                        if (lex_less(r, (int32_t)i, (int32_t)j, best, bi, bj)) {
                            best = r; bi = (int32_t)i; bj = (int32_t)j;
                        }
                    }
                }
            }
        }
    }
    if (lane != 0) { nwin = 0; ntl = 0; nviol = 0; }
    block_finish(best, bi, bj, nwin, ntl, nviol, partials + blockIdx.x);
}

// ------------------------------------------------------------------ tail: record + update

// Single wavefront.  Reduces the rescoring partials to the FP64 (min, i, j),
// records it, resets the coarse minimum for the next pass, and (do_step)
// applies the paper's update to P in FP64:
//   c = P^T s;  t = first argmax |c_t|;
//   if c = 0:   P' = [s, p_2, .., p_k]
//   else:       v = P c; modified Gram-Schmidt on (v, p_1..p_k without p_t);
//               u = unit((1-a) v + a (s - v))   [rule 1: unit vectors of v, s-v]
//               P' = [u, q_2, .., q_k]
// Vectors live in LDS: A (k x n), s (n), v (n), c (16).  Lane l owns components
// l, l+64, ...; every inner product is a wavefront butterfly sum.
template <typename TX>
__global__ __launch_bounds__(64) void k_tail(
    const Partial *__restrict__ partials, int nparts, uint32_t *__restrict__ gmin,
    double e_abs, double e_rel, const TX *__restrict__ X, int64_t ldx, int64_t N, int n, int k,
    double *__restrict__ P64t, void *__restrict__ Pr, int pr_kind, double alpha, int rule,
    int do_step, DevResult *__restrict__ res, double *__restrict__ tr_min,
    int64_t *__restrict__ tr_ij, int32_t *__restrict__ tr_cert, int it) {
    extern __shared__ double sm[];
    const int lane = threadIdx.x;

    double r = __builtin_huge_val();
    int32_t bi = 0x7fffffff, bj = 0x7fffffff, nres = 0, ntl = 0, nviol = 0;
    for (int p = lane; p < nparts; p += kWave) {
        const Partial pp = partials[p];
        if (lex_less(pp.r, pp.i, pp.j, r, bi, bj)) { r = pp.r; bi = pp.i; bj = pp.j; }
        nres += pp.n_rescored;
        ntl += pp.n_tiles;
        nviol += pp.n_viol;
    }
    wave_min_lex(r, bi, bj);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        nres += __shfl_xor(nres, o, kWave);
        ntl += __shfl_xor(ntl, o, kWave);
        nviol += __shfl_xor(nviol, o, kWave);
    }
    double coarse, tr;
    const uint32_t g = *gmin;
    (void)window_key(g, e_abs, e_rel, &coarse, &tr);
    const bool found = r < __builtin_huge_val();
    if (lane == 0) {
        res->min_norm = r;
        res->i = found ? bi : -1;
        res->j = found ? bj : -1;
        res->q = found ? pair_index(N, bi, bj) : -1;
        res->coarse_min = coarse;
        res->window = coarse >= 0.0 ? tr - coarse : 0.0;
        res->certified = (found && nviol == 0) ? 1 : 0;
        res->n_rescored = nres;
        res->n_tiles = ntl;
        res->t = -1;
        if (tr_min) tr_min[it] = r;
        if (tr_ij) { tr_ij[2 * it] = found ? bi : -1; tr_ij[2 * it + 1] = found ? bj : -1; }
        if (tr_cert) tr_cert[it] = (found && nviol == 0) ? 1 : 0;
        // the coarse minimum has been consumed (g was read above); arm it
        // for the next pass
        *gmin = kKeyNone;
    }
    if (!do_step || !found) return;

    double *A = sm;                       // k x n: MGS vectors
    double *s = sm + (size_t)k * n;       // unit secant
    double *v = s + n;                    // P P^T s
    double *c = v + n;                    // P^T s (uniform)
    const int64_t i = bi, j = bj;
    double d2 = 0.0;
    for (int l = lane; l < n; l += kWave) {
        const double dl = (double)X[i * ldx + l] - (double)X[j * ldx + l];
        s[l] = dl;
        d2 = __builtin_fma(dl, dl, d2);
    }
    const double d = sqrt(wave_sum(d2));
    for (int l = lane; l < n; l += kWave) s[l] = s[l] / d;

    // c = P^T s, t = first argmax |c|
    int t = 0;
    double cmax = -1.0;
    for (int q = 0; q < k; ++q) {
        double acc = 0.0;
        for (int l = lane; l < n; l += kWave) acc = __builtin_fma(P64t[(int64_t)q * n + l], s[l], acc);
        acc = wave_sum(acc);
        if (lane == 0) c[q] = acc;
        if (fabs(acc) > cmax) { cmax = fabs(acc); t = q; }
    }
    __syncthreads();
    if (lane == 0) res->t = t;

    if (cmax == 0.0) {
        for (int l = lane; l < n; l += kWave) P64t[l] = s[l];
    } else {
        for (int l = lane; l < n; l += kWave) {
            double acc = 0.0;
            for (int q = 0; q < k; ++q) acc = __builtin_fma(P64t[(int64_t)q * n + l], c[q], acc);
            v[l] = acc;
            A[l] = acc;
            for (int m = 1; m < k; ++m) {
                const int q = (m - 1 < t) ? m - 1 : m;
                A[(size_t)m * n + l] = P64t[(int64_t)q * n + l];
            }
        }
        // modified Gram-Schmidt, right-looking: once q_m is final, every later
        // vector loses its component along q_m (the same sequence of
        // subtractions, per vector, as the textbook column-by-column form)
        double vnorm = 0.0;
        for (int m = 0; m < k; ++m) {
            double *am = A + (size_t)m * n;
            double acc = 0.0;
            for (int l = lane; l < n; l += kWave) acc = __builtin_fma(am[l], am[l], acc);
            const double nrm = sqrt(wave_sum(acc));
            if (m == 0) vnorm = nrm;
            for (int l = lane; l < n; l += kWave) am[l] = am[l] / nrm;
            for (int jv = m + 1; jv < k; ++jv) {
                double *aj = A + (size_t)jv * n;
                double dot = 0.0;
                for (int l = lane; l < n; l += kWave) dot = __builtin_fma(am[l], aj[l], dot);
                dot = wave_sum(dot);
                for (int l = lane; l < n; l += kWave) aj[l] = aj[l] - dot * am[l];
            }
        }
        // the alpha shift toward the worst secant
        double wn = 1.0;
        if (rule == SAP_STEP_NORMALIZED) {
            double acc = 0.0;
            for (int l = lane; l < n; l += kWave) {
                const double w = s[l] - v[l];
                acc = __builtin_fma(w, w, acc);
            }
            wn = sqrt(wave_sum(acc));
        }
        double un = 0.0;
        for (int l = lane; l < n; l += kWave) {
            double u;
            if (rule == SAP_STEP_NORMALIZED)
                u = (1.0 - alpha) * (v[l] / vnorm) + (wn > 0.0 ? alpha * ((s[l] - v[l]) / wn) : 0.0);
            else
                u = (1.0 - alpha) * v[l] + alpha * (s[l] - v[l]);
            s[l] = u;  // s is no longer needed: reuse it for u
            un = __builtin_fma(u, u, un);
        }
        un = sqrt(wave_sum(un));
        for (int l = lane; l < n; l += kWave) {
            P64t[l] = s[l] / un;
            for (int m = 1; m < k; ++m) P64t[(int64_t)m * n + l] = A[(size_t)m * n + l];
        }
    }
    // the pass's own copy of P (plain form), row-major n x k
    if (pr_kind == 1) {
        float *pf = static_cast<float *>(Pr);
        for (int l = lane; l < n; l += kWave)
            for (int q = 0; q < k; ++q) pf[(int64_t)l * k + q] = (float)P64t[(int64_t)q * n + l];
    } else if (pr_kind == 2) {
        double *pd = static_cast<double *>(Pr);
        for (int l = lane; l < n; l += kWave)
            for (int q = 0; q < k; ++q) pd[(int64_t)l * k + q] = P64t[(int64_t)q * n + l];
    }
}

// ------------------------------------------------------------------ small helpers

// Write the plain pass's P copy (n x k row-major, T) from the FP64 master.
template <typename T>
__global__ void k_write_pass_P(const double *__restrict__ P64t, int n, int k, T *__restrict__ Pr) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int l = e / k, q = e % k;
    Pr[e] = (T)P64t[(int64_t)q * n + l];
}

// P_out (n x k row-major) <- master (k x n)
__global__ void k_P_out(const double *__restrict__ P64t, int n, int k, double *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int l = e / k, q = e % k;
    out[e] = P64t[(int64_t)q * n + l];
}

__global__ void k_arm_gmin(uint32_t *gmin) { *gmin = kKeyNone; }

}  // namespace sap
