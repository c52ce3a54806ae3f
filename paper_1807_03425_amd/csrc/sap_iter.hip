// Per-iteration kernels of the SAP library (gfx950).
//
// One iteration of the method (paper Sec. 4, Algorithm 1) is
//   evaluate  r_ij = ||P^T s_ij|| for every kept pair, min + argmin,
//   update    argmax basis vector, modified Gram-Schmidt, alpha shift.
// Here it runs as three launches (two for the plain form):
//   k_prep    (fused form) Y = (X - mu) P in FP64 on the matrix cores, rounded
//             to FP32;
//   k_pass    the coarse FP32 score of every pair, reduced to per-unit and
//             per-block minima (fused: ||y_i - y_j||^2 / d^2 per 16 x 64
//             sub-tile; plain: ||P^T s||^2 per 256-pair chunk, with the
//             chunk's argmin and second-smallest score); in the fused form
//             the same grid scores the short pairs (too short for the coarse
//             error bound) in FP64 on the matrix cores;
//   k_select  one block: global coarse minimum, the proven rescoring window,
//             FP64 rescoring of every in-window pair, the FP64 (min, i, j)
//             record, then the FP64 update of P by one wavefront.
// No two blocks ever contend on one address: each writes its own result
// slot, and the kernel boundary is the grid-wide barrier.  (Device-scope
// atomics on one address serialize across the eight XCDs of the part at tens
// of nanoseconds each, which costs more than a launch once there are more than
// a few hundred blocks.)
//
// The library is compiled with -ffp-contract=off: every FMA below is
// written explicitly, so a coarse value recomputed by the epilogue is
// bit-identical to the one the pass reduced.
#include "sap_common.h"

namespace sap {

typedef double double4_t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ wavefront sums

// DPP lane permutation of a double (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// v + (v of lane ^ 16) and v + (v of lane ^ 32), from gfx950's
// v_permlane16_swap / v_permlane32_swap: with both operands equal, the two
// results of the swap are {v_i, v_(i^16)} (resp. ^32) in some order, so their
// sum is the pair sum (lane semantics measured with an in-bounds probe).
__device__ __forceinline__ double pair_sum16(double v) {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double pair_sum32(double v) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// Sum over the 64 lanes, identical bits in every lane: each step adds two
// partial sums that every participating lane sees in swapped order, and
// floating-point addition is commutative.  Steps inside a 16-lane row use
// DPP (quad xor 1, quad xor 2, half-row mirror, row mirror); the two
// cross-row steps use the permlane swaps.  All VALU, no LDS traffic.
__device__ __forceinline__ double wave_sum_fast(double v) {
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);  // row_half_mirror
    v += dpp_f64<0x140>(v);  // row_mirror
    v = pair_sum16(v);
    return pair_sum32(v);
}

// v[from..NV-1] summed over the wavefront, the reductions interleaved.
template <int NV>
__device__ __forceinline__ void wave_sum_many(double (&v)[NV], int from = 0) {
#pragma unroll
    for (int a = 0; a < NV; ++a) if (a >= from) v[a] += dpp_f64<0xB1>(v[a]);
#pragma unroll
    for (int a = 0; a < NV; ++a) if (a >= from) v[a] += dpp_f64<0x4E>(v[a]);
#pragma unroll
    for (int a = 0; a < NV; ++a) if (a >= from) v[a] += dpp_f64<0x141>(v[a]);
#pragma unroll
    for (int a = 0; a < NV; ++a) if (a >= from) v[a] += dpp_f64<0x140>(v[a]);
#pragma unroll
    for (int a = 0; a < NV; ++a) if (a >= from) v[a] += __shfl_xor(v[a], 16, kWave);
#pragma unroll
    for (int a = 0; a < NV; ++a) if (a >= from) v[a] += __shfl_xor(v[a], 32, kWave);
}

// ------------------------------------------------------------------ GEMM

// 16 consecutive elements p[0..15] as FP64 (exact for FP32): 16-byte vector
// loads when vec (the caller guarantees p is 16-byte aligned), else scalar.
__device__ __forceinline__ void load16(const float *__restrict__ p, bool vec, double (&o)[16]) {
    if (vec) {
        const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float4 t = q[u];
            o[4 * u] = t.x; o[4 * u + 1] = t.y; o[4 * u + 2] = t.z; o[4 * u + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int u = 0; u < 16; ++u) o[u] = p[u];
    }
}
__device__ __forceinline__ void load16(const double *__restrict__ p, bool vec, double (&o)[16]) {
    if (vec) {
        const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double2 t = q[u];
            o[2 * u] = t.x; o[2 * u + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int u = 0; u < 16; ++u) o[u] = p[u];
    }
}

// Y[r][c] = fl32( sum_l (x_rl - mu_l) P_lc ), rows >= N and columns >= k set
// to 0.  One wavefront per 16-row block; v_mfma_f64_16x16x4_f64 with
//   A (16 x 4):  lane = row + 16 * kk   (row = lane % 16, kk = lane / 16)
//   B (4 x 16):  lane = col + 16 * kk
//   D (16 x 16): lane holds rows lane/16 + 4 v, v = 0..3, column lane % 16
//                (measured on gfx950 with an in-bounds probe of the builtin).
// In a 64-component chunk, k-slot kk of MFMA s carries component
// l0 + 16 kk + s, so each lane reads 16 consecutive components of its row
// (and of P's column): 16-byte loads when vx (X rows 16-byte aligned) and vp
// (n even).  Every operand load of a chunk is issued before its 16 MFMAs.
template <typename TX>
__device__ void gemm_block(const TX *__restrict__ X, int64_t ldx, int64_t N, int n, int k,
                           const double *__restrict__ mu, const double *__restrict__ P64t,
                           float *__restrict__ Y, int kp, int64_t Npad, bool vx, bool vp) {
    const int lane = threadIdx.x & 63;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (row0 >= Npad) return;
    const int m = lane & 15, kk = lane >> 4;
    const int64_t row = row0 + m;
    const bool rin = row < N;
    // out-of-range rows and columns read a valid element and are zeroed by a
    // mask afterwards, so that every load of a chunk is unconditional and the
    // 48 of them are in flight together (X is finite: checked at init)
    const double rmask = rin ? 1.0 : 0.0, pmask = m < k ? 1.0 : 0.0;
    const TX *xr = X + (rin ? row : N - 1) * ldx;
    const double *pc = P64t + (int64_t)(m < k ? m : k - 1) * n;
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
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64((xa[s] - ma[s]) * rmask, pb[s] * pmask,
                                                       acc, 0, 0, 0);
    }
    for (; l0 < n; l0 += 4) {
        const int l = l0 + kk;
        double a = 0.0, b = 0.0;
        if (l < n) {
            if (rin) a = (double)xr[l] - mu[l];
            if (m < k) b = pc[l];
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

// ------------------------------------------------------------------ coarse scores

// Coarse squared ratio of one pair: ||y_i - y_j||^2 * (1/d^2).  y_i is
// wavefront-uniform, y_j lives in the lane's registers.
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

// The lane's own row of Y (kp is a multiple of 4: float4 loads).
template <int K>
__device__ __forceinline__ void load_yj(const float *__restrict__ Y, int kp, int64_t row,
                                        float (&yj)[K]) {
    const float4 *p = reinterpret_cast<const float4 *>(Y + row * kp);
#pragma unroll
    for (int c4 = 0; c4 < (K + 3) / 4; ++c4) {
        const float4 v = p[c4];
        if (4 * c4 + 0 < K) yj[4 * c4 + 0] = v.x;
        if (4 * c4 + 1 < K) yj[4 * c4 + 1] = v.y;
        if (4 * c4 + 2 < K) yj[4 * c4 + 2] = v.z;
        if (4 * c4 + 3 < K) yj[4 * c4 + 3] = v.w;
    }
}

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

// Plain form: squared projected norms of the 4 consecutive stored secants
// q0..q0+3 (c = P^T s over the n components, then ||c||^2).
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

// ------------------------------------------------------------------ FP64 scores

// FP64 r of pair (i, j) from X: ||P^T (x_i - x_j)|| / ||x_i - x_j||, with
// P (K x n, FP64) in LDS.  Wavefront-cooperative (lanes split the n
// components); every lane returns the same value.
template <int K, typename TX>
__device__ double exact_r_wave(const TX *__restrict__ X, int64_t ldx, int n,
                               const double *P64t, int64_t i, int64_t j) {
    const int lane = threadIdx.x & 63;
    double v[K + 1];
#pragma unroll
    for (int q = 0; q <= K; ++q) v[q] = 0.0;
    for (int l = lane; l < n; l += kWave) {
        const double dl = (double)X[i * ldx + l] - (double)X[j * ldx + l];
        v[K] = __builtin_fma(dl, dl, v[K]);
#pragma unroll
        for (int q = 0; q < K; ++q) v[q] = __builtin_fma(P64t[(int64_t)q * n + l], dl, v[q]);
    }
    wave_sum_many<K + 1>(v);
    double r2 = 0.0;
#pragma unroll
    for (int q = 0; q < K; ++q) r2 = __builtin_fma(v[q], v[q], r2);
    return sqrt(r2) / sqrt(v[K]);
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

template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

__device__ __forceinline__ void lex_pick(double &r, int32_t &i, int32_t &j, double r2, int32_t i2,
                                         int32_t j2) {
    if (lex_less(r2, i2, j2, r, i, j)) { r = r2; i = i2; j = j2; }
}

template <int CTRL>
__device__ __forceinline__ void lex_step_dpp(double &r, int32_t &i, int32_t &j) {
    lex_pick(r, i, j, dpp_f64<CTRL>(r), dpp_i32<CTRL>(i), dpp_i32<CTRL>(j));
}

// Lexicographic (r, i, j) minimum over the wavefront, in every lane: the same
// six exchange steps as wave_sum_fast (four DPP steps inside 16-lane rows,
// then the permlane16 / permlane32 swaps, whose two results are the lane's
// own tuple and its partner's, in either order: the minimum of the two does
// not depend on that order).  No LDS traffic.
__device__ __forceinline__ void wave_min_lex_fast(double &r, int32_t &i, int32_t &j) {
    lex_step_dpp<0xB1>(r, i, j);
    lex_step_dpp<0x4E>(r, i, j);
    lex_step_dpp<0x141>(r, i, j);
    lex_step_dpp<0x140>(r, i, j);
    {
        const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(r), __double2loint(r), false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(r), __double2hiint(r), false, false);
        const auto ii = __builtin_amdgcn_permlane16_swap(i, i, false, false);
        const auto jj = __builtin_amdgcn_permlane16_swap(j, j, false, false);
        r = __hiloint2double(hi[0], lo[0]); i = ii[0]; j = jj[0];
        lex_pick(r, i, j, __hiloint2double(hi[1], lo[1]), ii[1], jj[1]);
    }
    {
        const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(r), __double2loint(r), false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(r), __double2hiint(r), false, false);
        const auto ii = __builtin_amdgcn_permlane32_swap(i, i, false, false);
        const auto jj = __builtin_amdgcn_permlane32_swap(j, j, false, false);
        r = __hiloint2double(hi[0], lo[0]); i = ii[0]; j = jj[0];
        lex_pick(r, i, j, __hiloint2double(hi[1], lo[1]), ii[1], jj[1]);
    }
}

// Integer sum over the wavefront, in every lane (same exchange pattern).
__device__ __forceinline__ int32_t wave_sum_i32_fast(int32_t v) {
    v += dpp_i32<0xB1>(v);
    v += dpp_i32<0x4E>(v);
    v += dpp_i32<0x141>(v);
    v += dpp_i32<0x140>(v);
    const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = a[0] + a[1];
    const auto b = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return b[0] + b[1];
}

// Block-wide reduction of a per-thread (r, i, j) and counters into *out
// (written by thread 0).  All 256 threads must call it.
__device__ void block_reduce_partial(double r, int32_t i, int32_t j, int32_t nres, int32_t ntl,
                                     int32_t nviol, Partial *out) {
    __shared__ Partial sb[kPairBlock / kWave];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    wave_min_lex_fast(r, i, j);
    nres = wave_sum_i32_fast(nres);
    ntl = wave_sum_i32_fast(ntl);
    nviol = wave_sum_i32_fast(nviol);
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
    __syncthreads();
}

// Unsigned minimum over the wavefront, in every lane (same exchange pattern
// as wave_sum_fast; the minimum of a swap's two results is order-free).
__device__ __forceinline__ uint32_t wave_min_u32_fast(uint32_t v) {
    v = min(v, (uint32_t)dpp_i32<0xB1>((int)v));
    v = min(v, (uint32_t)dpp_i32<0x4E>((int)v));
    v = min(v, (uint32_t)dpp_i32<0x141>((int)v));
    v = min(v, (uint32_t)dpp_i32<0x140>((int)v));
    const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = min((uint32_t)a[0], (uint32_t)a[1]);
    const auto b = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return min((uint32_t)b[0], (uint32_t)b[1]);
}

__device__ __forceinline__ uint32_t block_min_u32(uint32_t v) {
    __shared__ uint32_t sm[kPairBlock / kWave];
    v = wave_min_u32_fast(v);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t b = sm[0];
#pragma unroll
    for (int w = 1; w < kPairBlock / kWave; ++w) b = min(b, sm[w]);
    __syncthreads();
    return b;
}

// Load of a value another block of the same grid wrote (after the acquire
// in finished_last): a device-scope relaxed atomic load, never a scalar load.
__device__ __forceinline__ uint32_t ld_u32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ sweep

template <typename TX>
struct SweepArgs {
    // fused pass
    const float *Y;
    int kp;
    const float4 *invd2;
    const int2 *tiles;
    int64_t nhalf;       // 2 x tiles
    int64_t nb;          // tile rows (the tiles cover the upper triangle of nb x nb)
    // plain pass
    const TX *S;
    int64_t pcols;
    const TX *Pr;
    int64_t nchunks;
    // both passes
    int n;
    int npass;           // pass blocks; blocks >= npass are short-pair blocks
    uint32_t *unit_min;  // per sub-tile (fused) or chunk (plain)
    uint32_t *unit_min2; // plain: second-smallest key of the chunk
    uint32_t *unit_arg;  // plain: position (0..255) of the chunk's smallest key
    uint32_t *blk_min;   // per pass block
    // short pairs (fused)
    const int2 *close;    // short pairs (i, j), sorted
    const double *cd;     // their lengths ||x_i - x_j||
    int64_t nclose;
    Partial *spart;       // per short-pair block
    // selection
    double e_abs, e_rel;
    const TX *X;
    int64_t ldx, N;
    int vx, vp;           // 16-byte loads: X rows aligned; n even (rows of P64t)
    const double *P64t;
    uint32_t *gmin_out;
    DevResult *res;
    double *tr_min;
    int64_t *tr_ij;
    int32_t *tr_cert;
    int it;
};

// Fused pass block pb.  Wavefront w = 4 pb + slot takes half-tiles
// h = w, w + nw, ... (h = 2 t + half: rows 64 bi + 32 half .. +31 against the
// 64 columns of tile t = (bi, bj)).  Before scoring a half-tile it issues
// every load of the next one (8 weight float4 per lane, the lane's y_j, its
// share of the 32 y_i rows), so memory latency overlaps the arithmetic; the
// y_i rows go through the wavefront's own LDS slice (read back as
// broadcasts; no other wavefront touches it, so no block barrier).
// Per pair: K subtractions, K FMAs, one multiply, one unsigned min.
template <int K, typename TX>
__device__ uint32_t fused_pass_block(const SweepArgs<TX> &a, int pb) {
    __shared__ float4 s_y[kPairBlock / kWave][32 * kMaxK / 4];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)a.npass * (kPairBlock / kWave);
    const int kp = a.kp;
    float4 *yl = s_y[wv];
    const int nf4 = 8 * kp;                  // float4 count of 32 rows of Y (<= 128)
    uint32_t best = kKeyNone;
    int64_t h = (int64_t)pb * (kPairBlock / kWave) + wv;
    // loads of half-tile h: weights, y_j, and two float4 of the y_i rows per lane
    float4 w[8], yr0, yr1;
    float yj[K];
    auto fetch = [&](int64_t hh) {
        const int64_t t = hh >> 1;
        const int half = (int)(hh & 1);
        const float4 *tp = a.invd2 + t * (kTileElems / 4) + half * 512 + lane;
#pragma unroll
        for (int g = 0; g < 8; ++g) w[g] = tp[g * 64];
        const int2 b = a.tiles[t];
        const float4 *ysrc =
            reinterpret_cast<const float4 *>(a.Y + ((int64_t)b.x * kTile + 32 * half) * kp);
        yr0 = ysrc[lane < nf4 ? lane : 0];
        yr1 = ysrc[lane + 64 < nf4 ? lane + 64 : 0];
        load_yj<K>(a.Y, kp, (int64_t)b.y * kTile + lane, yj);
    };
    if (h < a.nhalf) fetch(h);
    for (; h < a.nhalf; h += nw) {
        float4 wc[8];
#pragma unroll
        for (int g = 0; g < 8; ++g) wc[g] = w[g];
        float yc[K];
#pragma unroll
        for (int c = 0; c < K; ++c) yc[c] = yj[c];
        __builtin_amdgcn_wave_barrier();
        if (lane < nf4) yl[lane] = yr0;
        if (lane + 64 < nf4) yl[lane + 64] = yr1;
        __builtin_amdgcn_wave_barrier();
        if (h + nw < a.nhalf) fetch(h + nw);     // next half-tile's loads in flight
        const float *yi0 = reinterpret_cast<const float *>(yl);
        uint32_t m0 = kKeyNone, m1 = kKeyNone;
#pragma unroll
        for (int g = 0; g < 8; ++g) {
            const float *yi = yi0 + 4 * g * kp;
            uint32_t m = min(__float_as_uint(pair_r2<K>(yi, yc, wc[g].x)),
                             __float_as_uint(pair_r2<K>(yi + kp, yc, wc[g].y)));
            m = min(m, __float_as_uint(pair_r2<K>(yi + 2 * kp, yc, wc[g].z)));
            m = min(m, __float_as_uint(pair_r2<K>(yi + 3 * kp, yc, wc[g].w)));
            if (g < 4) m0 = min(m0, m); else m1 = min(m1, m);
        }
        m0 = wave_min_u32_fast(m0);
        m1 = wave_min_u32_fast(m1);
        if (lane == 0) {
            a.unit_min[2 * h] = m0;
            a.unit_min[2 * h + 1] = m1;
        }
        best = min(best, min(m0, m1));
        __builtin_amdgcn_wave_barrier();
    }
    return block_min_u32(best);
}

// Plain pass block: one wavefront per 256-pair chunk (grid-stride).
template <int K, typename TX>
__device__ uint32_t plain_pass_block(const SweepArgs<TX> &a, int pb) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wid = (int64_t)pb * (kPairBlock / kWave) + wv;
    const int64_t nw = (int64_t)a.npass * (kPairBlock / kWave);
    uint32_t best = kKeyNone;
    for (int64_t ch = wid; ch < a.nchunks; ch += nw) {
        TX r2[4];
        plain_r2<K, TX>(a.S, a.pcols, a.n, a.Pr, ch * kChunk + lane * 4, r2);
        uint32_t kk[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) kk[e] = key_of<TX>(r2[e]);
        // the chunk's smallest and second-smallest keys: the selection
        // rescores a chunk's single window pair directly, without a rescan,
        // when the second-smallest key lies outside the window
        uint32_t m1 = min(kk[0], kk[1]), m2 = max(kk[0], kk[1]);
#pragma unroll
        for (int e = 2; e < 4; ++e) { m2 = min(m2, max(m1, kk[e])); m1 = min(m1, kk[e]); }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const uint32_t x1 = __shfl_xor(m1, o, kWave), x2 = __shfl_xor(m2, o, kWave);
            m2 = min(min(m2, x2), max(m1, x1));
            m1 = min(m1, x1);
        }
        // position of the first pair holding the smallest key
        const int ef = kk[0] == m1 ? 0 : kk[1] == m1 ? 1 : kk[2] == m1 ? 2 : kk[3] == m1 ? 3 : 4;
        const uint64_t bal = __ballot(ef < 4);
        const int fl = bal ? __builtin_ctzll(bal) : 0;
        const int arg = fl * 4 + __shfl(ef, fl, kWave);
        if (lane == 0) {
            a.unit_min[ch] = m1;
            a.unit_min2[ch] = m2;
            a.unit_arg[ch] = (uint32_t)arg;
        }
        best = min(best, m1);
    }
    return block_min_u32(best);
}

// c = P^T (x_i - x_j) for 16 short pairs in FP64 on the matrix cores, tiled
// exactly as gemm_block; lane (m = lane % 16, kk = lane / 16) passes pair m
// (pr, rin: whether it exists) and gets back c[pair kk + 4 v][component m]
// in element v (0 for m >= K).  The A operand is the pair's difference
// x_i - x_j formed from the two rows of X (exact in FP64 for FP32 inputs).
template <int K, typename TX>
__device__ __forceinline__ double4_t short_c16(const TX *__restrict__ X, int64_t ldx, int2 pr,
                                               bool rin, int n, const double *__restrict__ P64t,
                                               bool vx, bool vp) {
    const int lane = threadIdx.x & 63;
    const int m = lane & 15, kk = lane >> 4;
    const double pmask = m < K ? 1.0 : 0.0;
    const double *pc = P64t + (int64_t)(m < K ? m : K - 1) * n;
    const double rmask = rin ? 1.0 : 0.0;
    const TX *xi = X + (int64_t)pr.x * ldx;
    const TX *xj = X + (int64_t)pr.y * ldx;
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
    int l0 = 0;
    for (; l0 + 64 <= n; l0 += 64) {   // component l0 + 16 kk + q in k-slot kk of MFMA q
        double xa[16], xb[16], pb[16];
        const int lb = l0 + 16 * kk;
        load16(xi + lb, vx, xa);
        load16(xj + lb, vx, xb);
        load16(pc + lb, vp, pb);
#pragma unroll
        for (int q = 0; q < 16; ++q)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64((xa[q] - xb[q]) * rmask, pb[q] * pmask, acc, 0, 0, 0);
    }
    for (; l0 < n; l0 += 4) {
        const int l = l0 + kk;
        const double x = (l < n && rin) ? (double)xi[l] - (double)xj[l] : 0.0;
        const double p = (l < n && m < K) ? pc[l] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, p, acc, 0, 0, 0);
    }
    return acc;
}

// Sum over the 16 lanes of a DPP row (every lane of the row gets it).
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    return v + dpp_f64<0x140>(v);
}

// Short pairs of the iteration: r = ||c|| / d per pair (16 per wavefront,
// grid-stride), reduced to the block's lexicographic (r, i, j) minimum.
template <int K, typename TX>
__device__ void short_block(const SweepArgs<TX> &a, int sb, int nshort) {
    const int lane = threadIdx.x & 63;
    const int m = lane & 15, kk = lane >> 4;
    const int64_t ngroups = (a.nclose + 15) / 16;
    double best = __builtin_huge_val();
    int32_t bi = 0x7fffffff, bj = 0x7fffffff, cnt = 0;
    for (int64_t g16 = (int64_t)sb * (kPairBlock / kWave) + (threadIdx.x >> 6); g16 < ngroups;
         g16 += (int64_t)nshort * (kPairBlock / kWave)) {
        // pair m's indices and length, loaded once; the rows of X follow
        const int64_t row = g16 * 16 + m;
        const bool rin = row < a.nclose;
        const int2 pr = a.close[rin ? row : a.nclose - 1];
        const double dlen = a.cd[rin ? row : a.nclose - 1];
        const double4_t acc = short_c16<K, TX>(a.X, a.ldx, pr, rin, a.n, a.P64t, a.vx, a.vp);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const double q2 = row_sum16(acc[v] * acc[v]);
            const int src = kk + 4 * v;          // the lane (m = src) that loaded this pair
            const int pi = __shfl(pr.x, src, kWave), pj = __shfl(pr.y, src, kWave);
            const double dv = __shfl(dlen, src, kWave);
            const int64_t e = g16 * 16 + src;
            if (m == 0 && e < a.nclose) {
                const double r = sqrt(q2) / dv;
                ++cnt;
                if (lex_less(r, pi, pj, best, bi, bj)) { best = r; bi = pi; bj = pj; }
            }
        }
    }
    block_reduce_partial(best, bi, bj, cnt, 0, 0, a.spart + sb);
}

// Revisit one 16 x 64 sub-tile u (wavefront): every pair whose coarse value is
// inside the window is rescored in FP64 and its bound re-checked.
// Tile t of the upper triangle of nb x nb tiles, numbered row by row:
// t = bi nb - bi (bi - 1) / 2 + (bj - bi).
__device__ __forceinline__ int2 tile_coords(int64_t t, int64_t nb) {
    const double c = 2.0 * (double)nb + 1.0;
    const double disc = c * c - 8.0 * (double)t;
    int64_t bi = (int64_t)floor((c - sqrt(disc > 0.0 ? disc : 0.0)) * 0.5);
    if (bi < 0) bi = 0;
    if (bi > nb - 1) bi = nb - 1;
    while (bi > 0 && bi * nb - bi * (bi - 1) / 2 > t) --bi;
    while (bi < nb - 1 && (bi + 1) * nb - (bi + 1) * bi / 2 <= t) ++bi;
    const int64_t bj = t - (bi * nb - bi * (bi - 1) / 2) + bi;
    return make_int2((int)bi, (int)bj);
}

template <int K, typename TX>
__device__ void revisit_subtile(const SweepArgs<TX> &a, const double *Pl, int64_t u, uint32_t T2,
                                double &best, int32_t &bi, int32_t &bj, int32_t &nwin,
                                int32_t &nviol) {
    __shared__ float4 s_ry[kPairBlock / kWave][16 * kMaxK / 4];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int2 b = tile_coords(u >> 2, a.nb);
    const int32_t row0 = b.x * kTile + (int32_t)(u & 3) * 16;
    // every load of the sub-tile issued together; its 16 y_i rows go to this
    // wavefront's LDS slice (read back as broadcasts)
    const float4 *tp = a.invd2 + (u >> 2) * (kTileElems / 4) + (u & 3) * 256 + lane;
    const float4 w0 = tp[0], w1 = tp[64], w2 = tp[128], w3 = tp[192];
    float yj[K];
    load_yj<K>(a.Y, a.kp, (int64_t)b.y * kTile + lane, yj);
    const float4 *ysrc = reinterpret_cast<const float4 *>(a.Y + (int64_t)row0 * a.kp);
    __builtin_amdgcn_wave_barrier();
    if (lane < 4 * a.kp) s_ry[wv][lane] = ysrc[lane];
    __builtin_amdgcn_wave_barrier();
    const float *yi0 = reinterpret_cast<const float *>(s_ry[wv]);
    // loops kept rolled: one copy of the FP64 evaluation below
#pragma unroll 1
    for (int g = 0; g < 4; ++g) {
        const float4 w4 = g == 0 ? w0 : g == 1 ? w1 : g == 2 ? w2 : w3;
#pragma unroll 1
        for (int rr = 0; rr < 4; ++rr) {
            const float wr = rr == 0 ? w4.x : rr == 1 ? w4.y : rr == 2 ? w4.z : w4.w;
            const float r2 = pair_r2<K>(yi0 + (int64_t)(4 * g + rr) * a.kp, yj, wr);
            uint64_t cm = __ballot(__float_as_uint(r2) <= T2);
            while (cm) {
                const int ln = __builtin_ctzll(cm);
                cm &= cm - 1;
                const int32_t i = row0 + 4 * g + rr;
                const int32_t j = b.y * kTile + ln;
                const double r = exact_r_wave<K, TX>(a.X, a.ldx, a.n, Pl, i, j);
                const float r2c = __shfl(r2, ln, kWave);
                ++nwin;
                nviol += bound_broken(r, (double)r2c, a.e_abs, a.e_rel);
                if (lex_less(r, i, j, best, bi, bj)) { best = r; bi = i; bj = j; }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Rescan one 256-pair chunk of the plain form (wavefront): used only when the
// chunk may hold more than one window pair.
template <int K, typename TX>
__device__ void revisit_chunk(const SweepArgs<TX> &a, const double *Pl, int64_t ch, uint32_t T2,
                              double &best, int32_t &bi, int32_t &bj, int32_t &nwin,
                              int32_t &nviol) {
    const int lane = threadIdx.x & 63;
    TX r2[4];
    plain_r2<K, TX>(a.S, a.pcols, a.n, a.Pr, ch * kChunk + lane * 4, r2);
#pragma unroll 1
    for (int e = 0; e < 4; ++e) {   // rolled: one copy of the FP64 evaluation
        const TX re = e == 0 ? r2[0] : e == 1 ? r2[1] : e == 2 ? r2[2] : r2[3];
        uint64_t cm = __ballot(key_of<TX>(re) <= T2);
        while (cm) {
            const int ln = __builtin_ctzll(cm);
            cm &= cm - 1;
            int64_t i, j;
            decode_pair(ch * kChunk + ln * 4 + e, a.N, i, j);
            const double r = exact_r_wave<K, TX>(a.X, a.ldx, a.n, Pl, i, j);
            const TX r2c = __shfl(re, ln, kWave);
            ++nwin;
            nviol += bound_broken(r, (double)r2c, a.e_abs, a.e_rel);
            if (lex_less(r, (int32_t)i, (int32_t)j, best, bi, bj)) {
                best = r; bi = (int32_t)i; bj = (int32_t)j;
            }
        }
    }
}

// Selection (one block, after the pass): coarse minimum, window, FP64
// rescoring, record.  Wavefront w of the block revisits the units that
// wavefront slot w of each pass block produced, restricted to the pass
// blocks whose minimum lies inside the window.  Returns the winning pair in
// every thread (i < 0 if there is none).  Every dependent global round trip
// costs about a microsecond here, so each phase issues all of its loads
// before it uses any.
constexpr int kFlagCap = 512;        // flagged pass blocks listed in LDS (else a full scan)
constexpr int kBlkVec = 8;           // uint4 loads of block minima per thread: npass <= 8192
constexpr int kShortPerThread = 4;   // short-pair blocks per thread: <= 1024

template <int K, typename TX, bool FUSED>
__device__ int2 select_min(const SweepArgs<TX> &a, int nshort, const double *Pl) {
    __shared__ int s_flag[kFlagCap];
    __shared__ int s_nflag;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // per-block coarse minima (the array is padded with kKeyNone to a
    // multiple of 4 x 256 entries) and the short-pair partials (FP64)
    uint4 bm[kBlkVec];
    const int nvec = (a.npass + 4 * kPairBlock - 1) / (4 * kPairBlock);
#pragma unroll
    for (int m = 0; m < kBlkVec; ++m)
        bm[m] = m < nvec ? reinterpret_cast<const uint4 *>(a.blk_min)[threadIdx.x + m * kPairBlock]
                         : make_uint4(kKeyNone, kKeyNone, kKeyNone, kKeyNone);
    double best = __builtin_huge_val();
    int32_t bi = 0x7fffffff, bj = 0x7fffffff, nres_short = 0;
#pragma unroll
    for (int m = 0; m < kShortPerThread; ++m) {
        const int sb = (int)threadIdx.x + m * kPairBlock;
        if (sb < nshort) {
            const Partial p = a.spart[sb];
            if (lex_less(p.r, p.i, p.j, best, bi, bj)) { best = p.r; bi = p.i; bj = p.j; }
            nres_short += p.n_rescored;
        }
    }
    uint32_t g = kKeyNone;
#pragma unroll
    for (int m = 0; m < kBlkVec; ++m) g = min(g, min(min(bm[m].x, bm[m].y), min(bm[m].z, bm[m].w)));
    if (threadIdx.x == 0) s_nflag = 0;
    g = block_min_u32(g);
    double coarse, tr;
    const uint32_t T2 = window_key(g, a.e_abs, a.e_rel, &coarse, &tr);
    // pass blocks whose minimum lies inside the window: a bit mask of the
    // thread's 4 kBlkVec entries, then its set bits
    if (coarse >= 0.0) {
        uint32_t fm = 0;
#pragma unroll
        for (int m = 0; m < kBlkVec; ++m)
            fm |= (bm[m].x <= T2 ? 1u : 0u) << (4 * m) | (bm[m].y <= T2 ? 2u : 0u) << (4 * m) |
                  (bm[m].z <= T2 ? 4u : 0u) << (4 * m) | (bm[m].w <= T2 ? 8u : 0u) << (4 * m);
#pragma unroll 1
        while (fm) {
            const int bit = __builtin_ctz(fm);
            fm &= fm - 1;
            const int at = atomicAdd(&s_nflag, 1);
            if (at < kFlagCap) s_flag[at] = 4 * ((int)threadIdx.x + (bit >> 2) * kPairBlock) + (bit & 3);
        }
    }
    __syncthreads();
    const int nflag = s_nflag;
    int32_t nres = 0, ntl = 0, nviol = 0, nwin = 0;
    if (coarse >= 0.0) {
        const int64_t nw = (int64_t)a.npass * (kPairBlock / kWave);
        const int64_t nunits_w = FUSED ? a.nhalf : a.nchunks;   // work items of the pass
        // the list order depends on LDS atomics, but the set does not, and
        // the result is a lexicographic minimum over the set
        const bool listed = nflag <= kFlagCap;
        const int nscan = listed ? nflag : a.npass;
#pragma unroll 1
        for (int f = 0; f < nscan; ++f) {
            const int b = listed ? s_flag[f] : f;
            if (!listed && a.blk_min[b] > T2) continue;
            // the work items of wavefront slot wv of block b, 64 at a time
#pragma unroll 1
            for (int64_t h0 = (int64_t)b * (kPairBlock / kWave) + wv; h0 < nunits_w; h0 += kWave * nw) {
                const int64_t hl = h0 + lane * nw;
                uint32_t u0 = kKeyNone, u1 = kKeyNone, ag = 0;
                if (hl < nunits_w) {
                    if constexpr (FUSED) {
                        u0 = a.unit_min[2 * hl];
                        u1 = a.unit_min[2 * hl + 1];
                    } else {
                        u0 = a.unit_min[hl];
                        u1 = a.unit_min2[hl];
                        ag = a.unit_arg[hl];
                    }
                }
                uint64_t hits = __ballot((FUSED ? min(u0, u1) : u0) <= T2);
                while (hits) {
                    const int ln = __builtin_ctzll(hits);
                    hits &= hits - 1;
                    const int64_t h = h0 + (int64_t)ln * nw;
                    const uint32_t v0 = __shfl(u0, ln, kWave), v1 = __shfl(u1, ln, kWave);
                    if constexpr (FUSED) {
#pragma unroll 1
                        for (int x = 0; x < 2; ++x) {   // one call site
                            if ((x == 0 ? v0 : v1) <= T2) {
                                ++ntl;
                                revisit_subtile<K, TX>(a, Pl, 2 * h + x, T2, best, bi, bj, nwin, nviol);
                            }
                        }
                    } else {
                        ++ntl;
                        if (v1 > T2) {
                            // the chunk's only window pair: rescore it directly
                            int64_t i, j;
                            decode_pair(h * kChunk + __shfl(ag, ln, kWave), a.N, i, j);
                            const double r = exact_r_wave<K, TX>(a.X, a.ldx, a.n, Pl, i, j);
                            ++nwin;
                            nviol += bound_broken(r, (double)__uint_as_float(v0), a.e_abs, a.e_rel);
                            if (lex_less(r, (int32_t)i, (int32_t)j, best, bi, bj)) {
                                best = r; bi = (int32_t)i; bj = (int32_t)j;
                            }
                        } else {
                            revisit_chunk<K, TX>(a, Pl, h, T2, best, bi, bj, nwin, nviol);
                        }
                    }
                }
            }
        }
    }
    if (lane != 0) { nwin = 0; ntl = 0; nviol = 0; }
    nres = nwin + nres_short;
    __shared__ Partial s_fin;
    block_reduce_partial(best, bi, bj, nres, ntl, nviol, &s_fin);
    if (threadIdx.x == 0) {
        const Partial f = s_fin;
        const bool found = f.r < __builtin_huge_val();
        const int cert = (found && f.n_viol == 0) ? 1 : 0;
        DevResult *res = a.res;
        res->min_norm = f.r;
        res->i = found ? f.i : -1;
        res->j = found ? f.j : -1;
        res->q = found ? pair_index(a.N, f.i, f.j) : -1;
        res->coarse_min = coarse;
        res->window = coarse >= 0.0 ? tr - coarse : 0.0;
        res->certified = cert;
        res->n_rescored = f.n_rescored;
        res->n_tiles = f.n_tiles;
        res->t = -1;
        if (a.tr_min) a.tr_min[a.it] = f.r;
        if (a.tr_ij) {
            a.tr_ij[2 * a.it] = found ? f.i : -1;
            a.tr_ij[2 * a.it + 1] = found ? f.j : -1;
        }
        if (a.tr_cert) a.tr_cert[a.it] = cert;
        *a.gmin_out = g;
    }
    __syncthreads();
    const Partial f = s_fin;
    return f.r < __builtin_huge_val() ? make_int2(f.i, f.j) : make_int2(-1, -1);
}

// The pass.  Fused form: the first nshort blocks score the short pairs in
// FP64 (they need only P, and start first so that they run beside the
// coarse blocks), the other npass blocks score every pair coarsely.  Every
// block writes its own result slot; the kernel boundary is the grid-wide
// barrier before selection.
template <int K, typename TX, bool FUSED>
__global__ __launch_bounds__(kPairBlock) void k_pass(SweepArgs<TX> a, int nshort) {
    if constexpr (FUSED) {
        if ((int)blockIdx.x < nshort) {
            short_block<K, TX>(a, (int)blockIdx.x, nshort);
            return;
        }
    }
    const int pb = (int)blockIdx.x - (FUSED ? nshort : 0);
    uint32_t best;
    if constexpr (FUSED) best = fused_pass_block<K, TX>(a, pb);
    else best = plain_pass_block<K, TX>(a, pb);
    if (threadIdx.x == 0) a.blk_min[pb] = best;
}

// Fused form, before the pass: Y = (X - mu) P.
template <int K, typename TX>
__global__ __launch_bounds__(kPairBlock) void k_prep(SweepArgs<TX> a, const double *__restrict__ mu,
                                                     float *__restrict__ Y, int64_t Npad) {
    gemm_block<TX>(a.X, a.ldx, a.N, a.n, K, mu, a.P64t, Y, a.kp, Npad, a.vx, a.vp);
}

// ------------------------------------------------------------------ the update

// One wavefront: the paper's update of P in FP64, from the recorded pair:
//   c = P^T s;  t = first argmax |c_t|;
//   if c = 0:   P' = [s, p_2, .., p_k]
//   else:       v = P c; modified Gram-Schmidt on (v, p_1..p_k without p_t);
//               u = unit((1-a) v + a (s - v))   [rule 1: unit vectors of v, s-v]
//               P' = [u, q_2, .., q_k]
// The vectors live in LDS (A: K x n, then s, v, c); lane l owns components
// l, l+64, ...; every inner product is a wavefront sum.  Modified
// Gram-Schmidt runs right-looking: once q_m is final, every later vector
// loses its component along q_m (per vector, the same sequence of
// subtractions as the column-by-column form).  The loops are deliberately
// not unrolled: this code runs once per launch, and straight-line code is
// bound by instruction fetch.
template <int K, typename TX>
__device__ void apply_update(const TX *__restrict__ X, int64_t ldx, int n,
                             double *__restrict__ P64t, double *__restrict__ P64r,
                             void *__restrict__ Pr, int pr_kind, double alpha, int rule,
                             DevResult *__restrict__ res, int64_t i, int64_t j, double *sm) {
    const int lane = threadIdx.x & 63;
    double *A = sm;                       // K x n: P (loaded by the caller), then MGS vectors
    double *s = sm + (size_t)K * n;       // unit secant, later u
    double *v = s + n;                    // P P^T s
    double *c = v + n;                    // P^T s (16 slots)
    double d2 = 0.0;
    for (int l = lane; l < n; l += kWave) {
        const double dl = (double)X[i * ldx + l] - (double)X[j * ldx + l];
        s[l] = dl;
        d2 = __builtin_fma(dl, dl, d2);
    }
    const double d = sqrt(wave_sum_fast(d2));
    for (int l = lane; l < n; l += kWave) s[l] = s[l] / d;
    // c = P^T s, t = first argmax |c_t| (every lane holds the same sums)
    int t = 0;
    double cmax = -1.0;
#pragma unroll 1
    for (int q = 0; q < K; ++q) {
        double acc = 0.0;
        for (int l = lane; l < n; l += kWave) acc = __builtin_fma(A[(size_t)q * n + l], s[l], acc);
        acc = wave_sum_fast(acc);
        if (lane == 0) c[q] = acc;
        if (fabs(acc) > cmax) { cmax = fabs(acc); t = q; }
    }
    if (lane == 0) res->t = t;

    if (cmax == 0.0) {
        for (int l = lane; l < n; l += kWave) A[l] = s[l];
    } else {
        // v = P c; MGS input order (v, p_1..p_{t-1}, p_{t+1}..p_k), in place
        for (int l = lane; l < n; l += kWave) {
            double acc = 0.0;
#pragma unroll 1
            for (int q = 0; q < K; ++q) acc = __builtin_fma(A[(size_t)q * n + l], c[q], acc);
            v[l] = acc;
            for (int m = t; m > 0; --m) A[(size_t)m * n + l] = A[(size_t)(m - 1) * n + l];
            A[l] = acc;
        }
        double vnorm = 0.0;
#pragma unroll 1
        for (int m = 0; m < K; ++m) {
            double *am = A + (size_t)m * n;
            double nn = 0.0;
            for (int l = lane; l < n; l += kWave) nn = __builtin_fma(am[l], am[l], nn);
            const double nrm = sqrt(wave_sum_fast(nn));
            if (m == 0) vnorm = nrm;
            for (int l = lane; l < n; l += kWave) am[l] = am[l] / nrm;
#pragma unroll 1
            for (int jv = m + 1; jv < K; ++jv) {
                double *aj = A + (size_t)jv * n;
                double dot = 0.0;
                for (int l = lane; l < n; l += kWave) dot = __builtin_fma(am[l], aj[l], dot);
                dot = wave_sum_fast(dot);
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
            wn = sqrt(wave_sum_fast(acc));
        }
        double un = 0.0;
        for (int l = lane; l < n; l += kWave) {
            double u;
            if (rule == SAP_STEP_NORMALIZED)
                u = (1.0 - alpha) * (v[l] / vnorm) + (wn > 0.0 ? alpha * ((s[l] - v[l]) / wn) : 0.0);
            else
                u = (1.0 - alpha) * v[l] + alpha * (s[l] - v[l]);
            s[l] = u;
            un = __builtin_fma(u, u, un);
        }
        const double unrm = sqrt(wave_sum_fast(un));
        for (int l = lane; l < n; l += kWave) A[l] = s[l] / unrm;
    }
    // write back: master (K x n), row-major FP64 copy, and the plain pass's copy
    for (int l = lane; l < n; l += kWave) {
#pragma unroll 1
        for (int q = 0; q < K; ++q) {
            const double pv = A[(size_t)q * n + l];
            P64t[(int64_t)q * n + l] = pv;
            P64r[(int64_t)l * K + q] = pv;
            if (pr_kind == 1) static_cast<float *>(Pr)[(int64_t)l * K + q] = (float)pv;
            else if (pr_kind == 2) static_cast<double *>(Pr)[(int64_t)l * K + q] = pv;
        }
    }
}

// The same update with the vectors in registers, for n <= 64 M (lane l owns
// components l + 64 m) and small K M: every operation of apply_update, in the
// same order per vector, but without LDS round trips, and with the
// independent inner products of one step (c = P^T s; the projections of all
// later vectors on q_m) reduced together, so their latencies overlap.
template <int K, int M, typename TX>
__device__ __forceinline__ void apply_update_reg(const TX *__restrict__ X, int64_t ldx, int n, const double *Pl,
                                 double *__restrict__ P64t, double *__restrict__ P64r,
                                 void *__restrict__ Pr, int pr_kind, double alpha, int rule,
                                 DevResult *__restrict__ res, int64_t i, int64_t j) {
    const int lane = threadIdx.x & 63;
    double A[K][M], s[M], v[M];
    double d2 = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int l = lane + 64 * m;
        const bool in = l < n;
        const int lc = in ? l : 0;
        const double dl = in ? (double)X[i * ldx + lc] - (double)X[j * ldx + lc] : 0.0;
        s[m] = dl;
        d2 = __builtin_fma(dl, dl, d2);
#pragma unroll
        for (int q = 0; q < K; ++q) A[q][m] = in ? Pl[q * n + lc] : 0.0;
    }
    const double d = sqrt(wave_sum_fast(d2));
#pragma unroll
    for (int m = 0; m < M; ++m) s[m] = s[m] / d;
    double c[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        c[q] = 0.0;
#pragma unroll
        for (int m = 0; m < M; ++m) c[q] = __builtin_fma(A[q][m], s[m], c[q]);
    }
    wave_sum_many<K>(c);
    int t = 0;
    double cmax = -1.0;
#pragma unroll
    for (int q = 0; q < K; ++q)
        if (fabs(c[q]) > cmax) { cmax = fabs(c[q]); t = q; }
    if (lane == 0) res->t = t;
    if (cmax == 0.0) {
#pragma unroll
        for (int m = 0; m < M; ++m) A[0][m] = s[m];
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < K; ++q) acc = __builtin_fma(A[q][m], c[q], acc);
            v[m] = acc;
        }
        // MGS input order (v, p_1..p_{t-1}, p_{t+1}..p_k): rows 1..t take
        // rows 0..t-1 (selects, no dynamic register indexing)
#pragma unroll
        for (int q = K - 1; q >= 1; --q)
#pragma unroll
            for (int m = 0; m < M; ++m) A[q][m] = q <= t ? A[q - 1][m] : A[q][m];
#pragma unroll
        for (int m = 0; m < M; ++m) A[0][m] = v[m];
        double vnorm = 0.0;
#pragma unroll
        for (int mm = 0; mm < K; ++mm) {
            double nn = 0.0;
#pragma unroll
            for (int m = 0; m < M; ++m) nn = __builtin_fma(A[mm][m], A[mm][m], nn);
            const double nrm = sqrt(wave_sum_fast(nn));
            if (mm == 0) vnorm = nrm;
#pragma unroll
            for (int m = 0; m < M; ++m) A[mm][m] = A[mm][m] / nrm;
            double dots[K];
#pragma unroll
            for (int jv = 0; jv < K; ++jv) {
                dots[jv] = 0.0;
                if (jv > mm) {
#pragma unroll
                    for (int m = 0; m < M; ++m) dots[jv] = __builtin_fma(A[mm][m], A[jv][m], dots[jv]);
                }
            }
            wave_sum_many<K>(dots, mm + 1);
#pragma unroll
            for (int jv = mm + 1; jv < K; ++jv)
#pragma unroll
                for (int m = 0; m < M; ++m) A[jv][m] = A[jv][m] - dots[jv] * A[mm][m];
        }
        double wn = 1.0;
        if (rule == SAP_STEP_NORMALIZED) {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const double w = s[m] - v[m];
                acc = __builtin_fma(w, w, acc);
            }
            wn = sqrt(wave_sum_fast(acc));
        }
        double un = 0.0;
        double u[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (rule == SAP_STEP_NORMALIZED)
                u[m] = (1.0 - alpha) * (v[m] / vnorm) + (wn > 0.0 ? alpha * ((s[m] - v[m]) / wn) : 0.0);
            else
                u[m] = (1.0 - alpha) * v[m] + alpha * (s[m] - v[m]);
            un = __builtin_fma(u[m], u[m], un);
        }
        const double unrm = sqrt(wave_sum_fast(un));
#pragma unroll
        for (int m = 0; m < M; ++m) A[0][m] = u[m] / unrm;
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int l = lane + 64 * m;
        if (l < n) {
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const double pv = A[q][m];
                P64t[(int64_t)q * n + l] = pv;
                P64r[(int64_t)l * K + q] = pv;
                if (pr_kind == 1) static_cast<float *>(Pr)[(int64_t)l * K + q] = (float)pv;
                else if (pr_kind == 2) static_cast<double *>(Pr)[(int64_t)l * K + q] = pv;
            }
        }
    }
}

// Selection, record and (do_step) update, in one block.  Dynamic LDS holds
// P (read by the rescoring, then the update's working copy) and the update's
// vectors: (K + 2) n + 16 doubles.
template <int K, typename TX, bool FUSED>
__global__ __launch_bounds__(kPairBlock) void k_select(SweepArgs<TX> a, int nshort,
                                                       double *__restrict__ P64t,
                                                       double *__restrict__ P64r,
                                                       void *__restrict__ Pr, int pr_kind,
                                                       double alpha, int rule, int do_step) {
    extern __shared__ double sm_dyn[];
    // P into LDS now, so that its loads overlap the first phase (the block
    // barriers inside select_min order these writes before any read)
    for (int e = threadIdx.x; e < K * a.n; e += kPairBlock) sm_dyn[e] = a.P64t[e];
    const int2 ij = select_min<K, TX, FUSED>(a, nshort, sm_dyn);
    if (do_step && ij.x >= 0 && threadIdx.x < kWave) {
        // registers when every vector fits one 64-lane slice and K is
        // small, LDS otherwise
        if (K <= 8 && a.n <= 64)
            apply_update_reg<K, 1, TX>(a.X, a.ldx, a.n, sm_dyn, P64t, P64r, Pr, pr_kind, alpha, rule,
                                       a.res, ij.x, ij.y);
        else
            apply_update<K, TX>(a.X, a.ldx, a.n, P64t, P64r, Pr, pr_kind, alpha, rule, a.res, ij.x,
                                ij.y, sm_dyn);
    }
}

// ------------------------------------------------------------------ small helpers

// Write the row-major copies of P (FP64, and the plain pass's T) from the master.
template <typename T>
__global__ void k_write_P_copies(const double *__restrict__ P64t, int n, int k,
                                 double *__restrict__ P64r, T *__restrict__ Pr) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int l = e / k, q = e % k;
    const double pv = P64t[(int64_t)q * n + l];
    P64r[e] = pv;
    if (Pr) Pr[e] = (T)pv;
}

// P_out (n x k row-major) <- master (k x n)
__global__ void k_P_out(const double *__restrict__ P64t, int n, int k, double *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * k) return;
    const int l = e / k, q = e % k;
    out[e] = P64t[(int64_t)q * n + l];
}

// Lengths of the short pairs, once: cd[e] = ||x_i - x_j||, the differences
// formed in FP64 (exact for FP32 inputs).
template <typename TX>
__global__ void k_short_len(const TX *__restrict__ X, int64_t ldx, int n,
                            const int2 *__restrict__ close, int64_t nclose,
                            double *__restrict__ cd) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nclose) return;
    const int2 pr = close[e];
    double d2 = 0.0;
    for (int l = 0; l < n; ++l) {
        const double dl = (double)X[(int64_t)pr.x * ldx + l] - (double)X[(int64_t)pr.y * ldx + l];
        d2 = __builtin_fma(dl, dl, d2);
    }
    cd[e] = sqrt(d2);
}

}  // namespace sap
