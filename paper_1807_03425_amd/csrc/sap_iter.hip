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

// DPP lane permutation of a double (two 32-bit moves).  Every control used
// here (quad permutations, half-row and row mirrors, row rotations) reads a
// valid lane for every lane, so the moves take no "old" operand: that would
// cost a register initialisation per move.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
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

// v[from..NV-1] summed over the wavefront, the reductions interleaved (the
// same steps as wave_sum_fast, so each sum has the same bits).
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
    for (int a = 0; a < NV; ++a) if (a >= from) v[a] = pair_sum16(v[a]);
#pragma unroll
    for (int a = 0; a < NV; ++a) if (a >= from) v[a] = pair_sum32(v[a]);
}

// mine + (other of lane ^ 2^S), S < 4: quad xor 1, quad xor 2, xor 4 as a
// quad reversal followed by the half-row mirror (lane L reads lane L ^ 4),
// xor 8 as the 16-lane rotation by 8.  The partners are those of
// wave_sum_fast's steps (aligned lane groups of 2, 4, 8, 16), so a sum built
// from these steps and the permlane swaps has wave_sum_fast's bits.
template <int S>
__device__ __forceinline__ double xchg_add(double mine, double other) {
    if constexpr (S == 0) return mine + dpp_f64<0xB1>(other);
    else if constexpr (S == 1) return mine + dpp_f64<0x4E>(other);
    else if constexpr (S == 2) return mine + dpp_f64<0x141>(dpp_f64<0x1B>(other));
    else return mine + dpp_f64<0x128>(other);
}

// Wavefront sums of v[0..NV-1] (NV <= 16), transposed: the exchange at
// distance 2^s (s < H = ceil(log2 NV)) halves the values each lane carries
// -- the lane keeps the half whose index has bit s equal to its lane's bit
// s and receives its partner's share of that half -- and the later
// exchanges add whole sums.  Lane L ends with the total of index L mod 2^H,
// with the bits wave_sum_fast gives that index: about a quarter of the
// exchanges of NV separate reductions.
template <int NV>
__device__ __forceinline__ double wave_sum_transposed(const double (&v)[NV]) {
    static_assert(NV >= 1 && NV <= 16, "reduction batch");
    constexpr int H = NV <= 1 ? 0 : NV <= 2 ? 1 : NV <= 4 ? 2 : NV <= 8 ? 3 : 4;
    const int lane = threadIdx.x & (kWave - 1);
    double c[1 << H];
#pragma unroll
    for (int e = 0; e < (1 << H); ++e) c[e] = e < NV ? v[e] : 0.0;
#pragma unroll
    for (int st = 0; st < H; ++st) {
        const bool up = (lane >> st) & 1;
#pragma unroll
        for (int u = 0; u < (1 << (H - 1 - st)); ++u) {
            const double lo = c[2 * u], hi = c[2 * u + 1];
            const double mine = up ? hi : lo, other = up ? lo : hi;
            if (st == 0) c[u] = xchg_add<0>(mine, other);
            else if (st == 1) c[u] = xchg_add<1>(mine, other);
            else if (st == 2) c[u] = xchg_add<2>(mine, other);
            else c[u] = xchg_add<3>(mine, other);
        }
    }
    double t = c[0];
    if constexpr (H <= 0) t = xchg_add<0>(t, t);
    if constexpr (H <= 1) t = xchg_add<1>(t, t);
    if constexpr (H <= 2) t = xchg_add<2>(t, t);
    if constexpr (H <= 3) t = xchg_add<3>(t, t);
    t = pair_sum16(t);
    return pair_sum32(t);
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

// 16 consecutive elements in their own type (a prefetch: converted at use,
// so that no conversion waits for the load where it is issued).
template <typename T>
__device__ __forceinline__ void load16_raw(const T *__restrict__ p, bool vec, T (&o)[16]) {
    if (vec) {
        using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
        constexpr int W = 16 / (int)sizeof(T);
        const V *q = reinterpret_cast<const V *>(p);
#pragma unroll
        for (int u = 0; u < 16 / W; ++u) {
            const V t = q[u];
            const T *tv = reinterpret_cast<const T *>(&t);
#pragma unroll
            for (int w = 0; w < W; ++w) o[W * u + w] = tv[w];
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
// The lane's operands of gemm_block's first chunk (used when n >= 64 and X
// rows take 16-byte loads): 16 values of its X row (in X's type: converted
// at use, so that nothing waits for these loads where they are issued) and
// the matching 16 column means.  The loads are issued whether or not they
// are used (from `spare`, any 16-byte aligned 512 bytes of device memory,
// when not): with no branch around them, the wait for loads issued earlier
// stays exact.
template <typename TX>
__device__ __forceinline__ void gemm_first_x(const TX *__restrict__ X, int64_t ldx, int64_t N, int64_t row0,
                                             int l0, bool use, const void *spare, const double *__restrict__ mu,
                                             TX (&xa)[16], double (&ma)[16]) {
    const int lane = threadIdx.x & 63;
    const int64_t row = row0 + (lane & 15);
    const TX *xp = use ? X + (row < N ? row : N - 1) * ldx + l0 + 16 * (lane >> 4) : static_cast<const TX *>(spare);
    const double *mp = use ? mu + l0 + 16 * (lane >> 4) : static_cast<const double *>(spare);
    load16_raw(xp, true, xa);
    load16_raw(mp, true, ma);
}
// The same without 16-byte loads (X rows not 16-byte aligned).
template <typename TX>
__device__ __forceinline__ void gemm_first_x_scalar(const TX *__restrict__ X, int64_t ldx, int64_t N, int64_t Npad,
                                                    const double *__restrict__ mu, TX (&xa)[16], double (&ma)[16]) {
    const int lane = threadIdx.x & 63;
    const int64_t row0 = min(((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16, Npad - 16);
    const int64_t row = row0 + (lane & 15);
    load16_raw(X + (row < N ? row : N - 1) * ldx + 16 * (lane >> 4), false, xa);
    load16_raw(mu + 16 * (lane >> 4), true, ma);
}

typedef float float4_mfma __attribute__((ext_vector_type(4)));
typedef short bf16x4_bits __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float f) { return __builtin_bit_cast(short, static_cast<__bf16>(f)); }

// The same 16 x 16 tile of Y with FP32 or BF16 operands and FP32
// accumulation (gemm = SAP_GEMM_F32: v_mfma_f32_16x16x4f32, one component
// per lane and k-slot, components mapped as in the FP64 routine; SAP_GEMM_BF16:
// v_mfma_f32_16x16x16bf16_1k, lane (m, kk) feeding its 16 consecutive
// components of a 64-component chunk as k-slots 4 kk .. 4 kk + 3 of four
// MFMAs).  x - mu is formed in FP64 and rounded once to FP32 (then to BF16);
// P is rounded the same way.  Output layout of both instructions (measured on
// gfx950 with an in-bounds probe): lane holds rows 4 (lane / 16) + v,
// v = 0..3, column lane % 16.
template <typename TX>
__device__ __forceinline__ void gemm_block_lowp(const TX *__restrict__ X, int64_t ldx, int64_t N, int n, int k,
                                                const double *__restrict__ mu, const double *__restrict__ P64t,
                                                float *__restrict__ Y, int kp, int64_t row0, bool vx, bool vp,
                                                const TX (&x0)[16], const double (&m0)[16], bool use_x0,
                                                int gemm) {
    const int lane = threadIdx.x & 63;
    const int m = lane & 15, kk = lane >> 4;
    const int64_t row = row0 + m;
    const bool rin = row < N;
    const double rmask = rin ? 1.0 : 0.0, pmask = m < k ? 1.0 : 0.0;
    const TX *xr = X + (rin ? row : N - 1) * ldx;
    const double *pc = P64t + (int64_t)(m < k ? m : k - 1) * n;
    float4_mfma acc = {0.0f, 0.0f, 0.0f, 0.0f};
    int l0 = 0;
    for (; l0 + 64 <= n; l0 += 64) {
        double xa[16], ma[16], pb[16];
        const int lb = l0 + 16 * kk;
        if (use_x0 && l0 == 0) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                TX t = x0[u];
                asm volatile("" : "+v"(t));   // converted here, as in gemm_block
                xa[u] = (double)t;
                ma[u] = m0[u];
            }
        } else {
            load16(xr + lb, vx, xa);
            load16(mu + lb, true, ma);
        }
        load16(pc + lb, vp, pb);
        if (gemm == SAP_GEMM_F32) {
#pragma unroll
            for (int s = 0; s < 16; ++s)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)((xa[s] - ma[s]) * rmask), (float)(pb[s] * pmask),
                                                           acc, 0, 0, 0);
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                bf16x4_bits a4, b4;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a4[u] = bf16_bits((float)((xa[4 * s + u] - ma[4 * s + u]) * rmask));
                    b4[u] = bf16_bits((float)(pb[4 * s + u] * pmask));
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a4, b4, acc, 0, 0, 0);
            }
        }
    }
    if (gemm == SAP_GEMM_F32) {
        for (; l0 < n; l0 += 4) {
            const int l = l0 + kk;
            double a = 0.0, b = 0.0;
            if (l < n) {
                if (rin) a = (double)xr[l] - mu[l];
                if (m < k) b = pc[l];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, acc, 0, 0, 0);
        }
    } else {
        for (; l0 < n; l0 += 16) {
            bf16x4_bits a4, b4;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int l = l0 + 4 * kk + u;
                double a = 0.0, b = 0.0;
                if (l < n) {
                    if (rin) a = (double)xr[l] - mu[l];
                    if (m < k) b = pc[l];
                }
                a4[u] = bf16_bits((float)a);
                b4[u] = bf16_bits((float)b);
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a4, b4, acc, 0, 0, 0);
        }
    }
    if (m < kp) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t r = row0 + 4 * kk + v;
            Y[r * kp + m] = (r < N && m < k) ? acc[v] : 0.0f;
        }
    }
}

// x0, m0 (used when use_x0): the first chunk's X values and means, loaded
// earlier by k_selprep.  gemm: SAP_GEMM_F64 (below), or SAP_GEMM_F32 /
// SAP_GEMM_BF16 (gemm_block_lowp).  With the FP64 GEMM, Y64 (if not null)
// receives the same products unrounded (the short-pair bounds use them).
// A block covers 64 tpw rows; this call computes the wavefront's 16 rows of
// its tile-th group of 64.
template <typename TX>
__device__ __forceinline__ void gemm_block(const TX *__restrict__ X, int64_t ldx, int64_t N, int n, int k,
                           const double *__restrict__ mu, const double *__restrict__ P64t,
                           float *__restrict__ Y, double *__restrict__ Y64, int kp, int64_t Npad, bool vx,
                           bool vp, const TX (&x0)[16], const double (&m0)[16], bool use_x0, int gemm,
                           int tpw = 1, int tile = 0) {
    const int lane = threadIdx.x & 63;
    const int64_t row0 = (((int64_t)blockIdx.x * tpw + tile) * 4 + (threadIdx.x >> 6)) * 16;
    if (row0 >= Npad) return;
    if (gemm != SAP_GEMM_F64) {
        gemm_block_lowp<TX>(X, ldx, N, n, k, mu, P64t, Y, kp, row0, vx, vp, x0, m0, use_x0, gemm);
        return;
    }
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
    if (n >= 64) {
        // software-pipelined over 64-component chunks: the next chunk's
        // operands are in flight during this chunk's 16 MFMAs
        double xa[16], ma[16], pb[16];
        if (use_x0) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                // converted here, not where the prefetch was issued (the empty
                // asm pins the conversion after this point)
                TX t = x0[u];
                asm volatile("" : "+v"(t));
                xa[u] = (double)t;
                ma[u] = m0[u];
            }
        } else {
            load16(xr + 16 * kk, vx, xa);
            load16(mu + 16 * kk, true, ma);
        }
        load16(pc + 16 * kk, vp, pb);
        for (; l0 + 64 <= n; l0 += 64) {
            TX xn[16];
            double mn[16], pn[16];
            const bool more = l0 + 128 <= n;           // wavefront-uniform
            if (more) {
                const int lb = l0 + 64 + 16 * kk;
                load16_raw(xr + lb, vx, xn);
                load16_raw(mu + lb, true, mn);
                load16_raw(pc + lb, vp, pn);
            }
#pragma unroll
            for (int s = 0; s < 16; ++s)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64((xa[s] - ma[s]) * rmask, pb[s] * pmask,
                                                           acc, 0, 0, 0);
            if (more) {
#pragma unroll
                for (int u = 0; u < 16; ++u) { xa[u] = (double)xn[u]; ma[u] = mn[u]; pb[u] = pn[u]; }
            }
        }
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
            const double y = (r < N && m < k) ? acc[v] : 0.0;
            Y[r * kp + m] = (float)y;
            if (Y64) Y64[r * kp + m] = y;
        }
    }
}

// The 16-row tile (first row row0) and the range of 64-component chunks
// [cb, cb + nch) of the calling wavefront in gemm_block_deep.
__device__ __forceinline__ void deep_tile(bool split, int n, int64_t &row0, int &cb, int &nch) {
    const int w = threadIdx.x >> 6;
    if (split) {
        row0 = ((int64_t)blockIdx.x * 2 + (w & 1)) * 16;
        nch = n >> 7;
        cb = (w >> 1) * nch;
    } else {
        row0 = ((int64_t)blockIdx.x * 4 + w) * 16;
        nch = n >> 6;
        cb = 0;
    }
}

// The FP64 GEMM of gemm_block with P and the means in LDS and X streamed
// from memory four 64-component chunks deep: the lane's slices of chunks
// c + 1 .. c + 3 are in flight while chunk c's 16 MFMAs run, and the LDS
// operands of chunk c + 1 are read during them, so a long chain of chunks is
// bound by the matrix core rather than by one round trip per chunk.  X is
// the only global source inside the loop, so the wait for chunk c (in issue
// order) leaves the later chunks in flight.  Needs n a multiple of 256 and
// 16-byte X rows; x0 holds the wavefront's first chunk (prefetched in X's
// type, see deep_tile); loads past the last chunk re-read it.  Rows past N
// and columns past k read valid elements (row N - 1, column k - 1) and only
// feed outputs that are written as zeros, so no operand is masked.
//
// split (n a multiple of 512): a block covers 32 rows, and the wavefronts
// w and w + 2 share a 16-row tile, each taking half of the chunks; the
// second half's sums go through xch (LDS, 512 doubles) and are added to the
// first's (twice the blocks, half the chain per wavefront).  Every thread of
// the block must call it then.  A GEMM's rows are all computed one way or
// the other, so results do not depend on the kernel that computes them.
template <typename TX>
__device__ __forceinline__ void gemm_block_deep(const TX *__restrict__ X, int64_t ldx, int64_t N, int n, int k,
                                                const double *mu_l, const double *P_l, float *__restrict__ Y,
                                                double *__restrict__ Y64, int kp, int64_t Npad,
                                                const TX (&x0)[16], bool split, double *xch) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t row0;
    int cb, nch;
    deep_tile(split, n, row0, cb, nch);
    if (!split && row0 >= Npad) return;
    const int m = lane & 15, kk = lane >> 4;
    const int64_t row = row0 + m;
    const TX *xr = X + (row < N ? row : N - 1) * ldx + 64 * cb + 16 * kk;
    const double *pc = P_l + (m < k ? m : k - 1) * n + 64 * cb + 16 * kk;
    const double *mc = mu_l + 64 * cb + 16 * kk;
    TX xq[4][16];
#pragma unroll
    for (int u = 0; u < 16; ++u) xq[0][u] = x0[u];
#pragma unroll
    for (int c = 1; c < 4; ++c) load16_raw(xr + 64 * min(c, nch - 1), true, xq[c]);
    double ml[2][16], pl[2][16];   // LDS operands of chunks c (slot c & 1) and c + 1
    load16_raw(mc, true, ml[0]);
    load16_raw(pc, true, pl[0]);
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int g = 0; g < nch; g += 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = g + r;
            const int cn = min(c + 1, nch - 1);
            load16_raw(mc + 64 * cn, true, ml[(r + 1) & 1]);
            load16_raw(pc + 64 * cn, true, pl[(r + 1) & 1]);
            double xa[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                TX t = xq[r][u];
                asm volatile("" : "+v"(t));   // converted here, after chunk c has landed
                xa[u] = (double)t;
            }
            load16_raw(xr + 64 * min(c + 4, nch - 1), true, xq[r]);
#pragma unroll
            for (int s2 = 0; s2 < 16; ++s2)
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[s2] - ml[r & 1][s2], pl[r & 1][s2], acc, 0, 0, 0);
        }
    }
    if (split) {
        // the second half's sums, added to the first's in a fixed order
        double *xs = xch + ((w & 1) * kWave + lane) * 4;
        if (w >= 2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) xs[v] = acc[v];
        }
        __syncthreads();
        if (w >= 2) return;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = acc[v] + xs[v];
    }
    if (m < kp) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t r = row0 + kk + 4 * v;
            const double y = (r < N && m < k) ? acc[v] : 0.0;
            Y[r * kp + m] = (float)y;
            if (Y64) Y64[r * kp + m] = y;
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
        // P is read-only during the pass: its uniform row goes through the
        // constant address space (scalar loads), so it does not hold up the
        // vector loads of the next rows of S
        const __attribute__((address_space(4))) T *pl =
            (const __attribute__((address_space(4))) T *)(Pr + l * K);
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
// P (K x n, FP64, component-contiguous rows).  Wavefront-cooperative (lanes
// split the n components; every lane returns the same value).  The
// components come in groups of U per lane whose loads (clamped index,
// masked afterwards) are all issued before any is used.
template <int K, typename TX, int U = (K <= 8 ? 4 : 2)>
__device__ __forceinline__ double exact_r_wave(const TX *__restrict__ X, int64_t ldx, int n,
                                               const double *P64t, int64_t i, int64_t j) {
    const int lane = threadIdx.x & 63;
    const TX *xi = X + i * ldx, *xj = X + j * ldx;
    double v[K + 1];
#pragma unroll
    for (int q = 0; q <= K; ++q) v[q] = 0.0;
#pragma unroll 1
    for (int base = 0; base < n; base += U * kWave) {
        const int l0 = base + lane;
        double a[U], b[U], p[U][K];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int lc = min(l0 + u * kWave, n - 1);
            a[u] = (double)xi[lc];
            b[u] = (double)xj[lc];
#pragma unroll
            for (int q = 0; q < K; ++q) p[u][q] = P64t[(int64_t)q * n + lc];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double dl = l0 + u * kWave < n ? a[u] - b[u] : 0.0;
            v[K] = __builtin_fma(dl, dl, v[K]);
#pragma unroll
            for (int q = 0; q < K; ++q) v[q] = __builtin_fma(p[u][q], dl, v[q]);
        }
    }
    if constexpr (K + 1 <= 16) {
        // lane q holds the total of v[q]; read lanes 0..K back (uniform)
        const double t = wave_sum_transposed<K + 1>(v);
        const int tl = __double2loint(t), th = __double2hiint(t);
#pragma unroll
        for (int q = 0; q <= K; ++q)
            v[q] = __hiloint2double(__builtin_amdgcn_readlane(th, q), __builtin_amdgcn_readlane(tl, q));
    } else {
        wave_sum_many<K + 1>(v);
    }
    double r2 = 0.0;
#pragma unroll
    for (int q = 0; q < K; ++q) r2 = __builtin_fma(v[q], v[q], r2);
    return sqrt(r2) / sqrt(v[K]);
}

// exact_r_wave for two pairs at once (i1, j1) and (i2, j2): each group's
// loads of P serve both pairs, both pairs' rows are in flight together, and
// one transposed wavefront sum reduces the 2(K + 1) partial sums.  Each
// pair's partial sums are formed exactly as in exact_r_wave, so *r1 and *r2
// carry its bits.
template <int K, typename TX, int U = (K <= 8 ? 4 : 2)>
__device__ __forceinline__ void exact_r_wave2(const TX *__restrict__ X, int64_t ldx, int n, const double *P64t,
                                              int64_t i1, int64_t j1, int64_t i2, int64_t j2, double *r1,
                                              double *r2) {
    static_assert(2 * (K + 1) <= 16, "one transposed sum");
    const int lane = threadIdx.x & 63;
    const TX *xi1 = X + i1 * ldx, *xj1 = X + j1 * ldx;
    const TX *xi2 = X + i2 * ldx, *xj2 = X + j2 * ldx;
    double v[2 * (K + 1)];
#pragma unroll
    for (int q = 0; q < 2 * (K + 1); ++q) v[q] = 0.0;
#pragma unroll 1
    for (int base = 0; base < n; base += U * kWave) {
        const int l0 = base + lane;
        double a1[U], b1[U], a2[U], b2[U], p[U][K];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int lc = min(l0 + u * kWave, n - 1);
            a1[u] = (double)xi1[lc];
            b1[u] = (double)xj1[lc];
            a2[u] = (double)xi2[lc];
            b2[u] = (double)xj2[lc];
#pragma unroll
            for (int q = 0; q < K; ++q) p[u][q] = P64t[(int64_t)q * n + lc];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = l0 + u * kWave < n;
            const double d1 = in ? a1[u] - b1[u] : 0.0;
            const double d2 = in ? a2[u] - b2[u] : 0.0;
            v[K] = __builtin_fma(d1, d1, v[K]);
            v[2 * K + 1] = __builtin_fma(d2, d2, v[2 * K + 1]);
#pragma unroll
            for (int q = 0; q < K; ++q) {
                v[q] = __builtin_fma(p[u][q], d1, v[q]);
                v[K + 1 + q] = __builtin_fma(p[u][q], d2, v[K + 1 + q]);
            }
        }
    }
    // lane e holds the total of v[e]; read both pairs' sums back (uniform)
    const double t = wave_sum_transposed<2 * (K + 1)>(v);
    const int tl = __double2loint(t), th = __double2hiint(t);
#pragma unroll
    for (int e = 0; e < 2 * (K + 1); ++e)
        v[e] = __hiloint2double(__builtin_amdgcn_readlane(th, e), __builtin_amdgcn_readlane(tl, e));
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        s1 = __builtin_fma(v[q], v[q], s1);
        s2 = __builtin_fma(v[K + 1 + q], v[K + 1 + q], s2);
    }
    *r1 = sqrt(s1) / sqrt(v[K]);
    *r2 = sqrt(s2) / sqrt(v[2 * K + 1]);
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

// The window of a work item whose smallest key is m, in FP32 and rounded
// generously upward: T = (sqrt(m) (1 + e_rel) + 2 e_abs) / (1 - e_rel) = sqrt(m) wa + wb,
// and T^2 (1 + 1e-6) exceeds the exact square by more than the few FP32
// roundings of sqrt, multiply and add can lose.  A superset only costs
// rescoring time, never correctness.  A smallest key that is no valid value
// (an item of masked pairs only: negative or NaN bits) gets the empty window
// 0, which none of that item's keys is at or below.
__device__ __forceinline__ uint32_t item_window(uint32_t m, float wa, float wb) {
    if (m >= 0x7f800000u) return 0u;
    const float t = __builtin_fmaf(__builtin_amdgcn_sqrtf(__uint_as_float(m)), wa, wb);
    return __float_as_uint(t * t * 1.000001f);
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
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}

// (r, i, j) <- the lexicographic minimum of (r, i, j) and (r', i', j'), and r2
// <- the second-smallest value of the two top-2 sets: the smaller of the two
// second values and the first value of the tuple that lost.  The same pair
// on both sides (the lanes of a wavefront that rescored cooperatively hold
// identical results; a clamped duplicate load) is one element: only the
// second values merge.  Selects only: these merges form long dependent
// chains in single-wavefront code, where exec-mask branches cost far more
// than the few extra selects.
__device__ __forceinline__ void lex_pick2(double &r, int32_t &i, int32_t &j, double &r2, double rb, int32_t ib,
                                          int32_t jb, double r2b) {
    const bool same = (ib == i) & (jb == j);
    const bool less = !same & lex_less(rb, ib, jb, r, i, j);
    const double lost = less ? r : rb;   // the first value of the tuple that lost
    const double m2 = fmin(r2, r2b);
    r2 = same ? m2 : fmin(m2, lost);
    r = less ? rb : r;
    i = less ? ib : i;
    j = less ? jb : j;
}

template <int CTRL>
__device__ __forceinline__ void lex_step2_dpp(double &r, int32_t &i, int32_t &j, double &r2) {
    lex_pick2(r, i, j, r2, dpp_f64<CTRL>(r), dpp_i32<CTRL>(i), dpp_i32<CTRL>(j), dpp_f64<CTRL>(r2));
}

// Lexicographic (r, i, j) minimum over the wavefront and the second-smallest
// value r2 (over all lanes' top-2 sets), in every lane: the same six exchange
// steps as wave_sum_fast (four DPP steps inside 16-lane rows, then the
// permlane16 / permlane32 swaps, whose two results are the lane's own tuple
// and its partner's, in either order: the merge of the two does not depend on
// that order).  No LDS traffic.
__device__ __forceinline__ void wave_min_lex2_fast(double &r, int32_t &i, int32_t &j, double &r2) {
    lex_step2_dpp<0xB1>(r, i, j, r2);
    lex_step2_dpp<0x4E>(r, i, j, r2);
    lex_step2_dpp<0x141>(r, i, j, r2);
    lex_step2_dpp<0x140>(r, i, j, r2);
    {
        const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(r), __double2loint(r), false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(r), __double2hiint(r), false, false);
        const auto lo2 = __builtin_amdgcn_permlane16_swap(__double2loint(r2), __double2loint(r2), false, false);
        const auto hi2 = __builtin_amdgcn_permlane16_swap(__double2hiint(r2), __double2hiint(r2), false, false);
        const auto ii = __builtin_amdgcn_permlane16_swap(i, i, false, false);
        const auto jj = __builtin_amdgcn_permlane16_swap(j, j, false, false);
        r = __hiloint2double(hi[0], lo[0]); i = ii[0]; j = jj[0]; r2 = __hiloint2double(hi2[0], lo2[0]);
        lex_pick2(r, i, j, r2, __hiloint2double(hi[1], lo[1]), ii[1], jj[1], __hiloint2double(hi2[1], lo2[1]));
    }
    {
        const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(r), __double2loint(r), false, false);
        const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(r), __double2hiint(r), false, false);
        const auto lo2 = __builtin_amdgcn_permlane32_swap(__double2loint(r2), __double2loint(r2), false, false);
        const auto hi2 = __builtin_amdgcn_permlane32_swap(__double2hiint(r2), __double2hiint(r2), false, false);
        const auto ii = __builtin_amdgcn_permlane32_swap(i, i, false, false);
        const auto jj = __builtin_amdgcn_permlane32_swap(j, j, false, false);
        r = __hiloint2double(hi[0], lo[0]); i = ii[0]; j = jj[0]; r2 = __hiloint2double(hi2[0], lo2[0]);
        lex_pick2(r, i, j, r2, __hiloint2double(hi[1], lo[1]), ii[1], jj[1], __hiloint2double(hi2[1], lo2[1]));
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

// Block-wide reduction of a per-thread top-2 (r, i, j; r2), counters, the
// coarse minimum and the candidate-key limit, returned in every thread (and
// written to *out by thread 0 when out is non-null).  Every lane merges the
// four wavefront results in the same order, so the whole block holds the
// same value with one barrier.  All 256 threads must call it; sync_after
// adds the barrier a later call needs before it may reuse the staging slots.
// wave_uniform: every lane already holds its wavefront's values (lane 0's
// stand for the wavefront), so the wavefront reductions are skipped.
__device__ Partial block_reduce_partial(double r, int32_t i, int32_t j, double r2, int32_t nres, int32_t ntl,
                                        int32_t nviol, uint32_t kmin, uint32_t limit, Partial *out,
                                        bool sync_after, bool wave_uniform = false) {
    __shared__ Partial sb[kPairBlock / kWave];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (!wave_uniform) {
        wave_min_lex2_fast(r, i, j, r2);
        nres = wave_sum_i32_fast(nres);
        ntl = wave_sum_i32_fast(ntl);
        nviol = wave_sum_i32_fast(nviol);
        kmin = wave_min_u32_fast(kmin);
        limit = wave_min_u32_fast(limit);
    }
    if (lane == 0) sb[wv] = Partial{r, r2, i, j, nres, ntl, nviol, kmin, limit, 0};
    __syncthreads();
    Partial b = sb[0];
#pragma unroll
    for (int w = 1; w < kPairBlock / kWave; ++w) {
        const Partial o = sb[w];
        lex_pick2(b.r, b.i, b.j, b.r2, o.r, o.i, o.j, o.r2);
        b.n_rescored += o.n_rescored;
        b.n_units += o.n_units;
        b.n_viol += o.n_viol;
        b.kmin = min(b.kmin, o.kmin);
        b.limit = min(b.limit, o.limit);
    }
    if (out && threadIdx.x == 0) *out = b;
    if (sync_after) __syncthreads();
    return b;
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
    // plain pass
    const TX *S;
    int64_t pcols;
    const TX *Pr;
    int64_t nchunks;
    // both passes
    int n;
    int npass;           // pass blocks
    Partial *part;       // npass pass-block results, then one per short-pair block
    // short pairs (fused)
    const int2 *close;    // short pairs (i, j), sorted
    const double *cd;     // their lengths ||x_i - x_j||
    int64_t nclose;
    double *Y64;          // FP64 Y (FP64 GEMM; null otherwise): short-pair bounds
    double s_d2, s_eps;   // short-pair bound: |r~ - r| <= s_d2 / d + s_eps r~
    // FP64 rescoring and selection
    double e_abs, e_rel;
    float wa, wb;         // item_window coefficients: (1 + e_rel)/(1 - e_rel), 2 e_abs/(1 - e_rel),
                          // rounded up
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
    int cap;              // candidate-list capacity per wavefront, 1..kCandCap
    int gemm;             // arithmetic of the Y GEMM: SAP_GEMM_F64 | _F32 | _BF16
    int split;            // Y GEMM split over two wavefronts per tile (gemm_block_deep): k_prep
                          // and k_selprep then run n_pad / 32 blocks
    int gtiles;           // k_selprep: 64-row groups of Y per block (1 or 2: the TPW instance)
};

// Candidates of a pass block.  The block keeps its running minimum key in
// LDS; after a work item (a half-tile or a chunk) with smallest key m it is
// run = min(run, m), and every pair of the item with key <= T2(run) is a
// candidate.  The global window T2(global minimum) <= T2(block minimum) <=
// T2(run) at every point of the sweep, so every window pair of the
// iteration is a candidate of its own work item.  Each wavefront appends its
// candidates (i, j, key) to its LDS list during the pass; after the pass the
// block keeps those with key <= T2(block minimum) and rescores them in FP64
// (wavefront-cooperatively), re-checking each coarse value against the
// bound.
//
// A list that would overflow is first pruned to the current window.  If it
// would still overflow, the wavefront keeps its smallest keys: it lowers a
// key limit (only ever lowered) to the largest value that leaves at most
// three quarters of the capacity in the list, drops every entry above it and
// admits only keys at or below it from then on.  The limit is reported with
// the block's result; the evaluation stays certified as long as every limit
// is at or above the window of the global coarse minimum (no window pair was
// dropped), and is reported uncertified otherwise -- never silently wrong.
constexpr int kCandCap = 128;   // candidates per wavefront (largest capacity)

struct CandList {
    int2 *ij;
    uint32_t *key;
    int n;          // wavefront-uniform
    int cap;        // capacity, 1..kCandCap
    int lost;       // candidates dropped although no limit excluded them
    uint32_t limit; // candidate-key limit (kKeyNone: none)
};

struct WaveBest {
    double r, r2;   // best FP64 r (its pair i, j) and the second-smallest value
    int32_t i, j, nwin, nviol, nunits;
};

// Keep the list entries with key <= th, in order (lane-parallel: lane L holds
// entries L and L + 64; every entry is read before any is written).
__device__ __forceinline__ void prune_cands(CandList &cl, uint32_t th) {
    const int lane = threadIdx.x & 63;
    const bool v0 = lane < cl.n, v1 = lane + kWave < cl.n;
    int2 ij0 = make_int2(0, 0), ij1 = make_int2(0, 0);
    uint32_t k0 = kKeyNone, k1 = kKeyNone;
    if (v0) { ij0 = cl.ij[lane]; k0 = cl.key[lane]; }
    if (v1) { ij1 = cl.ij[lane + kWave]; k1 = cl.key[lane + kWave]; }
    const bool keep0 = v0 && k0 <= th, keep1 = v1 && k1 <= th;
    const uint64_t m0 = __ballot(keep0), m1 = __ballot(keep1);
    const int below0 = __builtin_amdgcn_mbcnt_hi((uint32_t)(m0 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m0, 0));
    const int below1 = __builtin_amdgcn_mbcnt_hi((uint32_t)(m1 >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m1, 0));
    const int n0 = __builtin_popcountll(m0);
    __builtin_amdgcn_wave_barrier();
    if (keep0) { cl.ij[below0] = ij0; cl.key[below0] = k0; }
    if (keep1) { cl.ij[n0 + below1] = ij1; cl.key[n0 + below1] = k1; }
    __builtin_amdgcn_wave_barrier();
    cl.n = n0 + __builtin_popcountll(m1);
}

// The largest key bound th <= te such that at most `target` keys -- list
// entries plus the lane keys flagged in `bits` -- are <= th, built bit by bit
// from the top (the count is monotone in th); but never below the smallest of
// those keys (when that key alone occurs more than `target` times, the list
// fills with it and the rest is counted as lost).
template <int NK>
__device__ __forceinline__ uint32_t cand_limit(const CandList &cl, const uint32_t (&key)[NK], uint32_t bits,
                                               uint32_t te, int target) {
    const int lane = threadIdx.x & 63;
    const uint32_t k0 = lane < cl.n ? cl.key[lane] : kKeyNone;
    const uint32_t k1 = lane + kWave < cl.n ? cl.key[lane + kWave] : kKeyNone;
    uint32_t th = 0;
#pragma unroll 1
    for (int b = 31; b >= 0; --b) {
        const uint32_t t = th | (1u << b);
        if (t > te) continue;   // wavefront-uniform
        int c = (k0 <= t ? 1 : 0) + (k1 <= t ? 1 : 0);
#pragma unroll
        for (int e = 0; e < NK; ++e) c += (((bits >> e) & 1u) && key[e] <= t) ? 1 : 0;
        if (wave_sum_i32_fast(c) <= target) th = t;
    }
    uint32_t m = min(k0, k1);
#pragma unroll
    for (int e = 0; e < NK; ++e) m = ((bits >> e) & 1u) ? min(m, key[e]) : m;
    return max(th, wave_min_u32_fast(m));
}

// Append the lanes' keys that are <= min(T2, limit) (T2: the window of the
// block's running minimum) to the wavefront's list.  key[e] belongs to the
// lane's pair pair(e, i, j); lmin is the lane's smallest key.  The few lanes
// holding candidates write their own entries, at offsets from a running count
// over those lanes, so no key has to move between lanes.
template <int NK, typename PairOf>
__device__ __forceinline__ void emit_cands(CandList &cl, const uint32_t (&key)[NK], uint32_t lmin,
                                           uint32_t T2, PairOf pair, WaveBest &wb) {
    const int lane = threadIdx.x & 63;
    uint32_t te = min(T2, cl.limit);
    uint32_t bits = 0;
    if (lmin <= te) {
#pragma unroll
        for (int e = 0; e < NK; ++e) bits |= (key[e] <= te ? 1u : 0u) << e;
    }
    int cnt = __builtin_popcount(bits);
    if (!__ballot(cnt > 0)) return;
    ++wb.nunits;
    int tot = wave_sum_i32_fast(cnt);
    if (cl.n + tot > cl.cap) {
        // rare: prune to the current window, then, if still full, keep the
        // smallest keys under a lowered limit
        prune_cands(cl, te);
        if (cl.n + tot > cl.cap) {
            const uint32_t th = cand_limit<NK>(cl, key, bits, te, max(1, (3 * cl.cap) / 4));
            cl.limit = th;
            te = th;
            prune_cands(cl, th);
#pragma unroll
            for (int e = 0; e < NK; ++e)
                if (key[e] > th) bits &= ~(1u << e);
            cnt = __builtin_popcount(bits);
            tot = wave_sum_i32_fast(cnt);
        }
    }
    uint64_t lanes = __ballot(cnt > 0);
    int base = 0, run = 0;
#pragma unroll 1
    while (lanes) {
        const int ln = __builtin_ctzll(lanes);
        lanes &= lanes - 1;
        if (lane == ln) base = run;
        run += __builtin_amdgcn_readlane(cnt, ln);
    }
    if (bits) {
        int pos = cl.n + base;
        if ((bits & (bits - 1u)) == 0u) {
            // one key in the window: it is the lane's smallest (the usual
            // case, a new running minimum)
            if (pos < cl.cap) {
                int32_t i, j;
                pair(__builtin_ctz(bits), i, j);
                cl.ij[pos] = make_int2(i, j);
                cl.key[pos] = lmin;
            }
        } else {
#pragma unroll
            for (int e = 0; e < NK; ++e) {
                if ((bits >> e) & 1u) {
                    if (pos < cl.cap) {
                        int32_t i, j;
                        pair(e, i, j);
                        cl.ij[pos] = make_int2(i, j);
                        cl.key[pos] = key[e];
                    }
                    ++pos;
                }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    const int room = cl.cap - cl.n;
    if (tot > room) cl.lost += tot - room;   // only if th = 0 still admitted too many
    cl.n += tot < room ? tot : room;
}

// The block's running minimum key, shared in LDS: after a work item with
// smallest key m, returns min(previous running minimum, m) and records it.
__device__ __forceinline__ uint32_t block_run_min(uint32_t *s_run, uint32_t m) {
    uint32_t old = 0;
    if ((threadIdx.x & 63) == 0) old = atomicMin(s_run, m);
    old = __builtin_amdgcn_readfirstlane(old);
    return old < m ? old : m;
}

// Fold the FP64 r of window pair ij (coarse key kv) into the wavefront's
// best, second-smallest value and counters.
template <typename TX>
__device__ __forceinline__ void take_window_pair(const SweepArgs<TX> &a, double r, int2 ij, uint32_t kv,
                                                 WaveBest &wb) {
    ++wb.nwin;
    wb.nviol += bound_broken(r, (double)__uint_as_float(kv), a.e_abs, a.e_rel);
    if (lex_less(r, ij.x, ij.y, wb.r, wb.i, wb.j)) {
        wb.r2 = wb.r;
        wb.r = r; wb.i = ij.x; wb.j = ij.y;
    } else {
        wb.r2 = fmin(wb.r2, r);
    }
}

// The first candidate at or after g, stepping by four over the four lists
// taken together (lengths n0, n1, n2, then the rest of tot), whose key lies
// in the window T2b: its key and pair, and g at it; false when none is left.
__device__ __forceinline__ bool next_window_entry(int &g, int tot, int n0, int n1, int n2,
                                                  const int2 (*cij)[kCandCap], const uint32_t (*ckey)[kCandCap],
                                                  uint32_t T2b, uint32_t &kv, int2 &ij) {
#pragma unroll 1
    for (; g < tot; g += kPairBlock / kWave) {
        int L = 0, c = g;   // (list, entry) of the g-th candidate (wavefront-uniform)
        if (c >= n0) {
            c -= n0; L = 1;
            if (c >= n1) {
                c -= n1; L = 2;
                if (c >= n2) { c -= n2; L = 3; }
            }
        }
        kv = ckey[L][c];
        ij = cij[L][c];
        if (kv <= T2b) return true;
    }
    return false;
}

// After every wavefront's sweep: the block's final minimum, then the four
// wavefronts share the rescoring of the block's candidates inside its window
// (every fourth entry of the four lists taken together, so that one long
// list does not hold the block back), and the block's result goes to its
// Partial slot.  The block window contains the window of the pass's global
// minimum, so every pair of the latter is rescored.  Every thread of the
// block must call it.
template <int K, typename TX>
__device__ __forceinline__ void finish_pass_block(const SweepArgs<TX> &a, const CandList &cl,
                                                  uint32_t kmin, const uint32_t *s_run, WaveBest &wb,
                                                  const int2 (*cij)[kCandCap], const uint32_t (*ckey)[kCandCap],
                                                  Partial *out) {
    __shared__ int s_cn[kPairBlock / kWave];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (lane == 0) s_cn[wv] = cl.n;
    __syncthreads();   // every list and the block minimum are final
    const uint32_t run = __builtin_amdgcn_readfirstlane(*(const volatile uint32_t *)s_run);
    if (run < 0x7f800000u) {
        const uint32_t T2b = item_window(run, a.wa, a.wb);
        const int n0 = s_cn[0], n1 = s_cn[1], n2 = s_cn[2], n3 = s_cn[3];
        const int tot = n0 + n1 + n2 + n3;
        int g = wv;
        uint32_t k1, k2;
        int2 p1, p2;
        bool paired = false;
        if constexpr (K <= 4) {
            // several component groups (n > 64): the wavefront's window
            // entries two at a time, the second pair's rows in flight with
            // the first's (the order of the folds does not change the result)
            if (a.n > kWave) {
                paired = true;
#pragma unroll 1
                while (next_window_entry(g, tot, n0, n1, n2, cij, ckey, T2b, k1, p1)) {
                    g += kPairBlock / kWave;
                    if (next_window_entry(g, tot, n0, n1, n2, cij, ckey, T2b, k2, p2)) {
                        g += kPairBlock / kWave;
                        double r1, r2;
                        exact_r_wave2<K, TX>(a.X, a.ldx, a.n, a.P64t, p1.x, p1.y, p2.x, p2.y, &r1, &r2);
                        take_window_pair(a, r1, p1, k1, wb);
                        take_window_pair(a, r2, p2, k2, wb);
                    } else {
                        take_window_pair(a, exact_r_wave<K, TX>(a.X, a.ldx, a.n, a.P64t, p1.x, p1.y), p1, k1, wb);
                    }
                }
            }
        }
        if (!paired) {
#pragma unroll 1
            while (next_window_entry(g, tot, n0, n1, n2, cij, ckey, T2b, k1, p1)) {
                g += kPairBlock / kWave;
                double r;
                // one group of components when n <= 64 (no clamped extra
                // loads; K <= 7, where the second instance fits the register
                // budget)
                if (K <= 7 && a.n <= kWave) r = exact_r_wave<K, TX, 1>(a.X, a.ldx, a.n, a.P64t, p1.x, p1.y);
                else r = exact_r_wave<K, TX>(a.X, a.ldx, a.n, a.P64t, p1.x, p1.y);
                take_window_pair(a, r, p1, k1, wb);
            }
        }
    }
    wb.nviol += cl.lost;   // dropped candidates: the result is not certified
    // every lane holds the wavefront's values: the rescoring's r is the same
    // in every lane (exact_r_wave), and the counters, kmin and the limit are
    // wavefront-uniform
    block_reduce_partial(wb.r, wb.i, wb.j, wb.r2, wb.nwin, wb.nunits, wb.nviol, kmin, cl.limit, out, false, true);
}

// Fused pass block pb.  Wavefront w = 4 pb + slot takes work items
// h = w, w + nw, ...: item h covers 4G rows of tile t = h / IPT = (bi, bj)
// (rows 64 bi + 4G (h % IPT) ..) against its 64 columns; G = 8 (a half-tile),
// or 4 for K >= 8.  An item's loads (G weight float4 per lane, the lane's y_j,
// its share of the item's y_i rows) are issued together once the tile's
// coordinates are in, at the end of the previous item; the y_i rows go
// through the wavefront's own LDS slice (read back as broadcasts; no other
// wavefront touches it, so no block barrier).
// Per pair: K subtractions, K FMAs, one multiply, one unsigned min.  Only an
// item whose minimum lies inside the window of the block's running minimum
// is scanned for candidates (emit_cands); they are rescored after the loop
// (finish_pass_block).
template <int K, typename TX>
__device__ void fused_pass_block(const SweepArgs<TX> &a, int pb) {
    __shared__ float4 s_y[kPairBlock / kWave][32 * kMaxK / 4];
    __shared__ int2 s_cij[kPairBlock / kWave][kCandCap];
    __shared__ uint32_t s_ckey[kPairBlock / kWave][kCandCap];
    __shared__ uint32_t s_run;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t nw = (int64_t)a.npass * (kPairBlock / kWave);
    const int kp = a.kp;
    float4 *yl = s_y[wv];
    if (threadIdx.x == 0) s_run = kKeyNone;
    __syncthreads();
    // work item: G groups of 4 rows against the tile's 64 columns (a
    // half-tile; a quarter-tile for K >= 8, which halves the registers the
    // item holds so that the pass keeps four wavefronts per SIMD)
    constexpr int G = K <= 7 ? 8 : 4;
    constexpr int IPT = 16 / G;              // items per tile
    const int64_t nitem = a.nhalf * (8 / G);
    const int nf4 = G * kp;                  // float4 count of the item's 4G rows of Y (<= 128)
    WaveBest wb{__builtin_huge_val(), __builtin_huge_val(), 0x7fffffff, 0x7fffffff, 0, 0, 0};
    CandList cl{s_cij[wv], s_ckey[wv], 0, a.cap, 0, kKeyNone};
    uint32_t kmin = kKeyNone;   // the wavefront's smallest key
    int64_t h = (int64_t)pb * (kPairBlock / kWave) + wv;
    // loads of item h: weights, tile, y_j, two float4 of the y_i rows per lane
    float4 w[G], yr0, yr1;
    float yj[K];
    int2 bt;
    auto fetch = [&](int64_t hh) __attribute__((always_inline)) {
        const int64_t t = hh / IPT;
        const int part = (int)(hh % IPT);
        const float4 *tp = a.invd2 + t * (kTileElems / 4) + part * (G * 64) + lane;
#pragma unroll
        for (int g = 0; g < G; ++g) w[g] = tp[g * 64];
        bt = a.tiles[t];
        const float4 *ysrc =
            reinterpret_cast<const float4 *>(a.Y + ((int64_t)bt.x * kTile + 4 * G * part) * kp);
        yr0 = ysrc[lane < nf4 ? lane : 0];
        yr1 = ysrc[lane + 64 < nf4 ? lane + 64 : 0];
        load_yj<K>(a.Y, kp, (int64_t)bt.y * kTile + lane, yj);
    };
    if (h < nitem) fetch(h);
    for (; h < nitem; h += nw) {
        float4 wc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) wc[g] = w[g];
        float yc[K];
#pragma unroll
        for (int c = 0; c < K; ++c) yc[c] = yj[c];
        const int32_t row0 = bt.x * kTile + 4 * G * (int32_t)(h % IPT), col0 = bt.y * kTile;
        __builtin_amdgcn_wave_barrier();
        if (lane < nf4) yl[lane] = yr0;
        if (lane + 64 < nf4) yl[lane + 64] = yr1;
        __builtin_amdgcn_wave_barrier();
        const float *yi0 = reinterpret_cast<const float *>(yl);
        // the lane's 4G keys (pair (row0 + e, col0 + lane) in key[e]) stay in
        // registers, replacing the weights they consume
        uint32_t key[4 * G];
        uint32_t lmin = kKeyNone;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const float *yi = yi0 + 4 * g * kp;
            key[4 * g] = __float_as_uint(pair_r2<K>(yi, yc, wc[g].x));
            key[4 * g + 1] = __float_as_uint(pair_r2<K>(yi + kp, yc, wc[g].y));
            key[4 * g + 2] = __float_as_uint(pair_r2<K>(yi + 2 * kp, yc, wc[g].z));
            key[4 * g + 3] = __float_as_uint(pair_r2<K>(yi + 3 * kp, yc, wc[g].w));
            lmin = min(lmin, min(min(key[4 * g], key[4 * g + 1]), min(key[4 * g + 2], key[4 * g + 3])));
        }
        const uint32_t m = wave_min_u32_fast(lmin);
        kmin = min(kmin, m);
        // the block window is at most the window of the block's running
        // minimum: a half-tile whose minimum lies outside it has no candidate
        const uint32_t T2 = item_window(block_run_min(&s_run, m), a.wa, a.wb);
        if (m <= T2)
            emit_cands(cl, key, lmin, T2,
                       [=](int e, int32_t &i, int32_t &j) __attribute__((always_inline)) {
                           i = row0 + e;
                           j = col0 + lane;
                       },
                       wb);
        __builtin_amdgcn_wave_barrier();
        if (h + nw < nitem) fetch(h + nw);       // the next item's loads
    }
    finish_pass_block<K, TX>(a, cl, kmin, &s_run, wb, s_cij, s_ckey, a.part + pb);
}

// Plain pass block: one wavefront per 256-pair chunk (grid-stride), the
// same candidate scheme per chunk.
template <int K, typename TX>
__device__ void plain_pass_block(const SweepArgs<TX> &a, int pb) {
    __shared__ int2 s_cij[kPairBlock / kWave][kCandCap];
    __shared__ uint32_t s_ckey[kPairBlock / kWave][kCandCap];
    __shared__ uint32_t s_run;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wid = (int64_t)pb * (kPairBlock / kWave) + wv;
    const int64_t nw = (int64_t)a.npass * (kPairBlock / kWave);
    WaveBest wb{__builtin_huge_val(), __builtin_huge_val(), 0x7fffffff, 0x7fffffff, 0, 0, 0};
    CandList cl{s_cij[wv], s_ckey[wv], 0, a.cap, 0, kKeyNone};
    uint32_t kmin = kKeyNone;   // the wavefront's smallest key
    if (threadIdx.x == 0) s_run = kKeyNone;
    __syncthreads();
    for (int64_t ch = wid; ch < a.nchunks; ch += nw) {
        TX r2[4];
        plain_r2<K, TX>(a.S, a.pcols, a.n, a.Pr, ch * kChunk + lane * 4, r2);
        uint32_t key[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) key[e] = key_of<TX>(r2[e]);
        const uint32_t lmin = min(min(key[0], key[1]), min(key[2], key[3]));
        const uint32_t m = wave_min_u32_fast(lmin);
        kmin = min(kmin, m);
        const uint32_t T2 = item_window(block_run_min(&s_run, m), a.wa, a.wb);
        if (m <= T2)
            emit_cands(cl, key, lmin, T2,
                       [=](int e, int32_t &i, int32_t &j) __attribute__((always_inline)) {
                           int64_t ii, jj;
                           decode_pair(ch * kChunk + lane * 4 + e, a.N, ii, jj);
                           i = (int32_t)ii;
                           j = (int32_t)jj;
                       },
                       wb);
    }
    finish_pass_block<K, TX>(a, cl, kmin, &s_run, wb, s_cij, s_ckey, a.part + pb);
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
    double best = __builtin_huge_val(), second = __builtin_huge_val();
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
                lex_pick2(best, bi, bj, second, r, pi, pj, __builtin_huge_val());
            }
        }
    }
    block_reduce_partial(best, bi, bj, second, cnt, 0, 0, kKeyNone, kKeyNone, a.part + a.npass + sb, false);
}

// Bounds of one short pair's value from the unrounded projection Y64:
// r~ = ||y64_i - y64_j|| / d with |r~ - r| <= s_d2 / d + s_eps r~ (each
// row of Y64 is within delta64 = 4 (n + 2) sqrt(k) u64 R of its exact value,
// s_d2 = 2 delta64; s_eps covers the rounding of the difference, the norm,
// the division and of d itself).
template <int K, typename TX>
__device__ __forceinline__ void short_bounds(const SweepArgs<TX> &a, int64_t e, double &lb, double &ub) {
    const int2 pr = a.close[e];
    const double d = a.cd[e];
    const double *yi = a.Y64 + (int64_t)pr.x * a.kp;
    const double *yj = a.Y64 + (int64_t)pr.y * a.kp;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const double t = yi[c] - yj[c];
        s = __builtin_fma(t, t, s);
    }
    const double rt = sqrt(s) / d;
    const double eb = a.s_d2 / d + a.s_eps * rt;
    lb = rt - eb;
    ub = rt + eb;
}

// (u1 <= u2) <- the two smallest of {u1, u2, v1, v2} (two sorted pairs of
// values of distinct pairs).
__device__ __forceinline__ void min2_merge(double &u1, double &u2, double v1, double v2) {
    const double s = fmin(fmax(u1, v1), fmin(u2, v2));
    u1 = fmin(u1, v1);
    u2 = s;
}

// Short pairs of the iteration from the FP64 Y, then exactly (FP64 GEMM).
// The block takes a contiguous range of the list.  First every pair's
// bounds [r~ - e, r~ + e]; U2 = the second-smallest upper bound, so at least
// two of the block's pairs are worth at most U2.  Then every pair with
// r~ - e <= U2 is evaluated exactly from X, one pair per wavefront step
// (exact_r_wave: a few dependent loads even for long rows, where the
// sixteen-pair matrix-core form walks the row in sixteen).  A pair left out
// is worth more than U2, hence more than the block's two smallest values,
// which are therefore exact FP64 evaluations, as with every pair evaluated
// exactly.
template <int K, typename TX>
__device__ void short_block_y64(const SweepArgs<TX> &a, int sb, int nshort) {
    __shared__ double s_u[kPairBlock / kWave][2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t per = (a.nclose + nshort - 1) / nshort;
    const int64_t e0 = (int64_t)sb * per;
    const int64_t e1 = e0 + per < a.nclose ? e0 + per : a.nclose;
    const double inf = __builtin_huge_val();
    double u1 = inf, u2 = inf;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kPairBlock) {
        double lb, ub;
        short_bounds<K, TX>(a, e, lb, ub);
        min2_merge(u1, u2, ub, inf);
    }
#pragma unroll 1
    for (int o = 32; o > 0; o >>= 1) {
        const double v1 = __shfl_xor(u1, o, kWave), v2 = __shfl_xor(u2, o, kWave);
        min2_merge(u1, u2, v1, v2);
    }
    if (lane == 0) { s_u[wv][0] = u1; s_u[wv][1] = u2; }
    __syncthreads();
    double U1 = s_u[0][0], U2 = s_u[0][1];
#pragma unroll
    for (int w = 1; w < kPairBlock / kWave; ++w) min2_merge(U1, U2, s_u[w][0], s_u[w][1]);
    double best = inf, second = inf;
    int32_t bi = 0x7fffffff, bj = 0x7fffffff, cnt = 0;
    for (int64_t c0 = e0 + (int64_t)wv * kWave; c0 < e1; c0 += kPairBlock) {
        const int64_t e = c0 + lane;
        bool cand = false;
        if (e < e1) {
            double lb, ub;
            short_bounds<K, TX>(a, e, lb, ub);
            cand = !(lb > U2);
        }
        uint64_t mask = __ballot(cand);
#pragma unroll 1
        while (mask) {
            const int64_t ee = c0 + __builtin_ctzll(mask);
            mask &= mask - 1;
            const int2 pr = a.close[ee];
            double r;
            if (K <= 7 && a.n <= kWave) r = exact_r_wave<K, TX, 1>(a.X, a.ldx, a.n, a.P64t, pr.x, pr.y);
            else r = exact_r_wave<K, TX>(a.X, a.ldx, a.n, a.P64t, pr.x, pr.y);
            ++cnt;
            lex_pick2(best, bi, bj, second, r, pr.x, pr.y, inf);
        }
    }
    block_reduce_partial(best, bi, bj, second, lane == 0 ? cnt : 0, 0, 0, kKeyNone, kKeyNone,
                         a.part + a.npass + sb, false);
}

// One step of the selection's loads: partials base + u * 256 + thread,
// u = 0..7, unconditional (clamped index, nparts >= 1): a guarded load would
// wait alone, and so would one whose registers are overwritten past the end.
template <typename TX>
__device__ __forceinline__ void select_load(const SweepArgs<TX> &a, int nparts, int base, Partial (&p)[8]) {
#pragma unroll
    for (int u = 0; u < 8; ++u) p[u] = a.part[min(base + u * kPairBlock + (int)threadIdx.x, nparts - 1)];
}

// Selection (one block, after the pass): the lexicographic minimum of every
// pass block's and short-pair block's FP64 result, the record, and the
// coarse minimum with its window (reported).  Eight partials per thread are
// loaded per step, all before any is used (each step is a round trip to
// memory written by other dies' caches).  The caller issues the first
// step's loads (select_load, base 0) and passes them in p, so that loads it
// issues next queue behind them.  Returns the winning pair in every thread
// (i < 0 if there is none).
//
// Certified: no rescored pair broke the coarse bound, no candidate was lost,
// and every block's candidate-key limit lies at or above the window of the
// global coarse minimum.  The runner-up: every pair left unevaluated in FP64
// has a coarse value above that window (or above its block's limit), hence a
// true value above r_lo = (sqrt(min(window, limit)) - e_abs) / (1 + e_rel);
// the reported runner_up is min(second-smallest evaluated value, r_lo), a
// lower bound of the true runner-up, exact when the evaluated value is the
// smaller.
template <int K, typename TX, bool FUSED>
__device__ int2 select_min(const SweepArgs<TX> &a, int nparts, bool record, Partial (&p)[8]) {
    double best = __builtin_huge_val(), second = __builtin_huge_val();
    int32_t bi = 0x7fffffff, bj = 0x7fffffff, nres = 0, nunits = 0, nviol = 0;
    uint32_t kmin = kKeyNone, limit = kKeyNone;
    // a clamped duplicate of the last partial (select_load) is the same
    // element to the top-2 merge and the minima; only its counts are masked
    auto merge_step = [&](int base) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool in = base + u * kPairBlock + (int)threadIdx.x < nparts;
            lex_pick2(best, bi, bj, second, p[u].r, p[u].i, p[u].j, p[u].r2);
            nres += in ? p[u].n_rescored : 0;
            nunits += in ? p[u].n_units : 0;
            nviol += in ? p[u].n_viol : 0;
            kmin = min(kmin, p[u].kmin);
            limit = min(limit, p[u].limit);
        }
    };
    merge_step(0);
#pragma unroll 1
    for (int base = 8 * kPairBlock; base < nparts; base += 8 * kPairBlock) {
        select_load(a, nparts, base, p);
        merge_step(base);
    }
    const Partial f = block_reduce_partial(best, bi, bj, second, nres, nunits, nviol, kmin, limit, nullptr, false);
    if (record && threadIdx.x == 0) {
        double coarse, tr;
        (void)window_key(f.kmin, a.e_abs, a.e_rel, &coarse, &tr);
        const bool found = f.r < __builtin_huge_val();
        const uint32_t wkey = f.kmin < 0x7f800000u ? item_window(f.kmin, a.wa, a.wb) : 0u;
        const int cert = (found && f.n_viol == 0 && f.limit >= wkey) ? 1 : 0;
        // lower bound of every unevaluated pair's true value
        double r_lo = __builtin_huge_val();
        if (coarse >= 0.0) {
            double t = tr;
            if (f.limit != kKeyNone) t = fmin(t, sqrt((double)__uint_as_float(f.limit)));
            r_lo = (t - a.e_abs) / (1.0 + a.e_rel) * (1.0 - 1e-9);
        }
        const double ru = fmin(f.r2, r_lo);
        DevResult *res = a.res;
        res->min_norm = f.r;
        res->runner_up = ru;
        res->runner_up_exact = (cert && f.r2 <= r_lo) ? 1 : 0;
        res->i = found ? f.i : -1;
        res->j = found ? f.j : -1;
        res->q = found ? pair_index(a.N, f.i, f.j) : -1;
        res->coarse_min = coarse;
        res->window = coarse >= 0.0 ? tr - coarse : 0.0;
        res->certified = cert;
        res->n_rescored = f.n_rescored;
        res->n_tiles = f.n_units;
        res->t = -1;
        if (a.tr_min) a.tr_min[a.it] = f.r;
        if (a.tr_ij) {
            a.tr_ij[2 * a.it] = found ? f.i : -1;
            a.tr_ij[2 * a.it + 1] = found ? f.j : -1;
        }
        if (a.tr_cert) a.tr_cert[a.it] = cert;
        *a.gmin_out = f.kmin;
    }
    return f.r < __builtin_huge_val() ? make_int2(f.i, f.j) : make_int2(-1, -1);
}

// The pass.  Fused form: the first nshort blocks score the short pairs in
// FP64 (they need only P, and start first so that they run beside the
// coarse blocks), the other npass blocks score every pair coarsely.  Every
// block writes its own result slot; the kernel boundary is the grid-wide
// barrier before selection.
// Occupancy: four wavefronts per SIMD (128 registers); three (168) for the
// plain form over FP64 data with K > 12, which would spill at 128.
template <int K, typename TX, bool FUSED>
__global__ __launch_bounds__(kPairBlock, (FUSED || sizeof(TX) == 4 || K <= 12) ? 4 : 3) void k_pass(SweepArgs<TX> a, int nshort) {
    if constexpr (FUSED) {
        if ((int)blockIdx.x < nshort) {
            if (a.Y64) short_block_y64<K, TX>(a, (int)blockIdx.x, nshort);
            else short_block<K, TX>(a, (int)blockIdx.x, nshort);
            return;
        }
    }
    const int pb = (int)blockIdx.x - (FUSED ? nshort : 0);
    if constexpr (FUSED) fused_pass_block<K, TX>(a, pb);
    else plain_pass_block<K, TX>(a, pb);
}

// The K x n FP64 P into LDS, eight loads in flight per thread before any
// is stored.
__device__ __forceinline__ void stage_P(const double *__restrict__ P, int kn, double *sm) {
#pragma unroll 1
    for (int e0 = threadIdx.x; e0 < kn; e0 += 8 * kPairBlock) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kPairBlock;
            t[u] = e < kn ? P[e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kPairBlock;
            if (e < kn) sm[e] = t[u];
        }
    }
}

// Fused form, before the pass: Y = (X - mu) P.
template <int K, typename TX>
__global__ __launch_bounds__(kPairBlock) void k_prep(SweepArgs<TX> a, const double *__restrict__ mu,
                                                     float *__restrict__ Y, int64_t Npad) {
    if (a.split) {
        // the split GEMM of k_selprep (the same tiles and order of sums):
        // P, the means and the exchange slots in LDS
        extern __shared__ __align__(16) double sm_pp[];
        int64_t row0;
        int cb, nch;
        deep_tile(true, a.n, row0, cb, nch);
        TX x0[16];
        double m0[16];
        gemm_first_x<TX>(a.X, a.ldx, a.N, row0, 64 * cb, true, a.invd2, mu, x0, m0);
        stage_P(a.P64t, K * a.n, sm_pp);
        double *mu_l = sm_pp + (size_t)K * a.n;
        for (int e = threadIdx.x; e < a.n; e += kPairBlock) mu_l[e] = mu[e];
        __syncthreads();
        gemm_block_deep<TX>(a.X, a.ldx, a.N, a.n, K, mu_l, sm_pp, Y, a.Y64, a.kp, Npad, x0, true, mu_l + a.n);
        return;
    }
    const TX nx[16] = {};
    const double none[16] = {};
    gemm_block<TX>(a.X, a.ldx, a.N, a.n, K, mu, a.P64t, Y, a.Y64, a.kp, Npad, a.vx, a.vp, nx, none, false,
                   a.gemm);
}

// ------------------------------------------------------------------ the update

// The modified Gram-Schmidt step of the update on coordinates in the basis
// P: the columns are c (v = P c) and e_q for q = 0..k-1 without t (the kept
// columns p_q = P e_q), in that order; since P has orthonormal columns,
// every inner product, hence every coefficient, equals that of the vectors
// themselves, and the orthonormalised vectors are P G[j].  vnorm = |c| =
// |v|.  Uniform: every lane computes the same K x K values.
template <int K>
__device__ __forceinline__ void coord_mgs(const double (&c)[K], int t, double (&G)[K][K], double &vnorm) {
#pragma unroll
    for (int jv = 0; jv < K; ++jv)
#pragma unroll
        for (int r = 0; r < K; ++r)
            G[jv][r] = jv == 0 ? c[r] : (r == (jv <= t ? jv - 1 : jv) ? 1.0 : 0.0);
#pragma unroll
    for (int mm = 0; mm < K; ++mm) {
        double nn = 0.0;
#pragma unroll
        for (int r = 0; r < K; ++r) nn = __builtin_fma(G[mm][r], G[mm][r], nn);
        const double nrm = sqrt(nn);
        if (mm == 0) vnorm = nrm;
        const double rn = 1.0 / nrm;
#pragma unroll
        for (int r = 0; r < K; ++r) G[mm][r] = G[mm][r] * rn;
#pragma unroll
        for (int jv = mm + 1; jv < K; ++jv) {
            double d = 0.0;
#pragma unroll
            for (int r = 0; r < K; ++r) d = __builtin_fma(G[mm][r], G[jv][r], d);
#pragma unroll
            for (int r = 0; r < K; ++r) G[jv][r] = G[jv][r] - d * G[mm][r];
        }
    }
}

// v[0..NV-1] summed over the block, the same bits in every thread:
// transposed wavefront sums, then the wavefronts' sums added in a fixed
// order.  Every thread of the block must call it.  red holds two
// alternating buffers (ph selects one and flips): a wavefront can rewrite a
// buffer only after the next call's barrier, which every wavefront reaches
// after reading it, so one barrier per call suffices.
template <int NV>
__device__ __forceinline__ void block_sum_many(double (&v)[NV], double (*red)[kPairBlock / kWave][16], int &ph) {
    const double t = wave_sum_transposed<NV>(v);
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    if (lane < NV) red[ph][w][lane] = t;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < NV; ++e) v[e] = (red[ph][0][e] + red[ph][1][e]) + (red[ph][2][e] + red[ph][3][e]);
    ph ^= 1;
}
__device__ __forceinline__ double block_sum(double x, double (*red)[kPairBlock / kWave][16], int &ph) {
    double v[1] = {x};
    block_sum_many<1>(v, red, ph);
    return v[0];
}

// The whole block: the paper's update of P in FP64, from the recorded pair:
//   c = P^T s;  t = first argmax |c_t|;
//   if c = 0:   P' = [s, p_2, .., p_k]
//   else:       v = P c; modified Gram-Schmidt on (v, p_1..p_k without p_t);
//               u = unit((1-a) v + a (s - v))   [rule 1: unit vectors of v, s-v]
//               P' = [u, q_2, .., q_k]
// The vectors live in LDS (A: K x n, then s, v); thread x owns components
// x, x+256, ... of every vector and is the only one to touch them, so the
// vectors need no barriers; every inner product is a block sum.  For K <= 12
// the Gram-Schmidt step runs on coordinates in the basis P (coord_mgs): no
// block sum, and the new vectors are P G.  For larger K it runs on the
// vectors, right-looking: once q_m is final, every later vector loses its
// component along q_m (per vector, the same sequence of subtractions as the
// column-by-column form), and the independent inner products of one step
// (the projections of all later vectors on q_m) are reduced together, so a
// step waits on two reductions (|a_m| and the batch).  Every thread of the
// block must call this.
template <int K, typename TX>
__device__ __forceinline__ void apply_update(const TX *__restrict__ X, int64_t ldx, int n,
                             double *__restrict__ P64t, void *__restrict__ Pr, int pr_kind,
                             double alpha, int rule, DevResult *__restrict__ res, int64_t i, int64_t j,
                             double *sm) {
    __shared__ double red[2][kPairBlock / kWave][16];
    int ph = 0;
    const int tid = threadIdx.x;
    double *A = sm;                       // K x n: P (loaded by the caller), then MGS vectors
    double *s = sm + (size_t)K * n;       // unit secant, later u
    double *v = s + n;                    // P P^T s
    double d2 = 0.0;
    for (int l = tid; l < n; l += kPairBlock) {
        const double dl = (double)X[i * ldx + l] - (double)X[j * ldx + l];
        s[l] = dl;
        d2 = __builtin_fma(dl, dl, d2);
    }
    const double d = sqrt(block_sum(d2, red, ph));
    // c = P^T s, t = first argmax |c_t| (every thread holds the same sums)
    double c[K];
#pragma unroll
    for (int q = 0; q < K; ++q) c[q] = 0.0;
    for (int l = tid; l < n; l += kPairBlock) {
        const double sl = s[l] / d;
        s[l] = sl;
#pragma unroll
        for (int q = 0; q < K; ++q) c[q] = __builtin_fma(A[(size_t)q * n + l], sl, c[q]);
    }
    block_sum_many<K>(c, red, ph);
    int t = 0;
    double cmax = -1.0;
#pragma unroll
    for (int q = 0; q < K; ++q)
        if (fabs(c[q]) > cmax) { cmax = fabs(c[q]); t = q; }
    if (res && tid == 0) res->t = t;

    if (cmax == 0.0) {
        for (int l = tid; l < n; l += kPairBlock) A[l] = s[l];
    } else {
        double vnorm = 0.0;
        if constexpr (K <= 12) {
            // v = P c; the Gram-Schmidt step on coordinates in the basis P
            // (as in apply_update_reg, the K x K coordinates the same in
            // every thread), then q_2..q_k = P G[1..k-1] in place
            for (int l = tid; l < n; l += kPairBlock) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < K; ++q) acc = __builtin_fma(A[(size_t)q * n + l], c[q], acc);
                v[l] = acc;
            }
            double G[K][K];
            coord_mgs<K>(c, t, G, vnorm);
            for (int l = tid; l < n; l += kPairBlock) {
                double x[K];   // every row read before any is written back
#pragma unroll
                for (int q = 0; q < K; ++q) x[q] = A[(size_t)q * n + l];
#pragma unroll
                for (int jv = 1; jv < K; ++jv) {
                    double acc = 0.0;
#pragma unroll
                    for (int q = 0; q < K; ++q) acc = __builtin_fma(x[q], G[jv][q], acc);
                    A[(size_t)jv * n + l] = acc;
                }
            }
        } else {
            // v = P c; MGS input order (v, p_1..p_{t-1}, p_{t+1}..p_k), in place
            for (int l = tid; l < n; l += kPairBlock) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < K; ++q) acc = __builtin_fma(A[(size_t)q * n + l], c[q], acc);
                v[l] = acc;
                for (int m = t; m > 0; --m) A[(size_t)m * n + l] = A[(size_t)(m - 1) * n + l];
                A[l] = acc;
            }
#pragma unroll 1
            for (int m = 0; m < K; ++m) {
                double *am = A + (size_t)m * n;
                double nn = 0.0;
                for (int l = tid; l < n; l += kPairBlock) nn = __builtin_fma(am[l], am[l], nn);
                const double nrm = sqrt(block_sum(nn, red, ph));
                if (m == 0) vnorm = nrm;
                if (m + 1 == K) {
                    for (int l = tid; l < n; l += kPairBlock) am[l] = am[l] / nrm;
                    break;
                }
                // every row's inner product with q_m, without branches (rows
                // up to m are final: their products go unused and the select
                // below rewrites them unchanged)
                double dots[K];
#pragma unroll
                for (int jv = 0; jv < K; ++jv) dots[jv] = 0.0;
                for (int l = tid; l < n; l += kPairBlock) {
                    const double q = am[l] / nrm;
                    am[l] = q;
#pragma unroll
                    for (int jv = 0; jv < K; ++jv) dots[jv] = __builtin_fma(q, A[(size_t)jv * n + l], dots[jv]);
                }
                block_sum_many<K>(dots, red, ph);
                for (int l = tid; l < n; l += kPairBlock) {
                    const double q = am[l];
                    double x[K];   // every row read before any is written back
#pragma unroll
                    for (int jv = 0; jv < K; ++jv) x[jv] = A[(size_t)jv * n + l];
#pragma unroll
                    for (int jv = 0; jv < K; ++jv) A[(size_t)jv * n + l] = jv > m ? x[jv] - dots[jv] * q : x[jv];
                }
            }
        }
        // the alpha shift toward the worst secant
        double wn = 1.0;
        if (rule == SAP_STEP_NORMALIZED) {
            double acc = 0.0;
            for (int l = tid; l < n; l += kPairBlock) {
                const double w = s[l] - v[l];
                acc = __builtin_fma(w, w, acc);
            }
            wn = sqrt(block_sum(acc, red, ph));
        }
        double un = 0.0;
        for (int l = tid; l < n; l += kPairBlock) {
            double u;
            if (rule == SAP_STEP_NORMALIZED)
                u = (1.0 - alpha) * (v[l] / vnorm) + (wn > 0.0 ? alpha * ((s[l] - v[l]) / wn) : 0.0);
            else
                u = (1.0 - alpha) * v[l] + alpha * (s[l] - v[l]);
            s[l] = u;
            un = __builtin_fma(u, u, un);
        }
        const double unrm = sqrt(block_sum(un, red, ph));
        for (int l = tid; l < n; l += kPairBlock) A[l] = s[l] / unrm;
    }
    // write back (each output optional; A itself holds the result): master
    // (K x n) and the plain pass's copy
    if (P64t || pr_kind) {
        for (int l = tid; l < n; l += kPairBlock) {
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const double pv = A[(size_t)q * n + l];
                if (P64t) P64t[(int64_t)q * n + l] = pv;
                if (pr_kind == 1) static_cast<float *>(Pr)[(int64_t)l * K + q] = (float)pv;
                else if (pr_kind == 2) static_cast<double *>(Pr)[(int64_t)l * K + q] = pv;
            }
        }
    }
}

// The same update with the vectors in registers, for n <= 64 M (lane l owns
// components l + 64 m) and small K M: the secant, c = P^T s, v and u as in
// apply_update but without LDS round trips, and the Gram-Schmidt step on
// coordinates in the basis P (see below), so that a step takes four
// wavefront reductions instead of 2K + 4.
template <int K, int M, typename TX>
__device__ __forceinline__ void apply_update_reg(const TX *__restrict__ X, int64_t ldx, int n, double *Pl,
                                 double *__restrict__ P64t, void *__restrict__ Pr, int pr_kind,
                                 double alpha, int rule, DevResult *__restrict__ res, int64_t i,
                                 int64_t j, bool to_lds) {
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
    if (res && lane == 0) res->t = t;
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
        // MGS of (v, p_1..p_{t-1}, p_{t+1}..p_k) on coordinates in the basis
        // P (coord_mgs): no wavefront reduction, and the new vectors are P G
        double G[K][K];
        double vnorm = 0.0;
        coord_mgs<K>(c, t, G, vnorm);
        // q_2..q_k = P G[1..k-1] (q_1, v's direction, gives way to u below)
        double Q[K][M];
#pragma unroll
        for (int jv = 1; jv < K; ++jv)
#pragma unroll
            for (int m = 0; m < M; ++m) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < K; ++q) acc = __builtin_fma(A[q][m], G[jv][q], acc);
                Q[jv][m] = acc;
            }
#pragma unroll
        for (int jv = 1; jv < K; ++jv)
#pragma unroll
            for (int m = 0; m < M; ++m) A[jv][m] = Q[jv][m];
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
    // outputs, each optional: master (K x n), the plain pass's copy, and
    // (to_lds) the K x n copy in LDS the update started from
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int l = lane + 64 * m;
        if (l < n) {
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const double pv = A[q][m];
                if (P64t) P64t[(int64_t)q * n + l] = pv;
                if (pr_kind == 1) static_cast<float *>(Pr)[(int64_t)l * K + q] = (float)pv;
                else if (pr_kind == 2) static_cast<double *>(Pr)[(int64_t)l * K + q] = pv;
                if (to_lds) Pl[q * n + l] = pv;
            }
        }
    }
}


// Selection, record and (do_step) update, in one block.  Dynamic LDS holds
// P (read by the rescoring, then the update's working copy) and the update's
// vectors: (K + 2) n doubles.
template <int K, typename TX, bool FUSED>
__global__ __launch_bounds__(kPairBlock) void k_select(SweepArgs<TX> a, int nshort,
                                                       double *__restrict__ P64t,
                                                       void *__restrict__ Pr, int pr_kind,
                                                       double alpha, int rule, int do_step) {
    extern __shared__ double sm_dyn[];
    // P into LDS now, so that its loads overlap the selection (the block
    // barriers inside select_min order these writes before the update)
    if (do_step) stage_P(a.P64t, K * a.n, sm_dyn);
    Partial p[8];
    select_load(a, a.npass + nshort, 0, p);
    const int2 ij = select_min<K, TX, FUSED>(a, a.npass + nshort, true, p);
    if (do_step && ij.x >= 0) {
        // one wavefront with the vectors in registers when every vector
        // fits one 64-lane slice and K is small, the whole block over LDS
        // otherwise
        if (K <= 8 && a.n <= 64) {
            if (threadIdx.x < kWave)
                apply_update_reg<K, 1, TX>(a.X, a.ldx, a.n, sm_dyn, P64t, Pr, pr_kind, alpha, rule,
                                           a.res, ij.x, ij.y, false);
        } else {
            apply_update<K, TX>(a.X, a.ldx, a.n, P64t, Pr, pr_kind, alpha, rule, a.res, ij.x,
                                ij.y, sm_dyn);
        }
    }
}

// Fused form inside a run: this iteration's selection and update (as
// k_select) followed by the next iteration's Y = (X - mu) P' (as k_prep), in
// every block of the GEMM's grid, so the run needs two launches per
// iteration.  Every block takes the same selection and computes the same P'
// (identical inputs, identical arithmetic) into its LDS, then its rows of Y
// from there.  Block 0 alone writes the record, the traces and P' to Pn, the
// other P buffer: blocks still reading the current P must not see P'.
template <int K, typename TX, int TPW>
__global__ __launch_bounds__(kPairBlock) void k_selprep(SweepArgs<TX> a, int nshort, double *__restrict__ Pn,
                                                        double alpha, int rule, const double *__restrict__ mu,
                                                        float *__restrict__ Y, int64_t Npad) {
    extern __shared__ __align__(16) double sm_sp[];
    const bool lead = blockIdx.x == 0;
    // small P (into registers, then to LDS after the selection, before the
    // barrier the update starts behind), the GEMM's first chunk of X and the
    // means are loaded right behind the selection's first loads: the
    // selection waits for its own loads only, and these land meanwhile
    const int kn = K * a.n;
    const bool small = kn <= 8 * kPairBlock;
    // the GEMM: four chunks deep with the means in LDS (FP64, 512 or 768 or
    // 1024 components, 16-byte X rows), else gemm_block; either takes its
    // first chunk prefetched here when X rows take 16-byte loads
    const bool pre_x = a.n >= 64 && a.vx;
    const bool deep = pre_x && a.gemm == SAP_GEMM_F64 && a.n >= 512 && a.n <= 4 * kPairBlock && a.n % 256 == 0;
    double *mu_l = sm_sp + (size_t)(K + 2) * a.n;   // past P and the update's two vectors
    TX x0[16];
    double m0[16], pre[8], mpre[4];
    Partial p[8];
    select_load(a, a.npass + nshort, 0, p);
    if (!small) stage_P(a.P64t, kn, sm_sp);
    // the wavefront's first chunk of X and the matching means, issued
    // unconditionally (the 1/d^2 tiles serve as the spare source)
    const bool split = deep && a.split;
    const int tpw = deep ? 1 : TPW;
    int64_t row0 = min(((int64_t)blockIdx.x * tpw * 4 + (threadIdx.x >> 6)) * 16, Npad - 16);
    int l0 = 0;
    if (deep) {
        int cb, nch;
        deep_tile(split, a.n, row0, cb, nch);
        l0 = 64 * cb;
    }
    gemm_first_x<TX>(a.X, a.ldx, a.N, row0, l0, pre_x, a.invd2, mu, x0, m0);
#pragma unroll
    for (int u = 0; u < 8; ++u) pre[u] = a.P64t[min((int)threadIdx.x + u * kPairBlock, kn - 1)];
#pragma unroll
    for (int u = 0; u < 4; ++u) mpre[u] = mu[min((int)threadIdx.x + u * kPairBlock, a.n - 1)];
    const int2 ij = select_min<K, TX, true>(a, a.npass + nshort, lead, p);
    if (small) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = (int)threadIdx.x + u * kPairBlock;
            if (e < kn) sm_sp[e] = pre[u];
        }
    }
    if (deep) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = (int)threadIdx.x + u * kPairBlock;
            if (e < a.n) mu_l[e] = mpre[u];
        }
    }
    if (small || deep) __syncthreads();
    if (ij.x >= 0) {
        if (K <= 8 && a.n <= 64) {
            if (threadIdx.x < kWave)
                apply_update_reg<K, 1, TX>(a.X, a.ldx, a.n, sm_sp, lead ? Pn : nullptr, nullptr, 0, alpha,
                                           rule, lead ? a.res : nullptr, ij.x, ij.y, true);
        } else {
            apply_update<K, TX>(a.X, a.ldx, a.n, lead ? Pn : nullptr, nullptr, 0, alpha, rule,
                                lead ? a.res : nullptr, ij.x, ij.y, sm_sp);
        }
    } else if (lead) {
        for (int e = threadIdx.x; e < K * a.n; e += kPairBlock) Pn[e] = sm_sp[e];   // P unchanged
    }
    __syncthreads();
    if (deep) {
        // (the update's vector s, past P, holds the split's exchange slots)
        gemm_block_deep<TX>(a.X, a.ldx, a.N, a.n, K, mu_l, sm_sp, Y, a.Y64, a.kp, Npad, x0, split,
                            sm_sp + (size_t)K * a.n);
        return;
    }
    // X rows without 16-byte loads: the first chunk is loaded now (scalar)
    if (a.n >= 64 && !pre_x) gemm_first_x_scalar<TX>(a.X, a.ldx, a.N, Npad, mu, x0, m0);
    gemm_block<TX>(a.X, a.ldx, a.N, a.n, K, mu, sm_sp, Y, a.Y64, a.kp, Npad, a.vx, (a.n & 1) == 0, x0, m0,
                   a.n >= 64, a.gemm, tpw, 0);
    // TPW = 2: a second group of 64 rows (more 64-row groups than compute
    // units: one round of blocks, each taking the selection and update once
    // for both)
    if constexpr (TPW == 2)
        gemm_block<TX>(a.X, a.ldx, a.N, a.n, K, mu, sm_sp, Y, a.Y64, a.kp, Npad, a.vx, (a.n & 1) == 0, x0, m0,
                       false, a.gemm, tpw, 1);
}

#ifndef SAP_KINST   // K-independent kernels: compiled once, in the host runtime unit
// ------------------------------------------------------------------ small helpers

// The plain pass's n x k row-major copy of P in X's dtype, from the master.
template <typename T>
__global__ void k_write_Pr(const double *__restrict__ P64t, int n, int k, T *__restrict__ Pr) {
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

#endif  // SAP_KINST

}  // namespace sap
