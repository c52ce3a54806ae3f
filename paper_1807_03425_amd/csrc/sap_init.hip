// One-time precomputation kernels of a SAP handle (gfx950).
//
//  * column means and the radius max_i ||x_i - mean|| (the error bound of the
//    fused pass is stated in terms of this radius);
//  * plain form: every unit secant s = (x_i - x_j)/||x_i - x_j|| stored once,
//    component-major (n x p), which is the paper's secant matrix S with the
//    secants as columns (Sec. 4);
//  * fused form: 1/d_ij^2 for every pair by direct differences in FP64,
//    packed by 64 x 64 tile, plus the list of short pairs that the coarse
//    FP32 pass cannot resolve and that are therefore evaluated in FP64.
// Pairs that the method drops (duplicates; secants shorter than the length
// threshold of Sec. 7) are masked in both forms.
#include "sap_common.h"

namespace sap {

// ---------------------------------------------------------------- moments

// Block b sums rows [b*rows, (b+1)*rows) of every column, in row order.
__global__ __launch_bounds__(256) void k_col_partial(const void *X, int dtype, int64_t ldx,
                                                     int64_t N, int n, int64_t rows,
                                                     double *part, int32_t *nonfinite) {
    const int64_t r0 = (int64_t)blockIdx.x * rows;
    const int64_t r1 = r0 + rows < N ? r0 + rows : N;
    int bad = 0;
    for (int l = threadIdx.x; l < n; l += blockDim.x) {
        double acc = 0.0;
        for (int64_t i = r0; i < r1; ++i) {
            double v = load_x(X, dtype, i * ldx + l);
            if (!isfinite(v)) bad = 1;
            acc += v;
        }
        part[(int64_t)blockIdx.x * n + l] = acc;
    }
    if (bad) atomicOr(nonfinite, 1);
}

__global__ __launch_bounds__(256) void k_col_mean(const double *part, int64_t nblk, int n,
                                                  int64_t N, double *mu) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    double acc = 0.0;
    for (int64_t b = 0; b < nblk; ++b) acc += part[b * n + l];
    mu[l] = acc / (double)N;
}

// One wavefront per row: ||x_i - mu||, folded into a max on the FP64 bits
// (non-negative doubles order like their bit patterns).
__global__ __launch_bounds__(256) void k_radius(const void *X, int dtype, int64_t ldx,
                                                int64_t N, int n, const double *mu,
                                                unsigned long long *rbits) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= N) return;
    double acc = 0.0;
    for (int l = lane; l < n; l += kWave) {
        double t = load_x(X, dtype, row * ldx + l) - mu[l];
        acc += t * t;
    }
    acc = wave_sum(acc);
    if (lane == 0) atomicMax(rbits, (unsigned long long)__double_as_longlong(sqrt(acc)));
}

// ---------------------------------------------------------------- plain form

// S[l * pcols + q] = component l of the unit secant of pair q (computed in
// FP64, stored in T).  Dropped pairs and the padding q >= p hold NaN.
template <typename T>
__global__ __launch_bounds__(256) void k_build_secants(const void *X, int dtype, int64_t ldx,
                                                       int64_t N, int n, double min_len,
                                                       T *S, int64_t pcols, int64_t p,
                                                       unsigned long long *kept,
                                                       unsigned long long *dropped) {
    __shared__ unsigned long long s_kept, s_drop;
    if (threadIdx.x == 0) { s_kept = 0; s_drop = 0; }
    __syncthreads();
    const T nanv = (T)__builtin_nan("");
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < pcols;
         q += (int64_t)gridDim.x * blockDim.x) {
        if (q >= p) {
            for (int l = 0; l < n; ++l) S[(int64_t)l * pcols + q] = nanv;
            continue;
        }
        int64_t i, j;
        decode_pair(q, N, i, j);
        double d2 = 0.0;
        for (int l = 0; l < n; ++l) {
            double t = load_x(X, dtype, i * ldx + l) - load_x(X, dtype, j * ldx + l);
            d2 += t * t;
        }
        double d = sqrt(d2);
        if (d == 0.0 || d < min_len) {
            for (int l = 0; l < n; ++l) S[(int64_t)l * pcols + q] = nanv;
            atomicAdd(&s_drop, 1ull);
            continue;
        }
        for (int l = 0; l < n; ++l) {
            double t = load_x(X, dtype, i * ldx + l) - load_x(X, dtype, j * ldx + l);
            S[(int64_t)l * pcols + q] = (T)(t / d);
        }
        atomicAdd(&s_kept, 1ull);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_kept) atomicAdd(kept, s_kept);
        if (s_drop) atomicAdd(dropped, s_drop);
    }
}

template __global__ void k_build_secants<float>(const void *, int, int64_t, int64_t, int,
                                                double, float *, int64_t, int64_t,
                                                unsigned long long *, unsigned long long *);
template __global__ void k_build_secants<double>(const void *, int, int64_t, int64_t, int,
                                                 double, double *, int64_t, int64_t,
                                                 unsigned long long *, unsigned long long *);

// ---------------------------------------------------------------- fused form

// Tile t = (bi, bj), bi <= bj, holds the 64 x 64 pairs
// (i = 64 bi + r, j = 64 bj + c) at float index (r/4)*256 + c*4 + r%4, i.e.
// a lane that owns column c reads rows 4g..4g+3 as one float4 at float4
// index 64 g + c: a wavefront load of 64 consecutive float4 (1 KiB).
//
// ladder[m] = (float)(1 / D_m^2), D_m = D_target * 2^(-m/4), increasing in m.
// A kept pair is counted in bin m when ladder[m] < invd2 <= ladder[m+1]
// (bin 63 takes everything above ladder[63]); the same FP32 comparison later
// decides membership of the close list, so the counts are exact.
__global__ __launch_bounds__(256) void k_build_invd2(const void *X, int dtype, int64_t ldx,
                                                     int64_t N, int n, const int2 *tiles,
                                                     int64_t ntiles, double min_len,
                                                     float4 *invd2, const float *ladder,
                                                     unsigned long long *hist,
                                                     unsigned long long *kept,
                                                     unsigned long long *dropped) {
    __shared__ unsigned long long s_hist[64];
    __shared__ unsigned long long s_kept, s_drop;
    __shared__ float s_ladder[64];
    if (threadIdx.x < 64) { s_hist[threadIdx.x] = 0; s_ladder[threadIdx.x] = ladder[threadIdx.x]; }
    if (threadIdx.x == 0) { s_kept = 0; s_drop = 0; }
    __syncthreads();
    const int c = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int2 b = tiles[t];
        const int64_t j = (int64_t)b.y * kTile + c;
        const bool jin = j < N;
        for (int m = 0; m < 4; ++m) {
            const int g = w + 4 * m;   // uniform within the wavefront
            const int64_t i0 = (int64_t)b.x * kTile + 4 * g;
            double d2[4] = {0.0, 0.0, 0.0, 0.0};
            if (jin) {
                for (int l = 0; l < n; ++l) {
                    const double xj = load_x(X, dtype, j * ldx + l);
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int64_t i = i0 + rr < N ? i0 + rr : N - 1;
                        const double t2 = load_x(X, dtype, i * ldx + l) - xj;
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
                    if (d == 0.0 || d < min_len) {
                        atomicAdd(&s_drop, 1ull);
                    } else {
                        v = (float)(1.0 / d2[rr]);
                        atomicAdd(&s_kept, 1ull);
                        if (v > s_ladder[0]) {
                            int lo = 0;  // largest m with ladder[m] < v
                            for (int hi = 63; lo < hi;) {
                                int mid = (lo + hi + 1) >> 1;
                                if (s_ladder[mid] < v) lo = mid; else hi = mid - 1;
                            }
                            atomicAdd(&s_hist[lo], 1ull);
                        }
                    }
                }
                out[rr] = v;
            }
            invd2[t * (kTileElems / 4) + g * 64 + c] = make_float4(out[0], out[1], out[2], out[3]);
        }
    }
    __syncthreads();
    if (threadIdx.x < 64 && s_hist[threadIdx.x]) atomicAdd(&hist[threadIdx.x], s_hist[threadIdx.x]);
    if (threadIdx.x == 0) {
        if (s_kept) atomicAdd(kept, s_kept);
        if (s_drop) atomicAdd(dropped, s_drop);
    }
}

// Pairs with 1/d^2 above thr become close pairs: masked in the tile array
// and appended (in no particular order; the host sorts the list) to `list`.
// Also folds the largest 1/d^2 left to the coarse pass into *keep_max (as
// float bits: positive floats order like their bit patterns); the coarse
// error bound is stated for the shortest pair the coarse pass still sees.
__global__ __launch_bounds__(256) void k_mark_close(float4 *invd2, const int2 *tiles,
                                                    int64_t ntiles, float thr, int2 *list,
                                                    int64_t cap, unsigned long long *count,
                                                    unsigned *keep_max) {
    __shared__ unsigned s_max;
    if (threadIdx.x == 0) s_max = 0u;
    __syncthreads();
    const int c = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    unsigned mx = 0u;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int2 b = tiles[t];
        for (int m = 0; m < 4; ++m) {
            const int g = w + 4 * m;
            float4 *ptr = invd2 + t * (kTileElems / 4) + g * 64 + c;
            float4 v = *ptr;
            float vv[4] = {v.x, v.y, v.z, v.w};
            bool hit = false;
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                if (vv[rr] > thr) {
                    unsigned long long at = atomicAdd(count, 1ull);
                    if ((int64_t)at < cap)
                        list[at] = make_int2(b.x * kTile + 4 * g + rr, b.y * kTile + c);
                    vv[rr] = kMaskClose;
                    hit = true;
                } else if (vv[rr] > 0.0f) {
                    mx = max(mx, __float_as_uint(vv[rr]));
                }
            }
            if (hit) *ptr = make_float4(vv[0], vv[1], vv[2], vv[3]);
        }
    }
    atomicMax(&s_max, mx);
    __syncthreads();
    if (threadIdx.x == 0 && s_max) atomicMax(keep_max, s_max);
}

}  // namespace sap
