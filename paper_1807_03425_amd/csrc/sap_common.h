// Internal declarations shared by the HIP kernels and the host runtime of
// the SAP library.  Not part of the public ABI (that is include/sap.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sap.h"

namespace sap {

constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kTile = 64;           // fused pass: 64 x 64 point-pair tiles
constexpr int kTileElems = kTile * kTile;
constexpr int kChunk = 256;         // plain pass: 256 consecutive pairs per chunk
constexpr int kMaxK = 16;           // widest projection handled (one MFMA N-tile)
constexpr int kPairBlock = 256;     // threads per block of the pair passes
constexpr uint32_t kKeyNone = 0xFFFFFFFFu;  // "no pair": loses every unsigned min

// Sentinels stored in the fused 1/d^2 array.  Both are negative, so the
// product with a sum of squares is <= -0.0, whose bit pattern as an
// unsigned integer exceeds that of every non-negative float: masked pairs
// lose the unsigned minimum without a branch.
constexpr float kMaskDropped = -1.0f;  // padding, i >= j, duplicate, d < l
constexpr float kMaskClose = -2.0f;    // evaluated in FP64 from the close list

// Per-block result of the pass: the best FP64-rescored pair of the block.
struct Partial {
    double r;         // best FP64 r in the block (+inf if none)
    double r2;        // second-smallest FP64 r evaluated in the block (+inf if none)
    int32_t i, j;     // the pair of r
    int32_t n_rescored;
    int32_t n_units;  // work items (half-tiles / chunks) with rescored pairs
    int32_t n_viol;   // rescored pairs whose coarse value broke the error bound,
                      // plus candidates dropped for want of list space
    uint32_t kmin;    // smallest coarse key of the block (kKeyNone: none)
    uint32_t limit;   // smallest candidate-key limit a full list imposed
                      // (kKeyNone: none): keys above it were not rescored
    int32_t pad;
};

// Device-resident record of the last evaluation (read back by the host).
struct DevResult {
    double min_norm;
    double runner_up;
    int64_t i, j, q;
    double coarse_min;
    double window;
    int32_t certified;
    int32_t runner_up_exact;
    int32_t n_rescored;
    int32_t t;
    int32_t n_tiles;
    int32_t pad;
};

// Mutable device-side scalars of a handle.
struct DevState {
    uint32_t gmin;       // min coarse key (bits of r~^2) over non-close pairs
    uint32_t pad;
    double radius;       // max_i ||x_i - mu|| (init)
    uint64_t radius_bits;
    int32_t nonfinite;   // init: X held NaN/Inf
    int32_t pad2;
    int64_t kept, dropped;  // init pair counts
    uint64_t hist[64];   // init: close-pair ladder counts
    int64_t n_close;     // init: length of the close list
    uint32_t sweep_counter;  // blocks of the running sweep that have finished
    uint32_t keep_max;       // init: largest 1/d^2 (float bits) left to the coarse pass
    // soft-min
    double sm_m, sm_s;   // running (reference, scaled sum)
    double sm_L;         // loss of the last forward
    int64_t sm_nzero;
};

__device__ __forceinline__ int64_t pair_index(int64_t N, int64_t i, int64_t j) {
    return i * N - i * (i + 1) / 2 + (j - i - 1);
}

// Pair (i, j), i < j, of pair index q (inverse of pair_index).
__device__ __forceinline__ void decode_pair(int64_t q, int64_t N, int64_t &i, int64_t &j) {
    double b = 2.0 * (double)N - 1.0;
    double disc = b * b - 8.0 * (double)q;
    int64_t ii = (int64_t)floor((b - sqrt(disc > 0.0 ? disc : 0.0)) * 0.5);
    if (ii < 0) ii = 0;
    if (ii > N - 2) ii = N - 2;
    while (ii > 0 && pair_index(N, ii, ii + 1) > q) --ii;
    while (ii < N - 2 && pair_index(N, ii + 1, ii + 2) <= q) ++ii;
    i = ii;
    j = q - pair_index(N, ii, ii + 1) + ii + 1;
}

__device__ __forceinline__ double load_x(const void *X, int dtype, int64_t off) {
    return dtype == SAP_F64 ? static_cast<const double *>(X)[off]
                            : static_cast<double>(static_cast<const float *>(X)[off]);
}

// Butterfly reductions over the 64 lanes of a wavefront.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t w = __shfl_xor(v, o, kWave);
        v = w < v ? w : v;
    }
    return v;
}

// lexicographic (r, i, j) order (no branches; false whenever r or r2 is NaN)
__device__ __forceinline__ bool lex_less(double r, int32_t i, int32_t j, double r2,
                                         int32_t i2, int32_t j2) {
    return (r < r2) | ((r == r2) & ((i < i2) | ((i == i2) & (j < j2))));
}

__device__ __forceinline__ void wave_min_lex(double &r, int32_t &i, int32_t &j) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double r2 = __shfl_xor(r, o, kWave);
        int32_t i2 = __shfl_xor(i, o, kWave);
        int32_t j2 = __shfl_xor(j, o, kWave);
        if (lex_less(r2, i2, j2, r, i, j)) { r = r2; i = i2; j = j2; }
    }
}

// Launch geometry of one kernel on the handle's stream; ea / eb (may be
// null) receive the dispatch's own start and end timestamps.
struct LaunchCfg {
    dim3 grid, block;
    uint32_t shmem;
    hipStream_t stream;
    hipEvent_t ea, eb;
};

}  // namespace sap

// Record the calling thread's last error (the message sap_last_error(NULL)
// returns); defined in the host runtime, used by every entry point.
void sap_internal_set_error(const char *msg);

// Dispatch a templated launch over the projection width K = 1..16.
#define SAP_DISPATCH_K(kval, ...)                                           \
    switch (kval) {                                                          \
        case 1: { constexpr int K = 1; __VA_ARGS__; } break;                 \
        case 2: { constexpr int K = 2; __VA_ARGS__; } break;                 \
        case 3: { constexpr int K = 3; __VA_ARGS__; } break;                 \
        case 4: { constexpr int K = 4; __VA_ARGS__; } break;                 \
        case 5: { constexpr int K = 5; __VA_ARGS__; } break;                 \
        case 6: { constexpr int K = 6; __VA_ARGS__; } break;                 \
        case 7: { constexpr int K = 7; __VA_ARGS__; } break;                 \
        case 8: { constexpr int K = 8; __VA_ARGS__; } break;                 \
        case 9: { constexpr int K = 9; __VA_ARGS__; } break;                 \
        case 10: { constexpr int K = 10; __VA_ARGS__; } break;               \
        case 11: { constexpr int K = 11; __VA_ARGS__; } break;               \
        case 12: { constexpr int K = 12; __VA_ARGS__; } break;               \
        case 13: { constexpr int K = 13; __VA_ARGS__; } break;               \
        case 14: { constexpr int K = 14; __VA_ARGS__; } break;               \
        case 15: { constexpr int K = 15; __VA_ARGS__; } break;               \
        case 16: { constexpr int K = 16; __VA_ARGS__; } break;               \
        default: break;                                                      \
    }
