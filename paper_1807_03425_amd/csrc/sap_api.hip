// Host runtime of the SAP library: argument validation, buffer ownership,
// launch sequencing and the extern "C" entry points declared in sap.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <utility>
#include <vector>

#include <hip/hip_ext.h>

#include "sap_common.h"

// The K-independent kernels are compiled into this translation unit; the
// kernels templated on K are compiled per K in sap_kinst.hip and reached
// through the KLaunch launchers.
#include "sap_init.hip"
#include "sap_iter.hip"
#include "sap_softmin.hip"
#include "sap_pca.hip"
#include "sap_launch.h"

using namespace sap;

// Grid sizing of the fused pass: short pairs per short-pair block.
#ifndef SAP_SHORT64_PER_BLOCK
#define SAP_SHORT64_PER_BLOCK 256   // short pairs per block when their bounds come from the FP64 Y
#endif
#ifndef SAP_SHORT_PER_BLOCK
#define SAP_SHORT_PER_BLOCK 64
#endif
// Automatic short-pair cap: p / (SAP_CLOSE_CAP_DIV n) pairs, within
// [1024, 2^20] (a short pair and a rescored window pair cost about the same:
// one FP64 product over n).
#ifndef SAP_CLOSE_CAP_DIV
#define SAP_CLOSE_CAP_DIV 1
#endif
// Automatic short-pair cutoff: the absolute coarse error it aims at.  A
// tighter target mostly adds short pairs (each an FP64 product over n every
// iteration) while the rescoring window it narrows holds few pairs.
#ifndef SAP_EABS_TARGET
#define SAP_EABS_TARGET 4e-6
#endif

// ---------------------------------------------------------------- context

struct sap_ctx {
    sap_config cfg{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool poisoned = false;
    std::string err;

    const void *X = nullptr;
    int64_t ldx = 0, N = 0, p = 0;
    bool vec_x = false, vec_p = false;   // 16-byte loads of X rows / P64t rows are aligned
    int n = 0, k = 0, kp = 0;

    // fused
    int64_t nb = 0, Npad = 0, ntiles = 0, nclose = 0;
    int2 *d_tiles = nullptr;
    float4 *d_invd2 = nullptr;
    float *d_Y = nullptr;
    double *d_Y64 = nullptr;  // FP64 GEMM with short pairs: the unrounded Y
    double s_d2 = 0, s_eps = 0;   // short-pair bound from d_Y64
    int2 *d_close = nullptr;
    double *d_cd = nullptr;   // short pairs: ||x_i - x_j||
    // the short-pair list (sorted by (i, j)) as CSR by i and by j
    int32_t *d_rp_i = nullptr, *d_rp_j = nullptr, *d_permj = nullptr;

    // plain
    void *d_S = nullptr;
    int64_t pcols = 0, nchunks = 0;
    void *d_Pr = nullptr;

    // common
    double *d_P64t = nullptr;       // the current P (FP64 master, K x n)
    double *d_P64t_alt = nullptr;   // fused: the other P buffer, written by k_selprep
    double *d_mu = nullptr;
    DevState *d_st = nullptr;
    Partial *d_part = nullptr;   // pass-block results, then one per short-pair block
    DevResult *d_res = nullptr;
    int pass_grid = 0, short_grid = 0;
    // fused FP64 Y GEMM split over two wavefronts per 16-row tile (k_prep and
    // k_selprep run n_pad / 32 blocks; see gemm_block_deep)
    bool gemm_split = false;
    // k_selprep: 64-row groups of Y per block (2 when there are more groups
    // than compute units, so that one round of blocks covers the rows)
    int gtiles = 1;
    int short_grid_it = 0;   // short-pair blocks of the iteration's pass (<= short_grid)
    int sm_grid = 0;   // fused: blocks of the soft-min tile passes
    size_t tail_lds = 0;

    // soft-min (allocated on first use)
    double *d_smP64t = nullptr;
    float *d_smP32 = nullptr;         // the forward's P as passed (n x k FP32)
    float *d_smY = nullptr;
    SmPart *d_smpart = nullptr;
    float *d_smZr = nullptr, *d_smZc = nullptr;
    double *d_smZ = nullptr, *d_zpair = nullptr, *d_smG = nullptr;
    int sm_chunks = 0;
    int64_t sm_rows = 0;
    bool sm_ready = false;
    double sm_tau = 0.0;

    double radius = 0, close_d = 0, e_abs = 0, e_rel = 0;
    int64_t kept = 0, dropped = 0;
    int64_t dev_bytes = 0;
    std::vector<void *> allocs;

    // per-kernel timing (sap_profile_enable)
    struct Mark { hipEvent_t a, b; int slot; };   // slots as in sap_profile_t
    bool prof_on = false;
    std::vector<Mark> marks;
    std::vector<hipEvent_t> ev_pool;
};

static thread_local std::string g_tls_err;

void sap_internal_set_error(const char *msg) { g_tls_err = msg; }

static sap_status fail(sap_ctx *h, sap_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) {
        h->err = buf;
        if (st == SAP_ERR_DEVICE) h->poisoned = true;
    }
    g_tls_err = buf;
    return st;
}

#define SAP_HIP(h, expr)                                                                  \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) {                                                           \
            if (e_ == hipErrorOutOfMemory)                                                \
                return fail(h, SAP_ERR_OUT_OF_MEMORY, "%s: %s", #expr, hipGetErrorString(e_)); \
            return fail(h, SAP_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));     \
        }                                                                                 \
    } while (0)

#define SAP_LAUNCHED(h, what)                                                             \
    do {                                                                                  \
        hipError_t e_ = hipGetLastError();                                                \
        if (e_ != hipSuccess)                                                             \
            return fail(h, SAP_ERR_DEVICE, "launch of %s: %s", what, hipGetErrorString(e_)); \
    } while (0)

template <typename T>
static sap_status dalloc(sap_ctx *h, T **ptr, size_t bytes) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, e == hipErrorOutOfMemory ? SAP_ERR_OUT_OF_MEMORY : SAP_ERR_DEVICE,
                    "hipMalloc(%zu bytes): %s", bytes, hipGetErrorString(e));
    }
    h->allocs.push_back(p);
    h->dev_bytes += (int64_t)bytes;
    *ptr = static_cast<T *>(p);
    return SAP_OK;
}

#define SAP_TRY(expr)                        \
    do {                                     \
        sap_status s_ = (expr);              \
        if (s_ != SAP_OK) return s_;         \
    } while (0)

static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

static constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24
static constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53

// Validation of a configuration; no HIP call.  Shared with sap_init.
static sap_status validate(const sap_config *c, int64_t ldx, const void *X, const void *P0,
                           const void *out) {
    if (!c || !X || !P0 || !out) return fail(nullptr, SAP_ERR_INVALID_ARG, "null pointer argument");
    if (c->N < 2) return fail(nullptr, SAP_ERR_INVALID_ARG, "N must be >= 2 (got %lld)", (long long)c->N);
    if (c->N >= (1ll << 31) - 64)
        return fail(nullptr, SAP_ERR_UNSUPPORTED, "N must be < 2^31 - 64");
    if (c->n < 1) return fail(nullptr, SAP_ERR_INVALID_ARG, "n must be >= 1");
    if (c->k < 1 || c->k > c->n)
        return fail(nullptr, SAP_ERR_INVALID_ARG, "k must satisfy 1 <= k <= n (k=%d, n=%d)", c->k, c->n);
    if (c->k > kMaxK) return fail(nullptr, SAP_ERR_UNSUPPORTED, "k > %d is not supported", kMaxK);
    if ((int64_t)c->n * (c->k + 3) > 19200)
        return fail(nullptr, SAP_ERR_UNSUPPORTED, "n*(k+3) must be <= 19200 (the update runs in LDS)");
    if (c->dtype != SAP_F64 && c->dtype != SAP_F32)
        return fail(nullptr, SAP_ERR_INVALID_ARG, "dtype must be SAP_F64 or SAP_F32");
    if (c->form != SAP_PLAIN && c->form != SAP_FUSED)
        return fail(nullptr, SAP_ERR_INVALID_ARG, "form must be SAP_PLAIN or SAP_FUSED");
    {
        // per-block records hold 32-bit pair (plain) or sub-tile (fused) indices
        const int64_t p = c->N * (c->N - 1) / 2, nb = (c->N + kTile - 1) / kTile;
        if (c->form == SAP_PLAIN && p >= (1ll << 32) - kChunk)
            return fail(nullptr, SAP_ERR_UNSUPPORTED, "the plain form needs N(N-1)/2 < 2^32 - 256");
        if (c->form == SAP_FUSED && 2 * nb * (nb + 1) >= (1ll << 32))
            return fail(nullptr, SAP_ERR_UNSUPPORTED, "the fused form needs fewer than 2^32 sub-tiles");
    }
    if (c->rule != SAP_STEP_LITERAL && c->rule != SAP_STEP_NORMALIZED)
        return fail(nullptr, SAP_ERR_INVALID_ARG, "rule must be SAP_STEP_LITERAL or SAP_STEP_NORMALIZED");
    if (!(c->alpha >= 0.0 && c->alpha <= 1.0))
        return fail(nullptr, SAP_ERR_INVALID_ARG, "alpha must lie in [0, 1]");
    if (!(c->min_len >= 0.0) || !std::isfinite(c->min_len))
        return fail(nullptr, SAP_ERR_INVALID_ARG, "min_len must be finite and >= 0");
    if (std::isnan(c->close_d) || std::isinf(c->close_d))
        return fail(nullptr, SAP_ERR_INVALID_ARG, "close_d must be finite (< 0 = automatic)");
    if (c->close_cap < 0) return fail(nullptr, SAP_ERR_INVALID_ARG, "close_cap must be >= 0");
    if (c->cand_cap < 0 || c->cand_cap > kCandCap)
        return fail(nullptr, SAP_ERR_INVALID_ARG, "cand_cap must lie in [0, %d] (0 = %d)", kCandCap, kCandCap);
    if (c->gemm != SAP_GEMM_F64 && c->gemm != SAP_GEMM_F32 && c->gemm != SAP_GEMM_BF16)
        return fail(nullptr, SAP_ERR_INVALID_ARG, "gemm must be SAP_GEMM_F64, SAP_GEMM_F32 or SAP_GEMM_BF16");
    if (c->gemm != SAP_GEMM_F64 && c->form != SAP_FUSED)
        return fail(nullptr, SAP_ERR_INVALID_ARG, "gemm selects the fused form's Y GEMM: plain form needs SAP_GEMM_F64");
    if (ldx < c->n) return fail(nullptr, SAP_ERR_INVALID_ARG, "ldx must be >= n");
    return SAP_OK;
}

static sap_status check_P_host(sap_ctx *h, const std::vector<double> &P, int n, int k) {
    for (double v : P)
        if (!std::isfinite(v)) return fail(h, SAP_ERR_NONFINITE, "P holds NaN or Inf");
    double e = 0.0;
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            double acc = 0.0;
            for (int l = 0; l < n; ++l) acc += P[(size_t)l * k + a] * P[(size_t)l * k + b];
            e = std::max(e, std::fabs(acc - (a == b ? 1.0 : 0.0)));
        }
    if (e > 1e-6) return fail(h, SAP_ERR_NOT_ORTHONORMAL, "max |P^T P - I| = %.3g > 1e-6", e);
    return SAP_OK;
}

// Load a device P (n x k row-major) into the FP64 master (k x n) after checks.
static sap_status load_P(sap_ctx *h, const double *P_dev) {
    const int n = h->n, k = h->k;
    std::vector<double> P((size_t)n * k), Pt((size_t)n * k);
    SAP_HIP(h, hipMemcpyAsync(P.data(), P_dev, sizeof(double) * n * k, hipMemcpyDeviceToHost, h->stream));
    SAP_HIP(h, hipStreamSynchronize(h->stream));
    SAP_TRY(check_P_host(h, P, n, k));
    for (int l = 0; l < n; ++l)
        for (int q = 0; q < k; ++q) Pt[(size_t)q * n + l] = P[(size_t)l * k + q];
    SAP_HIP(h, hipMemcpyAsync(h->d_P64t, Pt.data(), sizeof(double) * n * k, hipMemcpyHostToDevice,
                              h->stream));
    if (h->cfg.form == SAP_PLAIN) {
        const int blocks = (int)ceil_div((int64_t)n * k, 256);
        if (h->cfg.dtype == SAP_F64)
            hipLaunchKernelGGL(k_write_Pr<double>, dim3(blocks), dim3(256), 0, h->stream, h->d_P64t, n, k,
                               static_cast<double *>(h->d_Pr));
        else
            hipLaunchKernelGGL(k_write_Pr<float>, dim3(blocks), dim3(256), 0, h->stream, h->d_P64t, n, k,
                               static_cast<float *>(h->d_Pr));
        SAP_LAUNCHED(h, "k_write_Pr");
    }
    SAP_HIP(h, hipStreamSynchronize(h->stream));
    return SAP_OK;
}

// ---------------------------------------------------------------- init pieces

static sap_status init_moments(sap_ctx *h) {
    const int64_t rows = 256;
    const int64_t nblk = ceil_div(h->N, rows);
    double *part = nullptr;
    SAP_TRY(dalloc(h, &part, sizeof(double) * nblk * h->n));
    SAP_HIP(h, hipMemsetAsync(h->d_st, 0, sizeof(DevState), h->stream));
    hipLaunchKernelGGL(k_col_partial, dim3((unsigned)nblk), dim3(256), 0, h->stream, h->X,
                       h->cfg.dtype, h->ldx, h->N, h->n, rows, part, &h->d_st->nonfinite);
    SAP_LAUNCHED(h, "k_col_partial");
    hipLaunchKernelGGL(k_col_mean, dim3((unsigned)ceil_div(h->n, 256)), dim3(256), 0, h->stream,
                       part, nblk, h->n, h->N, h->d_mu);
    SAP_LAUNCHED(h, "k_col_mean");
    hipLaunchKernelGGL(k_radius, dim3((unsigned)ceil_div(h->N, 4)), dim3(256), 0, h->stream, h->X,
                       h->cfg.dtype, h->ldx, h->N, h->n, h->d_mu,
                       reinterpret_cast<unsigned long long *>(&h->d_st->radius_bits));
    SAP_LAUNCHED(h, "k_radius");
    DevState st;
    SAP_HIP(h, hipMemcpyAsync(&st, h->d_st, sizeof st, hipMemcpyDeviceToHost, h->stream));
    SAP_HIP(h, hipStreamSynchronize(h->stream));
    if (st.nonfinite) return fail(h, SAP_ERR_NONFINITE, "X holds NaN or Inf");
    double r;
    std::memcpy(&r, &st.radius_bits, sizeof r);
    h->radius = r;
    return SAP_OK;
}

static sap_status init_plain(sap_ctx *h) {
    const bool f64 = h->cfg.dtype == SAP_F64;
    const size_t es = f64 ? 8 : 4;
    h->pcols = ceil_div(h->p, kChunk) * kChunk;
    h->nchunks = h->pcols / kChunk;
    SAP_TRY(dalloc(h, &h->d_S, es * (size_t)h->n * (size_t)h->pcols));
    SAP_TRY(dalloc(h, &h->d_Pr, es * (size_t)h->n * h->k));
    const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(h->pcols, 256), 65536);
    auto *kept = reinterpret_cast<unsigned long long *>(&h->d_st->kept);
    auto *drop = reinterpret_cast<unsigned long long *>(&h->d_st->dropped);
    if (f64)
        hipLaunchKernelGGL(k_build_secants<double>, dim3(grid), dim3(256), 0, h->stream, h->X,
                           h->cfg.dtype, h->ldx, h->N, h->n, h->cfg.min_len,
                           static_cast<double *>(h->d_S), h->pcols, h->p, kept, drop);
    else
        hipLaunchKernelGGL(k_build_secants<float>, dim3(grid), dim3(256), 0, h->stream, h->X,
                           h->cfg.dtype, h->ldx, h->N, h->n, h->cfg.min_len,
                           static_cast<float *>(h->d_S), h->pcols, h->p, kept, drop);
    SAP_LAUNCHED(h, "k_build_secants");
    DevState st;
    SAP_HIP(h, hipMemcpyAsync(&st, h->d_st, sizeof st, hipMemcpyDeviceToHost, h->stream));
    SAP_HIP(h, hipStreamSynchronize(h->stream));
    h->kept = st.kept;
    h->dropped = st.dropped;
    // |c~ - c| <= (n+3) u sqrt(k) (rounded secants and P, FMA accumulation),
    // and the final sum of squares adds (k+2) u relative.
    const double u = f64 ? kU64 : kU32;
    h->e_abs = (h->n + 3) * u * std::sqrt((double)h->k) * 1.01;
    h->e_rel = (h->k + 4) * u + (f64 ? 2.0 * kU32 : 0.0);
    h->pass_grid = (int)std::min<int64_t>(ceil_div(h->nchunks, 4), 2048);
    return SAP_OK;
}

static sap_status init_fused(sap_ctx *h) {
    h->nb = ceil_div(h->N, kTile);
    h->Npad = h->nb * kTile;
    h->ntiles = h->nb * (h->nb + 1) / 2;
    h->kp = h->k <= 4 ? 4 : (h->k <= 8 ? 8 : (h->k <= 12 ? 12 : 16));
    std::vector<int2> tiles((size_t)h->ntiles);
    for (int64_t bi = 0, t = 0; bi < h->nb; ++bi)
        for (int64_t bj = bi; bj < h->nb; ++bj, ++t) tiles[(size_t)t] = make_int2((int)bi, (int)bj);
    SAP_TRY(dalloc(h, &h->d_tiles, sizeof(int2) * h->ntiles));
    SAP_TRY(dalloc(h, &h->d_invd2, sizeof(float) * (size_t)h->ntiles * kTileElems));
    SAP_TRY(dalloc(h, &h->d_Y, sizeof(float) * (size_t)h->Npad * h->kp));
    SAP_HIP(h, hipMemcpyAsync(h->d_tiles, tiles.data(), sizeof(int2) * h->ntiles,
                              hipMemcpyHostToDevice, h->stream));

    // Coarse error: ||y~_i - y_i|| <= delta, so |r~ - r| <= 2 delta / d.
    //   FP64 GEMM: delta = R (u32 + (n + 2) sqrt(k) 4 u64) (rounding Y to FP32);
    //   FP32 GEMM: operands rounded (u32 each) and FP32 accumulation over n
    //     terms: per component (n + 3) u32 sum_l |x_l - mu_l| |P_lc| <=
    //     (n + 3) u32 R, so delta = sqrt(k) (n + 3) u32 R;
    //   BF16 GEMM: operands rounded to BF16 (2^-8 each, through FP32), exact
    //     products, FP32 accumulation: delta = sqrt(k) (2^-7 + 2^-15 +
    //     (n + 1) u32) R.
    // The automatic cutoff aims at an absolute error of SAP_EABS_TARGET for
    // every pair left to the coarse pass.
    const double sk = std::sqrt((double)h->k);
    double delta = h->radius * (kU32 * 1.001 + (h->n + 2) * sk * kU64 * 4.0);
    if (h->cfg.gemm == SAP_GEMM_F32) delta = h->radius * sk * (h->n + 3) * kU32 * 1.01;
    if (h->cfg.gemm == SAP_GEMM_BF16)
        delta = h->radius * sk * (std::ldexp(1.0, -7) + std::ldexp(1.0, -15) + (h->n + 1) * kU32) * 1.01;
    const bool automatic = h->cfg.close_d < 0.0;
    // no pair is longer than 2R: an automatic ladder starts there at most
    // (a wide bound -- a BF16 GEMM -- would otherwise start it far above
    // every distance and let its 64 rungs end above the shortest pairs)
    double dtarget = automatic ? std::min(2.0 * delta / SAP_EABS_TARGET, 2.0 * h->radius * (1.0 + 1e-9))
                               : h->cfg.close_d;
    std::vector<float> ladder(64);
    for (int m = 0; m < 64; ++m) {
        const double D = dtarget * std::pow(2.0, -m / 4.0);
        ladder[m] = D > 0.0 ? (float)(1.0 / (D * D)) : std::numeric_limits<float>::infinity();
    }
    float *d_ladder = nullptr;
    SAP_TRY(dalloc(h, &d_ladder, sizeof(float) * 64));
    SAP_HIP(h, hipMemcpyAsync(d_ladder, ladder.data(), sizeof(float) * 64, hipMemcpyHostToDevice, h->stream));
    const unsigned grid = (unsigned)std::min<int64_t>(h->ntiles, 8192);
    hipLaunchKernelGGL(k_build_invd2, dim3(grid), dim3(256), 0, h->stream, h->X, h->cfg.dtype,
                       h->ldx, h->N, h->n, h->d_tiles, h->ntiles, h->cfg.min_len, h->d_invd2,
                       d_ladder, reinterpret_cast<unsigned long long *>(h->d_st->hist),
                       reinterpret_cast<unsigned long long *>(&h->d_st->kept),
                       reinterpret_cast<unsigned long long *>(&h->d_st->dropped));
    SAP_LAUNCHED(h, "k_build_invd2");
    DevState st;
    SAP_HIP(h, hipMemcpyAsync(&st, h->d_st, sizeof st, hipMemcpyDeviceToHost, h->stream));
    SAP_HIP(h, hipStreamSynchronize(h->stream));
    h->kept = st.kept;
    h->dropped = st.dropped;
    if (h->kept == 0) return SAP_OK;  // caller reports SAP_ERR_NO_PAIRS

    const int64_t cap = h->cfg.close_cap > 0
                            ? h->cfg.close_cap
                            : std::min<int64_t>(1 << 20, std::max<int64_t>(1024, h->p / (SAP_CLOSE_CAP_DIV * h->n)));
    // count(1/d^2 > ladder[m]) = sum of bins m..63
    int msel = -1;
    uint64_t tail = 0;
    std::vector<uint64_t> above(64);
    for (int m = 63; m >= 0; --m) { tail += st.hist[m]; above[m] = tail; }
    if (automatic) {
        for (int m = 0; m < 64; ++m)
            if ((int64_t)above[m] <= cap) { msel = m; break; }
        if (msel < 0)
            return fail(h, SAP_ERR_CAPACITY,
                        "%llu pairs are closer than %.3g: above the short-pair cap %lld",
                        (unsigned long long)above[63], dtarget * std::pow(2.0, -63 / 4.0), (long long)cap);
    } else {
        if ((int64_t)above[0] > cap)
            return fail(h, SAP_ERR_CAPACITY, "%llu pairs are closer than close_d=%.3g: above close_cap %lld",
                        (unsigned long long)above[0], dtarget, (long long)cap);
        msel = 0;
    }
    const float thr = ladder[msel];
    const int64_t want = (int64_t)above[msel];
    if (want > 0) SAP_TRY(dalloc(h, &h->d_close, sizeof(int2) * want));
    {
        unsigned long long *d_count = reinterpret_cast<unsigned long long *>(&h->d_st->n_close);
        hipLaunchKernelGGL(k_mark_close, dim3(grid), dim3(256), 0, h->stream, h->d_invd2, h->d_tiles,
                           h->ntiles, thr, h->d_close, want, d_count, &h->d_st->keep_max);
        SAP_LAUNCHED(h, "k_mark_close");
        SAP_HIP(h, hipMemcpyAsync(&st, h->d_st, sizeof st, hipMemcpyDeviceToHost, h->stream));
        SAP_HIP(h, hipStreamSynchronize(h->stream));
        if (st.n_close != want)
            return fail(h, SAP_ERR_DEVICE, "short-pair count mismatch (%lld vs %lld)",
                        (long long)st.n_close, (long long)want);
    }
    if (want > 0) {
        // deterministic order: sort by (i, j)
        std::vector<int2> lst((size_t)want);
        SAP_HIP(h, hipMemcpyAsync(lst.data(), h->d_close, sizeof(int2) * want, hipMemcpyDeviceToHost, h->stream));
        SAP_HIP(h, hipStreamSynchronize(h->stream));
        std::sort(lst.begin(), lst.end(), [](const int2 &a, const int2 &b) {
            return a.x != b.x ? a.x < b.x : a.y < b.y;
        });
        SAP_HIP(h, hipMemcpyAsync(h->d_close, lst.data(), sizeof(int2) * want, hipMemcpyHostToDevice, h->stream));
        // CSR by i (the list order) and by j (a permutation), for the
        // per-point sums of the soft-min gradient
        std::vector<int32_t> rp_i((size_t)h->N + 1, 0), rp_j((size_t)h->N + 1, 0), permj((size_t)want);
        for (const int2 &e : lst) { ++rp_i[(size_t)e.x + 1]; ++rp_j[(size_t)e.y + 1]; }
        for (int64_t p = 0; p < h->N; ++p) { rp_i[(size_t)p + 1] += rp_i[(size_t)p]; rp_j[(size_t)p + 1] += rp_j[(size_t)p]; }
        {
            std::vector<int32_t> fill(rp_j.begin(), rp_j.end() - 1);
            for (int64_t e = 0; e < want; ++e) permj[(size_t)fill[(size_t)lst[(size_t)e].y]++] = (int32_t)e;
        }
        SAP_TRY(dalloc(h, &h->d_rp_i, sizeof(int32_t) * (size_t)(h->N + 1)));
        SAP_TRY(dalloc(h, &h->d_rp_j, sizeof(int32_t) * (size_t)(h->N + 1)));
        SAP_TRY(dalloc(h, &h->d_permj, sizeof(int32_t) * (size_t)want));
        SAP_HIP(h, hipMemcpyAsync(h->d_rp_i, rp_i.data(), sizeof(int32_t) * (h->N + 1), hipMemcpyHostToDevice, h->stream));
        SAP_HIP(h, hipMemcpyAsync(h->d_rp_j, rp_j.data(), sizeof(int32_t) * (h->N + 1), hipMemcpyHostToDevice, h->stream));
        SAP_HIP(h, hipMemcpyAsync(h->d_permj, permj.data(), sizeof(int32_t) * want, hipMemcpyHostToDevice, h->stream));
        // the host vectors must outlive the asynchronous copies
        SAP_HIP(h, hipStreamSynchronize(h->stream));
        SAP_TRY(dalloc(h, &h->d_cd, sizeof(double) * (size_t)want));
        const unsigned gblk = (unsigned)ceil_div(want, 256);
        if (h->cfg.dtype == SAP_F64)
            hipLaunchKernelGGL(k_short_len<double>, dim3(gblk), dim3(256), 0, h->stream,
                               static_cast<const double *>(h->X), h->ldx, h->n, h->d_close, want,
                               h->d_cd);
        else
            hipLaunchKernelGGL(k_short_len<float>, dim3(gblk), dim3(256), 0, h->stream,
                               static_cast<const float *>(h->X), h->ldx, h->n, h->d_close, want,
                               h->d_cd);
        SAP_LAUNCHED(h, "k_short_len");
    }
    h->nclose = want;
    // every pair left to the coarse pass has fl32(1/d^2) <= w_max, hence
    // d >= 1/sqrt(w_max (1 + 2^-22)); no such pair: no coarse bound needed
    float wmax;
    std::memcpy(&wmax, &st.keep_max, sizeof wmax);
    h->close_d = dtarget * std::pow(2.0, -msel / 4.0);
    h->e_abs = st.keep_max ? 2.0 * delta * std::sqrt((double)wmax * (1.0 + std::ldexp(1.0, -22))) : 0.0;
    h->e_rel = (h->k + 4) * kU32;
    // iteration: 64 short pairs per block (16 per wavefront, on the matrix
    // cores); the soft-min's short-pair blocks use the same grid size
    h->short_grid = h->nclose > 0 ? (int)std::min<int64_t>(ceil_div(h->nclose, SAP_SHORT_PER_BLOCK), 1024) : 0;
    h->short_grid_it = h->short_grid;
    // FP64 GEMM: the iteration bounds each short pair from the unrounded Y
    // (error 2 delta64 / d, delta64 = 4 (n + 2) sqrt(k) u64 R) and evaluates
    // exactly only those that may hold one of its block's two smallest values
    if (h->nclose > 0 && h->cfg.gemm == SAP_GEMM_F64) {
        SAP_TRY(dalloc(h, &h->d_Y64, sizeof(double) * (size_t)h->Npad * h->kp));
        h->s_d2 = 2.0 * h->radius * (h->n + 2) * sk * kU64 * 4.0 * (1.0 + 1e-6);
        h->s_eps = 2.0 * (h->n + h->k + 12) * kU64;
        h->short_grid_it = (int)std::min<int64_t>(ceil_div(h->nclose, SAP_SHORT64_PER_BLOCK), 1024);
    }
    // pass blocks: with the short-pair blocks, one round of resident blocks
    // (four per compute unit), and at least one half-tile per wavefront; the
    // blocks stride over the rest of the tiles
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus <= 0)
        cus = 256;
    const int64_t slots = 4 * (int64_t)cus;
    // the split GEMM: 512 or 1024 components, 16-byte X rows, FP64, and fewer
    // 64-row blocks than compute units (the split doubles them)
    h->gemm_split = h->cfg.gemm == SAP_GEMM_F64 && h->vec_x && (h->n == 512 || h->n == 1024) &&
                    h->Npad / 64 < cus;
    h->gtiles = (h->n < 512 && h->Npad / 64 > cus) ? 2 : 1;
    h->pass_grid = (int)std::max<int64_t>(
        1, std::min<int64_t>(ceil_div(2 * h->ntiles, 4), std::max<int64_t>(slots / 4, slots - h->short_grid_it)));
    // soft-min tile passes (three or four blocks per compute unit): eight
    // half-tiles per block, many rounds
    h->sm_grid = (int)std::min<int64_t>(ceil_div(2 * h->ntiles, 8), 8192);
    return SAP_OK;
}

// ---------------------------------------------------------------- iteration

static sap_status ev_get(sap_ctx *h, hipEvent_t *e) {
    if (!h->ev_pool.empty()) { *e = h->ev_pool.back(); h->ev_pool.pop_back(); return SAP_OK; }
    SAP_HIP(h, hipEventCreate(e));
    return SAP_OK;
}

// Launch on the handle's stream.  With profiling on, the kernel's own start
// and end timestamps are taken (hipExtLaunchKernelGGL's event pair: no extra
// packets between launches) and accumulated in `slot`.
template <typename F, typename... Args>
static sap_status launch(sap_ctx *h, int slot, const char *what, F kernel, dim3 grid, dim3 block,
                         uint32_t shmem, Args... args) {
    hipEvent_t ea = nullptr, eb = nullptr;
    if (h->prof_on) {
        SAP_TRY(ev_get(h, &ea));
        SAP_TRY(ev_get(h, &eb));
    }
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, h->stream, ea, eb, 0, args...);
    SAP_LAUNCHED(h, what);
    if (ea) h->marks.push_back(sap_ctx::Mark{ea, eb, slot});
    return SAP_OK;
}

// Launch through a typed launcher fn(LaunchCfg) (the per-K kernels), with
// the same profiling as launch().
template <typename F>
static sap_status launch_with(sap_ctx *h, int slot, const char *what, dim3 grid, dim3 block, uint32_t shmem,
                              F &&fn) {
    hipEvent_t ea = nullptr, eb = nullptr;
    if (h->prof_on) {
        SAP_TRY(ev_get(h, &ea));
        SAP_TRY(ev_get(h, &eb));
    }
    const LaunchCfg c{grid, block, shmem, h->stream, ea, eb};
    const hipError_t e = fn(c);
    if (e != hipSuccess) return fail(h, SAP_ERR_DEVICE, "launch of %s: %s", what, hipGetErrorString(e));
    if (ea) h->marks.push_back(sap_ctx::Mark{ea, eb, slot});
    return SAP_OK;
}

template <typename TX>
static SweepArgs<TX> sweep_args(sap_ctx *h, double *tr_min, int64_t *tr_ij, int32_t *tr_cert,
                                int it) {
    SweepArgs<TX> a{};
    a.Y = h->d_Y;
    a.kp = h->kp;
    a.invd2 = h->d_invd2;
    a.tiles = h->d_tiles;
    a.nhalf = 2 * h->ntiles;
    a.S = static_cast<const TX *>(h->d_S);
    a.pcols = h->pcols;
    a.Pr = static_cast<const TX *>(h->d_Pr);
    a.nchunks = h->nchunks;
    a.n = h->n;
    a.npass = h->pass_grid;
    a.close = h->d_close;
    a.cd = h->d_cd;
    a.nclose = h->nclose;
    a.Y64 = h->d_Y64;
    a.s_d2 = h->s_d2;
    a.s_eps = h->s_eps;
    a.part = h->d_part;
    a.e_abs = h->e_abs;
    a.e_rel = h->e_rel;
    // item_window coefficients, rounded up to FP32
    a.wa = std::nextafter((float)((1.0 + h->e_rel) / (1.0 - h->e_rel)), std::numeric_limits<float>::infinity());
    a.wb = std::nextafter((float)(2.0 * h->e_abs / (1.0 - h->e_rel)), std::numeric_limits<float>::infinity());
    a.X = static_cast<const TX *>(h->X);
    a.ldx = h->ldx;
    a.vx = h->vec_x;
    a.vp = h->vec_p;
    a.N = h->N;
    a.P64t = h->d_P64t;
    a.gmin_out = &h->d_st->gmin;
    a.res = h->d_res;
    a.tr_min = tr_min;
    a.tr_ij = tr_ij;
    a.tr_cert = tr_cert;
    a.it = it;
    a.cap = h->cfg.cand_cap > 0 ? h->cfg.cand_cap : kCandCap;
    a.gemm = h->cfg.gemm;
    a.split = h->gemm_split ? 1 : 0;
    a.gtiles = h->gtiles;
    return a;
}

// Enqueue one evaluation (+ update when do_step).
template <typename TX>
static sap_status launch_prep(sap_ctx *h) {
    const int K = h->k;
    const SweepArgs<TX> a = sweep_args<TX>(h, nullptr, nullptr, nullptr, 0);
    const dim3 g0((unsigned)(h->Npad / (h->gemm_split ? 32 : 64))), blk(kPairBlock);
    // the split GEMM keeps P, the means and 512 exchange slots in LDS
    const uint32_t lds = h->gemm_split ? (uint32_t)(sizeof(double) * ((size_t)(K + 1) * h->n + 512)) : 0u;
    SAP_DISPATCH_K(K, SAP_TRY(launch_with(h, 0, "k_prep", g0, blk, lds, [&](const LaunchCfg &c) {
        return KLaunch<K, TX>::prep(c, a, h->d_mu, h->d_Y, h->Npad);
    })));
    return SAP_OK;
}

template <typename TX>
static sap_status launch_pass(sap_ctx *h) {
    const int K = h->k;
    const bool fused = h->cfg.form == SAP_FUSED;
    const SweepArgs<TX> a = sweep_args<TX>(h, nullptr, nullptr, nullptr, 0);
    const int nshort = fused ? h->short_grid_it : 0;
    const dim3 g1((unsigned)(h->pass_grid + nshort)), blk(kPairBlock);
    SAP_DISPATCH_K(K, SAP_TRY(launch_with(h, 1, "k_pass", g1, blk, 0, [&](const LaunchCfg &c) {
        return KLaunch<K, TX>::pass(c, fused, a, nshort);
    })));
    return SAP_OK;
}

template <typename TX>
static sap_status launch_select(sap_ctx *h, int do_step, double *tr_min, int64_t *tr_ij, int32_t *tr_cert,
                                int it) {
    const int K = h->k;
    const bool fused = h->cfg.form == SAP_FUSED;
    const SweepArgs<TX> a = sweep_args<TX>(h, tr_min, tr_ij, tr_cert, it);
    const int nshort = fused ? h->short_grid_it : 0;
    const int pr_kind = fused ? 0 : (h->cfg.dtype == SAP_F64 ? 2 : 1);
    const uint32_t lds = (uint32_t)h->tail_lds;
    const dim3 blk(kPairBlock);
    SAP_DISPATCH_K(K, SAP_TRY(launch_with(h, 2, "k_select", dim3(1), blk, lds, [&](const LaunchCfg &c) {
        return KLaunch<K, TX>::select(c, fused, a, nshort, h->d_P64t, h->d_Pr, pr_kind, h->cfg.alpha,
                                      h->cfg.rule, do_step);
    })));
    return SAP_OK;
}

// Blocks of k_selprep: 32 rows each with the split GEMM, else 64 gtiles.
static int64_t selprep_blocks(const sap_ctx *h) {
    if (h->gemm_split) return h->Npad / 32;
    const int64_t rows = 64 * (int64_t)h->gtiles;
    return (h->Npad + rows - 1) / rows;
}

// Fused form: selection + update of iteration it and the Y GEMM of the next
// P in one launch; the next P goes to the other buffer, which becomes the
// current one.
template <typename TX>
static sap_status launch_selprep(sap_ctx *h, double *tr_min, int64_t *tr_ij, int32_t *tr_cert, int it) {
    const int K = h->k;
    const SweepArgs<TX> a = sweep_args<TX>(h, tr_min, tr_ij, tr_cert, it);
    const dim3 g0((unsigned)selprep_blocks(h)), blk(kPairBlock);
    SAP_DISPATCH_K(K, SAP_TRY(launch_with(h, 6, "k_selprep", g0, blk, (uint32_t)h->tail_lds,
                                          [&](const LaunchCfg &c) {
        return KLaunch<K, TX>::selprep(c, a, h->short_grid_it, h->d_P64t_alt, h->cfg.alpha, h->cfg.rule,
                                       h->d_mu, h->d_Y, h->Npad);
    })));
    std::swap(h->d_P64t, h->d_P64t_alt);
    return SAP_OK;
}

// One evaluation (+ update when do_step): GEMM (fused), pass, selection.
template <typename TX>
static sap_status launch_iteration(sap_ctx *h, int do_step, double *tr_min, int64_t *tr_ij,
                                   int32_t *tr_cert, int it) {
    if (h->cfg.form == SAP_FUSED) SAP_TRY(launch_prep<TX>(h));
    SAP_TRY(launch_pass<TX>(h));
    return launch_select<TX>(h, do_step, tr_min, tr_ij, tr_cert, it);
}

// iters updates and a final evaluation.  Fused form with a small GEMM grid:
// the GEMM once, then per iteration the pass and the fused
// selection/update/GEMM (two launches).  Every block of the fused kernel
// reads all block results, so larger grids (more than 16 MB of such reads
// per iteration) keep the three launches.
template <typename TX>
static sap_status launch_run(sap_ctx *h, int32_t iters, double *tr_min, int64_t *tr_ij, int32_t *tr_cert) {
    // (counted per 64-row group: where the fused launch would read more, the
    // separate selection and GEMM launches are faster)
    const int64_t reads = (h->Npad / 64) * (int64_t)(h->pass_grid + h->short_grid_it) * (int64_t)sizeof(Partial);
    if (h->cfg.form != SAP_FUSED || reads > (16 << 20)) {
        for (int32_t it = 0; it <= iters; ++it)
            SAP_TRY(launch_iteration<TX>(h, it < iters ? 1 : 0, tr_min, tr_ij, tr_cert, it));
        return SAP_OK;
    }
    SAP_TRY(launch_prep<TX>(h));
    for (int32_t it = 0; it < iters; ++it) {
        SAP_TRY(launch_pass<TX>(h));
        SAP_TRY(launch_selprep<TX>(h, tr_min, tr_ij, tr_cert, it));
    }
    SAP_TRY(launch_pass<TX>(h));
    return launch_select<TX>(h, 0, tr_min, tr_ij, tr_cert, iters);
}

static sap_status enqueue_eval(sap_ctx *h, int do_step, double *tr_min, int64_t *tr_ij,
                               int32_t *tr_cert, int it) {
    if (h->cfg.dtype == SAP_F64) return launch_iteration<double>(h, do_step, tr_min, tr_ij, tr_cert, it);
    return launch_iteration<float>(h, do_step, tr_min, tr_ij, tr_cert, it);
}

static sap_status read_result(sap_ctx *h, sap_min_result *out) {
    DevResult r;
    SAP_HIP(h, hipMemcpyAsync(&r, h->d_res, sizeof r, hipMemcpyDeviceToHost, h->stream));
    SAP_HIP(h, hipStreamSynchronize(h->stream));
    out->min_norm = r.min_norm;
    out->runner_up = r.runner_up;
    out->i = r.i;
    out->j = r.j;
    out->pair_index = r.q;
    out->coarse_min = r.coarse_min;
    out->window = r.window;
    out->certified = r.certified;
    out->runner_up_exact = r.runner_up_exact;
    out->n_rescored = r.n_rescored;
    out->t = r.t;
    out->n_units = r.n_tiles;
    out->reserved = 0;
    return SAP_OK;
}

static sap_status usable(sap_ctx *h) {
    if (!h) return fail(nullptr, SAP_ERR_INVALID_ARG, "null handle");
    if (h->poisoned) return fail(h, SAP_ERR_POISONED, "handle poisoned by an earlier device error: %s", h->err.c_str());
    SAP_HIP(h, hipSetDevice(h->device));
    return SAP_OK;
}

static void destroy_ctx(sap_ctx *h) {
    if (!h) return;
    for (auto &m : h->marks) { (void)hipEventDestroy(m.a); (void)hipEventDestroy(m.b); }
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    for (void *p : h->allocs) (void)hipFree(p);
    delete h;
}

// ---------------------------------------------------------------- soft-min

static sap_status sm_check(sap_ctx *h, const float *P, double tau) {
    if (h->cfg.form != SAP_FUSED) return fail(h, SAP_ERR_UNSUPPORTED, "soft-min needs the fused form");
    if (!P) return fail(h, SAP_ERR_INVALID_ARG, "null P");
    if (!(tau >= 1e-6 && tau <= 1e6)) return fail(h, SAP_ERR_INVALID_ARG, "tau = %g outside [1e-6, 1e6]", tau);
    return SAP_OK;
}

static sap_status sm_alloc(sap_ctx *h) {
    if (h->d_smY) return SAP_OK;
    const int K = h->k;
    const int64_t nhalf = 2 * h->ntiles;
    h->sm_rows = std::max<int64_t>(64, ceil_div(h->N, 256));
    h->sm_chunks = (int)ceil_div(h->N, h->sm_rows);
    SAP_TRY(dalloc(h, &h->d_smP64t, sizeof(double) * h->n * K));
    SAP_TRY(dalloc(h, &h->d_smP32, sizeof(float) * h->n * K));
    SAP_TRY(dalloc(h, &h->d_smY, sizeof(float) * (size_t)h->Npad * h->kp));
    SAP_TRY(dalloc(h, &h->d_smpart, sizeof(SmPart) * (size_t)(h->sm_grid + h->short_grid)));
    SAP_TRY(dalloc(h, &h->d_smZr, sizeof(float) * (size_t)nhalf * K * 32));
    SAP_TRY(dalloc(h, &h->d_smZc, sizeof(float) * (size_t)nhalf * K * 64));
    SAP_TRY(dalloc(h, &h->d_smZ, sizeof(double) * (size_t)h->N * K));
    SAP_TRY(dalloc(h, &h->d_zpair, sizeof(double) * (size_t)std::max<int64_t>(h->nclose, 1) * K));
    SAP_TRY(dalloc(h, &h->d_smG, sizeof(double) * (size_t)h->sm_chunks * h->n * K));
    return SAP_OK;
}

static SmArgs sm_args(sap_ctx *h, double tau) {
    SmArgs a{};
    a.Y = h->d_smY;
    a.kp = h->kp;
    a.invd2 = h->d_invd2;
    a.tiles = h->d_tiles;
    a.nhalf = 2 * h->ntiles;
    a.npass = h->sm_grid;
    a.n = h->n;
    a.close = h->d_close;
    a.cd = h->d_cd;
    a.nclose = h->nclose;
    a.P64t = h->d_smP64t;
    a.vx = h->vec_x;
    a.vp = h->vec_p;
    a.gemm = h->cfg.gemm;
    a.tau = tau;
    a.c2 = (float)(1.4426950408889634 / tau);   // log2(e) / tau
    a.part = h->d_smpart;
    a.Lp = &h->d_st->sm_L;
    a.Zr = h->d_smZr;
    a.Zc = h->d_smZc;
    a.zpair = h->d_zpair;
    return a;
}

template <typename TX>
static sap_status sm_forward(sap_ctx *h, const float *P, double tau, float *loss) {
    const int K = h->k;
    const SmArgs a = sm_args(h, tau);
    const int gemm_blocks = (int)(h->Npad / 64);
    const int nshort = h->short_grid;
    const dim3 blk(kPairBlock);
    const TX *X = static_cast<const TX *>(h->X);
    SAP_TRY(launch(h, 5, "k_sm_loadP", k_sm_loadP, dim3((unsigned)ceil_div((int64_t)h->n * K, 256)),
                   dim3(256), 0, P, h->n, K, h->d_smP64t));
    SAP_DISPATCH_K(K, SAP_TRY(launch_with(h, 5, "k_sm_prep", dim3((unsigned)(gemm_blocks + nshort)), blk, 0,
                                          [&](const LaunchCfg &c) {
        return KLaunch<K, TX>::sm_prep(c, a, X, h->ldx, h->N, h->d_mu, h->d_smY, h->Npad, gemm_blocks, 0);
    })));
    SAP_DISPATCH_K(K, SAP_TRY(launch_with(h, 3, "k_sm_fwd", dim3((unsigned)h->sm_grid), blk, 0,
                                          [&](const LaunchCfg &c) { return KLaunch<K, TX>::sm_fwd(c, a); })));
    SAP_TRY(launch(h, 5, "k_sm_fin", k_sm_fin, dim3(1), blk, 0, (const SmPart *)h->d_smpart,
                   h->sm_grid + nshort, tau, loss, h->d_st));
    return SAP_OK;
}

template <typename TX>
static sap_status sm_backward(sap_ctx *h, double tau, const float *grad_loss, float *dP) {
    const int K = h->k;
    const SmArgs a = sm_args(h, tau);
    const int nshort = h->short_grid;
    const dim3 blk(kPairBlock);
    const TX *X = static_cast<const TX *>(h->X);
    if (nshort > 0)
        SAP_DISPATCH_K(K, SAP_TRY(launch_with(h, 5, "k_sm_prep", dim3((unsigned)nshort), blk, 0,
                                              [&](const LaunchCfg &c) {
            return KLaunch<K, TX>::sm_prep(c, a, X, h->ldx, h->N, h->d_mu, h->d_smY, h->Npad, 0, 1);
        })));
    SAP_DISPATCH_K(K, SAP_TRY(launch_with(h, 4, "k_sm_bwd", dim3((unsigned)h->sm_grid), blk, 0,
                                          [&](const LaunchCfg &c) { return KLaunch<K, TX>::sm_bwd(c, a); })));
    SAP_DISPATCH_K(K, SAP_TRY(launch_with(h, 5, "k_sm_zred", dim3((unsigned)h->nb), blk, 0,
                                          [&](const LaunchCfg &c) {
        return KLaunch<K, TX>::sm_zred(c, a, h->nb, h->N, h->d_rp_i, h->d_rp_j, h->d_permj, h->d_smZ);
    })));
    SAP_TRY(launch(h, 5, "k_sm_grad", k_sm_grad<TX>, dim3((unsigned)h->sm_chunks), dim3(256), 0,
                   X, h->ldx, h->N, h->n, K, (const double *)h->d_mu, (const double *)h->d_smZ,
                   h->sm_rows, h->d_smG));
    SAP_TRY(launch(h, 5, "k_sm_dP", k_sm_dP, dim3((unsigned)ceil_div((int64_t)h->n * K, 64)), dim3(256), 0,
                   (const double *)h->d_smG, h->sm_chunks, h->n, K, grad_loss, dP));
    return SAP_OK;
}

// ---------------------------------------------------------------- secant-PCA start

// Scratch of one PCA computation, freed on every exit path.
struct PcaScratch {
    std::vector<void *> ptrs;
    ~PcaScratch() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <typename T>
    hipError_t get(T **out, size_t bytes) {
        void *p = nullptr;
        const hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
        if (e == hipSuccess) ptrs.push_back(p);
        *out = static_cast<T *>(p);
        return e;
    }
};

template <typename TX>
static sap_status pca_run(sap_ctx *h, double *P_out, sap_pca_info *info, bool set_P) {
    const int n = h->n, k = h->k;
    const int64_t N = h->N, nb = ceil_div(N, kTile), ntiles = nb * (nb + 1) / 2;
    const int b = std::min(n, std::min(kPcaMaxB, std::max(k + 8, 2 * k)));
    const TX *X = static_cast<const TX *>(h->X);
    PcaScratch sc;
    int2 *d_tiles = nullptr;
    double *W = nullptr, *Z = nullptr, *Cm = nullptr, *Cs = nullptr, *V = nullptr, *T = nullptr, *out = nullptr,
           *P = nullptr;
    SAP_HIP(h, sc.get(&d_tiles, sizeof(int2) * ntiles));
    SAP_HIP(h, sc.get(&W, sizeof(double) * (size_t)ntiles * kTileElems));
    SAP_HIP(h, sc.get(&Z, sizeof(double) * (size_t)N * n));
    SAP_HIP(h, sc.get(&Cm, sizeof(double) * (size_t)n * n));
    SAP_HIP(h, sc.get(&Cs, sizeof(double) * (size_t)n * n));
    SAP_HIP(h, sc.get(&V, sizeof(double) * (size_t)n * b));
    SAP_HIP(h, sc.get(&T, sizeof(double) * (size_t)n * b));
    SAP_HIP(h, sc.get(&out, sizeof(double) * (kPcaMaxB + 1)));
    SAP_HIP(h, sc.get(&P, sizeof(double) * (size_t)n * k));
    std::vector<int2> tiles((size_t)ntiles);
    for (int64_t bi = 0, t = 0; bi < nb; ++bi)
        for (int64_t bj = bi; bj < nb; ++bj, ++t) tiles[(size_t)t] = make_int2((int)bi, (int)bj);
    SAP_HIP(h, hipMemcpyAsync(d_tiles, tiles.data(), sizeof(int2) * ntiles, hipMemcpyHostToDevice, h->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SAP_HIP(h, hipEventCreate(&e0));
    SAP_HIP(h, hipEventCreate(&e1));
    SAP_HIP(h, hipEventRecord(e0, h->stream));
    const unsigned gw = (unsigned)std::min<int64_t>(ntiles, 8192);
    hipLaunchKernelGGL(k_pca_w<TX>, dim3(gw), dim3(256), 0, h->stream, X, h->ldx, N, n, d_tiles, ntiles,
                       h->cfg.min_len, W);
    SAP_LAUNCHED(h, "k_pca_w");
    hipLaunchKernelGGL(k_pca_z<TX>, dim3((unsigned)nb, (unsigned)ceil_div(n, kTile)), dim3(256), 0, h->stream, X,
                       h->ldx, N, n, nb, (const double *)W, Z);
    SAP_LAUNCHED(h, "k_pca_z");
    const unsigned gn = (unsigned)ceil_div(n, kTile);
    hipLaunchKernelGGL(k_pca_gram<TX>, dim3(gn, gn), dim3(256), 0, h->stream, X, h->ldx, N, n,
                       (const double *)h->d_mu, (const double *)Z, Cm);
    SAP_LAUNCHED(h, "k_pca_gram");
    hipLaunchKernelGGL(k_pca_sym, dim3((unsigned)ceil_div((int64_t)n * n, 256)), dim3(256), 0, h->stream,
                       (const double *)Cm, n, Cs);
    SAP_LAUNCHED(h, "k_pca_sym");
    const dim3 gmv((unsigned)ceil_div((int64_t)n * b, 256));
    hipLaunchKernelGGL(k_pca_start, gmv, dim3(256), 0, h->stream, V, n, b);
    hipLaunchKernelGGL(k_pca_orth, dim3(1), dim3(256), 0, h->stream, V, n, b, 0);
    SAP_LAUNCHED(h, "k_pca_orth");
    double hout[kPcaMaxB + 1] = {0};
    int it = 0;
    bool conv = false;
    for (it = 1; it <= 400; ++it) {
        // two power steps, orthonormalisation, then the Rayleigh-Ritz check
        hipLaunchKernelGGL(k_pca_mv, gmv, dim3(256), 0, h->stream, (const double *)Cs, (const double *)V, n, b, T);
        hipLaunchKernelGGL(k_pca_mv, gmv, dim3(256), 0, h->stream, (const double *)Cs, (const double *)T, n, b, V);
        hipLaunchKernelGGL(k_pca_orth, dim3(1), dim3(256), 0, h->stream, V, n, b, it);
        hipLaunchKernelGGL(k_pca_mv, gmv, dim3(256), 0, h->stream, (const double *)Cs, (const double *)V, n, b, T);
        hipLaunchKernelGGL(k_pca_rr, dim3(1), dim3(256), 0, h->stream, V, T, n, b, k, out);
        SAP_LAUNCHED(h, "subspace iteration");
        SAP_HIP(h, hipMemcpyAsync(hout, out, sizeof(double) * (b + 1), hipMemcpyDeviceToHost, h->stream));
        SAP_HIP(h, hipStreamSynchronize(h->stream));
        if (hout[b] <= 1e-12) { conv = true; break; }
    }
    hipLaunchKernelGGL(k_pca_out, dim3(1), dim3(256), 0, h->stream, (const double *)V, n, b, k, P);
    SAP_LAUNCHED(h, "k_pca_out");
    SAP_HIP(h, hipEventRecord(e1, h->stream));
    if (P_out) SAP_HIP(h, hipMemcpyAsync(P_out, P, sizeof(double) * n * k, hipMemcpyDeviceToDevice, h->stream));
    SAP_HIP(h, hipStreamSynchronize(h->stream));
    float ms = 0.0f;
    SAP_HIP(h, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (info) {
        std::memset(info, 0, sizeof *info);
        for (int c = 0; c < k; ++c) info->sigma[c] = std::sqrt(std::max(hout[c], 0.0));
        info->residual = hout[b];
        info->ms = ms;
        info->iters = std::min(it, 400);
        info->converged = conv ? 1 : 0;
    }
    if (set_P) SAP_TRY(load_P(h, P));
    return SAP_OK;
}

// ---------------------------------------------------------------- C ABI// ---------------------------------------------------------------- C ABI

extern "C" {

sap_status sap_init(const sap_config *cfg, const void *X, int64_t ldx, const double *P0,
                    void *stream, sap_handle *out) {
    if (out) *out = nullptr;
    SAP_TRY(validate(cfg, ldx, X, P0, out));
    sap_ctx *h = new sap_ctx();
    h->cfg = *cfg;
    h->X = X;
    h->ldx = ldx;
    h->N = cfg->N;
    h->n = cfg->n;
    h->k = cfg->k;
    h->kp = cfg->k;
    h->p = cfg->N * (cfg->N - 1) / 2;
    {
        const size_t es = cfg->dtype == SAP_F64 ? 8 : 4;
        h->vec_x = (reinterpret_cast<uintptr_t>(X) % 16 == 0) && ((size_t)ldx * es) % 16 == 0;
        h->vec_p = cfg->n % 2 == 0;
    }
    h->stream = static_cast<hipStream_t>(stream);
    auto bail = [&](sap_status s) {
        g_tls_err = h->err.empty() ? g_tls_err : h->err;
        destroy_ctx(h);
        return s;
    };
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return bail(fail(h, SAP_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e)));
    sap_status s;
    if ((s = dalloc(h, &h->d_P64t, sizeof(double) * h->n * h->k)) != SAP_OK) return bail(s);
    if ((s = dalloc(h, &h->d_mu, sizeof(double) * h->n)) != SAP_OK) return bail(s);
    if ((s = dalloc(h, &h->d_st, sizeof(DevState))) != SAP_OK) return bail(s);
    if ((s = dalloc(h, &h->d_res, sizeof(DevResult))) != SAP_OK) return bail(s);
    if ((s = init_moments(h)) != SAP_OK) return bail(s);
    if ((s = (cfg->form == SAP_PLAIN ? init_plain(h) : init_fused(h))) != SAP_OK) return bail(s);
    if (h->kept == 0) return bail(fail(h, SAP_ERR_NO_PAIRS, "every pair is a duplicate or shorter than min_len"));
    if ((s = dalloc(h, &h->d_part, sizeof(Partial) * (size_t)(h->pass_grid + h->short_grid))) != SAP_OK)
        return bail(s);
    if (cfg->form == SAP_FUSED && (s = dalloc(h, &h->d_P64t_alt, sizeof(double) * h->n * h->k)) != SAP_OK)
        return bail(s);
    if ((s = load_P(h, P0)) != SAP_OK) return bail(s);
    // P, the update's two vectors and (k_selprep's GEMM) the column means
    h->tail_lds = sizeof(double) * ((size_t)h->k * h->n + 3 * (size_t)h->n);
    e = hipSuccess;
    SAP_DISPATCH_K(h->k, {
        e = KLaunch<K, float>::set_select_lds((int)h->tail_lds);
        if (e == hipSuccess) e = KLaunch<K, double>::set_select_lds((int)h->tail_lds);
    });
    if (e != hipSuccess) return bail(fail(h, SAP_ERR_DEVICE, "hipFuncSetAttribute: %s", hipGetErrorString(e)));
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return bail(fail(h, SAP_ERR_DEVICE, "init: %s", hipGetErrorString(e)));
    *out = h;
    return SAP_OK;
}

sap_status sap_min_secant(sap_handle h, sap_min_result *out) {
    SAP_TRY(usable(h));
    if (!out) return fail(h, SAP_ERR_INVALID_ARG, "null result pointer");
    SAP_TRY(enqueue_eval(h, 0, nullptr, nullptr, nullptr, 0));
    return read_result(h, out);
}

sap_status sap_step(sap_handle h, sap_min_result *out) {
    SAP_TRY(usable(h));
    SAP_TRY(enqueue_eval(h, 1, nullptr, nullptr, nullptr, 0));
    if (out) return read_result(h, out);
    return SAP_OK;
}

sap_status sap_run(sap_handle h, int32_t iters, double *min_trace, int64_t *ij_trace,
                   int32_t *cert_trace) {
    SAP_TRY(usable(h));
    if (iters < 0) return fail(h, SAP_ERR_INVALID_ARG, "iters must be >= 0");
    if (!min_trace) return fail(h, SAP_ERR_INVALID_ARG, "min_trace must not be NULL");
    if (h->cfg.dtype == SAP_F64) return launch_run<double>(h, iters, min_trace, ij_trace, cert_trace);
    return launch_run<float>(h, iters, min_trace, ij_trace, cert_trace);
}

sap_status sap_get_P(sap_handle h, double *P_out) {
    SAP_TRY(usable(h));
    if (!P_out) return fail(h, SAP_ERR_INVALID_ARG, "null P_out");
    hipLaunchKernelGGL(k_P_out, dim3((unsigned)ceil_div((int64_t)h->n * h->k, 256)), dim3(256), 0,
                       h->stream, h->d_P64t, h->n, h->k, P_out);
    SAP_LAUNCHED(h, "k_P_out");
    return SAP_OK;
}

sap_status sap_set_P(sap_handle h, const double *P) {
    SAP_TRY(usable(h));
    if (!P) return fail(h, SAP_ERR_INVALID_ARG, "null P");
    return load_P(h, P);
}

sap_status sap_pca_init(sap_handle h, double *P_out, sap_pca_info *info, int32_t set_P) {
    SAP_TRY(usable(h));
    if (h->cfg.dtype == SAP_F64) return pca_run<double>(h, P_out, info, set_P != 0);
    return pca_run<float>(h, P_out, info, set_P != 0);
}

sap_status sap_set_stream(sap_handle h, void *stream) {
    SAP_TRY(usable(h));
    h->stream = static_cast<hipStream_t>(stream);
    return SAP_OK;
}

sap_status sap_info(sap_handle h, sap_info_t *out) {
    SAP_TRY(usable(h));
    if (!out) return fail(h, SAP_ERR_INVALID_ARG, "null info pointer");
    SAP_HIP(h, hipStreamSynchronize(h->stream));
    out->n_pairs = h->kept;
    out->n_dropped = h->dropped;
    out->n_close = h->nclose;
    out->close_d = h->cfg.form == SAP_FUSED ? h->close_d : 0.0;
    out->e_abs = h->e_abs;
    out->e_rel = h->e_rel;
    out->radius = h->radius;
    if (h->cfg.form == SAP_FUSED)
        out->bytes_per_iter = (int64_t)h->ntiles * kTileElems * 4;
    else
        out->bytes_per_iter = (int64_t)h->n * h->pcols * (h->cfg.dtype == SAP_F64 ? 8 : 4);
    out->device_bytes = h->dev_bytes;
    out->n_tiles = h->cfg.form == SAP_FUSED ? h->ntiles : h->nchunks;
    return SAP_OK;
}

sap_status sap_softmin_fwd(sap_handle h, const float *P, double tau, float *loss) {
    SAP_TRY(usable(h));
    SAP_TRY(sm_check(h, P, tau));
    if (!loss) return fail(h, SAP_ERR_INVALID_ARG, "null loss pointer");
    SAP_TRY(sm_alloc(h));
    h->sm_ready = false;
    SAP_HIP(h, hipMemcpyAsync(h->d_smP32, P, sizeof(float) * h->n * h->k, hipMemcpyDeviceToDevice, h->stream));
    if (h->cfg.dtype == SAP_F64) SAP_TRY(sm_forward<double>(h, P, tau, loss));
    else SAP_TRY(sm_forward<float>(h, P, tau, loss));
    h->sm_ready = true;
    h->sm_tau = tau;
    return SAP_OK;
}

sap_status sap_softmin_bwd(sap_handle h, const float *P, double tau, const float *grad_loss,
                           float *dP) {
    SAP_TRY(usable(h));
    SAP_TRY(sm_check(h, P, tau));
    if (!grad_loss || !dP) return fail(h, SAP_ERR_INVALID_ARG, "null grad_loss or dP");
    if (!h->sm_ready || tau != h->sm_tau)
        return fail(h, SAP_ERR_INVALID_ARG, "sap_softmin_bwd must follow sap_softmin_fwd with the same tau");
    {
        // the gradient is that of the forward's P: P must be that projection
        // (compared bit for bit with the forward's copy)
        const size_t nk = (size_t)h->n * h->k;
        std::vector<float> a(nk), b(nk);
        SAP_HIP(h, hipMemcpyAsync(a.data(), P, sizeof(float) * nk, hipMemcpyDeviceToHost, h->stream));
        SAP_HIP(h, hipMemcpyAsync(b.data(), h->d_smP32, sizeof(float) * nk, hipMemcpyDeviceToHost, h->stream));
        SAP_HIP(h, hipStreamSynchronize(h->stream));
        if (std::memcmp(a.data(), b.data(), sizeof(float) * nk) != 0)
            return fail(h, SAP_ERR_INVALID_ARG,
                        "sap_softmin_bwd: P differs from the P of the latest sap_softmin_fwd");
    }
    if (h->cfg.dtype == SAP_F64) return sm_backward<double>(h, tau, grad_loss, dP);
    return sm_backward<float>(h, tau, grad_loss, dP);
}

sap_status sap_profile_enable(sap_handle h, int32_t on) {
    SAP_TRY(usable(h));
    h->prof_on = on != 0;
    return SAP_OK;
}

sap_status sap_profile_read(sap_handle h, sap_profile_t *out) {
    SAP_TRY(usable(h));
    if (!out) return fail(h, SAP_ERR_INVALID_ARG, "null profile pointer");
    SAP_HIP(h, hipStreamSynchronize(h->stream));
    std::memset(out, 0, sizeof *out);
    for (auto &m : h->marks) {
        float ms = 0.0f;
        SAP_HIP(h, hipEventElapsedTime(&ms, m.a, m.b));
        out->ms[m.slot] += ms;
        out->launches[m.slot] += 1;
        h->ev_pool.push_back(m.a);
        h->ev_pool.push_back(m.b);
    }
    h->marks.clear();
    return SAP_OK;
}

sap_status sap_destroy(sap_handle h) {
    if (!h) return SAP_OK;
    (void)hipSetDevice(h->device);
    if (!h->poisoned) (void)hipStreamSynchronize(h->stream);
    destroy_ctx(h);
    return SAP_OK;
}

const char *sap_last_error(sap_handle h) {
    if (h) return h->err.c_str();
    return g_tls_err.c_str();
}

}  // extern "C"
