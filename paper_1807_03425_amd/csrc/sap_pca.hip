// Algorithm 1's initial projection (Sec. 4, Algorithm 1 step 2): the first k
// columns of U in the SVD S = U Sigma V^T of the secant matrix S (every kept
// unit secant as a column), i.e. the top-k eigenvectors of
//     C = S S^T = sum_{kept i<j} s_ij s_ij^T,   sigma_c^2 = its eigenvalues,
// computed without forming S (gfx950, FP64 throughout):
//   k_pca_w     w_ij = 1/d_ij^2 for every kept pair (0 for dropped pairs,
//               i >= j and padding), by direct differences, 64 x 64 tiles;
//   k_pca_z     z_i = sum_j w_ij (x_i - x_j): the differences are formed
//               directly, never as deg_i x_i - (W X)_i, whose two terms cancel
//               on close pairs;
//   k_pca_gram  C = sum_i (x_i - mean) z_i^T (exact: sum_i z_i = 0, and
//               1/2 sum_ij w_ij (x_i - x_j)(x_i - x_j)^T = sum_i x_i z_i^T),
//               symmetrised;
//   subspace iteration on C with a block of b >= k vectors: products C V
//   (k_pca_mv), classical Gram-Schmidt applied twice (k_pca_orth), and a
//   Rayleigh-Ritz step (k_pca_rr: V^T C V diagonalised by a parallel cyclic
//   Jacobi) that reports the Ritz values and the residuals of the first k
//   Ritz vectors.
#include "sap_common.h"

namespace sap {

constexpr int kPcaMaxB = 32;   // subspace block size

// Sum of v[0..nv-1] over the block (256 threads), every thread gets the
// totals; sb: LDS scratch of 4 x kPcaMaxB doubles.  All threads call.
__device__ __forceinline__ void pca_block_sums(double *v, int nv, double *sb) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int e = 0; e < nv; ++e) {
        double t = v[e];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, kWave);
        if (lane == 0) sb[w * kPcaMaxB + e] = t;
    }
    __syncthreads();
    for (int e = 0; e < nv; ++e) v[e] = (sb[e] + sb[kPcaMaxB + e]) + (sb[2 * kPcaMaxB + e] + sb[3 * kPcaMaxB + e]);
    __syncthreads();
}

// 1/d^2 of every kept pair of tile t = (bi, bj), row-major 64 x 64 FP64;
// zero for dropped pairs (duplicates, d < min_len), i >= j and padding.
template <typename TX>
__global__ __launch_bounds__(256) void k_pca_w(const TX *__restrict__ X, int64_t ldx, int64_t N, int n,
                                               const int2 *__restrict__ tiles, int64_t ntiles, double min_len,
                                               double *__restrict__ W) {
    const int c = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int2 b = tiles[t];
        const int64_t j = (int64_t)b.y * kTile + c;
        const bool jin = j < N;
        const TX *xj = X + (jin ? j : N - 1) * ldx;
        for (int m = 0; m < 4; ++m) {
            const int g = w + 4 * m;
            const int64_t i0 = (int64_t)b.x * kTile + 4 * g;
            double d2[4] = {0.0, 0.0, 0.0, 0.0};
            if (jin) {
                for (int l = 0; l < n; ++l) {
                    const double xv = (double)xj[l];
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const int64_t i = i0 + rr < N ? i0 + rr : N - 1;
                        const double t2 = (double)X[i * ldx + l] - xv;
                        d2[rr] += t2 * t2;
                    }
                }
            }
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int64_t i = i0 + rr;
                double v = 0.0;
                if (jin && i < j) {
                    const double d = sqrt(d2[rr]);
                    if (!(d == 0.0 || d < min_len)) v = 1.0 / d2[rr];
                }
                W[t * kTileElems + (4 * g + rr) * kTile + c] = v;
            }
        }
    }
}

// z_i = sum_j w_ij (x_i - x_j) for the 64 rows of block I and the 64
// components of chunk ch: thread (r = tid / 4, u0 = (tid % 4) * 16) keeps
// z[r][u0 .. u0 + 15]; the loop runs over all column blocks J, with the
// w tile (transposed when J < I), X_I and X_J staged in LDS.
template <typename TX>
__global__ __launch_bounds__(256) void k_pca_z(const TX *__restrict__ X, int64_t ldx, int64_t N, int n, int64_t nb,
                                               const double *__restrict__ W, double *__restrict__ Z) {
    __shared__ double s_w[kTile][kTile + 1];
    __shared__ double s_xi[kTile][kTile + 1];
    __shared__ double s_xj[kTile][kTile + 1];
    const int64_t I = blockIdx.x;
    const int l0 = blockIdx.y * kTile;
    const int r = threadIdx.x >> 2, u0 = (threadIdx.x & 3) * 16;
    // X_I chunk
    for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
        const int rr = e / kTile, cc = e % kTile;
        const int64_t i = I * kTile + rr;
        s_xi[rr][cc] = (i < N && l0 + cc < n) ? (double)X[i * ldx + l0 + cc] : 0.0;
    }
    double z[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) z[u] = 0.0;
    for (int64_t J = 0; J < nb; ++J) {
        __syncthreads();
        const int64_t bi = I < J ? I : J, bj = I < J ? J : I;
        const double *T = W + (bi * nb - bi * (bi - 1) / 2 + (bj - bi)) * kTileElems;
        for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
            const int a = e / kTile, b = e % kTile;   // tile element (a, b): pair (64 bi + a, 64 bj + b)
            const double v = T[e];
            if (I < J) {
                s_w[a][b] = v;                         // w(I*64 + a, J*64 + b)
            } else if (I > J) {
                s_w[b][a] = v;                         // w(I*64 + b, J*64 + a)
            } else {
                if (a < b) { s_w[a][b] = v; s_w[b][a] = v; }
                else if (a == b) s_w[a][a] = 0.0;
            }
            const int64_t j = J * kTile + a;
            s_xj[a][b] = (j < N && l0 + b < n) ? (double)X[j * ldx + l0 + b] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int j = 0; j < kTile; ++j) {
            const double wv = s_w[r][j];
#pragma unroll
            for (int u = 0; u < 16; ++u) z[u] = __builtin_fma(wv, s_xi[r][u0 + u] - s_xj[j][u0 + u], z[u]);
        }
    }
    const int64_t i = I * kTile + r;
    if (i < N) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (l0 + u0 + u < n) Z[i * n + l0 + u0 + u] = z[u];
    }
}

// C[a][b] = sum_i (x_ia - mu_a) z_ib over all rows, for the 64 x 64 tile
// (blockIdx.x, blockIdx.y) of C (row-major n x n, unsymmetrised).
template <typename TX>
__global__ __launch_bounds__(256) void k_pca_gram(const TX *__restrict__ X, int64_t ldx, int64_t N, int n,
                                                  const double *__restrict__ mu, const double *__restrict__ Z,
                                                  double *__restrict__ Cm) {
    __shared__ double s_x[kTile][kTile + 1];
    __shared__ double s_z[kTile][kTile + 1];
    const int a0 = blockIdx.x * kTile, b0 = blockIdx.y * kTile;
    const int r = threadIdx.x >> 2, u0 = (threadIdx.x & 3) * 16;
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int64_t i0 = 0; i0 < N; i0 += kTile) {
        __syncthreads();
        for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
            const int rr = e / kTile, cc = e % kTile;
            const int64_t i = i0 + rr;
            const bool ok = i < N;
            s_x[rr][cc] = (ok && a0 + cc < n) ? (double)X[i * ldx + a0 + cc] - mu[a0 + cc] : 0.0;
            s_z[rr][cc] = (ok && b0 + cc < n) ? Z[i * n + b0 + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < kTile; ++rr) {
            const double xv = s_x[rr][r];
#pragma unroll
            for (int u = 0; u < 16; ++u) acc[u] = __builtin_fma(xv, s_z[rr][u0 + u], acc[u]);
        }
    }
    if (a0 + r < n) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (b0 + u0 + u < n) Cm[(int64_t)(a0 + r) * n + b0 + u0 + u] = acc[u];
    }
}

// C <- (C + C^T) / 2 into Cs.
__global__ void k_pca_sym(const double *__restrict__ Cm, int n, double *__restrict__ Cs) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int a = (int)(e / n), b = (int)(e % n);
    Cs[e] = 0.5 * (Cm[e] + Cm[(int64_t)b * n + a]);
}

// Deterministic start block (n x b row-major), entries in [-1, 1) from a
// counter hash (splitmix64 of the element index).
__device__ __forceinline__ double pca_hash(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void k_pca_start(double *__restrict__ V, int n, int b) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n * b) V[e] = pca_hash((uint64_t)e);
}

// Wout = C V (n x n times n x b, row-major): thread per output element.
__global__ __launch_bounds__(256) void k_pca_mv(const double *__restrict__ Cs, const double *__restrict__ V, int n,
                                                int b, double *__restrict__ Wout) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * b) return;
    const int l = (int)(e / b), c = (int)(e % b);
    const double *crow = Cs + (int64_t)l * n;
    double acc = 0.0;
    for (int m = 0; m < n; ++m) acc = __builtin_fma(crow[m], V[(int64_t)m * b + c], acc);
    Wout[e] = acc;
}

// Orthonormalise the b columns of V (n x b row-major) in place: classical
// Gram-Schmidt, twice per column; a column that cancels to below 1e-10 of
// its norm is replaced by a hashed vector and orthogonalised again.  One
// block of 256 threads.
__global__ __launch_bounds__(256) void k_pca_orth(double *__restrict__ V, int n, int b, int seed) {
    __shared__ double sb[4 * kPcaMaxB];
    for (int c = 0; c < b; ++c) {
        for (int attempt = 0; attempt < 2; ++attempt) {
            double nrm0;
            {
                double v[1] = {0.0};
                for (int l = threadIdx.x; l < n; l += 256) v[0] = __builtin_fma(V[l * b + c], V[l * b + c], v[0]);
                pca_block_sums(v, 1, sb);
                nrm0 = sqrt(v[0]);
            }
            for (int pass = 0; pass < 2; ++pass) {
                double d[kPcaMaxB];
                for (int a = 0; a < c; ++a) d[a] = 0.0;
                for (int l = threadIdx.x; l < n; l += 256) {
                    const double x = V[l * b + c];
                    for (int a = 0; a < c; ++a) d[a] = __builtin_fma(V[l * b + a], x, d[a]);
                }
                pca_block_sums(d, c, sb);
                for (int l = threadIdx.x; l < n; l += 256) {
                    double x = V[l * b + c];
                    for (int a = 0; a < c; ++a) x -= d[a] * V[l * b + a];
                    V[l * b + c] = x;
                }
                __syncthreads();
            }
            double v[1] = {0.0};
            for (int l = threadIdx.x; l < n; l += 256) v[0] = __builtin_fma(V[l * b + c], V[l * b + c], v[0]);
            pca_block_sums(v, 1, sb);
            const double nrm = sqrt(v[0]);
            if (nrm > 1e-10 * nrm0 && nrm > 1e-300) {
                for (int l = threadIdx.x; l < n; l += 256) V[l * b + c] = V[l * b + c] / nrm;
                __syncthreads();
                break;
            }
            // lost to cancellation: a fresh direction (the loop orthogonalises it)
            for (int l = threadIdx.x; l < n; l += 256)
                V[l * b + c] = pca_hash(0x51A9ull + (uint64_t)seed * 7919ull + (uint64_t)(c * n + l) * 131ull);
            __syncthreads();
        }
    }
}

// Rayleigh-Ritz on the orthonormal V with W = C V: H = (V^T W + W^T V) / 2
// (b x b), diagonalised by a parallel cyclic Jacobi (round-robin pairs, b/2
// rotations per step), Ritz values sorted descending, V <- V Q, W <- W Q,
// and out[0..b) = Ritz values, out[b] = max_{c<k} ||W_c - theta_c V_c|| /
// theta_0.  One block of 256 threads.
__global__ __launch_bounds__(256) void k_pca_rr(double *__restrict__ V, double *__restrict__ W, int n, int b, int k,
                                                double *__restrict__ out) {
    __shared__ double A[kPcaMaxB][kPcaMaxB + 1];
    __shared__ double Q[kPcaMaxB][kPcaMaxB + 1];
    __shared__ double rot[kPcaMaxB / 2][2];
    __shared__ int rpq[kPcaMaxB / 2][2];
    __shared__ int perm[kPcaMaxB];
    __shared__ double theta[kPcaMaxB];
    __shared__ double sb[4 * kPcaMaxB];
    __shared__ double s_off;
    const int bp = b + (b & 1);   // even number of players; the pad has A = 0
    // H, one entry per thread (b <= 32: at most 528 entries)
    for (int e = threadIdx.x; e < bp * bp; e += 256) {
        const int a = e / bp, c = e % bp;
        double h = 0.0;
        if (a < b && c < b && a <= c) {
            double s1 = 0.0, s2 = 0.0;
            for (int l = 0; l < n; ++l) {
                s1 = __builtin_fma(V[l * b + a], W[l * b + c], s1);
                s2 = __builtin_fma(W[l * b + a], V[l * b + c], s2);
            }
            h = 0.5 * (s1 + s2);
        }
        if (a <= c) { A[a][c] = h; A[c][a] = h; }
        Q[a][c] = a == c ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 30; ++sweep) {
        if (threadIdx.x == 0) {
            double off = 0.0, dia = 0.0;
            for (int p = 0; p < bp; ++p) {
                dia += A[p][p] * A[p][p];
                for (int q = p + 1; q < bp; ++q) off += A[p][q] * A[p][q];
            }
            s_off = off <= 1e-32 * dia ? -1.0 : off;
        }
        __syncthreads();
        if (s_off < 0.0) break;
        for (int step = 0; step < bp - 1; ++step) {
            if (threadIdx.x < bp / 2) {
                const int m = threadIdx.x;
                const int pa = m == 0 ? 0 : ((m - 1 + step) % (bp - 1)) + 1;
                const int mq = bp - 1 - m;
                const int pb = ((mq - 1 + step) % (bp - 1)) + 1;
                const int p = min(pa, pb), q = max(pa, pb);
                const double apq = A[p][q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                rot[m][0] = c; rot[m][1] = s;
                rpq[m][0] = p; rpq[m][1] = q;
            }
            __syncthreads();
            // rows p, q of A  (A <- J^T A)
            for (int e = threadIdx.x; e < (bp / 2) * bp; e += 256) {
                const int m = e / bp, j = e % bp;
                const int p = rpq[m][0], q = rpq[m][1];
                const double c = rot[m][0], s = rot[m][1];
                const double ap = A[p][j], aq = A[q][j];
                A[p][j] = c * ap - s * aq;
                A[q][j] = s * ap + c * aq;
            }
            __syncthreads();
            // columns p, q of A and of Q  (A <- A J, Q <- Q J)
            for (int e = threadIdx.x; e < (bp / 2) * bp; e += 256) {
                const int m = e / bp, i = e % bp;
                const int p = rpq[m][0], q = rpq[m][1];
                const double c = rot[m][0], s = rot[m][1];
                const double ap = A[i][p], aq = A[i][q];
                A[i][p] = c * ap - s * aq;
                A[i][q] = s * ap + c * aq;
                const double qp = Q[i][p], qq = Q[i][q];
                Q[i][p] = c * qp - s * qq;
                Q[i][q] = s * qp + c * qq;
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        // sort the b real Ritz values descending (the pad is excluded)
        for (int c = 0; c < b; ++c) perm[c] = c;
        for (int c = 0; c < b; ++c) {
            int best = c;
            for (int d = c + 1; d < b; ++d)
                if (A[perm[d]][perm[d]] > A[perm[best]][perm[best]]) best = d;
            const int t = perm[c]; perm[c] = perm[best]; perm[best] = t;
        }
        for (int c = 0; c < b; ++c) theta[c] = A[perm[c]][perm[c]];
    }
    __syncthreads();
    // V <- V Q, W <- W Q (each thread rewrites whole rows it owns)
    for (int l = threadIdx.x; l < n; l += 256) {
        double vr[kPcaMaxB], wr[kPcaMaxB];
        for (int a = 0; a < b; ++a) { vr[a] = V[l * b + a]; wr[a] = W[l * b + a]; }
        for (int c = 0; c < b; ++c) {
            double sv = 0.0, sw = 0.0;
            const int pc = perm[c];
            for (int a = 0; a < b; ++a) {
                sv = __builtin_fma(vr[a], Q[a][pc], sv);
                sw = __builtin_fma(wr[a], Q[a][pc], sw);
            }
            V[l * b + c] = sv;
            W[l * b + c] = sw;
        }
    }
    __syncthreads();
    // residuals of the first k Ritz pairs
    double res[kPcaMaxB];
    for (int c = 0; c < k; ++c) res[c] = 0.0;
    for (int l = threadIdx.x; l < n; l += 256)
        for (int c = 0; c < k; ++c) {
            const double d = W[l * b + c] - theta[c] * V[l * b + c];
            res[c] = __builtin_fma(d, d, res[c]);
        }
    pca_block_sums(res, k, sb);
    if (threadIdx.x == 0) {
        double mx = 0.0;
        for (int c = 0; c < k; ++c) mx = fmax(mx, sqrt(res[c]));
        for (int c = 0; c < b; ++c) out[c] = theta[c];
        out[b] = theta[0] > 0.0 ? mx / theta[0] : 0.0;
    }
}

// P (n x k row-major) from the first k columns of V (n x b), each column's
// largest-magnitude component made positive (the first on ties).  One block.
__global__ __launch_bounds__(256) void k_pca_out(const double *__restrict__ V, int n, int b, int k,
                                                 double *__restrict__ P) {
    __shared__ double sgn[kPcaMaxB];
    if (threadIdx.x < k) {
        const int c = threadIdx.x;
        int t = 0;
        double mx = -1.0;
        for (int l = 0; l < n; ++l)
            if (fabs(V[l * b + c]) > mx) { mx = fabs(V[l * b + c]); t = l; }
        sgn[c] = V[t * b + c] < 0.0 ? -1.0 : 1.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n * k; e += 256) {
        const int l = e / k, c = e % k;
        P[e] = sgn[c] * V[l * b + c];
    }
}

}  // namespace sap
