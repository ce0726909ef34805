// Dense FP64 building blocks for the randomized SVD (Algorithm 1) around the
// projection: CholeskyQR2 (Gram matrix, Cholesky, triangular inverse, Q =
// Y R^-1) and the small SVD (one-sided Jacobi).  The paper uses cuSOLVER for
// these steps (Sec. 5.1); here they are hand-written HIP kernels, FP64
// throughout (the Gram of the skinny Y is formed in FP64 from FP32 data).
//
// * gemm_acc64: C = alpha * op(A) op(B) (+ beta C) with arbitrary row/column
//   strides for every operand, FP64 products on v_mfma_f64_16x16x4f64, 64x64
//   output tiles staged through LDS in 16-deep slices; deterministic (fixed
//   summation order).
// * Cholesky (lower, in place): blocked right-looking, 64-wide blocks: the
//   diagonal block is factored in LDS by one workgroup, the panel below is
//   solved against it, the trailing matrix is updated with gemm_acc64.  A
//   non-positive pivot sets the NOT_SPD status bit and the factorization
//   continues on |pivot| so that every kernel still completes.
// * Inverse of a lower-triangular L: blocked; diagonal blocks inverted in LDS,
//   off-diagonal blocks X_ij = -X_ii (sum_{j<=l<i} L_il X_lj) row block by row
//   block with gemm_acc64.
// * One-sided Jacobi SVD of a small square matrix, parallel over column
//   pairs (round-robin ordering, one launch per round, rotation angles from
//   the 2x2 Gram of each pair, convergence when no pair has a relative
//   off-diagonal above the tolerance in a whole sweep).
// * C = A^T Q on FP32 MFMA; Gram products split along the contraction.
#include "rpmi_internal.h"
#include "gemm64_tile.h"

namespace rpmi {
namespace {

constexpr int GT = kG64Tile;   // output tile
constexpr int GK = kG64K;     // contraction slice
constexpr int NB = 64;      // block size of the factorizations
constexpr int kJacobiWavePairs = 2048;   // pairs per round from which a wave per pair is faster

template <class T>
__device__ __forceinline__ double ld(const T* p) { return (double)*p; }

// C[i][j] = alpha * sum_k A(i,k) B(k,j) + beta * C[i][j] on FP64 MFMA (one
// 64 x 64 tile per workgroup, gemm64_tile.h), batched over blockIdx.z:
// problem z uses a + z*sab, b + z*sbb, c + z*scb.
template <class TA, class TB, class TC>
__global__ __launch_bounds__(256) void gemm_acc64_kernel(
    int64_t M, int64_t N, int64_t K, double alpha, const TA* __restrict__ a, int64_t sam, int64_t sak,
    const TB* __restrict__ b, int64_t sbk, int64_t sbn, double beta, TC* __restrict__ c, int64_t scm,
    int64_t scn, int64_t sab, int64_t sbb, int64_t scb) {
    gemm64_tile<TA, TB, TC>(M, N, K, alpha, a + blockIdx.z * sab, sam, sak, b + blockIdx.z * sbb, sbk, sbn, beta,
                            c + blockIdx.z * scb, scm, scn, blockIdx.y * (int64_t)GT, blockIdx.x * (int64_t)GT);
}

// the same tiling in FP32 (FP32 MFMA, FP32 accumulation)
template <class TA, class TB, class TC>
__global__ __launch_bounds__(256) void gemm_f32_kernel(
    int64_t M, int64_t N, int64_t K, double alpha, const TA* __restrict__ a, int64_t sam, int64_t sak,
    const TB* __restrict__ b, int64_t sbk, int64_t sbn, double beta, TC* __restrict__ c, int64_t scm,
    int64_t scn, int64_t sab, int64_t sbb, int64_t scb) {
    gemm64_tile<TA, TB, TC, false, true>(M, N, K, alpha, a + blockIdx.z * sab, sam, sak, b + blockIdx.z * sbb, sbk,
                                         sbn, beta, c + blockIdx.z * scb, scm, scn, blockIdx.y * (int64_t)GT,
                                         blockIdx.x * (int64_t)GT);
}

// ---------------------------------------------------------------- Cholesky
// The nb x nb diagonal block at (k, k), nb <= NB, factored in place in LDS by
// one workgroup, right-looking: step j takes the pivot, scales column j and
// updates the trailing triangle, each wave whole rows of it (lane l column
// j + 1 + l), so a step is a few instructions per lane between barriers.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* A, int64_t lda, int64_t k, int nb,
                                                         unsigned int* status) {
    __shared__ double T[NB][NB + 1];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    for (int e = tid; e < nb * nb; e += 256) {
        const int i = e / nb, l = e % nb;
        T[i][l] = l <= i ? A[(k + i) * lda + k + l] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        double v = T[j][j];
        if (!(v > 0.0)) {                            // breakdown (or NaN): record, keep going
            if (tid == 0) atomicOr(status, kStatusNotSpd);
            v = fabs(v) > 0.0 ? fabs(v) : 1.0;
        }
        const double d = sqrt(v);
        __syncthreads();                             // T[j][j] read by every thread before it changes
        if (tid >= j && tid < nb) T[tid][j] = tid == j ? d : T[tid][j] / d;
        __syncthreads();
        const int l = j + 1 + tx;
        const double llj = l < nb ? T[l][j] : 0.0;
        for (int i = j + 1 + ty; i < nb; i += 4)
            if (l <= i) T[i][l] = T[i][l] - T[i][j] * llj;
        __syncthreads();
    }
    for (int e = tid; e < nb * nb; e += 256) {
        const int i = e / nb, l = e % nb;
        A[(k + i) * lda + k + l] = l <= i ? T[i][l] : 0.0;
    }
}

// Rows [k+nb, p) of block column k: X <- X L_kk^-T, one workgroup per 64
// rows with L_kk and the rows in LDS.  Right-looking: step j divides column j
// by L[j][j] (lane r: row r), then the four waves take the later columns in
// turn (x_l -= x_j L[l][j]), so each x_l receives its terms in the order
// l' = 0, 1, .. of the row-by-row substitution.
__global__ __launch_bounds__(256) void trsm_panel_kernel(double* A, int64_t lda, int64_t k, int nb,
                                                         int64_t p) {
    __shared__ double L[NB][NB + 1];
    __shared__ double X[64][NB + 1];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int64_t r0 = k + nb + blockIdx.x * 64;
    const int rows = (int)(p - r0 < 64 ? p - r0 : 64);
    for (int e = tid; e < nb * nb; e += 256) L[e / nb][e % nb] = A[(k + e / nb) * lda + k + e % nb];
    for (int e = tid; e < rows * nb; e += 256) X[e / nb][e % nb] = A[(r0 + e / nb) * lda + k + e % nb];
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (tid < rows) X[tid][j] = X[tid][j] / L[j][j];
        __syncthreads();
        if (tx < rows) {
            const double xj = X[tx][j];
            for (int l = j + 1 + ty; l < nb; l += 4) X[tx][l] = X[tx][l] - xj * L[l][j];
        }
        __syncthreads();
    }
    for (int e = tid; e < rows * nb; e += 256) A[(r0 + e / nb) * lda + k + e % nb] = X[e / nb][e % nb];
}

// ------------------------------------------------------- triangular inverse
// Invert each nb x nb diagonal block of lower-triangular L into X (one
// workgroup per block; column-wise forward substitution in LDS).
__global__ __launch_bounds__(256) void trtri_diag_kernel(const double* L, int64_t ldl, double* X,
                                                         int64_t ldx, int64_t p) {
    __shared__ double T[NB][NB + 1];
    __shared__ double V[NB][NB + 1];
    const int tid = threadIdx.x;
    const int64_t k = blockIdx.x * (int64_t)NB;
    const int nb = (int)(p - k < NB ? p - k : NB);
    for (int e = tid; e < nb * nb; e += 256) {
        T[e / nb][e % nb] = L[(k + e / nb) * ldl + k + e % nb];
        V[e / nb][e % nb] = 0.0;
    }
    __syncthreads();
    // column c of the inverse solves T v = e_c
    if (tid < nb) {
        const int cidx = tid;
        for (int i = cidx; i < nb; ++i) {
            double s = i == cidx ? 1.0 : 0.0;
            for (int l = cidx; l < i; ++l) s -= T[i][l] * V[l][cidx];
            V[i][cidx] = s / T[i][i];
        }
    }
    __syncthreads();
    for (int e = tid; e < nb * nb; e += 256) X[(k + e / nb) * ldx + k + e % nb] = V[e / nb][e % nb];
}

// Block row i of the inverse: X[i, 0:r0] currently holds T = L[i, 0:r0]
// X[0:r0, 0:r0]; replace it by -X_ii T.  One workgroup per 64-column chunk;
// X_ii and the chunk of T are staged in LDS.
__global__ __launch_bounds__(256) void trtri_apply_diag_kernel(double* X, int64_t ldx, int64_t r0, int rows) {
    __shared__ double D[NB][NB + 1];
    __shared__ double T[NB][NB + 1];
    const int tid = threadIdx.x;
    const int64_t c0 = blockIdx.x * (int64_t)NB;
    const int cols = (int)(r0 - c0 < NB ? r0 - c0 : NB);
    for (int e = tid; e < rows * rows; e += 256) D[e / rows][e % rows] = X[(r0 + e / rows) * ldx + r0 + e % rows];
    for (int e = tid; e < rows * cols; e += 256) T[e / cols][e % cols] = X[(r0 + e / cols) * ldx + c0 + e % cols];
    __syncthreads();
    for (int e = tid; e < rows * cols; e += 256) {
        const int i = e / cols, j = e % cols;
        double acc = 0.0;
        for (int l = 0; l <= i; ++l) acc += D[i][l] * T[l][j];
        X[(r0 + i) * ldx + c0 + j] = -acc;
    }
}

// Zero the strictly upper part of a p x p matrix (so that it is exactly lower).
__global__ void zero_upper_kernel(double* A, int64_t lda, int64_t p) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < p * p; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / p, j = e % p;
        if (j > i) A[i * lda + j] = 0.0;
    }
}


// G = sum over z of the split partials, in the fixed order z = 0, 1, ...
// One part z of G = Y^T Y (p x p, FP64) over contraction rows [z Kc, (z+1) Kc):
// block x enumerates the tiles (ti, tj), ti <= tj, of the upper triangle; each
// tile is written with its mirror.  out + z p^2 receives the part.
template <class T>
__global__ __launch_bounds__(256) void gram_sym_kernel(int64_t p, int64_t K, int64_t Kc, const T* Y, int64_t ldy,
                                                       double* out) {
    const int64_t nt = (p + GT - 1) / GT;
    int64_t t = blockIdx.x, ti = 0;
    while (t >= nt - ti) { t -= nt - ti; ++ti; }
    const int64_t tj = ti + t;
    const int64_t z = blockIdx.y, k0 = z * Kc;
    const int64_t kz = K - k0 < Kc ? K - k0 : Kc;
    const T* a = Y + k0 * ldy;
    gemm64_tile<T, T, double, true>(p, p, kz, 1.0, a, 1, ldy, a, ldy, 1, 0.0, out + z * p * p, p, 1, ti * GT, tj * GT);
}

__global__ void sum_partials_kernel(const double* __restrict__ part, int64_t count, int nsplit, double* __restrict__ G) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
        double acc = part[e];
        for (int z = 1; z < nsplit; ++z) acc += part[(int64_t)z * count + e];
        G[e] = acc;
    }
}

// ---------------------------------------------------------------- C = A^T Q on FP32 MFMA
// C (N x P, row-major, ldc) = A^T Q for A (K x N, row-major, lda) and Q
// (K x P, row-major, ldq), FP32 products with FP32 accumulation on
// v_mfma_f32_16x16x4f32 (lane 16g + c supplies A^T[c][g] and Q[g][c] of a
// 16 x 4 / 4 x 16 step).  A wave owns 64 rows x 64 columns of C as 4 x 4
// MFMA tiles with permuted rows and columns: row r of tile t is C row
// 4r + t of the wave's block (columns alike), so that lane c reads the four
// tiles' operands with one 16-byte load of 4 consecutive elements of a row
// of A (of Q).  Four waves take four consecutive 64-row blocks.  Requires
// lda, ldq, ldc multiples of 4 and 16-byte aligned A, Q and C.
__global__ __launch_bounds__(256) void gemm_tn_f32_kernel(int64_t N, int64_t P, int64_t K, const float* __restrict__ A,
                                                          int64_t lda, const float* __restrict__ Q, int64_t ldq,
                                                          float* __restrict__ C, int64_t ldc) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int64_t i0 = (blockIdx.y * 4 + wave) * 64, j0 = blockIdx.x * (int64_t)64;
    const int64_t ia = i0 + 4 * c, jq = j0 + 4 * c;       // this lane's 4 rows of C (tiles 0..3), 4 columns
    const bool a_full = ia + 3 < N, q_full = jq + 3 < P;
    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    auto load4 = [](const float* row, int64_t col, int64_t lim, bool full) -> f4 {
        if (full) return *reinterpret_cast<const f4*>(row + col);
        f4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = col + e < lim ? row[col + e] : 0.0f;
        return v;
    };
    for (int64_t k0 = 0; k0 < K; k0 += 16) {
        f4 av[4], qv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {                      // k = k0 + 4u + g
            const int64_t k = k0 + 4 * u + g;
            const bool in = k < K;
            av[u] = in ? load4(A + k * lda, ia, N, a_full) : f4{0.f, 0.f, 0.f, 0.f};
            qv[u] = in ? load4(Q + k * ldq, jq, P, q_full) : f4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u][a], qv[u][b], acc[a][b], 0, 0, 0);
    }
    // lane (g, c) holds D[4g + e][c] of tile (a, b): C row i0 + 4 (4g + e) + a, column j0 + 4c + b
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t i = i0 + 4 * (4 * g + e) + a;
            if (i >= N) continue;
            float* crow = C + i * ldc;
            if (q_full) {
                *reinterpret_cast<f4*>(crow + jq) = f4{acc[a][0][e], acc[a][1][e], acc[a][2][e], acc[a][3][e]};
            } else {
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (jq + b < P) crow[jq + b] = acc[a][b][e];
            }
        }
}

// ---------------------------------------------------------------- parallel one-sided Jacobi
// Many workgroups per round: one workgroup per column pair, one launch per
// round of the round-robin (circle) ordering, so that a sweep streams the
// columns at full-chip bandwidth instead of through one compute unit.  W and
// V are held column-major during the iteration (column j contiguous).  Per
// problem, flags[0] = converged, flags[1 + (sweep & 1)] = a rotation happened
// in that sweep, flags[3] = sweeps done.  Every kernel of a converged problem
// returns at once.
__global__ void jacobi_prep_kernel(const JacobiProb* tab) {
    const JacobiProb P = tab[blockIdx.y];
    const int n = P.n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / n), j = (int)(e % n);
        if (r < j) {                                  // transpose W in place: row-major -> column-major
            const double t = P.W[(int64_t)r * n + j];
            P.W[(int64_t)r * n + j] = P.W[(int64_t)j * n + r];
            P.W[(int64_t)j * n + r] = t;
        }
        P.V[e] = r == j ? 1.0 : 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x < 4) P.flags[threadIdx.x] = 0;
}

__device__ __forceinline__ double block_sum256(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// One round of the parallel one-sided Jacobi SVD.  WAVE = false: one
// workgroup per column pair, the pair's three dot products reduced over 256
// threads (about 2.5 rows per thread at n = 640, which keeps a round
// latency-short: 5.8 us at n = 640 against 10.3 us for one wave per pair).
// WAVE = true: one wave per pair, four pairs per workgroup, reduced within
// the wave with no workgroup barrier (faster when a round has thousands of
// pairs, as in the batched RSVD).
template <bool WAVE>
__global__ __launch_bounds__(256) void jacobi_round_kernel(const JacobiProb* tab, int count, int total_pairs,
                                                           int round, int sweep, double tol) {
    constexpr int STRIDE = WAVE ? 64 : 256;
    const int t0 = WAVE ? (threadIdx.x & 63) : threadIdx.x;
    const int b = WAVE ? blockIdx.x * 4 + (threadIdx.x >> 6) : blockIdx.x;
    if (b >= total_pairs) return;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].pair_start <= b) lo = mid;
        else hi = mid - 1;
    }
    const JacobiProb P = tab[lo];
    const int n = P.n, m = n + (n & 1);
    if (round >= m - 1 || P.flags[0]) return;
    const int k = b - P.pair_start;                   // pair k: positions k and m - 1 - k
    // circle method: position 0 holds player 0, position i >= 1 holds
    // 1 + ((i - 1 + round) mod (m - 1))
    auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (m - 1); };
    int a = player(k), c = player(m - 1 - k);
    if (a > c) { const int t = a; a = c; c = t; }
    if (c >= n) return;                               // the dummy of an odd n
    double* wa = P.W + (int64_t)a * n;
    double* wc = P.W + (int64_t)c * n;
    double* va = P.V + (int64_t)a * n;
    double* vc = P.V + (int64_t)c * n;
    // all four columns' elements of this thread in registers at once (n <=
    // 1024): one memory round trip before the reduction, none after it
    constexpr int PER = 1024 / STRIDE;
    double x[PER], y[PER], vx[PER], vy[PER];
    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int r = t0 + u * STRIDE;
        const bool in = r < n;
        x[u] = in ? wa[r] : 0.0;
        y[u] = in ? wc[r] : 0.0;
        vx[u] = in ? va[r] : 0.0;
        vy[u] = in ? vc[r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        al += x[u] * x[u]; be += y[u] * y[u]; ga += x[u] * y[u];
    }
    if constexpr (WAVE) {
        // butterfly: every lane ends with the same bits, so the lanes agree
        for (int off = 32; off > 0; off >>= 1) {
            al += __shfl_xor(al, off, 64);
            be += __shfl_xor(be, off, 64);
            ga += __shfl_xor(ga, off, 64);
        }
    } else {
        __shared__ double red[3][4];
        al = block_sum256(al, red[0]);
        be = block_sum256(be, red[1]);
        ga = block_sum256(ga, red[2]);
    }
    if (!(fabs(ga) > tol * sqrt(al * be)) || ga == 0.0) return;
    // the rotation that zeroes the off-diagonal of the pair's 2x2 Gram
    const double zeta = (be - al) / (2.0 * ga);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int r = t0 + u * STRIDE;
        if (r < n) {
            wa[r] = cs * x[u] - sn * y[u];
            wc[r] = sn * x[u] + cs * y[u];
            va[r] = cs * vx[u] - sn * vy[u];
            vc[r] = sn * vx[u] + cs * vy[u];
        }
    }
    if (t0 == 0) P.flags[1 + (sweep & 1)] = 1;
}

// One round of the block form of the one-sided Jacobi SVD: the columns are
// grouped in blocks of kJacobiBlock, the blocks are paired by the same
// round-robin ordering, and one workgroup takes a pair of blocks (up to 16
// columns of length n): it forms their 16 x 16 Gram H on FP64 MFMA, runs one
// cyclic sweep of the rotations of Algorithm 1's SVD on H (each rotation the
// one that zeroes H[p][q], as the column form computes it from the same dot
// products), accumulating them in Qm, and applies Qm to the block's columns
// of W and V.  Every pair of columns meets within some block pair in every
// sweep, so a sweep does at least the rotations of a column sweep, with
// p / 8 - 1 launches instead of p - 1.  A block paired with the padding block
// (odd block count) or a partial last block just has fewer columns.
// base[vid[i] n + r] = sum_j Qm[i][j] x[u][j] for the rows r = tid + 256 u < n
template <int JV, int NR>
__device__ __forceinline__ void jacobi_apply_rows(const double (&Qm)[JV][JV + 1], const int (&vid)[JV],
                                                  const double (&x)[NR][JV], double* base, int n, int tid) {
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const int r = tid + 256 * u;
        if (r >= n) continue;
#pragma unroll
        for (int i = 0; i < JV; ++i) {
            if (vid[i] < 0) continue;
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < JV; ++j) acc += Qm[i][j] * x[u][j];
            base[(int64_t)vid[i] * n + r] = acc;
        }
    }
}

// NR: rows per thread of the W and V updates (n <= 256 NR)
template <int NR>
__global__ __launch_bounds__(256) void jacobi_block_round_kernel(const JacobiProb* tab, int count, int total_bpairs,
                                                                 int round, int sweep, double tol) {
    typedef double double4_t __attribute__((ext_vector_type(4)));
    constexpr int JB = kJacobiBlock, JV = 2 * kJacobiBlock;   // 16 columns per block pair
    const int b = blockIdx.x;
    if (b >= total_bpairs) return;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tab[mid].bpair_start <= b) lo = mid;
        else hi = mid - 1;
    }
    const JacobiProb P = tab[lo];
    const int n = P.n, nb = (n + JB - 1) / JB, m = nb + (nb & 1);
    if (round >= m - 1 || P.flags[0]) return;
    const int k = b - P.bpair_start;
    auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (m - 1); };
    const int bi = player(k), bj = player(m - 1 - k);

    __shared__ int vid[JV];
    __shared__ double Hp[4][JV][JV + 1];
    __shared__ double H[JV][JV + 1];
    __shared__ double Qm[JV][JV + 1];
    __shared__ double rc[JV / 2], rs[JV / 2];
    __shared__ int rot_any;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < JV) {
        const int blk = tid < JB ? bi : bj, col = blk * JB + (tid % JB);
        vid[tid] = blk < nb && col < n ? col : -1;   // -1: no column (padding block, ragged end)
    }
    if (tid == 0) rot_any = 0;
    __syncthreads();

    // V's 16 columns of this thread's rows (up to NR per thread; NR <= 2),
    // loaded now so that their latency hides under the Gram and the inner
    // sweep; the update below takes W from memory and V from these registers
    // (with NR > 2 the registers would cost occupancy: V is loaded there too)
    constexpr bool PREV = NR <= 2;
    double xv[PREV ? NR : 1][JV];
    if constexpr (PREV) {
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int r = tid + 256 * u;
#pragma unroll
            for (int j = 0; j < JV; ++j) xv[u][j] = (r < n && vid[j] >= 0) ? P.V[(int64_t)vid[j] * n + r] : 0.0;
        }
    }

    // H = Wp Wp^T over the n rows: wave w takes rows [w R, (w + 1) R); lane l
    // holds W[vid[l mod 16]][r] for r = l / 16 + 4 s, which is both MFMA
    // operands (A[i][k] and B[k][j] of the same column set)
    {
        const int v = lane & 15, kk = lane >> 4;
        const int R = ((n + 15) / 16) * 4;            // rows per wave, a multiple of 4
        const int r0 = wave * R;
        const double* wv = vid[v] >= 0 ? P.W + (int64_t)vid[v] * n : nullptr;
        double4_t acc = {0.0, 0.0, 0.0, 0.0};
        constexpr int CH = 16;   // loads issued together, then their matrix instructions
        for (int r1 = r0 + kk; r1 < r0 + R; r1 += 4 * CH) {
            double xs[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int r = r1 + 4 * u;
                xs[u] = (wv && r < r0 + R && r < n) ? wv[r] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[u], xs[u], acc, 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) Hp[wave][kk + 4 * e][v] = acc[e];
    }
    __syncthreads();
    {
        const int i = tid / JV, j = tid % JV;
        H[i][j] = (Hp[0][i][j] + Hp[1][i][j]) + (Hp[2][i][j] + Hp[3][i][j]);
        Qm[i][j] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();

    // one cyclic sweep over the 16 local columns (round-robin, 8 disjoint
    // pairs per inner round); a rotation R = [[c, -s], [s, c]] on columns
    // (p, q) takes rows p, q of Qm and H to R (.) and then columns of H
    for (int ir = 0; ir < JV - 1; ++ir) {
        auto lp = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + ir) % (JV - 1); };
        if (tid < JV / 2) {
            int p = lp(tid), q = lp(JV - 1 - tid);
            if (p > q) { const int t = p; p = q; q = t; }
            const double al = H[p][p], be = H[q][q], ga = H[p][q];
            double c = 1.0, sn = 0.0;
            if (fabs(ga) > tol * sqrt(al * be) && ga != 0.0) {
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                c = 1.0 / sqrt(1.0 + t * t);
                sn = c * t;
                rot_any = 1;
            }
            rc[tid] = c;
            rs[tid] = sn;
        }
        __syncthreads();
        {   // rows: 8 pairs x 16 columns of H, and of Qm
            const int t = tid >> 5, col = tid & 15, which = (tid >> 4) & 1;   // which: H or Qm
            int p = lp(t), q = lp(JV - 1 - t);
            if (p > q) { const int u = p; p = q; q = u; }
            const double c = rc[t], sn = rs[t];
            double (*M)[JV + 1] = which ? Qm : H;
            const double xp = M[p][col], xq = M[q][col];
            M[p][col] = c * xp - sn * xq;
            M[q][col] = sn * xp + c * xq;
        }
        __syncthreads();
        if (tid < 128) {   // columns of H
            const int t = tid >> 4, row = tid & 15;
            int p = lp(t), q = lp(JV - 1 - t);
            if (p > q) { const int u = p; p = q; q = u; }
            const double c = rc[t], sn = rs[t];
            const double xp = H[row][p], xq = H[row][q];
            H[row][p] = c * xp - sn * xq;
            H[row][q] = sn * xp + c * xq;
        }
        __syncthreads();
    }
    if (!rot_any) return;
    if (tid == 0) P.flags[1 + (sweep & 1)] = 1;

    // W_new[i][r] = sum_j Qm[i][j] W[j][r] (and V), each thread its own rows r
    // (up to NR per thread, all loaded before any is used)
    for (int which = 0; which < (PREV ? 1 : 2); ++which) {
        double* base = which ? P.V : P.W;
        double x[NR][JV];
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int r = tid + 256 * u;
#pragma unroll
            for (int j = 0; j < JV; ++j) x[u][j] = (r < n && vid[j] >= 0) ? base[(int64_t)vid[j] * n + r] : 0.0;
        }
        jacobi_apply_rows(Qm, vid, x, base, n, tid);
    }
    if constexpr (PREV) jacobi_apply_rows(Qm, vid, xv, P.V, n, tid);
}

__global__ void set_jacobi_prob_kernel(JacobiProb* dst, JacobiProb v) {
    if (threadIdx.x == 0) *dst = v;
}

__global__ void jacobi_sweep_end_kernel(const JacobiProb* tab, int count, int sweep) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < count; g += gridDim.x * blockDim.x) {
        int* f = tab[g].flags;
        if (f[0]) continue;
        if (f[1 + (sweep & 1)] == 0) f[0] = 1;
        f[1 + ((sweep + 1) & 1)] = 0;
        f[3] = sweep + 1;
    }
}

__global__ void jacobi_final_kernel(const JacobiProb* tab, unsigned int* status) {
    const JacobiProb P = tab[blockIdx.y];
    const int n = P.n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / n), j = (int)(e % n);
        if (r < j) {                                  // back to row-major
            double t = P.W[(int64_t)r * n + j];
            P.W[(int64_t)r * n + j] = P.W[(int64_t)j * n + r];
            P.W[(int64_t)j * n + r] = t;
            t = P.V[(int64_t)r * n + j];
            P.V[(int64_t)r * n + j] = P.V[(int64_t)j * n + r];
            P.V[(int64_t)j * n + r] = t;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && !P.flags[0]) atomicOr(status, kStatusNotConverged);
}

// sigma_j = |w_j|; rank the columns by sigma descending (ties by index); write
// sigma in that order and the permutation (one workgroup, n <= 1024).
__global__ __launch_bounds__(1024) void svd_finish_kernel(const double* W, int n, double* sig_sorted,
                                                          int* order) {
    __shared__ double s[1024];
    const int tid = threadIdx.x;
    for (int j = tid; j < n; j += blockDim.x) {
        double a = 0.0;
        for (int r = 0; r < n; ++r) a += W[r * n + j] * W[r * n + j];
        s[j] = sqrt(a);
    }
    __syncthreads();
    for (int j = tid; j < n; j += blockDim.x) {
        // rank by (key, index) with NaN keyed below every sigma (>= 0), so that
        // the ranks are a permutation of 0 .. n-1 whatever W holds
        const double kj = s[j] == s[j] ? s[j] : -1.0;
        int rank = 0;
        for (int i = 0; i < n; ++i) {
            const double ki = s[i] == s[i] ? s[i] : -1.0;
            rank += (ki > kj) || (ki == kj && i < j);
        }
        sig_sorted[rank] = s[j];
        order[rank] = j;
    }
}

// U_r[:, c] = W[:, order[c]] / sigma_c (0 column when sigma_c == 0), V_r
// columns gathered in the same order; both n x ncols, row-major, FP64.
__global__ void svd_gather_kernel(const double* W, const double* Vin, int n, const double* sig,
                                  const int* order, int ncols, double* Ur, double* Vr) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * ncols;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / ncols), cidx = (int)(e % ncols);
        int src = order[cidx];
        src = src < 0 ? 0 : (src >= n ? n - 1 : src);   // a permutation by construction; never index past W
        const double sg = sig[cidx];
        Ur[e] = sg > 0.0 ? W[(int64_t)r * n + src] / sg : 0.0;
        Vr[e] = Vin[(int64_t)r * n + src];
    }
}

int grid1d(int64_t total, int block = 256) {
    int64_t g = (total + block - 1) / block;
    return (int)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

}  // namespace

// ------------------------------------------------------------------ launchers
template <class TA, class TB, class TC>
hipError_t gemm_acc64(int64_t M, int64_t N, int64_t K, double alpha, const TA* a, int64_t sam, int64_t sak,
                      const TB* b, int64_t sbk, int64_t sbn, double beta, TC* c, int64_t scm, int64_t scn,
                      hipStream_t s) {
    return gemm_acc64_batched<TA, TB, TC>(M, N, K, alpha, a, sam, sak, 0, b, sbk, sbn, 0, beta, c, scm, scn, 0, 1, s);
}

template <class TA, class TB, class TC>
hipError_t gemm_f32(int64_t M, int64_t N, int64_t K, double alpha, const TA* a, int64_t sam, int64_t sak,
                    const TB* b, int64_t sbk, int64_t sbn, double beta, TC* c, int64_t scm, int64_t scn,
                    hipStream_t s) {
    return gemm_f32_batched<TA, TB, TC>(M, N, K, alpha, a, sam, sak, 0, b, sbk, sbn, 0, beta, c, scm, scn, 0, 1, s);
}

template <class TA, class TB, class TC>
hipError_t gemm_f32_batched(int64_t M, int64_t N, int64_t K, double alpha, const TA* a, int64_t sam, int64_t sak,
                            int64_t sab, const TB* b, int64_t sbk, int64_t sbn, int64_t sbb, double beta, TC* c,
                            int64_t scm, int64_t scn, int64_t scb, int64_t batch, hipStream_t s) {
    if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
    const int64_t gx = (N + GT - 1) / GT, gm = (M + GT - 1) / GT;
    if (gx > 0x7FFFFFFF) return hipErrorInvalidValue;
    for (int64_t z0 = 0; z0 < batch; z0 += 65535) {
        const int64_t nb = batch - z0 < 65535 ? batch - z0 : 65535;
        for (int64_t y0 = 0; y0 < gm; y0 += 65535) {
            const int64_t ny = gm - y0 < 65535 ? gm - y0 : 65535;
            const int64_t r0 = y0 * GT;
            dim3 grid((unsigned)gx, (unsigned)ny, (unsigned)nb);
            hipLaunchKernelGGL((gemm_f32_kernel<TA, TB, TC>), grid, dim3(256), 0, s, M - r0, N, K, alpha,
                               a + z0 * sab + r0 * sam, sam, sak, b + z0 * sbb, sbk, sbn, beta,
                               c + z0 * scb + r0 * scm, scm, scn, sab, sbb, scb);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

template hipError_t gemm_f32<float, double, float>(int64_t, int64_t, int64_t, double, const float*, int64_t, int64_t,
                                                   const double*, int64_t, int64_t, double, float*, int64_t, int64_t,
                                                   hipStream_t);
template hipError_t gemm_f32<float, float, float>(int64_t, int64_t, int64_t, double, const float*, int64_t, int64_t,
                                                  const float*, int64_t, int64_t, double, float*, int64_t, int64_t,
                                                  hipStream_t);
template hipError_t gemm_f32_batched<float, float, float>(int64_t, int64_t, int64_t, double, const float*, int64_t,
                                                          int64_t, int64_t, const float*, int64_t, int64_t, int64_t,
                                                          double, float*, int64_t, int64_t, int64_t, int64_t,
                                                          hipStream_t);

template <class TA, class TB, class TC>
hipError_t gemm_acc64_batched(int64_t M, int64_t N, int64_t K, double alpha, const TA* a, int64_t sam, int64_t sak,
                              int64_t sab, const TB* b, int64_t sbk, int64_t sbn, int64_t sbb, double beta, TC* c,
                              int64_t scm, int64_t scn, int64_t scb, int64_t batch, hipStream_t s) {
    if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
    const int64_t gx = (N + GT - 1) / GT, gm = (M + GT - 1) / GT;
    if (gx > 0x7FFFFFFF) return hipErrorInvalidValue;
    // row tiles on grid.y and problems on grid.z, each in chunks of at most 65535
    for (int64_t z0 = 0; z0 < batch; z0 += 65535) {
        const int64_t nb = batch - z0 < 65535 ? batch - z0 : 65535;
        for (int64_t y0 = 0; y0 < gm; y0 += 65535) {
            const int64_t ny = gm - y0 < 65535 ? gm - y0 : 65535;
            const int64_t r0 = y0 * GT;
            dim3 grid((unsigned)gx, (unsigned)ny, (unsigned)nb);
            hipLaunchKernelGGL((gemm_acc64_kernel<TA, TB, TC>), grid, dim3(256), 0, s, M - r0, N, K, alpha,
                               a + z0 * sab + r0 * sam, sam, sak, b + z0 * sbb, sbk, sbn, beta,
                               c + z0 * scb + r0 * scm, scm, scn, sab, sbb, scb);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

template hipError_t gemm_acc64<float, float, double>(int64_t, int64_t, int64_t, double, const float*, int64_t,
                                                     int64_t, const float*, int64_t, int64_t, double, double*,
                                                     int64_t, int64_t, hipStream_t);
template hipError_t gemm_acc64<double, double, double>(int64_t, int64_t, int64_t, double, const double*,
                                                       int64_t, int64_t, const double*, int64_t, int64_t,
                                                       double, double*, int64_t, int64_t, hipStream_t);
template hipError_t gemm_acc64<float, double, float>(int64_t, int64_t, int64_t, double, const float*, int64_t,
                                                     int64_t, const double*, int64_t, int64_t, double, float*,
                                                     int64_t, int64_t, hipStream_t);
template hipError_t gemm_acc64<double, double, float>(int64_t, int64_t, int64_t, double, const double*,
                                                      int64_t, int64_t, const double*, int64_t, int64_t,
                                                      double, float*, int64_t, int64_t, hipStream_t);
template hipError_t gemm_acc64<float, double, double>(int64_t, int64_t, int64_t, double, const float*,
                                                      int64_t, int64_t, const double*, int64_t, int64_t,
                                                      double, double*, int64_t, int64_t, hipStream_t);
template hipError_t gemm_acc64<float, float, float>(int64_t, int64_t, int64_t, double, const float*, int64_t,
                                                    int64_t, const float*, int64_t, int64_t, double, float*,
                                                    int64_t, int64_t, hipStream_t);
template hipError_t gemm_acc64_batched<float, float, double>(int64_t, int64_t, int64_t, double, const float*, int64_t,
                                                             int64_t, int64_t, const float*, int64_t, int64_t, int64_t,
                                                             double, double*, int64_t, int64_t, int64_t, int64_t,
                                                             hipStream_t);
template hipError_t gemm_acc64_batched<double, double, double>(int64_t, int64_t, int64_t, double, const double*,
                                                               int64_t, int64_t, int64_t, const double*, int64_t,
                                                               int64_t, int64_t, double, double*, int64_t, int64_t,
                                                               int64_t, int64_t, hipStream_t);
template hipError_t gemm_acc64_batched<float, float, float>(int64_t, int64_t, int64_t, double, const float*, int64_t,
                                                            int64_t, int64_t, const float*, int64_t, int64_t, int64_t,
                                                            double, float*, int64_t, int64_t, int64_t, int64_t,
                                                            hipStream_t);

namespace {

// dst[i][bb][aa] = src[bb][i][aa] for src of shape [B, I, P] (C order): the
// mode-i unfolding of a C-order tensor made contiguous.  P == 1 is a plain
// transpose, tiled through LDS so that reads and writes are both coalesced;
// P > 1 copies runs of P contiguous elements.
__global__ __launch_bounds__(256) void transpose_tile_kernel(const float* __restrict__ src, int64_t B, int64_t I,
                                                             float* __restrict__ dst) {
    __shared__ float t[32][33];
    const int64_t b0 = blockIdx.x * 32, i0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t bb = b0 + ty + 8 * q, ii = i0 + tx;
        if (bb < B && ii < I) t[ty + 8 * q][tx] = src[bb * I + ii];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t ii = i0 + ty + 8 * q, bb = b0 + tx;
        if (bb < B && ii < I) dst[ii * B + bb] = t[tx][ty + 8 * q];
    }
}

__global__ __launch_bounds__(256) void swap01_kernel(const float* __restrict__ src, int64_t B, int64_t I, int64_t P,
                                                     float* __restrict__ dst) {
    const int64_t total = B * I * P;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int64_t aa = e % P, rest = e / P;
        const int64_t bb = rest % B, ii = rest / B;      // e indexes dst[ii][bb][aa]
        dst[e] = src[(bb * I + ii) * P + aa];
    }
}

}  // namespace

hipError_t launch_swap01(const float* src, int64_t B, int64_t I, int64_t P, float* dst, hipStream_t s) {
    if (B <= 0 || I <= 0 || P <= 0) return hipSuccess;
    if (P == 1) {
        const int64_t gb = (B + 31) / 32, gi = (I + 31) / 32;
        if (gi > 65535) return hipErrorInvalidValue;
        hipLaunchKernelGGL(transpose_tile_kernel, dim3((unsigned)gb, (unsigned)gi), dim3(256), 0, s, src, B, I, dst);
    } else {
        const int64_t total = B * I * P;
        int64_t g = (total + 255) / 256;
        g = g > 65536 ? 65536 : g;
        hipLaunchKernelGGL(swap01_kernel, dim3((unsigned)g), dim3(256), 0, s, src, B, I, P, dst);
    }
    return hipGetLastError();
}

hipError_t launch_trtri_apply_diag(double* X, int64_t ldx, int64_t r0, int64_t rows, hipStream_t s) {
    hipLaunchKernelGGL(trtri_apply_diag_kernel, dim3((unsigned)((r0 + NB - 1) / NB)), dim3(256), 0, s, X, ldx, r0,
                       (int)rows);
    return hipGetLastError();
}

template <class T>
hipError_t gram_acc64(int64_t p, int64_t K, const T* Y, int64_t ldy, double* G, double* partial, int max_split,
                      hipStream_t s) {
    if (p <= 0) return hipSuccess;
    const int64_t nt = (p + GT - 1) / GT, tri = nt * (nt + 1) / 2;
    int64_t S = (1024 + tri - 1) / tri;              // about 4 workgroups per compute unit
    S = S > max_split ? max_split : S;
    S = S > K / 512 ? K / 512 : S;                   // at least 512 contraction rows per part
    if (S < 1 || !partial) S = 1;
    const int64_t Kc = S == 1 ? K : ((K + S - 1) / S + GK - 1) / GK * GK;
    const int64_t parts = S == 1 ? 1 : (K + Kc - 1) / Kc;
    if (parts > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gram_sym_kernel<T>), dim3((unsigned)tri, (unsigned)parts), dim3(256), 0, s, p, K, Kc, Y, ldy,
                       parts == 1 ? G : partial);
    if (parts > 1)
        hipLaunchKernelGGL(sum_partials_kernel, dim3(grid1d(p * p)), dim3(256), 0, s, partial, p * p, (int)parts, G);
    return hipGetLastError();
}

template hipError_t gram_acc64<float>(int64_t, int64_t, const float*, int64_t, double*, double*, int, hipStream_t);
template hipError_t gram_acc64<double>(int64_t, int64_t, const double*, int64_t, double*, double*, int, hipStream_t);

hipError_t gemm_tn_f32(int64_t N, int64_t P, int64_t K, const float* A, int64_t lda, const float* Q, int64_t ldq,
                       float* C, int64_t ldc, hipStream_t s) {
    if (N <= 0 || P <= 0) return hipSuccess;
    const bool ok = lda % 4 == 0 && ldq % 4 == 0 && ldc % 4 == 0 && ((uintptr_t)A & 15) == 0 &&
                    ((uintptr_t)Q & 15) == 0 && ((uintptr_t)C & 15) == 0;
    if (!ok)   // off the 16-byte path: the FP64-accumulating GEMM
        return gemm_acc64<float, float, float>(N, P, K, 1.0, A, 1, lda, Q, ldq, 1, 0.0, C, ldc, 1, s);
    // column tiles of C on grid.x (up to 2^31 - 1), 256-row blocks on grid.y in
    // chunks of at most 65535
    const int64_t gx = (P + 63) / 64, gy = (N + 255) / 256;
    if (gx > 0x7FFFFFFF) return hipErrorInvalidValue;
    for (int64_t y0 = 0; y0 < gy; y0 += 65535) {
        const int64_t ny = gy - y0 < 65535 ? gy - y0 : 65535;
        const int64_t r0 = y0 * 256;
        hipLaunchKernelGGL(gemm_tn_f32_kernel, dim3((unsigned)gx, (unsigned)ny), dim3(256), 0, s, N - r0, P, K,
                           A + r0, lda, Q, ldq, C + r0 * ldc, ldc);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Rounds take the block form once a problem has more than one block pair.
// Its rotations come from the block's Gram, whose rounding keeps the last
// off-diagonal ratios near 1e-13 for a while (16 sweeps instead of 14 on a
// 640 x 640 R_B^T with sigma in [0.018, 1] at 1e-12), so it stops at 1e-12
// (singular values then agree to far below FP32 rounding) and may take up to
// 8 more sweeps.
static bool jacobi_block_form(int max_n) { return max_n > 2 * kJacobiBlock; }

int jacobi_group_sweep_bound(int max_n, int max_sweeps) {
    return jacobi_block_form(max_n) ? max_sweeps + 8 : max_sweeps;
}

hipError_t jacobi_group_prep(const JacobiProb* tab, int count, int max_n, hipStream_t s) {
    if (count <= 0 || max_n <= 0) return hipSuccess;
    if (max_n > 1024) return hipErrorInvalidValue;    // the round kernels hold n <= 1024 elements in registers
    const int gx = grid1d((int64_t)max_n * max_n) < 1024 ? grid1d((int64_t)max_n * max_n) : 1024;
    hipLaunchKernelGGL(jacobi_prep_kernel, dim3((unsigned)gx, (unsigned)count), dim3(256), 0, s, tab);
    return hipGetLastError();
}

hipError_t jacobi_group_sweeps(const JacobiProb* tab, int count, int total_pairs, int total_bpairs, int max_n,
                               int sweep_begin, int sweep_end, double tol, hipStream_t s, const int* poll_flag) {
    if (count <= 0 || max_n <= 0) return hipSuccess;
    if (max_n > 1024) return hipErrorInvalidValue;
    hipError_t e;
    const bool block = jacobi_block_form(max_n);
    const int max_nb = (max_n + kJacobiBlock - 1) / kJacobiBlock;
    const int max_m = block ? max_nb + (max_nb & 1) : max_n + (max_n & 1);
    const double btol = tol > 1e-12 ? tol : 1e-12;
    for (int sweep = sweep_begin; sweep < sweep_end; ++sweep) {
        for (int round = 0; round < max_m - 1; ++round) {
            if (block && max_n <= 256)
                hipLaunchKernelGGL(jacobi_block_round_kernel<1>, dim3((unsigned)total_bpairs), dim3(256), 0, s, tab,
                                   count, total_bpairs, round, sweep, btol);
            else if (block && max_n <= 512)
                hipLaunchKernelGGL(jacobi_block_round_kernel<2>, dim3((unsigned)total_bpairs), dim3(256), 0, s, tab,
                                   count, total_bpairs, round, sweep, btol);
            else if (block)
                hipLaunchKernelGGL(jacobi_block_round_kernel<4>, dim3((unsigned)total_bpairs), dim3(256), 0, s, tab,
                                   count, total_bpairs, round, sweep, btol);
            else if (total_pairs >= kJacobiWavePairs)
                hipLaunchKernelGGL(jacobi_round_kernel<true>, dim3((unsigned)((total_pairs + 3) / 4)), dim3(256), 0, s,
                                   tab, count, total_pairs, round, sweep, tol);
            else
                hipLaunchKernelGGL(jacobi_round_kernel<false>, dim3((unsigned)total_pairs), dim3(256), 0, s, tab,
                                   count, total_pairs, round, sweep, tol);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(jacobi_sweep_end_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, tab,
                           count, sweep);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (poll_flag) {   // one problem, not captured: stop once its converged flag is set
            int done = 0;
            if ((e = hipMemcpyAsync(&done, poll_flag, sizeof done, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
            if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
            if (done) break;
        }
    }
    return hipSuccess;
}

// *out = the number of problems whose converged flag is not set (one workgroup)
__global__ __launch_bounds__(256) void jacobi_open_kernel(const JacobiProb* tab, int count, int* out) {
    __shared__ int total;
    if (threadIdx.x == 0) total = 0;
    __syncthreads();
    int mine = 0;
    for (int g = threadIdx.x; g < count; g += blockDim.x) mine += tab[g].flags[0] ? 0 : 1;
    if (mine) atomicAdd(&total, mine);
    __syncthreads();
    if (threadIdx.x == 0) *out = total;
}

hipError_t jacobi_group_open(const JacobiProb* tab, int count, int* out, hipStream_t s) {
    hipLaunchKernelGGL(jacobi_open_kernel, dim3(1), dim3(256), 0, s, tab, count, out);
    return hipGetLastError();
}

hipError_t jacobi_group_final(const JacobiProb* tab, int count, int max_n, unsigned int* status, hipStream_t s) {
    if (count <= 0 || max_n <= 0) return hipSuccess;
    if (max_n > 1024) return hipErrorInvalidValue;
    const int gx = grid1d((int64_t)max_n * max_n) < 1024 ? grid1d((int64_t)max_n * max_n) : 1024;
    hipLaunchKernelGGL(jacobi_final_kernel, dim3((unsigned)gx, (unsigned)count), dim3(256), 0, s, tab, status);
    return hipGetLastError();
}

hipError_t jacobi_svd_group(const JacobiProb* tab, int count, int total_pairs, int total_bpairs, int max_n,
                            int max_sweeps, double tol, unsigned int* status, hipStream_t s, const int* poll_flag) {
    if (count <= 0 || max_n <= 0) return hipSuccess;
    if (max_n > 1024) return hipErrorInvalidValue;
    hipError_t e;
    if ((e = jacobi_group_prep(tab, count, max_n, s)) != hipSuccess) return e;
    if ((e = jacobi_group_sweeps(tab, count, total_pairs, total_bpairs, max_n, 0,
                                 jacobi_group_sweep_bound(max_n, max_sweeps), tol, s, poll_flag)) != hipSuccess)
        return e;
    return jacobi_group_final(tab, count, max_n, status, s);
}

hipError_t launch_set_jacobi_prob(JacobiProb* dst, const JacobiProb& v, hipStream_t s) {
    hipLaunchKernelGGL(set_jacobi_prob_kernel, dim3(1), dim3(64), 0, s, dst, v);
    return hipGetLastError();
}

hipError_t svd_finish(const double* W, const double* V, int n, int ncols, double* sig, int* order, double* Ur,
                      double* Vr, hipStream_t s) {
    hipLaunchKernelGGL(svd_finish_kernel, dim3(1), dim3(1024), 0, s, W, n, sig, order);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(svd_gather_kernel, dim3(grid1d((int64_t)n * ncols)), dim3(256), 0, s, W, V, n, sig, order,
                       ncols, Ur, Vr);
    return hipGetLastError();
}

hipError_t potrf_lower(double* A, int64_t lda, int64_t p, unsigned int* status, hipStream_t s) {
    hipError_t e;
    if ((e = launch_zero_upper(A, lda, p, s)) != hipSuccess) return e;
    for (int64_t k = 0; k < p; k += NB) {
        const int nb = (int)(p - k < NB ? p - k : NB);
        hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, A, lda, k, nb, status);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t below = p - k - nb;
        if (below <= 0) break;
        hipLaunchKernelGGL(trsm_panel_kernel, dim3((unsigned)((below + 63) / 64)), dim3(256), 0, s, A, lda, k,
                           nb, p);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        // trailing update: A22 -= L21 L21^T (full square; the upper part is
        // cleared again at the end)
        double* L21 = A + (k + nb) * lda + k;
        double* A22 = A + (k + nb) * lda + k + nb;
        if ((e = gemm_acc64<double, double, double>(below, below, nb, -1.0, L21, lda, 1, L21, 1, lda, 1.0, A22,
                                                    lda, 1, s)) != hipSuccess)
            return e;
    }
    return launch_zero_upper(A, lda, p, s);
}

hipError_t launch_zero_upper(double* A, int64_t lda, int64_t p, hipStream_t s) {
    if (p <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_upper_kernel, dim3(grid1d(p * p)), dim3(256), 0, s, A, lda, p);
    return hipGetLastError();
}

hipError_t trtri_lower(const double* L, int64_t ldl, double* X, int64_t ldx, int64_t p, hipStream_t s) {
    hipError_t e;
    const int64_t nblk = (p + NB - 1) / NB;
    hipLaunchKernelGGL(zero_upper_kernel, dim3(grid1d(p * p)), dim3(256), 0, s, X, ldx, p);   // upper = 0
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(trtri_diag_kernel, dim3((unsigned)nblk), dim3(256), 0, s, L, ldl, X, ldx, p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // block row i (i >= 1): X[i, 0:i] = -X_ii (L[i, 0:i] X[0:i, 0:i]); the
    // product T is written into block row i of X itself (those entries are
    // not read by it), then replaced by -X_ii T
    for (int64_t i = 1; i < nblk; ++i) {
        const int64_t r0 = i * NB;
        const int64_t rows = p - r0 < NB ? p - r0 : NB;
        double* Xi = X + r0 * ldx;                   // block row i, columns 0:r0
        // T = L[r0:r0+rows, 0:r0] X[0:r0, 0:r0]
        if ((e = gemm_acc64<double, double, double>(rows, r0, r0, 1.0, L + r0 * ldl, ldl, 1, X, ldx, 1, 0.0, Xi,
                                                    ldx, 1, s)) != hipSuccess)
            return e;
        // X[i, 0:i] = -X_ii T (in place, chunk by chunk in LDS)
        if ((e = launch_trtri_apply_diag(X, ldx, r0, rows, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rpmi
