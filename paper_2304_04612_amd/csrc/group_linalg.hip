// Grouped (table-driven) linear algebra for many small RSVD problems at once
// (the batched randomized SVD: Algorithm 1 for every problem of a set).  Each
// kernel reads a device table of jobs and runs all of them in one launch, so
// that a stage of Algorithm 1 costs one launch for the whole set instead of
// one (or a dozen) per problem:
//
// * gemm_acc64_group: C_g = alpha op(A_g) op(B_g) (+ beta C_g) with arbitrary
//   strides and FP64 MFMA products (64 x 64 output tiles); blocks find their
//   job by binary search over each job's first block.  Used for the Gram
//   matrices Y^T Y, the products Y R^-1 of CholeskyQR2, U = Q U_r, V = W V_r
//   and the product of the two Cholesky factors.
// * chol_inv_group: for every p x p FP64 Gram matrix G (p <= kCholGroupMaxP)
//   the lower Cholesky factor L (G = L L^T) and X = L^-1, one workgroup per
//   job with L held in LDS as a packed lower triangle.  A non-positive pivot
//   sets NOT_SPD and the factorisation continues on |pivot|.
// * gemm_tn_f32_group: C_g = A_g^T Q_g on FP32 MFMA for any leading
//   dimensions (16-byte loads where rows are 16-byte aligned, element loads
//   otherwise).
// * svd_finish_group: singular values of W (column norms after the Jacobi
//   iteration), their descending order, S, and the gathered U_r, V_r.
#include "rpmi_internal.h"
#include "gemm64_tile.h"

namespace rpmi {
namespace {

constexpr int GT = kG64Tile;   // output tile of gemm_acc64_group

__device__ __forceinline__ int find_job(const int64_t* starts, int count, int64_t b) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <class TA, class TB, class TC, bool ACC32 = false>
__global__ __launch_bounds__(256) void gemm_acc64_group_kernel(const GemmJob* __restrict__ jobs,
                                                               const int64_t* __restrict__ starts, int count) {
    const int64_t blk = blockIdx.x;
    const GemmJob J = jobs[find_job(starts, count, blk)];
    const int64_t local = blk - J.start;
    const int64_t ti = local / J.tiles_n, tj = local % J.tiles_n;
    gemm64_tile<TA, TB, TC, false, ACC32>(J.M, J.N, J.K, J.alpha, static_cast<const TA*>(J.a), J.sam, J.sak,
                                          static_cast<const TB*>(J.b), J.sbk, J.sbn, J.beta, static_cast<TC*>(J.c),
                                          J.scm, J.scn, ti * GT, tj * GT);
}

// G = Y^T Y per job: block b of the job is (kz, t) with t an upper-triangle
// 64 x 64 tile (ti <= tj, row by row); the tile's product over rows
// [kz kchunk, (kz + 1) kchunk) goes to partial kz (or straight to G when the
// job is not split), mirrored into the lower triangle.
template <class T>
__global__ __launch_bounds__(256) void gram_group_kernel(const GramJob* __restrict__ jobs,
                                                         const int64_t* __restrict__ starts, int count) {
    const int64_t blk = blockIdx.x;
    const GramJob J = jobs[find_job(starts, count, blk)];
    const int64_t local = blk - J.start;
    const int kz = (int)(local / J.tiles);
    int t = (int)(local - (int64_t)kz * J.tiles);
    const int tt = (int)((J.p + GT - 1) / GT);
    int ti = 0;
    while (t >= tt - ti) {
        t -= tt - ti;
        ++ti;
    }
    const int tj = ti + t;
    const int64_t k0 = kz * J.kchunk;
    const int64_t klen = J.R - k0 < J.kchunk ? J.R - k0 : J.kchunk;
    const T* y = static_cast<const T*>(J.y) + k0 * J.ldy;
    double* c = J.ksplit > 1 ? J.part + (int64_t)kz * J.p * J.p : J.G;
    gemm64_tile<T, T, double, true>(J.p, J.p, klen, 1.0, y, 1, J.ldy, y, J.ldy, 1, 0.0, c, J.p, 1, ti * GT, tj * GT);
}

// G = sum of the job's partials, in order (kSumBlocks workgroups per job)
constexpr int kSumBlocks = 16;
__global__ __launch_bounds__(256) void gram_sum_group_kernel(const GramJob* __restrict__ jobs) {
    const GramJob J = jobs[blockIdx.x];
    if (J.ksplit <= 1) return;
    const int64_t pp = J.p * J.p;
    for (int64_t e = blockIdx.y * 256 + threadIdx.x; e < pp; e += 256 * kSumBlocks) {
        double acc = 0.0;
        for (int z = 0; z < J.ksplit; ++z) acc += J.part[z * pp + e];
        J.G[e] = acc;
    }
}

// Packed lower triangle: element (i, l), l <= i, at i (i + 1) / 2 + l.
__device__ __forceinline__ int tri(int i, int l) { return i * (i + 1) / 2 + l; }

// Pivot of a Cholesky step; a non-positive (or NaN) pivot is reported by the
// caller and replaced by |v| (1 if zero) so that the factorization finishes.
__device__ __forceinline__ double chol_pivot(double v) { return v > 0.0 ? v : (fabs(v) > 0.0 ? fabs(v) : 1.0); }

constexpr int kCholThreads = 1024;

// One workgroup per problem, everything in LDS: the packed lower triangle T
// (p (p + 1) / 2 doubles) and two column buffers of p doubles.
//  * Cholesky, right-looking without scaled columns: step j subtracts
//    T_ij T_lj / T_jj from every T_il, j < l <= i (column j itself is not
//    written, so one barrier per step); afterwards d_j = sqrt(T_jj) and
//    L_ij = T_ij / d_j.
//  * X = L^-1 in place, last column first: from X L = I,
//    X_ij = -(sum_{l=j+1..i} X_il L_lj) / L_jj for i > j, X_jj = 1 / L_jj;
//    column j of L is copied to a buffer one step ahead (double buffer, one
//    barrier per step); four lanes share a row's sum.
__global__ __launch_bounds__(kCholThreads) void chol_inv_group_kernel(const CholJob* __restrict__ jobs,
                                                                      unsigned int* status) {
    extern __shared__ double T[];
    const CholJob J = jobs[blockIdx.x];
    const int p = J.p, tid = threadIdx.x;
    const int np = p * (p + 1) / 2;
    double* cb0 = T + np;
    double* cb1 = cb0 + p;
    for (int i = tid >> 5; i < p; i += kCholThreads / 32)
        for (int l = tid & 31; l <= i; l += 32) T[tri(i, l)] = J.G[(int64_t)i * p + l];
    __syncthreads();
    const int tx = tid & 31, ty = tid >> 5;
    for (int j = 0; j < p; ++j) {
        const double v = T[tri(j, j)];
        if (tid == 0 && !(v > 0.0)) atomicOr(status, kStatusNotSpd);
        const double rv = 1.0 / chol_pivot(v);
        for (int i = j + 1 + ty; i < p; i += kCholThreads / 32) {
            const double a = T[tri(i, j)] * rv;
            for (int l = j + 1 + tx; l <= i; l += 32) T[tri(i, l)] -= a * T[tri(l, j)];
        }
        __syncthreads();
    }
    for (int j = tid; j < p; j += kCholThreads) cb0[j] = sqrt(chol_pivot(T[tri(j, j)]));
    __syncthreads();
    for (int i = ty; i < p; i += kCholThreads / 32)
        for (int l = tx; l <= i; l += 32) T[tri(i, l)] = l == i ? cb0[i] : T[tri(i, l)] / cb0[l];
    __syncthreads();
    for (int e = tid; e < p * p; e += kCholThreads) {
        const int i = e / p, l = e % p;
        J.L[e] = l <= i ? T[tri(i, l)] : 0.0;
    }
    // inverse: cb holds column j of L (rows j..p-1) while column j is solved
    for (int l = p - 1 + tid; l < p; l += kCholThreads) cb0[l] = T[tri(l, p - 1)];
    __syncthreads();
    const int q = tid & 3, row = tid >> 2;
    for (int j = p - 1; j >= 0; --j) {
        double* cb = ((p - 1 - j) & 1) ? cb1 : cb0;
        double* nb = ((p - 1 - j) & 1) ? cb0 : cb1;
        if (j > 0)
            for (int l = j - 1 + tid; l < p; l += kCholThreads) nb[l] = T[tri(l, j - 1)];
        const int i = j + 1 + row;
        double acc = 0.0;
        if (i < p)
            for (int l = j + 1 + q; l <= i; l += 4) acc += T[tri(i, l)] * cb[l];
        acc += __shfl_xor(acc, 1);
        acc += __shfl_xor(acc, 2);
        if (i < p && q == 0) T[tri(i, j)] = -acc / cb[j];
        if (tid == 0) T[tri(j, j)] = 1.0 / cb[j];
        __syncthreads();
    }
    for (int e = tid; e < p * p; e += kCholThreads) {
        const int i = e / p, l = e % p;
        J.X[e] = l <= i ? T[tri(i, l)] : 0.0;
    }
}

// C (N x P) = A^T Q for A (K x N, lda) and Q (K x P, ldq) on
// v_mfma_f32_16x16x4f32: a wave owns 64 x 64 of C as 4 x 4 MFMA tiles; lane c
// reads column i0 + 16a + c of a row of A (and j0 + 16b + c of a row of Q), so
// the 16 lanes of a row read 64 consecutive bytes with each 4-byte load,
// whatever the alignment of lda, ldq and the bases.  The four waves of a
// workgroup take the job's wp 64-column tiles of P first (wp = min(tiles of P,
// 4)) and 4 / wp column blocks of A second, so that the waves sharing a block
// of A run on one compute unit and A leaves HBM once for all of P.  The next
// 16 rows are loaded before the products of the current ones.  Jobs come
// longest contraction chunk first (the host orders the table), so that the
// longest waves start first.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void gemm_tn_f32_group_kernel(const TnJob* __restrict__ jobs,
                                                                const int64_t* __restrict__ starts, int count) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int64_t blk = blockIdx.x;
    const TnJob J = jobs[find_job(starts, count, blk)];
    const int64_t local = blk - J.start;
    const int64_t per_k = J.tiles_x * J.tiles_y;
    const int kz = (int)(local / per_k);
    const int64_t rest = local - kz * per_k;
    const int64_t bx = rest % J.tiles_x, by = rest / J.tiles_x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wp = J.wp, wn = 4 / wp;
    if (wave >= wp * wn) return;              // wp = 3: the fourth wave has no tile (no barrier follows)
    const int64_t i0 = (by * wn + wave / wp) * 64, j0 = (bx * wp + wave % wp) * 64;
    if (i0 >= J.N || j0 >= J.P) return;
    const int64_t kbeg = kz * J.kchunk, kend = J.K < kbeg + J.kchunk ? J.K : kbeg + J.kchunk;
    float* const Cout = J.ksplit > 1 ? J.part + kz * J.N * J.P : J.C;
    const int64_t ldc = J.ksplit > 1 ? J.P : J.ldc;
    const int g = lane >> 4, c = lane & 15;
    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    auto load4 = [&](const float* row, int64_t base, int64_t lim) -> f4 {
        f4 v;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = base + 16 * e + c < lim ? row[base + 16 * e + c] : 0.0f;
        return v;
    };
    auto load_step = [&](int64_t k0, f4* av, f4* qv) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t k = k0 + 4 * u + g;
            const bool in = k < kend;
            av[u] = in ? load4(J.A + k * J.lda, i0, J.N) : f4{0.f, 0.f, 0.f, 0.f};
            qv[u] = in ? load4(J.Q + k * J.ldq, j0, J.P) : f4{0.f, 0.f, 0.f, 0.f};
        }
    };
    // 16 x 16 tiles wholly past N or P have no output: their products are
    // skipped (the tests are uniform over the wave)
    const int na = J.N - i0 >= 64 ? 4 : (int)((J.N - i0 + 15) / 16);
    const int nbt = J.P - j0 >= 64 ? 4 : (int)((J.P - j0 + 15) / 16);
    f4 av[4], qv[4];
    load_step(kbeg, av, qv);
    for (int64_t k0 = kbeg; k0 < kend; k0 += 16) {
        f4 an[4], qn[4];
        const bool more = k0 + 16 < kend;
        if (more) load_step(k0 + 16, an, qn);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (a < na && b < nbt)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u][a], qv[u][b], acc[a][b], 0, 0, 0);
        if (more) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                av[u] = an[u];
                qv[u] = qn[u];
            }
        }
    }
    // lane (c, g) holds D[4g + e][c] of every MFMA tile
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t i = i0 + 16 * a + 4 * g + e;
            if (i >= J.N) continue;
            float* crow = Cout + i * ldc;
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (j0 + 16 * b + c < J.P) crow[j0 + 16 * b + c] = acc[a][b][e];
        }
}

// sigma_j = |w_j| (column norms of W, row-major n x n); rank by sigma
// descending (ties by index); S (first ncols), sigma and the order.  One
// workgroup per job.
__global__ __launch_bounds__(1024) void svd_sigma_group_kernel(const SvdJob* __restrict__ jobs) {
    __shared__ double s[1024];
    const SvdJob J = jobs[blockIdx.x];
    const int n = J.n, tid = threadIdx.x;
    for (int j = tid; j < n; j += blockDim.x) {
        double a = 0.0;
        for (int r = 0; r < n; ++r) a += J.W[(int64_t)r * n + j] * J.W[(int64_t)r * n + j];
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
        J.sig[rank] = s[j];
        J.order[rank] = j;
        if (rank < J.ncols) J.S[rank] = s[j];
    }
}

// U_r[:, c] = W[:, order[c]] / sigma_c (0 when sigma_c == 0) and V_r[:, c] =
// V[:, order[c]], both n x ncols; grid.y = job.
__global__ void svd_gather_group_kernel(const SvdJob* __restrict__ jobs) {
    const SvdJob J = jobs[blockIdx.y];
    const int64_t total = (int64_t)J.n * J.ncols;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / J.ncols), cidx = (int)(e % J.ncols);
        int src = J.order[cidx];
        src = src < 0 ? 0 : (src >= J.n ? J.n - 1 : src);   // a permutation by construction; never index past W
        const double sg = J.sig[cidx];
        J.Ur[e] = sg > 0.0 ? J.W[(int64_t)r * J.n + src] / sg : 0.0;
        J.Vr[e] = J.V[(int64_t)r * J.n + src];
    }
}

}  // namespace

int64_t gemm_group_tiles(int64_t M, int64_t N) { return ((M + GT - 1) / GT) * ((N + GT - 1) / GT); }
int64_t gemm_group_tiles_n(int64_t N) { return (N + GT - 1) / GT; }

template <class TA, class TB, class TC>
hipError_t gemm_acc64_group(const GemmJob* jobs, const int64_t* starts, int count, int64_t blocks, hipStream_t s) {
    if (count <= 0 || blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_acc64_group_kernel<TA, TB, TC>), dim3((unsigned)blocks), dim3(256), 0, s, jobs, starts,
                       count);
    return hipGetLastError();
}

template <class TA, class TB, class TC>
hipError_t gemm_f32_group(const GemmJob* jobs, const int64_t* starts, int count, int64_t blocks, hipStream_t s) {
    if (count <= 0 || blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_acc64_group_kernel<TA, TB, TC, true>), dim3((unsigned)blocks), dim3(256), 0, s, jobs,
                       starts, count);
    return hipGetLastError();
}

template hipError_t gemm_f32_group<float, double, float>(const GemmJob*, const int64_t*, int, int64_t, hipStream_t);

template hipError_t gemm_acc64_group<float, float, double>(const GemmJob*, const int64_t*, int, int64_t, hipStream_t);
template hipError_t gemm_acc64_group<double, double, double>(const GemmJob*, const int64_t*, int, int64_t,
                                                             hipStream_t);
template hipError_t gemm_acc64_group<float, double, double>(const GemmJob*, const int64_t*, int, int64_t,
                                                            hipStream_t);
template hipError_t gemm_acc64_group<double, double, float>(const GemmJob*, const int64_t*, int, int64_t,
                                                            hipStream_t);
template hipError_t gemm_acc64_group<float, double, float>(const GemmJob*, const int64_t*, int, int64_t, hipStream_t);

int gram_group_tiles(int64_t p) {
    const int tt = (int)((p + GT - 1) / GT);
    return tt * (tt + 1) / 2;
}

template <class T>
hipError_t gram_group(const GramJob* jobs, const int64_t* starts, int count, int64_t blocks, bool any_split,
                      hipStream_t s) {
    if (count <= 0 || blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gram_group_kernel<T>), dim3((unsigned)blocks), dim3(256), 0, s, jobs, starts, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !any_split) return e;
    hipLaunchKernelGGL(gram_sum_group_kernel, dim3((unsigned)count, kSumBlocks), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

template hipError_t gram_group<float>(const GramJob*, const int64_t*, int, int64_t, bool, hipStream_t);
template hipError_t gram_group<double>(const GramJob*, const int64_t*, int, int64_t, bool, hipStream_t);

hipError_t chol_inv_group(const CholJob* jobs, int count, int max_p, unsigned int* status, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (max_p > kCholGroupMaxP) return hipErrorInvalidValue;
    const size_t lds = ((size_t)max_p * (max_p + 1) / 2 + 2 * (size_t)max_p) * sizeof(double);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_inv_group_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(chol_inv_group_kernel, dim3((unsigned)count), dim3(kCholThreads), lds, s, jobs, status);
    return hipGetLastError();
}

void tn_group_shape(TnJob& j) {
    const int64_t tp = (j.P + 63) / 64;
    j.wp = tp < 4 ? (int)(tp < 1 ? 1 : tp) : 4;
    j.tiles_x = (tp + j.wp - 1) / j.wp;
    j.tiles_y = (j.N + 64 * (4 / j.wp) - 1) / (64 * (4 / j.wp));
}

// C = sum of the job's partials, in order (kSumBlocks workgroups per job)
__global__ __launch_bounds__(256) void tn_sum_group_kernel(const TnJob* __restrict__ jobs) {
    const TnJob J = jobs[blockIdx.x];
    if (J.ksplit <= 1) return;
    const int64_t np = J.N * J.P;
    for (int64_t e = blockIdx.y * 256 + threadIdx.x; e < np; e += 256 * kSumBlocks) {
        float acc = 0.0f;
        for (int z = 0; z < J.ksplit; ++z) acc += J.part[z * np + e];
        const int64_t i = e / J.P, j = e - i * J.P;
        J.C[i * J.ldc + j] = acc;
    }
}

hipError_t gemm_tn_f32_group(const TnJob* jobs, const int64_t* starts, int count, int64_t blocks, bool any_split,
                             hipStream_t s) {
    if (count <= 0 || blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gemm_tn_f32_group_kernel, dim3((unsigned)blocks), dim3(256), 0, s, jobs, starts, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !any_split) return e;
    hipLaunchKernelGGL(tn_sum_group_kernel, dim3((unsigned)count, kSumBlocks), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

hipError_t svd_finish_group(const SvdJob* jobs, int count, int max_elems, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(svd_sigma_group_kernel, dim3((unsigned)count), dim3(1024), 0, s, jobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int gx = (max_elems + 255) / 256;
    gx = gx < 1 ? 1 : (gx > 1024 ? 1024 : gx);
    hipLaunchKernelGGL(svd_gather_group_kernel, dim3((unsigned)gx, (unsigned)count), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

}  // namespace rpmi
