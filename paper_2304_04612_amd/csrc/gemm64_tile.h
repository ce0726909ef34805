// One 64 x 64 output tile of C = alpha op(A) op(B) + beta C with FP64
// products on v_mfma_f64_16x16x4f64 (gfx950), shared by the plain, batched,
// grouped and Gram FP64-accumulating GEMMs of the library.
//
// Operands may be FP32 or FP64 with arbitrary row/column strides: A(i,k) =
// a[i*sam + k*sak], B(k,j) = b[k*sbk + j*sbn], C[i][j] = c[i*scm + j*scn].
// Slices of 16 contraction steps are staged through LDS as FP64 (the loader
// walks the unit-stride index fastest); the next slice is loaded into
// registers while the current one is multiplied, so the global-load latency
// overlaps the matrix instructions.  The 4 waves of the workgroup own the
// four 32 x 32 quadrants of the tile as 2 x 2 MFMA tiles; for
// v_mfma_f64_16x16x4f64 lane l supplies A[l mod 16][l / 16] and
// B[l / 16][l mod 16] and holds D[l / 16 + 4 e][l mod 16], e = 0..3 (the
// FP64 accumulator interleaves rows with stride 4, unlike the FP32 forms,
// whose lane holds 4 consecutive rows).  The contraction order is fixed
// (deterministic).  beta == 0 ignores C's old contents (NaN included).
// MIRROR (a tile with i0 <= j0 of a symmetric C = A A^T, beta 0) also
// writes C[j][i] = C[i][j].
// ACC32: the same tile in FP32 (operands rounded to FP32 as they are staged,
// v_mfma_f32_16x16x4f32, FP32 accumulation; lane l then holds
// D[4 (l / 16) + e][l mod 16]): the plain FP32 GEMM form, for the products
// outside CholeskyQR2 and the small SVD.
#pragma once
#include <type_traits>
#include "rpmi_internal.h"

namespace rpmi {
namespace {

constexpr int kG64Tile = 64;     // output tile
constexpr int kG64K = 16;        // contraction slice

template <class T>
__device__ __forceinline__ double g64_ld(const T* p) { return (double)*p; }

template <class TA, class TB, class TC, bool MIRROR = false, bool ACC32 = false>
__device__ __forceinline__ void gemm64_tile(int64_t M, int64_t N, int64_t K, double alpha, const TA* __restrict__ a,
                                            int64_t sam, int64_t sak, const TB* __restrict__ b, int64_t sbk,
                                            int64_t sbn, double beta, TC* __restrict__ c, int64_t scm, int64_t scn,
                                            int64_t i0, int64_t j0) {
    typedef double double4_t __attribute__((ext_vector_type(4)));
    typedef float g32x4_t __attribute__((ext_vector_type(4)));
    constexpr int GT = kG64Tile, GK = kG64K;
    typedef typename std::conditional<ACC32, float, double>::type TS;   // staging and product type
    __shared__ TS As[GK][GT + 1];
    __shared__ TS Bs[GK][GT + 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int qr = (wave >> 1) * 32, qc = (wave & 1) * 32;    // this wave's quadrant
    const int li = lane & 15, lk = lane >> 4;
    // this thread's 4 + 4 staging slots (the same in every slice)
    int ai[4], ak[4], bj[4], bk[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = tid + q * 256;          // 0..1023
        if (sak == 1) { ak[q] = e % GK; ai[q] = e / GK; } else { ai[q] = e % GT; ak[q] = e / GT; }
        if (sbn == 1) { bj[q] = e % GT; bk[q] = e / GT; } else { bk[q] = e % GK; bj[q] = e / GK; }
    }
    TS ra[4], rb[4];
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t gi = i0 + ai[q], gk = k0 + ak[q];
            ra[q] = (gi < M && gk < K) ? (TS)g64_ld(a + gi * sam + gk * sak) : (TS)0;
            const int64_t gj = j0 + bj[q], gkb = k0 + bk[q];
            rb[q] = (gj < N && gkb < K) ? (TS)g64_ld(b + gkb * sbk + gj * sbn) : (TS)0;
        }
    };
    g32x4_t acc32[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc32[u][v] = g32x4_t{0.f, 0.f, 0.f, 0.f};
    double4_t acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc[u][v] = double4_t{0.0, 0.0, 0.0, 0.0};
    if (K > 0) load(0);
    for (int64_t k0 = 0; k0 < K; k0 += GK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[ak[q]][ai[q]] = ra[q];
            Bs[bk[q]][bj[q]] = rb[q];
        }
        __syncthreads();
        if (k0 + GK < K) load(k0 + GK);      // in flight during this slice's products
#pragma unroll
        for (int ks = 0; ks < GK; ks += 4) {
            TS av[2], bv[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) av[u] = As[ks + lk][qr + 16 * u + li];
#pragma unroll
            for (int v = 0; v < 2; ++v) bv[v] = Bs[ks + lk][qc + 16 * v + li];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    if constexpr (ACC32)
                        acc32[u][v] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u], bv[v], acc32[u][v], 0, 0, 0);
                    else
                        acc[u][v] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[v], acc[u][v], 0, 0, 0);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t gi = i0 + qr + 16 * u + (ACC32 ? 4 * lk + e : lk + 4 * e);
                const int64_t gj = j0 + qc + 16 * v + li;
                const double d = ACC32 ? (double)acc32[u][v][e] : acc[u][v][e];
                if (gi < M && gj < N) {
                    TC* dst = c + gi * scm + gj * scn;
                    if constexpr (MIRROR) {
                        // a tile on the diagonal writes its upper triangle and
                        // mirrors it (exactly symmetric, one writer per element)
                        const TC val = (TC)(alpha * d);
                        if (i0 != j0 || gi <= gj) {
                            *dst = val;
                            if (gi != gj) c[gj * scm + gi * scn] = val;
                        }
                    } else {
                        if constexpr (ACC32) {
                            const float old = beta != 0.0 ? (float)*dst : 0.0f;
                            *dst = (TC)((float)alpha * acc32[u][v][e] + (float)beta * old);
                        } else {
                            const double old = beta != 0.0 ? (double)*dst : 0.0;
                            *dst = (TC)(alpha * d + beta * old);
                        }
                    }
                }
            }
}

}  // namespace
}  // namespace rpmi
