// Y = A * Omega on gfx950 matrix cores.
//
// Split-FP16 path (Sec. 4.1, eq:shgemm-1..3): every FP32 element a of A is
// split in registers, as it arrives from HBM, into
//     hi = RN16(a),   lo = RN16((a - hi) * 2^11)
// and the two FP16 products hi * Omega and lo * Omega run on
// v_mfma_f32_16x16x32_f16 with FP32 accumulation in two accumulators; the
// epilogue forms Y = acc_hi + 2^-11 acc_lo.  The split is never written to
// memory.  Omega is FP16 and arrives in fragment order (rpmi_internal.h), is
// staged through LDS once per workgroup and read back with one 16-byte LDS
// load per lane per fragment.
//
// FP32 path (the baseline form): the same tiling with v_mfma_f32_16x16x4_f32
// on FP32 A and FP32 Omega fragments.
//
// Tiling: a workgroup owns BM rows of A and BN columns of Y; its 4 waves form
// a WM x WN grid, each wave computing (16 TM) x (16 TN) outputs.  A is read
// straight into registers (two 16-byte loads per lane per 32-row block of the
// contraction; lanes of one row read 64 contiguous bytes per load); the next
// step's A and Omega are in flight while the current step computes (register
// double buffering for A, LDS double buffering for Omega, one barrier per
// step).  Rows beyond m are clamped for loads and masked for stores; a
// contraction tail shorter than a step is loaded with per-element guards and
// multiplies zero-padded Omega rows.
#include "rpmi_internal.h"

namespace rpmi {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int WM_, int WN_, int TM_, int TN_, int KS_>
struct Tile {
    static constexpr int WM = WM_, WN = WN_, TM = TM_, TN = TN_, KS = KS_;
    static constexpr int BM = WM * TM * 16;
    static constexpr int BN = WN * TN * 16;
    static constexpr int BK = kKBlock * KS;
    static constexpr int THREADS = WM * WN * 64;
    static constexpr int NTB = BN / kNTile;
};

using SplitTile = Tile<2, 2, 2, 8, 2>;   // 64 x 256 outputs, 64-deep steps
using F32Tile = Tile<2, 2, 4, 4, 1>;     // 128 x 128 outputs, 32-deep steps

// ------------------------------------------------------------------ split
__device__ __forceinline__ void split_one(float a, _Float16& hi, _Float16& lo) {
    hi = (_Float16)a;                                   // RN to FP16
    lo = (_Float16)((a - (float)hi) * 2048.0f);        // exact difference, exact scaling, RN
}

__device__ __forceinline__ void split8(const floatx4& a0, const floatx4& a1, half8& hi, half8& lo,
                                       float& amax) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        _Float16 h, l;
        split_one(a0[e], h, l);
        hi[e] = h; lo[e] = l;
        split_one(a1[e], h, l);
        hi[4 + e] = h; lo[4 + e] = l;
        amax = fmaxf(amax, fmaxf(fabsf(a0[e]), fabsf(a1[e])));
    }
}

// ------------------------------------------------------------------ A loads
// Row pointer per row subtile; per step the contraction offset `koff` of the
// step's first element (the step lies inside one contiguous run of A).
template <class T, bool MASK, bool VEC>
__device__ __forceinline__ void load_a(floatx4 (&a)[T::TM][T::KS][2], const float* const (&arow)[T::TM],
                                       int64_t koff, int64_t k0, int64_t n, int g) {
#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
        for (int kb = 0; kb < T::KS; ++kb)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int kl = kb * kKBlock + h * 16 + 4 * g;
                const float* p = arow[tm] + koff + kl;
                if (VEC && (!MASK || k0 + kl + 3 < n)) {
                    a[tm][kb][h] = *reinterpret_cast<const floatx4*>(p);
                } else if (!MASK) {
                    a[tm][kb][h] = floatx4{p[0], p[1], p[2], p[3]};
                } else {
                    floatx4 v;
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = (k0 + kl + e < n) ? p[e] : 0.0f;
                    a[tm][kb][h] = v;
                }
            }
}

// Contraction offset of step `it`: runs of k_inner contiguous elements,
// consecutive runs s_k_outer apart.
__device__ __forceinline__ int64_t step_offset(int64_t k0, int64_t k_inner, int64_t s_k_outer) {
    const int64_t o = k0 / k_inner;
    return o * s_k_outer + (k0 - o * k_inner);
}

// ------------------------------------------------------------------ split-FP16 kernel
template <class T, bool VEC>
__global__ __launch_bounds__(T::THREADS, 1) void project_split_f16_kernel(ProjArgs p) {
    __shared__ half8 lds[2][T::KS * T::NTB * 64];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int wm = wave % T::WM, wn = wave / T::WM;
    const int64_t bm = blockIdx.x, bn = blockIdx.y;

    const float* arow[T::TM];
#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm) {
        int64_t row = bm * T::BM + (wm * T::TM + tm) * 16 + c;
        row = row < p.m ? row : p.m - 1;
        arow[tm] = p.A + row * p.s_row;
    }

    const int64_t nsteps = (p.n + T::BK - 1) / T::BK;
    const bool tail = (p.n % T::BK) != 0;
    const half8* om = static_cast<const half8*>(p.omega);

    constexpr int CH = T::KS * T::NTB * 64 / T::THREADS;   // 16-byte chunks per thread
    static_assert(CH * T::THREADS == T::KS * T::NTB * 64, "Omega stage must split evenly");
    auto omega_src = [&](int64_t it, int i) -> const half8* {
        const int q = tid + i * T::THREADS;
        const int kbl = q / (T::NTB * 64), j = (q / 64) % T::NTB, ql = q % 64;
        return om + (((it * T::KS + kbl) * p.nt_count + bn * T::NTB + j) * 64 + ql);
    };

    floatx4 acc_hi[T::TM][T::TN], acc_lo[T::TM][T::TN];
#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
        for (int j = 0; j < T::TN; ++j) {
            acc_hi[tm][j] = floatx4{0.f, 0.f, 0.f, 0.f};
            acc_lo[tm][j] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    float amax = 0.0f;

    floatx4 abuf[2][T::TM][T::KS][2];
    half8 ostage[CH];

    // prologue: step 0
    if (nsteps == 1 && tail)
        load_a<T, true, VEC>(abuf[0], arow, step_offset(0, p.k_inner, p.s_k_outer), 0, p.n, g);
    else
        load_a<T, false, VEC>(abuf[0], arow, step_offset(0, p.k_inner, p.s_k_outer), 0, p.n, g);
#pragma unroll
    for (int i = 0; i < CH; ++i) ostage[i] = *omega_src(0, i);
#pragma unroll
    for (int i = 0; i < CH; ++i) lds[0][tid + i * T::THREADS] = ostage[i];
    __syncthreads();

    auto step = [&](int64_t it, floatx4 (&cur)[T::TM][T::KS][2], floatx4 (&nxt)[T::TM][T::KS][2]) {
        const int buf = (int)(it & 1);
        const bool more = it + 1 < nsteps;
        if (more) {
            const int64_t k1 = (it + 1) * T::BK;
            const int64_t off = step_offset(k1, p.k_inner, p.s_k_outer);
            if (tail && it + 2 == nsteps)
                load_a<T, true, VEC>(nxt, arow, off, k1, p.n, g);
            else
                load_a<T, false, VEC>(nxt, arow, off, k1, p.n, g);
#pragma unroll
            for (int i = 0; i < CH; ++i) ostage[i] = *omega_src(it + 1, i);
        }
#pragma unroll
        for (int kb = 0; kb < T::KS; ++kb) {
            half8 hi[T::TM], lo[T::TM];
#pragma unroll
            for (int tm = 0; tm < T::TM; ++tm) split8(cur[tm][kb][0], cur[tm][kb][1], hi[tm], lo[tm], amax);
#pragma unroll
            for (int j = 0; j < T::TN; ++j) {
                const half8 b = lds[buf][(kb * T::NTB + wn * T::TN + j) * 64 + lane];
#pragma unroll
                for (int tm = 0; tm < T::TM; ++tm) {
                    acc_hi[tm][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(hi[tm], b, acc_hi[tm][j], 0, 0, 0);
                    acc_lo[tm][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(lo[tm], b, acc_lo[tm][j], 0, 0, 0);
                }
            }
        }
        if (more) {
#pragma unroll
            for (int i = 0; i < CH; ++i) lds[buf ^ 1][tid + i * T::THREADS] = ostage[i];
        }
        __syncthreads();
    };

    int64_t it = 0;
    for (; it + 1 < nsteps; it += 2) {
        step(it, abuf[0], abuf[1]);
        step(it + 1, abuf[1], abuf[0]);
    }
    if (it < nsteps) step(it, abuf[0], abuf[1]);

    if (amax >= 65520.0f) atomicOr(p.status, kStatusRange);

    // epilogue: Y = acc_hi + 2^-11 acc_lo; lane (g, c) holds rows 4g..4g+3 of column c
#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
        for (int j = 0; j < T::TN; ++j) {
            const int64_t col = bn * T::BN + (wn * T::TN + j) * 16 + c;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = bm * T::BM + (wm * T::TM + tm) * 16 + 4 * g + e;
                if (row < p.m && col < p.r)
                    p.Y[row * p.ldy + col] = acc_hi[tm][j][e] + acc_lo[tm][j][e] * 0x1p-11f;
            }
        }
}

// ------------------------------------------------------------------ FP32 kernel
template <class T, bool VEC>
__global__ __launch_bounds__(T::THREADS, 1) void project_f32_kernel(ProjArgs p) {
    // FP32 fragments: 8 floats per lane = two 16-byte halves
    __shared__ floatx4 lds[2][T::KS * T::NTB * 64 * 2];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int wm = wave % T::WM, wn = wave / T::WM;
    const int64_t bm = blockIdx.x, bn = blockIdx.y;

    const float* arow[T::TM];
#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm) {
        int64_t row = bm * T::BM + (wm * T::TM + tm) * 16 + c;
        row = row < p.m ? row : p.m - 1;
        arow[tm] = p.A + row * p.s_row;
    }

    const int64_t nsteps = (p.n + T::BK - 1) / T::BK;
    const bool tail = (p.n % T::BK) != 0;
    const floatx4* om = static_cast<const floatx4*>(p.omega);

    constexpr int CH = T::KS * T::NTB * 64 * 2 / T::THREADS;
    static_assert(CH * T::THREADS == T::KS * T::NTB * 64 * 2, "Omega stage must split evenly");
    auto omega_src = [&](int64_t it, int i) -> const floatx4* {
        const int q = tid + i * T::THREADS;                  // 16-byte chunk in the stage
        const int kbl = q / (T::NTB * 128), rest = q % (T::NTB * 128);
        return om + ((it * T::KS + kbl) * p.nt_count + bn * T::NTB) * 128 + rest;
    };

    floatx4 acc[T::TM][T::TN];
#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
        for (int j = 0; j < T::TN; ++j) acc[tm][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    floatx4 abuf[2][T::TM][T::KS][2];
    floatx4 ostage[CH];

    if (nsteps == 1 && tail)
        load_a<T, true, VEC>(abuf[0], arow, step_offset(0, p.k_inner, p.s_k_outer), 0, p.n, g);
    else
        load_a<T, false, VEC>(abuf[0], arow, step_offset(0, p.k_inner, p.s_k_outer), 0, p.n, g);
#pragma unroll
    for (int i = 0; i < CH; ++i) ostage[i] = *omega_src(0, i);
#pragma unroll
    for (int i = 0; i < CH; ++i) lds[0][tid + i * T::THREADS] = ostage[i];
    __syncthreads();

    auto step = [&](int64_t it, floatx4 (&cur)[T::TM][T::KS][2], floatx4 (&nxt)[T::TM][T::KS][2]) {
        const int buf = (int)(it & 1);
        const bool more = it + 1 < nsteps;
        if (more) {
            const int64_t k1 = (it + 1) * T::BK;
            const int64_t off = step_offset(k1, p.k_inner, p.s_k_outer);
            if (tail && it + 2 == nsteps)
                load_a<T, true, VEC>(nxt, arow, off, k1, p.n, g);
            else
                load_a<T, false, VEC>(nxt, arow, off, k1, p.n, g);
#pragma unroll
            for (int i = 0; i < CH; ++i) ostage[i] = *omega_src(it + 1, i);
        }
#pragma unroll
        for (int kb = 0; kb < T::KS; ++kb) {
            floatx4 b[T::TN][2];
#pragma unroll
            for (int j = 0; j < T::TN; ++j) {
                const int f = ((kb * T::NTB + wn * T::TN + j) * 64 + lane) * 2;
                b[j][0] = lds[buf][f];
                b[j][1] = lds[buf][f + 1];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t)
#pragma unroll
                for (int j = 0; j < T::TN; ++j)
#pragma unroll
                    for (int tm = 0; tm < T::TM; ++tm)
                        acc[tm][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            cur[tm][kb][t >> 2][t & 3], b[j][t >> 2][t & 3], acc[tm][j], 0, 0, 0);
        }
        if (more) {
#pragma unroll
            for (int i = 0; i < CH; ++i) lds[buf ^ 1][tid + i * T::THREADS] = ostage[i];
        }
        __syncthreads();
    };

    int64_t it = 0;
    for (; it + 1 < nsteps; it += 2) {
        step(it, abuf[0], abuf[1]);
        step(it + 1, abuf[1], abuf[0]);
    }
    if (it < nsteps) step(it, abuf[0], abuf[1]);

#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
        for (int j = 0; j < T::TN; ++j) {
            const int64_t col = bn * T::BN + (wn * T::TN + j) * 16 + c;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = bm * T::BM + (wm * T::TM + tm) * 16 + 4 * g + e;
                if (row < p.m && col < p.r) p.Y[row * p.ldy + col] = acc[tm][j][e];
            }
        }
}

// ------------------------------------------------------------------ small kernels
__global__ void split_dump_kernel(const float* x, int64_t count, uint16_t* hi, uint16_t* lo) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        _Float16 h, l;
        split_one(x[i], h, l);
        hi[i] = __builtin_bit_cast(uint16_t, h);
        lo[i] = __builtin_bit_cast(uint16_t, l);
    }
}

__global__ void fill_f32_kernel(float* y, int64_t rows, int64_t cols, int64_t ld, float v) {
    const int64_t total = rows * cols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / cols;
        y[r * ld + (i - r * cols)] = v;
    }
}

// 16-byte loads need a 16-byte aligned base and row / run strides that
// keep every 4-element group aligned; otherwise the kernels load element-wise.
bool vector_ok(const ProjArgs& a) {
    return (reinterpret_cast<uintptr_t>(a.A) & 15) == 0 && (a.s_row & 3) == 0 &&
           (a.s_k_outer & 3) == 0 && (a.k_inner & 3) == 0;
}

int small_grid(int64_t total) {
    int64_t g = (total + 255) / 256;
    return (int)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

}  // namespace

int64_t split_f16_col_block() { return SplitTile::BN; }
int64_t f32_col_block() { return F32Tile::BN; }
int64_t proj_k_block() { return SplitTile::BK > F32Tile::BK ? SplitTile::BK : F32Tile::BK; }

hipError_t launch_project_split_f16(const ProjArgs& a, hipStream_t s) {
    using T = SplitTile;
    dim3 grid((unsigned)((a.m + T::BM - 1) / T::BM), (unsigned)((a.r + T::BN - 1) / T::BN));
    if (vector_ok(a))
        hipLaunchKernelGGL((project_split_f16_kernel<T, true>), grid, dim3(T::THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((project_split_f16_kernel<T, false>), grid, dim3(T::THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_project_f32(const ProjArgs& a, hipStream_t s) {
    using T = F32Tile;
    dim3 grid((unsigned)((a.m + T::BM - 1) / T::BM), (unsigned)((a.r + T::BN - 1) / T::BN));
    if (vector_ok(a))
        hipLaunchKernelGGL((project_f32_kernel<T, true>), grid, dim3(T::THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((project_f32_kernel<T, false>), grid, dim3(T::THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_split_dump(const float* x, int64_t count, uint16_t* hi, uint16_t* lo,
                             hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(split_dump_kernel, dim3(small_grid(count)), dim3(256), 0, s, x, count, hi, lo);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* y, int64_t rows, int64_t cols, int64_t ld, float v,
                           hipStream_t s) {
    if (rows * cols == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(small_grid(rows * cols)), dim3(256), 0, s, y, rows,
                       cols, ld, v);
    return hipGetLastError();
}

}  // namespace rpmi
