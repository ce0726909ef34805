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
#include "proj_lds.h"

namespace rpmi {
namespace {

// ------------------------------------------------------------------ split-FP16 kernel
// One (bm, bn) tile of Y = A Omega, the whole contraction.
template <class T, int D, bool VEC>
__device__ __forceinline__ void split_f16_body(const ProjArgs& p, int64_t bm, int64_t bn) {
    __shared__ half8 lds[2][T::KS * T::NTB * 64];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int wm = wave % T::WM, wn = wave / T::WM;
    // recomputation after a folded launch: only the rows of marked blocks
    if (p.fold_flags && p.fold_flags[((bm * T::BM) / WideCfg::BM) & (kFoldFlags - 1)] != p.fold_epoch) return;

    const AStream<T, VEC> as = make_astream<T, VEC>(p, bm, wm, c, g);
    // the split's scale of this lane's rows: the caller pre-scale, or each
    // row's own power of two
    float ascale[T::TM];
#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm) {
        ascale[tm] = p.a_scale;
        if (p.row_exp) {
            int64_t row = bm * T::BM + (wm * T::TM + tm) * 16 + c;
            row = row < p.m ? row : p.m - 1;
            ascale[tm] = ldexpf(1.0f, p.row_exp[row]);
        }
    }
    const int64_t nsteps = as.nsteps;
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

    floatx4 ring[D][T::TM][T::KS][2];
    half8 ostage[CH];

#pragma unroll
    for (int s = 0; s < D - 1; ++s) as.issue(ring[s], s);
#pragma unroll
    for (int i = 0; i < CH; ++i) ostage[i] = *omega_src(0, i);
#pragma unroll
    for (int i = 0; i < CH; ++i) lds[0][tid + i * T::THREADS] = ostage[i];
    __syncthreads();

    for (int64_t it0 = 0; it0 < nsteps; it0 += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) {
            const int64_t it = it0 + s;
            if (it < nsteps) {
                as.issue(ring[(s + D - 1) % D], it + D - 1);
                const bool more = it + 1 < nsteps;
                if (more) {
#pragma unroll
                    for (int i = 0; i < CH; ++i) ostage[i] = *omega_src(it + 1, i);
                }
                const int buf = (int)(it & 1);
#pragma unroll
                for (int kb = 0; kb < T::KS; ++kb) {
                    half8 hi[T::TM], lo[T::TM];
#pragma unroll
                    for (int tm = 0; tm < T::TM; ++tm)
                        split8(ring[s][tm][kb][0] * ascale[tm], ring[s][tm][kb][1] * ascale[tm], hi[tm], lo[tm]);
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
            }
        }
    }

    if (any_nonfinite(acc_lo)) atomicOr(p.status, kStatusRange);

    // epilogue: Y = (acc_hi + 2^-11 acc_lo) 2^-s; lane (g, c) holds rows 4g..4g+3 of column c
#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
        for (int j = 0; j < T::TN; ++j) {
            const int64_t col = bn * T::BN + (wn * T::TN + j) * 16 + c;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = bm * T::BM + (wm * T::TM + tm) * 16 + 4 * g + e;
                if (row < p.m && col < p.r) {
                    const float ys = p.row_exp ? ldexpf(1.0f, -p.row_exp[row]) : p.y_scale;
                    p.Y[row * p.ldy + col] = (acc_hi[tm][j][e] + acc_lo[tm][j][e] * 0x1p-11f) * ys;
                }
            }
        }
}

template <class T, int D, bool VEC>
__global__ __launch_bounds__(T::THREADS, 1) void project_split_f16_kernel(ProjArgs p) {
    split_f16_body<T, D, VEC>(p, blockIdx.x, blockIdx.y);
}

// Several projections off the 16-byte path in one launch (element loads,
// whole contraction per tile): dense block b (see xcd_dense_block) belongs to
// the problem g with table[g].start <= b < table[g + 1].start; inside it,
// blocks enumerate (bm, bn) with bn fastest.
template <class T, int D>
__global__ __launch_bounds__(T::THREADS, 1) void project_split_f16_general_grouped_kernel(
    const GroupEntry* __restrict__ table, int count) {
    const int64_t b = xcd_dense_block(blockIdx.x, gridDim.x);
    int lo = 0, hi = count - 1;
#pragma unroll 1
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].start <= b) lo = mid;
        else hi = mid - 1;
    }
    const GroupEntry& e = table[lo];
    const int64_t local = b - e.start;
    split_f16_body<T, D, false>(e.p, local / e.tiles_n, local % e.tiles_n);
}

// ------------------------------------------------------------------ FP32 kernel
template <class T, int D, bool VEC>
__global__ __launch_bounds__(T::THREADS, 1) void project_f32_kernel(ProjArgs p) {
    // FP32 fragments: 8 floats per lane = two 16-byte halves
    __shared__ floatx4 lds[2][T::KS * T::NTB * 64 * 2];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int wm = wave % T::WM, wn = wave / T::WM;
    const int64_t bm = blockIdx.x, bn = blockIdx.y;

    const AStream<T, VEC> as = make_astream<T, VEC>(p, bm, wm, c, g);
    const int64_t nsteps = as.nsteps;
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

    floatx4 ring[D][T::TM][T::KS][2];
    floatx4 ostage[CH];

#pragma unroll
    for (int s = 0; s < D - 1; ++s) as.issue(ring[s], s);
#pragma unroll
    for (int i = 0; i < CH; ++i) ostage[i] = *omega_src(0, i);
#pragma unroll
    for (int i = 0; i < CH; ++i) lds[0][tid + i * T::THREADS] = ostage[i];
    __syncthreads();

    for (int64_t it0 = 0; it0 < nsteps; it0 += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) {
            const int64_t it = it0 + s;
            if (it < nsteps) {
                as.issue(ring[(s + D - 1) % D], it + D - 1);
                const bool more = it + 1 < nsteps;
                if (more) {
#pragma unroll
                    for (int i = 0; i < CH; ++i) ostage[i] = *omega_src(it + 1, i);
                }
                const int buf = (int)(it & 1);
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
                                    ring[s][tm][kb][t >> 2][t & 3], b[j][t >> 2][t & 3], acc[tm][j], 0, 0, 0);
                }
                if (more) {
#pragma unroll
                    for (int i = 0; i < CH; ++i) lds[buf ^ 1][tid + i * T::THREADS] = ostage[i];
                }
                __syncthreads();
            }
        }
    }

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
    // the projection kernels' own split, two elements per thread
    for (int64_t i = 2 * (blockIdx.x * (int64_t)blockDim.x + threadIdx.x); i < count;
         i += 2 * (int64_t)gridDim.x * blockDim.x) {
        const float a0 = x[i], a1 = i + 1 < count ? x[i + 1] : 0.0f;
        uint32_t h, l;
        split_pair(a0, a1, h, l);
        hi[i] = (uint16_t)h;
        lo[i] = (uint16_t)l;
        if (i + 1 < count) {
            hi[i + 1] = (uint16_t)(h >> 16);
            lo[i + 1] = (uint16_t)(l >> 16);
        }
    }
}

__global__ void fill_u32_kernel(unsigned int* p, int64_t count, unsigned int v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
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

}  // namespace

bool split_fast_ok(const ProjArgs& a) { return vector_ok(a) && !a.two_acc && a.a_scale == 1.0f && !a.row_exp; }

namespace {

// One wave per row: the largest |a| of the row (as the bit pattern of a
// non-negative float), then the exponent that brings it into [2^14, 2^15).
__global__ __launch_bounds__(256) void row_exponent_kernel(ProjArgs p, int* row_exp) {
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= p.m) return;
    const float* base = p.A + row * p.s_row;
    unsigned int mx = 0u;
    for (int64_t k = lane; k < p.n; k += 64) {
        const int64_t off = (k % p.k_inner) + (k / p.k_inner) * p.s_k_outer;
        const unsigned int v = __float_as_uint(fabsf(base[off]));
        mx = v > mx ? v : mx;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned int o = __shfl_xor(mx, d);
        mx = o > mx ? o : mx;
    }
    if (lane == 0) {
        const float amax = __uint_as_float(mx);
        int e = 0;
        if (amax > 0.0f && amax <= 3.4028235e38f) {       // finite, non-zero
            e = 14 - ilogbf(amax);
            e = e < -126 ? -126 : (e > 126 ? 126 : e);
        }
        row_exp[row] = e;
    }
}

}  // namespace

hipError_t launch_row_exponents(const ProjArgs& a, int* row_exp, hipStream_t s) {
    if (a.m <= 0) return hipSuccess;
    const int64_t blocks = (a.m + 3) / 4;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(row_exponent_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, row_exp);
    return hipGetLastError();
}

namespace {

int small_grid(int64_t total) {
    int64_t g = (total + 255) / 256;
    return (int)(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

}  // namespace

// Projections with r <= kNarrowMax use the 128-column tile, wider ones the
// 256-column tile (several column tiles when r > 256); the packed Omega is
// padded to 128 columns for r <= 128 and to multiples of 256 beyond.
constexpr int64_t kNarrowMax = 128;
int64_t split_f16_col_block(int64_t r) { return r <= 128 ? 128 : 256; }
int64_t f32_col_block() { return F32Tile::BN; }
int64_t proj_k_block() { return 64; }   // multiple of every tile's step (SplitTile 64, DmaTile 32, F32Tile 32)
static_assert(64 % SplitTile::BK == 0 && 64 % DmaTile::BK == 0 && 64 % F32Tile::BK == 0, "k block");
static_assert(NarrowLdsCfg::BN == 128 && NarrowLdsCfg::BN == DmaTile128::BN, "both narrow forms read one packing");
static_assert(SplitTile::BN == DmaTile::BN && SplitTile128::BN == DmaTile128::BN && DmaTile128::BN == 128 &&
              DmaTile::BN == 256, "both split paths read the same packed Omega");

template <class C>
SplitPlan plan_for(int64_t m, int64_t n, int64_t r, int num_cus) {
    using T = typename C::Tile;
    SplitPlan plan{1, 0, 0};
    const int64_t tiles = ((m + T::BM - 1) / T::BM) * ((r + T::BN - 1) / T::BN);
    const int64_t nfull = n / T::BK;
    if (tiles <= 0 || nfull <= 0) return plan;
    int64_t k = num_cus / tiles;                    // fill the chip with tiles x k workgroups
    constexpr int64_t kSplitMax = 64;
    k = k > kSplitMax ? kSplitMax : k;
    k = k > nfull / (2 * C::Depth) ? nfull / (2 * C::Depth) : k;   // keep shares >= 2 groups
    if (k < 2) return plan;
    plan.ksplit = (int)k;
    plan.partial_bytes = (size_t)tiles * k * T::BM * T::BN * sizeof(float);
    plan.counter_bytes = (size_t)tiles * sizeof(unsigned int);
    return plan;
}

SplitPlan plan_split_f16(int64_t m, int64_t n, int64_t r, int num_cus) {
    return r <= kNarrowMax ? plan_for<NarrowCfg>(m, n, r, num_cus) : plan_for<WideCfg>(m, n, r, num_cus);
}

SplitPlan plan_split_f16_narrow_lds(int64_t m, int64_t n, int64_t r, int num_cus) {
    return plan_for<NarrowLdsCfg>(m, n, r, num_cus);
}
int64_t split_group_tile_m_narrow_lds() { return NarrowLdsCfg::BM; }

int64_t split_group_tile_m(int64_t r) { return r <= 128 ? DmaTile128::BM : DmaTile::BM; }
int64_t split_group_tile_n(int64_t r) { return r <= 128 ? DmaTile128::BN : DmaTile::BN; }

int64_t tcec_col_block() { return TcecCfg::BN; }
SplitPlan plan_tcec(int64_t m, int64_t n, int64_t r, int num_cus) { return plan_for<TcecCfg>(m, n, r, num_cus); }

hipError_t launch_project_tcec(const ProjArgs& a, hipStream_t s) {
    using C = TcecCfg;
    if (!split_fast_ok(a) || !a.omega_lo) return hipErrorInvalidValue;
    const int64_t tiles = ((a.m + C::BM - 1) / C::BM) * ((a.r + C::BN - 1) / C::BN);
    if (tiles <= 0) return hipSuccess;
    const int64_t blocks = tiles * (a.ksplit > 1 ? a.ksplit : 1);
    hipLaunchKernelGGL((project_tcec_lds_kernel<C>), dim3((unsigned)blocks), dim3(C::THREADS), 0, s, a);
    if (a.ksplit > 1)
        hipLaunchKernelGGL((split_lds_reduce_kernel<C>), dim3((unsigned)(tiles * C::TM * C::TN)), dim3(C::THREADS), 0,
                           s, a);
    return hipGetLastError();
}

hipError_t launch_project_split_f16_grouped(const GroupEntry* table, int count, int64_t blocks, bool narrow,
                                            hipStream_t s, const GroupEntry* one, int64_t rblocks) {
    return narrow ? launch_split_group_narrow(table, count, blocks, one, s)
                  : launch_split_group_wide(table, count, blocks, one, s, rblocks);
}

// A single projection on the 16-byte path goes to the fast kernel of its
// width, passed by value (a group of one); other requests (caller pre-scale,
// two accumulators, element loads) to the general kernel.  The wide fast
// kernel takes the folded split: it marks the 256-row blocks it could not
// take in a.fold_flags, and the general kernel then recomputes exactly those
// rows (its blocks of other rows return at once).
template <class C, class TS>
hipError_t launch_split_with(const ProjArgs& a, hipStream_t s) {
    using TD = typename C::Tile;
    dim3 grid((unsigned)((a.m + TS::BM - 1) / TS::BM), (unsigned)((a.r + TS::BN - 1) / TS::BN));
    if (split_fast_ok(a)) {
        const bool wide = TD::BN != 128;
        if (wide && (!a.fold_flags || a.fold_epoch == 0)) return hipErrorInvalidValue;
        GroupEntry e;
        e.p = a;
        e.tiles_m = (a.m + TD::BM - 1) / TD::BM;
        e.tiles_n = (a.r + TD::BN - 1) / TD::BN;
        e.start = 0;
        e.rstart = 0;
        hipError_t err = launch_project_split_f16_grouped(nullptr, 0, e.tiles_m * e.tiles_n * (a.ksplit > 1 ? a.ksplit : 1),
                                                          !wide, s, &e);
        if (err != hipSuccess || !wide) return err;
        ProjArgs fb = a;
        fb.ksplit = 1;
        hipLaunchKernelGGL((project_split_f16_kernel<TS, kSplitDepth, true>), grid, dim3(TS::THREADS), 0, s, fb);
        return hipGetLastError();
    }
    ProjArgs g = a;
    g.fold_flags = nullptr;
    hipLaunchKernelGGL((project_split_f16_kernel<TS, kSplitDepth, false>), grid, dim3(TS::THREADS), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_project_split_f16(const ProjArgs& a, hipStream_t s) {
    return a.r <= kNarrowMax ? launch_split_with<NarrowCfg, SplitTile128>(a, s)
                                  : launch_split_with<WideCfg, SplitTile>(a, s);
}

// general grouped tiles: 128 columns (r <= 128), 160 (r <= 160: the
// batched problems' k + oversampling, 37.5% fewer products than a 256-column
// tile), 256
using SplitTile160 = Tile<2, 2, 2, 5, 2>;
static_assert(SplitTile160::BN == 160 && SplitTile160::BM == SplitTile::BM && SplitTile128::BM == SplitTile::BM,
              "one row tile for every width");

int split_general_width_class(int64_t r) { return r <= kNarrowMax ? 0 : (r <= SplitTile160::BN ? 1 : 2); }
int64_t split_general_tile_m(int64_t r) {
    (void)r;
    return SplitTile::BM;
}
int64_t split_general_tile_n(int64_t r) {
    const int c = split_general_width_class(r);
    return c == 0 ? SplitTile128::BN : (c == 1 ? SplitTile160::BN : SplitTile::BN);
}

hipError_t launch_project_split_f16_general_grouped(const GroupEntry* table, int count, int64_t blocks,
                                                    int width_class, hipStream_t s) {
    if (count <= 0 || blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (width_class == 0)
        hipLaunchKernelGGL((project_split_f16_general_grouped_kernel<SplitTile128, kSplitDepth>), dim3((unsigned)blocks),
                           dim3(SplitTile128::THREADS), 0, s, table, count);
    else if (width_class == 1)
        hipLaunchKernelGGL((project_split_f16_general_grouped_kernel<SplitTile160, kSplitDepth>), dim3((unsigned)blocks),
                           dim3(SplitTile160::THREADS), 0, s, table, count);
    else
        hipLaunchKernelGGL((project_split_f16_general_grouped_kernel<SplitTile, kSplitDepth>), dim3((unsigned)blocks),
                           dim3(SplitTile::THREADS), 0, s, table, count);
    return hipGetLastError();
}

hipError_t launch_project_f32(const ProjArgs& a, hipStream_t s) {
    using T = F32Tile;
    dim3 grid((unsigned)((a.m + T::BM - 1) / T::BM), (unsigned)((a.r + T::BN - 1) / T::BN));
    if (vector_ok(a))
        hipLaunchKernelGGL((project_f32_kernel<T, kF32Depth, true>), grid, dim3(T::THREADS), 0, s, a);
    else
        hipLaunchKernelGGL((project_f32_kernel<T, kF32Depth, false>), grid, dim3(T::THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_split_dump(const float* x, int64_t count, uint16_t* hi, uint16_t* lo,
                             hipStream_t s) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(split_dump_kernel, dim3(small_grid(count)), dim3(256), 0, s, x, count, hi, lo);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int* p, int64_t count, unsigned int v, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(small_grid(count)), dim3(256), 0, s, p, count, v);
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
