// Gaussian random matrix Omega on the device (Sec. 3; Sec. 4.2 keeps it in FP16).
//
// Random source: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), one block
// per 4 columns of a row: element (i, j) takes word j mod 4 of the block with
// counter (i, floor(j/4), stream_id, 0) under key (seed, 0).  Low bit = sign,
// upper 63 bits = uniform u.  FP16: the magnitude is the FP16 pattern
// k = #{ t : T_t <= u } (thresholds built on the host, see lattice_host.cpp),
// so every bit is an exact integer function of (seed, stream_id, i, j) and
// identical on any device.  FP32: the same cell k, and a position inside it
// from the upper 32 bits of the word of the block with counter word 3 = 1;
// one exact FP64 product, one FP64 round-to-nearest add, one RN to FP32.
// Sparse Omega (eq:sp-rand, Sec. 2.2, without the sqrt(s) factor as Sec. 3.4
// allows): the whole word x against one threshold T = floor(2^64 / (2s)).
#include "rpmi_internal.h"

namespace rpmi {
namespace {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;

struct Words { uint64_t x[4]; };

__device__ __forceinline__ Words philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        if (rnd) { k0 += kW0; k1 += kW1; }
        const uint64_t lo0 = kM0 * c0, hi0 = __umul64hi(kM0, c0);
        const uint64_t lo1 = kM1 * c2, hi1 = __umul64hi(kM1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0;
        const uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    Words w;
    w.x[0] = c0; w.x[1] = c1; w.x[2] = c2; w.x[3] = c3;
    return w;
}

// k = #{ t : T_t <= u }: the guide table brackets k to one bucket of the
// top kGuideLog2 (16) bits of u, then a binary search inside the bucket.
__device__ __forceinline__ uint32_t f16_cell(uint64_t u, const uint64_t* __restrict__ T,
                                             const uint32_t* __restrict__ guide) {
    const uint32_t b = (uint32_t)(u >> (63 - kGuideLog2));
    uint32_t lo = guide[b], hi = guide[b + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (T[mid] <= u) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Sparse Omega (eq:sp-rand without sqrt(s)): +1, -1 or 0 from the whole word.
__device__ __forceinline__ int sparse_value(uint64_t x, uint64_t t) {
    if (x < t) return 1;
    return x - t < t ? -1 : 0;
}

__device__ __forceinline__ uint16_t f16_bits_from_word(uint64_t x, const OmegaTables& t) {
    if (t.sparse_t) {
        const int v = sparse_value(x, t.sparse_t);
        return v == 0 ? (uint16_t)0 : (v > 0 ? (uint16_t)0x3C00u : (uint16_t)0xBC00u);
    }
    const uint32_t k = f16_cell(x >> 1, t.thresholds, t.guide);
    return k == 0 ? (uint16_t)0 : (uint16_t)(k | ((uint32_t)(x & 1u) << 15));
}

// Exact value of the non-negative FP16 pattern `bits` as a double.
__device__ __forceinline__ double f16_value(uint32_t bits) {
    const uint32_t e = bits >> 10, m = bits & 0x3FFu;
    if (e == 0) return (double)m * 0x1p-24;
    return ldexp((double)(1024u + m), (int)e - 25);
}

__device__ __forceinline__ float f32_from_words(uint64_t x, uint64_t y, const OmegaTables& t) {
    if (t.sparse_t) return (float)sparse_value(x, t.sparse_t);
    const uint32_t k = f16_cell(x >> 1, t.thresholds, t.guide);
    const double upper = 0.5 * (f16_value(k) + f16_value(k + 1));
    const double lower = k == 0 ? 0.0 : 0.5 * (f16_value(k - 1) + f16_value(k));
    const double pos = ((double)(uint32_t)(y >> 32) + 0.5) * 0x1p-32;   // exact
    const double mag = __dadd_rn(lower, __dmul_rn(upper - lower, pos));  // product exact
    const float m32 = __double2float_rn(mag);
    return (x & 1u) ? -m32 : m32;
}

template <bool F32>
__global__ void omega_rowmajor_kernel(OmegaTables t, uint64_t seed, uint32_t stream_id,
                                      int64_t n, int64_t r, void* out, int64_t ldo) {
    const int64_t nb = (r + 3) >> 2;
    const int64_t total = n * nb;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / nb, b = q - i * nb;
        const Words w = philox4x64_10((uint64_t)i, (uint64_t)b, stream_id, 0, seed, 0);
        if (F32) {
            const Words v = philox4x64_10((uint64_t)i, (uint64_t)b, stream_id, 1, seed, 0);
            float* row = static_cast<float*>(out) + i * ldo;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (4 * b + e < r) row[4 * b + e] = f32_from_words(w.x[e], v.x[e], t);
        } else {
            uint16_t* row = static_cast<uint16_t*>(out) + i * ldo;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (4 * b + e < r) row[4 * b + e] = f16_bits_from_word(w.x[e], t);
        }
    }
}

__host__ __device__ __forceinline__ int frag_slot(int g, int e) {
    return e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4);
}

// One thread: fragment (kb, nt), lane group g, four adjacent columns c4.
// Eight Philox blocks (the eight rows of the group's slots) give 32 values,
// stored as the 16-byte fragments of lanes 16 g + 4 c4 + w, w = 0..3.
// FP16 Omega straight into fragment order.  A workgroup owns one 32-row
// block of the contraction and four 16-column tiles (64 columns: 4 KiB of
// fragments, contiguous in memory); each of its 256 threads runs two Philox
// blocks (one row, four consecutive columns each), places the 8 values in
// LDS at their fragment positions, and the workgroup then writes the 4 KiB
// with one 16-byte store per thread.
__device__ __forceinline__ void omega_packed_f16_block(const OmegaTables& t, uint64_t seed, uint32_t stream_id,
                                                       int64_t n, int64_t r, uint16_t* dst, int64_t nt_count,
                                                       int64_t blk) {
    __shared__ uint16_t frag[4 * 64 * 8];
    const int64_t groups = nt_count / 4;                       // 4-tile groups per 32-row block
    const int64_t kb = blk / groups, ntg = blk % groups;
    const int tid = threadIdx.x;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int pair = tid + 256 * h;                        // (rho, kappa): row in block, 4-column group
        const int rho = pair >> 4, kappa = pair & 15;
        const int64_t row = kb * kKBlock + rho;
        const int64_t j4 = ntg * 16 + kappa;                   // global 4-column group
        uint16_t v[4] = {0, 0, 0, 0};
        if (row < n && 4 * j4 < r) {
            const Words w = philox4x64_10((uint64_t)row, (uint64_t)j4, stream_id, 0, seed, 0);
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = 4 * j4 + c < r ? f16_bits_from_word(w.x[c], t) : (uint16_t)0;
        }
        // slot rho -> (g, e): rho = 4g + e (e < 4) or 16 + 4g + (e - 4)
        const int g = (rho & 15) >> 2, e = (rho & 3) + (rho >= 16 ? 4 : 0);
        const int f = kappa >> 2;
#pragma unroll
        for (int c = 0; c < 4; ++c) frag[(f * 64 + 16 * g + 4 * (kappa & 3) + c) * 8 + e] = v[c];
    }
    __syncthreads();
    const uint4 out = reinterpret_cast<const uint4*>(frag)[tid];
    reinterpret_cast<uint4*>(dst + (kb * nt_count + ntg * 4) * 64 * 8)[tid] = out;
}

__global__ __launch_bounds__(256) void omega_packed_f16_kernel(OmegaTables t, uint64_t seed, uint32_t stream_id,
                                                               int64_t n, int64_t r, uint16_t* dst,
                                                               int64_t kb_count, int64_t nt_count) {
    (void)kb_count;
    omega_packed_f16_block(t, seed, stream_id, n, r, dst, nt_count, blockIdx.x);
}

// Several problems' FP16 (or sparse) Omega in one launch: block b belongs to
// the job g with jobs[g].start <= b < jobs[g + 1].start.
__global__ __launch_bounds__(256) void omega_packed_f16_group_kernel(OmegaTables t,
                                                                     const OmegaJob* __restrict__ jobs, int count) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].start <= b) lo = mid;
        else hi = mid - 1;
    }
    const OmegaJob J = jobs[lo];
    OmegaTables tj = t;
    tj.sparse_t = J.sparse_t;
    omega_packed_f16_block(tj, J.seed, J.stream_id, J.n, J.r, static_cast<uint16_t*>(J.dst), J.nt_count,
                           b - J.start);
}

__device__ __forceinline__ float half_bits_to_float(uint16_t b) {
    return (float)__builtin_bit_cast(_Float16, b);
}

// Value of an e4m3fn code (OCP E4M3FN: bias 7, no infinities, S.1111.111 is
// NaN), exact in FP64.
__device__ __forceinline__ double e4m3_decode(uint32_t code) {
    const uint32_t e = (code >> 3) & 15u, m = code & 7u;
    double v;
    if (e == 15u && m == 7u) v = __builtin_nan("");
    else if (e == 0u) v = (double)m * 0x1p-9;
    else v = ldexp((double)(8u + m), (int)e - 10);
    return (code & 0x80u) ? -v : v;
}

// A power-of-two column scale inside [2^-7, 2^15], the range in which
// Omega8 / s is exact in FP16 for every e4m3 value.
__device__ __forceinline__ bool scale_ok(float sc) {
    int ex;
    const float f = frexpf(sc, &ex);
    return f == 0.5f && ex >= -6 && ex <= 16;
}

// Reorder a row-major Omega (FP16 bits, FP32, or e4m3 codes with column
// scales) into fragment order (FP16 or FP32 fragments).  Widening to FP32 and
// e4m3 / s_j into FP16 are exact; FP32 -> FP16 is not offered.  One thread per
// (fragment, lane).  FP16 fragments meant for the split kernels are checked:
// those kernels take the hi product against 2^11 Omega, exact below 32.
template <OmegaSrc SRC, bool DST_F32>
__global__ void pack_omega_kernel(const void* src, const float* col_scale, int64_t n, int64_t r, int64_t ldo,
                                  void* dst, int64_t kb_count, int64_t nt_count, unsigned int* flag,
                                  unsigned int flag_bit, unsigned int* status) {
    const int64_t total = kb_count * nt_count * 64;
    bool bad = false, bad_scale = false;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(q & 63), g = lane >> 4, c = lane & 15;
        const int64_t frag = q >> 6;
        const int64_t kb = frag / nt_count, nt = frag - kb * nt_count;
        const int64_t col = nt * kNTile + c;
        float fv[8];
        uint16_t hv[8];
        float sc = 1.0f;
        if (SRC == OmegaSrc::E4M3 && col < r) {
            sc = col_scale[col];
            bad_scale |= !scale_ok(sc);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t row = kb * kKBlock + frag_slot(g, e);
            const bool in = row < n && col < r;
            if (SRC == OmegaSrc::F32) {
                fv[e] = in ? static_cast<const float*>(src)[row * ldo + col] : 0.0f;
                hv[e] = 0;
            } else if (SRC == OmegaSrc::F16) {
                hv[e] = in ? static_cast<const uint16_t*>(src)[row * ldo + col] : (uint16_t)0;
                fv[e] = half_bits_to_float(hv[e]);
            } else {
                const uint32_t code = in ? static_cast<const uint8_t*>(src)[row * ldo + col] : 0u;
                fv[e] = (float)(e4m3_decode(code) / (double)sc);      // exact for a valid scale
                hv[e] = __builtin_bit_cast(uint16_t, (_Float16)fv[e]);
            }
            if (!DST_F32) bad |= (hv[e] & 0x7FFFu) >= 0x5000u;       // |v| >= 32, inf or NaN
        }
        if (DST_F32) {
            float4* d = reinterpret_cast<float4*>(static_cast<float*>(dst) + q * 8);
            d[0] = make_float4(fv[0], fv[1], fv[2], fv[3]);
            d[1] = make_float4(fv[4], fv[5], fv[6], fv[7]);
        } else {
            uint4 packed;
            packed.x = hv[0] | ((uint32_t)hv[1] << 16);
            packed.y = hv[2] | ((uint32_t)hv[3] << 16);
            packed.z = hv[4] | ((uint32_t)hv[5] << 16);
            packed.w = hv[6] | ((uint32_t)hv[7] << 16);
            *reinterpret_cast<uint4*>(static_cast<uint16_t*>(dst) + q * 8) = packed;
        }
    }
    if (flag && bad) atomicOr(flag, flag_bit);
    if (status && bad_scale) atomicOr(status, kStatusOmegaRange);
}

// TCEC packing of an FP32 right operand (eq:tcec-5): hi = RN16(w) and
// lo = RN16(2^11 (w - hi)) in fragment order, the lo fragments after all hi
// fragments.  w - hi is exact in FP32.  One thread per (fragment, lane).
__global__ void pack_omega_tcec_kernel(const float* src, int64_t n, int64_t r, int64_t ldo, uint16_t* dst,
                                       int64_t kb_count, int64_t nt_count, unsigned int* flag,
                                       unsigned int flag_bit) {
    const int64_t total = kb_count * nt_count * 64;
    bool bad = false;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(q & 63), g = lane >> 4, c = lane & 15;
        const int64_t frag = q >> 6;
        const int64_t kb = frag / nt_count, nt = frag - kb * nt_count;
        const int64_t col = nt * kNTile + c;
        uint16_t hv[8], lv[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int64_t row = kb * kKBlock + frag_slot(g, e);
            const float w = row < n && col < r ? src[row * ldo + col] : 0.0f;
            const _Float16 h = (_Float16)w;
            const _Float16 l = (_Float16)((w - (float)h) * 2048.0f);
            hv[e] = __builtin_bit_cast(uint16_t, h);
            lv[e] = __builtin_bit_cast(uint16_t, l);
            bad |= (hv[e] & 0x7FFFu) >= 0x5000u;      // |hi| >= 32, inf or NaN
        }
        uint4 ph, pl;
        ph.x = hv[0] | ((uint32_t)hv[1] << 16); ph.y = hv[2] | ((uint32_t)hv[3] << 16);
        ph.z = hv[4] | ((uint32_t)hv[5] << 16); ph.w = hv[6] | ((uint32_t)hv[7] << 16);
        pl.x = lv[0] | ((uint32_t)lv[1] << 16); pl.y = lv[2] | ((uint32_t)lv[3] << 16);
        pl.z = lv[4] | ((uint32_t)lv[5] << 16); pl.w = lv[6] | ((uint32_t)lv[7] << 16);
        *reinterpret_cast<uint4*>(dst + q * 8) = ph;
        *reinterpret_cast<uint4*>(dst + (total + q) * 8) = pl;
    }
    if (flag && bad) atomicOr(flag, flag_bit);
}

int grid_for(int64_t total, int block) {
    int64_t g = (total + block - 1) / block;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------- e4m3 Omega
// Per column j: s_j = 2^floor(log2(448 / max_i |w[i][j]|)) from the FP32
// Omega w; Omega8 = sat448(RNE_e4m3fn(w s_j)); the FP16 value Omega8 / s_j is
// exact (at most 4 significant bits, smallest step 2^-9 / s_j >= 2^-24).
__global__ void colmax_init_kernel(unsigned int* cmax, int64_t r, float* scale_one) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < r; j += (int64_t)gridDim.x * blockDim.x) {
        cmax[j] = 0u;
        if (scale_one) scale_one[j] = 1.0f;      // an empty column keeps scale 1
    }
}

// max |w| per column as the bit pattern of a non-negative float (the order of
// non-negative floats is the order of their patterns).  A block owns 64
// columns (blockIdx.x) and a strided share of the rows (blockIdx.y): each
// thread keeps the maximum of its rows, the block's four row lanes meet in
// LDS, and one atomic per column and block publishes it.
constexpr int kColmaxRowBlocks = 64;
__global__ __launch_bounds__(256) void colmax_kernel(const float* w, int64_t n, int64_t r, int64_t ldw,
                                                     unsigned int* cmax) {
    __shared__ unsigned int part[4][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + tx;
    unsigned int mx = 0u;
    if (j < r)
        for (int64_t i = (int64_t)blockIdx.y * 4 + ty; i < n; i += (int64_t)gridDim.y * 4) {
            const unsigned int v = __float_as_uint(fabsf(w[i * ldw + j]));
            mx = v > mx ? v : mx;
        }
    part[ty][tx] = mx;
    __syncthreads();
    if (ty == 0 && j < r) {
#pragma unroll
        for (int t = 1; t < 4; ++t) mx = part[t][tx] > mx ? part[t][tx] : mx;
        atomicMax(&cmax[j], mx);
    }
}

__device__ __forceinline__ double e4m3_scale(unsigned int cmax_bits) {
    const float c = __uint_as_float(cmax_bits);
    if (c == 0.0f) return 1.0;
    int ex;
    (void)frexp(448.0 / (double)c, &ex);          // 448 / c = f 2^ex, f in [1/2, 1)
    return ldexp(1.0, ex - 1);
}

__global__ void e4m3_quant_kernel(const float* w, int64_t n, int64_t r, int64_t ldw, const unsigned int* cmax,
                                  uint8_t* codes, int64_t ldc, uint16_t* f16, int64_t ldf, float* scale_out) {
    const int64_t total = n * r;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = q / r, j = q - i * r;
        const double sc = e4m3_scale(cmax[j]);
        const double x = (double)w[i * ldw + j] * sc;             // exact: power-of-two scaling
        const double a = fabs(x);
        double v = 0.0;
        if (a > 0.0) {
            const int e = ilogb(a) > -6 ? ilogb(a) : -6;
            const double qu = ldexp(1.0, e - 3);
            v = rint(a / qu) * qu;                                 // a / qu exact; rint is ties-to-even
            v = v > 448.0 ? 448.0 : v;
        }
        if (codes) {
            unsigned int code = 0;
            if (v > 0.0) {
                if (v >= 0x1p-6) {
                    const int ve = ilogb(v);
                    code = (unsigned)((ve + 7) << 3) | (unsigned)(ldexp(v, -ve) * 8.0 - 8.0);
                } else {
                    code = (unsigned)(v * 512.0);
                }
                if (x < 0.0) code |= 0x80u;
            }
            codes[i * ldc + j] = (uint8_t)code;
        }
        if (f16) {
            const double val = (x < 0.0 ? -v : v) / sc;
            f16[i * ldf + j] = v > 0.0 ? __builtin_bit_cast(uint16_t, (_Float16)(float)val) : (uint16_t)0;
        }
        if (scale_out && i == 0) scale_out[j] = (float)sc;
    }
}

}  // namespace

hipError_t launch_omega_e4m3(const OmegaTables& t, uint64_t seed, uint32_t stream_id, int64_t n, int64_t r,
                             float* w32, unsigned int* cmax, uint8_t* codes, int64_t ldc, uint16_t* f16, int64_t ldf,
                             float* scale, hipStream_t s) {
    if (r == 0) return hipSuccess;
    hipError_t e = launch_omega_rowmajor(t, seed, stream_id, n, r, true, w32, r, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colmax_init_kernel, dim3(grid_for(r, 256)), dim3(256), 0, s, cmax, r,
                       n == 0 ? scale : (float*)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    const int64_t rb = (n + 3) / 4 < kColmaxRowBlocks ? (n + 3) / 4 : kColmaxRowBlocks;
    hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)((r + 63) / 64), (unsigned)rb), dim3(256), 0, s, w32, n, r, r,
                       cmax);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(e4m3_quant_kernel, dim3(grid_for(n * r, 256)), dim3(256), 0, s, w32, n, r, r, cmax, codes, ldc,
                       f16, ldf, scale);
    return hipGetLastError();
}

namespace {
}  // namespace

hipError_t launch_omega_rowmajor(const OmegaTables& t, uint64_t seed, uint32_t stream_id,
                                 int64_t n, int64_t r, bool f32, void* out, int64_t ldo,
                                 hipStream_t s) {
    const int64_t total = n * ((r + 3) / 4);
    if (total == 0) return hipSuccess;
    const int block = 256, grid = grid_for(total, block);
    if (f32)
        hipLaunchKernelGGL(omega_rowmajor_kernel<true>, dim3(grid), dim3(block), 0, s, t, seed,
                           stream_id, n, r, out, ldo);
    else
        hipLaunchKernelGGL(omega_rowmajor_kernel<false>, dim3(grid), dim3(block), 0, s, t, seed,
                           stream_id, n, r, out, ldo);
    return hipGetLastError();
}

hipError_t launch_omega_packed_f16(const OmegaTables& t, uint64_t seed, uint32_t stream_id,
                                   int64_t n, int64_t r, const PackedOmega& dst, hipStream_t s) {
    if (dst.kb_count == 0 || dst.nt_count == 0) return hipSuccess;
    if (dst.nt_count % 4 != 0) return hipErrorInvalidValue;   // column blocks of 128 or 256
    const int64_t blocks = dst.kb_count * (dst.nt_count / 4);
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(omega_packed_f16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, t, seed, stream_id, n, r,
                       static_cast<uint16_t*>(dst.data), dst.kb_count, dst.nt_count);
    return hipGetLastError();
}

hipError_t launch_omega_packed_f16_group(const OmegaTables& t, const OmegaJob* jobs, int count, int64_t blocks,
                                         hipStream_t s) {
    if (count <= 0 || blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(omega_packed_f16_group_kernel, dim3((unsigned)blocks), dim3(256), 0, s, t, jobs, count);
    return hipGetLastError();
}

hipError_t launch_pack_omega_tcec(const float* src, int64_t n, int64_t r, int64_t ldo, const PackedOmega& dst,
                                  unsigned int* flag, unsigned int flag_bit, hipStream_t s) {
    const int64_t total = dst.kb_count * dst.nt_count * 64;
    if (total == 0) return hipSuccess;
    const int block = 256, grid = grid_for(total, block);
    hipLaunchKernelGGL(pack_omega_tcec_kernel, dim3(grid), dim3(block), 0, s, src, n, r, ldo,
                       static_cast<uint16_t*>(dst.data), dst.kb_count, dst.nt_count, flag, flag_bit);
    return hipGetLastError();
}

hipError_t launch_pack_omega(const void* src, OmegaSrc type, const float* col_scale, int64_t n, int64_t r,
                             int64_t ldo, const PackedOmega& dst, bool dst_f32, unsigned int* flag,
                             unsigned int flag_bit, unsigned int* status, hipStream_t s) {
    const int64_t total = dst.kb_count * dst.nt_count * 64;
    if (total == 0) return hipSuccess;
    const int block = 256, grid = grid_for(total, block);
    if (type == OmegaSrc::F32 && !dst_f32) return hipErrorInvalidValue;
#define RPMI_PACK(SRC, D32)                                                                                    \
    hipLaunchKernelGGL((pack_omega_kernel<SRC, D32>), dim3(grid), dim3(block), 0, s, src, col_scale, n, r, ldo, \
                       dst.data, dst.kb_count, dst.nt_count, flag, flag_bit, status)
    if (type == OmegaSrc::F32) RPMI_PACK(OmegaSrc::F32, true);
    else if (type == OmegaSrc::F16 && dst_f32) RPMI_PACK(OmegaSrc::F16, true);
    else if (type == OmegaSrc::F16) RPMI_PACK(OmegaSrc::F16, false);
    else if (dst_f32) RPMI_PACK(OmegaSrc::E4M3, true);
    else RPMI_PACK(OmegaSrc::E4M3, false);
#undef RPMI_PACK
    return hipGetLastError();
}

}  // namespace rpmi
