// Z = A^T Q with the TCEC products (Sec. 2.3, eq:tcec-5) on gfx950 FP16
// matrix cores: Algorithm 1 line 3 (B^T = A^T Q) and the power scheme's
// A^T Q, where neither operand is random and both are FP32.
//
// Both operands are split into FP16 hi = RN16(x) and lo = RN16(2^11 (x - hi)).
// One FP32 accumulator takes (2^11 hi_Q) hi_A + lo_Q hi_A + hi_Q lo_A per
// contraction step, 2^11 times the product; the epilogue scales by 2^-11.
// 2^11 hi_Q is exact in FP16 for |q| < 32 (Q has orthonormal columns).
//
// The product is formed as Z^T = Q^T A: the matrix-core A operand is Q^T
// (c rows, i contraction), read from Q packed in the projection kernels'
// fragment order (launch_pack_omega_tcec, Q as an m x p "Omega"), and the B
// operand is A (i contraction, j columns).  A is read in its own row-major
// order (rows i contiguous in j), split in registers and stored to LDS as
// FP16 rows; the B operand of a 16-column subtile then needs 8 contraction
// values per lane from 8 different rows, which ds_read_b64_tr_b16 (a
// transposing LDS read of gfx950: lane i of a 16-lane group receives element
// i mod 4 of the 8-byte chunks addressed by lanes 4e + i / 4, e = 0..3)
// delivers as two 4-row reads.
//
// Tile: a workgroup owns 128 columns c of Z (rows of Z^T) and 256 rows j of
// Z; its 8 waves form a 2 x 4 grid of 64 x 64 subtiles.  Per 32-deep step
// each thread loads 4 float4 of A (one 256-byte run per 16 lanes), splits
// and stores them; each wave loads one hi and one lo fragment of Q.  Both run
// two steps ahead in register rings (register loads only: with direct
// global->LDS loads in flight the compiler waits for every outstanding load
// before using A's registers), the LDS holds 3 stages; one workgroup barrier
// per step.  Rows beyond m are loaded clamped and zeroed; Q's padding rows
// are zero.
#include "proj_common.h"

namespace rpmi {
namespace {

constexpr int kTnBC = 128, kTnBJ = 256;       // workgroup tile: c x j
constexpr int kTnThreads = 512;
constexpr int kTnPitch = kTnBJ + 8;            // halves per LDS row of split A (bank offset per row)

typedef short v4i16 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int64_t tn_xcd_dense(int64_t b, int64_t total) {
    constexpr int kXcds = 8;
    if (total % kXcds != 0) return b;
    return (b % kXcds) * (total / kXcds) + b / kXcds;
}

// hi / lo of one float4 as two 8-byte chunks
__device__ __forceinline__ void split4(const floatx4& a, uint2& hi, uint2& lo) {
    uint32_t h0, h1, l0, l1;
    split_pair(a[0], a[1], h0, l0);
    split_pair(a[2], a[3], h1, l1);
    hi = make_uint2(h0, h1);
    lo = make_uint2(l0, l1);
}

__device__ __forceinline__ half8 tr_operand(const _Float16* rows0, const _Float16* rows16) {
    typedef __attribute__((address_space(3))) v4i16 lds_v4i16;
    const v4i16 x = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4i16*)(rows0));
    const v4i16 y = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4i16*)(rows16));
    typedef short v8i16 __attribute__((ext_vector_type(8)));
    const v8i16 v = {x[0], x[1], x[2], x[3], y[0], y[1], y[2], y[3]};
    return __builtin_bit_cast(half8, v);
}

template <bool QLO>
__global__ __launch_bounds__(kTnThreads, 1) void gemm_tn_tcec_kernel(TnTcecArgs t) {
    __shared__ _Float16 ahi0[32 * kTnPitch], ahi1[32 * kTnPitch], ahi2[32 * kTnPitch];
    __shared__ _Float16 alo0[32 * kTnPitch], alo1[32 * kTnPitch], alo2[32 * kTnPitch];
    __shared__ half8 qh0[8 * 64], qh1[8 * 64], qh2[8 * 64];
    __shared__ half8 ql0[8 * 64], ql1[8 * 64], ql2[8 * 64];
    auto ahi_at = [&](auto k) RPMI_INLINE -> _Float16* {
        if constexpr (decltype(k)::value == 0) return ahi0;
        else if constexpr (decltype(k)::value == 1) return ahi1;
        else return ahi2;
    };
    auto alo_at = [&](auto k) RPMI_INLINE -> _Float16* {
        if constexpr (decltype(k)::value == 0) return alo0;
        else if constexpr (decltype(k)::value == 1) return alo1;
        else return alo2;
    };
    auto qh_at = [&](auto k) RPMI_INLINE -> half8* {
        if constexpr (decltype(k)::value == 0) return qh0;
        else if constexpr (decltype(k)::value == 1) return qh1;
        else return qh2;
    };
    auto ql_at = [&](auto k) RPMI_INLINE -> half8* {
        if constexpr (decltype(k)::value == 0) return ql0;
        else if constexpr (decltype(k)::value == 1) return ql1;
        else return ql2;
    };

    const int64_t tiles_c = (t.p + kTnBC - 1) / kTnBC;
    const int64_t tiles = tiles_c * ((t.n + kTnBJ - 1) / kTnBJ);
    const int64_t dense = tn_xcd_dense(blockIdx.x, gridDim.x);
    const int kz = (int)(dense / tiles);
    const int64_t blk = dense - kz * tiles;
    const int64_t bc = blk % tiles_c, bj = blk / tiles_c;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wc = wave & 1, wj = wave >> 1;
    const int g = lane >> 4, c16 = lane & 15;
    // this chunk's steps: [s0, s0 + nsteps) of the (m + 31) / 32
    const int64_t all_steps = (t.m + 31) / 32;
    const int64_t s0 = t.ksplit > 1 ? kz * t.kchunk_steps : 0;
    const int64_t left = all_steps - s0;
    const int64_t nsteps = t.ksplit > 1 ? (left < t.kchunk_steps ? left : t.kchunk_steps) : all_steps;

    // A loads: thread row r (0..31), float4 columns q = (tid mod 16) + 16 u
    const int r = tid >> 4;
    const float* acol[4];
    bool colok[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int64_t j = bj * kTnBJ + 4 * ((tid & 15) + 16 * u);
        colok[u] = j < t.n;
        acol[u] = t.A + (colok[u] ? j : t.n - 4);
    }
    // (raw loads; rows past m and columns past n are zeroed when split, so
    // that no use of the loaded registers comes before that)
    auto load_a = [&](floatx4 (&dst)[4], int64_t step) RPMI_INLINE {
        const int64_t i = (s0 + step) * 32 + r;
        const int64_t ic = i < t.m ? i : t.m - 1;
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[u] = *reinterpret_cast<const floatx4*>(acol[u] + ic * t.lda);
    };
    // Q fragments: this wave loads fragment `wave` of the block's 8 (hi and
    // lo) into registers and stores them to the step's LDS stage.  (Register
    // loads throughout, rather than direct global->LDS loads, so that the
    // compiler's own waits on A count exactly.)
    const int64_t qoff = (bc * 8 + wave) * 64 + lane;
    const int64_t qstep = t.nt_count * 64;
    auto load_q = [&](half8 (&dst)[2], int64_t step) RPMI_INLINE {
        const int64_t st = s0 + (step < nsteps ? step : nsteps - 1);   // past the end: never stored
        dst[0] = static_cast<const half8*>(t.qhi)[st * qstep + qoff];
        if constexpr (QLO) dst[1] = static_cast<const half8*>(t.qlo)[st * qstep + qoff];
    };

    floatx4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

    floatx4 ra0[4], ra1[4], ra2[4];
    auto ra_at = [&](auto k) RPMI_INLINE -> floatx4(&)[4] {
        if constexpr (decltype(k)::value == 0) return ra0;
        else if constexpr (decltype(k)::value == 1) return ra1;
        else return ra2;
    };
    half8 rq0[2], rq1[2], rq2[2];
    auto rq_at = [&](auto k) RPMI_INLINE -> half8(&)[2] {
        if constexpr (decltype(k)::value == 0) return rq0;
        else if constexpr (decltype(k)::value == 1) return rq1;
        else return rq2;
    };

    // the B operand of j-subtile jb: rows 4g + s/4 (and 16 + ...), columns jb + 4 (s mod 4)
    const int trow = 4 * g + (c16 >> 2), tcol = 4 * (c16 & 3);

    auto step = [&](auto k, int64_t s) RPMI_INLINE {
        constexpr int K = decltype(k)::value;
        constexpr int K2 = (K + 2) % 3;
        // split this step's A (registers) into the LDS rows of slot K
        {
            _Float16* hrow = ahi_at(k) + r * kTnPitch;
            _Float16* lrow = alo_at(k) + r * kTnPitch;
            const bool rowok = (s0 + s) * 32 + r < t.m;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                uint2 h, l;
                split4(rowok && colok[u] ? ra_at(k)[u] : floatx4{0.f, 0.f, 0.f, 0.f}, h, l);
                const int col = 4 * ((tid & 15) + 16 * u);
                *reinterpret_cast<uint2*>(hrow + col) = h;
                *reinterpret_cast<uint2*>(lrow + col) = l;
            }
            qh_at(k)[wave * 64 + lane] = rq_at(k)[0];
            if constexpr (QLO) ql_at(k)[wave * 64 + lane] = rq_at(k)[1];
        }
        // every wave's A rows and Q fragments of this step are in LDS
        __syncthreads();
        load_a(ra_at(IntC<K2>{}), s + 2);
        load_q(rq_at(IntC<K2>{}), s + 2);
        // products
        const half8* qh = qh_at(k);
        const half8* ql = ql_at(k);
        half8 bh[4], bl[4], bh2[4];
#pragma unroll
        for (int tc = 0; tc < 4; ++tc) {
            bh[tc] = qh[(wc * 4 + tc) * 64 + lane];
            if constexpr (QLO) bl[tc] = ql[(wc * 4 + tc) * 64 + lane];
            bh2[tc] = scale_2p11(bh[tc]);
        }
        const _Float16* ah = ahi_at(k);
        const _Float16* al = alo_at(k);
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
            const int jb = wj * 64 + tj * 16 + tcol;
            const half8 xh = tr_operand(ah + trow * kTnPitch + jb, ah + (16 + trow) * kTnPitch + jb);
            const half8 xl = tr_operand(al + trow * kTnPitch + jb, al + (16 + trow) * kTnPitch + jb);
#pragma unroll
            for (int tc = 0; tc < 4; ++tc)
                acc[tc][tj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bh2[tc], xh, acc[tc][tj], 0, 0, 0);
            if constexpr (QLO) {
#pragma unroll
                for (int tc = 0; tc < 4; ++tc)
                    acc[tc][tj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bl[tc], xh, acc[tc][tj], 0, 0, 0);
            }
#pragma unroll
            for (int tc = 0; tc < 4; ++tc)
                acc[tc][tj] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bh[tc], xl, acc[tc][tj], 0, 0, 0);
        }
        // keep the next step's split (and its waits on A) out of this step
        __builtin_amdgcn_sched_barrier(0);
    };

    if (nsteps > 0) {
        load_a(ra0, 0);
        load_q(rq0, 0);
        load_a(ra1, 1);
        load_q(rq1, 1);
        const int64_t ngroups = nsteps / 3;
        for (int64_t grp = 0; grp < ngroups; ++grp)
            static_for<3>([&](auto k) RPMI_INLINE { step(k, grp * 3 + decltype(k)::value); });
        const int64_t rem = nsteps - ngroups * 3;
        static_for<3>([&](auto k) RPMI_INLINE {
            if (decltype(k)::value < rem) step(k, ngroups * 3 + decltype(k)::value);
        });
    }

    if (any_nonfinite(acc)) atomicOr(t.status, kStatusRange);

    // Z[j][c .. c + 3] = 2^-11 acc: lane (g, c16) of subtile (tc, tj) holds
    // Z^T rows c = 4g + e, column j = c16 (a chunk of a split: its partial)
    float* const zb = t.ksplit > 1 ? t.partial + kz * t.n * t.p : t.Z;
    const int64_t ldz = t.ksplit > 1 ? t.p : t.ldz;
    const bool vec = (ldz & 3) == 0 && (reinterpret_cast<uintptr_t>(zb) & 15) == 0;
#pragma unroll
    for (int tc = 0; tc < 4; ++tc)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
            const int64_t j = bj * kTnBJ + wj * 64 + tj * 16 + c16;
            const int64_t c0 = bc * kTnBC + wc * 64 + tc * 16 + 4 * g;
            if (j >= t.n) continue;
            float* dst = zb + j * ldz + c0;
            const floatx4 v = acc[tc][tj] * 0x1p-11f;
            if (vec && c0 + 3 < t.p) {
                *reinterpret_cast<floatx4*>(dst) = v;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (c0 + e < t.p) dst[e] = v[e];
            }
        }
}

// Z = the sum of the chunks' partials in a fixed order: lane group zg of a
// block adds chunks zg, zg + 8, ... of 32 consecutive outputs, then the 8
// group sums are added in group order
__global__ __launch_bounds__(256) void tn_tcec_reduce_kernel(TnTcecArgs t) {
    __shared__ float part[8][33];
    const int el = threadIdx.x & 31, zg = threadIdx.x >> 5;
    const int64_t np = t.n * t.p;
    const int64_t e = (int64_t)blockIdx.x * 32 + el;
    float acc = 0.0f;
    if (e < np)
        for (int z = zg; z < t.ksplit; z += 8) acc += t.partial[z * np + e];
    part[zg][el] = acc;
    __syncthreads();
    if (zg == 0 && e < np) {
        float sum = part[0][el];
#pragma unroll
        for (int q = 1; q < 8; ++q) sum += part[q][el];
        const int64_t j = e / t.p, c = e - j * t.p;
        t.Z[j * t.ldz + c] = sum;
    }
}

}  // namespace

int plan_tn_tcec_split(int64_t m, int64_t n, int64_t p, int cus, int64_t* chunk_steps) {
    const int64_t tiles = ((p + kTnBC - 1) / kTnBC) * ((n + kTnBJ - 1) / kTnBJ);
    const int64_t steps = (m + 31) / 32;
    *chunk_steps = steps;
    if (tiles <= 0 || steps <= 0) return 1;
    int64_t k = cus / tiles;
    k = k > steps / 16 ? steps / 16 : k;
    if (k < 2) return 1;
    const int64_t chunk = (steps + k - 1) / k;
    *chunk_steps = chunk;
    return (int)((steps + chunk - 1) / chunk);
}

hipError_t launch_gemm_tn_tcec(const TnTcecArgs& t, hipStream_t s) {
    if (t.n <= 0 || t.p <= 0) return hipSuccess;
    if ((t.n & 3) || (t.lda & 3) || (reinterpret_cast<uintptr_t>(t.A) & 15)) return hipErrorInvalidValue;
    if (t.nt_count * 16 < ((t.p + kTnBC - 1) / kTnBC) * kTnBC) return hipErrorInvalidValue;
    const int64_t steps = (t.m + 31) / 32;
    if (t.ksplit > 1 && (!t.partial || t.kchunk_steps <= 0 || (int64_t)(t.ksplit - 1) * t.kchunk_steps >= steps ||
                         (int64_t)t.ksplit * t.kchunk_steps < steps))
        return hipErrorInvalidValue;
    const int64_t tiles = ((t.p + kTnBC - 1) / kTnBC) * ((t.n + kTnBJ - 1) / kTnBJ);
    const int64_t blocks = tiles * (t.ksplit > 1 ? t.ksplit : 1);
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    if (t.qlo)
        hipLaunchKernelGGL(gemm_tn_tcec_kernel<true>, dim3((unsigned)blocks), dim3(kTnThreads), 0, s, t);
    else
        hipLaunchKernelGGL(gemm_tn_tcec_kernel<false>, dim3((unsigned)blocks), dim3(kTnThreads), 0, s, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || t.ksplit <= 1) return e;
    const int64_t g = (t.n * t.p + 31) / 32;
    if (g > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tn_tcec_reduce_kernel, dim3((unsigned)g), dim3(256), 0, s, t);
    return hipGetLastError();
}

}  // namespace rpmi
