// Device code shared by the projection kernels of librpmi (gfx950): tiles,
// the FP32 -> FP16 hi/lo split, A loads, pipeline helpers and the body of the
// deep-pipeline split-FP16 projection.  Included by project.hip and by the
// two files that instantiate the deep-pipeline kernel (one per column
// width), so that those heavy instantiations compile in parallel.
#pragma once
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

using SplitTile = Tile<2, 2, 2, 8, 2>;   // general split path: 64 x 256 outputs, 64-deep steps
using SplitTile128 = Tile<2, 2, 2, 4, 2>;   // same for r <= 128: 64 x 128 outputs
constexpr int kSplitDepth = 3;
// Fast path: tile and pipeline depth (A register ring and Omega LDS stages).
// Each wave owns 16 TM whole rows of the tile (A is read once per workgroup)
// and all its columns, so every Omega fragment read from LDS feeds 2 TM MFMAs.
template <class T, int D>
struct DmaCfg {
    using Tile = T;
    static constexpr int Depth = D;
};
using NarrowCfg = DmaCfg<Tile<4, 1, 2, 8, 1>, 6>; // r <= 128: 128 columns, 6-step pipeline
using DmaTile128 = NarrowCfg::Tile;
using F32Tile = Tile<2, 2, 4, 4, 1>;     // 128 x 128 outputs, 32-deep steps
constexpr int kF32Depth = 3;

// ------------------------------------------------------------------ split
// Two elements at a time: hi = RN16(a) for both with one v_cvt_pk_f16_f32,
// then lo = RN16(2^11 a - 2^11 hi) with v_fma_mix{lo,hi}_f16 reading hi as an
// FP16 half of the packed register.  2^11 a is exact in FP32 and so is the
// fused 2^11 a - 2^11 hi (a - hi is exact), so the only rounding of lo is the
// final RN16, exactly eq:shgemm-2.  2.5 VALU instructions per element.
__device__ __forceinline__ void split_pair(float a0, float a1, uint32_t& hi2, uint32_t& lo2) {
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    const half2_t h = {(_Float16)a0, (_Float16)a1};
    hi2 = __builtin_bit_cast(uint32_t, h);
    const float t0 = a0 * 2048.0f, t1 = a1 * 2048.0f;
    const float m = -2048.0f;
    uint32_t lo;
    asm("v_fma_mixlo_f16 %0, %1, %2, %3 op_sel_hi:[1,0,0]" : "=v"(lo) : "v"(hi2), "v"(m), "v"(t0));
    asm("v_fma_mixhi_f16 %0, %1, %2, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
        : "+v"(lo) : "v"(hi2), "v"(m), "v"(t1));
    lo2 = lo;
}

__device__ __forceinline__ void split8(const floatx4& a0, const floatx4& a1, half8& hi, half8& lo) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    uint32_t h0, h1, h2, h3, l0, l1, l2, l3;
    split_pair(a0[0], a0[1], h0, l0);
    split_pair(a0[2], a0[3], h1, l1);
    split_pair(a1[0], a1[1], h2, l2);
    split_pair(a1[2], a1[3], h3, l3);
    hi = __builtin_bit_cast(half8, u32x4{h0, h1, h2, h3});
    lo = __builtin_bit_cast(half8, u32x4{l0, l1, l2, l3});
}

// Single accumulator: Y = 2^-11 * sum(hi * (2^11 Omega) + lo * Omega), which
// is eq:shgemm-3 with the 2^-11 applied once in the epilogue.  2^11 Omega is
// exact in FP16 for |omega| < 32 (the Gaussian lattice stops at 9.09); a
// larger entry becomes inf and is reported like an A element out of range.
__device__ __forceinline__ half8 scale_2p11(const half8& b) {
    const _Float16 k = (_Float16)2048.0f;
    return b * half8{k, k, k, k, k, k, k, k};
}

// An element whose hi part overflows FP16 (finite |a| >= 65520), or a
// non-finite element, gives a non-finite lo part; multiplied by any Omega
// value (0 included) it leaves the lo accumulators of its whole row
// non-finite, and for in-range finite A they never are (|lo| <= 2^11 ulp(a)).
// So one check of the lo accumulators after the loop detects the condition.
template <int TM, int TN>
__device__ __forceinline__ bool any_nonfinite(const floatx4 (&acc)[TM][TN]) {
    float s = 0.0f;
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int j = 0; j < TN; ++j) s += (acc[tm][j][0] + acc[tm][j][1]) + (acc[tm][j][2] + acc[tm][j][3]);
    return !__builtin_isfinite(s * 0.0f);
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

// A register ring: the loads of step `it` land in ring slot it mod D and are
// issued D - 1 steps before they are consumed, so D - 1 steps of A stay in
// flight per wave.  The last step is loaded with per-element guards when the
// contraction length is not a multiple of the step.
template <class T, bool VEC>
struct AStream {
    const float* arow[T::TM];
    int64_t n, k_inner, s_k_outer, nsteps;
    int g;
    bool tail;

    __device__ __forceinline__ void issue(floatx4 (&dst)[T::TM][T::KS][2], int64_t it) const {
        if (it >= nsteps) return;
        const int64_t k0 = it * T::BK;
        const int64_t off = step_offset(k0, k_inner, s_k_outer);
        if (tail && it + 1 == nsteps) load_a<T, true, VEC>(dst, arow, off, k0, n, g);
        else load_a<T, false, VEC>(dst, arow, off, k0, n, g);
    }
};

template <class T, bool VEC>
__device__ __forceinline__ AStream<T, VEC> make_astream(const ProjArgs& p, int64_t bm, int wm, int c, int g) {
    AStream<T, VEC> s;
#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm) {
        int64_t row = bm * T::BM + (wm * T::TM + tm) * 16 + c;
        row = row < p.m ? row : p.m - 1;
        s.arow[tm] = p.A + row * p.s_row;
    }
    s.n = p.n; s.k_inner = p.k_inner; s.s_k_outer = p.s_k_outer;
    s.nsteps = (p.n + T::BK - 1) / T::BK;
    s.g = g;
    s.tail = (p.n % T::BK) != 0;
    return s;
}

// ------------------------------------------------------------------ split-FP16, deep pipeline
// The fast path for 16-byte aligned A.
//  * Omega reaches LDS by direct global->LDS loads (no register staging) into
//    a ring of D stages; A reaches registers through a ring of D steps.
//  * The split of step it+1 is computed while the MFMAs of step it run (two
//    sets of hi/lo registers), so the VALU work of the split hides under the
//    matrix-core work instead of adding to it.
//  * Every pipelined step issues exactly the same memory instructions (steps
//    past the end re-load the last full step into a slot nobody reads), so
//    the count of memory operations between two points is fixed and the waits
//    are exact vmcnt values: at the top of step it, everything issued before
//    the loads of step it+2 must have landed (that is: A of step it+1 for the
//    split that runs during this step, and this step's Omega stage), i.e. at
//    most D-3 steps' worth of operations may remain pending.
//  * A contraction tail shorter than a step is computed after the pipeline
//    drains, with guarded register loads.
#define RPMI_INLINE __attribute__((always_inline))
#define RPMI_LDS(p) ((__attribute__((address_space(3))) void*)(p))
#define RPMI_GLB(p) ((__attribute__((address_space(1))) void*)(p))

template <int I>
struct IntC { static constexpr int value = I; };

template <int N, class F, int I = 0>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(IntC<I>{});
        static_for<N, F, I + 1>(static_cast<F&&>(f));
    }
}

// s_waitcnt immediate for "at most N vector-memory operations pending":
// vmcnt in bits [3:0] and [15:14]; expcnt and lgkmcnt at their maxima.
template <int N>
struct VmCnt {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    static constexpr int value = (N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8);
};

// Wait until at most N vector-memory operations of this wave are pending,
// then a workgroup barrier.  The empty asm statements keep the compiler from
// moving memory accesses across.
template <int N>
__device__ __forceinline__ void wait_vm_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(VmCnt<N>::value);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// scheduling-group masks of __builtin_amdgcn_sched_group_barrier
constexpr int kSchedValu = 0x002, kSchedMfma = 0x008, kSchedVmemRead = 0x020, kSchedDsRead = 0x100;

// The body of the split-FP16 projection for output tile (bm, bn) and
// contraction share kz of problem p; tiles_n = number of column tiles of p.
template <class T, int D, bool TWO_ACC>
__device__ __forceinline__ void split_dma_body(const ProjArgs& p, const int64_t bm, const int64_t bn,
                                               const int kz, const int64_t tiles_n) {
    constexpr int STAGE = T::KS * T::NTB * 64;                 // 16-byte chunks per Omega stage
    constexpr int CH = STAGE / T::THREADS;                     // chunks per thread per stage
    constexpr int A_OPS = T::TM * T::KS * 2;                   // 16-byte A loads per step
    constexpr int OPS = CH + A_OPS;                            // memory instructions per issue
    static_assert(CH * T::THREADS == STAGE, "Omega stage must split evenly");
    static_assert(D >= 4 && D % 2 == 0, "pipeline depth: even, >= 4");
    static_assert((D - 2) * OPS < 64, "vmcnt range");
    static_assert(D <= 8, "at most 8 stages");
    // one LDS object per stage, so that the compiler can tell a stage being
    // read from the stages still being filled by direct loads
    __shared__ half8 st0[STAGE], st1[STAGE], st2[STAGE], st3[STAGE];
    __shared__ half8 st4[D > 4 ? STAGE : 1], st5[D > 5 ? STAGE : 1], st6[D > 6 ? STAGE : 1],
        st7[D > 7 ? STAGE : 1];
    auto stage_at = [&](auto slot_c) RPMI_INLINE -> half8* {
        constexpr int k = decltype(slot_c)::value;
        if constexpr (k == 0) return st0;
        else if constexpr (k == 1) return st1;
        else if constexpr (k == 2) return st2;
        else if constexpr (k == 3) return st3;
        else if constexpr (k == 4) return st4;
        else if constexpr (k == 5) return st5;
        else if constexpr (k == 6) return st6;
        else return st7;
    };

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int wm = wave % T::WM, wn = wave / T::WM;

    // this workgroup's share of the full contraction steps: [js, je)
    const int64_t nfull = p.n / T::BK;
    const int64_t nper = (nfull + p.ksplit - 1) / p.ksplit;
    const int64_t js = kz * nper < nfull ? kz * nper : nfull;
    const int64_t je = js + nper < nfull ? js + nper : nfull;
    const int64_t nsteps = je - js;
    const bool has_tail = kz == p.ksplit - 1 && nfull * T::BK < p.n;

    // A: per-lane row pointer with its 16-byte column group folded in
    const char* abase[T::TM];
#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm) {
        int64_t row = bm * T::BM + (wm * T::TM + tm) * 16 + c;
        row = row < p.m ? row : p.m - 1;
        abase[tm] = reinterpret_cast<const char*>(p.A + row * p.s_row) + 16 * g;
    }
    // Steps are issued in order from js; `jcur` is the step the next issue
    // loads and irun + iin its contraction offset inside A's runs (advanced
    // without divisions).  Issues past the last step of the share wrap back
    // to js; their data lands in slots nobody reads.
    const int64_t spr = p.k_inner / T::BK;                     // steps per contiguous run
    int64_t jcur = js;
    int64_t irun = nsteps > 0 ? (js / spr) * p.s_k_outer : 0;
    int64_t iin = nsteps > 0 ? (js % spr) * T::BK : 0;
    const int64_t irun0 = irun, iin0 = iin;
    // Omega: per-thread byte offset of its chunks inside one step's block
    const char* ombase = static_cast<const char*>(p.omega);
    const int64_t ostep = (int64_t)T::KS * p.nt_count * 64 * 16;   // bytes per step
    uint32_t ovoff[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
        const int q = tid + i * T::THREADS;
        const int kbl = q / (T::NTB * 64), jn = (q / 64) % T::NTB, ql = q % 64;
        ovoff[i] = (uint32_t)(((kbl * p.nt_count + bn * T::NTB + jn) * 64 + ql) * 16);
    }

    // accumulators: with TWO_ACC, acc holds the hi products and acc2 the lo
    // products (eq:shgemm-3 as written); otherwise one accumulator with the
    // hi products taken against 2^11 Omega
    floatx4 acc[T::TM][T::TN], acc2[TWO_ACC ? T::TM : 1][TWO_ACC ? T::TN : 1];
#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
        for (int j = 0; j < T::TN; ++j) acc[tm][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    if constexpr (TWO_ACC) {
#pragma unroll
        for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
            for (int j = 0; j < T::TN; ++j) acc2[tm][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    floatx4 ring[D][T::TM][T::KS][2];
    half8 hs[2][T::TM][T::KS], ls[2][T::TM][T::KS];   // split of the current / next step

    auto issue = [&](auto slot_c) RPMI_INLINE {
        constexpr int slot = decltype(slot_c)::value;
        const char* osrc = ombase + jcur * ostep;
#pragma unroll
        for (int i = 0; i < CH; ++i)
            __builtin_amdgcn_global_load_lds(RPMI_GLB(osrc + ovoff[i]),
                                             RPMI_LDS(stage_at(slot_c) + wave * 64 + i * T::THREADS), 16, 0, 0);
        const int64_t boff = (irun + iin) * 4;
#pragma unroll
        for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
            for (int kb = 0; kb < T::KS; ++kb)
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    ring[slot][tm][kb][h] = *reinterpret_cast<const floatx4*>(
                        abase[tm] + boff + (kb * kKBlock + h * 16) * 4);
        const bool last = jcur + 1 == je;
        iin += T::BK;
        const bool wrap = iin >= p.k_inner;
        irun += wrap ? p.s_k_outer : 0;
        iin = wrap ? 0 : iin;
        irun = last ? irun0 : irun;
        iin = last ? iin0 : iin;
        jcur = last ? js : jcur + 1;
    };

    auto split_step = [&](const floatx4 (&a)[T::TM][T::KS][2], half8 (&h)[T::TM][T::KS],
                          half8 (&l)[T::TM][T::KS]) RPMI_INLINE {
#pragma unroll
        for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
            for (int kb = 0; kb < T::KS; ++kb) split8(a[tm][kb][0], a[tm][kb][1], h[tm][kb], l[tm][kb]);
    };

    // MFMAs of one step: fragments in groups of FG; per group the hi
    // products (against 2^11 Omega) then the lo products, so the two updates
    // of one accumulator are FG * TM instructions apart.
    constexpr int FG = T::TN >= 4 ? 4 : T::TN;
    static_assert(T::TN % FG == 0, "fragment groups");
    auto mfma_step = [&](const half8 (&h)[T::TM][T::KS], const half8 (&l)[T::TM][T::KS],
                         const half8* stage) RPMI_INLINE {
#pragma unroll
        for (int kb = 0; kb < T::KS; ++kb)
#pragma unroll
            for (int j0 = 0; j0 < T::TN; j0 += FG) {
                half8 b[FG];
#pragma unroll
                for (int f = 0; f < FG; ++f) b[f] = stage[(kb * T::NTB + wn * T::TN + j0 + f) * 64 + lane];
                if constexpr (TWO_ACC) {
#pragma unroll
                    for (int f = 0; f < FG; ++f)
#pragma unroll
                        for (int tm = 0; tm < T::TM; ++tm) {
                            acc[tm][j0 + f] = __builtin_amdgcn_mfma_f32_16x16x32_f16(h[tm][kb], b[f], acc[tm][j0 + f], 0, 0, 0);
                            acc2[tm][j0 + f] = __builtin_amdgcn_mfma_f32_16x16x32_f16(l[tm][kb], b[f], acc2[tm][j0 + f], 0, 0, 0);
                        }
                } else {
#pragma unroll
                    for (int f = 0; f < FG; ++f) {
                        const half8 bs = scale_2p11(b[f]);
#pragma unroll
                        for (int tm = 0; tm < T::TM; ++tm)
                            acc[tm][j0 + f] = __builtin_amdgcn_mfma_f32_16x16x32_f16(h[tm][kb], bs, acc[tm][j0 + f], 0, 0, 0);
                    }
#pragma unroll
                    for (int f = 0; f < FG; ++f)
#pragma unroll
                        for (int tm = 0; tm < T::TM; ++tm)
                            acc[tm][j0 + f] = __builtin_amdgcn_mfma_f32_16x16x32_f16(l[tm][kb], b[f], acc[tm][j0 + f], 0, 0, 0);
                }
            }
    };

    // One pipelined step in slot s: wait + barrier (at most D-3 later issues
    // pending: this step's Omega stage and the next step's A have landed),
    // issue, then this step's MFMAs interleaved with the split of the next.
    auto step = [&](auto slot_c) RPMI_INLINE {
        constexpr int s = decltype(slot_c)::value;
        constexpr int cur = s & 1;
        wait_vm_barrier<(D - 3) * OPS>();
        // a scheduling region every kStepRegion steps (the barrier above
        // already orders the steps): larger regions schedule better, but the
        // interleaving solver's time grows steeply with the region (one region
        // per group of 6 steps takes minutes per instantiation)
        constexpr int kStepRegion = 3;
        if constexpr (s % kStepRegion == 0) __builtin_amdgcn_sched_barrier(0);
        issue(IntC<(s + D - 1) % D>{});
        mfma_step(hs[cur], ls[cur], stage_at(slot_c));
        split_step(ring[(s + 1) % D], hs[cur ^ 1], ls[cur ^ 1]);
        __builtin_amdgcn_sched_group_barrier(kSchedVmemRead, OPS, 0);
#pragma unroll
        for (int q = 0; q < 2 * T::TM * T::TN * T::KS; ++q) {
            if (q % (2 * FG * T::TM) == 0) __builtin_amdgcn_sched_group_barrier(kSchedDsRead, FG, 0);
            __builtin_amdgcn_sched_group_barrier(kSchedMfma, 1, 0);
            __builtin_amdgcn_sched_group_barrier(kSchedValu, 2, 0);
        }
    };

    if (nsteps > 0) {
        static_for<D - 1>([&](auto sc) RPMI_INLINE { issue(sc); });
        wait_vm_barrier<(D - 2) * OPS>();       // A of the first step (no LDS read yet)
        split_step(ring[0], hs[0], ls[0]);
        const int64_t ngroups = nsteps / D;
        for (int64_t grp = 0; grp < ngroups; ++grp)
            static_for<D>([&](auto sc) RPMI_INLINE { step(sc); });
        const int64_t rem = nsteps - ngroups * D;
        static_for<D>([&](auto sc) RPMI_INLINE {
            if (decltype(sc)::value < rem) step(sc);
        });
        wait_vm_barrier<0>();
    }

    if (has_tail) {   // contraction tail: guarded loads, zero-padded Omega rows
        const AStream<T, true> as = make_astream<T, true>(p, bm, wm, c, g);
        floatx4 a[T::TM][T::KS][2];
        const int64_t k0 = nfull * T::BK;
        load_a<T, true, true>(a, as.arow, step_offset(k0, p.k_inner, p.s_k_outer), k0, p.n, g);
        const half8* om = static_cast<const half8*>(p.omega);
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int q = tid + i * T::THREADS;
            const int kbl = q / (T::NTB * 64), jn = (q / 64) % T::NTB, ql = q % 64;
            st0[q] = om[((nfull * T::KS + kbl) * p.nt_count + bn * T::NTB + jn) * 64 + ql];
        }
        __syncthreads();
        split_step(a, hs[0], ls[0]);
        mfma_step(hs[0], ls[0], st0);
    }

    if constexpr (TWO_ACC) {
        // acc <- 2^11 acc_hi + acc_lo: the epilogue then scales by 2^-11 as in
        // the single-accumulator form (the 2^11 scaling is exact)
#pragma unroll
        for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
            for (int j = 0; j < T::TN; ++j) acc[tm][j] = acc[tm][j] * 2048.0f + acc2[tm][j];
    }
    if (any_nonfinite(acc)) atomicOr(p.status, kStatusRange);

    if (p.ksplit > 1) {
        // partial sums in lane order (16 bytes per lane per fragment), then the
        // last workgroup of the tile adds all ksplit partials in order z = 0, 1, ...
        const int64_t tile = bm * tiles_n + bn;
        constexpr int TILE_F4 = T::TM * T::TN * T::THREADS;      // float4s per partial tile
        floatx4* mine = reinterpret_cast<floatx4*>(p.partial) + (tile * p.ksplit + kz) * TILE_F4;
#pragma unroll
        for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
            for (int j = 0; j < T::TN; ++j) mine[(tm * T::TN + j) * T::THREADS + tid] = acc[tm][j];
        __threadfence();
        __shared__ unsigned int arrival;
        __syncthreads();
        if (tid == 0) arrival = atomicAdd(&p.counters[tile], 1u);
        __syncthreads();
        if (arrival != (unsigned)p.ksplit - 1) return;
        __threadfence();
        const floatx4* all = reinterpret_cast<const floatx4*>(p.partial) + tile * p.ksplit * TILE_F4;
#pragma unroll
        for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
            for (int j = 0; j < T::TN; ++j) {
                floatx4 sum = __builtin_nontemporal_load(&all[(tm * T::TN + j) * T::THREADS + tid]);
                for (int z = 1; z < p.ksplit; ++z)
                    sum += __builtin_nontemporal_load(&all[(z * TILE_F4) + (tm * T::TN + j) * T::THREADS + tid]);
                acc[tm][j] = sum;
            }
        if (tid == 0) p.counters[tile] = 0;   // ready for the next launch
    }

#pragma unroll
    for (int tm = 0; tm < T::TM; ++tm)
#pragma unroll
        for (int j = 0; j < T::TN; ++j) {
            const int64_t col = bn * T::BN + (wn * T::TN + j) * 16 + c;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = bm * T::BM + (wm * T::TM + tm) * 16 + 4 * g + e;
                if (row < p.m && col < p.r)
                    p.Y[row * p.ldy + col] = acc[tm][j][e] * 0x1p-11f;
            }
        }
}

// Several independent projections in one launch: block b belongs to the
// problem g with table[g].start <= b < table[g + 1].start (binary search);
// inside it, blocks enumerate (kz, bm, bn) with bn fastest.
// Several independent projections in one launch: block b belongs to the
// problem g with table[g].start <= b < table[g + 1].start (binary search on
// a block-uniform index, so the entry is read with scalar loads); inside it,
// blocks enumerate (kz, bm, bn) with bn fastest.
template <class T, int D, bool TWO_ACC>
__global__ __launch_bounds__(T::THREADS, 1) void project_split_f16_grouped_kernel(const GroupEntry* __restrict__ table,
                                                                                 int count) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = count - 1;
#pragma unroll 1
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].start <= b) lo = mid;
        else hi = mid - 1;
    }
    const GroupEntry& e = table[lo];
    const int64_t local = b - e.start;
    const int64_t tn = e.tiles_n, tm = e.tiles_m;
    const int64_t per_k = tm * tn;
    const int kz = (int)(local / per_k);
    const int64_t rest = local - kz * per_k;
    split_dma_body<T, D, TWO_ACC>(e.p, rest / tn, rest % tn, kz, tn);
}

// One projection, its arguments by value (kernel argument segment).
template <class T, int D, bool TWO_ACC>
__global__ __launch_bounds__(T::THREADS, 1) void project_split_f16_single_kernel(ProjArgs p) {
    const int64_t tn = (p.r + T::BN - 1) / T::BN, tm = (p.m + T::BM - 1) / T::BM;
    const int64_t b = blockIdx.x, per_k = tm * tn;
    const int kz = (int)(b / per_k);
    const int64_t rest = b - kz * per_k;
    split_dma_body<T, D, TWO_ACC>(p, rest / tn, rest % tn, kz, tn);
}

}  // namespace
}  // namespace rpmi
