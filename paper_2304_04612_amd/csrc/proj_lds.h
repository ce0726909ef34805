// The LDS-staged split-FP16 projection (Sec. 4.1, eq:shgemm-1..3) for gfx950:
// the form used for the wide (256-column) tiles.
//
//  * A workgroup of 8 waves owns BM = 256 rows of A and all BN = 256 columns
//    of its output tile; wave w owns rows [32 w, 32 w + 32) and every column,
//    so each A element is split by exactly one lane and each Omega fragment
//    read from LDS feeds 4 matrix instructions (2 row subtiles x hi, lo).
//  * Both operands reach LDS by direct global->LDS loads through a ring of 3
//    stages of one 32-deep contraction step.  A wave loads its own 32 rows of
//    A: each load instruction covers 8 whole rows of the step (8 lanes x 16
//    bytes = one 128-byte line per row), with the 16-byte chunks of a row
//    XOR-swizzled by the row so that the lanes' later 16-byte LDS reads of
//    their MFMA operand hit distinct banks.  The step's Omega fragments are
//    spread over the 8 waves (2 each).
//  * At the top of a step a wave waits for its own loads of that step (exact
//    vmcnt: every step issues the same memory instructions) and a workgroup
//    barrier makes the other waves' Omega visible; the loads of step i + 2 go
//    out into the slot step i - 1 used.
//  * Two waves share a SIMD (at most 256 registers per lane: 128 accumulator
//    registers and the rest), so one wave's waits hide under the other's
//    matrix instructions; the Omega fragments of the next group of 4 are
//    read while the current group's 16 MFMAs run.
//  * Matrix-instruction issue does not overlap vector ALU work on this chip,
//    so the split keeps the VALU count per MFMA low.  Folded form (single
//    projections): x = RN16(2^11 c a), y = RN16(2^11 c a - x) with c = 2^s the
//    caller pre-scale, both against Omega as stored, so that one FP32
//    accumulator holds 2^11 c (A Omega) with no per-fragment rescaling of
//    Omega; x + y carries a to within 2^-22 relative, as the hi/lo split of
//    eq:shgemm-1/2 does (x = 2^11 hi whenever hi is normal).  x overflows for
//    |c a| >= 2^16 / 2^11 - 2^-12 (about 32): the kernel then marks its
//    256-row block with the launch's epoch and a second kernel recomputes
//    exactly those rows with the two-accumulator form, which covers the whole
//    FP16 range.  Exact form (grouped launches): hi = RN16(a), lo =
//    RN16(2^11 (a - hi)) with the hi products against 2^11 Omega.
//  * A 256-row tile halves the Omega bytes each A byte costs against 128-row
//    tiles; the contraction split that fills the chip gives every XCD a
//    contiguous run of block ids (block ids are dealt to the XCDs round
//    robin), so the workgroups of one XCD share one slice of Omega in its L2.
//  * With a contraction split the single (folded) form only writes its
//    partial sums and a second kernel adds them.  Adding them in the last
//    workgroup to arrive needs a device-scope release per workgroup, which on
//    this chip writes back the XCD's L2; at 16384 x 16384 x 256 that epilogue
//    took 40-130 us after main loops that all ended near 210 us.
#pragma once
#include "proj_common.h"

namespace rpmi {
namespace {

template <int W_, int TM_, int TN_, int S_>
struct LdsCfg {
    static constexpr int WAVES = W_, TM = TM_, TN = TN_, S = S_;
    static constexpr int THREADS = W_ * 64;
    static constexpr int BM = W_ * TM_ * 16;
    static constexpr int BN = TN_ * 16;
    static constexpr int BK = kKBlock;          // one fragment block per step
    static constexpr int KS = 1;
    static constexpr int NTB = TN_;
    static constexpr int Depth = S_;
    static constexpr int A_OPS = TM_ * 2;        // 1 KiB A blocks per wave per step (8 rows each)
    static constexpr int O_OPS = TN_ / W_;       // Omega fragments per wave per step
    static constexpr int OPS = A_OPS + O_OPS;
    static constexpr int A_F4 = BM * BK / 4;     // float4s of A per stage
    static constexpr int O_H8 = TN_ * 64;        // half8s of Omega per stage
    using Tile = LdsCfg;
    static_assert(TN_ % W_ == 0, "Omega fragments split evenly over the waves");
    static_assert(TN_ % 4 == 0, "Omega fragments in groups of 4");
    static_assert(S_ == 3, "three stages (the LDS holds three)");
    static_assert((S_ - 2) * OPS < 64, "vmcnt range");
};

// r > 128: 256-column tiles, 8 waves of 32 rows (BM = 256)
using WideCfg = LdsCfg<8, 2, 16, 3>;
using DmaTile = WideCfg;

// Block id -> dense id such that each XCD gets a contiguous run (the hardware
// deals block ids to the 8 XCDs round robin); identity when the grid does not
// divide evenly.
__device__ __forceinline__ int64_t xcd_dense_block(int64_t b, int64_t total) {
    constexpr int kXcds = 8;
    if (total % kXcds != 0) return b;
    return (b % kXcds) * (total / kXcds) + b / kXcds;
}

// Folded split of two elements: x = RN16(t), y = RN16(t - x) for t = k a
// (k = 2^11 c, exact in FP32); v_fma_mix computes -x + t exactly and rounds
// once.  2.5 VALU instructions per element, as the hi/lo split.
__device__ __forceinline__ void split_pair_fold(float a0, float a1, float k, uint32_t& x2, uint32_t& y2) {
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    const float t0 = a0 * k, t1 = a1 * k;
    const half2_t h = {(_Float16)t0, (_Float16)t1};
    x2 = __builtin_bit_cast(uint32_t, h);
    const float m = -1.0f;
    uint32_t y;
    asm("v_fma_mixlo_f16 %0, %1, %2, %3 op_sel_hi:[1,0,0]" : "=v"(y) : "v"(x2), "v"(m), "v"(t0));
    asm("v_fma_mixhi_f16 %0, %1, %2, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(y) : "v"(x2), "v"(m), "v"(t1));
    y2 = y;
}

__device__ __forceinline__ void split8_fold(const floatx4& a0, const floatx4& a1, float k, half8& x, half8& y) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    uint32_t x0, x1, x2, x3, y0, y1, y2, y3;
    split_pair_fold(a0[0], a0[1], k, x0, y0);
    split_pair_fold(a0[2], a0[3], k, x1, y1);
    split_pair_fold(a1[0], a1[1], k, x2, y2);
    split_pair_fold(a1[2], a1[3], k, x3, y3);
    x = __builtin_bit_cast(half8, u32x4{x0, x1, x2, x3});
    y = __builtin_bit_cast(half8, u32x4{y0, y1, y2, y3});
}

// PARTIAL (grouped exact form): with a contraction split only the partial
// sums are written; split_lds_group_reduce_kernel adds them.
template <class C, bool FOLD, bool TCEC = false, bool PARTIAL = false>
__device__ __forceinline__ void split_lds_body(const ProjArgs& p, const int64_t bm, const int64_t bn, const int kz,
                                               const int64_t tiles_n) {
    static_assert(!(FOLD && TCEC), "the TCEC products take the exact split");
    constexpr int TM = C::TM, TN = C::TN, S = C::S;
    constexpr int OPS = C::A_OPS + (TCEC ? 2 : 1) * C::O_OPS;   // memory instructions per step
    static_assert((S - 2) * OPS < 64, "vmcnt range");
    __shared__ floatx4 sa0[C::A_F4], sa1[C::A_F4], sa2[C::A_F4];
    __shared__ half8 so0[C::O_H8], so1[C::O_H8], so2[C::O_H8];
    __shared__ half8 sd0[TCEC ? C::O_H8 : 1], sd1[TCEC ? C::O_H8 : 1], sd2[TCEC ? C::O_H8 : 1];
    auto sa_at = [&](auto slot_c) RPMI_INLINE -> floatx4* {
        constexpr int k = decltype(slot_c)::value;
        if constexpr (k == 0) return sa0;
        else if constexpr (k == 1) return sa1;
        else return sa2;
    };
    auto so_at = [&](auto slot_c) RPMI_INLINE -> half8* {
        constexpr int k = decltype(slot_c)::value;
        if constexpr (k == 0) return so0;
        else if constexpr (k == 1) return so1;
        else return so2;
    };
    auto sd_at = [&](auto slot_c) RPMI_INLINE -> half8* {
        constexpr int k = decltype(slot_c)::value;
        if constexpr (k == 0) return sd0;
        else if constexpr (k == 1) return sd1;
        else return sd2;
    };

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, c = lane & 15;
    if (kz >= p.ksplit) return;   // a grid larger than the plan: nothing of this block exists

    // this workgroup's share of the full contraction steps: [js, je)
    const int64_t nfull = p.n / C::BK;
    const int64_t nper = (nfull + p.ksplit - 1) / p.ksplit;
    const int64_t js = kz * nper < nfull ? kz * nper : nfull;
    const int64_t je = js + nper < nfull ? js + nper : nfull;
    const int64_t nsteps = je - js;
    const bool has_tail = kz == p.ksplit - 1 && nfull * C::BK < p.n;

    // A loads: instruction q covers rows 8q .. 8q + 7 of this wave; lane l
    // loads 16-byte chunk (l mod 8) xor (l / 8) of row 8q + l / 8.  Rows past
    // m are clamped for loads and masked at the store.
    const char* arq[TM * 2];
#pragma unroll
    for (int q = 0; q < TM * 2; ++q) {
        int64_t row = bm * C::BM + wave * TM * 16 + q * 8 + (lane >> 3);
        row = row < p.m ? row : p.m - 1;
        arq[q] = reinterpret_cast<const char*>(p.A + row * p.s_row) + 16 * ((lane & 7) ^ (lane >> 3));
    }
    // the MFMA operand of (row subtile tm, half h): lane (g, c) needs row
    // 16 tm + c, chunk 4 h + g; in instruction block q = 2 tm + c / 8 it is
    // slot 8 (c mod 8) + ((4 h + g) xor (c mod 8))
    auto aread = [&](const floatx4* sa, int tm, int h) RPMI_INLINE {
        const int rl = c & 7, q = 2 * tm + (c >> 3);
        return sa[(wave * TM * 2 + q) * 64 + rl * 8 + ((4 * h + g) ^ rl)];
    };

    // step cursor: `jcur` is the step the next issue loads, irun + iin its
    // contraction offset inside A's runs (advanced without divisions); issues
    // past the end of the share wrap back to js and land in slots nobody reads
    const int64_t spr = p.k_inner / C::BK;
    int64_t jcur = js;
    int64_t irun = nsteps > 0 ? (js / spr) * p.s_k_outer : 0;
    int64_t iin = nsteps > 0 ? (js % spr) * C::BK : 0;
    const int64_t irun0 = irun, iin0 = iin;
    // Omega: fragment (step, nt) at ((step * nt_count) + nt) KiB; this wave
    // loads fragments wave * O_OPS + i of the tile's TN
    const char* obase = static_cast<const char*>(p.omega) +
                        ((bn * TN + wave * C::O_OPS) * 64 + lane) * (int64_t)sizeof(half8);
    const int64_t ostep = p.nt_count * 64 * (int64_t)sizeof(half8);
    const char* obase_lo = TCEC ? static_cast<const char*>(p.omega_lo) + (obase - static_cast<const char*>(p.omega))
                                : nullptr;
    const float kfold = 2048.0f * p.a_scale;      // exact: a power of two

    floatx4 acc[TM][TN];
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[tm][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    auto issue = [&](auto slot_c) RPMI_INLINE {
        floatx4* sa = sa_at(slot_c);
        half8* so = so_at(slot_c);
        const int64_t boff = (irun + iin) * 4;
#pragma unroll
        for (int q = 0; q < TM * 2; ++q)
            __builtin_amdgcn_global_load_lds(RPMI_GLB(arq[q] + boff), RPMI_LDS(sa + (wave * TM * 2 + q) * 64), 16, 0,
                                             0);
        const char* osrc = obase + jcur * ostep;
#pragma unroll
        for (int i = 0; i < C::O_OPS; ++i)
            __builtin_amdgcn_global_load_lds(RPMI_GLB(osrc + i * 1024), RPMI_LDS(so + (wave * C::O_OPS + i) * 64), 16,
                                             0, 0);
        if constexpr (TCEC) {
            half8* sd = sd_at(slot_c);
            const char* dsrc = obase_lo + jcur * ostep;
#pragma unroll
            for (int i = 0; i < C::O_OPS; ++i)
                __builtin_amdgcn_global_load_lds(RPMI_GLB(dsrc + i * 1024), RPMI_LDS(sd + (wave * C::O_OPS + i) * 64),
                                                 16, 0, 0);
        }
        const bool last = jcur + 1 == je;
        iin += C::BK;
        const bool wrap = iin >= p.k_inner;
        irun += wrap ? p.s_k_outer : 0;
        iin = wrap ? 0 : iin;
        irun = last ? irun0 : irun;
        iin = last ? iin0 : iin;
        jcur = last ? js : jcur + 1;
    };

    // one step's products: the split of this wave's rows, then the Omega
    // fragments in groups of 4 (the next group's LDS reads in flight while
    // the current group's 16 MFMAs run; per group the hi products, then the
    // lo products, so that two updates of one accumulator are 8 apart)
    // (TCEC: a third set, hi_A lo_W, after the lo products)
    constexpr int FG = 4, NG = TN / FG;
    auto compute = [&](const floatx4 (&a)[TM][2], const half8* so, const half8* sd) RPMI_INLINE {
        half8 bq[2][FG], bd[2][TCEC ? FG : 1];
#pragma unroll
        for (int f = 0; f < FG; ++f) bq[0][f] = so[f * 64 + lane];
        if constexpr (TCEC) {
#pragma unroll
            for (int f = 0; f < FG; ++f) bd[0][f] = sd[f * 64 + lane];
        }
        half8 hi[TM], lo[TM];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
            if constexpr (FOLD) split8_fold(a[tm][0], a[tm][1], kfold, hi[tm], lo[tm]);
            else split8(a[tm][0], a[tm][1], hi[tm], lo[tm]);
        }
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            if (q + 1 < NG) {
#pragma unroll
                for (int f = 0; f < FG; ++f) bq[(q + 1) & 1][f] = so[((q + 1) * FG + f) * 64 + lane];
                if constexpr (TCEC) {
#pragma unroll
                    for (int f = 0; f < FG; ++f) bd[(q + 1) & 1][f] = sd[((q + 1) * FG + f) * 64 + lane];
                }
            }
            half8 bh[FG];
#pragma unroll
            for (int f = 0; f < FG; ++f) bh[f] = FOLD ? bq[q & 1][f] : scale_2p11(bq[q & 1][f]);
#pragma unroll
            for (int f = 0; f < FG; ++f)
#pragma unroll
                for (int tm = 0; tm < TM; ++tm)
                    acc[tm][q * FG + f] =
                        __builtin_amdgcn_mfma_f32_16x16x32_f16(hi[tm], bh[f], acc[tm][q * FG + f], 0, 0, 0);
#pragma unroll
            for (int f = 0; f < FG; ++f)
#pragma unroll
                for (int tm = 0; tm < TM; ++tm)
                    acc[tm][q * FG + f] =
                        __builtin_amdgcn_mfma_f32_16x16x32_f16(lo[tm], bq[q & 1][f], acc[tm][q * FG + f], 0, 0, 0);
            if constexpr (TCEC) {
#pragma unroll
                for (int f = 0; f < FG; ++f)
#pragma unroll
                    for (int tm = 0; tm < TM; ++tm)
                        acc[tm][q * FG + f] =
                            __builtin_amdgcn_mfma_f32_16x16x32_f16(hi[tm], bd[q & 1][f], acc[tm][q * FG + f], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };

    auto step = [&](auto slot_c) RPMI_INLINE {
        constexpr int s = decltype(slot_c)::value;
        wait_vm_barrier<(S - 2) * OPS>();
        issue(IntC<(s + S - 1) % S>{});
        const floatx4* sa = sa_at(slot_c);
        floatx4 a[TM][2];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) { a[tm][0] = aread(sa, tm, 0); a[tm][1] = aread(sa, tm, 1); }
        compute(a, so_at(slot_c), sd_at(slot_c));
    };

    if (nsteps > 0) {
        static_for<S - 1>([&](auto sc) RPMI_INLINE { issue(sc); });
        const int64_t ngroups = nsteps / S;
        for (int64_t grp = 0; grp < ngroups; ++grp) static_for<S>([&](auto sc) RPMI_INLINE { step(sc); });
        const int64_t rem = nsteps - ngroups * S;
        static_for<S>([&](auto sc) RPMI_INLINE {
            if (decltype(sc)::value < rem) step(sc);
        });
        wait_vm_barrier<0>();   // the wrapped loads past the end have landed
    }

    if (has_tail) {   // contraction tail: guarded register loads, zero-padded Omega rows
        const int64_t k0 = nfull * C::BK;
        const int64_t off = step_offset(k0, p.k_inner, p.s_k_outer);
        floatx4 a[TM][2];
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
            int64_t row = bm * C::BM + (wave * TM + tm) * 16 + c;
            row = row < p.m ? row : p.m - 1;
            const float* ar = p.A + row * p.s_row + off;
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int kl = h * 16 + 4 * g + e;
                    a[tm][h][e] = k0 + kl < p.n ? ar[kl] : 0.0f;
                }
        }
        const half8* om = static_cast<const half8*>(p.omega);
#pragma unroll
        for (int i = 0; i < C::O_OPS; ++i) {
            const int f = wave * C::O_OPS + i;
            so0[f * 64 + lane] = om[(nfull * p.nt_count + bn * TN + f) * 64 + lane];
            if constexpr (TCEC)
                sd0[f * 64 + lane] = static_cast<const half8*>(p.omega_lo)[(nfull * p.nt_count + bn * TN + f) * 64 + lane];
        }
        __syncthreads();
        compute(a, so0, sd0);
    }

    // Range: a non-finite accumulator means an element whose x (folded) or hi
    // part overflowed FP16, or a non-finite element.  The folded form marks
    // the row block for the exact recomputation (which reports the status);
    // the exact form reports it directly.
    if (any_nonfinite(acc)) {
        if constexpr (FOLD) p.fold_flags[bm & (kFoldFlags - 1)] = p.fold_epoch;
        else atomicOr(p.status, kStatusRange);
    }
    const float yscale = FOLD ? 0x1p-11f * p.y_scale : 0x1p-11f;

    if (p.ksplit > 1) {
        // partial sums in lane order (16 bytes per lane per fragment)
        const int64_t tile = bm * tiles_n + bn;
        constexpr int TILE_F4 = TM * TN * C::THREADS;
        floatx4* mine = reinterpret_cast<floatx4*>(p.partial) + (tile * p.ksplit + kz) * TILE_F4;
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int j = 0; j < TN; ++j) mine[(tm * TN + j) * C::THREADS + tid] = acc[tm][j];
        // a second kernel (split_lds_reduce_kernel, or the grouped one) adds
        // the partials, so no workgroup waits on a device-scope release (an L2
        // write-back on this chip); otherwise the last workgroup of the tile
        // to arrive adds all ksplit partials in order z = 0, 1, ...
        if constexpr (FOLD || TCEC || PARTIAL) return;
        __threadfence();
        __shared__ unsigned int arrival;
        __syncthreads();
        if (tid == 0) arrival = atomicAdd(&p.counters[tile], 1u);
        __syncthreads();
        if (arrival != (unsigned)p.ksplit - 1) return;
        __threadfence();
        const floatx4* all = reinterpret_cast<const floatx4*>(p.partial) + tile * p.ksplit * TILE_F4;
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const int idx = (tm * TN + j) * C::THREADS + tid;
                floatx4 sum = __builtin_nontemporal_load(&all[idx]);
                for (int z = 1; z < p.ksplit; ++z) sum += __builtin_nontemporal_load(&all[z * TILE_F4 + idx]);
                acc[tm][j] = sum;
            }
        if (tid == 0) p.counters[tile] = 0;   // ready for the next launch
    }

#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int64_t col = bn * C::BN + j * 16 + c;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = bm * C::BM + (wave * TM + tm) * 16 + 4 * g + e;
                if (row < p.m && col < p.r) p.Y[row * p.ldy + col] = acc[tm][j][e] * yscale;
            }
        }
}

// Several independent projections in one launch (exact form): dense block b
// (see xcd_dense_block) belongs to the problem g with table[g].start <= b <
// table[g + 1].start; inside it, blocks enumerate (kz, bm, bn) with bn fastest.
// A problem with a contraction split leaves partial sums for
// split_lds_group_reduce_kernel.
template <class C>
__global__ __launch_bounds__(C::THREADS, 1) void project_split_lds_grouped_kernel(const GroupEntry* __restrict__ table,
                                                                                 int count) {
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
    const int64_t tn = e.tiles_n, tm = e.tiles_m;
    const int64_t per_k = tm * tn;
    const int kz = (int)(local / per_k);
    const int64_t rest = local - kz * per_k;
    split_lds_body<C, false, false, true>(e.p, rest / tn, rest % tn, kz, tn);
}

// One projection (folded form), its arguments by value (kernel argument
// segment); rows whose folded split overflows are marked in p.fold_flags.
template <class C>
__global__ __launch_bounds__(C::THREADS, 1) void project_split_lds_single_kernel(ProjArgs p) {
    const int64_t tn = (p.r + C::BN - 1) / C::BN, tm = (p.m + C::BM - 1) / C::BM;
    const int64_t b = xcd_dense_block(blockIdx.x, gridDim.x), per_k = tm * tn;
    const int kz = (int)(b / per_k);
    const int64_t rest = b - kz * per_k;
    split_lds_body<C, true>(p, rest / tn, rest % tn, kz, tn);
}

// r <= 128 in the LDS-staged form: 128-column tiles, 8 waves of 32 rows (BM =
// 256); an alternative to the register-staged narrow kernel that the
// grouped launches' autotuner may pick
using NarrowLdsCfg = LdsCfg<8, 2, 8, 3>;

// TCEC products (eq:tcec-5, both operands split): 128-column tiles, so that
// the three stages hold A and both Omega arrays (3 x 48 KiB).
using TcecCfg = LdsCfg<8, 2, 8, 3>;

template <class C>
__global__ __launch_bounds__(C::THREADS, 1) void project_tcec_lds_kernel(ProjArgs p) {
    const int64_t tn = (p.r + C::BN - 1) / C::BN, tm = (p.m + C::BM - 1) / C::BM;
    const int64_t b = xcd_dense_block(blockIdx.x, gridDim.x), per_k = tm * tn;
    const int kz = (int)(b / per_k);
    const int64_t rest = b - kz * per_k;
    split_lds_body<C, false, true>(p, rest / tn, rest % tn, kz, tn);
}

// Second pass of a projection with a contraction split: Y = 2^-11 y_scale
// sum_z partial_z, summed in the fixed order z = 0, 1, ... (the result does not
// depend on the order in which the first pass's workgroups ran).  One block
// per (tile, fragment); thread t of the block holds what thread t of the
// first pass's workgroup held for that fragment.
template <class C>
__device__ __forceinline__ void split_lds_reduce_body(const ProjArgs& p, int64_t tn, int64_t rb) {
    constexpr int TM = C::TM, TN = C::TN, NF = TM * TN, TILE_F4 = NF * C::THREADS;
    const int64_t tile = rb / NF;
    const int f = (int)(rb % NF), tm = f / TN, j = f % TN;
    const int64_t bm = tile / tn, bn = tile % tn;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 4, c = lane & 15;
    const floatx4* src = reinterpret_cast<const floatx4*>(p.partial) + tile * p.ksplit * TILE_F4 + f * C::THREADS + tid;
    floatx4 sum = __builtin_nontemporal_load(src);
    for (int z = 1; z < p.ksplit; ++z) sum += __builtin_nontemporal_load(src + (int64_t)z * TILE_F4);
    const float yscale = 0x1p-11f * p.y_scale;
    const int64_t col = bn * C::BN + j * 16 + c;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t row = bm * C::BM + (wave * TM + tm) * 16 + 4 * g + e;
        if (row < p.m && col < p.r) p.Y[row * p.ldy + col] = sum[e] * yscale;
    }
}

// single folded or TCEC projection
template <class C>
__global__ __launch_bounds__(C::THREADS) void split_lds_reduce_kernel(ProjArgs p) {
    split_lds_reduce_body<C>(p, (p.r + C::BN - 1) / C::BN, blockIdx.x);
}

// grouped launch: block b belongs to the problem g with table[g].rstart <= b
// < table[g + 1].rstart (problems without a split own no blocks)
template <class C>
__global__ __launch_bounds__(C::THREADS) void split_lds_group_reduce_kernel(const GroupEntry* __restrict__ table,
                                                                            int count) {
    const int64_t b = blockIdx.x;
    int lo = 0, hi = count - 1;
#pragma unroll 1
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].rstart <= b) lo = mid;
        else hi = mid - 1;
    }
    const GroupEntry& e = table[lo];
    split_lds_reduce_body<C>(e.p, e.tiles_n, b - e.rstart);
}

}  // namespace
}  // namespace rpmi
