// Internal declarations shared by the host runtime and the kernel files of
// librpmi.  Not part of the public ABI (include/rpmi.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpmi {

// ---------------------------------------------------------------- Omega tables
constexpr int kF16TableMax = 20000;   // threshold table capacity (18571 used)
constexpr int kGuideLog2 = 16;        // guide table over the top 16 bits of u (256 KiB)
constexpr int kGuideSize = (1 << kGuideLog2) + 1;

struct OmegaTables {
    const uint64_t* thresholds;       // device, count entries
    const uint32_t* guide;            // device, kGuideSize entries
    int count;
    // 0: the Gaussian; else a sparse Omega of entries in {-1, 0, +1}: +1 for
    // a word x < sparse_t, -1 for sparse_t <= x < 2 sparse_t, else 0
    uint64_t sparse_t = 0;
};

// ---------------------------------------------------------------- packed Omega
// The projection kernels read Omega in "fragment" order: for every block of
// 32 contraction rows (kb) and 16 columns (nt) one fragment holds, for lane
// l = 16 g + c of a 64-wide wave, the 8 values Omega[32 kb + slot(g, e)][16 nt + c],
// e = 0..7, with slot(g, e) = 4 g + e for e < 4 and 16 + 4 g + (e - 4) for
// e >= 4.  A lane of the A operand holds A[row][32 kb + slot(g, e)] for the
// same (g, e), which makes its two 16-byte loads of A contiguous in memory.
// Fragments are stored kb-major: frag(kb, nt) at index kb * NT + nt.
// FP16 fragments are 64 x 8 halves (1 KiB), FP32 fragments 64 x 8 floats.
constexpr int kKBlock = 32;           // contraction rows per fragment
constexpr int kNTile = 16;            // columns per fragment

struct PackedOmega {
    void* data;                       // device
    int64_t kb_count;                 // number of 32-row blocks (covers n, zero padded)
    int64_t nt_count;                 // number of 16-column tiles (covers r, zero padded)
};

// ---------------------------------------------------------------- projection
struct ProjArgs {
    const float* A = nullptr;
    int64_t m = 0, n = 0;
    int64_t s_row = 0, k_inner = 1, s_k_outer = 0;
    const void* omega = nullptr;      // packed fragments (FP16 or FP32)
    int64_t nt_count = 0;             // fragment tiles per 32-row block
    float* Y = nullptr;
    int64_t ldy = 0, r = 0;
    unsigned int* status = nullptr;   // device status word
    // contraction split (split-FP16 path): ksplit workgroups share one output
    // tile; each writes its partial sums to `partial`, the last one to finish
    // (per-tile counter) adds them in a fixed order and writes Y
    int ksplit = 1;
    float* partial = nullptr;         // ksplit * tiles * BM * BN floats
    unsigned int* counters = nullptr; // one per output tile, zero between launches
    // caller pre-scale of A (split path): the split takes a_scale * A and the
    // epilogue multiplies by y_scale; a_scale = 2^s, y_scale = 2^-s, both exact
    float a_scale = 1.0f, y_scale = 1.0f;
    // host-side routing: take the general kernel with two accumulators
    // (eq:shgemm-3 as written), which has no bound on |Omega|
    bool two_acc = false;
    // folded split of single wide projections: a 256-row block whose folded
    // split overflowed is marked fold_flags[block mod kFoldFlags] =
    // fold_epoch, and the general kernel then recomputes the rows of marked
    // blocks (a block sharing a flag with a marked one is recomputed too,
    // which changes nothing); fold_epoch is distinct per launch and never 0
    unsigned int* fold_flags = nullptr;
    unsigned int fold_epoch = 0;
    // TCEC products (both operands split, eq:tcec-5): `omega` holds the FP16
    // hi fragments of the FP32 right operand and `omega_lo` its FP16
    // RN16(2^11 (w - hi)) fragments, in the same order
    const void* omega_lo = nullptr;
    // automatic per-row pre-scale (full FP32 exponent range of A): row i of
    // A is split as 2^row_exp[i] a and row i of Y multiplied by 2^-row_exp[i]
    // (a_scale and y_scale are then 1); general kernel only
    const int* row_exp = nullptr;
};
// row_exp[i] = the power of two that brings max_k |A[i][k]| into [2^14, 2^15)
// (clamped to [-126, 126]; 0 for an all-zero or non-finite row), over the
// unfolding layout of `a` (its A, m, n, s_row, k_inner, s_k_outer)
hipError_t launch_row_exponents(const ProjArgs& a, int* row_exp, hipStream_t s);
constexpr int kFoldFlags = 4096;      // flag table of the folded split (power of two)

// Several split-FP16 projections in one launch (all on the 16-byte path and
// of one column width: r <= 128 or r > 128).  The problem table lives in
// device memory; entry g owns blocks [start, start + tiles_m * tiles_n *
// ksplit), and entries are sorted by start.
constexpr int kMaxGroup = 8;          // modes of rp_hosvd
struct GroupEntry {
    ProjArgs p;
    int64_t tiles_m, tiles_n;
    int64_t start;
    int64_t rstart;                   // LDS-staged launches: first block of the reduction pass
};
// reduction-pass blocks of a problem with `tiles` output tiles and a
// contraction split on an LDS-staged grouped launch (narrow_lds: the
// r <= 128 form, else the wide one)
int64_t split_group_reduce_blocks(int64_t tiles, bool narrow_lds);
int64_t split_group_tile_m(int64_t r);
int64_t split_group_tile_n(int64_t r);
// `one` != NULL: a single problem passed by value (table and count unused)
// rblocks: blocks of the reduction pass (wide grouped launches)
hipError_t launch_project_split_f16_grouped(const GroupEntry* table, int count, int64_t blocks, bool narrow,
                                            hipStream_t s, const GroupEntry* one = nullptr, int64_t rblocks = 0);
hipError_t launch_split_group_wide(const GroupEntry* table, int count, int64_t blocks, const GroupEntry* one,
                                   hipStream_t s, int64_t rblocks = 0);
hipError_t launch_split_group_narrow(const GroupEntry* table, int count, int64_t blocks, const GroupEntry* one,
                                     hipStream_t s);
bool split_fast_ok(const ProjArgs& a);
// Projections of any layout (element loads, two accumulators, no contraction
// split; entries' fold_flags must be null) in one table-driven launch per
// column width class (0: r <= 128, 1: r <= 160, 2: wider); tiles from
// split_general_tile_m/_n.
int split_general_width_class(int64_t r);
int64_t split_general_tile_m(int64_t r);
int64_t split_general_tile_n(int64_t r);
hipError_t launch_project_split_f16_general_grouped(const GroupEntry* table, int count, int64_t blocks,
                                                    int width_class, hipStream_t s);

// Workspace the split-FP16 projection needs for (m, r) (0 if none) and the
// contraction split it will use; the counters must be zero initially.
struct SplitPlan {
    int ksplit;
    size_t partial_bytes;
    size_t counter_bytes;
};
SplitPlan plan_split_f16(int64_t m, int64_t n, int64_t r, int num_cus);
// The LDS-staged form of the narrow (r <= 128) grouped launch: its plan,
// its row tile (the column tile is 128 as in the register-staged form) and
// its launch.
SplitPlan plan_split_f16_narrow_lds(int64_t m, int64_t n, int64_t r, int num_cus);
int64_t split_group_tile_m_narrow_lds();
hipError_t launch_split_group_narrow_lds(const GroupEntry* table, int count, int64_t blocks, int64_t rblocks,
                                         hipStream_t s);

// Scratch of the no-allocation projection entry point (one static device
// array per device): partial sums first, then the arrival counters.  The
// planner never gives tiles x ksplit more workgroups than compute units, and
// a tile is at most 256 x 256 floats, so the partial sums of any split fit
// in num_cus x 256 KiB: 64 MiB on a 256-CU device.
constexpr size_t kNoAllocPartialBytes = size_t(64) << 20;
constexpr size_t kNoAllocCounterBytes = 4096;
// Device address of that array on the current device.
hipError_t noalloc_scratch_address(void** out);

constexpr unsigned int kStatusRange = 1u;
constexpr unsigned int kStatusNotSpd = 2u;
constexpr unsigned int kStatusNotConverged = 4u;
constexpr unsigned int kStatusOmegaRange = 8u;

// Column padding the packed Omega must provide for each algorithm: the
// kernels read whole column blocks.
int64_t split_f16_col_block(int64_t r);   // 128 for r <= 128, else 256
int64_t f32_col_block();
int64_t proj_k_block();               // contraction rows per main-loop step

hipError_t launch_omega_rowmajor(const OmegaTables& t, uint64_t seed, uint32_t stream_id,
                                 int64_t n, int64_t r, bool f32, void* out, int64_t ldo,
                                 hipStream_t s);
// e4m3 Omega (Omega8 = sat448(RNE_e4m3(w s_j)), s_j a power of two per
// column, w the FP32 Omega): w32 (n x r) and cmax (r) are scratch; codes
// (e4m3fn bytes), f16 (the exact FP16 values Omega8 / s_j) and scale (s_j) are
// written when not NULL.
hipError_t launch_omega_e4m3(const OmegaTables& t, uint64_t seed, uint32_t stream_id, int64_t n, int64_t r,
                             float* w32, unsigned int* cmax, uint8_t* codes, int64_t ldc, uint16_t* f16, int64_t ldf,
                             float* scale, hipStream_t s);
hipError_t launch_omega_packed_f16(const OmegaTables& t, uint64_t seed, uint32_t stream_id,
                                   int64_t n, int64_t r, const PackedOmega& dst, hipStream_t s);
// Several problems' packed FP16 (or sparse) Omega in one launch: job g owns
// blocks [start, start + kb_count * nt_count / 4) (jobs sorted by start;
// nt_count a multiple of 4), its own threshold sparse_t (0: Gaussian).
struct OmegaJob {
    uint64_t seed;
    uint32_t stream_id;
    int64_t n, r;
    void* dst;
    int64_t nt_count;
    uint64_t sparse_t;
    int64_t start;
};
hipError_t launch_omega_packed_f16_group(const OmegaTables& t, const OmegaJob* jobs, int count, int64_t blocks,
                                         hipStream_t s);
// Row-major Omega formats a caller can supply
enum class OmegaSrc { F16, F32, E4M3 };
// Reorder a caller (or generated) row-major Omega into fragment order.  For
// FP16 fragments every value v is checked: |v| >= 32 or a non-finite value
// sets `flag_bit` in *flag (when flag != NULL).  An e4m3 column scale outside
// the powers of two in [2^-7, 2^15] sets kStatusOmegaRange in *status (when
// status != NULL).
hipError_t launch_pack_omega(const void* src, OmegaSrc type, const float* col_scale, int64_t n, int64_t r,
                             int64_t ldo, const PackedOmega& dst, bool dst_f32, unsigned int* flag,
                             unsigned int flag_bit, unsigned int* status, hipStream_t s);
hipError_t launch_project_split_f16(const ProjArgs& a, hipStream_t s);
// Y = A W for an FP32 W with both operands split (eq:tcec-5): hi_A (2^11 hi_W)
// + lo_A hi_W + hi_A lo_W on FP16 MFMA into one FP32 accumulator.  Needs the
// 16-byte path (split_fast_ok) and W packed by launch_pack_omega_tcec.
hipError_t launch_project_tcec(const ProjArgs& a, hipStream_t s);
SplitPlan plan_tcec(int64_t m, int64_t n, int64_t r, int num_cus);
int64_t tcec_col_block();                 // 128
// Z = A^T Q (Z: n x p, row-major, ldz) for A m x n (row-major, lda) and Q
// m x p packed by launch_pack_omega_tcec (qhi = data, qlo = the lo
// fragments), with the TCEC products (eq:tcec-5).  Needs n and lda multiples
// of 4 and a 16-byte aligned A.  A non-finite product (|a| >= 65520 or a
// non-finite element) sets kStatusRange in *status.
struct TnTcecArgs {
    const float* A = nullptr;
    int64_t lda = 0;
    int64_t m = 0, n = 0, p = 0;
    const void* qhi = nullptr;
    const void* qlo = nullptr;
    int64_t nt_count = 0;
    float* Z = nullptr;
    int64_t ldz = 0;
    unsigned int* status = nullptr;
    // contraction split: chunk kz of ksplit takes 32-row steps
    // [kz kchunk_steps, (kz + 1) kchunk_steps) into partial + kz n p (ld p);
    // a second kernel adds the chunks, in a fixed order, into Z
    int ksplit = 1;
    int64_t kchunk_steps = 0;
    float* partial = nullptr;
};
// qlo == NULL: Q is FP16 (its lo part is zero), e.g. an FP16 Omega packed for
// the split projection; then Z = A^T Q is the split product of eq:shgemm-3 in
// its transposed form (two products per step instead of three).
hipError_t launch_gemm_tn_tcec(const TnTcecArgs& t, hipStream_t s);
// contraction split for an n x p output over m rows: about `cus` workgroups
// (chunks of at least 16 steps); 1 if no split pays
int plan_tn_tcec_split(int64_t m, int64_t n, int64_t p, int cus, int64_t* chunk_steps);
// Pack a row-major FP32 W (n x r, leading dimension ldo) for the TCEC
// kernels: FP16 hi fragments at dst.data, then the RN16(2^11 (w - hi))
// fragments; |hi| >= 32 or a non-finite value sets `flag_bit` in *flag (the
// hi products take 2^11 hi_W, exact in FP16 below 32).
hipError_t launch_pack_omega_tcec(const float* src, int64_t n, int64_t r, int64_t ldo, const PackedOmega& dst,
                                  unsigned int* flag, unsigned int flag_bit, hipStream_t s);
hipError_t launch_project_f32(const ProjArgs& a, hipStream_t s);
hipError_t launch_split_dump(const float* x, int64_t count, uint16_t* hi, uint16_t* lo,
                             hipStream_t s);
hipError_t launch_fill_f32(float* y, int64_t rows, int64_t cols, int64_t ld, float v,
                           hipStream_t s);
hipError_t launch_fill_u32(unsigned int* p, int64_t count, unsigned int v, hipStream_t s);

// ---------------------------------------------------------------- linalg.hip
// The same products as gemm_acc64 below with FP32 operands, FP32 MFMA and
// FP32 accumulation (B in FP64 is rounded to FP32 as it is loaded): the
// products outside CholeskyQR2 and the small SVD (U, V^T, the RP-HOSVD core).
template <class TA, class TB, class TC>
hipError_t gemm_f32(int64_t M, int64_t N, int64_t K, double alpha, const TA* a, int64_t sam, int64_t sak,
                    const TB* b, int64_t sbk, int64_t sbn, double beta, TC* c, int64_t scm, int64_t scn,
                    hipStream_t s);
template <class TA, class TB, class TC>
hipError_t gemm_f32_batched(int64_t M, int64_t N, int64_t K, double alpha, const TA* a, int64_t sam, int64_t sak,
                            int64_t sab, const TB* b, int64_t sbk, int64_t sbn, int64_t sbb, double beta, TC* c,
                            int64_t scm, int64_t scn, int64_t scb, int64_t batch, hipStream_t s);
template <class TA, class TB, class TC>
hipError_t gemm_acc64(int64_t M, int64_t N, int64_t K, double alpha, const TA* a, int64_t sam, int64_t sak,
                      const TB* b, int64_t sbk, int64_t sbn, double beta, TC* c, int64_t scm, int64_t scn,
                      hipStream_t s);
template <class TA, class TB, class TC>
hipError_t gemm_acc64_batched(int64_t M, int64_t N, int64_t K, double alpha, const TA* a, int64_t sam, int64_t sak,
                              int64_t sab, const TB* b, int64_t sbk, int64_t sbn, int64_t sbb, double beta, TC* c,
                              int64_t scm, int64_t scn, int64_t scb, int64_t batch, hipStream_t s);
// G = Y^T Y (p x p, row-major) for Y (K x p, leading dimension ldy), FP64
// accumulation; long contractions are split into up to max_split parts
// (partial: max_split * p * p doubles) summed in a fixed order.
constexpr int kGramSplit = 32;
template <class T>
hipError_t gram_acc64(int64_t p, int64_t K, const T* Y, int64_t ldy, double* G, double* partial, int max_split,
                      hipStream_t s);
// dst[i][b][p] = src[b][i][p], src of shape [B, I, P] in C order
hipError_t launch_swap01(const float* src, int64_t B, int64_t I, int64_t P, float* dst, hipStream_t s);
// C (N x P) = A^T Q, A K x N and Q K x P row-major: FP32 MFMA with FP32
// accumulation (FP64-accumulating fallback off the 16-byte path)
hipError_t gemm_tn_f32(int64_t N, int64_t P, int64_t K, const float* A, int64_t lda, const float* Q, int64_t ldq,
                       float* C, int64_t ldc, hipStream_t s);
hipError_t potrf_lower(double* A, int64_t lda, int64_t p, unsigned int* status, hipStream_t s);
hipError_t launch_zero_upper(double* A, int64_t lda, int64_t p, hipStream_t s);
hipError_t trtri_lower(const double* L, int64_t ldl, double* X, int64_t ldx, int64_t p, hipStream_t s);
hipError_t launch_trtri_apply_diag(double* X, int64_t ldx, int64_t r0, int64_t rows, hipStream_t s);
// One square problem of the parallel one-sided Jacobi SVD: W (n x n,
// row-major in and out) becomes W V with orthogonal columns; pair_start = sum
// of ceil(n/2) over the problems before it; flags: 4 ints of device scratch.
struct JacobiProb {
    double* W;
    double* V;
    int n;
    int pair_start;     // first global column pair of this problem (scalar rounds)
    int* flags;
    int bpair_start;    // first global block pair (block rounds: blocks of kJacobiBlock columns)
};
constexpr int kJacobiBlock = 8;
// block pairs of one problem per round: ceil(n / 8) blocks, padded to even, halved
inline int jacobi_block_pairs(int n) {
    const int nb = (n + kJacobiBlock - 1) / kJacobiBlock;
    return (nb + (nb & 1)) / 2;
}
// Write one Jacobi table entry from the kernel arguments (no host copy).
hipError_t launch_set_jacobi_prob(JacobiProb* dst, const JacobiProb& v, hipStream_t s);
// poll_flag != NULL (a single problem, stream not being captured): the
// host reads that device flag (the problem's flags[0], "converged") after
// every sweep, synchronising the stream, and stops issuing sweeps once set.
hipError_t jacobi_svd_group(const JacobiProb* tab, int count, int total_pairs, int total_bpairs, int max_n, int max_sweeps,
                            double tol, unsigned int* status, hipStream_t s, const int* poll_flag = nullptr);
// The phases of jacobi_svd_group, for a caller that runs the sweeps in parts:
// prep (W to column-major, V = I, flags cleared), sweeps [sweep_begin,
// sweep_end), final (W, V back to row-major; not-converged status).  The
// sweep bound is max_sweeps plus the block form's 8.  jacobi_group_open
// writes the number of problems not yet converged to *out (device int).
int jacobi_group_sweep_bound(int max_n, int max_sweeps);
hipError_t jacobi_group_prep(const JacobiProb* tab, int count, int max_n, hipStream_t s);
hipError_t jacobi_group_sweeps(const JacobiProb* tab, int count, int total_pairs, int total_bpairs, int max_n,
                               int sweep_begin, int sweep_end, double tol, hipStream_t s,
                               const int* poll_flag = nullptr);
hipError_t jacobi_group_open(const JacobiProb* tab, int count, int* out, hipStream_t s);
hipError_t jacobi_group_final(const JacobiProb* tab, int count, int max_n, unsigned int* status, hipStream_t s);
hipError_t svd_finish(const double* W, const double* V, int n, int ncols, double* sig, int* order, double* Ur,
                      double* Vr, hipStream_t s);

// ---------------------------------------------------------------- group_linalg.hip
// Job tables of the grouped kernels (device memory; every job of a launch is
// independent).  `start` is the job's first block and the launch's `starts`
// array repeats it, sorted, for the blocks' binary search.
struct GemmJob {                      // C = alpha op(A) op(B) + beta C, FP64 accumulation
    int64_t M, N, K;
    double alpha, beta;
    const void* a;
    int64_t sam, sak;
    const void* b;
    int64_t sbk, sbn;
    void* c;
    int64_t scm, scn;
    int64_t tiles_n, start;
};
int64_t gemm_group_tiles(int64_t M, int64_t N);
int64_t gemm_group_tiles_n(int64_t N);
template <class TA, class TB, class TC>
hipError_t gemm_acc64_group(const GemmJob* jobs, const int64_t* starts, int count, int64_t blocks, hipStream_t s);
// the FP32 form (FP32 MFMA and accumulation) of the same jobs
template <class TA, class TB, class TC>
hipError_t gemm_f32_group(const GemmJob* jobs, const int64_t* starts, int count, int64_t blocks, hipStream_t s);

struct GramJob {                      // G (p x p, FP64) = Y^T Y, Y (R x p, ld ldy, FP32 or FP64)
    const void* y;
    int64_t ldy, R, p;
    int64_t kchunk;                   // rows per contraction chunk
    double* G;
    double* part;                     // ksplit > 1: ksplit partial sums of p x p (G = their sum, in order)
    int ksplit, tiles;                // tiles: upper-triangle 64 x 64 tiles of G
    int64_t start;
};
int gram_group_tiles(int64_t p);
// One launch for the partial (or direct) products of every job, a second
// one (only when some job has ksplit > 1) for the sums; G is written whole
// (both triangles, exactly symmetric).
template <class T>
hipError_t gram_group(const GramJob* jobs, const int64_t* starts, int count, int64_t blocks, bool any_split,
                      hipStream_t s);

constexpr int kCholGroupMaxP = 199;   // p (p + 1) / 2 + 2 p doubles fit in 160 KiB of LDS
struct CholJob {                      // G (p x p) = L L^T; L (lower, zero above) and X = L^-1
    const double* G;
    double* L;                        // may equal G
    double* X;
    int p;
};
hipError_t chol_inv_group(const CholJob* jobs, int count, int max_p, unsigned int* status, hipStream_t s);

struct TnJob {                        // C (N x P) = A^T Q, A K x N, Q K x P, all FP32 row-major
    int64_t N, P, K;
    const float* A;
    int64_t lda;
    const float* Q;
    int64_t ldq;
    float* C;
    int64_t ldc;
    int64_t tiles_x, tiles_y, start;  // workgroups along P and along N (tn_group_shape)
    int wp;                           // 64-column tiles of P per workgroup (1 .. 4)
    int64_t kchunk;                   // rows of A per contraction chunk
    int ksplit;                       // > 1: chunk kz writes part + kz N P (ld P); C = their sum, in order
    float* part;
};
// sets wp, tiles_x and tiles_y from N and P
void tn_group_shape(TnJob& j);
hipError_t gemm_tn_f32_group(const TnJob* jobs, const int64_t* starts, int count, int64_t blocks,
                             bool any_split, hipStream_t s);

struct SvdJob {                       // after the Jacobi iteration on W (n x n) with V
    const double* W;
    const double* V;
    int n, ncols;
    double* sig;                      // n, descending
    int* order;                       // n
    double* S;                        // ncols (the caller's output)
    double* Ur;                       // n x ncols
    double* Vr;                       // n x ncols
};
hipError_t svd_finish_group(const SvdJob* jobs, int count, int max_elems, hipStream_t s);

}  // namespace rpmi

extern "C" int rpmi_build_f16_thresholds(uint64_t* table, int capacity);
extern "C" void rpmi_build_guide(const uint64_t* table, int count, uint32_t* guide, int buckets_log2);
