/*
 * rpmi.h - mixed-precision random projection for RandNLA on AMD MI355X (gfx950).
 *
 * C ABI of librpmi.so.  The library computes the random projection
 *     Y = A * Omega                                   (Sec. 2.2, eq:rp-vec)
 * of an FP32 matrix A (m x n, or an unfolding of a tensor) by a Gaussian
 * matrix Omega (n x r) kept in FP16, with each FP32 element of A split into an
 * FP16 hi part and a 2^11-scaled FP16 lo part and both products run on FP16
 * matrix cores with FP32 accumulation (Sec. 4.1, eq:shgemm-1..3).  A plain
 * FP32 GEMM path is provided as the baseline form.
 *
 * Conventions for every entry point:
 *   - Array pointers are DEVICE pointers owned by the caller unless the
 *     comment says "host".  No caller pointer is kept after the call returns.
 *   - Matrices are row-major with an explicit leading dimension (elements).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it and the call returns without synchronising.
 *   - Argument errors are detected on the host before anything is enqueued
 *     and leave outputs untouched; the call then returns a status != RP_OK
 *     and rp_last_error() describes it.
 *   - Conditions found on the device (FP16 range overflow of A) are recorded
 *     in a per-context device status word read by rp_get_device_status().
 *   - A context must not be used from two host threads at once.
 */
#ifndef RPMI_H
#define RPMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rp_ctx_s* rp_ctx;

typedef enum rp_status {
    RP_OK = 0,
    RP_ERR_INVALID_ARG = 1,   /* bad pointer, size, stride or enum value          */
    RP_ERR_UNSUPPORTED = 2,   /* valid request this build does not implement      */
    RP_ERR_RANGE = 3,         /* device: the FP16 split of A met an element whose
                                 hi part overflows (finite |a| >= 65520; Sec. 4.2:
                                 FP16 limits the exponent range of A) or a
                                 non-finite element (NaN, +-inf)                  */
    RP_ERR_NOT_SPD = 4,       /* device: Cholesky breakdown in CholeskyQR2        */
    RP_ERR_NOT_CONVERGED = 5, /* device: Jacobi SVD did not converge              */
    RP_ERR_NOMEM = 6,         /* device allocation failed                          */
    RP_ERR_HIP = 7,           /* a HIP runtime call failed (see rp_last_error)    */
    RP_ERR_OMEGA_RANGE = 8    /* device: a caller-supplied Omega packed for the
                                 split-FP16 kernels holds an entry with
                                 |omega| >= 32 or a non-finite one (the kernels
                                 take the hi product against 2^11 Omega, exact
                                 in FP16 only below 32; the generated Gaussian
                                 never exceeds 9.1), or an e4m3 column scale
                                 that is not a power of two in [2^-7, 2^15]     */
} rp_status;

/* Storage format of Omega (Sec. 3: a Gaussian matrix tolerates a short mantissa). */
typedef enum rp_omega_t {
    RP_OMEGA_F32 = 0,         /* FP32 Gaussian                                     */
    RP_OMEGA_F16 = 1,         /* FP16 Gaussian, exact sample of RN16(N(0,1))        */
    RP_OMEGA_E4M3 = 2,        /* FP8 e4m3fn of the FP32 Gaussian, power-of-two
                                 scale per column (rp_omega_generate_e4m3); the
                                 projections take Omega8 / s_j, exact in FP16     */
    /* Sparse random matrices of eq:sp-rand (Sec. 2.2) without their sqrt(s)
     * factor (Sec. 3.4: only the range of Y = A Omega is used): entries in
     * {-1, 0, +1}, +1 and -1 each with probability 1/(2s); exact in FP16 and
     * FP32, stored like RP_OMEGA_F16 (FP16 bits). */
    RP_OMEGA_SPARSE1 = 3,     /* s = 1: +-1 with probability 1/2 each           */
    RP_OMEGA_SPARSE3 = 4,     /* s = 3 (Achlioptas)                             */
    RP_OMEGA_VSPARSE = 5      /* s = sqrt(n) for an n-row Omega (very sparse)   */
} rp_omega_t;

/* How Y = A * Omega is computed. */
/* a_scale_exp value: a power-of-two pre-scale per row of A, chosen on the
 * device (see rp_project) */
#define RP_A_SCALE_AUTO_ROW 32767

typedef enum rp_algo_t {
    RP_ALGO_F32 = 0,          /* plain FP32 GEMM on FP32 matrix cores (baseline form);
                                 an FP16 Omega is widened exactly to FP32 first, as
                                 the paper does for its SGEMM comparison (Sec. 4.4.1) */
    RP_ALGO_SPLIT_F16 = 1,    /* A split into FP16 hi + 2^-11 lo on the fly, two FP16
                                 products with FP32 accumulation (Sec. 4.1); requires
                                 an FP16 Omega                                     */
    RP_ALGO_TCEC_F16 = 2      /* both operands split (the error-corrected product of
                                 Sec. 2.3, eq:tcec-5): A as for RP_ALGO_SPLIT_F16, an
                                 FP32 Omega into hi = RN16(w) and RN16(2^11 (w - hi));
                                 three FP16 products (hi_A hi_W, lo_A hi_W, hi_A lo_W)
                                 into one FP32 accumulator: FP32-level accuracy for a
                                 right operand that is not FP16 (the power scheme's
                                 A W).  Requires an FP32 Omega with |omega| < 32 and
                                 A on the 16-byte path (16-byte aligned, s_row,
                                 k_inner and s_k_outer multiples of 4)          */
} rp_algo_t;

/*
 * Descriptor of the logical m x n FP32 operand A (or a tensor unfolding,
 * Algorithm 2 line 2).  Element (i, k), 0 <= i < rows, 0 <= k < cols, is
 *     ptr[i * s_row + (k / k_inner) * s_k_outer + (k % k_inner) * s_k_inner]
 * A plain row-major matrix with leading dimension lda is
 *     { ptr, m, n, lda, n, 1, 0 }.
 * Supported by this build: s_k_inner == 1, and either k_inner == cols or
 * k_inner a multiple of 64 dividing cols; other layouts return
 * RP_ERR_UNSUPPORTED.  A 16-byte aligned ptr with s_row, k_inner and
 * s_k_outer multiples of 4 takes the 16-byte load path; any other
 * (4-byte aligned) layout is loaded element by element.
 */
typedef struct rp_desc {
    const float* ptr;
    int64_t rows;
    int64_t cols;
    int64_t s_row;
    int64_t k_inner;
    int64_t s_k_inner;
    int64_t s_k_outer;
} rp_desc;

/* Create a context on HIP device `device`: builds the FP16 inverse-CDF
 * threshold table on the host and uploads it, allocates the device status
 * word.  *out receives the handle.  Makes `device` current. */
rp_status rp_create(rp_ctx* out, int device);

/* Destroy a context (synchronises the device first).  NULL is allowed. */
rp_status rp_destroy(rp_ctx ctx);

/* Static text for a status code (host string, never NULL). */
const char* rp_status_string(rp_status s);

/* Text of the last error on this context (host string owned by the context,
 * valid until the next call on it).  Also works with ctx == NULL for errors of
 * rp_create. */
const char* rp_last_error(rp_ctx ctx);

/*
 * Generate the Gaussian matrix Omega (n x r, row-major, leading dimension ldo
 * >= r) for (seed, stream_id) into `omega` (uint16 FP16 bits for
 * RP_OMEGA_F16, float for RP_OMEGA_F32).  Sec. 3 / Sec. 4.2; the exact
 * definition of every bit:
 *   element (i, j) uses word j mod 4 of the Philox4x64-10 block with counter
 *   (i, floor(j/4), stream_id, 0) and key (seed, 0); the low bit is the sign,
 *   the upper 63 bits a uniform u.  FP16: magnitude = the FP16 value whose bit
 *   pattern is k = #{ t : T_t <= u }, T_t = floor(2^63 erf(mu_t / sqrt 2)),
 *   mu_t the midpoint between FP16 patterns t and t+1 (t = 0..18570); zero is
 *   +0.  FP32: same cell k, position from the upper 32 bits f of the same word
 *   of the block with counter word 3 = 1:
 *   RN32(mu_{k-1} + (mu_k - mu_{k-1}) (f + 1/2) 2^-32), mu_{-1} = 0.
 * The sparse types (FP16 bits) take the whole 64-bit word x of the same
 * element: +1 if x < T, -1 if T <= x < 2T, 0 otherwise, with
 * T = floor(2^64 / (2s)): 2^63 (s = 1), floor(2^64 / 6) (s = 3),
 * floor(2^63 / sqrt(n)) = isqrt(floor(2^126 / n)) (s = sqrt(n)); the
 * probabilities are 1/(2s) to within 2^-64.
 * n, r >= 0 (zero sizes enqueue nothing).
 */
rp_status rp_omega_generate(rp_ctx ctx, uint64_t seed, uint32_t stream_id,
                            int64_t n, int64_t r, rp_omega_t type,
                            void* omega, int64_t ldo, void* stream);

/*
 * Y = A * Omega (eq:rp-vec), Y row-major m x r with leading dimension ldy >= r.
 *   A          descriptor of the m x n operand (see rp_desc), read only.
 *   r          number of columns of Omega and Y (r >= 0).
 *   omega_type storage format of Omega.
 *   seed, stream_id  used when omega == NULL: Omega is generated exactly as
 *              rp_omega_generate (rp_omega_generate_e4m3 for RP_OMEGA_E4M3)
 *              would, into context-owned workspace.
 *   omega, ldo a caller-supplied Omega (n x r row-major: FP16 bits, FP32, or
 *              e4m3fn bytes according to omega_type), or NULL.
 *   col_scale  with a caller e4m3 Omega: r floats s_j (device), the power-of-
 *              two column scales of rp_omega_generate_e4m3; the projection
 *              takes Omega8[i][j] / s_j (exact in FP16 for s_j in
 *              [2^-7, 2^15]).  Ignored otherwise (may be NULL).
 *   algo       RP_ALGO_SPLIT_F16 (needs an FP16, e4m3 or sparse Omega), RP_ALGO_TCEC_F16
 *              (needs an FP32 Omega and A on the 16-byte path, otherwise
 *              RP_ERR_UNSUPPORTED) or RP_ALGO_F32.
 *   a_scale_exp  s: the split takes 2^s A instead of A and the epilogue
 *              multiplies by 2^-s (both exact while 2^s A and Y stay inside
 *              the FP32 normal range), so that an A whose magnitudes exceed
 *              the FP16 range (Sec. 4.2) can be brought inside it; 0 = off.
 *              |s| <= 64.  Ignored by RP_ALGO_F32 and RP_ALGO_TCEC_F16.
 *              RP_A_SCALE_AUTO_ROW: the full FP32 exponent range (the role
 *              of the paper's SHGEMM-TF32, Sec. 4.2, without a TF32 matrix
 *              core): each row i gets its own s_i, chosen on the device so
 *              that the row's largest |a| lands in [2^14, 2^15) (clamped to
 *              [-126, 126]; 0 for an all-zero or non-finite row); Y's row i
 *              is multiplied by 2^-s_i.  Exact scalings, so the elementwise
 *              bound of the split product holds for any row whose entries
 *              span fewer than about 28 binades below its maximum (smaller
 *              ones may fall into FP16 subnormals, an error below 2^-38
 *              of the row's maximum).  One extra read of A (the row maxima);
 *              the projection then runs on the two-accumulator kernel.
 *              Taken by rp_project and rsvd; other entry points return
 *              RP_ERR_UNSUPPORTED for it.
 * With RP_ALGO_SPLIT_F16 an element of 2^s A that overflows FP16 (finite
 * |2^s a| >= 65520), or a non-finite element, sets RP_ERR_RANGE in the device
 * status word; Y is then unspecified (a NaN element leaves NaN in its own
 * row of Y); the same holds for A with RP_ALGO_TCEC_F16, whose FP32 Omega
 * records RP_ERR_OMEGA_RANGE when an entry has |omega| >= 32 (the hi products
 * take 2^11 RN16(omega)) or is not finite.  A caller FP16 or e4m3 Omega is scanned on the device: when it
 * holds an entry with |omega| >= 32 the call takes the kernel with two
 * accumulators (eq:shgemm-3 as written), which has no such bound; the scan
 * is read back once, so such a call synchronises `stream`.
 * m, n or r equal to zero is allowed (n == 0 writes Y = 0).
 * May grow the context workspace (device allocation, which synchronises the
 * device when it happens).
 */
rp_status rp_project(rp_ctx ctx, const rp_desc* A, int64_t r,
                     rp_omega_t omega_type, uint64_t seed, uint32_t stream_id,
                     const void* omega, int64_t ldo, const float* col_scale,
                     rp_algo_t algo, int32_t a_scale_exp,
                     float* Y, int64_t ldy, void* stream);

/*
 * Omega in the projection kernels' fragment order, for callers that reuse one
 * Omega across many projections (e.g. the RSVD of many matrices sharing n and
 * r).  rp_omega_packed_size() gives the byte size of the buffer for (n, r,
 * algo) in *bytes (host pointer).  rp_omega_pack() fills `packed` (device,
 * caller-owned, that many bytes) from `omega` (n x r row-major: FP16 bits,
 * FP32, or e4m3fn bytes with col_scale, by `type`) or, when omega == NULL, by
 * generating Omega for (seed, stream_id) exactly as rp_omega_generate() (or
 * rp_omega_generate_e4m3()) does.  The split-FP16 algorithm takes FP16
 * fragments (type RP_OMEGA_F16, or RP_OMEGA_E4M3 whose values Omega8 / s_j
 * are exact in FP16); the FP32 algorithm takes FP32 fragments (an FP16 or
 * e4m3 Omega is widened exactly); the TCEC algorithm takes an FP32 Omega
 * (type RP_OMEGA_F32) as FP16 hi fragments followed by FP16 RN16(2^11 (w -
 * hi)) fragments (|omega| >= 32 records RP_ERR_OMEGA_RANGE).  col_scale: r floats (device) for a caller
 * e4m3 Omega, else ignored.  Packing a caller Omega for the split-FP16
 * algorithm records RP_ERR_OMEGA_RANGE in the device status word if an entry
 * has |omega| >= 32 or is not finite (or a column scale is not a power of two
 * in [2^-7, 2^15]); rp_project_packed() then leaves Y unspecified (rp_project()
 * handles such an Omega).  Zero padding beyond n rows and r columns is part
 * of the packed buffer.
 */
rp_status rp_omega_packed_size(int64_t n, int64_t r, rp_algo_t algo, size_t* bytes);
rp_status rp_omega_pack(rp_ctx ctx, uint64_t seed, uint32_t stream_id, const void* omega,
                        int64_t ldo, const float* col_scale, rp_omega_t type, int64_t n, int64_t r,
                        rp_algo_t algo, void* packed, void* stream);

/*
 * Y = A * Omega with Omega already packed by rp_omega_pack() for the same
 * (n = A->cols, r, algo).  Launches one projection kernel (none if m or r is
 * 0; a fill kernel if n is 0).  Same layout rules, a_scale_exp and device
 * status as rp_project().  When the output tiles of the split-FP16 path do
 * not fill the device, the contraction is split across workgroups whose
 * partial sums live in a context-owned workspace; growing it (first use of a
 * shape) allocates and synchronises the device.  Launches that share a
 * context must not run concurrently on different streams.
 */
rp_status rp_project_packed(rp_ctx ctx, const rp_desc* A, int64_t r, const void* packed,
                            rp_algo_t algo, int32_t a_scale_exp, float* Y, int64_t ldy, void* stream);

/*
 * rp_project_packed() for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, validation and result as rp_project_packed()
 * (bit for bit: the same kernels and the same contraction split), but the
 * partial sums and arrival counters of the contraction split live in one
 * static device array of the library (64 MiB of partial sums + 4 KiB of
 * counters) that each device holds until the process ends; no device memory
 * is allocated, and nothing synchronises.  A shape whose split needs more
 * than that returns RP_ERR_INVALID_ARG before anything is enqueued (the
 * planner never asks for more than 64 MiB on a device of up to 256 compute
 * units).  Each call first clears the counters it uses with a kernel.  All
 * calls on one device share the array and it keeps the last call's
 * contents: calls that overlap in time on one device (any contexts, any
 * streams) race and give undefined results.  algo RP_ALGO_F32 or
 * RP_ALGO_SPLIT_F16 (RP_ALGO_TCEC_F16 returns RP_ERR_INVALID_ARG).
 */
rp_status rp_project_packed_noalloc(rp_ctx ctx, const rp_desc* A, int64_t r, const void* packed,
                                    rp_algo_t algo, int32_t a_scale_exp, float* Y, int64_t ldy,
                                    void* stream);

/*
 * Z = A^T Q: the product of Algorithm 1 line 3 (B^T = A^T Q, Q with
 * orthonormal columns) and of the power scheme's A^T Q, for callers that run
 * the other steps themselves.  A m x n FP32 row-major (lda >= n), Q m x p
 * FP32 row-major (ldq >= p), Z n x p FP32 row-major (ldz >= p), all device.
 * algo RP_ALGO_F32: FP32 matrix cores.  RP_ALGO_TCEC_F16: both operands split
 * (Sec. 2.3, eq:tcec-5) on FP16 matrix cores; needs n and lda multiples of 4
 * and a 16-byte aligned A (otherwise RP_ERR_UNSUPPORTED), and records
 * RP_ERR_OMEGA_RANGE for an entry |q| >= 32 and RP_ERR_RANGE for an A
 * element with |a| >= 65520 or not finite (Z then unspecified).  The TCEC
 * form first packs Q into the context workspace (growing it allocates and
 * synchronises the device).  m == 0 writes Z = 0.
 */
rp_status rp_gemm_tn(rp_ctx ctx, int64_t m, int64_t n, int64_t p, const float* A, int64_t lda,
                     const float* Q, int64_t ldq, rp_algo_t algo, float* Z, int64_t ldz, void* stream);

/*
 * Randomized SVD (Algorithm 1, Sec. 2.2) of the m x n FP32 matrix A (row-major,
 * leading dimension lda >= n), with target rank k and oversampling s
 * (p = k + s columns of Omega, 1 <= k <= p <= min(m, n), p <= 1024) and
 * power_iters steps of the power scheme (Sec. 2.1), re-orthonormalised at
 * every half step:
 *     Y = A Omega;  repeat q times { Q = QR(Y); W = QR(A^T Q); Y = A W };
 *     Q = QR(Y);  B = Q^T A;  U', S, V' = SVD(B);  U = Q U'[:, :k].
 * Omega is generated from (seed, stream_id 0) in omega_type and the
 * projection runs with `algo` (RP_ALGO_SPLIT_F16 is the paper's method;
 * RP_ALGO_F32 the baseline); A^T Q (power scheme and B) and A W (power
 * scheme) run on the TCEC products (RP_ALGO_TCEC_F16, rp_gemm_tn) when algo
 * is RP_ALGO_SPLIT_F16, a_scale_exp is 0 and A is on the 16-byte path (n and
 * lda multiples of 4, 16-byte aligned), else on this library's FP32
 * matrix-core kernels; the
 * products with the small factors in FP32 with FP64 accumulation.  Every QR is CholeskyQR2 with the Gram
 * matrix, Cholesky factor and triangular inverse in FP64; the SVD of B is
 * taken as B^T = Q_B R_B (CholeskyQR2) followed by a one-sided Jacobi SVD of
 * R_B^T in FP64 (at most 16 sweeps).  Outside stream capture the call reads a
 * 4-byte convergence flag back after every Jacobi sweep (synchronising
 * `stream`) and stops sweeping once it is set; under capture every sweep is
 * recorded and the sweeps after convergence do no work.
 * Outputs (device): U m x k (ldu >= k), S k doubles in descending order, VT
 * k x n (ldvt >= n).  Singular vectors are determined up to sign.
 * a_scale_exp applies to the projection Y = A Omega as in rp_project().
 * Device conditions: RP_ERR_NOT_SPD (a Cholesky pivot was not positive:
 * Y numerically rank-deficient beyond FP64 Gram range), RP_ERR_NOT_CONVERGED
 * (Jacobi), RP_ERR_RANGE (split path, 2^s A outside FP16 range).
 * Workspace: with work == NULL the context workspace is used and grown as
 * needed (allocating and synchronising the device then), and the packed
 * Omega comes from the context cache described at rp_hosvd().  Otherwise `work`
 * (device, caller-owned, 256-byte aligned, contents undefined on entry) must
 * hold at least the bytes rsvd_workspace_size() reports for the same
 * arguments; the call then allocates nothing and synchronises only for the
 * Jacobi flag, and the caller keeps `work` alive until the work on `stream`
 * has finished.
 */
rp_status rsvd(rp_ctx ctx, int64_t m, int64_t n, const float* A, int64_t lda,
               int64_t k, int64_t oversample, int32_t power_iters,
               uint64_t seed, rp_omega_t omega_type, rp_algo_t algo, int32_t a_scale_exp,
               float* U, int64_t ldu, double* S, float* VT, int64_t ldvt,
               void* work, size_t work_bytes, void* stream);

/*
 * Bytes of caller workspace rsvd() needs for these arguments (host pointer
 * `bytes`).  Validates the arguments as rsvd() does, apart from pointers.
 */
rp_status rsvd_workspace_size(rp_ctx ctx, int64_t m, int64_t n, int64_t k, int64_t oversample,
                              int32_t power_iters, rp_omega_t omega_type, rp_algo_t algo, size_t* bytes);

/*
 * e4m3 Omega (the low-precision storage of Sec. 3 with the OCP FP8 E4M3FN
 * format of Table 1): for the FP32 Omega w of (seed, stream_id) and every
 * column j, s_j = 2^floor(log2(448 / max_i |w[i][j]|)) (1 for an empty
 * column) and Omega8[i][j] = sat448(RNE_e4m3(w[i][j] s_j)), so that
 * A Omega8[:, j] / s_j approximates A w[:, j].  omega: n x r e4m3fn bytes
 * (ldo >= r); col_scale: r floats s_j.  Device, caller-owned.  The projection
 * entry points use the values Omega8 / s_j, which are exact in FP16; they
 * take this Omega either generated (omega == NULL) or from the caller with
 * its col_scale.
 */
rp_status rp_omega_generate_e4m3(rp_ctx ctx, uint64_t seed, uint32_t stream_id, int64_t n, int64_t r,
                                 uint8_t* omega, int64_t ldo, float* col_scale, void* stream);

/*
 * One projection of a grouped call: Y = A Omega with Omega (A.cols x r, FP16
 * or e4m3) generated from (seed, stream_id).  A, Y: device, caller-owned.
 * a_scale_exp as in rp_project().
 */
typedef struct {
    rp_desc A;
    int64_t r;
    uint64_t seed;
    uint32_t stream_id;
    float* Y;
    int64_t ldy;
    int32_t a_scale_exp;
} rp_project_problem;

/*
 * Several split-FP16 projections (Sec. 4.1) of independent shapes in grouped
 * launches: the problems whose A is on the 16-byte path in one launch per
 * column width (r <= 128, r > 128), each problem's contraction split planned
 * for its share of the compute units (see the autotuner below); the others
 * in one launch of the general kernel per column width, longest
 * contraction first.  omega_type: RP_OMEGA_F16, RP_OMEGA_E4M3 or a sparse
 * type; a_scale_exp of a problem in [-64, 64].  probs: host array of count
 * problems, read during the call.  Same device conditions as rp_project.
 */
rp_status rp_project_grouped(rp_ctx ctx, int32_t count, const rp_project_problem* probs,
                             rp_omega_t omega_type, void* stream);

/* One randomized SVD of a batched call (arguments as in rsvd). */
typedef struct {
    int64_t m, n;
    const float* A;
    int64_t lda;
    int64_t k, oversample;
    float* U;
    int64_t ldu;
    double* S;
    float* VT;
    int64_t ldvt;
} rp_rsvd_problem;

/*
 * Many randomized SVDs (Algorithm 1) of different shapes in one call:
 * Omega_j from (seed, stream_id = j); RP_OMEGA_F16, RP_OMEGA_E4M3 and the
 * sparse types take the split-FP16 projection, RP_OMEGA_F32 the FP32 one.  The projections of all problems go
 * out in grouped launches whose contraction split is tuned once per
 * problem-shape signature (the grouped projection is timed at a few
 * compute-unit shares; the fastest is kept in the context).  The whole
 * sequence (Omega generation, projections, every problem's CholeskyQR2,
 * B, SVD and U, V^T stages) is captured in two HIP graphs on a context
 * stream and launched on `stream`; a later call with the same problems,
 * buffers and options replays them, reading A afresh.  The first graph ends
 * after the first 10 sweeps of the grouped Jacobi SVD (RPMI_BATCHED_GRAPH_SWEEPS
 * = an integer in [0, 1000] in the environment at rp_create sets another
 * count); the host then reads the number of problems not yet converged
 * (synchronising `stream`) and, while some are open and the sweep bound of
 * rsvd allows, issues one more sweep and reads it again; the second graph
 * holds the Jacobi final step and the U, V^T products.  Every call
 * therefore synchronises `stream` once; the first call of a problem set
 * synchronises the device.  Outputs per problem as in rsvd.
 */
rp_status rsvd_batched(rp_ctx ctx, int32_t count, const rp_rsvd_problem* probs, int32_t power_iters,
                       uint64_t seed, rp_omega_t omega_type, void* stream);

/*
 * Random-projection HOSVD (Algorithm 2, Sec. 5.2) of the ndim-way FP32 tensor
 * X (C order, dims[0] x ... x dims[ndim-1], 2 <= ndim <= 8), with target
 * ranks J_i = ranks[i] (oversampling included; 1 <= J_i <= dims[i],
 * J_i <= prod_{l != i} dims[l], J_i <= 1024):
 *     for each mode i:  W_i = X_(i) Omega_i;  Q_i = QR(W_i)
 *     core = X x_1 Q_1^T x_2 Q_2^T ... x_N Q_N^T
 * X_(i) is the mode-i unfolding: row index i_i, column index the C-order
 * linear index of the remaining modes.  Omega_i (prod_{l != i} dims[l] x J_i)
 * is generated from (seed, stream_id = i) in omega_type; the projections run
 * with `algo` (RP_ALGO_SPLIT_F16: all modes whose unfolding can be streamed in
 * place go out in grouped launches; the last mode streams X in place through
 * the transposed split kernel (see rp_hosvd_project); any other mode whose
 * columns are not contiguous in runs of a multiple of 64 elements is first
 * copied mode-first into workspace).  Each QR is CholeskyQR2 (FP64 Gram,
 * Cholesky and triangular inverse), so Q_i is the orthonormal factor with a
 * positive-diagonal R.  The core is contracted one mode at a time: the first
 * mode with FP32 MFMA products and FP32 accumulation, the others with FP64
 * accumulation.
 * Outputs (device): core, C order J_0 x ... x J_{ndim-1} FP32; factors is a
 * host array of ndim device pointers, factors[i] dims[i] x J_i row-major FP32.
 * dims, ranks, factors: host arrays owned by the caller, read during the call.
 * Device conditions: RP_ERR_NOT_SPD (a W_i numerically rank-deficient),
 * RP_ERR_RANGE (split path, X outside the FP16 range).  Grows the context
 * workspace as needed (synchronising the device then).  The packed Omega_i
 * are kept in a context cache (up to 1 GiB, least recently used freed first,
 * the device synchronised before a free) keyed by (seed, stream_id, n, r,
 * omega_type, algo), so a repeated call generates no Omega; a miss allocates.
 */
rp_status rp_hosvd(rp_ctx ctx, int32_t ndim, const int64_t* dims, const float* X,
                   const int64_t* ranks, uint64_t seed, rp_omega_t omega_type,
                   rp_algo_t algo, float* core, float* const* factors, void* stream);

/*
 * The projection step of RP-HOSVD alone (Algorithm 2 line 2, every mode):
 * W_i = X_(i) Omega_i into W[i] (device, dims[i] x J_i row-major, leading
 * dimension ldw[i] >= J_i), with the same X, dims, ranks, Omega_i and
 * arguments checks as rp_hosvd, and the same launches: with
 * RP_ALGO_SPLIT_F16 the modes whose unfolding streams in place go out
 * grouped, and the last mode, when dims[ndim-1] is a multiple of 4 and X is
 * 16-byte aligned, runs as W = M^T Omega for M = X viewed as
 * (prod_{l<N} dims[l]) x dims[N-1] row-major, on the transposed split kernel
 * (every element of X split into hi and lo as in eq:shgemm-1/2, both
 * against the FP16 Omega, one FP32 accumulator; X read in place); other
 * layouts are copied mode-first first.  W, ldw: host arrays of ndim entries.
 * Device condition: RP_ERR_RANGE (split path, X outside the FP16 range).
 */
rp_status rp_hosvd_project(rp_ctx ctx, int32_t ndim, const int64_t* dims, const float* X,
                           const int64_t* ranks, uint64_t seed, rp_omega_t omega_type,
                           rp_algo_t algo, float* const* W, const int64_t* ldw, void* stream);

/*
 * Split of an FP32 array into FP16 hi and lo (Sec. 4.1, eq:shgemm-1/2), as the
 * projection performs it in registers: hi = RN16(a), lo = RN16((a - hi) 2^11).
 * Exposed so that the split can be checked bit for bit.  x: count floats;
 * hi, lo: count uint16 each (device).
 */
rp_status rp_split_f16(rp_ctx ctx, const float* x, int64_t count,
                       uint16_t* hi, uint16_t* lo, void* stream);

/*
 * Synchronise `stream`, then return in *out the device status word of the
 * context as a status code (RP_OK if nothing was recorded; otherwise the
 * first recorded condition in the order RP_ERR_OMEGA_RANGE, RP_ERR_RANGE,
 * RP_ERR_NOT_SPD, RP_ERR_NOT_CONVERGED; an Omega outside its range makes the
 * products non-finite as well, so it is reported as the cause).  If `clear`
 * is non-zero the word is reset.
 */
rp_status rp_get_device_status(rp_ctx ctx, void* stream, int clear, rp_status* out);

/*
 * Autotuner cache of the grouped projections (the batching of Sec. 5's
 * many-problem runs and of Algorithm 2's per-mode projections): the first
 * rsvd_batched, rp_project_grouped, rp_hosvd or rp_hosvd_project call on a
 * problem set (shapes and layouts) times its grouped launch at several
 * contraction-split scales (the CU share each problem's split is planned
 * for), times two kernel forms for the 16-byte-path problems with r <= 128
 * (register-staged 128-row tiles, LDS-staged 256-row tiles), and keeps the
 * fastest per context; a stream under graph capture is not timed (scale 1,
 * register-staged form).  RPMI_GROUP_FORM=0 or 1 in the environment at
 * rp_create fixes the form.  The cache persists:
 *   - rp_tuning_save writes every entry to `path` as text, one line
 *     "<signature hex> <scale> <form>" per entry (replacing the file);
 *   - rp_tuning_load adds the entries of such a file (later lines win);
 *     a line that does not parse stops the load with RP_ERR_INVALID_ARG
 *     (entries read before it are kept); a missing file is RP_ERR_INVALID_ARG;
 *   - rp_tuning_count gives the number of entries.
 * If the environment variable RPMI_TUNING_FILE names a file when rp_create
 * runs, the context loads it (a missing or bad file is ignored) and writes
 * it back after each new tuning.  Signatures include the device's compute
 * unit count, so a file from another chip model matches nothing.  Host only.
 */
rp_status rp_tuning_save(rp_ctx ctx, const char* path);
rp_status rp_tuning_load(rp_ctx ctx, const char* path);
rp_status rp_tuning_count(rp_ctx ctx, int64_t* entries);

#ifdef __cplusplus
}
#endif

#endif /* RPMI_H */
