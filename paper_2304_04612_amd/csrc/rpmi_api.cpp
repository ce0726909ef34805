// C-ABI entry points of librpmi (declared in include/rpmi.h): argument
// validation, context state (Omega tables, status word, workspace) and
// dispatch to the kernels.  No C++ exception crosses the ABI.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "../../include/rpmi.h"
#include "rpmi_internal.h"

struct rp_ctx_s {
    int device = 0;
    uint64_t* d_thresholds = nullptr;
    uint32_t* d_guide = nullptr;
    int table_count = 0;
    unsigned int* d_status = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // contraction-split workspace of the split-FP16 projection: per-tile
    // counters (kept zero between launches) followed by partial sums
    void* split_ws = nullptr;
    size_t split_ws_bytes = 0;
    int num_cus = 0;
    std::string last_error;
};

namespace {

thread_local std::string g_create_error;

rp_status fail(rp_ctx ctx, rp_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->last_error = buf; else g_create_error = buf;
    return s;
}

rp_status hip_fail(rp_ctx ctx, hipError_t e, const char* what) {
    return fail(ctx, e == hipErrorOutOfMemory ? RP_ERR_NOMEM : RP_ERR_HIP, "%s: %s", what,
                hipGetErrorString(e));
}

#define RP_HIP(ctx, call)                                         \
    do {                                                          \
        hipError_t e_ = (call);                                   \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);  \
    } while (0)

rpmi::OmegaTables tables(rp_ctx ctx) {
    return rpmi::OmegaTables{ctx->d_thresholds, ctx->d_guide, ctx->table_count};
}

// Grow the context workspace to at least `bytes`.  Growing synchronises the
// device so that no queued kernel still uses the old buffer.
rp_status ensure_workspace(rp_ctx ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return RP_OK;
    RP_HIP(ctx, hipDeviceSynchronize());
    if (ctx->ws) {
        RP_HIP(ctx, hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    bytes = (bytes + 0xFFFFF) & ~size_t(0xFFFFF);
    RP_HIP(ctx, hipMalloc(&ctx->ws, bytes));
    ctx->ws_bytes = bytes;
    return RP_OK;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

bool desc_ok(rp_ctx ctx, const rp_desc* A, rp_status* st) {
    if (!A) { *st = fail(ctx, RP_ERR_INVALID_ARG, "A descriptor is NULL"); return false; }
    if (A->rows < 0 || A->cols < 0) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "negative A size (%lld x %lld)", (long long)A->rows,
                   (long long)A->cols);
        return false;
    }
    if (A->rows > 0 && A->cols > 0 && !A->ptr) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "A.ptr is NULL"); return false;
    }
    if (A->s_row < 0 || A->s_k_outer < 0 || A->k_inner <= 0) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "invalid A strides (s_row %lld, k_inner %lld, s_k_outer %lld)",
                   (long long)A->s_row, (long long)A->k_inner, (long long)A->s_k_outer);
        return false;
    }
    return true;
}

}  // namespace

extern "C" {

const char* rp_status_string(rp_status s) {
    switch (s) {
        case RP_OK: return "RP_OK";
        case RP_ERR_INVALID_ARG: return "RP_ERR_INVALID_ARG";
        case RP_ERR_UNSUPPORTED: return "RP_ERR_UNSUPPORTED";
        case RP_ERR_RANGE: return "RP_ERR_RANGE";
        case RP_ERR_NOT_SPD: return "RP_ERR_NOT_SPD";
        case RP_ERR_NOT_CONVERGED: return "RP_ERR_NOT_CONVERGED";
        case RP_ERR_NOMEM: return "RP_ERR_NOMEM";
        case RP_ERR_HIP: return "RP_ERR_HIP";
    }
    return "unknown rp_status";
}

const char* rp_last_error(rp_ctx ctx) {
    return ctx ? ctx->last_error.c_str() : g_create_error.c_str();
}

rp_status rp_create(rp_ctx* out, int device) {
    if (!out) return fail(nullptr, RP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
    if (device < 0 || device >= count)
        return fail(nullptr, RP_ERR_INVALID_ARG, "device %d out of range (%d devices)", device, count);
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");

    std::vector<uint64_t> thr(rpmi::kF16TableMax);
    const int n = rpmi_build_f16_thresholds(thr.data(), rpmi::kF16TableMax);
    if (n <= 0) return fail(nullptr, RP_ERR_HIP, "threshold table construction failed");
    std::vector<uint32_t> guide(rpmi::kGuideSize);
    rpmi_build_guide(thr.data(), n, guide.data(), rpmi::kGuideLog2);

    rp_ctx ctx = new (std::nothrow) rp_ctx_s;
    if (!ctx) return fail(nullptr, RP_ERR_NOMEM, "host allocation failed");
    ctx->device = device;
    ctx->table_count = n;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
    }
    auto cleanup = [&](hipError_t err, const char* what) {
        rp_status s = hip_fail(nullptr, err, what);
        rp_destroy(ctx);
        return s;
    };
    if ((e = hipMalloc(&ctx->d_thresholds, n * sizeof(uint64_t))) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMalloc(&ctx->d_guide, guide.size() * sizeof(uint32_t))) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMalloc(&ctx->d_status, sizeof(unsigned int))) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMemcpy(ctx->d_thresholds, thr.data(), n * sizeof(uint64_t), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMemcpy(ctx->d_guide, guide.data(), guide.size() * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMemset(ctx->d_status, 0, sizeof(unsigned int))) != hipSuccess) return cleanup(e, "hipMemset");
    *out = ctx;
    return RP_OK;
}

rp_status rp_destroy(rp_ctx ctx) {
    if (!ctx) return RP_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->d_thresholds) (void)hipFree(ctx->d_thresholds);
    if (ctx->d_guide) (void)hipFree(ctx->d_guide);
    if (ctx->d_status) (void)hipFree(ctx->d_status);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->split_ws) (void)hipFree(ctx->split_ws);
    delete ctx;
    return RP_OK;
}

rp_status rp_omega_generate(rp_ctx ctx, uint64_t seed, uint32_t stream_id, int64_t n, int64_t r,
                            rp_omega_t type, void* omega, int64_t ldo, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    if (n < 0 || r < 0) return fail(ctx, RP_ERR_INVALID_ARG, "negative size (n %lld, r %lld)", (long long)n, (long long)r);
    if (type != RP_OMEGA_F16 && type != RP_OMEGA_F32)
        return fail(ctx, RP_ERR_INVALID_ARG, "unknown omega type %d", (int)type);
    if (n == 0 || r == 0) return RP_OK;
    if (!omega) return fail(ctx, RP_ERR_INVALID_ARG, "omega is NULL");
    if (ldo < r) return fail(ctx, RP_ERR_INVALID_ARG, "ldo %lld < r %lld", (long long)ldo, (long long)r);
    RP_HIP(ctx, hipSetDevice(ctx->device));
    RP_HIP(ctx, rpmi::launch_omega_rowmajor(tables(ctx), seed, stream_id, n, r, type == RP_OMEGA_F32,
                                            omega, ldo, (hipStream_t)stream));
    return RP_OK;
}

}  // extern "C"

namespace {

// Validates A for the projection kernels; sets *st on failure.
bool proj_layout_ok(rp_ctx ctx, const rp_desc* A, rp_status* st) {
    const int64_t n = A->cols;
    const int64_t kstep = rpmi::proj_k_block();
    if (A->s_k_inner != 1) {
        *st = fail(ctx, RP_ERR_UNSUPPORTED, "A with s_k_inner != 1 is not supported");
        return false;
    }
    if (A->k_inner > n) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "k_inner %lld exceeds cols %lld", (long long)A->k_inner, (long long)n);
        return false;
    }
    if (A->k_inner < n && n % A->k_inner != 0) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "cols must be a multiple of k_inner");
        return false;
    }
    if (A->k_inner < n && A->k_inner % kstep != 0) {
        *st = fail(ctx, RP_ERR_UNSUPPORTED, "k_inner must equal cols or be a multiple of %lld", (long long)kstep);
        return false;
    }
    if (reinterpret_cast<uintptr_t>(A->ptr) & 3) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "A.ptr is not 4-byte aligned");
        return false;
    }
    return true;
}

rpmi::PackedOmega packed_geometry(int64_t n, int64_t r, rp_algo_t algo, void* data) {
    rpmi::PackedOmega pk;
    const int64_t col_block = algo == RP_ALGO_SPLIT_F16 ? rpmi::split_f16_col_block() : rpmi::f32_col_block();
    pk.kb_count = round_up(n, rpmi::proj_k_block()) / rpmi::kKBlock;
    pk.nt_count = round_up(r, col_block) / rpmi::kNTile;
    pk.data = data;
    return pk;
}

size_t packed_bytes(const rpmi::PackedOmega& pk, rp_algo_t algo) {
    return (size_t)pk.kb_count * pk.nt_count * 64 * 8 * (algo == RP_ALGO_SPLIT_F16 ? 2 : 4);
}

bool enums_ok(rp_ctx ctx, rp_omega_t type, rp_algo_t algo, rp_status* st) {
    if (type != RP_OMEGA_F16 && type != RP_OMEGA_F32) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "unknown omega type %d", (int)type);
        return false;
    }
    if (algo != RP_ALGO_F32 && algo != RP_ALGO_SPLIT_F16) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "unknown algorithm %d", (int)algo);
        return false;
    }
    if (algo == RP_ALGO_SPLIT_F16 && type != RP_OMEGA_F16) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "the split-FP16 projection needs an FP16 Omega");
        return false;
    }
    return true;
}

// Fill `pk` (fragment order for `algo`) from a caller Omega or from the
// generator; `scratch` holds a row-major FP32/FP16 Omega when one has to be
// generated before widening (FP32 algorithm without a caller Omega).
rp_status fill_packed(rp_ctx ctx, uint64_t seed, uint32_t stream_id, const void* omega, int64_t ldo,
                      rp_omega_t type, int64_t n, int64_t r, rp_algo_t algo,
                      const rpmi::PackedOmega& pk, void* scratch, hipStream_t s) {
    if (algo == RP_ALGO_SPLIT_F16) {
        if (omega) RP_HIP(ctx, rpmi::launch_pack_omega(omega, false, n, r, ldo, pk, false, s));
        else RP_HIP(ctx, rpmi::launch_omega_packed_f16(tables(ctx), seed, stream_id, n, r, pk, s));
        return RP_OK;
    }
    const bool src_f32 = type == RP_OMEGA_F32;
    const void* src = omega;
    if (!omega) {
        RP_HIP(ctx, rpmi::launch_omega_rowmajor(tables(ctx), seed, stream_id, n, r, src_f32, scratch, r, s));
        src = scratch;
        ldo = r;
    }
    RP_HIP(ctx, rpmi::launch_pack_omega(src, src_f32, n, r, ldo, pk, true, s));
    return RP_OK;
}

// Grow the split workspace to hold `counters` zeroed counter bytes plus
// `partials` bytes (synchronises the device when it grows).
rp_status ensure_split_workspace(rp_ctx ctx, size_t counters, size_t partials) {
    const size_t need = ((counters + 255) & ~size_t(255)) + partials;
    if (need <= ctx->split_ws_bytes) return RP_OK;
    RP_HIP(ctx, hipDeviceSynchronize());
    if (ctx->split_ws) {
        RP_HIP(ctx, hipFree(ctx->split_ws));
        ctx->split_ws = nullptr;
        ctx->split_ws_bytes = 0;
    }
    const size_t bytes = (need + 0xFFFFF) & ~size_t(0xFFFFF);
    RP_HIP(ctx, hipMalloc(&ctx->split_ws, bytes));
    RP_HIP(ctx, hipMemset(ctx->split_ws, 0, bytes));
    ctx->split_ws_bytes = bytes;
    return RP_OK;
}

rp_status launch_projection(rp_ctx ctx, const rp_desc* A, int64_t r, const rpmi::PackedOmega& pk,
                            rp_algo_t algo, float* Y, int64_t ldy, hipStream_t s) {
    rpmi::ProjArgs a;
    a.A = A->ptr; a.m = A->rows; a.n = A->cols;
    a.s_row = A->s_row;
    a.k_inner = A->k_inner;
    a.s_k_outer = A->s_k_outer;
    a.omega = pk.data; a.nt_count = pk.nt_count;
    a.Y = Y; a.ldy = ldy; a.r = r;
    a.status = ctx->d_status;
    a.ksplit = 1; a.partial = nullptr; a.counters = nullptr;
    if (algo == RP_ALGO_SPLIT_F16) {
        const rpmi::SplitPlan plan = rpmi::plan_split_f16(a.m, a.n, r, ctx->num_cus > 0 ? ctx->num_cus : 256);
        if (plan.ksplit > 1) {
            rp_status st = ensure_split_workspace(ctx, plan.counter_bytes, plan.partial_bytes);
            if (st != RP_OK) return st;
            a.ksplit = plan.ksplit;
            a.counters = static_cast<unsigned int*>(ctx->split_ws);
            a.partial = reinterpret_cast<float*>(static_cast<char*>(ctx->split_ws) +
                                                 ((plan.counter_bytes + 255) & ~size_t(255)));
        }
        RP_HIP(ctx, rpmi::launch_project_split_f16(a, s));
    } else {
        RP_HIP(ctx, rpmi::launch_project_f32(a, s));
    }
    return RP_OK;
}

}  // namespace

extern "C" {

rp_status rp_omega_packed_size(int64_t n, int64_t r, rp_algo_t algo, size_t* bytes) {
    if (!bytes || n < 0 || r < 0 || (algo != RP_ALGO_F32 && algo != RP_ALGO_SPLIT_F16))
        return fail(nullptr, RP_ERR_INVALID_ARG, "invalid arguments to rp_omega_packed_size");
    *bytes = packed_bytes(packed_geometry(n, r, algo, nullptr), algo);
    return RP_OK;
}

rp_status rp_omega_pack(rp_ctx ctx, uint64_t seed, uint32_t stream_id, const void* omega,
                        int64_t ldo, rp_omega_t type, int64_t n, int64_t r, rp_algo_t algo,
                        void* packed, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    rp_status st;
    if (!enums_ok(ctx, type, algo, &st)) return st;
    if (n < 0 || r < 0) return fail(ctx, RP_ERR_INVALID_ARG, "negative size");
    const rpmi::PackedOmega pk = packed_geometry(n, r, algo, packed);
    if (packed_bytes(pk, algo) == 0) return RP_OK;
    if (!packed) return fail(ctx, RP_ERR_INVALID_ARG, "packed is NULL");
    if (omega && ldo < r) return fail(ctx, RP_ERR_INVALID_ARG, "ldo %lld < r %lld", (long long)ldo, (long long)r);
    RP_HIP(ctx, hipSetDevice(ctx->device));
    void* scratch = nullptr;
    if (!omega && algo == RP_ALGO_F32) {
        if ((st = ensure_workspace(ctx, (size_t)n * r * (type == RP_OMEGA_F32 ? 4 : 2))) != RP_OK) return st;
        scratch = ctx->ws;
    }
    return fill_packed(ctx, seed, stream_id, omega, ldo, type, n, r, algo, pk, scratch, (hipStream_t)stream);
}

rp_status rp_project_packed(rp_ctx ctx, const rp_desc* A, int64_t r, const void* packed,
                            rp_algo_t algo, float* Y, int64_t ldy, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    rp_status st;
    if (!desc_ok(ctx, A, &st)) return st;
    if (algo != RP_ALGO_F32 && algo != RP_ALGO_SPLIT_F16)
        return fail(ctx, RP_ERR_INVALID_ARG, "unknown algorithm %d", (int)algo);
    if (r < 0) return fail(ctx, RP_ERR_INVALID_ARG, "negative r %lld", (long long)r);
    const int64_t m = A->rows, n = A->cols;
    if (m == 0 || r == 0) return RP_OK;
    if (!Y) return fail(ctx, RP_ERR_INVALID_ARG, "Y is NULL");
    if (ldy < r) return fail(ctx, RP_ERR_INVALID_ARG, "ldy %lld < r %lld", (long long)ldy, (long long)r);
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipSetDevice(ctx->device));
    if (n == 0) {
        RP_HIP(ctx, rpmi::launch_fill_f32(Y, m, r, ldy, 0.0f, s));
        return RP_OK;
    }
    if (!packed) return fail(ctx, RP_ERR_INVALID_ARG, "packed is NULL");
    if (!proj_layout_ok(ctx, A, &st)) return st;
    return launch_projection(ctx, A, r, packed_geometry(n, r, algo, const_cast<void*>(packed)), algo, Y, ldy, s);
}

rp_status rp_project(rp_ctx ctx, const rp_desc* A, int64_t r, rp_omega_t omega_type, uint64_t seed,
                     uint32_t stream_id, const void* omega, int64_t ldo, rp_algo_t algo, float* Y,
                     int64_t ldy, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    rp_status st;
    if (!desc_ok(ctx, A, &st)) return st;
    if (r < 0) return fail(ctx, RP_ERR_INVALID_ARG, "negative r %lld", (long long)r);
    if (!enums_ok(ctx, omega_type, algo, &st)) return st;
    const int64_t m = A->rows, n = A->cols;
    if (m == 0 || r == 0) return RP_OK;
    if (!Y) return fail(ctx, RP_ERR_INVALID_ARG, "Y is NULL");
    if (ldy < r) return fail(ctx, RP_ERR_INVALID_ARG, "ldy %lld < r %lld", (long long)ldy, (long long)r);
    if (omega && ldo < r) return fail(ctx, RP_ERR_INVALID_ARG, "ldo %lld < r %lld", (long long)ldo, (long long)r);
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipSetDevice(ctx->device));
    if (n == 0) {
        RP_HIP(ctx, rpmi::launch_fill_f32(Y, m, r, ldy, 0.0f, s));
        return RP_OK;
    }
    if (!proj_layout_ok(ctx, A, &st)) return st;
    rpmi::PackedOmega pk = packed_geometry(n, r, algo, nullptr);
    const size_t pbytes = packed_bytes(pk, algo);
    const bool need_raw = !omega && algo == RP_ALGO_F32;
    const size_t raw_off = (pbytes + 255) & ~size_t(255);
    const size_t raw_bytes = need_raw ? (size_t)n * r * (omega_type == RP_OMEGA_F32 ? 4 : 2) : 0;
    if ((st = ensure_workspace(ctx, raw_off + raw_bytes)) != RP_OK) return st;
    pk.data = ctx->ws;
    void* raw = static_cast<char*>(ctx->ws) + raw_off;
    if ((st = fill_packed(ctx, seed, stream_id, omega, ldo, omega_type, n, r, algo, pk, raw, s)) != RP_OK)
        return st;
    return launch_projection(ctx, A, r, pk, algo, Y, ldy, s);
}

rp_status rp_split_f16(rp_ctx ctx, const float* x, int64_t count, uint16_t* hi, uint16_t* lo,
                       void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    if (count < 0) return fail(ctx, RP_ERR_INVALID_ARG, "negative count");
    if (count == 0) return RP_OK;
    if (!x || !hi || !lo) return fail(ctx, RP_ERR_INVALID_ARG, "NULL pointer");
    RP_HIP(ctx, hipSetDevice(ctx->device));
    RP_HIP(ctx, rpmi::launch_split_dump(x, count, hi, lo, (hipStream_t)stream));
    return RP_OK;
}

rp_status rp_get_device_status(rp_ctx ctx, void* stream, int clear, rp_status* out) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    if (!out) return fail(ctx, RP_ERR_INVALID_ARG, "out is NULL");
    RP_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipStreamSynchronize(s));
    unsigned int word = 0;
    RP_HIP(ctx, hipMemcpy(&word, ctx->d_status, sizeof word, hipMemcpyDeviceToHost));
    if (clear) RP_HIP(ctx, hipMemset(ctx->d_status, 0, sizeof(unsigned int)));
    *out = (word & rpmi::kStatusRange) ? RP_ERR_RANGE
         : (word & rpmi::kStatusNotSpd) ? RP_ERR_NOT_SPD
         : (word & rpmi::kStatusNotConverged) ? RP_ERR_NOT_CONVERGED
         : RP_OK;
    return RP_OK;
}

}  // extern "C"
