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
    void* split_ws = nullptr;            // split-K partial sums (scratch)
    size_t split_ws_bytes = 0;
    unsigned int* split_counters = nullptr;   // per-tile arrival counters: zero
    size_t split_counter_bytes = 0;           // between launches (reset by each tile's last workgroup)
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
    if (ctx->split_counters) (void)hipFree(ctx->split_counters);
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
    const int64_t col_block = algo == RP_ALGO_SPLIT_F16 ? rpmi::split_f16_col_block(r) : rpmi::f32_col_block();
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

// Grow the split-K buffers: `counters` bytes of arrival counters in their own
// allocation (zeroed when allocated; every launch leaves them zero) and
// `partials` bytes of partial-sum scratch.  Synchronises the device when
// either grows.
rp_status ensure_split_workspace(rp_ctx ctx, size_t counters, size_t partials) {
    if (counters > ctx->split_counter_bytes) {
        RP_HIP(ctx, hipDeviceSynchronize());
        if (ctx->split_counters) {
            RP_HIP(ctx, hipFree(ctx->split_counters));
            ctx->split_counters = nullptr;
            ctx->split_counter_bytes = 0;
        }
        const size_t bytes = (counters + 0xFFFF) & ~size_t(0xFFFF);
        RP_HIP(ctx, hipMalloc(&ctx->split_counters, bytes));
        RP_HIP(ctx, hipMemset(ctx->split_counters, 0, bytes));
        RP_HIP(ctx, hipDeviceSynchronize());
        ctx->split_counter_bytes = bytes;
    }
    if (partials > ctx->split_ws_bytes) {
        RP_HIP(ctx, hipDeviceSynchronize());
        if (ctx->split_ws) {
            RP_HIP(ctx, hipFree(ctx->split_ws));
            ctx->split_ws = nullptr;
            ctx->split_ws_bytes = 0;
        }
        const size_t bytes = (partials + 0xFFFFF) & ~size_t(0xFFFFF);
        RP_HIP(ctx, hipMalloc(&ctx->split_ws, bytes));
        ctx->split_ws_bytes = bytes;
    }
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
            a.counters = ctx->split_counters;
            a.partial = static_cast<float*>(ctx->split_ws);
        }
        RP_HIP(ctx, rpmi::launch_project_split_f16(a, s));
    } else {
        RP_HIP(ctx, rpmi::launch_project_f32(a, s));
    }
    return RP_OK;
}

// Several split-FP16 projections in one grouped launch (every problem on the
// 16-byte path, all with r <= 128 or all with r > 128); the contraction split
// of each problem is planned for its share of the compute units, in
// proportion to its A bytes.  Returns RP_ERR_UNSUPPORTED (nothing launched)
// when the problems do not qualify; the caller then launches them one by one.
rp_status launch_projection_grouped(rp_ctx ctx, int count, const rp_desc* const* A, const int64_t* r,
                                    const rpmi::PackedOmega* pk, float* const* Y, const int64_t* ldy,
                                    hipStream_t s) {
    if (count <= 0 || count > rpmi::kMaxGroup) return RP_ERR_UNSUPPORTED;
    const bool narrow = r[0] <= 128;
    rpmi::GroupArgs ga;
    ga.count = count;
    double total = 0;
    for (int g = 0; g < count; ++g) total += (double)A[g]->rows * A[g]->cols;
    const int cus = ctx->num_cus > 0 ? ctx->num_cus : 256;
    size_t counter_bytes = 0, partial_bytes = 0;
    rpmi::SplitPlan plans[rpmi::kMaxGroup];
    for (int g = 0; g < count; ++g) {
        if ((r[g] <= 128) != narrow || A[g]->rows == 0 || A[g]->cols == 0 || r[g] == 0) return RP_ERR_UNSUPPORTED;
        rpmi::ProjArgs& a = ga.prob[g];
        a.A = A[g]->ptr; a.m = A[g]->rows; a.n = A[g]->cols;
        a.s_row = A[g]->s_row; a.k_inner = A[g]->k_inner; a.s_k_outer = A[g]->s_k_outer;
        a.omega = pk[g].data; a.nt_count = pk[g].nt_count;
        a.Y = Y[g]; a.ldy = ldy[g]; a.r = r[g];
        a.status = ctx->d_status;
        if (!rpmi::split_vector_ok(a)) return RP_ERR_UNSUPPORTED;
        int share = (int)(cus * ((double)a.m * a.n / total) + 0.5);
        plans[g] = rpmi::plan_split_f16(a.m, a.n, a.r, share > 0 ? share : 1);
        counter_bytes += (plans[g].counter_bytes + 255) & ~size_t(255);
        partial_bytes += (plans[g].partial_bytes + 255) & ~size_t(255);
    }
    rp_status st = ensure_split_workspace(ctx, counter_bytes, partial_bytes);
    if (st != RP_OK) return st;
    char* cbase = reinterpret_cast<char*>(ctx->split_counters);
    char* pbase = static_cast<char*>(ctx->split_ws);
    ga.start[0] = 0;
    for (int g = 0; g < count; ++g) {
        rpmi::ProjArgs& a = ga.prob[g];
        a.ksplit = plans[g].ksplit;
        a.counters = a.ksplit > 1 ? reinterpret_cast<unsigned int*>(cbase) : nullptr;
        a.partial = a.ksplit > 1 ? reinterpret_cast<float*>(pbase) : nullptr;
        cbase += (plans[g].counter_bytes + 255) & ~size_t(255);
        pbase += (plans[g].partial_bytes + 255) & ~size_t(255);
        ga.tiles_m[g] = (a.m + rpmi::split_group_tile_m(a.r) - 1) / rpmi::split_group_tile_m(a.r);
        ga.tiles_n[g] = (a.r + rpmi::split_group_tile_n(a.r) - 1) / rpmi::split_group_tile_n(a.r);
        ga.start[g + 1] = ga.start[g] + ga.tiles_m[g] * ga.tiles_n[g] * a.ksplit;
    }
    RP_HIP(ctx, rpmi::launch_project_split_f16_grouped(ga, narrow, s));
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

}  // extern "C"

namespace {

// Bump allocator over the context workspace (256-byte aligned pieces).
struct Arena {
    size_t used = 0;
    size_t take(size_t bytes) {
        const size_t off = used;
        used += (bytes + 255) & ~size_t(255);
        return off;
    }
};

// CholeskyQR2 of the m x p matrix Y (FP32, leading dimension ldy):
// Q (FP32, ldq) with orthonormal columns spanning Y, and, if M != NULL, the
// p x p lower-triangular product L1 L2 of the two Cholesky factors
// (= R^T for R = R2 R1, Y = Q R).  Scratch: Qd (m x p FP64), G, X (p x p FP64
// each) and L1 (p x p FP64, kept only when M is requested).
rp_status cholqr2(rp_ctx ctx, int64_t m, int64_t p, const float* Y, int64_t ldy, float* Q, int64_t ldq,
                  double* M, double* Qd, double* G, double* X, double* L1, hipStream_t s) {
    unsigned int* st = ctx->d_status;
    // pass 1: G = Y^T Y, G = L L^T, X = L^-1, Qd = Y X^T  (= Y R^-1)
    RP_HIP(ctx, (rpmi::gemm_acc64<float, float, double>(p, p, m, 1.0, Y, 1, ldy, Y, ldy, 1, 0.0, G, p, 1, s)));
    RP_HIP(ctx, rpmi::potrf_lower(G, p, p, st, s));
    RP_HIP(ctx, rpmi::trtri_lower(G, p, X, p, p, s));
    RP_HIP(ctx, (rpmi::gemm_acc64<float, double, double>(m, p, p, 1.0, Y, ldy, 1, X, 1, p, 0.0, Qd, p, 1, s)));
    if (M) RP_HIP(ctx, hipMemcpyAsync(L1, G, (size_t)p * p * sizeof(double), hipMemcpyDeviceToDevice, s));
    // pass 2 on Qd
    RP_HIP(ctx, (rpmi::gemm_acc64<double, double, double>(p, p, m, 1.0, Qd, 1, p, Qd, p, 1, 0.0, G, p, 1, s)));
    RP_HIP(ctx, rpmi::potrf_lower(G, p, p, st, s));
    RP_HIP(ctx, rpmi::trtri_lower(G, p, X, p, p, s));
    RP_HIP(ctx, (rpmi::gemm_acc64<double, double, float>(m, p, p, 1.0, Qd, p, 1, X, 1, p, 0.0, Q, ldq, 1, s)));
    if (M) RP_HIP(ctx, (rpmi::gemm_acc64<double, double, double>(p, p, p, 1.0, L1, p, 1, G, p, 1, 0.0, M, p, 1, s)));
    return RP_OK;
}

}  // namespace

extern "C" {

rp_status rsvd(rp_ctx ctx, int64_t m, int64_t n, const float* A, int64_t lda, int64_t k, int64_t oversample,
               int32_t power_iters, uint64_t seed, rp_omega_t omega_type, rp_algo_t algo, float* U, int64_t ldu,
               double* S, float* VT, int64_t ldvt, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    rp_status st;
    if (!enums_ok(ctx, omega_type, algo, &st)) return st;
    const int64_t p = k + oversample;
    if (m <= 0 || n <= 0 || k <= 0 || oversample < 0 || power_iters < 0)
        return fail(ctx, RP_ERR_INVALID_ARG, "invalid sizes (m %lld, n %lld, k %lld, s %lld, q %d)", (long long)m,
                    (long long)n, (long long)k, (long long)oversample, (int)power_iters);
    if (p > m || p > n || p > 1024)
        return fail(ctx, RP_ERR_INVALID_ARG, "k + oversample = %lld must be <= min(m, n) and <= 1024", (long long)p);
    if (!A || !U || !S || !VT) return fail(ctx, RP_ERR_INVALID_ARG, "NULL pointer");
    if (lda < n || ldu < k || ldvt < n) return fail(ctx, RP_ERR_INVALID_ARG, "leading dimension too small");
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipSetDevice(ctx->device));

    rp_desc dA{A, m, n, lda, n, 1, 0};
    if (!proj_layout_ok(ctx, &dA, &st)) return st;

    // workspace layout
    Arena ar;
    rpmi::PackedOmega pk = packed_geometry(n, p, algo, nullptr);
    const size_t o_pk = ar.take(packed_bytes(pk, algo));
    const rpmi::PackedOmega pkw_geom = packed_geometry(n, p, RP_ALGO_F32, nullptr);   // W for Y = A W
    const size_t o_pkw = ar.take(packed_bytes(pkw_geom, RP_ALGO_F32));
    const size_t o_raw = ar.take(algo == RP_ALGO_F32 ? (size_t)n * p * 4 : 0);       // raw Omega (FP32 path)
    const int64_t mx = m > n ? m : n;
    const size_t o_y = ar.take((size_t)m * p * 4);        // Y (m x p)
    const size_t o_q = ar.take((size_t)m * p * 4);        // Q (m x p)
    const size_t o_z = ar.take((size_t)n * p * 4);        // Z / B^T (n x p)
    const size_t o_w = ar.take((size_t)n * p * 4);        // W / Q_B (n x p)
    const size_t o_qd = ar.take((size_t)mx * p * 8);      // FP64 Q of the first CholeskyQR pass
    const size_t o_g = ar.take((size_t)p * p * 8);
    const size_t o_x = ar.take((size_t)p * p * 8);
    const size_t o_l1 = ar.take((size_t)p * p * 8);
    const size_t o_mw = ar.take((size_t)p * p * 8);       // R_B^T -> Jacobi W
    const size_t o_mv = ar.take((size_t)p * p * 8);       // Jacobi V
    const size_t o_sig = ar.take((size_t)p * 8);
    const size_t o_ord = ar.take((size_t)p * 4);
    const size_t o_ur = ar.take((size_t)p * k * 8);
    const size_t o_vr = ar.take((size_t)p * k * 8);
    if ((st = ensure_workspace(ctx, ar.used)) != RP_OK) return st;
    char* base = static_cast<char*>(ctx->ws);
    pk.data = base + o_pk;
    rpmi::PackedOmega pkw = pkw_geom;
    pkw.data = base + o_pkw;
    float* Y = reinterpret_cast<float*>(base + o_y);
    float* Q = reinterpret_cast<float*>(base + o_q);
    float* Z = reinterpret_cast<float*>(base + o_z);
    float* W = reinterpret_cast<float*>(base + o_w);
    double* Qd = reinterpret_cast<double*>(base + o_qd);
    double* G = reinterpret_cast<double*>(base + o_g);
    double* X = reinterpret_cast<double*>(base + o_x);
    double* L1 = reinterpret_cast<double*>(base + o_l1);
    double* MW = reinterpret_cast<double*>(base + o_mw);
    double* MV = reinterpret_cast<double*>(base + o_mv);
    double* sig = reinterpret_cast<double*>(base + o_sig);
    int* ord = reinterpret_cast<int*>(base + o_ord);
    double* Ur = reinterpret_cast<double*>(base + o_ur);
    double* Vr = reinterpret_cast<double*>(base + o_vr);

    // Algorithm 1 line 1: Y = A Omega
    if ((st = fill_packed(ctx, seed, 0, nullptr, 0, omega_type, n, p, algo, pk, base + o_raw, s)) != RP_OK) return st;
    if ((st = launch_projection(ctx, &dA, p, pk, algo, Y, p, s)) != RP_OK) return st;
    // power scheme, re-orthonormalised
    for (int32_t t = 0; t < power_iters; ++t) {
        if ((st = cholqr2(ctx, m, p, Y, p, Q, p, nullptr, Qd, G, X, L1, s)) != RP_OK) return st;
        // Z = A^T Q (n x p)
        RP_HIP(ctx, (rpmi::gemm_acc64<float, float, float>(n, p, m, 1.0, A, 1, lda, Q, p, 1, 0.0, Z, p, 1, s)));
        if ((st = cholqr2(ctx, n, p, Z, p, W, p, nullptr, Qd, G, X, L1, s)) != RP_OK) return st;
        // Y = A W (FP32 x FP32): the FP32 projection kernel with W (n x p) in
        // fragment order
        RP_HIP(ctx, rpmi::launch_pack_omega(W, true, n, p, p, pkw, true, s));
        if ((st = launch_projection(ctx, &dA, p, pkw, RP_ALGO_F32, Y, p, s)) != RP_OK) return st;
    }
    // Algorithm 1 line 2: Q = QR(Y)
    if ((st = cholqr2(ctx, m, p, Y, p, Q, p, nullptr, Qd, G, X, L1, s)) != RP_OK) return st;
    // line 3: B^T = A^T Q (n x p)
    RP_HIP(ctx, (rpmi::gemm_acc64<float, float, float>(n, p, m, 1.0, A, 1, lda, Q, p, 1, 0.0, Z, p, 1, s)));
    // line 4: B^T = Q_B R_B; R_B^T = L1 L2 (p x p lower) into MW
    if ((st = cholqr2(ctx, n, p, Z, p, W, p, MW, Qd, G, X, L1, s)) != RP_OK) return st;
    // SVD of R_B^T = U_r S V_r^T: then B = U_r S (Q_B V_r)^T
    RP_HIP(ctx, rpmi::jacobi_svd(MW, MV, (int)p, 40, 1e-14, ctx->d_status, s));
    RP_HIP(ctx, rpmi::svd_finish(MW, MV, (int)p, (int)k, sig, ord, Ur, Vr, s));
    RP_HIP(ctx, hipMemcpyAsync(S, sig, (size_t)k * sizeof(double), hipMemcpyDeviceToDevice, s));
    // line 5: U = Q U_r[:, :k] (m x k); V^T = (Q_B V_r[:, :k])^T (k x n)
    RP_HIP(ctx, (rpmi::gemm_acc64<float, double, float>(m, k, p, 1.0, Q, p, 1, Ur, k, 1, 0.0, U, ldu, 1, s)));
    RP_HIP(ctx, (rpmi::gemm_acc64<float, double, float>(n, k, p, 1.0, W, p, 1, Vr, k, 1, 0.0, VT, 1, ldvt, s)));
    return RP_OK;
}

rp_status rp_hosvd(rp_ctx ctx, int32_t ndim, const int64_t* dims, const float* X, const int64_t* ranks,
                   uint64_t seed, rp_omega_t omega_type, rp_algo_t algo, float* core, float* const* factors,
                   void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    rp_status st;
    if (!enums_ok(ctx, omega_type, algo, &st)) return st;
    if (ndim < 2 || ndim > rpmi::kMaxGroup)
        return fail(ctx, RP_ERR_INVALID_ARG, "ndim %d outside [2, %d]", (int)ndim, rpmi::kMaxGroup);
    if (!dims || !ranks || !X || !core || !factors) return fail(ctx, RP_ERR_INVALID_ARG, "NULL pointer");
    const int N = ndim;
    int64_t total = 1;
    for (int i = 0; i < N; ++i) {
        if (dims[i] <= 0) return fail(ctx, RP_ERR_INVALID_ARG, "dims[%d] = %lld", i, (long long)dims[i]);
        total *= dims[i];
    }
    for (int i = 0; i < N; ++i) {
        const int64_t cols = total / dims[i];
        if (ranks[i] <= 0 || ranks[i] > dims[i] || ranks[i] > cols || ranks[i] > 1024)
            return fail(ctx, RP_ERR_INVALID_ARG, "ranks[%d] = %lld must be in [1, min(dims[%d], %lld, 1024)]", i,
                        (long long)ranks[i], i, (long long)cols);
        if (!factors[i]) return fail(ctx, RP_ERR_INVALID_ARG, "factors[%d] is NULL", i);
    }
    if (reinterpret_cast<uintptr_t>(X) & 3) return fail(ctx, RP_ERR_INVALID_ARG, "X is not 4-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipSetDevice(ctx->device));

    // mode-i unfolding of the C-order tensor: rows i_i, columns the C-order
    // index of the other modes = (leading index) * after + (trailing index);
    // element offset = i_i * after + lead * (dims[i] * after) + trail
    int64_t after[rpmi::kMaxGroup], before[rpmi::kMaxGroup];
    for (int i = N - 1, a = 1; i >= 0; --i) { after[i] = a; a *= dims[i]; }
    for (int i = 0; i < N; ++i) before[i] = total / (dims[i] * after[i]);
    rp_desc desc[rpmi::kMaxGroup];
    bool permuted[rpmi::kMaxGroup];
    int64_t maxr = 0, maxd = 0, perm_elems = 0;
    for (int i = 0; i < N; ++i) {
        const int64_t cols = total / dims[i];
        desc[i] = rp_desc{X, dims[i], cols, after[i], after[i] == 1 && before[i] > 1 ? 1 : after[i], 1,
                          dims[i] * after[i]};
        if (before[i] == 1) desc[i].k_inner = cols;             // mode 1: plain row-major
        rp_status dummy;
        permuted[i] = !(before[i] == 1 || (after[i] % rpmi::proj_k_block() == 0 && after[i] > 1));
        if (!permuted[i] && !proj_layout_ok(ctx, &desc[i], &dummy)) permuted[i] = true;
        if (permuted[i]) perm_elems = total;
        maxr = ranks[i] > maxr ? ranks[i] : maxr;
        maxd = dims[i] > maxd ? dims[i] : maxd;
    }
    // core intermediates: after contracting modes 0..i, shape [J_0..J_i, I_{i+1}..]
    int64_t tmax = 0;
    {
        int64_t lead = 1;
        for (int i = 0; i < N - 1; ++i) {
            lead *= ranks[i];
            const int64_t e = lead * after[i];
            tmax = e > tmax ? e : tmax;
        }
    }
    Arena ar;
    size_t o_pk[rpmi::kMaxGroup], o_w[rpmi::kMaxGroup];
    rpmi::PackedOmega pk[rpmi::kMaxGroup];
    size_t raw_bytes = 0;
    for (int i = 0; i < N; ++i) {
        const int64_t cols = total / dims[i];
        pk[i] = packed_geometry(cols, ranks[i], algo, nullptr);
        o_pk[i] = ar.take(packed_bytes(pk[i], algo));
        o_w[i] = ar.take((size_t)dims[i] * ranks[i] * 4);
        if (algo == RP_ALGO_F32) {
            const size_t rb = (size_t)cols * ranks[i] * (omega_type == RP_OMEGA_F32 ? 4 : 2);
            raw_bytes = rb > raw_bytes ? rb : raw_bytes;
        }
    }
    const size_t o_raw = ar.take(raw_bytes);
    const size_t o_perm = ar.take((size_t)perm_elems * 4);
    const size_t o_qd = ar.take((size_t)maxd * maxr * 8);
    const size_t o_g = ar.take((size_t)maxr * maxr * 8);
    const size_t o_x = ar.take((size_t)maxr * maxr * 8);
    const size_t o_l1 = ar.take((size_t)maxr * maxr * 8);
    const size_t o_t0 = ar.take((size_t)tmax * 4);
    const size_t o_t1 = ar.take((size_t)tmax * 4);
    if ((st = ensure_workspace(ctx, ar.used)) != RP_OK) return st;
    char* base = static_cast<char*>(ctx->ws);
    float* W[rpmi::kMaxGroup];
    int64_t ldw[rpmi::kMaxGroup];
    const rp_desc* dp[rpmi::kMaxGroup];
    float* perm = reinterpret_cast<float*>(base + o_perm);

    // Algorithm 2, first loop: W_i = X_(i) Omega_i, Omega_i from stream i.
    // Modes whose unfolding the projection cannot stream in place are first
    // copied mode-first into one scratch tensor (one mode at a time, so those
    // projections run separately).
    for (int i = 0; i < N; ++i) {
        pk[i].data = base + o_pk[i];
        W[i] = reinterpret_cast<float*>(base + o_w[i]);
        ldw[i] = ranks[i];
        dp[i] = &desc[i];
        const int64_t cols = total / dims[i];
        if ((st = fill_packed(ctx, seed, (uint32_t)i, nullptr, 0, omega_type, cols, ranks[i], algo, pk[i],
                              base + o_raw, s)) != RP_OK)
            return st;
    }
    bool grouped_done = false;
    if (algo == RP_ALGO_SPLIT_F16) {
        const rp_desc* gA[rpmi::kMaxGroup];
        int64_t gr[rpmi::kMaxGroup], gld[rpmi::kMaxGroup];
        rpmi::PackedOmega gpk[rpmi::kMaxGroup];
        float* gY[rpmi::kMaxGroup];
        int cnt = 0;
        for (int i = 0; i < N; ++i) {
            if (permuted[i]) continue;
            gA[cnt] = dp[i]; gr[cnt] = ranks[i]; gld[cnt] = ldw[i]; gpk[cnt] = pk[i]; gY[cnt] = W[i];
            ++cnt;
        }
        bool same_width = true;
        for (int g = 1; g < cnt; ++g) same_width = same_width && ((gr[g] <= 128) == (gr[0] <= 128));
        if (cnt > 1 && same_width) {
            st = launch_projection_grouped(ctx, cnt, gA, gr, gpk, gY, gld, s);
            if (st == RP_OK) grouped_done = true;
            else if (st != RP_ERR_UNSUPPORTED) return st;
        }
    }
    for (int i = 0; i < N; ++i) {
        if (permuted[i]) {
            RP_HIP(ctx, rpmi::launch_swap01(X, before[i], dims[i], after[i], perm, s));
            const int64_t cols = total / dims[i];
            const rp_desc pd{perm, dims[i], cols, cols, cols, 1, 0};
            if ((st = launch_projection(ctx, &pd, ranks[i], pk[i], algo, W[i], ldw[i], s)) != RP_OK) return st;
        } else if (!grouped_done) {
            if ((st = launch_projection(ctx, dp[i], ranks[i], pk[i], algo, W[i], ldw[i], s)) != RP_OK) return st;
        }
    }
    // Q_i = QR(W_i) straight into the caller's factors
    double* Qd = reinterpret_cast<double*>(base + o_qd);
    double* G = reinterpret_cast<double*>(base + o_g);
    double* Xs = reinterpret_cast<double*>(base + o_x);
    double* L1 = reinterpret_cast<double*>(base + o_l1);
    for (int i = 0; i < N; ++i)
        if ((st = cholqr2(ctx, dims[i], ranks[i], W[i], ldw[i], factors[i], ranks[i], nullptr, Qd, G, Xs, L1, s)) !=
            RP_OK)
            return st;
    // core g = X x_1 Q_1^T ... x_N Q_N^T, one mode at a time: T has shape
    // [lead, I_i, after_i]; out[b][j][p] = sum_k Q_i[k][j] T[b][k][p]
    const float* T = X;
    float* bufs[2] = {reinterpret_cast<float*>(base + o_t0), reinterpret_cast<float*>(base + o_t1)};
    int64_t lead = 1;
    for (int i = 0; i < N; ++i) {
        float* out = i == N - 1 ? core : bufs[i & 1];
        const int64_t J = ranks[i], I = dims[i], P = after[i];
        if (P == 1) {
            RP_HIP(ctx, (rpmi::gemm_acc64<float, float, float>(lead, J, I, 1.0, T, I, 1, factors[i], J, 1, 0.0, out, J,
                                                                1, s)));
        } else {
            RP_HIP(ctx, (rpmi::gemm_acc64_batched<float, float, float>(J, P, I, 1.0, factors[i], 1, J, 0, T, P, 1,
                                                                        I * P, 0.0, out, P, 1, J * P, lead, s)));
        }
        T = out;
        lead *= J;
    }
    return RP_OK;
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
