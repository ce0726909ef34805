// C-ABI entry points of librpmi (declared in include/rpmi.h): argument
// validation, context state (Omega tables, status word, workspace) and
// dispatch to the kernels.  No C++ exception crosses the ABI.
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/rpmi.h"
#include "rpmi_internal.h"

struct rp_ctx_s {
    int device = 0;
    uint64_t* d_thresholds = nullptr;
    uint32_t* d_guide = nullptr;
    int table_count = 0;
    unsigned int* d_status = nullptr;
    unsigned int* d_scan = nullptr;      // result of scanning a caller Omega (read back by rp_project)
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // contraction-split workspace of the split-FP16 projection: per-tile
    // counters (kept zero between launches) followed by partial sums
    void* split_ws = nullptr;            // split-K partial sums (scratch)
    size_t split_ws_bytes = 0;
    rpmi::GroupEntry* table = nullptr;    // problem tables of grouped projections (device)
    size_t table_entries = 0;
    unsigned int* split_counters = nullptr;   // per-tile arrival counters: zero
    size_t split_counter_bytes = 0;           // between launches (reset by each tile's last workgroup)
    int num_cus = 0;
    // device address of the no-allocation scratch array on this device
    // (hipGetSymbolAddress at creation; never the array's host-side name)
    unsigned char* noalloc_scratch = nullptr;
    // flag table of the folded split (kFoldFlags words, zeroed at creation)
    // and the launch epoch written into it (never 0)
    unsigned int* fold_flags = nullptr;
    unsigned int fold_epoch = 0;
    std::string last_error;
    // batched RSVD: the captured graph of the last problem set (replayed while
    // the set, its buffers and the context buffers are unchanged), its own
    // device table of grouped projections, and the autotuner's choices
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;      // Omega .. the first graph_jac.graph_sweeps Jacobi sweeps
    hipGraphExec_t graph_exec2 = nullptr;     // the Jacobi final step and the finishing products
    uint64_t graph_key = 0;
    // the batched Jacobi between the two graphs: sweeps beyond the captured
    // ones run eagerly while a problem is open (d_jopen: open problems)
    struct {
        int count, pairs, bpairs, max_n, graph_sweeps, bound;
    } graph_jac = {0, 0, 0, 0, 0, 0};
    int* d_jopen = nullptr;
    rpmi::GroupEntry* graph_table = nullptr;
    size_t graph_table_entries = 0;
    rpmi::JacobiProb* graph_jtab = nullptr;   // the batched Jacobi table read by the graph
    size_t graph_jtab_entries = 0;
    char* graph_aux = nullptr;                // job tables of the grouped stages read by the graph
    size_t graph_aux_bytes = 0;
    // autotuner cache of the grouped projections: per problem-set signature
    // the contraction-split scale and the narrow kernel form (0: register-
    // staged, 1: LDS-staged)
    struct TuneEntry {
        double scale;
        int form;
    };
    std::unordered_map<uint64_t, TuneEntry> tuned_scale;
    std::string tuning_file;              // RPMI_TUNING_FILE at creation ("" if unset)
    int force_form = -1;                  // RPMI_GROUP_FORM at creation (0 or 1), else -1
    int graph_sweeps = -1;                // RPMI_BATCHED_GRAPH_SWEEPS at creation (>= 0), else -1: the default
    // generated Omega kept in device memory, keyed by what defines its bits
    // (seed, stream_id, n, r, type) and by the fragment format (algorithm);
    // least recently used entries are freed beyond kOmegaCacheBytes
    struct OmegaEntry {
        uint64_t seed;
        uint32_t stream_id;
        int64_t n, r;
        int type, algo;
        void* data;
        size_t bytes;
        uint64_t last_use;
    };
    std::vector<OmegaEntry> omega_cache;
    size_t omega_cache_bytes = 0;
    uint64_t omega_tick = 0;
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
    return rpmi::OmegaTables{ctx->d_thresholds, ctx->d_guide, ctx->table_count, 0};
}

bool sparse_type(rp_omega_t type) {
    return type == RP_OMEGA_SPARSE1 || type == RP_OMEGA_SPARSE3 || type == RP_OMEGA_VSPARSE;
}

// Threshold of a sparse Omega with n rows: floor(2^64 / (2s)).
uint64_t sparse_threshold(rp_omega_t type, int64_t n) {
    if (type == RP_OMEGA_SPARSE1) return uint64_t(1) << 63;
    if (type == RP_OMEGA_SPARSE3) return ~uint64_t(0) / 6;   // floor((2^64 - 1) / 6) = floor(2^64 / 6)
    // s = sqrt(n): floor(2^63 / sqrt(n)) = isqrt(floor(2^126 / n))
    const unsigned __int128 q = ((unsigned __int128)1 << 126) / (unsigned __int128)(n > 0 ? n : 1);
    uint64_t x = (uint64_t)1 << 63;                           // isqrt(q) < 2^63 for q < 2^126
    if (q < ((unsigned __int128)1 << 126)) {
        // Newton from above, integer
        unsigned __int128 y = (unsigned __int128)1 << 63;
        while (true) {
            const unsigned __int128 z = (y + q / y) >> 1;
            if (z >= y) break;
            y = z;
        }
        x = (uint64_t)y;
    }
    return x;
}

// The generator tables for Omega of `type` with n rows.
rpmi::OmegaTables tables(rp_ctx ctx, rp_omega_t type, int64_t n) {
    rpmi::OmegaTables t = tables(ctx);
    if (sparse_type(type)) t.sparse_t = sparse_threshold(type, n);
    return t;
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
        case RP_ERR_OMEGA_RANGE: return "RP_ERR_OMEGA_RANGE";
    }
    return "unknown rp_status";
}

const char* rp_last_error(rp_ctx ctx) {
    return ctx ? ctx->last_error.c_str() : g_create_error.c_str();
}

namespace {

rp_status tuning_load(rp_ctx ctx, const char* path) {
    FILE* f = fopen(path, "r");
    if (!f) return fail(ctx, RP_ERR_INVALID_ARG, "cannot open tuning file %s", path);
    char line[256];
    int lineno = 0;
    rp_status st = RP_OK;
    while (fgets(line, sizeof line, f)) {
        ++lineno;
        unsigned long long key = 0;
        double scale = 0.0;
        int form = 0;
        char extra = 0;
        if (line[0] == '\n' || line[0] == '\0') continue;
        if (sscanf(line, "%llx %lf %d %c", &key, &scale, &form, &extra) != 3 || !(scale > 0.0) || scale > 64.0 ||
            form < 0 || form > 1) {
            st = fail(ctx, RP_ERR_INVALID_ARG, "tuning file %s line %d does not parse", path, lineno);
            break;
        }
        ctx->tuned_scale[(uint64_t)key] = rp_ctx_s::TuneEntry{scale, form};
    }
    fclose(f);
    return st;
}

rp_status tuning_save(rp_ctx ctx, const char* path) {
    FILE* f = fopen(path, "w");
    if (!f) return fail(ctx, RP_ERR_INVALID_ARG, "cannot write tuning file %s", path);
    for (const auto& e : ctx->tuned_scale)
        fprintf(f, "%016llx %.17g %d\n", (unsigned long long)e.first, e.second.scale, e.second.form);
    const bool ok = fclose(f) == 0;
    return ok ? RP_OK : fail(ctx, RP_ERR_INVALID_ARG, "writing tuning file %s failed", path);
}

}  // namespace

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
    if ((e = hipMalloc(&ctx->d_scan, sizeof(unsigned int))) != hipSuccess) return cleanup(e, "hipMalloc");
    if ((e = hipMemcpy(ctx->d_thresholds, thr.data(), n * sizeof(uint64_t), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMemcpy(ctx->d_guide, guide.data(), guide.size() * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess)
        return cleanup(e, "hipMemcpy");
    if ((e = hipMemset(ctx->d_status, 0, sizeof(unsigned int))) != hipSuccess) return cleanup(e, "hipMemset");
    if ((e = hipMalloc(&ctx->table, 64 * sizeof(rpmi::GroupEntry))) != hipSuccess) return cleanup(e, "hipMalloc");
    ctx->table_entries = 64;
    if ((e = hipMalloc(&ctx->fold_flags, rpmi::kFoldFlags * sizeof(unsigned int))) != hipSuccess)
        return cleanup(e, "hipMalloc");
    if ((e = hipMemset(ctx->fold_flags, 0, rpmi::kFoldFlags * sizeof(unsigned int))) != hipSuccess)
        return cleanup(e, "hipMemset");
    {
        void* p = nullptr;
        if ((e = rpmi::noalloc_scratch_address(&p)) != hipSuccess || !p)
            return cleanup(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        ctx->noalloc_scratch = static_cast<unsigned char*>(p);
    }
    if (const char* gs = getenv("RPMI_BATCHED_GRAPH_SWEEPS")) {
        char* end = nullptr;
        const long v = strtol(gs, &end, 10);
        if (end != gs && *end == '\0' && v >= 0 && v <= 1000) ctx->graph_sweeps = (int)v;
    }
    if (const char* ff = getenv("RPMI_GROUP_FORM")) {
        if (ff[0] == '0' && ff[1] == '\0') ctx->force_form = 0;
        if (ff[0] == '1' && ff[1] == '\0') ctx->force_form = 1;
    }
    if (const char* tf = getenv("RPMI_TUNING_FILE")) {
        if (tf[0]) {
            ctx->tuning_file = tf;
            (void)tuning_load(ctx, tf);
            ctx->last_error.clear();
        }
    }
    *out = ctx;
    return RP_OK;
}


rp_status rp_tuning_save(rp_ctx ctx, const char* path) {
    if (!ctx || !path) return fail(ctx, RP_ERR_INVALID_ARG, "ctx or path is NULL");
    return tuning_save(ctx, path);
}

rp_status rp_tuning_load(rp_ctx ctx, const char* path) {
    if (!ctx || !path) return fail(ctx, RP_ERR_INVALID_ARG, "ctx or path is NULL");
    return tuning_load(ctx, path);
}

rp_status rp_tuning_count(rp_ctx ctx, int64_t* entries) {
    if (!ctx || !entries) return fail(ctx, RP_ERR_INVALID_ARG, "ctx or entries is NULL");
    *entries = (int64_t)ctx->tuned_scale.size();
    return RP_OK;
}

rp_status rp_destroy(rp_ctx ctx) {
    if (!ctx) return RP_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->d_thresholds) (void)hipFree(ctx->d_thresholds);
    if (ctx->d_guide) (void)hipFree(ctx->d_guide);
    if (ctx->d_status) (void)hipFree(ctx->d_status);
    if (ctx->d_scan) (void)hipFree(ctx->d_scan);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->split_ws) (void)hipFree(ctx->split_ws);
    if (ctx->split_counters) (void)hipFree(ctx->split_counters);
    if (ctx->table) (void)hipFree(ctx->table);
    if (ctx->fold_flags) (void)hipFree(ctx->fold_flags);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph_exec2) (void)hipGraphExecDestroy(ctx->graph_exec2);
    if (ctx->d_jopen) (void)hipFree(ctx->d_jopen);
    if (ctx->graph_table) (void)hipFree(ctx->graph_table);
    if (ctx->graph_jtab) (void)hipFree(ctx->graph_jtab);
    if (ctx->graph_aux) (void)hipFree(ctx->graph_aux);
    for (auto& e : ctx->omega_cache) (void)hipFree(e.data);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return RP_OK;
}

rp_status rp_omega_generate(rp_ctx ctx, uint64_t seed, uint32_t stream_id, int64_t n, int64_t r,
                            rp_omega_t type, void* omega, int64_t ldo, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    if (n < 0 || r < 0) return fail(ctx, RP_ERR_INVALID_ARG, "negative size (n %lld, r %lld)", (long long)n, (long long)r);
    if (type == RP_OMEGA_E4M3)
        return fail(ctx, RP_ERR_INVALID_ARG, "the e4m3 Omega comes with column scales: use rp_omega_generate_e4m3");
    if (type != RP_OMEGA_F16 && type != RP_OMEGA_F32 && !sparse_type(type))
        return fail(ctx, RP_ERR_INVALID_ARG, "unknown omega type %d", (int)type);
    if (n == 0 || r == 0) return RP_OK;
    if (!omega) return fail(ctx, RP_ERR_INVALID_ARG, "omega is NULL");
    if (ldo < r) return fail(ctx, RP_ERR_INVALID_ARG, "ldo %lld < r %lld", (long long)ldo, (long long)r);
    RP_HIP(ctx, hipSetDevice(ctx->device));
    RP_HIP(ctx, rpmi::launch_omega_rowmajor(tables(ctx, type, n), seed, stream_id, n, r, type == RP_OMEGA_F32,
                                            omega, ldo, (hipStream_t)stream));
    return RP_OK;
}

rp_status rp_omega_generate_e4m3(rp_ctx ctx, uint64_t seed, uint32_t stream_id, int64_t n, int64_t r,
                                 uint8_t* omega, int64_t ldo, float* col_scale, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    if (n < 0 || r < 0) return fail(ctx, RP_ERR_INVALID_ARG, "negative size (n %lld, r %lld)", (long long)n, (long long)r);
    if (r == 0) return RP_OK;
    if (!col_scale || (n > 0 && !omega)) return fail(ctx, RP_ERR_INVALID_ARG, "NULL pointer");
    if (n > 0 && ldo < r) return fail(ctx, RP_ERR_INVALID_ARG, "ldo %lld < r %lld", (long long)ldo, (long long)r);
    RP_HIP(ctx, hipSetDevice(ctx->device));
    rp_status st;
    const size_t w_bytes = ((size_t)n * r * 4 + 255) & ~size_t(255);
    if ((st = ensure_workspace(ctx, w_bytes + (size_t)r * 4)) != RP_OK) return st;
    float* w32 = static_cast<float*>(ctx->ws);
    unsigned int* cmax = reinterpret_cast<unsigned int*>(static_cast<char*>(ctx->ws) + w_bytes);
    RP_HIP(ctx, rpmi::launch_omega_e4m3(tables(ctx), seed, stream_id, n, r, w32, cmax, omega, ldo, nullptr, 0, col_scale,
                                        (hipStream_t)stream));
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
    const int64_t col_block = algo == RP_ALGO_SPLIT_F16  ? rpmi::split_f16_col_block(r)
                            : algo == RP_ALGO_TCEC_F16 ? rpmi::tcec_col_block()
                                                       : rpmi::f32_col_block();
    pk.kb_count = round_up(n, rpmi::proj_k_block()) / rpmi::kKBlock;
    pk.nt_count = round_up(r, col_block) / rpmi::kNTile;
    pk.data = data;
    return pk;
}

size_t packed_bytes(const rpmi::PackedOmega& pk, rp_algo_t algo) {
    // FP16 fragments; FP32 fragments; TCEC: FP16 hi and lo fragments
    return (size_t)pk.kb_count * pk.nt_count * 64 * 8 * (algo == RP_ALGO_SPLIT_F16 ? 2 : 4);
}

bool enums_ok(rp_ctx ctx, rp_omega_t type, rp_algo_t algo, rp_status* st) {
    if (type != RP_OMEGA_F16 && type != RP_OMEGA_F32 && type != RP_OMEGA_E4M3 && !sparse_type(type)) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "unknown omega type %d", (int)type);
        return false;
    }
    if (algo != RP_ALGO_F32 && algo != RP_ALGO_SPLIT_F16 && algo != RP_ALGO_TCEC_F16) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "unknown algorithm %d", (int)algo);
        return false;
    }
    if (algo == RP_ALGO_SPLIT_F16 && type == RP_OMEGA_F32) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "the split-FP16 projection needs an FP16 or e4m3 Omega");
        return false;
    }
    if (algo == RP_ALGO_TCEC_F16 && type != RP_OMEGA_F32) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "the TCEC products need an FP32 Omega");
        return false;
    }
    return true;
}

// Scratch bytes fill_packed needs to generate Omega of `type` for `algo`.
size_t raw_bytes(rp_omega_t type, rp_algo_t algo, int64_t n, int64_t r) {
    if (type == RP_OMEGA_E4M3) return (size_t)n * r * 6 + (((size_t)r * 4 + 255) & ~size_t(255)) + 256;
    if (algo == RP_ALGO_F32) return (size_t)n * r * (type == RP_OMEGA_F32 ? 4 : 2);
    if (algo == RP_ALGO_TCEC_F16) return (size_t)n * r * 4;
    return 0;
}

// Fill `pk` (fragment order for `algo`) from a caller Omega or from the
// generator; `scratch` holds a row-major FP32/FP16 Omega when one has to be
// generated before widening (FP32 algorithm without a caller Omega).  A
// caller Omega packed for the split algorithm is checked for entries outside
// the single-accumulator range: `flag_bit` is set in *flag if one is found.
rp_status fill_packed(rp_ctx ctx, uint64_t seed, uint32_t stream_id, const void* omega, int64_t ldo,
                      const float* col_scale, rp_omega_t type, int64_t n, int64_t r, rp_algo_t algo,
                      const rpmi::PackedOmega& pk, void* scratch, hipStream_t s, unsigned int* flag = nullptr,
                      unsigned int flag_bit = 0) {
    const bool dst_f32 = algo == RP_ALGO_F32;
    if (algo == RP_ALGO_TCEC_F16) {
        // FP32 Omega (the caller's, or generated row-major into scratch), then
        // its hi and lo fragments; entries with |omega| >= 32 are reported
        const float* w = static_cast<const float*>(omega);
        int64_t ld = ldo;
        if (!w) {
            RP_HIP(ctx, rpmi::launch_omega_rowmajor(tables(ctx), seed, stream_id, n, r, true, scratch, r, s));
            w = static_cast<const float*>(scratch);
            ld = r;
        }
        RP_HIP(ctx, rpmi::launch_pack_omega_tcec(w, n, r, ld, pk, ctx->d_status, rpmi::kStatusOmegaRange, s));
        return RP_OK;
    }
    if (omega) {
        const rpmi::OmegaSrc src = type == RP_OMEGA_F32 ? rpmi::OmegaSrc::F32
                                 : type == RP_OMEGA_E4M3 ? rpmi::OmegaSrc::E4M3 : rpmi::OmegaSrc::F16;
        if (src == rpmi::OmegaSrc::E4M3 && !col_scale)
            return fail(ctx, RP_ERR_INVALID_ARG, "a caller e4m3 Omega needs its col_scale");
        RP_HIP(ctx, rpmi::launch_pack_omega(omega, src, col_scale, n, r, ldo, pk, dst_f32, dst_f32 ? nullptr : flag,
                                            flag_bit, ctx->d_status, s));
        return RP_OK;
    }
    if (type == RP_OMEGA_E4M3) {
        // FP32 Omega, column maxima, then the exact FP16 values Omega8 / s_j
        char* b = static_cast<char*>(scratch);
        float* w32 = reinterpret_cast<float*>(b);
        uint16_t* f16 = reinterpret_cast<uint16_t*>(b + (size_t)n * r * 4);
        unsigned int* cmax = reinterpret_cast<unsigned int*>(b + (((size_t)n * r * 6 + 255) & ~size_t(255)));
        RP_HIP(ctx, rpmi::launch_omega_e4m3(tables(ctx), seed, stream_id, n, r, w32, cmax, nullptr, 0, f16, r, nullptr,
                                            s));
        RP_HIP(ctx, rpmi::launch_pack_omega(f16, rpmi::OmegaSrc::F16, nullptr, n, r, r, pk, dst_f32, nullptr, 0, nullptr,
                                            s));
        return RP_OK;
    }
    if (algo == RP_ALGO_SPLIT_F16) {
        RP_HIP(ctx, rpmi::launch_omega_packed_f16(tables(ctx, type, n), seed, stream_id, n, r, pk, s));
        return RP_OK;
    }
    const bool src_f32 = type == RP_OMEGA_F32;
    RP_HIP(ctx, rpmi::launch_omega_rowmajor(tables(ctx, type, n), seed, stream_id, n, r, src_f32, scratch, r, s));
    RP_HIP(ctx, rpmi::launch_pack_omega(scratch, src_f32 ? rpmi::OmegaSrc::F32 : rpmi::OmegaSrc::F16, nullptr, n, r, r,
                                        pk, true, nullptr, 0, nullptr, s));
    return RP_OK;
}

// Generated Omega from the context cache (a1: Omega depends only on seed,
// stream, n, r and type, so repeated calls reuse the packed fragments).  On a
// miss the fragments are generated into a new cache allocation (scratch: the
// generator's row-major staging), evicting least recently used entries
// beyond kOmegaCacheBytes; the device is synchronised before any free.
// Returns RP_ERR_UNSUPPORTED (nothing done) for an Omega larger than the
// cache.
constexpr size_t kOmegaCacheBytes = size_t(1) << 30;

// keep_after: entries used after this tick (by the caller's current call,
// whose kernels may still read them) are never evicted; when the new Omega
// does not fit without them, RP_ERR_UNSUPPORTED (nothing done).
rp_status cached_packed_omega(rp_ctx ctx, uint64_t seed, uint32_t stream_id, rp_omega_t type, int64_t n, int64_t r,
                              rp_algo_t algo, void* scratch, hipStream_t s, rpmi::PackedOmega* pk,
                              uint64_t keep_after) {
    *pk = packed_geometry(n, r, algo, nullptr);
    const size_t bytes = packed_bytes(*pk, algo);
    for (auto& e : ctx->omega_cache)
        if (e.seed == seed && e.stream_id == stream_id && e.n == n && e.r == r && e.type == (int)type &&
            e.algo == (int)algo) {
            e.last_use = ++ctx->omega_tick;
            pk->data = e.data;
            return RP_OK;
        }
    if (bytes == 0 || bytes > kOmegaCacheBytes) return RP_ERR_UNSUPPORTED;
    if (ctx->omega_cache_bytes + bytes > kOmegaCacheBytes) {
        size_t evictable = 0;
        for (const auto& e : ctx->omega_cache)
            if (e.last_use <= keep_after) evictable += e.bytes;
        if (ctx->omega_cache_bytes - evictable + bytes > kOmegaCacheBytes) return RP_ERR_UNSUPPORTED;
        RP_HIP(ctx, hipDeviceSynchronize());
        while (ctx->omega_cache_bytes + bytes > kOmegaCacheBytes) {
            size_t lru = ctx->omega_cache.size();
            for (size_t i = 0; i < ctx->omega_cache.size(); ++i)
                if (ctx->omega_cache[i].last_use <= keep_after &&
                    (lru == ctx->omega_cache.size() || ctx->omega_cache[i].last_use < ctx->omega_cache[lru].last_use))
                    lru = i;
            if (lru == ctx->omega_cache.size()) return RP_ERR_UNSUPPORTED;   // not reached (checked above)
            RP_HIP(ctx, hipFree(ctx->omega_cache[lru].data));
            ctx->omega_cache_bytes -= ctx->omega_cache[lru].bytes;
            ctx->omega_cache.erase(ctx->omega_cache.begin() + lru);
        }
    }
    void* data = nullptr;
    RP_HIP(ctx, hipMalloc(&data, bytes));
    pk->data = data;
    rp_status st = fill_packed(ctx, seed, stream_id, nullptr, 0, nullptr, type, n, r, algo, *pk, scratch, s);
    if (st != RP_OK) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(data);
        return st;
    }
    ctx->omega_cache.push_back({seed, stream_id, n, r, (int)type, (int)algo, data, bytes, ++ctx->omega_tick});
    ctx->omega_cache_bytes += bytes;
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

// Split-K buffers supplied by a caller workspace instead of the context's.
struct SplitBuffers {
    unsigned int* counters;           // zero on entry, left zero
    float* partial;
    size_t counter_bytes, partial_bytes;
};

rpmi::ProjArgs proj_args(rp_ctx ctx, const rp_desc* A, int64_t r, const void* omega, int64_t nt_count, float* Y,
                         int64_t ldy, int32_t a_scale_exp) {
    rpmi::ProjArgs a;
    a.A = A->ptr; a.m = A->rows; a.n = A->cols;
    a.s_row = A->s_row;
    a.k_inner = A->k_inner;
    a.s_k_outer = A->s_k_outer;
    a.omega = omega; a.nt_count = nt_count;
    a.Y = Y; a.ldy = ldy; a.r = r;
    a.status = ctx->d_status;
    const int32_t se = a_scale_exp == RP_A_SCALE_AUTO_ROW ? 0 : a_scale_exp;
    a.a_scale = ldexpf(1.0f, se);
    a.y_scale = ldexpf(1.0f, -se);
    return a;
}

// auto_row: the entry point takes RP_A_SCALE_AUTO_ROW
bool scale_exp_ok(rp_ctx ctx, int32_t s, rp_status* st, bool auto_row = false) {
    if (s == RP_A_SCALE_AUTO_ROW) {
        if (auto_row) return true;
        *st = fail(ctx, RP_ERR_UNSUPPORTED, "RP_A_SCALE_AUTO_ROW is taken by rp_project and rsvd only");
        return false;
    }
    if (s < -64 || s > 64) {
        *st = fail(ctx, RP_ERR_INVALID_ARG, "a_scale_exp %d outside [-64, 64]", (int)s);
        return false;
    }
    return true;
}

// row_exp_ws: m ints of device workspace, needed with RP_A_SCALE_AUTO_ROW
rp_status launch_projection(rp_ctx ctx, const rp_desc* A, int64_t r, const rpmi::PackedOmega& pk,
                            rp_algo_t algo, float* Y, int64_t ldy, hipStream_t s, int32_t a_scale_exp = 0,
                            bool two_acc = false, const SplitBuffers* sb = nullptr, int* row_exp_ws = nullptr) {
    rpmi::ProjArgs a = proj_args(ctx, A, r, pk.data, pk.nt_count, Y, ldy, a_scale_exp);
    a.two_acc = two_acc;
    if (algo == RP_ALGO_SPLIT_F16 && a_scale_exp == RP_A_SCALE_AUTO_ROW) {
        // full exponent range: every row's own power of two, then the general
        // kernel (two accumulators)
        if (!row_exp_ws) return fail(ctx, RP_ERR_INVALID_ARG, "no workspace for the row exponents");
        RP_HIP(ctx, rpmi::launch_row_exponents(a, row_exp_ws, s));
        a.row_exp = row_exp_ws;
        RP_HIP(ctx, rpmi::launch_project_split_f16(a, s));
        return RP_OK;
    }
    if (algo == RP_ALGO_TCEC_F16) {
        a.a_scale = a.y_scale = 1.0f;
        if (!rpmi::split_fast_ok(a))
            return fail(ctx, RP_ERR_UNSUPPORTED, "the TCEC products need A on the 16-byte path (16-byte aligned, "
                                                 "row and run strides multiples of 4)");
        a.omega_lo = static_cast<const char*>(pk.data) + (size_t)pk.kb_count * pk.nt_count * 64 * 8 * 2;
        const rpmi::SplitPlan plan = rpmi::plan_tcec(a.m, a.n, r, ctx->num_cus > 0 ? ctx->num_cus : 256);
        if (plan.ksplit > 1) {   // partial sums only: the TCEC form adds them in a second kernel
            if (sb) {
                if (plan.partial_bytes > sb->partial_bytes)
                    return fail(ctx, RP_ERR_INVALID_ARG, "workspace too small for the contraction split");
                a.partial = sb->partial;
            } else {
                rp_status st = ensure_split_workspace(ctx, 0, plan.partial_bytes);
                if (st != RP_OK) return st;
                a.partial = static_cast<float*>(ctx->split_ws);
            }
            a.ksplit = plan.ksplit;
        }
        RP_HIP(ctx, rpmi::launch_project_tcec(a, s));
        return RP_OK;
    }
    if (algo == RP_ALGO_SPLIT_F16) {
        a.fold_flags = ctx->fold_flags;
        a.fold_epoch = ++ctx->fold_epoch;
        if (a.fold_epoch == 0) a.fold_epoch = ++ctx->fold_epoch;
        if (rpmi::split_fast_ok(a)) {
            const rpmi::SplitPlan plan = rpmi::plan_split_f16(a.m, a.n, r, ctx->num_cus > 0 ? ctx->num_cus : 256);
            if (plan.ksplit > 1) {
                if (sb) {
                    if (plan.counter_bytes > sb->counter_bytes || plan.partial_bytes > sb->partial_bytes)
                        return fail(ctx, RP_ERR_INVALID_ARG, "workspace too small for the contraction split");
                    a.counters = sb->counters;
                    a.partial = sb->partial;
                } else {
                    rp_status st = ensure_split_workspace(ctx, plan.counter_bytes, plan.partial_bytes);
                    if (st != RP_OK) return st;
                    a.counters = ctx->split_counters;
                    a.partial = static_cast<float*>(ctx->split_ws);
                }
                a.ksplit = plan.ksplit;
            }
        }
        RP_HIP(ctx, rpmi::launch_project_split_f16(a, s));
    } else {
        RP_HIP(ctx, rpmi::launch_project_f32(a, s));
    }
    return RP_OK;
}

// Grow the device table of grouped projections to `entries` (synchronises
// the device when it grows).
rp_status ensure_table(rp_ctx ctx, size_t entries) {
    if (entries <= ctx->table_entries) return RP_OK;
    RP_HIP(ctx, hipDeviceSynchronize());
    RP_HIP(ctx, hipFree(ctx->table));
    ctx->table = nullptr;
    ctx->table_entries = 0;
    const size_t n = (entries + 255) & ~size_t(255);
    RP_HIP(ctx, hipMalloc(&ctx->table, n * sizeof(rpmi::GroupEntry)));
    ctx->table_entries = n;
    return RP_OK;
}

// Plan a set of split-FP16 projections as at most four grouped launches:
// problems on the 16-byte path (split_fast_ok) go to the fast kernels, one
// launch per column width, each with its contraction split planned for its
// share of the compute units (in proportion to its A bytes, times
// `cu_scale`) and its split-K counters and partials laid out in the context
// buffers; the others go to the general kernel, one launch per column width,
// longest contraction first (each of its tiles runs the whole contraction).
// Table order: fast narrow, fast wide, then the general kernel's three
// column widths (128, 160, 256).
struct GroupPlan {
    struct Seg {
        int first = 0, count = 0;
        int64_t blocks = 0;
        int64_t rblocks = 0;   // reduction-pass blocks (LDS-staged launches)
    };
    std::vector<rpmi::GroupEntry> entries;
    Seg seg[5];   // fast narrow, fast wide, general r <= 128, r <= 160, r > 160
    bool narrow_lds = false;   // fast narrow problems on the LDS-staged kernel
};

rp_status plan_group(rp_ctx ctx, const std::vector<rpmi::ProjArgs>& probs, double cu_scale, GroupPlan* out,
                     bool narrow_lds = false) {
    std::vector<int> fast, general;
    double total = 0;
    for (size_t g = 0; g < probs.size(); ++g) {
        if (rpmi::split_fast_ok(probs[g])) {
            fast.push_back((int)g);
            total += (double)probs[g].m * probs[g].n;
        } else {
            general.push_back((int)g);
        }
    }
    std::stable_sort(general.begin(), general.end(),
                     [&](int x, int y) { return probs[x].n > probs[y].n; });
    const int cus = ctx->num_cus > 0 ? ctx->num_cus : 256;
    std::vector<rpmi::SplitPlan> plans(probs.size(), rpmi::SplitPlan{1, 0, 0});
    size_t counter_bytes = 0, partial_bytes = 0;
    for (int g : fast) {
        const auto& a = probs[g];
        const int share = (int)(cus * cu_scale * ((double)a.m * a.n / total) + 0.5);
        plans[g] = narrow_lds && a.r <= 128 ? rpmi::plan_split_f16_narrow_lds(a.m, a.n, a.r, share > 0 ? share : 1)
                                             : rpmi::plan_split_f16(a.m, a.n, a.r, share > 0 ? share : 1);
        counter_bytes += (plans[g].counter_bytes + 255) & ~size_t(255);
        partial_bytes += (plans[g].partial_bytes + 255) & ~size_t(255);
    }
    if (!fast.empty()) {
        rp_status st = ensure_split_workspace(ctx, counter_bytes, partial_bytes);
        if (st != RP_OK) return st;
    }
    char* cbase = reinterpret_cast<char*>(ctx->split_counters);
    char* pbase = static_cast<char*>(ctx->split_ws);
    out->entries.clear();
    out->narrow_lds = narrow_lds;
    for (int sg = 0; sg < 5; ++sg) {
        const bool gen = sg >= 2, narrow = sg == 0;
        GroupPlan::Seg& seg = out->seg[sg];
        seg.first = (int)out->entries.size();
        int64_t start = 0, rstart = 0;
        const bool lds = sg == 1 || (sg == 0 && narrow_lds);
        for (int g : gen ? general : fast) {
            if (gen ? rpmi::split_general_width_class(probs[g].r) != sg - 2 : (probs[g].r <= 128) != narrow) continue;
            rpmi::GroupEntry e;
            e.p = probs[g];
            int64_t bm, bn;
            if (gen) {
                e.p.ksplit = 1;
                e.p.counters = nullptr;
                e.p.partial = nullptr;
                e.p.fold_flags = nullptr;
                bm = rpmi::split_general_tile_m(e.p.r);
                bn = rpmi::split_general_tile_n(e.p.r);
            } else {
                e.p.ksplit = plans[g].ksplit;
                e.p.counters = e.p.ksplit > 1 ? reinterpret_cast<unsigned int*>(cbase) : nullptr;
                e.p.partial = e.p.ksplit > 1 ? reinterpret_cast<float*>(pbase) : nullptr;
                cbase += (plans[g].counter_bytes + 255) & ~size_t(255);
                pbase += (plans[g].partial_bytes + 255) & ~size_t(255);
                bm = narrow && narrow_lds ? rpmi::split_group_tile_m_narrow_lds() : rpmi::split_group_tile_m(e.p.r);
                bn = rpmi::split_group_tile_n(e.p.r);
            }
            e.tiles_m = (e.p.m + bm - 1) / bm;
            e.tiles_n = (e.p.r + bn - 1) / bn;
            e.start = start;
            start += e.tiles_m * e.tiles_n * e.p.ksplit;
            e.rstart = rstart;
            if (lds && e.p.ksplit > 1) rstart += rpmi::split_group_reduce_blocks(e.tiles_m * e.tiles_n, sg == 0);
            out->entries.push_back(e);
        }
        seg.count = (int)out->entries.size() - seg.first;
        seg.blocks = start;
        seg.rblocks = rstart;
    }
    return RP_OK;
}

// Launch a planned group whose table is already on the device.
rp_status launch_group_kernels(rp_ctx ctx, const GroupPlan& gp, const rpmi::GroupEntry* table, hipStream_t s) {
    for (int sg = 0; sg < 5; ++sg) {
        const GroupPlan::Seg& seg = gp.seg[sg];
        if (seg.count == 0) continue;
        if (sg == 0 && gp.narrow_lds)
            RP_HIP(ctx, rpmi::launch_split_group_narrow_lds(table + seg.first, seg.count, seg.blocks, seg.rblocks, s));
        else if (sg < 2)
            RP_HIP(ctx, rpmi::launch_project_split_f16_grouped(table + seg.first, seg.count, seg.blocks, sg == 0, s,
                                                               nullptr, seg.rblocks));
        else
            RP_HIP(ctx, rpmi::launch_project_split_f16_general_grouped(table + seg.first, seg.count, seg.blocks,
                                                                       sg - 2, s));
    }
    return RP_OK;
}

// Write a planned group to `table` (device, stream-ordered) and launch it.
rp_status launch_group(rp_ctx ctx, const GroupPlan& gp, rpmi::GroupEntry* table, hipStream_t s) {
    if (gp.entries.empty()) return RP_OK;
    RP_HIP(ctx, hipMemcpyAsync(table, gp.entries.data(), gp.entries.size() * sizeof(rpmi::GroupEntry),
                               hipMemcpyHostToDevice, s));
    return launch_group_kernels(ctx, gp, table, s);
}

uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h;
}

// Autotuner of the grouped launches: time the launch of `probs` on `s` at
// every candidate (contraction-split scale x narrow kernel form; the form
// only where a narrow problem is on the 16-byte path) and keep the fastest
// under `sig` (each trial writes the problems' outputs).
rp_status tune_group(rp_ctx ctx, const std::vector<rpmi::ProjArgs>& probs, uint64_t sig, hipStream_t s,
                     rp_ctx_s::TuneEntry* out) {
    bool any_narrow = false;
    for (const auto& a : probs) any_narrow = any_narrow || (a.r <= 128 && rpmi::split_fast_ok(a));
    rp_status st;
    GroupPlan gp;
    hipEvent_t e0, e1;
    RP_HIP(ctx, hipEventCreate(&e0));
    RP_HIP(ctx, hipEventCreate(&e1));
    float best_ms = 1e30f;
    const int f0 = ctx->force_form >= 0 ? ctx->force_form : 0;
    const int f1 = ctx->force_form >= 0 ? ctx->force_form : (any_narrow ? 1 : 0);
    *out = rp_ctx_s::TuneEntry{1.0, f0};
    for (int form = f0; form <= f1; ++form)
        for (double scale : {0.5, 1.0, 2.0, 4.0}) {
            if ((st = plan_group(ctx, probs, scale, &gp, form == 1)) != RP_OK) return st;
            if ((st = ensure_table(ctx, gp.entries.size())) != RP_OK) return st;
            if ((st = launch_group(ctx, gp, ctx->table, s)) != RP_OK) return st;   // warm-up
            RP_HIP(ctx, hipEventRecord(e0, s));
            for (int rep = 0; rep < 3; ++rep)
                if ((st = launch_group(ctx, gp, ctx->table, s)) != RP_OK) return st;
            RP_HIP(ctx, hipEventRecord(e1, s));
            RP_HIP(ctx, hipEventSynchronize(e1));
            float ms = 0;
            RP_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
            if (ms < best_ms) {
                best_ms = ms;
                *out = rp_ctx_s::TuneEntry{scale, form};
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->tuned_scale[sig] = *out;
    if (!ctx->tuning_file.empty()) (void)tuning_save(ctx, ctx->tuning_file.c_str());
    return RP_OK;
}

// The plan of a grouped launch with the autotuner's choice for this problem
// set (shapes and layouts), tuned now on a miss.  A stream under graph
// capture takes scale 1 and the register-staged form untimed.
rp_status tuned_group_plan(rp_ctx ctx, const std::vector<rpmi::ProjArgs>& probs, hipStream_t s, GroupPlan* gp) {
    uint64_t sig = mix(mix(0x67726f7570ull, (uint64_t)probs.size()), (uint64_t)ctx->num_cus);
    bool any_fast = false;
    for (const auto& a : probs) {
        sig = mix(mix(mix(mix(sig, (uint64_t)a.m), (uint64_t)a.n), (uint64_t)a.r), (uint64_t)a.s_row);
        sig = mix(mix(mix(sig, (uint64_t)a.k_inner), (uint64_t)a.s_k_outer), (uint64_t)rpmi::split_fast_ok(a));
        any_fast = any_fast || rpmi::split_fast_ok(a);
    }
    rp_ctx_s::TuneEntry best{1.0, 0};
    auto it = ctx->tuned_scale.find(sig);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    RP_HIP(ctx, hipStreamIsCapturing(s, &cap));
    if (it != ctx->tuned_scale.end()) {
        best = it->second;
    } else if (any_fast && cap == hipStreamCaptureStatusNone) {
        rp_status st = tune_group(ctx, probs, sig, s, &best);
        if (st != RP_OK) return st;
    }
    if (ctx->force_form >= 0) best.form = ctx->force_form;
    return plan_group(ctx, probs, best.scale, gp, best.form == 1);
}

// Several split-FP16 projections in grouped launches.  Returns
// RP_ERR_UNSUPPORTED (nothing launched) when a problem is empty; the caller
// then launches them one by one.
rp_status launch_projection_grouped(rp_ctx ctx, int count, const rp_desc* const* A, const int64_t* r,
                                    const rpmi::PackedOmega* pk, float* const* Y, const int64_t* ldy,
                                    hipStream_t s) {
    if (count <= 0) return RP_ERR_UNSUPPORTED;
    std::vector<rpmi::ProjArgs> probs(count);
    for (int g = 0; g < count; ++g) {
        if (A[g]->rows == 0 || A[g]->cols == 0 || r[g] == 0) return RP_ERR_UNSUPPORTED;
        probs[g] = proj_args(ctx, A[g], r[g], pk[g].data, pk[g].nt_count, Y[g], ldy[g], 0);
    }
    GroupPlan gp;
    rp_status st = tuned_group_plan(ctx, probs, s, &gp);
    if (st != RP_OK) return st;
    if ((st = ensure_table(ctx, gp.entries.size())) != RP_OK) return st;
    return launch_group(ctx, gp, ctx->table, s);
}

}  // namespace

extern "C" {

rp_status rp_omega_packed_size(int64_t n, int64_t r, rp_algo_t algo, size_t* bytes) {
    if (!bytes || n < 0 || r < 0 || (algo != RP_ALGO_F32 && algo != RP_ALGO_SPLIT_F16 && algo != RP_ALGO_TCEC_F16))
        return fail(nullptr, RP_ERR_INVALID_ARG, "invalid arguments to rp_omega_packed_size");
    *bytes = packed_bytes(packed_geometry(n, r, algo, nullptr), algo);
    return RP_OK;
}

rp_status rp_omega_pack(rp_ctx ctx, uint64_t seed, uint32_t stream_id, const void* omega,
                        int64_t ldo, const float* col_scale, rp_omega_t type, int64_t n, int64_t r,
                        rp_algo_t algo, void* packed, void* stream) {
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
    if (!omega && raw_bytes(type, algo, n, r) > 0) {
        if ((st = ensure_workspace(ctx, raw_bytes(type, algo, n, r))) != RP_OK) return st;
        scratch = ctx->ws;
    }
    return fill_packed(ctx, seed, stream_id, omega, ldo, col_scale, type, n, r, algo, pk, scratch,
                       (hipStream_t)stream, ctx->d_status, rpmi::kStatusOmegaRange);
}

rp_status rp_project_packed(rp_ctx ctx, const rp_desc* A, int64_t r, const void* packed,
                            rp_algo_t algo, int32_t a_scale_exp, float* Y, int64_t ldy, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    rp_status st;
    if (!desc_ok(ctx, A, &st)) return st;
    if (algo != RP_ALGO_F32 && algo != RP_ALGO_SPLIT_F16 && algo != RP_ALGO_TCEC_F16)
        return fail(ctx, RP_ERR_INVALID_ARG, "unknown algorithm %d", (int)algo);
    if (!scale_exp_ok(ctx, a_scale_exp, &st)) return st;
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
    return launch_projection(ctx, A, r, packed_geometry(n, r, algo, const_cast<void*>(packed)), algo, Y, ldy, s,
                             algo == RP_ALGO_SPLIT_F16 ? a_scale_exp : 0);
}

rp_status rp_project_packed_noalloc(rp_ctx ctx, const rp_desc* A, int64_t r, const void* packed,
                                    rp_algo_t algo, int32_t a_scale_exp, float* Y, int64_t ldy, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    rp_status st;
    if (!desc_ok(ctx, A, &st)) return st;
    if (algo != RP_ALGO_F32 && algo != RP_ALGO_SPLIT_F16)
        return fail(ctx, RP_ERR_INVALID_ARG, "unknown algorithm %d", (int)algo);
    if (!scale_exp_ok(ctx, a_scale_exp, &st)) return st;
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
    SplitBuffers sb{reinterpret_cast<unsigned int*>(ctx->noalloc_scratch + rpmi::kNoAllocPartialBytes),
                    reinterpret_cast<float*>(ctx->noalloc_scratch), rpmi::kNoAllocCounterBytes,
                    rpmi::kNoAllocPartialBytes};
    if (algo == RP_ALGO_SPLIT_F16) {
        const rpmi::SplitPlan plan = rpmi::plan_split_f16(m, n, r, ctx->num_cus > 0 ? ctx->num_cus : 256);
        if (plan.ksplit > 1) {
            if (plan.partial_bytes > sb.partial_bytes || plan.counter_bytes > sb.counter_bytes)
                return fail(ctx, RP_ERR_INVALID_ARG,
                            "the contraction split of this shape needs %zu bytes of partial sums and %zu of "
                            "counters; the no-allocation scratch holds %zu and %zu",
                            plan.partial_bytes, plan.counter_bytes, sb.partial_bytes, sb.counter_bytes);
            // the counters must start at zero: cleared by a kernel (not a
            // memset node) so the call can be captured into a graph
            RP_HIP(ctx, rpmi::launch_fill_u32(sb.counters, (int64_t)(plan.counter_bytes / sizeof(unsigned int)), 0u,
                                              s));
        }
    }
    return launch_projection(ctx, A, r, packed_geometry(n, r, algo, const_cast<void*>(packed)), algo, Y, ldy, s,
                             algo == RP_ALGO_SPLIT_F16 ? a_scale_exp : 0, false, &sb);
}

rp_status rp_project(rp_ctx ctx, const rp_desc* A, int64_t r, rp_omega_t omega_type, uint64_t seed,
                     uint32_t stream_id, const void* omega, int64_t ldo, const float* col_scale, rp_algo_t algo,
                     int32_t a_scale_exp, float* Y, int64_t ldy, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    rp_status st;
    if (!desc_ok(ctx, A, &st)) return st;
    if (r < 0) return fail(ctx, RP_ERR_INVALID_ARG, "negative r %lld", (long long)r);
    if (!enums_ok(ctx, omega_type, algo, &st)) return st;
    if (!scale_exp_ok(ctx, a_scale_exp, &st, true)) return st;
    const int64_t m = A->rows, n = A->cols;
    if (m == 0 || r == 0) return RP_OK;
    if (!Y) return fail(ctx, RP_ERR_INVALID_ARG, "Y is NULL");
    if (ldy < r) return fail(ctx, RP_ERR_INVALID_ARG, "ldy %lld < r %lld", (long long)ldy, (long long)r);
    if (omega && ldo < r) return fail(ctx, RP_ERR_INVALID_ARG, "ldo %lld < r %lld", (long long)ldo, (long long)r);
    if (omega && omega_type == RP_OMEGA_E4M3 && !col_scale)
        return fail(ctx, RP_ERR_INVALID_ARG, "a caller e4m3 Omega needs its col_scale");
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipSetDevice(ctx->device));
    if (n == 0) {
        RP_HIP(ctx, rpmi::launch_fill_f32(Y, m, r, ldy, 0.0f, s));
        return RP_OK;
    }
    if (!proj_layout_ok(ctx, A, &st)) return st;
    rpmi::PackedOmega pk = packed_geometry(n, r, algo, nullptr);
    const size_t pbytes = packed_bytes(pk, algo);
    const size_t raw_off = (pbytes + 255) & ~size_t(255);
    const size_t rb = omega ? 0 : raw_bytes(omega_type, algo, n, r);
    const size_t rx_off = (raw_off + rb + 255) & ~size_t(255);
    const size_t rxb = a_scale_exp == RP_A_SCALE_AUTO_ROW ? (size_t)m * sizeof(int) : 0;
    if ((st = ensure_workspace(ctx, rx_off + rxb)) != RP_OK) return st;
    pk.data = ctx->ws;
    void* raw = static_cast<char*>(ctx->ws) + raw_off;
    int* row_exp = rxb ? reinterpret_cast<int*>(static_cast<char*>(ctx->ws) + rx_off) : nullptr;
    // a caller Omega for the split kernels is scanned; entries the single
    // accumulator cannot take route the call to the two-accumulator kernel
    const bool scan = omega && algo == RP_ALGO_SPLIT_F16;
    if (scan) RP_HIP(ctx, rpmi::launch_fill_u32(ctx->d_scan, 1, 0u, s));
    if ((st = fill_packed(ctx, seed, stream_id, omega, ldo, col_scale, omega_type, n, r, algo, pk, raw, s,
                          scan ? ctx->d_scan : nullptr, 1u)) != RP_OK)
        return st;
    bool two_acc = false;
    if (scan) {
        unsigned int word = 0;
        RP_HIP(ctx, hipMemcpyAsync(&word, ctx->d_scan, sizeof word, hipMemcpyDeviceToHost, s));
        RP_HIP(ctx, hipStreamSynchronize(s));
        two_acc = word != 0;
    }
    return launch_projection(ctx, A, r, pk, algo, Y, ldy, s, algo == RP_ALGO_SPLIT_F16 ? a_scale_exp : 0, two_acc,
                             nullptr, row_exp);
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
// each), L1 (p x p FP64, kept only when M is requested) and GP (split Gram
// partials, kGramSplit p x p FP64).
rp_status cholqr2(rp_ctx ctx, int64_t m, int64_t p, const float* Y, int64_t ldy, float* Q, int64_t ldq,
                  double* M, double* Qd, double* G, double* X, double* L1, double* GP, hipStream_t s) {
    unsigned int* st = ctx->d_status;
    // pass 1: G = Y^T Y, G = L L^T, X = L^-1, Qd = Y X^T  (= Y R^-1)
    RP_HIP(ctx, rpmi::gram_acc64<float>(p, m, Y, ldy, G, GP, rpmi::kGramSplit, s));
    RP_HIP(ctx, rpmi::potrf_lower(G, p, p, st, s));
    RP_HIP(ctx, rpmi::trtri_lower(G, p, X, p, p, s));
    RP_HIP(ctx, (rpmi::gemm_acc64<float, double, double>(m, p, p, 1.0, Y, ldy, 1, X, 1, p, 0.0, Qd, p, 1, s)));
    if (M) RP_HIP(ctx, hipMemcpyAsync(L1, G, (size_t)p * p * sizeof(double), hipMemcpyDeviceToDevice, s));
    // pass 2 on Qd
    RP_HIP(ctx, rpmi::gram_acc64<double>(p, m, Qd, p, G, GP, rpmi::kGramSplit, s));
    RP_HIP(ctx, rpmi::potrf_lower(G, p, p, st, s));
    RP_HIP(ctx, rpmi::trtri_lower(G, p, X, p, p, s));
    RP_HIP(ctx, (rpmi::gemm_acc64<double, double, float>(m, p, p, 1.0, Qd, p, 1, X, 1, p, 0.0, Q, ldq, 1, s)));
    if (M) RP_HIP(ctx, (rpmi::gemm_acc64<double, double, double>(p, p, p, 1.0, L1, p, 1, G, p, 1, 0.0, M, p, 1, s)));
    return RP_OK;
}

// Scratch of one RSVD after its projection (sized for m x n, rank k, p
// columns): Q, Z, W, the FP64 CholeskyQR2 and Jacobi buffers, and W in FP32
// fragment order for the power scheme's projections.
struct RsvdScratch {
    int64_t m = 0, n = 0, k = 0, p = 0;
    size_t o_q, o_z, o_w, o_qd, o_g, o_x, o_l1, o_gp, o_mw, o_mv, o_sig, o_ord, o_ur, o_vr, o_pkw, o_pkq, o_jt, o_jf,
        o_rx, bytes;
    float *Q, *Z, *W;
    double *Qd, *G, *X, *L1, *GP, *MW, *MV, *sig, *Ur, *Vr;
    int* ord;
    int* jflags;                       // Jacobi flags (4 ints)
    int* rowx;                         // row exponents of the automatic pre-scale (m ints)
    bool tcec_aw = false;              // power scheme's A W on the TCEC products (pkw in TCEC form)
    bool tcec_atq = false;             // A^T Q on the TCEC products (Q packed into pkq)
    const SplitBuffers* aw_sb = nullptr;   // contraction-split buffers for A W (else the context's)
    rpmi::JacobiProb* jtab;            // a one-entry Jacobi table (device)
    rpmi::PackedOmega pkw;
    rpmi::PackedOmega pkq;             // Q (m x p) in TCEC fragment form, for A^T Q

    // reserve the scratch in `ar` (one block); returns its offset
    size_t layout(Arena& outer, int64_t m_, int64_t n_, int64_t k_, int64_t p_, bool tcec_room = true) {
        m = m_; n = n_; k = k_; p = p_;
        Arena ar;
        const int64_t mx = m > n ? m : n;
        o_q = ar.take((size_t)m * p * 4);
        o_z = ar.take((size_t)n * p * 4);
        o_w = ar.take((size_t)n * p * 4);
        o_qd = ar.take((size_t)mx * p * 8);
        o_g = ar.take((size_t)p * p * 8);
        o_x = ar.take((size_t)p * p * 8);
        o_l1 = ar.take((size_t)p * p * 8);
        o_gp = ar.take((size_t)rpmi::kGramSplit * p * p * 8);
        o_mw = ar.take((size_t)p * p * 8);
        o_mv = ar.take((size_t)p * p * 8);
        o_sig = ar.take((size_t)p * 8);
        o_ord = ar.take((size_t)p * 4);
        o_ur = ar.take((size_t)p * k * 8);
        o_vr = ar.take((size_t)p * k * 8);
        pkw = packed_geometry(n, p, RP_ALGO_F32, nullptr);
        o_pkw = ar.take(packed_bytes(pkw, RP_ALGO_F32));
        pkq = packed_geometry(m, p, RP_ALGO_TCEC_F16, nullptr);
        o_pkq = ar.take(tcec_room ? packed_bytes(pkq, RP_ALGO_TCEC_F16) : 0);
        o_jt = ar.take(sizeof(rpmi::JacobiProb));
        o_jf = ar.take(4 * sizeof(int));
        o_rx = ar.take((size_t)m * sizeof(int));
        bytes = ar.used;
        return outer.take(bytes);
    }
    void bind(char* b) {
        Q = reinterpret_cast<float*>(b + o_q);
        Z = reinterpret_cast<float*>(b + o_z);
        W = reinterpret_cast<float*>(b + o_w);
        Qd = reinterpret_cast<double*>(b + o_qd);
        G = reinterpret_cast<double*>(b + o_g);
        X = reinterpret_cast<double*>(b + o_x);
        L1 = reinterpret_cast<double*>(b + o_l1);
        GP = reinterpret_cast<double*>(b + o_gp);
        MW = reinterpret_cast<double*>(b + o_mw);
        MV = reinterpret_cast<double*>(b + o_mv);
        sig = reinterpret_cast<double*>(b + o_sig);
        ord = reinterpret_cast<int*>(b + o_ord);
        Ur = reinterpret_cast<double*>(b + o_ur);
        Vr = reinterpret_cast<double*>(b + o_vr);
        pkw.data = b + o_pkw;
        pkq.data = b + o_pkq;
        jtab = reinterpret_cast<rpmi::JacobiProb*>(b + o_jt);
        jflags = reinterpret_cast<int*>(b + o_jf);
        rowx = reinterpret_cast<int*>(b + o_rx);
    }
};

constexpr int kJacobiSweeps = 16;
constexpr double kJacobiTol = 1e-14;
// Jacobi sweeps recorded in the batched call's first graph; the batched
// problems have converged within them (9 sweeps on 256 problems of width 26
// to 160), and any further sweep up to the bound runs eagerly, only while a
// problem is open
constexpr int kBatchedGraphSweeps = 10;

rp_status rsvd_check(rp_ctx ctx, const rp_rsvd_problem& q, int32_t power_iters) {
    const int64_t p = q.k + q.oversample;
    if (q.m <= 0 || q.n <= 0 || q.k <= 0 || q.oversample < 0 || power_iters < 0)
        return fail(ctx, RP_ERR_INVALID_ARG, "invalid sizes (m %lld, n %lld, k %lld, s %lld, q %d)", (long long)q.m,
                    (long long)q.n, (long long)q.k, (long long)q.oversample, (int)power_iters);
    if (p > q.m || p > q.n || p > 1024)
        return fail(ctx, RP_ERR_INVALID_ARG, "k + oversample = %lld must be <= min(m, n) and <= 1024", (long long)p);
    if (!q.A || !q.U || !q.S || !q.VT) return fail(ctx, RP_ERR_INVALID_ARG, "NULL pointer");
    if (q.lda < q.n || q.ldu < q.k || q.ldvt < q.n) return fail(ctx, RP_ERR_INVALID_ARG, "leading dimension too small");
    const rp_desc dA{q.A, q.m, q.n, q.lda, q.n, 1, 0};
    rp_status st;
    if (!proj_layout_ok(ctx, &dA, &st)) return st;
    return RP_OK;
}

// Algorithm 1 after Y = A Omega, up to the small SVD: the power scheme
// (re-orthonormalised), then Q = QR(Y), B^T = A^T Q, B^T = Q_B R_B with R_B^T
// left in w.MW.  Launches kernels only (capturable in a graph).
// Z = A^T Q (n x p, row-major) for A (m x n, lda) and Q (m x p).
// With `pkq` (TCEC form, m x p) the product takes the TCEC kernel (eq:tcec-5,
// Q packed first), else the FP32 matrix-core kernel.  `report_q` records an
// entry |q| >= 32 as RP_ERR_OMEGA_RANGE (a caller's Q; the algorithms' own
// orthonormal Q is inside the range unless A already was not finite, which
// its own report covers).
rp_status gemm_at_q(rp_ctx ctx, int64_t m, int64_t n, int64_t p, const float* A, int64_t lda, const float* Q,
                    int64_t ldq, float* Z, int64_t ldz, const rpmi::PackedOmega* pkq, hipStream_t s,
                    bool report_q = false) {
    if (!pkq) {
        RP_HIP(ctx, rpmi::gemm_tn_f32(n, p, m, A, lda, Q, ldq, Z, ldz, s));
        return RP_OK;
    }
    RP_HIP(ctx, rpmi::launch_pack_omega_tcec(Q, m, p, ldq, *pkq, report_q ? ctx->d_status : nullptr,
                                             rpmi::kStatusOmegaRange, s));
    rpmi::TnTcecArgs t;
    t.A = A; t.lda = lda; t.m = m; t.n = n; t.p = p;
    t.qhi = pkq->data;
    t.qlo = static_cast<const char*>(pkq->data) + (size_t)pkq->kb_count * pkq->nt_count * 64 * 8 * 2;
    t.nt_count = pkq->nt_count;
    t.Z = Z; t.ldz = ldz;
    t.status = ctx->d_status;
    RP_HIP(ctx, rpmi::launch_gemm_tn_tcec(t, s));
    return RP_OK;
}

rp_status rsvd_before_svd(rp_ctx ctx, const rp_desc& dA, const rp_rsvd_problem& q, int64_t p, int32_t power_iters,
                          float* Y, const RsvdScratch& w, hipStream_t s) {
    rp_status st;
    const int64_t m = q.m, n = q.n, lda = q.lda;
    const float* A = q.A;
    for (int32_t t = 0; t < power_iters; ++t) {
        if ((st = cholqr2(ctx, m, p, Y, p, w.Q, p, nullptr, w.Qd, w.G, w.X, w.L1, w.GP, s)) != RP_OK) return st;
        // Z = A^T Q (n x p)
        if ((st = gemm_at_q(ctx, m, n, p, A, lda, w.Q, p, w.Z, p, w.tcec_atq ? &w.pkq : nullptr, s)) != RP_OK)
            return st;
        if ((st = cholqr2(ctx, n, p, w.Z, p, w.W, p, nullptr, w.Qd, w.G, w.X, w.L1, w.GP, s)) != RP_OK) return st;
        // Y = A W (FP32 x FP32, W not random): the TCEC products (eq:tcec-5) or
        // the FP32 projection kernel, with W in fragment order (|w| <= 1: W
        // has orthonormal columns)
        if (w.tcec_aw) {
            RP_HIP(ctx, rpmi::launch_pack_omega_tcec(w.W, n, p, p, w.pkw, nullptr, 0, s));
            if ((st = launch_projection(ctx, &dA, p, w.pkw, RP_ALGO_TCEC_F16, Y, p, s, 0, false, w.aw_sb)) != RP_OK)
                return st;
        } else {
            RP_HIP(ctx, rpmi::launch_pack_omega(w.W, rpmi::OmegaSrc::F32, nullptr, n, p, p, w.pkw, true, nullptr, 0,
                                                nullptr, s));
            if ((st = launch_projection(ctx, &dA, p, w.pkw, RP_ALGO_F32, Y, p, s)) != RP_OK) return st;
        }
    }
    // Algorithm 1 line 2: Q = QR(Y)
    if ((st = cholqr2(ctx, m, p, Y, p, w.Q, p, nullptr, w.Qd, w.G, w.X, w.L1, w.GP, s)) != RP_OK) return st;
    // line 3: B^T = A^T Q (n x p)
    if ((st = gemm_at_q(ctx, m, n, p, A, lda, w.Q, p, w.Z, p, w.tcec_atq ? &w.pkq : nullptr, s)) != RP_OK) return st;
    // line 4: B^T = Q_B R_B; R_B^T = L1 L2 (p x p lower) into MW
    return cholqr2(ctx, n, p, w.Z, p, w.W, p, w.MW, w.Qd, w.G, w.X, w.L1, w.GP, s);
}

// After the Jacobi SVD of R_B^T = U_r S V_r^T (so B = U_r S (Q_B V_r)^T):
// S, U = Q U_r[:, :k] and V^T = (Q_B V_r[:, :k])^T.
rp_status rsvd_after_svd(rp_ctx ctx, const rp_rsvd_problem& q, int64_t p, const RsvdScratch& w, hipStream_t s) {
    const int64_t m = q.m, n = q.n, k = q.k;
    RP_HIP(ctx, rpmi::svd_finish(w.MW, w.MV, (int)p, (int)k, w.sig, w.ord, w.Ur, w.Vr, s));
    RP_HIP(ctx, hipMemcpyAsync(q.S, w.sig, (size_t)k * sizeof(double), hipMemcpyDeviceToDevice, s));
    // Algorithm 1 line 5 in FP32 (U_r, V_r rounded to FP32)
    RP_HIP(ctx, (rpmi::gemm_f32<float, double, float>(m, k, p, 1.0, w.Q, p, 1, w.Ur, k, 1, 0.0, q.U, q.ldu, 1, s)));
    RP_HIP(ctx, (rpmi::gemm_f32<float, double, float>(n, k, p, 1.0, w.W, p, 1, w.Vr, k, 1, 0.0, q.VT, 1, q.ldvt, s)));
    return RP_OK;
}

// The whole of Algorithm 1 after the projection, for one problem.
rp_status rsvd_after_projection(rp_ctx ctx, const rp_desc& dA, const rp_rsvd_problem& q, int64_t p,
                                int32_t power_iters, float* Y, const RsvdScratch& w, hipStream_t s) {
    rp_status st;
    if ((st = rsvd_before_svd(ctx, dA, q, p, power_iters, Y, w, s)) != RP_OK) return st;
    RP_HIP(ctx, rpmi::launch_set_jacobi_prob(w.jtab, rpmi::JacobiProb{w.MW, w.MV, (int)p, 0, w.jflags, 0}, s));
    // outside graph capture the sweeps stop at convergence (the host polls the
    // converged flag once per sweep); under capture all sweeps are recorded and
    // a converged problem's kernels return at once
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    RP_HIP(ctx, hipStreamIsCapturing(s, &cap));
    RP_HIP(ctx, rpmi::jacobi_svd_group(w.jtab, 1, (int)((p + 1) / 2), rpmi::jacobi_block_pairs((int)p), (int)p,
                                       kJacobiSweeps, kJacobiTol,
                                       ctx->d_status, s, cap == hipStreamCaptureStatusNone ? w.jflags : nullptr));
    return rsvd_after_svd(ctx, q, p, w, s);
}

// Workspace layout of one rsvd() call: packed Omega, generator scratch, Y,
// the per-problem scratch and the split-K counters and partials of the
// projection, all in one 256-byte aligned block.
struct RsvdPlan {
    rpmi::PackedOmega pk;
    RsvdScratch w;
    rpmi::SplitPlan sp;
    size_t o_pk, o_raw, o_y, o_w, o_cnt, o_part, bytes;
};

RsvdPlan rsvd_plan(rp_ctx ctx, int64_t m, int64_t n, int64_t k, int64_t oversample, rp_omega_t omega_type,
                   rp_algo_t algo) {
    RsvdPlan pl;
    const int64_t p = k + oversample;
    Arena ar;
    pl.pk = packed_geometry(n, p, algo, nullptr);
    pl.o_pk = ar.take(packed_bytes(pl.pk, algo));
    pl.o_raw = ar.take(raw_bytes(omega_type, algo, n, p));   // generator scratch
    pl.o_y = ar.take((size_t)m * p * 4);
    pl.o_w = pl.w.layout(ar, m, n, k, p);
    pl.sp = algo == RP_ALGO_SPLIT_F16 ? rpmi::plan_split_f16(m, n, p, ctx->num_cus > 0 ? ctx->num_cus : 256)
                                      : rpmi::SplitPlan{1, 0, 0};
    if (algo == RP_ALGO_SPLIT_F16) {   // the same buffer serves the power scheme's TCEC A W
        const rpmi::SplitPlan tp = rpmi::plan_tcec(m, n, p, ctx->num_cus > 0 ? ctx->num_cus : 256);
        if (tp.partial_bytes > pl.sp.partial_bytes) pl.sp.partial_bytes = tp.partial_bytes;
    }
    pl.o_cnt = ar.take(pl.sp.counter_bytes);
    pl.o_part = ar.take(pl.sp.partial_bytes);
    pl.bytes = ar.used;
    return pl;
}

// ------------------------------------------------------------------ grouped batched stages
// Host image of the job tables of the grouped kernels (group_linalg.hip) for
// one batched call; uploaded once per captured graph into ctx->graph_aux.
struct AuxImage {
    std::vector<char> bytes;
    size_t add(const void* p, size_t n) {
        const size_t off = (bytes.size() + 255) & ~size_t(255);
        bytes.resize(off + n);
        memcpy(bytes.data() + off, p, n);
        return off;
    }
};

struct GemmStage {
    size_t jobs = 0, starts = 0;
    int count = 0;
    int64_t blocks = 0;
};

GemmStage add_gemm_stage(AuxImage& im, std::vector<rpmi::GemmJob> jobs) {
    GemmStage st;
    std::vector<int64_t> starts(jobs.size());
    int64_t b = 0;
    for (size_t i = 0; i < jobs.size(); ++i) {
        jobs[i].tiles_n = rpmi::gemm_group_tiles_n(jobs[i].N);
        jobs[i].start = b;
        starts[i] = b;
        b += rpmi::gemm_group_tiles(jobs[i].M, jobs[i].N);
    }
    st.count = (int)jobs.size();
    st.blocks = b;
    if (!jobs.empty()) {
        st.jobs = im.add(jobs.data(), jobs.size() * sizeof(rpmi::GemmJob));
        st.starts = im.add(starts.data(), starts.size() * sizeof(int64_t));
    }
    return st;
}

rpmi::GemmJob gemm_job(int64_t M, int64_t N, int64_t K, const void* a, int64_t sam, int64_t sak, const void* b,
                       int64_t sbk, int64_t sbn, void* c, int64_t scm, int64_t scn) {
    rpmi::GemmJob j{};
    j.M = M; j.N = N; j.K = K;
    j.alpha = 1.0; j.beta = 0.0;
    j.a = a; j.sam = sam; j.sak = sak;
    j.b = b; j.sbk = sbk; j.sbn = sbn;
    j.c = c; j.scm = scm; j.scn = scn;
    return j;
}

struct CholStage {
    size_t jobs = 0;
    int count = 0, max_p = 0;
};

// Grouped Grams: each job's rows go out in ksplit chunks of at least 512
// rows (at most 16 chunks), so that a tall problem spreads over several
// workgroups per tile; the partial sums need ksplit p^2 doubles per job.
struct GramStage {
    size_t jobs = 0, starts = 0;
    int count = 0;
    int64_t blocks = 0;
    bool any_split = false;
};

int gram_split(int64_t R) {
    const int64_t s = R / 512;
    return (int)(s < 1 ? 1 : (s > 16 ? 16 : s));
}

size_t gram_part_bytes(const std::vector<int64_t>& rows, const std::vector<int64_t>& ps) {
    size_t b = 0;
    for (size_t i = 0; i < rows.size(); ++i) {
        const int s = gram_split(rows[i]);
        if (s > 1) b += ((size_t)s * ps[i] * ps[i] * sizeof(double) + 255) & ~size_t(255);
    }
    return b;
}

// jobs: (Y, R rows, p, G); part: gram_part_bytes of these rows
GramStage add_gram_stage(AuxImage& im, std::vector<rpmi::GramJob> jobs, char* part) {
    GramStage st;
    std::vector<int64_t> starts(jobs.size());
    int64_t b = 0;
    for (size_t i = 0; i < jobs.size(); ++i) {
        rpmi::GramJob& j = jobs[i];
        const int s = gram_split(j.R);
        j.kchunk = s > 1 ? (((j.R + s - 1) / s + 15) / 16) * 16 : (j.R > 0 ? j.R : 1);
        j.ksplit = (int)((j.R + j.kchunk - 1) / j.kchunk);
        j.ksplit = j.ksplit < 1 ? 1 : j.ksplit;
        j.part = nullptr;
        if (j.ksplit > 1) {
            j.part = reinterpret_cast<double*>(part);
            part += ((size_t)s * j.p * j.p * sizeof(double) + 255) & ~size_t(255);
            st.any_split = true;
        }
        j.tiles = rpmi::gram_group_tiles(j.p);
        j.start = b;
        starts[i] = b;
        b += (int64_t)j.tiles * j.ksplit;
    }
    st.count = (int)jobs.size();
    st.blocks = b;
    if (!jobs.empty()) {
        st.jobs = im.add(jobs.data(), jobs.size() * sizeof(rpmi::GramJob));
        st.starts = im.add(starts.data(), starts.size() * sizeof(int64_t));
    }
    return st;
}

rpmi::GramJob gram_job(const void* y, int64_t R, int64_t p, double* G) {
    rpmi::GramJob j{};
    j.y = y;
    j.ldy = p;
    j.R = R;
    j.p = p;
    j.G = G;
    return j;
}

template <class T>
hipError_t run_gram_stage(const GramStage& st, char* aux, hipStream_t s) {
    return rpmi::gram_group<T>(reinterpret_cast<const rpmi::GramJob*>(aux + st.jobs),
                               reinterpret_cast<const int64_t*>(aux + st.starts), st.count, st.blocks, st.any_split, s);
}

// CholeskyQR2 of every problem's Y (rows R_g x p_g, FP32, ld p_g) into Q
// (FP32, ld p_g), with scratch from its RsvdScratch; with_m: also M = L1 L2
// (into MW), the lower factor R^T of the triangular factor R.
struct CholQr2Group {
    GramStage gram1, gram2;
    GemmStage qd, q, m;
    CholStage chol1, chol2;
    bool with_m = false;
};

CholQr2Group build_cholqr2_group(AuxImage& im, const std::vector<int64_t>& rows, const std::vector<float*>& Y,
                                 const std::vector<float*>& Q, const std::vector<RsvdScratch>& ws, bool with_m,
                                 char* gram_part) {
    const size_t n = ws.size();
    std::vector<rpmi::GemmJob> qd, qq, mm;
    std::vector<rpmi::GramJob> g1, g2;
    std::vector<rpmi::CholJob> c1, c2;
    CholQr2Group G;
    G.with_m = with_m;
    for (size_t i = 0; i < n; ++i) {
        const RsvdScratch& w = ws[i];
        const int64_t p = w.p, R = rows[i];
        g1.push_back(gram_job(Y[i], R, p, w.G));
        c1.push_back(rpmi::CholJob{w.G, with_m ? w.L1 : w.G, w.X, (int)p});
        qd.push_back(gemm_job(R, p, p, Y[i], p, 1, w.X, 1, p, w.Qd, p, 1));
        g2.push_back(gram_job(w.Qd, R, p, w.G));
        c2.push_back(rpmi::CholJob{w.G, w.G, w.X, (int)p});
        qq.push_back(gemm_job(R, p, p, w.Qd, p, 1, w.X, 1, p, Q[i], p, 1));
        if (with_m) mm.push_back(gemm_job(p, p, p, w.L1, p, 1, w.G, p, 1, w.MW, p, 1));
        G.chol1.max_p = G.chol2.max_p = (int)p > G.chol1.max_p ? (int)p : G.chol1.max_p;
    }
    G.gram1 = add_gram_stage(im, g1, gram_part);
    G.chol1.jobs = im.add(c1.data(), n * sizeof(rpmi::CholJob));
    G.chol1.count = (int)n;
    G.qd = add_gemm_stage(im, qd);
    G.gram2 = add_gram_stage(im, g2, gram_part);
    G.chol2.jobs = im.add(c2.data(), n * sizeof(rpmi::CholJob));
    G.chol2.count = (int)n;
    G.q = add_gemm_stage(im, qq);
    if (with_m) G.m = add_gemm_stage(im, mm);
    return G;
}

template <class TA, class TB, class TC>
hipError_t run_gemm_stage(const GemmStage& st, char* aux, hipStream_t s) {
    return rpmi::gemm_acc64_group<TA, TB, TC>(reinterpret_cast<const rpmi::GemmJob*>(aux + st.jobs),
                                              reinterpret_cast<const int64_t*>(aux + st.starts), st.count, st.blocks,
                                              s);
}

rp_status run_cholqr2_group(rp_ctx ctx, const CholQr2Group& G, char* aux, hipStream_t s) {
    RP_HIP(ctx, run_gram_stage<float>(G.gram1, aux, s));
    RP_HIP(ctx, rpmi::chol_inv_group(reinterpret_cast<const rpmi::CholJob*>(aux + G.chol1.jobs), G.chol1.count,
                                     G.chol1.max_p, ctx->d_status, s));
    RP_HIP(ctx, (run_gemm_stage<float, double, double>(G.qd, aux, s)));
    RP_HIP(ctx, run_gram_stage<double>(G.gram2, aux, s));
    RP_HIP(ctx, rpmi::chol_inv_group(reinterpret_cast<const rpmi::CholJob*>(aux + G.chol2.jobs), G.chol2.count,
                                     G.chol2.max_p, ctx->d_status, s));
    RP_HIP(ctx, (run_gemm_stage<double, double, float>(G.q, aux, s)));
    if (G.with_m) RP_HIP(ctx, (run_gemm_stage<double, double, double>(G.m, aux, s)));
    return RP_OK;
}

// Z_g = A_g^T Q_g for every problem, as one grouped launch (plus the in-order
// sum of the contraction chunks where a problem is split).
struct TnGroup {
    size_t jobs = 0, starts = 0;
    int count = 0;
    int64_t blocks = 0;
    bool any_split = false;
};

int64_t tn_tiles(int64_t N, int64_t P) {
    rpmi::TnJob j{};
    j.N = N; j.P = P;
    rpmi::tn_group_shape(j);
    return j.tiles_x * j.tiles_y;
}

// Contraction split of a grouped A^T Q with few output tiles: enough chunks
// (of at least 1024 rows, at most 8) to give the problem about 24 workgroups.
int tn_split(int64_t K, int64_t N, int64_t P) {
    const int64_t tiles = tn_tiles(N, P);
    int64_t s = (24 + tiles - 1) / tiles;
    const int64_t kmax = K / 1024;
    s = s > kmax ? kmax : s;
    s = s > 8 ? 8 : s;
    return (int)(s < 1 ? 1 : s);
}

size_t tn_part_bytes(const rp_rsvd_problem* probs, int32_t count) {
    size_t b = 0;
    for (int32_t g = 0; g < count; ++g) {
        const int64_t p = probs[g].k + probs[g].oversample;
        const int s = tn_split(probs[g].m, probs[g].n, p);
        if (s > 1) b += ((size_t)s * probs[g].n * p * sizeof(float) + 255) & ~size_t(255);
    }
    return b;
}

TnGroup build_tn_group(AuxImage& im, const rp_rsvd_problem* probs, const std::vector<RsvdScratch>& ws, char* part) {
    TnGroup T;
    std::vector<rpmi::TnJob> jobs;
    std::vector<int64_t> starts;
    for (size_t i = 0; i < ws.size(); ++i) {
        const rp_rsvd_problem& q = probs[i];
        const RsvdScratch& w = ws[i];
        rpmi::TnJob j{};
        j.N = q.n; j.P = w.p; j.K = q.m;
        j.A = q.A; j.lda = q.lda; j.Q = w.Q; j.ldq = w.p; j.C = w.Z; j.ldc = w.p;
        const int sp = tn_split(q.m, q.n, w.p);
        j.kchunk = sp > 1 ? (((q.m + sp - 1) / sp + 15) / 16) * 16 : (q.m > 0 ? q.m : 1);
        j.ksplit = (int)((q.m + j.kchunk - 1) / j.kchunk);
        j.ksplit = j.ksplit < 1 ? 1 : j.ksplit;
        j.part = nullptr;
        if (j.ksplit > 1) {
            j.part = reinterpret_cast<float*>(part);
            part += ((size_t)sp * q.n * w.p * sizeof(float) + 255) & ~size_t(255);
            T.any_split = true;
        }
        rpmi::tn_group_shape(j);
        jobs.push_back(j);
    }
    // every wave of a job runs kchunk rows: longest first (a stable order, so
    // the table is the same on every call)
    std::stable_sort(jobs.begin(), jobs.end(),
                     [](const rpmi::TnJob& x, const rpmi::TnJob& y) { return x.kchunk > y.kchunk; });
    for (rpmi::TnJob& j : jobs) {
        j.start = T.blocks;
        starts.push_back(T.blocks);
        T.blocks += j.tiles_x * j.tiles_y * j.ksplit;
    }
    T.count = (int)jobs.size();
    if (!jobs.empty()) {
        T.jobs = im.add(jobs.data(), jobs.size() * sizeof(rpmi::TnJob));
        T.starts = im.add(starts.data(), starts.size() * sizeof(int64_t));
    }
    return T;
}

rp_status run_tn_group(rp_ctx ctx, const TnGroup& T, char* aux, hipStream_t s) {
    if (T.count > 0)
        RP_HIP(ctx, rpmi::gemm_tn_f32_group(reinterpret_cast<const rpmi::TnJob*>(aux + T.jobs),
                                            reinterpret_cast<const int64_t*>(aux + T.starts), T.count, T.blocks,
                                            T.any_split, s));
    return RP_OK;
}

// After the grouped Jacobi: S, U = Q U_r[:, :k], V^T = (Q_B V_r[:, :k])^T.
struct FinishGroup {
    size_t svd = 0;
    int count = 0, max_elems = 0;
    GemmStage u, vt;
};

FinishGroup build_finish_group(AuxImage& im, const rp_rsvd_problem* probs, const std::vector<RsvdScratch>& ws) {
    FinishGroup F;
    std::vector<rpmi::SvdJob> sj;
    std::vector<rpmi::GemmJob> uj, vj;
    for (size_t i = 0; i < ws.size(); ++i) {
        const rp_rsvd_problem& q = probs[i];
        const RsvdScratch& w = ws[i];
        const int64_t p = w.p, k = q.k;
        sj.push_back(rpmi::SvdJob{w.MW, w.MV, (int)p, (int)k, w.sig, w.ord, q.S, w.Ur, w.Vr});
        F.max_elems = (int)(p * k) > F.max_elems ? (int)(p * k) : F.max_elems;
        uj.push_back(gemm_job(q.m, k, p, w.Q, p, 1, w.Ur, k, 1, q.U, q.ldu, 1));
        vj.push_back(gemm_job(q.n, k, p, w.W, p, 1, w.Vr, k, 1, q.VT, 1, q.ldvt));
    }
    F.count = (int)sj.size();
    F.svd = im.add(sj.data(), sj.size() * sizeof(rpmi::SvdJob));
    F.u = add_gemm_stage(im, uj);
    F.vt = add_gemm_stage(im, vj);
    return F;
}

rp_status run_finish_group(rp_ctx ctx, const FinishGroup& F, char* aux, hipStream_t s) {
    RP_HIP(ctx, rpmi::svd_finish_group(reinterpret_cast<const rpmi::SvdJob*>(aux + F.svd), F.count, F.max_elems, s));
    // Algorithm 1 line 5 in FP32 (U_r, V_r rounded to FP32)
    RP_HIP(ctx, (rpmi::gemm_f32_group<float, double, float>(reinterpret_cast<const rpmi::GemmJob*>(aux + F.u.jobs),
                                                            reinterpret_cast<const int64_t*>(aux + F.u.starts),
                                                            F.u.count, F.u.blocks, s)));
    RP_HIP(ctx, (rpmi::gemm_f32_group<float, double, float>(reinterpret_cast<const rpmi::GemmJob*>(aux + F.vt.jobs),
                                                            reinterpret_cast<const int64_t*>(aux + F.vt.starts),
                                                            F.vt.count, F.vt.blocks, s)));
    return RP_OK;
}


}  // namespace

extern "C" {

rp_status rsvd_workspace_size(rp_ctx ctx, int64_t m, int64_t n, int64_t k, int64_t oversample,
                              int32_t power_iters, rp_omega_t omega_type, rp_algo_t algo, size_t* bytes) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    if (!bytes) return fail(ctx, RP_ERR_INVALID_ARG, "bytes is NULL");
    rp_status st;
    if (!enums_ok(ctx, omega_type, algo, &st)) return st;
    if (algo == RP_ALGO_TCEC_F16)
        return fail(ctx, RP_ERR_INVALID_ARG, "the randomized algorithms project with RP_ALGO_F32 or RP_ALGO_SPLIT_F16");
    const int64_t p = k + oversample;
    if (m <= 0 || n <= 0 || k <= 0 || oversample < 0 || power_iters < 0 || p > m || p > n || p > 1024)
        return fail(ctx, RP_ERR_INVALID_ARG, "invalid sizes (m %lld, n %lld, k %lld, s %lld, q %d)", (long long)m,
                    (long long)n, (long long)k, (long long)oversample, (int)power_iters);
    *bytes = rsvd_plan(ctx, m, n, k, oversample, omega_type, algo).bytes;
    return RP_OK;
}

rp_status rsvd(rp_ctx ctx, int64_t m, int64_t n, const float* A, int64_t lda, int64_t k, int64_t oversample,
               int32_t power_iters, uint64_t seed, rp_omega_t omega_type, rp_algo_t algo, int32_t a_scale_exp,
               float* U, int64_t ldu, double* S, float* VT, int64_t ldvt, void* work, size_t work_bytes,
               void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    rp_status st;
    if (!enums_ok(ctx, omega_type, algo, &st)) return st;
    if (algo == RP_ALGO_TCEC_F16)
        return fail(ctx, RP_ERR_INVALID_ARG, "the randomized algorithms project with RP_ALGO_F32 or RP_ALGO_SPLIT_F16");
    if (!scale_exp_ok(ctx, a_scale_exp, &st, true)) return st;
    const rp_rsvd_problem prob{m, n, A, lda, k, oversample, U, ldu, S, VT, ldvt};
    if ((st = rsvd_check(ctx, prob, power_iters)) != RP_OK) return st;
    const RsvdPlan pl = rsvd_plan(ctx, m, n, k, oversample, omega_type, algo);
    if (work) {
        if (reinterpret_cast<uintptr_t>(work) & 255) return fail(ctx, RP_ERR_INVALID_ARG, "work is not 256-byte aligned");
        if (work_bytes < pl.bytes)
            return fail(ctx, RP_ERR_INVALID_ARG, "work_bytes %zu < %zu (rsvd_workspace_size)", work_bytes, pl.bytes);
    }
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipSetDevice(ctx->device));
    const int64_t p = k + oversample;
    const rp_desc dA{A, m, n, lda, n, 1, 0};
    if (!work && (st = ensure_workspace(ctx, pl.bytes)) != RP_OK) return st;
    char* base = static_cast<char*>(work ? work : ctx->ws);
    rpmi::PackedOmega pk = pl.pk;
    pk.data = base + pl.o_pk;
    RsvdScratch w = pl.w;
    w.bind(base + pl.o_w);
    {
        // the power scheme's A W on the TCEC products when the projection is
        // split-FP16 and A is on their 16-byte path (pkw has the same size in
        // both forms; their contraction split uses the projection's buffer)
        // (with a caller pre-scale, which the TCEC kernels do not take, the
        // FP32 kernels, which need none)
        const rpmi::ProjArgs aw = proj_args(ctx, &dA, p, nullptr, 0, nullptr, p, 0);
        const bool tcec = algo == RP_ALGO_SPLIT_F16 && a_scale_exp == 0 && rpmi::split_fast_ok(aw);
        w.tcec_aw = tcec && power_iters > 0 &&
                    packed_geometry(n, p, RP_ALGO_TCEC_F16, nullptr).nt_count == w.pkw.nt_count;
        // A^T Q (Algorithm 1 line 3 and the power scheme) likewise
        w.tcec_atq = tcec;
    }
    float* Y = reinterpret_cast<float*>(base + pl.o_y);
    SplitBuffers sb{reinterpret_cast<unsigned int*>(base + pl.o_cnt), reinterpret_cast<float*>(base + pl.o_part),
                    pl.sp.counter_bytes, pl.sp.partial_bytes};
    w.aw_sb = &sb;
    if (pl.sp.counter_bytes)
        RP_HIP(ctx, rpmi::launch_fill_u32(sb.counters, (int64_t)(pl.sp.counter_bytes / 4), 0u, s));
    // Algorithm 1 line 1: Y = A Omega (Omega from the context cache, or
    // generated into the workspace when it does not fit the cache or the
    // caller's workspace rules out allocation)
    st = work ? RP_ERR_UNSUPPORTED
              : cached_packed_omega(ctx, seed, 0, omega_type, n, p, algo, base + pl.o_raw, s, &pk, ctx->omega_tick);
    if (st == RP_ERR_UNSUPPORTED) {
        pk.data = base + pl.o_pk;
        st = fill_packed(ctx, seed, 0, nullptr, 0, nullptr, omega_type, n, p, algo, pk, base + pl.o_raw, s);
    }
    if (st != RP_OK) return st;
    if ((st = launch_projection(ctx, &dA, p, pk, algo, Y, p, s, algo == RP_ALGO_SPLIT_F16 ? a_scale_exp : 0, false,
                                &sb, w.rowx)) != RP_OK)
        return st;
    return rsvd_after_projection(ctx, dA, prob, p, power_iters, Y, w, s);
}

rp_status rp_gemm_tn(rp_ctx ctx, int64_t m, int64_t n, int64_t p, const float* A, int64_t lda, const float* Q,
                     int64_t ldq, rp_algo_t algo, float* Z, int64_t ldz, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    if (m < 0 || n < 0 || p < 0) return fail(ctx, RP_ERR_INVALID_ARG, "negative size");
    if (algo != RP_ALGO_F32 && algo != RP_ALGO_TCEC_F16)
        return fail(ctx, RP_ERR_INVALID_ARG, "rp_gemm_tn takes RP_ALGO_F32 or RP_ALGO_TCEC_F16");
    if (n == 0 || p == 0) return RP_OK;
    if (!A || !Q || !Z) return fail(ctx, RP_ERR_INVALID_ARG, "NULL pointer");
    if (lda < n || ldq < p || ldz < p) return fail(ctx, RP_ERR_INVALID_ARG, "leading dimension too small");
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipSetDevice(ctx->device));
    if (m == 0) {
        RP_HIP(ctx, rpmi::launch_fill_f32(Z, n, p, ldz, 0.0f, s));
        return RP_OK;
    }
    if (algo == RP_ALGO_F32) return gemm_at_q(ctx, m, n, p, A, lda, Q, ldq, Z, ldz, nullptr, s);
    if ((n & 3) || (lda & 3) || (reinterpret_cast<uintptr_t>(A) & 15))
        return fail(ctx, RP_ERR_UNSUPPORTED, "the TCEC A^T Q needs n and lda multiples of 4 and a 16-byte aligned A");
    rpmi::PackedOmega pkq = packed_geometry(m, p, RP_ALGO_TCEC_F16, nullptr);
    rp_status st;
    if ((st = ensure_workspace(ctx, packed_bytes(pkq, RP_ALGO_TCEC_F16))) != RP_OK) return st;
    pkq.data = ctx->ws;
    return gemm_at_q(ctx, m, n, p, A, lda, Q, ldq, Z, ldz, &pkq, s, true);
}

rp_status rp_project_grouped(rp_ctx ctx, int32_t count, const rp_project_problem* probs, rp_omega_t omega_type,
                             void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    if (count < 0 || (count > 0 && !probs)) return fail(ctx, RP_ERR_INVALID_ARG, "invalid problem list");
    if (omega_type != RP_OMEGA_F16 && omega_type != RP_OMEGA_E4M3 && !sparse_type(omega_type))
        return fail(ctx, RP_ERR_UNSUPPORTED, "grouped projections take an FP16 or e4m3 Omega");
    rp_status st;
    for (int32_t g = 0; g < count; ++g) {
        const rp_project_problem& q = probs[g];
        if (!desc_ok(ctx, &q.A, &st)) return st;
        if (!scale_exp_ok(ctx, q.a_scale_exp, &st)) return st;
        if (q.r < 0) return fail(ctx, RP_ERR_INVALID_ARG, "problem %d: negative r", (int)g);
        if (q.A.rows > 0 && q.r > 0) {
            if (!q.Y || q.ldy < q.r) return fail(ctx, RP_ERR_INVALID_ARG, "problem %d: bad Y", (int)g);
            if (q.A.cols > 0 && !proj_layout_ok(ctx, &q.A, &st)) return st;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipSetDevice(ctx->device));
    Arena ar;
    std::vector<size_t> off(count);
    std::vector<rpmi::PackedOmega> pk(count);
    size_t rawb = 0;
    for (int32_t g = 0; g < count; ++g) {
        pk[g] = packed_geometry(probs[g].A.cols, probs[g].r, RP_ALGO_SPLIT_F16, nullptr);
        off[g] = ar.take(packed_bytes(pk[g], RP_ALGO_SPLIT_F16));
        const size_t rb = raw_bytes(omega_type, RP_ALGO_SPLIT_F16, probs[g].A.cols, probs[g].r);
        rawb = rb > rawb ? rb : rawb;
    }
    const size_t o_raw = ar.take(rawb);
    if ((st = ensure_workspace(ctx, ar.used)) != RP_OK) return st;
    std::vector<rpmi::ProjArgs> grouped;
    for (int32_t g = 0; g < count; ++g) {
        const rp_project_problem& q = probs[g];
        if (q.A.rows == 0 || q.r == 0) continue;
        if (q.A.cols == 0) {
            RP_HIP(ctx, rpmi::launch_fill_f32(q.Y, q.A.rows, q.r, q.ldy, 0.0f, s));
            continue;
        }
        pk[g].data = static_cast<char*>(ctx->ws) + off[g];
        if ((st = fill_packed(ctx, q.seed, q.stream_id, nullptr, 0, nullptr, omega_type, q.A.cols, q.r,
                              RP_ALGO_SPLIT_F16, pk[g], static_cast<char*>(ctx->ws) + o_raw, s)) != RP_OK)
            return st;
        grouped.push_back(proj_args(ctx, &q.A, q.r, pk[g].data, pk[g].nt_count, q.Y, q.ldy, q.a_scale_exp));
    }
    if (grouped.empty()) return RP_OK;
    GroupPlan gp;
    if ((st = tuned_group_plan(ctx, grouped, s, &gp)) != RP_OK) return st;
    if ((st = ensure_table(ctx, gp.entries.size())) != RP_OK) return st;
    return launch_group(ctx, gp, ctx->table, s);
}

// One batched call from its two graphs: the first (through the first Jacobi
// sweeps), then while some problem is open and the sweep bound allows, one
// eager sweep at a time (the host reads the open count after each: a stream
// synchronisation), then the second graph.
rp_status run_batched_graphs(rp_ctx ctx, hipStream_t s) {
    const auto& J = ctx->graph_jac;
    RP_HIP(ctx, hipGraphLaunch(ctx->graph_exec, s));
    const rpmi::JacobiProb* jtab = ctx->graph_jtab;
    for (int sweep = J.graph_sweeps; sweep < J.bound; ++sweep) {
        int open = 0;
        RP_HIP(ctx, rpmi::jacobi_group_open(jtab, J.count, ctx->d_jopen, s));
        RP_HIP(ctx, hipMemcpyAsync(&open, ctx->d_jopen, sizeof open, hipMemcpyDeviceToHost, s));
        RP_HIP(ctx, hipStreamSynchronize(s));
        if (open == 0) break;
        RP_HIP(ctx, rpmi::jacobi_group_sweeps(jtab, J.count, J.pairs, J.bpairs, J.max_n, sweep, sweep + 1,
                                              kJacobiTol, s));
    }
    RP_HIP(ctx, hipGraphLaunch(ctx->graph_exec2, s));
    return RP_OK;
}

rp_status rsvd_batched(rp_ctx ctx, int32_t count, const rp_rsvd_problem* probs, int32_t power_iters,
                       uint64_t seed, rp_omega_t omega_type, void* stream) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    if (count < 0 || (count > 0 && !probs)) return fail(ctx, RP_ERR_INVALID_ARG, "invalid problem list");
    if (omega_type != RP_OMEGA_F16 && omega_type != RP_OMEGA_F32 && omega_type != RP_OMEGA_E4M3 &&
        !sparse_type(omega_type))
        return fail(ctx, RP_ERR_INVALID_ARG, "unknown omega type %d", (int)omega_type);
    const rp_algo_t algo = omega_type == RP_OMEGA_F32 ? RP_ALGO_F32 : RP_ALGO_SPLIT_F16;
    rp_status st;
    for (int32_t g = 0; g < count; ++g)
        if ((st = rsvd_check(ctx, probs[g], power_iters)) != RP_OK) return st;
    if (count == 0) return RP_OK;
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipSetDevice(ctx->device));

    // workspace: per problem its packed Omega and Y; one scratch block sized
    // for the largest problem, shared (the per-problem stages run in order)
    Arena ar;
    std::vector<size_t> o_pk(count), o_y(count);
    std::vector<rpmi::PackedOmega> pk(count);
    int64_t mp = 0;
    size_t raw = 0;
    for (int32_t g = 0; g < count; ++g) {
        const rp_rsvd_problem& q = probs[g];
        const int64_t p = q.k + q.oversample;
        pk[g] = packed_geometry(q.n, p, algo, nullptr);
        o_pk[g] = ar.take(packed_bytes(pk[g], algo));
        o_y[g] = ar.take((size_t)q.m * p * 4);
        mp = p > mp ? p : mp;
        raw = raw_bytes(omega_type, algo, q.n, p) > raw ? raw_bytes(omega_type, algo, q.n, p) : raw;
    }
    const size_t o_raw = ar.take(raw);
    // per problem its own scratch (the stages before and after the grouped
    // Jacobi SVD keep Q, Q_B and R_B^T of every problem)
    std::vector<RsvdScratch> ws(count);
    std::vector<size_t> o_ws(count);
    for (int32_t g = 0; g < count; ++g)
        o_ws[g] = ws[g].layout(ar, probs[g].m, probs[g].n, probs[g].k, probs[g].k + probs[g].oversample, false);
    // partial sums of the grouped Grams (shared by every CholeskyQR2 stage, which run in turn)
    size_t o_gpart = 0;
    {
        std::vector<int64_t> mr(count), nr(count), pr(count);
        for (int32_t g = 0; g < count; ++g) {
            mr[g] = probs[g].m;
            nr[g] = probs[g].n;
            pr[g] = probs[g].k + probs[g].oversample;
        }
        const size_t bm = gram_part_bytes(mr, pr), bn = gram_part_bytes(nr, pr);
        o_gpart = ar.take(bm > bn ? bm : bn);
    }
    const size_t o_tnpart = ar.take(tn_part_bytes(probs, count));
    if ((st = ensure_workspace(ctx, ar.used)) != RP_OK) return st;
    char* base = static_cast<char*>(ctx->ws);
    for (int32_t g = 0; g < count; ++g) pk[g].data = base + o_pk[g];
    for (int32_t g = 0; g < count; ++g) ws[g].bind(base + o_ws[g]);

    // split-FP16 projections go out grouped (the 16-byte-path problems to the
    // fast kernels, the others to the general one)
    std::vector<rpmi::ProjArgs> grouped, grouped_fast;
    std::vector<int> single;
    uint64_t sig = mix(mix(0, (uint64_t)count), (uint64_t)ctx->num_cus);
    for (int32_t g = 0; g < count; ++g) {
        const rp_rsvd_problem& q = probs[g];
        const rp_desc dA{q.A, q.m, q.n, q.lda, q.n, 1, 0};
        const int64_t p = q.k + q.oversample;
        const rpmi::ProjArgs a = proj_args(ctx, &dA, p, pk[g].data, pk[g].nt_count,
                                           reinterpret_cast<float*>(base + o_y[g]), p, 0);
        if (algo == RP_ALGO_SPLIT_F16) {
            grouped.push_back(a);
            if (rpmi::split_fast_ok(a)) grouped_fast.push_back(a);
        } else {
            single.push_back(g);
        }
        sig = mix(mix(mix(mix(sig, (uint64_t)q.m), (uint64_t)q.n), (uint64_t)a.r), (uint64_t)rpmi::split_fast_ok(a));
    }

    // the graph of this exact call: problem set, buffers, options, context buffers
    auto call_key = [&]() {
        uint64_t key = mix(sig, seed);
        key = mix(mix(key, (uint64_t)power_iters), (uint64_t)omega_type);
        for (int32_t g = 0; g < count; ++g) {
            const rp_rsvd_problem& q = probs[g];
            key = mix(mix(mix(key, (uint64_t)(uintptr_t)q.A), (uint64_t)q.lda), (uint64_t)q.k);
            key = mix(mix(mix(key, (uint64_t)(uintptr_t)q.U), (uint64_t)(uintptr_t)q.S), (uint64_t)(uintptr_t)q.VT);
            key = mix(mix(mix(key, (uint64_t)q.ldu), (uint64_t)q.ldvt), (uint64_t)q.oversample);
        }
        key = mix(mix(key, (uint64_t)(uintptr_t)ctx->ws), (uint64_t)ctx->ws_bytes);
        key = mix(mix(key, (uint64_t)(uintptr_t)ctx->split_ws), (uint64_t)ctx->split_ws_bytes);
        return mix(mix(key, (uint64_t)(uintptr_t)ctx->split_counters), (uint64_t)ctx->split_counter_bytes);
    };
    if (ctx->graph_exec && ctx->graph_exec2 && call_key() == ctx->graph_key) return run_batched_graphs(ctx, s);

    auto gen_omega = [&](hipStream_t st_) -> rp_status {
        for (int32_t g = 0; g < count; ++g) {
            const rp_rsvd_problem& q = probs[g];
            rp_status r2 = fill_packed(ctx, seed, (uint32_t)g, nullptr, 0, nullptr, omega_type, q.n, q.k + q.oversample,
                                       algo, pk[g], base + o_raw, st_);
            if (r2 != RP_OK) return r2;
        }
        return RP_OK;
    };
    RP_HIP(ctx, hipStreamSynchronize(s));
    if (!ctx->cap_stream) RP_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = ctx->cap_stream;

    // autotuner: the contraction split of every grouped problem on the
    // 16-byte path follows its share of the compute units times a scale, and
    // the narrow ones take one of two kernel forms; both are chosen once per
    // problem-shape signature by timing the fast grouped launches
    GroupPlan gp;
    if (!grouped.empty()) {
        auto it = ctx->tuned_scale.find(sig);
        rp_ctx_s::TuneEntry best{1.0, 0};
        if (it != ctx->tuned_scale.end()) {
            best = it->second;
        } else if (!grouped_fast.empty()) {
            if ((st = gen_omega(cs)) != RP_OK) return st;
            if ((st = tune_group(ctx, grouped_fast, sig, cs, &best)) != RP_OK) return st;
        }
        if (ctx->force_form >= 0) best.form = ctx->force_form;
        if ((st = plan_group(ctx, grouped, best.scale, &gp, best.form == 1)) != RP_OK) return st;
        if (gp.entries.size() > ctx->graph_table_entries) {
            if (ctx->graph_table) RP_HIP(ctx, hipFree(ctx->graph_table));
            ctx->graph_table = nullptr;
            ctx->graph_table_entries = 0;
            RP_HIP(ctx, hipMalloc(&ctx->graph_table, gp.entries.size() * sizeof(rpmi::GroupEntry)));
            ctx->graph_table_entries = gp.entries.size();
        }
        RP_HIP(ctx, hipMemcpy(ctx->graph_table, gp.entries.data(), gp.entries.size() * sizeof(rpmi::GroupEntry),
                              hipMemcpyHostToDevice));
    }
    std::vector<rpmi::JacobiProb> jt(count);
    int jpairs = 0, jbpairs = 0;
    for (int32_t g = 0; g < count; ++g) {
        const int p = (int)(probs[g].k + probs[g].oversample);
        jt[g] = rpmi::JacobiProb{ws[g].MW, ws[g].MV, p, jpairs, ws[g].jflags, jbpairs};
        jpairs += (p + 1) / 2;
        jbpairs += rpmi::jacobi_block_pairs(p);
    }
    if ((size_t)count > ctx->graph_jtab_entries) {
        if (ctx->graph_jtab) RP_HIP(ctx, hipFree(ctx->graph_jtab));
        ctx->graph_jtab = nullptr;
        ctx->graph_jtab_entries = 0;
        RP_HIP(ctx, hipMalloc(&ctx->graph_jtab, (size_t)count * sizeof(rpmi::JacobiProb)));
        ctx->graph_jtab_entries = count;
    }
    rpmi::JacobiProb* jtab = ctx->graph_jtab;
    RP_HIP(ctx, hipMemcpy(jtab, jt.data(), jt.size() * sizeof(rpmi::JacobiProb), hipMemcpyHostToDevice));
    // every stage after the projections as grouped launches when every
    // problem's Cholesky factor fits the one-workgroup kernel
    const bool grouped_stages = mp <= rpmi::kCholGroupMaxP;
    AuxImage im;
    const bool omega_group = grouped_stages && algo == RP_ALGO_SPLIT_F16 &&
                             (omega_type == RP_OMEGA_F16 || sparse_type(omega_type));
    size_t om_jobs = 0;
    int64_t om_blocks = 0;
    CholQr2Group cq_yq, cq_zw, cq_zw_m;
    TnGroup tn;
    FinishGroup fin;
    if (grouped_stages) {
        std::vector<int64_t> mrows(count), nrows(count);
        std::vector<float*> ys(count), qs(count), zs(count), wsp(count);
        for (int32_t g = 0; g < count; ++g) {
            mrows[g] = probs[g].m;
            nrows[g] = probs[g].n;
            ys[g] = reinterpret_cast<float*>(base + o_y[g]);
            qs[g] = ws[g].Q;
            zs[g] = ws[g].Z;
            wsp[g] = ws[g].W;
        }
        char* gpart = base + o_gpart;
        cq_yq = build_cholqr2_group(im, mrows, ys, qs, ws, false, gpart);
        if (power_iters > 0) cq_zw = build_cholqr2_group(im, nrows, zs, wsp, ws, false, gpart);
        cq_zw_m = build_cholqr2_group(im, nrows, zs, wsp, ws, true, gpart);
        tn = build_tn_group(im, probs, ws, base + o_tnpart);
        fin = build_finish_group(im, probs, ws);
        if (omega_group) {
            // every problem's packed FP16 (or sparse) Omega in one launch
            std::vector<rpmi::OmegaJob> oj(count);
            for (int32_t g = 0; g < count; ++g) {
                const rp_rsvd_problem& q = probs[g];
                oj[g] = rpmi::OmegaJob{seed, (uint32_t)g, q.n, q.k + q.oversample, pk[g].data, pk[g].nt_count,
                                       sparse_type(omega_type) ? sparse_threshold(omega_type, q.n) : 0, om_blocks};
                om_blocks += pk[g].kb_count * (pk[g].nt_count / 4);
            }
            om_jobs = im.add(oj.data(), oj.size() * sizeof(rpmi::OmegaJob));
        }
        if (im.bytes.size() > ctx->graph_aux_bytes) {
            if (ctx->graph_aux) RP_HIP(ctx, hipFree(ctx->graph_aux));
            ctx->graph_aux = nullptr;
            ctx->graph_aux_bytes = 0;
            RP_HIP(ctx, hipMalloc(&ctx->graph_aux, im.bytes.size()));
            ctx->graph_aux_bytes = im.bytes.size();
        }
        RP_HIP(ctx, hipMemcpy(ctx->graph_aux, im.bytes.data(), im.bytes.size(), hipMemcpyHostToDevice));
    }
    char* aux = ctx->graph_aux;
    RP_HIP(ctx, hipDeviceSynchronize());

    // capture: Omega generation, the grouped projections, then every
    // problem's CholeskyQR2 / B / SVD stages
    if (ctx->graph_exec) {
        (void)hipGraphExecDestroy(ctx->graph_exec);
        ctx->graph_exec = nullptr;
    }
    if (ctx->graph_exec2) {
        (void)hipGraphExecDestroy(ctx->graph_exec2);
        ctx->graph_exec2 = nullptr;
    }
    if (!ctx->d_jopen) RP_HIP(ctx, hipMalloc(&ctx->d_jopen, sizeof(int)));
    const int jbound = rpmi::jacobi_group_sweep_bound((int)mp, kJacobiSweeps);
    const int jwant = ctx->graph_sweeps >= 0 ? ctx->graph_sweeps : kBatchedGraphSweeps;
    const int jgraph = jbound < jwant ? jbound : jwant;
    auto body = [&]() -> rp_status {
        rp_status r2 = RP_OK;
        if (omega_group) {
            RP_HIP(ctx, rpmi::launch_omega_packed_f16_group(tables(ctx), reinterpret_cast<const rpmi::OmegaJob*>(
                                                                aux + om_jobs), count, om_blocks, cs));
        } else if ((r2 = gen_omega(cs)) != RP_OK) {
            return r2;
        }
        if (!gp.entries.empty() && (r2 = launch_group_kernels(ctx, gp, ctx->graph_table, cs)) != RP_OK) return r2;
        for (int g : single) {
            const rp_rsvd_problem& q = probs[g];
            const rp_desc dA{q.A, q.m, q.n, q.lda, q.n, 1, 0};
            const int64_t p = q.k + q.oversample;
            if ((r2 = launch_projection(ctx, &dA, p, pk[g], algo, reinterpret_cast<float*>(base + o_y[g]), p, cs)) !=
                RP_OK)
                return r2;
        }
        if (grouped_stages) {
            // Algorithm 1 lines 2-4 for every problem at once (power scheme:
            // the products A W stay per problem)
            for (int32_t t = 0; t < power_iters; ++t) {
                if ((r2 = run_cholqr2_group(ctx, cq_yq, aux, cs)) != RP_OK) return r2;
                if ((r2 = run_tn_group(ctx, tn, aux, cs)) != RP_OK) return r2;
                if ((r2 = run_cholqr2_group(ctx, cq_zw, aux, cs)) != RP_OK) return r2;
                for (int32_t g = 0; g < count; ++g) {
                    const rp_rsvd_problem& q = probs[g];
                    const rp_desc dA{q.A, q.m, q.n, q.lda, q.n, 1, 0};
                    const int64_t p = q.k + q.oversample;
                    RP_HIP(ctx, rpmi::launch_pack_omega(ws[g].W, rpmi::OmegaSrc::F32, nullptr, q.n, p, p, ws[g].pkw,
                                                        true, nullptr, 0, nullptr, cs));
                    if ((r2 = launch_projection(ctx, &dA, p, ws[g].pkw, RP_ALGO_F32,
                                                reinterpret_cast<float*>(base + o_y[g]), p, cs)) != RP_OK)
                        return r2;
                }
            }
            if ((r2 = run_cholqr2_group(ctx, cq_yq, aux, cs)) != RP_OK) return r2;
            if ((r2 = run_tn_group(ctx, tn, aux, cs)) != RP_OK) return r2;
            if ((r2 = run_cholqr2_group(ctx, cq_zw_m, aux, cs)) != RP_OK) return r2;
        } else {
            for (int32_t g = 0; g < count; ++g) {
                const rp_rsvd_problem& q = probs[g];
                const rp_desc dA{q.A, q.m, q.n, q.lda, q.n, 1, 0};
                r2 = rsvd_before_svd(ctx, dA, q, q.k + q.oversample, power_iters,
                                     reinterpret_cast<float*>(base + o_y[g]), ws[g], cs);
                if (r2 != RP_OK) return r2;
            }
        }
        // one parallel Jacobi SVD over every problem's R_B^T: its first sweeps
        RP_HIP(ctx, rpmi::jacobi_group_prep(jtab, count, (int)mp, cs));
        RP_HIP(ctx, rpmi::jacobi_group_sweeps(jtab, count, jpairs, jbpairs, (int)mp, 0, jgraph, kJacobiTol, cs));
        return RP_OK;
    };
    // the second graph: the Jacobi final step and Algorithm 1 line 5
    auto body2 = [&]() -> rp_status {
        rp_status r2 = RP_OK;
        RP_HIP(ctx, rpmi::jacobi_group_final(jtab, count, (int)mp, ctx->d_status, cs));
        if (grouped_stages) return run_finish_group(ctx, fin, aux, cs);
        for (int32_t g = 0; g < count; ++g)
            if ((r2 = rsvd_after_svd(ctx, probs[g], probs[g].k + probs[g].oversample, ws[g], cs)) != RP_OK) return r2;
        return RP_OK;
    };
    auto capture = [&](const std::function<rp_status()>& fn, hipGraphExec_t* out) -> rp_status {
        RP_HIP(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        const rp_status body_st = fn();
        hipGraph_t graph = nullptr;
        const hipError_t ce = hipStreamEndCapture(cs, &graph);
        if (body_st != RP_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return body_st;
        }
        if (ce != hipSuccess) return hip_fail(ctx, ce, "hipStreamEndCapture");
        const hipError_t ie = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) return hip_fail(ctx, ie, "hipGraphInstantiate");
        return RP_OK;
    };
    rp_status cst = capture(body, &ctx->graph_exec);
    if (cst == RP_OK) cst = capture(body2, &ctx->graph_exec2);
    if (cst != RP_OK) {
        if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
        ctx->graph_exec = nullptr;
        return cst;
    }
    ctx->graph_jac = {count, jpairs, jbpairs, (int)mp, jgraph, jbound};
    ctx->graph_key = call_key();
    return run_batched_graphs(ctx, s);
}

}  // extern "C"

namespace {

// Algorithm 2 line 2 for every mode (W_i = X_(i) Omega_i), shared by rp_hosvd
// and rp_hosvd_project: the mode layouts, their workspace and the launches.
//  * A mode whose unfolding streams in place (rows i_i, column runs of a
//    multiple of 64 contiguous elements) is a plain projection; with the
//    split algorithm all of them go out in grouped launches.
//  * The last mode's unfolding is the transpose of X viewed as
//    (total / I_N) x I_N row-major: W_N = X^T Omega_N on the transposed split
//    kernel (X streamed in place, contraction split over its rows), when
//    I_N is a multiple of 4 and X 16-byte aligned.
//  * Any other mode is copied mode-first into workspace and projected.
struct HosvdModes {
    int N = 0;
    int64_t total = 1;
    int64_t after[rpmi::kMaxGroup], before[rpmi::kMaxGroup];
    rp_desc desc[rpmi::kMaxGroup];
    bool permuted[rpmi::kMaxGroup], tn_mode[rpmi::kMaxGroup];
    int tn_split_k[rpmi::kMaxGroup];
    int64_t tn_chunk[rpmi::kMaxGroup];
    rpmi::PackedOmega pk[rpmi::kMaxGroup];
    size_t o_pk[rpmi::kMaxGroup], o_tnp[rpmi::kMaxGroup];
    size_t o_raw = 0, o_perm = 0;
};

rp_status hosvd_check(rp_ctx ctx, int32_t ndim, const int64_t* dims, const float* X, const int64_t* ranks,
                      rp_omega_t omega_type, rp_algo_t algo, float* const* outs, const char* what) {
    if (!ctx) return fail(nullptr, RP_ERR_INVALID_ARG, "ctx is NULL");
    rp_status st;
    if (!enums_ok(ctx, omega_type, algo, &st)) return st;
    if (algo == RP_ALGO_TCEC_F16)
        return fail(ctx, RP_ERR_INVALID_ARG, "the randomized algorithms project with RP_ALGO_F32 or RP_ALGO_SPLIT_F16");
    if (ndim < 2 || ndim > rpmi::kMaxGroup)
        return fail(ctx, RP_ERR_INVALID_ARG, "ndim %d outside [2, %d]", (int)ndim, rpmi::kMaxGroup);
    if (!dims || !ranks || !X || !outs) return fail(ctx, RP_ERR_INVALID_ARG, "NULL pointer");
    int64_t total = 1;
    for (int i = 0; i < ndim; ++i) {
        if (dims[i] <= 0) return fail(ctx, RP_ERR_INVALID_ARG, "dims[%d] = %lld", i, (long long)dims[i]);
        total *= dims[i];
    }
    for (int i = 0; i < ndim; ++i) {
        const int64_t cols = total / dims[i];
        if (ranks[i] <= 0 || ranks[i] > dims[i] || ranks[i] > cols || ranks[i] > 1024)
            return fail(ctx, RP_ERR_INVALID_ARG, "ranks[%d] = %lld must be in [1, min(dims[%d], %lld, 1024)]", i,
                        (long long)ranks[i], i, (long long)cols);
        if (!outs[i]) return fail(ctx, RP_ERR_INVALID_ARG, "%s[%d] is NULL", what, i);
    }
    if (reinterpret_cast<uintptr_t>(X) & 3) return fail(ctx, RP_ERR_INVALID_ARG, "X is not 4-byte aligned");
    return RP_OK;
}

// Lay out the modes and take their workspace (packed Omega, raw Omega, the
// mode-first copy, the transposed kernel's partial sums) from `ar`.
void hosvd_plan_modes(rp_ctx ctx, int N, const int64_t* dims, const float* X, const int64_t* ranks,
                      rp_omega_t omega_type, rp_algo_t algo, Arena& ar, HosvdModes& hm) {
    hm.N = N;
    hm.total = 1;
    for (int i = 0; i < N; ++i) hm.total *= dims[i];
    const int64_t total = hm.total;
    // mode-i unfolding of the C-order tensor: rows i_i, columns the C-order
    // index of the other modes = (leading index) * after + (trailing index);
    // element offset = i_i * after + lead * (dims[i] * after) + trail
    for (int i = N - 1, a = 1; i >= 0; --i) { hm.after[i] = a; a *= dims[i]; }
    for (int i = 0; i < N; ++i) hm.before[i] = total / (dims[i] * hm.after[i]);
    int64_t perm_elems = 0;
    const int cus = ctx->num_cus > 0 ? ctx->num_cus : 256;
    for (int i = 0; i < N; ++i) {
        const int64_t cols = total / dims[i], after = hm.after[i], before = hm.before[i];
        hm.desc[i] = rp_desc{X, dims[i], cols, after, after == 1 && before > 1 ? 1 : after, 1, dims[i] * after};
        if (before == 1) hm.desc[i].k_inner = cols;             // mode 1: plain row-major
        rp_status dummy;
        hm.permuted[i] = !(before == 1 || (after % rpmi::proj_k_block() == 0 && after > 1));
        if (!hm.permuted[i] && !proj_layout_ok(ctx, &hm.desc[i], &dummy)) hm.permuted[i] = true;
        hm.tn_mode[i] = hm.permuted[i] && algo == RP_ALGO_SPLIT_F16 && after == 1 && before > 1 &&
                        dims[i] % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
        if (hm.permuted[i] && !hm.tn_mode[i]) perm_elems = total;
        hm.tn_split_k[i] = 1;
        hm.tn_chunk[i] = 0;
        hm.o_tnp[i] = 0;
        if (hm.tn_mode[i]) {
            hm.tn_split_k[i] = rpmi::plan_tn_tcec_split(before, dims[i], ranks[i], cus, &hm.tn_chunk[i]);
            if (hm.tn_split_k[i] > 1)
                hm.o_tnp[i] = ar.take((size_t)hm.tn_split_k[i] * dims[i] * ranks[i] * sizeof(float));
        }
    }
    size_t rawb = 0;
    for (int i = 0; i < N; ++i) {
        const int64_t cols = total / dims[i];
        hm.pk[i] = packed_geometry(cols, ranks[i], algo, nullptr);
        hm.o_pk[i] = ar.take(packed_bytes(hm.pk[i], algo));
        const size_t rb = raw_bytes(omega_type, algo, cols, ranks[i]);
        rawb = rb > rawb ? rb : rawb;
    }
    hm.o_raw = ar.take(rawb);
    hm.o_perm = ar.take((size_t)perm_elems * 4);
}

// Launch every mode's projection into W[i] (dims[i] x ranks[i], ld ldw[i]).
rp_status hosvd_run_projections(rp_ctx ctx, HosvdModes& hm, const int64_t* dims, const float* X,
                                const int64_t* ranks, uint64_t seed, rp_omega_t omega_type, rp_algo_t algo,
                                float* const* W, const int64_t* ldw, hipStream_t s) {
    const int N = hm.N;
    char* base = static_cast<char*>(ctx->ws);
    float* perm = reinterpret_cast<float*>(base + hm.o_perm);
    rp_status st;
    // the Omega_i of this call stay in the cache until all of them are placed
    const uint64_t call_tick = ctx->omega_tick;
    for (int i = 0; i < N; ++i) {
        const int64_t cols = hm.total / dims[i];
        st = cached_packed_omega(ctx, seed, (uint32_t)i, omega_type, cols, ranks[i], algo, base + hm.o_raw, s,
                                 &hm.pk[i], call_tick);
        if (st == RP_ERR_UNSUPPORTED) {
            hm.pk[i].data = base + hm.o_pk[i];
            st = fill_packed(ctx, seed, (uint32_t)i, nullptr, 0, nullptr, omega_type, cols, ranks[i], algo, hm.pk[i],
                             base + hm.o_raw, s);
        }
        if (st != RP_OK) return st;
    }
    bool grouped_done = false;
    if (algo == RP_ALGO_SPLIT_F16) {
        const rp_desc* gA[rpmi::kMaxGroup];
        int64_t gr[rpmi::kMaxGroup], gld[rpmi::kMaxGroup];
        rpmi::PackedOmega gpk[rpmi::kMaxGroup];
        float* gY[rpmi::kMaxGroup];
        int cnt = 0;
        for (int i = 0; i < N; ++i) {
            if (hm.permuted[i]) continue;
            gA[cnt] = &hm.desc[i]; gr[cnt] = ranks[i]; gld[cnt] = ldw[i]; gpk[cnt] = hm.pk[i]; gY[cnt] = W[i];
            ++cnt;
        }
        if (cnt > 1) {
            st = launch_projection_grouped(ctx, cnt, gA, gr, gpk, gY, gld, s);
            if (st == RP_OK) grouped_done = true;
            else if (st != RP_ERR_UNSUPPORTED) return st;
        }
    }
    for (int i = 0; i < N; ++i) {
        if (hm.tn_mode[i]) {
            rpmi::TnTcecArgs t;
            t.A = X;
            t.lda = dims[i];
            t.m = hm.before[i];
            t.n = dims[i];
            t.p = ranks[i];
            t.qhi = hm.pk[i].data;
            t.qlo = nullptr;
            t.nt_count = hm.pk[i].nt_count;
            t.Z = W[i];
            t.ldz = ldw[i];
            t.status = ctx->d_status;
            t.ksplit = hm.tn_split_k[i];
            t.kchunk_steps = hm.tn_chunk[i];
            t.partial = hm.tn_split_k[i] > 1 ? reinterpret_cast<float*>(base + hm.o_tnp[i]) : nullptr;
            RP_HIP(ctx, rpmi::launch_gemm_tn_tcec(t, s));
        } else if (hm.permuted[i]) {
            RP_HIP(ctx, rpmi::launch_swap01(X, hm.before[i], dims[i], hm.after[i], perm, s));
            const int64_t cols = hm.total / dims[i];
            const rp_desc pd{perm, dims[i], cols, cols, cols, 1, 0};
            if ((st = launch_projection(ctx, &pd, ranks[i], hm.pk[i], algo, W[i], ldw[i], s)) != RP_OK) return st;
        } else if (!grouped_done) {
            if ((st = launch_projection(ctx, &hm.desc[i], ranks[i], hm.pk[i], algo, W[i], ldw[i], s)) != RP_OK)
                return st;
        }
    }
    return RP_OK;
}

}  // namespace

extern "C" {

rp_status rp_hosvd_project(rp_ctx ctx, int32_t ndim, const int64_t* dims, const float* X, const int64_t* ranks,
                           uint64_t seed, rp_omega_t omega_type, rp_algo_t algo, float* const* W, const int64_t* ldw,
                           void* stream) {
    rp_status st = hosvd_check(ctx, ndim, dims, X, ranks, omega_type, algo, W, "W");
    if (st != RP_OK) return st;
    if (!ldw) return fail(ctx, RP_ERR_INVALID_ARG, "ldw is NULL");
    for (int i = 0; i < ndim; ++i)
        if (ldw[i] < ranks[i]) return fail(ctx, RP_ERR_INVALID_ARG, "ldw[%d] < ranks[%d]", i, i);
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipSetDevice(ctx->device));
    Arena ar;
    HosvdModes hm;
    hosvd_plan_modes(ctx, ndim, dims, X, ranks, omega_type, algo, ar, hm);
    if ((st = ensure_workspace(ctx, ar.used)) != RP_OK) return st;
    return hosvd_run_projections(ctx, hm, dims, X, ranks, seed, omega_type, algo, W, ldw, s);
}

rp_status rp_hosvd(rp_ctx ctx, int32_t ndim, const int64_t* dims, const float* X, const int64_t* ranks,
                   uint64_t seed, rp_omega_t omega_type, rp_algo_t algo, float* core, float* const* factors,
                   void* stream) {
    rp_status st = hosvd_check(ctx, ndim, dims, X, ranks, omega_type, algo, factors, "factors");
    if (st != RP_OK) return st;
    if (!core) return fail(ctx, RP_ERR_INVALID_ARG, "NULL pointer");
    const int N = ndim;
    hipStream_t s = (hipStream_t)stream;
    RP_HIP(ctx, hipSetDevice(ctx->device));
    Arena ar;
    HosvdModes hm;
    hosvd_plan_modes(ctx, N, dims, X, ranks, omega_type, algo, ar, hm);
    const int64_t* after = hm.after;
    int64_t maxr = 0, maxd = 0;
    for (int i = 0; i < N; ++i) {
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
    size_t o_w[rpmi::kMaxGroup];
    for (int i = 0; i < N; ++i) o_w[i] = ar.take((size_t)dims[i] * ranks[i] * 4);
    const size_t o_qd = ar.take((size_t)maxd * maxr * 8);
    const size_t o_g = ar.take((size_t)maxr * maxr * 8);
    const size_t o_x = ar.take((size_t)maxr * maxr * 8);
    const size_t o_l1 = ar.take((size_t)maxr * maxr * 8);
    const size_t o_gp = ar.take((size_t)rpmi::kGramSplit * maxr * maxr * 8);
    const size_t o_t0 = ar.take((size_t)tmax * 4);
    const size_t o_t1 = ar.take((size_t)tmax * 4);
    // the first core contraction on the TCEC products (split algorithm, X on
    // their 16-byte path): Q_0 in TCEC fragment form
    const bool core_tcec = algo == RP_ALGO_SPLIT_F16 && N >= 2 && after[0] % 4 == 0 &&
                           (reinterpret_cast<uintptr_t>(X) & 15) == 0;
    rpmi::PackedOmega pkq0 = packed_geometry(dims[0], ranks[0], RP_ALGO_TCEC_F16, nullptr);
    const size_t o_pkq0 = ar.take(core_tcec ? packed_bytes(pkq0, RP_ALGO_TCEC_F16) : 0);
    if ((st = ensure_workspace(ctx, ar.used)) != RP_OK) return st;
    char* base = static_cast<char*>(ctx->ws);
    float* W[rpmi::kMaxGroup];
    int64_t ldw[rpmi::kMaxGroup];
    for (int i = 0; i < N; ++i) {
        W[i] = reinterpret_cast<float*>(base + o_w[i]);
        ldw[i] = ranks[i];
    }
    // Algorithm 2, first loop: W_i = X_(i) Omega_i, Omega_i from stream i
    if ((st = hosvd_run_projections(ctx, hm, dims, X, ranks, seed, omega_type, algo, W, ldw, s)) != RP_OK) return st;
    // Q_i = QR(W_i) straight into the caller's factors
    double* Qd = reinterpret_cast<double*>(base + o_qd);
    double* G = reinterpret_cast<double*>(base + o_g);
    double* Xs = reinterpret_cast<double*>(base + o_x);
    double* L1 = reinterpret_cast<double*>(base + o_l1);
    double* GP = reinterpret_cast<double*>(base + o_gp);
    for (int i = 0; i < N; ++i)
        if ((st = cholqr2(ctx, dims[i], ranks[i], W[i], ldw[i], factors[i], ranks[i], nullptr, Qd, G, Xs, L1, GP, s)) !=
            RP_OK)
            return st;
    // core g = X x_1 Q_1^T ... x_N Q_N^T, one mode at a time: T has shape
    // [lead, I_i, after_i]; out[b][j][p] = sum_k Q_i[k][j] T[b][k][p] (the
    // first mode on the TCEC products or FP32 MFMA, the others with FP64
    // accumulation)
    const float* T = X;
    float* bufs[2] = {reinterpret_cast<float*>(base + o_t0), reinterpret_cast<float*>(base + o_t1)};
    int64_t lead = 1;
    for (int i = 0; i < N; ++i) {
        float* out = i == N - 1 ? core : bufs[i & 1];
        const int64_t J = ranks[i], I = dims[i], P = after[i];
        if (P == 1) {
            RP_HIP(ctx, (rpmi::gemm_f32<float, float, float>(lead, J, I, 1.0, T, I, 1, factors[i], J, 1, 0.0, out, J, 1,
                                                              s)));
        } else if (lead == 1 && core_tcec) {
            // out (J x P) = (T^T Q_i)^T: Z = T^T Q_i (P x J, into the other
            // buffer, free until the next mode) on the TCEC products, then
            // transposed
            float* z = bufs[(i + 1) & 1];
            pkq0.data = base + o_pkq0;
            if ((st = gemm_at_q(ctx, I, P, J, T, P, factors[i], J, z, J, &pkq0, s)) != RP_OK) return st;
            RP_HIP(ctx, rpmi::launch_swap01(z, P, J, 1, out, s));
        } else if (lead == 1) {
            // out (J x P) = Q_i^T T: the A^T Q form on FP32 MFMA
            RP_HIP(ctx, rpmi::gemm_tn_f32(J, P, I, factors[i], J, T, P, out, P, s));
        } else {
            RP_HIP(ctx, (rpmi::gemm_f32_batched<float, float, float>(J, P, I, 1.0, factors[i], 1, J, 0, T, P, 1,
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
    // an Omega outside its range also makes the products non-finite: it is
    // reported first, as the cause
    *out = (word & rpmi::kStatusOmegaRange) ? RP_ERR_OMEGA_RANGE
         : (word & rpmi::kStatusRange) ? RP_ERR_RANGE
         : (word & rpmi::kStatusNotSpd) ? RP_ERR_NOT_SPD
         : (word & rpmi::kStatusNotConverged) ? RP_ERR_NOT_CONVERGED
         : RP_OK;
    return RP_OK;
}

}  // extern "C"
