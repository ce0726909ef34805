"""Mixed-precision random projection for RandNLA on AMD MI355X (gfx950).

Thin ctypes binding over the C ABI of ``librpmi.so`` (include/rpmi.h).  The
functions carry the C names; they only marshal arguments (torch tensors give
device pointers, the current torch stream gives the HIP stream).  Every step
of the computation runs in the library's HIP kernels; there is no fallback:
if the library is missing or fails to load, every call raises.
"""
import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librpmi.so")

RP_OK = 0
RP_ERR_INVALID_ARG = 1
RP_ERR_UNSUPPORTED = 2
RP_ERR_RANGE = 3
RP_ERR_NOT_SPD = 4
RP_ERR_NOT_CONVERGED = 5
RP_ERR_NOMEM = 6
RP_ERR_HIP = 7
RP_ERR_OMEGA_RANGE = 8

RP_OMEGA_F32 = 0
RP_OMEGA_F16 = 1
RP_OMEGA_E4M3 = 2
RP_OMEGA_SPARSE1 = 3
RP_OMEGA_SPARSE3 = 4
RP_OMEGA_VSPARSE = 5
RP_ALGO_F32 = 0
RP_ALGO_SPLIT_F16 = 1
RP_ALGO_TCEC_F16 = 2

OMEGA_TYPES = {"f32": RP_OMEGA_F32, "f16": RP_OMEGA_F16, "e4m3": RP_OMEGA_E4M3, "sparse1": RP_OMEGA_SPARSE1,
               "sparse3": RP_OMEGA_SPARSE3, "vsparse": RP_OMEGA_VSPARSE}
ALGOS = {"f32": RP_ALGO_F32, "split_f16": RP_ALGO_SPLIT_F16, "tcec_f16": RP_ALGO_TCEC_F16}
RP_A_SCALE_AUTO_ROW = 32767   # a_scale_exp: one power-of-two pre-scale per row of A, chosen on the device


class RpError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


class rp_desc(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("s_row", ctypes.c_int64), ("k_inner", ctypes.c_int64),
                ("s_k_inner", ctypes.c_int64), ("s_k_outer", ctypes.c_int64)]


class rp_project_problem(ctypes.Structure):
    _fields_ = [("A", rp_desc), ("r", ctypes.c_int64), ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32),
                ("Y", ctypes.c_void_p), ("ldy", ctypes.c_int64), ("a_scale_exp", ctypes.c_int32)]


class rp_rsvd_problem(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("k", ctypes.c_int64), ("oversample", ctypes.c_int64), ("U", ctypes.c_void_p),
                ("ldu", ctypes.c_int64), ("S", ctypes.c_void_p), ("VT", ctypes.c_void_p), ("ldvt", ctypes.c_int64)]


_lib = None


def lib():
    """Load librpmi.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2304_04612_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, u64, u32, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    sig = {
        "rp_create": [ctypes.POINTER(vp), i32],
        "rp_destroy": [vp],
        "rp_status_string": [i32],
        "rp_last_error": [vp],
        "rp_omega_generate": [vp, u64, u32, i64, i64, i32, vp, i64, vp],
        "rp_project": [vp, ctypes.POINTER(rp_desc), i64, i32, u64, u32, vp, i64, vp, i32, i32, vp, i64, vp],
        "rp_split_f16": [vp, vp, i64, vp, vp, vp],
        "rp_omega_packed_size": [i64, i64, i32, ctypes.POINTER(ctypes.c_size_t)],
        "rp_omega_pack": [vp, u64, u32, vp, i64, vp, i32, i64, i64, i32, vp, vp],
        "rp_project_packed": [vp, ctypes.POINTER(rp_desc), i64, vp, i32, i32, vp, i64, vp],
        "rp_project_packed_noalloc": [vp, ctypes.POINTER(rp_desc), i64, vp, i32, i32, vp, i64, vp],
        "rp_gemm_tn": [vp, i64, i64, i64, vp, i64, vp, i64, i32, vp, i64, vp],
        "rp_get_device_status": [vp, vp, i32, ctypes.POINTER(i32)],
        "rsvd": [vp, i64, i64, vp, i64, i64, i64, i32, u64, i32, i32, i32, vp, i64, vp, vp, i64, vp,
                 ctypes.c_size_t, vp],
        "rsvd_workspace_size": [vp, i64, i64, i64, i64, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)],
        "rp_hosvd": [vp, i32, vp, vp, vp, u64, i32, i32, vp, vp, vp],
        "rp_hosvd_project": [vp, i32, vp, vp, vp, u64, i32, i32, vp, vp, vp],
        "rp_project_grouped": [vp, i32, vp, i32, vp],
        "rp_omega_generate_e4m3": [vp, u64, u32, i64, i64, vp, i64, vp, vp],
        "rsvd_batched": [vp, i32, vp, i32, u64, i32, vp],
        "rp_tuning_save": [vp, ctypes.c_char_p],
        "rp_tuning_load": [vp, ctypes.c_char_p],
        "rp_tuning_count": [vp, ctypes.POINTER(i64)],
        "rpmi_build_f16_thresholds": [vp, i32],
        "rpmi_build_guide": [vp, i32, vp, i32],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name in ("rp_status_string", "rp_last_error") else i32
    L.rpmi_build_guide.restype = None
    _lib = L
    return L


def status_string(s):
    return lib().rp_status_string(int(s)).decode()


def _check(ctx_handle, status):
    if status != RP_OK:
        msg = lib().rp_last_error(ctx_handle)
        raise RpError(status, msg.decode() if msg else "")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Context:
    """An rp_ctx on one HIP device (rp_create / rp_destroy)."""

    def __init__(self, device=0):
        h = ctypes.c_void_p()
        _check(None, lib().rp_create(ctypes.byref(h), int(device)))
        self.handle = h
        self.device = int(device)

    def close(self):
        if self.handle:
            lib().rp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def default_context(device=None):
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _default:
        _default[dev] = Context(dev)
    return _default[dev]


def desc_from_tensor(a, k_inner=None, s_k_outer=0, rows=None, cols=None, s_row=None):
    """rp_desc for a 2-D FP32 CUDA tensor with unit column stride (or an
    explicit unfolding layout)."""
    import torch
    if a.dtype != torch.float32 or not a.is_cuda:
        raise TypeError("A must be a float32 CUDA tensor")
    if rows is None:
        if a.dim() == 2 and a.numel() == 0:
            rows, cols, s_row = a.shape[0], a.shape[1], max(a.shape[1], 1)
        elif a.dim() != 2 or a.stride(1) != 1:
            raise ValueError("A must be 2-D with unit column stride (or give an explicit layout)")
        else:
            rows, cols, s_row = a.shape[0], a.shape[1], a.stride(0)
    k_inner = cols if k_inner is None else k_inner
    return rp_desc(a.data_ptr(), rows, cols, s_row, max(k_inner, 1), 1, s_k_outer)


def rp_omega_generate(n, r, seed, stream_id=0, omega="f16", out=None, ctx=None):
    """Omega (n x r) for (seed, stream_id): FP16 bits (int16) for the FP16
    and sparse types, float32 for "f32"."""
    import torch
    ctx = ctx or default_context()
    t = OMEGA_TYPES[omega]
    if out is None:
        out = torch.empty((n, r), dtype=torch.float32 if t == RP_OMEGA_F32 else torch.int16,
                          device=f"cuda:{ctx.device}")
    ldo = out.stride(0) if out.dim() == 2 and out.numel() else r
    _check(ctx.handle, lib().rp_omega_generate(ctx.handle, seed, stream_id, n, r, t, _ptr(out),
                                               ldo, _stream()))
    return out


def rp_project(a, r, seed=0, stream_id=0, omega=None, omega_type="f16", algo="split_f16",
               y=None, desc=None, col_scale=None, a_scale_exp=0, ctx=None):
    """Y = A Omega.  ``a``: float32 CUDA tensor (or ``desc`` for an unfolding
    layout, with ``a`` keeping the storage alive).  ``omega``: optional
    caller-supplied Omega (int16 FP16 bits, float32, or uint8 e4m3 codes with
    ``col_scale``, n x r).  ``a_scale_exp``: s, the split takes 2^s A."""
    import torch
    ctx = ctx or default_context()
    d = desc if desc is not None else desc_from_tensor(a)
    if y is None:
        y = torch.empty((d.rows, r), dtype=torch.float32, device=f"cuda:{ctx.device}")
    ldy = y.stride(0) if y.numel() else max(r, 1)
    ldo = omega.stride(0) if omega is not None and omega.numel() else max(r, 1)
    _check(ctx.handle, lib().rp_project(ctx.handle, ctypes.byref(d), r, OMEGA_TYPES[omega_type],
                                        seed, stream_id, _ptr(omega), ldo, _ptr(col_scale), ALGOS[algo],
                                        int(a_scale_exp), _ptr(y), ldy, _stream()))
    return y


def rp_omega_packed_size(n, r, algo="split_f16"):
    out = ctypes.c_size_t(0)
    _check(None, lib().rp_omega_packed_size(n, r, ALGOS[algo], ctypes.byref(out)))
    return out.value


def rp_omega_pack(n, r, seed=0, stream_id=0, omega=None, omega_type="f16", algo="split_f16",
                  out=None, col_scale=None, ctx=None):
    """Omega in the kernels' fragment order (a uint8 device buffer)."""
    import torch
    ctx = ctx or default_context()
    if out is None:
        out = torch.empty(rp_omega_packed_size(n, r, algo), dtype=torch.uint8,
                          device=f"cuda:{ctx.device}")
    ldo = omega.stride(0) if omega is not None and omega.numel() else max(r, 1)
    _check(ctx.handle, lib().rp_omega_pack(ctx.handle, seed, stream_id, _ptr(omega), ldo, _ptr(col_scale),
                                           OMEGA_TYPES[omega_type], n, r, ALGOS[algo], _ptr(out),
                                           _stream()))
    return out


def rp_project_packed(a, r, packed, algo="split_f16", y=None, desc=None, a_scale_exp=0, ctx=None):
    """Y = A Omega with Omega from rp_omega_pack (one kernel launch)."""
    import torch
    ctx = ctx or default_context()
    d = desc if desc is not None else desc_from_tensor(a)
    if y is None:
        y = torch.empty((d.rows, r), dtype=torch.float32, device=f"cuda:{ctx.device}")
    ldy = y.stride(0) if y.numel() else max(r, 1)
    _check(ctx.handle, lib().rp_project_packed(ctx.handle, ctypes.byref(d), r, _ptr(packed),
                                               ALGOS[algo], int(a_scale_exp), _ptr(y), ldy, _stream()))
    return y


def rp_project_packed_noalloc(a, r, packed, y, algo="split_f16", desc=None, a_scale_exp=0, ctx=None):
    """rp_project_packed into a caller-allocated y, with the library's static
    scratch instead of any device allocation."""
    ctx = ctx or default_context()
    d = desc if desc is not None else desc_from_tensor(a)
    ldy = y.stride(0) if y.numel() else max(r, 1)
    _check(ctx.handle, lib().rp_project_packed_noalloc(ctx.handle, ctypes.byref(d), r, _ptr(packed), ALGOS[algo],
                                                       int(a_scale_exp), _ptr(y), ldy, _stream()))
    return y


def rp_gemm_tn(a, q, algo="tcec_f16", z=None, ctx=None):
    """Z = A^T Q for float32 CUDA tensors a (m x n) and q (m x p), row-major
    with unit column stride; returns z (n x p)."""
    import torch
    ctx = ctx or default_context()
    m, n = a.shape
    p = q.shape[1]
    if z is None:
        z = torch.empty((n, p), dtype=torch.float32, device=a.device)
    _check(ctx.handle, lib().rp_gemm_tn(ctx.handle, m, n, p, _ptr(a), a.stride(0) if a.numel() else max(n, 1),
                                        _ptr(q), q.stride(0) if q.numel() else max(p, 1), ALGOS[algo], _ptr(z),
                                        z.stride(0) if z.numel() else max(p, 1), _stream()))
    return z


def rp_split_f16(x, ctx=None):
    """(hi, lo) FP16 bit patterns (int16 tensors) of the split of float32 x."""
    import torch
    ctx = ctx or default_context()
    x = x.contiguous()
    hi = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    lo = torch.empty(x.shape, dtype=torch.int16, device=x.device)
    _check(ctx.handle, lib().rp_split_f16(ctx.handle, _ptr(x), x.numel(), _ptr(hi), _ptr(lo), _stream()))
    return hi, lo


def rsvd_workspace_size(m, n, k, oversample=10, power_iters=0, omega_type="f16", algo="split_f16", ctx=None):
    """Bytes of caller workspace rsvd() needs for these arguments."""
    ctx = ctx or default_context()
    out = ctypes.c_size_t(0)
    _check(ctx.handle, lib().rsvd_workspace_size(ctx.handle, m, n, k, oversample, power_iters,
                                                 OMEGA_TYPES[omega_type], ALGOS[algo], ctypes.byref(out)))
    return out.value


def rsvd(a, k, oversample=10, power_iters=0, seed=0, omega_type="f16", algo="split_f16", a_scale_exp=0,
         work=None, outputs=None, ctx=None):
    """Randomized SVD (Algorithm 1) of the float32 CUDA matrix ``a`` (m x n).
    ``work``: optional caller workspace (a CUDA tensor of at least
    rsvd_workspace_size() bytes); None uses the context workspace.
    Returns (U m x k float32, S k float64, VT k x n float32)."""
    import torch
    ctx = ctx or default_context()
    if a.dtype != torch.float32 or not a.is_cuda or a.dim() != 2 or a.stride(1) != 1:
        raise TypeError("a must be a 2-D float32 CUDA tensor with unit column stride")
    m, n = a.shape
    dev = f"cuda:{ctx.device}"
    if outputs is not None:
        u, sv, vt = outputs
    else:
        u = torch.empty((m, k), dtype=torch.float32, device=dev)
        sv = torch.empty((k,), dtype=torch.float64, device=dev)
        vt = torch.empty((k, n), dtype=torch.float32, device=dev)
    wbytes = work.numel() * work.element_size() if work is not None else 0
    _check(ctx.handle, lib().rsvd(ctx.handle, m, n, _ptr(a), a.stride(0), k, oversample, power_iters, seed,
                                  OMEGA_TYPES[omega_type], ALGOS[algo], int(a_scale_exp), _ptr(u), u.stride(0),
                                  _ptr(sv), _ptr(vt), vt.stride(0), _ptr(work), wbytes, _stream()))
    return u, sv, vt


def rp_hosvd(x, ranks, seed=0, omega_type="f16", algo="split_f16", ctx=None):
    """Random-projection HOSVD (Algorithm 2) of the C-contiguous float32 CUDA
    tensor ``x`` with per-mode ranks; Omega_i from stream i.  Returns
    (core float32 of shape ranks, [factor_i float32 dims[i] x ranks[i]])."""
    import torch
    ctx = ctx or default_context()
    if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
        raise TypeError("x must be a C-contiguous float32 CUDA tensor")
    nd = x.dim()
    ranks = [int(r) for r in ranks]
    if len(ranks) != nd:
        raise ValueError("one rank per mode")
    dev = f"cuda:{ctx.device}"
    core = torch.empty(ranks, dtype=torch.float32, device=dev)
    factors = [torch.empty((x.shape[i], ranks[i]), dtype=torch.float32, device=dev) for i in range(nd)]
    dims_c = (ctypes.c_int64 * nd)(*x.shape)
    ranks_c = (ctypes.c_int64 * nd)(*ranks)
    fac_c = (ctypes.c_void_p * nd)(*[_ptr(f) for f in factors])
    _check(ctx.handle, lib().rp_hosvd(ctx.handle, nd, dims_c, _ptr(x), ranks_c, seed, OMEGA_TYPES[omega_type],
                                      ALGOS[algo], _ptr(core), fac_c, _stream()))
    return core, factors


def rp_hosvd_project(x, ranks, seed=0, omega_type="f16", algo="split_f16", out=None, ctx=None):
    """Algorithm 2 line 2 alone: [W_i = X_(i) Omega_i] (float32 dims[i] x
    ranks[i]) for the C-contiguous float32 CUDA tensor ``x``."""
    import torch
    ctx = ctx or default_context()
    if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
        raise TypeError("x must be a C-contiguous float32 CUDA tensor")
    nd = x.dim()
    ranks = [int(r) for r in ranks]
    if len(ranks) != nd:
        raise ValueError("one rank per mode")
    dev = f"cuda:{ctx.device}"
    ws = out if out is not None else [torch.empty((x.shape[i], ranks[i]), dtype=torch.float32, device=dev)
                                      for i in range(nd)]
    dims_c = (ctypes.c_int64 * nd)(*x.shape)
    ranks_c = (ctypes.c_int64 * nd)(*ranks)
    w_c = (ctypes.c_void_p * nd)(*[_ptr(w) for w in ws])
    ld_c = (ctypes.c_int64 * nd)(*[w.stride(0) for w in ws])
    _check(ctx.handle, lib().rp_hosvd_project(ctx.handle, nd, dims_c, _ptr(x), ranks_c, seed, OMEGA_TYPES[omega_type],
                                              ALGOS[algo], w_c, ld_c, _stream()))
    return ws


def rp_omega_generate_e4m3(n, r, seed=0, stream_id=0, ctx=None):
    """e4m3 Omega: (codes uint8 n x r, column scales float32 r)."""
    import torch
    ctx = ctx or default_context()
    dev = f"cuda:{ctx.device}"
    codes = torch.empty((n, r), dtype=torch.uint8, device=dev)
    scale = torch.empty((r,), dtype=torch.float32, device=dev)
    _check(ctx.handle, lib().rp_omega_generate_e4m3(ctx.handle, seed, stream_id, n, r, _ptr(codes), max(r, 1),
                                                    _ptr(scale), _stream()))
    return codes, scale


def rp_project_grouped(problems, omega_type="f16", ctx=None):
    """Grouped split-FP16 projections.  ``problems``: list of (a, r, seed,
    stream_id[, a_scale_exp]) with ``a`` a 2-D float32 CUDA tensor (unit
    column stride).  Returns the list of Y (float32, rows(a) x r)."""
    import torch
    ctx = ctx or default_context()
    n = len(problems)
    arr = (rp_project_problem * max(n, 1))()
    ys = []
    for i, prob in enumerate(problems):
        a, r, seed, sid = prob[:4]
        y = torch.empty((a.shape[0], r), dtype=torch.float32, device=f"cuda:{ctx.device}")
        ys.append(y)
        arr[i].A = desc_from_tensor(a)
        arr[i].r, arr[i].seed, arr[i].stream_id = r, seed, sid
        arr[i].a_scale_exp = int(prob[4]) if len(prob) > 4 else 0
        arr[i].Y, arr[i].ldy = _ptr(y), max(r, 1)
    _check(ctx.handle, lib().rp_project_grouped(ctx.handle, n, arr, OMEGA_TYPES[omega_type], _stream()))
    return ys


def rsvd_batched(mats, ks, oversamples, power_iters=0, seed=0, omega_type="f16", outputs=None, ctx=None):
    """Batched randomized SVD (Algorithm 1 per matrix; Omega_j from stream j).
    ``mats``: list of 2-D float32 CUDA tensors.  ``outputs``: optional list of
    (U, S, VT) to write into (a repeated call with the same tensors replays the
    captured graph).  Returns the list of (U, S, VT)."""
    import torch
    ctx = ctx or default_context()
    n = len(mats)
    arr = (rp_rsvd_problem * max(n, 1))()
    outs = []
    dev = f"cuda:{ctx.device}"
    for i, a in enumerate(mats):
        if a.dtype != torch.float32 or not a.is_cuda or a.dim() != 2 or a.stride(1) != 1:
            raise TypeError("matrices must be 2-D float32 CUDA tensors with unit column stride")
        m, nn = a.shape
        k = ks[i]
        if outputs is not None:
            u, sv, vt = outputs[i]
        else:
            u = torch.empty((m, k), dtype=torch.float32, device=dev)
            sv = torch.empty((k,), dtype=torch.float64, device=dev)
            vt = torch.empty((k, nn), dtype=torch.float32, device=dev)
        outs.append((u, sv, vt))
        arr[i].m, arr[i].n, arr[i].A, arr[i].lda = m, nn, _ptr(a), a.stride(0)
        arr[i].k, arr[i].oversample = k, oversamples[i]
        arr[i].U, arr[i].ldu, arr[i].S = _ptr(u), u.stride(0), _ptr(sv)
        arr[i].VT, arr[i].ldvt = _ptr(vt), vt.stride(0)
    _check(ctx.handle, lib().rsvd_batched(ctx.handle, n, arr, power_iters, seed, OMEGA_TYPES[omega_type], _stream()))
    return outs


def rp_tuning_save(path, ctx=None):
    """Write the context's autotuner entries to ``path``."""
    ctx = ctx or default_context()
    _check(ctx.handle, lib().rp_tuning_save(ctx.handle, os.fsencode(path)))


def rp_tuning_load(path, ctx=None):
    """Add the autotuner entries of ``path`` to the context."""
    ctx = ctx or default_context()
    _check(ctx.handle, lib().rp_tuning_load(ctx.handle, os.fsencode(path)))


def rp_tuning_count(ctx=None):
    ctx = ctx or default_context()
    out = ctypes.c_int64(0)
    _check(ctx.handle, lib().rp_tuning_count(ctx.handle, ctypes.byref(out)))
    return out.value


def rp_get_device_status(clear=True, ctx=None):
    ctx = ctx or default_context()
    out = ctypes.c_int(0)
    _check(ctx.handle, lib().rp_get_device_status(ctx.handle, _stream(), int(clear), ctypes.byref(out)))
    return out.value
