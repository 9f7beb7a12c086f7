"""ctypes binding of libhsumma.so (the C ABI declared in include/hsumma.h).

Argument marshalling only: every step of the local update runs in the HIP
kernels of the library.  PyTorch supplies device memory and the stream.
If the library is missing the first call raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# HSUMMA_LIBRARY selects another build of the library (e.g. the host-sanitized
# libhsumma_asan.so of `python -m paper_1306_4161_amd.build --sanitize`)
LIB_PATH = os.environ.get("HSUMMA_LIBRARY") or os.path.join(HERE, "libhsumma.so")

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_DEVICE, ERR_WORKSPACE = 0, -1, -2, -3, -4
FP64, SPLIT_BF16, SPLIT_FP8, SPLIT_INT8 = 0, 1, 2, 3
DIST_BLOCK, DIST_BLOCK_CYCLIC = 0, 1

EXPORTED = [
    "hsumma_opts_default", "hsumma_plan", "hsumma_plan_destroy", "hsumma_workspace_size",
    "hsumma_num_steps", "hsumma_num_outer_steps", "hsumma_groups", "hsumma_tile_shape",
    "hsumma_step_info", "hsumma_num_items", "hsumma_tile_config", "hsumma_local_update",
    "hsumma_outer_update",
    "hsumma_run", "hsumma_panel_slices", "hsumma_last_error", "hsumma_version",
    "hsumma_split_layout", "hsumma_mfma_exact_probe", "hsumma_outer_products",
    "hsumma_work_items", "hsumma_prepare_workspace", "hsumma_run_noalloc",
    "hsumma_noalloc_max_workspace", "hsumma_lu_plan", "hsumma_lu_workspace_size", "hsumma_lu",
    "hsumma_lu_plan_destroy",
    "hsumma_mlp_param_count", "hsumma_mlp_work_floats", "hsumma_mlp_forward", "hsumma_mlp_grad",
    "hsumma_mlp_adam", "hsumma_model_bcast", "hsumma_model_cost", "hsumma_model_dcomm_dgroups",
    "hsumma_model_select_groups", "hsumma_model_cost_levels",
]

BCAST_BINOMIAL, BCAST_VAN_DE_GEIJN = 0, 1


class Platform(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double)]


class Cost(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in (
        "comp", "latency_inner", "latency_outer", "bandwidth_inner", "bandwidth_outer", "comm",
        "total")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Opts(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("k", ctypes.c_int64),
        ("dist", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("nb", ctypes.c_int64),
        ("slices", ctypes.c_int32), ("min_slices", ctypes.c_int32), ("max_slices", ctypes.c_int32),
        ("tile_m", ctypes.c_int32), ("tile_n", ctypes.c_int32), ("kc", ctypes.c_int32),
        ("persistent", ctypes.c_int32), ("use_graph", ctypes.c_int32),
        ("tau_bits", ctypes.c_int32), ("staged", ctypes.c_int32), ("waves", ctypes.c_int32),
        ("lookahead", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 1),
    ]


class HsummaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("hsumma error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """Load libhsumma.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # Share torch's HIP runtime: torch must be loaded before the library,
        # otherwise the library's own libamdhip64 is mapped first and torch
        # later maps a second runtime into the process.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhsumma.so not built: run `python -m paper_1306_4161_amd.build` "
                               "(the HIP library is required; there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        P = ctypes.POINTER
        L.hsumma_opts_default.argtypes = [P(Opts)]
        L.hsumma_opts_default.restype = None
        L.hsumma_plan.argtypes = [P(vp), i64, i32, i32, i32, i64, i64, P(Opts)]
        L.hsumma_plan_destroy.argtypes = [vp]
        L.hsumma_plan_destroy.restype = None
        L.hsumma_workspace_size.argtypes = [vp, P(ctypes.c_size_t)]
        L.hsumma_num_steps.argtypes = [vp, P(i64)]
        L.hsumma_num_outer_steps.argtypes = [vp, P(i64)]
        L.hsumma_num_items.argtypes = [vp, P(i64)]
        L.hsumma_groups.argtypes = [vp, P(i32), P(i32)]
        L.hsumma_tile_shape.argtypes = [vp, i32, i32, P(i64), P(i64)]
        L.hsumma_step_info.argtypes = [vp, i64, P(i64), P(i64), P(i64), P(i32), P(i32),
                                       P(i32), P(i32), P(i32), P(i32)]
        upd = [vp, i64, vp, i64, vp, i64, vp, i64, vp, ctypes.c_size_t, vp]
        L.hsumma_local_update.argtypes = upd
        L.hsumma_outer_update.argtypes = upd
        L.hsumma_run.argtypes = [vp, vp, i64, vp, i64, vp, i64, vp, ctypes.c_size_t, vp]
        L.hsumma_outer_products.argtypes = upd
        L.hsumma_work_items.argtypes = [vp, P(i32), i64]
        L.hsumma_prepare_workspace.argtypes = [vp, vp, ctypes.c_size_t, vp]
        L.hsumma_run_noalloc.argtypes = [vp, vp, i64, vp, i64, vp, i64, vp]
        L.hsumma_noalloc_max_workspace.argtypes = []
        L.hsumma_lu_plan.argtypes = [P(vp), i64, i32, i32, i32, i64, i64, P(Opts)]
        L.hsumma_lu_workspace_size.argtypes = [vp, P(ctypes.c_size_t)]
        L.hsumma_lu.argtypes = [vp, vp, i64, vp, ctypes.c_size_t, vp]
        L.hsumma_lu_plan_destroy.argtypes = [vp]
        L.hsumma_lu_plan_destroy.restype = None
        L.hsumma_panel_slices.argtypes = [vp, vp, P(i32), vp]
        sz = ctypes.c_size_t
        L.hsumma_split_layout.argtypes = [vp, P(sz), P(sz), P(sz), P(sz), P(i32), P(i32)]
        L.hsumma_mfma_exact_probe.argtypes = [i32, vp, vp, i32, vp, vp]
        L.hsumma_mlp_param_count.argtypes = [i32, i32, i32]
        L.hsumma_mlp_work_floats.argtypes = [i32, i32, i32]
        L.hsumma_mlp_forward.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp]
        L.hsumma_mlp_grad.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.hsumma_mlp_adam.argtypes = [i64, vp, vp, vp, vp, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, ctypes.c_float, i32, vp]
        dbl = ctypes.c_double
        L.hsumma_model_bcast.argtypes = [i32, P(Platform), dbl, dbl, P(dbl)]
        L.hsumma_model_cost.argtypes = [i32, P(Platform), i64, i32, i32, i32, i64, i64, P(Cost)]
        L.hsumma_model_dcomm_dgroups.argtypes = [P(Platform), i64, dbl, dbl, i64, P(dbl)]
        L.hsumma_model_select_groups.argtypes = [i32, P(Platform), i64, i32, i32, i64, i64, P(i32),
                                                 P(Cost), P(Cost)]
        L.hsumma_model_cost_levels.argtypes = [i32, P(Platform), i64, i32, i32, i32, P(i32), P(i32),
                                               P(i64), P(Cost), P(dbl)]
        L.hsumma_last_error.restype = ctypes.c_char_p
        L.hsumma_last_error.argtypes = []
        L.hsumma_version.restype = ctypes.c_char_p
        L.hsumma_version.argtypes = []
        for name in EXPORTED:
            if name not in ("hsumma_opts_default", "hsumma_plan_destroy",
                            "hsumma_lu_plan_destroy", "hsumma_last_error", "hsumma_version"):
                getattr(L, name).restype = ctypes.c_int
        L.hsumma_noalloc_max_workspace.restype = ctypes.c_size_t
        L.hsumma_mlp_param_count.restype = i64
        L.hsumma_mlp_work_floats.restype = i64
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise HsummaError(rc, lib().hsumma_last_error().decode())


def _dev_ptr(t, what):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % what)
    if t.device.type != "cuda":
        raise ValueError("%s must live on the GPU" % what)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % what)
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("%s must be a 2-D row-major view (unit column stride)" % what)
    return ctypes.c_void_p(t.data_ptr()), t.stride(0)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


WS_ALIGN = 4096   # workspace alignment the library recommends (256 is required)


def _aligned_bytes(nbytes, device):
    """A uint8 device tensor of nbytes starting on a WS_ALIGN boundary: a view
    into a slightly larger allocation (the caching allocator may hand out
    blocks at any 512-byte offset)."""
    import torch
    raw = torch.empty(nbytes + WS_ALIGN, dtype=torch.uint8, device=device)
    start = (-raw.data_ptr()) % WS_ALIGN
    return raw[start:start + nbytes]


class Plan:
    """Host plan for C = A x B on a virtual P x Q grid with G groups."""

    def __init__(self, n, P, Q, G, b, M=None, *, m=0, k=0, dist=DIST_BLOCK, nb=0,
                 prec=FP64, slices=0, min_slices=0, max_slices=0, tile_m=0, tile_n=0,
                 kc=0, persistent=0, use_graph=0, tau_bits=0, staged=0, waves=0,
                 wgs_per_cu=0, lookahead=0):
        L = lib()
        o = Opts()
        L.hsumma_opts_default(ctypes.byref(o))
        o.m, o.k, o.dist, o.nb, o.prec = m, k, dist, nb, prec
        o.slices, o.min_slices, o.max_slices = slices, min_slices, max_slices
        o.tile_m, o.tile_n, o.kc = tile_m, tile_n, kc
        o.persistent, o.use_graph, o.tau_bits, o.staged = persistent, use_graph, tau_bits, staged
        o.waves, o.wgs_per_cu, o.lookahead = waves, wgs_per_cu, lookahead
        h = ctypes.c_void_p()
        _check(L.hsumma_plan(ctypes.byref(h), n, P, Q, G, b, M if M is not None else b,
                             ctypes.byref(o)))
        self._h = h
        self.n, self.m, self.k = n, (m or n), (k or n)
        self.P, self.Q, self.G, self.b = P, Q, G, b
        self.M = M if M is not None else b
        self.prec = prec

    def close(self):
        if getattr(self, "_h", None):
            lib().hsumma_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- queries ---------------------------------------------------------
    def _i64(self, fn):
        v = ctypes.c_int64()
        _check(fn(self._h, ctypes.byref(v)))
        return v.value

    @property
    def num_steps(self):
        return self._i64(lib().hsumma_num_steps)

    @property
    def num_outer_steps(self):
        return self._i64(lib().hsumma_num_outer_steps)

    @property
    def num_items(self):
        return self._i64(lib().hsumma_num_items)

    @property
    def tile_config(self):
        """(tile_m, tile_n, kc, waves) of the plan's update kernels."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().hsumma_tile_config(self._h, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    @property
    def workspace_size(self):
        v = ctypes.c_size_t()
        _check(lib().hsumma_workspace_size(self._h, ctypes.byref(v)))
        return v.value

    @property
    def groups(self):
        I, J = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().hsumma_groups(self._h, ctypes.byref(I), ctypes.byref(J)))
        return I.value, J.value

    def tile_shape(self, pr, pc):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().hsumma_tile_shape(self._h, pr, pc, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def step_info(self, s):
        v64 = [ctypes.c_int64() for _ in range(3)]
        v32 = [ctypes.c_int32() for _ in range(6)]
        _check(lib().hsumma_step_info(self._h, s, *[ctypes.byref(x) for x in v64],
                                      *[ctypes.byref(x) for x in v32]))
        keys = ["k0", "k1", "outer", "owner_col", "owner_row", "group_col", "group_row",
                "in_group_col", "in_group_row"]
        return dict(zip(keys, [x.value for x in v64 + v32]))

    # ---- compute ---------------------------------------------------------
    def workspace(self, device="cuda"):
        """A device workspace of hsumma_workspace_size() bytes, 4 KiB-aligned
        (torch owns it)."""
        return _aligned_bytes(self.workspace_size, device)

    def _args(self, A, B, C, ws):
        a, lda = _dev_ptr(A, "A")
        b, ldb = _dev_ptr(B, "B")
        c, ldc = _dev_ptr(C, "C")
        if tuple(A.shape) != (self.m, self.k) or tuple(B.shape) != (self.k, self.n) \
                or tuple(C.shape) != (self.m, self.n):
            raise ValueError("operand shapes do not match the plan")
        wsp = ctypes.c_void_p(ws.data_ptr() if ws is not None else 0)
        wsn = ws.numel() * ws.element_size() if ws is not None else 0
        return a, lda, b, ldb, c, ldc, wsp, wsn

    def local_update(self, step, A, B, C, ws=None, stream=None):
        a, lda, b, ldb, c, ldc, wsp, wsn = self._args(A, B, C, ws)
        _check(lib().hsumma_local_update(self._h, step, a, lda, b, ldb, c, ldc, wsp, wsn,
                                         _stream(stream)))

    def outer_update(self, g, A, B, C, ws=None, stream=None):
        a, lda, b, ldb, c, ldc, wsp, wsn = self._args(A, B, C, ws)
        _check(lib().hsumma_outer_update(self._h, g, a, lda, b, ldb, c, ldc, wsp, wsn,
                                         _stream(stream)))

    def outer_products(self, g, A, B, C, ws, stream=None):
        """Split forms: the product launch of outer step g on the planes in ws."""
        a, lda, b, ldb, c, ldc, wsp, wsn = self._args(A, B, C, ws)
        _check(lib().hsumma_outer_products(self._h, g, a, lda, b, ldb, c, ldc, wsp, wsn,
                                           _stream(stream)))

    def work_items(self):
        """The plan's work-item table (host): int32 array (items, 4) of r0, c0, h, w."""
        import numpy as np
        n = self.num_items
        out = (ctypes.c_int32 * (4 * max(1, n)))()
        _check(lib().hsumma_work_items(self._h, out, n))
        return np.frombuffer(out, dtype=np.int32)[:4 * n].reshape(n, 4).copy()

    def prepare_workspace(self, ws, stream=None):
        """Write the work-item table into ws (as every compute call does first)."""
        _check(lib().hsumma_prepare_workspace(self._h, ctypes.c_void_p(ws.data_ptr()),
                                              ws.numel() * ws.element_size(), _stream(stream)))

    def run(self, A, B, C, ws=None, stream=None):
        a, lda, b, ldb, c, ldc, wsp, wsn = self._args(A, B, C, ws)
        _check(lib().hsumma_run(self._h, a, lda, b, ldb, c, ldc, wsp, wsn, _stream(stream)))

    def run_noalloc(self, A, B, C, stream=None):
        """C = A x B with the library's scratch array as workspace (no allocation)."""
        a, lda, b, ldb, c, ldc, _, _ = self._args(A, B, C, None)
        _check(lib().hsumma_run_noalloc(self._h, a, lda, b, ldb, c, ldc, _stream(stream)))

    def panel_slices(self, ws, stream=None):
        n = self.num_outer_steps
        out = (ctypes.c_int32 * n)()
        _check(lib().hsumma_panel_slices(self._h, ctypes.c_void_p(ws.data_ptr()), out,
                                         _stream(stream)))
        return list(out)


    def split_layout(self):
        v = [ctypes.c_size_t() for _ in range(4)]
        w, np_ = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().hsumma_split_layout(self._h, *[ctypes.byref(x) for x in v],
                                         ctypes.byref(w), ctypes.byref(np_)))
        return dict(off_digA=v[0].value, off_digB=v[1].value, off_eA=v[2].value,
                    off_fB=v[3].value, Wp=w.value, planes=np_.value)


class LuPlan:
    """LU factorisation without pivoting whose trailing update is the HSUMMA
    local update (see hsumma_lu in include/hsumma.h)."""

    def __init__(self, n, P, Q, G, b, M, *, prec=FP64, **kw):
        L = lib()
        o = Opts()
        L.hsumma_opts_default(ctypes.byref(o))
        o.prec = prec
        for key, val in kw.items():
            setattr(o, key, val)
        h = ctypes.c_void_p()
        _check(L.hsumma_lu_plan(ctypes.byref(h), n, P, Q, G, b, M, ctypes.byref(o)))
        self._h = h
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            lib().hsumma_lu_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_size(self):
        v = ctypes.c_size_t()
        _check(lib().hsumma_lu_workspace_size(self._h, ctypes.byref(v)))
        return v.value

    def workspace(self, device="cuda"):
        """A device workspace of hsumma_lu_workspace_size() bytes, 4 KiB-aligned."""
        return _aligned_bytes(self.workspace_size, device)

    def factor(self, A, ws, stream=None):
        """A = L U in place (A: n x n float64 CUDA tensor, row-major)."""
        a, lda = _dev_ptr(A, "A")
        if tuple(A.shape) != (self.n, self.n):
            raise ValueError("A must be n x n")
        _check(lib().hsumma_lu(self._h, a, lda, ctypes.c_void_p(ws.data_ptr()),
                               ws.numel() * ws.element_size(), _stream(stream)))


def mfma_exact_probe(fmt, a_digits, b_digits, stream=None):
    """32 x 32 FP32 product of digit matrices on the matrix cores (see header)."""
    import torch
    k = a_digits.shape[1]
    if a_digits.shape[0] != 32 or b_digits.shape != (k, 32):
        raise ValueError("the probe takes a 32 x k and a k x 32 digit matrix")
    d = torch.empty((32, 32), dtype=torch.float32, device="cuda")
    _check(lib().hsumma_mfma_exact_probe(fmt, ctypes.c_void_p(a_digits.data_ptr()),
                                         ctypes.c_void_p(b_digits.data_ptr()), k,
                                         ctypes.c_void_p(d.data_ptr()), _stream(stream)))
    return d


def _f32_ptr(t, what, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32 \
            or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float32 CUDA tensor" % what)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %r, expected %r" % (what, tuple(t.shape), tuple(shape)))
    return ctypes.c_void_p(t.data_ptr())


def mlp_param_count(F, H, K):
    return int(lib().hsumma_mlp_param_count(F, H, K))


def mlp_work(N, H, K):
    import torch
    return torch.empty(int(lib().hsumma_mlp_work_floats(N, H, K)), dtype=torch.float32,
                       device="cuda")


def mlp_forward(X, params, H, K, work=None, stream=None):
    """Z = network(X) on the GPU (see hsumma_mlp_forward)."""
    import torch
    N, F = X.shape
    Z = torch.empty((N, K), dtype=torch.float32, device="cuda")
    work = mlp_work(N, H, K) if work is None else work
    _check(lib().hsumma_mlp_forward(N, F, H, K, _f32_ptr(X, "X"),
                                    _f32_ptr(params, "params", (mlp_param_count(F, H, K),)),
                                    _f32_ptr(Z, "Z"), _f32_ptr(work, "work"), _stream(stream)))
    return Z


def mlp_grad(X, T, mask, params, H, K, grads=None, work=None, stream=None):
    """(loss tensor on device, grads, Z) of the masked MSE (see hsumma_mlp_grad)."""
    import torch
    N, F = X.shape
    n = mlp_param_count(F, H, K)
    grads = torch.empty(n, dtype=torch.float32, device="cuda") if grads is None else grads
    Z = torch.empty((N, K), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    work = mlp_work(N, H, K) if work is None else work
    _check(lib().hsumma_mlp_grad(N, F, H, K, _f32_ptr(X, "X"), _f32_ptr(T, "T", (N, K)),
                                 _f32_ptr(mask, "mask", (N, K)), _f32_ptr(params, "params", (n,)),
                                 _f32_ptr(grads, "grads", (n,)), _f32_ptr(Z, "Z"),
                                 _f32_ptr(loss, "loss"), _f32_ptr(work, "work"), _stream(stream)))
    return loss, grads, Z


def mlp_adam(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    n = params.numel()
    _check(lib().hsumma_mlp_adam(n, _f32_ptr(params, "params"), _f32_ptr(grads, "grads"),
                                 _f32_ptr(m, "m"), _f32_ptr(v, "v"), lr, beta1, beta2, eps, step,
                                 _stream(stream)))


def version():
    return lib().hsumma_version().decode()


# -- communication-cost model (host only) ---------------------------------------

def model_bcast(algo, alpha, beta, m, q):
    """Seconds for one broadcast of m elements among q processes."""
    out = ctypes.c_double()
    pf = Platform(alpha, beta, 0.0)
    _check(lib().hsumma_model_bcast(algo, ctypes.byref(pf), float(m), float(q), ctypes.byref(out)))
    return out.value


def model_cost(algo, alpha, beta, gamma, n, P, Q, G, b, B):
    """Modelled cost (seconds) of C = A x B, n x n, on a P x Q grid with G groups."""
    c = Cost()
    pf = Platform(alpha, beta, gamma)
    _check(lib().hsumma_model_cost(algo, ctypes.byref(pf), n, P, Q, G, b, B, ctypes.byref(c)))
    return c.as_dict()


def model_dcomm_dgroups(alpha, beta, n, p, G, b):
    """Eq. (10): d(communication)/dG, Van de Geijn broadcasts, square grid, b = B."""
    out = ctypes.c_double()
    pf = Platform(alpha, beta, 0.0)
    _check(lib().hsumma_model_dcomm_dgroups(ctypes.byref(pf), n, float(p), float(G), b,
                                            ctypes.byref(out)))
    return out.value


def model_select_groups(algo, alpha, beta, gamma, n, P, Q, b, B):
    """(G with the least modelled communication, its cost, SUMMA's cost)."""
    g = ctypes.c_int32()
    best, summa = Cost(), Cost()
    pf = Platform(alpha, beta, gamma)
    _check(lib().hsumma_model_select_groups(algo, ctypes.byref(pf), n, P, Q, b, B, ctypes.byref(g),
                                            ctypes.byref(best), ctypes.byref(summa)))
    return g.value, best.as_dict(), summa.as_dict()


def model_cost_levels(algo, alpha, beta, gamma, n, P, Q, Is, Js, blocks):
    """(cost, per-level seconds) of a hierarchy of len(Is) levels, outermost first."""
    k = len(Is)
    if len(Js) != k or len(blocks) != k:
        raise ValueError("one I, J and block per level")
    ia = (ctypes.c_int32 * k)(*Is)
    ja = (ctypes.c_int32 * k)(*Js)
    ba = (ctypes.c_int64 * k)(*blocks)
    per = (ctypes.c_double * k)()
    c = Cost()
    pf = Platform(alpha, beta, gamma)
    _check(lib().hsumma_model_cost_levels(algo, ctypes.byref(pf), n, P, Q, k, ia, ja, ba,
                                          ctypes.byref(c), per))
    return c.as_dict(), list(per)
