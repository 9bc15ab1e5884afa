"""ctypes binding of libwenott (the C ABI in include/wenott.h).

Argument marshalling only: every step of the WENO-TT path runs in the HIP library.
Importing this module does not touch the GPU; the first call that needs the library
loads it and raises if it has not been built.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwenott.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ENONPHYS, ENAN, ENOTBUILT = 0, -1, -2, -3, -4, -5, -6, -7
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1

EXPORTED = ["wenott_default_opts", "wenott_init", "wenott_rhs", "wenott_rk3_step", "wenott_round",
            "wenott_to_dense", "wenott_get_state", "wenott_get_info", "wenott_max_wavespeed",
            "wenott_current_eps", "wenott_set_profiling", "wenott_last_error", "wenott_destroy",
            "wenott_strerror", "wenott_dense_init", "wenott_dense_max_wavespeed", "wenott_dense_rhs",
            "wenott_dense_rk3_step", "wenott_dense_destroy", "wenott_mlp_nparams", "wenott_mlp_workspace",
            "wenott_mlp_init_params", "wenott_mlp_forward", "wenott_mlp_loss_grad", "wenott_mlp_adam_step",
            "wenott_set_proposal", "wenott_set_cross_logging", "wenott_get_cross_log", "wenott_batch_rk3_step",
            "wenott_gemm_autotune", "wenott_gemm_autotune_table", "wenott_set_pivot_wait_limit", "wenott_finalize",
            "wenott_pivot_layout", "wenott_pivot_search", "wenott_max_wavespeed_noalloc", "wenott_set_inflow"]

MLP_IN, MLP_HID, MLP_OUT, MLP_RANK_CLASSES, MLP_BINS = 96, 128, 81, 17, 64


class wenott_grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("pad_", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
                ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3)]


class wenott_tt(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("ncomp", ctypes.c_int32), ("ranks", ctypes.POINTER(ctypes.c_int64)),
                ("cores", ctypes.POINTER(ctypes.c_void_p)), ("dtype", ctypes.c_int32), ("on_device", ctypes.c_int32)]


class wenott_opts(ctypes.Structure):
    _fields_ = [("c_eps", ctypes.c_double), ("eps0", ctypes.c_double), ("eps_mode", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("max_sweeps", ctypes.c_int32), ("kick_rank", ctypes.c_int32),
                ("rank_cap", ctypes.c_int32), ("probe_points", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("alpha_mode", ctypes.c_int32), ("use_proposal", ctypes.c_int32), ("alpha_given", ctypes.c_double),
                ("rounds_per_stage", ctypes.c_int32), ("graph_mode", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("conv_slack", ctypes.c_double), ("law", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("cross_ratio", ctypes.c_double)]


LAW_EULER, LAW_LINADV, LAW_BURGERS = 0, 1, 2


class wenott_info(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("ncomp", ctypes.c_int32), ("ranks", ctypes.c_int64 * 4),
                ("alpha", ctypes.c_double * 3), ("eps", ctypes.c_double), ("c_eps", ctypes.c_double),
                ("max_norm", ctypes.c_double), ("sweeps", (ctypes.c_int32 * 3) * 3),
                ("residual", (ctypes.c_double * 3) * 3), ("flux_rank", (ctypes.c_int64 * 3) * 3),
                ("sum_rank", ctypes.c_int64 * 3), ("fiber_points", ctypes.c_int64), ("fiber_ms", ctypes.c_double),
                ("fiber_launches", ctypes.c_int64), ("step_ms", ctypes.c_double),
                ("class_ms", ctypes.c_double * 4), ("class_launches", ctypes.c_int64 * 4),
                ("class_flops", ctypes.c_double * 4), ("class_bytes", ctypes.c_double * 4),
                ("proposals_tried", ctypes.c_int64), ("proposals_accepted", ctypes.c_int64),
                ("pivots_total", ctypes.c_int64), ("rank_capped", ctypes.c_int64),
                ("pivot_fallbacks", ctypes.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libwenott.so; raises RuntimeError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libwenott.so is not built ({path}); run paper_2405_12301_amd/build.py")
    # torch ships its own HIP runtime with the same SONAME as the system one; importing it
    # first makes the library bind to that already-loaded runtime (one runtime per process).
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    lib.wenott_default_opts.argtypes = [P(wenott_opts)]
    lib.wenott_default_opts.restype = None
    lib.wenott_init.argtypes = [P(vp), P(wenott_tt), P(wenott_grid), ctypes.c_double, P(ctypes.c_int32),
                                P(wenott_opts), vp]
    lib.wenott_rhs.argtypes = [vp, ctypes.c_double, P(wenott_tt)]
    lib.wenott_rk3_step.argtypes = [vp, ctypes.c_double, ctypes.c_double, P(ctypes.c_double)]
    lib.wenott_batch_rk3_step.argtypes = [P(vp), ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_double)]
    lib.wenott_round.argtypes = [vp, ctypes.c_double]
    lib.wenott_gemm_autotune.argtypes = [ctypes.c_int32]
    lib.wenott_gemm_autotune_table.argtypes = [P(ctypes.c_int32), ctypes.c_int32, P(ctypes.c_int32)]
    lib.wenott_to_dense.argtypes = [vp, vp, ctypes.c_int32]
    lib.wenott_get_state.argtypes = [vp, P(wenott_tt)]
    lib.wenott_get_info.argtypes = [vp, P(wenott_info)]
    lib.wenott_max_wavespeed.argtypes = [vp, P(ctypes.c_double)]
    lib.wenott_max_wavespeed_noalloc.argtypes = [vp, P(ctypes.c_double)]
    lib.wenott_current_eps.argtypes = [vp, P(ctypes.c_double)]
    lib.wenott_set_inflow.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double)]
    lib.wenott_set_profiling.argtypes = [vp, ctypes.c_int32]
    lib.wenott_set_pivot_wait_limit.argtypes = [ctypes.c_int32]
    lib.wenott_finalize.argtypes = []
    lib.wenott_pivot_layout.argtypes = [ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int32)]
    lib.wenott_pivot_search.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_int32, vp, vp, vp, P(ctypes.c_double), vp]
    lib.wenott_last_error.argtypes = [vp]
    lib.wenott_last_error.restype = ctypes.c_char_p
    lib.wenott_destroy.argtypes = [vp]
    lib.wenott_destroy.restype = None
    lib.wenott_strerror.argtypes = [ctypes.c_int]
    lib.wenott_strerror.restype = ctypes.c_char_p
    lib.wenott_dense_init.argtypes = [P(vp), P(wenott_grid), ctypes.c_double, P(ctypes.c_int32), vp]
    lib.wenott_dense_max_wavespeed.argtypes = [vp, vp, P(ctypes.c_double)]
    lib.wenott_dense_rhs.argtypes = [vp, vp, ctypes.c_double, vp]
    lib.wenott_dense_rk3_step.argtypes = [vp, vp, ctypes.c_double, P(ctypes.c_double), P(ctypes.c_double)]
    lib.wenott_dense_destroy.argtypes = [vp]
    lib.wenott_dense_destroy.restype = None
    lib.wenott_mlp_nparams.argtypes = []
    lib.wenott_mlp_nparams.restype = ctypes.c_int64
    lib.wenott_mlp_workspace.argtypes = [ctypes.c_int32]
    lib.wenott_mlp_workspace.restype = ctypes.c_int64
    lib.wenott_mlp_init_params.argtypes = [vp, ctypes.c_uint64, vp]
    lib.wenott_mlp_forward.argtypes = [vp, vp, ctypes.c_int32, vp, ctypes.c_int32, vp, vp]
    lib.wenott_mlp_loss_grad.argtypes = [vp, vp, vp, vp, ctypes.c_int32, vp, vp, vp, vp]
    lib.wenott_mlp_adam_step.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float, vp]
    lib.wenott_set_proposal.argtypes = [vp, vp]
    lib.wenott_set_cross_logging.argtypes = [vp, ctypes.c_int32]
    lib.wenott_get_cross_log.argtypes = [vp, vp, vp, vp, ctypes.c_int32, P(ctypes.c_int32)]
    for name in ("wenott_init", "wenott_rhs", "wenott_rk3_step", "wenott_batch_rk3_step", "wenott_round",
                 "wenott_gemm_autotune", "wenott_gemm_autotune_table", "wenott_to_dense",
                 "wenott_get_state", "wenott_get_info", "wenott_max_wavespeed", "wenott_max_wavespeed_noalloc",
                 "wenott_current_eps",
                 "wenott_set_profiling", "wenott_set_pivot_wait_limit", "wenott_finalize", "wenott_pivot_layout",
                 "wenott_pivot_search",
                 "wenott_dense_init", "wenott_dense_max_wavespeed", "wenott_dense_rhs",
                 "wenott_dense_rk3_step", "wenott_mlp_init_params", "wenott_mlp_forward", "wenott_mlp_loss_grad",
                 "wenott_mlp_adam_step", "wenott_set_proposal", "wenott_set_cross_logging", "wenott_get_cross_log"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    # drain and release the library's cached device blocks and events before the runtime goes
    import atexit
    atexit.register(_finalize_at_exit)
    return lib


_live = weakref.WeakSet()  # solvers not yet closed (closed at exit before the library finalizes)


def _finalize_at_exit():
    for s in list(_live):
        try:
            s.close()
        except Exception:
            pass
    if _lib is not None:
        _lib.wenott_finalize()


class WenottError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__(f"{load().wenott_strerror(status).decode()} ({status}) {msg}".strip())
        self.status = status


def _check(status: int, ctx=None):
    if status != OK:
        msg = load().wenott_last_error(ctx).decode()
        raise WenottError(status, msg)


def default_opts(**kw) -> wenott_opts:
    o = wenott_opts()
    load().wenott_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---- thin wrappers with the C names ---------------------------------------------------
def wenott_init(cores, n, lo, hi, gamma, bc, opts=None, stream=None):
    """cores: [ncomp][ndim] arrays (numpy host arrays or torch CUDA tensors), FP64,
    each of shape (R_{k-1}, N_k, R_k). bc: per dimension one wenott_bc code or a (low, high)
    pair. Returns a ctypes handle."""
    lib = load()
    ndim = len(n)
    ncomp = len(cores)
    g = wenott_grid()
    g.ndim = ndim
    for d in range(ndim):
        g.n[d], g.lo[d], g.hi[d] = int(n[d]), float(lo[d]), float(hi[d])
    ranks = (ctypes.c_int64 * (ncomp * (ndim + 1)))()
    ptrs = (ctypes.c_void_p * (ncomp * ndim))()
    keep = []
    on_device = 0
    for c in range(ncomp):
        for k in range(ndim):
            a = cores[c][k]
            if hasattr(a, "is_cuda") and a.is_cuda:
                import torch
                a = a.contiguous().to(torch.float64)
                on_device = 1
                ptrs[c * ndim + k] = a.data_ptr()
            else:
                a = np.ascontiguousarray(a, dtype=np.float64)
                ptrs[c * ndim + k] = a.ctypes.data
            keep.append(a)
            ranks[c * (ndim + 1) + k] = a.shape[0]
            if k == ndim - 1:
                ranks[c * (ndim + 1) + ndim] = a.shape[2]
    t = wenott_tt(ndim, ncomp, ranks, ptrs, 0, on_device)
    bcs = _bcs(bc)
    o = opts if opts is not None else default_opts()
    h = ctypes.c_void_p()
    st = _stream_handle() if stream is None else stream
    _check(lib.wenott_init(ctypes.byref(h), ctypes.byref(t), ctypes.byref(g), float(gamma), bcs, ctypes.byref(o), st))
    return h


def wenott_rhs(ctx, alpha=0.0):
    v = wenott_tt()
    _check(load().wenott_rhs(ctx, float(alpha), ctypes.byref(v)), ctx)
    return v


def wenott_rk3_step(ctx, dt, eps=0.0, alphas=None):
    a = None if alphas is None else (ctypes.c_double * 3)(*[float(x) for x in alphas])
    _check(load().wenott_rk3_step(ctx, float(dt), float(eps), a), ctx)


def wenott_batch_rk3_step(ctxs, dts, eps=None):
    """One SSP-RK3 step of each of len(ctxs) states in lock-step (one stream, same ndim)."""
    n = len(ctxs)
    if n == 0 or len(dts) != n or (eps is not None and len(eps) != n):
        raise ValueError("ctxs, dts and eps must have the same non-zero length")
    arr = (ctypes.c_void_p * n)(*ctxs)
    d = (ctypes.c_double * n)(*[float(x) for x in dts])
    e = None if eps is None else (ctypes.c_double * n)(*[float(x) for x in eps])
    _check(load().wenott_batch_rk3_step(arr, n, d, e), ctxs[0])


def wenott_gemm_autotune(mode):
    """1 tuned (default), 0 fixed 64x64 vector shape, 2 + k shape k everywhere (4: FP64 matrix cores)."""
    _check(load().wenott_gemm_autotune(int(mode)), None)


def wenott_gemm_autotune_table():
    """Rows (ta, tb, log2 M, log2 N, log2 K, log2 batch, shape or -1 while tuning)."""
    lib = load()
    n = ctypes.c_int32(0)
    _check(lib.wenott_gemm_autotune_table(None, 0, ctypes.byref(n)), None)
    buf = (ctypes.c_int32 * (7 * max(n.value, 1)))()
    _check(lib.wenott_gemm_autotune_table(buf, n.value, ctypes.byref(n)), None)
    return [tuple(buf[7 * i:7 * i + 7]) for i in range(n.value)]


def wenott_round(ctx, eps):
    _check(load().wenott_round(ctx, float(eps)), ctx)


def wenott_to_dense(ctx, out, on_device: bool):
    ptr = out.data_ptr() if on_device else out.ctypes.data
    _check(load().wenott_to_dense(ctx, ctypes.c_void_p(ptr), 1 if on_device else 0), ctx)


def wenott_get_state(ctx):
    v = wenott_tt()
    _check(load().wenott_get_state(ctx, ctypes.byref(v)), ctx)
    return v


def wenott_get_info(ctx) -> wenott_info:
    i = wenott_info()
    _check(load().wenott_get_info(ctx, ctypes.byref(i)), ctx)
    return i


def wenott_max_wavespeed(ctx) -> float:
    a = ctypes.c_double()
    _check(load().wenott_max_wavespeed(ctx, ctypes.byref(a)), ctx)
    return a.value


def wenott_max_wavespeed_noalloc(ctx) -> float:
    a = ctypes.c_double()
    _check(load().wenott_max_wavespeed_noalloc(ctx, ctypes.byref(a)), ctx)
    return a.value


def wenott_set_inflow(ctx, dim, side, prim):
    a = (ctypes.c_double * len(prim))(*[float(v) for v in prim])
    _check(load().wenott_set_inflow(ctx, int(dim), int(side), a), ctx)


def wenott_current_eps(ctx) -> float:
    a = ctypes.c_double()
    _check(load().wenott_current_eps(ctx, ctypes.byref(a)), ctx)
    return a.value


def wenott_set_profiling(ctx, on: bool):
    _check(load().wenott_set_profiling(ctx, 1 if on else 0), ctx)


def wenott_pivot_search(A, rmax: int, rel_tol2: float, allow_persistent: bool = True):
    """A: (m, n) float64 CUDA tensor. Returns (rank, rowpiv, colpiv, L (m x rmax tensor), resid2, tol2)."""
    import torch
    m, n = A.shape
    A = A.contiguous()
    rp = torch.zeros(rmax, dtype=torch.int32, device=A.device)
    cp = torch.zeros(rmax, dtype=torch.int32, device=A.device)
    L = torch.zeros((m, rmax), dtype=torch.float64, device=A.device)
    info = (ctypes.c_double * 3)()
    _check(load().wenott_pivot_search(_ptr(A), int(m), int(n), int(rmax), float(rel_tol2), 1 if allow_persistent else 0,
                                      _ptr(rp), _ptr(cp), _ptr(L), info, _stream_handle()), None)
    r = int(info[0])
    return r, rp[:r].cpu().numpy(), cp[:r].cpu().numpy(), L, info[1], info[2]


def wenott_pivot_layout(m: int, n: int):
    out = (ctypes.c_int32 * 7)()
    _check(load().wenott_pivot_layout(int(m), int(n), out), None)
    return list(out)


def wenott_set_pivot_wait_limit(polls: int):
    _check(load().wenott_set_pivot_wait_limit(int(polls)), None)


def _grid(n, lo, hi):
    g = wenott_grid()
    g.ndim = len(n)
    for d in range(len(n)):
        g.n[d], g.lo[d], g.hi[d] = int(n[d]), float(lo[d]), float(hi[d])
    return g


def _bcs(bc):
    """bc per dimension: one wenott_bc value for both sides, or a (low, high) pair."""
    b = (ctypes.c_int32 * 6)()
    for d in range(len(bc)):
        lo, hi = (bc[d], bc[d]) if isinstance(bc[d], (int, np.integer)) else bc[d]
        b[2 * d], b[2 * d + 1] = int(lo), int(hi)
    return b


def wenott_dense_init(n, lo, hi, gamma, bc, stream=None):
    h = ctypes.c_void_p()
    st = _stream_handle() if stream is None else stream
    _check(load().wenott_dense_init(ctypes.byref(h), ctypes.byref(_grid(n, lo, hi)), float(gamma), _bcs(bc), st))
    return h


def wenott_dense_max_wavespeed(ctx, U) -> float:
    a = ctypes.c_double()
    _check(load().wenott_dense_max_wavespeed(ctx, ctypes.c_void_p(U.data_ptr()), ctypes.byref(a)))
    return a.value


def wenott_dense_rhs(ctx, U, alpha, L):
    _check(load().wenott_dense_rhs(ctx, ctypes.c_void_p(U.data_ptr()), float(alpha), ctypes.c_void_p(L.data_ptr())))


def wenott_dense_rk3_step(ctx, U, dt, alphas=None):
    a = None if alphas is None else (ctypes.c_double * 3)(*[float(x) for x in alphas])
    used = (ctypes.c_double * 3)()
    _check(load().wenott_dense_rk3_step(ctx, ctypes.c_void_p(U.data_ptr()), float(dt), a, used))
    return [used[0], used[1], used[2]]


def wenott_dense_destroy(ctx):
    if ctx:
        load().wenott_dense_destroy(ctx)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def wenott_mlp_nparams() -> int:
    return int(load().wenott_mlp_nparams())


def wenott_mlp_workspace(batch: int) -> int:
    return int(load().wenott_mlp_workspace(int(batch)))


def wenott_mlp_init_params(params, seed: int):
    _check(load().wenott_mlp_init_params(_ptr(params), int(seed), _stream_handle()))


def wenott_mlp_forward(params, x, y, work, bf16: bool):
    _check(load().wenott_mlp_forward(_ptr(params), _ptr(x), int(x.shape[0]), _ptr(y), 1 if bf16 else 0, _ptr(work),
                                     _stream_handle()))


def wenott_mlp_loss_grad(params, x, cls, hist, grad, loss, work):
    _check(load().wenott_mlp_loss_grad(_ptr(params), _ptr(x), _ptr(cls), _ptr(hist), int(x.shape[0]), _ptr(grad),
                                       _ptr(loss), _ptr(work), _stream_handle()))


def wenott_mlp_adam_step(params, grad, m, v, t: int, lr: float):
    _check(load().wenott_mlp_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t), float(lr),
                                       _stream_handle()))


def wenott_set_proposal(ctx, params):
    _check(load().wenott_set_proposal(ctx, None if params is None else _ptr(params)), ctx)


def wenott_set_cross_logging(ctx, on: bool):
    _check(load().wenott_set_cross_logging(ctx, 1 if on else 0), ctx)


def wenott_get_cross_log(ctx, max_samples: int = 100000):
    x = np.zeros((max_samples, MLP_IN), dtype=np.float32)
    cls = np.zeros(max_samples, dtype=np.int32)
    hist = np.zeros((max_samples, MLP_BINS), dtype=np.float32)
    n = ctypes.c_int32()
    _check(load().wenott_get_cross_log(ctx, x.ctypes.data, cls.ctypes.data, hist.ctypes.data, max_samples,
                                       ctypes.byref(n)), ctx)
    k = n.value
    return x[:k].copy(), cls[:k].copy(), hist[:k].copy()


def wenott_destroy(ctx):
    if ctx:
        load().wenott_destroy(ctx)


class Solver:
    """Convenience owner of one context (state on the device)."""

    def __init__(self, flow, opts=None, stream=None):
        self.flow = flow
        self.n = tuple(flow.n)
        self.ncomp = flow.ncomp
        law = getattr(flow, "law", LAW_EULER)
        if opts is None:
            opts = default_opts(law=law)
        elif opts.law != law:
            opts = wenott_opts.from_buffer_copy(opts)
            opts.law = law
        self.ctx = wenott_init(flow.cores, flow.n, flow.lo, flow.hi, flow.gamma, flow.bc, opts, stream)
        _live.add(self)
        for (dim, side), prim in sorted((getattr(flow, "inflow", None) or {}).items()):
            wenott_set_inflow(self.ctx, dim, side, prim)

    def close(self):
        if self.ctx:
            wenott_destroy(self.ctx)
            self.ctx = None
        _live.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dense(self, device: bool = False):
        if device:
            import torch
            out = torch.empty((self.ncomp,) + self.n, dtype=torch.float64, device="cuda")
            wenott_to_dense(self.ctx, out, True)
            return out
        out = np.empty((self.ncomp,) + self.n)
        wenott_to_dense(self.ctx, out, False)
        return out

    def step(self, dt, eps=0.0, alphas=None):
        wenott_rk3_step(self.ctx, dt, eps, alphas)

    def info(self):
        return wenott_get_info(self.ctx)

    def max_wavespeed(self):
        return wenott_max_wavespeed(self.ctx)

    def eps(self):
        return wenott_current_eps(self.ctx)

    def round(self, eps):
        wenott_round(self.ctx, eps)

    def rhs_cores(self, alpha=0.0):
        """Host copies of the cores of the TT of L(U) computed by the library."""
        return _view_cores(wenott_rhs(self.ctx, alpha), self.n)

    def state_cores(self):
        return _view_cores(wenott_get_state(self.ctx), self.n)


def _view_cores(view: wenott_tt, n):
    """Host copies of the cores of a library view: [ncomp][ndim] numpy arrays."""
    import torch
    ndim, ncomp = view.ndim, view.ncomp
    torch.cuda.synchronize()
    cores = []
    for c in range(ncomp):
        comp = []
        for k in range(ndim):
            r0 = int(view.ranks[c * (ndim + 1) + k])
            r1 = int(view.ranks[c * (ndim + 1) + k + 1])
            arr = np.empty((r0, int(n[k]), r1))
            nbytes = arr.nbytes
            _memcpy_d2h(arr.ctypes.data, view.cores[c * ndim + k], nbytes)
            comp.append(arr)
        cores.append(comp)
    return cores


_hip = None


def _memcpy_d2h(dst, src, nbytes):
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    r = _hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), ctypes.c_size_t(nbytes), 2)
    if r != 0:
        raise RuntimeError(f"hipMemcpy failed ({r})")
