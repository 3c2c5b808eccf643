"""Thin Python binding over the C ABI (include/ph.h).

Marshalling only: numpy arrays for host inputs, torch tensors for device
buffers and the current HIP stream.  Every step of the online stage runs in
the library's HIP kernels; nothing here computes.
"""

import ctypes as C

import numpy as np

from . import _lib as L


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Tree:
    """Cluster tree and block cluster tree (ph_build_tree)."""

    def __init__(self, points, *, lo=0.0, hi=1.0, leaf_size=64, l_max=-1, eta2=None):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        if pts.ndim != 2:
            raise ValueError("points must be (n, d)")
        n, d = pts.shape
        num, den = eta2 if eta2 is not None else (d, 1)
        opts = L.TreeOpts(d, lo, hi, leaf_size, l_max, num, den)
        h = C.c_void_p()
        L.check(L.lib().ph_build_tree(_dptr(pts), n, C.byref(opts), C.byref(h)), "ph_build_tree")
        self._h = h
        info = L.TreeInfo()
        L.check(L.lib().ph_tree_info_get(h, C.byref(info)), "ph_tree_info_get")
        self.info = {k: getattr(info, k) for k, _ in L.TreeInfo._fields_}
        self.n, self.d = n, d

    def perm(self):
        out = np.empty(self.n, dtype=np.int64)
        L.check(L.lib().ph_tree_perm(self._h, out.ctypes.data_as(C.POINTER(C.c_int64))), "ph_tree_perm")
        return out

    def nodes(self):
        nn = self.info["n_nodes"]
        level = np.empty(nn, np.int32)
        coords = np.empty((nn, self.d), np.int32)
        begin = np.empty(nn, np.int64)
        end = np.empty(nn, np.int64)
        parent = np.empty(nn, np.int32)
        i32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        i64 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
        L.check(L.lib().ph_tree_nodes(self._h, i32(level), i32(coords), i64(begin), i64(end), i32(parent)),
                "ph_tree_nodes")
        return dict(level=level, coords=coords, begin=begin, end=end, parent=parent)

    def blocks(self):
        near = np.empty((self.info["n_near"], 2), np.int32)
        far = np.empty((self.info["n_far"], 2), np.int32)
        fcls = np.empty(self.info["n_far"], np.int32)
        i32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        L.check(L.lib().ph_tree_blocks(self._h, i32(near), i32(far), i32(fcls)), "ph_tree_blocks")
        return near, far, fcls

    def classes(self):
        lev = np.empty(self.info["n_classes"], np.int32)
        off = np.empty((self.info["n_classes"], self.d), np.int32)
        i32 = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        L.check(L.lib().ph_tree_classes(self._h, i32(lev), i32(off)), "ph_tree_classes")
        return lev, off

    def __del__(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and L is not None and L._lib is not None:   # (skip at interpreter shutdown)
            L._lib.ph_tree_free(h)


class Model:
    """Offline stage output on the device: ph_offline_compress (format "h2", the parametric
    H^2-matrix), ph_offline_compress_h (format "h", the parametric H-matrix),
    ph_offline_compress_gpu (offline="gpu": kernel tensors evaluated on the GPU), or
    ph_offline_compress_tt (compress="tt": TT-cross + TT-rounding; coupling="implicit" gives
    the format "h2_implicit")."""

    def __init__(self, tree, kernel, theta_lo, theta_hi, *, p_s, p_theta, tol, num_threads=0,
                 stream=None, format="h2", offline="host", compress="hosvd", coupling="materialized"):
        lo = np.atleast_1d(np.asarray(theta_lo, dtype=np.float64))
        hi = np.atleast_1d(np.asarray(theta_hi, dtype=np.float64))
        opts = L.OfflineOpts()
        opts.kernel = L.KERNELS[kernel]
        opts.d_theta = lo.shape[0]
        for k in range(lo.shape[0]):
            opts.theta_lo[k] = lo[k]
            opts.theta_hi[k] = hi[k]
        opts.p_s, opts.p_theta, opts.tol, opts.num_threads = p_s, p_theta, tol, num_threads
        h = C.c_void_p()
        if offline not in ("host", "gpu") or (offline == "gpu" and format != "h2"):
            raise ValueError('offline must be "host" or "gpu" (the GPU offline stage builds the H^2 format)')
        entry = {"h2": "ph_offline_compress", "h": "ph_offline_compress_h"}[format]
        if offline == "gpu":
            entry = "ph_offline_compress_gpu"
        if compress not in ("hosvd", "tt") or coupling not in L.COUPLINGS:
            raise ValueError('compress must be "hosvd" or "tt", coupling "materialized" or "implicit"')
        if compress == "tt":
            if format != "h2" or offline != "host":
                raise ValueError('compress="tt" builds the H^2 format on the host')
            entry = "ph_offline_compress_tt"
            L.check(L.lib().ph_offline_compress_tt(tree._h, C.byref(opts), L.COUPLINGS[coupling], _stream(stream),
                                                   C.byref(h)), entry)
        elif coupling != "materialized":
            raise ValueError('coupling="implicit" needs compress="tt"')
        else:
            L.check(getattr(L.lib(), entry)(tree._h, C.byref(opts), _stream(stream), C.byref(h)), entry)
        self._h = h
        fmt = C.c_int()
        L.check(L.lib().ph_model_format(h, C.byref(fmt)), "ph_model_format")
        self.format = {v: k for k, v in L.FORMATS.items()}[fmt.value]
        self.tree = tree
        info = L.ModelInfo()
        L.check(L.lib().ph_model_info_get(h, C.byref(info)), "ph_model_info_get")
        self.info = {k: getattr(info, k) for k, _ in L.ModelInfo._fields_}
        self.d_theta = lo.shape[0]

    def near_ranks(self):
        out = np.empty(self.tree.info["n_near"], np.int32)
        L.check(L.lib().ph_model_near_ranks(self._h, out.ctypes.data_as(C.POINTER(C.c_int32))),
                "ph_model_near_ranks")
        return out

    def class_ranks(self):
        out = np.empty((self.tree.info["n_classes"], 2 + self.d_theta), np.int32)
        L.check(L.lib().ph_model_class_ranks(self._h, out.ctypes.data_as(C.POINTER(C.c_int32))),
                "ph_model_class_ranks")
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and L is not None and L._lib is not None:   # (skip at interpreter shutdown)
            L._lib.ph_model_free(h)


class Instance:
    """An instantiated H^2-matrix for T parameter values (ph_instantiate / ph_instantiate_grad)."""

    def __init__(self, model, theta, *, dtype="f64", grad_dim=None, near="auto", stream=None):
        """near: "auto", "blocks" (near blocks written to memory) or "factored" (near blocks
        formed from the factors inside every MVM, never written); see ph_instantiate_ex."""
        self.model = model
        self._h = C.c_void_p()
        self.dtype = dtype
        self.near = near
        th = self._theta(theta)
        self.T = th.shape[0]
        self._call(th, grad_dim, stream)

    def _theta(self, theta):
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1, self.model.d_theta))
        return th

    def _call(self, th, grad_dim, stream):
        if self.near != "auto":
            code = L.lib().ph_instantiate_ex(self.model._h, _dptr(th), th.shape[0], L.DTYPES[self.dtype],
                                             L.NEAR_MODES[self.near], -1 if grad_dim is None else grad_dim,
                                             _stream(stream), C.byref(self._h))
            L.check(code, "ph_instantiate_ex")
        elif grad_dim is None:
            code = L.lib().ph_instantiate(self.model._h, _dptr(th), th.shape[0], L.DTYPES[self.dtype],
                                          _stream(stream), C.byref(self._h))
            L.check(code, "ph_instantiate")
        else:
            code = L.lib().ph_instantiate_grad(self.model._h, _dptr(th), th.shape[0], grad_dim,
                                               L.DTYPES[self.dtype], _stream(stream), C.byref(self._h))
            L.check(code, "ph_instantiate_grad")

    @property
    def factored(self):
        """True if the instance holds the factored near field (no near blocks in memory)."""
        f = C.c_int()
        L.check(L.lib().ph_inst_near_mode(self._h, C.byref(f)), "ph_inst_near_mode")
        return bool(f.value)

    def reinstantiate(self, theta, *, grad_dim=None, stream=None):
        """Re-instantiate in place (same T and dtype; no allocation)."""
        th = self._theta(theta)
        if th.shape[0] != self.T:
            raise ValueError("T must match the instance")
        self._call(th, grad_dim, stream)

    def matvec(self, x, y=None, *, alpha=1.0, beta=0.0, nugget=0.0, stream=None):
        """y = alpha (K~ + nugget I) x + beta y for device tensors x of shape (n,), (R, n) or (T, R, n)."""
        import torch
        want = torch.float64 if self.dtype == "f64" else torch.float32
        if x.dtype != want or not x.is_cuda:
            raise TypeError(f"x must be a {want} device tensor")
        x = x.contiguous()
        n = self.model.tree.n
        if x.shape[-1] != n:
            raise ValueError("last dimension of x must be n")
        R = 1 if x.dim() == 1 else x.shape[-2]
        if x.dim() == 3 and x.shape[0] != self.T:
            raise ValueError("leading dimension must be T")
        if x.dim() < 3 and self.T != 1:
            raise ValueError("x must be (T, R, n) for a T > 1 instance")
        if y is None:
            y = torch.empty_like(x)
            beta = 0.0
        elif y.shape != x.shape or y.dtype != want or not y.is_contiguous():
            raise ValueError("y must be a contiguous tensor shaped like x")
        code = L.lib().ph_matvec(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), R,
                                 alpha, beta, nugget, _stream(stream))
        L.check(code, "ph_matvec")
        return y

    def bilinear(self, u, x, *, stream=None):
        """out[t] = sum_r u_t[r] . K~_t x_t[r] as a device float64 tensor of length T (ph_bilinear)."""
        import torch
        want = torch.float64 if self.dtype == "f64" else torch.float32
        for a in (u, x):
            if a.dtype != want or not a.is_cuda:
                raise TypeError(f"u and x must be {want} device tensors")
        if u.shape != x.shape:
            raise ValueError("u and x must have the same shape")
        u = u.contiguous()
        x = x.contiguous()
        R = 1 if x.dim() == 1 else x.shape[-2]
        out = torch.empty(self.T, dtype=torch.float64, device=x.device)
        code = L.lib().ph_bilinear(self._h, C.c_void_p(u.data_ptr()), C.c_void_p(x.data_ptr()), R,
                                   C.c_void_p(out.data_ptr()), _stream(stream))
        L.check(code, "ph_bilinear")
        return out

    def autotune(self, x, y=None, *, stream=None):
        """Pick the MVM launch configuration by measurement (ph_autotune); returns it as a dict."""
        import torch
        x = x.contiguous()
        if y is None:
            y = torch.empty_like(x)
        R = 1 if x.dim() == 1 else x.shape[-2]
        info = L.TuneInfo()
        L.check(L.lib().ph_autotune(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), R,
                                    _stream(stream), C.byref(info)), "ph_autotune")
        return {k: getattr(info, k) for k, _ in L.TuneInfo._fields_}

    def record(self, x, y, *, nugget=0.0, stream=None):
        """Record instantiation + MVM (y = (K~ + nugget I) x) as one replayable graph (ph_graph_create)."""
        return Graph(self, x, y, nugget, stream)

    def near_block(self, b, t=0):
        near, _, _ = self.model.tree.blocks()
        nodes = self.model.tree.nodes()
        s, u = near[b]
        ns = nodes["end"][s] - nodes["begin"][s]
        nt = nodes["end"][u] - nodes["begin"][u]
        out = np.empty(ns * nt)
        L.check(L.lib().ph_inst_near_block(self._h, t, b, _dptr(out)), "ph_inst_near_block")
        return out.reshape(nt, ns).T

    def coupling(self, c, t=0):
        P = self.model.info["P"]
        out = np.empty(P * P)
        L.check(L.lib().ph_inst_coupling(self._h, t, c, _dptr(out)), "ph_inst_coupling")
        return out.reshape(P, P).T

    def __del__(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and L is not None and L._lib is not None:   # (skip at interpreter shutdown)
            L._lib.ph_inst_free(h)


class Graph:
    """A recorded instantiate + MVM launch of an instance; launch(theta) replays it."""

    def __init__(self, inst, x, y, nugget, stream):
        import torch
        if stream is None:
            raise ValueError("recording needs an explicit non-default torch.cuda.Stream")
        if not (x.is_contiguous() and y.is_contiguous()) or x.shape != y.shape:
            raise ValueError("x and y must be contiguous tensors of the same shape")
        self.inst, self.x, self.y, self.stream = inst, x, y, stream   # keep the bound buffers alive
        R = 1 if x.dim() == 1 else x.shape[-2]
        h = C.c_void_p()
        L.check(L.lib().ph_graph_create(inst._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), R, nugget,
                                        _stream(stream), C.byref(h)), "ph_graph_create")
        self._h = h

    def launch(self, theta=None, *, stream=None):
        th = None
        if theta is not None:
            th = self.inst._theta(theta)
            if th.shape[0] != self.inst.T:
                raise ValueError("theta must have T rows")
        L.check(L.lib().ph_graph_launch(self._h, _dptr(th) if th is not None else None,
                                        _stream(stream if stream is not None else self.stream)), "ph_graph_launch")
        return self.y

    def __del__(self):
        h = getattr(self, "_h", None)
        self._h = None
        if h and L is not None and L._lib is not None:   # (skip at interpreter shutdown)
            L._lib.ph_graph_free(h)


def kernel_eval(kernel, x, y, theta):
    """kappa(x_i, y_i; theta) for the rows of x and y (ph_kernel_eval, host arrays): x, y of
    shape (n, d), theta the kernel's d_theta parameters.  Returns a float64 array of n values."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    th = np.ascontiguousarray(np.atleast_1d(theta), dtype=np.float64)
    if x.ndim != 2 or x.shape != y.shape:
        raise ValueError("x and y must have the same shape (n, d)")
    out = np.empty(x.shape[0])
    L.check(L.lib().ph_kernel_eval(L.KERNELS[kernel], x.shape[1], _dptr(x), _dptr(y), x.shape[0], _dptr(th),
                                   _dptr(out)), "ph_kernel_eval")
    return out


def tt_far_ranks(tree, kernel, theta_lo, theta_hi, *, p_s, p_theta, tol, num_threads=0):
    """TT ranks of every translation class's far tensor after TT-cross + TT-rounding
    (ph_tt_far_ranks; host only, no model): an int32 array of shape (n_classes, 2 d + d_theta + 1)
    and the number of distinct kernel values evaluated."""
    lo = np.atleast_1d(np.asarray(theta_lo, dtype=np.float64))
    hi = np.atleast_1d(np.asarray(theta_hi, dtype=np.float64))
    opts = L.OfflineOpts()
    opts.kernel = L.KERNELS[kernel]
    opts.d_theta = lo.shape[0]
    for k in range(lo.shape[0]):
        opts.theta_lo[k] = lo[k]
        opts.theta_hi[k] = hi[k]
    opts.p_s, opts.p_theta, opts.tol, opts.num_threads = p_s, p_theta, tol, num_threads
    out = np.empty((tree.info["n_classes"], 2 * tree.d + lo.shape[0] + 1), np.int32)
    ev = C.c_int64()
    L.check(L.lib().ph_tt_far_ranks(tree._h, C.byref(opts), out.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(ev)),
            "ph_tt_far_ranks")
    return out, ev.value


def cg_solve(inst64, y, *, nugget, tol=1e-6, lo=None, max_iter=100000, inner_max=1000, inner_tol=1e-4,
             stream=None):
    """Solve (K~ + nugget I) a = y (ph_cg_solve, or ph_cg_solve_batch for several right-hand
    sides).  inst64: FP64 instance with T = 1; y: device float64 tensor of shape (n,) or (R, n);
    lo: optional FP32/BF16 instance of the same theta for FP64 iterative refinement.  Returns
    (a, stats dict); for R columns the stats are the largest iteration count and the worst
    residual."""
    import torch
    if y.dtype != torch.float64 or not y.is_cuda or y.dim() not in (1, 2):
        raise TypeError("y must be a float64 device tensor of shape (n,) or (R, n)")
    y = y.contiguous()
    a = torch.empty_like(y)
    st = L.CgStats()
    lo_h = lo._h if lo is not None else None
    if y.dim() == 1:
        code = L.lib().ph_cg_solve(inst64._h, lo_h, C.c_void_p(y.data_ptr()), C.c_void_p(a.data_ptr()), nugget,
                                   tol, max_iter, inner_max, inner_tol, C.byref(st), _stream(stream))
        L.check(code, "ph_cg_solve")
    else:
        code = L.lib().ph_cg_solve_batch(inst64._h, lo_h, C.c_void_p(y.data_ptr()), C.c_void_p(a.data_ptr()),
                                         y.shape[0], nugget, tol, max_iter, inner_max, inner_tol, C.byref(st),
                                         _stream(stream))
        L.check(code, "ph_cg_solve_batch")
    return a, {k: getattr(st, k) for k, _ in L.CgStats._fields_}


def _autograd_function():
    import torch

    class KThetaMatvec(torch.autograd.Function):
        """y = (K~(theta) + nugget I) x with gradients for theta and x.

        theta: (d_theta,) with x of shape (n,) or (R, n), or (T, d_theta) with x of shape
        (T, R, n).  Backward: dL/dx = (K~ + nugget I) g (K~ is symmetric by construction)
        and dL/dtheta_i = sum_r g_r . (dK~/dtheta_i) x_r, the bilinear form of the
        instance of ph_instantiate_grad, both computed by the library.  One instance per
        (model, T, dtype) is kept and re-instantiated in place for the forward product, the
        backward product and each derivative (no device allocation after the first call);
        backward re-instantiates at its own theta, so other forward calls in between are safe.
        """

        @staticmethod
        def _instance(model, th, dtype):
            cache = model.__dict__.setdefault("_autograd_instances", {})
            key = (th.shape[0], dtype)
            inst = cache.get(key)
            if inst is None:
                inst = cache[key] = Instance(model, th, dtype=dtype)
            else:
                inst.reinstantiate(th)
            return inst

        @staticmethod
        def forward(ctx, theta, x, model, nugget=0.0):
            th = theta.detach().to("cpu", torch.float64).numpy().reshape(-1, model.d_theta)
            dtype = "f64" if x.dtype == torch.float64 else "f32"
            inst = KThetaMatvec._instance(model, th, dtype)
            y = inst.matvec(x, nugget=nugget)
            ctx.save_for_backward(x)
            ctx.inst, ctx.model, ctx.nugget, ctx.th, ctx.theta_meta = inst, model, nugget, th, theta
            return y

        @staticmethod
        def backward(ctx, g):
            (x,) = ctx.saved_tensors
            g = g.contiguous()
            gtheta = gx = None
            if ctx.needs_input_grad[1]:
                ctx.inst.reinstantiate(ctx.th)
                gx = ctx.inst.matvec(g, nugget=ctx.nugget)
            if ctx.needs_input_grad[0]:
                cols = []
                for i in range(ctx.model.d_theta):
                    ctx.inst.reinstantiate(ctx.th, grad_dim=i)
                    cols.append(ctx.inst.bilinear(g, x))
                meta = ctx.theta_meta
                gtheta = torch.stack(cols, dim=-1).reshape(meta.shape).to(meta.dtype).to(meta.device)
            return gtheta, gx, None, None

    return KThetaMatvec


_KTM = None


def k_theta_matvec(model, theta, x, nugget=0.0):
    """Differentiable y = (K~(theta) + nugget I) x (see KThetaMatvec)."""
    global _KTM
    if _KTM is None:
        _KTM = _autograd_function()
    return _KTM.apply(theta, x, model, nugget)


def __getattr__(name):
    if name == "KThetaMatvec":
        global _KTM
        if _KTM is None:
            _KTM = _autograd_function()
        return _KTM
    raise AttributeError(name)
