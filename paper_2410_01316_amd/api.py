"""Python binding of libfastsum: argument checks and marshalling only.

Every step of the summation runs in the HIP library; PyTorch provides the
device buffers (tensor storage) and the current HIP stream.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _need(t, name, shape, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device != device:
        raise ValueError(f"{name} must be a contiguous float32 tensor on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


class Plan:
    """A fast-summation plan: kernel, directions xi (d x P), grid and window
    parameters, the bound R and workspace for up to n_max sources and m_max
    targets on one GPU.  See include/fastsum.h for every parameter.
    sorting=True (energy kernel) takes the exact 1-D sums by sorting instead
    of Fourier summation."""

    def __init__(self, xi, *, kernel, n_ft, R, scale=1.0, T=0.0, gmax_factor=0.0,
                 window_w=0, oversample=0, proj="fp32", grad=False, materialize=False,
                 sorting=False, n_max, m_max, device=None):
        lib = L.load()
        xi = np.ascontiguousarray(np.asarray(xi, dtype=np.float32))
        if xi.ndim != 2:
            raise ValueError("xi must be a (d, P) array")
        self.d, self.P = xi.shape
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.type != "cuda":
            raise ValueError("the plan lives on a GPU")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.kernel = kernel
        self.prm = L.Params(self.d, self.P, int(n_ft), int(window_w), int(oversample),
                            L.KERNELS[kernel], L.PROJ[proj],
                            (L.FLAG_GRAD if grad else 0) | (L.FLAG_MATERIALIZE if materialize else 0)
                            | (L.FLAG_SORTED if sorting else 0),
                            float(scale), float(T), float(gmax_factor), float(R))
        self.n_max, self.m_max = int(n_max), int(m_max)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = lib.fastsum_plan_create(ctypes.byref(self.prm), xi.ctypes.data_as(ctypes.c_void_p),
                                         self.n_max, self.m_max, _stream_ptr(self.device),
                                         ctypes.byref(self._h))
        L.check(st, "fastsum_plan_create")
        self._lib = lib
        self._last = None
        self.execs = 0                  # calls so far (FastSum checks it in backward)

    # -- forward / adjoint ------------------------------------------------
    def __call__(self, x, w, y=None, out=None):
        """s_m ~ sum_n w_n F(||x_n - y_m||); y defaults to x."""
        if y is None:
            y = x
        N, M = x.shape[0], y.shape[0]
        _need(x, "x", (N, self.d), self.device)
        _need(w, "w", (N,), self.device)
        _need(y, "y", (M, self.d), self.device)
        if out is None:
            out = torch.empty(M, dtype=torch.float32, device=self.device)
        _need(out, "out", (M,), self.device)
        with torch.cuda.device(self.device):
            st = self._lib.fastsum_exec(self._h, _ptr(x), N, _ptr(w), _ptr(y), M, _ptr(out),
                                        _stream_ptr(self.device))
        L.check(st, "fastsum_exec")
        self._last = (x, w, y)          # keep the inputs alive for grad
        self.execs += 1
        return out

    def grad(self, grad_s, want_y=True, want_w=True, want_x=False):
        """(grad_y, grad_w) of the last call for the cotangent grad_s, or
        (grad_x, grad_y, grad_w) when want_x is set."""
        if self._last is None:
            raise L.FastSumError(L.ESTATE, "grad before exec")
        x, w, y = self._last
        M, N = y.shape[0], x.shape[0]
        _need(grad_s, "grad_s", (M,), self.device)
        gx = torch.empty((N, self.d), dtype=torch.float32, device=self.device) if want_x else None
        gy = torch.empty((M, self.d), dtype=torch.float32, device=self.device) if want_y else None
        gw = torch.empty(N, dtype=torch.float32, device=self.device) if want_w else None
        opt = lambda t: _ptr(t) if t is not None else None
        with torch.cuda.device(self.device):
            st = self._lib.fastsum_grad_xyw(self._h, _ptr(grad_s), opt(gx), opt(gy), opt(gw),
                                            _stream_ptr(self.device))
        L.check(st, "fastsum_grad_xyw")
        return (gx, gy, gw) if want_x else (gy, gw)

    # -- diagnostics --------------------------------------------------------
    def check(self):
        """Raise FastSumError(ERANGE) if a point exceeded the bound R."""
        with torch.cuda.device(self.device):
            L.check(self._lib.fastsum_check(self._h), "fastsum_check")

    def info(self):
        inf = L.PlanInfo()
        L.check(self._lib.fastsum_get_info(self._h, ctypes.byref(inf)), "fastsum_get_info")
        return {k: getattr(inf, k) for k, _ in L.PlanInfo._fields_}

    def debug_read(self, which):
        """Copy of an internal buffer of the last exec: 0 x-projections (P,N),
        1 y-projections (P,M), 2 convolved grids (P, grid_nr)."""
        x, w, y = self._last
        inf = self.info()
        cols = {0: x.shape[0], 1: y.shape[0], 2: inf["grid_nr"]}[which]
        out = np.empty((self.P, cols), dtype=np.float32)
        with torch.cuda.device(self.device):
            st = self._lib.fastsum_debug_read(self._h, which, out.ctypes.data_as(ctypes.c_void_p),
                                              out.size)
        L.check(st, "fastsum_debug_read")
        return out

    def set_launch(self, chunk_len=0, dir_range=0):
        """Launch shape of later calls (0 = the plan's rule): sources per
        spreading workgroup (multiple of 4096), directions per fused
        gathering workgroup (multiple of 16)."""
        L.check(self._lib.fastsum_set_launch(self._h, int(chunk_len), int(dir_range)),
                "fastsum_set_launch")

    def profile(self, enable=True):
        """Record HIP events around every kernel launch of later calls."""
        L.check(self._lib.fastsum_profile(self._h, 1 if enable else 0), "fastsum_profile")

    def profile_read(self):
        """{phase: (total ms, launches)} since the last read (synchronises)."""
        ms = np.zeros(len(L.PHASES))
        cnt = np.zeros(len(L.PHASES), dtype=np.int64)
        with torch.cuda.device(self.device):
            st = self._lib.fastsum_profile_read(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                                cnt.ctypes.data_as(ctypes.c_void_p))
        L.check(st, "fastsum_profile_read")
        return {ph: (float(ms[i]), int(cnt[i])) for i, ph in enumerate(L.PHASES)}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.fastsum_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FastSum(torch.autograd.Function):
    """s = FastSum.apply(plan, x, y, w): differentiable in x, y and w (the
    plan must be created with grad=True).

    The library's adjoint reads what the plan kept from its last call.  When
    the plan ran again between this forward and its backward (one plan in
    several sums of one graph), backward first repeats this forward on the
    saved inputs; inputs modified in place since the forward make autograd
    raise instead of returning a wrong gradient."""

    @staticmethod
    def forward(ctx, plan, x, y, w):
        ctx.plan = plan
        ctx.same = y is x
        xd, yd, wd = x.detach(), y.detach(), w.detach()
        s = plan(xd, wd, xd if ctx.same else yd)
        ctx.exec_id = plan.execs
        ctx.save_for_backward(x, y, w)
        return s

    @staticmethod
    def backward(ctx, grad_s):
        plan = ctx.plan
        x, y, w = ctx.saved_tensors
        if plan.execs != ctx.exec_id:
            xd = x.detach()
            plan(xd, w.detach(), xd if ctx.same else y.detach())
            ctx.exec_id = plan.execs
        want_x, want_y, want_w = ctx.needs_input_grad[1:4]
        if not (want_x or want_y or want_w):
            return None, None, None, None
        r = plan.grad(grad_s.contiguous(), want_y=want_y, want_w=want_w, want_x=want_x)
        gx, gy, gw = r if want_x else (None, *r)
        return None, gx, gy, gw


def bound(x, y=None):
    """max ||x_n|| + max ||y_m|| (App. J, eq. radius_xy) computed on the
    device by fastsum_bound; y defaults to x.  Raises FastSumError(ERANGE)
    when a coordinate is not finite."""
    lib = L.load()
    if y is None:
        y = x
    d = x.shape[1]
    _need(x, "x", (x.shape[0], d), x.device)
    _need(y, "y", (y.shape[0], d), x.device)
    out = ctypes.c_double()
    with torch.cuda.device(x.device):
        st = lib.fastsum_bound(_ptr(x), x.shape[0], _ptr(y), y.shape[0], d,
                               _stream_ptr(x.device), ctypes.byref(out))
    L.check(st, "fastsum_bound")
    return out.value


def kernel_sum(x, y, w, xi, *, kernel, scale=1.0, n_ft=None, R=None, sorting=False, **kw):
    """One call of s_m ~ sum_n w_n F(||x_n - y_m||) (eq. kernel_sum by the
    slicing estimator with the directions xi, (d, P) unit columns) on a plan
    built for exactly these sizes and released afterwards.  R defaults to
    max ||x|| + max ||y|| (App. J, eq. radius_xy, from fastsum_bound), n_ft to
    choose_nft's rule (1024 for the energy kernel).  y may be x.  For
    repeated calls keep a Plan."""
    if R is None:
        R = bound(x, y)
        R = R * (1.0 + 1e-4) if R > 0 else 1.0
    if n_ft is None:
        n_ft = 1024 if kernel == "energy" else choose_nft(kernel, x.shape[1], R, scale=scale)
    plan = Plan(xi, kernel=kernel, n_ft=n_ft, R=R, scale=scale, sorting=sorting,
                n_max=x.shape[0], m_max=y.shape[0], device=x.device, **kw)
    try:
        s = plan(x, w, y)
        plan.check()
    finally:
        plan.close()
    return s


def distance_qmc(d, P, *, iters=400, lr=None, seed=0, rotate=True, device=None):
    """Distance QMC directions (App. H) built on the GPU by
    fastsum_distance_qmc: `iters` projected Adam steps from P seeded i.i.d.
    unit vectors (d <= 64), then, with `rotate`, a seeded Haar-random
    rotation (App. E) applied by fastsum_rotate_directions, so the sliced
    estimator stays unbiased.  Only the random draws (the start and the
    rotation matrix) are made here.  Returns the (d, P) float32 array of
    unit columns that Plan takes."""
    lib = L.load()
    rng = np.random.default_rng(seed)
    x0 = rng.standard_normal((P, d))
    x0 /= np.linalg.norm(x0, axis=1, keepdims=True)
    if lr is None:
        lr = 0.05 * P ** (-1.0 / max(d - 1, 1))
    dev = torch.device(device if device is not None else "cuda")
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    t = torch.from_numpy(x0.astype(np.float32)).to(dev)
    with torch.cuda.device(dev):
        st = lib.fastsum_distance_qmc(int(d), int(P), int(iters), float(lr), _ptr(t),
                                      _stream_ptr(dev))
        L.check(st, "fastsum_distance_qmc")
        if rotate:
            # a Haar draw: QR of a Gaussian matrix, columns signed by diag(R)
            q, r = np.linalg.qr(rng.standard_normal((d, d)))
            qd = torch.from_numpy((q * np.sign(np.diag(r))).astype(np.float32)).to(dev)
            st = lib.fastsum_rotate_directions(int(d), int(P), _ptr(qd), _ptr(t),
                                               _stream_ptr(dev))
            L.check(st, "fastsum_rotate_directions")
    return t.cpu().numpy().T.copy()


def host_tables(kernel, d, n_ft, R, scale=1.0, T=0.0, gmax_factor=0.0, window_w=0,
                oversample=0):
    """FP64 host precompute of a plan without touching a device:
    (tau, c_0..c_K, phihat_0..phihat_{n/2})."""
    lib = L.load()
    prm = L.Params(int(d), 1, int(n_ft), int(window_w), int(oversample), L.KERNELS[kernel], 0,
                   0, float(scale), float(T), float(gmax_factor), float(R))
    n = (oversample or 2) * n_ft
    tau = ctypes.c_double()
    ck = np.empty(n_ft // 2 + 1)
    ph = np.empty(n // 2 + 1)
    st = lib.fastsum_host_tables(ctypes.byref(prm), ctypes.byref(tau),
                                 ck.ctypes.data_as(ctypes.c_void_p),
                                 ph.ctypes.data_as(ctypes.c_void_p))
    L.check(st, "fastsum_host_tables")
    return tau.value, ck, ph


def choose_nft(kernel, d, R, scale=1.0, T=0.0, gmax_factor=0.0, candidates=(256, 512, 1024),
               tol=1e-4):
    """Smallest N_ft among candidates whose discarded Fourier-coefficient mass
    is at most tol times the total (FP64 host rule of the library)."""
    lib = L.load()
    prm = L.Params(int(d), 1, int(candidates[0]), 0, 0, L.KERNELS[kernel], 0, 0, float(scale),
                   float(T), float(gmax_factor), float(R))
    arr = (ctypes.c_int32 * len(candidates))(*[int(c) for c in candidates])
    out = ctypes.c_int32()
    L.check(lib.fastsum_choose_nft(ctypes.byref(prm), arr, len(candidates), float(tol),
                                   ctypes.byref(out)), "fastsum_choose_nft")
    return out.value


class Batch:
    """Many independent kernel sums (shared kernel, P, window, T) run by one
    launch per phase and replayed from a HIP graph.

    problems: list of dicts with keys xi (d x P), n_ft, scale, R, n_max, m_max.
    With every d <= 64 the projections are computed inside the spreading and
    gathering kernels (as in a single plan); materialize=True stores them.
    """

    TUNING_KEYS = ("blocks_per_cu", "spread_chunk", "gather_group", "use_graph")

    def __init__(self, problems, *, kernel, T=0.0, gmax_factor=0.0, window_w=0, oversample=0,
                 tuning=None, device=None, materialize=False):
        lib = L.load()
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        xis = [np.ascontiguousarray(np.asarray(p["xi"], dtype=np.float32)) for p in problems]
        P = {x.shape[1] for x in xis}
        if len(P) != 1:
            raise ValueError("every problem of a batch uses the same number of directions")
        self.P = P.pop()
        self.d = [x.shape[0] for x in xis]
        self.n_max = [int(p["n_max"]) for p in problems]
        self.m_max = [int(p["m_max"]) for p in problems]
        descs = (L.ProblemDesc * len(problems))()
        for i, (p, x) in enumerate(zip(problems, xis)):
            descs[i] = L.ProblemDesc(x.shape[0], int(p["n_ft"]), float(p.get("scale", 1.0)),
                                     float(p["R"]), x.ctypes.data_as(ctypes.c_void_p),
                                     self.n_max[i], self.m_max[i])
        flags = L.FLAG_MATERIALIZE if materialize else 0
        common = L.Params(0, self.P, 0, int(window_w), int(oversample), L.KERNELS[kernel], 0, flags,
                          1.0, float(T), float(gmax_factor), 1.0)
        self._h = ctypes.c_void_p()
        tun = self._tuning_struct(tuning or {})
        with torch.cuda.device(self.device):
            st = lib.fastsum_batch_create(ctypes.byref(common), descs, len(problems),
                                          ctypes.byref(tun), _stream_ptr(self.device),
                                          ctypes.byref(self._h))
        L.check(st, "fastsum_batch_create")
        self._lib = lib
        self.n = len(problems)
        self._keep = None
        self.tuning = dict(tuning or {})

    def _tuning_struct(self, t):
        return L.BatchTuning(*[int(t.get(k, 0)) for k in self.TUNING_KEYS])

    def set_tuning(self, **kw):
        tun = self._tuning_struct(kw)
        L.check(self._lib.fastsum_batch_set_tuning(self._h, ctypes.byref(tun)),
                "fastsum_batch_set_tuning")
        self.tuning = dict(kw)

    def __call__(self, xs, ws, ys, outs=None):
        """Run every problem; returns the list of result tensors."""
        if not (len(xs) == len(ws) == len(ys) == self.n):
            raise ValueError(f"expected {self.n} problems")
        if outs is None:
            outs = [torch.empty(y.shape[0], dtype=torch.float32, device=self.device) for y in ys]
        io = (L.ProblemIO * self.n)()
        for i in range(self.n):
            x, w, y, s = xs[i], ws[i], ys[i], outs[i]
            N, M = x.shape[0], y.shape[0]
            _need(x, f"x[{i}]", (N, self.d[i]), self.device)
            _need(w, f"w[{i}]", (N,), self.device)
            _need(y, f"y[{i}]", (M, self.d[i]), self.device)
            _need(s, f"s[{i}]", (M,), self.device)
            io[i] = L.ProblemIO(x.data_ptr(), w.data_ptr(), y.data_ptr(), s.data_ptr(), N, M)
        with torch.cuda.device(self.device):
            st = self._lib.fastsum_batch_exec(self._h, io, self.n, _stream_ptr(self.device))
        L.check(st, "fastsum_batch_exec")
        self._keep = (xs, ws, ys, outs)
        return outs

    def check(self):
        with torch.cuda.device(self.device):
            L.check(self._lib.fastsum_batch_check(self._h), "fastsum_batch_check")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.fastsum_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
