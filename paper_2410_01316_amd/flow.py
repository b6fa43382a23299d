"""MMD gradient flow with momentum driven by the fast sum (App. MMD flows).

For targets y (M points) and particles x (N points) the discrete MMD
functional is
    G_y(x) = 1/(2N^2) sum_ij K(x_i, x_j) - 1/(MN) sum_ij K(x_i, y_j)
             + 1/(2M^2) sum_ij K(y_i, y_j),
and grad_{x_i} G is the target derivative of ONE kernel sum: sources
z = [x; y] with weights [1/N^2 (N times), -1/(MN) (M times)], evaluated at
the targets x (the symmetric self term is counted twice, which cancels the
1/2).  A step is one fastsum_exec and one fastsum_grad (grad_y only), then
the momentum update of the paper,
    v <- grad G(x) + m v,   x <- x - tau v      (v starts at 0),
by fastsum_flow_update, which also writes the new particles into their
rows of z and returns their largest norm.  The bound R of the plan must
cover the moving particles: max ||z|| + max ||x|| = max(|x|, |y|) + |x|
with |y| taken once; the plan is rebuilt with a margin whenever they leave
it.
"""
import numpy as np
import torch

from . import _lib as L
from .api import Plan, bound, _ptr, _stream_ptr


class MMDFlow:
    """Particles flowing towards the targets y (M x d, float32 on the GPU).

    xi: (d, P) directions; kernel, n_ft, scale, T, window_w as in Plan;
    sorting: exact 1-D sums and derivatives by sorting (energy kernel);
    step: tau of the Euler step; momentum: m; margin: factor applied to the
    particles' current bound when the plan is (re)built.
    """

    def __init__(self, y, xi, n_particles, *, kernel="energy", n_ft=1024, scale=1.0, T=0.0,
                 window_w=0, sorting=False, step=1.0, momentum=0.9, margin=1.5):
        if not (isinstance(y, torch.Tensor) and y.dtype == torch.float32 and y.is_cuda):
            raise ValueError("y must be a float32 tensor on the GPU")
        self.y = y.contiguous()
        self.M, self.d = self.y.shape
        self.N = int(n_particles)
        self.xi = np.ascontiguousarray(np.asarray(xi, dtype=np.float32))
        if self.xi.shape[0] != self.d:
            raise ValueError("xi must be (d, P)")
        self.kernel, self.n_ft, self.scale, self.T, self.window_w = kernel, n_ft, scale, T, window_w
        self.sorting = bool(sorting)
        self.step_size, self.momentum, self.margin = float(step), float(momentum), float(margin)
        dev = self.y.device
        N, M = self.N, self.M
        self.z = torch.empty((N + M, self.d), dtype=torch.float32, device=dev)
        self.z[N:].copy_(self.y)
        self.w = torch.cat([torch.full((N,), 1.0 / N ** 2, dtype=torch.float32, device=dev),
                            torch.full((M,), -1.0 / (M * N), dtype=torch.float32, device=dev)])
        self.ones = torch.ones(N, dtype=torch.float32, device=dev)
        self.s = torch.empty(N, dtype=torch.float32, device=dev)
        self.plan, self.R, self.rebuilds = None, 0.0, 0
        self.y_norm = 0.5 * bound(self.y, self.y)           # max ||y_m||
        self.x_norm2 = torch.zeros(1, dtype=torch.float32, device=dev)
        self._synced = None      # (pointer, version) of the x that z[:N] and x_norm2 describe

    def _sync(self, x):
        """max ||x_n||; copies x into z first unless the last step wrote it
        (an in-place change of x since then shows in its version counter)."""
        if not (x.dtype == torch.float32 and x.is_cuda and x.shape == (self.N, self.d)
                and x.is_contiguous()):
            raise ValueError("x must be a contiguous (N, d) float32 tensor on the GPU")
        if self._synced == (x.data_ptr(), x._version):
            return float(torch.sqrt(self.x_norm2).item())
        self.z[: self.N].copy_(x)
        return 0.5 * bound(x, x)

    def _ensure_plan(self, x_norm):
        # sources z = [x; y] and targets x about the origin (App. J,
        # eq. radius_xy)
        need = max(x_norm, self.y_norm) + x_norm
        if self.plan is not None and need * (1.0 + 1e-4) <= self.R:
            return
        if self.plan is not None:
            self.plan.close()
        self.R = self.margin * need
        self.plan = Plan(self.xi, kernel=self.kernel, n_ft=self.n_ft, R=self.R, scale=self.scale,
                         T=self.T, window_w=self.window_w, grad=True, sorting=self.sorting,
                         n_max=self.N + self.M,
                         m_max=self.N, device=self.y.device)
        self.rebuilds += 1

    def gradient(self, x):
        """grad G_y at the particles x (N x d); returns a new tensor."""
        self._ensure_plan(self._sync(x))
        # targets: the particles as the first N rows of z (the plan projects
        # them once, as sources and as targets)
        self.plan(self.z, self.w, self.z[: self.N], out=self.s)
        gy, _ = self.plan.grad(self.ones, want_y=True, want_w=False)
        return gy

    def step(self, x, v):
        """One momentum step in place on x and v; returns the R used."""
        g = self.gradient(x)
        if not (v.dtype == torch.float32 and v.shape == x.shape and v.is_contiguous()
                and v.device == x.device):
            raise ValueError("v must be a contiguous float32 tensor shaped like x")
        st = L.load().fastsum_flow_update(self.N, self.d, self.momentum, self.step_size,
                                          _ptr(g), _ptr(v), _ptr(x), _ptr(self.z),
                                          _ptr(self.x_norm2), _stream_ptr(x.device))
        L.check(st, "fastsum_flow_update")
        self._synced = (x.data_ptr(), x._version)
        return self.R

    def run(self, x0, steps, callback=None):
        """Flow x0 (N x d, float32 on the GPU) for `steps` steps; callback(k, x, R)
        after each step.  Returns the final particles."""
        x = x0.clone().contiguous()
        v = torch.zeros_like(x)
        for k in range(steps):
            R = self.step(x, v)
            if callback is not None:
                callback(k, x, R)
        return x

    def close(self):
        if self.plan is not None:
            self.plan.close()
            self.plan = None
