"""Host-side checks of FastSum (the torch.autograd.Function over a plan):
which gradients it requests, how it unpacks the plan's adjoint, and that a
plan reused between a forward and its backward is re-run on the saved
inputs.  A CPU stand-in plan with the same call contract as Plan (exec
counter, grad returning (gy, gw) or (gx, gy, gw)) computes the dense
Gaussian sum and its exact adjoint; no GPU is involved."""
import pytest
import torch

from paper_2410_01316_amd.api import FastSum


class DensePlan:
    """Plan's contract on the CPU: s_m = sum_n w_n exp(-|x_n - y_m|^2 / 2)."""

    def __init__(self):
        self.execs = 0
        self._last = None

    def __call__(self, x, w, y=None, out=None):
        y = x if y is None else y
        self._last = (x, w, y)
        self.execs += 1
        return self._k(x, y).T @ w

    @staticmethod
    def _k(x, y):
        return torch.exp(-0.5 * torch.cdist(x, y) ** 2)          # (N, M)

    def grad(self, grad_s, want_y=True, want_w=True, want_x=False):
        x, w, y = self._last
        k = self._k(x, y)
        diff = x[:, None, :] - y[None, :, :]                      # (N, M, d)
        # d/dy_m of w_n k_nm = w_n k_nm (x_n - y_m)
        gy = torch.einsum("n,nm,nmd->md", w, k, diff) * grad_s[:, None] if want_y else None
        gw = k @ grad_s if want_w else None
        gx = -torch.einsum("n,nm,nmd,m->nd", w, k, diff, grad_s) if want_x else None
        return (gx, gy, gw) if want_x else (gy, gw)


def _inputs(seed=0, N=7, M=5, d=3):
    g = torch.Generator().manual_seed(seed)
    return (torch.randn(N, d, generator=g, dtype=torch.float64),
            torch.randn(M, d, generator=g, dtype=torch.float64),
            torch.rand(N, generator=g, dtype=torch.float64))


def _reference(x, y, w, v):
    x, y, w = [t.detach().clone().requires_grad_(True) for t in (x, y, w)]
    s = DensePlan._k(x, y).T @ w
    s.backward(v)
    return x.grad, y.grad, w.grad


@pytest.mark.parametrize("need", [(True, True, True), (False, True, True), (False, True, False),
                                  (False, False, True), (True, False, False)],
                         ids=["xyw", "yw", "y", "w", "x"])
def test_backward_requests_only_needed_gradients(need):
    """The canonical ds/dy, ds/dw use with fixed sources (x constant) and
    every other subset: the plan returns (gy, gw) without want_x."""
    x, y, w = _inputs()
    v = torch.linspace(-1.0, 1.0, y.shape[0], dtype=torch.float64)
    ref = _reference(x, y, w, v)
    ins = [t.clone().requires_grad_(r) for t, r in zip((x, y, w), need)]
    s = FastSum.apply(DensePlan(), *ins)
    s.backward(v)
    for t, r, g in zip(ins, need, ref):
        if r:
            assert torch.allclose(t.grad, g, rtol=1e-12, atol=1e-12)
        else:
            assert t.grad is None


def test_plan_reused_before_backward_is_rerun_on_saved_inputs():
    """Two sums on one plan in one graph: the first backward must not use
    the second call's kept state."""
    plan = DensePlan()
    x1, y1, w1 = [t.requires_grad_(True) for t in _inputs(1)]
    x2, y2, w2 = [t.requires_grad_(True) for t in _inputs(2)]
    s1 = FastSum.apply(plan, x1, y1, w1)
    s2 = FastSum.apply(plan, x2, y2, w2)
    v = torch.ones(y1.shape[0], dtype=torch.float64)
    (s1 @ v + 2.0 * (s2 @ v)).backward()
    for t, g in zip((x1, y1, w1), _reference(x1, y1, w1, v)):
        assert torch.allclose(t.grad, g, rtol=1e-12, atol=1e-12)
    for t, g in zip((x2, y2, w2), _reference(x2, y2, w2, 2.0 * v)):
        assert torch.allclose(t.grad, g, rtol=1e-12, atol=1e-12)
    assert plan.execs == 3          # the first sum was run again once


def test_inputs_modified_in_place_after_forward_raise():
    x, y, w = _inputs()
    y.requires_grad_(True)
    wl = w.clone()
    s = FastSum.apply(DensePlan(), x, y, wl)
    wl.mul_(2.0)                    # the sum no longer matches its inputs
    with pytest.raises(RuntimeError):
        s.sum().backward()


def test_targets_equal_to_sources():
    x, _, w = _inputs()
    x.requires_grad_(True)
    s = FastSum.apply(DensePlan(), x, x, w)
    v = torch.ones(x.shape[0], dtype=torch.float64)
    s.backward(v)
    xr = x.detach().clone().requires_grad_(True)
    (DensePlan._k(xr, xr).T @ w @ v).backward()
    assert torch.allclose(x.grad, xr.grad, rtol=1e-12, atol=1e-12)
