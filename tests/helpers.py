"""Shared test helpers: build inputs from the workload generators, run the
GPU library and the oracle on the same arrays, and compare."""
import numpy as np

DEFAULT_T = {"gauss": 0.3, "laplace": 0.1, "energy": 0.45,
             "matern32": 0.2, "matern52": 0.2, "matern72": 0.2}


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_rel(a, b):
    """max_i |a_i - b_i| / max_i |b_i|: the element-wise companion of rel_l2."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def err_scale(a, b, s_abs):
    """||a - b|| / ||s_abs||, s_abs_m = sum_n |w_n| |F(||x_n - y_m||)|:
    relative error that stays meaningful when s cancels under signed weights."""
    return float(np.linalg.norm(np.asarray(a, np.float64) - np.asarray(b, np.float64))
                 / max(np.linalg.norm(s_abs), 1e-300))


def gpu_plan(cfg, n_ft=None, proj="fp32", grad=False, window_w=0, oversample=0, xi=None,
             n_max=None, m_max=None, R=None, materialize=False):
    import paper_2410_01316_amd as F
    xi = cfg["xi"] if xi is None else xi
    return F.Plan(xi, kernel=cfg["kernel"], n_ft=n_ft or cfg["n_ft"], scale=cfg["scale"],
                  R=R or cfg["R"], T=DEFAULT_T[cfg["kernel"]], window_w=window_w,
                  oversample=oversample, proj=proj, grad=grad, materialize=materialize,
                  n_max=n_max or cfg["x"].shape[0], m_max=m_max or cfg["y"].shape[0])


def to_dev(*arrs):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in arrs]


def oracle_inputs(cfg, x32=True):
    """The inputs exactly as the GPU sees them (rounded to float32), in float64."""
    f = (lambda a: np.asarray(a, np.float32).astype(np.float64)) if x32 else (lambda a: a)
    return f(cfg["x"]), f(cfg["y"]), f(cfg["w"]), f(cfg["xi"])
