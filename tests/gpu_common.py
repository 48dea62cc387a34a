"""Shared helpers of the GPU parity tests (no test functions here)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import likelihood as lk  # noqa: E402
from paper_2508_12117_amd import spider, synth  # noqa: E402


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def make_ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return spider.Context(0)


def grad_scale(prob, bt, scale, theta):
    """S_m: per-event sum over the batch of the magnitudes that enter G_m,
    c (|T_i| + |T_j| + |tau| + |t_i - t_j|) / sigma_eff^2 * |d tau^/d theta_m|.
    FP32 rounding of the network perturbs G_m by a small multiple of S_m."""
    s_eff = prob.sigma ** 2 + 2 * prob.kappa ** 2 * bt.w
    dt = np.abs(theta[bt.ev_i, 3] - theta[bt.ev_j, 3])
    mag = scale * (np.abs(bt.T_i) + np.abs(bt.T_j) + np.abs(bt.tau) + dt) / s_eff
    S = np.zeros(prob.M)
    np.add.at(S, bt.ev_i, mag * np.sqrt((bt.gT_i ** 2).sum(1) + 1))
    np.add.at(S, bt.ev_j, mag * np.sqrt((bt.gT_j ** 2).sum(1) + 1))
    return S


def scaled_grad_error(G_gpu, G_ref, S, floor):
    err = np.linalg.norm(G_gpu - G_ref, axis=1)
    return float(np.max(err / np.maximum(S, floor)))


__all__ = ["torch", "lk", "spider", "synth", "dev", "host", "make_ctx", "grad_scale",
           "scaled_grad_error"]
