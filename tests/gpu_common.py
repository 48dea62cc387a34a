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
    sig, kap = prob.row_sigma_kappa(bt.phase)
    s_eff = sig ** 2 + 2 * kap ** 2 * bt.w
    dt = np.abs(theta[bt.ev_i, 3] - theta[bt.ev_j, 3])
    mag = scale * (np.abs(bt.T_i) + np.abs(bt.T_j) + np.abs(bt.tau) + dt) / s_eff
    S = np.zeros(prob.M)
    np.add.at(S, bt.ev_i, mag * np.sqrt((bt.gT_i ** 2).sum(1) + 1))
    np.add.at(S, bt.ev_j, mag * np.sqrt((bt.gT_j ** 2).sum(1) + 1))
    return S


def sigma_apply(z, w, group, ev_i, ev_j, M, sigma, kappa, mode):
    """Sigma_B z for the batch covariance of eq:marginal_sigma (matrix-free):
    sigma^2 z + kappa^2 U (U^T z), U = diag(sqrt w) A_B, where row n of A_B
    has +1 at node (group_n, ev_i_n) and -1 at node (group_n, ev_j_n).  sigma
    and kappa are scalars or per-row values (a row's group's phase)."""
    s2 = np.asarray(sigma, np.float64) ** 2
    k2 = np.asarray(kappa, np.float64) ** 2
    if mode == lk.WHITEN_NONE or np.all(k2 == 0.0):
        return s2 * z
    if mode == lk.WHITEN_DIAG:
        return (s2 + 2.0 * k2 * w) * z
    key_i = np.asarray(group, np.int64) * M + ev_i
    key_j = np.asarray(group, np.int64) * M + ev_j
    nodes, inv = np.unique(np.concatenate([key_i, key_j]), return_inverse=True)
    n = z.shape[0]
    sw = np.sqrt(k2 * w) * np.ones(n)  # kappa_n sqrt(w_n): groups never mix phases
    utz = np.bincount(inv[:n], sw * z, nodes.shape[0]) - np.bincount(inv[n:], sw * z,
                                                                       nodes.shape[0])
    return s2 * z + sw * (utz[inv[:n]] - utz[inv[n:]])


def whitening_residual(r, z, bt, prob, mode):
    """max |Sigma_B z - r| / (|r| + 1e-3 s): how exactly z solves the batch
    system for the residuals r it was computed from."""
    sig, kap = prob.row_sigma_kappa(bt.phase)
    Sz = sigma_apply(z, bt.w, bt.group, bt.ev_i, bt.ev_j, prob.M, sig, kap, mode)
    return float(np.max(np.abs(Sz - r) / (np.abs(r) + 1e-3)))


def woodbury_floor(r, w, group, ev_i, ev_j, M, sigma, kappa):
    """The rounding floor of the Woodbury form the GPU uses, for the same r:
    y from a direct sparse FP64 solve of (lambda I + U^T U) y = U^T r
    (lambda = sigma^2/kappa^2, U = W^1/2 A_B), then z = (r - U y)/sigma^2;
    returns whitening_residual's measure of that z.  The subtraction r - U y
    cancels most of r where groups are dense, so this floor sits well above
    that of a direct solve of Sigma_B z = r."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    key_i = np.asarray(group, np.int64) * M + ev_i
    key_j = np.asarray(group, np.int64) * M + ev_j
    nodes, inv = np.unique(np.concatenate([key_i, key_j]), return_inverse=True)
    n = r.shape[0]
    sw = np.sqrt(w)
    rows = np.concatenate([np.arange(n), np.arange(n)])
    U = sp.csr_matrix((np.concatenate([sw, -sw]), (rows, inv)), shape=(n, nodes.shape[0]))
    lam = sigma ** 2 / kappa ** 2
    K = (sp.identity(nodes.shape[0]) * lam + U.T @ U).tocsc()
    y = spla.spsolve(K, U.T @ r)
    z = (r - U @ y) / sigma ** 2
    Sz = sigma_apply(z, w, group, ev_i, ev_j, M, sigma, kappa, lk.WHITEN_EXACT)
    return float(np.max(np.abs(Sz - r) / (np.abs(r) + 1e-3)))


def psgld_update_tolerance(theta, v, G, dG, cfg, eta):
    """How far one pSGLD update (state theta, v) can move when its gradient G
    is off by up to dG per entry: the drift eps G / (sqrt(v') + eps_p) is
    monotone in G, v' = beta2 v + (1 - beta2) G^2 and the noise
    sqrt(2 eps / (sqrt(v') + eps_p)) eta depend on |G| only, so each term's
    extremes over [G - dG, G + dG] lie at the ends or at G = 0.  Returns
    (theta tolerance, v tolerance): twice the extreme deviations, plus FP64
    rounding."""
    def parts(g):
        vn = cfg.beta2 * v + (1.0 - cfg.beta2) * g * g
        q = np.sqrt(vn) + cfg.eps_p
        return vn, cfg.step * g / q, cfg.noise_scale * np.sqrt(2.0 * cfg.step / q) * eta
    v0, d0, n0 = parts(G)
    tv = np.zeros_like(G)
    td = np.zeros_like(G)
    tn = np.zeros_like(G)
    for g in (G - dG, G + dG, np.where(np.abs(G) <= dG, 0.0, G)):
        vn, d, n = parts(g)
        tv = np.maximum(tv, np.abs(vn - v0))
        td = np.maximum(td, np.abs(d - d0))
        tn = np.maximum(tn, np.abs(n - n0))
    return (2.0 * (td + tn) + 1e-13 * (np.abs(theta) + np.abs(d0) + np.abs(n0)),
            2.0 * tv + 1e-13 * np.abs(v0))


def scaled_grad_error(G_gpu, G_ref, S, floor):
    err = np.linalg.norm(G_gpu - G_ref, axis=1)
    return float(np.max(err / np.maximum(S, floor)))


__all__ = ["torch", "lk", "spider", "synth", "dev", "host", "make_ctx", "grad_scale",
           "scaled_grad_error", "sigma_apply", "whitening_residual", "psgld_update_tolerance",
           "woodbury_floor"]
