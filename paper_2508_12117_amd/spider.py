"""ctypes binding of libspider (include/spider.h): argument marshalling only.

Every computation runs in the HIP library.  Device arrays are torch tensors
on the context's device; the binding passes their pointers and the current
torch stream.  The library must have been built (``__graft_entry__.build()``
or ``python -m paper_2508_12117_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as ct
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspider.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "spider.h")

OK, E_INVALID, E_OOM, E_HIP, E_STATE, E_UNSUPPORTED, E_NUMERIC = 0, -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
WHITEN_NONE, WHITEN_DIAG, WHITEN_EXACT = 0, 1, 2
FP32, BF16 = 0, 1
GRAD_PRIOR, GRAD_CENTROID, GRAD_L1 = 1, 2, 4
MAX_LAYERS = 16

_ERRNAMES = {E_INVALID: "invalid", E_OOM: "out of memory", E_HIP: "HIP error",
             E_STATE: "bad state", E_UNSUPPORTED: "unsupported", E_NUMERIC: "numeric"}


class SpiderError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class CatalogDesc(ct.Structure):
    _fields_ = [("M", ct.c_int32), ("L", ct.c_int32), ("P", ct.c_int32), ("N", ct.c_int64),
                ("mem", ct.c_int32),
                ("hypo0", ct.c_void_p), ("stations", ct.c_void_p),
                ("pair_i", ct.c_void_p), ("pair_j", ct.c_void_p),
                ("obs_pair", ct.c_void_p), ("obs_sta", ct.c_void_p), ("obs_dt", ct.c_void_p),
                ("sigma", ct.c_double), ("kappa", ct.c_double), ("p", ct.c_double),
                ("ell", ct.c_double), ("eps_w", ct.c_double),
                ("prior_sigma", ct.c_double * 4), ("centroid_sigma", ct.c_double * 4),
                ("stream", ct.c_uint32), ("whiten", ct.c_int32),
                ("obs_phase", ct.c_void_p), ("sigma_s", ct.c_double), ("kappa_s", ct.c_double)]


class NetDesc(ct.Structure):
    _fields_ = [("D", ct.c_int32), ("H", ct.c_int32), ("mem", ct.c_int32),
                ("W", ct.c_void_p * (MAX_LAYERS + 1)), ("b", ct.c_void_p * (MAX_LAYERS + 1)),
                ("v0", ct.c_double), ("center", ct.c_double * 3),
                ("half_extent", ct.c_double * 3)]


class ChainSet(ct.Structure):
    _fields_ = [("cat_id", ct.c_int32), ("net_id", ct.c_int32), ("n_chains", ct.c_int32),
                ("precision", ct.c_int32), ("batch", ct.c_int64)]


class SgldCfg(ct.Structure):
    _fields_ = [("step", ct.c_double), ("beta2", ct.c_double), ("eps_p", ct.c_double),
                ("noise_scale", ct.c_double), ("precond", ct.c_int32), ("noise_ramp", ct.c_int32),
                ("n_steps", ct.c_int64), ("burn_in", ct.c_int64), ("thin", ct.c_int64),
                ("seed", ct.c_uint64), ("noise_scale_end", ct.c_double)]


class MapCfg(ct.Structure):
    _fields_ = [("lr", ct.c_double), ("beta1", ct.c_double), ("beta2", ct.c_double),
                ("eps", ct.c_double), ("n_steps", ct.c_int64), ("seed", ct.c_uint64)]


_P = ct.c_void_p
_SIGS = {
    "spider_version": ([], ct.c_int),
    "spider_create": ([ct.POINTER(_P), ct.c_int, _P], ct.c_int),
    "spider_destroy": ([_P], None),
    "spider_last_error": ([_P], ct.c_char_p),
    "spider_sync": ([_P], ct.c_int),
    "spider_load_catalog": ([_P, ct.POINTER(CatalogDesc), ct.POINTER(ct.c_int32)], ct.c_int),
    "spider_load_net": ([_P, ct.POINTER(NetDesc), ct.POINTER(ct.c_int32)], ct.c_int),
    "spider_travel_time": ([_P, ct.c_int32, ct.c_int32, _P, _P, ct.c_int64, _P, _P], ct.c_int),
    "spider_tt_forward": ([_P, ct.c_int32, ct.c_int32, _P, _P, ct.c_int64, _P], ct.c_int),
    "spider_tt_backward": ([_P, ct.c_int32, ct.c_int32, _P, _P, _P, ct.c_int64, _P], ct.c_int),
    "spider_travel_time_noalloc": ([_P, ct.c_int32, ct.c_int32, _P, _P, ct.c_int64, _P, _P],
                                   ct.c_int),
    "spider_grad": ([_P, ct.c_int32, ct.c_int32, ct.c_int32, _P, _P, ct.c_int64, ct.c_uint64,
                     ct.c_int32, ct.c_int64, ct.c_uint32, _P, _P], ct.c_int),
    "spider_batch_terms": ([_P, ct.c_int32, ct.c_int32, ct.c_int32, _P, _P, ct.c_int64,
                            ct.c_uint64, ct.c_int32, ct.c_int64, _P, _P, _P, _P, _P, _P],
                           ct.c_int),
    "spider_batch_indices": ([_P, ct.c_int32, ct.c_uint64, ct.c_int32, ct.c_int64, ct.c_int64,
                              _P], ct.c_int),
    "spider_noise": ([_P, ct.c_int32, ct.c_uint64, ct.c_int32, ct.c_int64, _P], ct.c_int),
    "spider_reset_chains": ([_P, ct.c_int32, ct.c_int32], ct.c_int),
    "spider_sgld_steps": ([_P, ct.POINTER(ChainSet), ct.c_int32, ct.POINTER(SgldCfg)], ct.c_int),
    "spider_set_graphs": ([_P, ct.c_int], ct.c_int),
    "spider_map_steps": ([_P, ct.POINTER(ChainSet), ct.c_int32, ct.POINTER(MapCfg)], ct.c_int),
    "spider_outliers": ([_P, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_double, _P,
                         ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)],
                        ct.c_int),
    "spider_set_phase_net": ([_P, ct.c_int32, ct.c_int32], ct.c_int),
    "spider_linearity": ([_P, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_double, _P,
                          ct.POINTER(ct.c_int64)], ct.c_int),
    "spider_set_sample_buffer": ([_P, ct.c_int32, _P, ct.c_int64], ct.c_int),
    "spider_quantiles": ([_P, _P, ct.c_int64, ct.c_int64, _P, ct.c_int32, _P], ct.c_int),
    "spider_sample_ranks": ([_P, _P, ct.c_int64, ct.c_int64, _P, _P], ct.c_int),
    "spider_ess": ([_P, _P, ct.c_int64, ct.c_int32, ct.c_int64, _P], ct.c_int),
    "spider_noise_ratio": ([_P, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int64,
                            ct.c_int32, _P, _P, ct.POINTER(ct.c_double)], ct.c_int),
    "spider_moments": ([_P, ct.c_int32, ct.c_int32, _P, _P, ct.POINTER(ct.c_int64)], ct.c_int),
    "spider_get_state": ([_P, ct.c_int32, ct.c_int32, _P, _P, ct.POINTER(ct.c_int64)], ct.c_int),
    "spider_set_state": ([_P, ct.c_int32, ct.c_int32, _P, _P, ct.c_int64], ct.c_int),
    "spider_profile": ([_P, ct.c_int], ct.c_int),
    "spider_network_variant": ([_P, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32),
                                ct.POINTER(ct.c_int32)], ct.c_int),
    "spider_profile_read": ([_P, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64),
                             ct.POINTER(ct.c_int64)], ct.c_int),
}

_lib = None


def header_functions():
    """Names of the functions include/spider.h declares."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spider_[a-z_0-9]+)\s*\(", text)))


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2508_12117_amd.build`")
        L = ct.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ct.c_void_p(t.data_ptr())


def _np_ptr(a):
    return ct.c_void_p(a.ctypes.data)


class Context:
    """One libspider context on a device, enqueueing on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = ct.c_void_p()
        rc = lib().spider_create(ct.byref(h), device, ct.c_void_p(stream.cuda_stream))
        if rc != OK:
            raise SpiderError(rc, f"spider_create(device={device}) failed")
        self._h = h
        self._keep = []
        self._n_obs = {}  # observations of each loaded catalog
        self._n_ev = {}   # and its events

    def close(self):
        if getattr(self, "_h", None):
            lib().spider_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc):
        if rc != OK:
            raise SpiderError(rc, lib().spider_last_error(self._h).decode())

    def sync(self):
        self._check(lib().spider_sync(self._h))

    # ---- loading
    def load_catalog(self, cat, whiten=WHITEN_EXACT, stream_id=0, sigma=None, kappa=None,
                     p=None, ell=None, eps_w=None, sigma_s=None, kappa_s=None) -> int:
        """Load a catalog; one with S observations (cat.obs_phase) also needs
        set_phase_net before it is evaluated."""
        wl = cat.wl
        arrays = dict(
            hypo0=np.ascontiguousarray(cat.hypo0, np.float64),
            stations=np.ascontiguousarray(cat.stations, np.float64),
            pair_i=np.ascontiguousarray(cat.pair_i, np.int32),
            pair_j=np.ascontiguousarray(cat.pair_j, np.int32),
            obs_pair=np.ascontiguousarray(cat.obs_pair, np.int32),
            obs_sta=np.ascontiguousarray(cat.obs_sta, np.int16),
            obs_dt=np.ascontiguousarray(cat.obs_dt, np.float32))
        phase = getattr(cat, "obs_phase", None)
        if phase is not None:
            arrays["obs_phase"] = np.ascontiguousarray(phase, np.int8)
        d = CatalogDesc()
        d.M, d.L, d.P, d.N = cat.M, cat.L, cat.P, cat.N
        d.mem = MEM_HOST
        for k, a in arrays.items():
            setattr(d, k, _np_ptr(a))
        d.sigma = wl.sigma if sigma is None else sigma
        d.kappa = wl.kappa if kappa is None else kappa
        d.p = wl.p if p is None else p
        d.ell = wl.ell if ell is None else ell
        d.eps_w = wl.eps_w if eps_w is None else eps_w
        d.prior_sigma[:] = list(wl.prior_sigma)
        d.centroid_sigma[:] = list(wl.centroid_sigma)
        d.stream = stream_id
        d.whiten = whiten
        d.sigma_s = getattr(wl, "sigma_s", d.sigma) if sigma_s is None else sigma_s
        d.kappa_s = getattr(wl, "kappa_s", d.kappa) if kappa_s is None else kappa_s
        cid = ct.c_int32()
        self._check(lib().spider_load_catalog(self._h, ct.byref(d), ct.byref(cid)))
        self._n_obs[cid.value] = cat.N
        self._n_ev[cid.value] = cat.M
        return cid.value

    def set_phase_net(self, cat_id, net_id):
        """The S-phase network of a two-phase catalog."""
        self._check(lib().spider_set_phase_net(self._h, cat_id, net_id))

    def load_net(self, net) -> int:
        W = [np.ascontiguousarray(w, np.float32) for w in net.W]
        B = [np.ascontiguousarray(b, np.float32) for b in net.b]
        d = NetDesc()
        d.D, d.H, d.mem = net.D, net.H, MEM_HOST
        for l in range(net.D + 1):
            d.W[l] = W[l].ctypes.data
            d.b[l] = B[l].ctypes.data
        d.v0 = net.v0
        d.center[:] = list(map(float, net.center))
        d.half_extent[:] = list(map(float, net.half_extent))
        nid = ct.c_int32()
        self._check(lib().spider_load_net(self._h, ct.byref(d), ct.byref(nid)))
        return nid.value

    # ---- hot path
    def travel_time(self, net_id, x_src, s, T, gradT=None, precision=FP32):
        self._check(lib().spider_travel_time(self._h, net_id, precision, _ptr(x_src), _ptr(s),
                                             x_src.shape[0], _ptr(T), _ptr(gradT)))

    def travel_time_noalloc(self, net_id, x_src, s, T, gradT=None, precision=FP32):
        self._check(lib().spider_travel_time_noalloc(self._h, net_id, precision, _ptr(x_src),
                                                     _ptr(s), x_src.shape[0], _ptr(T),
                                                     _ptr(gradT)))

    def tt_forward(self, net_id, x_src, s, T, precision=FP32):
        self._check(lib().spider_tt_forward(self._h, net_id, precision, _ptr(x_src), _ptr(s),
                                            x_src.shape[0], _ptr(T)))

    def tt_backward(self, net_id, x_src, s, grad_T, grad_x, precision=FP32):
        self._check(lib().spider_tt_backward(self._h, net_id, precision, _ptr(x_src), _ptr(s),
                                             _ptr(grad_T), x_src.shape[0], _ptr(grad_x)))

    def grad(self, cat_id, net_id, theta, grad_out, batch_idx=None, n=None, seed=0, chain=0,
             step=0, flags=GRAD_PRIOR | GRAD_CENTROID, logpost=None, precision=FP32):
        n = batch_idx.shape[0] if batch_idx is not None else n
        self._check(lib().spider_grad(self._h, cat_id, net_id, precision, _ptr(theta),
                                      _ptr(batch_idx), n, seed, chain, step, flags,
                                      _ptr(grad_out), _ptr(logpost)))

    def batch_terms(self, cat_id, net_id, theta, batch_idx=None, n=None, seed=0, chain=0, step=0,
                    precision=FP32, out=None):
        """Returns dict of T_i, T_j, gT_i, gT_j, r, z device tensors."""
        torch = self._torch
        n = batch_idx.shape[0] if batch_idx is not None else n
        dev = theta.device
        if out is None:
            out = dict(T_i=torch.empty(n, dtype=torch.float64, device=dev),
                       T_j=torch.empty(n, dtype=torch.float64, device=dev),
                       gT_i=torch.empty(n, 3, dtype=torch.float64, device=dev),
                       gT_j=torch.empty(n, 3, dtype=torch.float64, device=dev),
                       r=torch.empty(n, dtype=torch.float64, device=dev),
                       z=torch.empty(n, dtype=torch.float64, device=dev))
        self._check(lib().spider_batch_terms(
            self._h, cat_id, net_id, precision, _ptr(theta), _ptr(batch_idx), n, seed, chain,
            step, _ptr(out["T_i"]), _ptr(out["T_j"]), _ptr(out["gT_i"]), _ptr(out["gT_j"]),
            _ptr(out["r"]), _ptr(out["z"])))
        return out

    def batch_indices(self, cat_id, seed, chain, step, n, out):
        self._check(lib().spider_batch_indices(self._h, cat_id, seed, chain, step, n, _ptr(out)))

    def noise(self, cat_id, seed, chain, step, out):
        self._check(lib().spider_noise(self._h, cat_id, seed, chain, step, _ptr(out)))

    def reset_chains(self, cat_id, n_chains):
        self._check(lib().spider_reset_chains(self._h, cat_id, n_chains))

    def sgld_steps(self, sets, n_steps, step=1e-4, beta2=0.99, eps_p=1e-5, noise_scale=1.0,
                   precond=1, burn_in=0, thin=1, seed=0, noise_scale_end=None):
        """sets: list of (cat_id, net_id, n_chains, batch, precision).  With
        noise_scale_end the noise amplitude ramps linearly from noise_scale
        over the call (step k uses noise_scale + (end - noise_scale) k / n_steps)."""
        arr = (ChainSet * len(sets))()
        for k, (cid, nid, C, n, prec) in enumerate(sets):
            arr[k].cat_id, arr[k].net_id, arr[k].n_chains = cid, nid, C
            arr[k].precision, arr[k].batch = prec, n
        ramp = noise_scale_end is not None
        cfg = SgldCfg(step=step, beta2=beta2, eps_p=eps_p, noise_scale=noise_scale,
                      precond=precond, noise_ramp=1 if ramp else 0, n_steps=n_steps,
                      burn_in=burn_in, thin=thin, seed=seed,
                      noise_scale_end=noise_scale_end if ramp else 0.0)
        self._check(lib().spider_sgld_steps(self._h, arr, len(sets), ct.byref(cfg)))

    def set_graphs(self, enable: bool):
        """Replay sampler steps from a captured HIP graph (default) or launch
        every step on the stream."""
        self._check(lib().spider_set_graphs(self._h, 1 if enable else 0))

    def map_steps(self, sets, n_steps, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0):
        """Stage 1: Adam on the minibatch L1 loss of the dd residuals, no priors.
        sets: list of (cat_id, net_id, n_chains, batch, precision)."""
        arr = (ChainSet * len(sets))()
        for k, (cid, nid, C, n, prec) in enumerate(sets):
            arr[k].cat_id, arr[k].net_id, arr[k].n_chains = cid, nid, C
            arr[k].precision, arr[k].batch = prec, n
        cfg = MapCfg(lr=lr, beta1=beta1, beta2=beta2, eps=eps, n_steps=n_steps, seed=seed)
        self._check(lib().spider_map_steps(self._h, arr, len(sets), ct.byref(cfg)))

    def outliers(self, cat_id, net_id, chain=0, k_mad=4.0, precision=FP32):
        """Outlier screening at a chain's state: (keep [N] uint8 device
        tensor, kept count, median, MAD) of the residuals of all observations."""
        torch = self._torch
        keep = torch.empty(self._n_obs.get(cat_id, 0), dtype=torch.uint8,
                           device=f"cuda:{self.device}")
        n, med, mad = ct.c_int64(), ct.c_double(), ct.c_double()
        self._check(lib().spider_outliers(self._h, cat_id, net_id, precision, chain, k_mad,
                                          _ptr(keep), ct.byref(n), ct.byref(med), ct.byref(mad)))
        return keep, n.value, med.value, mad.value

    def linearity(self, cat_id, net_id, chain=0, max_rel_err=0.05, precision=FP32):
        """Linear-regime data filter at a chain's state: (keep [N] uint8
        device tensor, kept count)."""
        torch = self._torch
        keep = torch.empty(self._n_obs.get(cat_id, 0), dtype=torch.uint8,
                           device=f"cuda:{self.device}")
        n = ct.c_int64()
        self._check(lib().spider_linearity(self._h, cat_id, net_id, precision, chain,
                                           max_rel_err, _ptr(keep), ct.byref(n)))
        return keep, n.value

    def set_sample_buffer(self, cat_id, samples):
        """Attach a device tensor [K, C, M, 4] (float64) that receives the
        recorded states of the catalog's C chains; None detaches."""
        if samples is None:
            self._check(lib().spider_set_sample_buffer(self._h, cat_id, None, 0))
            return
        self._keep.append(samples)
        self._check(lib().spider_set_sample_buffer(self._h, cat_id, _ptr(samples),
                                                   samples.shape[0]))

    def quantiles(self, samples, probs):
        """Percentiles over the first axis of a device tensor [S, ...]:
        returns [len(probs), ...]."""
        torch = self._torch
        S = samples.shape[0]
        P = samples.numel() // S
        pr = np.ascontiguousarray(probs, np.float64)
        out = torch.empty((len(pr),) + tuple(samples.shape[1:]), dtype=torch.float64,
                          device=samples.device)
        self._check(lib().spider_quantiles(self._h, _ptr(samples), S, P, _np_ptr(pr), len(pr),
                                           _ptr(out)))
        return out

    def sample_ranks(self, samples, values):
        """Position of values [...] among samples [S, ...] (fractions)."""
        torch = self._torch
        S = samples.shape[0]
        out = torch.empty(values.shape, dtype=torch.float64, device=samples.device)
        self._check(lib().spider_sample_ranks(self._h, _ptr(samples), S, values.numel(),
                                              _ptr(values), _ptr(out)))
        self.sync()
        return out

    def ess(self, samples):
        """Effective sample size of draws [K, C, ...]: returns [...]."""
        torch = self._torch
        K, C = samples.shape[0], samples.shape[1]
        out = torch.empty(tuple(samples.shape[2:]), dtype=torch.float64, device=samples.device)
        self._check(lib().spider_ess(self._h, _ptr(samples), K, C, out.numel(), _ptr(out)))
        self.sync()
        return out

    def noise_ratio(self, cat_id, net_id, chain, batch, n_batches, step=1e-4, eps_p=1e-5,
                    noise_scale=1.0, precond=1, seed=0, precision=FP32):
        """Gradient-noise to injected-noise variance ratio [M, 4] at a
        chain's state, and its mean."""
        torch = self._torch
        cfg = SgldCfg(step=step, beta2=0.99, eps_p=eps_p, noise_scale=noise_scale,
                      precond=precond, noise_ramp=0, n_steps=0, burn_in=0, thin=1, seed=seed,
                      noise_scale_end=noise_scale)
        out = torch.empty(self._n_ev.get(cat_id, 0), 4, dtype=torch.float64,
                          device=f"cuda:{self.device}")
        mean = ct.c_double()
        self._check(lib().spider_noise_ratio(self._h, cat_id, net_id, precision, chain, batch,
                                             n_batches, ct.byref(cfg), _ptr(out),
                                             ct.byref(mean)))
        return out, mean.value

    def sgld_stages(self, sets, warmup, ramp, sample, thin=1, **kw):
        """The sampler stages that follow the initial solution (Sec. 3.2):
        `warmup` steps with the injected noise off, `ramp` steps raising it
        linearly to full amplitude, `sample` steps at full amplitude whose
        states enter the posterior moments (every `thin`-th)."""
        try:
            t0 = self.get_state(sets[0][0], 0)
        except SpiderError:  # no chains yet: they start at step 0
            t0 = 0
        burn = t0 + warmup + ramp  # global step of the first sample
        if warmup > 0:
            self.sgld_steps(sets, warmup, noise_scale=0.0, burn_in=burn, thin=thin, **kw)
        if ramp > 0:
            self.sgld_steps(sets, ramp, noise_scale=0.0, noise_scale_end=1.0, burn_in=burn,
                            thin=thin, **kw)
        if sample > 0:
            self.sgld_steps(sets, sample, noise_scale=1.0, burn_in=burn, thin=thin, **kw)

    def moments(self, cat_id, chain, mean, cov):
        cnt = ct.c_int64()
        self._check(lib().spider_moments(self._h, cat_id, chain, _ptr(mean), _ptr(cov),
                                         ct.byref(cnt)))
        return cnt.value

    def get_state(self, cat_id, chain, theta=None, v=None):
        step = ct.c_int64()
        self._check(lib().spider_get_state(self._h, cat_id, chain, _ptr(theta), _ptr(v),
                                           ct.byref(step)))
        return step.value

    def profile(self, enable: bool):
        self._check(lib().spider_profile(self._h, 1 if enable else 0))

    def network_variant(self, net_id, precision=FP32):
        """(waves per workgroup, 16-row tiles per workgroup) of the chosen kernel."""
        w, r = ct.c_int32(), ct.c_int32()
        self._check(lib().spider_network_variant(self._h, net_id, precision, ct.byref(w),
                                                 ct.byref(r), None))
        return w.value, r.value

    def network_schedule(self, net_id, precision=FP32):
        """Schedule of the chosen kernel: 0 one barrier per layer, 1 row-half
        ping-pong with a one-layer weight ring, 2 the same with a 1.5-layer ring."""
        sc = ct.c_int32()
        self._check(lib().spider_network_variant(self._h, net_id, precision, None, None,
                                                 ct.byref(sc)))
        return sc.value

    def profile_read(self):
        """(summed network-kernel ms, launches, rows) since profile(True)."""
        ms, n, rows = ct.c_double(), ct.c_int64(), ct.c_int64()
        self._check(lib().spider_profile_read(self._h, ct.byref(ms), ct.byref(n), ct.byref(rows)))
        return ms.value, n.value, rows.value

    def set_state(self, cat_id, chain, theta, v=None, step=0):
        self._check(lib().spider_set_state(self._h, cat_id, chain, _ptr(theta), _ptr(v), step))
