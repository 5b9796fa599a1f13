"""ctypes binding of the screening entry points (include/rimp2_screen.h) and a
small training driver.  Argument marshalling and loop control only: features,
network passes, gradients and Adam steps run in the library's HIP kernels."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from .rimp2 import _check, _ptr, _stream_handle, lib

N_PARAMS = 64 * 4 + 64 + 64 * 64 + 64 + 64 + 1
_bound = False


def _L():
    global _bound
    L = lib()
    if not _bound:
        i32, i64, sz, vp, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_double
        L.rimp2_features_workspace_size.restype = sz
        L.rimp2_features_workspace_size.argtypes = [i32, i32]
        L.rimp2_pair_features.restype = ctypes.c_int
        L.rimp2_pair_features.argtypes = [i32, i32, i32] + [vp] * 6 + [vp, sz, vp]
        L.rimp2_mlp_forward.restype = ctypes.c_int
        L.rimp2_mlp_forward.argtypes = [i64, vp, vp, vp, vp]
        L.rimp2_mlp_workspace_size.restype = sz
        L.rimp2_mlp_workspace_size.argtypes = [i64]
        L.rimp2_mlp_loss_grad.restype = ctypes.c_int
        L.rimp2_mlp_loss_grad.argtypes = [i64, vp, vp, vp, vp, vp, vp, sz, vp]
        L.rimp2_mlp_adam.restype = ctypes.c_int
        L.rimp2_mlp_adam.argtypes = [vp, vp, vp, vp, i64, dbl, dbl, dbl, dbl, vp]
        L.rimp2_log_energy.restype = ctypes.c_int
        L.rimp2_log_energy.argtypes = [i64, vp, vp, vp]
        L.rimp2_screen_mask.restype = ctypes.c_int
        L.rimp2_screen_mask.argtypes = [i32, vp, dbl, vp, vp, vp]
        _bound = True
    return L


def pair_features(B, eps_occ, eps_vir, centroids, bound: bool = True, stream=None):
    """(features [nocc*nocc][4], bound [nocc][nocc] or None) on the GPU."""
    nocc, nvir, naux = B.shape
    L = _L()
    f64 = dict(dtype=torch.float64, device=B.device)
    feat = torch.empty((nocc * nocc, 4), **f64)
    bd = torch.empty((nocc, nocc), **f64) if bound else None
    ws = torch.empty(L.rimp2_features_workspace_size(nocc, naux), dtype=torch.uint8, device=B.device)
    _check(L.rimp2_pair_features(nocc, nvir, naux, _ptr(B), _ptr(eps_occ), _ptr(eps_vir), _ptr(centroids),
                                 _ptr(feat), _ptr(bd), _ptr(ws), ws.numel(), _stream_handle(stream)))
    return feat, bd


def mlp_forward(x, params, stream=None):
    y = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
    _check(_L().rimp2_mlp_forward(x.shape[0], _ptr(x), _ptr(params), _ptr(y), _stream_handle(stream)))
    return y


def mlp_loss_grad(x, t, params, workspace=None, stream=None):
    L = _L()
    n = x.shape[0]
    if workspace is None:
        workspace = torch.empty(L.rimp2_mlp_workspace_size(n), dtype=torch.uint8, device=x.device)
    loss = torch.empty(1, dtype=torch.float64, device=x.device)
    grad = torch.empty(N_PARAMS, dtype=torch.float64, device=x.device)
    _check(L.rimp2_mlp_loss_grad(n, _ptr(x), _ptr(t), _ptr(params), _ptr(loss), _ptr(grad), _ptr(workspace),
                                 workspace.numel(), _stream_handle(stream)))
    return loss, grad


def adam(grad, params, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_L().rimp2_mlp_adam(_ptr(grad), _ptr(params), _ptr(m), _ptr(v), step, lr, beta1, beta2, eps,
                               _stream_handle(stream)))


def log_energy(e, stream=None):
    out = torch.empty_like(e)
    _check(_L().rimp2_log_energy(e.numel(), _ptr(e), _ptr(out), _stream_handle(stream)))
    return out


def screen_mask(pred, nocc, threshold_log10, stream=None):
    """(skip mask uint8 [nocc][nocc], predicted skipped energy [1])."""
    skip = torch.empty((nocc, nocc), dtype=torch.uint8, device=pred.device)
    se = torch.empty(1, dtype=torch.float64, device=pred.device)
    _check(_L().rimp2_screen_mask(nocc, _ptr(pred), threshold_log10, _ptr(skip), _ptr(se), _stream_handle(stream)))
    return skip, se


def init_params(seed: int, device) -> torch.Tensor:
    """Glorot-uniform weights, zero biases (host RNG, seeded)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((4, 64), (64, 64), (64, 1)):
        a = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-a, a, fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return torch.from_numpy(np.concatenate(parts)).to(device)


def save_params(path: str, params: torch.Tensor, **meta) -> None:
    """Checkpoint of a trained network: the parameter vector (layout of
    include/rimp2_screen.h) and JSON-serialisable metadata (training seeds,
    feature scaling, loss), in an .npz file that loads without pickle."""
    import json
    np.savez(path, params=params.detach().cpu().numpy().astype(np.float64),
             meta=np.frombuffer(json.dumps(meta, sort_keys=True).encode(), dtype=np.uint8))


def load_params(path: str, device) -> tuple[torch.Tensor, dict]:
    """(params on ``device``, metadata) from save_params' file."""
    import json
    with np.load(path, allow_pickle=False) as z:
        p = z["params"]
        meta = json.loads(bytes(z["meta"]).decode()) if "meta" in z else {}
    if p.shape != (N_PARAMS,) or p.dtype != np.float64:
        raise ValueError("%s: expected %d float64 parameters, got %s %s" % (path, N_PARAMS, p.shape, p.dtype))
    return torch.from_numpy(p.copy()).to(device), meta


def budget_threshold(pred: torch.Tensor, nocc: int, budget_Eh: float, iters: int = 60) -> float:
    """The largest log10 threshold whose predicted skipped energy (sum of
    10^pred over the pairs it skips, rimp2_screen_mask) is at most budget_Eh,
    by bisection over [-30, 0]."""
    lo, hi = -30.0, 0.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        _, se = screen_mask(pred, nocc, mid)
        if float(se) <= budget_Eh:
            lo = mid
        else:
            hi = mid
    return lo


def bound_mask(bound: torch.Tensor, budget_Eh: float) -> torch.Tensor:
    """The rigorous-bound screen (the method without the network): skip the
    pairs i < j with the smallest bounds while twice their summed bound (both
    orders) stays within budget_Eh, so the exact skipped energy is within it
    too.  Host-side selection over the bound matrix; returns a symmetric uint8
    mask on the bound's device."""
    bd = bound.detach().cpu().numpy()
    n = bd.shape[0]
    iu = np.triu_indices(n, 1)
    order = np.argsort(bd[iu], kind="stable")
    csum = np.cumsum(2.0 * bd[iu][order])
    nb = int(np.searchsorted(csum, budget_Eh, side="right"))
    m = np.zeros((n, n), dtype=np.uint8)
    m[iu[0][order[:nb]], iu[1][order[:nb]]] = 1
    m |= m.T
    return torch.from_numpy(m).to(bound.device)


class Trainer:
    """Adam on the mean squared error, minibatches drawn by a seeded host RNG."""

    def __init__(self, params: torch.Tensor, lr: float = 1e-3):
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step = 0
        self.lr = lr
        self._ws = {}

    def fit(self, x: torch.Tensor, t: torch.Tensor, steps: int, batch: int, seed: int = 0) -> float:
        rng = np.random.default_rng(seed)
        n = x.shape[0]
        b = min(batch, n)
        if b not in self._ws:
            self._ws[b] = torch.empty(_L().rimp2_mlp_workspace_size(b), dtype=torch.uint8, device=x.device)
        loss = None
        for _ in range(steps):
            idx = torch.from_numpy(rng.choice(n, size=b, replace=False)).to(x.device)
            xb = x.index_select(0, idx).contiguous()
            tb = t.index_select(0, idx).contiguous()
            loss, grad = mlp_loss_grad(xb, tb, self.params, workspace=self._ws[b])
            self.step += 1
            adam(grad, self.params, self.m, self.v, self.step, self.lr)
        return float(loss) if loss is not None else float("nan")
