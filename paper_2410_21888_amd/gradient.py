"""ctypes binding of include/rimp2_gradient.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from .rimp2 import _check, _ptr, _stream_handle, lib

_bound = False


def _L():
    global _bound
    L = lib()
    if not _bound:
        i32, vp = ctypes.c_int32, ctypes.c_void_p
        L.rimp2_gamma_metric.restype = ctypes.c_int
        L.rimp2_gamma_metric.argtypes = [i32, i32, i32, vp, vp, vp, vp]
        _bound = True
    return L


def gamma_metric(Gamma: torch.Tensor, Jm: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
    """out[i, a, P] = sum_Q Gamma[i, a, Q] Jm[P, Q] on the GPU (rimp2_gamma_metric)."""
    nocc, nvir, naux = Gamma.shape
    if Jm.shape != (naux, naux) or Gamma.dtype != torch.float64 or Jm.dtype != torch.float64:
        raise ValueError("Gamma [nocc][nvir][naux] and Jm [naux][naux], float64")
    if not (Gamma.is_contiguous() and Jm.is_contiguous()):
        raise ValueError("Gamma and Jm must be contiguous")
    if out is None:
        out = torch.empty_like(Gamma)
    _check(_L().rimp2_gamma_metric(nocc, nvir, naux, _ptr(Gamma), _ptr(Jm), _ptr(out), _stream_handle(stream)))
    return out
