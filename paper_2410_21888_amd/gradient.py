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
        i32, vp, sz = ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
        L.rimp2_gamma_metric.restype = ctypes.c_int
        L.rimp2_gamma_metric.argtypes = [i32, i32, i32, vp, vp, vp, vp]
        L.rimp2_gamma_ao_workspace_size.restype = ctypes.c_int
        L.rimp2_gamma_ao_workspace_size.argtypes = [i32, i32, i32, ctypes.POINTER(sz)]
        L.rimp2_gamma_ao.restype = ctypes.c_int
        L.rimp2_gamma_ao.argtypes = [i32] * 6 + [vp] * 5 + [sz, vp]
        L.rimp2_l_terms_workspace_size.restype = ctypes.c_int
        L.rimp2_l_terms_workspace_size.argtypes = [i32, i32, i32, i32, ctypes.POINTER(sz)]
        L.rimp2_l_terms.restype = ctypes.c_int
        L.rimp2_l_terms.argtypes = [i32] * 4 + [vp] * 6 + [sz, vp]
        i64, dbl = ctypes.c_int64, ctypes.c_double
        L.rimp2_antisym_workspace_size.restype = ctypes.c_int
        L.rimp2_antisym_workspace_size.argtypes = [i32] * 4 + [ctypes.POINTER(sz)]
        L.rimp2_antisym_term.restype = ctypes.c_int
        L.rimp2_antisym_term.argtypes = [i32] * 6 + [vp, vp, vp, i64, vp, sz, vp]
        L.rimp2_zvector_workspace_size.restype = ctypes.c_int
        L.rimp2_zvector_workspace_size.argtypes = [i32] * 3 + [ctypes.POINTER(sz)]
        L.rimp2_zvector.restype = ctypes.c_int
        L.rimp2_zvector.argtypes = [i32] * 3 + [vp] * 8 + [dbl, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp, sz,
                                                           vp]
        L.rimp2_energy_weighted_density_workspace_size.restype = ctypes.c_int
        L.rimp2_energy_weighted_density_workspace_size.argtypes = [i32] * 3 + [ctypes.POINTER(sz)]
        L.rimp2_energy_weighted_density.restype = ctypes.c_int
        L.rimp2_energy_weighted_density.argtypes = [i32] * 3 + [vp] * 9 + [vp, sz, vp]
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


def _need(t: torch.Tensor, shape, name):
    if tuple(t.shape) != tuple(shape) or t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("%s must be a contiguous float64 GPU tensor of shape %s" % (name, tuple(shape)))


def gamma_ao(Gamma: torch.Tensor, C_occ: torch.Tensor, C_vir: torch.Tensor, p0: int = 0,
             pcount: Optional[int] = None, out: Optional[torch.Tensor] = None, workspace=None, stream=None):
    """out[m, n, P - p0] = sum_ia C_occ[i, m] Gamma[i, a, P] C_vir[a, n] for P in
    [p0, p0 + pcount) on the GPU (rimp2_gamma_ao)."""
    nocc, nvir, naux = Gamma.shape
    nao = C_occ.shape[1]
    pcount = naux - p0 if pcount is None else pcount
    _need(Gamma, (nocc, nvir, naux), "Gamma")
    _need(C_occ, (nocc, nao), "C_occ")
    _need(C_vir, (nvir, nao), "C_vir")
    if out is None:
        out = torch.empty((nao, nao, pcount), dtype=torch.float64, device=Gamma.device)
    _need(out, (nao, nao, pcount), "out")
    L = _L()
    if workspace is None:
        n = ctypes.c_size_t(0)
        _check(L.rimp2_gamma_ao_workspace_size(nocc, nao, pcount, ctypes.byref(n)))
        workspace = torch.empty(n.value, dtype=torch.uint8, device=Gamma.device)
    _check(L.rimp2_gamma_ao(nocc, nvir, nao, naux, p0, pcount, _ptr(Gamma), _ptr(C_occ), _ptr(C_vir), _ptr(out),
                            _ptr(workspace), workspace.numel(), _stream_handle(stream)))
    return out


def l_terms(Gamma: torch.Tensor, I_qa: Optional[torch.Tensor], I_iq: Optional[torch.Tensor], workspace=None,
            stream=None):
    """(L' [nocc][nmo], L'' [nvir][nmo]) on the GPU (rimp2_l_terms); either
    integral tensor may be None, and its term is then None."""
    nocc, nvir, naux = Gamma.shape
    nmo = (I_qa if I_qa is not None else I_iq).shape[0 if I_qa is not None else 1]
    _need(Gamma, (nocc, nvir, naux), "Gamma")
    f64 = dict(dtype=torch.float64, device=Gamma.device)
    L1 = L2 = None
    if I_qa is not None:
        _need(I_qa, (nmo, nvir, naux), "I_qa")
        L1 = torch.empty((nocc, nmo), **f64)
    if I_iq is not None:
        _need(I_iq, (nocc, nmo, naux), "I_iq")
        L2 = torch.empty((nvir, nmo), **f64)
    L = _L()
    if workspace is None:
        n = ctypes.c_size_t(0)
        _check(L.rimp2_l_terms_workspace_size(nocc, nvir, nmo, naux, ctypes.byref(n)))
        workspace = torch.empty(n.value, dtype=torch.uint8, device=Gamma.device)
    _check(L.rimp2_l_terms(nocc, nvir, nmo, naux, _ptr(Gamma), _ptr(I_qa), _ptr(I_iq), _ptr(L1), _ptr(L2),
                           _ptr(workspace), workspace.numel(), _stream_handle(stream)))
    return L1, L2


def _ws(size_fn, *args, device):
    n = ctypes.c_size_t(0)
    _check(size_fn(*args, ctypes.byref(n)))
    return torch.empty(n.value, dtype=torch.uint8, device=device)


def antisym_term(Bf: torch.Tensor, D: torch.Tensor, rows=None, cols=None, stream=None) -> torch.Tensor:
    """F[p, q] = sum_rs G_pq^rs D[r, s] for p in range(*rows), q in range(*cols)
    (default: every MO) on the GPU (rimp2_antisym_term)."""
    nmo, nmo2, naux = Bf.shape
    if nmo2 != nmo:
        raise ValueError("Bf must be [nmo][nmo][naux]")
    _need(Bf, (nmo, nmo, naux), "Bf")
    _need(D, (nmo, nmo), "D")
    r0, r1 = rows if rows is not None else (0, nmo)
    c0, c1 = cols if cols is not None else (0, nmo)
    F = torch.empty((r1 - r0, c1 - c0), dtype=torch.float64, device=Bf.device)
    L = _L()
    ws = _ws(L.rimp2_antisym_workspace_size, nmo, naux, r1 - r0, c1 - c0, device=Bf.device)
    _check(L.rimp2_antisym_term(nmo, naux, r0, r1 - r0, c0, c1 - c0, _ptr(Bf), _ptr(D), _ptr(F), c1 - c0, _ptr(ws),
                                ws.numel(), _stream_handle(stream)))
    return F


def zvector(Bf, eps_occ, eps_vir, P_ij, P_ab, L1, L2, tol: float = 1e-12, max_iter: int = 500, stream=None):
    """(D_ai [nvir][nocc], iterations, relative residual) from the Z-vector
    equation on the GPU (rimp2_zvector); raises Rimp2Error(RIMP2_ENOCONV)
    when CG does not reach tol."""
    nocc, nvir = eps_occ.shape[0], eps_vir.shape[0]
    nmo, naux = nocc + nvir, Bf.shape[2]
    _need(Bf, (nmo, nmo, naux), "Bf")
    for t, shp, name in ((P_ij, (nocc, nocc), "P_ij"), (P_ab, (nvir, nvir), "P_ab"), (L1, (nocc, nmo), "L1"),
                         (L2, (nvir, nmo), "L2"), (eps_occ, (nocc,), "eps_occ"), (eps_vir, (nvir,), "eps_vir")):
        _need(t, shp, name)
    D_ai = torch.empty((nvir, nocc), dtype=torch.float64, device=Bf.device)
    L = _L()
    ws = _ws(L.rimp2_zvector_workspace_size, nocc, nvir, naux, device=Bf.device)
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)
    _check(L.rimp2_zvector(nocc, nvir, naux, _ptr(Bf), _ptr(eps_occ), _ptr(eps_vir), _ptr(P_ij), _ptr(P_ab),
                           _ptr(L1), _ptr(L2), _ptr(D_ai), tol, max_iter, ctypes.byref(it), ctypes.byref(res),
                           _ptr(ws), ws.numel(), _stream_handle(stream)))
    return D_ai, it.value, res.value


def energy_weighted_density(Bf, eps_occ, eps_vir, P_ij, P_ab, D_ai, L1, L2, stream=None) -> torch.Tensor:
    """W [nmo][nmo] on the GPU (rimp2_energy_weighted_density)."""
    nocc, nvir = eps_occ.shape[0], eps_vir.shape[0]
    nmo, naux = nocc + nvir, Bf.shape[2]
    _need(Bf, (nmo, nmo, naux), "Bf")
    W = torch.empty((nmo, nmo), dtype=torch.float64, device=Bf.device)
    L = _L()
    ws = _ws(L.rimp2_energy_weighted_density_workspace_size, nocc, nvir, naux, device=Bf.device)
    _check(L.rimp2_energy_weighted_density(nocc, nvir, naux, _ptr(Bf), _ptr(eps_occ), _ptr(eps_vir), _ptr(P_ij),
                                           _ptr(P_ab), _ptr(D_ai), _ptr(L1), _ptr(L2), _ptr(W), _ptr(ws), ws.numel(),
                                           _stream_handle(stream)))
    return W
