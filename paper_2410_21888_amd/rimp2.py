"""ctypes binding of librimp2.so: the same entry points as include/rimp2.h,
taking torch tensors for device buffers and a torch stream.

Argument marshalling only: every step of the computation runs in the HIP
library, and loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import NamedTuple, Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librimp2.so")

RIMP2_OK, RIMP2_EINVAL, RIMP2_ENOMEM, RIMP2_EWORKSPACE = 0, -1, -2, -3
RIMP2_EDEVICE, RIMP2_EGAP, RIMP2_ENOTSUP, RIMP2_ENOCONV = -4, -5, -6, -7
FP64, SPLIT_INT8 = 0, 1
WANT_GAMMA, WANT_DENSITY = 1, 2


class Rimp2Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_status_name(code), code, msg))
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("split_slices", ctypes.c_int32),
        ("slab_group", ctypes.c_int32),
        ("split_slices_gamma", ctypes.c_int32),
        ("slab_budget_bytes", ctypes.c_size_t),
        ("pair_skip", ctypes.c_void_p),
        ("autotune", ctypes.c_int32),
        ("gemm_loader", ctypes.c_int32),
    ]


class FragDesc(ctypes.Structure):
    _fields_ = [
        ("nocc", ctypes.c_int32), ("nvir", ctypes.c_int32), ("naux", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("B", ctypes.c_void_p), ("eps_occ", ctypes.c_void_p), ("eps_vir", ctypes.c_void_p),
        ("E", ctypes.c_void_p), ("Gamma", ctypes.c_void_p), ("P_ij", ctypes.c_void_p),
        ("P_ab", ctypes.c_void_p), ("e_pair", ctypes.c_void_p),
    ]


class TuneStat(ctypes.Structure):
    _fields_ = [("role", ctypes.c_char * 32), ("device", ctypes.c_int32), ("nvar", ctypes.c_int32),
                ("best", ctypes.c_int32), ("vec", ctypes.c_int32), ("M", ctypes.c_int64), ("N", ctypes.c_int64),
                ("K", ctypes.c_int64), ("kchunk", ctypes.c_int64), ("tile_m", ctypes.c_int32 * 4),
                ("tile_n", ctypes.c_int32 * 4), ("timed", ctypes.c_int32 * 4), ("min_ms", ctypes.c_double * 4),
                ("uses", ctypes.c_int64)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("alg_flops", ctypes.c_double), ("exec_flops", ctypes.c_double), ("alg_bytes", ctypes.c_double)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("librimp2.so is not built (run __graft_entry__.build()); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        i32, sz, vp = ctypes.c_int32, ctypes.c_size_t, ctypes.c_void_p
        L.rimp2_version.restype = ctypes.c_int
        L.rimp2_last_error.restype = ctypes.c_char_p
        L.rimp2_status_string.restype = ctypes.c_char_p
        L.rimp2_status_string.argtypes = [ctypes.c_int]
        L.rimp2_workspace_size.restype = ctypes.c_int
        L.rimp2_workspace_size.argtypes = [i32, i32, i32, i32, ctypes.POINTER(Opts), ctypes.POINTER(sz)]
        L.rimp2_fragment.restype = ctypes.c_int
        L.rimp2_fragment.argtypes = [i32, i32, i32] + [vp] * 8 + [vp, sz, ctypes.POINTER(Opts), vp]
        L.rimp2_read_status.restype = ctypes.c_int
        L.rimp2_read_status.argtypes = [vp, vp, ctypes.POINTER(i32)]
        L.rimp2_batch_workspace_size.restype = ctypes.c_int
        L.rimp2_batch_workspace_size.argtypes = [i32, ctypes.POINTER(FragDesc), ctypes.POINTER(Opts),
                                                 ctypes.POINTER(sz)]
        L.rimp2_fragment_batch.restype = ctypes.c_int
        L.rimp2_fragment_batch.argtypes = [i32, ctypes.POINTER(FragDesc), vp, vp, sz, ctypes.POINTER(Opts), vp]
        L.rimp2_batch_create.restype = ctypes.c_int
        L.rimp2_batch_create.argtypes = [i32, ctypes.POINTER(FragDesc), ctypes.POINTER(Opts), ctypes.POINTER(vp),
                                         ctypes.POINTER(sz)]
        L.rimp2_batch_run.restype = ctypes.c_int
        L.rimp2_batch_run.argtypes = [vp, vp, vp, sz, vp]
        L.rimp2_batch_destroy.restype = ctypes.c_int
        L.rimp2_batch_destroy.argtypes = [vp]
        L.rimp2_timing_enable.restype = ctypes.c_int
        L.rimp2_timing_enable.argtypes = [ctypes.c_int]
        L.rimp2_timing_collect.restype = ctypes.c_int
        L.rimp2_timing_collect.argtypes = [ctypes.POINTER(KernelStat), i32, ctypes.POINTER(i32)]
        L.rimp2_autotune_report.restype = ctypes.c_int
        L.rimp2_autotune_report.argtypes = [ctypes.POINTER(TuneStat), i32, ctypes.POINTER(i32)]
        L.rimp2_autotune_reset.restype = ctypes.c_int
        L.rimp2_autotune_reset.argtypes = []
        _lib = L
    return _lib


def _status_name(code: int) -> str:
    names = {0: "RIMP2_OK", -1: "RIMP2_EINVAL", -2: "RIMP2_ENOMEM", -3: "RIMP2_EWORKSPACE", -4: "RIMP2_EDEVICE",
             -5: "RIMP2_EGAP", -6: "RIMP2_ENOTSUP", -7: "RIMP2_ENOCONV"}
    return names.get(code, "unknown")


def _check(rc: int):
    if rc != RIMP2_OK:
        raise Rimp2Error(rc, lib().rimp2_last_error().decode())


def version() -> int:
    return lib().rimp2_version()


def make_opts(precision: int = FP64, split_slices: int = 0, slab_group: int = 0, slab_budget_bytes: int = 0,
              pair_skip: Optional[torch.Tensor] = None, split_slices_gamma: int = 0, autotune: bool = False,
              gemm_loader: int = 0) -> Opts:
    o = Opts()
    o.autotune = 1 if autotune else 0
    o.gemm_loader = gemm_loader
    o.precision, o.split_slices, o.slab_group = precision, split_slices, slab_group
    o.split_slices_gamma = split_slices_gamma
    o.slab_budget_bytes = slab_budget_bytes
    o.pair_skip = pair_skip.data_ptr() if pair_skip is not None else None
    # the struct holds a raw device address: keep the mask tensor alive with it
    o._pair_skip_ref = pair_skip
    return o


def workspace_size(nocc: int, nvir: int, naux: int, gamma: bool = True, density: bool = True,
                   opts: Optional[Opts] = None) -> int:
    n = ctypes.c_size_t(0)
    want = (WANT_GAMMA if gamma else 0) | (WANT_DENSITY if density else 0)
    _check(lib().rimp2_workspace_size(nocc, nvir, naux, want, ctypes.byref(opts) if opts else None, ctypes.byref(n)))
    return n.value


class Result(NamedTuple):
    E: torch.Tensor                  # device [2]: (hi, lo)
    Gamma: Optional[torch.Tensor]
    P_ij: Optional[torch.Tensor]
    P_ab: Optional[torch.Tensor]
    e_pair: Optional[torch.Tensor]

    @property
    def E_hi(self) -> float:
        return float(self.E[0])

    @property
    def E_lo(self) -> float:
        return float(self.E[1])


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _validate(B, eps_occ, eps_vir):
    for name, t in (("B", B), ("eps_occ", eps_occ), ("eps_vir", eps_vir)):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("%s must be a contiguous float64 tensor on the GPU" % name)
    if B.dim() != 3 or eps_occ.shape != (B.shape[0],) or eps_vir.shape != (B.shape[1],):
        raise ValueError("shapes: B [nocc][nvir][naux], eps_occ [nocc], eps_vir [nvir]")


def fragment_into(B, eps_occ, eps_vir, E, Gamma=None, P_ij=None, P_ab=None, e_pair=None, *, workspace,
                  opts: Optional[Opts] = None, stream=None) -> None:
    """Enqueue the kernel writing into caller-owned outputs (no allocation,
    no synchronisation)."""
    nocc, nvir, naux = B.shape
    rc = lib().rimp2_fragment(nocc, nvir, naux, _ptr(B), _ptr(eps_occ), _ptr(eps_vir), _ptr(E), _ptr(Gamma),
                              _ptr(P_ij), _ptr(P_ab), _ptr(e_pair), _ptr(workspace), workspace.numel(),
                              ctypes.byref(opts) if opts else None, _stream_handle(stream))
    _check(rc)


def read_status(workspace: torch.Tensor, stream=None) -> int:
    s = ctypes.c_int32(0)
    _check(lib().rimp2_read_status(_ptr(workspace), _stream_handle(stream), ctypes.byref(s)))
    return s.value


def fragment(B: torch.Tensor, eps_occ: torch.Tensor, eps_vir: torch.Tensor, *, gamma: bool = True,
             density: bool = True, pairs: bool = True, opts: Optional[Opts] = None, workspace=None, stream=None,
             check: bool = True) -> Result:
    """Run the fragment kernel, allocating outputs (and the workspace unless
    given).  With ``check`` the device status is read back (synchronising) and
    a gap violation raises Rimp2Error(RIMP2_EGAP)."""
    _validate(B, eps_occ, eps_vir)
    nocc, nvir, naux = B.shape
    dev = B.device
    f64 = dict(dtype=torch.float64, device=dev)
    E = torch.zeros(2, **f64)
    G = torch.empty((nocc, nvir, naux), **f64) if gamma else None
    Pij = torch.empty((nocc, nocc), **f64) if density else None
    Pab = torch.empty((nvir, nvir), **f64) if density else None
    ep = torch.empty((nocc, nocc), **f64) if pairs else None
    if workspace is None:
        workspace = torch.empty(workspace_size(nocc, nvir, naux, gamma, density, opts), dtype=torch.uint8,
                                device=dev)
    fragment_into(B, eps_occ, eps_vir, E, G, Pij, Pab, ep, workspace=workspace, opts=opts, stream=stream)
    if check:
        st = read_status(workspace, stream)
        if st != RIMP2_OK:
            raise Rimp2Error(st, "device status")
    return Result(E, G, Pij, Pab, ep)


def _descs(frags: Sequence[dict]):
    arr = (FragDesc * len(frags))()
    for d, f in zip(arr, frags):
        B = f["B"]
        d.nocc, d.nvir, d.naux = B.shape
        d.B, d.eps_occ, d.eps_vir, d.E = _ptr(B), _ptr(f["eps_occ"]), _ptr(f["eps_vir"]), _ptr(f["E"])
        d.Gamma, d.P_ij, d.P_ab, d.e_pair = (_ptr(f.get("Gamma")), _ptr(f.get("P_ij")), _ptr(f.get("P_ab")),
                                             _ptr(f.get("e_pair")))
    return arr


def batch_workspace_size(frags: Sequence[dict], opts: Optional[Opts] = None) -> int:
    n = ctypes.c_size_t(0)
    arr = _descs(frags)
    _check(lib().rimp2_batch_workspace_size(len(frags), arr, ctypes.byref(opts) if opts else None, ctypes.byref(n)))
    return n.value


def fragment_batch(frags: Sequence[dict], *, status: Optional[torch.Tensor] = None, workspace=None,
                   opts: Optional[Opts] = None, stream=None) -> None:
    """Enqueue many fragments.  Each dict holds device tensors B, eps_occ,
    eps_vir, E and optionally Gamma, P_ij, P_ab, e_pair."""
    arr = _descs(frags)
    if workspace is None:
        workspace = torch.empty(batch_workspace_size(frags, opts), dtype=torch.uint8, device=frags[0]["B"].device)
    _check(lib().rimp2_fragment_batch(len(frags), arr, _ptr(status), _ptr(workspace), workspace.numel(),
                                      ctypes.byref(opts) if opts else None, _stream_handle(stream)))


def flops(nocc: int, nvir: int, naux: int, gamma: bool = True, density: bool = True) -> dict:
    """Algorithmic FLOP counts of the path (2 per multiply-add): (ia|jb) over
    unordered pairs, Gamma, P_ab and P_ij; and the plain GEMM FLOPs with the
    (ia|jb) slabs over ordered pairs (the kernels run less where tiles are
    triangular or mirrored; rimp2_timing_collect reports what they execute)."""
    o, v, x = float(nocc), float(nvir), float(naux)
    alg = {"ints": o * (o + 1) * v * v * x}
    exe = {"ints": 2 * o * o * v * v * x}
    if gamma:
        alg["gamma"] = exe["gamma"] = 2 * o * o * v * v * x
    if density:
        alg["p_ab"] = exe["p_ab"] = 2 * o * o * v ** 3
        alg["p_ij"] = exe["p_ij"] = 2 * o ** 3 * v * v
    return {"algorithmic": sum(alg.values()), "executed": sum(exe.values()), "parts": alg}


def timing_enable(on: bool = True) -> None:
    """Start (discarding earlier records) or stop per-launch event timing."""
    _check(lib().rimp2_timing_enable(1 if on else 0))


def timing_collect() -> list:
    """Per-role kernel statistics recorded since timing was enabled."""
    arr = (KernelStat * 32)()
    n = ctypes.c_int32(0)
    _check(lib().rimp2_timing_collect(arr, 32, ctypes.byref(n)))
    return [dict(name=a.name.decode(), launches=a.launches, total_ms=a.total_ms, alg_flops=a.alg_flops,
                 exec_flops=a.exec_flops, alg_bytes=a.alg_bytes) for a in arr[:n.value]]


def autotune_report() -> list:
    """Shapes seen by the in-situ tile autotuner, with candidates, trial
    timings and the decision (best = -1 while trials are pending)."""
    arr = (TuneStat * 512)()
    n = ctypes.c_int32(0)
    _check(lib().rimp2_autotune_report(arr, 512, ctypes.byref(n)))
    out = []
    for a in arr[:n.value]:
        nv = a.nvar
        out.append(dict(role=a.role.decode(), device=a.device, best=a.best, vec=a.vec, M=a.M, N=a.N, K=a.K,
                        kchunk=a.kchunk, tiles=[(a.tile_m[v], a.tile_n[v]) for v in range(nv)],
                        timed=list(a.timed[:nv]), min_ms=list(a.min_ms[:nv]), uses=a.uses))
    return out


def autotune_reset() -> None:
    _check(lib().rimp2_autotune_reset())


class Batch:
    """A planned batch (rimp2_batch_create): run() enqueues it without host
    synchronisation, so it can be captured into a graph and replayed while the
    handle lives.  The tensors named in ``frags`` must stay alive."""

    def __init__(self, frags: Sequence[dict], opts: Optional[Opts] = None):
        self._frags = list(frags)
        self._arr = _descs(self._frags)
        h = ctypes.c_void_p(None)
        n = ctypes.c_size_t(0)
        _check(lib().rimp2_batch_create(len(self._frags), self._arr, ctypes.byref(opts) if opts else None,
                                        ctypes.byref(h), ctypes.byref(n)))
        self._h = h
        self.workspace_bytes = n.value

    def run(self, workspace: torch.Tensor, status: Optional[torch.Tensor] = None, stream=None) -> None:
        _check(lib().rimp2_batch_run(self._h, _ptr(status), _ptr(workspace), workspace.numel(),
                                     _stream_handle(stream)))

    def close(self) -> None:
        if self._h:
            lib().rimp2_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
