"""Seeded synthetic inputs for the closed-shell RI-MP2 fragment kernel.

This package holds the input generators and the workload registry, and nothing
of the MP2 arithmetic.  Both the CPU oracle (through the tests) and the HIP path
(through the tests and the benchmark) take their inputs from here.

Workloads (all energies in hartree, distances in angstrom):

* ``small``   nocc=20,  nvir=100,  naux=400,  B = 0.3 N(0,1) exp(-P/80)
* ``large``   nocc=200, nvir=1800, naux=6000, B = 0.3 N(0,1) exp(-P/1200)
* ``split``   the ``large`` shapes and seed, for the split-precision products
* ``mbe3``    4096 fragments: 30% monomers, 40% dimers, 30% trimers with
              nocc ~ U{5..60} per monomer (summed), nvir = 5 nocc,
              naux = 3 (nocc + nvir)
* ``screen``  nocc=400, nvir=2400, naux=7200 with occupied and auxiliary
              centroids uniform in a 40 A cube and
              B = 0.3 N(0,1) exp(-|r_i - r_P| / 3 A)

Orbital energies: eps_occ ~ U[-20, -0.3], eps_vir ~ U[0.1, 5], each sorted
ascending, so every MP2 denominator is at most -0.4 Eh.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csynth.c")
_LIB = os.path.join(_HERE, "_csynth.so")
_DSRC = os.path.join(_HERE, "dsynth.hip")
_DLIB = os.path.join(_HERE, "_dsynth.so")

# tensor ids inside one fragment's key space
T_B, T_EOCC, T_EVIR, T_ROCC, T_RAUX, T_SIZES = 0, 1, 2, 3, 4, 5
GOLDEN = 0x9E3779B97F4A7C15


def build(force: bool = False) -> str:
    """Compile the C generator in place (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def build_device(force: bool = False) -> str:
    """Compile the device twin of the generator (hipcc, gfx950) in place."""
    if force or not os.path.exists(_DLIB) or os.path.getmtime(_DLIB) < os.path.getmtime(_DSRC):
        tmp = _DLIB + ".tmp%d" % os.getpid()
        hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-Xclang", "-target-feature",
                               "-Xclang", "-packed-fp32-ops", "-o", tmp, _DSRC],
                              stderr=subprocess.DEVNULL)
        os.replace(tmp, _DLIB)
    return _DLIB


_dlib = None


def three_index_device(k: int, nocc: int, nvir: int, naux: int, scale, out, i0: int = 0, i1: int | None = None,
                       stream=None):
    """Rows [i0, i1) of the three-index tensor generated on the GPU into the
    torch tensor ``out`` (float64, [i1-i0][nvir][naux]); ``scale`` as in
    three_index (numpy)."""
    global _dlib
    import torch
    if _dlib is None:
        if not os.path.exists(_DLIB):
            raise RuntimeError("synth/_dsynth.so is not built (run __graft_entry__.build())")
        lib = ctypes.CDLL(_DLIB)
        lib.dsynth_three_index.restype = ctypes.c_int
        lib.dsynth_three_index.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_void_p]
        _dlib = lib
    i1 = nocc if i1 is None else i1
    sc = torch.as_tensor(np.ascontiguousarray(scale, dtype=np.float64)).to(out.device)
    per_i = 1 if sc.dim() == 2 else 0
    assert out.dtype == torch.float64 and out.is_contiguous() and tuple(out.shape) == (i1 - i0, nvir, naux)
    st = (stream or torch.cuda.current_stream()).cuda_stream
    rc = _dlib.dsynth_three_index(k, i0, i1, nvir, naux, sc.data_ptr(), per_i, out.data_ptr(), st)
    if rc != 0:
        raise RuntimeError("device generator launch failed")
    torch.cuda.current_stream().synchronize()
    return out


_lib = None


def _clib():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        u64, i64, pd = ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        lib.synth_key.restype = u64
        lib.synth_key.argtypes = [u64, u64, u64]
        lib.synth_draw.restype = u64
        lib.synth_draw.argtypes = [u64, u64]
        lib.synth_uniform.argtypes = [u64, u64, i64, pd]
        lib.synth_normal.argtypes = [u64, u64, i64, pd]
        lib.synth_three_index.argtypes = [u64, i64, i64, i64, i64, pd, ctypes.c_int, pd]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def key(seed: int, frag: int, tensor: int) -> int:
    return int(_clib().synth_key(seed, frag, tensor))


def uniform(k: int, first: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _clib().synth_uniform(k, first, count, _ptr(out))
    return out


def normal(k: int, first: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _clib().synth_normal(k, first, count, _ptr(out))
    return out


def decay_scale(naux: int, decay: float, amp: float = 0.3) -> np.ndarray:
    """amp * exp(-P / decay) for P = 0 .. naux-1 (P is 0-based)."""
    return amp * np.exp(-np.arange(naux, dtype=np.float64) / decay)


def three_index(k: int, nocc: int, nvir: int, naux: int, scale: np.ndarray,
                i0: int = 0, i1: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Rows [i0, i1) of B[i][a][P] = normal(k, (i*nvir+a)*naux+P) * scale.

    ``scale`` is either one row of ``naux`` values or an ``[nocc][naux]`` array
    (per occupied orbital)."""
    i1 = nocc if i1 is None else i1
    scale = np.ascontiguousarray(scale, dtype=np.float64)
    per_i = 1 if scale.ndim == 2 else 0
    if per_i:
        assert scale.shape == (nocc, naux)
    else:
        assert scale.shape == (naux,)
    if out is None:
        out = np.empty((i1 - i0, nvir, naux), dtype=np.float64)
    assert out.flags.c_contiguous and out.dtype == np.float64 and out.shape == (i1 - i0, nvir, naux)
    _clib().synth_three_index(k, i0, i1, nvir, naux, _ptr(scale), per_i, _ptr(out))
    return out


def orbital_energies(seed: int, frag: int, nocc: int, nvir: int):
    eo = np.sort(-20.0 + (-0.3 + 20.0) * uniform(key(seed, frag, T_EOCC), 0, nocc))
    ev = np.sort(0.1 + (5.0 - 0.1) * uniform(key(seed, frag, T_EVIR), 0, nvir))
    return eo, ev


@dataclass(frozen=True)
class Fragment:
    nocc: int
    nvir: int
    naux: int
    seed: int
    frag: int = 0
    decay: float = 80.0        # exp(-P/decay) aux decay (used when ``centroids`` is False)
    centroids: bool = False    # spatial decay exp(-|r_i - r_P| / length)
    box: float = 40.0          # cube edge (angstrom) for centroids
    length: float = 3.0        # spatial decay length (angstrom)

    @property
    def key_B(self) -> int:
        return key(self.seed, self.frag, T_B)

    def scale(self) -> np.ndarray:
        if not self.centroids:
            return decay_scale(self.naux, self.decay)
        r_i, r_P = self.positions()
        d = np.sqrt(((r_i[:, None, :] - r_P[None, :, :]) ** 2).sum(-1))
        return 0.3 * np.exp(-d / self.length)

    def positions(self):
        """Occupied and auxiliary centroids, uniform in the cube (angstrom)."""
        r_i = self.box * uniform(key(self.seed, self.frag, T_ROCC), 0, 3 * self.nocc).reshape(self.nocc, 3)
        r_P = self.box * uniform(key(self.seed, self.frag, T_RAUX), 0, 3 * self.naux).reshape(self.naux, 3)
        return r_i, r_P

    def B(self, i0: int = 0, i1: int | None = None, out=None) -> np.ndarray:
        return three_index(self.key_B, self.nocc, self.nvir, self.naux, self.scale(), i0, i1, out)

    def B_device(self, out):
        """The whole B generated on the GPU into a torch tensor."""
        return three_index_device(self.key_B, self.nocc, self.nvir, self.naux, self.scale(), out)

    def eps(self):
        return orbital_energies(self.seed, self.frag, self.nocc, self.nvir)

    def arrays(self):
        eo, ev = self.eps()
        return self.B(), eo, ev

    def bytes_B(self) -> int:
        return 8 * self.nocc * self.nvir * self.naux


SMALL = Fragment(20, 100, 400, seed=1000, decay=80.0)
LARGE = Fragment(200, 1800, 6000, seed=1001, decay=1200.0)
SPLIT = LARGE
SCREEN = Fragment(400, 2400, 7200, seed=4200, centroids=True)


def screen_system(seed: int, nocc: int = 400, nvir: int = 2400, naux: int = 7200) -> Fragment:
    """One spatially decaying system of the screening workload (training seeds
    4000..4199, held-out evaluation seed 4200)."""
    return Fragment(nocc, nvir, naux, seed=seed, centroids=True)


def mbe3_sizes(nfrag: int = 4096, seed: int = 1003):
    """(kind, nocc) per fragment: ids [0, 0.3n) monomers, [0.3n, 0.7n) dimers,
    the rest trimers; nocc is the sum of 1/2/3 draws from U{5..60}."""
    n_mono = int(round(0.3 * nfrag))
    n_di = int(round(0.4 * nfrag))
    out = []
    for f in range(nfrag):
        kind = 1 if f < n_mono else (2 if f < n_mono + n_di else 3)
        u = uniform(key(seed, f, T_SIZES), 0, kind)
        nocc = int(sum(5 + min(55, int(x * 56)) for x in u))
        out.append((kind, nocc))
    return out


def mbe3_fragment(f: int, nocc: int, seed: int = 1003) -> Fragment:
    nvir = 5 * nocc
    return Fragment(nocc, nvir, 3 * (nocc + nvir), seed=seed, frag=f, decay=80.0)


def random_fragment(nocc: int, nvir: int, naux: int, seed: int, decay: float = 80.0) -> Fragment:
    return Fragment(nocc, nvir, naux, seed=seed, decay=decay)
