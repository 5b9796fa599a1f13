"""Helpers shared by the GPU tests (device transfer and comparisons)."""
import math

import numpy as np
import torch


def dev():
    return torch.device("cuda:0")


def to_dev(*arrays):
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dev()) for a in arrays]


def rel_fro(got, ref):
    got = np.asarray(got)
    ref = np.asarray(ref)
    n = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / n) if n > 0 else float(np.linalg.norm(got))


def energy_error(E_dev, ref_hi, ref_lo):
    """|E_gpu - E_oracle| evaluated exactly from the two (hi, lo) pairs."""
    e = E_dev.cpu().numpy()
    return abs(math.fsum([float(e[0]), float(e[1]), -ref_hi, -ref_lo]))


def say(*args):
    print(*args, flush=True)


def assert_elementwise(got, ref, rtol, atol, name=""):
    """Every element within rtol |ref| + atol max|ref row|, where a row is the
    last index (a Gamma row over P, a row of P_ij or P_ab, a row of e_pair):
    the relative part bounds large elements, the row part bounds elements
    that cancel to near zero (their rounding error scales with the row's
    magnitude, not their own).  Raises with the worst element otherwise."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    rowmax = np.max(np.abs(ref), axis=-1, keepdims=True) if ref.ndim else np.abs(ref)
    bound = rtol * np.abs(ref) + atol * rowmax
    err = np.abs(got - ref)
    bad = ~(err <= bound)
    if bad.any():
        ratio = np.where(bound > 0, err / np.where(bound > 0, bound, 1.0), np.inf)
        w = np.unravel_index(np.argmax(np.where(bad, ratio, -1.0)), ref.shape)
        raise AssertionError("%s: %d of %d elements outside rtol=%g atol=%g (x row max); worst at %s: got %r ref %r"
                             % (name, int(bad.sum()), bad.size, rtol, atol, tuple(int(i) for i in w),
                                float(got[w]), float(ref[w])))
