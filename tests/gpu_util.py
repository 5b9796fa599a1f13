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
