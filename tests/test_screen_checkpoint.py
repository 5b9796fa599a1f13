"""The committed screening checkpoint (paper_2410_21888_amd/screen_model.npz,
written by `bench.py --workload screen --screen-save ...` on the GPU): it
loads without pickle, holds the network's parameter vector with its
metadata, and the CPU oracle's forward pass on it predicts pair energies
that fall with distance, as the training data do."""
import os

import numpy as np
import pytest
import torch

from oracle import screen_oracle as S
from paper_2410_21888_amd import screen as SC

PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2410_21888_amd",
                    "screen_model.npz")


@pytest.mark.skipif(not os.path.exists(PATH), reason="no trained checkpoint committed")
def test_checkpoint_loads_and_predicts():
    p, meta = SC.load_params(PATH, "cpu")
    assert p.dtype == torch.float64 and p.numel() == S.NP == SC.N_PARAMS
    assert meta["target"] == "log10|e_ij|" and len(meta["size"]) == 3
    assert meta["rmse_log10_eval"] < 0.5
    x = np.zeros((5, 4))
    x[:, 0] = np.linspace(0.2, 4.0, 5)          # |r_i - r_j| / 10 from 2 to 40 A
    x[:, 1] = x[:, 2] = -1.0                    # log ||B_i||
    x[:, 3] = -1.0                              # (eps_i + eps_j) / 10
    y = S.forward(x, p.numpy())
    assert np.all(np.isfinite(y)) and np.all(np.diff(y) < 0)


def test_save_load_roundtrip(tmp_path):
    p = SC.init_params(3, "cpu")
    path = os.path.join(str(tmp_path), "m.npz")
    SC.save_params(path, p, size=[4, 5, 6], note="roundtrip")
    q, meta = SC.load_params(path, "cpu")
    assert torch.equal(p, q) and meta == {"note": "roundtrip", "size": [4, 5, 6]}
