"""Screening kernels and the energy-only symmetric path against the CPU oracles."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import rimp2_oracle as O
from oracle import screen_oracle as S
import paper_2410_21888_amd as rm
from paper_2410_21888_amd import screen as SC
from gpu_util import to_dev, rel_fro, say
import pins

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_features_and_bound_match_oracle():
    f = synth.screen_system(4000, nocc=9, nvir=20, naux=40)
    B, eo, ev = f.arrays()
    r, _ = f.positions()
    feat, bd = SC.pair_features(*to_dev(B, eo, ev, r))
    assert rel_fro(feat.cpu().numpy(), S.pair_features(B, eo, r)) <= 1e-14
    assert rel_fro(bd.cpu().numpy(), S.pair_bound(B, eo, ev)) <= 1e-13


def test_mlp_forward_and_gradient_match_oracle():
    rng = np.random.default_rng(5)
    for n in (1, 31, 100):
        x = rng.standard_normal((n, 4))
        t = rng.standard_normal(n)
        p = rng.standard_normal(S.NP) * 0.3
        dx, dt, dp = to_dev(x, t, p)
        y = SC.mlp_forward(dx, dp).cpu().numpy()
        assert rel_fro(y, S.forward(x, p)) <= 1e-13
        loss, grad = SC.mlp_loss_grad(dx, dt, dp)
        L, g = S.loss_grad(x, t, p)
        assert abs(float(loss) - L) <= 1e-13 * L
        assert rel_fro(grad.cpu().numpy(), g) <= 1e-12, n


def test_adam_matches_oracle():
    rng = np.random.default_rng(6)
    p, g = rng.standard_normal(S.NP), rng.standard_normal(S.NP)
    dp, dg = to_dev(p, g)
    m = torch.zeros_like(dp)
    v = torch.zeros_like(dp)
    pr, mr, vr = p, np.zeros(S.NP), np.zeros(S.NP)
    for step in (1, 2, 3):
        SC.adam(dg, dp, m, v, step, 1e-2)
        pr, mr, vr = S.adam(pr, g, mr, vr, step, 1e-2)
    assert rel_fro(dp.cpu().numpy(), pr) <= 1e-14


def test_screen_mask_and_log_energy():
    rng = np.random.default_rng(7)
    n = 11
    pred = rng.uniform(-12, -4, (n, n))
    skip, se = SC.screen_mask(torch.from_numpy(pred.ravel()).to(DEV), n, -8.0)
    s = skip.cpu().numpy()
    up = np.triu(pred, 1)
    ref = np.zeros((n, n), dtype=np.uint8)
    iu = np.triu_indices(n, 1)
    ref[iu] = pred[iu] < -8.0
    ref = ref | ref.T
    assert np.array_equal(s, ref)
    full = np.where(np.triu(np.ones((n, n)), 1) > 0, pred, 0) + np.where(np.triu(np.ones((n, n)), 1) > 0, pred, 0).T
    ref_e = sum(10 ** full[i, j] for i in range(n) for j in range(n) if ref[i, j])
    assert abs(float(se) - ref_e) <= 1e-13 * ref_e
    e = -np.abs(rng.standard_normal(20)) * 1e-3
    out = SC.log_energy(torch.from_numpy(e).to(DEV)).cpu().numpy()
    assert np.allclose(out, np.log10(-e), rtol=0, atol=1e-14)


@pytest.mark.parametrize("shape,g", [((7, 30, 50), 0), ((9, 33, 64), 2), ((5, 64, 128), 1)])
def test_energy_only_symmetric_path(shape, g):
    f = synth.random_fragment(*shape, seed=sum(shape))
    B, eo, ev = f.arrays()
    ref = O.fragment(B, eo, ev, gamma=False, density=False)
    r = rm.fragment(*to_dev(B, eo, ev), gamma=False, density=False, opts=rm.make_opts(slab_group=g))
    ep = r.e_pair.cpu().numpy()
    assert np.all(np.abs(ep - ref["e_pair"]) <= 1e-12 * np.abs(ref["e_pair"]) + 1e-15)
    e = r.E.cpu().numpy()
    assert abs(math.fsum([e[0], e[1], -ref["E_hi"], -ref["E_lo"]])) <= 1e-12 * abs(ref["E_hi"])


@pytest.mark.parametrize("density", [False, True])
def test_pair_skip_sums_unskipped_pairs(density):
    f = synth.screen_system(4001, nocc=10, nvir=40, naux=80)
    B, eo, ev = f.arrays()
    ref = O.fragment(B, eo, ev, gamma=False, density=False)
    rng = np.random.default_rng(8)
    m = np.triu(rng.random((10, 10)) < 0.4, 1)
    m = (m | m.T).astype(np.uint8)
    dB, deo, dev_ = to_dev(B, eo, ev)
    skip = torch.from_numpy(m).to(DEV)
    r = rm.fragment(dB, deo, dev_, gamma=density, density=density, opts=rm.make_opts(pair_skip=skip, slab_group=3))
    ep = r.e_pair.cpu().numpy()
    assert np.all(ep[m > 0] == 0)
    keep = m == 0
    assert np.all(np.abs(ep[keep] - ref["e_pair"][keep]) <= 1e-12 * np.abs(ref["e_pair"][keep]))
    e = r.E.cpu().numpy()
    want = math.fsum(ref["e_pair"][keep].tolist())
    assert abs(math.fsum([e[0], e[1], -want])) <= 1e-12 * abs(want)


def test_training_reduces_loss():
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, 1, (4096, 4))
    t = np.sin(2 * x[:, 0]) + x[:, 1] * x[:, 2] - 0.5 * x[:, 3]
    dx, dt = to_dev(x, t)
    p = SC.init_params(0, DEV)
    tr = SC.Trainer(p, lr=3e-3)
    l0 = float(SC.mlp_loss_grad(dx, dt, p)[0])
    tr.fit(dx, dt, steps=400, batch=512)
    l1 = float(SC.mlp_loss_grad(dx, dt, tr.params)[0])
    say("training loss %.3e -> %.3e" % (l0, l1))
    assert l1 < l0 / 20
