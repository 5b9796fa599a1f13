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
from gpu_util import to_dev, rel_fro, say, assert_elementwise
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


# The screened path against the oracle with the same mask (oracle.fragment's
# skip): every element of e_pair, Gamma, P_ij and P_ab.  Slab groups of 3 put
# skipped pairs both inside one group (blocks formed from their mirror) and
# across groups (blocks formed on their own); slab_group=0 puts every pair in
# one group; density=False with gamma=False takes the energy-only path.
@pytest.mark.parametrize("outputs,g", [("energy", 3), ("gamma", 3), ("all", 3), ("all", 0), ("all", 1)])
def test_pair_skip_matches_oracle_with_mask(outputs, g):
    nocc = 10
    f = synth.screen_system(4001, nocc=nocc, nvir=40, naux=80)
    B, eo, ev = f.arrays()
    gamma, density = outputs in ("gamma", "all"), outputs == "all"
    rng = np.random.default_rng(8)
    m = np.triu(rng.random((nocc, nocc)) < 0.4, 1)
    m[2, 3] = m[0, 9] = True        # one pair inside the first group, one across groups
    m = (m | m.T).astype(np.uint8)
    ref = O.fragment(B, eo, ev, gamma=gamma, density=density, skip=m)
    dB, deo, dev_ = to_dev(B, eo, ev)
    say("pair skip: outputs=%s slab_group=%d skipped pairs=%d" % (outputs, g, int(m.sum()) // 2))
    r = rm.fragment(dB, deo, dev_, gamma=gamma, density=density,
                    opts=rm.make_opts(pair_skip=torch.from_numpy(m).to(DEV), slab_group=g))
    ep = r.e_pair.cpu().numpy()
    assert np.all(ep[m > 0] == 0)
    assert_elementwise(ep, ref["e_pair"], 1e-12, 1e-15, "e_pair")
    e = r.E.cpu().numpy()
    assert abs(math.fsum([e[0], e[1], -ref["E_hi"], -ref["E_lo"]])) <= 1e-12 * abs(ref["E_hi"])
    if gamma:
        G = r.Gamma.cpu().numpy()
        assert_elementwise(G, ref["Gamma"], 1e-12, 1e-12, "Gamma")
    if density:
        assert_elementwise(r.P_ij.cpu().numpy(), ref["P_ij"], 1e-12, 1e-12, "P_ij")
        assert_elementwise(r.P_ab.cpu().numpy(), ref["P_ab"], 1e-12, 1e-12, "P_ab")


@pytest.mark.parametrize("outputs", ["energy", "all"])
def test_pair_skip_mask_names_unordered_pairs(outputs):
    """A mask with only (i, j) or only (j, i) set screens the pair out in
    both orders: bitwise the same outputs as the symmetric mask, whatever the
    slab grouping, and equal to the oracle."""
    nocc = 9
    f = synth.screen_system(4002, nocc=nocc, nvir=36, naux=72)
    B, eo, ev = f.arrays()
    gamma = density = outputs == "all"
    rng = np.random.default_rng(10)
    up = np.triu(rng.random((nocc, nocc)) < 0.35, 1)
    sym = (up | up.T).astype(np.uint8)
    # each pair marked on one side only, the side chosen at random
    side = rng.random((nocc, nocc)) < 0.5
    asym = np.zeros_like(sym)
    asym[up & side] = 1
    asym[(up & ~side).T] = 1
    dB, deo, dev_ = to_dev(B, eo, ev)
    ref = O.fragment(B, eo, ev, gamma=gamma, density=density, skip=sym)
    for g in (1, 4, 0):
        outs = []
        for mask in (sym, asym):
            r = rm.fragment(dB, deo, dev_, gamma=gamma, density=density,
                            opts=rm.make_opts(pair_skip=torch.from_numpy(mask).to(DEV), slab_group=g))
            outs.append(r)
        for name, a, b in zip(outs[0]._fields, outs[0], outs[1]):
            if a is not None:
                assert torch.equal(a, b), (g, name)
        assert_elementwise(outs[1].e_pair.cpu().numpy(), ref["e_pair"], 1e-12, 1e-15, "e_pair")
        if gamma:
            assert_elementwise(outs[1].Gamma.cpu().numpy(), ref["Gamma"], 1e-12, 1e-12, "Gamma")
            assert_elementwise(outs[1].P_ab.cpu().numpy(), ref["P_ab"], 1e-12, 1e-12, "P_ab")
            assert_elementwise(outs[1].P_ij.cpu().numpy(), ref["P_ij"], 1e-12, 1e-12, "P_ij")


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
