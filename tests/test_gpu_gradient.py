"""Metric contraction of Gamma on the GPU (rimp2_gamma_metric) against the
oracle, element by element (|d| <= 1e-12 |ref| + 1e-12 max|ref row|) and by
relative Frobenius norm; the metric is not symmetric, so a transposed operand
would show."""
import numpy as np
import pytest
import torch

import synth
from oracle import rimp2_oracle as O
import paper_2410_21888_amd as rm
from paper_2410_21888_amd import gradient as G
from gpu_util import to_dev, rel_fro, say, assert_elementwise

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 17, 33), (5, 40, 300), (4, 130, 257), (2, 64, 128)])
def test_gamma_metric_matches_oracle(shape):
    nocc, nvir, naux = shape
    rng = np.random.default_rng(sum(shape))
    Gam = rng.standard_normal((nocc, nvir, naux))
    Jm = rng.standard_normal((naux, naux))
    say("gamma_metric %s" % (shape,))
    dG, dJ = to_dev(Gam, Jm)
    got = G.gamma_metric(dG, dJ).cpu().numpy()
    torch.cuda.synchronize()
    ref = O.gamma_metric(Gam, Jm)
    assert rel_fro(got, ref) <= 1e-13
    assert_elementwise(got, ref, 1e-12, 1e-12, "gamma_metric")


def test_gamma_metric_after_the_fragment_kernel():
    f = synth.random_fragment(6, 50, 96, seed=41)
    B, eo, ev = f.arrays()
    Jm = np.random.default_rng(42).standard_normal((96, 96))
    r = rm.fragment(*to_dev(B, eo, ev), density=False)
    got = G.gamma_metric(r.Gamma, to_dev(Jm)[0]).cpu().numpy()
    ref = O.gamma_metric(O.fragment(B, eo, ev, density=False)["Gamma"], Jm)
    assert rel_fro(got, ref) <= 1e-13
    assert_elementwise(got, ref, 1e-12, 1e-12, "gamma_metric")


def test_gamma_metric_rejects_overlap():
    g = torch.zeros((2, 3, 4), dtype=torch.float64, device="cuda:0")
    j = torch.eye(4, dtype=torch.float64, device="cuda:0")
    with pytest.raises(rm.Rimp2Error):
        G.gamma_metric(g, j, out=g)


# AO back-transform: rectangular, different coefficient matrices (a swapped or
# transposed one would show), odd and even nao (the M-contiguous loader's
# fast and masked paths), auxiliary chunks that start at odd offsets.
@pytest.mark.parametrize("shape", [(1, 1, 1, 1, 0, 1), (2, 3, 5, 4, 0, 4), (3, 17, 24, 33, 5, 20),
                                   (5, 40, 50, 64, 0, 64), (4, 60, 71, 130, 3, 127), (6, 130, 140, 40, 8, 32)])
def test_gamma_ao_matches_oracle(shape):
    nocc, nvir, nao, naux, p0, pc = shape
    rng = np.random.default_rng(sum(shape) + 1)
    Gam = rng.standard_normal((nocc, nvir, naux))
    Co = rng.standard_normal((nocc, nao))
    Cv = rng.standard_normal((nvir, nao))
    say("gamma_ao %s" % (shape,))
    dG, dCo, dCv = to_dev(Gam, Co, Cv)
    got = G.gamma_ao(dG, dCo, dCv, p0=p0, pcount=pc).cpu().numpy()
    ref = O.gamma_ao(Gam[:, :, p0:p0 + pc], Co, Cv)
    assert rel_fro(got, ref) <= 1e-13
    assert_elementwise(got, ref, 1e-12, 1e-12, "gamma_ao")


def test_gamma_ao_chunks_tile_the_full_tensor():
    nocc, nvir, nao, naux = 4, 30, 36, 50
    rng = np.random.default_rng(3)
    dG, dCo, dCv = to_dev(rng.standard_normal((nocc, nvir, naux)), rng.standard_normal((nocc, nao)),
                          rng.standard_normal((nvir, nao)))
    full = G.gamma_ao(dG, dCo, dCv)
    parts = [G.gamma_ao(dG, dCo, dCv, p0=p0, pcount=min(16, naux - p0)) for p0 in range(0, naux, 16)]
    assert torch.equal(torch.cat(parts, dim=2), full)


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 4), (3, 17, 33), (5, 40, 64), (4, 60, 130), (7, 33, 18)])
def test_l_terms_match_oracle(shape):
    nocc, nvir, naux = shape
    nmo = nocc + nvir
    rng = np.random.default_rng(sum(shape) + 2)
    Gam = rng.standard_normal((nocc, nvir, naux))
    I_qa = rng.standard_normal((nmo, nvir, naux))
    I_iq = rng.standard_normal((nocc, nmo, naux))
    say("l_terms %s" % (shape,))
    L1, L2 = G.l_terms(*to_dev(Gam, I_qa, I_iq))
    ref1, ref2 = O.l_prime(Gam, I_qa), O.l_dprime(Gam, I_iq)
    for got, ref, name in ((L1, ref1, "L'"), (L2, ref2, "L''")):
        g = got.cpu().numpy()
        assert rel_fro(g, ref) <= 1e-13, name
        assert_elementwise(g, ref, 1e-12, 1e-12, name)
    only1, none2 = G.l_terms(*to_dev(Gam, I_qa), None)
    assert none2 is None and torch.equal(only1, L1)


def test_l_terms_after_the_fragment_kernel():
    """The chain the Appendix describes: fragment Gamma, its metric
    contraction, then L' and L'' against the oracle's same chain."""
    nocc, nvir, naux = 5, 30, 48
    nmo = nocc + nvir
    f = synth.random_fragment(nocc, nvir, naux, seed=43)
    B, eo, ev = f.arrays()
    rng = np.random.default_rng(44)
    Jm = rng.standard_normal((naux, naux))
    I_qa = rng.standard_normal((nmo, nvir, naux))
    I_iq = rng.standard_normal((nocc, nmo, naux))
    r = rm.fragment(*to_dev(B, eo, ev), density=False)
    Gm = G.gamma_metric(r.Gamma, to_dev(Jm)[0])
    L1, L2 = G.l_terms(Gm, *to_dev(I_qa, I_iq))
    Gref = O.gamma_metric(O.fragment(B, eo, ev, density=False)["Gamma"], Jm)
    assert_elementwise(L1.cpu().numpy(), O.l_prime(Gref, I_qa), 1e-11, 1e-11, "L'")
    assert_elementwise(L2.cpu().numpy(), O.l_dprime(Gref, I_iq), 1e-11, 1e-11, "L''")
