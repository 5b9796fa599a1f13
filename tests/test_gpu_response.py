"""Orbital response on the GPU (antisymmetrised-integral term, Z-vector
solve, energy-weighted density W) against the CPU oracle, element by element.

Inputs: a seeded three-index factor Bf over every pair of molecular orbitals
(symmetric in the pair, 0.05 N(0,1) exp(-P/40): small enough that the orbital
Hessian is positive definite, as for a stable closed-shell reference), orbital
energies as in the fragment workloads, and the fragment kernel's own P_ij,
P_ab and Gamma for the chain test.  Bars: the antisymmetrised term and W to
|d| <= 1e-12 |ref| + 1e-12 max|ref row|; D_ai, an iterative solution, to
1e-9 |ref| + 1e-9 max|ref row| with CG run to a relative residual of 1e-13.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import rimp2_oracle as O
import paper_2410_21888_amd as rm
from paper_2410_21888_amd import gradient as G
from gpu_util import to_dev, say, assert_elementwise

pytestmark = pytest.mark.gpu


def full_factor(nocc, nvir, naux, seed, scale=0.05, decay=40.0):
    rng = np.random.default_rng(seed)
    nmo = nocc + nvir
    Bf = scale * rng.standard_normal((nmo, nmo, naux)) * np.exp(-np.arange(naux) / decay)
    Bf = 0.5 * (Bf + Bf.transpose(1, 0, 2))
    eo = np.sort(rng.uniform(-20.0, -0.3, nocc))
    ev = np.sort(rng.uniform(0.1, 5.0, nvir))
    return np.ascontiguousarray(Bf), eo, ev


@pytest.mark.parametrize("shape,rows,cols", [((2, 3, 4), None, None), ((5, 17, 33), (5, 22), (0, 5)),
                                             ((4, 40, 70), (0, 4), None), ((7, 60, 130), (3, 50), (10, 61)),
                                             ((3, 129, 16), None, (0, 3))])
def test_antisym_term_matches_oracle(shape, rows, cols):
    nocc, nvir, naux = shape
    nmo = nocc + nvir
    Bf, _, _ = full_factor(nocc, nvir, naux, sum(shape), scale=0.3)
    D = np.random.default_rng(sum(shape) + 1).standard_normal((nmo, nmo))
    say("antisym %s rows %s cols %s" % (shape, rows, cols))
    got = G.antisym_term(*to_dev(Bf, D), rows=rows, cols=cols).cpu().numpy()
    r0, r1 = rows if rows else (0, nmo)
    c0, c1 = cols if cols else (0, nmo)
    ref = O.antisym_term(Bf, D)[r0:r1, c0:c1]
    assert_elementwise(got, ref, 1e-12, 1e-12, "antisym")


@pytest.mark.parametrize("shape", [(1, 1, 3), (3, 8, 20), (6, 30, 64), (8, 45, 100)])
def test_zvector_matches_oracle(shape):
    nocc, nvir, naux = shape
    nmo = nocc + nvir
    Bf, eo, ev = full_factor(nocc, nvir, naux, 3 * sum(shape))
    rng = np.random.default_rng(sum(shape) + 2)
    D_oo = rng.standard_normal((nocc, nocc))
    D_vv = rng.standard_normal((nvir, nvir))
    D_oo, D_vv = D_oo + D_oo.T, D_vv + D_vv.T
    L1 = rng.standard_normal((nocc, nmo))
    L2 = rng.standard_normal((nvir, nmo))
    say("zvector %s" % (shape,))
    D_ai, it, res = G.zvector(*to_dev(Bf, eo, ev, D_oo, D_vv, L1, L2), tol=1e-13, max_iter=400)
    say("  %d iterations, relative residual %.2e" % (it, res))
    assert res <= 1e-13
    ref = O.zvector(Bf, eo, ev, D_oo, D_vv, L1, L2)
    assert_elementwise(D_ai.cpu().numpy(), ref, 1e-9, 1e-9, "D_ai")


def test_zvector_reports_no_convergence():
    """One iteration cannot reach 1e-13: RIMP2_ENOCONV, forced from the host."""
    nocc, nvir, naux = 6, 30, 64
    nmo = nocc + nvir
    Bf, eo, ev = full_factor(nocc, nvir, naux, 7)
    rng = np.random.default_rng(8)
    args = to_dev(Bf, eo, ev, np.eye(nocc), np.eye(nvir), rng.standard_normal((nocc, nmo)),
                  rng.standard_normal((nvir, nmo)))
    with pytest.raises(rm.Rimp2Error) as ei:
        G.zvector(*args, tol=1e-13, max_iter=1)
    assert ei.value.code == rm.RIMP2_ENOCONV


@pytest.mark.parametrize("shape", [(2, 3, 4), (5, 24, 50), (7, 40, 90)])
def test_energy_weighted_density_matches_oracle(shape):
    nocc, nvir, naux = shape
    nmo = nocc + nvir
    Bf, eo, ev = full_factor(nocc, nvir, naux, 5 * sum(shape), scale=0.3)
    rng = np.random.default_rng(sum(shape) + 3)
    D_oo = rng.standard_normal((nocc, nocc))
    D_vv = rng.standard_normal((nvir, nvir))
    D_oo, D_vv = D_oo + D_oo.T, D_vv + D_vv.T
    D_vo = rng.standard_normal((nvir, nocc))
    L1 = rng.standard_normal((nocc, nmo))
    L2 = rng.standard_normal((nvir, nmo))
    say("W %s" % (shape,))
    W = G.energy_weighted_density(*to_dev(Bf, eo, ev, D_oo, D_vv, D_vo, L1, L2)).cpu().numpy()
    ref = O.energy_weighted_density(Bf, eo, ev, D_oo, D_vv, D_vo, L1, L2)
    assert_elementwise(W, ref, 1e-12, 1e-12, "W")


def test_response_chain_from_the_fragment_kernel():
    """The Appendix's sequence on one synthetic system: fragment kernel (E,
    Gamma, P_ij, P_ab) -> metric contraction of Gamma -> L', L'' -> Z-vector
    D_ai -> W, on the GPU, against the oracle's same sequence."""
    nocc, nvir, naux = 6, 36, 80
    nmo = nocc + nvir
    Bf, eo, ev = full_factor(nocc, nvir, naux, 99)
    B = np.ascontiguousarray(Bf[:nocc, nocc:])                 # (P|ia) J^-1/2 block
    Jm = np.eye(naux) + 0.01 * np.random.default_rng(100).standard_normal((naux, naux))
    I_qa = np.ascontiguousarray(np.transpose(Bf[:, nocc:], (0, 1, 2)))   # (P|qa) stand-in [nmo][nvir][naux]
    I_iq = np.ascontiguousarray(Bf[:nocc])                      # (P|iq) stand-in [nocc][nmo][naux]
    dB, deo, dev_ = to_dev(B, eo, ev)
    r = rm.fragment(dB, deo, dev_)
    Gm = G.gamma_metric(r.Gamma, to_dev(Jm)[0])
    L1, L2 = G.l_terms(Gm, *to_dev(I_qa, I_iq))
    dBf = to_dev(Bf)[0]
    D_ai, it, res = G.zvector(dBf, deo, dev_, r.P_ij, r.P_ab, L1, L2, tol=1e-13, max_iter=400)
    W = G.energy_weighted_density(dBf, deo, dev_, r.P_ij, r.P_ab, D_ai, L1, L2)
    say("chain: Z-vector %d iterations, residual %.2e" % (it, res))
    ref = O.fragment(B, eo, ev)
    Gref = O.gamma_metric(ref["Gamma"], Jm)
    L1r, L2r = O.l_prime(Gref, I_qa), O.l_dprime(Gref, I_iq)
    Dr = O.zvector(Bf, eo, ev, ref["P_ij"], ref["P_ab"], L1r, L2r)
    Wr = O.energy_weighted_density(Bf, eo, ev, ref["P_ij"], ref["P_ab"], Dr, L1r, L2r)
    assert_elementwise(L1.cpu().numpy(), L1r, 1e-11, 1e-11, "L'")
    assert_elementwise(L2.cpu().numpy(), L2r, 1e-11, 1e-11, "L''")
    assert_elementwise(D_ai.cpu().numpy(), Dr, 1e-9, 1e-9, "D_ai")
    assert_elementwise(W.cpu().numpy(), Wr, 1e-9, 1e-9, "W")
