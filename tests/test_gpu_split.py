"""Split-precision path (INT8 digit products, Ozaki scheme) against the CPU oracle.

Bar: |dE| <= 1 uEh (exact evaluation of the (hi, lo) pairs) and relative
Frobenius error <= 1e-8 for Gamma, P_ij and P_ab, with the default digit
counts (7 for (ia|jb), 5 for Gamma); every element of Gamma, P_ij, P_ab and
e_pair is also held to |d| <= 1e-8 |ref| + 1e-8 max|ref row|.  The error must
also fall steeply with the number of digits (about 2^-7 per digit).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import rimp2_oracle as O
import paper_2410_21888_amd as rm
from gpu_util import to_dev, rel_fro, energy_error, say, assert_elementwise

pytestmark = pytest.mark.gpu


def split_opts(sv=0, sg=0, g=0):
    return rm.make_opts(precision=rm.SPLIT_INT8, split_slices=sv, split_slices_gamma=sg, slab_group=g)


def check(f, opts, e_tol=1e-6, rel_tol=1e-8):
    B, eo, ev = f.arrays()
    say("split case nocc=%d nvir=%d naux=%d" % (f.nocc, f.nvir, f.naux))
    r = rm.fragment(*to_dev(B, eo, ev), opts=opts)
    ref = O.fragment(B, eo, ev)
    dE = energy_error(r.E, ref["E_hi"], ref["E_lo"])
    assert dE <= e_tol, dE
    for key, got in (("Gamma", r.Gamma), ("P_ij", r.P_ij), ("P_ab", r.P_ab), ("e_pair", r.e_pair)):
        g = got.cpu().numpy()
        err = rel_fro(g, ref[key])
        assert err <= rel_tol, (key, err)
        assert_elementwise(g, ref[key], rel_tol, rel_tol, key)
    return dE


def test_split_small_workload():
    check(synth.SMALL, split_opts())


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 17, 33), (5, 70, 130), (2, 129, 65)])
def test_split_ragged(shape):
    nocc, nvir, naux = shape
    check(synth.random_fragment(nocc, nvir, naux, seed=sum(shape) + 3), split_opts(g=2))


@pytest.mark.parametrize("sv", [5, 7])
def test_split_long_reduction_windows(sv):
    """naux = 70000: the (ia|jb) product's reduction runs in windows, one
    launch each, every later window adding into the output (25 windows of 2816)."""
    check(synth.random_fragment(2, 8, 70000, seed=41), split_opts(sv=sv))


def test_split_gamma_windows():
    """nocc * nvir = 8400 (padded to 8448): the Gamma product's reduction runs
    in three windows of 2816, the later ones adding into the first's output."""
    f = synth.random_fragment(2, 4200, 24, seed=43)
    B, eo, ev = f.arrays()
    say("split Gamma windows nocc=2 nvir=4200 naux=24")
    r = rm.fragment(*to_dev(B, eo, ev), density=False, opts=split_opts())
    ref = O.fragment(B, eo, ev, density=False)
    assert energy_error(r.E, ref["E_hi"], ref["E_lo"]) <= 1e-6
    g = r.Gamma.cpu().numpy()
    assert rel_fro(g, ref["Gamma"]) <= 1e-8
    assert_elementwise(g, ref["Gamma"], 1e-8, 1e-8, "Gamma")


@pytest.mark.parametrize("g", [0, 1, 3])
def test_split_symmetric_e_gamma(g):
    """E and Gamma without P take the symmetric path with split products: the
    (ia|jb) products over pairs j >= k0, the Gamma row-block products and the
    transposed-block products, group after group (g orbitals per group; 0 =
    the planner's choice, one group here)."""
    f = synth.random_fragment(7, 90, 150, seed=51)
    B, eo, ev = f.arrays()
    say("split symmetric path nocc=7 nvir=90 naux=150 g=%d" % g)
    r = rm.fragment(*to_dev(B, eo, ev), density=False, opts=split_opts(g=g))
    ref = O.fragment(B, eo, ev, density=False)
    assert energy_error(r.E, ref["E_hi"], ref["E_lo"]) <= 1e-6
    for key, got in (("Gamma", r.Gamma), ("e_pair", r.e_pair)):
        got = got.cpu().numpy()
        assert rel_fro(got, ref[key]) <= 1e-8, key
        assert_elementwise(got, ref[key], 1e-8, 1e-8, key)


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 17, 33), (2, 129, 65), (5, 70, 130)])
def test_split_symmetric_ragged(shape):
    """Ragged sizes on the symmetric split path, one orbital per group."""
    nocc, nvir, naux = shape
    f = synth.random_fragment(nocc, nvir, naux, seed=sum(shape) + 7)
    B, eo, ev = f.arrays()
    say("split symmetric ragged %s" % (shape,))
    r = rm.fragment(*to_dev(B, eo, ev), density=False, opts=split_opts(g=1))
    ref = O.fragment(B, eo, ev, density=False)
    assert energy_error(r.E, ref["E_hi"], ref["E_lo"]) <= 1e-6
    for key, got in (("Gamma", r.Gamma), ("e_pair", r.e_pair)):
        got = got.cpu().numpy()
        assert rel_fro(got, ref[key]) <= 1e-8, key
        assert_elementwise(got, ref[key], 1e-8, 1e-8, key)


def test_split_symmetric_windows():
    """Symmetric path, one orbital per group: the first group's row-block
    product reduces over 9000 (windowed, the first window storing), the later
    groups' row products add onto the transposed blocks already in their rows."""
    f = synth.random_fragment(3, 3000, 16, seed=53)
    B, eo, ev = f.arrays()
    say("split symmetric path nocc=3 nvir=3000 naux=16 g=1")
    r = rm.fragment(*to_dev(B, eo, ev), density=False, opts=split_opts(g=1))
    ref = O.fragment(B, eo, ev, density=False)
    assert energy_error(r.E, ref["E_hi"], ref["E_lo"]) <= 1e-6
    g = r.Gamma.cpu().numpy()
    assert rel_fro(g, ref["Gamma"]) <= 1e-8
    assert_elementwise(g, ref["Gamma"], 1e-8, 1e-8, "Gamma")


def test_split_error_falls_with_digits():
    f = synth.random_fragment(6, 60, 200, seed=21)
    B, eo, ev = f.arrays()
    ref = O.fragment(B, eo, ev, gamma=True, density=False)
    dB, deo, dev_ = to_dev(B, eo, ev)
    errs = []
    for s in (3, 4, 5, 6, 7):
        r = rm.fragment(dB, deo, dev_, density=False, opts=split_opts(sv=s, sg=s))
        errs.append((energy_error(r.E, ref["E_hi"], ref["E_lo"]) / abs(ref["E_hi"]),
                     rel_fro(r.Gamma.cpu().numpy(), ref["Gamma"])))
        say("digits %d: rel dE %.3e, Gamma %.3e" % (s, errs[-1][0], errs[-1][1]))
    for (e0, g0), (e1, g1) in zip(errs, errs[1:]):
        assert g1 < g0 / 20 or g1 < 1e-14
        assert e1 < e0 / 4 or e1 < 1e-14   # E partly cancels: noisier than Gamma


def test_split_deterministic():
    f = synth.random_fragment(4, 50, 90, seed=31)
    d = to_dev(*f.arrays())
    r1 = rm.fragment(*d, opts=split_opts())
    r2 = rm.fragment(*d, opts=split_opts())
    for a, b in zip(r1, r2):
        assert torch.equal(a, b)
