"""The symmetric Gamma path (E and Gamma without P_ij and P_ab) against the
CPU oracle, element by element.

Without P the library forms (ia|jb) for pairs j >= k only.  Gamma rows of a
slab group get T_kj B_j over those pairs from one GEMM, and the rows of every
later orbital j get the transposed blocks, sum over (k, a) of T_kj[a, b]
B_k[a, P] (T_jk = T_kj^T), from a second GEMM that reads the T slab as an
M-contiguous operand.  Contributions reach each row in a fixed order (earlier
groups first), so results are bitwise reproducible.

Bar: |dE| <= 1e-12 |E| from exact (hi, lo) sums; e_ij within 1e-12 relative;
every Gamma element within 1e-12 |ref| + 1e-12 max|ref row|, and relative
Frobenius <= 1e-8.  The shapes reach the M-contiguous loader's fast path
(even M = rows past the group times nvir), its general masked path (odd
nvir), ragged reductions (K = g nvir not a multiple of 16), one-orbital
groups, groups that grow under a small slab budget, and a single group.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import rimp2_oracle as O
import paper_2410_21888_amd as rm
from gpu_util import to_dev, rel_fro, energy_error, say, assert_elementwise

pytestmark = pytest.mark.gpu


def run_sym(f, opts=None, ref=None):
    B, eo, ev = f.arrays()
    say("symmetric case nocc=%d nvir=%d naux=%d seed=%d" % (f.nocc, f.nvir, f.naux, f.seed))
    r = rm.fragment(*to_dev(B, eo, ev), density=False, opts=opts)
    torch.cuda.synchronize()
    if ref is None:
        ref = O.fragment(B, eo, ev, density=False)
    assert energy_error(r.E, ref["E_hi"], ref["E_lo"]) <= 1e-12 * abs(ref["E_hi"]) + 1e-15
    ep = r.e_pair.cpu().numpy()
    assert np.all(np.abs(ep - ref["e_pair"]) <= 1e-12 * np.abs(ref["e_pair"]) + 1e-15)
    assert np.array_equal(ep, ep.T)   # each unordered pair is formed once and written to both
    G = r.Gamma.cpu().numpy()
    assert rel_fro(G, ref["Gamma"]) <= 1e-8
    assert_elementwise(G, ref["Gamma"], 1e-12, 1e-12, "Gamma")
    return r, ref


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 4), (3, 17, 33), (5, 33, 100), (4, 130, 257),
                                   (9, 64, 128), (3, 40, 16), (6, 16, 160), (7, 64, 130), (6, 25, 100),
                                   (5, 30, 36), (2, 129, 17)])
def test_symmetric_gamma_shapes(shape):
    nocc, nvir, naux = shape
    run_sym(synth.random_fragment(nocc, nvir, naux, seed=5 * nocc + nvir + naux))


@pytest.mark.parametrize("g", [1, 2, 3, 4])
def test_symmetric_gamma_slab_groups(g):
    run_sym(synth.random_fragment(9, 40, 90, seed=78), opts=rm.make_opts(slab_group=g))


def test_symmetric_gamma_growing_groups():
    """A slab budget that fits two orbitals' slabs at the start: later groups
    (fewer columns j >= k0) take more orbitals."""
    nocc, nvir, naux = 11, 48, 70
    budget = 2 * 2 * 8 * nocc * nvir * nvir
    f = synth.random_fragment(nocc, nvir, naux, seed=79)
    r, ref = run_sym(f, opts=rm.make_opts(slab_budget_bytes=budget))
    # the same with fixed groups of one orbital gives the same values to rounding
    run_sym(f, opts=rm.make_opts(slab_group=1), ref=ref)


def test_symmetric_gamma_small_workload():
    run_sym(synth.SMALL)


def test_symmetric_gamma_deterministic_and_loaders():
    """Run twice: bitwise equal.  The general loader only (opts.gemm_loader =
    1) and the autotuner's tile choices sum in the same order: bitwise equal
    too."""
    f = synth.random_fragment(8, 70, 150, seed=80)
    d = to_dev(*f.arrays())
    base = rm.make_opts(slab_group=3)
    r1 = rm.fragment(*d, density=False, opts=base)
    r2 = rm.fragment(*d, density=False, opts=base)
    r3 = rm.fragment(*d, density=False, opts=rm.make_opts(slab_group=3, gemm_loader=1))
    for a, b, c in zip(r1, r2, r3):
        if a is not None:
            assert torch.equal(a, b) and torch.equal(a, c)
    rm.autotune_reset()
    tuned = rm.make_opts(slab_group=3, autotune=True)
    for call in range(6):
        r = rm.fragment(*d, density=False, opts=tuned)
        for name, a, b in zip(r._fields, r, r1):
            if a is not None:
                assert torch.equal(a, b), (call, name)
    roles = {e["role"] for e in rm.autotune_report()}
    assert {"ints_gemm", "gamma_gemm", "gamma_t_gemm"} <= roles
    rm.autotune_reset()


def test_symmetric_gamma_matches_ordered_path():
    """E from the symmetric path equals the ordered path's (with P) to
    rounding, and Gamma too: the two paths share no GEMM launch shapes."""
    f = synth.random_fragment(7, 45, 80, seed=81)
    d = to_dev(*f.arrays())
    rs = rm.fragment(*d, density=False)
    ro = rm.fragment(*d)
    assert abs((rs.E_hi - ro.E_hi) + (rs.E_lo - ro.E_lo)) <= 1e-12 * abs(ro.E_hi)
    assert_elementwise(rs.Gamma.cpu().numpy(), ro.Gamma.cpu().numpy(), 1e-12, 1e-12, "Gamma")
