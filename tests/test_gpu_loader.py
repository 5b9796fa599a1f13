"""The FP64 GEMMs' two operand loaders against each other (opts.gemm_loader).

The fast loader (two chunks of global loads in flight, clamped edge rows,
per-thread run steps, a ragged last chunk loaded once after the loop) and the
general loader sum every output element in the same order, so the whole
fragment path must give bitwise identical outputs with either.  The shapes
reach every branch of the fast loader: reductions of one to several chunks,
ragged last chunks, edge tiles in M and N, runs that end inside a chunk, and
slab groups; a batch covers the grouped launches' loader lists.
"""
import pytest
import torch

import synth
import paper_2410_21888_amd as rm
from gpu_util import to_dev, say

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 2), (2, 3, 4), (3, 40, 16), (4, 30, 54), (6, 20, 2), (5, 48, 64), (7, 64, 130), (3, 144, 96),
          (9, 150, 260), (4, 600, 64), (10, 150, 130)]


def _run(dB, deo, dev_, **kw):
    r = rm.fragment(dB, deo, dev_, opts=rm.make_opts(**kw))
    torch.cuda.synchronize()
    return r


@pytest.mark.parametrize("shape", SHAPES)
def test_fast_and_general_loaders_agree_bitwise(shape):
    nocc, nvir, naux = shape
    f = synth.random_fragment(nocc, nvir, naux, seed=11 * nocc + nvir + naux)
    dB, deo, dev_ = to_dev(*f.arrays())
    for g in sorted({0, max(1, nocc // 3)}):
        say("loaders nocc=%d nvir=%d naux=%d slab_group=%d" % (nocc, nvir, naux, g))
        fast = _run(dB, deo, dev_, slab_group=g)
        general = _run(dB, deo, dev_, slab_group=g, gemm_loader=1)
        for name, a, b in zip(fast._fields, fast, general):
            assert torch.equal(a, b), (shape, g, name)


def test_batch_loaders_agree_bitwise():
    sizes = [(5, 25, 90), (12, 60, 216), (7, 35, 126), (3, 15, 54), (8, 40, 144), (6, 30, 108), (4, 20, 72)]
    outs = []
    for loader in (0, 1):
        frags = []
        for n, (nocc, nvir, naux) in enumerate(sizes):
            B, eo, ev = synth.Fragment(nocc, nvir, naux, seed=1007, frag=n).arrays()
            dB, deo, dev_ = to_dev(B, eo, ev)
            kw = dict(dtype=torch.float64, device=dB.device)
            frags.append(dict(B=dB, eps_occ=deo, eps_vir=dev_, E=torch.zeros(2, **kw), Gamma=torch.empty_like(dB),
                              P_ij=torch.empty((nocc, nocc), **kw), P_ab=torch.empty((nvir, nvir), **kw),
                              e_pair=torch.empty((nocc, nocc), **kw)))
        say("batch of %d fragments, gemm_loader=%d" % (len(frags), loader))
        # a small wave budget: the largest fragments run alone, the rest in grouped waves
        rm.fragment_batch(frags, opts=rm.make_opts(slab_budget_bytes=3 << 20, gemm_loader=loader))
        torch.cuda.synchronize()
        outs.append(frags)
    for n, (a, b) in enumerate(zip(*outs)):
        for key in ("E", "Gamma", "P_ij", "P_ab", "e_pair"):
            assert torch.equal(a[key], b[key]), (n, key)
