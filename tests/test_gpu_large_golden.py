"""The large fragment (nocc=200, nvir=1800, naux=6000) at full size, in the
launch configuration bench.py times (default options: slab groups of 6
occupied orbitals, every output), against the CPU oracle's stored outputs.

tests/golden/large_oracle.npz was written by tests/golden/make_large_golden.py,
which calls only oracle/ and synth/ (about 1.7 h on 6 cores).  Gamma is not
stored; its rows are computed here with oracle.gamma_rows, at every tile edge
of the virtual index (a = 0, 127, 128, 1799 against 128-wide GEMM tiles) for
occupied orbitals at the edges of the slab groups of 6 (k = 0, 5, 6) and in
the last, ragged group (k = 198, 199), plus two interior ones.  Every element
is held to |d| <= 1e-12 |ref| + 1e-12 max|ref row|.  The symmetric path (E and
Gamma without P) runs at full size too and is held to the same bars.
"""
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import rimp2_oracle as O
import paper_2410_21888_amd as rm
from gpu_util import rel_fro, say, assert_elementwise

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_oracle.npz")


@pytest.mark.timeout(900)
@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden file not generated")
def test_large_fragment_against_stored_oracle():
    g = np.load(GOLDEN)
    f = synth.LARGE
    assert tuple(g["shape"]) == (f.nocc, f.nvir, f.naux) and int(g["seed"]) == f.seed
    assert float(g["decay"]) == f.decay
    say("large golden: generating inputs")
    B, eo, ev = f.arrays()
    dev = torch.device("cuda:0")
    dB = torch.from_numpy(B).to(dev)
    deo, dev_ = torch.from_numpy(eo).to(dev), torch.from_numpy(ev).to(dev)
    say("large golden: running the fragment kernel")
    r = rm.fragment(dB, deo, dev_)
    torch.cuda.synchronize()
    E = r.E.cpu().numpy()
    dE = abs(math.fsum([float(E[0]), float(E[1]), -float(g["E"][0]), -float(g["E"][1])]))
    say("large golden: |dE| = %.3e Eh (E = %.6e)" % (dE, float(g["E"][0])))
    assert dE <= 1e-6
    ep = r.e_pair.cpu().numpy()
    ref_ep = g["e_pair"]
    assert np.all(np.abs(ep - ref_ep) <= 1e-12 * np.abs(ref_ep) + 1e-15)
    pij = r.P_ij.cpu().numpy()
    assert rel_fro(pij, g["P_ij"]) <= 1e-12
    assert_elementwise(pij, g["P_ij"], 1e-12, 1e-12, "P_ij")
    pab = r.P_ab.cpu().numpy()
    rows = g["P_ab_row_index"]
    assert rel_fro(pab[rows], g["P_ab_rows"]) <= 1e-12
    assert_elementwise(pab[rows], g["P_ab_rows"], 1e-12, 1e-12, "P_ab rows")
    assert rel_fro(np.diag(pab), g["P_ab_diag"]) <= 1e-12
    assert abs(np.linalg.norm(pab) - float(g["P_ab_fro"])) <= 1e-12 * float(g["P_ab_fro"])
    # the same at full size through the symmetric path (E and Gamma without P:
    # each unordered pair once, the transposed blocks through the second GEMM);
    # rows past the first slab group get their earlier-group contributions
    # from the transposed GEMM
    Gam_full = {}
    avals = [0, 127, 128, 900, 1799]
    irows = (0, 5, 6, 57, 120, 198, 199)
    for i in irows:
        Gam_full[i] = r.Gamma[i, avals].cpu().numpy()
    del r
    torch.cuda.empty_cache()
    say("large golden: running the symmetric path (E and Gamma only)")
    rs = rm.fragment(dB, deo, dev_, density=False)
    torch.cuda.synchronize()
    Es = rs.E.cpu().numpy()
    dEs = abs(math.fsum([float(Es[0]), float(Es[1]), -float(g["E"][0]), -float(g["E"][1])]))
    say("large golden: symmetric path |dE| = %.3e Eh" % dEs)
    assert dEs <= 1e-6
    eps_ = rs.e_pair.cpu().numpy()
    assert np.all(np.abs(eps_ - ref_ep) <= 1e-12 * np.abs(ref_ep) + 1e-15)
    Gam_sym = {i: rs.Gamma[i, avals].cpu().numpy() for i in irows}
    del rs, dB
    torch.cuda.empty_cache()
    for i in irows:
        ref = O.gamma_rows(B, eo, ev, i, avals)
        for name, got in (("ordered", Gam_full[i]), ("symmetric", Gam_sym[i])):
            err = rel_fro(got, ref)
            say("large golden: %s Gamma[%d, %s, :] rel err %.2e" % (name, i, avals, err))
            assert err <= 1e-12
            assert_elementwise(got, ref, 1e-12, 1e-12, "%s Gamma[%d]" % (name, i))
