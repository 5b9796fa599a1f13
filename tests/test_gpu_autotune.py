"""In-situ tile autotuning of the FP64 GEMMs (opts.autotune).

Every candidate tile shape sums each output element in the same order, so a
tuned call must reproduce the untuned call bit for bit, on the trial calls
and after the decision alike; the decision itself must be taken once every
candidate has been timed.
"""
import pytest
import torch

import synth
from oracle import rimp2_oracle as O
import paper_2410_21888_amd as rm
from gpu_util import to_dev, rel_fro, energy_error, say, assert_elementwise

pytestmark = pytest.mark.gpu


def _outputs(dB, deo, dev_, opts):
    r = rm.fragment(dB, deo, dev_, opts=opts)
    torch.cuda.synchronize()
    return r


def test_autotune_bitwise_and_decides():
    # 5 slab groups of 2 occupied orbitals (the last one ragged): two shapes per role
    f = synth.random_fragment(9, 150, 260, seed=31)
    B, eo, ev = f.arrays()
    dB, deo, dev_ = to_dev(B, eo, ev)
    say("autotune case nocc=9 nvir=150 naux=260 slab_group=2")
    ref = _outputs(dB, deo, dev_, rm.make_opts(slab_group=2))
    orc = O.fragment(B, eo, ev)
    assert energy_error(ref.E, orc["E_hi"], orc["E_lo"]) <= 1e-12 * abs(orc["E_hi"])
    assert rel_fro(ref.Gamma.cpu().numpy(), orc["Gamma"]) <= 1e-13
    for key in ("Gamma", "P_ij", "P_ab"):
        assert_elementwise(getattr(ref, key).cpu().numpy(), orc[key], 1e-12, 1e-12, key)
    rm.autotune_reset()
    opts = rm.make_opts(slab_group=2, autotune=True)
    for call in range(8):
        r = _outputs(dB, deo, dev_, opts)
        for name, a, b in zip(r._fields, r, ref):
            assert torch.equal(a, b), (call, name)
    rep = rm.autotune_report()
    roles = {e["role"] for e in rep}
    assert roles == {"ints_gemm", "gamma_gemm", "pab_gemm", "pij_gemm"}
    for e in rep:
        say("tuned %s M=%d N=%d K=%d -> %s timed=%s ms=%s" % (e["role"], e["M"], e["N"], e["K"],
                                                              e["tiles"][e["best"]] if e["best"] >= 0 else None,
                                                              e["timed"], ["%.3f" % t for t in e["min_ms"]]))
        assert e["best"] >= 0, e
        assert all(t == 2 for t in e["timed"]), e
        assert all(ms >= 0 for ms in e["min_ms"]), e
        assert e["uses"] >= 8
    rm.autotune_reset()
    assert rm.autotune_report() == []


def test_autotune_under_graph_capture_takes_no_trials():
    f = synth.random_fragment(6, 70, 130, seed=32)
    dB, deo, dev_ = to_dev(*f.arrays())
    ref = _outputs(dB, deo, dev_, None)
    rm.autotune_reset()
    opts = rm.make_opts(autotune=True)
    outs = dict(E=torch.zeros(2, dtype=torch.float64, device=dB.device), Gamma=torch.empty_like(dB),
                P_ij=torch.empty_like(ref.P_ij), P_ab=torch.empty_like(ref.P_ab), e_pair=torch.empty_like(ref.e_pair))
    ws = torch.empty(rm.workspace_size(6, 70, 130, opts=opts), dtype=torch.uint8, device=dB.device)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rm.fragment_into(dB, deo, dev_, outs["E"], outs["Gamma"], outs["P_ij"], outs["P_ab"], outs["e_pair"],
                         workspace=ws, opts=opts)
    rep = rm.autotune_report()
    assert rep and all(sum(e["timed"]) == 0 and e["best"] == -1 for e in rep)
    for rep_i in range(3):
        g.replay()
        torch.cuda.synchronize()
        for name in ("E", "Gamma", "P_ij", "P_ab", "e_pair"):
            assert torch.equal(outs[name], getattr(ref, name)), (rep_i, name)
    rm.autotune_reset()
