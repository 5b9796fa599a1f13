"""Batched fragments (grouped persistent launches, solo fragments, waves,
graph capture) against the CPU oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import rimp2_oracle as O
import paper_2410_21888_amd as rm
from gpu_util import to_dev, rel_fro, energy_error, say, assert_elementwise

pytestmark = pytest.mark.gpu


def make_frags(sizes, seed=1003, outputs=("Gamma", "P", "e_pair")):
    frags, refs = [], []
    for n, (nocc, nvir, naux) in enumerate(sizes):
        f = synth.Fragment(nocc, nvir, naux, seed=seed, frag=n)
        B, eo, ev = f.arrays()
        refs.append(O.fragment(B, eo, ev, gamma="Gamma" in outputs, density="P" in outputs))
        dB, deo, dev_ = to_dev(B, eo, ev)
        kw = dict(dtype=torch.float64, device=dB.device)
        d = dict(B=dB, eps_occ=deo, eps_vir=dev_, E=torch.zeros(2, **kw))
        if "Gamma" in outputs:
            d["Gamma"] = torch.empty_like(dB)
        if "P" in outputs:
            d["P_ij"] = torch.empty((nocc, nocc), **kw)
            d["P_ab"] = torch.empty((nvir, nvir), **kw)
        if "e_pair" in outputs:
            d["e_pair"] = torch.empty((nocc, nocc), **kw)
        frags.append(d)
    return frags, refs


def check(frags, refs, rtol=1e-12, atol=1e-12):
    """E within 1e-12 relative; Gamma, P_ij, P_ab and e_pair element by
    element, |d| <= rtol |ref| + atol max|ref row| (FP64: only the summation
    order of the GEMMs differs), and by relative Frobenius norm <= 1e-8."""
    for d, ref in zip(frags, refs):
        assert energy_error(d["E"], ref["E_hi"], ref["E_lo"]) <= 1e-12 * abs(ref["E_hi"]) + 1e-15
        for key in ("Gamma", "P_ij", "P_ab", "e_pair"):
            if key in d:
                got = d[key].cpu().numpy()
                assert rel_fro(got, ref[key]) <= 1e-8, key
                assert_elementwise(got, ref[key], rtol, atol, key)


MBE_LIKE = [(5, 25, 90), (12, 60, 216), (7, 35, 126), (3, 15, 54), (9, 45, 162), (6, 30, 108), (2, 10, 36)]


def test_grouped_waves_and_solo_match_oracle():
    frags, refs = make_frags(MBE_LIKE)
    # a small wave budget: the largest fragments run alone, the rest in several waves
    opts = rm.make_opts(slab_budget_bytes=3 << 20)
    status = torch.full((len(frags),), 7, dtype=torch.int32, device="cuda:0")
    say("batch of %d fragments, small wave budget" % len(frags))
    rm.fragment_batch(frags, status=status, opts=opts)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0] * len(frags)
    check(frags, refs)


def test_batch_output_subsets():
    frags, refs = make_frags(MBE_LIKE[:4], outputs=("e_pair",))
    say("energy-only batch")
    rm.fragment_batch(frags)
    torch.cuda.synchronize()
    check(frags, refs)


def test_batch_gap_status_per_fragment():
    frags, refs = make_frags(MBE_LIKE[:3])
    bad = frags[1]
    ev = bad["eps_vir"].clone()
    ev[0] = bad["eps_occ"].max() - 1e-3
    bad["eps_vir"] = ev
    status = torch.full((3,), 7, dtype=torch.int32, device="cuda:0")
    rm.fragment_batch(frags, status=status)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0, rm.RIMP2_EGAP, 0]
    check([frags[0], frags[2]], [refs[0], refs[2]])


def test_batch_graph_capture_replays():
    frags, refs = make_frags(MBE_LIKE[:5])
    b = rm.Batch(frags)
    ws = torch.empty(b.workspace_bytes, dtype=torch.uint8, device="cuda:0")
    status = torch.zeros(len(frags), dtype=torch.int32, device="cuda:0")
    b.run(ws, status)
    torch.cuda.synchronize()
    check(frags, refs)
    eager = [{k: v.clone() for k, v in d.items() if k not in ("B", "eps_occ", "eps_vir")} for d in frags]
    # capture (warm-up on the side stream first, as torch recommends)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run(ws, status)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run(ws, status)
    for rep in range(3):
        for d in frags:   # scribble over the outputs with eager work between replays
            for k, v in d.items():
                if k not in ("B", "eps_occ", "eps_vir"):
                    v.fill_(float("nan") if v.dtype == torch.float64 else 0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say("graph replay %d" % rep)
        for d, e in zip(frags, eager):
            for k, v in e.items():
                assert torch.equal(d[k], v), (rep, k)
    b.close()


def test_batch_autotune_bitwise_and_decides():
    frags, refs = make_frags(MBE_LIKE)
    outs = ("E", "Gamma", "P_ij", "P_ab", "e_pair")
    b0 = rm.Batch(frags)
    ws = torch.empty(b0.workspace_bytes, dtype=torch.uint8, device="cuda:0")
    b0.run(ws)
    torch.cuda.synchronize()
    check(frags, refs)
    ref = [{k: d[k].clone() for k in outs} for d in frags]
    b0.close()
    rm.autotune_reset()
    b = rm.Batch(frags, opts=rm.make_opts(autotune=True))
    assert b.workspace_bytes <= ws.numel()
    for call in range(6):
        say("autotuned batch run %d" % call)
        for d in frags:
            for k in outs:
                d[k].fill_(float("nan"))
        b.run(ws)
        torch.cuda.synchronize()
        for d, r in zip(frags, ref):
            for k in outs:
                assert torch.equal(d[k], r[k]), (call, k)
    rep = [e for e in rm.autotune_report() if e["vec"] == 2]
    assert {e["role"] for e in rep} == {"ints_gemm", "gamma_gemm", "pab_gemm", "pij_gemm"}
    for e in rep:
        say("grouped %s: tiles %s timed %s ms %s -> %s" % (e["role"], e["tiles"], e["timed"], e["min_ms"], e["best"]))
        assert e["best"] >= 0 and e["timed"] == [2, 2], e
    b.close()
    rm.autotune_reset()


def check_split(frags, refs):
    """Split-precision bar: |dE| <= 1 uEh; every element of Gamma, P_ij, P_ab
    and e_pair within 1e-8 |ref| + 1e-8 max|ref row|, and relative Frobenius
    error <= 1e-8."""
    for d, ref in zip(frags, refs):
        assert energy_error(d["E"], ref["E_hi"], ref["E_lo"]) <= 1e-6
        for key in ("Gamma", "P_ij", "P_ab", "e_pair"):
            got = d[key].cpu().numpy()
            assert rel_fro(got, ref[key]) <= 1e-8, key
            assert_elementwise(got, ref[key], 1e-8, 1e-8, key)


def run_split_batch(frags, **kw):
    status = torch.full((len(frags),), 7, dtype=torch.int32, device="cuda:0")
    rm.fragment_batch(frags, status=status, opts=rm.make_opts(precision=rm.SPLIT_INT8, **kw))
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0] * len(frags)


def test_batch_split_precision_matches_oracle():
    """One wave: grouped split products of every fragment."""
    frags, refs = make_frags(MBE_LIKE)
    say("split-precision batch of %d fragments" % len(frags))
    run_split_batch(frags)
    check_split(frags, refs)


def test_batch_split_waves_and_solo_match_oracle():
    """A small wave budget: the largest fragments run alone (their own split
    plan), the rest in several waves of grouped split products."""
    frags, refs = make_frags(MBE_LIKE)
    say("split-precision batch of %d fragments, small wave budget" % len(frags))
    run_split_batch(frags, slab_budget_bytes=3 << 20)
    check_split(frags, refs)


def test_batch_split_windows_match_oracle():
    """Reductions longer than one window in a wave: the Gamma product of the
    first fragment (nocc * nvir = 6000) and the (ia|jb) product of the second
    (naux = 6000) run in three windows of 2816; the other fragments have one,
    and skip their items in the later launches."""
    frags, refs = make_frags([(3, 2000, 24), (2, 8, 6000), (5, 25, 90), (2, 10, 36)])
    say("split-precision batch with windowed products")
    run_split_batch(frags)
    check_split(frags, refs)


def test_batch_split_gap_status_per_fragment():
    """A gap violation in one fragment of a grouped split wave: its status is
    RIMP2_EGAP, and the digit splits and split products of the others run."""
    frags, refs = make_frags(MBE_LIKE[:3])
    bad = frags[1]
    ev = bad["eps_vir"].clone()
    ev[0] = bad["eps_occ"].max() - 1e-3
    bad["eps_vir"] = ev
    status = torch.full((3,), 7, dtype=torch.int32, device="cuda:0")
    rm.fragment_batch(frags, status=status, opts=rm.make_opts(precision=rm.SPLIT_INT8))
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0, rm.RIMP2_EGAP, 0]
    check_split([frags[0], frags[2]], [refs[0], refs[2]])


def test_batch_split_graph_capture_replays():
    frags, refs = make_frags(MBE_LIKE[:5])
    b = rm.Batch(frags, opts=rm.make_opts(precision=rm.SPLIT_INT8))
    ws = torch.empty(b.workspace_bytes, dtype=torch.uint8, device="cuda:0")
    status = torch.zeros(len(frags), dtype=torch.int32, device="cuda:0")
    b.run(ws, status)
    torch.cuda.synchronize()
    check_split(frags, refs)
    eager = [{k: v.clone() for k, v in d.items() if k not in ("B", "eps_occ", "eps_vir")} for d in frags]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run(ws, status)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run(ws, status)
    for rep in range(3):
        for d in frags:
            for k, v in d.items():
                if k not in ("B", "eps_occ", "eps_vir"):
                    v.fill_(float("nan") if v.dtype == torch.float64 else 0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say("split graph replay %d" % rep)
        for d, e in zip(frags, eager):
            for k, v in e.items():
                assert torch.equal(d[k], v), (rep, k)
    b.close()
