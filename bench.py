"""Benchmark of the RI-MP2 fragment kernel on one MI355X.

A step is one pass of the whole path -- (ia|jb) slabs, amplitudes and pair
energies, E, Gamma, P_ab and P_ij -- over the large synthetic fragment
(nocc=200, nvir=1800, naux=6000, B = 0.3 N(0,1) exp(-P/1200), seed 1001), with
every input already resident in HBM.  Prints one JSON line.

  value      algorithmic FP64 TFLOP/s of the whole step: (ia|jb) over unordered
             pairs nocc(nocc+1) nvir^2 naux, Gamma 2 nocc^2 nvir^2 naux,
             P_ab 2 nocc^2 nvir^3, P_ij 2 nocc^3 nvir^2
  roofline   the dominant kernel's algorithmic rate from HIP events recorded
             around each of its launches on its stream, against the FP64
             MFMA peak (78.6 TFLOP/s)
  cpu_baseline  the CPU oracle on one occupied slab (k = 0) of the same
             workload, i.e. 1/nocc of the job, timed on this host's cores
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
METRIC = "RI-MP2 E+Γ TFLOP/s & %peak; split-prec/batched vs FP64 speedup at |ΔE|≤1µEh"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2410_21888_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode() + f.read())
    return h.hexdigest()[:16]


def measured_traffic(role: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 PMC runs, if they were
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(workload, {}).get(role)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(B, eo, ev, nocc, alg_total, sample_slabs):
    from oracle import rimp2_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = sum(p.get("num_threads", 0) for p in threadpool_info() if p.get("user_api") == "blas") or os.cpu_count()
    except Exception:
        cores = os.cpu_count()
    t0 = time.perf_counter()
    ref = O.fragment(B, eo, ev, slabs=sample_slabs)
    dt = time.perf_counter() - t0
    flops = alg_total * len(sample_slabs) / nocc
    return ref, {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
                 "sample": "occupied slab(s) %s of %d (all pairs (k,j), Gamma rows k, their P_ab/P_ij terms); "
                           "%.3g algorithmic FLOP in %.1f s" % (list(sample_slabs), nocc, flops, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["large", "mbe3"], default="large",
                    help="large: one fragment 200/1800/6000; mbe3: a batch of MBE3 fragments")
    ap.add_argument("--mbe3-stride", type=int, default=32,
                    help="mbe3: take every n-th of the 4096 recipe fragments")
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nocc", type=int, default=200)
    ap.add_argument("--nvir", type=int, default=1800)
    ap.add_argument("--naux", type=int, default=6000)
    ap.add_argument("--decay", type=float, default=1200.0)
    ap.add_argument("--seed", type=int, default=1001)
    ap.add_argument("--slab-group", type=int, default=0)
    ap.add_argument("--precision", choices=["fp64", "split"], default="fp64",
                    help="split: (ia|jb) and Gamma as INT8 digit products (Ozaki scheme)")
    ap.add_argument("--split-slices", type=int, default=0, help="digits per operand of (ia|jb) (0 = 7)")
    ap.add_argument("--split-slices-gamma", type=int, default=0, help="digits per operand of Gamma (0 = 5)")
    ap.add_argument("--compare-fp64", action="store_true",
                    help="after the timed steps run one FP64 step and report the differences")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stats", action="store_true", help="print per-kernel statistics to stderr")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, copy 1 GiB device-to-device (a plain copy of known size, for "
                         "scaling profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2410_21888_amd as rm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "mbe3":
        return bench_mbe3(args, torch, synth, rm, dev)
    f = synth.Fragment(args.nocc, args.nvir, args.naux, seed=args.seed, decay=args.decay)
    nocc, nvir, naux = f.nocc, f.nvir, f.naux
    large = (nocc, nvir, naux, args.seed, args.decay) == (200, 1800, 6000, 1001, 1200.0)
    workload = "large" if large else "custom"
    print("[bench] generating inputs nocc=%d nvir=%d naux=%d" % (nocc, nvir, naux), file=sys.stderr, flush=True)
    B_host = torch.empty((nocc, nvir, naux), dtype=torch.float64, pin_memory=True)
    f.B(out=B_host.numpy())
    eo, ev = f.eps()
    B = B_host.to(dev, non_blocking=True)
    deo = torch.from_numpy(eo).to(dev)
    dev_ = torch.from_numpy(ev).to(dev)
    f64 = dict(dtype=torch.float64, device=dev)
    E = torch.zeros(2, **f64)
    G = torch.empty((nocc, nvir, naux), **f64)
    Pij = torch.empty((nocc, nocc), **f64)
    Pab = torch.empty((nvir, nvir), **f64)
    ep = torch.empty((nocc, nocc), **f64)
    opts = rm.make_opts(slab_group=args.slab_group,
                        precision=rm.SPLIT_INT8 if args.precision == "split" else rm.FP64,
                        split_slices=args.split_slices, split_slices_gamma=args.split_slices_gamma)
    ws = torch.empty(rm.workspace_size(nocc, nvir, naux, True, True, opts), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step():
        rm.fragment_into(B, deo, dev_, E, G, Pij, Pab, ep, workspace=ws, opts=opts)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print("[bench] warmup step %d done" % w, file=sys.stderr, flush=True)
    if rm.read_status(ws) != rm.RIMP2_OK:
        raise SystemExit("device status not OK (orbital-energy gap)")

    rm.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = rm.timing_collect()
    rm.timing_enable(False)
    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    print("[bench] timed %d step(s) in %.3f s" % (args.steps, t1 - t0), file=sys.stderr, flush=True)

    fl = rm.flops(nocc, nvir, naux)
    dt = (t1 - t0) / args.steps
    value = fl["algorithmic"] / dt / 1e12
    dom = max(stats, key=lambda s: s["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    achieved = dom["alg_flops"] / (dom["total_ms"] / 1e3) / 1e12
    traffic = measured_traffic(dom["name"], workload)
    if args.stats:
        for s in sorted(stats, key=lambda s: -s["total_ms"]):
            print("[bench] %-14s launches=%5d total=%10.2f ms avg=%9.3f ms alg=%7.2f TF/s exec=%7.2f TF/s "
                  "alg_bytes/s=%8.1f GB/s" % (s["name"], s["launches"], s["total_ms"], s["total_ms"] / s["launches"],
                                              s["alg_flops"] / s["total_ms"] / 1e9,
                                              s["exec_flops"] / s["total_ms"] / 1e9,
                                              s["alg_bytes"] / s["total_ms"] / 1e6), file=sys.stderr)

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s fragment nocc=%d nvir=%d naux=%d" % (workload, nocc, nvir, naux),
                   "nocc": nocc, "nvir": nvir, "naux": naux, "seed": args.seed, "aux_decay": args.decay,
                   "outputs": "E, e_ij, Gamma, P_ij, P_ab", "flops_counted": "algorithmic E+Gamma+P_ab+P_ij",
                   "slab_group": args.slab_group or "auto"},
        "frac_fp64_peak": round(value / FP64_PEAK_TFLOPS, 4),
        "tflops_executed": round(fl["executed"] / dt / 1e12, 4),
        "roofline": {"bound": "mfma", "kernel": dom["name"], "achieved": round(achieved, 4),
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                     "avg_launch_ms": round(avg_ms, 4), "launches": dom["launches"],
                     "alg_flops_per_launch": dom["alg_flops"] / dom["launches"],
                     "traffic": traffic},
        "E_hi": float(E[0]), "E_lo": float(E[1]),
    }
    if args.precision == "split":
        out["dtype"] = "int8 digit products (Ozaki), f64 elsewhere"
        out["config"]["precision"] = "split-int8 ints=%d gamma=%d digits" % (args.split_slices or 7,
                                                                             args.split_slices_gamma or 5)
        out["roofline"]["note"] = "FP64-equivalent rate of the split kernel against the FP64 peak"
    if args.compare_fp64:
        import math
        G_s, ep_s, Pij_s, Pab_s, E_s = G.clone(), ep.clone(), Pij.clone(), Pab.clone(), E.clone()
        del ws
        torch.cuda.empty_cache()
        o64 = rm.make_opts(slab_group=args.slab_group)
        ws64 = torch.empty(rm.workspace_size(nocc, nvir, naux, True, True, o64), dtype=torch.uint8, device=dev)
        t2 = time.perf_counter()
        rm.fragment_into(B, deo, dev_, E, G, Pij, Pab, ep, workspace=ws64, opts=o64)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        e64 = E.cpu().numpy()
        es = E_s.cpu().numpy()
        rel = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
        out["vs_fp64"] = {
            "abs_dE_Eh": abs(math.fsum([float(es[0]), float(es[1]), -float(e64[0]), -float(e64[1])])),
            "gamma_rel_fro": rel(G_s, G), "p_ij_rel_fro": rel(Pij_s, Pij), "p_ab_rel_fro": rel(Pab_s, Pab),
            "e_pair_rel_fro": rel(ep_s, ep), "fp64_step_s": t3 - t2,
            "speedup_vs_fp64": (t3 - t2) / dt,
        }
    if not args.no_cpu_baseline:
        B_np = B_host.numpy()
        ref, cb = cpu_baseline(B_np, eo, ev, nocc, fl["algorithmic"], [0])
        out["cpu_baseline"] = cb
        g_ep = ep[0].cpu().numpy()
        g_G0 = G[0].cpu().numpy()
        out["sampled_parity"] = {
            "e_pair_row0_max_rel": float(np.max(np.abs(g_ep - ref["e_pair"][0]) / np.abs(ref["e_pair"][0]))),
            "gamma_row0_rel_fro": float(np.linalg.norm(g_G0 - ref["Gamma"][0]) / np.linalg.norm(ref["Gamma"][0])),
        }
    print(json.dumps(out))


def bench_mbe3(args, torch, synth, rm, dev):
    """Batch of MBE3 fragments: every n-th of the 4096-fragment recipe (30% monomers,
    40% dimers, 30% trimers), B generated on the GPU.  Times the grouped batch, the
    same batch replayed from a captured graph, and one rimp2_fragment call per
    fragment; value = algorithmic TFLOP/s of the grouped batch."""
    sizes = synth.mbe3_sizes(4096)
    ids = list(range(0, 4096, args.mbe3_stride))
    frags, total_alg, kinds = [], 0.0, {1: 0, 2: 0, 3: 0}
    print("[bench] generating %d fragments on the GPU" % len(ids), file=sys.stderr, flush=True)
    f64 = dict(dtype=torch.float64, device=dev)
    for f in ids:
        kind, nocc = sizes[f]
        kinds[kind] += 1
        F = synth.mbe3_fragment(f, nocc)
        B = torch.empty((F.nocc, F.nvir, F.naux), **f64)
        F.B_device(B)
        eo, ev = F.eps()
        frags.append(dict(B=B, eps_occ=torch.from_numpy(eo).to(dev), eps_vir=torch.from_numpy(ev).to(dev),
                          E=torch.zeros(2, **f64), Gamma=torch.empty_like(B),
                          P_ij=torch.empty((F.nocc, F.nocc), **f64), P_ab=torch.empty((F.nvir, F.nvir), **f64),
                          e_pair=torch.empty((F.nocc, F.nocc), **f64)))
        total_alg += rm.flops(F.nocc, F.nvir, F.naux)["algorithmic"]
    batch = rm.Batch(frags)
    ws = torch.empty(batch.workspace_bytes, dtype=torch.uint8, device=dev)
    status = torch.zeros(len(frags), dtype=torch.int32, device=dev)

    def timed(fn, reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    for _ in range(args.warmup):
        batch.run(ws, status)
    torch.cuda.synchronize()
    if int(status.abs().sum()) != 0:
        raise SystemExit("device status not OK")
    E_batch = torch.stack([d["E"] for d in frags]).clone()
    rm.timing_enable(True)
    t_batch = timed(lambda: batch.run(ws, status), args.steps)
    stats = rm.timing_collect()
    rm.timing_enable(False)
    print("[bench] grouped batch %.3f s" % t_batch, file=sys.stderr, flush=True)
    # graph capture of the same batch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run(ws, status)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.run(ws, status)
    t_graph = timed(g.replay, args.steps)
    print("[bench] graph replay %.3f s" % t_graph, file=sys.stderr, flush=True)
    # one call per fragment (largest first), each with its own default plan
    order = sorted(range(len(frags)), key=lambda i: -frags[i]["B"].numel() * frags[i]["B"].shape[0])
    ws1 = torch.empty(max(rm.workspace_size(*frags[i]["B"].shape) for i in order), dtype=torch.uint8, device=dev)

    def loop():
        for i in order:
            d = frags[i]
            rm.fragment_into(d["B"], d["eps_occ"], d["eps_vir"], d["E"], d["Gamma"], d["P_ij"], d["P_ab"],
                             d["e_pair"], workspace=ws1)
    loop()
    t_loop = timed(loop, args.steps)
    print("[bench] per-fragment loop %.3f s" % t_loop, file=sys.stderr, flush=True)
    E_loop = torch.stack([d["E"] for d in frags])
    dE = float((E_loop - E_batch).abs().max())
    if args.stats:
        for st in sorted(stats, key=lambda x: -x["total_ms"]):
            print("[bench] %-14s launches=%5d total=%10.2f ms" % (st["name"], st["launches"], st["total_ms"]),
                  file=sys.stderr)
    gemm = [st for st in stats if st["name"].endswith("_gemm")]
    dom = max(gemm, key=lambda x: x["total_ms"])
    value = total_alg / t_batch / 1e12
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_batch * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "mbe3 batch: %d of the 4096 recipe fragments (every %d-th): %d monomers, %d dimers, "
                               "%d trimers" % (len(ids), args.mbe3_stride, kinds[1], kinds[2], kinds[3]),
                   "fragments": len(ids), "flops_counted": "algorithmic E+Gamma+P_ab+P_ij"},
        "frac_fp64_peak": round(value / FP64_PEAK_TFLOPS, 4),
        "graph_replay_tflops": round(total_alg / t_graph / 1e12, 4),
        "per_fragment_loop_tflops": round(total_alg / t_loop / 1e12, 4),
        "speedup_batch_vs_loop": round(t_loop / t_batch, 4),
        "speedup_graph_vs_loop": round(t_loop / t_graph, 4),
        "max_abs_dE_batch_vs_loop_Eh": dE,
        "roofline": {"bound": "mfma", "kernel": dom["name"] + " (grouped)", "achieved": None, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": None, "traffic": None,
                     "note": "grouped launches mix fragments; per-launch algorithmic FLOPs are not split by role"},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
