"""Benchmark of the RI-MP2 fragment kernel on one MI355X.

A step is one pass of the hot path over the large synthetic fragment
(nocc=200, nvir=1800, naux=6000, B = 0.3 N(0,1) exp(-P/1200), seed 1001), with
every input already resident in HBM (B is generated on the GPU).  By default
(--outputs eg) a step forms the metric's own outputs, E (with every e_ij) and
Gamma: (ia|jb) slabs over unordered pairs, amplitudes and pair energies, and
the Gamma GEMMs of the symmetric path.  --outputs all adds P_ab and P_ij (the
whole path, on ordered pairs).  Prints one JSON line.

  value      algorithmic FP64 TFLOP/s of the step: (ia|jb) over unordered
             pairs nocc(nocc+1) nvir^2 naux, Gamma 2 nocc^2 nvir^2 naux, and
             with --outputs all P_ab 2 nocc^2 nvir^3 and P_ij 2 nocc^3 nvir^2
  roofline   the dominant kernel's algorithmic rate from HIP events recorded
             around each of its launches on its stream, against the FP64
             MFMA peak (78.6 TFLOP/s)
  whole_path / e_gamma_only   the same fragment in the other --outputs form
  split_e_gamma  (FP64 E+Gamma line) the same E+Gamma step with split-precision
             INT8 products, its speedup over the FP64 step and its differences
             from the FP64 result
  digit_sweep  (--digit-sweep) the split E+Gamma step once per digit count,
             each with its speedup and its differences from the FP64 result
  cpu_baseline  the CPU oracle on one occupied slab (k = 0) of the same
             workload, i.e. 1/nocc of the job, timed on this host's cores
             (--workload mbe3: three whole fragments of the batch; --workload
             screen: six pair energies); its outputs are the references of
             the line's sampled parity checks

A step of the large fragment takes tens of seconds, so the run keeps to a
wall-clock budget (--budget-s, from process start): the first step is always
a warmup step, and the timed steps are cut to what fits after it, with room
kept for the sub-record and the CPU baseline.  ``steps`` and ``warmup`` in the
line are the counts that ran; ``requested`` holds the ones asked for.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

T_START = time.perf_counter()

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
INT8_PEAK_TOPS = 5000.0      # dense INT8 MFMA, 5.0 POP/s
METRIC = "RI-MP2 E+Γ TFLOP/s & %peak; split-prec/batched vs FP64 speedup at |ΔE|≤1µEh"


def kernel_source_hash() -> str:
    from paper_2410_21888_amd.profsum import kernel_source_hash as h
    return h()


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


def blas_cores() -> int:
    try:
        from threadpoolctl import threadpool_info
        return int(sum(p.get("num_threads", 0) for p in threadpool_info() if p.get("user_api") == "blas")
                   or os.cpu_count())
    except Exception:
        return int(os.cpu_count())


def cpu_baseline(B, eo, ev, nocc, alg_total, sample_slabs, density=True):
    """The CPU oracle on some occupied slabs of one fragment: its outputs (the
    references of the sampled parity checks) and the baseline record."""
    from oracle import rimp2_oracle as O
    cores = blas_cores()
    t0 = time.perf_counter()
    ref = O.fragment(B, eo, ev, density=density, slabs=sample_slabs)
    dt = time.perf_counter() - t0
    flops = alg_total * len(sample_slabs) / nocc
    return ref, {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
                 "sample": "occupied slab(s) %s of %d (all pairs (k,j), Gamma rows k%s); %.3g algorithmic FLOP "
                           "(the slabs' share of the job's) in %.1f s"
                           % (list(sample_slabs), nocc, ", their P_ab/P_ij terms" if density else "", flops, dt)}


def cpu_baseline_fragments(arrays, alg_flops):
    """The CPU oracle on whole fragments (arrays: (B, eps_occ, eps_vir) per
    fragment, alg_flops: each one's algorithmic FLOPs): the references and the
    baseline record."""
    from oracle import rimp2_oracle as O
    t0 = time.perf_counter()
    refs = [O.fragment(B, eo, ev) for B, eo, ev in arrays]
    dt = time.perf_counter() - t0
    flops = float(sum(alg_flops))
    return refs, {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": blas_cores(), "kind": "oracle",
                  "sample": "%d whole fragments (nocc %s; E, e_ij, Gamma, P_ij, P_ab); %.3g algorithmic FLOP in %.3g s"
                            % (len(arrays), [int(a[0].shape[0]) for a in arrays], flops, dt)}


def cpu_baseline_pairs(B, eo, ev, pairs):
    """The CPU oracle's pair energies e_ij for some occupied pairs of one
    fragment (each pair's (ia|jb) block: 2 nvir^2 naux FLOP, its share of the
    symmetric count): the references and the baseline record."""
    from oracle import rimp2_oracle as O
    nvir, naux = B.shape[1], B.shape[2]
    t0 = time.perf_counter()
    refs = [float(O.pair_energy(B, eo, ev, i, j)) for i, j in pairs]
    dt = time.perf_counter() - t0
    flops = 2.0 * nvir * nvir * naux * len(pairs)
    return refs, {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": blas_cores(), "kind": "oracle",
                  "sample": "pair energies of %d occupied pairs (their share of the energy-only count); %.3g "
                            "algorithmic FLOP in %.3g s" % (len(pairs), flops, dt)}


def plan_steps(req_steps: int, req_warmup: int, budget_s: float, elapsed_s: float, step_s: float,
               reserve_s: float, margin: float = 1.05) -> tuple[int, int]:
    """Warmup and timed step counts that fit the wall-clock budget.

    Called after the first warmup step has run (it took ``step_s`` and the
    process has used ``elapsed_s`` so far); ``reserve_s`` is the time kept
    for the work after the timed steps.  Timed steps come first: at least
    one, at most ``req_steps``.  Further warmup steps (beyond the one already
    run) are added only where they fit as well.  Returns (warmup, steps),
    the warmup count including the step already run."""
    room = budget_s - elapsed_s - reserve_s
    fit = int(room // (step_s * margin)) if step_s > 0 else req_steps
    steps = max(1, min(req_steps, fit))
    extra = max(0, min(req_warmup - 1, fit - steps))
    return 1 + extra, steps


class Watchdog:
    """Prints the main record and ends the process if the hard deadline
    passes while optional extras are still running; without a record it ends
    the process with status 3.  ``emit`` prints the record exactly once."""

    def __init__(self, t_start: float, deadline_s: float):
        import threading
        self.rec = None
        self._lock = threading.Lock()
        self._done = False
        self._timer = threading.Timer(max(1.0, deadline_s - (time.perf_counter() - t_start)), self._fire)
        self._timer.daemon = True
        self._timer.start()

    def emit(self, rec: dict) -> bool:
        with self._lock:
            if self._done:
                return False
            self._done = True
        self._timer.cancel()
        sys.stdout.write(json.dumps(rec) + "\n")
        sys.stdout.flush()
        return True

    def _fire(self):
        if self.rec is not None:
            rec = dict(self.rec)
            rec["truncated"] = "hard deadline reached: the extras after the timed steps are missing"
            if self.emit(rec):
                os._exit(0)
            return
        sys.stderr.write("[bench] hard deadline reached before the timed steps finished\n")
        sys.stderr.flush()
        os._exit(3)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["large", "mbe3", "screen"], default="large",
                    help="large: one fragment 200/1800/6000; mbe3: a batch of MBE3 fragments; "
                         "screen: learned pair screening on spatially decaying systems")
    ap.add_argument("--screen-train", type=int, default=200, help="screen: training systems (seeds 4000..)")
    ap.add_argument("--screen-pairs", type=int, default=128, help="screen: sampled pairs per training system")
    ap.add_argument("--screen-size", type=str, default="400,2400,7200", help="screen: nocc,nvir,naux")
    ap.add_argument("--screen-save", type=str, default="",
                    help="screen: write the trained network (parameters and metadata, .npz) to this path")
    ap.add_argument("--mbe3-stride", type=int, default=32,
                    help="mbe3: take every n-th of the 4096 recipe fragments")
    ap.add_argument("--mbe3-kinds", type=str, default="1,2,3",
                    help="mbe3: polymer orders to keep (1 monomers, 2 dimers, 3 trimers)")
    ap.add_argument("--mbe3-batch-only", action="store_true",
                    help="mbe3: time the grouped batch only (no graph replay, per-fragment loop or autotuning)")
    ap.add_argument("--mbe3-chunk-gb", type=float, default=0.0,
                    help="mbe3: process the fragments in chunks of at most this many GB of B and Gamma, each "
                         "generated on the GPU before it runs (for sets that do not fit in HBM); times the "
                         "batches only")
    ap.add_argument("--steps", type=int, default=3, help="timed steps requested (large: capped by --budget-s)")
    ap.add_argument("--warmup", type=int, default=1,
                    help="warmup steps requested (large: at least one runs, unless 0 is asked for, as profiler runs "
                         "do: then the first step is timed, one step only)")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="large: wall-clock budget of the whole run from process start; the timed step count "
                         "is cut to what fits after the first warmup step")
    ap.add_argument("--deadline-s", type=float, default=0.0,
                    help="large: hard deadline from process start (0 = budget + 120 s); past it the main record "
                         "is printed without the extras and the process ends")
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
    ap.add_argument("--outputs", choices=["eg", "all"], default=None,
                    help="large: outputs of the timed steps: eg = E, e_ij and Gamma (the metric's pair, on the "
                         "symmetric path; the default), all = also P_ij and P_ab (the whole path, ordered pairs)")
    ap.add_argument("--no-split-sub", action="store_true",
                    help="large, FP64, E+Gamma: skip the split-precision E+Gamma step after the timed steps")
    ap.add_argument("--digit-sweep", action="store_true",
                    help="large, FP64, E+Gamma: after the timed steps run the split-precision E+Gamma step once per "
                         "digit count ((ia|jb) 3..7 digits with Gamma at 5, Gamma 3..7 with (ia|jb) at 7) and "
                         "report each one's time and differences from the FP64 result (digit_sweep)")
    ap.add_argument("--no-sub", "--no-e-gamma", dest="no_sub", action="store_true",
                    help="large: skip the sub-record (the same fragment in the other --outputs form)")
    ap.add_argument("--autotune", action="store_true",
                    help="large: in-situ tile autotuning (the warmup steps take the trials)")
    ap.add_argument("--stats", action="store_true", help="print per-kernel statistics to stderr")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, copy 1 GiB device-to-device (a plain copy of known size, for "
                         "scaling profiler byte counters)")
    args = ap.parse_args()
    if args.outputs is None:
        args.outputs = "eg"
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2410_21888_amd as rm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "mbe3" and args.mbe3_chunk_gb > 0:
        return bench_mbe3_chunked(args, torch, synth, rm, dev)
    if args.workload == "mbe3":
        return bench_mbe3(args, torch, synth, rm, dev)
    if args.workload == "screen":
        return bench_screen(args, torch, synth, rm, dev)
    return bench_large(args, torch, synth, rm, dev)


def log(msg: str):
    print("[bench %6.1fs] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)


def bench_large(args, torch, synth, rm, dev):
    """One fragment; see the module docstring."""
    wd = Watchdog(T_START, args.deadline_s or args.budget_s + 120.0)
    f = synth.Fragment(args.nocc, args.nvir, args.naux, seed=args.seed, decay=args.decay)
    nocc, nvir, naux = f.nocc, f.nvir, f.naux
    large = (nocc, nvir, naux, args.seed, args.decay) == (200, 1800, 6000, 1001, 1200.0)
    workload = "large" if large else "custom"
    eg_main = args.outputs == "eg"
    log("generating inputs on the GPU: nocc=%d nvir=%d naux=%d" % (nocc, nvir, naux))
    f64 = dict(dtype=torch.float64, device=dev)
    B = torch.empty((nocc, nvir, naux), **f64)
    f.B_device(B)
    eo, ev = f.eps()
    deo = torch.from_numpy(eo).to(dev)
    dev_ = torch.from_numpy(ev).to(dev)
    E = torch.zeros(2, **f64)
    G = torch.empty((nocc, nvir, naux), **f64)
    Pij = torch.empty((nocc, nocc), **f64)
    Pab = torch.empty((nvir, nvir), **f64)
    ep = torch.empty((nocc, nocc), **f64)
    opts = rm.make_opts(slab_group=args.slab_group,
                        precision=rm.SPLIT_INT8 if args.precision == "split" else rm.FP64,
                        split_slices=args.split_slices, split_slices_gamma=args.split_slices_gamma,
                        autotune=args.autotune)
    # the main record's outputs and the sub-record's (the other form), unless
    # --no-sub; the FP64 E+Gamma line also times the split-precision E+Gamma step
    need_full = not eg_main or not args.no_sub
    need_eg = eg_main or not args.no_sub
    split_sub = eg_main and args.precision == "fp64" and not args.no_split_sub
    opts_split = rm.make_opts(slab_group=args.slab_group, precision=rm.SPLIT_INT8) if split_sub else None
    sweep = eg_main and args.precision == "fp64" and args.digit_sweep
    if args.digit_sweep and not sweep:
        log("--digit-sweep runs with the FP64 E+Gamma line only (--precision fp64 --outputs eg): not run")
    sweep_pts = ([(sv, 5) for sv in range(3, 8)] + [(7, sg) for sg in (3, 4, 6, 7)]) if sweep else []
    sweep_opts = [rm.make_opts(slab_group=args.slab_group, precision=rm.SPLIT_INT8, split_slices=sv,
                               split_slices_gamma=sg) for sv, sg in sweep_pts]
    ws = torch.empty(max([rm.workspace_size(nocc, nvir, naux, True, True, opts) if need_full else 0,
                          rm.workspace_size(nocc, nvir, naux, True, False, opts) if need_eg else 0,
                          rm.workspace_size(nocc, nvir, naux, True, False, opts_split) if split_sub else 0] +
                         [rm.workspace_size(nocc, nvir, naux, True, False, o) for o in sweep_opts]),
                     dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step_full():
        rm.fragment_into(B, deo, dev_, E, G, Pij, Pab, ep, workspace=ws, opts=opts)

    def step_eg():
        rm.fragment_into(B, deo, dev_, E, G, None, None, ep, workspace=ws, opts=opts)

    step, step_sub = (step_eg, step_full) if eg_main else (step_full, step_eg)
    fl = rm.flops(nocc, nvir, naux, gamma=True, density=not eg_main)
    fl_sub = rm.flops(nocc, nvir, naux, gamma=True, density=eg_main)

    # the first step is a warmup step (the paper discards its first time
    # step), unless --warmup 0 asks for a single timed step (profiler runs)
    cold = args.warmup == 0
    step_s = 0.0
    if not cold:
        t0 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        step_s = time.perf_counter() - t0
        log("warmup step 0: %.2f s" % step_s)
        if rm.read_status(ws) != rm.RIMP2_OK:
            raise SystemExit("device status not OK (orbital-energy gap)")
    # work kept for after the timed steps: the sub-record (up to two steps:
    # the whole path takes about 1.45 times an E+Gamma step), the CPU baseline
    # and the copies
    sub_s = step_s * (1.45 if eg_main else 0.75)
    cpu_est = 0.0 if args.no_cpu_baseline else 20.0 + 3.0e-12 * fl["algorithmic"] / nocc
    reserve = (0.0 if args.no_sub else 2.0 * sub_s) + cpu_est + 15.0
    if split_sub:   # a split E+Gamma step takes about 0.66 of the FP64 one
        reserve += 2.0 * 0.7 * step_s + 10.0
    if args.compare_fp64:
        reserve += 1.2 * step_s
    if sweep:       # about 0.5-0.9 of an FP64 E+Gamma step per point, plus a warm call
        reserve += 0.8 * step_s * (len(sweep_pts) + 1)
    if cold:
        warmup, steps = 0, 1
    else:
        warmup, steps = plan_steps(args.steps, args.warmup, args.budget_s, time.perf_counter() - T_START, step_s,
                                   reserve)
    log("plan: %d timed step(s), %d warmup step(s) (requested %d and %d, budget %.0f s, reserve %.0f s)"
        % (steps, warmup, args.steps, args.warmup, args.budget_s, reserve))
    for w in range(1, warmup):
        step()
        torch.cuda.synchronize()
        log("warmup step %d done" % w)

    rm.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = rm.timing_collect()
    rm.timing_enable(False)
    log("timed %d step(s) in %.3f s" % (steps, t1 - t0))
    if cold:
        step_s = t1 - t0
        sub_s = step_s * (1.45 if eg_main else 0.75)
        if rm.read_status(ws) != rm.RIMP2_OK:
            raise SystemExit("device status not OK (orbital-energy gap)")
    E_main = E.cpu().numpy().copy()
    ep0_main = ep[0].cpu().numpy().copy()
    G0_main = G[0].cpu().numpy().copy()
    if args.calib_copy:
        src = torch.ones(1 << 27, **f64)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    dt = (t1 - t0) / steps
    value = fl["algorithmic"] / dt / 1e12
    dom = max(stats, key=lambda s: s["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    achieved = dom["alg_flops"] / (dom["total_ms"] / 1e3) / 1e12
    executed = dom["exec_flops"] / (dom["total_ms"] / 1e3) / 1e12
    traffic = measured_traffic(dom["name"], workload + ("_eg" if eg_main else ""))
    if args.stats:
        print_stats(stats)
    outputs_main = "E, e_ij, Gamma" if eg_main else "E, e_ij, Gamma, P_ij, P_ab"
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s fragment nocc=%d nvir=%d naux=%d" % (workload, nocc, nvir, naux),
                   "nocc": nocc, "nvir": nvir, "naux": naux, "seed": args.seed, "aux_decay": args.decay,
                   "outputs": outputs_main,
                   "flops_counted": "algorithmic E+Gamma" if eg_main else "algorithmic E+Gamma+P_ab+P_ij",
                   "path": ("symmetric: (ia|jb) over pairs j >= k only" if eg_main
                            else "ordered pairs (P needs every ordered pair's T and X)"),
                   "slab_group": args.slab_group or "auto", "autotune": bool(args.autotune),
                   "inputs": "B generated on the GPU (seeded counter-based normals), resident in HBM"},
        "requested": {"steps": args.steps, "warmup": args.warmup, "budget_s": args.budget_s},
        "frac_fp64_peak": round(value / FP64_PEAK_TFLOPS, 4),
        "tflops_executed": round(sum(s["exec_flops"] for s in stats) / (t1 - t0) / 1e12, 4),
        "roofline": {"bound": "mfma", "kernel": dom["name"], "achieved": round(achieved, 4),
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                     "avg_launch_ms": round(avg_ms, 4), "launches": dom["launches"],
                     "alg_flops_per_launch": dom["alg_flops"] / dom["launches"],
                     "traffic": traffic,
                     "executed_tflops": round(executed, 4), "frac_executed": round(executed / FP64_PEAK_TFLOPS, 4)},
        "kernels": {s["name"]: {"launches": s["launches"], "ms": round(s["total_ms"] / steps, 2)}
                    for s in sorted(stats, key=lambda s: -s["total_ms"])},
        "E_hi": float(E_main[0]), "E_lo": float(E_main[1]),
    }
    if dom["name"] == "ints_gemm" and not eg_main:
        out["roofline"]["note"] = ("the (ia|jb) GEMM computes ordered pairs (twice the symmetric algorithmic count) "
                                   "so that Gamma and P read complete slab rows; executed_tflops is its MFMA rate")
    if args.autotune:
        out["autotune"] = [dict(role=e["role"], M=e["M"], N=e["N"], K=e["K"], tile=e["tiles"][e["best"]]
                                if e["best"] >= 0 else None, min_ms=[round(t, 3) for t in e["min_ms"]])
                           for e in rm.autotune_report()]
    if args.precision == "split":
        out["dtype"] = "int8 digit products (Ozaki), f64 elsewhere"
        out["config"]["precision"] = "split-int8 ints=%d gamma=%d digits" % (args.split_slices or 7,
                                                                             args.split_slices_gamma or 5)
        # the split products run on INT8 MFMA: their roofline is the INT8 peak, on the
        # INT8 operations executed (S(S+1)/2 digit products per FP64-equivalent product)
        if dom["name"] in ("ints_oz8", "gamma_oz8", "gamma_t_oz8"):
            S = (args.split_slices or 7) if dom["name"] == "ints_oz8" else (args.split_slices_gamma or 5)
            ops = dom["exec_flops"] * S * (S + 1) / 2 / (dom["total_ms"] / 1e3) / 1e12
            out["roofline"].update({
                "achieved": round(ops, 2), "peak": INT8_PEAK_TOPS, "unit": "TOP/s",
                "frac": round(ops / INT8_PEAK_TOPS, 4), "digits": S,
                "fp64_equivalent_tflops": round(executed, 4),
                "note": "INT8 digit products executed per second against the dense INT8 MFMA peak; "
                        "fp64_equivalent_tflops is the same launch's FP64-equivalent rate"})
    wd.rec = out

    def left():
        return args.budget_s - (time.perf_counter() - T_START)

    if args.compare_fp64 and left() > 1.2 * step_s + cpu_est:
        G_s, ep_s, Pij_s, Pab_s, E_s = G.clone(), ep.clone(), Pij.clone(), Pab.clone(), E.clone()
        o64 = rm.make_opts(slab_group=args.slab_group)
        ws64 = torch.empty(rm.workspace_size(nocc, nvir, naux, True, not eg_main, o64), dtype=torch.uint8,
                           device=dev)
        t2 = time.perf_counter()
        rm.fragment_into(B, deo, dev_, E, G, None if eg_main else Pij, None if eg_main else Pab, ep,
                         workspace=ws64, opts=o64)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        del ws64
        e64 = E.cpu().numpy()
        es = E_s.cpu().numpy()
        rel = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
        out["vs_fp64"] = {
            "abs_dE_Eh": abs(math.fsum([float(es[0]), float(es[1]), -float(e64[0]), -float(e64[1])])),
            "gamma_rel_fro": rel(G_s, G), "e_pair_rel_fro": rel(ep_s, ep), "fp64_step_s": t3 - t2,
            "speedup_vs_fp64": (t3 - t2) / dt,
        }
        if not eg_main:
            out["vs_fp64"].update({"p_ij_rel_fro": rel(Pij_s, Pij), "p_ab_rel_fro": rel(Pab_s, Pab)})
        del G_s, ep_s, Pij_s, Pab_s, E_s
        log("FP64 comparison step: %.2f s" % (t3 - t2))

    # the split-precision E+Gamma step on the same inputs (warm, then timed),
    # against this run's FP64 E+Gamma result: the split-vs-FP64 speedup of the
    # metric's own outputs
    if split_sub and left() > 1.5 * step_s + cpu_est + (sub_s if not args.no_sub else 0.0):
        G64, ep64 = G.clone(), ep.clone()
        t_split = []
        for rep in range(2):
            rm.timing_enable(rep == 1)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            rm.fragment_into(B, deo, dev_, E, G, None, None, ep, workspace=ws, opts=opts_split)
            torch.cuda.synchronize()
            t_split.append(time.perf_counter() - t2)
            st_split = rm.timing_collect() if rep == 1 else None
            rm.timing_enable(False)
            if rep == 0 and left() < t_split[0] * 1.05 + cpu_est + (sub_s if not args.no_sub else 0.0):
                break
        ts = t_split[-1]
        E_s = E.cpu().numpy().copy()
        rel = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
        out["split_e_gamma"] = {
            "value": round(fl["algorithmic"] / ts / 1e12, 4), "unit": "TFLOP/s",
            "flops_counted": "algorithmic E+Gamma (FP64-equivalent)",
            "ms_per_step": round(ts * 1e3, 3), "steps": 1, "warmup": len(t_split) - 1,
            "digits": "ints=7 gamma=5", "dtype": "int8 digit products (Ozaki), f64 elsewhere",
            "speedup_vs_fp64": round(dt / ts, 4),
            "abs_dE_vs_fp64_Eh": abs(math.fsum([float(E_s[0]), float(E_s[1]), -float(E_main[0]), -float(E_main[1])])),
            "gamma_rel_fro_vs_fp64": rel(G, G64), "e_pair_rel_fro_vs_fp64": rel(ep, ep64)}
        if st_split:
            out["split_e_gamma"]["kernels"] = {x["name"]: {"launches": x["launches"], "ms": round(x["total_ms"], 2)}
                                               for x in sorted(st_split, key=lambda x: -x["total_ms"])}
        G.copy_(G64)
        ep.copy_(ep64)
        del G64, ep64
        log("split E+Gamma step: %.2f s (%.3fx the FP64 step)" % (ts, dt / ts))

    # digit-count sweep of the split E+Gamma step against this run's FP64
    # E+Gamma result (one warm call at the first point, then one timed call per
    # point; points that do not fit the budget are left out)
    if sweep:
        G64, ep64 = G.clone(), ep.clone()
        ep64_np = ep64.cpu().numpy()
        rel = lambda a, b: float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
        pts = []
        rm.fragment_into(B, deo, dev_, E, G, None, None, ep, workspace=ws, opts=sweep_opts[-1])
        torch.cuda.synchronize()
        for (sv, sg), o in zip(sweep_pts, sweep_opts):
            if left() < 1.1 * step_s + cpu_est:
                log("digit sweep: no time left for ints=%d gamma=%d" % (sv, sg))
                break
            t2 = time.perf_counter()
            rm.fragment_into(B, deo, dev_, E, G, None, None, ep, workspace=ws, opts=o)
            torch.cuda.synchronize()
            ts = time.perf_counter() - t2
            if rm.read_status(ws) != rm.RIMP2_OK:
                raise SystemExit("device status not OK in the digit sweep")
            E_s = E.cpu().numpy().copy()
            dE = abs(math.fsum([float(E_s[0]), float(E_s[1]), -float(E_main[0]), -float(E_main[1])]))
            ep_np = ep.cpu().numpy()
            pts.append({"ints_digits": sv, "gamma_digits": sg, "ms_per_step": round(ts * 1e3, 3),
                        "speedup_vs_fp64": round(dt / ts, 4), "abs_dE_vs_fp64_Eh": dE,
                        "gamma_rel_fro_vs_fp64": rel(G, G64), "e_pair_rel_fro_vs_fp64": rel(ep, ep64),
                        "e_pair_max_abs_vs_fp64_Eh": float(np.max(np.abs(ep_np - ep64_np))),
                        "within_tolerances": bool(dE <= 1e-6 and rel(G, G64) <= 1e-8)})
            log("digit sweep ints=%d gamma=%d: %.2f s (%.3fx), |dE| = %.3g Eh, Gamma %.3g"
                % (sv, sg, ts, dt / ts, dE, pts[-1]["gamma_rel_fro_vs_fp64"]))
        ok = [q for q in pts if q["within_tolerances"]]
        out["digit_sweep"] = {"points": pts, "tolerances": "|dE| <= 1e-6 Eh and Gamma relative Frobenius <= 1e-8 "
                                                           "against this run's FP64 E+Gamma step",
                              "fastest_within_tolerances": (max(ok, key=lambda q: q["speedup_vs_fp64"])
                                                            if ok else None)}
        G.copy_(G64)
        ep.copy_(ep64)
        del G64, ep64

    # the sub-record: the same fragment in the other form (the whole path when
    # the main record is E+Gamma, E+Gamma alone otherwise), timed the same way
    sub = None
    if not args.no_sub and left() > sub_s + cpu_est:
        sub_warm = 0
        if cold:
            rm.timing_enable(True)
        t2 = time.perf_counter()
        step_sub()
        torch.cuda.synchronize()
        sub_first = time.perf_counter() - t2
        st_first = rm.timing_collect() if cold else []
        if cold:
            rm.timing_enable(False)
        if not cold and left() > sub_first * 1.05 + cpu_est:
            sub_warm = 1
            rm.timing_enable(True)
            t2 = time.perf_counter()
            step_sub()
            torch.cuda.synchronize()
            sub_t = time.perf_counter() - t2
            st_sub = rm.timing_collect()
            rm.timing_enable(False)
        else:
            sub_t, st_sub = sub_first, st_first
        E_sub = E.cpu().numpy().copy()
        sub = {"value": round(fl_sub["algorithmic"] / sub_t / 1e12, 4), "unit": "TFLOP/s",
               "ms_per_step": round(sub_t * 1e3, 3), "steps": 1, "warmup": sub_warm,
               "frac_fp64_peak": round(fl_sub["algorithmic"] / sub_t / 1e12 / FP64_PEAK_TFLOPS, 4),
               "flops_counted": "algorithmic E+Gamma+P_ab+P_ij" if eg_main else "algorithmic E+Gamma",
               "outputs": "E, e_ij, Gamma, P_ij, P_ab" if eg_main else "E, e_ij, Gamma",
               "E_hi": float(E_sub[0]), "E_lo": float(E_sub[1]),
               "abs_dE_vs_main_Eh": abs(math.fsum([float(E_sub[0]), float(E_sub[1]), -float(E_main[0]),
                                                   -float(E_main[1])]))}
        if st_sub:
            sub["kernels"] = {s["name"]: {"launches": s["launches"], "ms": round(s["total_ms"], 2)}
                              for s in sorted(st_sub, key=lambda s: -s["total_ms"])}
        ep0_sub = ep[0].cpu().numpy().copy()
        G0_sub = G[0].cpu().numpy().copy()
        sub_key = "whole_path" if eg_main else "e_gamma_only"
        out[sub_key] = sub
        log("%s step: %.2f s (%.2f TFLOP/s)" % (sub_key, sub_t, sub["value"]))

    if not args.no_cpu_baseline and left() > cpu_est * 0.5:
        B_np = B.cpu().numpy()
        ref, cb = cpu_baseline(B_np, eo, ev, nocc, fl["algorithmic"], [0], density=not eg_main)
        out["cpu_baseline"] = cb

        def rows(ep0, G0):
            return {"e_pair_row0_max_rel": float(np.max(np.abs(ep0 - ref["e_pair"][0]) / np.abs(ref["e_pair"][0]))),
                    "gamma_row0_rel_fro": float(np.linalg.norm(G0 - ref["Gamma"][0]) /
                                                np.linalg.norm(ref["Gamma"][0])),
                    "gamma_row0_max_abs_over_max": float(np.max(np.abs(G0 - ref["Gamma"][0])) /
                                                         np.max(np.abs(ref["Gamma"][0])))}
        sp = rows(ep0_main, G0_main)
        if sub is not None:
            sp["whole_path" if eg_main else "e_gamma_only"] = rows(ep0_sub, G0_sub)
        out["sampled_parity"] = sp
        del B_np
        log("CPU baseline: %.3f TFLOP/s on %d cores" % (cb["value"], cb["cores"]))
    out["wall_s"] = round(time.perf_counter() - T_START, 1)
    wd.emit(out)


def print_stats(stats):
    for s in sorted(stats, key=lambda s: -s["total_ms"]):
        print("[bench] %-14s launches=%5d total=%10.2f ms avg=%9.3f ms alg=%7.2f TF/s exec=%7.2f TF/s "
              "alg_bytes/s=%8.1f GB/s" % (s["name"], s["launches"], s["total_ms"], s["total_ms"] / s["launches"],
                                          s["alg_flops"] / s["total_ms"] / 1e9,
                                          s["exec_flops"] / s["total_ms"] / 1e9,
                                          s["alg_bytes"] / s["total_ms"] / 1e6), file=sys.stderr)


def bench_mbe3(args, torch, synth, rm, dev):
    """Batch of MBE3 fragments: every n-th of the 4096-fragment recipe (30% monomers,
    40% dimers, 30% trimers), B generated on the GPU.  Times the grouped batch, the
    same batch replayed from a captured graph, and one rimp2_fragment call per
    fragment; value = algorithmic TFLOP/s of the grouped batch."""
    sizes = synth.mbe3_sizes(4096)
    keep = {int(k) for k in args.mbe3_kinds.split(",")}
    ids = [f for f in range(0, 4096, args.mbe3_stride) if sizes[f][0] in keep]
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
    # --mbe3-batch-only --precision split: the grouped split-precision batch alone
    split_only = args.mbe3_batch_only and args.precision == "split"
    batch = rm.Batch(frags, opts=rm.make_opts(precision=rm.SPLIT_INT8) if split_only else None)
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
    # sampled parity in the timed launch configuration: the smallest, a middle
    # and the largest fragment of at most 40 occupied orbitals, against the
    # CPU oracle on the device's own B (read back)
    sampled, cb = [], None
    if not args.no_cpu_baseline:
        cand = sorted((i for i in range(len(frags)) if frags[i]["B"].shape[0] <= 40),
                      key=lambda i: frags[i]["B"].shape[0])
        picks = sorted({cand[0], cand[len(cand) // 2], cand[-1]} if cand else set())
        arrays = [(frags[i]["B"].cpu().numpy(), frags[i]["eps_occ"].cpu().numpy(), frags[i]["eps_vir"].cpu().numpy())
                  for i in picks]
        refs = []
        if arrays:
            refs, cb = cpu_baseline_fragments(
                arrays, [rm.flops(*a[0].shape, gamma=True, density=True)["algorithmic"] for a in arrays])
        del arrays
        for i, ref in zip(picks, refs):
            d = frags[i]
            e = E_batch[i].cpu().numpy()
            g = d["Gamma"].cpu().numpy()
            sampled.append({"nocc": int(d["B"].shape[0]),
                            "abs_dE_Eh": abs(math.fsum([float(e[0]), float(e[1]), -ref["E_hi"], -ref["E_lo"]])),
                            "gamma_rel_fro": float(np.linalg.norm(g - ref["Gamma"]) / np.linalg.norm(ref["Gamma"])),
                            "p_ab_rel_fro": float(np.linalg.norm(d["P_ab"].cpu().numpy() - ref["P_ab"]) /
                                                  np.linalg.norm(ref["P_ab"]))})
    rm.timing_enable(True)
    t_batch = timed(lambda: batch.run(ws, status), args.steps)
    stats = rm.timing_collect()
    rm.timing_enable(False)
    print("[bench] grouped batch %.3f s" % t_batch, file=sys.stderr, flush=True)
    if args.mbe3_batch_only:   # the grouped batch alone (profiler runs)
        value = total_alg / t_batch / 1e12
        gemm = [st for st in stats if st["name"].endswith("_gemm")]
        print(json.dumps({
            "metric": METRIC, "value": round(value, 4), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(t_batch * 1e3, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "int8 digit products (Ozaki), f64 elsewhere" if split_only else "f64", "data": "synthetic",
            "config": {"workload": "mbe3 batch (grouped %sbatch only): %d of the 4096 recipe fragments (every %d-th, "
                                   "orders %s): %d monomers, %d dimers, %d trimers"
                                   % ("split-precision " if split_only else "", len(ids), args.mbe3_stride,
                                      args.mbe3_kinds, kinds[1], kinds[2], kinds[3]),
                       "fragments": len(ids), "flops_counted": "algorithmic E+Gamma+P_ab+P_ij"},
            "frac_fp64_peak": round(value / FP64_PEAK_TFLOPS, 4), "sampled_parity": sampled, "cpu_baseline": cb,
            "kernels": {st["name"]: {"launches": st["launches"], "ms": round(st["total_ms"] / args.steps, 2)}
                        for st in sorted(stats, key=lambda x: -x["total_ms"])},
            "roofline": {"bound": "mfma", "kernel": max(gemm, key=lambda x: x["total_ms"])["name"] + " (grouped)",
                         "achieved": None, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": None,
                         "traffic": None,
                         "note": "grouped launches mix fragments; per-launch algorithmic FLOPs are not split by role"}}))
        return
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
    n_ws1 = max(rm.workspace_size(*frags[i]["B"].shape) for i in order)
    ws1 = [torch.empty(n_ws1, dtype=torch.uint8, device=dev)]   # released while the split batch runs

    def loop(opts=None):
        for i in order:
            d = frags[i]
            rm.fragment_into(d["B"], d["eps_occ"], d["eps_vir"], d["E"], d["Gamma"], d["P_ij"], d["P_ab"],
                             d["e_pair"], workspace=ws1[0], opts=opts)
    loop()
    t_loop = timed(loop, args.steps)
    print("[bench] per-fragment loop %.3f s" % t_loop, file=sys.stderr, flush=True)
    E_loop = torch.stack([d["E"] for d in frags]).clone()
    dE = float((E_loop - E_batch).abs().max())
    split = None
    if args.precision == "split":   # grouped split products for (ia|jb) and Gamma
        ws1[0] = None
        torch.cuda.empty_cache()
        sb = rm.Batch(frags, opts=rm.make_opts(precision=rm.SPLIT_INT8))
        ws_s = torch.empty(sb.workspace_bytes, dtype=torch.uint8, device=dev)
        sb.run(ws_s, status)
        torch.cuda.synchronize()
        rm.timing_enable(True)
        t_split = timed(lambda: sb.run(ws_s, status), args.steps)
        st_split = rm.timing_collect()
        rm.timing_enable(False)
        E_s = torch.stack([d["E"] for d in frags])
        dE_s = max(abs(math.fsum([float(a[0]), float(a[1]), -float(b[0]), -float(b[1])]))
                   for a, b in zip(E_s.cpu().numpy(), E_batch.cpu().numpy()))
        sb.close()
        del ws_s
        torch.cuda.empty_cache()
        ws1[0] = torch.empty(n_ws1, dtype=torch.uint8, device=dev)
        split = {"split_batch_tflops": round(total_alg / t_split / 1e12, 4),
                 "speedup_split_vs_fp64_batch": round(t_batch / t_split, 4), "max_abs_dE_vs_fp64_Eh": dE_s,
                 "kernels": {x["name"]: {"launches": x["launches"], "ms": round(x["total_ms"] / args.steps, 2)}
                             for x in sorted(st_split, key=lambda x: -x["total_ms"])},
                 "fp64_kernels": {x["name"]: {"launches": x["launches"], "ms": round(x["total_ms"] / args.steps, 2)}
                                  for x in sorted(stats, key=lambda x: -x["total_ms"])}}
        print("[bench] split-precision batch %.3f s" % t_split, file=sys.stderr, flush=True)
    # in-situ tile autotuning: the first passes trial the candidates, later passes use the choices
    rm.autotune_reset()
    tb = rm.Batch(frags, opts=rm.make_opts(autotune=True))
    for _ in range(6):   # trial passes: two per candidate of every grouped launch
        tb.run(ws, status)
        torch.cuda.synchronize()
        if all(e["best"] >= 0 for e in rm.autotune_report() if e["vec"] == 2):
            break
    t_batch_tuned = timed(lambda: tb.run(ws, status), args.steps)
    E_bt = torch.stack([d["E"] for d in frags]).clone()
    batch_tuned_bitwise = bool(torch.equal(E_bt, E_batch))
    tb.close()
    print("[bench] grouped batch, autotuned: %.3f s" % t_batch_tuned, file=sys.stderr, flush=True)
    tuned = rm.make_opts(autotune=True)
    t_trial = timed(lambda: loop(tuned), 1)
    loop(tuned)
    torch.cuda.synchronize()
    t_tuned = timed(lambda: loop(tuned), args.steps)
    rep = rm.autotune_report()
    E_tuned = torch.stack([d["E"] for d in frags])
    tuned_bitwise = bool(torch.equal(E_tuned, E_loop))
    n_changed = sum(1 for e in rep if e["best"] > 0)
    decisions = {}
    for e in rep:
        if e["best"] >= 0:
            key = "%dx%d" % tuple(e["tiles"][e["best"]])
            d = decisions.setdefault(e["role"], {})
            d[key] = d.get(key, 0) + 1
        if args.stats:
            print("[tune] %-10s M=%6d N=%6d K=%9d kchunk=%9d best=%s ms=%s" % (
                e["role"], e["M"], e["N"], e["K"], e["kchunk"], e["tiles"][e["best"]] if e["best"] >= 0 else None,
                " ".join("%dx%d:%.3f" % (t[0], t[1], m) for t, m in zip(e["tiles"], e["min_ms"]))), file=sys.stderr)
    print("[bench] per-fragment loop, autotuned: trial pass %.3f s, tuned %.3f s; %d of %d shapes off the default"
          % (t_trial, t_tuned, n_changed, len(rep)), file=sys.stderr, flush=True)
    rm.autotune_reset()
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
        "config": {"workload": "mbe3 batch: %d of the 4096 recipe fragments (every %d-th, orders %s): %d monomers, "
                               "%d dimers, %d trimers" % (len(ids), args.mbe3_stride, args.mbe3_kinds, kinds[1],
                                                          kinds[2], kinds[3]),
                   "fragments": len(ids), "flops_counted": "algorithmic E+Gamma+P_ab+P_ij"},
        "frac_fp64_peak": round(value / FP64_PEAK_TFLOPS, 4),
        "graph_replay_tflops": round(total_alg / t_graph / 1e12, 4),
        "per_fragment_loop_tflops": round(total_alg / t_loop / 1e12, 4),
        "speedup_batch_vs_loop": round(t_loop / t_batch, 4),
        "speedup_graph_vs_loop": round(t_loop / t_graph, 4),
        "autotune": {"batch_tuned_tflops": round(total_alg / t_batch_tuned / 1e12, 4),
                     "speedup_tuned_vs_fixed_batch": round(t_batch / t_batch_tuned, 4),
                     "batch_E_bitwise_equal_to_fixed": batch_tuned_bitwise,
                     "loop_tuned_tflops": round(total_alg / t_tuned / 1e12, 4),
                     "loop_trial_pass_tflops": round(total_alg / t_trial / 1e12, 4),
                     "speedup_tuned_vs_fixed_loop": round(t_loop / t_tuned, 4),
                     "shapes": len(rep), "shapes_off_default": n_changed, "E_bitwise_equal_to_fixed": tuned_bitwise,
                     "chosen_tiles": decisions},
        "max_abs_dE_batch_vs_loop_Eh": dE,
        "sampled_parity": sampled,
        "cpu_baseline": cb,
        "split": split,
        "roofline": {"bound": "mfma", "kernel": dom["name"] + " (grouped)", "achieved": None, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": None, "traffic": None,
                     "note": "grouped launches mix fragments; per-launch algorithmic FLOPs are not split by role"},
    }
    print(json.dumps(out))


def bench_mbe3_chunked(args, torch, synth, rm, dev):
    """MBE3 fragments (every n-th of the 4096-fragment recipe, or all of them)
    in chunks that fit in HBM, largest fragments first: each chunk's B is
    generated on the GPU (not timed), then the chunk runs as one batch (timed,
    one run, no warm-up); value = algorithmic TFLOP/s of all the batches."""
    sizes = synth.mbe3_sizes(4096)
    keep = {int(k) for k in args.mbe3_kinds.split(",")}
    ids = [f for f in range(0, 4096, args.mbe3_stride) if sizes[f][0] in keep]
    dims = {f: (sizes[f][1], 5 * sizes[f][1], 3 * 6 * sizes[f][1]) for f in ids}
    ids.sort(key=lambda f: -(dims[f][0] ** 2 * dims[f][1] ** 2 * dims[f][2]))
    budget = args.mbe3_chunk_gb * 1e9
    chunks, cur, used = [], [], 0.0
    for f in ids:
        o, v, x = dims[f]
        b = 16.0 * o * v * x
        if cur and used + b > budget:
            chunks.append(cur)
            cur, used = [], 0.0
        cur.append(f)
        used += b
    if cur:
        chunks.append(cur)
    f64 = dict(dtype=torch.float64, device=dev)
    total_alg, t_total, kinds = 0.0, 0.0, {1: 0, 2: 0, 3: 0}
    E_all = []
    for c, chunk in enumerate(chunks):
        frags = []
        for f in chunk:
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
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.run(ws, status)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t_total += dt
        if int(status.abs().sum()) != 0:
            raise SystemExit("device status not OK in chunk %d" % c)
        E_all.append(torch.stack([d["E"] for d in frags]).cpu())
        batch.close()
        del frags, ws, batch, status
        torch.cuda.empty_cache()
        print("[bench] chunk %d/%d: %d fragments in %.2f s (total %.1f s)" % (c + 1, len(chunks), len(chunk), dt,
                                                                           t_total), file=sys.stderr, flush=True)
    value = total_alg / t_total / 1e12
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "TFLOP/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(t_total * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "mbe3: %d of the 4096 recipe fragments (every %d-th, orders %s; %d monomers, %d "
                               "dimers, %d trimers) in %d chunks of <= %.0f GB generated on the GPU"
                               % (len(ids), args.mbe3_stride, args.mbe3_kinds, kinds[1], kinds[2], kinds[3],
                                  len(chunks), args.mbe3_chunk_gb),
                   "fragments": len(ids), "flops_counted": "algorithmic E+Gamma+P_ab+P_ij",
                   "timed": "the batch runs only (input generation excluded)"},
        "frac_fp64_peak": round(value / FP64_PEAK_TFLOPS, 4),
        "E_total_hi": float(sum(float(e[0]) for E in E_all for e in E)),
        "roofline": {"bound": "mfma", "kernel": "grouped and solo GEMMs", "achieved": None, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": None, "traffic": None},
    }
    print(json.dumps(out))


def bench_screen(args, torch, synth, rm, dev):
    """Learned pair screening.  Training: for each system (seeds 4000..), the
    energy-only kernel runs on distance-stratified sampled pairs (all others
    skipped) and its e_ij become log10|e_ij| targets for the 4-64-64-1 network,
    trained with the library's kernels.  Evaluation (held-out seed 4200): an
    unscreened energy-only run judges the screens; value = algorithmic TFLOP/s
    of the full energy (nocc(nocc+1) nvir^2 naux) over the screened run's time,
    with the threshold chosen so the predicted skipped energy is <= 0.5 uEh."""
    import math
    from paper_2410_21888_amd import screen as SC
    nocc, nvir, naux = (int(v) for v in args.screen_size.split(","))
    f64 = dict(dtype=torch.float64, device=dev)
    B = torch.empty((nocc, nvir, naux), **f64)
    e_pair = torch.empty((nocc, nocc), **f64)
    E = torch.zeros(2, **f64)
    ws = torch.empty(rm.workspace_size(nocc, nvir, naux, False, False), dtype=torch.uint8, device=dev)

    def load(seed):
        F = synth.screen_system(seed, nocc, nvir, naux)
        F.B_device(B)
        eo, ev = F.eps()
        r, _ = F.positions()
        return (torch.from_numpy(eo).to(dev), torch.from_numpy(ev).to(dev), torch.from_numpy(r).to(dev), r)

    def run(eo, ev, skip=None):
        opts = rm.make_opts(pair_skip=skip)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rm.fragment_into(B, eo, ev, E, e_pair=e_pair, workspace=ws, opts=opts)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    iu = np.triu_indices(nocc, 1)
    xs, ts = [], []
    t_data = time.perf_counter()
    for n in range(args.screen_train):
        seed = 4000 + n
        eo, ev, r_dev, r = load(seed)
        feat, _ = SC.pair_features(B, eo, ev, r_dev, bound=False)
        # sample pairs i < j uniformly over distance bins
        d = np.sqrt(((r[iu[0]] - r[iu[1]]) ** 2).sum(-1))
        rng = np.random.default_rng(seed)
        bins = np.minimum((d / d.max() * 16).astype(int), 15)
        w = 1.0 / np.bincount(bins, minlength=16)[bins]
        pick = rng.choice(len(d), size=min(args.screen_pairs, len(d)), replace=False, p=w / w.sum())
        pi, pj = iu[0][pick], iu[1][pick]
        mask = np.ones((nocc, nocc), dtype=np.uint8)
        mask[pi, pj] = 0
        mask[pj, pi] = 0
        run(eo, ev, torch.from_numpy(mask).to(dev))
        flat = torch.from_numpy(pi * nocc + pj).to(dev)
        ts.append(SC.log_energy(e_pair.reshape(-1).index_select(0, flat).contiguous()))
        xs.append(feat.index_select(0, flat))
        if n % 20 == 0:
            print("[bench] training system %d/%d" % (n + 1, args.screen_train), file=sys.stderr, flush=True)
    t_data = time.perf_counter() - t_data
    X = torch.cat(xs).contiguous()
    T = torch.cat(ts).contiguous()
    params = SC.init_params(0, dev)
    tr = SC.Trainer(params, lr=2e-3)
    t_fit = time.perf_counter()
    loss = tr.fit(X, T, steps=3000, batch=4096, seed=1)
    tr.lr = 3e-4
    loss = tr.fit(X, T, steps=2000, batch=4096, seed=2)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t_fit
    print("[bench] trained on %d pairs: final minibatch loss %.4f (log10 units^2)" % (len(T), loss),
          file=sys.stderr, flush=True)

    # evaluation system
    eo, ev, r_dev, r = load(4200)
    feat, bound = SC.pair_features(B, eo, ev, r_dev, bound=True)
    pred = SC.mlp_forward(feat, tr.params)
    rm.timing_enable(True)
    t0 = run(eo, ev)
    st0 = rm.timing_collect()
    rm.timing_enable(False)
    print("[bench] unscreened energy-only run %.3f s" % t0, file=sys.stderr, flush=True)
    ep0 = e_pair.cpu().numpy().copy()
    E0 = E.cpu().numpy().copy()
    # sampled parity at full size, in the launch configuration timed: e_ij of
    # 6 pairs (near, middle and far) against the CPU baseline's oracle run on
    # the device's own B
    B_np = B.cpu().numpy()
    eo_np, ev_np = eo.cpu().numpy(), ev.cpu().numpy()
    dist = np.sqrt(((r[:, None, :] - r[None, :, :]) ** 2).sum(-1))
    iu_all = np.triu_indices(nocc, 1)
    order_d = np.argsort(dist[iu_all])
    picks = [order_d[0], order_d[len(order_d) // 3], order_d[len(order_d) // 2], order_d[2 * len(order_d) // 3],
             order_d[-1]]
    pair_checks = [(0, 0)] + [(int(iu_all[0][q]), int(iu_all[1][q])) for q in picks]
    max_rel_pair, cb = None, None
    if not args.no_cpu_baseline:
        refs, cb = cpu_baseline_pairs(B_np, eo_np, ev_np, pair_checks)
        max_rel_pair = max(abs(ep0[pi_, pj_] - ref_e) / abs(ref_e) for (pi_, pj_), ref_e in zip(pair_checks, refs))
    del B_np
    off = ~np.eye(nocc, dtype=bool)
    ptrue = np.log10(np.maximum(-ep0[iu], 1e-300))
    pp = pred.reshape(nocc, nocc).cpu().numpy()[iu]
    rmse = float(np.sqrt(np.mean((pp - ptrue) ** 2)))

    def exact_error(mask):
        return abs(math.fsum(ep0[mask > 0].tolist()))

    # literal threshold (1e-7 Eh) and the budgeted threshold
    lit, lit_e = SC.screen_mask(pred, nocc, -7.0)
    lo = SC.budget_threshold(pred, nocc, 0.5e-6)
    # the unscreened run judges each screened run; over the 1 uEh budget the
    # threshold is lowered by half a decade and the screened run repeated, and
    # after three failures the unscreened result stands (the fallback)
    attempts, t_screened, fallback = [], 0.0, False
    while True:
        bud, bud_e = SC.screen_mask(pred, nocc, lo)
        t1 = run(eo, ev, bud)
        t_screened += t1
        E1 = E.cpu().numpy().copy()
        dE_run = abs(math.fsum([float(E1[0]), float(E1[1]), -float(E0[0]), -float(E0[1])]))
        attempts.append({"threshold_log10": lo, "s": round(t1, 3), "abs_dE_Eh": dE_run})
        print("[bench] screened run %.3f s, |dE| %.3g Eh" % (t1, dE_run), file=sys.stderr, flush=True)
        if dE_run <= 1e-6:
            break
        if len(attempts) == 3:
            fallback = True
            t1, E1, dE_run = t0, E0, 0.0
            break
        lo -= 0.5
    # rigorous bound screen with the same budget: skip the smallest bounds while their sum <= 1 uEh
    bmask = SC.bound_mask(bound, 1e-6).cpu().numpy()
    nb = int(bmask[iu].sum())
    if args.screen_save:
        SC.save_params(args.screen_save, tr.params, train_seeds=[4000, 4000 + args.screen_train - 1],
                       pairs_per_system=args.screen_pairs, size=[nocc, nvir, naux], eval_seed=4200,
                       rmse_log10_eval=rmse, features="|r_i-r_j|/10, log||B_i||, log||B_j||, (eps_i+eps_j)/10",
                       target="log10|e_ij|")
    npairs = nocc * (nocc - 1)
    lit_np, bud_np = lit.cpu().numpy(), bud.cpu().numpy()
    alg = float(nocc) * (nocc + 1) * nvir * nvir * naux
    value = alg / t1 / 1e12
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "TFLOP/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(t1 * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "learned pair screening: energy-only, nocc=%d nvir=%d naux=%d, 40 A cube, 3 A decay"
                               % (nocc, nvir, naux), "train_systems": args.screen_train,
                   "train_pairs": int(len(T)), "eval_seed": 4200,
                   "flops_counted": "algorithmic full energy nocc(nocc+1) nvir^2 naux"},
        "unscreened_s": round(t0, 3), "screened_s": round(t1, 3), "speedup_screened_vs_unscreened": round(t0 / t1, 4),
        "judge": {"budget_Eh": 1e-6, "passed": not fallback, "fallback_to_unscreened": fallback,
                  "attempts": attempts, "screened_time_incl_failed_attempts_s": round(t_screened, 3)},
        "screen_budgeted": {"threshold_log10": lo, "skipped_pair_fraction": float(bud_np[off].mean()),
                            "predicted_skipped_Eh": float(bud_e), "exact_skipped_Eh": exact_error(bud_np),
                            "abs_dE_run_Eh": dE_run},
        "screen_literal_1e-7": {"skipped_pair_fraction": float(lit_np[off].mean()),
                                "predicted_skipped_Eh": float(lit_e), "exact_skipped_Eh": exact_error(lit_np)},
        "bound_screen_1uEh": {"skipped_pair_fraction": nb * 2 / npairs, "exact_skipped_Eh": exact_error(bmask)},
        "model": {"rmse_log10_eval": rmse, "train_data_s": round(t_data, 1), "train_fit_s": round(t_fit, 1),
                  "saved_to": args.screen_save or None},
        "E_unscreened": [float(E0[0]), float(E0[1])],
        "sampled_parity": {"pairs": pair_checks, "e_pair_max_rel": max_rel_pair},
        "cpu_baseline": cb,
    }
    # roofline of the unscreened run's dominant kernel (HIP events around each launch)
    dom = max(st0, key=lambda x: x["total_ms"])
    ach = dom["alg_flops"] / (dom["total_ms"] / 1e3) / 1e12
    out["roofline"] = {"bound": "mfma", "kernel": dom["name"], "achieved": round(ach, 4), "peak": FP64_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(ach / FP64_PEAK_TFLOPS, 4),
                       "avg_launch_ms": round(dom["total_ms"] / dom["launches"], 4), "launches": dom["launches"],
                       "traffic": None, "run": "unscreened energy-only run"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
