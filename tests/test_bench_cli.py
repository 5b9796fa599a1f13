"""bench.py on the CPU: its command line refuses more than one GPU with a
message and exit status 2, before touching any device; its step planner keeps
the driver's request (20 timed steps after 5 warmup steps) inside the
wall-clock budget when one step takes tens of seconds."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def simulate(req_steps, req_warmup, budget, import_s, setup_s, step_s, reserve_s, extras_s):
    """Wall clock of a run whose steps take step_s: import and setup, the
    first warmup step, the planned steps, then the extras."""
    elapsed = import_s + setup_s + step_s
    warmup, steps = bench.plan_steps(req_steps, req_warmup, budget, elapsed, step_s, reserve_s)
    total = elapsed + (warmup - 1 + steps) * step_s + extras_s
    return warmup, steps, total


def test_planner_clamps_a_51s_step_to_the_budget():
    # 51 s per step, as the large fragment took; the driver asks for 20 + 5
    for import_s in (2.0, 60.0, 120.0):
        reserve = 2 * 51.0 + 63.0 + 15.0
        warmup, steps, total = simulate(20, 5, 420.0, import_s, 10.0, 51.0, reserve, reserve)
        assert warmup >= 1 and steps >= 1
        assert steps < 20 and warmup < 5
        assert total <= 420.0 + 1e-9, (import_s, warmup, steps, total)
        # the counts that ran times the step time stay under the driver's 600 s
        assert steps * 51.0 <= 600.0


def test_planner_keeps_the_request_when_steps_are_short():
    warmup, steps = bench.plan_steps(20, 5, 420.0, 5.0, 0.5, 30.0)
    assert (warmup, steps) == (5, 20)


def test_planner_runs_one_timed_step_even_when_nothing_fits():
    warmup, steps = bench.plan_steps(20, 5, 100.0, 90.0, 51.0, 80.0)
    assert (warmup, steps) == (1, 1)


def test_planner_prefers_timed_steps_over_extra_warmup():
    # room for 6 steps: all go to timed steps, the one warmup step already ran
    warmup, steps = bench.plan_steps(20, 5, 420.0, 60.0, 50.0, 45.0)
    assert steps == 6 and warmup == 1
    # room for 6 with 4 requested: the other 2 become warmup steps
    warmup, steps = bench.plan_steps(4, 5, 420.0, 60.0, 50.0, 45.0)
    assert steps == 4 and warmup == 3


def test_cpu_baseline_legs_return_the_oracle_and_a_rate():
    """The MBE3 and screening CPU baselines time the oracle on whole fragments
    and on single pair energies; their outputs are the oracle's own (the
    references of the sampled parity checks)."""
    import numpy as np
    import synth
    from oracle import rimp2_oracle as O
    import paper_2410_21888_amd as rm
    f = synth.random_fragment(3, 10, 24, seed=5)
    B, eo, ev = f.arrays()
    refs, cb = bench.cpu_baseline_fragments([(B, eo, ev)], [rm.flops(3, 10, 24, gamma=True, density=True)["algorithmic"]])
    ref = O.fragment(B, eo, ev)
    assert refs[0]["E_hi"] == ref["E_hi"] and np.array_equal(refs[0]["Gamma"], ref["Gamma"])
    assert cb["kind"] == "oracle" and cb["unit"] == "TFLOP/s" and cb["value"] > 0 and cb["cores"] >= 1
    pairs = [(0, 0), (0, 2)]
    prefs, pcb = bench.cpu_baseline_pairs(B, eo, ev, pairs)
    assert prefs == [float(O.pair_energy(B, eo, ev, i, j)) for i, j in pairs]
    assert prefs[1] == ref["e_pair"][0, 2] or abs(prefs[1] - ref["e_pair"][0, 2]) <= 1e-12 * abs(ref["e_pair"][0, 2])
    assert pcb["value"] > 0 and "2 occupied pairs" in pcb["sample"]
