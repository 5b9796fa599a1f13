"""Summaries of rocprofv3 output for the library's kernels (measurement
tooling; no part of the compute path).

    python -m paper_2410_21888_amd.profsum trace <kernel_stats.csv>
        per-kernel totals of a `rocprofv3 --kernel-trace --stats
        --output-format csv` run, with each kernel's role

    python -m paper_2410_21888_amd.profsum traffic <fetch.csv> <write.csv> \\
            --workload large --json profiles/hbm_traffic.json
        HBM bytes per launch and role from two `rocprofv3 --pmc FETCH_SIZE` /
        `--pmc WRITE_SIZE` runs (counter_collection.csv), each counter scaled
        by what it read for the largest runtime copy kernel of the run (the
        1 GiB device-to-device copy `bench.py --calib-copy` makes), and tagged
        with the hash of the kernel sources it was measured on

    python -m paper_2410_21888_amd.profsum mfma <counter_collection.csv>
        per-role matrix-unit occupancy and clock from one `rocprofv3 --pmc
        SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE` run: busy cycles over all
        SIMDs divided by (GPU-active cycles per XCC x SIMD count), and
        GPU-active cycles per XCC over the dispatch's duration
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_KERNEL = "__amd_rocclr_copyBuffer"
CALIB_BYTES = 1 << 30        # bench.py --calib-copy moves 1 GiB each way

_GEMM_ROLES = {"0": "ints_gemm", "1": "gamma_gemm", "2": "pab_gemm", "3": "pij_gemm", "4": "gamma_t_gemm",
               "5": "gamma_ao_gemm", "6": "l_terms_gemm"}


# the sources the fragment path's kernels are built from (screening and the
# adjacent gradient steps have their own files and do not enter it)
FRAGMENT_SOURCES = ("batch.hpp", "common.hpp", "gemm_f64.hpp", "kernels.hpp", "rimp2.hip", "split_int8.hpp")


def strip_comments(src: str) -> str:
    """C/C++ source without its comments (string and character literals kept)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return "".join(out)


def sources_hash(read) -> str:
    """Hash of the fragment path's kernel sources: names, and contents without
    comments with every run of white space read as one blank; read(name)
    returns a file's text."""
    h = hashlib.sha256()
    for fn in FRAGMENT_SOURCES:
        h.update(fn.encode() + " ".join(strip_comments(read(fn)).split()).encode())
    return h.hexdigest()[:16]


def kernel_source_hash() -> str:
    """Hash of the fragment path's kernel sources as they are in the tree
    (comments do not enter it)."""
    def read(fn):
        with open(os.path.join(CSRC, fn), encoding="utf-8") as f:
            return f.read()
    return sources_hash(read)


def role_of(name: str) -> str:
    """The library role of a kernel symbol (the names rimp2_timing_collect uses)."""
    m = re.search(r"gemm_f64_(?:kernel|grouped)<\s*\d+,\s*\d+,\s*\d+,\s*(true|false),\s*(\d)", name)
    if m:
        if m.group(2) == "1" and m.group(1) == "false":   # K-contiguous B: the metric contraction of Gamma
            return "gamma_metric"
        return _GEMM_ROLES[m.group(2)]
    for key, role in (("gemm_oz8_", None), ("amplitude", "amplitude"),
                      ("pair_energy_reduce", "amplitude (pair energy reduce)"),
                      ("splitk_reduce", "splitk_reduce"), ("reduce_grouped", "splitk_reduce"),
                      ("energy_sum", "energy_sum"), ("gap_check", "gap_check"), ("split_rows", "digit_split"),
                      ("split_cols", "digit_split"), ("colmax", "digit_split"), ("zero_u64", "digit_split"),
                      ("digit_split_grouped", "digit_split"), ("relocate_digit", "status_copy"),
                      ("copy_status", "status_copy"), ("status_copy", "status_copy"),
                      ("relocate_tables", "status_copy"), ("relocate_oz", "status_copy"),
                      ("zero_counters", "status_copy"),
                      (COPY_KERNEL, "(runtime copy)"), ("at::native", "(torch)"), ("three_index", "(input generator)")):
        if key in name:
            if role is None:   # the split-precision products, by digit count
                m2 = re.search(r"gemm_oz8_(kernel|grouped)<\s*(\d+)", name)
                if not m2:
                    return "oz8"
                return "oz8 S=%s%s" % (m2.group(2), " (grouped)" if m2.group(1) == "grouped" else "")
            return role
    return "(other)"


def _rows(path: str) -> list:
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _num(x: str) -> float:
    return float(x) if x not in ("", None) else 0.0


def _col(r: dict, *names) -> float:
    for n in names:
        if n in r:
            return _num(r[n])
    return 0.0


def trace_summary(stats_csv: str) -> str:
    """Markdown table of a kernel statistics CSV (rocprofv3 --stats, or
    rocpd2summary's kernels summary)."""
    rows = _rows(stats_csv)
    tot_of = lambda r: _col(r, "TotalDurationNs", "Duration (Nsec)")
    total = sum(tot_of(r) for r in rows) or 1.0
    out = ["| role | kernel | calls | total ms | average ms | % |", "|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -tot_of(r)):
        name = r["Name"]
        tot = tot_of(r)
        calls = int(_col(r, "Calls"))
        avg = _col(r, "AverageNs", "Average (Nsec)")
        short = name if len(name) <= 70 else name[:70]
        out.append("| %s | `%s` | %d | %.1f | %.3f | %.2f |" % (role_of(name), short, calls, tot / 1e6, avg / 1e6,
                                                              100.0 * tot / total))
    return "\n".join(out)


def _per_kernel(counter_csv: str, counter: str):
    """{dispatch id: (kernel name, value)} for one counter (values summed over
    dimensions of the same dispatch)."""
    d = {}
    for r in _rows(counter_csv):
        if r["Counter_Name"] != counter:
            continue
        key = r["Dispatch_Id"]
        name, v = d.get(key, (r["Kernel_Name"], 0.0))
        d[key] = (name, v + _num(r["Counter_Value"]))
    return d


def _split_roles(vals: dict, first: dict) -> dict:
    """Per dispatch (in dispatch order) the role, with the launches of a role
    past the first first[role] ones named "<role> (later)"."""
    seen = defaultdict(int)
    out = {}
    for key in sorted(vals, key=lambda k: int(k)):
        name, _ = vals[key]
        role = role_of(name)
        if role in first:
            seen[role] += 1
            if seen[role] > first[role]:
                role = role + " (later)"
        out[key] = role
    return out


def traffic(fetch_csv: str, write_csv: str, first: dict | None = None):
    """Calibrated HBM bytes per launch and role.  ``first`` = {role: N} keeps
    the first N launches of a role under its name and the rest as
    "<role> (later)" (two runs of the same kernel in one process)."""
    first = first or {}
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    # calibration: the largest runtime copy of each run moved CALIB_BYTES each way
    f_copy = max((v for n, v in fetch.values() if COPY_KERNEL in n), default=0.0)
    w_copy = max((v for n, v in write.values() if COPY_KERNEL in n), default=0.0)
    if f_copy <= 0 or w_copy <= 0:
        raise SystemExit("no calibration copy found (run bench.py with --calib-copy)")
    fs, ws = CALIB_BYTES / (f_copy * 1024.0), CALIB_BYTES / (w_copy * 1024.0)
    acc = defaultdict(lambda: [0, 0.0, 0.0])
    n_f = defaultdict(int)
    for vals, idx in ((fetch, 1), (write, 2)):
        roles = _split_roles(vals, first)
        for key, (name, v) in vals.items():
            role = roles[key]
            if role.startswith("("):
                continue
            acc[role][idx] += v
            if idx == 1:
                n_f[role] += 1
    out = {}
    for role, (_, f_kib, w_kib) in acc.items():
        n = n_f[role] or 1
        out[role] = {"launches": n, "fetch_kib_raw": f_kib / n, "write_kib_raw": w_kib / n,
                     "bytes_per_launch": (f_kib * fs + w_kib * ws) * 1024.0 / n}
    return out, {"fetch_scale": fs, "write_scale": ws, "fetch_copy_kib": f_copy, "write_copy_kib": w_copy}


def _agent(counter_csv: str):
    """(SIMD count, XCC count) of the GPU agent, from the agent_info.csv that
    rocprofv3 writes beside the counter file."""
    path = counter_csv.replace("counter_collection.csv", "agent_info.csv")
    for r in _rows(path):
        if _num(r.get("Simd_Count", "")) > 0:
            return int(_num(r["Simd_Count"])), max(1, int(_num(r.get("Num_Xcc", "1"))))
    raise SystemExit("no GPU agent in %s" % path)


def mfma(counter_csv: str, simds: int = 0, xccs: int = 0, first: dict | None = None):
    """{role: {launches, avg_ms, clock_ghz, mfma_busy}} from one PMC run of
    SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE (values summed over
    dimensions; GRBM_GUI_ACTIVE counts once per XCC).  ``first`` splits
    repeated roles as in traffic()."""
    if not simds:
        simds, xccs = _agent(counter_csv)
    busy = _per_kernel(counter_csv, "SQ_VALU_MFMA_BUSY_CYCLES")
    roles = _split_roles(busy, first or {})
    gui = _per_kernel(counter_csv, "GRBM_GUI_ACTIVE")
    lds = _per_kernel(counter_csv, "SQ_LDS_IDX_ACTIVE")
    conf = _per_kernel(counter_csv, "SQ_LDS_BANK_CONFLICT")
    dur = {}
    for r in _rows(counter_csv):
        dur[r["Dispatch_Id"]] = _num(r["End_Timestamp"]) - _num(r["Start_Timestamp"])
    acc = defaultdict(lambda: [0, 0.0, 0.0, 0.0, 0.0, 0.0])
    for key, (name, b) in busy.items():
        role = roles[key]
        if role.startswith("(") or key not in gui:
            continue
        e = acc[role]
        e[0] += 1
        e[1] += dur.get(key, 0.0)
        e[2] += b
        e[3] += gui[key][1] / xccs
        e[4] += lds[key][1] if key in lds else 0.0
        e[5] += conf[key][1] if key in conf else 0.0
    out = {}
    cus = simds // 4
    for role, (n, ns, b, cyc, li, lc) in acc.items():
        out[role] = {"launches": n, "avg_ms": ns / n / 1e6, "clock_ghz": cyc / ns if ns > 0 else 0.0,
                     "mfma_busy": b / (cyc * simds) if cyc > 0 else 0.0}
        if lds:   # LDS busy with indexed accesses, per CU, and the bank-conflict share of those cycles
            out[role]["lds_util"] = li / (cyc * cus) if cyc > 0 else 0.0
            out[role]["lds_conflict"] = lc / li if li > 0 else 0.0
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2410_21888_amd.profsum")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("stats_csv")
    h = sub.add_parser("traffic")
    h.add_argument("fetch_csv")
    h.add_argument("write_csv")
    h.add_argument("--workload", required=True)
    h.add_argument("--json", help="merge the result into this JSON file")
    h.add_argument("--first", action="append", default=[], metavar="ROLE=N",
                   help="keep the first N launches of ROLE under its name, the rest as 'ROLE (later)'")
    h.add_argument("--later-workload", default="",
                   help="with --json: file the 'ROLE (later)' entries under this workload, as ROLE")
    m = sub.add_parser("mfma")
    m.add_argument("counter_csv")
    m.add_argument("--first", action="append", default=[], metavar="ROLE=N",
                   help="keep the first N launches of ROLE under its name, the rest as 'ROLE (later)'")
    a = ap.parse_args(argv)
    if a.cmd == "mfma":
        print("Kernel sources hash: %s\n" % kernel_source_hash())
        res = mfma(a.counter_csv, first={kv.split("=")[0]: int(kv.split("=")[1]) for kv in a.first})
        with_lds = any("lds_util" in e for e in res.values())
        print("| role | launches | average ms | clock GHz | matrix units busy |" + (" LDS busy | LDS bank-conflict cycles |"
                                                                             if with_lds else ""))
        print("|---|---|---|---|---|" + ("---|---|" if with_lds else ""))
        for role, e in sorted(res.items(), key=lambda kv: -kv[1]["avg_ms"] * kv[1]["launches"]):
            line = "| %s | %d | %.3f | %.2f | %.1f%% |" % (role, e["launches"], e["avg_ms"], e["clock_ghz"],
                                                         100.0 * e["mfma_busy"])
            if with_lds:
                line += " %.1f%% | %.1f%% |" % (100.0 * e.get("lds_util", 0.0), 100.0 * e.get("lds_conflict", 0.0))
            print(line)
        return 0
    if a.cmd == "trace":
        print("Kernel sources hash: %s\n" % kernel_source_hash())
        print(trace_summary(a.stats_csv))
        return 0
    first = {kv.split("=")[0]: int(kv.split("=")[1]) for kv in a.first}
    roles, cal = traffic(a.fetch_csv, a.write_csv, first)
    src = kernel_source_hash()
    print("Calibration: FETCH_SIZE x%.4f, WRITE_SIZE x%.4f (copy read %.0f / %.0f KiB for 1 GiB)\n" % (
        cal["fetch_scale"], cal["write_scale"], cal["fetch_copy_kib"], cal["write_copy_kib"]))
    print("Kernel sources hash: %s\n" % src)
    print("| role | launches | FETCH_SIZE KiB/launch (raw) | WRITE_SIZE KiB/launch (raw) | HBM bytes/launch (scaled) |")
    print("|---|---|---|---|---|")
    for role, e in sorted(roles.items(), key=lambda kv: -kv[1]["bytes_per_launch"] * kv[1]["launches"]):
        print("| %s | %d | %.4g | %.4g | %.4g |" % (role, e["launches"], e["fetch_kib_raw"], e["write_kib_raw"],
                                                    e["bytes_per_launch"]))
    if a.json:
        d = {}
        if os.path.exists(a.json):
            with open(a.json) as fh:
                d = json.load(fh)
        later = " (later)"
        if a.later_workload:
            d[a.workload] = {r: dict(e, source_hash=src) for r, e in roles.items() if not r.endswith(later)}
            d[a.later_workload] = {r[:-len(later)]: dict(e, source_hash=src) for r, e in roles.items()
                                   if r.endswith(later)}
        else:
            d[a.workload] = {r: dict(e, source_hash=src) for r, e in roles.items()}
        d["calibration"] = cal
        with open(a.json, "w") as f:
            json.dump(d, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
