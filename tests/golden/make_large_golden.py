"""Writes tests/golden/large_oracle.npz: the CPU oracle's outputs for the large
fragment (nocc=200, nvir=1800, naux=6000, B = 0.3 N(0,1) exp(-P/1200), seed
1001) -- E as (hi, lo), every e_ij, P_ij, and P_ab's diagonal, Frobenius norm
and rows 0, 1, 899 and 1799 (the full P_ab is 26 MB).  Gamma is not stored.

Calls only oracle/ and synth/.  About 2.9 h on 6 cores and 28 GB of memory:

    OPENBLAS_NUM_THREADS=6 python tests/golden/make_large_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import rimp2_oracle as O  # noqa: E402

ROWS = [0, 1, 899, 1799]


def main():
    f = synth.LARGE
    t0 = time.time()
    B, eo, ev = f.arrays()
    print("inputs generated in %.1f s" % (time.time() - t0), flush=True)
    t0 = time.time()
    r = O.fragment(B, eo, ev, gamma=False, density=True)
    print("oracle finished in %.1f s" % (time.time() - t0), flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_oracle.npz")
    np.savez(out, E=np.array([r["E_hi"], r["E_lo"]]), e_pair=r["e_pair"], P_ij=r["P_ij"],
             P_ab_diag=np.diag(r["P_ab"]).copy(), P_ab_fro=np.array(np.linalg.norm(r["P_ab"])),
             P_ab_rows=r["P_ab"][ROWS].copy(), P_ab_row_index=np.array(ROWS),
             shape=np.array([f.nocc, f.nvir, f.naux]), seed=np.array(f.seed), decay=np.array(f.decay))
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
