"""Writes the stored expected values under tests/golden/ from the oracle alone.

Run from the repository root: python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402


def main():
    # every file is rewritten; the 64-shell table takes about a minute and 9 GB
    # |S_s| for unit-width shells s = 1..64 (full periodic grid large enough to hold them).
    S = O.shell_mode_counts(132, 64, 1.0)
    np.savetxt(os.path.join(HERE, "shell_modes_width1.txt"),
               np.stack([np.arange(1, 65), S], axis=1), fmt="%d",
               header="shell |S_s| for width 1 k_f, shell s = [(s-1/2), (s+1/2)) k_f")
    # Triangle counts of the 64^3 grid with 16 unit-width shells.
    cand = O.candidate_tuples(3, 16, True)
    n = O.polygon_counts(64, 3, 16, 1.0, cand)
    keep = n > 0
    np.savetxt(os.path.join(HERE, "bispec_64_counts.txt"),
               np.concatenate([cand[keep], n[keep, None]], axis=1), fmt="%d",
               header="t1 t2 t3 n_t: closed ordered triangles, N=64, 16 shells of width 1 k_f")
    # Triangle counts of 64 unit-width shells.  3 (64 + 1/2) <= 256, so no closure wraps
    # around the periodic grid and the counts are the number of integer vector triangles:
    # the same for every alias-free N (the 256^3 and 512^3 workloads share this table).
    cand = O.candidate_tuples(3, 64, True)
    n = O.polygon_counts(256, 3, 64, 1.0, cand)
    keep = n > 0
    np.savetxt(os.path.join(HERE, "bispec_64shells_counts.txt.gz"),
               np.concatenate([cand[keep], n[keep, None]], axis=1), fmt="%d",
               header="t1 t2 t3 n_t: closed ordered triangles, 64 shells of width 1 k_f, any alias-free N "
                      "(computed at N=256)")


if __name__ == "__main__":
    main()
