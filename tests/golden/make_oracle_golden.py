"""Writes tests/golden/oracle_*.json: loss probabilities computed by the
FP64 CPU oracle (dense LU, no FFT) for workloads too slow to solve inside a
test.  Calls only oracle/ and the seeded input generators.

    python tests/golden/make_oracle_golden.py
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle.dda import solve_point  # noqa: E402


def c1():
    w = W.c1_single_solve()
    r = solve_point(w.mask, w.d, w.eps_dipoles(0), w.m_h, w.beta, w.r0[0],
                    float(w.energies[0]), pol=w.polarizability, method="lu")
    return {
        "workload": w.name,
        "recipe": "workloads.c1_single_solve(): 16^3 sphere R = 8 nm, d = 1 nm, eps = -10+1i, "
                  "m_h = 1.45, beta = 0.55, r0 = (10, 0, 0) nm, E = 2.5 eV, LDR",
        "solver": "dense LU (oracle.solve.lu_solve)",
        "n_occ": int(w.n_occ),
        "rel_residual": r.residual,
        "p_eels": r.p_eels, "p_ext": r.p_ext, "p_abs": r.p_abs, "p_cl": r.p_cl,
    }


if __name__ == "__main__":
    out = os.path.join(HERE, "oracle_c1.json")
    with open(out, "w") as f:
        json.dump(c1(), f, indent=1)
    print("wrote", out)
