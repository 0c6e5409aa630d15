"""Writes table1_oracle.txt: the oracle's PCG iteration count and condition
number estimate for Table 1's BDDC-SO(vef) problems (Section 5.1: (10k)^3
hexahedra, 10^3 subdomains of k^3, subobjects of 4h, f = 1, residual
reduced by 10^6).  Calls only oracle/ and workloads/; k = 8 takes several
minutes of CPU time, so the GPU test reads the stored result.

    python tests/golden/make_table1_oracle.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import bddc, pcg  # noqa: E402


def main():
    lines = ["# The oracle on Table 1's BDDC-SO(vef) problems (Section 5.1), written by",
             "# tests/golden/make_table1_oracle.py: method k coarse_size iterations kappa"]
    for k in (4, 8):
        p = W.table1_problem(k)
        o = bddc.from_problem(p)
        r = pcg.solve(o, p.f[0], rtol=1e-6)
        lines.append(f"BDDC-SO(vef) {k} {o.cls.n_coarse} {r.iters} {r.kappa:.12e}")
        print(lines[-1], flush=True)
    with open(os.path.join(HERE, "table1_oracle.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
