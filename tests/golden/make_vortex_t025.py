"""Writes vortex_t025_oracle.txt: the FP64 oracle's error on the isentropic vortex (Algorithm 1
with the correction, CFL 0.3, periodic [0,10]^2) at t = 0.25, against the exact cell averages
of the translated vortex.  (One period, t = 10, is out of reach: the linearised scheme about
the background state (1,1,1,1) has spectral radius 1.0068 per step at CFL 0.3, and a 128^2 run
stops with a non-admissible value at t = 7.0.)  Calls only the oracle and the input generators.

    python tests/golden/make_vortex_t025.py 128 256
"""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2508_06273_amd import inputs as I  # noqa: E402

N_GL = 3
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "vortex_t025_oracle.txt")
T_END = 0.25


def main(sizes):
    lines = ["# FP64 oracle, isentropic vortex (strength 5, centre (5,5), background (1,1,1,1),",
             "# gamma 1.4) on the periodic [0,10]^2, Algorithm 1 with the correction, CFL 0.3,",
             f"# initial averages by {N_GL}x{N_GL} Gauss-Legendre, run to t = {T_END}.",
             "# Error vs the exact cell averages of the translated vortex (same quadrature).",
             "# columns: n steps L1_rho L1_rhou L1_rhov L1_E Linf_rho Linf_rhou Linf_rhov Linf_E"]
    for n in sizes:
        st = I.shu_vortex(n, n_gl=N_GL)
        ref = I.cell_average(I.shu_vortex_field(T_END), st.grid, n_gl=N_GL)
        t0 = time.time()
        e, steps, _ = oracle.run(st, T_END, 0.3)
        assert e == 0 and st.t == T_END, (e, st.t)
        l1, linf = I.norms(st.avg, ref, st.grid)
        lines.append(f"{n} {steps} " + " ".join(f"{v:.12e}" for v in list(l1) + list(linf)))
        print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [128, 256])
