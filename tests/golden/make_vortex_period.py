"""Writes vortex_period_oracle.txt: the FP64 oracle's error after one period of the isentropic
vortex (Algorithm 1 with the correction, CFL 0.3, t = 10 on the periodic [0,10]^2), against the
exact cell averages (the initial ones: after one period the exact solution is the initial
state).  Calls only the oracle and the input generators.

    python tests/golden/make_vortex_period.py 128 256
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
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "vortex_period_oracle.txt")


def main(sizes):
    lines = ["# FP64 oracle, isentropic vortex (strength 5, centre (5,5), background (1,1,1,1),",
             "# gamma 1.4) on the periodic [0,10]^2, Algorithm 1 with the correction, CFL 0.3,",
             f"# initial averages by {N_GL}x{N_GL} Gauss-Legendre, run to t = 10 (one period).",
             "# Error vs the exact averages (= the initial averages after one period).",
             "# columns: n steps L1_rho L1_rhou L1_rhov L1_E Linf_rho Linf_rhou Linf_rhov Linf_E"]
    for n in sizes:
        st = I.shu_vortex(n, n_gl=N_GL)
        ref = st.avg.copy()
        t0 = time.time()
        e, steps, _ = oracle.run(st, 10.0, 0.3)
        assert e == 0 and st.t == 10.0, (e, st.t)
        l1, linf = I.norms(st.avg, ref, st.grid)
        lines.append(f"{n} {steps} " + " ".join(f"{v:.12e}" for v in list(l1) + list(linf)))
        print(lines[-1], f"({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [128, 256])
