"""Host logic of bench.py, on the CPU: the benchmark refuses more than one GPU before it touches
one, and its algorithmic FLOP model is the sum of the per-part counts it documents (the
roofline's `achieved` rests on it)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_flop_model_is_the_sum_of_its_parts():
    eg2 = 1443 + 575 + 580          # corner, x-edge, y-edge EG2 (set-up included)
    per_dof = 213 + 197 + 197       # derivatives, correction, assembly, fluxes, wave speed
    per_cell = 440                  # inverse Simpson, centre value, average, monomials
    # Algorithm 1: three EG2 evaluations per DOF; the averaged linearisation: two, plus the
    # mean of the adjacent averages
    assert bench.flops_per_cell(0, "fp32") == 3 * eg2 + per_dof + per_cell == 8841
    assert bench.flops_per_cell(0, "fp64") == 8841
    assert bench.flops_per_cell(1, "fp64") == 2 * eg2 + per_dof + per_cell + 32
    # the non-packed issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
    assert abs(bench.PEAK_NONPACKED - 256 * 4 * 16 * 2 * 2.4e9 / 1e12) < 0.05


@pytest.mark.parametrize("args,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(args, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args,
                       env={**os.environ, **env}, capture_output=True, text=True, timeout=300)
    assert r.returncode == 2, r.stderr
    assert "one GPU only" in r.stderr
