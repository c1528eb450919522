"""CPU-side checks of the C ABI: the library is built for gfx950, loads, and exports every
symbol that include/af.h declares.  No compute call is made here."""
import ctypes as ct
import os
import re
import subprocess

import pytest

from paper_2508_06273_amd import af

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "af.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(af_[a-z_]+)\s*\(", txt)))


def test_header_matches_binding_list():
    assert declared_symbols() == sorted(af.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(af.LIB_PATH):
        pytest.skip("libaf.so not built")
    out = subprocess.check_output(["nm", "-D", "--defined-only", af.LIB_PATH], text=True)
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    lib = ct.CDLL(af.LIB_PATH)
    for s in declared_symbols():
        assert hasattr(lib, s)


def test_library_contains_gfx950_code():
    if not os.path.exists(af.LIB_PATH):
        pytest.skip("libaf.so not built")
    data = open(af.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_binding_fails_loudly_without_library(tmp_path):
    with pytest.raises(FileNotFoundError):
        af._lib = None
        af.load(str(tmp_path / "missing.so"))
    af._lib = None


@pytest.mark.parametrize("grid,gamma,bc,what", [
    ((8, 8, 0.0, float("inf"), 0.0, 1.0), 1.4, (0, 0, 0, 0), "finite"),
    ((8, 8, float("nan"), 1.0, 0.0, 1.0), 1.4, (0, 0, 0, 0), "finite"),
    ((8, 8, 0.0, 1.0, 1.0, 1.0), 1.4, (0, 0, 0, 0), "empty domain"),
    ((8, 8, 0.0, 1e-300, 0.0, 1.0), 1.4, (0, 0, 0, 0), "cell size"),
    ((1, 8, 0.0, 1.0, 0.0, 1.0), 1.4, (0, 0, 0, 0), "nx, ny"),
    ((8, 8, 0.0, 1.0, 0.0, 1.0), float("inf"), (0, 0, 0, 0), "gamma"),
    ((8, 8, 0.0, 1.0, 0.0, 1.0), 1.0, (0, 0, 0, 0), "gamma"),
    ((8, 8, 0.0, 1.0, 0.0, 1.0), 1.4, (0, 1, 0, 0), "periodic"),
    ((8, 8, 0.0, 1.0, 0.0, 1.0), 1.4, (7, 7, 0, 0), "boundary kind"),
])
def test_create_rejects_bad_arguments(grid, gamma, bc, what):
    """Argument checks of af_create and af_create_batch come before any HIP call: a bad grid,
    gamma or side set is refused with AF_ERR_INVALID_ARG and a message naming the problem."""
    if not os.path.exists(af.LIB_PATH):
        pytest.skip("libaf.so not built")
    af._lib = None
    L = af.load()
    G = af.Grid(*grid)
    B = af.Bc(*bc)
    h = ct.c_void_p()
    assert L.af_create(ct.byref(G), gamma, ct.byref(B), ct.byref(h)) == af.AF_ERR_INVALID_ARG
    assert not h.value
    assert what in L.af_last_error(None).decode()
    assert L.af_create_batch(1, ct.byref(G), gamma, ct.byref(B), ct.byref(h)) == \
        af.AF_ERR_INVALID_ARG
    assert what in L.af_last_error(None).decode()
