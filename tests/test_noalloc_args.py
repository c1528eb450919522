"""Argument checks of af_step_noalloc, on the CPU: they reject a grid too large for the static
scratch array and bad pitches before any device work (no GPU call is made)."""
import pytest

from paper_2508_06273_amd import af


@pytest.fixture(scope="module")
def lib():
    try:
        return af.load()
    except FileNotFoundError:
        pytest.skip("libaf.so not built")


def test_rejects_grid_beyond_scratch(lib):
    with pytest.raises(af.AfError) as e:
        af.step_noalloc((2048, 2048, 0.0, 1.0, 0.0, 1.0), 1.4, (0, 0, 0, 0), [16] * 4,
                        [32] * 4, 2048, 2048, 1e-3)
    assert e.value.code == af.AF_ERR_INVALID_ARG and "scratch" in str(e.value)


@pytest.mark.parametrize("pa,pp", [(9, 64), (8, 63), (6, 64), (8, 6)])
def test_rejects_bad_pitches(lib, pa, pp):
    with pytest.raises(af.AfError) as e:
        af.step_noalloc((8, 8, 0.0, 1.0, 0.0, 1.0), 1.4, (1, 1, 0, 0), [16] * 4, [32] * 4,
                        pa, pp, 1e-3)
    assert e.value.code == af.AF_ERR_INVALID_ARG and "pitch" in str(e.value)


def test_rejects_aliasing_misalignment_and_options(lib):
    g = (8, 8, 0.0, 1.0, 0.0, 1.0)
    with pytest.raises(af.AfError) as e:
        af.step_noalloc(g, 1.4, (0, 0, 0, 0), [16, 48, 80, 112], [48, 32, 32, 32], 32, 64, 1e-3)
    assert "alias" in str(e.value)
    with pytest.raises(af.AfError) as e:
        af.step_noalloc(g, 1.4, (0, 0, 0, 0), [16] * 4, [40] * 4, 32, 64, 1e-3)
    assert "aligned" in str(e.value)
    with pytest.raises(af.AfError) as e:
        af.step_noalloc(g, 1.4, (0, 0, 0, 0), [16] * 4, [32] * 4, 32, 64, 1e-3, precision=7)
    assert "option" in str(e.value)
    with pytest.raises(af.AfError) as e:
        af.step_noalloc(g, 1.4, (3, 1, 0, 0), [16] * 4, [32] * 4, 32, 64, 1e-3)
    assert "inflow" in str(e.value)
