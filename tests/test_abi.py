"""The C-ABI library loads and exports every entry point include/bem.h
declares; argument validation that precedes any device call (CPU only)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bem.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bem_\w+)\s*\(", text)))


def test_header_declares_core_entry_points():
    names = declared_functions()
    for n in ("bem_influence", "bem_influence_ex", "bem_convolve", "bem_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1612_08395_amd import bem
    out = subprocess.run(["nm", "-D", "--defined-only", bem.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(bem_\w+)$", out, flags=re.M))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert hasattr(bem._lib, n)


@pytest.mark.parametrize("args", [
    (0, 8, 0.1, 0.3, 0.3),        # empty grid
    (8, 8, -0.1, 0.3, 0.3),       # negative element size
    (8, 8, 0.1, 1.0, 0.3),        # k outside (-1, 1), Eq. 1
    (8, 8, 0.1, -1.2, 0.3),
    (8, 8, 0.1, 0.3, 0.5),        # nu outside [0, 0.5)
    (8, 8, float("nan"), 0.3, 0.3),
])
def test_invalid_arguments_rejected(args):
    from paper_1612_08395_amd import bem
    with pytest.raises(bem.BemError) as e:
        bem.bem_influence(*args)
    assert e.value.code == bem.BEM_EINVAL
    assert bem.bem_last_error()


def test_oversized_grid_unsupported():
    from paper_1612_08395_amd import bem
    with pytest.raises(bem.BemError) as e:
        bem.bem_influence(bem.BEM_MAX_N + 1, 8, 0.1, 0.3, 0.3)
    assert e.value.code == bem.BEM_EUNSUPPORTED


def test_solver_clock_host_paths():
    from paper_1612_08395_amd import bem
    with pytest.raises(bem.BemError) as e:         # no clock running on this thread
        bem.bem_clock_stop()
    assert e.value.code == bem.BEM_EINVAL
    bem.bem_clock_start()
    c = bem.bem_clock_stop()                       # no solve in between: nothing timed
    assert c.iterations == 0 and c.skipped == 0 and list(c.launches) == [0] * 6
