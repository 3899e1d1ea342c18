"""Iteration counts of the GPU solve on the standard setup of Sec. 5 (constant medium, 101 points
per subdomain and direction, 10 points per wavelength, four narrow sources, tolerance 1e-6)
against Tab. PMLeffect, with the package's default PML constant (16 ln omega)."""
import json
import os
import sys

import pytest

from paper_1909_01467_amd import trend

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def test_standard_setup_iterations_follow_paper_table():
    """1-wavelength PML: at most one iteration more than the paper at q = 2 ... 16; a PML of two
    wavelengths never needs more iterations than one of one wavelength (Sec. 5.1: a thicker PML
    makes the preconditioner more effective)."""
    with open(os.path.join(GOLDEN, "pml_effect_iterations.json")) as fh:
        table = json.load(fh)
    for row in table["rows"]:
        its = {}
        for w in (1, 2):
            r = trend.case(row["q"], w)
            say("q", row["q"], "wavelengths", w, "iterations", r["iterations"], "paper",
                row["iterations_pml_1_wavelength"] if w == 1 else row["iterations_pml_2_wavelengths"])
            assert r["converged"] and r["relres"] <= 1e-6
            its[w] = r["iterations"]
        assert its[1] <= row["iterations_pml_1_wavelength"] + 1, (row, its)
        assert its[2] <= its[1], (row, its)
