"""The per-subdomain check of the GPU parity tests catches an error confined to one subdomain
that the whole-grid norm lets through (a planted error on the CPU; no GPU)."""
import numpy as np
import pytest

from oracle.lsweep import partition
from paper_1909_01467_amd import inputs
from tests.parity_check import block_errors, check


class _Cdd:
    def __init__(self, n, p, q, r):
        self.xlo, self.xhi, _ = partition(n, p, r)
        self.ylo, self.yhi, _ = partition(n, p, q)


def test_error_confined_to_one_subdomain_is_caught():
    n, p, q = 60, 6, 4
    cdd = _Cdd(n, p, q, q)
    shape = (n + 2 * p, n + 2 * p)
    ref = inputs.complex_normal(shape, 1)
    got = ref.copy()
    y0, y1, x0, x1 = cdd.ylo[2], cdd.yhi[2], cdd.xlo[1], cdd.xhi[1]
    got[y0:y1, x0:x1] *= 1 + 3e-12          # 3e-12 on one of 16 subdomains: 7e-13 in the whole norm
    be = block_errors(got, ref, shape, cdd)
    assert int(be.argmax()) == 2 * q + 1 and be.max() == pytest.approx(3e-12, rel=1e-3)
    check("planted whole-norm only", got, ref, 1e-12)                  # passes without the partition
    with pytest.raises(AssertionError):
        check("planted per subdomain", got, ref, 1e-12, cdd=cdd, shape=shape, block_bar=2e-12)


def test_quiet_subdomain_is_measured_against_the_floor():
    n, p, q = 40, 4, 2
    cdd = _Cdd(n, p, q, q)
    shape = (n + 2 * p, n + 2 * p)
    ref = inputs.complex_normal(shape, 2)
    ref[: cdd.yhi[0], : cdd.xhi[0]] *= 1e-9   # a quiet corner: its own norm is no scale for an error
    got = ref + 1e-14 * inputs.complex_normal(shape, 3)
    assert block_errors(got, ref, shape, cdd).max() < 1e-12
