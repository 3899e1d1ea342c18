"""Pins of the oracle's scenario 4 (Sec. 2.1, arbitrary sources): four shifted CDDs and a
partition of unity.  The windows are pinned by what the paper asks of them (they sum to one
and each vanishes on the skeleton of its own CDD); the composition by the paper's claim that
the sum of the four windowed sweeps reconstructs A^-1 f for any source, up to the PML error."""
import math

import numpy as np
import pytest

from oracle.direct import SparseLU
from oracle.discretization import GlobalProblem
from oracle.lsweep import LSweep2D, partition
from oracle.scenario4 import Scenario4, axis_window, default_shift
from paper_1909_01467_amd import inputs


def test_shifted_partition_translates_every_group_start():
    lo, hi, sizes = partition(127, 10, 4, 16)
    assert sizes == [32, 32, 32, 31]
    assert lo == [0, 26, 58, 90, 122] and hi == [26, 58, 90, 122, 147]
    assert partition(127, 10, 4, 0)[0] == [0, 42, 74, 106]
    assert default_shift(127, 4) == 15 and default_shift(511, 8) == 31


def test_axis_window_ramps_between_the_two_skeletons():
    lo = [0, 20, 40]
    los = [0, 10, 30, 50]
    a = axis_window(70, lo, los)
    assert np.all(a[:11] == 1) and np.all(a[49:] == 1)
    for b in (20, 40):                    # trace lines of an interface of the CDD
        assert a[b - 1] == 0 and a[b] == 0
    for b in (10, 30, 50):                # trace lines of a shifted interface
        assert a[b - 1] == 1 and a[b] == 1
    # linear ramp from d = 1 to d' = 1: at x = 25, d = 5.5 and d' = 4.5
    assert a[25] == pytest.approx(4.5 / (4.5 + 3.5), abs=1e-15)
    assert np.all(np.diff(a[20:30]) >= 0) and np.all(np.diff(a[40:50]) >= 0)
    assert np.all(np.diff(a[10:20]) <= 0) and np.all(np.diff(a[30:40]) <= 0)


@pytest.fixture(scope="module")
def strong_pml():
    """Constant medium, thick strong PML (as for the scenario-3 pins)."""
    n, q, p, C = 89, 3, 30, 40.0
    omega = 2 * math.pi * n / 10
    m = np.ones((n + 2 * p,) * 2)
    gp = GlobalProblem(m, omega, n, p, C)
    return gp, SparseLU(gp.A), Scenario4(m, omega, n, p, q, q, C)


def _skeleton_mask(ls: LSweep2D):
    """The trace lines of every interior interface of one CDD (Sec. 2.2)."""
    mask = np.zeros((ls.Ney, ls.Nex), dtype=bool)
    for lo in ls.ylo[1:]:
        mask[lo - 1:lo + 1, :] = True
    for lo in ls.xlo[1:]:
        mask[:, lo - 1:lo + 1] = True
    return mask


def test_windows_are_a_partition_of_unity_vanishing_on_their_skeletons(strong_pml):
    _, _, s4 = strong_pml
    total = sum(s4.windows)
    assert np.max(np.abs(total - 1.0)) < 1e-15
    for k, (ls, phi) in enumerate(zip(s4.cdds, s4.windows)):
        assert phi.min() >= 0.0 and phi.max() <= 1.0
        assert np.all(phi[_skeleton_mask(ls)] == 0.0), k
        # and each window is nonzero on part of every other CDD's skeleton
        for l, other in enumerate(s4.cdds):
            if l != k:
                assert np.any(phi[_skeleton_mask(other)] > 0.5), (k, l)


def _cross_point(ls, gp):
    p, h = ls.px, gp.h
    return ((ls.xlo[1] - 0.5 - p + 1) * h, (ls.ylo[1] - 0.5 - p + 1) * h)


@pytest.mark.parametrize("source", ["cross_point", "random"])
def test_sources_on_the_skeleton_are_reconstructed(strong_pml, source):
    """u = sum_k u^{phi_k} (Sec. 2.1): a Gaussian on the CDD's cross point and a random vector
    (both nonzero on every skeleton) are reconstructed up to the PML error."""
    gp, lu, s4 = strong_pml
    if source == "cross_point":
        b = gp.rhs(inputs.gaussian_source(gp.n[0], _cross_point(s4.cdds[0], gp)))
    else:
        b = inputs.complex_normal(gp.size, 31)
    u = lu.solve(b)
    assert np.linalg.norm(s4.apply(b) - u) / np.linalg.norm(u) < 5e-6


def test_each_shifted_cdd_is_a_valid_sweep(strong_pml):
    """Each of the four CDDs alone reconstructs its own windowed source."""
    gp, lu, s4 = strong_pml
    b = inputs.complex_normal(gp.size, 32).reshape(s4.Ney, s4.Nex)
    for ls, phi in zip(s4.cdds, s4.windows):
        bk = (phi * b).ravel()
        u = lu.solve(bk)
        assert np.linalg.norm(ls.apply(bk) - u) / np.linalg.norm(u) < 5e-6


def test_planted_dropped_window_is_detected(strong_pml, monkeypatch):
    """A plausible mistake (one of the four windowed sweeps left out) fails the pin above."""
    gp, lu, s4 = strong_pml
    b = inputs.complex_normal(gp.size, 33)
    u = lu.solve(b)
    monkeypatch.setattr(s4, "cdds", s4.cdds[:3])
    assert np.linalg.norm(s4.apply(b) - u) / np.linalg.norm(u) > 1e-2


def test_needs_two_groups_per_axis():
    m = np.ones((30, 30))
    with pytest.raises(ValueError):
        Scenario4(m, 10.0, 20, 5, 1, 3, 4.0)


def test_shift_must_keep_the_skeletons_apart():
    m = np.ones((40, 40))
    with pytest.raises(ValueError):
        Scenario4(m, 10.0, 30, 5, 2, 2, 4.0, shift=(2, 5))
    with pytest.raises(ValueError):
        Scenario4(m, 10.0, 30, 5, 2, 2, 4.0, shift=(5, 13))


def test_3d_beams_reconstruct_a_random_source():
    """Scenario 4 over beams (windows of the (x, y) cross-section on every z plane): constant
    medium, strong PML, a random source (nonzero on every skeleton) is reconstructed up to the PML
    error, as the 3D scenario-3 pins require of sources inside beams."""
    n, q, p, C = 13, 2, 6, 30.0
    omega = 2 * math.pi * n / 8
    m = np.ones((n + 2 * p,) * 3)
    gp = GlobalProblem(m, omega, n, p, C)
    s4 = Scenario4(m, omega, n, p, q, q, C)
    assert s4.shift == (3, 3)
    assert np.max(np.abs(sum(s4.windows) - 1.0)) < 1e-15
    b = inputs.complex_normal(gp.size, 34)
    u = SparseLU(gp.A).solve(b)
    assert np.linalg.norm(s4.apply(b) - u) / np.linalg.norm(u) < 1e-3   # PML error 2.6e-4 at this width
