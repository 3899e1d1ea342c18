"""Pins of the oracle's 3D beam L-sweep (Alg. Scenario3 over a q x r CDD in (x, y), beams over
all z) against exact identities and the exact-reconstruction property of Sec. 2."""
import math

import numpy as np
import pytest

from oracle.direct import SparseLU
from oracle.discretization import GlobalProblem, extend_normal
from oracle.lsweep3d import LSweep3D
from paper_1909_01467_amd import inputs


def _medium3d(n, seed):
    rng = np.random.default_rng(seed)
    x = inputs.bulk_coords(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    a, b, c = rng.uniform(1, 3, 3)
    return 1.0 + 0.3 * np.sin(a * X + b * Y) * np.cos(c * Z)


def test_3d_single_beam_is_the_exact_inverse():
    n, p = 9, 5
    m = extend_normal(_medium3d(n, 31), p)
    omega = 2 * math.pi * n / 8
    ls = LSweep3D(m, omega, n, p, 1, 1, C=5.0)
    gp = GlobalProblem(m, omega, n, p, C=5.0)
    b = inputs.complex_normal(gp.size, 32)
    u = SparseLU(gp.A).solve(b)
    assert np.linalg.norm(ls.apply(b) - u) / np.linalg.norm(u) < 1e-12


@pytest.fixture(scope="module")
def small3d():
    n, p = 11, 4
    m = extend_normal(_medium3d(n, 33), p)
    return LSweep3D(m, 2 * math.pi * n / 8, n, p, 2, 2, C=4.0)


@pytest.mark.parametrize("ij,side", [((1, 1), "B"), ((1, 1), "L"), ((0, 0), "T"), ((0, 0), "R")])
def test_3d_annihilation_straight(small3d, ij, side):
    """Sec. 1.3 in 3D: the polarized field of v = A^-1 g built from v's trace planes is chi*v
    when g vanishes on the receiving side, and -(1-chi)*v when g lives only there."""
    ls, (i, j) = small3d, ij
    chi = ls.receiving_mask(i, j, side)
    rng = np.random.default_rng(34)
    for support, expect in ((~chi, lambda v: chi * v), (chi, lambda v: -(1.0 - chi) * v)):
        g = np.where(support, rng.standard_normal(chi.shape) + 1j * rng.standard_normal(chi.shape), 0)
        v = ls.solve_local(i, j, g)
        lam = ls.extract(v, i, j)[side]
        U = ls.polarized(i, j, side, ls.straight_field(i, j, side, lam))
        assert np.linalg.norm(U - expect(v)) / np.linalg.norm(v) < 1e-12


@pytest.mark.parametrize("ij,hv", [((1, 1), ("B", "L")), ((0, 0), ("T", "R")), ((1, 0), ("B", "R")),
                                   ((0, 1), ("T", "L"))])
def test_3d_annihilation_corner(small3d, ij, hv):
    ls, (i, j) = small3d, ij
    hside, vside = hv
    chi = ls.receiving_mask(i, j, hside + vside)
    rng = np.random.default_rng(35)
    g = np.where(~chi, rng.standard_normal(chi.shape) + 1j * rng.standard_normal(chi.shape), 0)
    v = ls.solve_local(i, j, g)
    t = ls.extract(v, i, j)
    U = ls.polarized(i, j, hside + vside, ls.corner_field(i, j, hside, t[hside], vside, t[vside]))
    assert np.linalg.norm(U - chi * v) / np.linalg.norm(v) < 1e-12


def test_3d_linearity(small3d):
    ls = small3d
    N = ls.Nex * ls.Ney * ls.Nez
    x, y = inputs.complex_normal(N, 36), inputs.complex_normal(N, 37)
    a = 0.3 - 1.2j
    lhs = ls.apply(x + a * y)
    assert np.linalg.norm(lhs - ls.apply(x) - a * ls.apply(y)) / np.linalg.norm(lhs) < 1e-12


@pytest.fixture(scope="module")
def strong_pml3d():
    """Constant medium, strong PML: sources inside a beam are reconstructed up to the PML error."""
    n, q, p, C = 11, 2, 8, 30.0
    omega = 2 * math.pi * n / 8
    m = np.ones((n + 2 * p,) * 3)
    gp = GlobalProblem(m, omega, n, p, C)
    return gp, SparseLU(gp.A), LSweep3D(m, omega, n, p, q, q, C)


def _centre3d(ls, gp, i, j, z=0.4):
    p, h = ls.px, gp.h
    return (((ls.xlo[j] + ls.xhi[j] - 1) / 2 - p + 1) * h, ((ls.ylo[i] + ls.yhi[i] - 1) / 2 - p + 1) * h, z)


@pytest.mark.parametrize("ij", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_3d_point_source_is_reconstructed(strong_pml3d, ij):
    gp, lu, ls = strong_pml3d
    b = gp.rhs(inputs.gaussian_source(ls.nx, _centre3d(ls, gp, *ij)))
    u = lu.solve(b)
    assert np.linalg.norm(ls.apply(b) - u) / np.linalg.norm(u) < 1e-4


def test_3d_planted_full_line_legs_are_detected(strong_pml3d, monkeypatch):
    """The plausible mistake of L legs over full window planes must fail the pin above."""
    gp, lu, ls = strong_pml3d

    def full_lines(self, i, j, hside, hlam, vside, vlam):
        ut = np.zeros(self.shape(i, j), dtype=np.complex128)
        a, b = self.lines(i, j, vside)
        ut[:, :, a], ut[:, :, b] = vlam[0], vlam[1]
        a, b = self.lines(i, j, hside)
        ut[:, a, :], ut[:, b, :] = hlam[0], hlam[1]
        return ut

    monkeypatch.setattr(LSweep3D, "corner_field", full_lines)
    b = gp.rhs(inputs.gaussian_source(ls.nx, _centre3d(ls, gp, 0, 0)))
    u = lu.solve(b)
    assert np.linalg.norm(ls.apply(b) - u) / np.linalg.norm(u) > 1e-3
