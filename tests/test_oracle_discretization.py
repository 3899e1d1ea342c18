"""Pins of the oracle's discretisation (App. A) against closed forms and library routines."""
import math

import numpy as np
import pytest
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.special as ssp

from oracle.direct import SparseLU, solve_banded, solve_dense
from oracle.discretization import GlobalProblem, extend_normal
from paper_1909_01467_amd import inputs


def _rand_smooth(shape, seed):
    rng = np.random.default_rng(seed)
    return 1.0 + 0.3 * rng.uniform(size=shape)


def test_operator_is_complex_symmetric():
    m = extend_normal(_rand_smooth((17, 20), 0), (4, 5))
    gp = GlobalProblem(m, 30.0, (20, 17), (4, 5), C=6.0)
    D = (gp.A - gp.A.T).tocoo()
    assert D.nnz == 0 or np.max(np.abs(D.data)) == 0.0
    # not Hermitian: the PML makes the coefficients complex
    assert abs(gp.A - gp.A.conj().T).max() > 0.0


def test_normal_extension_copies_nearest_bulk_value():
    mb = _rand_smooth((6, 9), 1)
    me = extend_normal(mb, (3, 2))      # 3 points in x, 2 in y
    assert me.shape == (10, 15)
    assert np.array_equal(me[2:-2, 3:-3], mb)
    assert np.all(me[0, 3:-3] == mb[0]) and np.all(me[-1, 3:-3] == mb[-1])
    assert np.all(me[2:-2, 0] == mb[:, 0]) and me[0, 0] == mb[0, 0]


def _dst_eigs(n, h):
    k = np.arange(1, n + 1)
    return 4.0 / h**2 * np.sin(np.pi * k / (2 * (n + 1))) ** 2


def test_no_pml_2d_matches_dst_closed_form():
    """n_pml = 0, constant m: the textbook Dirichlet 5-point Helmholtz, diagonalised by DST-I."""
    nx, ny, omega = 15, 11, 7.3
    h = 1.0 / (nx + 1)
    gp = GlobalProblem(np.full((ny, nx), 1.0), omega, (nx, ny), 0, C=3.0)
    f = inputs.complex_normal((ny, nx), 3)
    u = solve_banded(gp.A, f.ravel()).reshape(ny, nx)
    lam = _dst_eigs(ny, h)[:, None] + _dst_eigs(nx, h)[None, :] - omega**2
    u_cf = sfft.idstn(sfft.dstn(f, type=1, norm="ortho") / lam, type=1, norm="ortho")
    assert np.linalg.norm(u - u_cf) / np.linalg.norm(u_cf) < 1e-12


def test_no_pml_2d_medium_varying_in_x_reduces_to_1d_solves():
    """m = m(x): DST-I in y, then one textbook tridiagonal solve in x per y-mode."""
    nx, ny, omega = 13, 9, 9.1
    h = 1.0 / (nx + 1)
    mx = 1.0 + 0.5 * np.sin(np.arange(nx))
    gp = GlobalProblem(np.tile(mx, (ny, 1)), omega, (nx, ny), 0, C=3.0)
    f = inputs.complex_normal((ny, nx), 4)
    u = solve_banded(gp.A, f.ravel()).reshape(ny, nx)
    fh = sfft.dst(f, type=1, norm="ortho", axis=0)
    uh = np.zeros_like(fh)
    muy = _dst_eigs(ny, h)
    for k in range(ny):
        ab = np.zeros((3, nx), dtype=np.complex128)
        ab[0, 1:] = -1.0 / h**2
        ab[2, :-1] = -1.0 / h**2
        ab[1] = 2.0 / h**2 + muy[k] - omega**2 * mx
        uh[k] = sla.solve_banded((1, 1), ab, fh[k])
    u_cf = sfft.idst(uh, type=1, norm="ortho", axis=0)
    assert np.linalg.norm(u - u_cf) / np.linalg.norm(u_cf) < 1e-12


def test_no_pml_3d_matches_dst_closed_form():
    nx, ny, nz, omega = 7, 6, 5, 4.1
    h = 1.0 / (nx + 1)
    gp = GlobalProblem(np.full((nz, ny, nx), 1.0), omega, (nx, ny, nz), 0, C=3.0)
    f = inputs.complex_normal((nz, ny, nx), 5)
    u = solve_dense(gp.A, f.ravel()).reshape(nz, ny, nx)
    lam = (_dst_eigs(nz, h)[:, None, None] + _dst_eigs(ny, h)[None, :, None]
           + _dst_eigs(nx, h)[None, None, :] - omega**2)
    u_cf = sfft.idstn(sfft.dstn(f, type=1, norm="ortho") / lam, type=1, norm="ortho")
    assert np.linalg.norm(u - u_cf) / np.linalg.norm(u_cf) < 1e-12


@pytest.mark.parametrize("C", [2.0, 4.0, 8.0])
def test_pml_normal_incidence_reflection_is_exp_minus_C_over_2(C):
    """1-D: the cubic profile integrates to C/4 over the layer, so a wave crossing it twice
    comes back with modulus exp(-C/2) (fine grid)."""
    n, p, omega = 2000, 400, 2 * math.pi * 5
    gp = GlobalProblem(np.ones(n + 2 * p), omega, n, p, C=C)
    h = gp.h
    b = np.zeros(n + 2 * p, dtype=np.complex128)
    src = p + n // 4
    b[src] = 1.0 / h
    u = solve_banded(gp.A, b)
    k = math.acos(1.0 - (omega * h) ** 2 / 2.0) / h       # discrete wavenumber
    idx = np.arange(src + 20, p + n - 20)
    x = gp.x_int[0][idx]
    M = np.stack([np.exp(1j * k * x), np.exp(-1j * k * x)], axis=1)
    (a, bb), *_ = np.linalg.lstsq(M, u[idx], rcond=None)
    assert abs(abs(bb / a) - math.exp(-C / 2)) / math.exp(-C / 2) < 2e-3


def test_converges_to_free_space_hankel_at_second_order():
    """Constant speed, strong PML: u -> (i/4) H0(omega r) * exp(-omega^2 w^2/4) on an annulus."""
    omega = 2 * math.pi * 4
    errs = []
    for n in (63, 127, 255):
        h = 1.0 / (n + 1)
        p = int(round(0.25 / h))                 # one wavelength of PML
        gp = GlobalProblem(np.ones((n + 2 * p,) * 2), omega, n, p, C=20.0)
        f = inputs.gaussian_source(n, (0.5, 0.5))
        u = SparseLU(gp.A).solve(gp.rhs(f)).reshape(gp.m.shape)[p:-p, p:-p]
        X, Y = np.meshgrid(inputs.bulk_coords(n), inputs.bulk_coords(n))
        r = np.hypot(X - 0.5, Y - 0.5)
        ring = (r >= 0.15) & (r <= 0.35)
        w = 2 * h
        exact = 0.25j * ssp.hankel1(0, omega * r[ring]) * math.exp(-(omega * w) ** 2 / 4)
        errs.append(np.max(np.abs(u[ring] - exact)) / np.max(np.abs(exact)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 0.01
    assert all(1.7 < o < 2.3 for o in orders), (errs, orders)


def test_pml_constant_reading_truncates_one_wavelength_pml_best():
    """App. A leaves the scale of C open.  For a PML of one wavelength (10 points at 10 points
    per wavelength) the bulk solution with C = 16 ln(omega) agrees with a thick-PML reference
    far better than with 4 ln(omega) or the literal ln(omega): the reading of the default C."""
    n = 63
    omega = 2 * math.pi * n / 10
    f = inputs.four_point_sources(n)

    def bulk(p, C):
        gp = GlobalProblem(np.ones((n + 2 * p,) * 2), omega, n, p, C=C)
        return SparseLU(gp.A).solve(gp.rhs(f)).reshape(gp.m.shape)[p:-p, p:-p]

    ref = bulk(60, 8 * math.log(omega))
    err = {cf: np.linalg.norm(bulk(10, cf * math.log(omega)) - ref) / np.linalg.norm(ref) for cf in (1, 4, 16)}
    assert err[16] < err[4] / 20 < err[1] / 20, err


def test_banded_sparse_and_dense_solvers_agree_2d():
    m = extend_normal(_rand_smooth((17, 20), 6), (6, 5))
    gp = GlobalProblem(m, 40.0, (20, 17), (6, 5), C=5.0)
    b = inputs.complex_normal(gp.size, 7)
    ud = solve_dense(gp.A, b)
    for u in (solve_banded(gp.A, b), SparseLU(gp.A).solve(b)):
        assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-12


def test_banded_sparse_and_dense_solvers_agree_3d():
    m = extend_normal(_rand_smooth((6, 4, 5), 8), 2)
    gp = GlobalProblem(m, 12.0, (5, 4, 6), 2, C=5.0)
    b = inputs.complex_normal(gp.size, 9)
    ud = solve_dense(gp.A, b)
    for u in (solve_banded(gp.A, b), SparseLU(gp.A).solve(b)):
        assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-12
