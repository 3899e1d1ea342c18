"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (relative L2 over the whole vector, and on every subdomain Omega_ij at 10x the bar):
  * y = A x (FP64 stencil)                               1e-13
  * z = M^-1 r, FP64 sweeps (block LU vs SuperLU)        1e-12 (largest measured 1.2e-13)
  * z = M^-1 r, complex64 sweeps                         1e-6 (small cases, largest measured 3.5e-7),
                                                         2e-6 (lens2d and 147-point windows, 6.8e-7)
  * GMRES solve vs the exact solve: 1e-6 (FP64) and 1e-4 (mixed) at tol 1e-8,
    and the true residual computed by the oracle's own matrix <= tol.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle.direct import SparseLU, solve_banded
from oracle.discretization import GlobalProblem, extend_normal
from oracle.fgmres import fgmres
from oracle.gradient import FWIProblem
from oracle.lsweep import LSweep2D
from oracle.scenario4 import Scenario4
from paper_1909_01467_amd import inputs
from paper_1909_01467_amd.lsweeps import LSW_EINVAL, LSW_ENAN, HelmholtzSolve, LswError, Solver, extend_medium
from tests.parity_check import check

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def smooth_medium(nx, ny, seed):
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.arange(1, nx + 1) / (nx + 1), np.arange(1, ny + 1) / (nx + 1))
    a, b, c = rng.uniform(1, 3, 3)
    return 1.0 + 0.3 * np.sin(a * X + b * Y) * np.cos(c * Y)


class Case:
    def __init__(self, name, nx, ny, px, py, q, r, medium="smooth", pl=None, C=None, ppw=10.0):
        self.name = name
        self.nx, self.ny, self.px, self.py, self.q, self.r, self.pl = nx, ny, px, py, q, r, pl
        mb = np.ones((ny, nx)) if medium == "const" else smooth_medium(nx, ny, 5)
        self.m = np.pad(mb, ((py, py), (px, px)), mode="edge")   # problem input, extended by np.pad
        self.h = 1.0 / (nx + 1)
        self.omega = 2 * math.pi * nx / ppw
        self.C = 4 * math.log(self.omega) if C is None else C
        self._oracle = None
        self._gp = None

    @property
    def oracle(self):
        if self._oracle is None:
            self._oracle = LSweep2D(self.m, self.omega, (self.nx, self.ny), (self.px, self.py), self.q, self.r,
                                    self.C, n_pml_local=self.pl, h=self.h)
        return self._oracle

    @property
    def gp(self):
        if self._gp is None:
            self._gp = GlobalProblem(self.m, self.omega, (self.nx, self.ny), (self.px, self.py), self.C, h=self.h)
        return self._gp

    def solver(self, **kw):
        say(self.name, kw)
        return Solver(torch.from_numpy(self.m).cuda(), self.omega, self.h, (self.nx, self.ny), (self.px, self.py),
                      self.q, self.r, C=self.C, n_pml_local=self.pl, **kw)

    @property
    def N(self):
        return self.m.size


CASES = {
    "const127_4x4": Case("const127_4x4", 127, 127, 10, 10, 4, 4, medium="const"),
    "ragged_45x38_3x2": Case("ragged_45x38_3x2", 45, 38, 5, 4, 3, 2),
    "single_1x1": Case("single_1x1", 30, 26, 6, 6, 1, 1),
    "row_1x3": Case("row_1x3", 50, 21, 5, 5, 1, 3),
    "col_3x1": Case("col_3x1", 21, 50, 5, 5, 3, 1),
    "thin_local_pml": Case("thin_local_pml", 64, 64, 8, 8, 3, 3, pl=3),
    "no_pml": Case("no_pml", 33, 29, 0, 0, 2, 2, C=1.0),
    "wide_4x5": Case("wide_4x5", 150, 131, 10, 10, 4, 5),
    "wide_windows_2x2": Case("wide_windows_2x2", 250, 180, 10, 10, 2, 2),   # windows 147 x 112
    "widest_windows_2x2": Case("widest_windows_2x2", 280, 90, 10, 10, 2, 2),   # windows 162 x 67
}


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a).ravel() - np.asarray(b).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def to_np(t):
    return t.detach().cpu().numpy().ravel()


@pytest.mark.parametrize("name", ["const127_4x4", "ragged_45x38_3x2", "no_pml"])
def test_matvec_matches_oracle(name):
    c = CASES[name]
    x = inputs.complex_normal(c.N, 1)
    s = c.solver()
    y = s.matvec(torch.from_numpy(x).cuda())
    assert rel(to_np(y), c.gp.A @ x) < 1e-13
    s.close()


@pytest.mark.parametrize("mode", ["compressed", "chain"])
@pytest.mark.parametrize("name", list(CASES))
def test_apply_fp64_matches_oracle(name, mode):
    c = CASES[name]
    r = inputs.complex_normal(c.N, 2)
    s = c.solver(sweep_mode=mode)
    z = to_np(s.apply(torch.from_numpy(r).cuda()))
    zo = c.oracle.apply(r)
    check(f"{name} {mode} apply fp64", z, zo, 1e-12, cdd=c.oracle, shape=c.m.shape)
    s.close()


def test_apply_single_subdomain_is_exact_inverse():
    c = CASES["single_1x1"]
    b = inputs.complex_normal(c.N, 3)
    s = c.solver()
    z = to_np(s.apply(torch.from_numpy(b).cuda()))
    check("single_1x1 apply = A^-1", z, solve_banded(c.gp.A, b), 1e-12)
    s.close()


@pytest.mark.parametrize("mode", ["compressed", "chain"])
@pytest.mark.parametrize("name", ["const127_4x4", "ragged_45x38_3x2", "wide_4x5"])
def test_apply_mixed_matches_oracle(name, mode):
    c = CASES[name]
    r = inputs.complex_normal(c.N, 4)
    s = c.solver(precision="mixed", sweep_mode=mode)
    z = to_np(s.apply(torch.from_numpy(r).cuda()))
    check(f"{name} {mode} apply mixed", z, c.oracle.apply(r), 1e-6, cdd=c.oracle, shape=c.m.shape)
    s.close()


@pytest.mark.parametrize("mode", ["compressed", "chain"])
def test_apply_is_deterministic_and_batches_rhs_exactly(mode, monkeypatch):
    """One right-hand side per workgroup: a batch is bitwise the single applications, and
    repeated applications are bitwise equal (the batched-workgroup kernels are compared to
    tolerance in test_batched_substitutions_carry_several_rhs_per_workgroup)."""
    monkeypatch.setenv("LSW_RHS_PER_WORKGROUP", "1")
    c = CASES["ragged_45x38_3x2"]
    R = inputs.complex_normal((3, c.N), 5)
    s = c.solver(nrhs_max=3, sweep_mode=mode)
    Rt = torch.from_numpy(R).cuda()
    Z = s.apply(Rt)
    Z2 = s.apply(Rt)
    assert torch.equal(Z, Z2)
    for k in range(3):
        assert torch.equal(Z[k].reshape(-1), s.apply(Rt[k]).reshape(-1))
    s.close()


def test_solve_const2d_matches_direct_solve_fp64():
    """127^2, 4x4, centre source: tol 1e-6 in 3 iterations and 1e-8 in 4, as the oracle."""
    c = CASES["const127_4x4"]
    wl = inputs.workload("const2d")
    b = c.gp.rhs(wl.sources[0])
    u_ref = solve_banded(c.gp.A, b)
    bt = torch.from_numpy(b).cuda()
    for tol, its in ((1e-6, 3), (1e-8, 4)):
        s = c.solver(tol=tol)
        u, info = s.solve(bt)
        un = to_np(u)
        say("const2d fp64", tol, info)
        assert info["converged"] == [True] and info["iterations"] == [its]
        assert np.linalg.norm(b - c.gp.A @ un) / np.linalg.norm(b) <= tol
        if tol == 1e-8:
            assert rel(un, u_ref) < 1e-6
        s.close()


def test_solve_const2d_mixed_precision():
    c = CASES["const127_4x4"]
    wl = inputs.workload("const2d")
    b = c.gp.rhs(wl.sources[0])
    u_ref = solve_banded(c.gp.A, b)
    s = c.solver(precision="mixed", tol=1e-8)
    u, info = s.solve(torch.from_numpy(b).cuda())
    un = to_np(u)
    say("const2d mixed", info)
    assert info["converged"] == [True] and info["iterations"][0] <= 6
    assert np.linalg.norm(b - c.gp.A @ un) / np.linalg.norm(b) <= 1e-8
    assert rel(un, u_ref) < 1e-4
    s.close()


def test_solve_iterations_match_oracle_fgmres():
    c = CASES["ragged_45x38_3x2"]
    b = inputs.complex_normal(c.N, 6)
    res = fgmres(lambda v: c.gp.A @ v, c.oracle.apply, b, tol=1e-8)
    s = c.solver(tol=1e-8)
    u, info = s.solve(torch.from_numpy(b).cuda())
    assert info["iterations"] == [res.iterations]
    assert rel(to_np(u), res.x) < 1e-7
    s.close()


def test_multi_rhs_solve_matches_single_solves():
    c = CASES["ragged_45x38_3x2"]
    B = inputs.complex_normal((2, c.N), 7)
    s = c.solver(tol=1e-9, nrhs_max=2)
    U, info = s.solve(torch.from_numpy(B).cuda())
    for k in range(2):
        u1, i1 = s.solve(torch.from_numpy(B[k]).cuda())
        assert i1["iterations"][0] == info["iterations"][k]
        assert rel(to_np(U[k]), to_np(u1)) < 1e-12
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gram_schmidt_in_three_sweeps_equals_four(monkeypatch, precision):
    """Classical Gram-Schmidt with reorthogonalisation in three sweeps over the Krylov basis (the
    first update fused with the second pass's dot products, up to 24 basis vectors) against the four
    separate sweeps (LSW_FUSED_GS=0): the same sums in the same order, so bitwise the same iterates.
    Without PML (C = 1) the solve takes 32 iterations in one restart cycle of 40, so the later
    steps cross over to the four-sweep form."""
    c = CASES["no_pml"]
    B = inputs.complex_normal((3, c.N), 6)
    # the same substitution and sweep kernels in both solvers (the setup tuners time them and may
    # pick different shapes, whose FP32 sums differ in order)
    monkeypatch.setenv("LSW_SYM_CONFIG", "0" if precision == "mixed" else "7")
    monkeypatch.setenv("LSW_RHS_PER_WORKGROUP", "1")
    monkeypatch.setenv("LSW_GEMV_MMA", "0")
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("LSW_FUSED_GS", mode)
        s = c.solver(tol=1e-10, restart=40, nrhs_max=3, precision=precision)
        U, info = s.solve(torch.from_numpy(B).cuda())
        out[mode] = (U.cpu().numpy(), info["iterations"])
        s.close()
    monkeypatch.delenv("LSW_FUSED_GS", raising=False)
    say("gram-schmidt", precision, "iterations", out["1"][1])
    assert out["1"][1] == out["0"][1]
    assert max(out["1"][1]) > 24
    assert np.array_equal(out["1"][0], out["0"][0])
    if precision == "fp64":
        res = fgmres(lambda v: c.gp.A @ v, c.oracle.apply, B[0], tol=1e-10, restart=40)
        assert out["1"][1][0] == res.iterations
        assert rel(out["1"][0][0], res.x) < 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gram_schmidt_update_sums_its_own_coefficients(monkeypatch, precision):
    """The four-sweep Gram-Schmidt passes with the coefficients summed from the dot products'
    workgroup partials inside the update (up to 64 basis vectors) against a finishing launch for
    every sum (LSW_GS_FINISH_MAX=0, the form beyond 64 basis vectors): the same partials added in
    the same order, so bitwise the same iterates (32 steps in one restart cycle)."""
    c = CASES["no_pml"]
    B = inputs.complex_normal((3, c.N), 7)
    monkeypatch.setenv("LSW_SYM_CONFIG", "0" if precision == "mixed" else "7")
    monkeypatch.setenv("LSW_RHS_PER_WORKGROUP", "1")
    monkeypatch.setenv("LSW_GEMV_MMA", "0")
    monkeypatch.setenv("LSW_FUSED_GS", "0")
    out = {}
    for mode in ("0", "64"):
        monkeypatch.setenv("LSW_GS_FINISH_MAX", mode)
        s = c.solver(tol=1e-10, restart=40, nrhs_max=3, precision=precision)
        U, info = s.solve(torch.from_numpy(B).cuda())
        out[mode] = (U.cpu().numpy(), info["iterations"])
        s.close()
    monkeypatch.delenv("LSW_GS_FINISH_MAX", raising=False)
    say("gram-schmidt coefficients in the update", precision, "iterations", out["64"][1])
    assert out["64"][1] == out["0"][1]
    assert max(out["64"][1]) > 24
    assert np.array_equal(out["64"][0], out["0"][0])
    if precision == "fp64":
        res = fgmres(lambda v: c.gp.A @ v, c.oracle.apply, B[0], tol=1e-10, restart=40)
        assert out["64"][1][0] == res.iterations
        assert rel(out["64"][0][0], res.x) < 1e-8


@pytest.mark.parametrize("restart", [2, 3])
def test_restarted_fgmres_follows_the_oracle_across_cycles(restart):
    """FGMRES(restart) over several restart cycles (the thin local PML case takes 7 iterations with
    either restart, the oracle's as well) against the oracle's FGMRES with the same restart: the
    same iteration count and solution, each cycle starting again from the true residual (FP64)."""
    c = CASES["thin_local_pml"]
    b = inputs.complex_normal(c.N, 9)
    s = c.solver(tol=1e-10, restart=restart, maxit=100, precision="fp64")
    u, info = s.solve(torch.from_numpy(b).cuda())
    s.close()
    res = fgmres(lambda v: c.gp.A @ v, c.oracle.apply, b, tol=1e-10, restart=restart, maxit=100)
    say("restarted fgmres", restart, "iterations", info["iterations"], "oracle", res.iterations)
    assert info["converged"] == [True] and res.converged
    assert info["iterations"][0] > 2 * restart
    assert info["iterations"][0] == res.iterations
    assert rel(to_np(u), res.x) < 1e-8


def test_adjoint_solves_the_conjugate_transpose_system():
    c = CASES["ragged_45x38_3x2"]
    g = inputs.complex_normal(c.N, 8)
    s = c.solver(tol=1e-10)
    v, info = s.adjoint(torch.from_numpy(g).cuda())
    assert info["converged"] == [True]
    v_ref = np.conj(solve_banded(c.gp.A, np.conj(g)))
    assert rel(to_np(v), v_ref) < 1e-7
    s.close()


def test_noconvergence_returns_last_iterate():
    c = CASES["ragged_45x38_3x2"]
    b = inputs.complex_normal(c.N, 9)
    s = c.solver(tol=1e-12, maxit=1)
    u, info = s.solve(torch.from_numpy(b).cuda())
    assert info["converged"] == [False] and info["iterations"] == [1]
    assert 0 < info["relres"][0] < 1
    s.close()


def test_input_errors():
    c = CASES["ragged_45x38_3x2"]
    m = torch.from_numpy(c.m).cuda().clone()
    m[3, 4] = float("nan")
    with pytest.raises(LswError) as e:
        Solver(m, c.omega, c.h, (c.nx, c.ny), (c.px, c.py), c.q, c.r)
    assert e.value.code == LSW_ENAN
    s = c.solver(nrhs_max=1)
    with pytest.raises(ValueError):
        s.apply(torch.zeros(2, c.N, dtype=torch.complex128, device="cuda"))
    rc = s._lib.lsw_apply(s._h, None, None, 1)
    assert rc == LSW_EINVAL
    s.close()


def test_fwi_gradient_matches_oracle_and_finite_differences():
    n, p, q = 40, 6, 2
    omega = 2 * math.pi * n / 10
    C = 4 * math.log(omega)
    srcs = np.stack([inputs.gaussian_source(n, (x, 0.8)) for x in (0.3, 0.7)])
    rec = inputs.receiver_indices(n, np.linspace(0.1, 0.9, 9), 0.75) + p
    prob = FWIProblem(omega, n, p, C, srcs, rec)
    mb_true = 1.0 / inputs.speed_lens_blobs(n) ** 2
    mb0 = 1.0 / inputs.speed_lens(n, 2) ** 2
    d_obs = prob.data(extend_normal(mb_true, p))
    J_ref, g_ref = prob.gradient(extend_normal(mb0, p), d_obs)

    kw = dict(omega=omega, h=1.0 / (n + 1), n=n, n_pml=p, q=q, r=q, C=C, tol=1e-12, nrhs_max=2)
    m_t = torch.from_numpy(mb0).cuda().requires_grad_(True)
    m_ext = extend_medium(m_t, p)
    gp = GlobalProblem(extend_normal(mb0, p), omega, n, p, C)
    F = torch.from_numpy(np.stack([gp.rhs(f) for f in srcs])).cuda()
    U = HelmholtzSolve.apply(m_ext, F, kw)
    Uf = U.reshape(2, n + 2 * p, n + 2 * p)
    rec_t = torch.from_numpy(rec).cuda()
    res = Uf[:, rec_t[:, 0], rec_t[:, 1]] - torch.from_numpy(d_obs).cuda()
    J = 0.5 * (res.abs() ** 2).sum()
    J.backward()
    assert abs(J.item() - J_ref) / J_ref < 1e-9
    # oracle gradient on the extended grid folded onto the bulk (adjoint of the extension)
    from oracle.gradient import restrict_to_bulk
    gb_ref = restrict_to_bulk(g_ref, p)
    err = rel(m_t.grad.cpu().numpy(), gb_ref)
    say("fwi gradient rel err", err)
    assert err < 1e-7


def test_helmholtz_solve_passes_gradcheck_on_a_tiny_grid():
    """torch.autograd.gradcheck of a real misfit through HelmholtzSolve, with respect to the bulk
    squared slowness (real) and the right-hand side (complex): checks the adjoint backward and
    PyTorch's conjugate-Wirtinger convention for the complex input against finite differences."""
    n, p, q = 10, 4, 2
    omega = 2 * math.pi * n / 10
    kw = dict(omega=omega, h=1.0 / (n + 1), n=n, n_pml=p, q=q, r=q, C=16 * math.log(omega), tol=1e-13,
              precision="fp64")
    N = n + 2 * p
    rec = torch.tensor([[p + 2, p + 1], [p + 5, p + 7], [p + 8, p + 3]], device="cuda")
    d = torch.from_numpy(inputs.complex_normal(3, 31)).cuda()

    def misfit(mb, f):
        U = HelmholtzSolve.apply(extend_medium(mb, p), f, kw).reshape(N, N)
        return 0.5 * ((U[rec[:, 0], rec[:, 1]] - d).abs() ** 2).sum()

    mb = torch.from_numpy(1.0 / inputs.speed_lens(n, 2) ** 2).cuda().requires_grad_(True)
    f = torch.from_numpy(inputs.complex_normal((N, N), 32)).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(misfit, (mb, f), eps=1e-6, atol=1e-7, rtol=1e-5, fast_mode=True)


@pytest.mark.parametrize("precision,tol_err", [("fp64", 1e-6), ("mixed", 1e-4)])
def test_lens2d_full_size_solve(precision, tol_err):
    """511^2, 8x8 CDD, lens + 5% smooth noise (the benchmark workload) at tol 1e-8."""
    wl = inputs.workload("lens2d")
    m = extend_normal(wl.slowness2, wl.n_pml)
    gp = GlobalProblem(m, wl.omega, wl.n, wl.n_pml, wl.C)
    b = gp.rhs(wl.sources[0])
    say("lens2d", precision)
    s = Solver(torch.from_numpy(m).cuda(), wl.omega, wl.h, wl.n, wl.n_pml, wl.q, wl.r, C=wl.C,
               precision=precision, tol=1e-8)
    u, info = s.solve(torch.from_numpy(b).cuda())
    un = to_np(u)
    say("lens2d", precision, info)
    assert info["converged"] == [True]
    assert np.linalg.norm(b - gp.A @ un) / np.linalg.norm(b) <= 1e-8
    u_ref = SparseLU(gp.A).solve(b)
    assert rel(un, u_ref) < tol_err
    s.close()


def test_lens2d_full_size_apply_matches_oracle():
    wl = inputs.workload("lens2d")
    m = extend_normal(wl.slowness2, wl.n_pml)
    r = inputs.complex_normal(m.size, 10)
    ls = LSweep2D(m, wl.omega, wl.n, wl.n_pml, wl.q, wl.r, wl.C)
    zo = ls.apply(r)
    for mode in ("compressed", "chain"):
        for precision, tol in (("fp64", 1e-12), ("mixed", 2e-6)):
            s = Solver(torch.from_numpy(m).cuda(), wl.omega, wl.h, wl.n, wl.n_pml, wl.q, wl.r, C=wl.C,
                       precision=precision, sweep_mode=mode)
            check(f"lens2d apply {mode} {precision}", to_np(s.apply(torch.from_numpy(r).cuda())), zo, tol,
                  cdd=ls, shape=m.shape)
            s.close()


def test_sweep_modes_agree():
    """The trace-compressed and the chained sweeps are two implementations of the same M^-1."""
    c = CASES["wide_4x5"]
    r = torch.from_numpy(inputs.complex_normal(c.N, 12)).cuda()
    a = c.solver(sweep_mode="compressed")
    b = c.solver(sweep_mode="chain")
    za, zb = to_np(a.apply(r)), to_np(b.apply(r))
    assert rel(za, zb) < 1e-11
    a.close()
    b.close()


def test_lazy_conjugate_views_are_materialised():
    c = CASES["ragged_45x38_3x2"]
    x = torch.from_numpy(inputs.complex_normal(c.N, 11)).cuda()
    s = c.solver()
    assert torch.equal(s.apply(torch.conj(x)), s.apply(torch.conj_physical(x)))
    s.close()


@pytest.mark.parametrize("R", [1, 2, 4, 16, 32])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_substitutions_carry_several_rhs_per_workgroup(R, precision, monkeypatch):
    """R right-hand sides per workgroup of the stage-1 / final substitutions (every factor
    block read once per group; R = 16 and 32 on matrix cores, 32 in complex64 only) give the same
    applications as one right-hand side at a time."""
    if R == 32 and precision == "fp64":
        pytest.skip("32 right-hand sides per workgroup are a complex64 configuration")
    c = CASES["wide_4x5"]
    X = torch.from_numpy(np.stack([inputs.complex_normal(c.N, 70 + k) for k in range(5)])).cuda()
    monkeypatch.setenv("LSW_RHS_PER_WORKGROUP", str(R))
    s = c.solver(precision=precision, nrhs_max=5)
    assert s.stats()["rhs_per_workgroup"] == R
    Z = s.apply(X).cpu().numpy().reshape(5, -1)
    singles = np.stack([s.apply(X[k:k + 1]).cpu().numpy().ravel() for k in range(5)])
    s.close()
    # R = 1 runs on the packed symmetric blocks, R > 1 on the full blocks: the two agree to rounding
    for k in range(5):
        assert rel(Z[k], singles[k]) < (1e-12 if precision == "fp64" else 2e-6), (R, k)
    zo = c.oracle.apply(X[2].cpu().numpy())
    check(f"wide_4x5 R={R} batched apply {precision}", Z[2], zo, 1e-12 if precision == "fp64" else 1e-6,
          cdd=c.oracle, shape=c.m.shape)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
@pytest.mark.parametrize("name", ["ragged_45x38_3x2", "wide_4x5", "thin_local_pml", "row_1x3"])
def test_packed_symmetric_factors_match_full_blocks(name, precision, tol, monkeypatch):
    """The substitutions on the packed symmetric blocks (odd and even window widths, several
    right-hand sides, one per workgroup) give the applications of the full blocks."""
    c = CASES[name]
    X = torch.from_numpy(inputs.complex_normal((2, c.N), 6)).cuda()
    monkeypatch.setenv("LSW_RHS_PER_WORKGROUP", "1")
    s = c.solver(precision=precision, nrhs_max=2)
    st = s.stats()
    assert st["symmetric_factors"] == 1 and st["packed_factor_elems"] > 0
    Z = s.apply(X).cpu().numpy().reshape(2, -1)
    s.close()
    monkeypatch.setenv("LSW_SYMMETRIC_FACTORS", "0")
    s = c.solver(precision=precision, nrhs_max=2)
    assert s.stats()["symmetric_factors"] == 0
    Z0 = s.apply(X).cpu().numpy().reshape(2, -1)
    s.close()
    for k in range(2):
        check(f"{name} {precision} packed vs full blocks", Z[k], Z0[k], tol, cdd=c.oracle, shape=c.m.shape)


def test_packed_factors_of_wide_windows(monkeypatch):
    """Windows 147 points wide (three packed tiles per lane in complex64) against the oracle and
    against the full blocks."""
    c = CASES["wide_windows_2x2"]
    X = torch.from_numpy(inputs.complex_normal((2, c.N), 7)).cuda()
    monkeypatch.setenv("LSW_RHS_PER_WORKGROUP", "1")
    s = c.solver(precision="mixed", nrhs_max=2)
    st = s.stats()
    assert st["symmetric_factors"] == 1 and st["W_max"] == 147
    Z = s.apply(X).cpu().numpy().reshape(2, -1)
    s.close()
    monkeypatch.setenv("LSW_SYMMETRIC_FACTORS", "0")
    s = c.solver(precision="mixed", nrhs_max=2)
    Z0 = s.apply(X).cpu().numpy().reshape(2, -1)
    s.close()
    zo = c.oracle.apply(X[0].cpu().numpy())
    for k in range(2):
        check("wide windows packed vs full blocks", Z[k], Z0[k], 2e-6, cdd=c.oracle, shape=c.m.shape)
    check("wide windows packed vs oracle", Z[0], zo, 2e-6, cdd=c.oracle, shape=c.m.shape)


SYM_SHAPE_INDICES = range(10)   # the shapes of the packed substitution kernel (LSW_SYM_CONFIG)


@pytest.mark.parametrize("name,precision,min_shapes", [
    ("ragged_45x38_3x2", "mixed", 7), ("ragged_45x38_3x2", "fp64", 3), ("wide_4x5", "mixed", 5),
    ("wide_windows_2x2", "mixed", 2), ("widest_windows_2x2", "mixed", 1)])
def test_every_packed_kernel_shape_gives_the_oracle_application(name, precision, min_shapes, monkeypatch):
    """Each shape of the one-right-hand-side packed substitutions (lanes per workgroup, tiles per
    lane, ring depth, lanes per row) that the windows fit, forced with LSW_SYM_CONFIG, against the
    oracle's application and against each other; widest_windows_2x2 has windows 162 wide."""
    c = CASES[name]
    X = torch.from_numpy(inputs.complex_normal((2, c.N), 8)).cuda()
    zo = c.oracle.apply(X[1].cpu().numpy())
    monkeypatch.setenv("LSW_RHS_PER_WORKGROUP", "1")
    bar = 1e-12 if precision == "fp64" else 2e-6
    seen = {}
    for i in SYM_SHAPE_INDICES:
        monkeypatch.setenv("LSW_SYM_CONFIG", str(i))
        s = c.solver(precision=precision, nrhs_max=2)
        st = s.stats()
        assert st["symmetric_factors"] == 1
        shape = (st["sym_threads"], st["sym_tiles_per_lane"], st["sym_ring"], st["sym_lanes_per_row"])
        if shape in seen:
            s.close()
            continue
        Z = s.apply(X).cpu().numpy().reshape(2, -1)
        s.close()
        check(f"{name} {precision} packed shape {shape} vs oracle", Z[1], zo, bar, cdd=c.oracle, shape=c.m.shape)
        seen[shape] = Z
    say(name, precision, "shapes", sorted(seen))
    assert len(seen) >= min_shapes
    first = next(iter(seen.values()))
    for shape, Z in seen.items():
        for k in range(2):
            assert rel(Z[k], first[k]) < (1e-13 if precision == "fp64" else 2e-6), (shape, k)


def test_packed_kernel_shape_is_tuned_at_setup(monkeypatch):
    monkeypatch.delenv("LSW_SYM_CONFIG", raising=False)
    c = CASES["const127_4x4"]
    s = c.solver(precision="mixed", nrhs_max=1)
    st = s.stats()
    s.close()
    say("packed shape", st["sym_threads"], st["sym_tiles_per_lane"], st["sym_ring"], st["sym_lanes_per_row"],
        "timed", st["sym_shapes_timed"], st["sym_tune_best_ms"], st["sym_tune_worst_ms"])
    assert st["sym_shapes_timed"] >= 2 and 0 < st["sym_tune_best_ms"] <= st["sym_tune_worst_ms"]


@pytest.mark.parametrize("nrhs", [5, 19])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sweep_levels_on_matrix_cores(nrhs, precision, monkeypatch):
    """The sweep levels of several right-hand sides on matrix cores (LSW_GEMV_MMA=1; 19 right-hand
    sides take two 16-wide groups in complex128 and one 32-wide group in complex64) against the
    batched GEMVs (LSW_GEMV_MMA=0) and the oracle's application."""
    c = CASES["wide_4x5"]
    X = torch.from_numpy(inputs.complex_normal((nrhs, c.N), 10)).cuda()
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("LSW_GEMV_MMA", mode)
        s = c.solver(precision=precision, nrhs_max=nrhs)
        assert s.stats()["gemv_mma"] == int(mode)
        out[mode] = s.apply(X).cpu().numpy().reshape(nrhs, -1)
        s.close()
    bar = 1e-12 if precision == "fp64" else 2e-6
    for k in range(nrhs):
        assert rel(out["1"][k], out["0"][k]) < bar, k
    zo = c.oracle.apply(X[nrhs - 1].cpu().numpy())
    check(f"wide_4x5 {nrhs} rhs sweeps on matrix cores {precision}", out["1"][nrhs - 1], zo, bar,
          cdd=c.oracle, shape=c.m.shape)


def test_sweep_kernel_is_tuned_at_setup(monkeypatch):
    monkeypatch.delenv("LSW_GEMV_MMA", raising=False)
    c = CASES["const127_4x4"]
    s = c.solver(precision="mixed", nrhs_max=8)
    st = s.stats()
    s.close()
    say("sweeps on matrix cores", st["gemv_mma"], st["gemv_tune_ms"])
    assert all(t > 0 for t in st["gemv_tune_ms"])
    assert st["gemv_mma"] == (1 if st["gemv_tune_ms"][1] < st["gemv_tune_ms"][0] else 0)


def test_windows_of_the_largest_width():
    """Windows exactly 256 points wide, the largest the kernels take (257 is refused: test_abi): the
    blocked Gauss-Jordan on 256 x 256 line blocks, the unit solves for Q on matrix cores and the
    full-block substitutions (wider than the packed kernel takes), against the oracle's application
    in both precisions."""
    c = Case("max_window_1x2", 484, 30, 6, 6, 1, 2, pl=6)   # windows of 256 x 42 points
    x = inputs.complex_normal(c.N, 11)
    zo = c.oracle.apply(x)
    for precision, bar in (("fp64", 1e-12), ("mixed", 2e-6)):
        s = c.solver(precision=precision)
        st = s.stats()
        assert st["W_max"] == 256 and st["symmetric_factors"] == 0
        z = s.apply(torch.from_numpy(x).cuda()).cpu().numpy().ravel()
        s.close()
        check(f"max_window_1x2 (W = 256) apply {precision}", z, zo, bar, cdd=c.oracle, shape=c.m.shape)


def test_rhs_per_workgroup_is_tuned_at_setup():
    c = CASES["const127_4x4"]
    s = c.solver(precision="mixed", nrhs_max=8)
    st = s.stats()
    s.close()
    say("tuned R", st["rhs_per_workgroup"], st["tune_ms"])
    assert st["rhs_per_workgroup"] in (1, 2, 4, 16)
    assert all(t > 0 for t in st["tune_ms"][:4]) and st["tune_ms"][4] == 0   # 32 needs more than 16


@pytest.mark.parametrize("windows", [False, True])
def test_workspace_in_the_torch_caching_allocator(windows, monkeypatch):
    """torch_allocator=True: every workspace buffer comes from PyTorch's caching allocator (the
    allocated bytes grow by at least the Krylov basis and return to where they were after close),
    and the results are bitwise those of the hipMalloc workspace (with the packed kernel's shape
    fixed, since the setup tuner of either solver may pick another shape, whose sums differ in order)."""
    monkeypatch.setenv("LSW_SYM_CONFIG", "7")
    c = CASES["ragged_45x38_3x2"]
    r = torch.from_numpy(inputs.complex_normal(c.N, 61)).cuda()
    b = torch.from_numpy(inputs.complex_normal(c.N, 62)).cuda()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    s = c.solver(torch_allocator=True, windows=windows, tol=1e-8)
    grown = torch.cuda.memory_allocated() - before
    assert grown >= 51 * c.N * 16   # the Krylov basis V alone (restart 50)
    z1 = s.apply(r).cpu()
    u1, i1 = s.solve(b)
    u1 = u1.cpu()
    s.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    s2 = c.solver(windows=windows, tol=1e-8)
    z2 = s2.apply(r).cpu()
    u2, i2 = s2.solve(b)
    u2 = u2.cpu()
    s2.close()
    say("torch allocator", windows, "workspace MB", grown / 1e6, "iterations", i1["iterations"], i2["iterations"])
    assert torch.equal(z1, z2) and torch.equal(u1, u2) and i1["iterations"] == i2["iterations"]


def test_random_geometries_match_oracle():
    """Seeded random grids, PML widths, local PML widths and CDD shapes (ragged splits, thin
    groups, single rows or columns): one FP64 application against the oracle's, 1e-12."""
    rng = np.random.default_rng(2024)
    done = 0
    while done < 10:
        nx, ny = (int(v) for v in rng.integers(16, 80, 2))
        px, py = (int(v) for v in rng.integers(0, 9, 2))
        q, r = (int(v) for v in rng.integers(1, 5, 2))
        pl = None if rng.random() < 0.5 else int(rng.integers(1, max(2, px + 1)))
        c = Case(f"random_{done}", nx, ny, px, py, q, r, pl=pl, C=None if px and py else 1.0)
        try:
            oracle = c.oracle
        except ValueError:   # a group or window that does not fit: the library must refuse it too
            with pytest.raises(LswError):
                c.solver()
            continue
        x = inputs.complex_normal(c.N, 70 + done)
        s = c.solver()
        z = to_np(s.apply(torch.from_numpy(x).cuda()))
        s.close()
        check(f"random geometry {(nx, ny, px, py, q, r, pl)} apply fp64", z, oracle.apply(x), 1e-12,
              cdd=oracle, shape=c.m.shape)
        if q >= 2 and r >= 2 and min(nx // r, ny // q) >= 6:   # scenario 4 with the default shifts
            s4 = Scenario4(c.m, c.omega, (nx, ny), (px, py), q, r, c.C, n_pml_local=pl, h=c.h)
            s = c.solver(windows=True)
            z = to_np(s.apply(torch.from_numpy(x).cuda()))
            s.close()
            check(f"random geometry {(nx, ny, px, py, q, r, pl)}, windows {s4.shift} apply fp64", z, s4.apply(x),
                  1e-12, cdd=oracle, shape=c.m.shape)
        done += 1
