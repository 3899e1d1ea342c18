"""Scenario 4 (Sec. 2.1) on the HIP path through the C ABI, against the FP64 oracle.

Tolerances (relative L2, whole vector and 10x on every subdomain of the unshifted CDD) as for
scenario 3: 1e-12 for the FP64 sweeps, 1e-6 for the complex64 sweeps (largest measured 7.4e-15 and
2.1e-7); the windowed solve reaches the exact solve to 1e-6 at tol 1e-8.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle.direct import SparseLU
from oracle.discretization import GlobalProblem
from oracle.lsweep import LSweep2D
from oracle.scenario4 import Scenario4
from paper_1909_01467_amd import inputs
from paper_1909_01467_amd.lsweeps import Solver
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
    def __init__(self, name, nx, ny, px, py, q, r, medium="smooth", shift=None):
        self.name, self.nx, self.ny, self.px, self.py, self.q, self.r = name, nx, ny, px, py, q, r
        mb = np.ones((ny, nx)) if medium == "const" else smooth_medium(nx, ny, 5)
        self.m = np.pad(mb, ((py, py), (px, px)), mode="edge")
        self.h = 1.0 / (nx + 1)
        self.omega = 2 * math.pi * nx / 10
        self.C = 4 * math.log(self.omega)
        self.shift = shift
        self._oracle = None

    @property
    def N(self):
        return self.m.size

    @property
    def oracle(self):
        if self._oracle is None:
            self._oracle = Scenario4(self.m, self.omega, (self.nx, self.ny), (self.px, self.py), self.q, self.r,
                                     self.C, h=self.h, shift=self.shift)
        return self._oracle

    def solver(self, **kw):
        say(self.name, kw)
        return Solver(torch.from_numpy(self.m).cuda(), self.omega, self.h, (self.nx, self.ny), (self.px, self.py),
                      self.q, self.r, C=self.C, windows=True, shift=self.shift or (0, 0), **kw)


CASES = {
    "const127_4x4": Case("const127_4x4", 127, 127, 10, 10, 4, 4, medium="const"),
    "ragged_45x38_3x2": Case("ragged_45x38_3x2", 45, 38, 5, 4, 3, 2),
    "shift_5x7_wide_4x5": Case("shift_5x7_wide_4x5", 150, 131, 10, 10, 4, 5, shift=(5, 7)),
}


def rel(a, b):
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_np(t):
    return t.detach().cpu().numpy().ravel()


@pytest.mark.parametrize("mode", ["compressed", "chain"])
@pytest.mark.parametrize("name", list(CASES))
def test_windowed_apply_fp64_matches_oracle(name, mode):
    c = CASES[name]
    r = inputs.complex_normal(c.N, 41)
    s = c.solver(sweep_mode=mode)
    st = s.stats()
    assert st["cdd_count"] == 4 and tuple(st["window_shift"]) == c.oracle.shift
    z = to_np(s.apply(torch.from_numpy(r).cuda()))
    check(f"{name} {mode} windowed apply fp64", z, c.oracle.apply(r), 1e-12, cdd=c.oracle.cdds[0],
          shape=c.m.shape)
    s.close()


@pytest.mark.parametrize("name", ["const127_4x4", "ragged_45x38_3x2"])
def test_windowed_apply_mixed_matches_oracle(name):
    c = CASES[name]
    r = inputs.complex_normal(c.N, 42)
    s = c.solver(precision="mixed")
    check(f"{name} windowed apply mixed", to_np(s.apply(torch.from_numpy(r).cuda())), c.oracle.apply(r), 1e-6,
          cdd=c.oracle.cdds[0], shape=c.m.shape)
    s.close()


def test_shifted_cdd_alone_matches_oracle():
    """A single shifted CDD (windows off; one more group along each shifted axis) against the
    oracle's sweep on the same shifted CDD."""
    c = CASES["ragged_45x38_3x2"]
    ls = LSweep2D(c.m, c.omega, (c.nx, c.ny), (c.px, c.py), c.q, c.r, c.C, h=c.h, shift=(7, 4))
    s = Solver(torch.from_numpy(c.m).cuda(), c.omega, c.h, (c.nx, c.ny), (c.px, c.py), c.q, c.r, C=c.C,
               shift=(7, 4))
    r = inputs.complex_normal(c.N, 43)
    check("shifted CDD alone apply fp64", to_np(s.apply(torch.from_numpy(r).cuda())), ls.apply(r), 1e-12,
          cdd=ls, shape=c.m.shape)
    s.close()


def test_windowed_apply_batches_rhs():
    c = CASES["ragged_45x38_3x2"]
    R = inputs.complex_normal((3, c.N), 44)
    s = c.solver(nrhs_max=3)
    Rt = torch.from_numpy(R).cuda()
    Z = s.apply(Rt)
    assert torch.equal(Z, s.apply(Rt))   # the four CDDs run concurrently; the sum order is fixed
    for k in range(3):
        assert rel(to_np(Z[k]), to_np(s.apply(Rt[k]))) < 1e-13
    # the work of the windowed plan is that of its four CDDs built alone
    st = s.stats()
    sx, sy = st["window_shift"]
    alone = [Solver(torch.from_numpy(c.m).cuda(), c.omega, c.h, (c.nx, c.ny), (c.px, c.py), c.q, c.r, C=c.C,
                    shift=sh).stats() for sh in ((0, 0), (sx, 0), (0, sy), (sx, sy))]
    assert [(a["q"], a["r"]) for a in alone] == [(c.q, c.r), (c.q, c.r + 1), (c.q + 1, c.r), (c.q + 1, c.r + 1)]
    for key in ("n_subdomains", "solves_per_apply", "factor_elems", "gemv_items"):
        assert st[key] == sum(a[key] for a in alone), key
    s.close()


@pytest.mark.parametrize("precision,tol_err", [("fp64", 1e-6), ("mixed", 1e-4)])
def test_windowed_solve_of_a_skeleton_source_matches_direct_solve(precision, tol_err):
    """127^2, 4x4, a Gaussian on the CDD's cross point (nonzero on the skeleton): GMRES with the
    windowed preconditioner reaches the exact solve; the iteration counts of both scenarios are
    reported."""
    c = CASES["const127_4x4"]
    gp = GlobalProblem(c.m, c.omega, c.nx, c.px, c.C, h=c.h)
    ls = LSweep2D(c.m, c.omega, c.nx, c.px, c.q, c.r, c.C, h=c.h)
    xc = (ls.xlo[2] - 0.5 - c.px + 1) * c.h
    b = gp.rhs(inputs.gaussian_source(c.nx, (xc, xc)))
    u = SparseLU(gp.A).solve(b)
    its = {}
    for windows in (False, True):
        s = Solver(torch.from_numpy(c.m).cuda(), c.omega, c.h, c.nx, c.px, c.q, c.r, C=c.C, windows=windows,
                   precision=precision, tol=1e-8)
        x, info = s.solve(torch.from_numpy(b).cuda())
        err = rel(to_np(x), u)
        its[windows] = info["iterations"][0]
        say(precision, "windows" if windows else "scenario 3", "iterations", its[windows], "err", err)
        assert info["converged"][0] and err < tol_err
        s.close()
    assert its[True] <= its[False] + 1
