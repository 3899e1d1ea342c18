"""FWI misfit and its adjoint-state gradient with respect to the squared slowness (oracle; test infrastructure only).

The paper motivates fast Helmholtz solves by full-waveform inversion (Sec. 1); it gives
no formula, so this is the textbook adjoint-state method for eq. LS written out:

    J(m) = 1/2 sum_s || P u_s - d_s ||^2,      A(m) u_s = b_s,
    A(m) = A_0 - omega^2 diag(w m),            w = 1/prod(alpha)  (App. A mass term),
    dJ/dm = omega^2 Re( sum_s lambda_s * w * u_s ),   lambda_s = A^-1 conj(P^T (P u_s - d_s)),

using A = A^T (the symmetric PML form), so A^-H y = conj(A^-1 conj(y)).  P samples the
wavefield at receiver grid points.  m is parameterised on the extended grid; the bulk
gradient is the adjoint of the normal extension (a scatter-add onto the edge points).

Pinned by central finite differences of J (tests/test_oracle_gradient.py).
"""
from __future__ import annotations

import numpy as np

from .direct import SparseLU
from .discretization import GlobalProblem


class FWIProblem:
    def __init__(self, omega, n, n_pml, C, sources_bulk, receivers_ext):
        """receivers_ext: (k, 2) array of (iy, ix) indices on the extended grid."""
        self.omega, self.n, self.n_pml, self.C = omega, n, n_pml, C
        self.sources = np.asarray(sources_bulk)
        self.rec = np.asarray(receivers_ext)

    def _system(self, m_ext):
        gp = GlobalProblem(m_ext, self.omega, self.n, self.n_pml, self.C)
        return gp, SparseLU(gp.A)

    def sample(self, gp, u):
        U = u.reshape(gp.m.shape)
        return U[self.rec[:, 0], self.rec[:, 1]]

    def data(self, m_ext):
        gp, lu = self._system(m_ext)
        return np.stack([self.sample(gp, lu.solve(gp.rhs(f))) for f in self.sources])

    def misfit(self, m_ext, d_obs):
        gp, lu = self._system(m_ext)
        J = 0.0
        for f, d in zip(self.sources, d_obs):
            res = self.sample(gp, lu.solve(gp.rhs(f))) - d
            J += 0.5 * float(np.vdot(res, res).real)
        return J

    def gradient(self, m_ext, d_obs):
        gp, lu = self._system(m_ext)
        w = gp.inv_prod_alpha().ravel()
        J = 0.0
        grad = np.zeros(gp.m.size)
        for f, d in zip(self.sources, d_obs):
            u = lu.solve(gp.rhs(f))
            res = self.sample(gp, u) - d
            J += 0.5 * float(np.vdot(res, res).real)
            adj = np.zeros(gp.m.shape, dtype=np.complex128)
            np.add.at(adj, (self.rec[:, 0], self.rec[:, 1]), res)
            lam = lu.solve(np.conj(adj.ravel()))
            grad += self.omega**2 * np.real(lam * w * u)
        return J, grad.reshape(gp.m.shape)


def restrict_to_bulk(g_ext: np.ndarray, n_pml: int) -> np.ndarray:
    """Adjoint of the normal extension: fold every PML value onto its nearest bulk point."""
    p = n_pml
    g = np.array(g_ext, dtype=np.float64)
    Ny, Nx = g.shape
    ny, nx = Ny - 2 * p, Nx - 2 * p
    out = np.zeros((ny, nx))
    iy = np.clip(np.arange(Ny) - p, 0, ny - 1)
    ix = np.clip(np.arange(Nx) - p, 0, nx - 1)
    np.add.at(out, (iy[:, None], ix[None, :]), g)
    return out
