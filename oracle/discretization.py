"""PML-truncated Helmholtz operator, written out plainly (oracle; test infrastructure only).

Follows App. A of the paper:
  * coordinate stretching d/dx_k -> alpha_k d/dx_k, alpha_k = 1/(1 + i sigma_k/omega);
  * cubic profile sigma_k = (C/delta)(dist/delta)^3 outside the bulk, 0 inside;
  * symmetric form  -div(Lambda grad u) - omega^2 m/(prod alpha) u = f/(prod alpha),
    Lambda_kk = alpha_k^2 / prod(alpha)  (2D: s1 = alpha1/alpha2, s2 = alpha2/alpha1);
  * second-order differences with the coefficient taken at half points.
The medium is extended into the PML by its normal (constant) extension (Sec. 1.1).

Readings (where the paper is silent or garbled):
  * grid: n bulk points per axis at x = h..n h, h = 1/(n+1) by default; n_pml extra
    points per side at x = 0, -h, ..., -(n_pml-1)h (and mirrored), Dirichlet ghosts at
    x = -n_pml h and 1 + n_pml h, so delta = n_pml h and the bulk interval is [0, (n+1)h];
  * the undefined beta in Lambda is prod(alpha); the mass term is -omega^2 m/prod(alpha) u;
  * 3D uses the 7-point stencil (second order);
  * C is a parameter (the printed profile absorbs only exp(-C/2) at normal incidence).

The operator is assembled as  A = sum_k D_k^T S_k D_k - diag(omega^2 m / prod alpha),
with D_k the forward difference from grid points to half points along axis k (zero
Dirichlet ghosts) and S_k = diag(Lambda_kk at the half points).  This is the same
5/7-point stencil as App. A, written as a product of sparse factors.

Pins (tests/test_oracle_discretization.py): exact symmetry; n_pml = 0 reduces to the
textbook Dirichlet Laplacian solved in closed form by DST-I (2D and 3D); 1-D normal
incidence reflection equals exp(-C/2); convergence to the free-space Hankel function
at second order; banded vs dense solves.

Arrays are indexed [y, x] (2D) and [z, y, x] (3D); vectors flatten them with x fastest.
Physical axis k = 0, 1, 2 (x, y, z) is array axis d-1-k.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def extend_normal(m_bulk: np.ndarray, n_pml) -> np.ndarray:
    """Normal (constant) extension of the medium into the PML (Sec. 1.1, Fig. 1b)."""
    d = m_bulk.ndim
    p = [n_pml] * d if np.isscalar(n_pml) else list(n_pml)
    # p is given per physical axis (x, y, z); np.pad wants array-axis order
    pad = [(p[d - 1 - a], p[d - 1 - a]) for a in range(d)]
    return np.pad(m_bulk, pad, mode="edge")


def axis_points(n: int, n_pml: int, h: float):
    """Integer points x_a (a = 0..N-1) and half points x_{a-1/2} (a = 0..N) of one axis."""
    N = n + 2 * n_pml
    x_int = (np.arange(N) - n_pml + 1) * h
    x_half = (np.arange(N + 1) - n_pml + 0.5) * h
    return x_int, x_half


def cubic_sigma(x: np.ndarray, left: float, right: float, delta: float, C: float) -> np.ndarray:
    """App. A profile: (C/delta)((distance outside [left, right])/delta)^3."""
    if delta <= 0.0:
        return np.zeros_like(x)
    dist = np.maximum(0.0, np.maximum(left - x, x - right))
    return (C / delta) * (dist / delta) ** 3


def alpha_of(sigma: np.ndarray, omega: float) -> np.ndarray:
    """App. A: alpha = 1/(1 + i sigma/omega)."""
    return 1.0 / (1.0 + 1j * sigma / omega)


def diff_matrix(N: int, h: float) -> sp.csr_matrix:
    """Forward difference onto the N+1 half points: (Du)_{a-1/2} = (u_a - u_{a-1})/h, u_{-1} = u_N = 0."""
    main = np.full(N, 1.0 / h)
    low = np.full(N, -1.0 / h)
    return sp.diags([main, low], [0, -1], shape=(N + 1, N), format="csr")


def assemble(alpha_int, alpha_half, m_box: np.ndarray, omega: float, h: float) -> sp.csr_matrix:
    """Assemble A on a box with zero Dirichlet data just outside it.

    alpha_int[k]  : alpha of physical axis k at the box's integer points (length N_k)
    alpha_half[k] : alpha of axis k at the box's half points (length N_k + 1)
    m_box         : squared slowness on the box (array order z, y, x)
    """
    d = m_box.ndim
    shape = m_box.shape                       # array order
    Ns = [shape[d - 1 - k] for k in range(d)]  # physical order
    A = None
    for k in range(d):
        t = d - 1 - k                          # array axis of physical axis k
        factors = []
        for a in range(d):
            if a == t:
                factors.append(diff_matrix(shape[a], h))
            else:
                factors.append(sp.identity(shape[a], format="csr"))
        Dk = factors[0]
        for f in factors[1:]:
            Dk = sp.kron(Dk, f, format="csr")
        # Lambda_kk = alpha_k(half) / prod_{l != k} alpha_l(int), on the half-point grid of axis k
        coeff = np.ones([shape[a] + (1 if a == t else 0) for a in range(d)], dtype=np.complex128)
        for l in range(d):
            al = d - 1 - l
            bshape = [1] * d
            if l == k:
                bshape[al] = Ns[l] + 1
                coeff = coeff * np.asarray(alpha_half[l]).reshape(bshape)
            else:
                bshape[al] = Ns[l]
                coeff = coeff / np.asarray(alpha_int[l]).reshape(bshape)
        term = Dk.T @ sp.diags(coeff.ravel()) @ Dk
        A = term if A is None else A + term
    prod_alpha = np.ones(shape, dtype=np.complex128)
    for l in range(d):
        bshape = [1] * d
        bshape[d - 1 - l] = Ns[l]
        prod_alpha = prod_alpha * np.asarray(alpha_int[l]).reshape(bshape)
    mass = omega**2 * m_box / prod_alpha
    return (A - sp.diags(mass.ravel())).tocsr()


class GlobalProblem:
    """The PML-extended global system A u = b (eq. LS) on the extended grid."""

    def __init__(self, m_ext: np.ndarray, omega: float, n, n_pml, C: float, h: float | None = None):
        self.d = m_ext.ndim
        d = self.d
        self.n = [n] * d if np.isscalar(n) else list(n)
        self.n_pml = [n_pml] * d if np.isscalar(n_pml) else list(n_pml)
        self.h = 1.0 / (self.n[0] + 1) if h is None else h
        self.omega = omega
        self.C = C
        self.m = np.asarray(m_ext, dtype=np.float64)
        self.N = [self.n[k] + 2 * self.n_pml[k] for k in range(d)]
        assert tuple(self.N[::-1]) == self.m.shape, (self.N, self.m.shape)
        self.x_int, self.x_half, self.sig_int, self.sig_half = [], [], [], []
        for k in range(d):
            xi, xh = axis_points(self.n[k], self.n_pml[k], self.h)
            L = (self.n[k] + 1) * self.h
            delta = self.n_pml[k] * self.h
            self.x_int.append(xi)
            self.x_half.append(xh)
            self.sig_int.append(cubic_sigma(xi, 0.0, L, delta, C))
            self.sig_half.append(cubic_sigma(xh, 0.0, L, delta, C))
        self.alpha_int = [alpha_of(s, omega) for s in self.sig_int]
        self.alpha_half = [alpha_of(s, omega) for s in self.sig_half]
        self.A = assemble(self.alpha_int, self.alpha_half, self.m, omega, self.h)

    @property
    def size(self) -> int:
        return int(np.prod(self.N))

    def inv_prod_alpha(self) -> np.ndarray:
        """w = 1/prod(alpha) on the grid (1 in the bulk): the weight of m in the mass term."""
        d = self.d
        w = np.ones(self.m.shape, dtype=np.complex128)
        for l in range(d):
            bshape = [1] * d
            bshape[d - 1 - l] = self.N[l]
            w = w / self.alpha_int[l].reshape(bshape)
        return w

    def rhs(self, f_bulk: np.ndarray) -> np.ndarray:
        """b = f/prod(alpha) with f extended by zero into the PML (= f there)."""
        pad = [(self.n_pml[self.d - 1 - a],) * 2 for a in range(self.d)]
        f_ext = np.pad(np.asarray(f_bulk, dtype=np.complex128), pad)
        return (f_ext * self.inv_prod_alpha()).ravel()
