"""L-sweeps for the 3D problem over a beam CDD (oracle; test infrastructure only).

The 3D discretisation is the 7-point form of App. A (oracle.discretization.assemble with
three axes).  The checkerboard decomposition is the 2D one of Sec. 2 applied in (x, y);
every subdomain is a beam over the full extended z range, so its local problem keeps the
global PML at both z ends and adds local PML only on its interior x/y sides (the beam
reading of the 3D example of Sec. 5).  Alg. Scenario3 is then unchanged: the traces are
the two grid planes on either side of each vertical interface (two lines of the 2D CDD
times all z), the receiving region chi of a subdomain is the 2D half plane or quadrant
times all z, and the polarized sources follow eq. DiscPol2 with the neighbours of the
7-point stencil (the z neighbours never cross the boundary of chi).

Arrays are indexed [z, y, x] (x fastest).  Trace arrays hold [line, z, along-side index].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import alpha_of, assemble, axis_points, cubic_sigma
from .lsweep import SIDES, LSweep2D, partition


class LSweep3D(LSweep2D):
    """Alg. Scenario3 for a q x r beam CDD of a 3D box (n_x, n_y, n_z bulk points); `shift` as for
    LSweep2D (the shifted CDDs of scenario 4, in x and y)."""

    def __init__(self, m_ext: np.ndarray, omega: float, n, n_pml, q: int, r: int, C: float,
                 n_pml_local: int | None = None, h: float | None = None, shift=(0, 0)):
        nx, ny, nz = (n, n, n) if np.isscalar(n) else n
        px, py, pz = (n_pml, n_pml, n_pml) if np.isscalar(n_pml) else n_pml
        self.nx, self.ny, self.nz, self.px, self.py, self.pz = nx, ny, nz, px, py, pz
        self.h = 1.0 / (nx + 1) if h is None else h
        self.omega, self.C = omega, C
        self.q, self.r = q, r
        self.pl = px if n_pml_local is None else n_pml_local
        self.e = 2 + self.pl
        self.m = np.asarray(m_ext, dtype=np.float64)
        self.Nex, self.Ney, self.Nez = nx + 2 * px, ny + 2 * py, nz + 2 * pz
        assert self.m.shape == (self.Nez, self.Ney, self.Nex)
        self.shift = tuple(shift)
        self.xlo, self.xhi, _ = partition(nx, px, r, self.shift[0])
        self.ylo, self.yhi, _ = partition(ny, py, q, self.shift[1])
        q, r = self.q, self.r = len(self.ylo), len(self.xlo)   # a shifted axis has one more group
        for lo, hi, N in ((self.xlo, self.xhi, self.Nex), (self.ylo, self.yhi, self.Ney)):
            for g in range(len(lo)):
                if hi[g] - lo[g] < 2 or (g > 0 and lo[g] < self.e) or \
                        (g < len(lo) - 1 and hi[g] + self.e > N):
                    raise ValueError("each group needs 2 points and its window must fit in the grid")
        self.xw = [self._window(self.xlo, self.xhi, j, r, self.Nex) for j in range(r)]
        self.yw = [self._window(self.ylo, self.yhi, i, q, self.Ney) for i in range(q)]
        self.ax = [self._axis_alpha(nx, px, self.xlo, self.xhi, j, r, self.xw[j]) for j in range(r)]
        self.ay = [self._axis_alpha(ny, py, self.ylo, self.yhi, i, q, self.yw[i]) for i in range(q)]
        # z: the beam spans the whole extended range, global PML only
        zi, zh = axis_points(nz, pz, self.h)
        Lz, dz = (nz + 1) * self.h, pz * self.h
        self.az = (alpha_of(cubic_sigma(zi, 0.0, Lz, dz, C), omega), alpha_of(cubic_sigma(zh, 0.0, Lz, dz, C), omega))
        self.A, self.lu = {}, {}
        for i in range(q):
            for j in range(r):
                (y0, y1), (x0, x1) = self.yw[i], self.xw[j]
                A = assemble([self.ax[j][0], self.ay[i][0], self.az[0]], [self.ax[j][1], self.ay[i][1], self.az[1]],
                             self.m[:, y0:y1, x0:x1], omega, self.h)
                self.A[i, j] = A.tocsr()
                self.lu[i, j] = spla.splu(sp.csc_matrix(A))
        self._coupling = {}
        self.solves = 0

    # ------------------------------------------------------------------ geometry
    def shape(self, i, j):
        (y0, y1), (x0, x1) = self.yw[i], self.xw[j]
        return (self.Nez, y1 - y0, x1 - x0)

    def mask2d(self, i, j, kind):
        """chi in the (y, x) cross-section: the half plane or quadrant receiving the wave."""
        _, H, W = self.shape(i, j)
        (r0, r1), (c0, c1) = self.omega_box(i, j)
        rows = np.arange(H)[:, None]
        cols = np.arange(W)[None, :]
        m = np.ones((H, W), dtype=bool)
        if "B" in kind:
            m &= rows >= r0
        if "T" in kind:
            m &= rows < r1
        if "L" in kind:
            m &= cols >= c0
        if "R" in kind:
            m &= cols < c1
        return m

    def receiving_mask(self, i, j, kind):
        return np.broadcast_to(self.mask2d(i, j, kind), self.shape(i, j)).copy()

    # ------------------------------------------------------------------ primitives
    def extract(self, u, i, j):
        Nz, H, W = self.shape(i, j)
        out = {}
        for s in SIDES:
            if s in ("B", "T"):
                t = np.zeros((2, Nz, W), dtype=np.complex128)
                if self.has_side(i, j, s):
                    a, b = self.lines(i, j, s)
                    t[0], t[1] = u[:, a, :], u[:, b, :]
            else:
                t = np.zeros((2, Nz, H), dtype=np.complex128)
                if self.has_side(i, j, s):
                    a, b = self.lines(i, j, s)
                    t[0], t[1] = u[:, :, a], u[:, :, b]
            out[s] = t
        return out

    def solve_local(self, i, j, g):
        self.solves += 1
        return self.lu[i, j].solve(g.ravel()).reshape(self.shape(i, j))

    def straight_field(self, i, j, side, lam):
        ut = np.zeros(self.shape(i, j), dtype=np.complex128)
        a, b = self.lines(i, j, side)
        if side in ("B", "T"):
            ut[:, a, :], ut[:, b, :] = lam[0], lam[1]
        else:
            ut[:, :, a], ut[:, :, b] = lam[0], lam[1]
        return ut

    def corner_field(self, i, j, hside, hlam, vside, vlam):
        """L-shaped interface times all z: legs restricted to the quadrant, horizontal leg wins."""
        ut = np.zeros(self.shape(i, j), dtype=np.complex128)
        chi = self.mask2d(i, j, hside + vside)
        rows_in = chi.any(axis=1)
        cols_in = chi.any(axis=0)
        a, b = self.lines(i, j, vside)
        ut[:, rows_in, a] = vlam[0][:, rows_in]
        ut[:, rows_in, b] = vlam[1][:, rows_in]
        a, b = self.lines(i, j, hside)
        ut[:, a, cols_in] = hlam[0][:, cols_in]
        ut[:, b, cols_in] = hlam[1][:, cols_in]
        return ut

    def _zeros_like_sides(self, sides):
        out = {}
        for s in sides:
            d = {}
            for i in range(self.q):
                for j in range(self.r):
                    Nz, H, W = self.shape(i, j)
                    d[i, j] = np.zeros((2, Nz, W if s in ("B", "T") else H), dtype=np.complex128)
            out[s] = d
        return out

    # ------------------------------------------------------------------ Alg. Scenario3
    def apply(self, rvec: np.ndarray) -> np.ndarray:
        q, r = self.q, self.r
        R = np.asarray(rvec, dtype=np.complex128).reshape(self.Nez, self.Ney, self.Nex)
        u, lam = {}, {s: {} for s in SIDES}
        for i in range(q):
            for j in range(r):
                f = np.zeros(self.shape(i, j), dtype=np.complex128)
                (r0, r1), (c0, c1) = self.omega_box(i, j)
                (y0, _), (x0, _) = self.yw[i], self.xw[j]
                f[:, r0:r1, c0:c1] = R[:, y0 + r0:y0 + r1, x0 + c0:x0 + c1]
                u[i, j] = self.solve_local(i, j, f)
                t = self.extract(u[i, j], i, j)
                for s in SIDES:
                    lam[s][i, j] = t[s]
        R_up, L_up = self._vertical(u, lam["T"], up=True)
        R_dn, L_dn = self._vertical(u, lam["B"], up=False)
        B_lf, T_lf = self._horizontal(u, lam["L"], right=False)
        B_rt, T_rt = self._horizontal(u, lam["R"], right=True)
        self._diagonal(u, "B", T_rt, "L", R_up)   # BL2TR(R^up, T^right)
        self._diagonal(u, "T", B_lf, "R", L_dn)   # TR2BL(L^down, B^left)
        self._diagonal(u, "B", T_lf, "R", L_up)   # BR2TL(L^up, T^left)
        self._diagonal(u, "T", B_rt, "L", R_dn)   # TL2BR(R^down, B^right)
        Z = np.zeros((self.Nez, self.Ney, self.Nex), dtype=np.complex128)
        for i in range(q):
            for j in range(r):
                (r0, r1), (c0, c1) = self.omega_box(i, j)
                (y0, _), (x0, _) = self.yw[i], self.xw[j]
                Z[:, y0 + r0:y0 + r1, x0 + c0:x0 + c1] = u[i, j][:, r0:r1, c0:c1]
        return Z.ravel()
