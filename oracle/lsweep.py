"""The L-sweeps preconditioner z = M^-1 r, run literally and sequentially (oracle; test infrastructure only).

This is Alg. Scenario3 of App. C in the paper's own order: stage 1 (local solutions,
addLocSols), the four cardinal sweeps (up, down, left, right), then the four diagonal
sweeps (BL->TR, TR->BL, BR->TL, TL->BR), and the assembly of z from the Omega_ij parts.
Every local solve is a SuperLU solve of the local matrix A_ij; every polarized
wavefield is built from eq. DiscPol2:

    g[Gamma_1] = A_ij[Gamma_1, Gamma_2] u~[Gamma_2],   g[Gamma_2] = -A_ij[Gamma_2, Gamma_1] u~[Gamma_1],
    U = A_ij^-1 g,

where Gamma_2 are the points of the receiving region chi adjacent to its outside and
Gamma_1 the outside points adjacent to chi (Sec. 1.3).  They are found from the
sparsity of A_ij itself, so g = A_ij(chi u~) - chi (A_ij u~) exactly.

Discrete conventions (Sec. 2.2; where the paper leaves them open, the readings below):
  * CDD: the bulk points of each axis are split into q (rows, along y) or r (columns,
    along x) contiguous groups, the first (n mod q) one point larger; the first and last
    groups also own the global PML points.  Row i = 0 is at the bottom, column j = 0 at
    the left.
  * Local problem: Omega_ij extended on each interior side by 2 overlap lines (the
    2-delta layer, delta = 1 for the 5-point stencil) and then n_pml_local PML lines whose
    cubic profile starts (sigma = 0) at the third appended line; Dirichlet beyond.  The
    local sigma is added to the global one; m is the global m at the same points.
  * Traces: the two lines on either side of each interface, over the full window
    extent: B = rows {lo-1, lo}, T = rows {hi-1, hi}, L = cols {lo-1, lo},
    R = cols {hi-1, hi}.  Line 0 is the one with the smaller index.
  * L-shaped traces: each leg is restricted to the receiving range of the other side
    (the L-shaped set surrounding the quadrant); on the one point shared by both legs
    the horizontal (B or T) trace is used, as in the paper's convention.
  * Diagonal sweeps take their inputs by call site (the bodies' names disagree with the
    parameter names): BL2TR(R^up, T^right), TR2BL(L^down, B^left), BR2TL(L^up, T^left),
    TL2BR(R^down, B^right), each visiting anti-diagonals in its sweep direction.

Pins (tests/test_oracle_lsweep.py): the discrete annihilation identity for every side
and quadrant; M^-1 = A^-1 for a 1x1 CDD; for sources in any subdomain of a constant
medium with a strong PML, M^-1 f reproduces A^-1 f up to the PML error (exact
reconstruction claimed in Sec. 2); linearity.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import alpha_of, assemble, axis_points, cubic_sigma


def partition(n_bulk: int, n_pml: int, groups: int, shift: int = 0):
    """[lo, hi) of each group along one axis (extended-grid indices).

    shift > 0 gives the shifted CDD of scenario 4 (Sec. 2.1): every group start of the even split,
    the first bulk point included, moves by `shift` points towards larger indices, so the axis has
    one more group (the first holds the PML and `shift` bulk points).  The returned sizes are those
    of the even split."""
    sizes = [n_bulk // groups + (1 if g < n_bulk % groups else 0) for g in range(groups)]
    first = 1 if shift == 0 else 0
    bounds = [n_pml + sum(sizes[:g]) + shift for g in range(first, groups)]
    lo = [0] + bounds
    hi = bounds + [n_bulk + 2 * n_pml]
    return lo, hi, sizes


SIDES = ("B", "R", "T", "L")


class LSweep2D:
    """Alg. Scenario3 for a 2D q x r CDD; `shift` = (sx, sy) shifts the group boundaries of each
    axis (the shifted CDDs of scenario 4; a shifted axis has one more group)."""

    def __init__(self, m_ext: np.ndarray, omega: float, n, n_pml, q: int, r: int, C: float,
                 n_pml_local: int | None = None, h: float | None = None, shift=(0, 0)):
        nx, ny = (n, n) if np.isscalar(n) else n
        px, py = (n_pml, n_pml) if np.isscalar(n_pml) else n_pml
        self.nx, self.ny, self.px, self.py = nx, ny, px, py
        self.h = 1.0 / (nx + 1) if h is None else h
        self.omega, self.C = omega, C
        self.q, self.r = q, r
        self.pl = px if n_pml_local is None else n_pml_local
        self.e = 2 + self.pl
        self.m = np.asarray(m_ext, dtype=np.float64)
        self.Nex, self.Ney = nx + 2 * px, ny + 2 * py
        assert self.m.shape == (self.Ney, self.Nex)
        self.shift = tuple(shift)
        self.xlo, self.xhi, _ = partition(nx, px, r, self.shift[0])
        self.ylo, self.yhi, _ = partition(ny, py, q, self.shift[1])
        q, r = self.q, self.r = len(self.ylo), len(self.xlo)
        for lo, hi, N in ((self.xlo, self.xhi, self.Nex), (self.ylo, self.yhi, self.Ney)):
            for g in range(len(lo)):
                if hi[g] - lo[g] < 2 or (g > 0 and lo[g] < self.e) or \
                        (g < len(lo) - 1 and hi[g] + self.e > N):
                    raise ValueError("each group needs 2 points and its window must fit in the grid")
        self.xw = [self._window(self.xlo, self.xhi, j, r, self.Nex) for j in range(r)]
        self.yw = [self._window(self.ylo, self.yhi, i, q, self.Ney) for i in range(q)]
        # per-axis alpha tables of each column / row group's window
        self.ax = [self._axis_alpha(nx, px, self.xlo, self.xhi, j, r, self.xw[j]) for j in range(r)]
        self.ay = [self._axis_alpha(ny, py, self.ylo, self.yhi, i, q, self.yw[i]) for i in range(q)]
        self.A, self.lu = {}, {}
        for i in range(q):
            for j in range(r):
                (y0, y1), (x0, x1) = self.yw[i], self.xw[j]
                A = assemble([self.ax[j][0], self.ay[i][0]], [self.ax[j][1], self.ay[i][1]],
                             self.m[y0:y1, x0:x1], omega, self.h)
                self.A[i, j] = A.tocsr()
                self.lu[i, j] = spla.splu(sp.csc_matrix(A))
        self._coupling = {}
        self.solves = 0

    # ------------------------------------------------------------------ geometry
    def _window(self, lo, hi, g, G, N):
        w0 = lo[g] - (self.e if g > 0 else 0)
        w1 = hi[g] + (self.e if g < G - 1 else 0)
        return (w0, w1)

    def _axis_alpha(self, n, p, lo, hi, g, G, win):
        """alpha at the window's integer and half points: global sigma + local cubic layers."""
        x_int, x_half = axis_points(n, p, self.h)
        w0, w1 = win
        xi = x_int[w0:w1]
        xh = x_half[w0:w1 + 1]
        L = (n + 1) * self.h
        dl = self.pl * self.h

        def sig(x):
            s = cubic_sigma(x, 0.0, L, p * self.h, self.C)
            if self.pl > 0 and g > 0:       # local layer below/left: starts at line lo-3
                s = s + cubic_sigma(x, x_int[lo[g] - 3], np.inf, dl, self.C)
            if self.pl > 0 and g < G - 1:   # local layer above/right: starts at line hi+2
                s = s + cubic_sigma(x, -np.inf, x_int[hi[g] + 2], dl, self.C)
            return s

        return alpha_of(sig(xi), self.omega), alpha_of(sig(xh), self.omega)

    def shape(self, i, j):
        (y0, y1), (x0, x1) = self.yw[i], self.xw[j]
        return (y1 - y0, x1 - x0)

    def omega_box(self, i, j):
        """Window-local [row0, row1) x [col0, col1) of Omega_ij."""
        (y0, _), (x0, _) = self.yw[i], self.xw[j]
        return (self.ylo[i] - y0, self.yhi[i] - y0), (self.xlo[j] - x0, self.xhi[j] - x0)

    def lines(self, i, j, side):
        """Window-local indices (2 lines) of a trace side."""
        (r0, r1), (c0, c1) = self.omega_box(i, j)
        return {"B": (r0 - 1, r0), "T": (r1 - 1, r1), "L": (c0 - 1, c0), "R": (c1 - 1, c1)}[side]

    def has_side(self, i, j, side):
        return {"B": i > 0, "T": i < self.q - 1, "L": j > 0, "R": j < self.r - 1}[side]

    # ------------------------------------------------------------------ primitives
    def extract(self, u, i, j):
        """extractTraces: the 2-line traces of a local field (zero on exterior sides)."""
        H, W = self.shape(i, j)
        out = {}
        for s in SIDES:
            if s in ("B", "T"):
                t = np.zeros((2, W), dtype=np.complex128)
                if self.has_side(i, j, s):
                    a, b = self.lines(i, j, s)
                    t[0], t[1] = u[a], u[b]
            else:
                t = np.zeros((2, H), dtype=np.complex128)
                if self.has_side(i, j, s):
                    a, b = self.lines(i, j, s)
                    t[0], t[1] = u[:, a], u[:, b]
            out[s] = t
        return out

    def solve_local(self, i, j, g):
        self.solves += 1
        H, W = self.shape(i, j)
        return self.lu[i, j].solve(g.ravel()).reshape(H, W)

    def receiving_mask(self, i, j, kind):
        """chi: the half plane (one side) or quadrant (two sides) that receives the wave."""
        H, W = self.shape(i, j)
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

    def _couplings(self, i, j, kind):
        key = (i, j, kind)
        if key not in self._coupling:
            chi = self.receiving_mask(i, j, kind).ravel()
            inn = np.flatnonzero(chi)
            out = np.flatnonzero(~chi)
            A = self.A[i, j]
            self._coupling[key] = (inn, out, A[out][:, inn].tocsr(), A[inn][:, out].tocsr())
        return self._coupling[key]

    def polarized(self, i, j, kind, ut):
        """U = A_ij^-1 [A_ij, chi] u~ via the block form of eq. DiscPol2."""
        inn, out, A_out_in, A_in_out = self._couplings(i, j, kind)
        v = ut.ravel()
        g = np.zeros(v.size, dtype=np.complex128)
        g[out] = A_out_in @ v[inn]
        g[inn] = -(A_in_out @ v[out])
        return self.solve_local(i, j, g.reshape(ut.shape))

    def straight_field(self, i, j, side, lam):
        """u~ holding one incoming 2-line trace on its own lines (full window extent)."""
        ut = np.zeros(self.shape(i, j), dtype=np.complex128)
        a, b = self.lines(i, j, side)
        if side in ("B", "T"):
            ut[a], ut[b] = lam[0], lam[1]
        else:
            ut[:, a], ut[:, b] = lam[0], lam[1]
        return ut

    def corner_field(self, i, j, hside, hlam, vside, vlam):
        """u~ for an L-shaped interface: legs restricted to the quadrant; horizontal leg wins."""
        ut = np.zeros(self.shape(i, j), dtype=np.complex128)
        chi = self.receiving_mask(i, j, hside + vside)
        rows_in = chi.any(axis=1)        # receiving range of the horizontal side
        cols_in = chi.any(axis=0)        # receiving range of the vertical side
        a, b = self.lines(i, j, vside)   # vertical leg: columns a, b on the quadrant's rows
        ut[rows_in, a] = vlam[0][rows_in]
        ut[rows_in, b] = vlam[1][rows_in]
        a, b = self.lines(i, j, hside)   # horizontal leg: rows a, b on the quadrant's columns
        ut[a, cols_in] = hlam[0][cols_in]
        ut[b, cols_in] = hlam[1][cols_in]
        return ut

    # ------------------------------------------------------------------ Alg. Scenario3
    def apply(self, rvec: np.ndarray) -> np.ndarray:
        q, r = self.q, self.r
        R = np.asarray(rvec, dtype=np.complex128).reshape(self.Ney, self.Nex)
        u, lam = {}, {s: {} for s in SIDES}
        # stage 1: addLocSols
        for i in range(q):
            for j in range(r):
                f = np.zeros(self.shape(i, j), dtype=np.complex128)
                (r0, r1), (c0, c1) = self.omega_box(i, j)
                (y0, _), (x0, _) = self.yw[i], self.xw[j]
                f[r0:r1, c0:c1] = R[y0 + r0:y0 + r1, x0 + c0:x0 + c1]
                u[i, j] = self.solve_local(i, j, f)
                t = self.extract(u[i, j], i, j)
                for s in SIDES:
                    lam[s][i, j] = t[s]
        # stage 2: cardinal sweeps (addUpSweeps, addDownSweeps, addLeftSweeps, addRightSweeps)
        R_up, L_up = self._vertical(u, lam["T"], up=True)
        R_dn, L_dn = self._vertical(u, lam["B"], up=False)
        B_lf, T_lf = self._horizontal(u, lam["L"], right=False)
        B_rt, T_rt = self._horizontal(u, lam["R"], right=True)
        # stage 3: diagonal sweeps, inputs bound by call site
        self._diagonal(u, "B", T_rt, "L", R_up)   # BL2TR(R^up, T^right)
        self._diagonal(u, "T", B_lf, "R", L_dn)   # TR2BL(L^down, B^left)
        self._diagonal(u, "B", T_lf, "R", L_up)   # BR2TL(L^up, T^left)
        self._diagonal(u, "T", B_rt, "L", R_dn)   # TL2BR(R^down, B^right)
        Z = np.zeros((self.Ney, self.Nex), dtype=np.complex128)
        for i in range(q):
            for j in range(r):
                (r0, r1), (c0, c1) = self.omega_box(i, j)
                (y0, _), (x0, _) = self.yw[i], self.xw[j]
                Z[y0 + r0:y0 + r1, x0 + c0:x0 + c1] = u[i, j][r0:r1, c0:c1]
        return Z.ravel()

    def _zeros_like_sides(self, sides):
        out = {}
        for s in sides:
            d = {}
            for i in range(self.q):
                for j in range(self.r):
                    H, W = self.shape(i, j)
                    d[i, j] = np.zeros((2, W if s in ("B", "T") else H), dtype=np.complex128)
            out[s] = d
        return out

    def _vertical(self, u, run, up: bool):
        """Up sweep (incoming B, running T) or down sweep (incoming T, running B)."""
        q, r = self.q, self.r
        side_in, side_run = ("B", "T") if up else ("T", "B")
        outs = self._zeros_like_sides(("R", "L"))
        order = range(1, q) if up else range(q - 2, -1, -1)
        for i in order:
            src = i - 1 if up else i + 1
            for j in range(r):
                U = self.polarized(i, j, side_in, self.straight_field(i, j, side_in, run[src, j]))
                t = self.extract(U, i, j)
                u[i, j] = u[i, j] + U
                run[i, j] = run[i, j] + t[side_run]
                outs["R"][i, j] = t["R"]
                outs["L"][i, j] = t["L"]
        return outs["R"], outs["L"]

    def _horizontal(self, u, run, right: bool):
        """Right sweep (incoming L, running R) or left sweep (incoming R, running L)."""
        q, r = self.q, self.r
        side_in, side_run = ("L", "R") if right else ("R", "L")
        outs = self._zeros_like_sides(("B", "T"))
        order = range(1, r) if right else range(r - 2, -1, -1)
        for i in range(q):
            for j in order:
                src = j - 1 if right else j + 1
                U = self.polarized(i, j, side_in, self.straight_field(i, j, side_in, run[i, src]))
                t = self.extract(U, i, j)
                u[i, j] = u[i, j] + U
                run[i, j] = run[i, j] + t[side_run]
                outs["B"][i, j] = t["B"]
                outs["T"][i, j] = t["T"]
        return outs["B"], outs["T"]

    def _diagonal(self, u, hside, hrun, vside, vrun):
        """One corner-to-corner sweep.  hside/vside are the incoming sides of each visited
        subdomain; hrun/vrun the running horizontal/vertical trace arrays (updated in place)."""
        q, r = self.q, self.r
        di = -1 if hside == "B" else 1          # horizontal trace comes from row i+di
        dj = -1 if vside == "L" else 1          # vertical trace comes from column j+dj
        rows = range(1, q) if hside == "B" else range(0, q - 1)
        cols = range(1, r) if vside == "L" else range(0, r - 1)
        hout = "T" if hside == "B" else "B"
        vout = "R" if vside == "L" else "L"

        def depth(i, j):  # distance from the sweep's starting corner
            return (i if hside == "B" else q - 1 - i) + (j if vside == "L" else r - 1 - j)

        cells = sorted(((i, j) for i in rows for j in cols), key=lambda c: (depth(*c), c))
        for i, j in cells:
            ut = self.corner_field(i, j, hside, hrun[i + di, j], vside, vrun[i, j + dj])
            U = self.polarized(i, j, hside + vside, ut)
            t = self.extract(U, i, j)
            u[i, j] = u[i, j] + U
            hrun[i, j] = hrun[i, j] + t[hout]
            vrun[i, j] = vrun[i, j] + t[vout]
