"""Scenario 4 of Sec. 2.1: L-sweeps for arbitrary sources through four shifted CDDs and a
partition of unity (oracle; test infrastructure only).

The paper takes the CDD, three more CDDs obtained from it by a horizontal, a vertical and
a combined shift, and four window functions phi_1..phi_4 that sum to one, each vanishing on
the skeleton of one of the four CDDs.  Each windowed source phi_k f then avoids the
skeleton of its own CDD, scenario 3 on that CDD handles it, and the approximate solution is
the sum of the four results:  z = sum_k M_k^-1 (phi_k r).

The paper fixes neither the shift nor the windows; the readings taken here:
  * Shift: the CDD's grid of interfaces is translated by s points towards larger indices along
    the shifted axis: every group start of the even split, the first bulk point included, moves
    by s, so the shifted axis has one more group (the first holds the PML and s bulk points, the
    last the remaining bulk points and the PML) and no group is larger than in the CDD.  By
    default s is half of the smallest bulk group.  The skeletons of the two CDDs of one axis are
    then disjoint and interleaved, the shifted one on both ends.
  * Windows: tensor products phi = a(x) b(y).  Along one axis, with interfaces at
    P = lo - 1/2 (CDD) and P' = lo' - 1/2 (shifted CDD), d and d' the distances of a point to the
    nearest P and P', and w(t) = max(0, t - 1):
        a = w(d) / (w(d) + w(d')) between the first and the last interface,
        a = 1 beyond them (the nearest interface there is a shifted one).
    a vanishes on the two trace lines of every interface of the CDD (d = 1/2) and equals 1 on those
    of every shifted one; between them it is a linear ramp.  The CDD unshifted along this axis
    takes a, the shifted one 1 - a, so the four products sum to one.

Pins (tests/test_oracle_scenario4.py): the shifted partition; the window ramp; the partition of
unity and its vanishing on each CDD's skeleton; reconstruction of A^-1 f up to the PML error for
sources on the skeleton; each shifted CDD alone reconstructing its windowed source; a planted
dropped window failing the reconstruction.
"""
from __future__ import annotations

import numpy as np

from .lsweep import LSweep2D, partition
from .lsweep3d import LSweep3D


def default_shift(n_bulk: int, groups: int) -> int:
    """Half of the smallest bulk group of the even split."""
    return (n_bulk // groups) // 2


def axis_window(N: int, lo: list[int], lo_shifted: list[int]) -> np.ndarray:
    """The window a(x) of one axis on its N extended-grid points (see the module notes).
    lo / lo_shifted are the group starts of the CDD and of the shifted CDD (lo[0] = 0)."""
    P = np.asarray(lo[1:], dtype=np.float64) - 0.5
    Ps = np.asarray(lo_shifted[1:], dtype=np.float64) - 0.5
    first, last = min(P.min(), Ps.min()), max(P.max(), Ps.max())
    a = np.empty(N)
    for x in range(N):
        d, ds = np.abs(x - P).min(), np.abs(x - Ps).min()
        if x < first or x > last:
            a[x] = 1.0 if ds < d else 0.0
        else:
            w, ws = max(0.0, d - 1.0), max(0.0, ds - 1.0)
            a[x] = w / (w + ws)
    return a


class Scenario4:
    """z = sum over the four CDDs k of M_k^-1 (phi_k r).  In 3D (m_ext of shape [z, y, x], beams
    over all z) the CDDs and windows are those of the (x, y) cross-section, the same on every plane."""

    def __init__(self, m_ext: np.ndarray, omega: float, n, n_pml, q: int, r: int, C: float,
                 n_pml_local: int | None = None, h: float | None = None, shift=None):
        dim = np.asarray(m_ext).ndim
        ns = (n,) * dim if np.isscalar(n) else tuple(n)
        ps = (n_pml,) * dim if np.isscalar(n_pml) else tuple(n_pml)
        nx, ny, px, py = ns[0], ns[1], ps[0], ps[1]
        if q < 2 or r < 2:
            raise ValueError("scenario 4 needs at least two groups along each axis")
        sx, sy = (default_shift(nx, r), default_shift(ny, q)) if shift is None else shift
        if not (3 <= sx <= nx // r - 3 and 3 <= sy <= ny // q - 3):
            raise ValueError("the shift must lie in [3, smallest group - 3] so that the skeletons are disjoint")
        self.shift = (sx, sy)
        self.shape = np.asarray(m_ext).shape
        self.Nex, self.Ney = nx + 2 * px, ny + 2 * py
        ax = axis_window(self.Nex, partition(nx, px, r)[0], partition(nx, px, r, sx)[0])
        ay = axis_window(self.Ney, partition(ny, py, q)[0], partition(ny, py, q, sy)[0])
        cls = LSweep2D if dim == 2 else LSweep3D
        self.cdds, self.windows = [], []
        for kx, ky in ((0, 0), (1, 0), (0, 1), (1, 1)):
            self.cdds.append(cls(m_ext, omega, ns, ps, q, r, C, n_pml_local, h, shift=(kx * sx, ky * sy)))
            wx = 1.0 - ax if kx else ax
            wy = 1.0 - ay if ky else ay
            self.windows.append(np.outer(wy, wx))   # [y, x]; broadcast over z in 3D

    def apply(self, rvec: np.ndarray) -> np.ndarray:
        R = np.asarray(rvec, dtype=np.complex128).reshape(self.shape)
        z = np.zeros(R.size, dtype=np.complex128)
        for ls, phi in zip(self.cdds, self.windows):
            z += ls.apply((phi * R).ravel())
        return z

    @property
    def solves(self) -> int:
        return sum(ls.solves for ls in self.cdds)
