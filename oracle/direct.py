"""The exact target of the preconditioned solve: u = A^-1 b (oracle; test infrastructure only).

Plain definition of what GMRES + L-sweeps converges to (Sec. 3, eq. PrecLS): the solution
of the global linear system eq. LS.  Three library solvers:
  * solve_banded : LAPACK zgbsv on the band of A (kl = ku = N_x N_y ... of all faster axes);
  * SparseLU     : SuperLU (scipy.sparse.linalg.splu), for grids whose band storage is large;
  * solve_dense  : numpy.linalg.solve on the dense matrix (tiny grids only).
Pins: the three agree to 1e-12 on tiny 2D/3D grids, and solve the closed-form DST
problems (tests/test_oracle_discretization.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def bandwidth(A: sp.spmatrix) -> int:
    coo = A.tocoo()
    return int(np.max(np.abs(coo.row - coo.col))) if coo.nnz else 0


def to_band(A: sp.spmatrix, kl: int, ku: int) -> np.ndarray:
    """LAPACK band storage: ab[ku + i - j, j] = A[i, j]."""
    coo = A.tocoo()
    N = A.shape[0]
    ab = np.zeros((kl + ku + 1, N), dtype=np.complex128)
    ab[ku + coo.row - coo.col, coo.col] = coo.data
    return ab


def solve_banded(A: sp.spmatrix, b: np.ndarray) -> np.ndarray:
    """u = A^-1 b by banded LU with partial pivoting (zgbsv)."""
    bw = bandwidth(A)
    ab = to_band(A, bw, bw)
    return sla.solve_banded((bw, bw), ab, np.asarray(b, dtype=np.complex128),
                            overwrite_ab=True, check_finite=False)


def solve_dense(A: sp.spmatrix, b: np.ndarray) -> np.ndarray:
    return np.linalg.solve(A.toarray(), np.asarray(b, dtype=np.complex128))


class SparseLU:
    """One SuperLU factorisation reused for many right-hand sides (and for A^T = A)."""

    def __init__(self, A: sp.spmatrix):
        self.lu = spla.splu(sp.csc_matrix(A))

    def solve(self, b: np.ndarray) -> np.ndarray:
        return self.lu.solve(np.asarray(b, dtype=np.complex128))


def relative_residual(A: sp.spmatrix, u: np.ndarray, b: np.ndarray) -> float:
    """||b - A u||_2 / ||b||_2 in FP64 (the stop criterion of the solve)."""
    return float(np.linalg.norm(b - A @ u) / np.linalg.norm(b))
