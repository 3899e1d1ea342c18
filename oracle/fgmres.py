"""Right-preconditioned flexible GMRES, FP64 (oracle; test infrastructure only).

Sec. 3 (Phase 3) solves the preconditioned system with GMRES from a zero initial guess,
with restarts, to a relative residual tolerance (1e-6 in 2D).  Readings: right
preconditioning (so the monitored residual is the true residual of A u = b), the flexible
variant (it stores z_j = M^-1 v_j, which keeps the method exact for a preconditioner
applied in lower precision), classical Gram-Schmidt applied twice, restart length 50,
and the stop test ||b - A u||_2 <= tol ||b||_2 confirmed on the true residual.
An iteration is one application of the preconditioner.

Pinned by: convergence to the direct solution of eq. LS on small problems, and the
iteration counts of the paper's tables as soft bands (tests/test_oracle_lsweep.py).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class FGMRESResult:
    x: np.ndarray
    iterations: int
    converged: bool
    relres: float
    history: list = field(default_factory=list)


def fgmres(matvec, precond, b, tol=1e-6, restart=50, maxit=500, x0=None) -> FGMRESResult:
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    if nb == 0.0:
        return FGMRESResult(np.zeros_like(b), 0, True, 0.0)
    it = 0
    history = []
    while True:
        rvec = b - matvec(x)
        beta = np.linalg.norm(rvec)
        relres = beta / nb
        if relres <= tol or it >= maxit:
            return FGMRESResult(x, it, relres <= tol, relres, history)
        m = restart
        V = np.zeros((m + 1, b.size), dtype=np.complex128)
        Z = np.zeros((m, b.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = rvec / beta
        k = 0
        for k in range(m):
            Z[k] = precond(V[k])
            w = matvec(Z[k])
            h = np.zeros(k + 2, dtype=np.complex128)
            for _ in range(2):   # classical Gram-Schmidt, twice
                c = V[:k + 1].conj() @ w
                w = w - c @ V[:k + 1]
                h[:k + 1] += c
            h[k + 1] = np.linalg.norm(w)
            if h[k + 1] != 0.0:
                V[k + 1] = w / h[k + 1]
            # apply the previous Givens rotations G_l = [[conj(c), conj(s)], [-s, c]]
            for l in range(k):
                a, bb = h[l], h[l + 1]
                h[l] = np.conj(cs[l]) * a + np.conj(sn[l]) * bb
                h[l + 1] = -sn[l] * a + cs[l] * bb
            rho = np.sqrt(abs(h[k]) ** 2 + abs(h[k + 1]) ** 2)
            if rho == 0.0:
                cs[k], sn[k] = 1.0, 0.0
            else:
                cs[k], sn[k] = h[k] / rho, h[k + 1] / rho
            h[k] = rho
            h[k + 1] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = np.conj(cs[k]) * g[k]
            H[:k + 2, k] = h
            it += 1
            history.append(abs(g[k + 1]) / nb)
            if abs(g[k + 1]) <= tol * nb or it >= maxit:
                break
        kk = k + 1
        y = np.linalg.solve(np.triu(H[:kk, :kk]), g[:kk])
        x = x + y @ Z[:kk]
