"""Parity checks shared by the GPU tests: relative L2 error over the whole vector and on every
subdomain Omega_ij of the CDD, so that an error confined to one subdomain or one PML corner
cannot hide inside the whole-grid norm.

Every measured error is appended as one JSON line to the file named by $LSW_PARITY_LOG (when set),
which is how the measured table of errors against their bars is collected.
"""
from __future__ import annotations

import json
import os

import numpy as np

# a subdomain whose reference norm is far below the average (a quiet PML corner) is measured
# against this fraction of the norm it would have with the grid's mean magnitude
BLOCK_FLOOR = 0.05


def rel(a, b) -> float:
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def block_errors(got, ref, shape, cdd) -> np.ndarray:
    """Relative error on every Omega_ij (all right-hand sides and z planes of the subdomain
    together).  `shape` is the extended grid ((Nz,) Ny, Nx); `cdd` carries the partition
    (xlo, xhi, ylo, yhi) of the extended grid, edge groups owning the PML."""
    G = np.asarray(got).reshape(-1, *shape)
    R = np.asarray(ref).reshape(-1, *shape)
    total = np.linalg.norm(R)
    N = R.size
    errs = []
    for y0, y1 in zip(cdd.ylo, cdd.yhi):
        for x0, x1 in zip(cdd.xlo, cdd.xhi):
            g = G[..., y0:y1, x0:x1]
            r = R[..., y0:y1, x0:x1]
            floor = BLOCK_FLOOR * total * np.sqrt(r.size / N)
            errs.append(np.linalg.norm(g - r) / max(np.linalg.norm(r), floor))
    return np.asarray(errs)


def record(label: str, **fields) -> None:
    path = os.environ.get("LSW_PARITY_LOG")
    if not path:
        return
    with open(path, "a") as fh:
        fh.write(json.dumps({"case": label, **fields}) + "\n")


def check(label: str, got, ref, bar: float, *, cdd=None, shape=None, block_bar: float | None = None) -> float:
    """Asserts rel(got, ref) < bar and, with a CDD, every subdomain's error < block_bar
    (default 10 bar: an error confined to one of q r subdomains shows there about sqrt(q r)
    times larger than in the whole-grid norm)."""
    err = rel(got, ref)
    worst = None
    if cdd is not None:
        block_bar = 10 * bar if block_bar is None else block_bar
        be = block_errors(got, ref, shape, cdd)
        worst = float(be.max())
    record(label, err=err, bar=bar, block_err=worst, block_bar=block_bar)
    print("[case]", label, "rel err", err, "worst subdomain", worst, flush=True)
    assert err < bar, (label, err, bar)
    if worst is not None:
        assert worst < block_bar, (label, "subdomain", int(be.argmax()), worst, block_bar)
    return err
