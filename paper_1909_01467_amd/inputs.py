"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmarks.

This module produces *problem data only*: wave speeds on the bulk grid, source
densities on the bulk grid, receiver positions, frequencies and random complex
vectors.  It contains none of the method's arithmetic (no PML, no normal
extension of the medium, no stencil, no sweep): each side that consumes these
inputs performs those steps with its own code.

Media stand in for the paper's numerical examples (Sec. 5): a constant speed
(Sec. 5.1-5.2), a smooth random medium (Sec. 5.3), a reflective layered medium
(stand-in for the BP model of Sec. 5.4, which is not available) and a 3D smooth
lens (Sec. 5.6).  Frequencies follow the paper's 10 points per minimum
wavelength rule (Sec. 5): omega = 2*pi*c_min*n/ppw.

Bulk grid convention: n points per axis at x = h, 2h, ..., n*h with
h = 1/(n+1), so the bulk is the unit interval with its Dirichlet end points
removed.  Arrays are indexed [y, x] in 2D and [z, y, x] in 3D (x fastest).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage


def bulk_h(n: int) -> float:
    return 1.0 / (n + 1)


def bulk_coords(n: int) -> np.ndarray:
    h = bulk_h(n)
    return h * np.arange(1, n + 1, dtype=np.float64)


def _mesh(n: int, dim: int):
    x = bulk_coords(n)
    # indexing 'ij' over (slowest ... fastest) = (z, y, x) / (y, x)
    return np.meshgrid(*([x] * dim), indexing="ij")


# ----------------------------------------------------------------------------
# wave speeds on the bulk grid
# ----------------------------------------------------------------------------

def speed_constant(n: int, dim: int = 2, c: float = 1.0) -> np.ndarray:
    return np.full((n,) * dim, c, dtype=np.float64)


def speed_lens(n: int, dim: int = 2, depth: float = 0.4, radius: float = 0.1) -> np.ndarray:
    """Gaussian low-velocity lens centred in the box: c = 1 - depth*exp(-|x-x0|^2/radius^2)."""
    X = _mesh(n, dim)
    r2 = sum((xi - 0.5) ** 2 for xi in X)
    return 1.0 - depth * np.exp(-r2 / radius**2)


def speed_lens_noise(n: int, seed: int = 2, amp: float = 0.05, corr: float = 0.05) -> np.ndarray:
    """Lens times (1 + p), p = seeded white noise low-pass filtered to correlation
    length `corr` and scaled to max|p| = amp (smooth random medium, Sec. 5.3)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n))
    p = ndimage.gaussian_filter(w, sigma=corr / bulk_h(n), mode="reflect")
    p *= amp / np.max(np.abs(p))
    return speed_lens(n, 2) * (1.0 + p)


def speed_random_smooth(n: int, seed: int = 5, amp: float = 0.3, corr: float = 0.1) -> np.ndarray:
    """c = 1 + amp p, p = seeded white noise low-pass filtered to correlation length `corr` and
    scaled to max|p| = 1 (stands in for the random smooth wave speed of Sec. 5.3)."""
    rng = np.random.default_rng(seed)
    p = ndimage.gaussian_filter(rng.standard_normal((n, n)), sigma=corr / bulk_h(n), mode="reflect")
    return 1.0 + amp * p / np.max(np.abs(p))


def speed_waveguide(n: int, contrast: float = 2.0, width: float = 0.1) -> np.ndarray:
    """A straight horizontal wave-guide (stand-in for the wave-guide of Sec. 5): c = 1 in the
    channel |y - 1/2| < width/2, c = contrast elsewhere."""
    Y, X = _mesh(n, 2)
    return np.where(np.abs(Y - 0.5) < width / 2, 1.0, float(contrast)) + 0.0 * X


def speed_depth_gradient(n: int, top: float = 1.5, bottom: float = 3.0) -> np.ndarray:
    """Smooth background whose speed grows linearly with depth (1 - y), from `top` at y = 1 to
    `bottom` at y = 0 (stand-in for the smooth background BG1 of Sec. 5)."""
    Y, X = _mesh(n, 2)
    return top + (bottom - top) * (1.0 - Y) + 0.0 * X


def speed_salt(n: int, seed: int = 6, salt: float = 4.5, blobs: int = 3) -> np.ndarray:
    """The depth-gradient background with a salt body of speed `salt`: the region where a sum of
    `blobs` seeded Gaussian bumps (centres in [0.3, 0.7] x [0.35, 0.6], radii 0.08-0.15) exceeds
    1/2 (stand-in for BG1 with the salt body of Sec. 5)."""
    rng = np.random.default_rng(seed)
    Y, X = _mesh(n, 2)
    bump = np.zeros_like(X)
    for _ in range(blobs):
        cx, cy = rng.uniform(0.3, 0.7), rng.uniform(0.35, 0.6)
        r = rng.uniform(0.08, 0.15)
        bump += np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / r**2)
    return np.where(bump > 0.5, float(salt), speed_depth_gradient(n))


def speed_layered_faults(n: int, seed: int = 3, layers: int = 12, faults: int = 3,
                         cmin: float = 1.5, cmax: float = 4.5) -> np.ndarray:
    """Piecewise-constant dipping layers cut by vertical faults (reflective medium)."""
    rng = np.random.default_rng(seed)
    y_k = np.sort(rng.uniform(0.0, 1.0, layers - 1))
    theta = math.radians(rng.uniform(5.0, 20.0))
    x_f = np.sort(rng.uniform(0.15, 0.85, faults))
    shifts = rng.uniform(-0.05, 0.05, faults)
    c_k = rng.uniform(cmin, cmax, layers)
    Y, X = _mesh(n, 2)
    offset = np.zeros_like(X)
    for xf, s in zip(x_f, shifts):
        offset += np.where(X > xf, s, 0.0)
    layer = np.zeros(X.shape, dtype=np.int64)
    for yk in y_k:
        iface = yk + math.tan(theta) * (X - 0.5) + offset
        layer += (Y > iface).astype(np.int64)
    return c_k[layer]


def speed_lens_blobs(n: int, seed: int = 4, blobs: int = 6, amp: float = 0.05,
                     radius: float = 0.05) -> np.ndarray:
    """Lens plus +/-amp Gaussian blobs (the 'true' model of the FWI workload)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.2, 0.8, (blobs, 2))
    signs = rng.choice([-1.0, 1.0], blobs)
    Y, X = _mesh(n, 2)
    pert = np.zeros_like(X)
    for (cx, cy), s in zip(centres, signs):
        pert += s * amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / radius**2)
    return speed_lens(n, 2) * (1.0 + pert)


# ----------------------------------------------------------------------------
# sources, receivers, random vectors
# ----------------------------------------------------------------------------

def gaussian_source(n: int, centre, width: float | None = None) -> np.ndarray:
    """Unit-mass Gaussian f = exp(-|x-xs|^2/w^2)/(pi w^2)^(d/2), default w = 2h."""
    dim = len(centre)
    w = 2.0 * bulk_h(n) if width is None else width
    X = _mesh(n, dim)
    # mesh order is (.., y, x); centre is given as (x, y[, z])
    r2 = sum((X[dim - 1 - k] - centre[k]) ** 2 for k in range(dim))
    return np.exp(-r2 / w**2) / (math.pi * w**2) ** (dim / 2.0)


def four_point_sources(n: int) -> np.ndarray:
    """The sources of the standard setup of Sec. 5: narrow Gaussians of amplitude n^2/pi and
    width 1/n at (0.125, 0.125), (0.125, 0.875), (0.875, 0.125) and (0.875, 0.875)."""
    pts = ((0.125, 0.125), (0.125, 0.875), (0.875, 0.125), (0.875, 0.875))
    return sum(gaussian_source(n, c, width=1.0 / n) for c in pts)


def entrance_source(n: int) -> np.ndarray:
    """One narrow Gaussian (amplitude n^2/pi, width 1/n) at the entrance (0.125, 0.5) of the
    wave-guide."""
    return gaussian_source(n, (0.125, 0.5), width=1.0 / n)


def receiver_indices(n: int, xs, y: float) -> np.ndarray:
    """Nearest bulk grid points (iy, ix) of receivers at (x, y) for x in xs."""
    h = bulk_h(n)
    ix = np.clip(np.rint(np.asarray(xs) / h).astype(np.int64) - 1, 0, n - 1)
    iy = int(np.clip(round(y / h) - 1, 0, n - 1))
    return np.stack([np.full_like(ix, iy), ix], axis=1)


def complex_normal(shape, seed: int) -> np.ndarray:
    """Seeded CN(0,1) samples, complex128."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def smooth_direction(n: int, seed: int, corr: float = 0.05) -> np.ndarray:
    """Seeded N(0,1) field on the bulk grid, low-pass filtered to correlation length `corr`
    and scaled to max-abs 1 (a direction for finite-difference checks of a gradient)."""
    rng = np.random.default_rng(seed)
    d = ndimage.gaussian_filter(rng.standard_normal((n, n)), sigma=corr / bulk_h(n), mode="reflect")
    return d / np.max(np.abs(d))


def omega_for(n: int, c: np.ndarray, ppw: float = 10.0) -> float:
    """Angular frequency giving `ppw` points per minimum wavelength."""
    return 2.0 * math.pi * float(np.min(c)) * n / ppw


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    dim: int
    n: int
    n_pml: int
    q: int
    r: int
    speed: np.ndarray            # bulk grid
    omega: float
    sources: np.ndarray           # [nrhs, *bulk shape]
    tol: float
    precision: str                # "fp64" | "mixed"
    receivers: np.ndarray | None = None
    background: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    @property
    def h(self) -> float:
        return bulk_h(self.n)

    @property
    def C(self) -> float:
        """Default PML absorption constant: 16 ln(omega) (reading of App. A: the most accurate
        truncation for PMLs of one wavelength, and the iteration counts of Tab. PMLeffect)."""
        return 16.0 * math.log(self.omega)

    @property
    def slowness2(self) -> np.ndarray:
        return 1.0 / self.speed**2


def workload(name: str, n: int | None = None, q: int | None = None) -> Workload:
    """Named synthetic workloads.  `n`/`q` override the size for scaled-down parity runs
    (the medium recipe is unchanged)."""
    if name == "const2d":          # 127^2, 4x4, c = 1, centre source on the CDD cross-point
        n = n or 127
        q = q or 4
        c = speed_constant(n)
        src = gaussian_source(n, (0.5, 0.5))[None]
        return Workload(name, 2, n, 10, q, q, c, omega_for(n, c), src, 1e-8, "fp64")
    if name == "lens2d":           # 511^2, 8x8, lens + 5% smooth noise
        n = n or 511
        q = q or 8
        c = speed_lens_noise(n)
        src = gaussian_source(n, (0.5, 0.15))[None]
        return Workload(name, 2, n, 10, q, q, c, omega_for(n, c), src, 1e-6, "mixed")
    if name == "layered2d":        # 2047^2, 16x16, 12 dipping layers + 3 faults, 32 RHS
        n = n or 2047
        q = q or 16
        c = speed_layered_faults(n)
        xs = (np.arange(32) + 0.5) / 32
        src = np.stack([gaussian_source(n, (x, 0.98)) for x in xs])
        return Workload(name, 2, n, 15, q, q, c, omega_for(n, c), src, 1e-6, "mixed")
    if name == "fwi2d":            # 1023^2, 8x8, 8 sources, 64 receivers
        n = n or 1023
        q = q or 8
        c_true = speed_lens_blobs(n)
        c_bg = speed_lens(n, 2)
        xs = (np.arange(8) + 0.5) / 8
        src = np.stack([gaussian_source(n, (x, 0.98)) for x in xs])
        rec = receiver_indices(n, (np.arange(64) + 0.5) / 64, 0.96)
        return Workload(name, 2, n, 10, q, q, c_true, omega_for(n, c_bg), src, 1e-10,
                        "fp64", receivers=rec, background=c_bg)
    if name == "lens3d":           # 95^3, 4x4 beams, 8 ppw
        n = n or 95
        q = q or 4
        c = speed_lens(n, 3)
        src = gaussian_source(n, (0.5, 0.5, 0.25))[None]
        return Workload(name, 3, n, 8, q, q, c, omega_for(n, c, ppw=8.0), src, 1e-6, "mixed")
    raise KeyError(name)
