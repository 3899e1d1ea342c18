"""Pin of the oracle's FWI gradient against central finite differences of the misfit."""
import math

import numpy as np

from oracle.discretization import extend_normal
from oracle.gradient import FWIProblem, restrict_to_bulk
from paper_1909_01467_amd import inputs


def _problem(n=24, p=5):
    omega = 2 * math.pi * n / 10
    srcs = np.stack([inputs.gaussian_source(n, (x, 0.8)) for x in (0.25, 0.5, 0.75)])
    rec_b = inputs.receiver_indices(n, np.linspace(0.1, 0.9, 7), 0.75)
    return FWIProblem(omega, n, p, 4 * math.log(omega), srcs, rec_b + p)


def test_gradient_matches_central_differences_on_extended_grid():
    n, p = 24, 5
    prob = _problem(n, p)
    m_true = extend_normal(1.0 / inputs.speed_lens_blobs(n) ** 2, p)
    m0 = extend_normal(1.0 / inputs.speed_lens(n, 2) ** 2, p)
    d = prob.data(m_true)
    J, g = prob.gradient(m0, d)
    assert J > 0
    rng = np.random.default_rng(1000)
    for _ in range(3):
        dm = rng.standard_normal(m0.shape)
        dm /= np.max(np.abs(dm))
        eps = 1e-4
        fd = (prob.misfit(m0 + eps * dm, d) - prob.misfit(m0 - eps * dm, d)) / (2 * eps)
        an = float(np.sum(g * dm))
        assert abs(fd - an) <= 1e-6 * abs(an) + 1e-12 * J, (fd, an)


def test_bulk_gradient_is_the_adjoint_of_normal_extension():
    n, p = 24, 5
    prob = _problem(n, p)
    mb_true = 1.0 / inputs.speed_lens_blobs(n) ** 2
    mb0 = 1.0 / inputs.speed_lens(n, 2) ** 2
    d = prob.data(extend_normal(mb_true, p))
    _, g = prob.gradient(extend_normal(mb0, p), d)
    gb = restrict_to_bulk(g, p)
    rng = np.random.default_rng(1001)
    dm = rng.standard_normal(mb0.shape)
    dm /= np.max(np.abs(dm))
    eps = 1e-4
    fd = (prob.misfit(extend_normal(mb0 + eps * dm, p), d)
          - prob.misfit(extend_normal(mb0 - eps * dm, p), d)) / (2 * eps)
    an = float(np.sum(gb * dm))
    assert abs(fd - an) <= 1e-6 * abs(an)
