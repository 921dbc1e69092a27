"""Pins of the oracle's Gaussian splat (the ground density of the
differentiable form): closed forms of a normalised 2-D Gaussian, which its
cell sums must reproduce independently of how the oracle writes it.

* Mass: with the truncation far out, the cell sums times the cell area equal
  the photon's weight. A Riemann sum of a Gaussian on a grid of spacing h
  differs from its integral by about 2 exp(-2 pi^2 sigma^2 / h^2) (Poisson
  summation), below 1e-15 here.
* Second moment: sum of D (x_g - x)^2 times the cell area equals w sigma^2
  (catches a wrong factor in the exponent).
* Peak: a photon on a cell centre gives w / (2 pi sigma^2) there.
* Truncation: cells farther than trunc * sigma in x or in y get nothing;
  the cell exactly at the limit keeps its Gaussian value.
* Every cell against scipy's bivariate normal density.
* Superposition; photons that did not land add nothing.
"""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

import oracle.oracle as O


def photons_at(xy, status=None):
    ph = np.zeros(len(xy), O.PHOTON_DTYPE)
    ph["xl"] = [p[0] for p in xy]
    ph["yl"] = [p[1] for p in xy]
    ph["status"] = O.LANDED if status is None else status
    return ph


@pytest.mark.parametrize("pos", [(0.0, 0.0), (1.37, -2.91), (-4.999, 3.3)])
def test_mass_equals_weight(oracle, pos):
    sigma, cell, w = 5.0, 2.0, 0.7316
    D = O.splat(photons_at([pos]), np.array([w]), -100.0, -100.0, cell, 100, 100, sigma, trunc=12.0)
    assert abs(D.sum() * cell * cell - w) < 1e-13


@pytest.mark.parametrize("pos", [(0.0, 0.0), (1.37, -2.91)])
def test_second_moment(oracle, pos):
    sigma, cell, w = 5.0, 2.0, 1.9
    D = O.splat(photons_at([pos]), np.array([w]), -100.0, -100.0, cell, 100, 100, sigma, trunc=12.0)
    g = -100.0 + (np.arange(100) + 0.5) * cell
    mx = (D.sum(0) * (g - pos[0]) ** 2).sum() * cell * cell
    my = (D.sum(1) * (g - pos[1]) ** 2).sum() * cell * cell
    assert abs(mx - w * sigma**2) < 1e-11 and abs(my - w * sigma**2) < 1e-11


def test_peak_on_a_cell_centre(oracle):
    sigma, cell, w = 5.0, 5.0, 3.0
    # cell (ix, iy) = (10, 7) has its centre at (-320 + 52.5, -320 + 37.5)
    x, y = -320.0 + 10.5 * cell, -320.0 + 7.5 * cell
    D = O.splat(photons_at([(x, y)]), np.array([w]), -320.0, -320.0, cell, 128, 128, sigma)
    assert D[7, 10] == pytest.approx(w / (2.0 * np.pi * sigma**2), rel=1e-15)
    assert D.max() == D[7, 10]


def test_truncation(oracle):
    """trunc = 4: cells whose centre is more than 4 sigma away in x or in y
    are empty; at exactly 4 sigma along an axis the Gaussian value stays."""
    sigma, cell, w = 5.0, 5.0, 1.0
    x, y = -320.0 + 64.5 * cell, -320.0 + 64.5 * cell
    D = O.splat(photons_at([(x, y)]), np.array([w]), -320.0, -320.0, cell, 128, 128, sigma, trunc=4.0)
    nz = np.argwhere(D > 0)
    assert nz[:, 0].min() == 60 and nz[:, 0].max() == 68 and nz[:, 1].min() == 60 and nz[:, 1].max() == 68
    assert len(nz) == 81
    norm = w / (2.0 * np.pi * sigma**2)
    assert D[64, 68] == pytest.approx(norm * np.exp(-8.0), rel=1e-14)
    assert D[68, 68] == pytest.approx(norm * np.exp(-16.0), rel=1e-14)


def test_against_scipy_density(oracle):
    rng = np.random.default_rng(3)
    sigma, cell = 5.0, 5.0
    xy = rng.uniform(-250.0, 250.0, size=(40, 2))
    w = rng.uniform(0.1, 1.0, 40)
    D = O.splat(photons_at([tuple(p) for p in xy]), w, -320.0, -320.0, cell, 128, 128, sigma, trunc=4.0)
    g = -320.0 + (np.arange(128) + 0.5) * cell
    gx, gy = np.meshgrid(g, g)
    ref = np.zeros_like(D)
    for p, wi in zip(xy, w):
        inside = (np.abs(gx - p[0]) <= 4.0 * sigma) & (np.abs(gy - p[1]) <= 4.0 * sigma)
        pdf = multivariate_normal(mean=p, cov=sigma**2 * np.eye(2)).pdf(np.stack([gx, gy], -1))
        ref += wi * pdf * inside
    assert np.abs(D - ref).max() <= 1e-14 * ref.max()


def test_superposition_and_status(oracle):
    sigma, cell = 5.0, 5.0
    a, b = (12.3, -40.0), (-7.7, 21.0)
    Da = O.splat(photons_at([a]), np.array([0.3]), -320.0, -320.0, cell, 128, 128, sigma)
    Db = O.splat(photons_at([b]), np.array([0.9]), -320.0, -320.0, cell, 128, 128, sigma)
    both = photons_at([a, b, (0.0, 0.0), (5.0, 5.0)], status=[O.LANDED, O.LANDED, O.UP, O.BELOW])
    Dab = O.splat(both, np.array([0.3, 0.9, 5.0, 5.0]), -320.0, -320.0, cell, 128, 128, sigma)
    assert np.abs(Dab - (Da + Db)).max() <= 1e-16
