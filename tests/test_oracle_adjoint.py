"""Pins of the reference gradient of the splatted ground density.

The complex-step gradient (oracle.adjoint) is checked against what does not
come from it: its forward against the C oracle's photons (adaptive
Gauss-Kronrod quadrature, pinned by the propagation tests), its derivatives
against five-point central differences of the C oracle's density, and the
invariants of the parametrisation (directions are normalised inside, layers
above every emission point do not matter).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from oracle.adjoint import SplatModel
from paper_2309_15861_amd import workloads as wl

SEED = 5


@pytest.fixture(scope="module")
def case():
    seg = wl.subsample(wl.differentiable(200_000, 5), np.arange(60))
    atm_d = wl.default_atmosphere(absorption=True)
    atm = orc.Atmosphere.from_dict(atm_d)
    cnt, mu, _ = orc.counts(seg, atm, "cherenkov", SEED)
    g = wl.splat_grid_128()
    # wide truncation: the finite differences then see no jump at the window edge
    g["trunc"] = 10.0
    H1, e1, d1 = wl.perturbed_parameters(atm_d, seg, 77)
    atm1 = dict(atm_d, scale_height=H1, n0_minus_1=e1)
    seg1 = dict(seg, dx=d1[:, 0].copy(), dy=d1[:, 1].copy(), dz=d1[:, 2].copy())
    T = orc.splat_density(seg1, orc.Atmosphere.from_dict(atm1), cnt, mu, SEED, g, g["sigma"], g["trunc"])
    M = SplatModel(seg, atm_d, SEED, cnt, mu, g, g["sigma"], g["trunc"])
    grad = M.gradient(T, atm_d["scale_height"], atm_d["n0_minus_1"], seg["dx"], seg["dy"], seg["dz"])
    return dict(seg=seg, atm_d=atm_d, atm=atm, cnt=cnt, mu=mu, g=g, T=T, M=M, grad=grad)


def _loss_c(c, atm_d, seg):
    g = c["g"]
    D = orc.splat_density(seg, orc.Atmosphere.from_dict(atm_d), c["cnt"], c["mu"], SEED, g, g["sigma"],
                          g["trunc"])
    return float(np.sum((D - c["T"]) ** 2))


def _fd5(f, h):
    return (8.0 * (f(h) - f(-h)) - (f(2.0 * h) - f(-2.0 * h))) / (12.0 * h)


def test_forward_matches_c_oracle(case):
    c = case
    M, seg, atm_d = c["M"], c["seg"], c["atm_d"]
    x, y, W, landed = M.photons(atm_d["scale_height"], atm_d["n0_minus_1"], seg["dx"], seg["dy"], seg["dz"])
    ph = orc.photons(seg, c["atm"], "cherenkov", SEED, M.s_list, M.j_list)
    ok = ph["status"] == orc.LANDED
    assert np.array_equal(ok, landed)
    assert ok.sum() > 1000
    dist = np.maximum(np.hypot(ph["xl"] - ph["xe"], ph["yl"] - ph["ye"]), 1.0)
    assert np.max(np.abs(x.real - ph["xl"])[ok] / dist[ok]) < 1e-12
    assert np.max(np.abs(y.real - ph["yl"])[ok] / dist[ok]) < 1e-12
    assert np.max(np.abs(W.real - ph["weight"])[ok] / ph["weight"][ok]) < 1e-12
    D = M.density(atm_d["scale_height"], atm_d["n0_minus_1"], seg["dx"], seg["dy"], seg["dz"]).real
    g = c["g"]
    D2 = orc.splat_density(seg, c["atm"], c["cnt"], c["mu"], SEED, g, g["sigma"], g["trunc"])
    assert np.max(np.abs(D - D2)) < 1e-12 * np.max(np.abs(D2))


def test_weight_ratio_is_one_at_nominal(case):
    """mu(theta)/mu(theta0) = 1 at the nominal parameters: the weights are the
    plain transmissions."""
    c = case
    M, seg, atm_d = c["M"], c["seg"], c["atm_d"]
    _, _, W, landed = M.photons(atm_d["scale_height"], atm_d["n0_minus_1"], seg["dx"], seg["dy"], seg["dz"])
    ph = orc.photons(seg, c["atm"], "cherenkov", SEED, M.s_list, M.j_list)
    assert np.allclose(W.real[landed], np.exp(-ph["tau"][landed]), rtol=1e-13, atol=0)


def test_global_gradient_matches_central_differences(case):
    c = case
    atm_d, seg = c["atm_d"], c["seg"]
    gH, ge, _ = c["grad"]
    H0 = np.asarray(atm_d["scale_height"], float)
    for l in (0, 1):
        def f(h, l=l):
            Hh = H0.copy()
            Hh[l] += h
            return _loss_c(c, dict(atm_d, scale_height=Hh), seg)
        v = _fd5(f, 1e-3 * H0[l])
        assert abs(gH[l] - v) <= 1e-7 * abs(v), (l, gH[l], v)
    e0 = atm_d["n0_minus_1"]
    v = _fd5(lambda h: _loss_c(c, dict(atm_d, n0_minus_1=e0 + h), seg), 1e-3 * e0)
    assert abs(ge - v) <= 1e-7 * abs(v), (ge, v)


def test_direction_gradient_matches_central_differences(case):
    c = case
    atm_d, seg = c["atm_d"], c["seg"]
    gd = c["grad"][2]
    rows = [s for s in range(len(seg["x0"])) if np.abs(gd[s]).max() > 0][:3]
    assert len(rows) == 3
    for s in rows:
        for k, key in enumerate(("dx", "dy", "dz")):
            def f(h, s=s, key=key):
                arr = seg[key].copy()
                arr[s] += h
                return _loss_c(c, atm_d, dict(seg, **{key: arr}))
            v = _fd5(f, 2e-6)
            assert abs(gd[s, k] - v) <= 1e-6 * np.abs(gd[s]).max(), (s, key, gd[s, k], v)


def test_direction_gradient_is_orthogonal(case):
    """The direction is normalised inside: scaling d does not change L."""
    c = case
    gd = c["grad"][2]
    seg = c["seg"]
    d = np.stack([seg["dx"], seg["dy"], seg["dz"]], axis=1)
    assert np.max(np.abs(np.sum(gd * d, axis=1))) <= 1e-12 * np.abs(gd).max()


def test_layers_above_emission_have_zero_gradient(case):
    """Scale heights above every emission point (40 km and up) enter no
    photon: their derivative is exactly zero."""
    c = case
    gH = c["grad"][0]
    assert np.max(c["seg"]["z0"]) < 40000.0
    assert gH[3] == 0.0 and gH[4] == 0.0
    assert gH[0] != 0.0 and gH[1] != 0.0
