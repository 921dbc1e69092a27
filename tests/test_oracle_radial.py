"""Pins of the oracle's radial profiles (section 3.1: photon density and mean
arrival time in rings about the shower core).

Bins are checked on photons placed at known radii and against numpy's
digitize on shower photons; the profiles against a hand-computed case and
the invariants that fix them (the density integrated over the rings gives
back the binned weight, the mean time lies within its bin's times and does
not depend on the reference time).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2309_15861_amd import workloads as wl


def _placed(radii, phi=0.0, core=(0.0, 0.0), w=None, t=None, status=None):
    ph = np.zeros(len(radii), orc.PHOTON_DTYPE)
    r = np.asarray(radii, float)
    ph["xl"] = core[0] + r * np.cos(phi)
    ph["yl"] = core[1] + r * np.sin(phi)
    ph["weight"] = 1.0 if w is None else w
    ph["tl"] = 0.0 if t is None else t
    ph["status"] = orc.LANDED if status is None else status
    return ph


def test_edges():
    assert np.allclose(orc.radial_edges(10, 0.0, 100.0, False), np.arange(0.0, 101.0, 10.0), rtol=0, atol=1e-12)
    assert np.allclose(orc.radial_edges(3, 1.0, 1000.0, True), [1.0, 10.0, 100.0, 1000.0], rtol=1e-14)


def test_placed_photons():
    e = orc.radial_edges(10, 0.0, 100.0, False)
    ph = _placed([5.0, 15.0, 25.5, 99.999, 100.0, 100.5])
    assert orc.radial_bins(ph, (0.0, 0.0), e).tolist() == [0, 1, 2, 9, -1, -1]
    el = orc.radial_edges(3, 1.0, 1000.0, True)
    ph = _placed([5.0, 50.0, 500.0, 0.5], core=(30.0, -20.0))
    assert orc.radial_bins(ph, (30.0, -20.0), el).tolist() == [0, 1, 2, -1]
    ph = _placed([5.0, 15.0], status=np.array([orc.LANDED, 2], np.int32))
    assert orc.radial_bins(ph, (0.0, 0.0), e).tolist() == [0, -1]


def test_hand_computed_profile():
    e = orc.radial_edges(2, 0.0, 20.0, False)
    ph = _placed([3.0, 7.0, 15.0], w=np.array([1.0, 0.5, 0.25]), t=np.array([10.0, 20.0, 40.0]))
    cnt, w, dens, mt = orc.radial_profile(ph, (0.0, 0.0), e)
    assert cnt.tolist() == [2, 1]
    assert np.allclose(w, [1.5, 0.25])
    assert np.allclose(dens, [1.5 / (np.pi * 100.0), 0.25 / (np.pi * 300.0)])
    assert np.allclose(mt, [(10.0 + 0.5 * 20.0) / 1.5, 40.0])


@pytest.fixture(scope="module")
def shower_photons():
    seg = wl.subsample(wl.shower_cherenkov(), np.arange(0, 200_000, 20))
    atm = orc.Atmosphere.from_dict(wl.default_atmosphere(absorption=True))
    cnt, _, _ = orc.counts(seg, atm, "cherenkov", 2)
    off = np.concatenate([[0], np.cumsum(cnt.astype(np.int64))]).astype(np.uint64)
    return orc.photons_all(seg, atm, "cherenkov", 2, off)


@pytest.mark.parametrize("log_bins", [False, True])
def test_bins_match_digitize(shower_photons, log_bins):
    ph = shower_photons
    e = orc.radial_edges(60, 1.0 if log_bins else 0.0, 600.0, log_bins)
    core = (3.0, -2.0)
    b = orc.radial_bins(ph, core, e)
    r = np.hypot(ph["xl"] - core[0], ph["yl"] - core[1])
    ref = np.digitize(r, e) - 1
    ref[(ref < 0) | (ref >= len(e) - 1) | (ph["status"] != orc.LANDED)] = -1
    gap = np.min(np.abs(r[:, None] - e[None, :]), axis=1)
    clear = gap > 1e-9 * np.maximum(r, 1.0)
    assert np.array_equal(b[clear], ref[clear])
    assert (b >= 0).sum() > 10000


def test_profile_invariants(shower_photons):
    ph = shower_photons
    e = orc.radial_edges(40, 1.0, 800.0, True)
    core = (0.0, 0.0)
    cnt, w, dens, mt = orc.radial_profile(ph, core, e, t_ref=0.0)
    b = orc.radial_bins(ph, core, e)
    area = np.pi * (e[1:] ** 2 - e[:-1] ** 2)
    assert np.isclose(np.sum(dens * area), ph["weight"][b >= 0].sum(), rtol=1e-12)
    assert cnt.sum() == (b >= 0).sum()
    for k in np.nonzero(cnt)[0]:
        tk = ph["tl"][b == k]
        assert tk.min() - 1e-9 <= mt[k] <= tk.max() + 1e-9
    _, _, _, mt2 = orc.radial_profile(ph, core, e, t_ref=float(np.median(ph["tl"])))
    ok = cnt > 0
    assert np.allclose(mt[ok], mt2[ok], rtol=0, atol=1e-7)
    assert np.all(np.isnan(mt[~ok]))
