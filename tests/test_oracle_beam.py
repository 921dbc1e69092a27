"""Pins of the oracle's fluorescence beaming (section 1.1.1).

Beamed emission sends a segment's photons into a cone that contains the
emission area (a sphere around every telescope) and scales the photon number
by the cone's solid-angle fraction. The pins check the oracle against what
does not come from its own code: the cone from arcsin and cos of the summed
angle, directions inside the cone and uniform on it, every isotropic photon
that reaches a telescope leaving inside its segment's cone (so nothing that
can hit is lost), and the expected hit number unchanged.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import oracle as orc
from paper_2309_15861_amd import workloads as wl

SEED = 13
MARGIN = np.radians(1.0)
LINES = wl.fluorescence_lines()
YIELD = 10.0


def _tel(radius=40.0):
    return wl.telescopes_16(radius=radius)


def _area(tel):
    c = tel[:, :3].mean(axis=0)
    return c, float(np.max(np.linalg.norm(tel[:, :3] - c, axis=1) + tel[:, 3]))


def _cone_numpy(seg, centre, radius, margin):
    """(beamed, half angle, axis) per segment from arcsin and the unit vector."""
    d = np.stack([seg["dx"], seg["dy"], seg["dz"]], axis=1)
    u = d / np.linalg.norm(d, axis=1, keepdims=True)
    m = np.stack([seg["x0"], seg["y0"], seg["z0"]], axis=1) + 0.5 * seg["length"][:, None] * u
    v = np.asarray(centre)[None, :] - m
    D = np.linalg.norm(v, axis=1)
    reach = radius + 0.5 * seg["length"]
    beamed = reach < D
    half = np.where(beamed, np.arcsin(np.minimum(reach / D, 1.0)) + margin, np.pi)
    return beamed, half, v / D[:, None]


def _atm():
    return orc.Atmosphere.from_dict(wl.default_atmosphere(absorption=True))


def _all_photons(seg, seed, beam, yield_per_MeV=YIELD):
    atm = _atm()
    cnt, mu, _ = orc.counts(seg, atm, "fluorescence", seed, yield_per_MeV=yield_per_MeV, beam=beam)
    off = np.concatenate([[0], np.cumsum(cnt.astype(np.int64))]).astype(np.uint64)
    ph = orc.photons_all(seg, atm, "fluorescence", seed, off, yield_per_MeV=yield_per_MeV, lines_nm=LINES[0],
                         line_rel=LINES[1], beam=beam)
    s_of = np.repeat(np.arange(len(cnt)), cnt.astype(np.int64))
    return ph, s_of, cnt, mu


def test_cone_matches_trigonometry():
    seg = wl.fluorescence_near_array(400)
    far = wl.fluorescence(2000, seed=3)
    c, r = _area(_tel())
    for s in (seg, far):
        on, om, ax = orc.beam_cap(s, (c, r, MARGIN))
        b, half, axis = _cone_numpy(s, c, r, MARGIN)
        assert np.array_equal(on, b)
        assert np.allclose(om[b], 1.0 - np.cos(half[b]), rtol=1e-12, atol=0)
        assert np.allclose(ax[b], axis[b], rtol=0, atol=1e-14)
        assert np.all(om[~b] == 2.0)
    # a sphere containing the segment: isotropic
    on, om, _ = orc.beam_cap(seg, (c, 1e7, MARGIN))
    assert not on.any() and np.all(om == 2.0)


def test_beamed_mean_is_the_isotropic_mean_times_the_solid_angle_fraction():
    seg = wl.fluorescence_near_array(400)
    c, r = _area(_tel())
    atm = _atm()
    _, mu0, _ = orc.counts(seg, atm, "fluorescence", SEED, yield_per_MeV=YIELD)
    _, mu1, _ = orc.counts(seg, atm, "fluorescence", SEED, yield_per_MeV=YIELD, beam=(c, r, MARGIN))
    b, half, _ = _cone_numpy(seg, c, r, MARGIN)
    frac = np.where(b, 0.5 * (1.0 - np.cos(half)), 1.0)
    assert np.allclose(mu1, mu0 * frac, rtol=1e-12, atol=0)
    assert np.all(mu1 <= mu0) and b.sum() > 300


def test_beamed_directions_fill_the_cone_uniformly():
    seg = wl.fluorescence_near_array(400)
    c, r = _area(_tel())
    ph, s_of, _, _ = _all_photons(seg, SEED, (c, r, MARGIN), yield_per_MeV=200.0)
    b, half, axis = _cone_numpy(seg, c, r, MARGIN)
    keep = b[s_of]
    assert keep.sum() > 20000
    u = ph["ue"][keep]
    a = axis[s_of[keep]]
    cosang = np.sum(u * a, axis=1)
    assert np.all(cosang >= np.cos(half[s_of[keep]]) - 1e-12)
    # 1 - cos(angle) / (1 - cos(half)) is uniform on (0, 1)
    q = (1.0 - cosang) / (1.0 - np.cos(half[s_of[keep]]))
    assert stats.kstest(q, "uniform").pvalue > 1e-3
    # azimuth about the axis, in a frame built from the axis
    ref = np.where(np.abs(a[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    e1 = np.cross(a, ref)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(a, e1)
    phi = np.arctan2(np.sum(u * e2, axis=1), np.sum(u * e1, axis=1))
    assert stats.kstest((phi + np.pi) / (2.0 * np.pi), "uniform").pvalue > 1e-3
    # unit directions
    assert np.allclose(np.linalg.norm(ph["ue"], axis=1), 1.0, atol=1e-14)


def test_every_isotropic_hit_leaves_inside_its_cone():
    seg = wl.fluorescence_near_array(400)
    tel = _tel()
    c, r = _area(tel)
    atm = _atm()
    ph, s_of, _, _ = _all_photons(seg, SEED, None)
    tid, _ = orc.telescopes(ph, tel, atm.index(wl.H_OBS))
    hit = tid >= 0
    assert hit.sum() > 300
    b, half, axis = _cone_numpy(seg, c, r, MARGIN)
    ang = np.arccos(np.clip(np.sum(ph["ue"][hit] * axis[s_of[hit]], axis=1), -1.0, 1.0))
    inside = ang <= half[s_of[hit]]
    assert inside.all()
    # and without the margin too: refraction bends these rays by far less than a degree
    b0, half0, _ = _cone_numpy(seg, c, r, 0.0)
    assert np.all(ang <= half0[s_of[hit]])


def test_expected_hits_unchanged():
    """Isotropic hits against the mean over seeds of beamed hits (4 sigma)."""
    seg = wl.fluorescence_near_array(400)
    tel = _tel()
    c, r = _area(tel)
    atm = _atm()
    n_obs = atm.index(wl.H_OBS)
    ph, _, cnt0, _ = _all_photons(seg, SEED, None, yield_per_MeV=40.0)
    h_iso = int((orc.telescopes(ph, tel, n_obs)[0] >= 0).sum())
    hb = []
    n_beam = 0
    for k in range(16):
        phb, _, cnt1, _ = _all_photons(seg, 1000 + k, (c, r, MARGIN), yield_per_MeV=40.0)
        hb.append(int((orc.telescopes(phb, tel, n_obs)[0] >= 0).sum()))
        n_beam += int(cnt1.sum())
    mean_b = float(np.mean(hb))
    sigma = np.sqrt(h_iso + mean_b / len(hb))
    assert abs(h_iso - mean_b) <= 4.0 * sigma, (h_iso, mean_b, sigma)
    assert h_iso > 1000
    # the photon reduction: at least the 50% the paper reports as the worst case
    assert n_beam / 16 < 0.5 * cnt0.sum()


def test_segments_inside_the_area_stay_isotropic():
    seg = wl.fluorescence_near_array(400)
    c, _ = _area(_tel())
    atm = _atm()
    cnt0, mu0, _ = orc.counts(seg, atm, "fluorescence", SEED, yield_per_MeV=YIELD)
    cnt1, mu1, _ = orc.counts(seg, atm, "fluorescence", SEED, yield_per_MeV=YIELD, beam=(c, 1e6, MARGIN))
    assert np.array_equal(cnt0, cnt1) and np.array_equal(mu0, mu1)
    ph, s_of, _, _ = _all_photons(seg, SEED, (c, 1e6, MARGIN), yield_per_MeV=50.0)
    # isotropic: the vertical component is uniform on (-1, 1)
    assert stats.kstest((ph["ue"][:, 2] + 1.0) / 2.0, "uniform").pvalue > 1e-3


@pytest.mark.parametrize("margin_deg", [0.0, 5.0])
def test_margin_widens_the_cone(margin_deg):
    seg = wl.fluorescence_near_array(100)
    c, r = _area(_tel())
    _, om0, _ = orc.beam_cap(seg, (c, r, 0.0))
    _, om1, _ = orc.beam_cap(seg, (c, r, np.radians(margin_deg)))
    if margin_deg == 0.0:
        assert np.array_equal(om0, om1)
    else:
        assert np.all(om1[om0 < 2.0] > om0[om0 < 2.0])
