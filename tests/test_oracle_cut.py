"""Pins of the oracle's Cherenkov angular particle cut (section 1.2.1,
Fig. 2).

The cut keeps a segment when the angle between its flight direction and the
vector from its midpoint to a target point (the array centre, or each
telescope) is at most the cut angle. The pins check the oracle's test
against angles computed here with arccos on unit vectors, on constructed
geometry with known angles, and check that the cut only removes segments:
kept segments draw the same counts as without the cut, cut ones draw none.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2309_15861_amd import workloads as wl

SEED = 11
SHOWER = wl.shower_cherenkov(200_000, 2)
TEL = wl.telescopes_16()
CENTRE = [[0.0, 0.0, wl.H_OBS]]


def _angles_deg(seg, points):
    """Minimum angle (deg) per segment between direction and midpoint->point."""
    d = np.stack([seg["dx"], seg["dy"], seg["dz"]], axis=1)
    u = d / np.linalg.norm(d, axis=1, keepdims=True)
    m = np.stack([seg["x0"], seg["y0"], seg["z0"]], axis=1) + 0.5 * seg["length"][:, None] * u
    best = np.full(len(u), np.inf)
    for p in np.asarray(points, float).reshape(-1, 3):
        v = p[None, :] - m
        v = v / np.linalg.norm(v, axis=1, keepdims=True)
        c = np.clip(np.sum(u * v, axis=1), -1.0, 1.0)
        best = np.minimum(best, np.degrees(np.arccos(c)))
    return best


def _segments(dirs, starts, length=10.0):
    n = len(dirs)
    return wl._segments(n, starts[:, 0], starts[:, 1], starts[:, 2], np.asarray(dirs, float),
                        np.full(n, length), np.full(n, 1000.0), np.zeros(n))


def test_constructed_angles():
    """Segments aimed at known angles from the target at the origin: 0, 5.9,
    6.1, 90 and 180 degrees, with a 6 degree cut."""
    angs = np.radians([0.0, 5.9, 6.1, 90.0, 180.0])
    z = 10000.0
    # midpoint at (0, 0, z); direction tilted from straight down (towards the origin) by a
    dirs = np.stack([np.sin(angs), np.zeros_like(angs), -np.cos(angs)], axis=1)
    starts = np.array([[0.0, 0.0, z]]) - 5.0 * dirs  # length 10: midpoint at (0, 0, z)
    seg = _segments(dirs, starts)
    keep = orc.passes_cut(seg, [[0.0, 0.0, 0.0]], np.cos(np.radians(6.0)))
    assert keep.tolist() == [True, True, False, False, False]


def test_angle_is_taken_at_the_midpoint():
    """Long segments near the target, where the angle changes along the track:
    one fails at its midpoint but passes at its start, the other passes at its
    midpoint but fails at its end."""
    z, L = 5000.0, 2000.0
    seg_rows = []
    for a_mid in (6.1, 5.9):
        a = np.radians(a_mid)
        d = np.array([np.sin(a), 0.0, -np.cos(a)])
        seg_rows.append((np.array([0.0, 0.0, z]) - 0.5 * L * d, d))
    starts = np.array([r[0] for r in seg_rows])
    dirs = np.array([r[1] for r in seg_rows])
    seg = _segments(dirs, starts, length=L)

    def angle_at(t):
        pos = starts + t * dirs
        v = -pos / np.linalg.norm(pos, axis=1, keepdims=True)
        return np.degrees(np.arccos(np.sum(v * dirs, axis=1)))

    a0, am, a1 = angle_at(0.0), angle_at(0.5 * L), angle_at(L)
    assert a0[0] < 6.0 < am[0] and am[1] < 6.0 < a1[1]
    keep = orc.passes_cut(seg, [[0.0, 0.0, 0.0]], np.cos(np.radians(6.0)))
    assert keep.tolist() == [False, True]


def test_matches_arccos_on_shower_segments():
    seg = wl.subsample(SHOWER, np.arange(0, 200_000, 97))
    pts = TEL[:, :3]
    for cut_deg, points in ((6.0, CENTRE), (6.0, pts), (2.0, pts), (20.0, pts[:3])):
        ang = _angles_deg(seg, points)
        keep = orc.passes_cut(seg, points, np.cos(np.radians(cut_deg)))
        clear = np.abs(ang - cut_deg) > 1e-6
        assert clear.sum() > 0.99 * len(ang)
        assert np.array_equal(keep[clear], (ang <= cut_deg)[clear]), cut_deg
        assert 0 < keep.sum() < len(keep)


def test_minimum_over_points_is_union():
    seg = wl.subsample(SHOWER, np.arange(0, 200_000, 211))
    pts = TEL[:, :3]
    c = np.cos(np.radians(4.0))
    union = np.zeros(len(seg["x0"]), bool)
    for p in pts:
        union |= orc.passes_cut(seg, [p], c)
    assert np.array_equal(orc.passes_cut(seg, pts, c), union)


def test_no_points_or_full_angle_keeps_everything():
    seg = wl.subsample(SHOWER, np.arange(0, 200_000, 401))
    n = len(seg["x0"])
    assert orc.passes_cut(seg, np.zeros((0, 3)), 1.0).all()
    assert orc.passes_cut(seg, [[0.0, 0.0, 0.0]], -1.0).sum() == n


@pytest.mark.parametrize("points,cut_deg", [(CENTRE, 6.0), (None, 6.0)])
def test_cut_only_removes_segments(points, cut_deg):
    """Kept segments draw the same count as without the cut (same random
    stream); cut segments have mean 0 and count 0."""
    seg = wl.subsample(SHOWER, np.arange(0, 200_000, 53))
    pts = TEL[:, :3] if points is None else points
    atm = orc.Atmosphere.from_dict(wl.default_atmosphere(absorption=True))
    c = np.cos(np.radians(cut_deg))
    cnt0, mu0, _ = orc.counts(seg, atm, "cherenkov", SEED)
    cnt1, mu1, _ = orc.counts(seg, atm, "cherenkov", SEED, cut=(pts, c))
    keep = orc.passes_cut(seg, pts, c)
    assert np.array_equal(cnt1[keep], cnt0[keep])
    assert np.array_equal(mu1[keep], mu0[keep])
    assert np.all(cnt1[~keep] == 0) and np.all(mu1[~keep] == 0.0)
    assert keep.sum() < len(keep)


def test_fluorescence_ignores_cut():
    seg = wl.subsample(SHOWER, np.arange(0, 200_000, 307))
    atm = orc.Atmosphere.from_dict(wl.default_atmosphere(absorption=True))
    cnt0, _, _ = orc.counts(seg, atm, "fluorescence", SEED)
    cnt1, _, _ = orc.counts(seg, atm, "fluorescence", SEED, cut=([[0.0, 0.0, 0.0]], 1.0))
    assert np.array_equal(cnt0, cnt1)
