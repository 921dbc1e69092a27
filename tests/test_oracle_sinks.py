"""Pins of the oracle's collection step by brute force on tiny inputs.

Telescope hits: distance from each sphere centre to the arrival line
|(c - r) x u| against R, entry point by projection; ground grid: direct
floor binning; per-telescope and per-cell photon counts by brute force.
"""
import numpy as np

from paper_2309_15861_amd import workloads as W


def small_run(oracle, n_seg=40, seed=12):
    a = W.default_atmosphere(absorption=True)
    atm = oracle.Atmosphere.from_dict(a)
    seg = W.plain_cherenkov(n_seg, seed=seed)
    cnt = oracle.counts(seg, atm, "cherenkov", seed)[0]
    off = oracle.offsets_of(cnt)
    ph = oracle.photons_all(seg, atm, "cherenkov", seed, off)
    return a, atm, ph


def brute_telescopes(ph, tel, n_obs):
    C = 0.299792458
    tid = np.full(len(ph), -1)
    rec = np.zeros((len(ph), 5))
    for q in range(len(ph)):
        if ph["status"][q] != 0:
            continue
        r = np.array([ph["xl"][q], ph["yl"][q], ph["zl"][q]])
        u = ph["ul"][q]
        best, best_s = -1, np.inf
        for k, (cx, cy, cz, R) in enumerate(tel):
            c = np.array([cx, cy, cz])
            dist = np.linalg.norm(np.cross(c - r, u))
            if dist > R:
                continue
            s = np.dot(c - r, u) - np.sqrt(R * R - dist * dist)
            if s < best_s:
                best, best_s = k, s
        if best >= 0:
            tid[q] = best
            p = r + best_s * u
            rec[q] = (p[0], p[1], p[2], ph["tl"][q] + n_obs * best_s / C, best_s)
    return tid, rec


def test_telescope_hits_brute_force(oracle):
    a, atm, ph = small_run(oracle)
    # large spheres around where this small sample lands, so that many hit
    tel = W.telescopes_16(h_obs=a["h_obs"], radius=45.0, spacing=100.0)
    tel[:, 0] += np.median(ph["xl"])
    tel[:, 1] += np.median(ph["yl"])
    n_obs = atm.index(a["h_obs"])
    tid, rec = oracle.telescopes(ph, tel, n_obs)
    tid_b, rec_b = brute_telescopes(ph, tel, n_obs)
    assert (tid_b >= 0).sum() > 50
    assert np.array_equal(tid, tid_b)
    hit = tid >= 0
    assert np.allclose(rec[hit], rec_b[hit], rtol=1e-12, atol=1e-8)
    # the entry point lies on the sphere
    c = tel[tid[hit], :3]
    assert np.allclose(np.linalg.norm(rec[hit, :3] - c, axis=1), tel[tid[hit], 3], rtol=1e-10)
    # per-telescope counts
    assert np.array_equal(np.bincount(tid[hit], minlength=16), np.bincount(tid_b[tid_b >= 0], minlength=16))


def test_ground_grid_brute_force(oracle):
    a, atm, ph = small_run(oracle, n_seg=60, seed=13)
    g = dict(x_min=-600.0, y_min=-550.0, cell=25.0, nx=40, ny=36)
    cell = oracle.grid(ph, g["x_min"], g["y_min"], g["cell"], g["nx"], g["ny"])
    ix = np.floor((ph["xl"] - g["x_min"]) / g["cell"]).astype(int)
    iy = np.floor((ph["yl"] - g["y_min"]) / g["cell"]).astype(int)
    inside = (ix >= 0) & (iy >= 0) & (ix < g["nx"]) & (iy < g["ny"]) & (ph["status"] == 0)
    ref = np.where(inside, iy * g["nx"] + ix, -1)
    assert np.array_equal(cell, ref)
    assert inside.sum() > 100 and (~inside).sum() > 0
    hist = np.bincount(cell[cell >= 0], minlength=g["nx"] * g["ny"])
    hist_b = np.zeros(g["nx"] * g["ny"], int)
    for q in range(len(ph)):
        if inside[q]:
            hist_b[iy[q] * g["nx"] + ix[q]] += 1
    assert np.array_equal(hist, hist_b)
