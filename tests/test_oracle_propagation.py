"""Pins of the oracle's propagation (quadrature of the ray integrals).

* Closed forms of the four layer integrals, obtained by antidifferentiation
  in eps = n - 1 (log branch for S < 1, arcsine branch for S > 1), evaluated
  in 40-digit mpmath: a different route from the oracle's Gauss-Kronrod
  quadrature of the plain integrands.
* An RK4 integration of the ray equation d(n dr/ds)/ds = grad n (Fermat's
  principle), which does not assume Snell's invariant.
* Homogeneous medium: straight line, t = n L / c, Beer-Lambert exp(-k L).
* Vertical ray: no displacement, delay = eta0 * column density / c.
* Snell invariant, azimuth, unit arrival direction; UP and BELOW statuses.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from paper_2309_15861_amd import workloads as W

C = 0.299792458
INF = float("inf")


def atm_dict(h_obs=2200.0, absorption=False):
    return W.default_atmosphere(absorption=absorption, h_obs=h_obs)


# ------------------------------------------------------------- closed forms --
def mp_density(h, hb, H):
    """rho/rho0 of the layered model in mpmath (input model, pinned in
    test_oracle_generation)."""
    rho = mp.mpf(1)
    i = 0
    for k in range(len(hb)):
        if hb[k] <= h:
            i = k
    for k in range(i):
        rho *= mp.e ** (-(mp.mpf(hb[k + 1]) - hb[k]) / H[k])
    return rho * mp.e ** (-(mp.mpf(h) - hb[i]) / H[i]), i


def mp_piece(eps_a, eps_b, H, S, a, b, eta0):
    """Closed-form layer integrals over [a, b] (a < b) with eps = eta0*rho
    falling exponentially with scale height H."""
    na, nb = 1 + eps_a, 1 + eps_b
    ra, rb = mp.sqrt(na * na - S * S), mp.sqrt(nb * nb - S * S)
    if S < 1:
        Cc = mp.sqrt(1 - S * S)
        ds = (b - a) / Cc + (H / Cc) * mp.log((Cc * rb + Cc * Cc + eps_b) / (Cc * ra + Cc * Cc + eps_a))
    else:
        Kk = mp.sqrt(S * S - 1)
        ds = (H / Kk) * (mp.asin((eps_a - Kk * Kk) / (eps_a * S)) - mp.asin((eps_b - Kk * Kk) / (eps_b * S)))
    Lg = mp.log((na + ra) / (nb + rb))
    P = ds + H * Lg
    O = ds + H * Lg + H * (ra - rb)
    T = (H / eta0) * (ra - rb)
    return [ds, P, O, T]


def mp_ray_integrals(atm, z_e, cos_e, h_lo):
    mp.mp.dps = 40
    hb = [mp.mpf(x) for x in atm["h_base"]]
    H = [mp.mpf(x) for x in atm["scale_height"]]
    eta0 = mp.mpf(atm["n0_minus_1"])
    z_e = mp.mpf(z_e)
    rho_e, le = mp_density(z_e, hb, H)
    ne = 1 + eta0 * rho_e
    S = ne * mp.sqrt(1 - mp.mpf(cos_e) ** 2)
    G = [mp.mpf(0)] * 4
    for l in range(le + 1):
        lo = max(mp.mpf(h_lo), hb[l]) if l > 0 else mp.mpf(h_lo)
        hi = hb[l + 1] if l < le else z_e
        if not lo < hi:
            continue
        ea = eta0 * mp_density(lo, hb, H)[0]
        eb = ea * mp.e ** (-(hi - lo) / H[l])      # layer l's own exponential up to hi
        piece = mp_piece(ea, eb, H[l], S, lo, hi, eta0)
        G = [g + p for g, p in zip(G, piece)]
    return [float(g) for g in G]


@pytest.mark.parametrize("z_e", [2500.0, 4000.0, 10000.0, 25000.0])
@pytest.mark.parametrize("zenith", [0.0, 1.4, 20.0, 45.0, 60.0, 85.0, 88.5, 89.5, 89.9, 89.99])
def test_ray_integrals_match_closed_forms(oracle, z_e, zenith):
    a = atm_dict()
    atm = oracle.Atmosphere.from_dict(a)
    ce = math.cos(math.radians(zenith))
    got = atm.ray_integrals(z_e, ce, 2200.0)
    ref = mp_ray_integrals(a, z_e, ce, 2200.0)
    tol = 1e-12 if zenith < 88 else 2e-11
    for g, r in zip(got, ref):
        assert abs(g - r) <= tol * abs(r), (zenith, z_e, got, ref)


def test_closed_form_reference_values(oracle):
    """Horizontal displacements S*G0 (m) from 2.2 km up to the emission
    height for a few rays of the default atmosphere."""
    atm = oracle.Atmosphere.from_dict(atm_dict())
    cases = [(4000.0, 20.0, 655.132576), (30000.0, 60.0, None), (10000.0, 85.0, None),
             (4000.0, 89.9, 343756.35)]
    for z_e, zen, ref in cases:
        ce = math.cos(math.radians(zen))
        G = atm.ray_integrals(z_e, ce, 2200.0)
        disp = atm.index(z_e) * math.sin(math.radians(zen)) * G[0]
        straight = (z_e - 2200.0) * math.tan(math.radians(zen))
        assert disp < straight                      # refraction bends towards the vertical
        if ref is not None:
            assert abs(disp - ref) < 1e-6 * ref


# ---------------------------------------------------------- ray equation RK4 --
def np_density(z, hb, H):
    hb = np.asarray(hb)
    H = np.asarray(H)
    rb = np.ones(len(hb))
    for k in range(len(hb) - 1):
        rb[k + 1] = rb[k] * np.exp(-(hb[k + 1] - hb[k]) / H[k])
    i = np.clip(np.searchsorted(hb, z, side="right") - 1, 0, len(hb) - 1)
    return rb[i] * np.exp(-(z - hb[i]) / H[i]), H[i]


def trace_rays(a, ze, u, steps=400):
    """RK4 in z of the ray equation: p = n dr/ds, dp/ds = grad n, so p_x, p_y
    are constant and dp_z/dz = n n'(z)/p_z, dx/dz = p_x/p_z, and the path,
    optical path and density-weighted path grow by n/p_z, n^2/p_z,
    rho n/p_z per dz (z decreasing, p_z < 0). Pieces are aligned with layer
    boundaries."""
    hb, H, eta0, h_obs = a["h_base"], a["scale_height"], a["n0_minus_1"], a["h_obs"]
    rho_e, _ = np_density(ze, hb, H)
    ne = 1 + eta0 * rho_e
    px, py, pz = ne * u[:, 0], ne * u[:, 1], ne * u[:, 2]
    x = np.zeros(len(ze))
    y = np.zeros(len(ze))
    P = np.zeros(len(ze))
    O = np.zeros(len(ze))
    T = np.zeros(len(ze))

    def rhs(z, state, qx, qy):
        _, _, pzz, _, _, _ = state
        rho, Hl = np_density(z, hb, H)
        n = 1 + eta0 * rho
        dn = -eta0 * rho / Hl
        return (qx / pzz, qy / pzz, n * dn / pzz, n / pzz, n * n / pzz, rho * n / pzz)

    # break points: emission, layer boundaries below it, observation level;
    # the first and last stage of a step are evaluated just inside the piece
    for i in range(len(ze)):
        pts = [ze[i]] + [h for h in sorted(hb, reverse=True) if h_obs < h < ze[i]] + [h_obs]
        st = (0.0, 0.0, pz[i], 0.0, 0.0, 0.0)
        qx, qy = px[i], py[i]
        for top, bot in zip(pts[:-1], pts[1:]):
            dz = (bot - top) / steps
            z = top
            for _ in range(steps):
                k1 = rhs(z + 1e-9 * dz, st, qx, qy)
                k2 = rhs(z + 0.5 * dz, tuple(s + 0.5 * dz * k for s, k in zip(st, k1)), qx, qy)
                k3 = rhs(z + 0.5 * dz, tuple(s + 0.5 * dz * k for s, k in zip(st, k2)), qx, qy)
                k4 = rhs(z + dz * (1 - 1e-9), tuple(s + dz * k for s, k in zip(st, k3)), qx, qy)
                st = tuple(s + dz / 6 * (q1 + 2 * q2 + 2 * q3 + q4)
                           for s, q1, q2, q3, q4 in zip(st, k1, k2, k3, k4))
                z += dz
        x[i], y[i], pzf, P[i], O[i], T[i] = st
        pz[i] = pzf
    rho_o, _ = np_density(h_obs, hb, H)
    n_obs = 1 + eta0 * rho_o
    return x, y, P, O, T, np.stack([px / n_obs, py / n_obs, pz / n_obs], 1)


def test_propagation_matches_ray_equation(oracle):
    a = atm_dict(absorption=True)
    atm = oracle.Atmosphere.from_dict(a)
    n = 12
    seg = W.plain_cherenkov(200, seed=21)
    cnt = oracle.counts(seg, atm, "cherenkov", 9)[0]
    s_list = np.nonzero(cnt)[0][:n]
    ph = oracle.photons(seg, atm, "cherenkov", 9, s_list, np.zeros(n, np.uint32))
    # add a few steeper and slanted rays from fluorescence-like directions
    fz = np.array([-0.9, -0.5, -0.2])
    extra = np.stack([np.sqrt(1 - fz ** 2) * 0.6, np.sqrt(1 - fz ** 2) * 0.8, fz], 1)
    ze = np.concatenate([ph["ze"], [12000.0, 7000.0, 3000.0]])
    u = np.concatenate([ph["ue"], extra])
    x, y, P, O, T, ul = trace_rays(a, ze, u, steps=300)
    for i in range(len(ze)):
        G = atm.ray_integrals(ze[i], -u[i, 2], a["h_obs"])
        ne = atm.index(ze[i])
        disp = np.hypot(u[i, 0], u[i, 1]) * ne * G[0]
        assert abs(ne * u[i, 0] * G[0] - x[i]) <= 1e-9 * max(disp, 1.0)
        assert abs(ne * u[i, 1] * G[0] - y[i]) <= 1e-9 * max(disp, 1.0)
        assert abs(G[1] - P[i]) <= 1e-10 * P[i]
        assert abs(G[2] - O[i]) <= 1e-10 * O[i]
        assert abs(G[3] - T[i]) <= 1e-10 * T[i]
    # the oracle's photons, end to end
    for i in range(n):
        assert abs(ph["xl"][i] - ph["xe"][i] - x[i]) <= 1e-9 * max(abs(x[i]), 1.0)
        assert abs((ph["tl"][i] - ph["te"][i]) - O[i] / C) < 1e-6
        assert abs(ph["path"][i] - P[i]) < 1e-6
        assert np.allclose(ph["ul"][i], ul[i], atol=1e-12)
        k = atm.abs_k(ph["lam"][i])
        assert abs(ph["weight"][i] - math.exp(-k * T[i])) < 1e-12


# ------------------------------------------------------ homogeneous / vertical --
def test_homogeneous_medium_is_straight_line(oracle):
    lam = np.array([300.0, 400.0, 600.0])
    kk = np.array([3e-5, 2e-5, 1e-5])
    eta0 = 2.9e-4
    atm = oracle.Atmosphere([0.0, 5000.0, 20000.0], [INF, INF, INF], eta0, 1000.0, lam, kk)
    seg = W.plain_cherenkov(50, seed=8)
    cnt = oracle.counts(seg, atm, "cherenkov", 2)[0]
    s_list = np.repeat(np.nonzero(cnt)[0], 3)
    j_list = np.tile([0, 1, 2], len(s_list) // 3)
    ph = oracle.photons(seg, atm, "cherenkov", 2, s_list, j_list)
    ue = ph["ue"]
    L = (ph["ze"] - 1000.0) / -ue[:, 2]
    assert np.allclose(ph["xl"], ph["xe"] + ue[:, 0] * L, rtol=0, atol=1e-9 * L.max())
    assert np.allclose(ph["yl"], ph["ye"] + ue[:, 1] * L, rtol=0, atol=1e-9 * L.max())
    assert np.allclose(ph["path"], L, rtol=1e-12)
    assert np.allclose(ph["tl"] - ph["te"], (1 + eta0) * L / C, rtol=1e-12)
    k = np.interp(ph["lam"], lam, kk)
    assert np.allclose(ph["weight"], np.exp(-k * L), rtol=1e-12)
    assert np.allclose(ph["ul"], ue, atol=1e-15)


def test_vertical_ray_closed_forms(oracle):
    a = atm_dict()
    atm = oracle.Atmosphere.from_dict(a)
    G = atm.ray_integrals(10000.0, 1.0, 2200.0)
    # column density: sum over pieces of H_i (rho(bottom) - rho(top))
    col = 0.0
    pieces = [(2200.0, 4000.0, 0), (4000.0, 10000.0, 1)]
    for lo, hi, l in pieces:
        col += a["scale_height"][l] * (atm.density(lo) - atm.density(hi * (1 - 1e-16)))
    assert abs(G[3] - col) < 1e-12 * col
    assert abs(col - 4226.757) < 1e-3
    assert abs(G[1] - 7800.0) < 1e-10                     # path = height difference
    delay = (G[2] - 7800.0) / C                           # refraction delay [ns]
    assert abs(delay - a["n0_minus_1"] * col / C) < 1e-9
    assert abs(delay - 4.0887) < 1e-4


def test_snell_invariant_and_statuses(oracle):
    a = atm_dict(absorption=True)
    atm = oracle.Atmosphere.from_dict(a)
    lines, rel = W.fluorescence_lines()
    seg = W.fluorescence(30, seed=4)
    cnt = oracle.counts(seg, atm, "fluor", 4)[0]
    s_list = np.repeat(np.arange(30), 40)
    j_list = np.tile(np.arange(40), 30)
    ph = oracle.photons(seg, atm, "fluor", 4, s_list, j_list, lines_nm=lines, line_rel=rel)
    up = ph["ue"][:, 2] >= 0
    assert np.all(ph["status"][up] == oracle.UP)
    ok = ~up
    assert np.all(ph["status"][ok] == oracle.LANDED)
    n_e = np.array([atm.index(z) for z in ph["ze"][ok]])
    n_o = atm.index(a["h_obs"])
    s_e = np.hypot(ph["ue"][ok, 0], ph["ue"][ok, 1])
    s_o = np.hypot(ph["ul"][ok, 0], ph["ul"][ok, 1])
    assert np.allclose(n_o * s_o, n_e * s_e, rtol=1e-14, atol=1e-15)
    az_e = np.arctan2(ph["ue"][ok, 1], ph["ue"][ok, 0])
    az_o = np.arctan2(ph["ul"][ok, 1], ph["ul"][ok, 0])
    assert np.allclose(az_e, az_o, atol=1e-12)
    assert np.allclose(np.linalg.norm(ph["ul"][ok], axis=1), 1.0, atol=1e-14)
    # below the observation level
    b = atm_dict(h_obs=40000.0)
    atm_b = oracle.Atmosphere.from_dict(b)
    ph_b = oracle.photons(seg, atm_b, "fluor", 4, s_list[:50], j_list[:50], lines_nm=lines,
                          line_rel=rel)
    down = ph_b["ue"][:, 2] < 0
    assert np.all(ph_b["status"][down] == oracle.BELOW)


def test_absorption_table_interpolation(oracle):
    lam = np.array([300.0, 350.0, 500.0])
    kk = np.array([4e-5, 2e-5, 1e-5])
    atm = oracle.Atmosphere([0.0], [8000.0], 2.9e-4, 0.0, lam, kk)
    assert atm.abs_k(250.0) == 4e-5 and atm.abs_k(700.0) == 1e-5
    for x in (300.0, 350.0, 500.0):
        assert atm.abs_k(x) == kk[list(lam).index(x)]
    assert abs(atm.abs_k(325.0) - 3e-5) < 1e-18
    assert abs(atm.abs_k(425.0) - 1.5e-5) < 1e-18
