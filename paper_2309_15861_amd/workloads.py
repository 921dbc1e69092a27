"""Seeded synthetic inputs: track segments, atmosphere, lines, telescopes.

These generators only shape the inputs (segment geometry, energies, tables).
They contain none of the photon method's arithmetic and serve the HIP path,
the oracle, the tests and the benchmark alike. Every array is float64 except
the integer id fields, and every draw comes from numpy's PCG64 seeded per
workload, so each consumer sees identical inputs.

The paper's own workloads (summed 500 GeV gamma showers from full cascade
simulations, section 3.1) are not available; the shapes below stand in for
them.
"""
from __future__ import annotations

import numpy as np

ME_MEV = 0.51099895          # electron rest energy [MeV]
C_M_PER_NS = 0.299792458     # speed of light [m/ns]

# Five exponential layers with boundaries 0/4/10/40/100 km.  The first four
# scale heights are close to the US-standard (Linsley) parametrisation; any
# positive values are valid inputs.
H_BASE = (0.0, 4000.0, 10000.0, 40000.0, 100000.0)
SCALE_HEIGHT = (9941.8638, 8781.5355, 6361.4304, 7721.7016, 7721.7016)
N0_MINUS_1 = 2.9e-4
H_OBS = 2200.0

# Rayleigh-like absorption k(lambda) = K400 (lambda/400 nm)^-4 at sea-level
# density; K400 makes the vertical transmission from 10 km down to 2.2 km at
# 400 nm about 0.85.
K400_PER_M = 3.845e-5


def default_atmosphere(absorption: bool = False, h_obs: float = H_OBS) -> dict:
    atm = dict(h_base=np.array(H_BASE), scale_height=np.array(SCALE_HEIGHT),
               n0_minus_1=N0_MINUS_1, h_obs=float(h_obs))
    if absorption:
        lam = np.arange(290.0, 611.0, 10.0)
        atm["abs_lambda_nm"] = lam
        atm["abs_k_per_m"] = K400_PER_M * (lam / 400.0) ** -4
    else:
        atm["abs_lambda_nm"] = None
        atm["abs_k_per_m"] = None
    return atm


def beta_from_energy(e_total_mev):
    """Speed of an electron of total energy E (kinematics of the input)."""
    g = np.asarray(e_total_mev, dtype=np.float64) / ME_MEV
    return np.sqrt((g - 1.0) * (g + 1.0)) / g


def telescopes_16(h_obs: float = H_OBS, radius: float = 6.0, spacing: float = 100.0) -> np.ndarray:
    """16 spheres on a 4x4 grid of 100 m pitch around the core, centres at
    the observation level; rows (x, y, z, R)."""
    xs = (np.arange(4) - 1.5) * spacing
    rows = [(x, y, h_obs, radius) for y in xs for x in xs]
    return np.array(rows, dtype=np.float64)


def grid_64() -> dict:
    """64 x 64 ground grid of 10 m cells centred on the core."""
    return dict(x_min=-320.0, y_min=-320.0, cell=10.0, nx=64, ny=64)


def _segments(n, x0, y0, z0, d, length, e, t0, dedx=None, shower=None, index=None):
    seg = dict(x0=np.ascontiguousarray(x0, np.float64), y0=np.ascontiguousarray(y0, np.float64),
               z0=np.ascontiguousarray(z0, np.float64),
               dx=np.ascontiguousarray(d[:, 0]), dy=np.ascontiguousarray(d[:, 1]),
               dz=np.ascontiguousarray(d[:, 2]), length=np.ascontiguousarray(length, np.float64),
               beta=beta_from_energy(e), t0=np.ascontiguousarray(t0, np.float64),
               dedx=None if dedx is None else np.ascontiguousarray(dedx, np.float64),
               charge=np.full(n, -1, np.int32),
               shower=np.zeros(n, np.uint32) if shower is None else shower.astype(np.uint32),
               index_in_shower=(np.arange(n, dtype=np.uint32) if index is None
                                else index.astype(np.uint32)))
    seg["energy_mev"] = np.asarray(e, np.float64)
    return seg


def _cone_dirs(rng, n, axis, half_angle_rad):
    """Directions uniform in solid angle within half_angle of the unit axis."""
    ct = rng.uniform(np.cos(half_angle_rad), 1.0, n)
    st = np.sqrt((1.0 - ct) * (1.0 + ct))
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    e1, e2 = _perp_basis(axis)
    return (ct[:, None] * axis[None, :] + (st * np.cos(ph))[:, None] * e1[None, :]
            + (st * np.sin(ph))[:, None] * e2[None, :])


def _perp_basis(axis):
    axis = np.asarray(axis, np.float64)
    helper = np.array([1.0, 0.0, 0.0]) if abs(axis[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(axis, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(axis, e1)
    return e1, e2


def plain_cherenkov(n: int = 1000, seed: int = 1) -> dict:
    """1,000 electron segments: start height U(5,30) km, length U(1,50) m,
    direction within 5 degrees of the downward vertical, total energy
    log-uniform 50 MeV..1 GeV; t0 counts from a front at 30 km."""
    rng = np.random.default_rng(seed)
    z0 = rng.uniform(5000.0, 30000.0, n)
    length = rng.uniform(1.0, 50.0, n)
    d = _cone_dirs(rng, n, np.array([0.0, 0.0, -1.0]), np.radians(5.0))
    e = np.exp(rng.uniform(np.log(50.0), np.log(1000.0), n))
    t0 = (30000.0 - z0) / C_M_PER_NS
    return _segments(n, np.zeros(n), np.zeros(n), z0, d, length, e, t0)


def _shower_profile(rng, n, zenith_deg, azimuth_deg, core, h_obs, e_range, lateral_sigma,
                    length_range, smear=True):
    """Segments of a synthetic electromagnetic shower: longitudinal depth from a
    gamma-distribution profile, Gaussian lateral spread about the axis,
    power-law E^-2 energies and direction smear ~ 21.2 MeV / E."""
    th, az = np.radians(zenith_deg), np.radians(azimuth_deg)
    axis = np.array([np.sin(th) * np.cos(az), np.sin(th) * np.sin(az), -np.cos(th)])
    e1, e2 = _perp_basis(axis)
    x0_rad = 36.62          # radiation length of air [g/cm^2]
    b = 0.5
    e_max = e_range[1]
    t_max = np.log(e_max / 87.0) + 0.5
    a = b * t_max + 1.0
    out = {k: np.empty(0) for k in ("x0", "y0", "z0", "e", "L")}
    dirs = np.empty((0, 3))
    need = n
    while need > 0:
        m = int(need * 1.3) + 16
        depth = rng.gamma(a, 1.0 / b, m) * x0_rad                  # slant depth
        xv = depth * np.cos(th)                                   # vertical depth
        xv = np.minimum(xv, 1030.0)
        h = -8400.0 * np.log(xv / 1036.0)                         # isothermal overburden
        lam = (h - core[2]) / np.cos(th)                          # back up along the axis
        p = core[None, :] - lam[:, None] * axis[None, :]
        g1 = rng.normal(0.0, lateral_sigma, m)
        g2 = rng.normal(0.0, lateral_sigma, m)
        p = p + g1[:, None] * e1[None, :] + g2[:, None] * e2[None, :]
        u = rng.uniform(0.0, 1.0, m)
        e = 1.0 / (1.0 / e_range[0] - u * (1.0 / e_range[0] - 1.0 / e_range[1]))
        if smear:
            sig = np.minimum(21.2 / e, 0.5)
            ang = sig * np.sqrt(rng.normal(size=m) ** 2 + rng.normal(size=m) ** 2)
        else:
            ang = np.zeros(m)
        phi = rng.uniform(0.0, 2.0 * np.pi, m)
        d = (np.cos(ang)[:, None] * axis[None, :]
             + (np.sin(ang) * np.cos(phi))[:, None] * e1[None, :]
             + (np.sin(ang) * np.sin(phi))[:, None] * e2[None, :])
        L = rng.uniform(length_range[0], length_range[1], m)
        ok = (p[:, 2] > h_obs + 1.0) & (p[:, 2] + L * d[:, 2] > h_obs + 1.0)
        take = np.nonzero(ok)[0][:need]
        out["x0"] = np.concatenate([out["x0"], p[take, 0]])
        out["y0"] = np.concatenate([out["y0"], p[take, 1]])
        out["z0"] = np.concatenate([out["z0"], p[take, 2]])
        out["e"] = np.concatenate([out["e"], e[take]])
        out["L"] = np.concatenate([out["L"], L[take]])
        dirs = np.concatenate([dirs, d[take]])
        need = n - len(out["x0"])
    # time: distance travelled along the axis from the 30 km plane at c
    lam_top = (30000.0 - core[2]) / np.cos(th)
    along = lam_top - ((out["z0"] - core[2]) / np.cos(th))
    t0 = along / C_M_PER_NS
    return out, dirs, t0


def shower_cherenkov(n: int = 200_000, seed: int = 2) -> dict:
    """Shower-shaped Cherenkov input: 1 TeV gamma-like longitudinal profile,
    electron energies E^-2 from 20 MeV, lateral sigma 50 m, zenith 20 deg,
    lengths U(1,30) m."""
    rng = np.random.default_rng(seed)
    out, d, t0 = _shower_profile(rng, n, 20.0, 0.0, np.array([0.0, 0.0, H_OBS]), H_OBS,
                                 (20.0, 1.0e6), 50.0, (1.0, 30.0))
    return _segments(n, out["x0"], out["y0"], out["z0"], d, out["L"], out["e"], t0)


def fluorescence(n: int = 100_000, seed: int = 3) -> dict:
    """Fluorescence input: geometry as the plain Cherenkov set, dE/dx
    log-uniform 1..10 MeV/m."""
    seg = plain_cherenkov(n, seed)
    rng = np.random.default_rng(seed + 1000)
    seg["dedx"] = np.exp(rng.uniform(0.0, np.log(10.0), n))
    return seg


def fluorescence_near_array(n: int = 400, seed: int = 6) -> dict:
    """Fluorescence tracks 0.3..2.8 km above the observation level within
    800 m of the array centre, isotropic directions, lengths 5..30 m, dE/dx
    log-uniform 1..10 MeV/m: close enough that isotropic emission hits the
    telescopes often, for comparing beamed and isotropic emission."""
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-800.0, 800.0, n)
    y0 = rng.uniform(-800.0, 800.0, n)
    z0 = H_OBS + rng.uniform(300.0, 2800.0, n)
    ct = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    st = np.sqrt(1.0 - ct * ct)
    d = np.stack([st * np.cos(phi), st * np.sin(phi), ct], axis=1)
    length = rng.uniform(5.0, 30.0, n)
    e = np.exp(rng.uniform(np.log(50.0), np.log(5000.0), n))
    seg = _segments(n, x0, y0, z0, d, length, e, np.zeros(n))
    seg["dedx"] = np.exp(rng.uniform(0.0, np.log(10.0), n))
    return seg


def fluorescence_lines(seed: int = 3, n_lines: int = 21):
    """21 emission lines, wavelengths sorted U(300,430) nm, relative yields
    U(0.05,1)."""
    rng = np.random.default_rng(seed + 2000)
    lam = np.sort(rng.uniform(300.0, 430.0, n_lines))
    rel = rng.uniform(0.05, 1.0, n_lines)
    return lam, rel


FLUOR_YIELD_PER_MEV = 10.0


def batched_showers(seed: int = 4, n_showers: int = 64, n_min: float = 1e3, n_max: float = 1e6,
                    scale: float = 1.0) -> dict:
    """Many showers of uneven size: per shower, segment count log-uniform in
    [n_min, n_max) (times scale), zenith U(0,60) deg, azimuth U(0,360) deg;
    segments start on the shower axis at U(5,30) km with directions within 5
    degrees of it and energies log-uniform 50 MeV..1 GeV."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_showers)) * scale)
    sizes = np.maximum(sizes, 1).astype(np.int64)
    zen = np.radians(rng.uniform(0.0, 60.0, n_showers))
    azi = rng.uniform(0.0, 2.0 * np.pi, n_showers)
    parts = []
    for s in range(n_showers):
        m = int(sizes[s])
        axis = np.array([np.sin(zen[s]) * np.cos(azi[s]), np.sin(zen[s]) * np.sin(azi[s]),
                         -np.cos(zen[s])])
        z0 = rng.uniform(5000.0, 30000.0, m)
        lam = (z0 - H_OBS) / np.cos(zen[s])
        p = np.array([0.0, 0.0, H_OBS])[None, :] - lam[:, None] * axis[None, :]
        d = _cone_dirs(rng, m, axis, np.radians(5.0))
        length = rng.uniform(1.0, 50.0, m)
        e = np.exp(rng.uniform(np.log(50.0), np.log(1000.0), m))
        t0 = ((30000.0 - H_OBS) / np.cos(zen[s]) - lam) / C_M_PER_NS
        parts.append((p, d, length, e, t0, np.full(m, s, np.uint32), np.arange(m, dtype=np.uint32)))
    p = np.concatenate([q[0] for q in parts])
    d = np.concatenate([q[1] for q in parts])
    seg = _segments(len(p), p[:, 0], p[:, 1], p[:, 2], d, np.concatenate([q[2] for q in parts]),
                    np.concatenate([q[3] for q in parts]), np.concatenate([q[4] for q in parts]),
                    shower=np.concatenate([q[5] for q in parts]),
                    index=np.concatenate([q[6] for q in parts]))
    seg["shower_sizes"] = sizes
    return seg


def differentiable(n: int = 1_000_000, seed: int = 5) -> dict:
    """Input of the gradient workload: the shower recipe at 1e6 segments."""
    return shower_cherenkov(n, seed)


def subsample(seg: dict, idx) -> dict:
    """Rows idx of every per-segment array (ids are kept, so random streams
    are unchanged)."""
    idx = np.asarray(idx)
    n = len(seg["x0"])
    out = {}
    for k, v in seg.items():
        if isinstance(v, np.ndarray) and v.ndim >= 1 and len(v) == n:
            out[k] = np.ascontiguousarray(v[idx])
        else:
            out[k] = v
    return out


def splat_grid_128() -> dict:
    """Ground grid of the differentiable form: 128 x 128 cells of 5 m centred
    on the core, Gaussian width 5 m, square truncation at 4 sigma."""
    return dict(x_min=-320.0, y_min=-320.0, cell=5.0, nx=128, ny=128, sigma=5.0, trunc=4.0)


def perturbed_parameters(atm: dict, seg: dict, seed: int):
    """Parameters of the target density of the differentiable form: scale
    heights H_l (1 + 0.02 xi_l) with xi_l = +-1, n0 - 1 times 0.97, and every
    segment direction turned by 0.2 degrees about a random axis (Rodrigues'
    rotation), drawn from numpy's PCG64 under seed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H = np.asarray(atm["scale_height"], np.float64)
    xi = rng.choice([-1.0, 1.0], size=len(H))
    H1 = H * (1.0 + 0.02 * xi)
    eta1 = float(atm["n0_minus_1"]) * 0.97
    d = np.stack([seg["dx"], seg["dy"], seg["dz"]], axis=1).astype(np.float64)
    k = rng.normal(size=d.shape)
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    a = np.deg2rad(0.2)
    d1 = (d * np.cos(a) + np.cross(k, d) * np.sin(a)
          + k * np.sum(k * d, axis=1, keepdims=True) * (1.0 - np.cos(a)))
    return H1, eta1, d1
