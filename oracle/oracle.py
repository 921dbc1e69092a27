"""Python access to the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module. It shares nothing with the HIP
library; inputs come from the seeded generators and are passed as plain
numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LANDED, HIT, UP, BELOW, OFFGRID, ABSORBED, INVALID = 0, 1, 2, 3, 4, 5, 6


def build(openmp: bool = True) -> str:
    """Compiles oracle.c with gcc (no FMA contraction) into liboracle.so."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11",
           "-Wall", _SRC, "-o", _LIB + ".tmp", "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Atm(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("h_base", C.c_double * 8), ("H", C.c_double * 8),
                ("eta0", C.c_double), ("h_obs", C.c_double), ("n_abs", C.c_int32),
                ("abs_lambda", C.c_double * 64), ("abs_k", C.c_double * 64),
                ("rho_base", C.c_double * 8)]


class _Seg(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, C.c_void_p) for f in
                ("x0", "y0", "z0", "dx", "dy", "dz", "length", "beta", "t0", "dedx",
                 "charge", "shower", "index_in_shower")]


class _Photon(C.Structure):
    _fields_ = [("xe", C.c_double), ("ye", C.c_double), ("ze", C.c_double), ("te", C.c_double),
                ("ue", C.c_double * 3), ("lam", C.c_double), ("status", C.c_int32),
                ("xl", C.c_double), ("yl", C.c_double), ("zl", C.c_double), ("tl", C.c_double),
                ("ul", C.c_double * 3), ("path", C.c_double), ("tau", C.c_double),
                ("weight", C.c_double)]


PHOTON_DTYPE = np.dtype([("xe", "f8"), ("ye", "f8"), ("ze", "f8"), ("te", "f8"), ("ue", "f8", 3),
                         ("lam", "f8"), ("status", "i4"), ("xl", "f8"), ("yl", "f8"),
                         ("zl", "f8"), ("tl", "f8"), ("ul", "f8", 3), ("path", "f8"),
                         ("tau", "f8"), ("weight", "f8")], align=True)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.or_philox.argtypes = [P, P, P]
        L.or_uniform.argtypes = [C.c_uint32]
        L.or_uniform.restype = C.c_double
        L.or_atm_prepare.argtypes = [P]
        L.or_exp_fixed.argtypes = [C.c_double]
        L.or_exp_fixed.restype = C.c_double
        L.or_density.argtypes = [P, C.c_double]
        L.or_density.restype = C.c_double
        L.or_index.argtypes = [P, C.c_double]
        L.or_index.restype = C.c_double
        L.or_abs_k.argtypes = [P, C.c_double]
        L.or_abs_k.restype = C.c_double
        L.or_frank_tamm_K.argtypes = [C.c_double, C.c_double]
        L.or_frank_tamm_K.restype = C.c_double
        L.or_poisson.argtypes = [C.c_double, C.c_uint64, C.c_uint32, C.c_uint32, P]
        L.or_poisson.restype = C.c_uint32
        L.or_counts.argtypes = [P, P, C.c_int, P, C.c_uint64, P, P, P]
        L.or_counts_ex.argtypes = [P, P, C.c_int, P, C.c_uint64, C.c_int32, C.c_double, P, P, P, P, P]
        L.or_beam_cap.argtypes = [P, C.c_int64, P, P, P]
        L.or_beam_cap.restype = C.c_int
        L.or_passes_cut.argtypes = [P, C.c_int64, C.c_int32, C.c_double, P]
        L.or_passes_cut.restype = C.c_int
        L.or_rotation_matrix.argtypes = [C.c_double, C.c_double, C.c_double, P]
        L.or_line_cdf.argtypes = [P, C.c_int32, P]
        L.or_ray_integrals.argtypes = [P, C.c_double, C.c_double, C.c_double, P]
        L.or_photons.argtypes = [P, P, C.c_int, P, P, P, C.c_int32, C.c_uint64, P, P, P, C.c_int64, P]
        L.or_photons_all.argtypes = [P, P, C.c_int, P, P, P, C.c_int32, C.c_uint64, P, P, P]
        L.or_telescopes.argtypes = [P, C.c_int64, P, C.c_int32, C.c_double, P, P]
        L.or_radial_bins.argtypes = [P, C.c_int64, C.c_double, C.c_double, P, C.c_int32, P]
        L.or_table_build.argtypes = [P, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, P, P]
        L.or_propagate_table.argtypes = [P, C.c_int64, P, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                         C.c_int32, P, P]
        L.or_grid.argtypes = [P, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int32,
                              C.c_int32, P]
        L.or_splat.argtypes = [P, P, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32,
                               C.c_double, C.c_double, P]
        L.or_num_threads.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def num_threads() -> int:
    return int(lib().or_num_threads())


# ---------------------------------------------------------------- inputs --
class Atmosphere:
    """Holds the ctypes atmosphere (the oracle derives its own base densities)."""

    def __init__(self, h_base, scale_height, n0_minus_1, h_obs, abs_lambda=None, abs_k=None):
        a = _Atm()
        nl = len(h_base)
        a.n_layers = nl
        for i in range(nl):
            a.h_base[i] = float(h_base[i])
            a.H[i] = float(scale_height[i])
        a.eta0 = float(n0_minus_1)
        a.h_obs = float(h_obs)
        if abs_lambda is not None and len(abs_lambda):
            a.n_abs = len(abs_lambda)
            for i in range(a.n_abs):
                a.abs_lambda[i] = float(abs_lambda[i])
                a.abs_k[i] = float(abs_k[i])
        else:
            a.n_abs = 0
        lib().or_atm_prepare(C.byref(a))
        self.c = a

    @classmethod
    def from_dict(cls, d):
        return cls(d["h_base"], d["scale_height"], d["n0_minus_1"], d["h_obs"],
                   d.get("abs_lambda_nm"), d.get("abs_k_per_m"))

    def density(self, h):
        return lib().or_density(C.byref(self.c), float(h))

    def index(self, h):
        return lib().or_index(C.byref(self.c), float(h))

    def abs_k(self, lam):
        return lib().or_abs_k(C.byref(self.c), float(lam))

    @property
    def rho_base(self):
        return np.array(self.c.rho_base[: self.c.n_layers])

    def ray_integrals(self, z_e, cos_e, h_lo):
        """(int dh/r, int n/r dh, int n^2/r dh, int rho n/r dh) from h_lo up to
        the emission height z_e for a ray with |cos zenith| = cos_e there."""
        G = np.zeros(4)
        lib().or_ray_integrals(C.byref(self.c), float(z_e), float(cos_e), float(h_lo), _ptr(G))
        return G


class Segments:
    """Keeps contiguous numpy copies alive for the ctypes struct."""

    FIELDS = ("x0", "y0", "z0", "dx", "dy", "dz", "length", "beta", "t0")

    def __init__(self, seg: dict):
        self.arrays = {}
        n = len(seg["x0"])
        s = _Seg()
        s.n = n
        for f in self.FIELDS:
            self.arrays[f] = np.ascontiguousarray(seg[f], dtype=np.float64)
            setattr(s, f, self.arrays[f].ctypes.data)
        if seg.get("dedx") is not None:
            self.arrays["dedx"] = np.ascontiguousarray(seg["dedx"], dtype=np.float64)
            s.dedx = self.arrays["dedx"].ctypes.data
        for f, dt in (("charge", np.int32), ("shower", np.uint32), ("index_in_shower", np.uint32)):
            if seg.get(f) is not None:
                self.arrays[f] = np.ascontiguousarray(seg[f], dtype=dt)
                setattr(s, f, self.arrays[f].ctypes.data)
        self.c = s
        self.n = n


# ------------------------------------------------------------- functions --
def philox(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 of each row of ctr (N,4) uint32 under key (k0, k1)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty_like(ctr)
    L = lib()
    for i in range(ctr.shape[0]):
        L.or_philox(ctr[i].ctypes.data, k.ctypes.data, out[i].ctypes.data)
    return out


def exp_fixed(x) -> np.ndarray:
    """The specified exp of the count path (or_exp_fixed), elementwise."""
    f = lib().or_exp_fixed
    return np.array([f(float(v)) for v in np.ravel(x)], np.float64).reshape(np.shape(x))


def uniform(x) -> np.ndarray:
    return np.array([lib().or_uniform(int(v)) for v in np.ravel(x)])


def frank_tamm_K(lmin, lmax):
    return lib().or_frank_tamm_K(float(lmin), float(lmax))


def poisson(mu, seed, idx, shower):
    m = C.c_double()
    k = lib().or_poisson(float(mu), int(seed), int(idx), int(shower), C.byref(m))
    return int(k), m.value


def _beam_arr(beam):
    """beam = (centre (3,), radius, margin in radians) or None."""
    if beam is None:
        return None
    c, r, m = beam
    return np.array([c[0], c[1], c[2], r, m], dtype=np.float64)


def counts(seg: dict, atm: Atmosphere, kind: str, seed: int, *, lambda_nm=(300.0, 600.0),
           yield_per_MeV=10.0, cut=None, beam=None):
    """Per-segment (counts u32, mean f64, decision margin f64). cut = (points
    (k, 3), cos of the cut angle) applies the Cherenkov angular particle cut;
    beam = (centre, radius, margin rad) the fluorescence beaming."""
    S = Segments(seg)
    n = S.n
    cnt = np.zeros(n, np.uint32)
    mu = np.zeros(n)
    mg = np.zeros(n)
    if kind == "cherenkov":
        par = np.array(lambda_nm, dtype=np.float64)
        kd = 0
    else:
        par = np.array([yield_per_MeV], dtype=np.float64)
        kd = 1
    if cut is None and beam is None:
        lib().or_counts(C.byref(S.c), C.byref(atm.c), kd, _ptr(par), int(seed), _ptr(cnt), _ptr(mu),
                        _ptr(mg))
    else:
        pts = (np.zeros((0, 3)) if cut is None else
               np.ascontiguousarray(cut[0], dtype=np.float64).reshape(-1, 3))
        cos_cut = 1.0 if cut is None else float(cut[1])
        b = _beam_arr(beam)
        lib().or_counts_ex(C.byref(S.c), C.byref(atm.c), kd, _ptr(par), int(seed), len(pts), cos_cut,
                           _ptr(pts), _ptr(b), _ptr(cnt), _ptr(mu), _ptr(mg))
    return cnt, mu, mg


def beam_cap(seg: dict, beam):
    """Per segment (beamed?, 1 - cos of the cone half angle, unit axis (n, 3))."""
    S = Segments(seg)
    b = _beam_arr(beam)
    om = np.zeros(1)
    ax = np.zeros(3)
    on = np.zeros(S.n, bool)
    oms = np.zeros(S.n)
    axes = np.zeros((S.n, 3))
    for i in range(S.n):
        on[i] = bool(lib().or_beam_cap(C.byref(S.c), i, _ptr(b), _ptr(om), _ptr(ax)))
        oms[i] = om[0]
        axes[i] = ax
    return on, oms, axes


def passes_cut(seg: dict, points, cos_cut) -> np.ndarray:
    """Per segment: kept by the Cherenkov angular particle cut."""
    S = Segments(seg)
    pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    return np.array([bool(lib().or_passes_cut(C.byref(S.c), i, len(pts), float(cos_cut), _ptr(pts)))
                     for i in range(S.n)])


def offsets_of(cnt: np.ndarray) -> np.ndarray:
    off = np.zeros(len(cnt) + 1, np.uint64)
    np.cumsum(cnt.astype(np.uint64), out=off[1:])
    return off


def _gen_args(kind, lambda_nm, yield_per_MeV, lines_nm, line_rel):
    if kind == "cherenkov":
        return 0, np.array(lambda_nm, dtype=np.float64), None, None, 0
    ln = np.ascontiguousarray(lines_nm, dtype=np.float64)
    lr = np.ascontiguousarray(line_rel, dtype=np.float64)
    return 1, np.array([yield_per_MeV], dtype=np.float64), ln, lr, len(ln)


def photons(seg: dict, atm: Atmosphere, kind: str, seed: int, s_list, j_list, *,
            lambda_nm=(300.0, 600.0), yield_per_MeV=10.0, lines_nm=None, line_rel=None, beam=None):
    """Generated + propagated photons for the listed (segment, j) pairs."""
    S = Segments(seg)
    kd, par, ln, lr, nl = _gen_args(kind, lambda_nm, yield_per_MeV, lines_nm, line_rel)
    s_list = np.ascontiguousarray(s_list, dtype=np.int64)
    j_list = np.ascontiguousarray(j_list, dtype=np.uint32)
    out = np.zeros(len(s_list), PHOTON_DTYPE)
    b = _beam_arr(beam)
    lib().or_photons(C.byref(S.c), C.byref(atm.c), kd, _ptr(par), _ptr(ln), _ptr(lr), nl,
                     int(seed), _ptr(b), _ptr(s_list), _ptr(j_list), len(s_list), _ptr(out))
    return out


def photons_all(seg: dict, atm: Atmosphere, kind: str, seed: int, offsets, *,
                lambda_nm=(300.0, 600.0), yield_per_MeV=10.0, lines_nm=None, line_rel=None, beam=None):
    """Every photon in slot order (offsets has n+1 entries)."""
    S = Segments(seg)
    kd, par, ln, lr, nl = _gen_args(kind, lambda_nm, yield_per_MeV, lines_nm, line_rel)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    out = np.zeros(int(off[-1]), PHOTON_DTYPE)
    b = _beam_arr(beam)
    lib().or_photons_all(C.byref(S.c), C.byref(atm.c), kd, _ptr(par), _ptr(ln), _ptr(lr), nl,
                         int(seed), _ptr(b), _ptr(off), _ptr(out))
    return out


def telescopes(ph: np.ndarray, tel: np.ndarray, n_obs: float):
    """(telescope id or -1, hit record x,y,z,t,s) per photon."""
    ph = np.ascontiguousarray(ph)
    tel = np.ascontiguousarray(tel, dtype=np.float64).reshape(-1, 4)
    tid = np.zeros(len(ph), np.int32)
    hits = np.zeros((len(ph), 5))
    lib().or_telescopes(_ptr(ph), len(ph), _ptr(tel), tel.shape[0], float(n_obs), _ptr(tid),
                        _ptr(hits))
    return tid, hits


class Table:
    """Correction tables of the straight-line propagation (section 2):
    corr (n_h, n_q, 3) = (g, dP, dX) and vert (n_v, 2) = (rho/rho0, VX)."""

    def __init__(self, atm: Atmosphere, n_h: int, n_q: int, h_max: float, q_max: float, n_v: int):
        self.n_h, self.n_q, self.h_max, self.q_max, self.n_v = int(n_h), int(n_q), float(h_max), float(q_max), int(n_v)
        self.corr = np.zeros((self.n_h, self.n_q, 3))
        self.vert = np.zeros((self.n_v, 2))
        lib().or_table_build(C.byref(atm.c), self.n_h, self.n_q, self.h_max, self.q_max, self.n_v,
                             _ptr(self.corr), _ptr(self.vert))


def propagate_table(ph: np.ndarray, atm: Atmosphere, table: Table) -> np.ndarray:
    """A copy of generated photons carried to the ground by the table method."""
    out = np.ascontiguousarray(ph).copy()
    lib().or_propagate_table(_ptr(out), len(out), C.byref(atm.c), table.n_h, table.n_q, table.h_max,
                             table.q_max, table.n_v, _ptr(table.corr), _ptr(table.vert))
    return out


def radial_edges(n_bins, r_min, r_max, log_bins):
    """Bin edges: uniform in r, or in ln r (r_min > 0); the last is r_max."""
    k = np.arange(n_bins + 1) / n_bins
    e = r_min * (r_max / r_min) ** k if log_bins else r_min + (r_max - r_min) * k
    e[-1] = r_max
    return e


def radial_bins(ph: np.ndarray, core, edges):
    """Bin per photon (-1: not landed or outside the edges)."""
    ph = np.ascontiguousarray(ph)
    e = np.ascontiguousarray(edges, dtype=np.float64)
    out = np.zeros(len(ph), np.int32)
    lib().or_radial_bins(_ptr(ph), len(ph), float(core[0]), float(core[1]), _ptr(e), len(e) - 1, _ptr(out))
    return out


def radial_profile(ph: np.ndarray, core, edges, t_ref=0.0):
    """Section 3.1 profiles: per bin (count, sum of weights, density in
    photons/m^2 = weight / ring area, mean arrival time weighted by w)."""
    b = radial_bins(ph, core, edges)
    n = len(edges) - 1
    m = b >= 0
    cnt = np.bincount(b[m], minlength=n)
    w = np.bincount(b[m], weights=ph["weight"][m], minlength=n)
    wt = np.bincount(b[m], weights=ph["weight"][m] * (ph["tl"][m] - t_ref), minlength=n)
    area = np.pi * (edges[1:] ** 2 - edges[:-1] ** 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        mean_t = np.where(w > 0, t_ref + wt / w, np.nan)
    return cnt, w, w / area, mean_t


def grid(ph: np.ndarray, x_min, y_min, cell, nx, ny):
    """Flat cell index per photon (-1 = off grid or not landed)."""
    ph = np.ascontiguousarray(ph)
    cell_of = np.zeros(len(ph), np.int32)
    lib().or_grid(_ptr(ph), len(ph), float(x_min), float(y_min), float(cell), int(nx), int(ny),
                  _ptr(cell_of))
    return cell_of


def rotation_matrix(d):
    M = np.zeros(9)
    lib().or_rotation_matrix(float(d[0]), float(d[1]), float(d[2]), _ptr(M))
    return M.reshape(3, 3)


def line_cdf(rel):
    rel = np.ascontiguousarray(rel, dtype=np.float64)
    cdf = np.zeros(len(rel))
    lib().or_line_cdf(_ptr(rel), len(rel), _ptr(cdf))
    return cdf


def splat(ph: np.ndarray, weight: np.ndarray, x_min, y_min, cell, nx, ny, sigma, trunc=4.0):
    """Gaussian-splatted density (ny, nx) of landed photons with weights."""
    ph = np.ascontiguousarray(ph)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    D = np.zeros(int(ny) * int(nx))
    lib().or_splat(_ptr(ph), _ptr(w), len(ph), float(x_min), float(y_min), float(cell), int(nx), int(ny),
                   float(sigma), float(trunc), _ptr(D))
    return D.reshape(int(ny), int(nx))


def splat_density(seg: dict, atm: "Atmosphere", counts0, mu0, seed, grid: dict, sigma, trunc=4.0,
                  lambda_nm=(300.0, 600.0)):
    """Density of the differentiable form: Cherenkov photons of every segment
    with its frozen count counts0 (drawn at the nominal parameters), generated
    and propagated under the parameters in seg/atm, weighted by
    mu(theta)/mu0 (the mean at the current parameters over the nominal one)
    times the transmission exp(-tau)."""
    cnt = np.asarray(counts0, np.int64)
    s_list = np.repeat(np.arange(len(cnt)), cnt)
    off = np.concatenate([[0], np.cumsum(cnt)])
    j_list = np.arange(off[-1]) - off[s_list]
    ph = photons(seg, atm, "cherenkov", seed, s_list, j_list, lambda_nm=lambda_nm)
    _, mu, _ = counts(seg, atm, "cherenkov", seed, lambda_nm=lambda_nm)
    ratio = np.where(np.asarray(mu0) > 0, mu / np.where(np.asarray(mu0) > 0, mu0, 1.0), 0.0)
    w = ratio[s_list] * ph["weight"]
    return splat(ph, w, grid["x_min"], grid["y_min"], grid["cell"], grid["nx"], grid["ny"], sigma, trunc)
