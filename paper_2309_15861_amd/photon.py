"""Python binding of libphoton (C ABI in include/photon.h).

Argument marshalling only: every step of the photon path runs in the HIP
kernels of libphoton.so. PyTorch supplies device memory (tensor data
pointers) and the stream (the current torch stream). There is no CPU
fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphoton.so")

OK, EINVAL, ECAPACITY, EHIP, ENODEV = 0, -1, -2, -3, -4
FP64, FP32 = 0, 1
CHERENKOV, FLUORESCENCE = 0, 1
LANDED, HIT, UP, BELOW, OFFGRID, ABSORBED, INVALID = 0, 1, 2, 3, 4, 5, 6
HORIZON_FLOAT = 7          # totals slot: near-horizon rays evaluated in float (queue full)
N_STATUS = 8
SINK_STATUS, SINK_TELESCOPES, SINK_GRID, SINK_PLANE, SINK_RADIAL = 0, 1, 2, 3, 4
MAX_RADIAL_BINS = 1024
MAX_LAYERS, MAX_ABS, MAX_LINES, MAX_TELESCOPES, MAX_CUT_POINTS = 8, 40, 32, 32, 32

P = C.c_void_p


class Atmosphere(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("h_base", C.c_double * MAX_LAYERS),
                ("scale_height", C.c_double * MAX_LAYERS), ("n0_minus_1", C.c_double),
                ("h_obs", C.c_double), ("n_abs", C.c_int32), ("abs_lambda_nm", C.c_double * MAX_ABS),
                ("abs_k_per_m", C.c_double * MAX_ABS), ("table", P)]


class TableStruct(C.Structure):
    _fields_ = [("n_h", C.c_int32), ("n_q", C.c_int32), ("n_v", C.c_int32), ("h_max", C.c_double),
                ("q_max", C.c_double), ("corr", P), ("vert", P), ("atm_hash", C.c_uint64)]


class Segments(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, P) for f in (
        "x0", "y0", "z0", "dx", "dy", "dz", "length", "beta", "t0", "dedx", "charge", "shower",
        "index_in_shower")]


class Emission(C.Structure):
    _fields_ = [("kind", C.c_int32), ("lambda_min_nm", C.c_double), ("lambda_max_nm", C.c_double),
                ("yield_per_MeV", C.c_double), ("n_lines", C.c_int32),
                ("line_nm", C.c_double * MAX_LINES), ("line_rel_yield", C.c_double * MAX_LINES),
                ("n_cut_points", C.c_int32), ("cut_cos", C.c_double),
                ("cut_points", (C.c_double * 3) * MAX_CUT_POINTS),
                ("beam", C.c_int32), ("beam_center", C.c_double * 3), ("beam_radius", C.c_double),
                ("beam_margin_rad", C.c_double)]


class Block(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("n_photons", C.c_int64), ("precision", C.c_int32)] + [
        (f, P) for f in ("x", "y", "ux", "uy", "uz", "wavelength_nm", "weight", "z", "t_ns", "path_m",
                         "segment", "j", "status")]


class Hits(C.Structure):
    _fields_ = [("capacity", C.c_int64)] + [(f, P) for f in (
        "count", "segment", "j", "telescope", "x", "y", "z", "t_ns", "ux", "uy", "uz", "wavelength_nm",
        "weight")]


class Sink(C.Structure):
    _fields_ = [("kind", C.c_int32), ("status_totals", P), ("n_tel", C.c_int32),
                ("tel", (C.c_double * 4) * MAX_TELESCOPES), ("hits", Hits), ("x_min", C.c_double),
                ("y_min", C.c_double), ("cell", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32),
                ("grid_count", P), ("grid_weight", P), ("plane", P),
                ("core_x", C.c_double), ("core_y", C.c_double), ("r_min", C.c_double), ("r_max", C.c_double),
                ("t_ref_ns", C.c_double), ("n_bins", C.c_int32), ("log_bins", C.c_int32),
                ("radial_count", P), ("radial_weight", P), ("radial_wt", P)]


class Tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("chunk", C.c_int32), ("blocks_per_cu", C.c_int32)]


class SplatGrid(C.Structure):
    _fields_ = [("x_min", C.c_double), ("y_min", C.c_double), ("cell", C.c_double), ("nx", C.c_int32),
                ("ny", C.c_int32), ("sigma", C.c_double), ("trunc", C.c_double)]


class PhotonError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libphoton error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Loads libphoton.so; raises if it has not been built, or was built from
    other sources than the ones beside it."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.photon_version.restype = C.c_char_p
        built = L.photon_version().decode().rsplit(" ", 1)[-1]
        want = _build.source_hash()
        if built != want:
            raise RuntimeError(f"{LIB_PATH} was built from sources {built}, the sources are now {want}: "
                               "rebuild it with __graft_entry__.build()")
        L.photon_last_error.restype = C.c_char_p
        L.photon_init.restype = C.c_int
        L.photon_gen_cherenkov.argtypes = [P, P, C.c_double, C.c_double, C.c_uint64, C.c_int32, P, P, P, P]
        L.photon_gen_fluor.argtypes = [P, P, P, P, C.c_int32, C.c_double, C.c_uint64, C.c_int32, P, P, P, P]
        L.photon_propagate.argtypes = [P, P, P]
        L.photon_collect.argtypes = [P, P, P, P]
        L.photon_run_fused.argtypes = [P, P, P, C.c_uint64, C.c_int32, P, C.c_int64, P, P, P]
        L.photon_run_fused_noalloc.argtypes = [P, P, P, C.c_uint64, C.c_int32, P, C.c_int64, P, P, P]
        L.photon_plan_create.argtypes = [P, P, P, C.c_uint64, C.c_int32, P, P, P, P, P]
        L.photon_plan_launch.argtypes = [P, P]
        L.photon_plan_destroy.argtypes = [P]
        L.photon_autotune.argtypes = [P, P, P, C.c_uint64, C.c_int32, P, P, P, C.c_int32, C.c_int32, P, P, P]
        L.photon_means.argtypes = [P, P, P, P, P]
        L.photon_count.argtypes = [P, P, P, C.c_uint64, P, P, P]
        L.photon_generate.argtypes = [P, P, P, C.c_uint64, C.c_int32, P, P, P]
        L.photon_radial_profile.argtypes = [P, P, P, P]
        L.photon_table_build.argtypes = [P, P, P]
        L.photon_kernel_timing.argtypes = [C.c_int32]
        L.photon_fused_kernel_ms.argtypes = [P]
        L.photon_fused_deferred_ms.argtypes = [P]
        L.photon_set_defer_capacity.argtypes = [C.c_int64]
        L.photon_peak_run.argtypes = [C.c_int32, P, C.c_int64, C.c_int32, P, P, P]
        L.photon_splat_forward.argtypes = [P, P, C.c_double, C.c_double, C.c_uint64, C.c_int32, P, P, P, P, P, P]
        L.photon_splat_backward.argtypes = [P, P, C.c_double, C.c_double, C.c_uint64, C.c_int32, P, P, P, P,
                                            P, P, P, P, P, P]
        for f in ("photon_gen_cherenkov", "photon_gen_fluor", "photon_propagate", "photon_collect",
                  "photon_run_fused", "photon_run_fused_noalloc", "photon_plan_create", "photon_plan_launch", "photon_plan_destroy",
                  "photon_autotune", "photon_means", "photon_splat_forward", "photon_splat_backward",
                  "photon_count", "photon_kernel_timing", "photon_fused_kernel_ms", "photon_fused_deferred_ms", "photon_set_defer_capacity", "photon_peak_run"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise PhotonError(rc, lib().photon_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def version():
    return lib().photon_version().decode()


def init():
    _check(lib().photon_init())


# ------------------------------------------------------------------ inputs --
class PropagationTable:
    """Correction tables of the straight-line propagation (section 2) for one
    atmosphere, resident on the GPU; built on construction."""

    def __init__(self, atm: Atmosphere, n_h=257, n_q=257, h_max=40000.0, q_max=float(np.tan(np.radians(80.0))),
                 n_v=4097, device="cuda"):
        self.corr = torch.zeros(4 * n_h * n_q, dtype=torch.float32, device=device)
        self.vert = torch.zeros(2 * n_v, dtype=torch.float32, device=device)
        self.s = TableStruct()
        self.s.n_h, self.s.n_q, self.s.n_v = int(n_h), int(n_q), int(n_v)
        self.s.h_max, self.s.q_max = float(h_max), float(q_max)
        self.s.corr, self.s.vert = self.corr.data_ptr(), self.vert.data_ptr()
        _check(lib().photon_table_build(C.byref(atm), C.byref(self.s), _stream()))

    def attach(self, atm: Atmosphere) -> Atmosphere:
        """A copy of atm that propagates with this table (keeps the table alive)."""
        a = Atmosphere.from_buffer_copy(atm)
        a.table = C.addressof(self.s)
        a._table_owner = self
        return a


def atmosphere(d: dict) -> Atmosphere:
    a = Atmosphere()
    hb, H = d["h_base"], d["scale_height"]
    a.n_layers = len(hb)
    for i in range(min(len(hb), MAX_LAYERS)):
        a.h_base[i] = float(hb[i])
        a.scale_height[i] = float(H[i])
    a.n0_minus_1 = float(d["n0_minus_1"])
    a.h_obs = float(d["h_obs"])
    lam, k = d.get("abs_lambda_nm"), d.get("abs_k_per_m")
    if lam is not None and len(lam):
        a.n_abs = len(lam)
        for i in range(min(len(lam), MAX_ABS)):
            a.abs_lambda_nm[i] = float(lam[i])
            a.abs_k_per_m[i] = float(k[i])
    return a


class DeviceSegments:
    """Segment arrays resident on the GPU (float64 / int32 / uint32)."""

    F64 = ("x0", "y0", "z0", "dx", "dy", "dz", "length", "beta", "t0")

    def __init__(self, seg: dict, device="cuda"):
        self.t = {}
        for f in self.F64:
            self.t[f] = torch.as_tensor(np.ascontiguousarray(seg[f], np.float64), device=device)
        if seg.get("dedx") is not None:
            self.t["dedx"] = torch.as_tensor(np.ascontiguousarray(seg["dedx"], np.float64), device=device)
        if seg.get("charge") is not None:
            self.t["charge"] = torch.as_tensor(np.ascontiguousarray(seg["charge"], np.int32), device=device)
        for f in ("shower", "index_in_shower"):
            if seg.get(f) is not None:
                a = np.ascontiguousarray(seg[f], np.uint32).view(np.int32)
                self.t[f] = torch.as_tensor(a, device=device)
        self.n = int(self.t["x0"].numel())

    def struct(self) -> Segments:
        s = Segments()
        s.n = self.n
        for f in self.F64 + ("dedx", "charge", "shower", "index_in_shower"):
            if f in self.t:
                setattr(s, f, self.t[f].data_ptr())
        return s


class PhotonBlock:
    """The common photon block (structure of arrays) on the GPU."""

    REAL = ("x", "y", "ux", "uy", "wavelength_nm", "weight")

    def __init__(self, capacity: int, precision: int, device="cuda"):
        dt = torch.float64 if precision == FP64 else torch.float32
        self.precision = precision
        self.capacity = int(capacity)
        self.n_photons = 0
        n = max(self.capacity, 1)
        self.t = {f: torch.empty(n, dtype=dt, device=device) for f in self.REAL}
        self.t["uz"] = torch.empty(n, dtype=torch.float64, device=device)   # double in both precisions
        self.t["z"] = torch.empty(n, dtype=torch.float64, device=device)
        self.t["t_ns"] = torch.empty(n, dtype=torch.float64, device=device)
        self.t["path_m"] = torch.empty(n, dtype=torch.float64, device=device)
        self.t["segment"] = torch.empty(n, dtype=torch.int32, device=device)
        self.t["j"] = torch.empty(n, dtype=torch.int32, device=device)
        self.t["status"] = torch.empty(n, dtype=torch.int32, device=device)

    def struct(self) -> Block:
        b = Block()
        b.capacity = self.capacity
        b.n_photons = self.n_photons
        b.precision = self.precision
        for f, v in self.t.items():
            setattr(b, f, v.data_ptr())
        return b

    def numpy(self) -> dict:
        n = self.n_photons
        out = {f: v[:n].cpu().numpy() for f, v in self.t.items()}
        out["segment"] = out["segment"].view(np.uint32)
        out["j"] = out["j"].view(np.uint32)
        return out


class HitBuffer:
    """Telescope hit records on the GPU."""

    def __init__(self, capacity: int, device="cuda"):
        self.capacity = int(capacity)
        n = max(self.capacity, 1)
        self.t = dict(count=torch.zeros(1, dtype=torch.int64, device=device),
                      segment=torch.empty(n, dtype=torch.int32, device=device),
                      j=torch.empty(n, dtype=torch.int32, device=device),
                      telescope=torch.empty(n, dtype=torch.int32, device=device))
        for f in ("x", "y", "z", "t_ns"):
            self.t[f] = torch.empty(n, dtype=torch.float64, device=device)
        for f in ("ux", "uy", "uz", "wavelength_nm", "weight"):
            self.t[f] = torch.empty(n, dtype=torch.float32, device=device)

    def clear(self):
        self.t["count"].zero_()

    def struct(self) -> Hits:
        h = Hits()
        h.capacity = self.capacity
        for f, v in self.t.items():
            setattr(h, f, v.data_ptr())
        return h

    def count(self) -> int:
        return int(self.t["count"].item())

    def numpy(self) -> dict:
        n = min(self.count(), self.capacity)
        out = {f: v[:n].cpu().numpy() for f, v in self.t.items() if f != "count"}
        out["segment"] = out["segment"].view(np.uint32)
        out["j"] = out["j"].view(np.uint32)
        return out


def status_totals(device="cuda"):
    return torch.zeros(N_STATUS, dtype=torch.int64, device=device)


def sink_status(totals) -> Sink:
    s = Sink()
    s.kind = SINK_STATUS
    s.status_totals = _ptr(totals).value
    return s


def sink_telescopes(tel: np.ndarray, hits: HitBuffer, totals=None) -> Sink:
    s = Sink()
    s.kind = SINK_TELESCOPES
    s.status_totals = None if totals is None else totals.data_ptr()
    tel = np.asarray(tel, np.float64).reshape(-1, 4)
    s.n_tel = tel.shape[0]
    for k in range(min(tel.shape[0], MAX_TELESCOPES)):
        for c in range(4):
            s.tel[k][c] = float(tel[k, c])
    s.hits = hits.struct()
    return s


def sink_grid(x_min, y_min, cell, nx, ny, grid_count, grid_weight, totals=None) -> Sink:
    s = Sink()
    s.kind = SINK_GRID
    s.status_totals = None if totals is None else totals.data_ptr()
    s.x_min, s.y_min, s.cell, s.nx, s.ny = float(x_min), float(y_min), float(cell), int(nx), int(ny)
    s.grid_count = grid_count.data_ptr()
    s.grid_weight = grid_weight.data_ptr()
    return s


class RadialProfile:
    """Accumulators of a radial profile sink on the GPU (count, weight in
    units of 2^-32, w (t - t_ref) in units of 2^-8 ns) and its geometry."""

    def __init__(self, n_bins, r_min, r_max, log_bins=False, core=(0.0, 0.0), t_ref_ns=0.0, device="cuda"):
        self.n_bins, self.r_min, self.r_max = int(n_bins), float(r_min), float(r_max)
        self.log_bins, self.core, self.t_ref_ns = bool(log_bins), (float(core[0]), float(core[1])), float(t_ref_ns)
        n = max(self.n_bins, 1)
        self.count = torch.zeros(n, dtype=torch.int64, device=device)
        self.weight = torch.zeros(n, dtype=torch.int64, device=device)
        self.wt = torch.zeros(n, dtype=torch.int64, device=device)

    def edges(self) -> np.ndarray:
        k = np.arange(self.n_bins + 1) / self.n_bins
        if self.log_bins:
            e = self.r_min * (self.r_max / self.r_min) ** k
        else:
            e = self.r_min + (self.r_max - self.r_min) * k
        e[-1] = self.r_max
        return e


def sink_radial(prof: RadialProfile, totals=None) -> Sink:
    """Radial photon-density and arrival-time profile about prof.core."""
    s = Sink()
    s.kind = SINK_RADIAL
    s.status_totals = None if totals is None else totals.data_ptr()
    s.core_x, s.core_y = prof.core
    s.r_min, s.r_max, s.t_ref_ns = prof.r_min, prof.r_max, prof.t_ref_ns
    s.n_bins, s.log_bins = prof.n_bins, int(prof.log_bins)
    s.radial_count = prof.count.data_ptr()
    s.radial_weight = prof.weight.data_ptr()
    s.radial_wt = prof.wt.data_ptr()
    return s


def radial_profile(prof: RadialProfile):
    """(density [photons/m^2], mean arrival time [ns]) per bin as float64
    tensors; NaN time where a bin holds no weight."""
    density = torch.empty(max(prof.n_bins, 1), dtype=torch.float64, device=prof.count.device)
    mean_t = torch.empty_like(density)
    s = sink_radial(prof)
    _check(lib().photon_radial_profile(C.byref(s), _ptr(density), _ptr(mean_t), _stream()))
    return density[:prof.n_bins], mean_t[:prof.n_bins]


def sink_plane(block: PhotonBlock, totals=None) -> Sink:
    """Every photon's final state written at its slot of `block`."""
    s = Sink()
    s.kind = SINK_PLANE
    s.status_totals = None if totals is None else totals.data_ptr()
    s._plane = block.struct()          # kept alive with the sink
    s.plane = C.addressof(s._plane)
    return s


def emission_cherenkov(lmin=300.0, lmax=600.0, cut_points=None, cut_angle_deg=6.0) -> Emission:
    """Cherenkov emission; cut_points (k x 3) enables the angular particle cut
    (a segment emits only if its direction is within cut_angle_deg of the
    direction from its midpoint to one of the points)."""
    e = Emission()
    e.kind = CHERENKOV
    e.lambda_min_nm, e.lambda_max_nm = float(lmin), float(lmax)
    if cut_points is not None:
        pts = np.asarray(cut_points, np.float64).reshape(-1, 3)
        e.n_cut_points = len(pts)
        e.cut_cos = float(np.cos(np.radians(cut_angle_deg)))
        for k in range(min(len(pts), MAX_CUT_POINTS)):
            for d in range(3):
                e.cut_points[k][d] = float(pts[k, d])
    return e


def emission_fluor(line_nm, line_rel, yield_per_MeV, beam_area=None, beam_margin_deg=1.0) -> Emission:
    """Fluorescence emission; beam_area = (centre (3,), radius) beams every
    segment into the cone that contains that sphere (plus beam_margin_deg),
    with the photon number scaled by the cone's solid-angle fraction."""
    e = Emission()
    e.kind = FLUORESCENCE
    e.yield_per_MeV = float(yield_per_MeV)
    e.n_lines = len(line_nm)
    for k in range(min(len(line_nm), MAX_LINES)):
        e.line_nm[k] = float(line_nm[k])
        e.line_rel_yield[k] = float(line_rel[k])
    if beam_area is not None:
        c, r = beam_area
        e.beam = 1
        for d in range(3):
            e.beam_center[d] = float(c[d])
        e.beam_radius = float(r)
        e.beam_margin_rad = float(np.radians(beam_margin_deg))
    return e


def enclosing_sphere(tel) -> tuple:
    """(centre, radius) of a sphere around telescope spheres (rows x, y, z, R):
    centred on the mean of their centres, reaching the far side of each."""
    tel = np.asarray(tel, np.float64).reshape(-1, 4)
    c = tel[:, :3].mean(axis=0)
    return c, float(np.max(np.linalg.norm(tel[:, :3] - c, axis=1) + tel[:, 3]))


# --------------------------------------------------------------- entry points --
def gen_cherenkov(seg: DeviceSegments, atm: Atmosphere, lmin, lmax, seed, precision, counts, offsets,
                  block: PhotonBlock | None = None):
    s = seg.struct()
    b = None if block is None else block.struct()
    _check(lib().photon_gen_cherenkov(C.byref(s), C.byref(atm), float(lmin), float(lmax), int(seed),
                                      int(precision), _ptr(counts), _ptr(offsets),
                                      None if b is None else C.byref(b), _stream()))


def gen_fluor(seg: DeviceSegments, atm: Atmosphere, line_nm, line_rel, yield_per_MeV, seed, precision,
              counts, offsets, block: PhotonBlock | None = None):
    s = seg.struct()
    b = None if block is None else block.struct()
    ln = np.ascontiguousarray(line_nm, np.float64)
    lr = np.ascontiguousarray(line_rel, np.float64)
    _check(lib().photon_gen_fluor(C.byref(s), C.byref(atm), ln.ctypes.data, lr.ctypes.data, len(ln),
                                  float(yield_per_MeV), int(seed), int(precision), _ptr(counts),
                                  _ptr(offsets), None if b is None else C.byref(b), _stream()))


def count(seg: DeviceSegments, atm: Atmosphere, em: Emission, seed, device="cuda"):
    """Counts (u32 as int32 tensor) and offsets (u64 as int64 tensor) for an
    emission model (honouring its angular cut)."""
    counts = torch.empty(max(seg.n, 1), dtype=torch.int32, device=device)
    offsets = torch.empty(seg.n + 1, dtype=torch.int64, device=device)
    s = seg.struct()
    _check(lib().photon_count(C.byref(s), C.byref(atm), C.byref(em), int(seed), _ptr(counts), _ptr(offsets),
                              _stream()))
    return counts[:seg.n], offsets


def generate(seg: DeviceSegments, atm: Atmosphere, em: Emission, seed, precision, offsets,
             block: PhotonBlock):
    """Fills the block for the emission model (beaming included)."""
    s = seg.struct()
    _check(lib().photon_generate(C.byref(s), C.byref(atm), C.byref(em), int(seed), int(precision),
                                 _ptr(offsets), C.byref(block.struct()), _stream()))


def propagate(block: PhotonBlock, atm: Atmosphere):
    b = block.struct()
    _check(lib().photon_propagate(C.byref(b), C.byref(atm), _stream()))


def collect(block: PhotonBlock, atm: Atmosphere, sink: Sink):
    b = block.struct()
    _check(lib().photon_collect(C.byref(b), C.byref(atm), C.byref(sink), _stream()))


def run_fused(seg: DeviceSegments, atm: Atmosphere, em: Emission, seed, precision, offsets, n_photons,
              sink: Sink, tuning: Tuning | None = None):
    s = seg.struct()
    _check(lib().photon_run_fused(C.byref(s), C.byref(atm), C.byref(em), int(seed), int(precision),
                                  _ptr(offsets), int(n_photons), C.byref(sink),
                                  None if tuning is None else C.byref(tuning), _stream()))


def run_fused_noalloc(seg: DeviceSegments, atm: Atmosphere, em: Emission, seed, precision, offsets, n_photons,
                      sink: Sink, tuning: Tuning | None = None):
    """run_fused working in the library's static device scratch: the call
    allocates nothing (photon_run_fused_noalloc)."""
    s = seg.struct()
    _check(lib().photon_run_fused_noalloc(C.byref(s), C.byref(atm), C.byref(em), int(seed), int(precision),
                                          _ptr(offsets), int(n_photons), C.byref(sink),
                                          None if tuning is None else C.byref(tuning), _stream()))


def kernel_timing(on: bool):
    """Events around every fused kernel launched on the current device
    outside a stream capture (photon_kernel_timing)."""
    _check(lib().photon_kernel_timing(1 if on else 0))


def fused_kernel_ms() -> float:
    """Kernel time of the last fused launch timed on the current device
    (waits for it)."""
    ms = C.c_float(0.0)
    _check(lib().photon_fused_kernel_ms(C.byref(ms)))
    return float(ms.value)


PEAK_KINDS = ("fp32_fma", "fp64_fma", "int_mad64", "fp32_exp2", "fp32_fma_exp2", "hbm_read", "lds_add32_rtn",
              "lds_add64")


def peak_run(kind: int, work: torch.Tensor, iters: int = 4096):
    """One micro-benchmark launch (photon_peak_run): (lane operations or
    bytes, kernel ms)."""
    ops = C.c_double(0.0)
    ms = C.c_float(0.0)
    _check(lib().photon_peak_run(int(kind), _ptr(work), work.numel() * work.element_size(), int(iters),
                                 C.byref(ops), C.byref(ms), _stream()))
    return ops.value, ms.value


def set_defer_capacity(rays: int):
    """Length of the current device's near-horizon queue for later calls
    (photon_set_defer_capacity)."""
    _check(lib().photon_set_defer_capacity(int(rays)))


def fused_deferred_ms() -> float:
    """Time of the near-horizon double pass after the last timed fused
    launch (0 when it had none)."""
    ms = C.c_float(0.0)
    _check(lib().photon_fused_deferred_ms(C.byref(ms)))
    return float(ms.value)


def tuning(block=256, chunk=4096, blocks_per_cu=0) -> Tuning:
    t = Tuning()
    t.block, t.chunk, t.blocks_per_cu = int(block), int(chunk), int(blocks_per_cu)
    return t


class Plan:
    """One whole step (counts, offsets, cleared sink, fused kernel) captured
    into a HIP graph by the library; replay with launch()."""

    def __init__(self, seg: DeviceSegments, atm: Atmosphere, em: Emission, seed, precision, counts, offsets,
                 sink: Sink, tuning: Tuning | None = None):
        self._keep = (seg, counts, offsets, sink)      # buffers the graph points at
        self._seg = seg.struct()
        self.handle = C.c_void_p()
        _check(lib().photon_plan_create(C.byref(self._seg), C.byref(atm), C.byref(em), int(seed),
                                        int(precision), _ptr(counts), _ptr(offsets), C.byref(sink),
                                        None if tuning is None else C.byref(tuning), C.byref(self.handle)))

    def launch(self):
        _check(lib().photon_plan_launch(self.handle, _stream()))

    def close(self):
        if self.handle:
            torch.cuda.synchronize()
            _check(lib().photon_plan_destroy(self.handle))
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(seg: DeviceSegments, atm: Atmosphere, em: Emission, seed, precision, offsets, sink: Sink,
             candidates, reps=5):
    """Fastest fused launch shape among candidates [(block, chunk, blocks_per_cu)]:
    returns (Tuning, median ms)."""
    arr = (Tuning * len(candidates))()
    for i, (b, c, o) in enumerate(candidates):
        arr[i].block, arr[i].chunk, arr[i].blocks_per_cu = int(b), int(c), int(o)
    best = Tuning()
    ms = C.c_float()
    s = seg.struct()
    _check(lib().photon_autotune(C.byref(s), C.byref(atm), C.byref(em), int(seed), int(precision),
                                 _ptr(offsets), C.byref(sink), arr, len(candidates), int(reps), C.byref(best),
                                 C.byref(ms), _stream()))
    return best, ms.value


# ------------------------------------------------------ differentiable form --
def means(seg: DeviceSegments, atm: Atmosphere, em: Emission, device="cuda"):
    """Per-segment means (float64 tensor), as the count step evaluates them."""
    out = torch.empty(max(seg.n, 1), dtype=torch.float64, device=device)
    s = seg.struct()
    _check(lib().photon_means(C.byref(s), C.byref(atm), C.byref(em), _ptr(out), _stream()))
    return out[:seg.n]


def splat_grid(d: dict) -> SplatGrid:
    g = SplatGrid()
    g.x_min, g.y_min, g.cell = float(d["x_min"]), float(d["y_min"]), float(d["cell"])
    g.nx, g.ny = int(d["nx"]), int(d["ny"])
    g.sigma, g.trunc = float(d["sigma"]), float(d["trunc"])
    return g


def _seg_with_dirs(seg: DeviceSegments, dx, dy, dz) -> Segments:
    s = seg.struct()
    if dx is not None:
        s.dx, s.dy, s.dz = dx.data_ptr(), dy.data_ptr(), dz.data_ptr()
    return s


def splat_forward(seg: DeviceSegments, atm: Atmosphere, lmin, lmax, seed, precision, offsets, mean0,
                  grid: SplatGrid, totals=None, dirs=None):
    """Splatted ground density (ny, nx): float64 (FP64) or float32 (FP32)
    tensor. dirs = (dx, dy, dz) device float64 tensors replacing the
    segments' directions."""
    dt = torch.float64 if precision == FP64 else torch.float32
    D = torch.empty((grid.ny, grid.nx), dtype=dt, device=offsets.device)
    s = _seg_with_dirs(seg, *(dirs if dirs is not None else (None, None, None)))
    _check(lib().photon_splat_forward(C.byref(s), C.byref(atm), float(lmin), float(lmax), int(seed),
                                      int(precision), _ptr(offsets), _ptr(mean0), C.byref(grid), _ptr(D),
                                      _ptr(totals), _stream()))
    return D


def splat_backward(seg: DeviceSegments, atm: Atmosphere, lmin, lmax, seed, precision, offsets, mean0,
                   grid: SplatGrid, grad_density, dirs=None):
    """(dL/dH per layer, dL/d(n0-1), dL/ddx, dL/ddy, dL/ddz) as float64 tensors."""
    dev = offsets.device
    dt = torch.float64 if precision == FP64 else torch.float32
    gD = grad_density.to(dtype=dt).contiguous()
    gH = torch.zeros(int(atm.n_layers), dtype=torch.float64, device=dev)
    ge = torch.zeros(1, dtype=torch.float64, device=dev)
    n = max(seg.n, 1)
    gx, gy, gz = (torch.empty(n, dtype=torch.float64, device=dev) for _ in range(3))
    s = _seg_with_dirs(seg, *(dirs if dirs is not None else (None, None, None)))
    _check(lib().photon_splat_backward(C.byref(s), C.byref(atm), float(lmin), float(lmax), int(seed),
                                       int(precision), _ptr(offsets), _ptr(mean0), C.byref(grid), _ptr(gD),
                                       _ptr(gH), _ptr(ge), _ptr(gx), _ptr(gy), _ptr(gz), _stream()))
    return gH, ge[0], gx[:seg.n], gy[:seg.n], gz[:seg.n]


class SplatProblem:
    """The frozen part of the differentiable form: segments on the device,
    atmosphere layout, band, seed, precision, grid, and the counts' offsets
    and means at the nominal parameters."""

    def __init__(self, seg: DeviceSegments, atm_dict: dict, seed, precision, grid: dict, lmin=300.0, lmax=600.0):
        self.seg = seg
        self.atm_dict = dict(atm_dict)
        self.seed, self.precision = int(seed), int(precision)
        self.lmin, self.lmax = float(lmin), float(lmax)
        self.grid = splat_grid(grid)
        a0 = atmosphere(self.atm_dict)
        em = emission_cherenkov(self.lmin, self.lmax)
        self.counts, self.offsets = count(seg, a0, em, self.seed)
        self.mean0 = means(seg, a0, em)

    def atmosphere(self, H, eta0) -> Atmosphere:
        d = dict(self.atm_dict)
        d["scale_height"] = [float(v) for v in H]
        d["n0_minus_1"] = float(eta0)
        return atmosphere(d)


class SplatDensity(torch.autograd.Function):
    """D(H, n0 - 1, dx, dy, dz): splatted ground density of the frozen
    problem; backward runs the adjoint kernel (photon_splat_backward)."""

    @staticmethod
    def forward(ctx, H, eta0, dx, dy, dz, problem: SplatProblem):
        atm = problem.atmosphere(H.detach().cpu().tolist(), float(eta0.detach().cpu()))
        dirs = tuple(t.detach().to(torch.float64).contiguous() for t in (dx, dy, dz))
        D = splat_forward(problem.seg, atm, problem.lmin, problem.lmax, problem.seed, problem.precision,
                          problem.offsets, problem.mean0, problem.grid, dirs=dirs)
        ctx.problem, ctx.atm, ctx.dirs = problem, atm, dirs
        ctx.h_meta = (H.dtype, H.device, eta0.dtype, eta0.device)
        return D

    @staticmethod
    def backward(ctx, gD):
        p = ctx.problem
        gH, ge, gx, gy, gz = splat_backward(p.seg, ctx.atm, p.lmin, p.lmax, p.seed, p.precision, p.offsets,
                                            p.mean0, p.grid, gD, dirs=ctx.dirs)
        hd, hdev, ed, edev = ctx.h_meta
        return (gH.to(dtype=hd, device=hdev), ge.to(dtype=ed, device=edev).reshape(()), gx, gy, gz, None)
