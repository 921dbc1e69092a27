"""The C ABI on the host: the library loads, exports every declared entry
point, and validates arguments before touching a device (no GPU needed)."""
import ctypes as C
import os
import re

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "photon.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(photon_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def ph():
    from paper_2309_15861_amd import photon
    photon.lib()
    return photon


def test_every_declared_symbol_is_exported(ph):
    names = declared_functions()
    assert {"photon_gen_cherenkov", "photon_gen_fluor", "photon_propagate", "photon_collect",
            "photon_run_fused", "photon_init", "photon_last_error", "photon_version"} <= set(names)
    L = ph.lib()
    for n in names:
        assert hasattr(L, n), n


def test_version(ph):
    assert "gfx950" in ph.version()
    # the library reports the hash of the sources it was built from
    assert ph.version().endswith(ph._build.source_hash())


def test_stale_library_is_refused(ph, monkeypatch):
    """A library built from other sources than the ones beside it does not
    load: the binding raises instead of running stale kernels."""
    monkeypatch.setattr(ph, "_lib", None)
    monkeypatch.setattr(ph._build, "source_hash", lambda: "0000000000000000")
    with pytest.raises(RuntimeError, match="rebuild"):
        ph.lib()


def _valid_atm(ph):
    from paper_2309_15861_amd import workloads as W
    return ph.atmosphere(W.default_atmosphere(absorption=True))


def _fake_segments(ph, n=10):
    s = ph.Segments()
    s.n = n
    for f in ("x0", "y0", "z0", "dx", "dy", "dz", "length", "beta", "t0"):
        setattr(s, f, 0x1000)
    return s


def _gen(ph, seg, atm, lmin=300.0, lmax=600.0, prec=0, counts=0x2000, offsets=0x3000, block=None):
    L = ph.lib()
    return L.photon_gen_cherenkov(None if seg is None else C.byref(seg), None if atm is None else C.byref(atm),
                                  lmin, lmax, 1, prec, counts, offsets,
                                  None if block is None else C.byref(block), None)


def test_validation_errors(ph):
    atm = _valid_atm(ph)
    seg = _fake_segments(ph)
    assert _gen(ph, None, atm) == ph.EINVAL
    assert _gen(ph, seg, None) == ph.EINVAL
    assert _gen(ph, seg, atm, lmin=600.0, lmax=300.0) == ph.EINVAL
    assert "lambda" in ph.lib().photon_last_error().decode()
    assert _gen(ph, seg, atm, lmin=0.0) == ph.EINVAL
    assert _gen(ph, seg, atm, prec=7) == ph.EINVAL
    assert _gen(ph, seg, atm, offsets=None) == ph.EINVAL
    bad = _fake_segments(ph)
    bad.n = -1
    assert _gen(ph, bad, atm) == ph.EINVAL
    nul = _fake_segments(ph)
    nul.beta = None
    assert _gen(ph, nul, atm) == ph.EINVAL
    assert "beta" in ph.lib().photon_last_error().decode()
    for mutate in (lambda a: setattr(a, "n_layers", 0), lambda a: setattr(a, "n_layers", 9),
                   lambda a: a.scale_height.__setitem__(2, 0.0),
                   lambda a: a.h_base.__setitem__(2, 3000.0), lambda a: a.h_base.__setitem__(0, 5.0),
                   lambda a: setattr(a, "n0_minus_1", -1e-4), lambda a: setattr(a, "n_abs", 41),
                   lambda a: a.abs_lambda_nm.__setitem__(3, 100.0),
                   lambda a: a.abs_k_per_m.__setitem__(0, -1.0),
                   lambda a: setattr(a, "h_obs", float("nan"))):
        a = _valid_atm(ph)
        mutate(a)
        assert _gen(ph, seg, a) == ph.EINVAL


def test_fluorescence_and_block_validation(ph):
    import numpy as np
    L = ph.lib()
    atm = _valid_atm(ph)
    seg = _fake_segments(ph)
    lines = np.array([337.0, 357.0])
    rel = np.array([1.0, 0.5])
    # dedx missing for fluorescence
    rc = L.photon_gen_fluor(C.byref(seg), C.byref(atm), lines.ctypes.data, rel.ctypes.data, 2, 10.0, 1, 0,
                            0x2000, 0x3000, None, None)
    assert rc == ph.EINVAL and "dedx" in L.photon_last_error().decode()
    seg.dedx = 0x1000
    zero = np.zeros(2)
    rc = L.photon_gen_fluor(C.byref(seg), C.byref(atm), lines.ctypes.data, zero.ctypes.data, 2, 10.0, 1, 0,
                            0x2000, 0x3000, None, None)
    assert rc == ph.EINVAL
    rc = L.photon_gen_fluor(C.byref(seg), C.byref(atm), lines.ctypes.data, rel.ctypes.data, 0, 10.0, 1, 0,
                            0x2000, 0x3000, None, None)
    assert rc == ph.EINVAL
    rc = L.photon_gen_fluor(C.byref(seg), C.byref(atm), lines.ctypes.data, rel.ctypes.data, 2, -1.0, 1, 0,
                            0x2000, 0x3000, None, None)
    assert rc == ph.EINVAL
    # photon block over capacity
    blk = ph.Block()
    blk.capacity, blk.n_photons, blk.precision = 10, 11, 0
    assert _gen(ph, _fake_segments(ph), atm, block=blk) == ph.ECAPACITY
    blk.n_photons, blk.precision = 5, 1
    assert _gen(ph, _fake_segments(ph), atm, block=blk) == ph.EINVAL   # precision mismatch


def test_sink_validation(ph):
    L = ph.lib()
    atm = _valid_atm(ph)
    blk = ph.Block()
    blk.capacity, blk.n_photons, blk.precision = 0, 0, 0
    s = ph.Sink()
    s.kind = 9
    assert L.photon_collect(C.byref(blk), C.byref(atm), C.byref(s), None) == ph.EINVAL
    s.kind = ph.SINK_TELESCOPES
    s.n_tel = 0
    assert L.photon_collect(C.byref(blk), C.byref(atm), C.byref(s), None) == ph.EINVAL
    s.n_tel = 1
    s.tel[0][3] = -1.0
    assert L.photon_collect(C.byref(blk), C.byref(atm), C.byref(s), None) == ph.EINVAL
    s.kind = ph.SINK_GRID
    s.nx, s.ny, s.cell = 0, 4, 1.0
    assert L.photon_collect(C.byref(blk), C.byref(atm), C.byref(s), None) == ph.EINVAL


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-device path")
def test_valid_arguments_without_device_report_enodev(ph):
    atm = _valid_atm(ph)
    assert _gen(ph, _fake_segments(ph), atm) == ph.ENODEV
    assert ph.lib().photon_init() == ph.ENODEV


def test_kernel_timing_without_device(ph):
    """The timing entry points: a NULL output is rejected before any device
    access; switching timing on needs a device."""
    L = ph.lib()
    assert L.photon_fused_kernel_ms(None) == ph.EINVAL
    assert L.photon_kernel_timing(1) == ph.ENODEV
    assert L.photon_kernel_timing(0) == ph.ENODEV


def test_binding_refuses_to_run_without_library(monkeypatch, tmp_path):
    from paper_2309_15861_amd import photon
    monkeypatch.setattr(photon, "_lib", None)
    monkeypatch.setattr(photon, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        photon.lib()


def test_splat_validation_errors(ph):
    """The differentiable form's entry points validate before any device work."""
    L = ph.lib()
    atm = _valid_atm(ph)
    seg = _fake_segments(ph)

    def grid(**kw):
        g = ph.SplatGrid()
        g.x_min, g.y_min, g.cell, g.nx, g.ny, g.sigma, g.trunc = -320.0, -320.0, 5.0, 128, 128, 5.0, 4.0
        for k, v in kw.items():
            setattr(g, k, v)
        return g

    def fwd(g, density=0x5000, mean0=0x4000, offsets=0x3000, prec=0):
        return L.photon_splat_forward(C.byref(seg), C.byref(atm), 300.0, 600.0, 1, prec, offsets, mean0,
                                      None if g is None else C.byref(g), density, None, None)

    def bwd(g, grad=0x5000, gH=0x6000, ge=0x7000, gd=0x8000):
        return L.photon_splat_backward(C.byref(seg), C.byref(atm), 300.0, 600.0, 1, 0, 0x3000, 0x4000,
                                       C.byref(g), grad, gH, ge, gd, gd, gd, None)

    assert fwd(None) == ph.EINVAL
    for bad in (dict(nx=0), dict(ny=-1), dict(nx=4096, ny=4096), dict(cell=0.0), dict(sigma=0.0),
                dict(trunc=0.0), dict(trunc=100.0), dict(x_min=float("nan"))):
        assert fwd(grid(**bad)) == ph.EINVAL, bad
    assert fwd(grid(), density=None) == ph.EINVAL
    assert fwd(grid(), mean0=None) == ph.EINVAL
    assert fwd(grid(), offsets=None) == ph.EINVAL
    assert fwd(grid(), prec=3) == ph.EINVAL
    assert bwd(grid(), grad=None) == ph.EINVAL
    assert bwd(grid(), gH=None) == ph.EINVAL
    assert bwd(grid(), gd=None) == ph.EINVAL
    em = ph.emission_cherenkov()
    assert L.photon_means(C.byref(seg), C.byref(atm), C.byref(em), None, None) == ph.EINVAL
    if not torch.cuda.is_available():
        assert fwd(grid()) == ph.ENODEV
        assert bwd(grid()) == ph.ENODEV
        assert L.photon_means(C.byref(seg), C.byref(atm), C.byref(em), 0x4000, None) == ph.ENODEV


def test_tuning_validation(ph):
    """Launch shapes are checked before any device work: block 128/256/512,
    chunk a multiple of block and at most 16384, blocks per CU >= 0."""
    L = ph.lib()
    atm = _valid_atm(ph)
    seg = _fake_segments(ph)
    em = ph.emission_cherenkov()
    sink = ph.Sink()
    sink.kind = ph.SINK_STATUS
    for b, c, o in ((100, 400, 0), (256, 300, 0), (256, 16384 + 256, 0), (512, 0, 0), (256, 4096, -1)):
        t = ph.tuning(b, c, o)
        rc = L.photon_run_fused(C.byref(seg), C.byref(atm), C.byref(em), 1, 1, 0x3000, -1, C.byref(sink),
                                C.byref(t), None)
        assert rc == ph.EINVAL, (b, c, o)
        assert "tuning" in L.photon_last_error().decode()


def test_cut_validation(ph):
    """The angular particle cut is validated before any device work."""
    L = ph.lib()
    atm = _valid_atm(ph)
    seg = _fake_segments(ph)

    def count(em):
        return L.photon_count(C.byref(seg), C.byref(atm), C.byref(em), 1, 0x2000, 0x3000, None)

    em = ph.emission_cherenkov(cut_points=[[0.0, 0.0, 2200.0]])
    assert count(em) == ph.ENODEV
    em.n_cut_points = ph.MAX_CUT_POINTS + 1
    assert count(em) == ph.EINVAL
    em.n_cut_points = -1
    assert count(em) == ph.EINVAL
    em = ph.emission_cherenkov(cut_points=[[0.0, 0.0, 2200.0]])
    em.cut_cos = 1.5
    assert count(em) == ph.EINVAL
    em.cut_cos = float("nan")
    assert count(em) == ph.EINVAL
    em = ph.emission_cherenkov(cut_points=[[0.0, float("inf"), 2200.0]])
    assert count(em) == ph.EINVAL
    assert b"not finite" in L.photon_last_error()


def test_beam_validation(ph):
    """Fluorescence beaming is validated before any device work."""
    L = ph.lib()
    atm = _valid_atm(ph)
    seg = _fake_segments(ph)
    seg.dedx = 0x1000

    def count(em):
        return L.photon_count(C.byref(seg), C.byref(atm), C.byref(em), 1, 0x2000, 0x3000, None)

    def em(**kw):
        e = ph.emission_fluor([391.0], [1.0], 10.0, beam_area=((0.0, 0.0, 2200.0), 200.0))
        for k, v in kw.items():
            setattr(e, k, v)
        return e

    assert count(em()) == ph.ENODEV
    assert count(em(beam=2)) == ph.EINVAL
    assert count(em(beam_radius=-1.0)) == ph.EINVAL
    assert count(em(beam_radius=float("nan"))) == ph.EINVAL
    assert count(em(beam_margin_rad=-0.1)) == ph.EINVAL
    assert count(em(beam_margin_rad=2.0)) == ph.EINVAL
    e = em()
    e.beam_center[1] = float("inf")
    assert count(e) == ph.EINVAL
    # photon_generate needs a block
    assert L.photon_generate(C.byref(seg), C.byref(atm), C.byref(em()), 1, 0, 0x3000, None, None) == ph.EINVAL


def test_radial_validation(ph):
    """The radial profile sink and its finish validate before device work."""
    L = ph.lib()

    def sink(**kw):
        s = ph.Sink()
        s.kind = ph.SINK_RADIAL
        s.core_x, s.core_y, s.r_min, s.r_max, s.t_ref_ns = 0.0, 0.0, 1.0, 1000.0, 0.0
        s.n_bins, s.log_bins = 100, 1
        s.radial_count, s.radial_weight, s.radial_wt = 0x1000, 0x2000, 0x3000
        for k, v in kw.items():
            setattr(s, k, v)
        return s

    def prof(s, out=0x4000):
        return L.photon_radial_profile(C.byref(s), out, out, None)

    assert prof(sink()) == ph.ENODEV
    for bad in (dict(n_bins=0), dict(n_bins=ph.MAX_RADIAL_BINS + 1), dict(log_bins=2), dict(r_min=0.0),
                dict(r_max=1.0), dict(r_min=-1.0, log_bins=0), dict(core_x=float("nan")),
                dict(t_ref_ns=float("inf")), dict(radial_wt=None), dict(kind=ph.SINK_GRID)):
        assert prof(sink(**bad)) == ph.EINVAL, bad
    assert prof(sink(), out=None) == ph.EINVAL
    assert prof(sink(r_min=0.0, log_bins=0)) == ph.ENODEV


def test_table_validation(ph):
    """Correction tables: shape checks and the atmosphere fingerprint, before
    device work."""
    L = ph.lib()
    atm = _valid_atm(ph)

    def table(**kw):
        t = ph.TableStruct()
        t.n_h, t.n_q, t.n_v, t.h_max, t.q_max, t.corr, t.vert = 17, 17, 257, 40000.0, 5.0, 0x1000, 0x2000
        for k, v in kw.items():
            setattr(t, k, v)
        return t

    assert L.photon_table_build(C.byref(atm), C.byref(table()), None) == ph.ENODEV
    for bad in (dict(n_h=1), dict(n_q=5000), dict(n_v=1), dict(h_max=1000.0), dict(q_max=0.0),
                dict(q_max=float("nan")), dict(corr=None)):
        assert L.photon_table_build(C.byref(atm), C.byref(table(**bad)), None) == ph.EINVAL, bad
    # a table that was never built (hash 0) or built for another atmosphere
    t = table()
    a2 = ph.Atmosphere.from_buffer_copy(atm)
    a2.table = C.addressof(t)
    seg = _fake_segments(ph)
    assert _gen(ph, seg, a2) == ph.EINVAL
    assert b"not built for this atmosphere" in L.photon_last_error()


def test_noalloc_entry_validates_like_run_fused(ph):
    """photon_run_fused_noalloc checks its arguments exactly as
    photon_run_fused does, before any device work."""
    L = ph.lib()
    atm = _valid_atm(ph)
    seg = _fake_segments(ph)
    em = ph.emission_cherenkov()
    sink = ph.Sink()
    sink.kind = ph.SINK_STATUS
    for fn in (L.photon_run_fused, L.photon_run_fused_noalloc):
        t = ph.tuning(100, 400, 0)
        assert fn(C.byref(seg), C.byref(atm), C.byref(em), 1, 1, 0x3000, -1, C.byref(sink), C.byref(t),
                  None) == ph.EINVAL
        assert fn(C.byref(seg), C.byref(atm), C.byref(em), 1, 1, None, -1, C.byref(sink), None,
                  None) == ph.EINVAL
        assert fn(C.byref(seg), C.byref(atm), C.byref(em), 1, 1, 0x3000, -2, C.byref(sink), None,
                  None) == ph.EINVAL
        assert fn(C.byref(seg), C.byref(atm), C.byref(em), 1, 7, 0x3000, -1, C.byref(sink), None,
                  None) == ph.EINVAL
        if not torch.cuda.is_available():
            assert fn(C.byref(seg), C.byref(atm), C.byref(em), 1, 1, 0x3000, -1, C.byref(sink), None,
                      None) == ph.ENODEV


def test_peak_run_validation(ph):
    """The micro-benchmark entry point checks kind, iterations and pointers
    before any device work."""
    L = ph.lib()
    ops, ms = C.c_double(), C.c_float()
    assert L.photon_peak_run(8, 0x1000, 1 << 20, 16, C.byref(ops), C.byref(ms), None) == ph.EINVAL
    assert L.photon_peak_run(-1, 0x1000, 1 << 20, 16, C.byref(ops), C.byref(ms), None) == ph.EINVAL
    assert L.photon_peak_run(0, 0x1000, 1 << 20, 0, C.byref(ops), C.byref(ms), None) == ph.EINVAL
    assert L.photon_peak_run(0, None, 1 << 20, 16, C.byref(ops), C.byref(ms), None) == ph.EINVAL
    assert L.photon_peak_run(0, 0x1000, 1 << 20, 16, None, C.byref(ms), None) == ph.EINVAL
    if not torch.cuda.is_available():
        assert L.photon_peak_run(0, 0x1000, 1 << 20, 16, C.byref(ops), C.byref(ms), None) == ph.ENODEV
