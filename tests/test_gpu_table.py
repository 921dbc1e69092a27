"""GPU parity of the straight-line propagation with correction tables
(section 2).

Bars: the GPU's table (float storage) matches the oracle's table to float
rounding; every photon of the unfused FP64 path and of the fused plane sink
(both precisions) matches the oracle's table method on the same inputs
(FP64: landing 1e-4 m, time 1e-3 ns, weight 1e-6, direction 1e-7 rad, the
float storage of the corrections; FP32: the FP32 bars on every photon, the
slant factor taken from the double zenith cosine); photons outside the
table take the exact integrals; and at the default resolution (257 x 257
nodes) the method stays within 0.15 m and 0.5 ns of the exact propagation on
the full shower (rms below 1 mm).
"""
import numpy as np
import pytest
import torch

import oracle.oracle as O
from paper_2309_15861_amd import photon as ph
from paper_2309_15861_amd import workloads as W
from test_gpu_parity import TOL32, check_propagated, run_fused_plane

pytestmark = pytest.mark.gpu

SEED = 2
H_MAX = 40000.0
Q_MAX = float(np.tan(np.radians(80.0)))
TOL64_TABLE = dict(land=1e-9, land_abs=1e-4, t=1e-3, w=1e-6, dir=1e-7)


def _check64(g, ref):
    landed = ref["status"] == O.LANDED
    assert np.array_equal(g["status"], ref["status"])
    d = np.hypot(g["x"] - ref["xl"], g["y"] - ref["yl"])[landed]
    scale = np.maximum(np.hypot(ref["xl"] - ref["xe"], ref["yl"] - ref["ye"]), 1.0)[landed]
    assert np.all(d <= TOL64_TABLE["land_abs"] + TOL64_TABLE["land"] * scale), d.max()
    assert np.max(np.abs(g["t_ns"] - ref["tl"])[landed]) <= TOL64_TABLE["t"]
    assert np.max((np.abs(g["weight"] - ref["weight"]) / ref["weight"])[landed]) <= TOL64_TABLE["w"]
    u = np.stack([g["ux"], g["uy"], g["uz"]], 1)
    assert np.max(np.linalg.norm(u - ref["ul"], axis=1)[landed]) <= TOL64_TABLE["dir"]


@pytest.fixture(scope="module")
def setup():
    a = W.default_atmosphere(absorption=True)
    atm0 = ph.atmosphere(a)
    tab = ph.PropagationTable(atm0, 65, 65, H_MAX, Q_MAX, 1025)
    atm_t = tab.attach(atm0)
    oatm = O.Atmosphere.from_dict(a)
    otab = O.Table(oatm, 65, 65, H_MAX, Q_MAX, 1025)
    seg = W.subsample(W.shower_cherenkov(), np.arange(0, 200_000, 40))
    d = ph.DeviceSegments(seg)
    em = ph.emission_cherenkov()
    counts, offsets = ph.count(d, atm0, em, SEED)
    torch.cuda.synchronize()
    off = offsets.cpu().numpy().view(np.uint64)
    gen = O.photons_all(seg, oatm, "cherenkov", SEED, off)
    ref = O.propagate_table(gen, oatm, otab)
    return dict(a=a, atm0=atm0, tab=tab, atm_t=atm_t, oatm=oatm, otab=otab, seg=seg, d=d, em=em,
                offsets=offsets, total=int(off[-1]), gen=gen, ref=ref)


def test_table_matches_oracle_table(setup):
    s = setup
    corr = s["tab"].corr.cpu().numpy().reshape(65, 65, 4)[:, :, :3].astype(np.float64)
    vert = s["tab"].vert.cpu().numpy().reshape(1025, 2).astype(np.float64)
    oc, ov = s["otab"].corr, s["otab"].vert
    for c in range(3):
        scale = np.max(np.abs(oc[:, :, c]))
        assert np.max(np.abs(corr[:, :, c] - oc[:, :, c])) <= 1e-6 * scale + 1e-9, c
    assert np.max(np.abs(vert - ov) / np.maximum(np.abs(ov), 1e-30)) <= 2e-7


def test_unfused_fp64_every_photon(setup):
    s = setup
    blk = ph.PhotonBlock(s["total"], ph.FP64)
    blk.n_photons = s["total"]
    ph.generate(s["d"], s["atm0"], s["em"], SEED, ph.FP64, s["offsets"], blk)
    ph.propagate(blk, s["atm_t"])
    torch.cuda.synchronize()
    _check64(blk.numpy(), s["ref"])


@pytest.mark.parametrize("prec", [ph.FP64, ph.FP32])
def test_fused_plane_every_photon(setup, prec):
    s = setup
    g, tot = run_fused_plane(s["d"], s["atm_t"], s["em"], SEED, prec, s["offsets"], s["total"])
    assert tot[:7].sum() == s["total"]
    if prec == ph.FP64:
        _check64(g, s["ref"])
    else:
        _check32(g, s["ref"])


def _check32(g, ref):
    """The fused kernel carries each photon's zenith cosine in double, so
    every photon meets the FP32 bars, grazing rays included."""
    assert np.array_equal(g["status"], ref["status"])
    check_propagated(g, ref, TOL32)


def test_exact_fp32_on_the_same_shower_photons(setup):
    """The exact FP32 fused path on these shower photons, against the exact
    oracle, with the same bars."""
    s = setup
    g, tot = run_fused_plane(s["d"], s["atm0"], s["em"], SEED, ph.FP32, s["offsets"], s["total"])
    _check32(g, s["gen"])


def test_outside_the_table_is_exact(setup):
    """A table that no photon falls into: the run equals the exact one."""
    s = setup
    tiny = ph.PropagationTable(s["atm0"], 2, 2, W.H_OBS + 1.0, 1e-6, 2)
    atm_x = tiny.attach(s["atm0"])
    g0, _ = run_fused_plane(s["d"], s["atm0"], s["em"], SEED, ph.FP64, s["offsets"], s["total"])
    g1, _ = run_fused_plane(s["d"], atm_x, s["em"], SEED, ph.FP64, s["offsets"], s["total"])
    assert np.array_equal(g0["status"], g1["status"])
    for f in ("x", "y", "t_ns", "weight", "ux"):
        assert np.allclose(g0[f], g1[f], rtol=1e-12, atol=1e-12), f


def test_differentiable_form_refuses_tables(setup):
    s = setup
    gdict = W.splat_grid_128()
    with pytest.raises(ph.PhotonError, match="exact propagation"):
        mean0 = ph.means(s["d"], s["atm0"], s["em"])
        ph.splat_forward(s["d"], s["atm_t"], 300.0, 600.0, SEED, ph.FP32, s["offsets"], mean0,
                         ph.splat_grid(gdict))


def test_default_table_accuracy_on_the_shower():
    """The benchmarked shower, FP64: the 257 x 257 table against the exact
    integrals, every photon."""
    a = W.default_atmosphere(absorption=True)
    atm0 = ph.atmosphere(a)
    tab = ph.PropagationTable(atm0)
    atm_t = tab.attach(atm0)
    seg = W.shower_cherenkov()
    d = ph.DeviceSegments(seg)
    em = ph.emission_cherenkov()
    counts, offsets = ph.count(d, atm0, em, SEED)
    torch.cuda.synchronize()
    total = int(offsets[-1].item())
    g0, _ = run_fused_plane(d, atm0, em, SEED, ph.FP64, offsets, total)
    g1, _ = run_fused_plane(d, atm_t, em, SEED, ph.FP64, offsets, total)
    landed = g0["status"] == ph.LANDED
    assert np.array_equal(g0["status"], g1["status"])
    dxy = np.hypot(g1["x"] - g0["x"], g1["y"] - g0["y"])[landed]
    dt = np.abs(g1["t_ns"] - g0["t_ns"])[landed]
    dw = (np.abs(g1["weight"] - g0["weight"]) / g0["weight"])[landed]
    print(f"257x257 table vs exact: landing max {dxy.max():.3e} m rms {np.sqrt(np.mean(dxy**2)):.3e} m, "
          f"time max {dt.max():.3e} ns, weight max {dw.max():.3e}")
    # worst where a table cell straddles the 10 km layer base at 78-80 degrees
    # (first order there); measured 0.10 m, 0.34 ns, rms 0.3 mm
    assert dxy.max() < 0.15 and dt.max() < 0.5 and np.sqrt(np.mean(dxy ** 2)) < 1e-3 and dw.max() < 1e-5
