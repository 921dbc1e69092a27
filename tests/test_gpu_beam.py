"""GPU parity of fluorescence beaming (section 1.1.1).

Bars: counts and means bit-exact against the oracle (both evaluate the cone
in FP64 without contraction in the same order); every beamed photon of the
unfused and the fused paths within the fluorescence tolerances of the
isotropic path; the fused FP64 telescope hit set equal to the oracle's; and
at full size the expected hit number of beamed emission equal to that of
isotropic emission within 4 sigma, with far fewer photons.
"""
import numpy as np
import pytest
import torch

import oracle.oracle as O
from paper_2309_15861_amd import photon as ph
from paper_2309_15861_amd import workloads as W
from test_gpu_parity import (TOL32, TOL64, check_propagated, run_block,
                             run_fused_plane)

pytestmark = pytest.mark.gpu

SEED = 3
MARGIN_DEG = 1.0


def _setup(seg, tel, yield_per_MeV=W.FLUOR_YIELD_PER_MEV, beam=True, seed=SEED):
    a = W.default_atmosphere(absorption=True)
    lam, rel = W.fluorescence_lines()
    area = ph.enclosing_sphere(tel)
    em = ph.emission_fluor(lam, rel, yield_per_MeV, beam_area=area if beam else None,
                           beam_margin_deg=MARGIN_DEG)
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    counts, offsets = ph.count(d, atm, em, seed)
    torch.cuda.synchronize()
    ob = (area[0], area[1], em.beam_margin_rad) if beam else None
    return a, lam, rel, em, d, atm, counts, offsets, ob


@pytest.mark.parametrize("name", ["c3", "near"])
def test_counts_and_means_bit_exact(name):
    seg = W.fluorescence() if name == "c3" else W.fluorescence_near_array(2000)
    tel = W.telescopes_16(radius=40.0)
    a, lam, rel, em, d, atm, counts, offsets, ob = _setup(seg, tel)
    gcnt = counts.cpu().numpy().view(np.uint32)[:len(seg["x0"])]
    gmu = ph.means(d, atm, em).cpu().numpy()
    ocnt, omu, mg = O.counts(seg, O.Atmosphere.from_dict(a), "fluorescence", SEED,
                             yield_per_MeV=W.FLUOR_YIELD_PER_MEV, beam=ob)
    assert np.array_equal(gmu, omu)
    assert np.array_equal(gcnt, ocnt)
    off = offsets.cpu().numpy().view(np.uint64)
    assert np.array_equal(off, O.offsets_of(ocnt))


@pytest.fixture(scope="module")
def beam_run():
    seg = W.fluorescence_near_array(400)
    tel = W.telescopes_16(radius=40.0)
    a, lam, rel, em, d, atm, counts, offsets, ob = _setup(seg, tel, yield_per_MeV=200.0)
    off = offsets.cpu().numpy().view(np.uint64)
    ref = O.photons_all(seg, O.Atmosphere.from_dict(a), "fluorescence", SEED, off, yield_per_MeV=200.0,
                        lines_nm=lam, line_rel=rel, beam=ob)
    return a, seg, tel, d, atm, em, offsets, int(off[-1]), ref


def test_unfused_fp64_every_photon(beam_run):
    a, seg, tel, d, atm, em, offsets, total, ref = beam_run
    assert total > 20000
    blk, e, g = run_block(d, atm, em, SEED, ph.FP64, offsets, total)
    ue = np.stack([e["ux"], e["uy"], e["uz"]], 1)
    assert np.max(np.abs(ue - ref["ue"])) < 1e-12
    assert np.array_equal(e["wavelength_nm"], ref["lam"])
    assert np.array_equal(g["status"], ref["status"])
    check_propagated(g, ref, TOL64)


def test_unfused_fp32_every_photon(beam_run):
    a, seg, tel, d, atm, em, offsets, total, ref = beam_run
    blk, e, g = run_block(d, atm, em, SEED, ph.FP32, offsets, total)
    ue = np.stack([e["ux"], e["uy"], e["uz"]], 1).astype(np.float64)
    assert np.max(np.abs(ue - ref["ue"])) < 2e-6
    diff = g["status"] != ref["status"]
    assert np.all(np.abs(ref["ue"][diff, 2]) < 1e-5)
    check_propagated(g, ref, TOL32, mask=~diff)


@pytest.mark.parametrize("prec", [ph.FP64, ph.FP32])
def test_fused_plane_every_photon(beam_run, prec):
    a, seg, tel, d, atm, em, offsets, total, ref = beam_run
    g, tot = run_fused_plane(d, atm, em, SEED, prec, offsets, total)
    assert tot[:7].sum() == total and tot[ph.HORIZON_FLOAT] == 0
    assert np.array_equal(g["status"], ref["status"])
    check_propagated(g, ref, TOL64 if prec == ph.FP64 else TOL32)


def test_fused_fp64_hits_match_oracle(beam_run):
    a, seg, tel, d, atm, em, offsets, total, ref = beam_run
    oatm = O.Atmosphere.from_dict(a)
    tid, rec = O.telescopes(ref, tel, oatm.index(a["h_obs"]))
    off = offsets.cpu().numpy().view(np.uint64)
    s_of = np.repeat(np.arange(len(seg["x0"])), np.diff(off).astype(np.int64))
    j_of = np.arange(total) - off[s_of].astype(np.int64)
    hit = tid >= 0
    assert hit.sum() > 1000
    key_ref = (s_of[hit].astype(np.int64) << 32) | j_of[hit]
    hits = ph.HitBuffer(total)
    ph.run_fused(d, atm, em, SEED, ph.FP64, offsets, total, ph.sink_telescopes(tel, hits))
    torch.cuda.synchronize()
    h = hits.numpy()
    key = (h["segment"].astype(np.int64) << 32) | h["j"].astype(np.int64)
    assert np.array_equal(np.sort(key), np.sort(key_ref))
    assert np.array_equal(h["telescope"][np.argsort(key)], tid[hit][np.argsort(key_ref)])


def _fused_hits(d, atm, em, seed, tel):
    """(photons, hits) of one fused FP32 telescope run; hits are counted in
    the status totals, records are not kept."""
    _, o = ph.count(d, atm, em, seed)
    total = int(o[-1].item())
    hits = ph.HitBuffer(1)
    totals = ph.status_totals()
    ph.run_fused(d, atm, em, seed, ph.FP32, o, total, ph.sink_telescopes(tel, hits, totals))
    torch.cuda.synchronize()
    tot = totals.cpu().numpy()
    assert int(tot[:7].sum()) == total
    return total, int(tot[ph.HIT])


def test_full_size_expected_hits_unchanged():
    """The 1e5-segment fluorescence workload, 16 telescopes of R = 40 m:
    isotropic hits (one seed) against the mean of beamed hits over 64 seeds."""
    seg = W.fluorescence()
    tel = W.telescopes_16(radius=40.0)
    a, lam, rel, em_b, d, atm, _, _, _ = _setup(seg, tel)
    em_i = ph.emission_fluor(lam, rel, W.FLUOR_YIELD_PER_MEV)
    n_iso, h_iso = _fused_hits(d, atm, em_i, SEED, tel)
    hb, nb = [], []
    for k in range(64):
        n, h = _fused_hits(d, atm, em_b, 100 + k, tel)
        hb.append(h)
        nb.append(n)
    mean_b = float(np.mean(hb))
    sigma = np.sqrt(h_iso + mean_b / len(hb))
    assert h_iso > 5000
    assert abs(h_iso - mean_b) <= 4.0 * sigma, (h_iso, mean_b, sigma)
    assert np.mean(nb) < 0.01 * n_iso
