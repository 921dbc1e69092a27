"""GPU parity of the Cherenkov angular particle cut (section 1.2.1, Fig. 2).

Bars: counts and the per-segment keep decision bit-exact against the oracle
(both sides evaluate d.v >= cos(cut)|v| in FP64 in the same order); the
fused telescope run with the cut produces exactly the hits of the kept
segments of the uncut run (a kept segment draws the same photons); hits the
cut removes come only from segments closer to the hit telescope than 15
telescope radii, the limit the paper gives for a 6 degree cut.
"""
import numpy as np
import pytest
import torch

import oracle.oracle as O
from paper_2309_15861_amd import photon as ph
from paper_2309_15861_amd import workloads as W

pytestmark = pytest.mark.gpu

SEED = 2
CUT_DEG = 6.0


@pytest.fixture(scope="module")
def shower():
    a = W.default_atmosphere(absorption=True)
    seg = W.shower_cherenkov()
    tel = W.telescopes_16()
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    return a, seg, tel, d, atm


def _targets(name, tel):
    return np.array([[0.0, 0.0, W.H_OBS]]) if name == "centre" else tel[:, :3]


def _keys(h):
    return (h["segment"].astype(np.int64) << 32) | h["j"].astype(np.int64)


@pytest.mark.parametrize("target", ["centre", "telescopes"])
def test_counts_and_means_with_cut_bit_exact(shower, target):
    a, seg, tel, d, atm = shower
    pts = _targets(target, tel)
    em = ph.emission_cherenkov(cut_points=pts, cut_angle_deg=CUT_DEG)
    counts, offsets = ph.count(d, atm, em, SEED)
    mu = ph.means(d, atm, em)
    torch.cuda.synchronize()
    gcnt = counts.cpu().numpy().view(np.uint32)[:len(seg["x0"])]
    gmu = mu.cpu().numpy()
    oatm = O.Atmosphere.from_dict(a)
    ocnt, omu, mg = O.counts(seg, oatm, "cherenkov", SEED, cut=(pts, em.cut_cos))
    keep = O.passes_cut(seg, pts, em.cut_cos)
    # the keep decision: every segment above threshold has a positive mean
    assert np.array_equal(gmu > 0, keep & (omu > 0)) and np.array_equal(omu > 0, keep & (omu > 0))
    assert np.all(gmu[~keep] == 0.0) and np.all(gcnt[~keep] == 0)
    assert np.array_equal(gmu, omu)
    assert np.array_equal(gcnt, ocnt)
    off = offsets.cpu().numpy().view(np.uint64)
    assert np.array_equal(off, O.offsets_of(ocnt))
    assert 0.05 < keep.mean() < 0.5


def test_fused_hits_with_cut_are_the_kept_segments_hits(shower):
    a, seg, tel, d, atm = shower
    pts = tel[:, :3]
    runs = {}
    for cut in (False, True):
        em = ph.emission_cherenkov(cut_points=pts if cut else None, cut_angle_deg=CUT_DEG)
        counts, offsets = ph.count(d, atm, em, SEED)
        total = int(offsets[-1].item())
        hits = ph.HitBuffer(max(total // 100, 1))
        totals = ph.status_totals()
        ph.run_fused(d, atm, em, SEED, ph.FP32, offsets, total, ph.sink_telescopes(tel, hits, totals))
        torch.cuda.synchronize()
        assert hits.count() <= hits.capacity
        assert int(totals.sum().item()) == total
        runs[cut] = (hits.numpy(), total, em)
    h0, total0, _ = runs[False]
    h1, total1, em = runs[True]
    keep = O.passes_cut(seg, pts, em.cut_cos)
    k0, k1 = _keys(h0), _keys(h1)
    kept0 = keep[h0["segment"]]
    assert np.array_equal(np.sort(k1), np.sort(k0[kept0]))
    assert total1 < 0.5 * total0
    # hits lost to the cut come from segments within 15 telescope radii
    lost = np.nonzero(~kept0)[0]
    s = h0["segment"][lost]
    dvec = np.stack([seg["dx"], seg["dy"], seg["dz"]], 1)[s]
    u = dvec / np.linalg.norm(dvec, axis=1, keepdims=True)
    m = np.stack([seg["x0"], seg["y0"], seg["z0"]], 1)[s] + 0.5 * seg["length"][s, None] * u
    tk = h0["telescope"][lost]
    dist = np.linalg.norm(tel[tk, :3] - m, axis=1)
    assert np.all(dist <= 15.0 * tel[tk, 3])
    assert len(k1) > 0.9 * len(k0)


def test_cut_hits_match_oracle_on_subsample():
    """Every photon of a shower subsample through the oracle with the cut
    applied to its counts: the FP64 fused hit set is the oracle's."""
    a = W.default_atmosphere(absorption=True)
    seg = W.subsample(W.shower_cherenkov(), np.arange(0, 200_000, 25))
    tel = W.telescopes_16(radius=20.0)
    pts = tel[:, :3]
    em = ph.emission_cherenkov(cut_points=pts, cut_angle_deg=CUT_DEG)
    oatm = O.Atmosphere.from_dict(a)
    ocnt, _, _ = O.counts(seg, oatm, "cherenkov", SEED, cut=(pts, em.cut_cos))
    off = np.concatenate([[0], np.cumsum(ocnt.astype(np.int64))])
    total = int(off[-1])
    s_of = np.repeat(np.arange(len(ocnt)), ocnt.astype(np.int64))
    j_of = (np.arange(total) - off[s_of]).astype(np.uint32)
    ref = O.photons(seg, oatm, "cherenkov", SEED, s_of.astype(np.uint64), j_of)
    tid, _ = O.telescopes(ref, tel, oatm.index(a["h_obs"]))
    hit = tid >= 0
    key_ref = (s_of[hit].astype(np.int64) << 32) | j_of[hit].astype(np.int64)
    assert hit.sum() > 200
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    counts, offsets = ph.count(d, atm, em, SEED)
    torch.cuda.synchronize()
    assert np.array_equal(offsets.cpu().numpy().view(np.uint64), off.astype(np.uint64))
    hits = ph.HitBuffer(total)
    ph.run_fused(d, atm, em, SEED, ph.FP64, offsets, total, ph.sink_telescopes(tel, hits))
    torch.cuda.synchronize()
    h = hits.numpy()
    assert np.array_equal(np.sort(_keys(h)), np.sort(key_ref))
    assert np.array_equal(h["telescope"][np.argsort(_keys(h))], tid[hit][np.argsort(key_ref)])
