"""GPU parity of the batched form (many showers of uneven size in one
persistent launch, replayed from a captured graph) against the FP64 oracle.

Each shower's segments are numbered from 0 (index_in_shower restarts), so
the shower id is the only part of the random-number counter that tells the
showers apart: the oracle draws other counts when it is dropped, and the GPU
must match the oracle with it, count by count and photon by photon.

Tolerances are those of the single-shower parity tests (test_gpu_parity):
counts and offsets bit-exact; FP64 landing 1e-9 relative, time 1e-6 ns;
FP32 landing 1e-5, time 0.1 ns, direction 1e-6 rad.
"""
import numpy as np
import pytest
import torch

import oracle.oracle as O
from paper_2309_15861_amd import photon as ph
from paper_2309_15861_amd import workloads as W
from test_gpu_parity import TOL32, TOL64, check_propagated, gpu_counts

pytestmark = pytest.mark.gpu

SEED = 4


def hit_tolerance(ref, rec, prec):
    """Bound on a hit record's entry point: the landing tolerance (relative
    to the displacement from the emission point) plus the direction
    tolerance over the distance from the landing point to the entry point."""
    tol = TOL64 if prec == ph.FP64 else TOL32
    scale = np.maximum(np.hypot(ref["xl"] - ref["xe"], ref["yl"] - ref["ye"]), 1.0)
    return tol["land"] * scale + tol["dir"] * np.abs(rec[:, 4]) + 1e-9


@pytest.fixture(scope="module")
def batched_run():
    a = W.default_atmosphere(absorption=True)
    seg = W.batched_showers(seed=SEED, n_showers=16, n_min=30, n_max=300)
    em = ph.emission_cherenkov()
    d, atm, counts, offsets = gpu_counts(seg, a, em, SEED)
    oatm = O.Atmosphere.from_dict(a)
    ocnt = O.counts(seg, oatm, "cherenkov", SEED)[0]
    off = O.offsets_of(ocnt)
    ref = O.photons_all(seg, oatm, "cherenkov", SEED, off)
    return a, seg, d, atm, em, counts, offsets, ocnt, off, ref


def test_batched_input_shape(batched_run):
    """Sixteen showers with ids 0..15, every one numbered from 0."""
    a, seg, d, atm, em, counts, offsets, ocnt, off, ref = batched_run
    assert np.array_equal(np.unique(seg["shower"]), np.arange(16))
    for s in range(16):
        rows = np.nonzero(seg["shower"] == s)[0]
        assert np.array_equal(seg["index_in_shower"][rows], np.arange(len(rows)))


def test_batched_counts_bit_exact(batched_run):
    a, seg, d, atm, em, counts, offsets, ocnt, off, ref = batched_run
    gcnt = counts.cpu().numpy().view(np.uint32)
    assert np.array_equal(gcnt, ocnt)
    assert np.array_equal(offsets.cpu().numpy().view(np.uint64), off)
    # the shower id enters the count stream: without it the oracle draws
    # other counts on almost every segment with a sizeable mean
    seg0 = dict(seg, shower=np.zeros_like(seg["shower"]))
    ocnt0, mu, _ = O.counts(seg0, O.Atmosphere.from_dict(a), "cherenkov", SEED)
    big = (mu > 20.0) & (seg["shower"] > 0)
    assert big.sum() > 500
    assert (ocnt0[big] != ocnt[big]).mean() > 0.8


@pytest.mark.parametrize("prec", [ph.FP64, ph.FP32])
def test_batched_fused_every_photon(batched_run, prec):
    """The persistent kernel over all showers at once, final state of every
    photon (plane sink, slot order) against the oracle's photon."""
    a, seg, d, atm, em, counts, offsets, ocnt, off, ref = batched_run
    total = int(off[-1])
    plane = ph.PhotonBlock(total, prec)
    plane.n_photons = total
    totals = ph.status_totals()
    ph.run_fused(d, atm, em, SEED, prec, offsets, -1, ph.sink_plane(plane, totals), ph.tuning(256, 4096, 0))
    torch.cuda.synchronize()
    g = plane.numpy()
    tot = totals.cpu().numpy()
    assert tot[:7].sum() == total and tot[ph.HORIZON_FLOAT] == 0
    s_of = np.repeat(np.arange(len(seg["x0"]), dtype=np.uint32), ocnt.astype(np.int64))
    assert np.array_equal(g["segment"], s_of)
    assert np.array_equal(g["j"], (np.arange(total, dtype=np.uint64) - off[s_of]).astype(np.uint32))
    assert np.array_equal(g["status"], ref["status"])
    check_propagated(g, ref, TOL64 if prec == ph.FP64 else TOL32)


@pytest.mark.parametrize("prec", [ph.FP64, ph.FP32])
def test_batched_plan_hits_against_oracle(batched_run, prec):
    """The captured step (counts, offsets, cleared outputs, fused kernel)
    replayed three times with eager work between the replays: every replay's
    counts and telescope hit set equal the oracle's."""
    a, seg, d, atm, em, counts, offsets, ocnt, off, ref = batched_run
    tel = W.telescopes_16(radius=30.0)
    n_obs = O.Atmosphere.from_dict(a).index(a["h_obs"])
    tid, rec = O.telescopes(ref, tel, n_obs)
    hit = tid >= 0
    assert hit.sum() > 200
    s_of = np.repeat(np.arange(len(seg["x0"]), dtype=np.int64), ocnt.astype(np.int64))
    j_of = np.arange(len(ref), dtype=np.int64) - off[s_of].astype(np.int64)
    key_ref = (s_of[hit] << 32) | j_of[hit]
    order_ref = np.argsort(key_ref)
    c2 = torch.empty_like(counts)
    o2 = torch.empty_like(offsets)
    hits = ph.HitBuffer(int(off[-1]))
    totals = ph.status_totals()
    plan = ph.Plan(d, atm, em, SEED, prec, c2, o2, ph.sink_telescopes(tel, hits, totals), ph.tuning(256, 4096, 0))
    try:
        for rep in range(3):
            c2.fill_(-1)
            plan.launch()
            torch.cuda.synchronize()
            assert np.array_equal(c2.cpu().numpy().view(np.uint32), ocnt)
            h = hits.numpy()
            key = (h["segment"].astype(np.int64) << 32) | h["j"].astype(np.int64)
            order = np.argsort(key)
            assert np.array_equal(key[order], key_ref[order_ref]), rep
            assert np.array_equal(h["telescope"][order], tid[hit][order_ref])
            hp = np.stack([h["x"], h["y"], h["z"]], 1)[order]
            err = np.linalg.norm(hp - rec[hit][order_ref, :3], axis=1)
            assert np.all(err <= hit_tolerance(ref[hit][order_ref], rec[hit][order_ref], prec)), err.max()
            assert np.abs(h["t_ns"][order] - rec[hit][order_ref, 3]).max() < (1e-6 if prec == ph.FP64 else 0.1)
            tot = totals.cpu().numpy()
            assert tot[:7].sum() == off[-1] and tot[ph.HIT] == hit.sum()
            # eager work on the stream between replays
            torch.cuda.synchronize()
            _ = (counts.double() * 2.0).sum().item()
    finally:
        plan.close()


def test_batched_full_size_sampled_against_oracle():
    """The batched workload as benchmarked (64 showers, 1e3..1e6 segments
    each, zenith 0..60 deg; FP32 bulk; 16 telescopes R = 6 m; graph replay
    at 256 threads, 16384-photon chunks): counts bit-exact on 2e5 sampled
    segments, and the hit set checked on 1e5 sampled photons that the oracle
    recomputes one by one."""
    a = W.default_atmosphere(absorption=True)
    seg = W.batched_showers(seed=SEED)
    n = len(seg["x0"])
    print(f"batched workload: {n} segments", flush=True)
    em = ph.emission_cherenkov()
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    tel = W.telescopes_16()
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    hits = ph.HitBuffer(1 << 23)
    totals = ph.status_totals()
    plan = ph.Plan(d, atm, em, SEED, ph.FP32, counts, offsets, ph.sink_telescopes(tel, hits, totals),
                   ph.tuning(256, 16384, 0))
    try:
        plan.launch()
        torch.cuda.synchronize()
    finally:
        plan.close()
    gcnt = counts.cpu().numpy().view(np.uint32)
    off = offsets.cpu().numpy().view(np.uint64)
    total = int(off[-1])
    assert total > 1e9
    tot = totals.cpu().numpy()
    assert int(tot[:7].sum()) == total and tot[ph.HORIZON_FLOAT] == 0
    assert hits.count() <= hits.capacity
    assert hits.count() == tot[ph.HIT]
    oatm = O.Atmosphere.from_dict(a)
    rng = np.random.default_rng(1)
    rows = np.sort(rng.choice(n, 200_000, replace=False))
    sub = W.subsample(seg, rows)
    assert np.array_equal(gcnt[rows], O.counts(sub, oatm, "cherenkov", SEED)[0])
    assert np.array_equal(np.diff(off).astype(np.uint32), gcnt)
    h = hits.numpy()
    gkey = (h["segment"].astype(np.int64) << 32) | h["j"].astype(np.int64)
    q = np.sort(rng.choice(total, 100_000, replace=False)).astype(np.uint64)
    s = np.searchsorted(off, q, side="right") - 1
    j = (q - off[s]).astype(np.uint32)
    ref = O.photons(seg, oatm, "cherenkov", SEED, s, j)
    tid, rec = O.telescopes(ref, tel, oatm.index(a["h_obs"]))
    skey = (s.astype(np.int64) << 32) | j.astype(np.int64)
    in_gpu = np.isin(skey, gkey)
    mismatch = in_gpu != (tid >= 0)
    for i in np.nonzero(mismatch)[0]:   # only rays that graze a sphere may differ
        r = np.array([ref["xl"][i], ref["yl"][i], ref["zl"][i]])
        u = ref["ul"][i]
        dmin = min(abs(np.linalg.norm(np.cross(tel[k, :3] - r, u)) - tel[k, 3]) for k in range(len(tel)))
        assert dmin < 1e-3, (i, dmin)
    assert (tid >= 0).sum() >= 50
    pos = {k: i for i, k in enumerate(gkey.tolist())}
    both = np.nonzero(in_gpu & (tid >= 0))[0]
    idx = np.array([pos[k] for k in skey[both]])
    hp = np.stack([h["x"][idx], h["y"][idx], h["z"][idx]], 1)
    err = np.linalg.norm(hp - rec[both, :3], axis=1)
    assert np.all(err <= hit_tolerance(ref[both], rec[both], ph.FP32)), err.max()
    assert np.abs(h["t_ns"][idx] - rec[both, 3]).max() < 0.1
    assert np.array_equal(h["telescope"][idx], tid[both])
