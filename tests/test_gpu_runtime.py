"""GPU tests of the runtime around the fused kernel: HIP-graph plans and the
launch-shape autotuner."""
import numpy as np
import pytest
import torch

from paper_2309_15861_amd import photon as ph
from paper_2309_15861_amd import workloads as W

pytestmark = pytest.mark.gpu


def hit_keys(hits):
    h = hits.numpy()
    return np.sort((h["segment"].astype(np.int64) << 32) | h["j"].astype(np.int64))


@pytest.fixture(scope="module")
def batched():
    a = W.default_atmosphere(absorption=True)
    seg = W.batched_showers(seed=4, n_showers=12, n_min=100, n_max=3000)
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    em = ph.emission_cherenkov()
    counts, offsets = ph.count(d, atm, em, 4)
    torch.cuda.synchronize()
    return a, seg, d, atm, em, counts, offsets, int(offsets[-1].item())


@pytest.mark.parametrize("prec", [ph.FP32, ph.FP64])
def test_plan_replays_match_direct_run(batched, prec):
    a, seg, d, atm, em, counts, offsets, total = batched
    tel = W.telescopes_16(radius=20.0)
    # direct run
    hits0 = ph.HitBuffer(total)
    tot0 = ph.status_totals()
    ph.run_fused(d, atm, em, 4, prec, offsets, total, ph.sink_telescopes(tel, hits0, tot0))
    torch.cuda.synchronize()
    ref_keys, ref_tot = hit_keys(hits0), tot0.cpu().numpy()
    assert ref_tot.sum() == total and len(ref_keys) > 0
    # captured step: counts, offsets, cleared outputs and the fused kernel
    c2 = torch.full_like(counts, -1)
    o2 = torch.full_like(offsets, -1)
    hits = ph.HitBuffer(total)
    tot = ph.status_totals()
    plan = ph.Plan(d, atm, em, 4, prec, c2, o2, ph.sink_telescopes(tel, hits, tot))
    scratch = torch.zeros(1 << 20, device="cuda")
    for r in range(4):
        # eager work and a dirty output between replays
        scratch.add_(1.0)
        hits.t["count"].fill_(12345)
        tot.fill_(7)
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        assert torch.equal(c2, counts), r
        assert torch.equal(o2, offsets), r
        assert np.array_equal(tot.cpu().numpy(), ref_tot), r
        assert np.array_equal(hit_keys(hits), ref_keys), r
    plan.close()


def test_plan_with_grid_sink(batched):
    a, seg, d, atm, em, counts, offsets, total = batched
    g = W.grid_64()
    n = g["nx"] * g["ny"]
    gc0 = torch.zeros(n, dtype=torch.int32, device="cuda")
    gw0 = torch.zeros(n, dtype=torch.int64, device="cuda")
    ph.run_fused(d, atm, em, 4, ph.FP32, offsets, total,
                 ph.sink_grid(g["x_min"], g["y_min"], g["cell"], g["nx"], g["ny"], gc0, gw0))
    gc = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    gw = torch.full((n,), 99, dtype=torch.int64, device="cuda")
    c2 = torch.empty_like(counts)
    o2 = torch.empty_like(offsets)
    plan = ph.Plan(d, atm, em, 4, ph.FP32, c2, o2,
                   ph.sink_grid(g["x_min"], g["y_min"], g["cell"], g["nx"], g["ny"], gc, gw))
    for _ in range(3):
        plan.launch()
        torch.cuda.synchronize()
        assert torch.equal(gc, gc0) and torch.equal(gw, gw0)
    assert int(gc0.sum().item()) > 0
    plan.close()


def test_autotune_picks_a_candidate_with_identical_results(batched):
    a, seg, d, atm, em, counts, offsets, total = batched
    tel = W.telescopes_16(radius=20.0)
    hits = ph.HitBuffer(total)
    sink = ph.sink_telescopes(tel, hits)
    cands = [(128, 1024, 0), (256, 4096, 0), (256, 16384, 0), (512, 8192, 1)]
    best, ms = ph.autotune(d, atm, em, 4, ph.FP32, offsets, sink, cands, reps=3)
    assert (best.block, best.chunk, best.blocks_per_cu) in cands
    assert ms > 0
    keys = []
    for tun in (None, best):
        hits.clear()
        ph.run_fused(d, atm, em, 4, ph.FP32, offsets, total, sink, tun)
        torch.cuda.synchronize()
        keys.append(hit_keys(hits))
    assert np.array_equal(keys[0], keys[1])


def test_device_total_matches_explicit_total(batched):
    """n_photons = -1 (total read on the device) equals passing the total,
    and a too-large explicit count marks the extra slots INVALID."""
    a, seg, d, atm, em, counts, offsets, total = batched
    res = []
    for n_ph in (total, -1, total + 1000):
        tot = ph.status_totals()
        ph.run_fused(d, atm, em, 4, ph.FP32, offsets, n_ph, ph.sink_status(tot))
        torch.cuda.synchronize()
        res.append(tot.cpu().numpy())
    assert np.array_equal(res[0], res[1])
    extra = res[2] - res[0]
    assert extra[ph.INVALID] == 1000 and extra.sum() == 1000


@pytest.mark.parametrize("prec", [ph.FP32, ph.FP64])
@pytest.mark.parametrize("dilution", [400.0, 8000.0])
def test_chunk_pieces_do_not_change_photons(prec, dilution):
    """Sparse segments (fluorescence at 1/400 of the yield: a few photons
    each): a work chunk spans many more segments than the LDS window holds and
    is processed in pieces. At 1/8000 (most segments empty, fewer photons than
    segments in a chunk) chunks look their segments up in global memory
    instead. Every photon comes out the same for every launch shape, bit for
    bit."""
    a = W.default_atmosphere(absorption=True)
    lam, rel = W.fluorescence_lines()
    seg = W.fluorescence(40_000, seed=5)
    em = ph.emission_fluor(lam, rel, W.FLUOR_YIELD_PER_MEV / dilution)
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    counts, offsets = ph.count(d, atm, em, 5)
    torch.cuda.synchronize()
    total = int(offsets[-1].item())
    per_seg = total / len(seg["x0"])
    assert 16384 / max(per_seg, 1e-9) > 4 * 128  # chunks of 16384 span many windows
    assert (per_seg < 1.0) == (dilution > 1000.0) and total > 1000
    outs = []
    for tun in (ph.tuning(128, 1024, 0), ph.tuning(256, 4096, 0), ph.tuning(512, 16384, 0),
                ph.tuning(256, 16384, 0)):
        plane = ph.PhotonBlock(total, prec)
        plane.n_photons = total
        totals = ph.status_totals()
        ph.run_fused(d, atm, em, 5, prec, offsets, -1, ph.sink_plane(plane, totals), tun)
        torch.cuda.synchronize()
        outs.append((plane.numpy(), totals.cpu().numpy()))
    g0, t0 = outs[0]
    assert t0[:7].sum() == total
    for g, t in outs[1:]:
        assert np.array_equal(t, t0)
        for f in g0:
            assert np.array_equal(g[f], g0[f], equal_nan=np.issubdtype(g0[f].dtype, np.floating)), f


def test_kernel_timing(batched):
    """The library's events around the persistent kernel: positive, below the
    time of the whole fused call (which adds the clearing and the
    near-horizon pass), and absent while switched off or under capture."""
    a, seg, d, atm, em, counts, offsets, total = batched
    sink = ph.sink_status(ph.status_totals())
    ph.kernel_timing(True)
    with pytest.raises(ph.PhotonError):
        ph.fused_kernel_ms()           # nothing timed yet
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ph.run_fused(d, atm, em, 4, ph.FP32, offsets, -1, sink, ph.tuning(256, 4096, 0))
    e1.record(stream)
    k = ph.fused_kernel_ms()
    torch.cuda.synchronize()
    assert 0.0 < k <= e0.elapsed_time(e1)
    # a captured step records no events
    plan = ph.Plan(d, atm, em, 4, ph.FP32, counts, offsets, sink, ph.tuning(256, 4096, 0))
    ph.kernel_timing(True)
    plan.launch()
    torch.cuda.synchronize()
    with pytest.raises(ph.PhotonError):
        ph.fused_kernel_ms()
    plan.close()
    ph.kernel_timing(False)


def _fluor_set():
    a = W.default_atmosphere(absorption=True)
    lam, rel = W.fluorescence_lines()
    seg = W.fluorescence(1500, seed=3)
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    em = ph.emission_fluor(lam, rel, W.FLUOR_YIELD_PER_MEV)
    counts, offsets = ph.count(d, atm, em, 3)
    torch.cuda.synchronize()
    return d, atm, em, counts, offsets, int(offsets[-1].item())


def test_two_plans_on_two_streams(batched):
    """Plans own their work cursor and near-horizon queue: two plans (a
    Cherenkov batch and an isotropic fluorescence set, both FP32, both with
    near-horizon rays for the double pass of the fluorescence one) replayed
    interleaved on two streams without synchronising give exactly the results
    of sequential direct runs."""
    a, seg, d, atm, em, counts, offsets, total = batched
    tel = W.telescopes_16(radius=20.0)
    fd, fatm, fem, fcounts, foffsets, ftotal = _fluor_set()
    ref = []
    for dd, aa, ee, seed, off, tt in ((d, atm, em, 4, offsets, total), (fd, fatm, fem, 3, foffsets, ftotal)):
        h = ph.HitBuffer(tt)
        t = ph.status_totals()
        ph.run_fused(dd, aa, ee, seed, ph.FP32, off, tt, ph.sink_telescopes(tel, h, t))
        torch.cuda.synchronize()
        ref.append((hit_keys(h), t.cpu().numpy()))
    assert ref[1][1][ph.HORIZON_FLOAT] == 0 and ref[1][1][ph.LANDED] > 0
    outs, plans = [], []
    for dd, aa, ee, seed, cc, off, tt in ((d, atm, em, 4, counts, offsets, total),
                                          (fd, fatm, fem, 3, fcounts, foffsets, ftotal)):
        h = ph.HitBuffer(tt)
        t = ph.status_totals()
        c2, o2 = torch.empty_like(cc), torch.empty_like(off)
        plans.append(ph.Plan(dd, aa, ee, seed, ph.FP32, c2, o2, ph.sink_telescopes(tel, h, t)))
        outs.append((h, t))
    s = [torch.cuda.Stream(), torch.cuda.Stream()]
    try:
        torch.cuda.synchronize()
        for rep in range(4):
            for k in (0, 1):
                with torch.cuda.stream(s[k]):
                    plans[k].launch()
            torch.cuda.synchronize()
            for k in (0, 1):
                assert np.array_equal(outs[k][1].cpu().numpy(), ref[k][1]), (rep, k)
                assert np.array_equal(hit_keys(outs[k][0]), ref[k][0]), (rep, k)
    finally:
        for p in plans:
            p.close()


def test_eager_calls_on_two_streams(batched):
    """Eager fused calls on two streams, enqueued back to back, are ordered on
    the device (they share its work cursor): both results are exact."""
    a, seg, d, atm, em, counts, offsets, total = batched
    tel = W.telescopes_16(radius=20.0)
    fd, fatm, fem, fcounts, foffsets, ftotal = _fluor_set()
    runs = ((d, atm, em, 4, offsets, total), (fd, fatm, fem, 3, foffsets, ftotal))
    ref = []
    for dd, aa, ee, seed, off, tt in runs:
        t = ph.status_totals()
        ph.run_fused(dd, aa, ee, seed, ph.FP32, off, tt, ph.sink_status(t))
        torch.cuda.synchronize()
        ref.append(t.cpu().numpy())
    s = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(3):
        tots = [ph.status_totals(), ph.status_totals()]
        torch.cuda.synchronize()
        for k, (dd, aa, ee, seed, off, tt) in enumerate(runs):
            with torch.cuda.stream(s[k]):
                ph.run_fused(dd, aa, ee, seed, ph.FP32, off, tt, ph.sink_status(tots[k]))
        torch.cuda.synchronize()
        for k in (0, 1):
            assert np.array_equal(tots[k].cpu().numpy(), ref[k]), (rep, k)
