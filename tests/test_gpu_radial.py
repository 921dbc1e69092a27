"""GPU parity of the radial profile sink (section 3.1: photon density and
mean arrival time in rings about the shower core).

Bars: a photon goes to the oracle's bin unless its oracle landing radius
lies within the path's landing tolerance of a bin edge, where either
neighbouring bin is valid. So each GPU bin lies between the oracle's sum over
its unambiguous photons and that sum plus the ambiguous photons that may
fall in it: counts exactly, weights within the fixed-point rounding (2^-33
per photon) and the weight tolerance. Mean times agree within 2^-9 ns plus
the time tolerance plus the most the ambiguous photons can move the mean. Integer sums make the
accumulators independent of the launch shape: bit-exact across tunings.
"""
import numpy as np
import pytest
import torch

import oracle.oracle as O
from paper_2309_15861_amd import photon as ph
from paper_2309_15861_amd import workloads as W

pytestmark = pytest.mark.gpu

SEED = 2
LAND_TOL = {ph.FP64: 1e-9, ph.FP32: 1e-5}
T_TOL = {ph.FP64: 1e-6, ph.FP32: 0.1}
W_TOL = {ph.FP64: 1e-12, ph.FP32: 2e-6}


def _oracle_sums(ref, core, edges, prec, t_ref):
    """Oracle sums per bin over the photons whose bin is certain, and the
    ambiguous photons: those within the landing tolerance of their nearest
    edge m, which may be in bin m - 1 or m (candidate bins, weight, t - t_ref)."""
    n = len(edges) - 1
    b = O.radial_bins(ref, core, edges)
    landed = ref["status"] == O.LANDED
    r = np.hypot(ref["xl"] - core[0], ref["yl"] - core[1])
    scale = np.maximum(np.hypot(ref["xl"] - ref["xe"], ref["yl"] - ref["ye"]), 1.0)
    tol = LAND_TOL[prec] * scale + 1e-12 * np.maximum(r, 1.0)
    m = np.clip(np.searchsorted(edges, r), 0, n)
    below = np.maximum(m - 1, 0)
    m = np.where((m > 0) & (np.abs(r - edges[below]) < np.abs(edges[m] - r)), below, m)
    amb = landed & (np.abs(r - edges[m]) <= tol)
    w = ref["weight"]
    tau = ref["tl"] - t_ref
    sure = (b >= 0) & ~amb
    return dict(cnt=np.bincount(b[sure], minlength=n)[:n].astype(np.int64),
                w=np.bincount(b[sure], weights=w[sure], minlength=n)[:n],
                wt=np.bincount(b[sure], weights=(w * tau)[sure], minlength=n)[:n],
                amb_k=np.stack([m[amb] - 1, m[amb]], axis=1), amb_w=w[amb], amb_tau=tau[amb])


def _merge(a, b):
    out = {k: a[k] + b[k] for k in ("cnt", "w", "wt")}
    for k in ("amb_k", "amb_w", "amb_tau"):
        out[k] = np.concatenate([a[k], b[k]])
    return out


def _check(prof, sums, prec, t_ref):
    """Each GPU bin against the oracle's certain photons plus any subset of
    the ambiguous ones that may fall in it."""
    n = prof.n_bins
    c = prof.count.cpu().numpy()
    wg = prof.weight.cpu().numpy().astype(np.float64) * 2.0**-32
    tg = prof.wt.cpu().numpy().astype(np.float64) * 2.0**-8
    cnt_hi, w_hi = sums["cnt"].copy(), sums["w"].copy()
    msure = np.divide(sums["wt"], sums["w"], out=np.zeros(n), where=sums["w"] > 0)
    dev = np.zeros(n)
    for col in (0, 1):
        k = sums["amb_k"][:, col]
        sel = (k >= 0) & (k < n)
        cnt_hi += np.bincount(k[sel], minlength=n)[:n]
        w_hi += np.bincount(k[sel], weights=sums["amb_w"][sel], minlength=n)[:n]
        dev += np.bincount(k[sel], weights=sums["amb_w"][sel] * np.abs(sums["amb_tau"][sel] - msure[k[sel]]),
                           minlength=n)[:n]
    assert np.all(c >= sums["cnt"]) and np.all(c <= cnt_hi)
    slack = c * 2.0**-33 + W_TOL[prec] * w_hi + 1e-300
    assert np.all(wg >= sums["w"] - slack) and np.all(wg <= w_hi + slack)
    ok = (c > 0) & (sums["w"] > 0)
    assert ok.sum() > 10
    # the mean over the certain photons plus ambiguous ones moves by at most dev / w
    bound = 2.0**-9 + T_TOL[prec] + 1e-9 * np.abs(t_ref + msure[ok]) + dev[ok] / sums["w"][ok]
    assert np.all(np.abs(tg[ok] / wg[ok] - msure[ok]) <= bound)
    d, mt = ph.radial_profile(prof)
    torch.cuda.synchronize()
    e = prof.edges()
    area = np.pi * (e[1:] ** 2 - e[:-1] ** 2)
    # r1^2 - r0^2 of thin far bins cancels: edges built in another order differ by ~r/dr ulps
    assert np.allclose(d.cpu().numpy(), wg / area, rtol=1e-12, atol=0)
    mtc = mt.cpu().numpy()
    assert np.all(np.isnan(mtc[c == 0]))
    assert np.allclose(mtc[c > 0], t_ref + tg[c > 0] / wg[c > 0], rtol=1e-14, atol=0)


@pytest.fixture(scope="module")
def run():
    a = W.default_atmosphere(absorption=True)
    seg = W.subsample(W.shower_cherenkov(), np.arange(0, 200_000, 20))
    em = ph.emission_cherenkov()
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    counts, offsets = ph.count(d, atm, em, SEED)
    torch.cuda.synchronize()
    off = offsets.cpu().numpy().view(np.uint64)
    ref = O.photons_all(seg, O.Atmosphere.from_dict(a), "cherenkov", SEED, off)
    t_ref = float(np.median(ref["tl"][ref["status"] == O.LANDED]))
    return a, seg, d, atm, em, offsets, int(off[-1]), ref, t_ref


@pytest.mark.parametrize("prec", [ph.FP64, ph.FP32])
@pytest.mark.parametrize("log_bins", [False, True])
def test_fused_profile_matches_oracle(run, prec, log_bins):
    a, seg, d, atm, em, offsets, total, ref, t_ref = run
    core = (1.5, -2.5)
    prof = ph.RadialProfile(80, 2.0 if log_bins else 0.0, 700.0, log_bins=log_bins, core=core, t_ref_ns=t_ref)
    totals = ph.status_totals()
    ph.run_fused(d, atm, em, SEED, prec, offsets, -1, ph.sink_radial(prof, totals))
    torch.cuda.synchronize()
    tot = totals.cpu().numpy()
    assert tot[:7].sum() == total
    assert int(prof.count.sum().item()) == tot[ph.LANDED]
    _check(prof, _oracle_sums(ref, core, prof.edges(), prec, t_ref), prec, t_ref)


def test_unfused_profile_matches_oracle(run):
    a, seg, d, atm, em, offsets, total, ref, t_ref = run
    core = (0.0, 0.0)
    prof = ph.RadialProfile(50, 1.0, 1000.0, log_bins=True, core=core, t_ref_ns=t_ref)
    blk = ph.PhotonBlock(total, ph.FP64)
    blk.n_photons = total
    ph.generate(d, atm, em, SEED, ph.FP64, offsets, blk)
    ph.propagate(blk, atm)
    ph.collect(blk, atm, ph.sink_radial(prof))
    torch.cuda.synchronize()
    _check(prof, _oracle_sums(ref, core, prof.edges(), ph.FP64, t_ref), ph.FP64, t_ref)


def test_accumulators_do_not_depend_on_launch_shape(run):
    a, seg, d, atm, em, offsets, total, ref, t_ref = run
    out = []
    for tun in (ph.tuning(256, 4096, 0), ph.tuning(512, 8192, 1), ph.tuning(128, 512, 2)):
        prof = ph.RadialProfile(200, 1.0, 2000.0, log_bins=True, t_ref_ns=t_ref)
        ph.run_fused(d, atm, em, SEED, ph.FP32, offsets, total, ph.sink_radial(prof), tun)
        torch.cuda.synchronize()
        out.append(np.stack([prof.count.cpu().numpy(), prof.weight.cpu().numpy(), prof.wt.cpu().numpy()]))
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_graph_step_clears_and_repeats(run):
    """The captured step clears the accumulators: replays give the same bins."""
    a, seg, d, atm, em, offsets, total, ref, t_ref = run
    prof = ph.RadialProfile(100, 0.0, 500.0, t_ref_ns=t_ref)
    counts = torch.empty(d.n, dtype=torch.int32, device="cuda")
    offs = torch.empty(d.n + 1, dtype=torch.int64, device="cuda")
    plan = ph.Plan(d, atm, em, SEED, ph.FP32, counts, offs, ph.sink_radial(prof), ph.tuning(256, 4096, 0))
    res = []
    for _ in range(3):
        plan.launch()
        torch.cuda.synchronize()
        res.append(np.stack([prof.count.cpu().numpy(), prof.weight.cpu().numpy(), prof.wt.cpu().numpy()]))
        prof.count.fill_(7)  # eager work between replays
        torch.cuda.synchronize()
    plan.close()
    assert np.array_equal(res[0], res[1]) and np.array_equal(res[0], res[2])
    assert res[0][0].sum() > 0


def test_full_size_shower_profile():
    """The benchmarked shower (2.4e7 photons), fused FP32: the profile
    against the oracle over every photon, in batches of segments."""
    a = W.default_atmosphere(absorption=True)
    seg = W.shower_cherenkov()
    em = ph.emission_cherenkov()
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    counts, offsets = ph.count(d, atm, em, SEED)
    prof = ph.RadialProfile(100, 1.0, 3000.0, log_bins=True, t_ref_ns=30000.0)
    totals = ph.status_totals()
    ph.run_fused(d, atm, em, SEED, ph.FP32, offsets, -1, ph.sink_radial(prof, totals), ph.tuning(512, 8192, 0))
    torch.cuda.synchronize()
    off = offsets.cpu().numpy().view(np.uint64)
    oatm = O.Atmosphere.from_dict(a)
    acc = None
    n = len(seg["x0"])
    for s0 in range(0, n, 20000):
        idx = np.arange(s0, min(n, s0 + 20000))
        sub = W.subsample(seg, idx)
        o = (off[s0:idx[-1] + 2] - off[s0]).astype(np.uint64)
        ref = O.photons_all(sub, oatm, "cherenkov", SEED, o)
        part = _oracle_sums(ref, (0.0, 0.0), prof.edges(), ph.FP32, 30000.0)
        acc = part if acc is None else _merge(acc, part)
    assert int(prof.count.sum().item()) == int(totals.cpu().numpy()[ph.LANDED])
    _check(prof, acc, ph.FP32, 30000.0)
