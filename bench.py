#!/usr/bin/env python3
"""Photons propagated per second on one MI355X.

Workload: shower-shaped Cherenkov input (2e5 electron segments following a
1 TeV gamma longitudinal profile, E^-2 energies from 20 MeV, lateral
sigma 50 m, zenith 20 deg), five-layer exponential atmosphere with
wavelength-dependent absorption, 16 telescope spheres (R = 6 m, 100 m grid)
at 2.2 km. One step = the whole hot path on resident inputs: per-segment
counts and offsets, clearing the outputs, and the fused persistent kernel
(generation, propagation, telescope collection). The headline value is the
FP32-bulk form (float generation and bending, double time and path); the
plain FP64 form is timed beside it. The FP64 CPU oracle is timed on the
host's cores over the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_SLOTS = 256 * 4 * 16 * 2.4e9          # VALU lane-slots/s: CUs x SIMDs x lanes x clock
# Algorithmic VALU issue slots per photon (quarter-rate operations count 4):
# Philox4x32-10 (10 rounds of two 32x32->64 multiplies and two 3-way xors,
# ~100-120), uniforms (~8), cone/rotation/translation/wavelength (~30),
# propagation over ~2 layer pieces (~90), absorption (~15), telescope
# selection and hit test (~30).
SLOTS_PER_PHOTON = {"fp32": 300.0, "fp64": 750.0}
PMC_FILE = os.path.join(ROOT, "profiles", "fused_shower_fp32_traffic.json")
# launch shapes the autotuner chooses from: (block, chunk, blocks per CU; 0 = as many as fit)
FP32_TUNING = "256,3072,0"
TUNING_CANDIDATES = [(256, 3072, 0), (256, 4096, 0), (256, 8192, 0), (256, 16384, 0), (512, 8192, 0),
                     (512, 16384, 0), (128, 4096, 0), (256, 8192, 2)]


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("photon.hip", "photon_device.hpp", "photon_adjoint.hpp"):
        with open(os.path.join(ROOT, "paper_2309_15861_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per fused launch from the committed rocprofv3 counter runs,
    if they were taken on the current kernel source."""
    try:
        with open(PMC_FILE) as fh:
            d = json.load(fh)
    except OSError:
        return None
    if d.get("source_hash") != source_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(seg, atm_dict, tel, seed, max_threads=16):
    """The FP64 oracle on the host: counts, photon generation + propagation
    and telescope test for every segment, in batches of 20000 segments."""
    import numpy as np

    import oracle.oracle as O
    from paper_2309_15861_amd import workloads as W

    threads = max(1, min(max_threads, len(os.sched_getaffinity(0))))
    O.set_threads(threads)
    oatm = O.Atmosphere.from_dict(atm_dict)
    n_obs = oatm.index(atm_dict["h_obs"])
    n = len(seg["x0"])
    photons = 0
    t0 = time.perf_counter()
    for b0 in range(0, n, 20000):
        sub = W.subsample(seg, np.arange(b0, min(n, b0 + 20000)))
        cnt = O.counts(sub, oatm, "cherenkov", seed)[0]
        off = O.offsets_of(cnt)
        ph = O.photons_all(sub, oatm, "cherenkov", seed, off)
        O.telescopes(ph, tel, n_obs)
        photons += int(off[-1])
    dt = time.perf_counter() - t0
    return dict(value=photons / dt, unit="photons/s", cores=O.num_threads(), kind="oracle",
                sample=f"all {n} segments ({photons} photons) in batches of 20000 segments; "
                       f"counts + generation + quadrature propagation + telescope test; {dt:.1f} s")


def batched_showers(args):
    """64 showers (segment counts log-uniform 1e3..1e6, zenith 0..60 deg) in
    one graph-captured step, FP32 bulk, telescope sink per shower core."""
    import torch

    from paper_2309_15861_amd import photon as ph
    from paper_2309_15861_amd import workloads as W

    seg = W.batched_showers(seed=4)
    a = W.default_atmosphere(absorption=True)
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    em = ph.emission_cherenkov(300.0, 600.0)
    counts = torch.empty(d.n, dtype=torch.int32, device="cuda")
    offsets = torch.empty(d.n + 1, dtype=torch.int64, device="cuda")
    ph.gen_cherenkov(d, atm, 300.0, 600.0, 4, ph.FP64, counts, offsets)
    torch.cuda.synchronize()
    total = int(offsets[-1].item())
    hits = ph.HitBuffer(1 << 22)       # hits beyond the capacity are still counted in the totals
    totals = ph.status_totals()
    sink = ph.sink_telescopes(W.telescopes_16(), hits, totals)
    best, _ = ph.autotune(d, atm, em, 4, ph.FP32, offsets, sink, TUNING_CANDIDATES, reps=2)
    plan = ph.Plan(d, atm, em, 4, ph.FP32, counts, offsets, sink, best)
    plan.launch()
    torch.cuda.synchronize()
    steps = max(2, args.steps // 4)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        plan.launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    tot = totals.cpu().numpy()
    assert int(tot[:7].sum()) == total
    plan.close()
    return dict(workload="64 showers, segments log-uniform 1e3..1e6 per shower, zenith 0..60 deg",
                segments=d.n, photons=total, hits=int(tot[ph.HIT]), ms_per_step=ms,
                photons_per_s=total / (ms * 1e-3),
                precision="fp32 bulk, fp64 time/path", steps=steps,
                tuning=[best.block, best.chunk, best.blocks_per_cu])


def angular_cut(args, d, atm, tel, seed, best, uncut):
    """The shower step with the Cherenkov angular particle cut at 6 degrees,
    to the array centre and to each telescope: emitting segments, photons and
    hits kept, and the step time against the uncut step (same launch shape)."""
    import numpy as np
    import torch

    from paper_2309_15861_amd import photon as ph
    from paper_2309_15861_amd import workloads as W

    em0 = ph.emission_cherenkov(300.0, 600.0)
    emitting0 = int((ph.means(d, atm, em0) > 0).sum().item())
    out = dict(cut_deg=6.0, uncut=dict(emitting_segments=emitting0, photons=uncut["photons"],
                                       hits=uncut["hits"], ms_per_step=uncut["ms_per_step"]))
    for name, pts in (("centre", np.array([[0.0, 0.0, W.H_OBS]])), ("telescopes", tel[:, :3])):
        em = ph.emission_cherenkov(300.0, 600.0, cut_points=pts, cut_angle_deg=6.0)
        emitting = int((ph.means(d, atm, em) > 0).sum().item())
        counts = torch.empty(d.n, dtype=torch.int32, device="cuda")
        offsets = torch.empty(d.n + 1, dtype=torch.int64, device="cuda")
        hits = ph.HitBuffer(max(uncut["photons"] // 8, 1024))
        totals = ph.status_totals()
        plan = ph.Plan(d, atm, em, seed, ph.FP32, counts, offsets, ph.sink_telescopes(tel, hits, totals), best)
        for _ in range(args.warmup):
            plan.launch()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            plan.launch()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        photons = int(offsets[-1].item())
        assert int(totals.cpu().numpy()[:7].sum()) == photons
        nh = hits.count()
        plan.close()
        out[name] = dict(emitting_segments=emitting, segments_kept_frac=emitting / max(emitting0, 1),
                         photons=photons, photons_kept_frac=photons / uncut["photons"], hits=nh,
                         hits_kept_frac=nh / max(uncut["hits"], 1), ms_per_step=ms,
                         speedup=uncut["ms_per_step"] / ms)
    return out


def fluorescence_beaming(args, best):
    """The fluorescence step (1e5 segments, 21 lines, 16 telescopes R = 6 m)
    with isotropic and with beamed emission (a cone per segment around a
    sphere enclosing the array, 1 degree margin): photons, hits and step time."""
    import torch

    from paper_2309_15861_amd import photon as ph
    from paper_2309_15861_amd import workloads as W

    seg = W.fluorescence()
    a = W.default_atmosphere(absorption=True)
    tel = W.telescopes_16()
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    lam, rel = W.fluorescence_lines()
    out = dict(workload="1e5 fluorescence segments 5..30 km, dE/dx 1..10 MeV/m, 21 lines, 10 photons/MeV; "
                        "16 telescopes R=6 m", margin_deg=1.0)
    for name, area in (("isotropic", None), ("beamed", ph.enclosing_sphere(tel))):
        em = ph.emission_fluor(lam, rel, W.FLUOR_YIELD_PER_MEV, beam_area=area, beam_margin_deg=1.0)
        counts = torch.empty(d.n, dtype=torch.int32, device="cuda")
        offsets = torch.empty(d.n + 1, dtype=torch.int64, device="cuda")
        hits = ph.HitBuffer(1 << 16)
        totals = ph.status_totals()
        plan = ph.Plan(d, atm, em, 3, ph.FP32, counts, offsets, ph.sink_telescopes(tel, hits, totals), best)
        for _ in range(args.warmup):
            plan.launch()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            plan.launch()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        photons = int(offsets[-1].item())
        tot = totals.cpu().numpy()
        assert int(tot[:7].sum()) == photons
        plan.close()
        out[name] = dict(photons=photons, hits=int(tot[ph.HIT]), ms_per_step=ms,
                         photons_per_s=photons / (ms * 1e-3))
    out["photons_kept_frac"] = out["beamed"]["photons"] / out["isotropic"]["photons"]
    out["speedup"] = out["isotropic"]["ms_per_step"] / out["beamed"]["ms_per_step"]
    return out


def radial_profile(args, d, atm, seed, best):
    """The shower step collected as the radial profiles of section 3.1
    (100 bins uniform in ln r from 1 m to 3 km about the core): step time and
    a few points of the photon density and mean arrival time."""
    import numpy as np
    import torch

    from paper_2309_15861_amd import photon as ph
    from paper_2309_15861_amd import workloads as W

    em = ph.emission_cherenkov(300.0, 600.0)
    prof = ph.RadialProfile(100, 1.0, 3000.0, log_bins=True, t_ref_ns=0.0)
    counts = torch.empty(d.n, dtype=torch.int32, device="cuda")
    offsets = torch.empty(d.n + 1, dtype=torch.int64, device="cuda")
    totals = ph.status_totals()
    plan = ph.Plan(d, atm, em, seed, ph.FP32, counts, offsets, ph.sink_radial(prof, totals), best)
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    plan.close()
    photons = int(offsets[-1].item())
    dens, mt = (x.cpu().numpy() for x in ph.radial_profile(prof))
    cnt = prof.count.cpu().numpy()
    e = prof.edges()
    mid = np.sqrt(e[:-1] * e[1:])
    points = {}
    for r in (30.0, 100.0, 150.0, 300.0, 1000.0):
        k = int(np.searchsorted(e, r) - 1)
        points[f"{r:g} m"] = dict(density_per_m2=float(dens[k]), mean_t_ns=float(mt[k]), photons=int(cnt[k]))
    return dict(bins="100, uniform in ln r, 1 m..3 km", photons=photons, binned=int(cnt.sum()), ms_per_step=ms,
                photons_per_s=photons / (ms * 1e-3), at_r=points,
                peak_density_r_m=float(mid[int(np.argmax(dens))]))


def table_propagation(args, d, atm, tel, seed, best, exact_ms):
    """The shower step with the straight-line propagation and tabulated
    refraction corrections of section 2 (257 x 257 nodes up to 40 km and
    80 degrees, FP32): step time against the exact closed forms."""
    import torch

    from paper_2309_15861_amd import photon as ph

    tab = ph.PropagationTable(atm)
    atm_t = tab.attach(atm)
    em = ph.emission_cherenkov(300.0, 600.0)
    counts = torch.empty(d.n, dtype=torch.int32, device="cuda")
    offsets = torch.empty(d.n + 1, dtype=torch.int64, device="cuda")
    hits = ph.HitBuffer(1 << 20)
    totals = ph.status_totals()
    plan = ph.Plan(d, atm_t, em, seed, ph.FP32, counts, offsets, ph.sink_telescopes(tel, hits, totals), best)
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    photons = int(offsets[-1].item())
    plan.close()
    return dict(table="257 x 257 nodes, h_obs..40 km, tan(zenith) 0..tan(80 deg); 4097 vertical nodes",
                photons=photons, hits=hits.count(), ms_per_step=ms, photons_per_s=photons / (ms * 1e-3),
                speedup_vs_exact=exact_ms / ms)


def differentiable(args):
    """The differentiable form at 1e6 segments: splatted ground density
    (128 x 128 cells of 5 m, sigma 5 m) with counts frozen at the nominal
    parameters, and its adjoint for L = sum (D - T)^2 with T the density at
    perturbed parameters; FP32 bulk, FP64 beside it."""
    import torch

    from paper_2309_15861_amd import photon as ph
    from paper_2309_15861_amd import workloads as W

    seg = W.differentiable()
    a = W.default_atmosphere(absorption=True)
    g = W.splat_grid_128()
    d = ph.DeviceSegments(seg)
    H1, e1, d1 = W.perturbed_parameters(a, seg, 77)
    dirs1 = tuple(torch.as_tensor(np.ascontiguousarray(d1[:, k]), device="cuda") for k in range(3))
    out = dict(workload="1e6 shower segments, splat 128 x 128 cells of 5 m, sigma 5 m, trunc 4 sigma; "
                        "L = sum (D - T)^2, T at perturbed H, n0-1, directions")
    steps = max(2, args.steps // 4)
    for name, prec in (("fp32", ph.FP32), ("fp64", ph.FP64)):
        p = ph.SplatProblem(d, a, 5, prec, g)
        atm0 = ph.atmosphere(a)
        T = ph.splat_forward(d, p.atmosphere(H1, e1), 300.0, 600.0, 5, prec, p.offsets, p.mean0, p.grid, dirs=dirs1)
        D = ph.splat_forward(d, atm0, 300.0, 600.0, 5, prec, p.offsets, p.mean0, p.grid)
        G = (2.0 * (D - T)).contiguous()
        ph.splat_backward(d, atm0, 300.0, 600.0, 5, prec, p.offsets, p.mean0, p.grid, G)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        for _ in range(steps):
            ph.splat_forward(d, atm0, 300.0, 600.0, 5, prec, p.offsets, p.mean0, p.grid)
        ev[1].record()
        for _ in range(steps):
            grads = ph.splat_backward(d, atm0, 300.0, 600.0, 5, prec, p.offsets, p.mean0, p.grid, G)
        ev[2].record()
        torch.cuda.synchronize()
        total = int(p.offsets[-1].item())
        fwd = ev[0].elapsed_time(ev[1]) / steps
        bwd = ev[1].elapsed_time(ev[2]) / steps
        out["segments"] = d.n
        out["photons"] = total
        out[name] = dict(forward_ms=fwd, backward_ms=bwd, forward_photons_per_s=total / (fwd * 1e-3),
                         backward_photons_per_s=total / (bwd * 1e-3), steps=steps,
                         loss=float(((D - T).double() ** 2).sum()),
                         grad_scale_height=[float(v) for v in grads[0].cpu()], grad_n0_minus_1=float(grads[1]))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy (HBM counter calibration)")
    ap.add_argument("--fp32-only", action="store_true", help="time only the FP32 form (profiling runs)")
    ap.add_argument("--batched", action=argparse.BooleanOptionalAction, default=True,
                    help="also time 64 showers of 1e3..1e6 segments in one graph-captured step")
    ap.add_argument("--tuning", default=None,
                    help="block,chunk,blocks_per_cu of the fused kernel for both forms instead of the defaults "
                         "(profiling runs)")
    ap.add_argument("--fp32-tuning", default=FP32_TUNING,
                    help="launch shape of the FP32 form: the fastest on this workload in repeated sweeps of the "
                         "tuning candidates (a single autotuner pass is within its noise); 'auto' to autotune")
    ap.add_argument("--cut", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the shower step with the 6 degree Cherenkov angular particle cut")
    ap.add_argument("--table", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the shower step with the straight-line + correction-table propagation")
    ap.add_argument("--radial", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the shower step collected as radial density and arrival-time profiles")
    ap.add_argument("--beam", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the fluorescence step with isotropic and beamed emission")
    ap.add_argument("--adjoint", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the differentiable form (splat forward and adjoint, 1e6 segments)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the photon path would shard by whole showers or by photon-prefix ranges, "
              "with one all-reduce of the small grids); use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2309_15861_amd import photon as ph
    from paper_2309_15861_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(64 * 2**20, dtype=torch.float64, device="cuda")   # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "launches": 3}))
        return
    seed = 2
    seg = W.shower_cherenkov()
    a = W.default_atmosphere(absorption=True)
    tel = W.telescopes_16()
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    em = ph.emission_cherenkov(300.0, 600.0)
    n = d.n
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    ph.gen_cherenkov(d, atm, 300.0, 600.0, seed, ph.FP64, counts, offsets)
    torch.cuda.synchronize()
    total = int(offsets[-1].item())
    hits = ph.HitBuffer(max(total // 8, 1024))
    totals = ph.status_totals()
    sink = ph.sink_telescopes(tel, hits, totals)
    stream = torch.cuda.current_stream()

    results = {}
    forms = (("fp32", ph.FP32),) if args.fp32_only else (("fp32", ph.FP32), ("fp64", ph.FP64))
    for name, prec in forms:
        # launch shape from the autotuner, then the whole step captured in a graph
        if args.tuning:
            best = ph.tuning(*(int(v) for v in args.tuning.split(",")))
        elif prec == ph.FP32 and args.fp32_tuning != "auto":
            best = ph.tuning(*(int(v) for v in args.fp32_tuning.split(",")))
        else:
            best, _ = ph.autotune(d, atm, em, seed, prec, offsets, sink, TUNING_CANDIDATES, reps=3)
        plan = ph.Plan(d, atm, em, seed, prec, counts, offsets, sink, best)
        for _ in range(args.warmup):
            plan.launch()
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(args.steps):
            plan.launch()
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        tot = totals.cpu().numpy()
        assert int(tot[:7].sum()) == total, (tot, total)
        assert hits.count() <= hits.capacity
        nhits = hits.count()
        plan.close()
        # the persistent kernel alone, same shape: the library's HIP events
        # around its launch on the stream it runs on
        ph.kernel_timing(True)
        kms = []
        for _ in range(args.steps):
            ph.run_fused(d, atm, em, seed, prec, offsets, -1, sink, best)
            kms.append(ph.fused_kernel_ms())
        ph.kernel_timing(False)
        fused_ms = float(np.mean(kms))
        results[name] = dict(ms_per_step=ms / args.steps, fused_ms=fused_ms,
                             photons_per_s=total * args.steps / (ms * 1e-3), hits=nhits,
                             status_totals=[int(x) for x in tot],
                             tuning=[best.block, best.chunk, best.blocks_per_cu])

    r32 = results["fp32"]
    achieved = SLOTS_PER_PHOTON["fp32"] * total / (r32["fused_ms"] * 1e-3)
    roofline = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_SLOTS / 1e12, unit="Tslot/s",
                    frac=achieved / PEAK_SLOTS, traffic=traffic_per_launch(),
                    kernel=f"k_fused<float, {r32['tuning'][0]}, 0>", slots_per_photon=SLOTS_PER_PHOTON["fp32"],
                    fused_ms=r32["fused_ms"], tuning=r32["tuning"])
    r64 = results.get("fp64", r32)
    out = {
        "metric": "photons propagated/s on 1 MI355X (FP64 vs FP32-split, batched) + % roofline",
        "value": r32["photons_per_s"], "unit": "photons/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r32["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "shower-shaped Cherenkov: 2e5 segments, 1 TeV gamma profile, zenith 20 deg, "
                               "16 telescopes R=6 m on a 100 m grid, absorption, 300-600 nm",
                   "segments": n, "photons": total, "precision": "fp32 bulk, fp64 time/path"},
        "roofline": roofline,
        "fp64": {"value": r64["photons_per_s"], "ms_per_step": r64["ms_per_step"], "fused_ms": r64["fused_ms"],
                 "frac": SLOTS_PER_PHOTON["fp64"] * total / (r64["fused_ms"] * 1e-3) / PEAK_SLOTS},
        "hits": r32["hits"],
    }
    if args.cut:
        out["angular_cut"] = angular_cut(args, d, atm, tel, seed, ph.tuning(*r32["tuning"]),
                                         dict(photons=total, hits=r32["hits"], ms_per_step=r32["ms_per_step"]))
    if args.table:
        out["table_propagation"] = table_propagation(args, d, atm, tel, seed, ph.tuning(*r32["tuning"]),
                                                     r32["ms_per_step"])
    if args.radial:
        out["radial_profile"] = radial_profile(args, d, atm, seed, ph.tuning(*r32["tuning"]))
    if args.beam:
        out["fluorescence_beaming"] = fluorescence_beaming(args, ph.tuning(*r32["tuning"]))
    if args.batched:
        out["batched"] = batched_showers(args)
    if args.adjoint:
        out["differentiable"] = differentiable(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(seg, a, tel, seed)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
