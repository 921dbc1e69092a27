#!/usr/bin/env python3
"""Photons propagated per second on one MI355X: FP32-split vs FP64, batched.

Headline workload: 64 showers in one persistent launch (segment counts
log-uniform 1e3..1e6 per shower, zenith 0..60 deg, electron segments 5..30 km
with directions within 5 deg of the shower axis, energies log-uniform
50 MeV..1 GeV; 1.38e7 segments, 2.3e9 photons), five-layer exponential
atmosphere with wavelength-dependent absorption, 16 telescope spheres
(R = 6 m, 100 m grid) at 2.2 km. One step = the whole hot path on resident
inputs, replayed from a captured graph: per-segment counts and offsets,
clearing of the outputs, the fused persistent kernel (generation,
propagation, telescope collection) and the near-horizon double pass. The
launch shape comes from the library's autotuner. The headline value is the
FP32-split form (float generation and bending, double time and path); the
plain FP64 form of the same step is timed beside it.

Also reported: the shower workload (2e5 segments) in both forms, the plain
FP64 Cherenkov workload through the materialised photon block (count,
generate, propagate: HBM-bound), the fluorescence workload on its 64 x 64
ground grid in both forms, the angular cut, the correction-table
propagation, radial profiles, fluorescence beaming and the differentiable
form. Every timed form carries its largest error against the FP64 oracle on
a sample of its photons. The oracle itself is timed on the host's cores
(all of them and one) on a sample of the headline workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_SLOTS = 256 * 4 * 16 * 2.4e9          # VALU lane-slots/s: CUs x SIMDs x lanes x clock
PEAK_HBM = 8.0e12                          # B/s
PEAK_LDS_BYTES = 256 * 128 * 2.4e9         # B/s of LDS: CUs x 128 B per clock x clock
# Algorithmic VALU issue slots per photon (quarter-rate operations count 4):
# Philox4x32-10 (10 rounds of two 32x32->64 multiplies and two 3-way xors,
# ~100-120), uniforms (~8), cone/rotation/translation/wavelength (~30),
# propagation over ~2 layer pieces (~90), absorption (~15), telescope
# selection and hit test (~30). The double form is priced at 750 (its
# transcendentals are instruction sequences).
SLOTS_PER_PHOTON = {"fp32": 300.0, "fp64": 750.0}
# Algorithmic HBM bytes per photon of the materialised FP64 path: the
# generator writes x, y, ux, uy, uz, lambda, w, z, t, path (f64), segment, j
# (u32) and status (i32) = 92 B; propagation reads 84 B (all but segment and
# j) and writes 76 B (all but segment, j and lambda). The propagated block is
# the observation-plane output in slot order.
BLOCK_BYTES = {"gen": 92.0, "propagate": 160.0}
# The differentiable form's algorithmic slots: the forward adds, per photon
# landing within reach of the grid, 81 cells x (the Gaussian factor's
# multiply, the fixed-point conversion, the LDS add) = 243; the adjoint
# regenerates and propagates each photon and sweeps its layer pieces back
# (twice the forward's per-photon slots) and, per photon in reach, reads
# 81 cells of dL/dD with the weight and both position derivatives
# (5 slots each) = 405.
SPLAT_SLOTS = {"forward": 243.0, "adjoint": 405.0}
COUNTERS = os.path.join(ROOT, "profiles", "counters.json")
# launch shapes the autotuner chooses from: (block, chunk, blocks per CU; 0 = as many as fit)
TUNING_CANDIDATES = [(256, 3072, 0), (256, 4096, 0), (256, 8192, 0), (256, 16384, 0), (512, 8192, 0),
                     (512, 16384, 0), (128, 4096, 0), (256, 8192, 2)]
SHOWER_FP32_TUNING = (256, 3072, 0)   # fastest on the shower workload in repeated sweeps


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("photon.hip", "photon_device.hpp", "photon_adjoint.hpp"):
        with open(os.path.join(ROOT, "paper_2309_15861_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counters(key):
    """Counter figures of one kernel and workload from the committed
    rocprofv3 runs, if they were taken on the current kernel source."""
    try:
        with open(COUNTERS) as fh:
            d = json.load(fh)
    except OSError:
        return None
    if d.get("source_hash") != source_hash():
        return None
    return d.get("kernels", {}).get(key)


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(model=model or platform.processor(), nproc=os.cpu_count(),
                affinity=len(os.sched_getaffinity(0)), omp_num_threads=os.environ.get("OMP_NUM_THREADS"))


def host_threads():
    """Threads the host share allows: the CPUs this process may run on,
    limited by OMP_NUM_THREADS when it is set."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


# ------------------------------------------------------------------ timing --
def time_steps(fn, steps, warmup):
    """ms per call of fn (which enqueues on the current stream), HIP events
    around `steps` calls after `warmup` untimed ones."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def kernel_times(d, atm, em, seed, prec, offsets, sink, tun, reps):
    """Mean time of the persistent kernel alone and of the near-horizon
    double pass after it (the library's HIP events on the kernel's stream)."""
    from paper_2309_15861_amd import photon as ph
    ph.kernel_timing(True)
    k, dfr = [], []
    for _ in range(reps):
        ph.run_fused(d, atm, em, seed, prec, offsets, -1, sink, tun)
        k.append(ph.fused_kernel_ms())
        dfr.append(ph.fused_deferred_ms())
    ph.kernel_timing(False)
    return float(np.mean(k)), float(np.mean(dfr))


def alu_roofline(kernel, key, form, photons, kernel_ms, deferred_ms, tun):
    """Roofline object of a fused kernel: algorithmic lane-slots per photon
    over the kernel's mean launch time, against the VALU issue peak; the
    measured VALU instruction rate and HBM bytes from the committed counters
    when they match the current source."""
    achieved = SLOTS_PER_PHOTON[form] * photons / (kernel_ms * 1e-3)
    r = dict(bound="alu", achieved=achieved / 1e12, peak=PEAK_SLOTS / 1e12, unit="Tslot/s",
             frac=achieved / PEAK_SLOTS, traffic=None, kernel=kernel, slots_per_photon=SLOTS_PER_PHOTON[form],
             photons_per_launch=photons, kernel_ms=kernel_ms, deferred_pass_ms=deferred_ms,
             tuning=[tun.block, tun.chunk, tun.blocks_per_cu])
    c = counters(key)
    if c:
        r["traffic"] = c["fetch_bytes"] + c["write_bytes"]
        # from the committed rocprofv3 runs of this kernel and workload: executed
        # instructions per photon, rocprofv3's VALUBusy and VALUUtilization
        # (gfx950 can issue two VALU instructions per SIMD quad-cycle, so the
        # busy figure can pass 100), FLOP rates against 157.3 (FP32, packed)
        # and 78.6 TFLOP/s (FP64), and the traced mean kernel time
        r["measured"] = dict(valu_lane_instr_per_photon=c["valu_per_photon"],
                             salu_per_photon=c["salu_per_photon"], lds_per_photon=c.get("lds_per_photon"),
                             valu_busy_pct=c.get("valu_busy_pct"), valu_util_pct=c.get("valu_util_pct"),
                             fp32_tflops=c.get("fp32_tflops"), fp64_tflops=c.get("fp64_tflops"),
                             profiled_kernel_ms=c["avg_ns"] * 1e-6,
                             hbm_bytes_per_photon=(c["fetch_bytes"] + c["write_bytes"]) / photons)
    return r


# ------------------------------------------------------- errors vs oracle --
def photon_errors(g, ref, ok=None):
    """Largest errors of GPU photons g against the oracle's ref, over photons
    both call landed: landing |dr| / max(|r_land - r_emit|, 1 m), arrival
    time (ns), relative weight, direction (rad)."""
    import oracle.oracle as O
    landed = (ref["status"] == O.LANDED) & (g["status"] == O.LANDED)
    if ok is not None:
        landed &= ok
    if not landed.any():
        return dict(landed=0)
    r = ref[landed]
    scale = np.maximum(np.hypot(r["xl"] - r["xe"], r["yl"] - r["ye"]), 1.0)
    gx = g["x"][landed].astype(np.float64)
    gy = g["y"][landed].astype(np.float64)
    u = np.stack([g["ux"][landed], g["uy"][landed], g["uz"][landed]], 1).astype(np.float64)
    ang = np.arctan2(np.linalg.norm(np.cross(u, r["ul"]), axis=1), (u * r["ul"]).sum(1))
    return dict(landed=int(landed.sum()),
                landing_rel=float((np.hypot(gx - r["xl"], gy - r["yl"]) / scale).max()),
                landing_m=float(np.hypot(gx - r["xl"], gy - r["yl"]).max()),
                time_ns=float(np.abs(g["t_ns"][landed] - r["tl"]).max()),
                weight_rel=float((np.abs(g["weight"][landed].astype(np.float64) - r["weight"]) / r["weight"]).max()),
                direction_rad=float(ang.max()))


def sampled_errors(seg, a, kind, em, seed, prec, rows, tun=None, lines=None, atm=None):
    """The fused kernel's photons of the segments `rows` (ids kept, so they
    are the photons of the full run) through the plane sink, against the
    oracle's: counts and statuses compared exactly, the rest by photon_errors."""
    import torch

    import oracle.oracle as O
    from paper_2309_15861_amd import photon as ph
    from paper_2309_15861_amd import workloads as W
    sub = W.subsample(seg, rows)
    d = ph.DeviceSegments(sub)
    atm = atm if atm is not None else ph.atmosphere(a)
    counts, offsets = ph.count(d, atm, em, seed)
    oatm = O.Atmosphere.from_dict(a)
    ocnt = O.counts(sub, oatm, kind, seed)[0]
    gcnt = counts.cpu().numpy().view(np.uint32)
    total = int(offsets[-1].item())
    plane = ph.PhotonBlock(total, prec)
    plane.n_photons = total
    ph.run_fused(d, atm, em, seed, prec, offsets, -1, ph.sink_plane(plane), tun)
    torch.cuda.synchronize()
    g = plane.numpy()
    kw = {} if lines is None else dict(lines_nm=lines[0], line_rel=lines[1])
    ref = O.photons_all(sub, oatm, kind, seed, O.offsets_of(ocnt), **kw)
    out = dict(segments=len(rows), photons=total, counts_equal=bool(np.array_equal(gcnt, ocnt)),
               status_equal=bool(len(g["status"]) == len(ref) and np.array_equal(g["status"], ref["status"])))
    out.update(photon_errors(g, ref))
    return out


def every_kth(n, target, per_segment):
    """Every k-th row so that about `target` photons are sampled."""
    k = max(1, int(n * per_segment / max(target, 1)))
    return np.arange(0, n, k)


# --------------------------------------------------------------- workloads --
def fused_form(name, seg, a, kind, em, seed, prec, sink_fn, args, tun=None, mode=16):
    """One workload in one precision: autotuned launch shape (unless given),
    the whole step captured in a graph and timed, the persistent kernel
    timed alone at the same shape, the sink's results. mode: the fused
    kernel instance's template mode (16: Cherenkov into telescopes, 40:
    fluorescence into the grid)."""
    import torch

    from paper_2309_15861_amd import photon as ph
    d = ph.DeviceSegments(seg)
    atm = ph.atmosphere(a)
    counts, offsets = ph.count(d, atm, em, seed)
    torch.cuda.synchronize()
    total = int(offsets[-1].item())
    sink, outs = sink_fn(total)
    if tun is None:
        tun, _ = ph.autotune(d, atm, em, seed, prec, offsets, sink, TUNING_CANDIDATES, reps=3)
    plan = ph.Plan(d, atm, em, seed, prec, counts, offsets, sink, tun)
    try:
        ms = time_steps(plan.launch, args.steps, args.warmup)
    finally:
        plan.close()
    res = dict(photons=total, ms_per_step=ms, photons_per_s=total / (ms * 1e-3),
               tuning=[tun.block, tun.chunk, tun.blocks_per_cu])
    res.update(outs())
    kms, dms = kernel_times(d, atm, em, seed, prec, offsets, sink, tun, max(3, args.steps // 4))
    form = "fp64" if prec == ph.FP64 else "fp32"
    kern = f"k_fused<{'double' if prec == ph.FP64 else 'float'}, {tun.block}, {mode}>"
    res["roofline"] = alu_roofline(kern, f"{kern} {name}", form, total, kms, dms, tun)
    return res, d, atm, counts, offsets, tun


def telescope_sink(tel, capacity_hint=None):
    from paper_2309_15861_amd import photon as ph

    def make(total):
        # capacity from the photon total (hits are a few per cent of the photons)
        hits = ph.HitBuffer(capacity_hint or max(total // 16, 1 << 16))
        totals = ph.status_totals()

        def outs():
            tot = totals.cpu().numpy()
            return dict(hits=hits.count(), hit_capacity=hits.capacity, hits_dropped=max(0, hits.count() - hits.capacity),
                        status_totals=[int(x) for x in tot])
        return ph.sink_telescopes(tel, hits, totals), outs
    return make


def grid_sink(g):
    import torch

    from paper_2309_15861_amd import photon as ph

    def make(total):
        gc = torch.zeros(g["nx"] * g["ny"], dtype=torch.int32, device="cuda")
        gw = torch.zeros(g["nx"] * g["ny"], dtype=torch.int64, device="cuda")
        totals = ph.status_totals()

        def outs():
            tot = totals.cpu().numpy()
            return dict(on_grid=int(gc.sum().item()), grid_weight=float(gw.double().sum().item()) / 2**32,
                        status_totals=[int(x) for x in tot])
        return ph.sink_grid(g["x_min"], g["y_min"], g["cell"], g["nx"], g["ny"], gc, gw, totals), outs
    return make


def batched(args, forms):
    """The headline workload in the requested forms, with sampled errors."""
    from paper_2309_15861_amd import photon as ph
    from paper_2309_15861_amd import workloads as W
    seg = W.batched_showers(seed=4)
    a = W.default_atmosphere(absorption=True)
    em = ph.emission_cherenkov(300.0, 600.0)
    tel = W.telescopes_16()
    out = dict(workload="64 showers in one persistent launch, segments log-uniform 1e3..1e6 per shower, zenith "
                        "0..60 deg, Cherenkov 300-600 nm, absorption, 16 telescopes R=6 m on a 100 m grid",
               segments=len(seg["x0"]))
    for name, prec, tun in forms:
        r, *_ = fused_form("batched", seg, a, "cherenkov", em, 4, prec, telescope_sink(tel, 1 << 23), args, tun)
        if not args.no_errors:
            rows = every_kth(len(seg["x0"]), 2e5, r["photons"] / len(seg["x0"]))
            r["error_vs_oracle"] = sampled_errors(seg, a, "cherenkov", em, 4, prec, rows,
                                                  ph.tuning(*r["tuning"]))
        out[name] = r
    return out


def shower(args):
    """The shower workload (2e5 segments) in both forms."""
    from paper_2309_15861_amd import photon as ph
    from paper_2309_15861_amd import workloads as W
    seg = W.shower_cherenkov()
    a = W.default_atmosphere(absorption=True)
    em = ph.emission_cherenkov(300.0, 600.0)
    tel = W.telescopes_16()
    out = dict(workload="shower-shaped Cherenkov: 2e5 segments, 1 TeV gamma profile, zenith 20 deg, 16 telescopes "
                        "R=6 m on a 100 m grid, absorption, 300-600 nm", segments=len(seg["x0"]))
    extra = None
    for name, prec, tun in (("fp32", ph.FP32, ph.tuning(*SHOWER_FP32_TUNING)), ("fp64", ph.FP64, None)):
        r, d, atm, counts, offsets, tun = fused_form("shower", seg, a, "cherenkov", em, 2, prec,
                                                     telescope_sink(tel), args, tun)
        if not args.no_errors:
            rows = every_kth(len(seg["x0"]), 2e5, r["photons"] / len(seg["x0"]))
            r["error_vs_oracle"] = sampled_errors(seg, a, "cherenkov", em, 2, prec, rows, tun)
        out[name] = r
        if name == "fp32":
            extra = (seg, a, d, atm, tel, tun, r)
    return out, extra


def plain_block(args, which=("plain", "shower_scale")):
    """The plain FP64 Cherenkov workload (1,000 segments) through the
    materialised photon block: counts and offsets, generation into the
    block, propagation in place (the propagated block is the observation
    plane in slot order). The same path on the shower workload shows the
    HBM-bound regime: algorithmic bytes per photon over the kernel times."""
    import torch

    import oracle.oracle as O
    from paper_2309_15861_amd import photon as ph
    from paper_2309_15861_amd import workloads as W
    a = W.default_atmosphere(absorption=False)
    out = {}
    cases = {"plain": (W.plain_cherenkov, 1, False), "shower_scale": (W.shower_cherenkov, 2, True)}
    for name in which:
        make, seed, absorb = cases[name]
        seg = make()
        a = W.default_atmosphere(absorption=absorb)
        d = ph.DeviceSegments(seg)
        atm = ph.atmosphere(a)
        em = ph.emission_cherenkov(300.0, 600.0)
        counts, offsets = ph.count(d, atm, em, seed)
        torch.cuda.synchronize()
        total = int(offsets[-1].item())
        blk = ph.PhotonBlock(total, ph.FP64)
        blk.n_photons = total
        c2, o2 = torch.empty_like(counts), torch.empty_like(offsets)

        def step():
            # the boundary's calls: counts and offsets, the photon block, propagation in place
            ph.gen_cherenkov(d, atm, 300.0, 600.0, seed, ph.FP64, c2, o2)
            ph.gen_cherenkov(d, atm, 300.0, 600.0, seed, ph.FP64, c2, o2, blk)
            ph.propagate(blk, atm)
        ms = time_steps(step, args.steps, args.warmup)
        # the two photon kernels alone (each entry point is one kernel on the current stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        g_ms, p_ms = [], []
        for _ in range(max(3, args.steps // 2)):
            ev[0].record()
            ph.generate(d, atm, em, seed, ph.FP64, offsets, blk)
            ev[1].record()
            ph.propagate(blk, atm)
            ev[2].record()
            torch.cuda.synchronize()
            g_ms.append(ev[0].elapsed_time(ev[1]))
            p_ms.append(ev[1].elapsed_time(ev[2]))
        gms, pms = float(np.mean(g_ms)), float(np.mean(p_ms))
        bytes_ = (BLOCK_BYTES["gen"] + BLOCK_BYTES["propagate"]) * total
        r = dict(segments=len(seg["x0"]), photons=total, ms_per_step=ms, photons_per_s=total / (ms * 1e-3),
                 gen_ms=gms, propagate_ms=pms,
                 roofline=dict(bound="hbm", achieved=bytes_ / ((gms + pms) * 1e-3) / 1e9, peak=PEAK_HBM / 1e9,
                               unit="GB/s", frac=bytes_ / ((gms + pms) * 1e-3) / PEAK_HBM,
                               bytes_per_photon=BLOCK_BYTES["gen"] + BLOCK_BYTES["propagate"],
                               kernels="k_gen<double> + k_propagate<double, false>", traffic=None))
        cg, cp = counters(f"k_gen<double> {name}"), counters(f"k_propagate<double, false> {name}")
        if cg and cp:
            r["roofline"]["traffic"] = cg["fetch_bytes"] + cg["write_bytes"] + cp["fetch_bytes"] + cp["write_bytes"]
        if not args.no_errors:
            g = blk.numpy()
            oatm = O.Atmosphere.from_dict(a)
            off = offsets.cpu().numpy().astype(np.int64)
            rows = np.arange(len(seg["x0"])) if name == "plain" else every_kth(len(seg["x0"]), 2e5, total / len(seg["x0"]))
            sub = W.subsample(seg, rows)
            ocnt = O.counts(sub, oatm, "cherenkov", seed)[0]
            gcnt = np.diff(off)[rows].astype(np.uint32)
            ref = O.photons_all(sub, oatm, "cherenkov", seed, O.offsets_of(ocnt))
            slots = np.concatenate([np.arange(off[s], off[s + 1], dtype=np.int64) for s in rows])
            gs = {k: v[slots] for k, v in g.items()}
            e = dict(segments=len(rows), photons=len(slots), counts_equal=bool(np.array_equal(gcnt, ocnt)),
                     status_equal=bool(np.array_equal(gs["status"], ref["status"])))
            e.update(photon_errors(gs, ref))
            r["error_vs_oracle"] = e
        out[name] = r
        del blk
        torch.cuda.empty_cache()
    out["workload"] = ("plain FP64 Cherenkov: 1000 segments 5..30 km within 5 deg of vertical, 50 MeV..1 GeV, "
                       "plane at 2.2 km, no absorption; and the same materialised path on the 2e5-segment shower")
    return out


def fluorescence_grid(args):
    """The fluorescence workload (1e5 segments, 1e8 photons) on the 64 x 64
    ground grid of 10 m cells, FP32 and FP64."""
    from paper_2309_15861_amd import photon as ph
    from paper_2309_15861_amd import workloads as W
    seg = W.fluorescence()
    a = W.default_atmosphere(absorption=True)
    lam, rel = W.fluorescence_lines()
    em = ph.emission_fluor(lam, rel, W.FLUOR_YIELD_PER_MEV)
    g = W.grid_64()
    out = dict(workload="fluorescence: 1e5 segments 5..30 km, dE/dx 1..10 MeV/m, 10 photons/MeV, 21 lines, "
                        "isotropic; 64 x 64 grid of 10 m cells at 2.2 km", segments=len(seg["x0"]))
    for name, prec in (("fp32", ph.FP32), ("fp64", ph.FP64)):
        r, *_ = fused_form("fluorescence", seg, a, "fluor", em, 3, prec, grid_sink(g), args, mode=40)
        if not args.no_errors:
            rows = every_kth(len(seg["x0"]), 1e6, r["photons"] / len(seg["x0"]))
            r["error_vs_oracle"] = sampled_errors(seg, a, "fluor", em, 3, prec, rows, ph.tuning(*r["tuning"]),
                                                  lines=(lam, rel))
        out[name] = r
    return out


def angular_cut(args, d, atm, tel, seed, best, uncut):
    """The shower step with the Cherenkov angular particle cut at 6 degrees,
    to the array centre and to each telescope: emitting segments, photons and
    hits kept, and the step time against the uncut step (same launch shape)."""
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
        try:
            ms = time_steps(plan.launch, args.steps, args.warmup)
        finally:
            plan.close()
        photons = int(offsets[-1].item())
        assert int(totals.cpu().numpy()[:7].sum()) == photons
        nh = hits.count()
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
        try:
            ms = time_steps(plan.launch, args.steps, args.warmup)
        finally:
            plan.close()
        photons = int(offsets[-1].item())
        tot = totals.cpu().numpy()
        assert int(tot[:7].sum()) == photons
        out[name] = dict(photons=photons, hits=int(tot[ph.HIT]), ms_per_step=ms, photons_per_s=photons / (ms * 1e-3))
    out["photons_kept_frac"] = out["beamed"]["photons"] / out["isotropic"]["photons"]
    out["speedup"] = out["isotropic"]["ms_per_step"] / out["beamed"]["ms_per_step"]
    return out


def radial_profile(args, d, atm, seed, best):
    """The shower step collected as the radial profiles of section 3.1
    (100 bins uniform in ln r from 1 m to 3 km about the core): step time and
    a few points of the photon density and mean arrival time."""
    import torch

    from paper_2309_15861_amd import photon as ph
    em = ph.emission_cherenkov(300.0, 600.0)
    prof = ph.RadialProfile(100, 1.0, 3000.0, log_bins=True, t_ref_ns=0.0)
    counts = torch.empty(d.n, dtype=torch.int32, device="cuda")
    offsets = torch.empty(d.n + 1, dtype=torch.int64, device="cuda")
    totals = ph.status_totals()
    plan = ph.Plan(d, atm, em, seed, ph.FP32, counts, offsets, ph.sink_radial(prof, totals), best)
    try:
        ms = time_steps(plan.launch, args.steps, args.warmup)
    finally:
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


def table_propagation(args, seg, a, d, atm, tel, seed, best, exact_ms):
    """The shower step with the straight-line propagation and tabulated
    refraction corrections of section 2 (257 x 257 nodes up to 40 km and
    80 degrees, FP32): step time against the exact closed forms, and the
    method's error against the exact FP64 oracle on sampled photons."""
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
    try:
        ms = time_steps(plan.launch, args.steps, args.warmup)
    finally:
        plan.close()
    photons = int(offsets[-1].item())
    out = dict(table="257 x 257 nodes, h_obs..40 km, tan(zenith) 0..tan(80 deg); 4097 vertical nodes",
               photons=photons, hits=hits.count(), ms_per_step=ms, photons_per_s=photons / (ms * 1e-3),
               speedup_vs_exact=exact_ms / ms)
    if not args.no_errors:
        rows = every_kth(len(seg["x0"]), 2e5, photons / len(seg["x0"]))
        out["error_vs_exact_oracle"] = sampled_errors(seg, a, "cherenkov", em, seed, ph.FP32, rows, best,
                                                      atm=atm_t)
    return out


def differentiable(args):
    """The differentiable form at 1e6 segments: splatted ground density
    (128 x 128 cells of 5 m, sigma 5 m) with counts frozen at the nominal
    parameters, and its adjoint for L = sum (D - T)^2 with T the density at
    perturbed parameters; FP32 bulk, FP64 beside it; the FP32 results'
    relative difference from the FP64 ones."""
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
    kept = {}
    for name, prec in (("fp32", ph.FP32), ("fp64", ph.FP64)):
        p = ph.SplatProblem(d, a, 5, prec, g)
        atm0 = ph.atmosphere(a)
        T = ph.splat_forward(d, p.atmosphere(H1, e1), 300.0, 600.0, 5, prec, p.offsets, p.mean0, p.grid, dirs=dirs1)
        totals = ph.status_totals()
        D = ph.splat_forward(d, atm0, 300.0, 600.0, 5, prec, p.offsets, p.mean0, p.grid, totals=totals)
        in_reach = int(totals[ph.LANDED].item())
        G = (2.0 * (D - T)).contiguous()
        grads = ph.splat_backward(d, atm0, 300.0, 600.0, 5, prec, p.offsets, p.mean0, p.grid, G)
        torch.cuda.synchronize()
        fwd = time_steps(lambda: ph.splat_forward(d, atm0, 300.0, 600.0, 5, prec, p.offsets, p.mean0, p.grid),
                         steps, 1)
        bwd = time_steps(lambda: ph.splat_backward(d, atm0, 300.0, 600.0, 5, prec, p.offsets, p.mean0, p.grid, G),
                         steps, 1)
        total = int(p.offsets[-1].item())
        out["segments"] = d.n
        out["photons"] = total
        base = SLOTS_PER_PHOTON[name]
        fw_slots = base * total + SPLAT_SLOTS["forward"] * in_reach
        bw_slots = 2.0 * base * total + SPLAT_SLOTS["adjoint"] * in_reach
        out[name] = dict(forward_ms=fwd, backward_ms=bwd, forward_photons_per_s=total / (fwd * 1e-3),
                         backward_photons_per_s=total / (bwd * 1e-3), steps=steps, photons_in_reach=in_reach,
                         forward_roofline=dict(bound="alu", achieved=fw_slots / (fwd * 1e-3) / 1e12,
                                               peak=PEAK_SLOTS / 1e12, unit="Tslot/s",
                                               frac=fw_slots / (fwd * 1e-3) / PEAK_SLOTS,
                                               slots=f"{base:g}/photon + {SPLAT_SLOTS['forward']:g}/photon in reach"),
                         backward_roofline=dict(bound="alu", achieved=bw_slots / (bwd * 1e-3) / 1e12,
                                                peak=PEAK_SLOTS / 1e12, unit="Tslot/s",
                                                frac=bw_slots / (bwd * 1e-3) / PEAK_SLOTS,
                                                slots=f"{2 * base:g}/photon + {SPLAT_SLOTS['adjoint']:g}/photon in reach"),
                         loss=float(((D - T).double() ** 2).sum()),
                         grad_scale_height=[float(v) for v in grads[0].cpu()], grad_n0_minus_1=float(grads[1]))
        kept[name] = (D.double().cpu().numpy(), [x.double().cpu().numpy() for x in grads])
    D32, g32 = kept["fp32"]
    D64, g64 = kept["fp64"]
    gdir32 = np.stack(g32[2:5], 1)
    gdir64 = np.stack(g64[2:5], 1)
    out["fp32_vs_fp64"] = dict(
        density_max_abs_over_max=float(np.abs(D32 - D64).max() / np.abs(D64).max()),
        grad_scale_height_rel=float(np.abs(g32[0] - g64[0]).max() / np.abs(g64[0]).max()),
        grad_n0_minus_1_rel=float(abs(g32[1] - g64[1]) / abs(g64[1])),
        grad_direction_rel_norm=float(np.linalg.norm(gdir32 - gdir64) / np.linalg.norm(gdir64)))
    return out


def peaks(args):
    """Measured device rates (library micro-benchmarks, best of three
    launches) beside the nominal ones the rooflines use: FP32 and FP64 FMA
    lanes, the 32x32->64 integer multiply-add of Philox, FP32 exp2, FMA and
    exp2 interleaved, HBM reads of a 2 GiB buffer, and the splat's LDS
    integer adds (32-bit returning, 64-bit)."""
    import torch

    from paper_2309_15861_amd import photon as ph
    nominal = {"fp32_fma": PEAK_SLOTS, "fp64_fma": PEAK_SLOTS, "int_mad64": PEAK_SLOTS / 4,
               "fp32_exp2": PEAK_SLOTS / 4, "fp32_fma_exp2": PEAK_SLOTS, "hbm_read": PEAK_HBM,
               "lds_add32_rtn": PEAK_LDS_BYTES / 4, "lds_add64": PEAK_LDS_BYTES / 8}
    out = {}
    small = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    big = torch.ones(1 << 29, dtype=torch.float32, device="cuda")   # 2 GiB
    for k, name in enumerate(ph.PEAK_KINDS):
        work = big if name == "hbm_read" else small
        best = None
        for _ in range(3):
            ops, ms = ph.peak_run(k, work, 2048)
            rate = ops / (ms * 1e-3)
            best = rate if best is None or rate > best else best
        unit = "B/s" if name == "hbm_read" else "lane-op/s"
        out[name] = dict(measured=best, nominal=nominal[name], unit=unit, frac_of_nominal=best / nominal[name])
    del big
    torch.cuda.empty_cache()
    out["note"] = ("nominal: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz for full-rate VALU operations, a quarter of it "
                   "for 32x32->64 multiplies and transcendentals, 8 TB/s HBM, 128 B per clock per CU of LDS for "
                   "the LDS adds; the FMA+exp2 mix can exceed one instruction per lane-cycle because the "
                   "transcendental unit issues beside the VALU")
    return out


def cpu_baseline(seconds_all=12.0, seconds_one=8.0):
    """The FP64 oracle on the host, on the headline workload: counts,
    photon generation and quadrature propagation and the telescope test,
    segment batches of every 53rd segment taken in order until the time
    budget is spent; on all the threads the host share allows and on one."""
    import oracle.oracle as O
    from paper_2309_15861_amd import workloads as W
    seg = W.batched_showers(seed=4)
    a = W.default_atmosphere(absorption=True)
    tel = W.telescopes_16()
    oatm = O.Atmosphere.from_dict(a)
    n_obs = oatm.index(a["h_obs"])
    rows_all = np.arange(0, len(seg["x0"]), 53)
    res = {}
    for label, threads, budget in (("all", host_threads(), seconds_all), ("one", 1, seconds_one)):
        O.set_threads(threads)
        photons = segs = 0
        t0 = time.perf_counter()
        for b0 in range(0, len(rows_all), 4000):
            sub = W.subsample(seg, rows_all[b0:b0 + 4000])
            cnt = O.counts(sub, oatm, "cherenkov", 4)[0]
            off = O.offsets_of(cnt)
            phs = O.photons_all(sub, oatm, "cherenkov", 4, off)
            O.telescopes(phs, tel, n_obs)
            photons += int(off[-1])
            segs += len(cnt)
            if time.perf_counter() - t0 > budget:
                break
        dt = time.perf_counter() - t0
        res[label] = dict(photons_per_s=photons / dt, threads=O.num_threads(), photons=photons, segments=segs,
                          seconds=dt)
    info = cpu_info()
    return dict(value=res["all"]["photons_per_s"], unit="photons/s", cores=res["all"]["threads"], kind="oracle",
                sample=(f"64-shower workload, every 53rd segment in batches of 4000 until the time budget: "
                        f"{res['all']['segments']} segments ({res['all']['photons']} photons) on "
                        f"{res['all']['threads']} threads in {res['all']['seconds']:.1f} s; counts + generation + "
                        f"quadrature propagation + telescope test"),
                single_thread=res["one"], cpu=info)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-errors", action="store_true", help="skip the sampled errors against the oracle")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device-to-device copy (HBM counter calibration)")
    ap.add_argument("--only", default=None,
                    help="comma-separated sections to run (profiling runs): batched32, batched64, shower, plain, "
                         "blockshower, grid, cut, table, radial, beam, adjoint, peaks")
    ap.add_argument("--tuning", default=None,
                    help="block,chunk,blocks_per_cu of the headline FP32 step instead of the autotuner's choice")
    ap.add_argument("--tuning64", default=None,
                    help="block,chunk,blocks_per_cu of the headline FP64 step instead of the autotuner's choice")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the photon path would shard by whole showers or by photon-prefix ranges, "
              "with one all-reduce of the small grids); use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2309_15861_amd import photon as ph

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(64 * 2**20, dtype=torch.float64, device="cuda")   # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 8, "launches": 3}))
        return
    sections = set(args.only.split(",")) if args.only else {
        "batched32", "batched64", "shower", "plain", "blockshower", "grid", "cut", "table", "radial", "beam", "adjoint",
        "peaks"}
    tun32 = ph.tuning(*(int(v) for v in args.tuning.split(","))) if args.tuning else None
    tun64 = ph.tuning(*(int(v) for v in args.tuning64.split(","))) if args.tuning64 else None
    forms = [f for f in (("fp32", ph.FP32, tun32), ("fp64", ph.FP64, tun64))
             if ("batched32" if f[0] == "fp32" else "batched64") in sections]
    out = {}
    b = batched(args, forms) if forms else None
    head = b["fp32"] if b and "fp32" in b else None
    out = {
        "metric": "photons propagated/s on 1 MI355X (FP64 vs FP32-split, batched) + % roofline",
        "value": head["photons_per_s"] if head else None, "unit": "photons/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"] if head else None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": b["workload"] if b else None, "segments": b["segments"] if b else None,
                   "photons": head["photons"] if head else None,
                   "precision": "fp32 bulk, fp64 time/path and near-horizon rays",
                   "step": "counts + offsets + clear + fused kernel + near-horizon double pass, graph replay"},
        "roofline": head["roofline"] if head else None,
    }
    if b:
        out["batched"] = b
        if "fp64" in b:
            out["fp64"] = dict(value=b["fp64"]["photons_per_s"], ms_per_step=b["fp64"]["ms_per_step"],
                               frac=b["fp64"]["roofline"]["frac"],
                               speedup_fp32_over_fp64=(b["fp64"]["ms_per_step"] / head["ms_per_step"]) if head else None)
        if head and "error_vs_oracle" in head:
            out["error_vs_oracle"] = head["error_vs_oracle"]
    extra = None
    if "shower" in sections or sections & {"cut", "table", "radial"}:
        out["shower"], extra = shower(args)
    which = tuple(k for k, sec in (("plain", "plain"), ("shower_scale", "blockshower")) if sec in sections)
    if which:
        out["plain_fp64_block"] = plain_block(args, which)
    if "grid" in sections:
        out["fluorescence_grid"] = fluorescence_grid(args)
    if extra:
        seg, a, d, atm, tel, tun, r32 = extra
        if "cut" in sections:
            out["angular_cut"] = angular_cut(args, d, atm, tel, 2, tun,
                                             dict(photons=r32["photons"], hits=r32["hits"],
                                                  ms_per_step=r32["ms_per_step"]))
        if "table" in sections:
            out["table_propagation"] = table_propagation(args, seg, a, d, atm, tel, 2, tun, r32["ms_per_step"])
        if "radial" in sections:
            out["radial_profile"] = radial_profile(args, d, atm, 2, tun)
    if "beam" in sections:
        out["fluorescence_beaming"] = fluorescence_beaming(args, ph.tuning(*SHOWER_FP32_TUNING))
    if "adjoint" in sections:
        out["differentiable"] = differentiable(args)
    if "peaks" in sections:
        out["peaks"] = peaks(args)
    if not args.no_cpu_baseline and not args.only:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
