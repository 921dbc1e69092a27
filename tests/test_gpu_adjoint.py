"""Parity of the differentiable form on the GPU: splatted density
(photon_splat_forward) against the C oracle, and the adjoint
(photon_splat_backward) against the oracle's complex-step gradient, central
differences of the GPU's own FP64 forward, and at full size on sampled
segments.

The density gradient G handed to the adjoint never comes from the HIP path:
it is 2 (D_oracle - T) or a seeded random field."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle.adjoint import SplatModel
from paper_2309_15861_amd import photon as ph
from paper_2309_15861_amd import workloads as W

pytestmark = pytest.mark.gpu
SEED = 5
BAND = (300.0, 600.0)
# FP64 adjoint against the FP64 reference: relative 1e-8; FP32 bulk: 1e-3 (norm-wise)
TOL_G64, TOL_G32 = 1e-8, 1e-3


def _oracle_density(seg, atm_d, cnt, mu, g):
    return O.splat_density(seg, O.Atmosphere.from_dict(atm_d), cnt, mu, SEED, g, g["sigma"], g["trunc"])


def _perturbed(seg, atm_d):
    H1, e1, d1 = W.perturbed_parameters(atm_d, seg, 77)
    atm1 = dict(atm_d, scale_height=H1, n0_minus_1=e1)
    seg1 = dict(seg, dx=d1[:, 0].copy(), dy=d1[:, 1].copy(), dz=d1[:, 2].copy())
    return atm1, seg1


@pytest.fixture(scope="module")
def case():
    seg = W.subsample(W.differentiable(200_000, 5), np.arange(200))
    atm_d = W.default_atmosphere(absorption=True)
    g = W.splat_grid_128()
    cnt, mu, _ = O.counts(seg, O.Atmosphere.from_dict(atm_d), "cherenkov", SEED)
    atm1, seg1 = _perturbed(seg, atm_d)
    T = _oracle_density(seg1, atm1, cnt, mu, g)
    D0 = _oracle_density(seg, atm_d, cnt, mu, g)
    M = SplatModel(seg, atm_d, SEED, cnt, mu, g, g["sigma"], g["trunc"])
    G = 2.0 * (D0 - T)
    ref = M.vjp(G, atm_d["scale_height"], atm_d["n0_minus_1"], seg["dx"], seg["dy"], seg["dz"])
    d = ph.DeviceSegments(seg)
    return dict(seg=seg, atm_d=atm_d, g=g, cnt=cnt, mu=mu, atm1=atm1, seg1=seg1, T=T, D0=D0, G=G, ref=ref,
                d=d, M=M)


def _problem(c, prec, grid=None, atm_d=None):
    return ph.SplatProblem(c["d"], atm_d or c["atm_d"], SEED, prec, grid or c["g"], *BAND)


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


def fp32_cell_bound(seg, atm_d, cnt, mu, g, land_rel=1e-5, w_rel=1e-6, w_tau=6e-7):
    """Per-cell bound on |D_fp32 - D_oracle| implied by the FP32 photon bars.
    A photon of weight w landing within eps = land_rel max(displacement, 1 m)
    of the oracle's point changes its contribution c = w N exp(-d^2/2 sigma^2)
    to a cell at distance d by at most c (|d| eps + eps^2)/sigma^2 (for
    eps < sigma/4, where the Gaussian's log changes by |d| eps/sigma^2 +
    eps^2/(2 sigma^2), and e^x - 1 <= 2x for x <= 1/2); its weight error adds
    c (w_rel + w_tau tau); a photon within eps of the 4-sigma window's edge
    may add or drop a term of at most w N e^-8 (one coordinate at the edge);
    the float Gaussian factor adds 1e-6 c, and the float form's fixed-point
    sum (units of 2^-24 of weight) 2^-25 per photon and cell."""
    oatm = O.Atmosphere.from_dict(atm_d)
    c64 = np.asarray(cnt, np.int64)
    s_list = np.repeat(np.arange(len(c64)), c64)
    off = np.concatenate([[0], np.cumsum(c64)])
    j_list = np.arange(off[-1]) - off[s_list]
    ref = O.photons(seg, oatm, "cherenkov", SEED, s_list, j_list)
    mu_now = O.counts(seg, oatm, "cherenkov", SEED)[1]
    mu0 = np.asarray(mu)
    ratio = np.where(mu0 > 0, mu_now / np.where(mu0 > 0, mu0, 1.0), 0.0)[s_list]
    land = ref["status"] == O.LANDED
    r = ref[land]
    w = r["weight"] * ratio[land]
    eps = land_rel * np.maximum(np.hypot(r["xl"] - r["xe"], r["yl"] - r["ye"]), 1.0)
    sig, reach = g["sigma"], g["trunc"] * g["sigma"]
    assert np.all(eps < sig / 4)
    N = 1.0 / (2.0 * np.pi * sig * sig)
    gx = g["x_min"] + (np.arange(g["nx"]) + 0.5) * g["cell"]
    gy = g["y_min"] + (np.arange(g["ny"]) + 0.5) * g["cell"]
    B = np.zeros((g["ny"], g["nx"]))
    for q in range(len(r)):
        dx = gx - r["xl"][q]
        dy = gy - r["yl"][q]
        ix = np.nonzero(np.abs(dx) <= reach + eps[q])[0]
        iy = np.nonzero(np.abs(dy) <= reach + eps[q])[0]
        if len(ix) == 0 or len(iy) == 0:
            continue
        DX, DY = np.meshgrid(dx[ix], dy[iy])
        d = np.hypot(DX, DY)
        c = w[q] * N * np.exp(-(d * d) / (2 * sig * sig))
        b = c * ((d * eps[q] + eps[q] ** 2) / (sig * sig) + w_rel + w_tau * r["tau"][q] + 1e-6)
        edge = (np.abs(np.abs(DX) - reach) <= eps[q]) | (np.abs(np.abs(DY) - reach) <= eps[q])
        b = b + edge * w[q] * N * np.exp(-8.0) * 1.01
        B[np.ix_(iy, ix)] += b + N * 2.0**-25
    return B


def test_frozen_counts_and_means_match_oracle(case):
    c = case
    p = _problem(c, ph.FP64)
    assert np.array_equal(p.counts.cpu().numpy().view(np.uint32), c["cnt"])
    assert np.array_equal(p.mean0.cpu().numpy(), c["mu"])


@pytest.mark.parametrize("prec", [ph.FP64, ph.FP32])
def test_density_matches_oracle(case, prec):
    c = case
    p = _problem(c, prec)
    totals = ph.status_totals()
    D = ph.splat_forward(c["d"], ph.atmosphere(c["atm_d"]), *BAND, SEED, prec, p.offsets, p.mean0, p.grid,
                         totals=totals).double().cpu().numpy()
    tot = totals.cpu().numpy().view(np.uint64)
    assert tot.sum() == c["cnt"].sum()
    assert tot[ph.LANDED] > 1000
    D0 = c["D0"]
    if prec == ph.FP64:
        assert np.abs(D - D0).max() <= 1e-10 * np.abs(D0).max()
    else:
        assert _rel(D, D0) <= 1e-4
        # cell by cell, within what the FP32 photon bars allow
        B = fp32_cell_bound(c["seg"], c["atm_d"], c["cnt"], c["mu"], c["g"])
        assert np.all(np.abs(D - D0) <= B), (np.abs(D - D0) / np.maximum(B, 1e-300)).max()


@pytest.mark.parametrize("prec", [ph.FP64, ph.FP32])
def test_density_at_perturbed_parameters(case, prec):
    """Current parameters differ from the nominal ones: weights carry
    mu(theta)/mu(theta0) and the photons move."""
    c = case
    p = _problem(c, prec)
    s1 = c["seg1"]
    dirs = tuple(torch.as_tensor(np.ascontiguousarray(s1[k]), device="cuda") for k in ("dx", "dy", "dz"))
    D = ph.splat_forward(c["d"], ph.atmosphere(c["atm1"]), *BAND, SEED, prec, p.offsets, p.mean0, p.grid,
                         dirs=dirs).double().cpu().numpy()
    T = c["T"]
    if prec == ph.FP64:
        assert np.abs(D - T).max() <= 1e-10 * np.abs(T).max()
    else:
        assert _rel(D, T) <= 1e-4
        B = fp32_cell_bound(s1, c["atm1"], c["cnt"], c["mu"], c["g"])
        assert np.all(np.abs(D - T) <= B), (np.abs(D - T) / np.maximum(B, 1e-300)).max()


def _gpu_vjp(c, prec, G, grid=None, atm_d=None):
    p = _problem(c, prec, grid, atm_d)
    gD = torch.as_tensor(np.ascontiguousarray(G), device="cuda")
    gH, ge, gx, gy, gz = ph.splat_backward(c["d"], ph.atmosphere(atm_d or c["atm_d"]), *BAND, SEED, prec,
                                           p.offsets, p.mean0, p.grid, gD)
    gd = torch.stack([gx, gy, gz], 1).cpu().numpy()
    return gH.cpu().numpy(), float(ge.cpu()), gd


@pytest.mark.parametrize("k", [200.0, 1.0e4])
def test_fp32_fixed_point_carries(case, k):
    """Frozen means divided by k multiply every photon's weight by k. At
    k = 200 (weights below 256) each cell of the float form's 32-bit LDS grid
    takes one conversion, and the cell sums pass 2^32 units: the densest cell
    holds more than 256 weight units per 3072 photons, so any split of the
    photons into chunks of at least that size wraps a cell in some block and
    carries into the global grid. At k = 1e4 single contributions pass 2^32
    units (their high words go to the global grid directly). The float
    density must still match the double one (whose 64-bit cells never wrap)
    to the FP32 bar."""
    c = case
    p32, p64 = _problem(c, ph.FP32), _problem(c, ph.FP64)
    N = 1.0 / (2.0 * np.pi * c["g"]["sigma"] ** 2)
    atm = ph.atmosphere(c["atm_d"])
    D = {}
    for prec, p in ((ph.FP32, p32), (ph.FP64, p64)):
        m0 = (p.mean0 / k).contiguous()
        D[prec] = ph.splat_forward(c["d"], atm, *BAND, SEED, prec, p.offsets, m0, p.grid).double().cpu().numpy()
    photons = int(c["cnt"].sum())
    if k == 200.0:
        assert D[ph.FP64].max() / N > 256.0 * (photons / 3072.0 + 1.0)
    assert np.abs(D[ph.FP64] - k * c["D0"]).max() <= 1e-10 * k * np.abs(c["D0"]).max()
    assert _rel(D[ph.FP32], D[ph.FP64]) <= 1e-4
    assert np.abs(D[ph.FP32] - D[ph.FP64]).max() <= 1e-4 * np.abs(D[ph.FP64]).max()


def test_adjoint_fp64_matches_reference(case):
    c = case
    gH, ge, gd = _gpu_vjp(c, ph.FP64, c["G"])
    rH, re, rd = c["ref"]
    for l in (0, 1, 2):
        assert abs(gH[l] - rH[l]) <= TOL_G64 * abs(rH[l]), (l, gH[l], rH[l])
    assert gH[3] == 0.0 and gH[4] == 0.0 and rH[3] == 0.0 and rH[4] == 0.0
    assert abs(ge - re) <= TOL_G64 * abs(re), (ge, re)
    assert np.count_nonzero(np.abs(rd).max(1)) > 20
    assert _rel(gd, rd) <= TOL_G64
    assert np.abs(gd - rd).max() <= TOL_G64 * np.abs(rd).max()


def test_adjoint_fp32_matches_reference(case):
    c = case
    gH, ge, gd = _gpu_vjp(c, ph.FP32, c["G"].astype(np.float32))
    rH, re, rd = c["ref"]
    assert _rel(gH, rH) <= TOL_G32
    assert abs(ge - re) <= TOL_G32 * abs(re)
    assert _rel(gd, rd) <= TOL_G32


def test_direction_gradient_orthogonal(case):
    c = case
    _, _, gd = _gpu_vjp(c, ph.FP64, c["G"])
    s = c["seg"]
    d = np.stack([s["dx"], s["dy"], s["dz"]], 1)
    assert np.abs(np.sum(gd * d, 1)).max() <= 1e-12 * np.abs(gd).max()


def test_adjoint_matches_central_differences_of_gpu_forward(case):
    """dL/dtheta of L = sum (D - T)^2 against five-point differences of the
    FP64 GPU forward (wide truncation: no jumps at the window edge)."""
    c = case
    g = dict(c["g"], trunc=10.0)
    p = _problem(c, ph.FP64, g)
    T = torch.as_tensor(c["T"], device="cuda")
    a0 = c["atm_d"]
    s = c["seg"]

    def loss(atm_d, dirs=None):
        D = ph.splat_forward(c["d"], ph.atmosphere(atm_d), *BAND, SEED, ph.FP64, p.offsets, p.mean0, p.grid,
                             dirs=dirs)
        return float(((D - T) ** 2).sum())

    D = ph.splat_forward(c["d"], ph.atmosphere(a0), *BAND, SEED, ph.FP64, p.offsets, p.mean0, p.grid)
    gH, ge, gx, gy, gz = ph.splat_backward(c["d"], ph.atmosphere(a0), *BAND, SEED, ph.FP64, p.offsets, p.mean0,
                                           p.grid, 2.0 * (D - T))

    def fd(f, h):
        return (8.0 * (f(h) - f(-h)) - (f(2.0 * h) - f(-2.0 * h))) / (12.0 * h)

    H0 = np.asarray(a0["scale_height"], float)
    for l in (0, 1):
        def f(h, l=l):
            Hh = H0.copy()
            Hh[l] += h
            return loss(dict(a0, scale_height=Hh))
        v = fd(f, 1e-3 * H0[l])
        assert abs(float(gH[l]) - v) <= 1e-5 * abs(v), (l, float(gH[l]), v)
    e0 = a0["n0_minus_1"]
    v = fd(lambda h: loss(dict(a0, n0_minus_1=e0 + h)), 1e-3 * e0)
    assert abs(float(ge) - v) <= 1e-5 * abs(v)
    gd = torch.stack([gx, gy, gz], 1).cpu().numpy()
    row = int(np.argmax(np.abs(gd).max(1)))
    base = [torch.as_tensor(np.ascontiguousarray(s[k]), device="cuda") for k in ("dx", "dy", "dz")]
    for k in range(3):
        def f(h, k=k):
            dirs = [t.clone() for t in base]
            dirs[k][row] += h
            return loss(a0, tuple(dirs))
        v = fd(f, 2e-6)
        assert abs(gd[row, k] - v) <= 1e-5 * np.abs(gd[row]).max(), (k, gd[row, k], v)


@pytest.mark.parametrize("prec", [ph.FP64, ph.FP32])
def test_autograd_function(case, prec):
    """torch.autograd through SplatDensity gives the adjoint of
    L = sum (D - T)^2 at the reference's tolerance."""
    c = case
    p = _problem(c, prec)
    a0 = c["atm_d"]
    s = c["seg"]
    H = torch.tensor(np.asarray(a0["scale_height"], float), requires_grad=True)
    eta = torch.tensor(float(a0["n0_minus_1"]), dtype=torch.float64, requires_grad=True)
    dirs = [torch.tensor(np.ascontiguousarray(s[k]), device="cuda", requires_grad=True) for k in ("dx", "dy", "dz")]
    D = ph.SplatDensity.apply(H, eta, *dirs, p)
    T = torch.as_tensor(c["T"], device="cuda", dtype=D.dtype)
    L = ((D - T) ** 2).sum()
    L.backward()
    rH, re, rd = c["ref"]
    tol = TOL_G64 if prec == ph.FP64 else TOL_G32
    # the reference is the product with 2 (D_oracle - T); the GPU's D differs from it by rounding only
    tol_d = max(tol, 1e-9) if prec == ph.FP64 else tol
    assert _rel(H.grad.numpy(), rH) <= tol_d
    assert abs(float(eta.grad) - re) <= tol_d * abs(re)
    gd = torch.stack([t.grad for t in dirs], 1).cpu().numpy()
    assert _rel(gd, rd) <= tol_d


def test_homogeneous_layer_has_zero_gradient(case):
    c = case
    a = dict(c["atm_d"])
    H = np.asarray(a["scale_height"], float).copy()
    H[1] = np.inf
    a["scale_height"] = H
    cnt, mu, _ = O.counts(c["seg"], O.Atmosphere.from_dict(a), "cherenkov", SEED)
    M = SplatModel(c["seg"], a, SEED, cnt, mu, c["g"], c["g"]["sigma"], c["g"]["trunc"])
    rng = np.random.Generator(np.random.PCG64(11))
    G = rng.normal(size=(c["g"]["ny"], c["g"]["nx"]))
    rH, re, rd = M.vjp(G, H, a["n0_minus_1"], c["seg"]["dx"], c["seg"]["dy"], c["seg"]["dz"])
    gH, ge, gd = _gpu_vjp(c, ph.FP64, G, atm_d=a)
    assert gH[1] == 0.0 and rH[1] == 0.0
    assert abs(gH[0] - rH[0]) <= TOL_G64 * abs(rH[0])
    assert abs(ge - re) <= TOL_G64 * abs(re)
    assert _rel(gd, rd) <= TOL_G64


def test_empty_and_out_of_reach():
    atm = W.default_atmosphere(absorption=True)
    g = W.splat_grid_128()
    seg = W.subsample(W.differentiable(200_000, 5), np.arange(0))
    d = ph.DeviceSegments(seg) if len(seg["x0"]) else None
    # no segments
    s0 = ph.Segments()
    s0.n = 0
    gr = ph.splat_grid(g)
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    D = torch.full((g["ny"], g["nx"]), 7.0, dtype=torch.float64, device="cuda")
    L = ph.lib()
    import ctypes as C
    pa = ph.atmosphere(atm)
    rc = L.photon_splat_forward(C.byref(s0), C.byref(pa), 300.0, 600.0, SEED, ph.FP64, ph._ptr(off), None,
                                C.byref(gr), ph._ptr(D), None, ph._stream())
    assert rc == 0
    assert float(D.abs().max()) == 0.0
    gH = torch.full((5,), 3.0, dtype=torch.float64, device="cuda")
    ge = torch.full((1,), 3.0, dtype=torch.float64, device="cuda")
    rc = L.photon_splat_backward(C.byref(s0), C.byref(pa), 300.0, 600.0, SEED, ph.FP64, ph._ptr(off), None,
                                 C.byref(gr), ph._ptr(D), ph._ptr(gH), ph._ptr(ge), None, None, None, ph._stream())
    assert rc == 0
    assert float(gH.abs().max()) == 0.0 and float(ge.abs().max()) == 0.0
    assert d is None
    # a grid far from every landing point: zero density and zero gradient
    seg = W.subsample(W.differentiable(200_000, 5), np.arange(50))
    d = ph.DeviceSegments(seg)
    far = dict(g, x_min=50_000.0)
    p = ph.SplatProblem(d, atm, SEED, ph.FP64, far, *BAND)
    totals = ph.status_totals()
    D = ph.splat_forward(d, ph.atmosphere(atm), *BAND, SEED, ph.FP64, p.offsets, p.mean0, p.grid, totals=totals)
    assert float(D.abs().max()) == 0.0
    tot = totals.cpu().numpy().view(np.uint64)
    assert tot[ph.LANDED] == 0 and tot[ph.OFFGRID] > 0
    gH, ge, gx, gy, gz = ph.splat_backward(d, ph.atmosphere(atm), *BAND, SEED, ph.FP64, p.offsets, p.mean0, p.grid,
                                           torch.ones_like(D))
    assert float(gH.abs().max()) == 0.0 and float(ge) == 0.0
    assert float(torch.stack([gx, gy, gz]).abs().max()) == 0.0


@pytest.fixture(scope="module")
def full():
    seg = W.differentiable()
    d = ph.DeviceSegments(seg)
    return seg, d


@pytest.mark.parametrize("prec", [ph.FP64, ph.FP32])
def test_full_size_sampled_segments(full, prec):
    """1e6 segments (the gradient workload) with a seeded random density
    gradient: the direction gradients of sampled segments against the
    oracle, which needs only those segments' photons; orthogonality of every
    direction gradient and zero gradients of the layers above 40 km."""
    seg, d = full
    atm = W.default_atmosphere(absorption=True)
    g = W.splat_grid_128()
    p = ph.SplatProblem(d, atm, SEED, prec, g, *BAND)
    rng = np.random.Generator(np.random.PCG64(12))
    G = rng.normal(size=(g["ny"], g["nx"]))
    gD = torch.as_tensor(G.astype(np.float64 if prec == ph.FP64 else np.float32), device="cuda")
    gH, ge, gx, gy, gz = ph.splat_backward(d, ph.atmosphere(atm), *BAND, SEED, prec, p.offsets, p.mean0, p.grid,
                                           gD)
    gd = torch.stack([gx, gy, gz], 1).cpu().numpy()
    assert int(p.counts.sum()) > 100_000_000
    dd = np.stack([seg["dx"], seg["dy"], seg["dz"]], 1)
    orth = np.abs(np.sum(gd * dd, 1)) / np.maximum(np.linalg.norm(gd, axis=1), 1e-300)
    assert orth.max() <= (1e-12 if prec == ph.FP64 else 1e-6)
    gHn = gH.cpu().numpy()
    assert gHn[3] == 0.0 and gHn[4] == 0.0 and gHn[0] != 0.0
    # sampled segments with a nonzero gradient, spread over the index range
    nz = np.nonzero(np.abs(gd).max(1) > 0)[0]
    rows = nz[np.linspace(0, len(nz) - 1, 24).astype(int)]
    sub = W.subsample(seg, rows)
    cnt, mu, _ = O.counts(sub, O.Atmosphere.from_dict(atm), "cherenkov", SEED)
    assert np.array_equal(cnt, p.counts.cpu().numpy().view(np.uint32)[rows])
    M = SplatModel(sub, atm, SEED, cnt, mu, g, g["sigma"], g["trunc"])
    _, _, rd = M.vjp(G, atm["scale_height"], atm["n0_minus_1"], sub["dx"], sub["dy"], sub["dz"])
    tol = TOL_G64 if prec == ph.FP64 else TOL_G32
    for i in range(len(rows)):
        assert np.linalg.norm(gd[rows[i]] - rd[i]) <= tol * np.linalg.norm(rd[i]) + 1e-300, (rows[i], gd[rows[i]],
                                                                                          rd[i])


def test_full_size_fp32_against_fp64_and_differences(full):
    """1e6 segments, L = sum (D - T)^2 with a seeded target T of the
    density's scale and a wide window (no jumps at its edge): the FP32 adjoint
    against the FP64 adjoint element by element (scale heights, n0 - 1 and
    every segment's direction gradient), and the FP64 adjoint's dL/dH_0 and
    dL/d(n0 - 1) against five-point differences of the FP64 forward."""
    seg, d = full
    atm = W.default_atmosphere(absorption=True)
    g = dict(W.splat_grid_128(), trunc=10.0)
    p64 = ph.SplatProblem(d, atm, SEED, ph.FP64, g, *BAND)
    p32 = ph.SplatProblem(d, atm, SEED, ph.FP32, g, *BAND)
    a0 = ph.atmosphere(atm)
    D = ph.splat_forward(d, a0, *BAND, SEED, ph.FP64, p64.offsets, p64.mean0, p64.grid)
    rng = np.random.Generator(np.random.PCG64(21))
    T = torch.as_tensor(D.cpu().numpy() * rng.uniform(0.8, 1.2, size=(g["ny"], g["nx"])), device="cuda")

    def loss(atm_d):
        Dh = ph.splat_forward(d, ph.atmosphere(atm_d), *BAND, SEED, ph.FP64, p64.offsets, p64.mean0, p64.grid)
        return float(((Dh - T) ** 2).sum())

    G = (2.0 * (D - T)).contiguous()
    g64 = ph.splat_backward(d, a0, *BAND, SEED, ph.FP64, p64.offsets, p64.mean0, p64.grid, G)
    g32 = ph.splat_backward(d, a0, *BAND, SEED, ph.FP32, p32.offsets, p32.mean0, p32.grid, G.float().contiguous())
    H64, e64 = g64[0].cpu().numpy(), float(g64[1].cpu())
    H32, e32 = g32[0].cpu().numpy(), float(g32[1].cpu())
    print(f"dL/dH fp64 {H64} fp32 {H32}; dL/d(n0-1) {e64} {e32}", flush=True)
    for l in (0, 1, 2):
        assert abs(H32[l] - H64[l]) <= TOL_G32 * abs(H64[l]), l
    assert H64[3] == H32[3] == 0.0 and H64[4] == H32[4] == 0.0
    assert abs(e32 - e64) <= TOL_G32 * abs(e64)
    d64 = torch.stack(g64[2:5], 1).cpu().numpy()
    d32 = torch.stack(g32[2:5], 1).cpu().numpy()
    n64 = np.linalg.norm(d64, axis=1)
    err = np.linalg.norm(d32 - d64, axis=1)
    assert np.count_nonzero(n64) > 100_000
    # a segment's gradient sums its photons' terms of both signs (moving a
    # landing point raises the density on one side and lowers it on the
    # other), so the float error is relative to the terms, not to their sum:
    # the bar is 1e-3 of the segment's gradient plus 1e-3 of the rms gradient
    rms = np.sqrt(np.mean(n64[n64 > 0] ** 2))
    bound = TOL_G32 * (n64 + rms)
    print(f"direction gradients: worst error / bound {(err / bound).max():.3f}, rms {rms:.3e}, "
          f"norm-wise {np.linalg.norm(d32 - d64) / np.linalg.norm(d64):.2e}", flush=True)
    assert np.linalg.norm(d32 - d64) <= TOL_G32 * np.linalg.norm(d64)
    assert np.all(err <= bound)

    def fd(f, h):
        return (8.0 * (f(h) - f(-h)) - (f(2.0 * h) - f(-2.0 * h))) / (12.0 * h)

    # steps: small enough that the loss is near its tangent over +-2h (at
    # 1e-3 (n0 - 1) the differences are still 1.2% off; at 1e-4 they agree
    # to 1e-7), large enough that the density's 2^-32 fixed-point steps stay
    # below the change of the loss (below 1e-6 relative they reach 1e-5)
    H0 = np.asarray(atm["scale_height"], float)
    for l in (0, 1):
        def fH(h, l=l):
            Hh = H0.copy()
            Hh[l] += h
            return loss(dict(atm, scale_height=Hh))
        v = fd(fH, 1e-3 * H0[l])
        print(f"dL/dH_{l} adjoint {H64[l]} differences {v}", flush=True)
        assert abs(H64[l] - v) <= 1e-5 * abs(v), l
    e0 = atm["n0_minus_1"]
    v = fd(lambda h: loss(dict(atm, n0_minus_1=e0 + h)), 1e-4 * e0)
    print(f"dL/d(n0-1) adjoint {e64} differences {v}", flush=True)
    assert abs(e64 - v) <= 1e-5 * abs(v)
