"""Reference gradient of the splatted ground photon density (FP64, CPU).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this module. It shares nothing with the HIP
library.

The differentiable form: the Cherenkov photons of every segment, with the
counts frozen at the nominal parameters, each weighted by mu_s(theta) /
mu_s(theta_0) (the Frank-Tamm mean of its segment at the current parameters
over the nominal one) times its transmission exp(-tau), are splatted on a
ground grid with a truncated Gaussian of width sigma normalised per square
metre. The loss is L = sum_g (D_g - T_g)^2. The parameters are the layer
scale heights H_l, n0 - 1 and the raw direction vector of every segment (it
is normalised inside, so its gradient is orthogonal to it).

Derivatives are taken by the complex step: the forward below is written in
plain numpy arithmetic that accepts complex parameters, and for a real
analytic f, f'(x) = Im f(x + i h) / h + O(h^2) with no subtractive
cancellation, so h = 1e-30 gives the derivative to rounding. Each step of the
forward follows the method's own description:

* generation (section 1.2): n at the segment midpoint, cone half angle
  cos(Theta_c) = 1/(beta n), the photon vector at azimuth 2 pi u1 rotated by
  M_Rod (section 1.2.1, the entries as printed), emission point u0 L along
  the track, wavelength from the 1/lambda^2 spectrum;
* propagation (section 2): S = n sin(zenith) is conserved; the horizontal
  displacement is S int dh/r and the density-weighted path int rho n/r dh,
  r = sqrt(n^2 - S^2), integrated over each layer piece by Gauss-Legendre
  quadrature after the substitution h = top - (top - bottom) t^2, which keeps
  the integrand smooth for rays leaving nearly horizontally;
* the Frank-Tamm mean mu = 2 pi alpha z^2 (1/lambda_1 - 1/lambda_2) L
  (1 - 1/(beta n)^2) for the weight ratio;
* the splat: every cell whose centre lies within trunc*sigma of the landing
  point in x and in y receives w exp(-d^2/(2 sigma^2)) / (2 pi sigma^2).
  The cell set is taken from the real part of the landing point, so the
  gradient is the derivative almost everywhere (the truncation edge is not
  differentiated), like the kernel's.
"""
from __future__ import annotations

import numpy as np

from . import oracle as orc

STEP = 1e-30


def _uniforms(seg: dict, seed: int, s_list: np.ndarray, j_list: np.ndarray) -> np.ndarray:
    """u0, u1, u2 of the Cherenkov draws of photons (s, j): counter
    (j, index in shower, shower, 1) under key (seed low, seed high), u = (x + 1/2) 2^-32."""
    n = len(seg["x0"])
    idx = seg.get("index_in_shower")
    idx = np.arange(n, dtype=np.uint32) if idx is None else np.asarray(idx, np.uint32)
    sh = seg.get("shower")
    sh = np.zeros(n, np.uint32) if sh is None else np.asarray(sh, np.uint32)
    ctr = np.stack([np.asarray(j_list, np.uint32), idx[s_list], sh[s_list],
                    np.ones(len(s_list), np.uint32)], axis=1)
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)
    words = orc.philox(ctr, key)
    return (words[:, :3].astype(np.float64) + 0.5) * 2.0 ** -32


class SplatModel:
    """Frozen photon list (segment, j) and random numbers of the differentiable
    form; evaluates density, loss and the reference gradient."""

    def __init__(self, seg: dict, atm: dict, seed: int, counts0, mu0, grid: dict, sigma: float,
                 trunc: float = 4.0, lambda_nm=(300.0, 600.0), n_gl: int = 64):
        self.seg = {k: (np.asarray(v) if isinstance(v, np.ndarray) else v) for k, v in seg.items()}
        self.atm = atm
        self.seed = int(seed)
        cnt = np.asarray(counts0, np.int64)
        self.s_list = np.repeat(np.arange(len(cnt)), cnt)
        off = np.concatenate([[0], np.cumsum(cnt)])
        self.j_list = (np.arange(off[-1]) - off[self.s_list]).astype(np.int64)
        self.mu0 = np.asarray(mu0, np.float64)
        self.grid = dict(grid)
        self.sigma = float(sigma)
        self.trunc = float(trunc)
        self.lmin, self.lmax = float(lambda_nm[0]), float(lambda_nm[1])
        self.K = orc.frank_tamm_K(self.lmin, self.lmax)
        u = _uniforms(self.seg, self.seed, self.s_list, self.j_list)
        self.u0, self.u1, self.u2 = u[:, 0], u[:, 1], u[:, 2]
        inv1, inv2 = 1.0 / self.lmin, 1.0 / self.lmax
        lam = 1.0 / (inv1 - self.u2 * (inv1 - inv2))
        if atm.get("abs_lambda_nm") is not None and len(atm["abs_lambda_nm"]):
            # piecewise linear in lambda, clamped to the end values
            self.kabs = np.interp(lam, atm["abs_lambda_nm"], atm["abs_k_per_m"])
        else:
            self.kabs = np.zeros(len(lam))
        x, w = np.polynomial.legendre.leggauss(n_gl)
        self.t_gl = 0.5 * (x + 1.0)
        self.w_gl = 0.5 * w

    # --------------------------------------------------------------- forward --
    def _atm(self, H, eta0):
        hb = np.asarray(self.atm["h_base"], np.float64)
        nl = len(hb)
        H = [H[l] for l in range(nl)]
        rb = [1.0 + 0j]
        for l in range(nl - 1):
            rb.append(rb[-1] * np.exp(-(hb[l + 1] - hb[l]) / H[l]))
        return hb, H, rb, eta0

    @staticmethod
    def _layer_of(hb, h):
        l = np.zeros(np.shape(h), np.int64)
        for k in range(1, len(hb)):
            l = np.where(hb[k] <= h, k, l)
        return l

    def _density(self, hb, H, rb, l, h):
        """rho/rho0 at heights h inside layers l (arrays of one shape)."""
        out = np.zeros(np.shape(h), np.complex128)
        for k in range(len(hb)):
            m = l == k
            if np.any(m):
                out[m] = rb[k] * np.exp(-(h[m] - hb[k]) / H[k])
        return out

    def photons(self, H, eta0, dx, dy, dz):
        """Landing point (x, y), weight W and landed flag of every photon for
        parameters that may be complex."""
        hb, Hs, rb, eta0 = self._atm(H, eta0)
        hobs = float(self.atm["h_obs"])
        sg = self.seg
        s = self.s_list
        dxs, dys, dzs = np.asarray(dx)[s], np.asarray(dy)[s], np.asarray(dz)[s]
        dn = np.sqrt(dxs * dxs + dys * dys + dzs * dzs)
        vx, vy, vz = dxs / dn, dys / dn, dzs / dn
        L = np.asarray(sg["length"], np.float64)[s]
        beta = np.asarray(sg["beta"], np.float64)[s]
        zz = np.ones(len(s)) if sg.get("charge") is None else np.asarray(sg["charge"], np.float64)[s] ** 2
        # refractive index at the segment midpoint
        zc = np.asarray(sg["z0"], np.float64)[s] + 0.5 * L * vz
        lc = self._layer_of(hb, zc.real)
        n_s = 1.0 + eta0 * self._density(hb, Hs, rb, lc, zc)
        cos_c = 1.0 / (beta * n_s)
        sin_c = np.sqrt((1.0 - cos_c) * (1.0 + cos_c))
        mu = self.K * zz * L * (1.0 - 1.0 / (beta * n_s) ** 2)
        mu0 = self.mu0[s]
        ratio = np.where(mu0 > 0, mu / np.where(mu0 > 0, mu0, 1.0), 0.0)
        # photon vector on the cone and M_Rod (section 1.2.1 entries)
        c = 2.0 * np.pi * self.u1
        p = (np.cos(c) * sin_c, np.sin(c) * sin_c, -cos_c)
        ax, ay, az = vx, vy, vz - 1.0
        an = np.sqrt(ax * ax + ay * ay + az * az)
        ax, ay, az = ax / an, ay / an, az / an
        M = ((-2.0 * ay * ay - 2.0 * az * az + 1.0, 2.0 * ax * ay, 2.0 * ax * az),
             (2.0 * ax * ay, -2.0 * ax * ax - 2.0 * az * az + 1.0, 2.0 * ay * az),
             (2.0 * ax * az, 2.0 * ay * az, -2.0 * ax * ax - 2.0 * ay * ay + 1.0))
        ux = M[0][0] * p[0] + M[0][1] * p[1] + M[0][2] * p[2]
        uy = M[1][0] * p[0] + M[1][1] * p[1] + M[1][2] * p[2]
        uz = M[2][0] * p[0] + M[2][1] * p[1] + M[2][2] * p[2]
        along = self.u0 * L
        xe = np.asarray(sg["x0"], np.float64)[s] + along * vx
        ye = np.asarray(sg["y0"], np.float64)[s] + along * vy
        ze = np.asarray(sg["z0"], np.float64)[s] + along * vz
        landed = (uz.real < 0.0) & (ze.real >= hobs)
        # propagation (section 2)
        le = self._layer_of(hb, ze.real)
        rho_e = self._density(hb, Hs, rb, le, ze)
        n_e = 1.0 + eta0 * rho_e
        se2 = ux * ux + uy * uy
        ce2 = uz * uz
        l_obs = int(self._layer_of(hb, np.array([hobs]))[0])
        G0 = np.zeros(len(s), np.complex128)
        G3 = np.zeros(len(s), np.complex128)
        t, wq = self.t_gl, self.w_gl
        for l in range(l_obs, len(hb)):
            m = landed & (le >= l)
            if not np.any(m):
                continue
            bot = hobs if l == l_obs else hb[l]
            top = np.where(le[m] == l, ze[m], hb[l + 1] if l + 1 < len(hb) else 0.0)
            span = top - bot
            h = top[:, None] - span[:, None] * (t * t)[None, :]
            rho = rb[l] * np.exp(-(h - hb[l]) / Hs[l])
            n = 1.0 + eta0 * rho
            ne_m = n_e[m][:, None]
            # r^2 = n^2 - S^2 = (n_e cos_e)^2 + (n - n_e)(n + n_e)
            r2 = ne_m * ne_m * ce2[m][:, None] + eta0 * (rho - rho_e[m][:, None]) * (n + ne_m)
            r = np.sqrt(r2)
            jac = 2.0 * span[:, None] * t[None, :]
            G0[m] += np.sum(wq[None, :] * jac / r, axis=1)
            G3[m] += np.sum(wq[None, :] * jac * rho * n / r, axis=1)
        x = xe + ux * n_e * G0
        y = ye + uy * n_e * G0
        W = ratio * np.exp(-self.kabs * G3)
        return x, y, W, landed

    def _cells(self, x, y):
        """(photon, flat cell, dx, dy) of every photon-cell pair of the splat,
        with the cell set decided on the real landing point."""
        g = self.grid
        reach = self.trunc * self.sigma
        cell, nx, ny = float(g["cell"]), int(g["nx"]), int(g["ny"])
        xr, yr = x.real, y.real
        m = int(np.floor(2.0 * reach / cell)) + 3
        ix0 = np.floor((xr - reach - g["x_min"]) / cell - 0.5).astype(np.int64) - 1
        iy0 = np.floor((yr - reach - g["y_min"]) / cell - 0.5).astype(np.int64) - 1
        k = np.arange(m)
        ix = ix0[:, None] + k[None, :]
        iy = iy0[:, None] + k[None, :]
        gx = g["x_min"] + (ix + 0.5) * cell
        gy = g["y_min"] + (iy + 0.5) * cell
        okx = (ix >= 0) & (ix < nx) & (np.abs(gx - xr[:, None]) <= reach)
        oky = (iy >= 0) & (iy < ny) & (np.abs(gy - yr[:, None]) <= reach)
        q, a, b = np.nonzero(oky[:, :, None] & okx[:, None, :])
        flat = iy[q, a] * nx + ix[q, b]
        return q, flat, gx[q, b] - x[q], gy[q, a] - y[q]

    def contributions(self, H, eta0, dx, dy, dz):
        """Photon-cell pairs and their (possibly complex) density contributions."""
        x, y, W, landed = self.photons(H, eta0, dx, dy, dz)
        sel = np.nonzero(landed)[0]
        q, flat, ddx, ddy = self._cells(x[sel], y[sel])
        norm = 1.0 / (2.0 * np.pi * self.sigma * self.sigma)
        v = W[sel][q] * norm * np.exp(-(ddx * ddx + ddy * ddy) / (2.0 * self.sigma * self.sigma))
        return sel[q], flat, v

    def density(self, H, eta0, dx, dy, dz):
        _, flat, v = self.contributions(H, eta0, dx, dy, dz)
        g = self.grid
        D = np.zeros(int(g["nx"]) * int(g["ny"]), np.complex128)
        np.add.at(D, flat, v)
        return D.reshape(int(g["ny"]), int(g["nx"]))

    def loss(self, T, H, eta0, dx, dy, dz):
        D = self.density(H, eta0, dx, dy, dz)
        return np.sum((D - T) ** 2)

    # -------------------------------------------------------------- gradient --
    def vjp(self, G, H, eta0, dx, dy, dz):
        """sum_g G_g dD_g/dtheta for a fixed array G (ny, nx): per-layer
        scale heights, n0 - 1 and the per-segment directions, by the complex
        step. Layers with infinite scale height get 0."""
        H = np.asarray(H, np.float64)
        dx, dy, dz = (np.asarray(v, np.float64) for v in (dx, dy, dz))
        Gf = np.asarray(G, np.float64).ravel()

        def dot(qq_flat_v):
            _, flat, v = qq_flat_v
            return float(np.sum(Gf[flat] * v.imag)) / STEP

        g_H = np.zeros(len(H))
        for l in range(len(H)):
            if not np.isfinite(H[l]):
                continue
            Hc = H.astype(np.complex128)
            Hc[l] += 1j * STEP
            g_H[l] = dot(self.contributions(Hc, eta0, dx, dy, dz))
        g_eta = dot(self.contributions(H, eta0 + 1j * STEP, dx, dy, dz))
        # per-segment directions: every photon depends on its own segment
        # only, so one complex step per component gives all segments at once
        g_d = np.zeros((len(dx), 3))
        for c in range(3):
            d = [dx.astype(np.complex128), dy.astype(np.complex128), dz.astype(np.complex128)]
            d[c] = d[c] + 1j * STEP
            qq, flat, v = self.contributions(H, eta0, *d)
            np.add.at(g_d[:, c], self.s_list[qq], Gf[flat] * v.imag / STEP)
        return g_H, g_eta, g_d

    def gradient(self, T, H, eta0, dx, dy, dz):
        """dL/dH (per layer), dL/d(n0 - 1) and dL/d(dx, dy, dz) (per segment)
        of L = sum (D - T)^2: the product with G = dL/dD = 2 (D - T)."""
        D = self.density(H, eta0, dx, dy, dz).real
        return self.vjp(2.0 * (D - np.asarray(T, np.float64)), H, eta0, dx, dy, dz)
