// Splatted ground density and its adjoint (the differentiable form).
//
// Forward: every landed Cherenkov photon adds w norm exp(-d^2/(2 sigma^2))
// to each grid cell whose centre lies within reach = trunc sigma of its
// landing point in x and in y (norm = 1/(2 pi sigma^2)); its weight w is the
// segment's Frank-Tamm mean at the current parameters over the frozen
// nominal mean, times the transmission exp(-tau).
//
// Adjoint: with the random numbers fixed, every photon is regenerated from
// its counter and carried forward once more (no stored paths); the density
// gradient gives the seeds dL/dx, dL/dy, dL/dw at its landing point, which
// are carried back through the layer integrals of section 2, the emission
// point, M_Rod and the cone of section 1.2.1, and the refractive index at the
// segment midpoint, into the layer scale heights, n0 - 1 and the segment
// direction.
#pragma once

#include "photon_device.hpp"

namespace ph {

// ----------------------------------------------------------------- splat --
struct SplatGeom {
  double x_min, y_min, cell, inv_cell;
  double reach, norm, inv_2s2;  // trunc sigma, 1/(2 pi sigma^2), 1/(2 sigma^2)
  double q;  // exp(-cell^2 / sigma^2): ratio of successive Gaussian ratios
  int32_t nx, ny;
};

// Cells along one axis within reach of coordinate x: first index i0, count
// n, offset d0 of the first centre from x. Centres and the reach test are
// evaluated in double without contraction, so the cell set is that of any
// IEEE evaluation of c = lo + (i + 1/2) cell, |c - x| <= reach. The first
// guess of the index range takes the reciprocal of the cell (inv_cell): off
// by at most one from the quotient, which the margin of one cell and the
// exact tests of the loops absorb.
__device__ __forceinline__ void splat_axis(double lo, double cell, double inv_cell, int nc, double reach, double x,
                                           int& i0, int& n, double& d0) {
#pragma clang fp contract(off)
  i0 = 0;
  n = 0;
  d0 = 0.0;
  if (!isfinite(x)) return;
  double fa = floor((x - reach - lo) * inv_cell - 0.5) - 1.0;
  double fb = floor((x + reach - lo) * inv_cell - 0.5) + 1.0;
  fa = fmax(fa, 0.0);
  fb = fmin(fb, (double)(nc - 1));
  if (!(fa <= fb)) return;
  int a = (int)fa, b = (int)fb;
  while (a <= b && !(fabs((lo + ((double)a + 0.5) * cell) - x) <= reach)) ++a;
  while (b >= a && !(fabs((lo + ((double)b + 0.5) * cell) - x) <= reach)) --b;
  if (a > b) return;
  i0 = a;
  n = b - a + 1;
  d0 = (lo + ((double)a + 0.5) * cell) - x;
}

// A cheap first test that a photon landing at (x, y) may have a cell in
// reach: false only when x or y lies more than 1 m outside the grid grown by
// the reach (the margin is far above the float rounding of coordinates below
// 1e6 m and of the bounds; farther out the distance alone decides), and for
// non-finite coordinates. splat_axis's exact tests decide the rest, so the
// cell sets do not change.
template <typename C>
__device__ __forceinline__ bool splat_near(const SplatGeom& g, C x, C y) {
  const C x0 = (C)(g.x_min - g.reach - 1.0), x1 = (C)(g.x_min + g.nx * g.cell + g.reach + 1.0);
  const C y0 = (C)(g.y_min - g.reach - 1.0), y1 = (C)(g.y_min + g.ny * g.cell + g.reach + 1.0);
  return x >= x0 && x <= x1 && y >= y0 && y <= y1;
}

// Gaussian factors along one axis, e_k = exp(-(d0 + k cell)^2 / (2 sigma^2)),
// by the recurrence e_{k+1} = e_k r_k, r_{k+1} = r_k q (two exponentials per
// axis instead of one per cell).
template <typename T>
__device__ __forceinline__ void gauss_start(const SplatGeom& g, double d0, T& e0, T& r0) {
  e0 = Fm<T>::exp_((T)(-(d0 * d0) * g.inv_2s2));
  r0 = Fm<T>::exp_((T)(-(2.0 * d0 * g.cell + g.cell * g.cell) * g.inv_2s2));
}

// Fixed point of the splat accumulation: every cell sums w exp(-d^2/(2 sigma^2))
// (the density without its normalisation) in a 64-bit integer, in units of
// 2^-32 of weight in the double form and 2^-24 in the float form (the
// float's own resolution at weight 1: a contribution below 256 then takes one
// rounding and one 32-bit conversion). Integer sums do not depend on the
// order of the additions, and integer atomics are the fast ones in LDS. A
// cell overflows only beyond 2^32 (double form) or 2^40 (float form) weight
// units.
template <typename T>
__host__ __device__ constexpr double splat_unit() {
  return sizeof(T) == 4 ? 16777216.0 : 4294967296.0;  // 2^24, 2^32
}

// Float, s = v splat_unit (exact): r = its nearest integer (ties to even) is
// a float with at most 24 significant bits, and its high and low 32-bit
// halves are exact in float too, so the 64-bit value equals the
// round-to-nearest conversion of s, from 32-bit conversions only.
__device__ __forceinline__ unsigned long long to_fixed(float s) {
  const float r = __builtin_rintf(s);
  const float hf = __builtin_truncf(r * 0x1p-32f);
  const uint32_t hi = (uint32_t)hf;
  const uint32_t lo = (uint32_t)__builtin_fmaf(-hf, 0x1p32f, r);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long to_fixed(double s) { return __double2ull_rn(s); }

// Rows of at most kSplatCols cells (a 4-sigma window of cells no narrower
// than sigma) take unrolled rows: the column factors e_a come once per photon
// from the same recurrence (the same products, so the same values), and each
// cell costs a multiply, a conversion and the LDS add at an immediate offset.
constexpr int kSplatCols = 9;

// The cells of one photon, rows iy0.. of the accumulator from row (nyw rows
// of nxw cells), wy0 its weight in fixed-point units; NARROW: every
// contribution is below 2^32 units (one 32-bit conversion).
template <typename T, bool NARROW>
__device__ __forceinline__ void splat_cells(unsigned long long* row, int nx, int nxw, int nyw, T wy0, T ex0, T rx0,
                                            T ey, T ry, T q) {
  for (int b = 0; b < nyw; ++b) {
    const T wy = wy0 * ey;
    T ex = ex0, rx = rx0;
    for (int a = 0; a < nxw; ++a) {
      const T v = wy * ex;
      if constexpr (NARROW)
        atomicAdd(&row[a], (unsigned long long)(uint32_t)__builtin_rintf(v));
      else
        atomicAdd(&row[a], to_fixed(v));
      ex *= rx;
      rx *= q;
    }
    row += nx;
    ey *= ry;
    ry *= q;
  }
}

// The same in unrolled rows of at most kSplatCols cells.
template <typename T, bool NARROW>
__device__ __forceinline__ void splat_cells_rows(unsigned long long* row, int nx, int nxw, int nyw, T wy0, T ex0,
                                                 T rx0, T ey, T ry, T q) {
  T ea[kSplatCols];
  {
    T ex = ex0, rx = rx0;
#pragma unroll
    for (int a = 0; a < kSplatCols; ++a) {
      ea[a] = ex;
      ex *= rx;
      rx *= q;
    }
  }
  for (int b = 0; b < nyw; ++b) {
    const T wy = wy0 * ey;
#pragma unroll
    for (int a = 0; a < kSplatCols; ++a) {
      if (a < nxw) {
        const T v = wy * ea[a];
        if constexpr (NARROW)
          atomicAdd(&row[a], (unsigned long long)(uint32_t)__builtin_rintf(v));
        else
          atomicAdd(&row[a], to_fixed(v));
      }
    }
    row += nx;
    ey *= ry;
    ry *= q;
  }
}

// Adds a photon of weight w landing at (x, y) to the fixed-point
// accumulator acc (row-major, ny rows of nx cells). Returns false when no
// cell is within reach.
template <typename T>
__device__ __forceinline__ bool splat_add(const SplatGeom& g, double x, double y, T w, unsigned long long* acc) {
  if (!splat_near<T>(g, (T)x, (T)y)) return false;
  int ix0, nxw, iy0, nyw;
  double dx0, dy0;
  splat_axis(g.x_min, g.cell, g.inv_cell, g.nx, g.reach, x, ix0, nxw, dx0);
  splat_axis(g.y_min, g.cell, g.inv_cell, g.ny, g.reach, y, iy0, nyw, dy0);
  if (nxw == 0 || nyw == 0) return false;
  T ex0, rx0, ey, ry;
  gauss_start<T>(g, dx0, ex0, rx0);
  gauss_start<T>(g, dy0, ey, ry);
  const T q = (T)g.q;
  unsigned long long* row = acc + (int64_t)iy0 * g.nx + ix0;
  // the Gaussian factors are at most 1: a weight below 2^32 units bounds
  // every contribution
  const T ws = w * (T)splat_unit<T>();
  const bool narrow = sizeof(T) == 4 && ws < (T)4294967296.0;
  if (nxw <= kSplatCols) {
    if (narrow)
      splat_cells_rows<T, sizeof(T) == 4>(row, g.nx, nxw, nyw, ws, ex0, rx0, ey, ry, q);
    else
      splat_cells_rows<T, false>(row, g.nx, nxw, nyw, ws, ex0, rx0, ey, ry, q);
  } else if (narrow) {
    splat_cells<T, sizeof(T) == 4>(row, g.nx, nxw, nyw, ws, ex0, rx0, ey, ry, q);
  } else {
    splat_cells<T, false>(row, g.nx, nxw, nyw, ws, ex0, rx0, ey, ry, q);
  }
  return true;
}

// The float form's block accumulator in LDS with 32-bit cells (units of
// 2^-24 of weight, as splat_add): the adds return the old value, and a wrap
// past 2^32 carries 2^32 into the global 64-bit cell (gacc), so that the
// global cell plus the LDS cell is the exact 64-bit sum. NARROW: every
// contribution is below 2^32 units; otherwise each one's high word goes to
// the global cell directly.
template <bool NARROW>
__device__ __forceinline__ void splat_cells32(uint32_t* row, unsigned long long* grow, int nx, int nxw, int nyw,
                                              float wy0, float ex0, float rx0, float ey, float ry, float q) {
  for (int b = 0; b < nyw; ++b) {
    const float wy = wy0 * ey;
    float ex = ex0, rx = rx0;
    for (int a = 0; a < nxw; ++a) {
      const float v = wy * ex;
      uint32_t lo;
      if constexpr (NARROW) {
        lo = (uint32_t)__builtin_rintf(v);
      } else {
        const unsigned long long f = to_fixed(v);
        lo = (uint32_t)f;
        if (f >> 32) atomicAdd(&grow[a], f & 0xffffffff00000000ull);
      }
      const uint32_t old = atomicAdd(&row[a], lo);
      if (old > 0xffffffffu - lo) atomicAdd(&grow[a], 1ull << 32);
      ex *= rx;
      rx *= q;
    }
    row += nx;
    grow += nx;
    ey *= ry;
    ry *= q;
  }
}

__device__ __forceinline__ void splat_cells32_rows(uint32_t* row, unsigned long long* grow, int nx, int nxw, int nyw,
                                                   float wy0, float ex0, float rx0, float ey, float ry, float q) {
  float ea[kSplatCols];
  {
    float ex = ex0, rx = rx0;
#pragma unroll
    for (int a = 0; a < kSplatCols; ++a) {
      ea[a] = ex;
      ex *= rx;
      rx *= q;
    }
  }
  for (int b = 0; b < nyw; ++b) {
    const float wy = wy0 * ey;
#pragma unroll
    for (int a = 0; a < kSplatCols; ++a) {
      if (a < nxw) {
        const uint32_t lo = (uint32_t)__builtin_rintf(wy * ea[a]);
        const uint32_t old = atomicAdd(&row[a], lo);
        uint32_t sum;
        if (__builtin_add_overflow(old, lo, &sum)) atomicAdd(&grow[a], 1ull << 32);
      }
    }
    row += nx;
    grow += nx;
    ey *= ry;
    ry *= q;
  }
}

__device__ __forceinline__ bool splat_add32(const SplatGeom& g, double x, double y, float w, uint32_t* acc,
                                            unsigned long long* gacc) {
  if (!splat_near<float>(g, (float)x, (float)y)) return false;
  int ix0, nxw, iy0, nyw;
  double dx0, dy0;
  splat_axis(g.x_min, g.cell, g.inv_cell, g.nx, g.reach, x, ix0, nxw, dx0);
  splat_axis(g.y_min, g.cell, g.inv_cell, g.ny, g.reach, y, iy0, nyw, dy0);
  if (nxw == 0 || nyw == 0) return false;
  float ex0, rx0, ey, ry;
  gauss_start<float>(g, dx0, ex0, rx0);
  gauss_start<float>(g, dy0, ey, ry);
  const int64_t base = (int64_t)iy0 * g.nx + ix0;
  const float ws = w * (float)splat_unit<float>();
  if (ws < 4294967296.0f && nxw <= kSplatCols)
    splat_cells32_rows(acc + base, gacc + base, g.nx, nxw, nyw, ws, ex0, rx0, ey, ry, (float)g.q);
  else if (ws < 4294967296.0f)
    splat_cells32<true>(acc + base, gacc + base, g.nx, nxw, nyw, ws, ex0, rx0, ey, ry, (float)g.q);
  else
    splat_cells32<false>(acc + base, gacc + base, g.nx, nxw, nyw, ws, ex0, rx0, ey, ry, (float)g.q);
  return true;
}

// Whether a photon landing at (x, y) has a cell in reach (the test of
// splat_add, exactly).
__device__ __forceinline__ bool splat_reach(const SplatGeom& g, double x, double y) {
  if (!splat_near<double>(g, x, y)) return false;
  int i0, n;
  double d0;
  splat_axis(g.x_min, g.cell, g.inv_cell, g.nx, g.reach, x, i0, n, d0);
  if (n == 0) return false;
  splat_axis(g.y_min, g.cell, g.inv_cell, g.ny, g.reach, y, i0, n, d0);
  return n != 0;
}

// Seeds of one photon from the density gradient G: dL/dx, dL/dy (through
// the Gaussian) and dL/dw. Returns false when no cell is within reach.
template <typename T, typename Gt>
__device__ __forceinline__ bool splat_seeds(const SplatGeom& g, double x, double y, T w, const Gt* G, T& xb, T& yb,
                                            T& wb) {
  if (!splat_near<double>(g, x, y)) return false;
  int ix0, nxw, iy0, nyw;
  double dx0, dy0;
  splat_axis(g.x_min, g.cell, g.inv_cell, g.nx, g.reach, x, ix0, nxw, dx0);
  splat_axis(g.y_min, g.cell, g.inv_cell, g.ny, g.reach, y, iy0, nyw, dy0);
  if (nxw == 0 || nyw == 0) return false;
  T ex0, rx0, ey, ry;
  gauss_start<T>(g, dx0, ex0, rx0);
  gauss_start<T>(g, dy0, ey, ry);
  const T q = (T)g.q, cell = (T)g.cell;
  T s0 = (T)0, sx = (T)0, sy = (T)0;
  const Gt* row = G + (int64_t)iy0 * g.nx + ix0;
  T dy = (T)dy0;
  if (nxw <= kSplatCols) {
    // unrolled rows (as splat_cells32_rows): the column factors and offsets
    // from the same recurrences, the same sums in the same order
    T ea[kSplatCols], da[kSplatCols];
    {
      T ex = ex0, rx = rx0, dx = (T)dx0;
#pragma unroll
      for (int a = 0; a < kSplatCols; ++a) {
        ea[a] = ex;
        da[a] = dx;
        ex *= rx;
        rx *= q;
        dx += cell;
      }
    }
    for (int b = 0; b < nyw; ++b) {
      T r0 = (T)0, r1 = (T)0;
#pragma unroll
      for (int a = 0; a < kSplatCols; ++a) {
        if (a < nxw) {
          const T v = (T)row[a] * ea[a];
          r0 += v;
          r1 += v * da[a];
        }
      }
      s0 += ey * r0;
      sx += ey * r1;
      sy += ey * dy * r0;
      row += g.nx;
      ey *= ry;
      ry *= q;
      dy += cell;
    }
  } else {
    for (int b = 0; b < nyw; ++b) {
      T ex = ex0, rx = rx0, dx = (T)dx0;
      T r0 = (T)0, r1 = (T)0;
      for (int a = 0; a < nxw; ++a) {
        const T v = (T)row[a] * ex;
        r0 += v;
        r1 += v * dx;
        ex *= rx;
        rx *= q;
        dx += cell;
      }
      s0 += ey * r0;
      sx += ey * r1;
      sy += ey * dy * r0;
      row += g.nx;
      ey *= ry;
      ry *= q;
      dy += cell;
    }
  }
  const T n = (T)g.norm, is2 = (T)(2.0 * g.inv_2s2);  // 1/sigma^2
  wb = n * s0;
  xb = w * n * is2 * sx;
  yb = w * n * is2 * sy;
  return true;
}

// ---------------------------------------------------------------- adjoint --
// Per-lane sums of the global adjoints, kept in lane-private LDS slots
// (word k of lane i at p[k * stride]): dL/d ln rb[m] (rb[m] = rho/rho0 at the
// base of layer m, a function of the scale heights below it) in words
// 0..7, the direct dL/dH_l in words 8..15, dL/d(n0 - 1) in word 16.
constexpr int kAdjWords = 2 * PHOTON_MAX_LAYERS + 1;
constexpr int kAdjLnrb = 0, kAdjH = PHOTON_MAX_LAYERS, kAdjEta = 2 * PHOTON_MAX_LAYERS;

struct AdjAcc {
  double* p;
  int stride;
  __device__ __forceinline__ void add(int k, double v) { p[k * stride] += v; }
  __device__ __forceinline__ void lnrb(int l, double v) { add(kAdjLnrb + l, v); }
  __device__ __forceinline__ void H(int l, double v) { add(kAdjH + l, v); }
  __device__ __forceinline__ void eta(double v) { add(kAdjEta, v); }
};

// Raw segment record as read for the adjoint.
struct SegRaw {
  double x0, y0, z0, dx, dy, dz, len, beta, zz, mu0;
  uint32_t idx, shower;
};

// Per-segment constants of the adjoint, in double, computed once per segment
// (adj_seg_setup): the unit track direction v and 1/|d|, the cone (cos and
// sin of its angle, cc/sc, cc/ns), the unit bisector A of the half turn and
// 1/|b| (0 when v points straight down), the weight ratio mu/mu0 at the
// frozen counts and its factor d ratio/d cos, and the index at the midpoint
// (layer lc, rho_c, eta0 rho_c) with the factors its adjoint takes to H_lc and
// to v_z. ok: the segment emits (beta n > 1, mu0 > 0, a valid record).
struct AdjSeg {
  double x0, y0, z0, len;
  double vx, vy, vz, inv_dn;
  double cc, sc, cc_sc, cc_ns;
  double Ax, Ay, Az, inv_bn;
  double ratio, ratio_cc;
  double rho_c, eta_rho_c, hfac_c, vfac_c;
  int32_t lc;
  uint32_t idx, shower;
  int32_t ok;
};

// The constants of segment sg (section 1.2: index at the midpoint, cone
// angle; the half turn about the bisector of the track and the downward
// normal), K the Frank-Tamm factor.
__device__ __forceinline__ void adj_seg_setup(const AtmDev& a, const AtmLane& L, const SegRaw& sg, bool valid,
                                              double K, AdjSeg& o) {
  o.x0 = sg.x0;
  o.y0 = sg.y0;
  o.z0 = sg.z0;
  o.len = sg.len;
  o.idx = sg.idx;
  o.shower = sg.shower;
  const double dn = sqrt((sg.dx * sg.dx + sg.dy * sg.dy) + sg.dz * sg.dz);
  const double vx = sg.dx / dn, vy = sg.dy / dn, vz = sg.dz / dn;
  o.vx = vx;
  o.vy = vy;
  o.vz = vz;
  o.inv_dn = 1.0 / dn;
  const double zc = sg.z0 + (0.5 * sg.len) * vz;
  const int lc = layer_of(a, zc);
  const double rho_c = L.rb[lc] * exp(-(zc - L.hb[lc]) * L.invH[lc]);
  const double ns = 1.0 + a.eta0 * rho_c;
  const double bn = sg.beta * ns;
  const double cc = 1.0 / bn;
  const double sc2 = (1.0 - cc) * (1.0 + cc);
  o.ok = valid && sc2 > 0.0 && sg.mu0 > 0.0;
  const double sc = sqrt(fmax(sc2, 0.0));
  const double kzl = (K * sg.zz) * sg.len;
  o.cc = cc;
  o.sc = sc;
  o.cc_sc = cc / sc;
  o.cc_ns = cc / ns;
  o.ratio = (kzl * (1.0 - 1.0 / (bn * bn))) / sg.mu0;
  o.ratio_cc = -2.0 * cc * kzl / sg.mu0;
  const double bx = vx, by = vy, bz = vz - 1.0;
  const double bnorm = sqrt((bx * bx + by * by) + bz * bz);
  const bool rot = bnorm > 0.0;
  o.Ax = rot ? bx / bnorm : 1.0;
  o.Ay = rot ? by / bnorm : 0.0;
  o.Az = rot ? bz / bnorm : 0.0;
  o.inv_bn = rot ? 1.0 / bnorm : 0.0;
  o.lc = lc;
  o.rho_c = rho_c;
  o.eta_rho_c = a.eta0 * rho_c;
  o.hfac_c = (zc - L.hb[lc]) * L.invH[lc] * L.invH[lc];
  o.vfac_c = -0.5 * sg.len * L.invH[lc];
}

// Closed-form layer piece with its partial derivatives. Variables of the
// formulas: C2 = 1 - S^2, eps_a / eps_b (n - 1 at the bottom / top), H, dh,
// and for the density-weighted path rho_a / rho_b. For a piece [a, b]:
//   C2 > 0: G = dh/C + (H/C) ln(P_b/P_a),   P = C r + C2 + eps
//   C2 < 0: G = (H/K) [asin(v_a) - asin(v_b)],  v = (eps - K^2)/(eps S), K^2 = -C2
//   C2 = 0: G = H (r_b/eps_b - r_a/eps_a)
//   homogeneous: G = dh/r
//   Col = H (rho_a - rho_b)(2 + eps_a + eps_b)/(r_a + r_b)   (homogeneous: rho (1 + eps) dh/r)
// with r = sqrt(C2 + eps (2 + eps)) = sqrt(n^2 - S^2). The derivatives use
//   d ln P/d eps = (2 + eps)/(r (r + C)),  d ln P/d C2 = (r + C)^2/(2 C r P),
//   (r + C)^2 = 2 P + eps^2,
//   d asin(v)/d eps = K/(eps r),  d asin(v)/d K^2 = -(2 + K^2 + eps)/(2 S^2 K r), S^2 = 1 + K^2.
template <typename T>
struct PieceD {
  double g;       // int dh/r
  T col;          // int rho n/r dh
  T g_C2, g_ea, g_eb, g_H, g_dh;
  T c_C2, c_ea, c_eb, c_ra, c_rb, c_H, c_dh;
};

template <typename T, bool DERIV>
__device__ __forceinline__ void piece_d(T rho_a, T em, double dh, T H, bool homog, T eta0, T C2, T Cc, T invC,
                                        double invCd, T S, T ra, T rb, PieceD<T>& o) {
  using F = Fm<T>;
  const T eps_a = eta0 * rho_a;
  const T dht = (T)dh;
  if (homog) {
    const T ira = F::rcp(ra);
    const T n_a = (T)1 + eps_a;
    o.g = dh / (double)ra;
    o.col = rho_a * n_a * dht * ira;
    if (DERIV) {
      const T ira3 = ira * ira * ira;
      o.g_dh = ira;
      o.g_C2 = -(T)0.5 * dht * ira3;
      o.g_ea = -dht * n_a * ira3;
      o.g_eb = (T)0;
      o.g_H = (T)0;
      o.c_dh = rho_a * n_a * ira;
      o.c_ra = n_a * dht * ira;
      o.c_ea = rho_a * dht * (ira - n_a * n_a * ira3);
      o.c_C2 = -(T)0.5 * rho_a * n_a * dht * ira3;
      o.c_eb = o.c_rb = o.c_H = (T)0;
    }
    return;
  }
  const T drho = rho_a * em;  // rho_b - rho_a
  const T d = eta0 * drho;    // eps_b - eps_a
  const T eps_b = eps_a + d;
  const T rs = ra + rb;
  const T irs = F::rcp(rs);
  const T two_e = (T)2 + eps_a + eps_b;
  const T Q = two_e * irs;
  o.col = -H * drho * Q;
  T gc;
  if (C2 > (T)0) {
    const T Pa = Cc * ra + C2 + eps_a;
    const T delta = d * ((T)1 + Cc * Q);  // P_b - P_a
    const T lq = F::log1p_(delta * F::rcp(Pa));
    gc = H * invC * lq;
    o.g = dh * invCd + (double)gc;
    if (DERIV) {
      const T Pb = Pa + delta;
      const T rd = -d * Q;  // r_a - r_b
      o.g_dh = invC;
      o.g_H = invC * lq;
      o.g_ea = -(H * invC) * ((T)2 + eps_a) * F::rcp(ra * (ra + Cc));
      o.g_eb = (H * invC) * ((T)2 + eps_b) * F::rcp(rb * (rb + Cc));
      o.g_C2 = ((T)(-o.g) + H * ((T)2 * rd * F::rcp(ra * rb) + eps_b * eps_b * F::rcp(rb * Pb) -
                                  eps_a * eps_a * F::rcp(ra * Pa))) *
               F::rcp((T)2 * C2);
    }
  } else if (C2 < (T)0) {
    const T K2 = -C2;
    const T Kk = F::sqrt_(K2);
    const T A = asin((eps_a - K2) / (eps_a * S)), B = asin((eps_b - K2) / (eps_b * S));
    gc = (H / Kk) * (A - B);
    o.g = (double)gc;
    if (DERIV) {
      const T S2 = (T)1 + K2;
      o.g_dh = (T)0;
      o.g_H = (A - B) / Kk;
      o.g_ea = H / (eps_a * ra);
      o.g_eb = -H / (eps_b * rb);
      const T da = -((T)2 + K2 + eps_a) / ((T)2 * S2 * Kk * ra);
      const T db = -((T)2 + K2 + eps_b) / ((T)2 * S2 * Kk * rb);
      // d G/d C2 = -d G/d K^2
      o.g_C2 = gc / ((T)2 * K2) - (H / Kk) * (da - db);
    }
  } else {
    gc = H * (rb / eps_b - ra / eps_a);
    o.g = (double)gc;
    if (DERIV) {
      o.g_dh = (T)0;
      o.g_H = rb / eps_b - ra / eps_a;
      o.g_ea = H / (eps_a * ra);
      o.g_eb = -H / (eps_b * rb);
      o.g_C2 = (T)0;  // C2 exactly 0: a set of measure zero
    }
  }
  if (DERIV) {
    const T dr = -drho;  // rho_a - rho_b
    o.c_H = dr * Q;
    o.c_ra = H * Q;
    o.c_rb = -H * Q;
    o.c_ea = H * dr * ((T)1 - Q * ((T)1 + eps_a) * F::rcp(ra)) * irs;
    o.c_eb = H * dr * ((T)1 - Q * ((T)1 + eps_b) * F::rcp(rb)) * irs;
    o.c_C2 = -(T)0.5 * H * dr * Q * (F::rcp(ra) + F::rcp(rb)) * irs;
    o.c_dh = (T)0;
  }
}

// Outcome of adjoint_photon.
constexpr int kAdjNone = 0, kAdjDone = 1, kAdjDeferred = 2;

// Adjoint of one Cherenkov photon (segment sg, number j) of the splatted
// density with gradient G. Adds its contributions to the global sums acc and
// returns the segment-direction adjoint in dd (kAdjDone), or kAdjNone when
// the photon contributes nothing (not landed, outside every cell's reach, or
// its segment below threshold). The float form returns kAdjDeferred for rays
// within about 3 degrees of the horizontal (C^2 <= 0.0025), which the double
// form finishes; with FORCE_FLOAT it evaluates them in float.
template <typename T, typename Gt, bool FORCE_FLOAT = false>
__device__ __forceinline__ int adjoint_photon(const AtmDev& a, const AtmLane& L, const AdjSeg& sg, uint32_t j,
                                              uint32_t k0, uint32_t k1, double inv_l1, double inv_dl,
                                              const SplatGeom& g, const Gt* G, AdjAcc acc, double dd[3]) {
  using F = Fm<T>;
  dd[0] = dd[1] = dd[2] = 0.0;
  if (!sg.ok) return kAdjNone;
  const double vx = sg.vx, vy = sg.vy, vz = sg.vz;

  // photon j (section 1.2.1): cone vector, M_Rod p = 2 (A.p) A - p
  const U4 r = philox(j, sg.idx, sg.shower, kDomCher, k0, k1);
  const T u0 = u01<T>(r.w[0]), u1 = u01<T>(r.w[1]), u2 = u01<T>(r.w[2]);
  T sp, cp;
  cone_sincos(u1, &sp, &cp);
  const T tsc = (T)sg.sc, tcc = (T)sg.cc;
  const T Ax = (T)sg.Ax, Ay = (T)sg.Ay, Az = (T)sg.Az;
  const T px = cp * tsc, py = sp * tsc, pz = -tcc;
  const T ap = Ax * px + Ay * py + Az * pz;
  T ux = (T)2 * ap * Ax - px, uy = (T)2 * ap * Ay - py, uz = (T)2 * ap * Az - pz;
  const T s = u0 * (T)sg.len;
  const double ze = sg.z0 + (double)(s * (T)vz);
  if (!(uz < (T)0) || !(ze >= a.hobs)) return kAdjNone;
  const double xe = sg.x0 + (double)(s * (T)vx), ye = sg.y0 + (double)(s * (T)vy);
  const T lambda = F::rcp((T)inv_l1 - u2 * (T)inv_dl);
  const T kabs = abs_coeff<T>(a, L, lambda);
  const T inv_un = F::rcp(F::sqrt_(ux * ux + uy * uy + uz * uz));
  ux *= inv_un;
  uy *= inv_un;
  uz *= inv_un;

  // propagation (section 2), first sweep: values
  const double ced = -(double)uz;
  const double sed = sqrt((1.0 - ced) * (1.0 + ced));
  const int le = layer_of(a, ze);
  const double bot_e = L.pc[le][kPcBot];
  const double rho_bot_e = L.pc[le][kPcRho];
  const bool homog_e = (a.homog_mask >> le) & 1;
  const T eta0 = (T)a.eta0;
  const T em_e = homog_e ? (T)0 : F::expm1_((T)(-(ze - bot_e) * L.invH[le]));
  const T rho_e = (T)rho_bot_e * ((T)1 + em_e);
  const T eps_e = eta0 * rho_e;
  const T ne = (T)1 + eps_e;
  const double epsd = (double)eps_e;
  const double C2d = (ced * ced / (1.0 + sed) - epsd * sed) * (1.0 + (1.0 + epsd) * sed);
  if constexpr (sizeof(T) == 4 && !FORCE_FLOAT) {
    if (!(C2d > (double)kNearHorizonC2)) return kAdjDeferred;
  }
  const T C2 = (T)C2d;
  const T S = ne * (T)sed;
  const T Cc = C2 > (T)0 ? F::sqrt_(C2) : (T)0;
  const T invC = C2 > (T)0 ? F::rcp(Cc) : (T)0;
  const double invCd = C2 > (T)0 ? (sizeof(T) == 8 ? (double)invC : rsqrt_refined(C2d)) : 0.0;
  const T r_e = ne * (T)ced;  // r at the emission point
  double g0 = 0.0;
  T col = (T)0;
  // piece constants from the LDS record of each layer (as in the forward
  // propagation)
  {
    T r_top = r_e;
    for (int l = a.nl - 1; l >= a.l_obs; --l) {
      if (l > le) continue;
      const double* pc = L.pc[l];
      const double top = (l == le) ? ze : pc[kPcTop];
      const double dh = top - pc[kPcBot];
      if (!(dh > 0.0)) continue;
      const bool homog = (a.homog_mask >> l) & 1;
      const double H_l = pc[kPcH];
      const T rho_a = (T)pc[kPcRho];
      const T em = (l == le) ? em_e : (T)pc[kPcEm];
      const T eps_a = eta0 * rho_a;
      const T ra = F::sqrt_(C2 + eps_a * ((T)2 + eps_a));
      PieceD<T> o;
      piece_d<T, false>(rho_a, em, dh, (T)H_l, homog, eta0, C2, Cc, invC, invCd, S, ra, r_top, o);
      g0 += o.g;
      col += o.col;
      r_top = ra;
    }
  }
  const double disp = (double)ne * g0;
  const double xl = xe + (double)ux * disp, yl = ye + (double)uy * disp;
  const T w = F::exp_(-kabs * col);
  const T W = (T)sg.ratio * w;

  // seeds from the density gradient
  T xb, yb, Wb;
  if (!splat_seeds<T, Gt>(g, xl, yl, W, G, xb, yb, Wb)) return kAdjNone;
  const T ratio_b = Wb * w;
  const T col_b = -kabs * w * (T)sg.ratio * Wb;
  const T g0t = (T)g0;
  const T g0_b = (xb * ux + yb * uy) * ne;
  T ne_b = (xb * ux + yb * uy) * g0t;
  const T ux_b = xb * ne * g0t, uy_b = yb * ne * g0t;
  T uz_b = (T)0;
  T C2_b = (T)0, rhoe_b = (T)0;
  double ze_b = 0.0;

  // second sweep: partial derivatives of every piece
  {
    T r_top = r_e;
    for (int l = a.nl - 1; l >= a.l_obs; --l) {
      if (l > le) continue;
      const double* pc = L.pc[l];
      const double top = (l == le) ? ze : pc[kPcTop];
      const double bot = pc[kPcBot];
      const double dh = top - bot;
      if (!(dh > 0.0)) continue;
      const bool homog = (a.homog_mask >> l) & 1;
      const bool is_obs = l == a.l_obs;
      const double H_l = pc[kPcH];
      const double invH_l = L.invH[l];
      const T rho_a = (T)pc[kPcRho];
      const T em = (l == le) ? em_e : (T)pc[kPcEm];
      const T rho_b = rho_a * ((T)1 + em);
      const T eps_a = eta0 * rho_a;
      const T ra = F::sqrt_(C2 + eps_a * ((T)2 + eps_a));
      PieceD<T> o;
      piece_d<T, true>(rho_a, em, dh, (T)H_l, homog, eta0, C2, Cc, invC, invCd, S, ra, r_top, o);
      C2_b += g0_b * o.g_C2 + col_b * o.c_C2;
      const T ea_b = g0_b * o.g_ea + col_b * o.c_ea;
      const T eb_b = g0_b * o.g_eb + col_b * o.c_eb;
      T ra_b = col_b * o.c_ra + eta0 * ea_b;
      T rb_b = col_b * o.c_rb + eta0 * eb_b;
      acc.eta((double)(ea_b * rho_a + eb_b * rho_b));
      if (!homog) acc.H(l, (double)(g0_b * o.g_H + col_b * o.c_H));
      const T dh_b = g0_b * o.g_dh + col_b * o.c_dh;
      if (homog) {
        ra_b += rb_b;  // the density is the same at both ends
        rb_b = (T)0;
      }
      // density at the bottom of the piece: rb[l], or at h_obs
      // rho_obs = rb[l_obs] exp(-(h_obs - hb[l_obs])/H[l_obs])
      const double tb = (double)(ra_b * rho_a);
      acc.lnrb(l, tb);
      if (is_obs) acc.H(l, tb * (bot - L.hb[l]) * invH_l * invH_l);
      // density at the top: rb[l + 1], or rho_e for the emission piece
      if (l == le) {
        rhoe_b += rb_b;
        ze_b += (double)dh_b;
      } else {
        acc.lnrb(l + 1, (double)(rb_b * rho_b));
      }
      r_top = ra;
    }
  }
  // C2 = 1 - ne^2 (1 - uz^2)
  const T se2 = (T)((1.0 - ced) * (1.0 + ced));
  uz_b += C2_b * (T)2 * ne * ne * uz;
  ne_b += -C2_b * (T)2 * ne * se2;
  acc.eta((double)(ne_b * rho_e));
  rhoe_b += ne_b * eta0;
  // rho_e = rb[le] exp(-(ze - hb[le])/H[le])
  {
    const double t = (double)(rhoe_b * rho_e);
    acc.lnrb(le, t);
    acc.H(le, t * (ze - L.hb[le]) * L.invH[le] * L.invH[le]);
    ze_b -= t * L.invH[le];
  }
  // emission point x_e = x0 + s v (v the unit track direction)
  const double sd = (double)s;
  double vxb = (double)xb * sd, vyb = (double)yb * sd, vzb = ze_b * sd;
  // u = 2 (A.p) A - p
  const T Au = Ax * ux_b + Ay * uy_b + Az * uz_b;
  const T Axb = (T)2 * (Au * px + ap * ux_b), Ayb = (T)2 * (Au * py + ap * uy_b), Azb = (T)2 * (Au * pz + ap * uz_b);
  const T pxb = (T)2 * Au * Ax - ux_b, pyb = (T)2 * Au * Ay - uy_b, pzb = (T)2 * Au * Az - uz_b;
  if (sg.inv_bn > 0.0) {
    // A = b/|b|, b = v - (0, 0, 1)
    const double AdA = sg.Ax * (double)Axb + sg.Ay * (double)Ayb + sg.Az * (double)Azb;
    vxb += ((double)Axb - sg.Ax * AdA) * sg.inv_bn;
    vyb += ((double)Ayb - sg.Ay * AdA) * sg.inv_bn;
    vzb += ((double)Azb - sg.Az * AdA) * sg.inv_bn;
  }
  // p = (cos c sin Tc, sin c sin Tc, -cos Tc); the weight ratio ~ 1 - cos^2 Tc
  const double scb = (double)(pxb * cp + pyb * sp);
  double ccb = -(double)pzb - scb * sg.cc_sc;
  ccb += (double)ratio_b * sg.ratio_cc;
  // cos Tc = 1/(beta ns), ns = 1 + eta0 rho_c, rho_c = rb[lc] exp(-(zc - hb[lc])/H[lc])
  const double nsb = -ccb * sg.cc_ns;
  acc.eta(nsb * sg.rho_c);
  const double t = nsb * sg.eta_rho_c;
  acc.lnrb(sg.lc, t);
  acc.H(sg.lc, t * sg.hfac_c);
  vzb += t * sg.vfac_c;
  // v = d/|d|
  const double vdot = vx * vxb + vy * vyb + vz * vzb;
  dd[0] = (vxb - vx * vdot) * sg.inv_dn;
  dd[1] = (vyb - vy * vdot) * sg.inv_dn;
  dd[2] = (vzb - vz * vdot) * sg.inv_dn;
  return kAdjDone;
}

}  // namespace ph
