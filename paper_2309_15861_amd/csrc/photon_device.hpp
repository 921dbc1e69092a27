// Device-side building blocks of the photon pipeline (gfx950, wave64).
//
// Paper: Baack & Alameddine, arXiv:2309.15861 (ICRC2023). Section 1.1
// (fluorescence yield), section 1.2 (Frank-Tamm count, cone generation),
// section 1.2.1 (photon vector p, rotation M_Rod), section 2 (propagation).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "photon.h"

namespace ph {

constexpr double kPi = 3.141592653589793;
constexpr double kAlpha = 7.2973525693e-3;   // fine-structure constant (CODATA 2018)
constexpr double kC = 0.299792458;           // m/ns
constexpr uint32_t kDomCount = 0u, kDomCher = 1u, kDomFluo = 2u;
constexpr double kPoissonChunk = 128.0;
constexpr uint32_t kPoissonKmax = 1000u;
constexpr double kMaxMean = 1e7;   // a segment with a larger mean is invalid

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x32
// S-box; each round multiplies words 0 and 2 by the published constants,
// crosses the high halves with words 1 and 3 and the key, and the key gets
// the Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t w[4];
};

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      // the keys are wave-uniform: bumped per round with scalar adds (an
      // empty asm keeps the compiler from precomputing all ten round keys,
      // which would occupy scalar registers through the whole photon loop)
      asm volatile("" : "+s"(k0), "+s"(k1));
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  return U4{{c0, c1, c2, c3}};
}

// (x + 1/2) 2^-32: exact in double, strictly inside (0,1).
__device__ __forceinline__ double u01d(uint32_t x) { return (double)x * 0x1p-32 + 0x1p-33; }
// Float form: the 32-bit word converted with one rounding, so u keeps about
// 6e-8 relative precision down to 2^-33 (1 - u is taken as u(~x)).
__device__ __forceinline__ float u01f(uint32_t x) { return __builtin_fmaf((float)x, 0x1p-32f, 0x1p-33f); }

template <typename T>
__device__ __forceinline__ T u01(uint32_t x);
template <>
__device__ __forceinline__ double u01<double>(uint32_t x) { return u01d(x); }
template <>
__device__ __forceinline__ float u01<float>(uint32_t x) { return u01f(x); }

// ---------------------------------------------------------------------------
// Atmosphere as passed to kernels (by value). rb = rho/rho0 at each layer
// base, computed on the host by the recurrence rb[i+1] = rb[i]
// exp(-(h[i+1]-h[i])/H[i]); rho_obs and n_obs at the observation level.
// ---------------------------------------------------------------------------
struct AtmDev {
  int32_t nl;
  int32_t n_abs;
  double hb[PHOTON_MAX_LAYERS + 1];  // +inf beyond the last layer (hb[l + 1] is the top of layer l)
  double H[PHOTON_MAX_LAYERS];
  double rb[PHOTON_MAX_LAYERS];
  double eta0, hobs, rho_obs, n_obs;
  int32_t l_obs;          // layer of h_obs
  int32_t homog_mask;     // bit i set: layer i has infinite scale height
  double invH[PHOTON_MAX_LAYERS];
  double em_full[PHOTON_MAX_LAYERS];  // expm1(-(hb[l+1] - hb[l]) / H[l]): density ratio - 1 across layer l
  double em_obs;                      // expm1(-(top of the observation layer - hobs) / H[l_obs])
  int32_t abs_uniform;                // absorption nodes equally spaced
  double abs_l[PHOTON_MAX_ABS];
  double abs_k[PHOTON_MAX_ABS];
  // first node and nodes per nm (uniform nodes: the first guess of the node
  // index in either precision, corrected by one comparison each way)
  float absf_l0, absf_inv_step;
  float absf_l_lo, absf_l_hi, absf_k_lo, absf_k_hi;  // first and last nodes in float
  // straight-line propagation with correction tables (tcorr = NULL: exact)
  const float4* tcorr;                // (g, dP, dX, 0) per node, q fastest
  const float2* tvert;                // (rho/rho0, vertical column) per height node
  int32_t tn_h, tn_q, tn_v;
  double t_hmax, t_qmax;
  double t_fi, t_fj, t_fk;            // nodes per metre of height, per unit of q, per metre (vertical)
};

// The exponential of the count path (the index at the segment midpoint, the
// layer base densities it uses, and exp(-mean) of the Poisson draw): a count
// is an integer decided on these values, and library exp routines differ in
// the last bit, so every step is fixed here as a sequence of IEEE double
// operations without contraction that any implementation of the same steps
// reproduces bit for bit. Argument reduction after Cody and Waite (1980):
// x = k ln 2 + r with k the nearest integer to x/ln 2 (ties to even) and
// ln 2 split into a head with 21 trailing zero bits (k ln2_hi exact) and a
// tail; e^r as its Taylor series through r^13 (|r| <= ln 2 / 2, first
// omitted term below 5e-18) in Horner form from the highest power with
// coefficients 1/i! rounded to double; scaled by 2^k. About 1 ulp.
__host__ __device__ inline double exp_fixed(double x) {
#pragma clang fp contract(off)
  if (x != x) return x;
  if (x > 709.78) return HUGE_VAL;
  if (x < -745.2) return 0.0;
  const double k = rint(x * 0x1.71547652b82fep+0);
  const double r = (x - k * 0x1.62e42fee00000p-1) - k * 0x1.a39ef35793c76p-33;
  double p = 0x1.6124613a86d09p-33;   // 1/13!
  p = p * r + 0x1.1eed8eff8d898p-29;  // 1/12!
  p = p * r + 0x1.ae64567f544e4p-26;  // 1/11!
  p = p * r + 0x1.27e4fb7789f5cp-22;  // 1/10!
  p = p * r + 0x1.71de3a556c734p-19;  // 1/9!
  p = p * r + 0x1.a01a01a01a01ap-16;  // 1/8!
  p = p * r + 0x1.a01a01a01a01ap-13;  // 1/7!
  p = p * r + 0x1.6c16c16c16c17p-10;  // 1/6!
  p = p * r + 0x1.1111111111111p-7;   // 1/5!
  p = p * r + 0x1.5555555555555p-5;   // 1/4!
  p = p * r + 0x1.5555555555555p-3;   // 1/3!
  p = p * r + 0.5;
  p = p * r + 1.0;
  p = p * r + 1.0;
  return ldexp(p, (int)k);
}

// Layer of height h: the last k with hb[k] <= h (hb is +inf beyond the last
// layer; layer 0 also extends below hb[0]).
__device__ __forceinline__ int layer_of(const AtmDev& a, double h) {
  int l = 0;
#pragma unroll
  for (int k = 1; k < PHOTON_MAX_LAYERS; ++k)
    if (a.hb[k] <= h) l = k;
  return l;
}

// ---------------------------------------------------------------------------
// Per-segment mean and Poisson count (section 1.2 Frank-Tamm, section 1.1
// yield). Evaluated in double without contraction in a fixed order so that
// counts are reproducible bit for bit by any IEEE implementation of the
// same steps.
// ---------------------------------------------------------------------------
struct SegView {
  const double *x0, *y0, *z0, *dx, *dy, *dz, *len, *beta, *t0, *dedx;
  const int32_t* charge;
  const uint32_t *shower, *idx;
};

__device__ __forceinline__ uint32_t seg_idx(const SegView& s, int64_t i) {
  return s.idx ? s.idx[i] : (uint32_t)i;
}
__device__ __forceinline__ uint32_t seg_shower(const SegView& s, int64_t i) {
  return s.shower ? s.shower[i] : 0u;
}

__device__ __forceinline__ bool seg_ok(const SegView& s, int64_t i) {
#pragma clang fp contract(off)
  const double v[9] = {s.x0[i], s.y0[i], s.z0[i], s.dx[i], s.dy[i], s.dz[i], s.len[i], s.beta[i], s.t0[i]};
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 9; ++k) ok = ok && isfinite(v[k]);
  ok = ok && (s.beta[i] > 0.0) && (s.beta[i] < 1.0) && (s.len[i] >= 0.0);
  const double dn2 = (s.dx[i] * s.dx[i] + s.dy[i] * s.dy[i]) + s.dz[i] * s.dz[i];
  return ok && (dn2 > 0.0);
}

// n at the segment midpoint (the medium is homogeneous along a short step).
__device__ __forceinline__ double seg_index(const SegView& s, int64_t i, const AtmDev& a) {
#pragma clang fp contract(off)
  const double dx = s.dx[i], dy = s.dy[i], dz = s.dz[i];
  const double dn = sqrt((dx * dx + dy * dy) + dz * dz);
  const double dzh = dz / dn;
  const double zc = s.z0[i] + (0.5 * s.len[i]) * dzh;
  const int l = layer_of(a, zc);
  const double rho = a.rb[l] * exp_fixed(-(zc - a.hb[l]) / a.H[l]);
  return 1.0 + a.eta0 * rho;
}

__device__ __forceinline__ double mean_cherenkov(const SegView& s, int64_t i, const AtmDev& a, double K) {
#pragma clang fp contract(off)
  if (!seg_ok(s, i)) return 0.0;
  const double n = seg_index(s, i, a);
  const double bn = s.beta[i] * n;
  const double f = 1.0 - 1.0 / (bn * bn);
  double zz = 1.0;
  if (s.charge) zz = (double)(s.charge[i] * s.charge[i]);
  return (f > 0.0) ? ((K * zz) * s.len[i]) * f : 0.0;
}

__device__ __forceinline__ double mean_fluor(const SegView& s, int64_t i, double Y) {
#pragma clang fp contract(off)
  if (!seg_ok(s, i)) return 0.0;
  const double e = s.dedx[i];
  if (!(isfinite(e) && e >= 0.0)) return 0.0;
  return (Y * e) * s.len[i];
}

// Cherenkov angular particle cut (the optimisation of section 1.2.1): a
// segment passes when the angle between its unit direction and the vector
// from its midpoint to one of the points is at most the cut angle,
// d.v >= cos_cut |v|. FP64 without contraction in a fixed order, so that any
// IEEE evaluation of the same steps decides alike.
struct CutDev {
  int32_t n;  // 0: no cut
  double cos_cut;
  double pts[PHOTON_MAX_CUT_POINTS][3];
};

__device__ __forceinline__ bool passes_cut(const SegView& s, int64_t i, const CutDev& c) {
#pragma clang fp contract(off)
  if (c.n <= 0) return true;
  const double dx = s.dx[i], dy = s.dy[i], dz = s.dz[i];
  const double dn = sqrt((dx * dx + dy * dy) + dz * dz);
  const double ux = dx / dn, uy = dy / dn, uz = dz / dn;
  const double hl = 0.5 * s.len[i];
  const double mx = s.x0[i] + hl * ux, my = s.y0[i] + hl * uy, mz = s.z0[i] + hl * uz;
  for (int k = 0; k < c.n && k < PHOTON_MAX_CUT_POINTS; ++k) {
    const double vx = c.pts[k][0] - mx, vy = c.pts[k][1] - my, vz = c.pts[k][2] - mz;
    const double dot = (ux * vx + uy * vy) + uz * vz;
    const double nv = sqrt((vx * vx + vy * vy) + vz * vz);
    if (dot >= c.cos_cut * nv) return true;
  }
  return false;
}

// Fluorescence beaming (the optimisation of section 1.1.1): a track emits
// into a cone that contains an emission area enclosing every telescope, a
// sphere of centre c and radius r, and its photon number is scaled by the
// cone's solid-angle fraction. Seen from the track midpoint m, at distance D
// from c, the sphere grown by half the track length (which contains the
// sphere as seen from every point of the track) subtends the half angle
// alpha, sin(alpha) = (r + L/2)/D; the cone adds a margin for the bending of
// rays by refraction. Returns om = 1 - cos(alpha + margin), so that the
// solid-angle fraction is om/2, and the unit cone axis (m to c). A track
// inside the grown sphere stays isotropic: om = 2, axis straight down. FP64
// without contraction in a fixed order, like the angular cut.
struct BeamDev {
  int32_t on;
  double cx, cy, cz, r;
  double cos_m, sin_m;  // cosine and sine of the margin angle
};

__device__ __forceinline__ double beam_cap(const SegView& s, int64_t i, const BeamDev& b, double* ax, double* ay,
                                           double* az) {
#pragma clang fp contract(off)
  const double dx = s.dx[i], dy = s.dy[i], dz = s.dz[i];
  const double dn = sqrt((dx * dx + dy * dy) + dz * dz);
  const double ux = dx / dn, uy = dy / dn, uz = dz / dn;
  const double hl = 0.5 * s.len[i];
  const double mx = s.x0[i] + hl * ux, my = s.y0[i] + hl * uy, mz = s.z0[i] + hl * uz;
  const double vx = b.cx - mx, vy = b.cy - my, vz = b.cz - mz;
  const double D = sqrt((vx * vx + vy * vy) + vz * vz);
  const double reach = b.r + hl;
  if (!(reach < D)) {
    *ax = 0.0;
    *ay = 0.0;
    *az = -1.0;
    return 2.0;
  }
  const double sa = reach / D;
  const double ca = sqrt((1.0 - sa) * (1.0 + sa));
  const double cb = ca * b.cos_m - sa * b.sin_m;
  *ax = vx / D;
  *ay = vy / D;
  *az = vz / D;
  return 1.0 - cb;
}

// Mean photon number of a fluorescence segment with beaming: the isotropic
// mean times the cone's solid-angle fraction.
__device__ __forceinline__ double beamed_mean(const SegView& s, int64_t i, const BeamDev& b, double mu) {
#pragma clang fp contract(off)
  if (!b.on || !(mu > 0.0)) return mu;
  double ax, ay, az;
  const double om = beam_cap(s, i, b, &ax, &ay, &az);
  return mu * (0.5 * om);
}

// Chunking of a mean for the Poisson draw: m chunks of mean mc (m = 0 when
// the segment emits nothing).
__device__ __forceinline__ uint32_t poisson_chunks(double mu) {
#pragma clang fp contract(off)
  if (!(mu > 0.0) || !(mu <= kMaxMean)) return 0u;
  return (mu <= kPoissonChunk) ? 1u : (uint32_t)ceil(mu / kPoissonChunk);
}

// One chunk: the smallest k with F(k) >= u for Poisson(mc), p0 = exp(-mc),
// capped at kPoissonKmax; rk[k] = 1/(k+1), 16-byte aligned. The terms are
// taken four at a time: the products and sums are the ones of the step-by-step
// recurrence in the same order, and F never decreases, so one test of the
// fourth sum decides whether all four steps are taken (one table read and one
// loop test per four steps), and the result is the same.
__device__ __forceinline__ uint32_t poisson_chunk(double u, double mc, double p0, const double* rk) {
#pragma clang fp contract(off)
  static_assert(kPoissonKmax % 4u == 0u, "the cap is a multiple of the step group");
  double p = p0, F = p0;
  if (!(u > F)) return 0u;
  for (uint32_t k = 0; k < kPoissonKmax; k += 4u) {
    const double2 r01 = *reinterpret_cast<const double2*>(rk + k);
    const double2 r23 = *reinterpret_cast<const double2*>(rk + k + 2);
    const double p1 = (p * mc) * r01.x, F1 = F + p1;
    const double p2 = (p1 * mc) * r01.y, F2 = F1 + p2;
    const double p3 = (p2 * mc) * r23.x, F3 = F2 + p3;
    const double p4 = (p3 * mc) * r23.y, F4 = F3 + p4;
    if (!(u > F4)) return k + (!(u > F1) ? 1u : !(u > F2) ? 2u : !(u > F3) ? 3u : 4u);
    p = p4;
    F = F4;
  }
  return kPoissonKmax;
}

// Precision-specific primitives: the float path uses the hardware
// reciprocal, square root and logarithm (about 1 ulp); the double path uses
// correctly rounded IEEE operations and the library functions.
template <typename T>
struct Fm;
template <>
struct Fm<double> {
  // reciprocal: the hardware estimate refined by two Newton steps, within an
  // ulp of 1/x for the finite, normal arguments of the photon path (the
  // IEEE division takes about twice the instructions)
  static __device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
  }
  // square root: the hardware reciprocal square root refined by two coupled
  // Newton steps for g = sqrt(x) and h = 1/(2 sqrt(x)), then one correction
  // of g from its residual x - g^2 (within an ulp)
  static __device__ __forceinline__ double sqrt_(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    r = __builtin_fma(-g, h, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    g = __builtin_fma(__builtin_fma(-g, g, x), h, g);
    return x > 0.0 ? g : (x == 0.0 ? 0.0 : __builtin_nan(""));
  }
  // log1p: below |x| = 1/8 (the layer integrals' arguments, except on rays
  // grazing the horizon) 2 atanh(s) with s = x/(2 + x) by its odd series,
  // 2 s (1 + s^2/3 + ... + s^16/17) (|s| < 1/15, so the next term is below
  // 1e-20 relative); elsewhere the library routine
  static __device__ __forceinline__ double log1p_(double x) {
    if (__builtin_fabs(x) < 0.125) {
      const double s = x * rcp(2.0 + x);
      const double s2 = s * s;
      double q = 1.0 / 17.0;
      q = __builtin_fma(q, s2, 1.0 / 15.0);
      q = __builtin_fma(q, s2, 1.0 / 13.0);
      q = __builtin_fma(q, s2, 1.0 / 11.0);
      q = __builtin_fma(q, s2, 1.0 / 9.0);
      q = __builtin_fma(q, s2, 1.0 / 7.0);
      q = __builtin_fma(q, s2, 1.0 / 5.0);
      q = __builtin_fma(q, s2, 1.0 / 3.0);
      const double s3 = s * s2;
      return 2.0 * __builtin_fma(s3, q, s);
    }
    return log1p(x);
  }
  static __device__ __forceinline__ double expm1_(double x) { return expm1(x); }
  static __device__ __forceinline__ double exp_(double x) { return exp(x); }
};
template <>
struct Fm<float> {
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
  // log1p(x) = log(u) x / (u - 1) with u = 1 + x rounded (exact u - 1);
  // log(u) = log2(u) ln 2 from the hardware log2 (u lies near 1 here: no
  // denormal or infinite argument to guard against)
  // For |x| < 1/32 (the arguments of the float path's layer integrals but
  // those of rays within a few degrees of the horizon) a degree-6 Taylor
  // polynomial instead: truncation x^7/7, below 1e-10 relative.
  static __device__ __forceinline__ float log1p_(float x) {
    if (fabsf(x) < 0.03125f) {
      float p = -1.66666667e-01f;
      p = __builtin_fmaf(p, x, 0.2f);
      p = __builtin_fmaf(p, x, -0.25f);
      p = __builtin_fmaf(p, x, 3.33333333e-01f);
      p = __builtin_fmaf(p, x, -0.5f);
      p = __builtin_fmaf(p, x, 1.0f);
      return p * x;
    }
    const float u = 1.0f + x;
    return (__builtin_amdgcn_logf(u) * 0.693147180559945309f) * (x * __builtin_amdgcn_rcpf(u - 1.0f));
  }
  // expm1 for x <= 0: Taylor polynomial to x^8 for |x| < 0.5 (truncation
  // 1e-8 relative), else exp(x) - 1, where 1 - e^x > 0.39 keeps the
  // subtraction well conditioned; about 2e-7 relative either way
  static __device__ __forceinline__ float expm1_(float x) {
    float p = 2.48015873e-05f;  // 1/8!
    p = __builtin_fmaf(p, x, 1.98412698e-04f);
    p = __builtin_fmaf(p, x, 1.38888889e-03f);
    p = __builtin_fmaf(p, x, 8.33333333e-03f);
    p = __builtin_fmaf(p, x, 4.16666667e-02f);
    p = __builtin_fmaf(p, x, 1.66666667e-01f);
    p = __builtin_fmaf(p, x, 0.5f);
    p = __builtin_fmaf(p, x, 1.0f);
    return fabsf(x) < 0.5f ? p * x : __expf(x) - 1.0f;
  }
  static __device__ __forceinline__ float exp_(float x) { return __expf(x); }
};

// ---------------------------------------------------------------------------
// Per-segment constants of photon generation, computed once per segment
// (one lane per segment) and shared by all of its photons.
// ---------------------------------------------------------------------------
// Float form: the cone's dominant vertical terms in double. A photon's
// vertical direction component is 2 (A.p) A_z - p_z, dominated by A_z p_z;
// rounded to float its absolute error (a few 1e-7) becomes a relative error
// of the slant path of 1/cos(zenith) times that, about 0.15 ns on steep rays.
template <typename T>
struct SegHi {
  double cos_cd;  // cone cosine (Cherenkov) or 1 - cos of the beaming cone (beamed fluorescence)
  double azd;     // vertical component of the M_Rod bisector
};
template <>
struct SegHi<double> {};

template <typename T>
struct SegConst : SegHi<T> {
  T x0, y0;                        // start point (horizontal: in the working precision)
  double z0, t0, inv_bc;           // start height, start time, 1/(beta c)
  T dx, dy, dz, len;               // unit direction, length
  T cos_c, sin_c;                  // Cherenkov cone (section 1.2); beamed fluorescence: cos_c = om
  T ax, ay, az;                    // unit bisector of the cone axis and (0,0,-1)
  uint32_t idx, shower;
  int32_t layer;                   // the layer holding the whole segment (1 mm margin), else -1
};

// Unit bisector A of a cone axis d and the downward normal: M_Rod
// (section 1.2.1) is the half turn 2 A A^T - 1 about it, which maps the
// downward axis onto d. For d straight up the bisector vanishes and the
// half turn about x is used.
__device__ __forceinline__ void rod_bisector(double ux, double uy, double uz, double* bx, double* by, double* bz) {
  double x = ux, y = uy, z = uz - 1.0;
  const double bn = sqrt((x * x + y * y) + z * z);
  if (bn > 0.0) {
    x /= bn;
    y /= bn;
    z /= bn;
  } else {
    x = 1.0;
    y = 0.0;
    z = 0.0;
  }
  *bx = x;
  *by = y;
  *bz = z;
}

// The cone axis is the track direction for Cherenkov light and the beaming
// axis for beamed fluorescence.
template <typename T>
__device__ __forceinline__ void seg_const(const SegView& s, int64_t i, const AtmDev& a, bool cherenkov,
                                          const BeamDev& beam, SegConst<T>& c) {
  const double dx = s.dx[i], dy = s.dy[i], dz = s.dz[i];
  const double dn = sqrt((dx * dx + dy * dy) + dz * dz);
  const double ux = dx / dn, uy = dy / dn, uz = dz / dn;
  c.x0 = (T)s.x0[i];
  c.y0 = (T)s.y0[i];
  c.z0 = s.z0[i];
  c.t0 = s.t0[i];
  c.inv_bc = 1.0 / (s.beta[i] * kC);
  c.dx = (T)ux;
  c.dy = (T)uy;
  c.dz = (T)uz;
  c.len = (T)s.len[i];
  c.idx = seg_idx(s, i);
  c.shower = seg_shower(s, i);
  {
    // emission heights z0 + s dz, s in [0, len], rounded in either precision
    const double z1 = c.z0 + s.len[i] * uz;
    const double m = 1e-3 + 1e-6 * s.len[i];
    const int l0 = layer_of(a, fmin(c.z0, z1) - m), l1 = layer_of(a, fmax(c.z0, z1) + m);
    c.layer = l0 == l1 ? l0 : -1;
  }
  if (cherenkov) {
    const double n = seg_index(s, i, a);
    const double cc = 1.0 / (s.beta[i] * n);
    c.cos_c = (T)cc;
    c.sin_c = (T)sqrt((1.0 - cc) * (1.0 + cc));
    double bx, by, bz;
    rod_bisector(ux, uy, uz, &bx, &by, &bz);
    c.ax = (T)bx;
    c.ay = (T)by;
    c.az = (T)bz;
    if constexpr (sizeof(T) == 4) {
      c.cos_cd = cc;
      c.azd = bz;
    }
  } else if (beam.on) {
    double ax, ay, az, bx, by, bz;
    const double om = beam_cap(s, i, beam, &ax, &ay, &az);
    c.cos_c = (T)om;
    c.sin_c = (T)0;
    rod_bisector(ax, ay, az, &bx, &by, &bz);
    c.ax = (T)bx;
    c.ay = (T)by;
    c.az = (T)bz;
    if constexpr (sizeof(T) == 4) {
      c.cos_cd = om;
      c.azd = bz;
    }
  } else {
    c.cos_c = c.sin_c = c.ax = c.ay = c.az = (T)0;
  }
}

// One photon in registers. The height z, the time and the path length are
// double in both precisions: along slant paths of hundreds of km a float
// height (2 mm ulp at 30 km) would cost about 0.1 ns of arrival time.
// uzd is the vertical direction component in double: exact for isotropic
// photons (from the 32-bit word), the float value otherwise. The float path
// takes the ray's C^2 and its long-path terms from it.
template <typename T>
struct Photon {
  T x, y, ux, uy, uz, lambda, w;
  double z, t, path, uzd;
  int32_t status;
};

__device__ __forceinline__ void sincos2pi(double u, double* s, double* c) { sincospi(2.0 * u, s, c); }
__device__ __forceinline__ void sincos2pi(float u, float* s, float* c) { sincospif(2.0f * u, s, c); }
// Cone azimuth: in float the hardware sine/cosine, whose argument is in
// revolutions (u in (0,1)); its error enters the direction scaled by the
// small sin(theta_c).
__device__ __forceinline__ void cone_sincos(double u, double* s, double* c) { sincospi(2.0 * u, s, c); }
__device__ __forceinline__ void cone_sincos(float u, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(u);
  *c = __builtin_amdgcn_cosf(u);
}

// Photon j of a Cherenkov segment (section 1.2, Fig. 1): cone vector
// p = (cos c sin Tc, sin c sin Tc, -cos Tc) at azimuth c = 2 pi u1
// (section 1.2.1), rotated by M_Rod p = 2 (A.p) A - p, moved to the emission
// point u0 along the track; wavelength from the 1/lambda^2 spectrum.
template <typename T>
__device__ __forceinline__ void gen_cherenkov(const SegConst<T>& c, uint32_t j, uint32_t k0, uint32_t k1,
                                              T inv_l1, T inv_dl, Photon<T>& p) {
  const U4 r = philox(j, c.idx, c.shower, kDomCher, k0, k1);
  const T u0 = u01<T>(r.w[0]), u1 = u01<T>(r.w[1]), u2 = u01<T>(r.w[2]);
  const T s = u0 * c.len;
  p.x = c.x0 + s * c.dx;
  p.y = c.y0 + s * c.dy;
  p.z = c.z0 + (double)(s * c.dz);
  p.t = c.t0 + (double)s * c.inv_bc;
  T sp, cp;
  cone_sincos(u1, &sp, &cp);
  const T px = cp * c.sin_c, py = sp * c.sin_c, pz = -c.cos_c;
  const T ap2 = (T)2 * (c.ax * px + c.ay * py + c.az * pz);
  p.ux = ap2 * c.ax - px;
  p.uy = ap2 * c.ay - py;
  if constexpr (sizeof(T) == 4) {
    // the dominant A_z p_z term in double (the small horizontal terms in float)
    const double pzd = -c.cos_cd;
    p.uzd = 2.0 * ((double)(c.ax * px + c.ay * py) + c.azd * pzd) * c.azd - pzd;
    p.uz = (T)p.uzd;
  } else {
    p.uz = ap2 * c.az - pz;
    p.uzd = p.uz;
  }
  p.lambda = Fm<T>::rcp(inv_l1 - u2 * inv_dl);
  p.w = (T)1;
  p.path = 0.0;
  p.status = PHOTON_LANDED;
}

// Photon j of a fluorescence segment (section 1.1): isotropic direction,
// emission point u0 along the track, line k = smallest k with u3 < cdf[k],
// decided exactly on the 32-bit word against integer thresholds
// thr[k] = ceil(cdf[k] 2^32 - 1/2). Beamed (section 1.1.1): uniform on the
// segment's cone, 1 - cos(theta) = u1 om from the axis and azimuth 2 pi u2,
// generated about the downward normal and turned onto the axis by M_Rod.
template <typename T>
__device__ __forceinline__ void gen_fluor(const SegConst<T>& c, uint32_t j, uint32_t k0, uint32_t k1,
                                          const uint64_t* thr, const T* line_nm, int n_lines, bool beam,
                                          Photon<T>& p) {
  const U4 r = philox(j, c.idx, c.shower, kDomFluo, k0, k1);
  const T u0 = u01<T>(r.w[0]), u1 = u01<T>(r.w[1]), u2 = u01<T>(r.w[2]);
  const T s = u0 * c.len;
  p.x = c.x0 + s * c.dx;
  p.y = c.y0 + s * c.dy;
  p.z = c.z0 + (double)(s * c.dz);
  p.t = c.t0 + (double)s * c.inv_bc;
  if (beam) {
    const T v = u1 * c.cos_c;
    const T ct = (T)1 - v;
    const T st = Fm<T>::sqrt_(v * ((T)2 - v));
    T sp, cp;
    sincos2pi(u2, &sp, &cp);
    const T px = st * cp, py = st * sp, pz = -ct;
    const T ap2 = (T)2 * (c.ax * px + c.ay * py + c.az * pz);
    p.ux = ap2 * c.ax - px;
    p.uy = ap2 * c.ay - py;
    if constexpr (sizeof(T) == 4) {
      // the dominant A_z p_z term in double, p_z = -(1 - u1 om)
      const double vd = u01<double>(r.w[1]) * c.cos_cd;
      const double pz2 = vd - 1.0;
      p.uzd = 2.0 * ((double)(c.ax * px + c.ay * py) + c.azd * pz2) * c.azd - pz2;
      p.uz = (T)p.uzd;
    } else {
      p.uz = ap2 * c.az - pz;
      p.uzd = p.uz;
    }
  } else {
    // cos = 1 - 2 u1 = -(w - 2^31 + 1/2) 2^-31, and 1 - u1 = u(~w): both
    // taken from the 32-bit word, so rays near the horizon keep their
    // relative precision in either arithmetic
    const int32_t sw = (int32_t)(r.w[1] ^ 0x80000000u);
    const double ctd = -((double)sw + 0.5) * 0x1p-31;
    const T ct = (T)ctd;
    const T st = (T)2 * Fm<T>::sqrt_(u01<T>(r.w[1]) * u01<T>(~r.w[1]));
    T sp, cp;
    sincos2pi(u2, &sp, &cp);
    p.ux = st * cp;
    p.uy = st * sp;
    p.uz = ct;
    p.uzd = ctd;
  }
  int k = 0;
  const uint64_t w3 = r.w[3];
  while (k < n_lines - 1 && !(w3 < thr[k])) ++k;
  p.lambda = line_nm[k];
  p.w = (T)1;
  p.path = 0.0;
  p.status = PHOTON_LANDED;
}

// ---------------------------------------------------------------------------
// Propagation (section 2). With n sin(theta) = S conserved, the layer
// integrals of dh/r, n dh/r, n^2 dh/r and rho n dh/r (r = sqrt(n^2 - S^2))
// have closed forms in eps = n - 1 = eta0 rho, which falls exponentially
// with scale height H inside a layer. For a piece [a, b] (a below b):
//   C^2 = 1 - S^2 > 0:  int dh/r = (b-a)/C + (H/C) log((C r_b + C^2 + eps_b)
//                                                   / (C r_a + C^2 + eps_a))
//   C^2 < 0, K^2 = -C^2: int dh/r = (H/K) [asin((eps_a - K^2)/(eps_a S))
//                                        - asin((eps_b - K^2)/(eps_b S))]
//   C^2 = 0:           int dh/r = H (r_b/eps_b - r_a/eps_a)
//   int n dh/r   = int dh/r + H log((n_a + r_a)/(n_b + r_b))
//   int n^2 dh/r = int n dh/r + H (r_a - r_b)
//   int rho n dh/r = H (rho_a - rho_b) (2 + eps_a + eps_b)/(r_a + r_b)
// Differences are formed from eps_a expm1(-(b-a)/H) so that thin pieces and
// nearly vertical rays keep full relative precision.
// ---------------------------------------------------------------------------
// Integrals over one layer piece [a, b] (a below b) of dh/r, n dh/r,
// n^2 dh/r and rho n dh/r, with r = sqrt(n^2 - S^2) and eps = n - 1 falling
// exponentially with scale height H. rho_a is rho/rho0 at a and
// em = rho_b/rho_a - 1; ra and rb are r at both ends. C2 = 1 - S^2.
//   C2 > 0:  int dh/r = (b-a)/C + (H/C) log((C r_b + C^2 + eps_b) / (C r_a + C^2 + eps_a))
//   C2 < 0:  int dh/r = (H/K) [asin((eps_a - K^2)/(eps_a S)) - asin((eps_b - K^2)/(eps_b S))], K^2 = -C2
//   C2 = 0:  int dh/r = H (r_b/eps_b - r_a/eps_a)
//   int n dh/r   = int dh/r + H log((n_a + r_a)/(n_b + r_b))
//   int n^2 dh/r = int n dh/r + H (r_a - r_b)
//   int rho n dh/r = H (rho_a - rho_b)(2 + eps_a + eps_b)/(r_a + r_b)
// The log arguments are written as 1 + (small difference) and the
// differences come from em, so thin pieces and near-vertical rays keep their
// relative precision. The dominant term of int dh/r, (b-a)/C (or (b-a)/r in a
// homogeneous layer), is left to the caller, which adds it in double; the
// piece returns the remainder g0c and the path increments lgH = int n dh/r -
// int dh/r and rdH = int n^2 dh/r - int n dh/r, all small.
template <typename T>
struct PieceOut {
  T g0c, lgH, rdH, col;
};

template <typename T>
__device__ __forceinline__ void piece_integrals(T rho_a, T em, T dh, T H, bool homog, T eta0, T C2, T Cc, T invC,
                                                T S, T ra, T rb, PieceOut<T>& o) {
  using F = Fm<T>;
  const T eps_a = eta0 * rho_a;
  if (homog) {
    const T g = dh * F::rcp(ra);
    o.g0c = (T)0;
    o.lgH = eps_a * g;
    o.rdH = eps_a * ((T)1 + eps_a) * g;
    o.col = rho_a * ((T)1 + eps_a) * g;
    return;
  }
  const T drho = rho_a * em;            // rho_b - rho_a
  const T d = eta0 * drho;              // eps_b - eps_a
  const T eps_b = eps_a + d;
  const T nb = (T)1 + eps_b;
  const T inv_rs = F::rcp(ra + rb);
  const T two_e = (T)2 + eps_a + eps_b;
  const T rd = -d * two_e * inv_rs;     // r_a - r_b
  if (C2 > (T)0) {
    const T den = Cc * ra + C2 + eps_a;
    const T delta = d * ((T)1 + Cc * two_e * inv_rs);
    o.g0c = (H * invC) * F::log1p_(delta * F::rcp(den));
  } else if (C2 < (T)0) {
    const T K2 = -C2;
    const T Kk = F::sqrt_(K2);
    o.g0c = (H / Kk) * (asin((eps_a - K2) / (eps_a * S)) - asin((eps_b - K2) / (eps_b * S)));
  } else {
    o.g0c = H * (rb / eps_b - ra / eps_a);
  }
  o.lgH = H * F::log1p_((-d + rd) * F::rcp(nb + rb));
  o.rdH = H * rd;
  o.col = -H * drho * two_e * inv_rs;
}

// Tables that photons index by their own layer or wavelength bin, mirrored
// into LDS by every kernel that propagates (lane-indexed reads of a kernel
// argument would be vector memory loads). abs_s[i] is the slope of the
// absorption coefficient on [abs_l[i], abs_l[i+1]].
// pc[l]: the piece of layer l a downward ray crosses, with the observation
// layer folded in: bottom (h_obs in the observation layer, else the layer
// base), top (the next base, +inf for the top layer), rho/rho0 at the
// bottom, expm1 of the density drop from bottom to top, scale height, and
// the thickness top - bottom. A ray loop reads it with its wave-uniform layer
// index (broadcast LDS reads: neither scalar registers nor vector memory).
// pcf[l]: the float form's copy (thickness, rho, em, H), so that its loop
// converts nothing. pfg[l], pfh[l]: what a whole layer's piece needs that
// does not depend on the ray, for the float form (below).
enum { kPcBot = 0, kPcTop, kPcRho, kPcEm, kPcH, kPcDh, kPcWords };
struct AtmLane {
  double hb[PHOTON_MAX_LAYERS], rb[PHOTON_MAX_LAYERS], invH[PHOTON_MAX_LAYERS];
  double abs_l[PHOTON_MAX_ABS], abs_k[PHOTON_MAX_ABS], abs_s[PHOTON_MAX_ABS];
  double pc[PHOTON_MAX_LAYERS][kPcWords];
  float4 pcf[PHOTON_MAX_LAYERS];
  float4 pfg[PHOTON_MAX_LAYERS], pfh[PHOTON_MAX_LAYERS];
  float abs_lf[PHOTON_MAX_ABS], abs_kf[PHOTON_MAX_ABS], abs_sf[PHOTON_MAX_ABS];
};

// Block-cooperative copy; the caller synchronises before use.
__device__ __forceinline__ void atm_lane_fill(const AtmDev& a, AtmLane* L) {
  for (int i = threadIdx.x; i < PHOTON_MAX_LAYERS; i += blockDim.x) {
    L->hb[i] = a.hb[i];
    L->rb[i] = a.rb[i];
    L->invH[i] = a.invH[i];
  }
  for (int i = threadIdx.x; i < PHOTON_MAX_LAYERS; i += blockDim.x) {
    const bool obs = i == a.l_obs;
    L->pc[i][kPcBot] = obs ? a.hobs : a.hb[i];
    L->pc[i][kPcTop] = a.hb[i + 1];
    L->pc[i][kPcRho] = obs ? a.rho_obs : a.rb[i];
    L->pc[i][kPcEm] = obs ? a.em_obs : a.em_full[i];
    L->pc[i][kPcH] = a.H[i];
    L->pc[i][kPcDh] = L->pc[i][kPcTop] - L->pc[i][kPcBot];
    L->pcf[i] = make_float4((float)L->pc[i][kPcDh], (float)L->pc[i][kPcRho], (float)L->pc[i][kPcEm], (float)a.H[i]);
    // eps_a, eps_a (2 + eps_a), d = eps_b - eps_a, d (2 + eps_a + eps_b);
    // n_b, -H drho (2 + eps_a + eps_b), H
    const double eps_a = a.eta0 * L->pc[i][kPcRho];
    const double d = eps_a * L->pc[i][kPcEm];
    const double two_e = 2.0 + eps_a + (eps_a + d);
    const bool homog = (a.homog_mask >> i) & 1;
    L->pfg[i] = make_float4((float)eps_a, (float)(eps_a * (2.0 + eps_a)), (float)d, (float)(d * two_e));
    L->pfh[i] = make_float4((float)(1.0 + eps_a + d),
                            homog ? 0.0f : (float)(-a.H[i] * L->pc[i][kPcRho] * L->pc[i][kPcEm] * two_e),
                            (float)a.H[i], 0.0f);
  }
  for (int i = threadIdx.x; i < PHOTON_MAX_ABS; i += blockDim.x) {
    L->abs_l[i] = a.abs_l[i];
    L->abs_k[i] = a.abs_k[i];
    L->abs_s[i] = (i + 1 < a.n_abs) ? (a.abs_k[i + 1] - a.abs_k[i]) / (a.abs_l[i + 1] - a.abs_l[i]) : 0.0;
    L->abs_lf[i] = (float)a.abs_l[i];
    L->abs_kf[i] = (float)a.abs_k[i];
    L->abs_sf[i] = (float)L->abs_s[i];
  }
}

// Absorption coefficient at rho/rho0 = 1: piecewise linear in lambda,
// clamped to the end values outside the table.
template <typename T>
__device__ __forceinline__ T abs_coeff_double(const AtmDev& a, const AtmLane& L, T lambda) {
  if (a.n_abs <= 0) return (T)0;
  const double l = (double)lambda;
  if (l <= a.abs_l[0]) return (T)a.abs_k[0];
  if (l >= a.abs_l[a.n_abs - 1]) return (T)a.abs_k[a.n_abs - 1];
  int lo;
  if (a.abs_uniform) {
    lo = (int)((l - (double)a.absf_l0) * (double)a.absf_inv_step);
    lo = lo < 0 ? 0 : (lo > a.n_abs - 2 ? a.n_abs - 2 : lo);
    // guard against the last bit of the index computation
    if (l < L.abs_l[lo]) --lo;
    else if (!(l < L.abs_l[lo + 1])) ++lo;
  } else {
    lo = 0;
    int hi = a.n_abs - 1;  // abs_l[lo] <= l < abs_l[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (L.abs_l[mid] <= l) lo = mid; else hi = mid;
    }
  }
  return (T)(L.abs_k[lo] + (l - L.abs_l[lo]) * L.abs_s[lo]);
}

// The float form: the same interpolation on float copies of the nodes (the
// function is continuous, so a node decided differently by rounding moves
// the value by rounding only).
__device__ __forceinline__ float abs_coeff_float(const AtmDev& a, const AtmLane& L, float l) {
  if (a.n_abs <= 0) return 0.0f;
  if (l <= a.absf_l_lo) return a.absf_k_lo;
  if (l >= a.absf_l_hi) return a.absf_k_hi;
  int lo;
  if (a.abs_uniform) {
    lo = (int)((l - a.absf_l0) * a.absf_inv_step);
    lo = lo < 0 ? 0 : (lo > a.n_abs - 2 ? a.n_abs - 2 : lo);
    if (l < L.abs_lf[lo]) --lo;
    else if (!(l < L.abs_lf[lo + 1])) ++lo;
  } else {
    lo = 0;
    int hi = a.n_abs - 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (L.abs_lf[mid] <= l) lo = mid; else hi = mid;
    }
  }
  return L.abs_kf[lo] + (l - L.abs_lf[lo]) * L.abs_sf[lo];
}

template <typename T>
__device__ __forceinline__ T abs_coeff(const AtmDev& a, const AtmLane& L, T lambda) {
  if constexpr (sizeof(T) == 4) return abs_coeff_float(a, L, lambda);
  else return abs_coeff_double<T>(a, L, lambda);
}

// Double square root and reciprocal square root for the float path: the
// float hardware seed (about 1 ulp) refined by one Newton step in double
// (relative error below 1e-13; the square root gets one more correction),
// at a fraction of the cost of the correctly rounded double routines.
__device__ __forceinline__ double rsqrt_refined(double x) {
  const double r = (double)__builtin_amdgcn_rsqf((float)x);
  return r * (1.5 - 0.5 * x * r * r);
}
__device__ __forceinline__ double sqrt_refined(double x) {
  if (!(x > 0.0)) return 0.0;
  const double r = rsqrt_refined(x);
  const double s = x * r;
  return s + 0.5 * r * (x - s * s);
}

// Rays with C^2 = 1 - S^2 below this (within about 3 degrees of the
// horizontal) are not evaluated in float: the float closed forms and the
// float direction lose digits there. In the unfused path they are evaluated
// in double in place; the fused path hands them to a double pass. (Measured
// on the fluorescence parity set: the float rays nearest the limit, zenith
// cosines 0.05..0.07, arrive within 0.011 ns of the oracle, a ninth of the
// 0.1 ns bar; with the limit at 0.001 the nearest come within 0.041 ns.)
constexpr float kNearHorizonC2 = 0.0025f;
// Internal status of a photon left to the double pass (never reported).
constexpr int kDeferred = 7;

// C^2 = 1 - S^2 of a ray with zenith cosine ced and sine se where
// eps = n - 1 is epsd, in double. Double form: 1 - S = ce^2/(1 + se) - eps se,
// free of cancellation up to the horizon. Float form (taken to decide the
// float rays, C^2 > 0.01): ce^2 - eps (2 + eps)(1 - ce)(1 + ce), whose terms
// differ by a factor of 16 or more there.
template <typename C>
__device__ __forceinline__ double ray_c2(double ced, C se, double epsd) {
  if constexpr (sizeof(C) == 8) {
    return (ced * ced / (1.0 + se) - epsd * se) * (1.0 + (1.0 + epsd) * se);
  } else {
    return ced * ced - epsd * (2.0 + epsd) * ((1.0 - ced) * (1.0 + ced));
  }
}

// Layer pieces from the emission height ze down to h_obs in precision C.
// rho_e = rho_bot (1 + em_e) is the density at ze, se/ce the sine/cosine of
// the zenith angle at emission. Accumulates in double int dh/r (g0), the path
// and the optical path, and in C the density-weighted path (col).
// ced: cosine of the emission zenith angle in double, se its sine; the float
// form takes the dominant 1/C from C2d, C^2 in double (ray_c2).
template <typename C>
__device__ __forceinline__ void ray_pieces(const AtmDev& a, const AtmLane& L, int le, double ze, C em_e, C rho_e,
                                           C se, double ced, double C2d, double& g0, double& pth, double& opt,
                                           C& col, C& ne) {
  using F = Fm<C>;
  const C eta0 = (C)a.eta0;
  const C eps_e = eta0 * rho_e;
  ne = (C)1 + eps_e;
  const C S = ne * se;
  const C C2 = (C)C2d;
  const C Cc = C2 > (C)0 ? F::sqrt_(C2) : (C)0;
  const C invC = C2 > (C)0 ? F::rcp(Cc) : (C)0;
  // 1/C in double for the dominant (b - a)/C terms of long slant paths
  const double invCd = C2 > (C)0 ? (sizeof(C) == 8 ? (double)invC : rsqrt_refined(C2d)) : 0.0;
  const C ce = (C)ced;
  C r_top = ne * ce;  // r at ze: sqrt(ne^2 - S^2) = ne cos
  // the dominant terms (b - a)/C of the pieces add up to (ze - h_obs)/C,
  // taken once in double; a homogeneous layer's own term dh/r_a enters the
  // sum below as its difference from dh/C
  const bool cpos = C2 > (C)0;
  g0 = cpos ? (ze - a.hobs) * invCd : 0.0;
  col = (C)0;
  const C dh_e = (C)(ze - L.pc[le][kPcBot]);
  // the piece remainders and the small path and optical-path corrections,
  // summed in the working precision and added to the double totals once
  C g_sum = (C)0, lg_sum = (C)0, rd_sum = (C)0;
  // one piece: its remainder of int dh/r, the path and optical-path
  // corrections and the column go to the sums
  auto add_piece = [&](C dh, C rho_a, C em, C H_l, bool homog) {
    const C eps_a = eta0 * rho_a;
    const C ra = F::sqrt_(C2 + eps_a * ((C)2 + eps_a));
    PieceOut<C> o;
    piece_integrals<C>(rho_a, em, dh, H_l, homog, eta0, C2, Cc, invC, S, ra, r_top, o);
    // homogeneous: dh/r_a - dh/C = -dh (r_a^2 - C^2) / (r_a C (r_a + C))
    const C gm = !homog ? (C)0
                        : (cpos ? -dh * eps_a * ((C)2 + eps_a) * F::rcp(ra * Cc * (ra + Cc)) : dh * F::rcp(ra));
    g_sum += gm + o.g0c;
    lg_sum += o.lgH;
    rd_sum += o.rdH;
    col += o.col;
    r_top = ra;
  };
  if constexpr (sizeof(C) == 4) {
    // the emission layer's piece per lane, then the whole layers below it
    // with the wave-uniform layer index (lanes at or above it skip the
    // iteration), whose ray-independent terms come precomputed (LDS)
    if (dh_e > (C)0) {
      const float4 q = L.pcf[le];
      add_piece(dh_e, q.y, em_e, q.w, (a.homog_mask >> le) & 1);
    }
#pragma unroll 1
    for (int l = a.nl - 2; l >= a.l_obs; --l) {
      if (l >= le) continue;
      const bool homog = (a.homog_mask >> l) & 1;
      if (homog || !cpos) {
        const float4 q = L.pcf[l];
        add_piece(q.x, q.y, q.z, q.w, homog);
        continue;
      }
      // piece_integrals for C^2 > 0 with the layer's constants folded:
      // r_a - r_b = -d (2 + eps_a + eps_b)/(r_a + r_b), and so on
      const float4 g = L.pfg[l];  // eps_a, eps_a (2 + eps_a), d, d (2 + eps_a + eps_b)
      const float4 h = L.pfh[l];  // n_b, -H drho (2 + eps_a + eps_b), H
      const C ra = F::sqrt_(C2 + g.y);
      const C inv_rs = F::rcp(ra + r_top);
      const C rd = -g.w * inv_rs;
      const C den = Cc * ra + C2 + g.x;
      const C delta = g.z + Cc * g.w * inv_rs;
      g_sum += (h.z * invC) * F::log1p_(delta * F::rcp(den));
      lg_sum += h.z * F::log1p_((rd - g.z) * F::rcp(h.x + r_top));
      rd_sum += h.z * rd;
      col += h.y * inv_rs;
      r_top = ra;
    }
  } else {
    // the layer index runs wave-uniformly (lanes above their emission layer
    // skip the iteration); the piece constants come from the LDS record of
    // the layer (a kernel-argument array indexed under per-lane selects
    // would be read by vector loads with their full latency)
#pragma unroll 1
    for (int l = a.nl - 1; l >= a.l_obs; --l) {
      if (l > le) continue;
      const double* pc = L.pc[l];
      const C dh = (l == le) ? dh_e : (C)pc[kPcDh];
      if (!(dh > (C)0)) continue;
      add_piece(dh, (C)pc[kPcRho], (l == le) ? em_e : (C)pc[kPcEm], (C)pc[kPcH], (a.homog_mask >> l) & 1);
    }
  }
  g0 += (double)g_sum;
  pth = g0 + (double)lg_sum;
  opt = pth + (double)rd_sum;
}

// DEFER (float only): a near-horizon ray is only marked kDeferred.
// FORCE_FLOAT (float only): every ray is evaluated in float.
// The exact integrals in double of a ray from height ze (zenith cosine ced,
// sine sed) down to h_obs; em_out: expm1 of the density drop from the
// emission layer's base to ze.
__device__ __forceinline__ void exact_ray_double(const AtmDev& a, const AtmLane& L, double ze, double sed, double ced,
                                                 double& g0, double& pth, double& opt, double& col, double& ne,
                                                 double& em_out, double& rho_bot_out) {
  const int le = layer_of(a, ze);
  // the emission layer's piece record (LDS): a select between a kernel
  // argument and an LDS array would become a generic (flat) load
  const double bot = L.pc[le][kPcBot];
  const double rho_bot = L.pc[le][kPcRho];
  const bool homog_e = (a.homog_mask >> le) & 1;
  const double em_e = homog_e ? 0.0 : expm1(-(ze - bot) * L.invH[le]);
  const double rho_e = rho_bot * (1.0 + em_e);
  const double C2d = ray_c2<double>(ced, sed, a.eta0 * rho_e);
  ray_pieces<double>(a, L, le, ze, em_e, rho_e, sed, ced, C2d, g0, pth, opt, col, ne);
  em_out = em_e;
  rho_bot_out = rho_bot;
}

template <typename T>
__device__ __forceinline__ T lerp_t(T a, T b, T t) {
  return a + (b - a) * t;
}

// Straight line plus tabulated corrections (section 2) for a downward photon
// at or above h_obs (unit direction ux, uy; zenith cosine mu, its double
// value mud, sine se). The slant factor 1/mu of the dominant straight path
// is taken from the double cosine: a float cosine's rounding (6e-8) would
// become a path error of 6e-8/mu^2 relative, 0.2 ns on steep-angle rays.
// Returns false when the photon lies outside the table (above h_max or
// steeper than q_max): the caller then takes the exact integrals.
template <typename T>
__device__ __forceinline__ bool propagate_table(const AtmDev& a, const AtmLane& L, T ux, T uy, T mu, double mud,
                                                T se, Photon<T>& p) {
  using F = Fm<T>;
  const double dh = p.z - a.hobs;
  const T q = se * F::rcp(mu);
  if (!(p.z <= a.t_hmax) || !(q <= (T)a.t_qmax)) return false;
  const T fi = (T)(dh * a.t_fi), fj = q * (T)a.t_fj;
  const int i = min((int)fi, a.tn_h - 2), j = min((int)fj, a.tn_q - 2);
  const T ta = fi - (T)i, tb = fj - (T)j;
  const float4* c = a.tcorr + (size_t)i * (size_t)a.tn_q + (size_t)j;
  const float4 c00 = c[0], c01 = c[1], c10 = c[a.tn_q], c11 = c[a.tn_q + 1];
  const T g = lerp_t(lerp_t((T)c00.x, (T)c01.x, tb), lerp_t((T)c10.x, (T)c11.x, tb), ta);
  const T dP = lerp_t(lerp_t((T)c00.y, (T)c01.y, tb), lerp_t((T)c10.y, (T)c11.y, tb), ta);
  const T dX = lerp_t(lerp_t((T)c00.z, (T)c01.z, tb), lerp_t((T)c10.z, (T)c11.z, tb), ta);
  const T fk = (T)(dh * a.t_fk);
  const int k = min((int)fk, a.tn_v - 2);
  const T tk = fk - (T)k;
  const float2 v0 = a.tvert[k], v1 = a.tvert[k + 1];
  const T rho_e = lerp_t((T)v0.x, (T)v1.x, tk);
  const T VX = lerp_t((T)v0.y, (T)v1.y, tk);
  const double sec = 1.0 / mud;
  const double P = dh * sec + (double)dP;
  const T X = (T)sec * VX + dX;
  const double O = P + a.eta0 * (double)X;
  const double disp = (dh + (double)g) * sec;
  p.x = (T)((double)p.x + (double)ux * disp);
  p.y = (T)((double)p.y + (double)uy * disp);
  p.z = a.hobs;
  p.t = p.t + O * (1.0 / kC);
  p.path = P;
  p.w = F::exp_(-(abs_coeff<T>(a, L, p.lambda) * X));
  const T r = ((T)1 + (T)a.eta0 * rho_e) * (T)(1.0 / a.n_obs);
  const T sl = r * se;
  p.ux = ux * r;
  p.uy = uy * r;
  p.uz = -F::sqrt_(((T)1 - sl) * ((T)1 + sl));
  p.status = PHOTON_LANDED;
  return true;
}

// TABLE: try the straight line with corrections first (a.tcorr set).
// layer_hint: the emission layer when the caller knows it (>= 0), else -1.
template <typename T, bool DEFER = false, bool FORCE_FLOAT = false, bool TABLE = false>
__device__ __forceinline__ void propagate(const AtmDev& a, const AtmLane& L, Photon<T>& p, int layer_hint = -1) {
  using F = Fm<T>;
  if (p.status != PHOTON_LANDED) return;
  if (!(p.uz < (T)0)) {
    p.status = PHOTON_UP;
    return;
  }
  const double ze = p.z;
  if (ze < a.hobs) {
    p.status = PHOTON_BELOW;
    return;
  }
  // the float form's directions are unit to rounding (a half turn of a unit
  // vector, or drawn on the sphere): used as they are; the double form
  // renormalises
  const T inv_un = sizeof(T) == 8 ? F::rcp(F::sqrt_(p.ux * p.ux + p.uy * p.uy + p.uz * p.uz)) : (T)1;
  const T ux = p.ux * inv_un, uy = p.uy * inv_un;
  // zenith cosine and sine in double from the double vertical component
  const double ced = sizeof(T) == 8 ? -p.uzd * (double)inv_un : -p.uzd;
  const double omc = (1.0 - ced) * (1.0 + ced);
  // the sine in double only where a double pass in place needs it (the
  // float form enters it in float terms only)
  double sed = 0.0;
  T se;
  if constexpr (sizeof(T) == 8) {
    sed = sqrt(omc);
    se = sed;
  } else if constexpr (DEFER) {
    se = F::sqrt_((T)omc);
  } else {
    sed = sqrt_refined(omc);
    se = (T)sed;
  }
  const T ce = (T)ced;
  if constexpr (TABLE) {
    if (propagate_table<T>(a, L, ux, uy, ce, ced, se, p)) return;
  }
  int le = layer_hint;
  if (le < 0) le = layer_of(a, ze);
  // the emission layer's piece record (LDS): a select between a kernel
  // argument and an LDS array would become a generic (flat) load
  const double bot = L.pc[le][kPcBot];
  const double rho_bot = L.pc[le][kPcRho];
  const double invH_e = L.invH[le];
  const bool homog_e = (a.homog_mask >> le) & 1;

  T col, ne, em_out;
  double g0, pth, opt;
  bool done = false;
  if (sizeof(T) == 4) {
    // near the horizon the float closed forms lose digits: use double there
    const T em_e = homog_e ? (T)0 : F::expm1_((T)(-(ze - bot) * invH_e));
    const T rho_e = (T)rho_bot * ((T)1 + em_e);
    const T eps_e = (T)a.eta0 * rho_e;
    const double C2d = ray_c2<T>(ced, se, (double)eps_e);
    if (FORCE_FLOAT || C2d > (double)kNearHorizonC2) {
      ray_pieces<T>(a, L, le, ze, em_e, rho_e, se, ced, C2d, g0, pth, opt, col, ne);
      em_out = em_e;
      done = true;
    } else if (DEFER) {
      p.status = kDeferred;
      return;
    }
  }
  if (!done) {
    double cold, ned, emd, rbd;
    exact_ray_double(a, L, ze, sed, ced, g0, pth, opt, cold, ned, emd, rbd);
    col = (T)cold;
    ne = (T)ned;
    em_out = (T)emd;
  }
  if constexpr (sizeof(T) == 4) {
    // the horizontal displacement to float rounding (the landing point is float)
    const T disp = ne * (T)g0;
    p.x = p.x + ux * disp;
    p.y = p.y + uy * disp;
  } else {
    const double disp = (double)ne * g0;
    p.x = p.x + ux * disp;
    p.y = p.y + uy * disp;
  }
  p.z = a.hobs;
  p.t = p.t + opt * (1.0 / kC);
  p.path = pth;
  const T tau = abs_coeff<T>(a, L, p.lambda) * col;
  p.w = F::exp_(-tau);
  // arrival direction by Snell: horizontal part scaled by q = ne/n_obs and
  // u_z^2 = ce^2 + se^2 (1 - q)(1 + q), with 1 - q = eta0 (rho_obs - rho_e)/n_obs
  // formed from density differences (no cancellation near the horizon)
  const T drho = (T)(a.rho_obs - rho_bot) - (T)rho_bot * em_out;
  const T omq = (T)a.eta0 * drho * (T)(1.0 / a.n_obs);
  const T q = (T)1 - omq;
  p.ux = ux * q;
  p.uy = uy * q;
  p.uz = -F::sqrt_(ce * ce + se * se * omq * ((T)2 - omq));
  p.status = PHOTON_LANDED;
}

// ---------------------------------------------------------------------------
// Telescope test: first sphere along the straight arrival line.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int telescope_hit(const Photon<T>& p, const double (*tel)[4], int n_tel, T& s_hit) {
  int best = -1;
  T best_s = (T)INFINITY;
  for (int k = 0; k < n_tel; ++k) {
    const T ox = p.x - (T)tel[k][0], oy = p.y - (T)tel[k][1], oz = (T)(p.z - tel[k][2]);
    const T R = (T)tel[k][3];
    const T b = p.ux * ox + p.uy * oy + p.uz * oz;
    const T cc = (ox * ox + oy * oy + oz * oz) - R * R;
    const T disc = b * b - cc;
    if (disc < (T)0) continue;
    const T s = -b - Fm<T>::sqrt_(disc);
    if (s < best_s) {
      best_s = s;
      best = k;
    }
  }
  s_hit = best_s;
  return best;
}

// Same test restricted to the spheres whose bits are set in mask.
template <typename T>
__device__ __forceinline__ int telescope_hit_masked(const Photon<T>& p, const double (*tel)[4], uint32_t mask,
                                                    T& s_hit) {
  int best = -1;
  T best_s = (T)INFINITY;
  while (mask) {
    const int k = __builtin_ctz(mask);
    mask &= mask - 1u;
    const T ox = p.x - (T)tel[k][0], oy = p.y - (T)tel[k][1], oz = (T)(p.z - tel[k][2]);
    const T R = (T)tel[k][3];
    const T b = p.ux * ox + p.uy * oy + p.uz * oz;
    const T cc = (ox * ox + oy * oy + oz * oz) - R * R;
    const T disc = b * b - cc;
    if (disc < (T)0) continue;
    const T s = -b - Fm<T>::sqrt_(disc);
    if (s < best_s) {
      best_s = s;
      best = k;
    }
  }
  s_hit = best_s;
  return best;
}

// The float form on float centres (x, y, z - h_obs, R^2); pz_rel = z - h_obs
// of the photon.
__device__ __forceinline__ int telescope_hit_masked_f(const Photon<float>& p, const float (*tel)[4], float pz_rel,
                                                      uint32_t mask, float& s_hit) {
  // entry distance along the line to sphere k, or +inf when the line misses it
  auto entry = [&](int k) {
    const float4 c = *reinterpret_cast<const float4*>(tel[k]);
    const float ox = p.x - c.x, oy = p.y - c.y, oz = pz_rel - c.z;
    const float b = p.ux * ox + p.uy * oy + p.uz * oz;
    const float cc = (ox * ox + oy * oy + oz * oz) - c.w;
    const float disc = b * b - cc;
    return disc < 0.0f ? INFINITY : -b - __builtin_amdgcn_sqrtf(disc);
  };
  int best = -1;
  float best_s = INFINITY;
  // the first candidate (usually the only one) outside the loop
  if (mask) {
    const int k = __builtin_ctz(mask);
    mask &= mask - 1u;
    best_s = entry(k);
    best = best_s < INFINITY ? k : -1;
  }
  while (mask) {
    const int k = __builtin_ctz(mask);
    mask &= mask - 1u;
    const float s = entry(k);
    if (s < best_s) {
      best_s = s;
      best = k;
    }
  }
  s_hit = best_s;
  return best;
}

}  // namespace ph
