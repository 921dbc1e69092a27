/*
 * oracle.c -- plain, slow FP64 CPU oracle for the optical-photon hot path:
 * per-segment photon counts, Cherenkov and fluorescence photon generation,
 * propagation through a layered exponential atmosphere with refraction and
 * absorption, and collection on an observation plane, telescope spheres or a
 * ground grid.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library. It shares no code, header,
 * table or constant generator with the HIP library; it derives every table
 * it needs (layer base densities, yield prefactor, line CDF) itself.
 *
 * Paper: D. Baack, J.-M. Alameddine, "Comparison and efficiency of GPU
 * accelerated optical light propagation in CORSIKA 8", ICRC2023,
 * arXiv:2309.15861.  Citations below name the paper's sections/equations.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared [-fopenmp] oracle.c -lm
 * (no FMA contraction: the per-segment mean and the Poisson search must be
 * evaluated in exactly the order written, operation by operation).
 *
 * Parity status: every function here is pinned by CPU tests against closed
 * forms, published test vectors, library routines or brute force; see the
 * test files named test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- physical constants ------------------------------------------------ */
#define OR_PI 3.141592653589793
#define OR_ALPHA 7.2973525693e-3    /* fine-structure constant, CODATA 2018 */
#define OR_C_M_PER_NS 0.299792458   /* speed of light in vacuum [m/ns]    */

/* ---- counter domains of the random stream ------------------------------ */
#define OR_DOM_COUNT 0u
#define OR_DOM_CHER 1u
#define OR_DOM_FLUO 2u

/* ---- photon status codes ------------------------------------------------ */
#define OR_LANDED 0
#define OR_HIT 1
#define OR_UP 2
#define OR_BELOW 3
#define OR_OFFGRID 4
#define OR_INVALID 6

#define OR_MAX_LAYERS 8
#define OR_MAX_ABS 64

/* ------------------------------------------------------------------------ */
/* Data the oracle works on (its own definitions).                          */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_layers;               /* 1..8                                  */
  double h_base[OR_MAX_LAYERS];   /* m, h_base[0] = 0, strictly increasing */
  double H[OR_MAX_LAYERS];        /* scale height per layer, m (inf = flat)*/
  double eta0;                    /* n - 1 at h_base[0]                    */
  double h_obs;                   /* observation level, m                  */
  int32_t n_abs;                  /* 0 = no absorption                     */
  double abs_lambda[OR_MAX_ABS];  /* nm, strictly increasing               */
  double abs_k[OR_MAX_ABS];       /* 1/m at rho/rho0 = 1                   */
  double rho_base[OR_MAX_LAYERS]; /* filled by or_atm_prepare               */
} or_atmosphere;

typedef struct {
  int64_t n;
  const double *x0, *y0, *z0, *dx, *dy, *dz, *length, *beta, *t0, *dedx;
  const int32_t *charge;          /* NULL: |z| = 1                         */
  const uint32_t *shower;         /* NULL: shower 0                        */
  const uint32_t *index_in_shower;/* NULL: the segment's own index         */
} or_segments;

typedef struct {
  /* emission (generation step) */
  double xe, ye, ze, te, ue[3], lambda;
  /* propagation result */
  int32_t status;
  double xl, yl, zl, tl, ul[3], path, tau, weight;
} or_photon;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,        */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11. Ten rounds of the   */
/* 4x32 S-box with the published multipliers and Weyl key increments.        */
/* ------------------------------------------------------------------------ */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* A 32-bit word to a double strictly inside (0,1): (x + 1/2) / 2^32. */
double or_uniform(uint32_t x) { return ((double)x + 0.5) / 4294967296.0; }

static void draw4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t dom,
                  double u[4], uint32_t w[4]) {
  uint32_t ctr[4] = {c0, c1, c2, dom};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t o[4];
  or_philox(ctr, key, o);
  for (int i = 0; i < 4; ++i) {
    u[i] = or_uniform(o[i]);
    if (w) w[i] = o[i];
  }
}

/* ------------------------------------------------------------------------ */
/* The exponential wherever it decides an integer (the Poisson count, via   */
/* the refractive index at the segment midpoint and exp(-mean), and the     */
/* layer base densities those use). A library exp is only faithful to about */
/* one unit in the last place and differs between libraries, which would    */
/* let a count differ between two correct implementations. This one is a    */
/* fully specified sequence of IEEE double operations (no contraction), so  */
/* any implementation of the same steps gets the same bits:                 */
/*   k = nearest integer to x / ln 2 (ties to even);                        */
/*   r = (x - k ln2_hi) - k ln2_lo   (W. J. Cody, W. Waite, "Software Manual */
/*       for the Elementary Functions", 1980: ln 2 split so that k ln2_hi is  */
/*       exact; |r| <= ln 2 / 2);                                           */
/*   e^r = sum of r^i / i! for i = 0..13 (Taylor series; the first omitted   */
/*       term is below 5e-18 for |r| <= ln 2 / 2), by Horner from i = 13;    */
/*   exp(x) = e^r 2^k (ldexp).                                              */
/* The coefficients are 1/i! rounded to double.                             */
/* ------------------------------------------------------------------------ */
static const double OR_INV_FACT[14] = {
    1.0, 1.0, 0.5, 0x1.5555555555555p-3, 0x1.5555555555555p-5, 0x1.1111111111111p-7,
    0x1.6c16c16c16c17p-10, 0x1.a01a01a01a01ap-13, 0x1.a01a01a01a01ap-16, 0x1.71de3a556c734p-19,
    0x1.27e4fb7789f5cp-22, 0x1.ae64567f544e4p-26, 0x1.1eed8eff8d898p-29, 0x1.6124613a86d09p-33};

double or_exp_fixed(double x) {
  if (isnan(x)) return x;
  if (x > 709.78) return INFINITY;
  if (x < -745.2) return 0.0;
  const double ln2_hi = 0x1.62e42fee00000p-1;   /* 21 trailing zero bits */
  const double ln2_lo = 0x1.a39ef35793c76p-33;
  const double inv_ln2 = 0x1.71547652b82fep+0;
  double k = rint(x * inv_ln2);
  double r = (x - k * ln2_hi) - k * ln2_lo;
  double p = OR_INV_FACT[13];
  for (int i = 12; i >= 0; --i) p = p * r + OR_INV_FACT[i];
  return ldexp(p, (int)k);
}

/* ------------------------------------------------------------------------ */
/* Atmosphere: plane-parallel, piecewise exponential density, refractive    */
/* index n(h) = 1 + (n0 - 1) rho(h)/rho0. Layer i covers                     */
/* [h_base[i], h_base[i+1]); layer 0 also extends below h_base[0] and the   */
/* top layer has no upper cut. The density is continuous at the boundaries. */
/* ------------------------------------------------------------------------ */
void or_atm_prepare(or_atmosphere* a) {
  a->rho_base[0] = 1.0;
  for (int i = 0; i + 1 < a->n_layers; ++i)
    a->rho_base[i + 1] = a->rho_base[i] * or_exp_fixed(-(a->h_base[i + 1] - a->h_base[i]) / a->H[i]);
}

int or_layer_of(const or_atmosphere* a, double h) {
  int i = 0;
  for (int k = 0; k < a->n_layers; ++k)
    if (a->h_base[k] <= h) i = k;
  return i;
}

/* rho(h)/rho0 */
double or_density(const or_atmosphere* a, double h) {
  int i = or_layer_of(a, h);
  return a->rho_base[i] * exp(-(h - a->h_base[i]) / a->H[i]);
}

double or_index(const or_atmosphere* a, double h) { return 1.0 + a->eta0 * or_density(a, h); }

/* Absorption coefficient at rho/rho0 = 1: piecewise linear in lambda,
   clamped to the end values outside the table. */
double or_abs_k(const or_atmosphere* a, double lambda) {
  if (a->n_abs <= 0) return 0.0;
  if (lambda <= a->abs_lambda[0]) return a->abs_k[0];
  if (lambda >= a->abs_lambda[a->n_abs - 1]) return a->abs_k[a->n_abs - 1];
  int i = 0;
  while (!(lambda < a->abs_lambda[i + 1])) ++i;
  double f = (lambda - a->abs_lambda[i]) / (a->abs_lambda[i + 1] - a->abs_lambda[i]);
  return a->abs_k[i] + f * (a->abs_k[i + 1] - a->abs_k[i]);
}

/* ------------------------------------------------------------------------ */
/* Per-segment mean photon number.                                          */
/* ------------------------------------------------------------------------ */
static uint32_t seg_index(const or_segments* s, int64_t i) {
  return s->index_in_shower ? s->index_in_shower[i] : (uint32_t)i;
}
static uint32_t seg_shower(const or_segments* s, int64_t i) { return s->shower ? s->shower[i] : 0u; }

static int seg_valid(const or_segments* s, int64_t i) {
  double v[9] = {s->x0[i], s->y0[i], s->z0[i], s->dx[i], s->dy[i], s->dz[i],
                 s->length[i], s->beta[i], s->t0[i]};
  for (int k = 0; k < 9; ++k)
    if (!isfinite(v[k])) return 0;
  if (!(s->beta[i] > 0.0 && s->beta[i] < 1.0)) return 0;
  if (!(s->length[i] >= 0.0)) return 0;
  double dn2 = (s->dx[i] * s->dx[i] + s->dy[i] * s->dy[i]) + s->dz[i] * s->dz[i];
  if (!(dn2 > 0.0)) return 0;
  return 1;
}

/* Refractive index for a segment: the step is short enough that the medium
   is taken as homogeneous along it (section 1.2, text after the Frank-Tamm
   formula); the value used is n at the height of the segment midpoint.
   Fixed evaluation order, no contraction. */
double or_segment_index(const or_segments* s, int64_t i, const or_atmosphere* a) {
  double dx = s->dx[i], dy = s->dy[i], dz = s->dz[i];
  double dn = sqrt((dx * dx + dy * dy) + dz * dz);
  double dzh = dz / dn;
  double zc = s->z0[i] + (0.5 * s->length[i]) * dzh;
  int l = 0;
  for (int k = 0; k < a->n_layers; ++k)
    if (a->h_base[k] <= zc) l = k;
  double rho = a->rho_base[l] * or_exp_fixed(-(zc - a->h_base[l]) / a->H[l]);
  return 1.0 + a->eta0 * rho;
}

/* Frank-Tamm prefactor (section 1.2 equation): mu_r pi z^2 e^2/(h eps0 c0)
   = 2 pi alpha z^2 for mu_r = 1, times the wavelength integral of 1/lambda^2
   over [lambda1, lambda2] (n does not depend on lambda) in 1/m. */
double or_frank_tamm_K(double lambda_min_nm, double lambda_max_nm) {
  return (2.0 * OR_PI * OR_ALPHA) * ((1e9 / lambda_min_nm) - (1e9 / lambda_max_nm));
}

/* Mean Cherenkov photon number of a segment: the Frank-Tamm formula
   (section 1.2) integrated over the segment length with n constant along
   it; the step function gives zero below threshold (beta n <= 1). */
double or_mean_cherenkov(const or_segments* s, int64_t i, const or_atmosphere* a, double K) {
  if (!seg_valid(s, i)) return 0.0;
  double n = or_segment_index(s, i, a);
  double bn = s->beta[i] * n;
  double f = 1.0 - 1.0 / (bn * bn);
  double zz = 1.0;
  if (s->charge) zz = (double)(s->charge[i] * s->charge[i]);
  return (f > 0.0) ? ((K * zz) * s->length[i]) * f : 0.0;
}

/* Mean fluorescence photon number (section 1.1 equation dN/dx = Y dE/dx with
   a constant yield Y and dE/dx the segment's total energy loss per metre). */
double or_mean_fluor(const or_segments* s, int64_t i, double yield_per_MeV) {
  if (!seg_valid(s, i) || !s->dedx || !isfinite(s->dedx[i]) || s->dedx[i] < 0.0) return 0.0;
  return (yield_per_MeV * s->dedx[i]) * s->length[i];
}

/* Poisson(mu) count by sequential inverse CDF on the COUNT stream.
   mu is split into m equal chunks of at most 128 (exp(-mu) would underflow
   for large mu); each chunk draws the smallest k with F(k) >= u, F the
   Poisson(mu/m) CDF summed term by term p_k = (p_{k-1} * mc) * (1/k), with
   1/k rounded to double and p_0 = exp(-mc) by or_exp_fixed. The sum of m
   independent Poisson(mu/m) variates is Poisson(mu).
   *margin receives min over chunks of |u - F(k)| at the accepted k and at
   k-1 (how close the decision was). */
#define OR_POISSON_CHUNK 128.0
#define OR_POISSON_KMAX 1000u
#define OR_MAX_MEAN 1e7  /* larger means mark the segment invalid: no photons */
uint32_t or_poisson(double mu, uint64_t seed, uint32_t idx, uint32_t shower, double* margin) {
  double best = INFINITY;
  if (!(mu > 0.0) || !(mu <= OR_MAX_MEAN)) {
    if (margin) *margin = best;
    return 0u;
  }
  uint32_t m = (mu <= OR_POISSON_CHUNK) ? 1u : (uint32_t)ceil(mu / OR_POISSON_CHUNK);
  double mc = mu / (double)m;
  uint32_t total = 0;
  for (uint32_t c = 0; c < m; ++c) {
    double u[4];
    draw4(seed, c, idx, shower, OR_DOM_COUNT, u, 0);
    uint32_t k = 0;
    double p = or_exp_fixed(-mc);
    double F = p, Fprev = 0.0;
    while (u[0] > F && k < OR_POISSON_KMAX) {
      k += 1;
      p = (p * mc) * (1.0 / (double)k);
      Fprev = F;
      F = F + p;
    }
    double d1 = fabs(u[0] - F), d0 = fabs(u[0] - Fprev);
    if (d1 < best) best = d1;
    if (k > 0 && d0 < best) best = d0;
    total += k;
  }
  if (margin) *margin = best;
  return total;
}

/* kind 0 = Cherenkov (params: lambda_min_nm, lambda_max_nm),
   kind 1 = fluorescence (params: yield per MeV). */
void or_counts(const or_segments* s, const or_atmosphere* a, int kind, const double* params,
               uint64_t seed, uint32_t* counts, double* mu_out, double* margin_out) {
  double K = (kind == 0) ? or_frank_tamm_K(params[0], params[1]) : 0.0;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < s->n; ++i) {
    double mu = (kind == 0) ? or_mean_cherenkov(s, i, a, K) : or_mean_fluor(s, i, params[0]);
    double mg;
    counts[i] = or_poisson(mu, seed, seg_index(s, i), seg_shower(s, i), &mg);
    if (mu_out) mu_out[i] = mu;
    if (margin_out) margin_out[i] = mg;
  }
}

/* Cherenkov angular particle cut (section 1.2.1, optimisation): a particle
   is handled only when the angle between its flight direction and the
   vector from its position to the experiment centre (or to one of the
   telescopes) is at most the cut angle. The position is the segment
   midpoint; angle <= cut is tested as d.v >= cos(cut) |v|. */
int or_passes_cut(const or_segments* s, int64_t i, int32_t n_pts, double cos_cut, const double* pts) {
  if (n_pts <= 0) return 1;
  double dx = s->dx[i], dy = s->dy[i], dz = s->dz[i];
  double dn = sqrt((dx * dx + dy * dy) + dz * dz);
  double ux = dx / dn, uy = dy / dn, uz = dz / dn;
  double hl = 0.5 * s->length[i];
  double mx = s->x0[i] + hl * ux, my = s->y0[i] + hl * uy, mz = s->z0[i] + hl * uz;
  for (int32_t k = 0; k < n_pts; ++k) {
    double vx = pts[3 * k] - mx, vy = pts[3 * k + 1] - my, vz = pts[3 * k + 2] - mz;
    double dot = (ux * vx + uy * vy) + uz * vz;
    double nv = sqrt((vx * vx + vy * vy) + vz * vz);
    if (dot >= cos_cut * nv) return 1;
  }
  return 0;
}

/* Fluorescence beaming (section 1.1.1, optimisation): instead of emitting
   isotropically, a track emits into a cone that contains an emission area
   enclosing every telescope, and its photon number is scaled by the cone's
   solid-angle fraction. The area is a sphere beam = (cx, cy, cz, R); the
   margin beam[4] (radians) widens the cone for the bending of rays by
   refraction. Seen from the track midpoint m, at distance D from the
   centre, the sphere grown by half the track length subtends the half
   angle alpha with sin(alpha) = (R + L/2)/D; the grown sphere seen from m
   contains the sphere seen from every point of the track. The cone has half
   angle alpha + margin about the unit vector from m to the centre; om is
   1 - cos(alpha + margin) and the solid-angle fraction om/2. A track inside
   the grown sphere (R + L/2 >= D) stays isotropic: om = 2, axis straight
   down. Returns 1 when beamed. */
int or_beam_cap(const or_segments* s, int64_t i, const double* beam, double* om, double* axis) {
  double dx = s->dx[i], dy = s->dy[i], dz = s->dz[i];
  double dn = sqrt((dx * dx + dy * dy) + dz * dz);
  double ux = dx / dn, uy = dy / dn, uz = dz / dn;
  double hl = 0.5 * s->length[i];
  double mx = s->x0[i] + hl * ux, my = s->y0[i] + hl * uy, mz = s->z0[i] + hl * uz;
  double vx = beam[0] - mx, vy = beam[1] - my, vz = beam[2] - mz;
  double D = sqrt((vx * vx + vy * vy) + vz * vz);
  double reach = beam[3] + hl;
  if (!(reach < D)) {
    *om = 2.0;
    axis[0] = 0.0; axis[1] = 0.0; axis[2] = -1.0;
    return 0;
  }
  double sa = reach / D;
  double ca = sqrt((1.0 - sa) * (1.0 + sa));
  double cb = ca * cos(beam[4]) - sa * sin(beam[4]);
  *om = 1.0 - cb;
  axis[0] = vx / D; axis[1] = vy / D; axis[2] = vz / D;
  return 1;
}

/* Counts with the angular cut applied to Cherenkov segments (n_pts > 0)
   and beaming applied to fluorescence segments (beam != NULL). */
void or_counts_ex(const or_segments* s, const or_atmosphere* a, int kind, const double* params, uint64_t seed,
                  int32_t n_pts, double cos_cut, const double* pts, const double* beam, uint32_t* counts,
                  double* mu_out, double* margin_out) {
  double K = (kind == 0) ? or_frank_tamm_K(params[0], params[1]) : 0.0;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < s->n; ++i) {
    double mu;
    if (kind == 0) {
      mu = or_passes_cut(s, i, n_pts, cos_cut, pts) ? or_mean_cherenkov(s, i, a, K) : 0.0;
    } else {
      mu = or_mean_fluor(s, i, params[0]);
      if (beam && mu > 0.0) {
        double om, ax[3];
        or_beam_cap(s, i, beam, &om, ax);
        mu = mu * (0.5 * om);
      }
    }
    double mg;
    counts[i] = or_poisson(mu, seed, seg_index(s, i), seg_shower(s, i), &mg);
    if (mu_out) mu_out[i] = mu;
    if (margin_out) margin_out[i] = mg;
  }
}

/* ------------------------------------------------------------------------ */
/* Photon generation.                                                       */
/* ------------------------------------------------------------------------ */

/* Emission point uniform along the track (section 1.1 "randomly distributed
   along the track"; section 1.2 emission point), time from the particle
   speed. */
static void emission_point(const or_segments* s, int64_t i, double u0, or_photon* p) {
  double dx = s->dx[i], dy = s->dy[i], dz = s->dz[i];
  double dn = sqrt((dx * dx + dy * dy) + dz * dz);
  double along = u0 * s->length[i];
  p->xe = s->x0[i] + along * (dx / dn);
  p->ye = s->y0[i] + along * (dy / dn);
  p->ze = s->z0[i] + along * (dz / dn);
  p->te = s->t0[i] + along / (s->beta[i] * OR_C_M_PER_NS);
}

/* The rotation of section 1.2.1: M_Rod = 1 + 2 R_Rod^2 with R_Rod the cross
   product matrix of the unit vector A bisecting the particle direction and
   the downward normal (0,0,-1); M_Rod = 2 A A^T - 1 is the half turn about A
   and maps (0,0,-1) onto the particle direction. The matrix is written out
   entry by entry exactly as printed in section 1.2.1. For a direction
   pointing straight up the bisector vanishes; any half turn about a
   horizontal axis is then correct and the one about x is used. */
void or_rotation_matrix(double dxh, double dyh, double dzh, double M[9]) {
  double ax = dxh, ay = dyh, az = dzh - 1.0;
  double an = sqrt((ax * ax + ay * ay) + az * az);
  if (!(an > 0.0)) {
    ax = 1.0; ay = 0.0; az = 0.0;
  } else {
    ax /= an; ay /= an; az /= an;
  }
  M[0] = -2.0 * ay * ay - 2.0 * az * az + 1.0;
  M[1] = 2.0 * ax * ay;
  M[2] = 2.0 * ax * az;
  M[3] = 2.0 * ax * ay;
  M[4] = -2.0 * ax * ax - 2.0 * az * az + 1.0;
  M[5] = 2.0 * ay * az;
  M[6] = 2.0 * ax * az;
  M[7] = 2.0 * ay * az;
  M[8] = -2.0 * ax * ax - 2.0 * ay * ay + 1.0;
}

/* j-th Cherenkov photon of segment i (section 1.2, Fig. 1): generated
   downward at the origin on the cone of half angle Theta_c with
   cos Theta_c = 1/(beta n), random azimuth c_rng; the photon vector of
   section 1.2.1 is rotated by M_Rod into the track frame, then moved to the
   emission point. Wavelength from the 1/lambda^2 spectrum of the Frank-Tamm
   integrand by inverse CDF. */
void or_gen_cherenkov_one(const or_segments* s, int64_t i, uint32_t j, const or_atmosphere* a,
                          double lambda_min_nm, double lambda_max_nm, uint64_t seed,
                          or_photon* p) {
  memset(p, 0, sizeof(*p));
  double u[4];
  draw4(seed, j, seg_index(s, i), seg_shower(s, i), OR_DOM_CHER, u, 0);
  emission_point(s, i, u[0], p);

  double n = or_segment_index(s, i, a);
  double cos_c = 1.0 / (s->beta[i] * n);
  double sin_c = sqrt((1.0 - cos_c) * (1.0 + cos_c));
  double c_rng = 2.0 * OR_PI * u[1];
  double pv[3] = {cos(c_rng) * sin_c, sin(c_rng) * sin_c, -cos_c};

  double dx = s->dx[i], dy = s->dy[i], dz = s->dz[i];
  double dn = sqrt((dx * dx + dy * dy) + dz * dz);
  double M[9];
  or_rotation_matrix(dx / dn, dy / dn, dz / dn, M);
  for (int r = 0; r < 3; ++r) p->ue[r] = M[3 * r] * pv[0] + M[3 * r + 1] * pv[1] + M[3 * r + 2] * pv[2];

  double inv1 = 1.0 / lambda_min_nm, inv2 = 1.0 / lambda_max_nm;
  p->lambda = 1.0 / (inv1 - u[2] * (inv1 - inv2));
  p->status = OR_LANDED;
}

/* Normalised cumulative line yields, summed in index order; the last entry
   is exactly 1. */
void or_line_cdf(const double* rel_yield, int32_t n_lines, double* cdf) {
  double acc = 0.0;
  for (int k = 0; k < n_lines; ++k) {
    acc = acc + rel_yield[k];
    cdf[k] = acc;
  }
  for (int k = 0; k < n_lines; ++k) cdf[k] = cdf[k] / acc;
  cdf[n_lines - 1] = 1.0;
}

/* j-th fluorescence photon of segment i (section 1.1): isotropic direction,
   emission point uniform along the track, emission line drawn with
   probability proportional to its relative yield. With beaming (beam !=
   NULL, section 1.1.1) the direction is uniform on the cone of or_beam_cap:
   1 - cos(theta) = u1 om from the cone axis, azimuth 2 pi u2, generated
   about the downward normal and turned onto the axis by the half turn of
   or_rotation_matrix (which maps (0,0,-1) onto the axis). */
void or_gen_fluor_one(const or_segments* s, int64_t i, uint32_t j, const double* line_nm,
                      const double* cdf, int32_t n_lines, uint64_t seed, const double* beam, or_photon* p) {
  memset(p, 0, sizeof(*p));
  double u[4];
  draw4(seed, j, seg_index(s, i), seg_shower(s, i), OR_DOM_FLUO, u, 0);
  emission_point(s, i, u[0], p);
  if (beam) {
    double om, ax[3], M[9];
    or_beam_cap(s, i, beam, &om, ax);
    double v = u[1] * om;
    double ct = 1.0 - v;
    double st = sqrt(v * (2.0 - v));
    double ph = 2.0 * OR_PI * u[2];
    double pv[3] = {st * cos(ph), st * sin(ph), -ct};
    or_rotation_matrix(ax[0], ax[1], ax[2], M);
    for (int r = 0; r < 3; ++r) p->ue[r] = M[3 * r] * pv[0] + M[3 * r + 1] * pv[1] + M[3 * r + 2] * pv[2];
  } else {
    double ct = 1.0 - 2.0 * u[1];
    double st = sqrt((1.0 - ct) * (1.0 + ct));
    double ph = 2.0 * OR_PI * u[2];
    p->ue[0] = st * cos(ph);
    p->ue[1] = st * sin(ph);
    p->ue[2] = ct;
  }
  int k = 0;
  while (k < n_lines - 1 && !(u[3] < cdf[k])) ++k;
  p->lambda = line_nm[k];
  p->status = OR_LANDED;
}

/* ------------------------------------------------------------------------ */
/* Propagation (section 2): the photon is carried from its emission point   */
/* to the observation level through the refracting atmosphere. In a         */
/* plane-parallel medium n(h) sin(theta(h)) = S is conserved (Snell), and   */
/* along the ray, per unit height,                                          */
/*   horizontal displacement  dX/dh = S / r,                                */
/*   geometric length         dP/dh = n / r,                                */
/*   optical length           dO/dh = n^2 / r,                              */
/*   density-weighted length  dT/dh = (rho/rho0) n / r,                      */
/* with r = sqrt(n^2 - S^2). The oracle integrates these plain integrands   */
/* by adaptive Gauss-Kronrod (7,15) quadrature layer piece by layer piece.  */
/* ------------------------------------------------------------------------ */

/* Kronrod 15-point nodes/weights and the embedded 7-point Gauss weights
   (QUADPACK qk15 values). */
static const double XGK[8] = {0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
                              0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
                              0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
                              0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double WGK[8] = {0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
                              0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
                              0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
                              0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
static const double WG[4] = {0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
                             0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

typedef struct {
  const or_atmosphere* a;
  int layer;              /* layer of the piece being integrated          */
  int layer_e;            /* layer of the emission height                 */
  double ze, ne, rho_e, ce;  /* emission height, index, density, |cos|   */
} ray_ctx;

/* rho(h) - rho(z_e) for h <= z_e, written as a sum of positive per-layer
   increments rho(lower) - rho(upper) = rho(upper) expm1(dh/H), so that it
   keeps full relative precision when h is close to z_e. */
static double density_rise(const ray_ctx* c, double h) {
  const or_atmosphere* a = c->a;
  int l = c->layer, le = c->layer_e;
  if (l == le) return c->rho_e * expm1((c->ze - h) / a->H[l]);
  double d = a->rho_base[l + 1] * expm1((a->h_base[l + 1] - h) / a->H[l]);
  for (int k = l + 1; k < le; ++k) d += a->rho_base[k + 1] * expm1((a->h_base[k + 1] - a->h_base[k]) / a->H[k]);
  d += c->rho_e * expm1((c->ze - a->h_base[le]) / a->H[le]);
  return d;
}

static void integrand(const ray_ctx* c, double h, double f[4]) {
  double drho = density_rise(c, h);
  double rho = c->rho_e + drho;
  double n = 1.0 + c->a->eta0 * rho;
  /* n^2 - S^2 = ne^2 cos^2 + (n - ne)(n + ne), with n - ne = eta0 (rho - rho_e) */
  double r2 = c->ne * c->ne * c->ce * c->ce + c->a->eta0 * drho * (n + c->ne);
  double r = sqrt(r2);
  f[0] = 1.0 / r;
  f[1] = n / r;
  f[2] = n * n / r;
  f[3] = rho * n / r;
}

static void gk15(const ray_ctx* c, double lo, double hi, double K[4], double E[4]) {
  double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
  double fc[4];
  integrand(c, mid, fc);
  double g[4], k[4];
  for (int q = 0; q < 4; ++q) {
    g[q] = WG[3] * fc[q];
    k[q] = WGK[7] * fc[q];
  }
  for (int j = 0; j < 7; ++j) {
    double f1[4], f2[4];
    integrand(c, mid - half * XGK[j], f1);
    integrand(c, mid + half * XGK[j], f2);
    for (int q = 0; q < 4; ++q) {
      k[q] += WGK[j] * (f1[q] + f2[q]);
      if (j % 2 == 1) g[q] += WG[j / 2] * (f1[q] + f2[q]);
    }
  }
  for (int q = 0; q < 4; ++q) {
    K[q] = k[q] * half;
    E[q] = fabs((k[q] - g[q]) * half);
  }
}

/* Globally adaptive quadrature over one layer piece: keep bisecting the
   interval with the largest error estimate until the summed estimate is
   below 1e-13 of the integral for all four integrands, or the budget of
   GK_LIMIT intervals is used (rounding noise of the integrand then bounds
   the accuracy, about 1e-12 for rays within 1e-4 of the horizontal). */
#define GK_LIMIT 400
static void integrate_piece(const ray_ctx* c, double lo, double hi, double acc[4]) {
  static _Thread_local double A[GK_LIMIT], B[GK_LIMIT], K[GK_LIMIT][4], E[GK_LIMIT][4];
  int m = 1;
  A[0] = lo;
  B[0] = hi;
  gk15(c, lo, hi, K[0], E[0]);
  for (;;) {
    double tot[4] = {0, 0, 0, 0}, err[4] = {0, 0, 0, 0};
    for (int i = 0; i < m; ++i)
      for (int q = 0; q < 4; ++q) {
        tot[q] += K[i][q];
        err[q] += E[i][q];
      }
    int ok = 1;
    for (int q = 0; q < 4; ++q)
      if (err[q] > 1e-13 * fabs(tot[q])) ok = 0;
    if (ok || m >= GK_LIMIT) {
      for (int q = 0; q < 4; ++q) acc[q] += tot[q];
      return;
    }
    int w = 0;
    double wmax = -1.0;
    for (int i = 0; i < m; ++i) {
      double e = 0.0;
      for (int q = 0; q < 4; ++q) {
        double rel = E[i][q] / fabs(tot[q]);
        if (rel > e) e = rel;
      }
      if (e > wmax) {
        wmax = e;
        w = i;
      }
    }
    double mid = 0.5 * (A[w] + B[w]);
    A[m] = mid;
    B[m] = B[w];
    B[w] = mid;
    gk15(c, A[w], B[w], K[w], E[w]);
    gk15(c, A[m], B[m], K[m], E[m]);
    ++m;
  }
}

/* Integrals G = (int dh/r, int n/r dh, int n^2/r dh, int rho n/r dh) from
   h_lo up to the emission height ze, split at layer boundaries. */
void or_ray_integrals(const or_atmosphere* a, double ze, double ce, double h_lo, double G[4]) {
  for (int q = 0; q < 4; ++q) G[q] = 0.0;
  int le = or_layer_of(a, ze);
  double rho_e = or_density(a, ze);
  double ne = 1.0 + a->eta0 * rho_e;
  for (int l = 0; l <= le; ++l) {
    double lo = (l == 0) ? -INFINITY : a->h_base[l];
    double hi = (l < le) ? a->h_base[l + 1] : ze;
    if (lo < h_lo) lo = h_lo;
    if (!(lo < hi)) continue;
    ray_ctx c = {a, l, le, ze, ne, rho_e, ce};
    integrate_piece(&c, lo, hi, G);
  }
}

/* Carries an emitted photon to the observation level h_obs. */
void or_propagate_one(or_photon* p, const or_atmosphere* a) {
  if (p->status == OR_INVALID) return;
  double un = sqrt((p->ue[0] * p->ue[0] + p->ue[1] * p->ue[1]) + p->ue[2] * p->ue[2]);
  double ux = p->ue[0] / un, uy = p->ue[1] / un, uz = p->ue[2] / un;
  if (!(uz < 0.0)) { p->status = OR_UP; return; }
  if (p->ze < a->h_obs) { p->status = OR_BELOW; return; }

  double ne = or_index(a, p->ze);
  double nobs = or_index(a, a->h_obs);
  double G[4];
  or_ray_integrals(a, p->ze, -uz, a->h_obs, G);

  /* horizontal displacement S*G0 along the unit horizontal direction
     (ux,uy)/sin; with S = ne*sin this is (ux,uy)*ne*G0 */
  p->xl = p->xe + ux * ne * G[0];
  p->yl = p->ye + uy * ne * G[0];
  p->zl = a->h_obs;
  p->tl = p->te + G[2] / OR_C_M_PER_NS;
  p->path = G[1];
  p->tau = or_abs_k(a, p->lambda) * G[3];
  p->weight = exp(-p->tau);
  /* arrival direction: Snell, n_e sin_e = n_obs sin_obs, azimuth kept */
  double q = ne / nobs;
  p->ul[0] = ux * q;
  p->ul[1] = uy * q;
  double sl2 = p->ul[0] * p->ul[0] + p->ul[1] * p->ul[1];
  p->ul[2] = -sqrt((1.0 - sl2));
  p->status = OR_LANDED;
}

/* ------------------------------------------------------------------------ */
/* Collection.                                                              */
/* ------------------------------------------------------------------------ */

/* Telescope spheres (centre x,y,z, radius R per row of tel): the photon hits
   a sphere when the straight line through its landing point along its
   arrival direction meets the sphere; the entry point (smaller root of the
   line parameter s) of the first sphere along the ray is recorded, with
   time t_l + n_obs s / c. Returns the sphere index or -1. */
int or_telescope_one(const or_photon* p, const double* tel, int32_t n_tel, double n_obs,
                     double hit[5]) {
  if (p->status != OR_LANDED) return -1;
  int best = -1;
  double best_s = INFINITY;
  for (int k = 0; k < n_tel; ++k) {
    double ox = p->xl - tel[4 * k], oy = p->yl - tel[4 * k + 1], oz = p->zl - tel[4 * k + 2];
    double R = tel[4 * k + 3];
    double b = p->ul[0] * ox + p->ul[1] * oy + p->ul[2] * oz;
    double cc = (ox * ox + oy * oy + oz * oz) - R * R;
    double disc = b * b - cc;
    if (disc < 0.0) continue;
    double s = -b - sqrt(disc);
    if (s < best_s) {
      best_s = s;
      best = k;
    }
  }
  if (best >= 0) {
    hit[0] = p->xl + best_s * p->ul[0];
    hit[1] = p->yl + best_s * p->ul[1];
    hit[2] = p->zl + best_s * p->ul[2];
    hit[3] = p->tl + n_obs * best_s / OR_C_M_PER_NS;
    hit[4] = best_s;
  }
  return best;
}

/* Ground grid: half-open cells [x_min + i*cell, x_min + (i+1)*cell). */
int32_t or_grid_cell(const or_photon* p, double x_min, double y_min, double cell, int32_t nx,
                     int32_t ny) {
  if (p->status != OR_LANDED) return -1;
  double fx = floor((p->xl - x_min) / cell), fy = floor((p->yl - y_min) / cell);
  if (fx < 0.0 || fy < 0.0 || fx >= (double)nx || fy >= (double)ny) return -1;
  return (int32_t)fy * nx + (int32_t)fx;
}

/* ------------------------------------------------------------------------ */
/* Straight line plus correction factors (section 2): the fast propagation  */
/* of the paper. A photon is carried to the observation level along a       */
/* straight line at its emission zenith angle; tabulated corrections then   */
/* move its landing point, path, optical path and column density to what   */
/* the refracting atmosphere gives, and the arrival angle follows Snell.    */
/*                                                                          */
/* Tables, built from the exact integrals at their nodes:                   */
/*  2-D over emission height h_i = h_obs + (h_max - h_obs) i/(n_h - 1) and  */
/*  q_j = tan(zenith) = q_max j/(n_q - 1), three values per node:           */
/*    g  = (D - dh q)/q  (horizontal displacement D; at q = 0 the limit,    */
/*         taken at q = 1e-4 q_max),                                        */
/*    dP = P - dh sec,   dX = X - sec VX(h_i)                               */
/*  with dh = h_i - h_obs, sec = sqrt(1 + q^2), P the geometric path and X  */
/*  the column (integral of rho/rho0 ds);                                   */
/*  1-D over height v_k = h_obs + (h_max - h_obs) k/(n_v - 1): rho/rho0 and */
/*  the vertical column VX(v_k) from h_obs.                                 */
/* A photon then lands at x_e + ux (dh + g)/mu (mu = -uz), with path        */
/* dh sec + dP, column sec VX(h_e) + dX, optical path path + eta0 column;    */
/* values between nodes by bilinear (2-D) and linear (1-D) interpolation.    */
/* Photons above h_max or steeper than q_max take the exact integrals.      */
/* ------------------------------------------------------------------------ */

static void node_integrals(const or_atmosphere* a, double h, double q, double G[4], double* D) {
  double ce = 1.0 / sqrt(1.0 + q * q);
  double se = q * ce;
  or_ray_integrals(a, h, ce, a->h_obs, G);
  *D = or_index(a, h) * se * G[0];
}

void or_table_build(const or_atmosphere* a, int32_t n_h, int32_t n_q, double h_max, double q_max, int32_t n_v,
                    double* corr, double* vert) {
  double span = h_max - a->h_obs;
#pragma omp parallel for schedule(dynamic, 4)
  for (int32_t i = 0; i < n_h; ++i) {
    double h = a->h_obs + span * ((double)i / (double)(n_h - 1));
    double dh = h - a->h_obs;
    double Gv[4], Dv;
    node_integrals(a, h, 0.0, Gv, &Dv);
    double VX = Gv[3];
    for (int32_t j = 0; j < n_q; ++j) {
      double q = q_max * ((double)j / (double)(n_q - 1));
      double G[4], D, *c = corr + 3 * ((int64_t)i * n_q + j);
      if (dh <= 0.0) { c[0] = c[1] = c[2] = 0.0; continue; }
      if (j == 0) {
        double qs = 1e-4 * q_max, G2[4], D2;
        node_integrals(a, h, qs, G2, &D2);
        c[0] = (D2 - dh * qs) / qs;
      }
      node_integrals(a, h, q, G, &D);
      double sec = sqrt(1.0 + q * q);
      if (j > 0) c[0] = (D - dh * q) / q;
      c[1] = G[1] - dh * sec;
      c[2] = G[3] - sec * VX;
    }
  }
  for (int32_t k = 0; k < n_v; ++k) {
    double h = a->h_obs + span * ((double)k / (double)(n_v - 1));
    double G[4], D;
    node_integrals(a, h, 0.0, G, &D);
    vert[2 * k] = or_density(a, h);
    vert[2 * k + 1] = (h > a->h_obs) ? G[3] : 0.0;
  }
}

static double lerp(double a, double b, double t) { return a + (b - a) * t; }

void or_propagate_table_one(or_photon* p, const or_atmosphere* a, int32_t n_h, int32_t n_q, double h_max,
                            double q_max, int32_t n_v, const double* corr, const double* vert) {
  if (p->status == OR_INVALID) return;
  double un = sqrt((p->ue[0] * p->ue[0] + p->ue[1] * p->ue[1]) + p->ue[2] * p->ue[2]);
  double ux = p->ue[0] / un, uy = p->ue[1] / un, uz = p->ue[2] / un;
  if (!(uz < 0.0)) { p->status = OR_UP; return; }
  if (p->ze < a->h_obs) { p->status = OR_BELOW; return; }
  double mu = -uz;
  double se = sqrt(ux * ux + uy * uy);
  double q = se / mu;
  if (p->ze > h_max || q > q_max) { or_propagate_one(p, a); return; }
  double span = h_max - a->h_obs;
  double dh = p->ze - a->h_obs;
  double sec = 1.0 / mu;
  /* cell and weights */
  double fi = dh / span * (double)(n_h - 1), fj = q / q_max * (double)(n_q - 1);
  int32_t i = (int32_t)floor(fi), j = (int32_t)floor(fj);
  if (i > n_h - 2) i = n_h - 2;
  if (j > n_q - 2) j = n_q - 2;
  double ta = fi - i, tb = fj - j;
  double val[3];
  for (int c = 0; c < 3; ++c) {
    double v00 = corr[3 * ((int64_t)i * n_q + j) + c], v01 = corr[3 * ((int64_t)i * n_q + j + 1) + c];
    double v10 = corr[3 * ((int64_t)(i + 1) * n_q + j) + c], v11 = corr[3 * ((int64_t)(i + 1) * n_q + j + 1) + c];
    val[c] = lerp(lerp(v00, v01, tb), lerp(v10, v11, tb), ta);
  }
  double fk = dh / span * (double)(n_v - 1);
  int32_t k = (int32_t)floor(fk);
  if (k > n_v - 2) k = n_v - 2;
  double tk = fk - k;
  double rho_e = lerp(vert[2 * k], vert[2 * k + 2], tk);
  double VX = lerp(vert[2 * k + 1], vert[2 * k + 3], tk);
  double P = dh * sec + val[1];
  double X = sec * VX + val[2];
  double O = P + a->eta0 * X;
  p->xl = p->xe + ux * (dh + val[0]) / mu;
  p->yl = p->ye + uy * (dh + val[0]) / mu;
  p->zl = a->h_obs;
  p->tl = p->te + O / OR_C_M_PER_NS;
  p->path = P;
  p->tau = or_abs_k(a, p->lambda) * X;
  p->weight = exp(-p->tau);
  /* arrival direction: Snell with the interpolated emission index */
  double ne = 1.0 + a->eta0 * rho_e, nobs = or_index(a, a->h_obs);
  double r = ne / nobs;
  double sl = r * se;
  p->ul[0] = ux * r;
  p->ul[1] = uy * r;
  p->ul[2] = -sqrt((1.0 - sl) * (1.0 + sl));
  p->status = OR_LANDED;
}

/* ------------------------------------------------------------------------ */
/* Batch drivers.                                                           */
/* ------------------------------------------------------------------------ */

/* Generates and propagates photons (s_list[q], j_list[q]) for q < count. */
void or_photons(const or_segments* s, const or_atmosphere* a, int kind, const double* params,
                const double* line_nm, const double* line_rel, int32_t n_lines, uint64_t seed,
                const double* beam, const int64_t* s_list, const uint32_t* j_list, int64_t count,
                or_photon* out) {
  double cdf[64];
  if (kind == 1) or_line_cdf(line_rel, n_lines, cdf);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t q = 0; q < count; ++q) {
    int64_t i = s_list[q];
    if (kind == 0)
      or_gen_cherenkov_one(s, i, j_list[q], a, params[0], params[1], seed, &out[q]);
    else
      or_gen_fluor_one(s, i, j_list[q], line_nm, cdf, n_lines, seed, beam, &out[q]);
    or_propagate_one(&out[q], a);
  }
}

/* Every photon of every segment, in slot order given by offsets (n+1). */
void or_photons_all(const or_segments* s, const or_atmosphere* a, int kind, const double* params,
                    const double* line_nm, const double* line_rel, int32_t n_lines,
                    uint64_t seed, const double* beam, const uint64_t* offsets, or_photon* out) {
  double cdf[64];
  if (kind == 1) or_line_cdf(line_rel, n_lines, cdf);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < s->n; ++i) {
    for (uint64_t q = offsets[i]; q < offsets[i + 1]; ++q) {
      uint32_t j = (uint32_t)(q - offsets[i]);
      if (kind == 0)
        or_gen_cherenkov_one(s, i, j, a, params[0], params[1], seed, &out[q]);
      else
        or_gen_fluor_one(s, i, j, line_nm, cdf, n_lines, seed, beam, &out[q]);
      or_propagate_one(&out[q], a);
    }
  }
}

/* Radial profile bin of each photon (section 3.1: density and mean
   arrival time in rings about the shower core): the k with
   edges[k] <= r < edges[k+1], r the distance of the landing point from
   (cx, cy); -1 for photons that did not land or fall outside the edges.
   Found by bisection over the n_bins + 1 increasing edges. */
void or_radial_bins(const or_photon* ph, int64_t count, double cx, double cy, const double* edges, int32_t n_bins,
                    int32_t* bin) {
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < count; ++q) {
    bin[q] = -1;
    if (ph[q].status != OR_LANDED) continue;
    double dx = ph[q].xl - cx, dy = ph[q].yl - cy;
    double r = sqrt(dx * dx + dy * dy);
    if (!(r >= edges[0]) || !(r < edges[n_bins])) continue;
    int32_t lo = 0, hi = n_bins; /* edges[lo] <= r < edges[hi] */
    while (hi - lo > 1) {
      int32_t mid = (lo + hi) / 2;
      if (edges[mid] <= r) lo = mid; else hi = mid;
    }
    bin[q] = lo;
  }
}

/* Propagates generated photons (emission fields set) by the table method. */
void or_propagate_table(or_photon* ph, int64_t count, const or_atmosphere* a, int32_t n_h, int32_t n_q, double h_max,
                        double q_max, int32_t n_v, const double* corr, const double* vert) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t q = 0; q < count; ++q) {
    if (ph[q].status != OR_INVALID) ph[q].status = OR_LANDED;
    or_propagate_table_one(&ph[q], a, n_h, n_q, h_max, q_max, n_v, corr, vert);
  }
}

void or_telescopes(const or_photon* ph, int64_t count, const double* tel, int32_t n_tel,
                   double n_obs, int32_t* tel_id, double* hits /* 5 per photon */) {
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < count; ++q) tel_id[q] = or_telescope_one(&ph[q], tel, n_tel, n_obs, &hits[5 * q]);
}

void or_grid(const or_photon* ph, int64_t count, double x_min, double y_min, double cell, int32_t nx,
             int32_t ny, int32_t* cell_of) {
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < count; ++q) cell_of[q] = or_grid_cell(&ph[q], x_min, y_min, cell, nx, ny);
}

/* ------------------------------------------------------------------------ */
/* Ground photon density by Gaussian splatting (the differentiable form).   */
/* Each landed photon adds w * exp(-|r_g - r_l|^2 / (2 sigma^2)) /         */
/* (2 pi sigma^2) to every cell whose centre r_g lies within trunc*sigma   */
/* of the landing point in x and in y.                                      */
/* ------------------------------------------------------------------------ */
void or_splat(const or_photon* ph, const double* weight, int64_t count, double x_min, double y_min,
              double cell, int32_t nx, int32_t ny, double sigma, double trunc, double* D) {
  const double norm = 1.0 / (2.0 * OR_PI * sigma * sigma);
  const double reach = trunc * sigma;
  for (int64_t q = 0; q < count; ++q) {
    if (ph[q].status != OR_LANDED) continue;
    const double x = ph[q].xl, y = ph[q].yl;
    for (int32_t iy = 0; iy < ny; ++iy) {
      const double gy = y_min + (iy + 0.5) * cell;
      if (fabs(gy - y) > reach) continue;
      for (int32_t ix = 0; ix < nx; ++ix) {
        const double gx = x_min + (ix + 0.5) * cell;
        if (fabs(gx - x) > reach) continue;
        const double r2 = (gx - x) * (gx - x) + (gy - y) * (gy - y);
        D[(int64_t)iy * nx + ix] += weight[q] * norm * exp(-r2 / (2.0 * sigma * sigma));
      }
    }
  }
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
