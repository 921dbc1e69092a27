/*
 * photon.h -- C ABI of the MI355X optical-photon library (libphoton.so).
 *
 * The library computes, for charged-particle track segments, the optical
 * photons of the method of Baack & Alameddine, "Comparison and efficiency of
 * GPU accelerated optical light propagation in CORSIKA 8" (ICRC2023,
 * arXiv:2309.15861):
 *   - Cherenkov photon numbers from the Frank-Tamm formula (section 1.2) and
 *     fluorescence photon numbers from dN/dx = Y dE/dx (section 1.1),
 *     Poisson-sampled per segment;
 *   - Cherenkov photons on the cone cos(theta) = 1/(beta n), generated
 *     downward, rotated by M_Rod into the track frame and moved to their
 *     emission point (section 1.2, Fig. 1, section 1.2.1); isotropic
 *     fluorescence photons on emission lines (section 1.1);
 *   - propagation to the observation level through a plane-parallel layered
 *     exponential atmosphere, n(h) = 1 + (n0 - 1) rho(h)/rho0, with
 *     refraction, arrival time and absorption (section 2);
 *   - collection on telescope spheres or a ground grid.
 *
 * Conventions shared by every call:
 *   - z is the altitude above sea level [m], z points up; times in ns;
 *     wavelengths in nm; c = 0.299792458 m/ns.
 *   - Pointers named "device" are HIP device pointers owned by the caller;
 *     the library never frees or keeps them. Structs passed by pointer are
 *     host memory, read during the call only.
 *   - Every call validates its arguments on the host before any HIP call,
 *     then enqueues its kernels on `stream` (a hipStream_t; NULL = the null
 *     stream) and returns without synchronising.
 *   - Return value: PHOTON_OK (0) or a negative error code; the message of
 *     the last error of the calling thread is photon_last_error().
 *   - Randomness: Philox4x32-10 (Salmon et al., SC'11) with key = seed and
 *     counter (j or chunk, index_in_shower, shower, domain); results are a
 *     pure function of (inputs, seed), independent of batching and of the
 *     order of segments.
 *   - Device scratch. Eager calls of the fused, splat and adjoint forms work
 *     in the device's own scratch, allocated on first use: a 64 KB work area
 *     (work cursor, per-block counts), the FP32 form's near-horizon queue
 *     (2^24 rays, 128 MB, photon_set_defer_capacity), the adjoint's partial
 *     sums (1.1 MB) and the splat's accumulator (8 B per cell). Such calls
 *     are ordered on the device whatever their streams: a call on another
 *     stream than the previous one waits for it (an event recorded after
 *     each call; not inside a stream capture). photon_init() creates the
 *     work area up front. A captured plan owns its scratch (photon_plan_*),
 *     and photon_run_fused_noalloc works in a static array: neither touches
 *     the device's scratch.
 */
#ifndef PHOTON_H
#define PHOTON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define PHOTON_OK 0
#define PHOTON_EINVAL (-1)      /* invalid argument (message says which)   */
#define PHOTON_ECAPACITY (-2)   /* output buffer too small                 */
#define PHOTON_EHIP (-3)        /* a HIP runtime call failed               */
#define PHOTON_ENODEV (-4)      /* no usable gfx950 device                 */

/* ---- precision --------------------------------------------------------- */
#define PHOTON_FP64 0           /* all arithmetic in double                 */
#define PHOTON_FP32 1           /* generation and bending in float; time,
                                   path and near-horizon pieces in double  */

/* ---- emission kinds ------------------------------------------------------ */
#define PHOTON_CHERENKOV 0
#define PHOTON_FLUORESCENCE 1

/* ---- per-photon status -------------------------------------------------- */
#define PHOTON_LANDED 0         /* reached the observation level            */
#define PHOTON_HIT 1            /* landed and hit a telescope sphere        */
#define PHOTON_UP 2             /* emitted with u_z >= 0: never lands        */
#define PHOTON_BELOW 3          /* emitted below the observation level      */
#define PHOTON_OFFGRID 4        /* landed outside the ground grid           */
#define PHOTON_INVALID 6        /* slot without a valid segment             */
#define PHOTON_N_STATUS 8
/* Slot 7 of the status totals is not a photon status: it counts rays near
   the horizon that a fused FP32 run evaluated in place (in double, as the
   photon-block path does, at a lower speed) because its deferral queue was
   full (2^24 rays per device unless resized, shared evenly among the
   kernel's blocks); slots 0..6 partition the photons. */
#define PHOTON_HORIZON_FLOAT 7

/* ---- sink kinds ---------------------------------------------------------- */
#define PHOTON_SINK_STATUS 0    /* per-status photon totals only            */
#define PHOTON_SINK_TELESCOPES 1
#define PHOTON_SINK_GRID 2
#define PHOTON_SINK_PLANE 3     /* every photon written at its slot         */
#define PHOTON_SINK_RADIAL 4    /* radial density and arrival-time profile  */

#define PHOTON_MAX_LAYERS 8
#define PHOTON_MAX_ABS 40
#define PHOTON_MAX_LINES 32
#define PHOTON_MAX_TELESCOPES 32
#define PHOTON_MAX_CUT_POINTS 32
#define PHOTON_MAX_RADIAL_BINS 1024

/* Plane-parallel atmosphere (host struct). Layer i covers
   [h_base[i], h_base[i+1]); layer 0 extends below h_base[0] = 0 and the top
   layer has no upper bound. rho/rho0 is continuous, equals 1 at h = 0 and
   falls as exp(-h/scale_height[i]) inside layer i (scale_height = +inf:
   constant density). n(h) = 1 + n0_minus_1 * rho(h)/rho0. Absorption
   coefficient k(lambda) * rho/rho0 [1/m], k piecewise linear in lambda
   between the table nodes and clamped outside; n_abs = 0: no absorption.
   table: NULL for the exact propagation (the closed-form layer integrals);
   else the straight-line propagation with that correction table (built by
   photon_table_build for this atmosphere) for every call that propagates.
   Errors: n_layers outside 1..8, h_base[0] != 0 or not strictly increasing,
   scale_height <= 0 or NaN, n0_minus_1 < 0 or not finite, h_obs not finite,
   n_abs outside 0..40, abs_lambda_nm not strictly increasing, abs_k < 0, a
   table built for another atmosphere (layers, scale heights, n0_minus_1 or
   h_obs differ) or not built. */
struct photon_table;
typedef struct {
  int32_t n_layers;
  double h_base[PHOTON_MAX_LAYERS];
  double scale_height[PHOTON_MAX_LAYERS];
  double n0_minus_1;
  double h_obs;
  int32_t n_abs;
  double abs_lambda_nm[PHOTON_MAX_ABS];
  double abs_k_per_m[PHOTON_MAX_ABS];
  const struct photon_table* table;
} photon_atmosphere;

/* Correction tables of the straight-line propagation (section 2: photons
   are carried to the ground on a straight line and correction factors then
   change arrival position, time and angle for refraction). With
   dh = h_e - h_obs, mu = cos(zenith), q = tan(zenith), sec = 1/mu:
     landing point  x_e + ux (dh + g)/mu   (ux, uy: unit direction)
     path           P = dh sec + dP
     column         X = sec VX(h_e) + dX   (VX: vertical column from h_obs,
                                            column = integral of rho/rho0 ds)
     time           t_e + (P + n0_minus_1 X)/c,   weight exp(-k(lambda) X)
     direction      Snell: horizontal part times n(h_e)/n(h_obs)
   g, dP, dX are the exact integrals minus the straight line, tabulated at
   heights h_i = h_obs + (h_max - h_obs) i/(n_h - 1) and q_j = q_max j/(n_q - 1)
   (g at q = 0: its limit, taken at q = 1e-4 q_max) and interpolated
   bilinearly; rho/rho0 and VX at v_k = h_obs + (h_max - h_obs) k/(n_v - 1),
   interpolated linearly. Photons above h_max or with q > q_max, and every
   photon of the differentiable form, take the exact integrals.
   Caller-owned device arrays: corr float[4 n_h n_q], node (i, j) at
   4 (i n_q + j) as (g, dP, dX, 0); vert float[2 n_v] as (rho/rho0, VX).
   atm_hash is written by photon_table_build. */
typedef struct photon_table {
  int32_t n_h, n_q, n_v;
  double h_max, q_max;
  float* corr;
  float* vert;
  uint64_t atm_hash;
} photon_table;

/* Track segments, structure of arrays of length n (device pointers).
   Start point (x0,y0,z0) [m], direction (dx,dy,dz) (normalised inside),
   length [m], speed beta in (0,1), start time t0 [ns], energy loss dedx
   [MeV/m] (fluorescence only), charge number (NULL: |z| = 1), shower id
   (NULL: 0) and index of the segment in its shower (NULL: the row number);
   the last two are Philox counter words. A segment with a non-finite field,
   beta outside (0,1), negative length or zero direction emits no photons. */
typedef struct {
  int64_t n;
  const double *x0, *y0, *z0, *dx, *dy, *dz, *length, *beta, *t0;
  const double *dedx;
  const int32_t *charge;
  const uint32_t *shower;
  const uint32_t *index_in_shower;
} photon_segments;

/* Emission model (host struct).
   Cherenkov: wavelength band [lambda_min_nm, lambda_max_nm], 0 < min < max.
   Fluorescence: total yield [photons/MeV] >= 0 and n_lines (1..32) lines
   with wavelengths line_nm and relative yields line_rel_yield (>= 0, not
   all zero); a photon takes line k with probability rel[k]/sum(rel).
   Cherenkov angular particle cut (the optimisation of section 1.2.1): with
   n_cut_points in 1..32, a segment emits no photons unless, for at least one
   point P, the angle between its unit direction d and v = P - m (m its
   midpoint) is at most the cut angle: d.v >= cut_cos |v|, evaluated in FP64
   without contraction. One point is the array centre; the telescope centres
   give the per-telescope form. n_cut_points = 0: no cut (zero-initialise).
   Photons of the remaining segments are unchanged (their random numbers
   depend only on their own ids). Ignored for fluorescence.
   Fluorescence beaming (the optimisation of section 1.1.1), beam = 1: each
   segment emits into a cone that contains the emission area, a sphere of
   centre beam_center and radius beam_radius enclosing every telescope, and
   its mean photon number is scaled by the cone's solid-angle fraction
   (1 - cos(half angle))/2. Seen from the segment midpoint m at distance D
   from the centre, the half angle is asin((beam_radius + L/2)/D) plus
   beam_margin_rad (in [0, pi/2]; a margin for refractive bending), about
   the direction from m to the centre; directions are uniform on the cone.
   A segment with beam_radius + L/2 >= D stays isotropic. beam = 0: isotropic
   emission. Ignored for Cherenkov. Expected telescope hits are unchanged as
   long as every photon that can reach a telescope leaves within the cone. */
typedef struct {
  int32_t kind;                       /* PHOTON_CHERENKOV / PHOTON_FLUORESCENCE */
  double lambda_min_nm, lambda_max_nm;
  double yield_per_MeV;
  int32_t n_lines;
  double line_nm[PHOTON_MAX_LINES];
  double line_rel_yield[PHOTON_MAX_LINES];
  int32_t n_cut_points;
  double cut_cos;
  double cut_points[PHOTON_MAX_CUT_POINTS][3];
  int32_t beam;
  double beam_center[3];
  double beam_radius;
  double beam_margin_rad;
} photon_emission;

/* The common photon block (section 1: photons of both generators are
   written to one memory block and processed downstream), structure of
   arrays with `capacity` slots (device pointers). Slot q holds photon j of
   segment `segment[q]`, with q = offsets[segment] + j. Horizontal position,
   the horizontal direction components, wavelength and weight are double
   (PHOTON_FP64) or float (PHOTON_FP32); the vertical direction component,
   the height z, the time and the path length are double in both (near the
   horizon the zenith cosine sets the slant path and must keep its double
   digits from generation to propagation). After generation: emission point,
   time and direction, path 0, weight 1, status LANDED (or INVALID). After
   propagation: landing point (z = h_obs), arrival time, arrival direction,
   geometric path length, transmission weight exp(-tau) and status. */
typedef struct {
  int64_t capacity;
  int64_t n_photons;                  /* slots in use = offsets[n]          */
  int32_t precision;
  void *x, *y, *ux, *uy;
  double *uz;
  void *wavelength_nm, *weight;
  double *z, *t_ns, *path_m;
  uint32_t *segment, *j;
  int32_t *status;
} photon_block;

/* Telescope hit records, appended in arbitrary order (device pointers).
   *count (device) is incremented once per hit; records beyond capacity
   are dropped but still counted, so *count > capacity signals overflow. */
typedef struct {
  int64_t capacity;
  unsigned long long *count;
  uint32_t *segment, *j;
  int32_t *telescope;
  double *x, *y, *z, *t_ns;           /* entry point on the sphere and time  */
  float *ux, *uy, *uz, *wavelength_nm, *weight;
} photon_hits;

/* Where photons are collected (host struct). Outputs accumulate: the caller
   clears them. status_totals (device, 8 x u64, may be NULL) receives the
   number of photons per status. TELESCOPES: spheres (x,y,z,R) [m]; a
   landed photon hits when the straight line through its landing point
   along its arrival direction meets a sphere; the entry point of the first
   sphere along the ray is recorded with time t + n_obs * s / c (s the
   signed distance from the landing point). GRID: nx * ny cells of size
   `cell` from (x_min, y_min), half-open; grid_count[iy*nx+ix] counts landed
   photons, grid_weight the sum of their weights in units of 2^-32. PLANE:
   every photon's final state is written at its slot q = offsets[s] + j of
   `plane` (a photon block of the run's precision, its vertical direction
   in double; capacity >= number of photons;
   slots beyond the capacity are not written), as photon_propagate leaves a
   photon block. RADIAL (the profiles of section 3.1): a landed photon at
   distance r = |(x, y) - (core_x, core_y)| from the core falls in bin
   k = floor((r - r_min) n_bins / (r_max - r_min)) (log_bins = 0) or
   k = floor(ln(r / r_min) n_bins / ln(r_max / r_min)) (log_bins = 1,
   r_min > 0), FP64, when 0 <= k < n_bins (1..1024 bins), else its status
   becomes OFFGRID. Per bin, radial_count counts photons, radial_weight sums
   their weights in units of 2^-32 and radial_wt sums w (t - t_ref_ns), each
   term rounded to units of 2^-8 ns, as two's-complement int64 in the u64
   array. Integer sums: the result does not depend on the order. */
typedef struct {
  int32_t kind;
  unsigned long long *status_totals;
  int32_t n_tel;
  double tel[PHOTON_MAX_TELESCOPES][4];
  photon_hits hits;
  double x_min, y_min, cell;
  int32_t nx, ny;
  uint32_t *grid_count;
  unsigned long long *grid_weight;
  const photon_block *plane;
  double core_x, core_y, r_min, r_max, t_ref_ns;
  int32_t n_bins, log_bins;
  unsigned long long *radial_count, *radial_weight, *radial_wt;
} photon_sink;

/* Launch shape of the fused kernel: threads per block (128, 256 or 512),
   photons per work chunk (a multiple of block, at most 16384), blocks per
   CU (0 = as many as fit). NULL = 256 threads, 4096-photon chunks, as many
   blocks as fit. Errors: EINVAL for any other shape. */
typedef struct {
  int32_t block;
  int32_t chunk;
  int32_t blocks_per_cu;
} photon_tuning;

/* Creates the per-device work area on the current device and looks up the
   device's address of the static scratch of photon_run_fused_noalloc.
   Optional; returns PHOTON_ENODEV without a gfx950 device. */
int photon_init(void);

/* Length of the current device's near-horizon queue of the FP32 form
   (default 2^24 rays, 8 B each), for calls made after this one and plans
   created after it: a block of a fused launch queues at most rays / (its
   blocks) rays, and evaluates the rest in place, in double, at a lower
   speed (counted in PHOTON_HORIZON_FLOAT).
   Waits for the device to be idle and frees the current queue (it is
   allocated again on first use). Errors: EINVAL (rays outside 1..2^28). */
int photon_set_defer_capacity(int64_t rays);

/* Version string ("libphoton <version> (gfx950) source <hash>", the hash
   being the first 16 hex digits of the SHA-256 of the library's source
   files and this header) and the message of the calling thread's last
   error. */
const char* photon_version(void);
const char* photon_last_error(void);

/* Cherenkov generation (section 1.2). With out == NULL: per-segment mean
   from the Frank-Tamm formula with n taken at the segment midpoint and
   constant along it, mu = 2 pi alpha z^2 (1/lambda_min - 1/lambda_max) L
   (1 - 1/(beta n)^2) for beta n > 1, else 0; Poisson count by sequential
   inverse CDF in chunks of mean <= 128 on the COUNT stream -> counts[n]
   (device u32); exclusive prefix sums -> offsets[n+1] (device u64,
   offsets[n] = total). With out != NULL: fills slots [0, out->n_photons)
   from the given offsets (which must come from a call with out == NULL):
   cone angle cos = 1/(beta n), azimuth 2 pi u1, photon vector of section
   1.2.1 rotated by M_Rod about the bisector of the track direction and
   (0,0,-1), emission point u0 along the track, time t0 + s/(beta c),
   wavelength from the 1/lambda^2 spectrum. Errors: EINVAL (NULL pointer,
   n < 0, band, atmosphere, precision, n_photons > capacity). */
int photon_gen_cherenkov(const photon_segments* seg, const photon_atmosphere* atm,
                         double lambda_min_nm, double lambda_max_nm, uint64_t seed,
                         int32_t precision, uint32_t* counts, uint64_t* offsets,
                         photon_block* out, void* stream);

/* Fluorescence generation (section 1.1): mean Y dE/dx L, Poisson count and
   offsets as above (out == NULL); photons (out != NULL) isotropic,
   cos(theta) = 1 - 2 u1, phi = 2 pi u2, emission point u0 along the track,
   line = smallest k with u3 < cdf[k]. Errors: as photon_gen_cherenkov, plus
   n_lines outside 1..32, negative or all-zero relative yields, yield < 0,
   dedx == NULL. */
int photon_gen_fluor(const photon_segments* seg, const photon_atmosphere* atm,
                     const double* line_nm, const double* line_rel_yield, int32_t n_lines,
                     double yield_per_MeV, uint64_t seed, int32_t precision, uint32_t* counts,
                     uint64_t* offsets, photon_block* out, void* stream);

/* Propagation (section 2), in place on slots [0, inout->n_photons): u_z >= 0
   -> UP; emission below h_obs -> BELOW; otherwise the exact refracted ray of
   the plane-parallel atmosphere (n sin(theta) conserved) is carried to
   h_obs with closed-form layer integrals: landing point, arrival time
   t + (optical path)/c, path length, arrival direction (Snell), weight
   exp(-k(lambda) * column density along the ray). Directions are taken as
   unit vectors in FP32 (the generators' are, to rounding) and normalised in
   FP64. Errors: EINVAL. */
int photon_propagate(photon_block* inout, const photon_atmosphere* atm, void* stream);

/* Collection of a propagated block into `sink` (status totals, telescope
   hits or ground grid). Errors: EINVAL (sink kind, n_tel outside 1..32,
   R <= 0, grid shape, NULL outputs). */
int photon_collect(const photon_block* in, const photon_atmosphere* atm, const photon_sink* sink,
                   void* stream);

/* Fused persistent form: generation, propagation and collection of every
   photon of `seg` in registers, without a photon block, by one persistent
   kernel that takes work chunks of the photon index space from an atomic
   queue. `offsets` (n+1, device) comes from a generation call with
   out == NULL for the same segments, emission and seed. n_photons is the
   number of photon slots to process: offsets[n], or -1 to have the kernel
   read offsets[n] on the device (no host round trip; slots beyond
   offsets[n] count as INVALID). Results equal those of gen + propagate +
   collect. In the FP32 form, rays within about 3 degrees of the horizon are
   handed to a second, double kernel that regenerates them from their random
   numbers (the device's queue of 2^24 rays, allocated on the first such
   call; see PHOTON_HORIZON_FLOAT). Works in the device's scratch: calls on
   one device are ordered whatever their streams (see the conventions). */
int photon_run_fused(const photon_segments* seg, const photon_atmosphere* atm,
                     const photon_emission* em, uint64_t seed, int32_t precision,
                     const uint64_t* offsets, int64_t n_photons, const photon_sink* sink,
                     const photon_tuning* tuning, void* stream);

/* photon_run_fused for callers that cannot allocate device memory (code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): same arguments, kernels and results, but it allocates nothing.
   Its scratch (work cursor, per-block near-horizon counts and their prefix
   sums, and a queue of 2^20 near-horizon rays: 8.1 MiB) is a static device
   array that every GPU the library runs on holds until the process ends; its
   address is looked up once per device (photon_init, else the first call).
   Limit: the FP32 form queues at most 2^20 / (blocks of the launch)
   near-horizon rays per block for the double pass; a block that queues more
   evaluates the excess in place in double and counts it in
   PHOTON_HORIZON_FLOAT, as photon_run_fused does beyond its 2^24-ray
   queue. Every call on one GPU
   works in that GPU's one array and leaves its contents behind (the cursor
   is cleared at the start of each call): calls that overlap on one GPU, on
   any streams, race. Errors: as photon_run_fused; PHOTON_EHIP if the
   array's address cannot be looked up. */
int photon_run_fused_noalloc(const photon_segments* seg, const photon_atmosphere* atm,
                             const photon_emission* em, uint64_t seed, int32_t precision,
                             const uint64_t* offsets, int64_t n_photons, const photon_sink* sink,
                             const photon_tuning* tuning, void* stream);

/* Kernel timing, a measurement aid. With on != 0, every fused launch on the
   current device outside a stream capture (photon_run_fused, the splat
   forward) records a pair of HIP events on its stream around the persistent
   kernel alone (not the clearing, count or near-horizon kernels around it).
   photon_fused_kernel_ms waits for the last such launch and returns its
   kernel time in ms; PHOTON_EINVAL if none was timed since timing was last
   switched. Events are created on the first call with on != 0 and kept for
   the process. */
int photon_kernel_timing(int32_t on);
int photon_fused_kernel_ms(float* ms);

/* Time of the near-horizon double pass (the scan of the per-block queues and
   the double kernel) that followed the last timed fused kernel, in ms: the
   interval from the end of that kernel to the end of the double pass; 0 when
   that launch had none (FP64 form). Errors as photon_fused_kernel_ms. */
int photon_fused_deferred_ms(float* ms);

/* Micro-benchmark of one device rate the photon kernels' rooflines use (a
   measurement aid): kind 0 FP32 fused multiply-adds, 1 FP64 fused
   multiply-adds, 2 32x32->64 integer multiply-adds (the Philox rounds'
   operation), 3 FP32 exp2 on the transcendental unit, 4 FP32 FMAs and
   exp2 interleaved one to one, 5 reads of the device buffer `work`, 6 LDS
   32-bit integer adds returning the old value (the float splat's cell
   update), 7 LDS 64-bit integer adds (the double splat's), each wave's lanes
   on consecutive words. ALU and LDS kinds run `iters` steps of eight
   independent chains in every thread of eight 256-thread blocks per CU and
   write one value per thread to `work` (device, at least 2 KiB per block);
   kind 5 reads work[64 KiB ..
   work_bytes) once and writes one float per block at `work`. Writes the
   lane operations (or bytes) done to *ops and the kernel time measured with
   HIP events on `stream` to *ms; synchronises `stream`. Errors: EINVAL
   (kind, iters outside 1..2^20, NULL pointers, work_bytes too small). */
int photon_peak_run(int32_t kind, void* work, int64_t work_bytes, int32_t iters, double* ops, float* ms,
                    void* stream);

/* ---- captured steps (HIP graphs) and launch-shape tuning ------------------ */

/* A plan is one whole step captured into a HIP graph: per-segment counts and
   offsets (as photon_gen_cherenkov / photon_gen_fluor with out == NULL),
   clearing of the sink outputs (status totals, hit counter, grid) by fill
   kernels, and the fused persistent kernel reading the photon total on the
   device. Replays reuse the pointers given at creation; the caller keeps those
   buffers alive and unchanged in size until photon_plan_destroy. Creation
   validates like photon_run_fused and allocates the plan's own scratch (a
   128 KB work area and, for FP32, a near-horizon queue of the device's
   queue length), so that plans replayed on different streams do not
   interfere; replays of one plan must not overlap each other. */
typedef struct photon_plan_s* photon_plan;

int photon_plan_create(const photon_segments* seg, const photon_atmosphere* atm,
                       const photon_emission* em, uint64_t seed, int32_t precision,
                       uint32_t* counts, uint64_t* offsets, const photon_sink* sink,
                       const photon_tuning* tuning, photon_plan* out);

/* Enqueues one replay of the plan on `stream`. */
int photon_plan_launch(photon_plan plan, void* stream);

/* Releases the graph (after the last replay has completed). NULL is a no-op. */
int photon_plan_destroy(photon_plan plan);

/* Launch-shape tuning of the fused kernel: runs photon_run_fused once per
   candidate shape (after one untimed run each), `reps` timed runs per
   candidate measured with HIP events on `stream`, and returns the fastest in
   *best with its median time in *best_ms. Every run starts from cleared
   sink outputs (status totals, hit counter, grid, radial bins), and they are
   left cleared. Synchronises `stream`.
   Errors: EINVAL (no candidates, reps < 1, invalid candidate), as
   photon_run_fused otherwise. */
int photon_autotune(const photon_segments* seg, const photon_atmosphere* atm,
                    const photon_emission* em, uint64_t seed, int32_t precision,
                    const uint64_t* offsets, const photon_sink* sink,
                    const photon_tuning* candidates, int32_t n_candidates, int32_t reps,
                    photon_tuning* best, float* best_ms, void* stream);

/* ---- differentiable form: splatted ground density and its adjoint ---------- */

/* Ground grid of the splat: cell (ix, iy) has its centre at
   (x_min + (ix + 1/2) cell, y_min + (iy + 1/2) cell), row-major (ny rows of
   nx cells). A landed photon of weight w adds
   w exp(-d^2 / (2 sigma^2)) / (2 pi sigma^2) (per m^2) to every cell whose
   centre lies within trunc * sigma of its landing point in x and in y.
   Limits: nx ny <= 2^22, trunc sigma <= 64 cells. */
typedef struct {
  double x_min, y_min, cell;
  int32_t nx, ny;
  double sigma, trunc;
} photon_splat_grid;

/* Radial profiles from the accumulators of a RADIAL sink (section 3.1):
   density[k] = (sum of weights) / (pi (r_{k+1}^2 - r_k^2)) [photons/m^2]
   and mean_t_ns[k] = t_ref_ns + (sum of w (t - t_ref)) / (sum of weights),
   NaN where a bin holds no weight; bin edges r_k as the sink defines them.
   density and mean_t_ns: device f64[n_bins]. Errors: EINVAL (the sink's
   RADIAL fields as photon_run_fused checks them, NULL outputs). */
int photon_radial_profile(const photon_sink* sink, double* density, double* mean_t_ns, void* stream);

/* Fills a correction table for an atmosphere (its `table` field is
   ignored) from the exact FP64 integrals at every node, and stamps it with
   the atmosphere's hash. n_h, n_q in 2..4096, n_v in 2..65536,
   h_max > h_obs, 0 < q_max <= 1e3, corr and vert non-NULL. Errors: EINVAL. */
int photon_table_build(const photon_atmosphere* atm, photon_table* table, void* stream);

/* Per-segment counts and offsets for an emission model (as the generation
   calls with out == NULL), honouring the Cherenkov angular particle cut of
   `em`. counts: device u32[n]; offsets: device u64[n+1], offsets[n] = total.
   Errors: EINVAL (as photon_gen_cherenkov / photon_gen_fluor, plus
   n_cut_points outside 0..32, cut_cos outside [-1, 1], non-finite points,
   beam not 0 or 1, a non-finite beam centre, a negative beam radius, or a
   margin outside [0, pi/2]). */
int photon_count(const photon_segments* seg, const photon_atmosphere* atm, const photon_emission* em,
                 uint64_t seed, uint32_t* counts, uint64_t* offsets, void* stream);

/* Fills a photon block for an emission model (as the generation calls with
   a block), with the model's fluorescence beaming; offsets from photon_count
   with the same model, seed and segments. Errors: EINVAL (as photon_count,
   plus a NULL, mismatched or too small block). */
int photon_generate(const photon_segments* seg, const photon_atmosphere* atm, const photon_emission* em,
                    uint64_t seed, int32_t precision, const uint64_t* offsets, photon_block* out,
                    void* stream);

/* Per-segment means (device f64, n) exactly as the count step evaluates
   them: Frank-Tamm (section 1.2) or Y dE/dx L (section 1.1); 0 for
   invalid segments and for segments removed by the angular cut; beamed
   fluorescence means include the solid-angle fraction.
   Errors: EINVAL. */
int photon_means(const photon_segments* seg, const photon_atmosphere* atm,
                 const photon_emission* em, double* mean, void* stream);

/* Splatted ground density D of the Cherenkov photons of `seg` with the
   counts frozen: `offsets` (n+1, device) and `mean0` (n, device f64) are
   the offsets and means of the nominal parameters (photon_gen_cherenkov with
   out == NULL and photon_means), while `seg` and `atm` hold the current
   ones. Each landed photon carries the weight mu(current)/mean0 of its
   segment (0 where mean0 <= 0) times its transmission exp(-tau); the random
   numbers of photon (segment, j) are those of the plain form. density:
   device, ny*nx values of the precision's type (double for PHOTON_FP64,
   float for PHOTON_FP32), overwritten. status_totals: optional device
   u64[PHOTON_N_STATUS]; landed photons with no cell in reach count as
   OFFGRID. Cells sum w exp(-d^2/(2 sigma^2)) in 64-bit fixed point (units
   of 2^-32 of weight for PHOTON_FP64, 2^-24 for PHOTON_FP32) before the
   normalisation, so the density does not depend on the order of the
   additions (a cell overflows only beyond 2^32 or 2^40 weight units
   respectively); each block accumulates the whole grid in LDS when it
   fits (on gfx950 up to about 37,000 cells in 32-bit words with carries
   into the global grid for PHOTON_FP32, 17,600 cells in 64-bit words for
   PHOTON_FP64; larger grids add to the global grid directly). The library
   keeps a per-device accumulator
   of 8 bytes per cell, grown on the first call with a larger grid; calls
   are ordered on the device as the conventions say. Errors: EINVAL (NULL
   pointers, band, atmosphere, precision, grid). */
int photon_splat_forward(const photon_segments* seg, const photon_atmosphere* atm,
                         double lambda_min_nm, double lambda_max_nm, uint64_t seed,
                         int32_t precision, const uint64_t* offsets, const double* mean0,
                         const photon_splat_grid* grid, void* density,
                         unsigned long long* status_totals, void* stream);

/* Adjoint of photon_splat_forward (same arguments): given the gradient
   grad_density = dL/dD (device, the precision's type, ny*nx), writes
   dL/dH_l for l < n_layers (grad_scale_height, device f64; 0 for layers of
   infinite scale height), dL/d(n0 - 1) (grad_n0_minus_1, device f64, one
   value) and the gradient with respect to each segment's direction vector
   (dx, dy, dz) as given (grad_dx/dy/dz, device f64, n each; the direction
   is normalised inside, so the gradient is orthogonal to it). Every photon
   is regenerated from its random numbers and carried forward and back; the
   truncation edge of the splat is not differentiated. Direction gradients
   are summed with atomic adds (order varies between runs); the global ones
   in a fixed order of per-block partial sums. Works in the device's
   scratch (ordered as the conventions say). Errors: as
   photon_splat_forward. */
int photon_splat_backward(const photon_segments* seg, const photon_atmosphere* atm,
                          double lambda_min_nm, double lambda_max_nm, uint64_t seed,
                          int32_t precision, const uint64_t* offsets, const double* mean0,
                          const photon_splat_grid* grid, const void* grad_density,
                          double* grad_scale_height, double* grad_n0_minus_1, double* grad_dx,
                          double* grad_dy, double* grad_dz, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PHOTON_H */
