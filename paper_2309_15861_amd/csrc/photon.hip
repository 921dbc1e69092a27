// libphoton: HIP kernels for gfx950 and the C ABI declared in photon.h.
//
// Kernels (all wave64):
//   k_count      one lane per segment: mean (Frank-Tamm, section 1.2, or
//                Y dE/dx, section 1.1) and Poisson count; block totals for
//                the scan.
//   k_scan_tops  one workgroup: inclusive scan of the block totals in place.
//   k_scan_final one lane per segment: exclusive offsets.
//   k_gen        one lane per photon slot: Cherenkov (section 1.2, 1.2.1) or
//                fluorescence (section 1.1) photon into the photon block.
//   k_propagate  one lane per photon: refracted ray to the observation level
//                (section 2).
//   k_collect    one lane per photon: status totals, telescope hits, grid.
//   k_fused      persistent: work chunks of the photon index space from an
//                atomic queue; generation + propagation + collection in
//                registers, per-segment constants staged in LDS.
//   k_splat_adjoint persistent like k_fused: every photon regenerated and
//                carried forward and back through the adjoint of the
//                splatted ground density.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>

#include "photon.h"
#include "photon_device.hpp"
#include "photon_adjoint.hpp"
#include "photon_peaks.hpp"

using namespace ph;

// Scratch of photon_run_fused_noalloc, the entry point for callers that cannot
// allocate: words [0, 8192) hold the work-queue cursor (word 0) and the
// per-block counts of queued near-horizon rays (from word 64), words
// [8192, 16384) their prefix sums, and the rest a queue of 2^20 rays
// (segment row, photon number). 8.1 MiB; every device that runs the entry
// point holds its own copy until the process ends. Host code never uses this
// name as an address: it takes each device's address from
// hipGetSymbolAddress.
constexpr size_t kScratchAreaWords = 8192;
constexpr int64_t kScratchDeferRays = 1 << 20;
constexpr size_t kScratchWords = 2 * kScratchAreaWords + (size_t)kScratchDeferRays;
static __device__ __align__(256) unsigned long long scratch[kScratchWords];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(PHOTON_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int kScanBlock = 256;
constexpr int kWaveSize = 64;

// ------------------------------------------------------------------ views --
template <typename T>
struct BlockView {
  T *x, *y, *ux, *uy, *lam, *w;
  double *uz, *z, *t, *path;  // uz in double: the zenith cosine near the horizon
  uint32_t *seg, *j;
  int32_t* status;
};

struct GenParams {
  int32_t kind;
  int32_t n_lines;
  double inv_l1, inv_dl;                // Cherenkov: 1/lambda_min, 1/lambda_min - 1/lambda_max
  double K;                             // Frank-Tamm prefactor (Cherenkov) or yield per MeV
  uint64_t thr[PHOTON_MAX_LINES];       // fluorescence line thresholds on the 32-bit word
  double line_nm[PHOTON_MAX_LINES];
  BeamDev beam;                         // fluorescence beaming (on = 0: isotropic)
};

// Candidate grid of the telescope test: a landed photon whose arrival
// direction is within kCapZenith of the vertical can only hit sphere k if its
// landing point lies within R_k / cos(cap) + |z_k - h_obs| tan(cap) of the
// sphere centre horizontally (the line's closest approach is at least the
// horizontal offset at the centre's height times cos(zenith)). Each cell of
// a coarse grid over those capture disks keeps a bitmask of the spheres whose
// disk touches it; steeper photons test every sphere.
constexpr int kCandCells = 12;
constexpr double kCapCos = 0.5;  // cos(60 deg)

struct SinkDev {
  int32_t kind;
  int32_t n_tel;
  unsigned long long* totals;
  double tel[PHOTON_MAX_TELESCOPES][4];
  // h_obs (the float form's LDS table holds x, y, z - h_obs, R^2); the
  // candidate grid's origin and cells per metre (float: the lists carry a
  // 1 mm margin for the rounding)
  double tel_hobs;
  float cand_x0, cand_y0, cand_inv_cell;
  uint32_t cand_mask[kCandCells * kCandCells];
  photon_hits hits;
  double x_min, y_min, cell;
  int32_t nx, ny;
  uint32_t* grid_count;
  unsigned long long* grid_weight;
  // PLANE: every photon written at its slot (arrays of the run's precision)
  int64_t plane_capacity;
  void *px, *py, *pux, *puy, *plam, *pw;
  double *puz, *pz, *pt, *ppath;  // the vertical direction in double, as in the photon block
  uint32_t *pseg, *pj;
  int32_t* pstatus;
  // SPLAT (differentiable form): fixed-point accumulator of the whole grid
  // (global), frozen nominal means; splat_lds: each block accumulates in LDS
  // first and adds its grid to acc once
  SplatGeom sg;
  unsigned long long* splat_acc;
  const double* mu0;
  int32_t splat_lds;
  // RADIAL: profile bins about the core (r_inv = bins per unit of r or ln r)
  double core_x, core_y, r_min, r_inv, t_ref;
  int32_t n_bins, log_bins;
  unsigned long long *rad_count, *rad_w, *rad_wt;
};
// Sink of the differentiable form (reached through photon_splat_forward only).
constexpr int32_t kSinkSplat = 16;

// ------------------------------------------------------ wave/block helpers --
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Lanes of the wave mask m below this lane (its rank among them).
__device__ __forceinline__ unsigned int lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// The value v of lane src (the same src on every lane), read with scalar
// lane reads rather than a cross-lane permute.
__device__ __forceinline__ unsigned long long lane_value(unsigned long long v, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned int lane_value(unsigned int v, int src) {
  return (unsigned int)__builtin_amdgcn_readlane((int)v, src);
}

__device__ __forceinline__ unsigned long long wave_incl_scan(unsigned long long v) {
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWaveSize; d <<= 1) {
    const unsigned long long o = __shfl_up(v, d, kWaveSize);
    if (lane >= d) v += o;
  }
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int d = kWaveSize / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWaveSize);
  return v;
}

// Largest s in [0, n] with off[s] <= key (off nondecreasing, off[0] = 0),
// found by one wave with 64-way splits (a few dependent loads).
__device__ int64_t wave_upper_index(const uint64_t* off, int64_t n, uint64_t key) {
  const int lane = lane_id();
  int64_t lo = 0, hi = n;
  while (hi - lo >= kWaveSize) {
    const int64_t step = (hi - lo + kWaveSize) / kWaveSize;
    const int64_t pos = lo + (int64_t)lane * step;
    const bool le = (pos <= hi) && (off[pos] <= key);
    const int c = max(__popcll(__ballot(le)) - 1, 0);
    const int64_t nlo = lo + (int64_t)c * step;
    const int64_t nhi = min(nlo + step - 1, hi);
    lo = nlo;
    hi = nhi;
  }
  const int64_t pos = lo + lane;
  const bool le = (pos <= hi) && (off[pos] <= key);
  return lo + max(__popcll(__ballot(le)) - 1, 0);
}

// Largest s in [0, n) with off[s] <= key, one lane.
__device__ __forceinline__ int64_t lane_upper_index(const uint64_t* off, int64_t n, uint64_t key) {
  int64_t lo = 0, hi = n;  // off[lo] <= key < off[hi] for key < off[n]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= key) lo = mid; else hi = mid;
  }
  return lo;
}

// ------------------------------------------------------------- count+scan --
// Mean of segment i (i < n) and its Poisson chunking: m chunks of mean mc,
// p0 = exp(-mc); the segment's random-stream ids. Zero chunks beyond n.
template <int KIND>
__device__ __forceinline__ void count_setup(const SegView& seg, int64_t n, int64_t i, const AtmDev& atm, double K,
                                            const CutDev& cut, const BeamDev& beam, uint32_t& m, double& mc,
                                            double& p0, uint32_t& idx, uint32_t& sh) {
  if (i < n) {
#pragma clang fp contract(off)
    const double mu = (KIND == PHOTON_CHERENKOV) ? (passes_cut(seg, i, cut) ? mean_cherenkov(seg, i, atm, K) : 0.0)
                                                 : beamed_mean(seg, i, beam, mean_fluor(seg, i, K));
    m = poisson_chunks(mu);
    if (m) {
      mc = mu / (double)m;
      p0 = exp_fixed(-mc);
    }
    idx = seg_idx(seg, i);
    sh = seg_shower(seg, i);
  }
}

// Counts: lane i computes the mean of segment i and its number of Poisson
// chunks; each wave then spreads the (segment, chunk) draws of its 64
// segments over its lanes, so that lanes do not idle while one segment with
// a large mean draws chunk after chunk. Chunk results are summed per segment
// with LDS atomics (integer sums: the order does not matter).
template <int KIND>
__global__ __launch_bounds__(kScanBlock) void k_count(SegView seg, int64_t n, AtmDev atm, double K, uint32_t k0,
                                                      uint32_t k1, CutDev cut, BeamDev beam,
                                                      uint32_t* __restrict__ counts,
                                                      uint64_t* __restrict__ offsets) {
  __shared__ unsigned long long part[kScanBlock / kWaveSize];
  __shared__ __align__(16) double rk[kPoissonKmax];
  __shared__ double s_mc[kScanBlock], s_p0[kScanBlock];
  __shared__ uint32_t s_start[kScanBlock], s_cnt[kScanBlock], s_idx[kScanBlock], s_sh[kScanBlock];
  const int tid = threadIdx.x;
  for (int k = tid; k < (int)kPoissonKmax; k += kScanBlock) rk[k] = 1.0 / (double)(k + 1);
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + tid;
  uint32_t m = 0;
  double mc = 0.0, p0 = 0.0;
  uint32_t idx = 0, sh = 0;
  count_setup<KIND>(seg, n, i, atm, K, cut, beam, m, mc, p0, idx, sh);
  const unsigned long long incl = wave_incl_scan((unsigned long long)m);
  const uint32_t total = (uint32_t)__shfl(incl, kWaveSize - 1, kWaveSize);
  s_start[tid] = (uint32_t)(incl - m);
  s_mc[tid] = mc;
  s_p0[tid] = p0;
  s_cnt[tid] = 0u;
  s_idx[tid] = idx;
  s_sh[tid] = sh;
  __syncthreads();
  const int wb = (tid / kWaveSize) * kWaveSize;
  for (uint32_t t = (uint32_t)lane_id(); t < total; t += kWaveSize) {
    // the segment lane L of item t: the last L with start[L] <= t
    int lo = 0, hi = kWaveSize;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_start[wb + mid] <= t) lo = mid; else hi = mid;
    }
    const int L = wb + lo;
    const uint32_t c = t - s_start[L];
    const double u = u01d(philox(c, s_idx[L], s_sh[L], kDomCount, k0, k1).w[0]);
    atomicAdd(&s_cnt[L], poisson_chunk(u, s_mc[L], s_p0[L], rk));
  }
  __syncthreads();
  const uint32_t cnt = s_cnt[tid];
  if (i < n) counts[i] = cnt;
  const unsigned long long s = wave_sum((unsigned long long)cnt);
  if (lane_id() == 0) part[tid / kWaveSize] = s;
  __syncthreads();
  if (tid == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kScanBlock / kWaveSize; ++w) t += part[w];
    const int64_t pos = min((int64_t)(blockIdx.x + 1) * kScanBlock, n);
    offsets[pos] = t;
  }
}

// The same counts for inputs of few segments (kCountWideMaxBlocks blocks or
// fewer): the draws of a block's kScanBlock segments are spread over all
// kCountWide threads of the block instead of over the 64 lanes of each
// segment's wave. A Poisson search is a chain of dependent multiplies and adds,
// and a small input at one wave per 64 segments leaves a few waves per SIMD to
// hide its latency; four times the waves per segment do.
constexpr int kCountWide = 1024;
constexpr int64_t kCountWideMaxBlocks = 2048;
template <int KIND>
__global__ __launch_bounds__(kCountWide) void k_count_wide(SegView seg, int64_t n, AtmDev atm, double K,
                                                           uint32_t k0, uint32_t k1, CutDev cut, BeamDev beam,
                                                           uint32_t* __restrict__ counts,
                                                           uint64_t* __restrict__ offsets) {
  constexpr int kW = kScanBlock / kWaveSize;  // the waves holding one segment per lane
  __shared__ unsigned long long part[kW];
  __shared__ uint32_t s_wt[kW];
  __shared__ __align__(16) double rk[kPoissonKmax];
  __shared__ double s_mc[kScanBlock], s_p0[kScanBlock];
  __shared__ uint32_t s_start[kScanBlock], s_cnt[kScanBlock], s_idx[kScanBlock], s_sh[kScanBlock];
  const int tid = threadIdx.x;
  for (int k = tid; k < (int)kPoissonKmax; k += kCountWide) rk[k] = 1.0 / (double)(k + 1);
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + tid;
  if (tid < kScanBlock) {
    uint32_t m = 0;
    double mc = 0.0, p0 = 0.0;
    uint32_t idx = 0, sh = 0;
    count_setup<KIND>(seg, n, i, atm, K, cut, beam, m, mc, p0, idx, sh);
    const unsigned long long incl = wave_incl_scan((unsigned long long)m);
    if (lane_id() == kWaveSize - 1) s_wt[tid / kWaveSize] = (uint32_t)incl;
    s_start[tid] = (uint32_t)(incl - m);  // within the wave; the waves before are added below
    s_mc[tid] = mc;
    s_p0[tid] = p0;
    s_cnt[tid] = 0u;
    s_idx[tid] = idx;
    s_sh[tid] = sh;
  }
  __syncthreads();
  uint32_t total = 0, before = 0;
  for (int w = 0; w < kW; ++w) {
    if (w < tid / kWaveSize) before += s_wt[w];
    total += s_wt[w];
  }
  if (tid < kScanBlock) s_start[tid] += before;
  __syncthreads();
  for (uint32_t t = (uint32_t)tid; t < total; t += kCountWide) {
    // the segment L of item t: the last L with start[L] <= t
    int lo = 0, hi = kScanBlock;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_start[mid] <= t) lo = mid; else hi = mid;
    }
    const uint32_t c = t - s_start[lo];
    const double u = u01d(philox(c, s_idx[lo], s_sh[lo], kDomCount, k0, k1).w[0]);
    atomicAdd(&s_cnt[lo], poisson_chunk(u, s_mc[lo], s_p0[lo], rk));
  }
  __syncthreads();
  if (tid < kScanBlock) {
    const uint32_t cnt = s_cnt[tid];
    if (i < n) counts[i] = cnt;
    const unsigned long long s = wave_sum((unsigned long long)cnt);
    if (lane_id() == 0) part[tid / kWaveSize] = s;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kW; ++w) t += part[w];
    const int64_t pos = min((int64_t)(blockIdx.x + 1) * kScanBlock, n);
    offsets[pos] = t;
  }
}

// In-place inclusive scan of the block totals at positions min((b+1)B, n),
// one workgroup, in tiles of 1024 x P totals: each thread loads its P
// consecutive totals into registers (all loads in flight together), the
// thread sums are scanned across the workgroup, and each thread writes its
// running sums back; a carry links the tiles (one tile up to 8.4e6
// segments).
__global__ __launch_bounds__(1024) void k_scan_tops(uint64_t* __restrict__ offsets, int64_t n, int64_t nb) {
  constexpr int P = 32;
  __shared__ unsigned long long part[1024 / kWaveSize];
  unsigned long long carry = 0;
  for (int64_t base = 0; base < nb; base += (int64_t)1024 * P) {
    const int64_t b0 = base + (int64_t)threadIdx.x * P;
    unsigned long long v[P];
    unsigned long long sum = 0;
#pragma unroll
    for (int k = 0; k < P; ++k) v[k] = (b0 + k < nb) ? offsets[min((b0 + k + 1) * kScanBlock, n)] : 0ull;
#pragma unroll
    for (int k = 0; k < P; ++k) sum += v[k];
    const unsigned long long incl = wave_incl_scan(sum);
    const int w = threadIdx.x / kWaveSize;
    if (lane_id() == kWaveSize - 1) part[w] = incl;
    __syncthreads();
    unsigned long long run = carry + incl - sum, tile = 0;
    for (int k = 0; k < 1024 / kWaveSize; ++k) {
      if (k < w) run += part[k];
      tile += part[k];
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
      run += v[k];
      if (b0 + k < nb) offsets[min((b0 + k + 1) * kScanBlock, n)] = run;
    }
    carry += tile;
    __syncthreads();  // part[] is rewritten by the next tile
  }
  if (threadIdx.x == 0) offsets[0] = 0;
}
__global__ __launch_bounds__(kScanBlock) void k_scan_final(const uint32_t* __restrict__ counts,
                                                           uint64_t* __restrict__ offsets, int64_t n) {
  __shared__ unsigned long long part[kScanBlock / kWaveSize];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  const int64_t i = base + threadIdx.x;
  const unsigned long long prefix = offsets[base];
  const unsigned long long c = (i < n) ? counts[i] : 0u;
  const unsigned long long incl = wave_incl_scan(c);
  const int w = threadIdx.x / kWaveSize;
  if (lane_id() == kWaveSize - 1) part[w] = incl;
  __syncthreads();
  unsigned long long add = prefix;
  for (int k = 0; k < w; ++k) add += part[k];
  if (i < n) offsets[i] = add + incl - c;
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Up to kZeroLists arrays of 64-bit words and one of 32-bit words cleared by
// one launch (the sink outputs and the work cursor of a step).
constexpr int kZeroLists = 6;
struct ZeroList {
  unsigned long long* p[kZeroLists];
  int32_t n[kZeroLists];
  int32_t k = 0;
  uint32_t* p32 = nullptr;
  int32_t n32 = 0;
  void add(unsigned long long* q, int32_t m) {
    p[k] = q;
    n[k++] = m;
  }
};

__global__ void k_zero_list(ZeroList z) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  for (int i = 0; i < z.k; ++i)
    for (int j = t; j < z.n[i]; j += stride) z.p[i][j] = 0ull;
  for (int j = t; j < z.n32; j += stride) z.p32[j] = 0u;
}

void launch_zero_list(const ZeroList& z, hipStream_t st) {
  int m = z.n32;
  for (int i = 0; i < z.k; ++i) m = m > z.n[i] ? m : z.n[i];
  if (m <= 0) return;
  const int blocks = (int)std::min<int64_t>((m + 255) / 256, 64);
  hipLaunchKernelGGL(k_zero_list, dim3((unsigned)blocks), dim3(256), 0, st, z);
}

// Grid-stride clear of n 64-bit words (a kernel, not a memset node, so that
// captured graphs replay it faithfully).
__global__ void k_zero64_n(unsigned long long* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// -------------------------------------------------------------- generation --
template <typename T>
__device__ __forceinline__ void generate(const SegConst<T>& c, uint32_t j, const GenParams& g, uint32_t k0,
                                         uint32_t k1, const uint64_t* thr, const T* lines, Photon<T>& p) {
  if (g.kind == PHOTON_CHERENKOV)
    gen_cherenkov<T>(c, j, k0, k1, (T)g.inv_l1, (T)g.inv_dl, p);
  else
    gen_fluor<T>(c, j, k0, k1, thr, lines, g.n_lines, g.beam.on != 0, p);
}

// The same with the emission kind fixed at compile time.
template <typename T, bool CHER>
__device__ __forceinline__ void generate_kind(const SegConst<T>& c, uint32_t j, const GenParams& g, uint32_t k0,
                                              uint32_t k1, const uint64_t* thr, const T* lines, Photon<T>& p) {
  if constexpr (CHER)
    gen_cherenkov<T>(c, j, k0, k1, (T)g.inv_l1, (T)g.inv_dl, p);
  else
    gen_fluor<T>(c, j, k0, k1, thr, lines, g.n_lines, g.beam.on != 0, p);
}

// Photons [256 b, 256 b + 256) of the block: their segments are found once
// per block (a wave-parallel search for the first and the last) and, when
// they are at most kGenWin, staged in LDS with their constants, so that each
// photon looks its segment up among a few LDS offsets instead of searching
// the offsets in global memory and recomputing the segment's constants.
constexpr int kGenWin = 64;

template <typename T>
__global__ __launch_bounds__(256) void k_gen(SegView seg, int64_t n_seg, AtmDev atm, GenParams g, uint32_t k0,
                                             uint32_t k1, const uint64_t* __restrict__ offsets, int64_t n_ph,
                                             BlockView<T> out) {
  __shared__ uint64_t s_thr[PHOTON_MAX_LINES];
  __shared__ T s_lines[PHOTON_MAX_LINES];
  __shared__ SegConst<T> s_seg[kGenWin];
  __shared__ uint64_t s_off[kGenWin + 1];
  __shared__ int64_t s_lo, s_hi;
  const int tid = threadIdx.x;
  if (tid < PHOTON_MAX_LINES) {
    s_thr[tid] = g.thr[tid];
    s_lines[tid] = (T)g.line_nm[tid];
  }
  const uint64_t total = offsets[n_seg];
  const int64_t q0 = (int64_t)blockIdx.x * blockDim.x;
  // the block's valid photons [q0, qe)
  const int64_t qe = min(min(q0 + (int64_t)blockDim.x, n_ph), (int64_t)total);
  const int wave = tid / kWaveSize;
  if (qe > q0) {
    if (wave == 0) {
      const int64_t sl = wave_upper_index(offsets, n_seg, (uint64_t)q0);
      if (lane_id() == 0) s_lo = sl;
    } else if (wave == 1) {
      const int64_t sh = wave_upper_index(offsets, n_seg, (uint64_t)(qe - 1));
      if (lane_id() == 0) s_hi = sh;
    }
  }
  __syncthreads();
  // both ends in [0, n_seg) for offsets from the count call; the clamps keep
  // every index in bounds for any offsets array
  const int64_t lo = qe > q0 ? min(s_lo, n_seg - 1) : 0;
  const int64_t W = qe > q0 ? min(s_hi, n_seg - 1) - lo + 1 : 0;
  const bool win = W >= 1 && W <= kGenWin;
  const bool cher = g.kind == PHOTON_CHERENKOV;
  if (win) {
    for (int t = tid; t < W; t += blockDim.x) seg_const<T>(seg, lo + t, atm, cher, g.beam, s_seg[t]);
    for (int t = tid; t <= W; t += blockDim.x) s_off[t] = offsets[lo + t];
  }
  __syncthreads();
  const int64_t q = q0 + tid;
  if (q >= n_ph) return;
  Photon<T> p;
  uint32_t s32 = 0xffffffffu, j = 0;
  if ((uint64_t)q < total) {
    int64_t s;
    uint64_t off_s;
    SegConst<T> c;
    int a = 0;
    if (win) {
      int b = (int)W;  // s_off[a] <= q < s_off[b]
      while (b - a > 1) {
        const int mid = (a + b) >> 1;
        if (s_off[mid] <= (uint64_t)q) a = mid; else b = mid;
      }
      s = lo + a;
      c = s_seg[a];
      off_s = s_off[a];
      // keeps the LDS load and the global one below apart
      asm volatile("" : "+v"(off_s));
    } else {
      s = lane_upper_index(offsets, n_seg, (uint64_t)q);
      seg_const<T>(seg, s, atm, cher, g.beam, c);
      off_s = offsets[s];
    }
    j = (uint32_t)((uint64_t)q - off_s);
    generate<T>(c, j, g, k0, k1, s_thr, s_lines, p);
    s32 = (uint32_t)s;
  } else {
    p = Photon<T>{};
    p.status = PHOTON_INVALID;
  }
  out.x[q] = p.x;
  out.y[q] = p.y;
  out.z[q] = p.z;
  out.ux[q] = p.ux;
  out.uy[q] = p.uy;
  out.uz[q] = p.uzd;
  out.lam[q] = p.lambda;
  out.w[q] = p.w;
  out.t[q] = p.t;
  out.path[q] = p.path;
  out.seg[q] = s32;
  out.j[q] = j;
  out.status[q] = p.status;
}

// ------------------------------------------------------------- propagation --
// TABLE: the straight line with tabulated corrections (atm.tcorr set); a
// separate instance, so that the exact path carries none of its registers.
template <typename T, bool TABLE>
__global__ __launch_bounds__(256) void k_propagate(AtmDev atm, BlockView<T> b, int64_t n_ph) {
  __shared__ AtmLane s_lane;
  atm_lane_fill(atm, &s_lane);
  __syncthreads();
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_ph) return;
  Photon<T> p;
  p.x = b.x[q];
  p.y = b.y[q];
  p.z = b.z[q];
  p.ux = b.ux[q];
  p.uy = b.uy[q];
  p.uzd = b.uz[q];
  p.uz = (T)p.uzd;
  p.lambda = b.lam[q];
  p.w = b.w[q];
  p.t = b.t[q];
  p.path = b.path[q];
  p.status = b.status[q];
  propagate<T, false, false, TABLE>(atm, s_lane, p);
  b.x[q] = p.x;
  b.y[q] = p.y;
  b.z[q] = p.z;
  b.ux[q] = p.ux;
  b.uy[q] = p.uy;
  // the arrival direction is in the working precision; photons that did not
  // land keep their emitted component
  b.uz[q] = p.status == PHOTON_LANDED ? (double)p.uz : p.uzd;
  b.w[q] = p.w;
  b.t[q] = p.t;
  b.path[q] = p.path;
  b.status[q] = p.status;
}

// -------------------------------------------------------------- collection --
struct StatusCounter {
  uint32_t c[PHOTON_N_STATUS];
  __device__ void clear() {
#pragma unroll
    for (int k = 0; k < PHOTON_N_STATUS; ++k) c[k] = 0;
  }
  __device__ void add(int st) {
#pragma unroll
    for (int k = 0; k < PHOTON_N_STATUS; ++k) c[k] += (st == k) ? 1u : 0u;
  }
};

// Per-lane status counts of one work chunk, eight 8-bit fields in one
// 64-bit register (a lane sees at most chunk / block <= 128 photons of a
// chunk). At the chunk's end each wave adds them up, two fields per 32-bit
// word in 16-bit halves (a wave's field sum stays below 2^14), and one lane
// adds the sums to the block's LDS totals.
__device__ __forceinline__ uint64_t status_inc(int st) {
  return st >= 0 ? (1ull << (8 * st)) : 0ull;
}

__device__ __forceinline__ void flush_lane_status(uint64_t pk, unsigned long long* s_stat) {
  const uint32_t lo = (uint32_t)pk, hi = (uint32_t)(pk >> 32);
  uint32_t w[4] = {(lo & 0xffu) | ((lo & 0xff00u) << 8), ((lo >> 16) & 0xffu) | ((lo >> 8) & 0xff0000u),
                   (hi & 0xffu) | ((hi & 0xff00u) << 8), ((hi >> 16) & 0xffu) | ((hi >> 8) & 0xff0000u)};
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int d = kWaveSize / 2; d > 0; d >>= 1) w[k] += __shfl_xor(w[k], d, kWaveSize);
  if (lane_id() == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (w[k] & 0xffffu) atomicAdd(&s_stat[2 * k], (unsigned long long)(w[k] & 0xffffu));
      if (w[k] >> 16) atomicAdd(&s_stat[2 * k + 1], (unsigned long long)(w[k] >> 16));
    }
  }
}

// Block-wide reduction of per-lane status counters into global totals.
__device__ void flush_status(StatusCounter& sc, unsigned long long* totals) {
  __shared__ unsigned long long s_tot[PHOTON_N_STATUS];
  if (threadIdx.x < PHOTON_N_STATUS) s_tot[threadIdx.x] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PHOTON_N_STATUS; ++k) {
    const unsigned long long v = wave_sum((unsigned long long)sc.c[k]);
    if (lane_id() == 0 && v) atomicAdd(&s_tot[k], v);
  }
  __syncthreads();
  if (threadIdx.x < PHOTON_N_STATUS && s_tot[threadIdx.x]) atomicAdd(&totals[threadIdx.x], s_tot[threadIdx.x]);
}

// A telescope hit record as staged in LDS.
struct HitRec {
  double x, y, z, t;
  uint32_t seg, j;
  int32_t tel;
  float ux, uy, uz, lam, w;
};
constexpr int kHitStage = 64;  // hit records staged per block and work chunk

struct HitStage {
  unsigned int n;
  HitRec rec[kHitStage];
};

__device__ __forceinline__ void write_hit(const photon_hits& h, unsigned long long slot, const HitRec& r) {
  h.segment[slot] = r.seg;
  h.j[slot] = r.j;
  h.telescope[slot] = r.tel;
  h.x[slot] = r.x;
  h.y[slot] = r.y;
  h.z[slot] = r.z;
  h.t_ns[slot] = r.t;
  h.ux[slot] = r.ux;
  h.uy[slot] = r.uy;
  h.uz[slot] = r.uz;
  h.wavelength_nm[slot] = r.lam;
  h.weight[slot] = r.w;
}

// Block-wide: moves the staged hits to the output with one global atomic.
__device__ __forceinline__ void flush_hits(HitStage* st, const photon_hits& h) {
  __shared__ unsigned long long s_base;
  __syncthreads();
  const unsigned int n = st->n < (unsigned int)kHitStage ? st->n : (unsigned int)kHitStage;
  if (threadIdx.x == 0) s_base = n ? atomicAdd(h.count, (unsigned long long)n) : 0ull;
  __syncthreads();
  for (unsigned int i = threadIdx.x; i < n; i += blockDim.x) {
    const unsigned long long slot = s_base + i;
    if (slot < (unsigned long long)h.capacity) write_hit(h, slot, st->rec[i]);
  }
  __syncthreads();
  if (threadIdx.x == 0) st->n = 0u;
}

// Radial profile bin of a landing point, or -1 outside [r_min, r_max).
__device__ __forceinline__ int radial_bin(const SinkDev& sk, double x, double y) {
#pragma clang fp contract(off)
  const double dx = x - sk.core_x, dy = y - sk.core_y;
  const double r = sqrt(dx * dx + dy * dy);
  const double f = sk.log_bins ? log(r / sk.r_min) * sk.r_inv : (r - sk.r_min) * sk.r_inv;
  return (f >= 0.0 && f < (double)sk.n_bins) ? (int)f : -1;
}

// Fixed-point terms of one photon: weight in units of 2^-32 and
// w (t - t_ref) in units of 2^-8 ns (two's complement).
__device__ __forceinline__ unsigned long long radial_wfix(double w) {
  return (unsigned long long)(w * 4294967296.0 + 0.5);
}
__device__ __forceinline__ unsigned long long radial_tfix(double w, double t, double t_ref) {
  return (unsigned long long)(long long)rint(w * (t - t_ref) * 256.0);
}

// LDS of the hit stage; the splat variant has none (its LDS holds the grid).
template <bool SPLAT>
struct HitStageLds {
  HitStage st;
  __device__ HitStage* get() { return &st; }
};
template <>
struct HitStageLds<true> {
  __device__ HitStage* get() { return nullptr; }
};

// Applies the sink to one propagated photon (in the lanes that hold one);
// returns the final status. Hit records are compacted per wave: one atomic
// per wave reserves the slots, lanes write at their rank among the hits.
// SPLAT: the sink of the differentiable form only; RADIAL: the radial
// profile only (separate instantiations, so that the other sinks' kernels
// carry none of their code). lds_acc: the block's LDS accumulator (the
// splat grid, or the radial bins as count, weight, w t), or NULL to add to
// the global arrays directly.
template <typename T, bool SPLAT = false, bool RADIAL = false, bool TEL_ONLY = false, bool GRID_ONLY = false>
__device__ __forceinline__ int sink_photon(const SinkDev& sk, const double (*tel)[4], const float (*telf)[4],
                                           double n_over_c, Photon<T>& p,
                                           uint32_t seg_row, uint32_t j, bool active, uint64_t slot_q,
                                           HitStage* stage, unsigned long long* lds_acc,
                                           const uint32_t* cand) {
  int st = active ? p.status : -1;
  if constexpr (SPLAT) {
    if (active && st == PHOTON_LANDED) {
      // one call per address space (no generic pointer)
      const bool in = lds_acc ? splat_add<T>(sk.sg, (double)p.x, (double)p.y, p.w, lds_acc)
                              : splat_add<T>(sk.sg, (double)p.x, (double)p.y, p.w, sk.splat_acc);
      if (!in) st = PHOTON_OFFGRID;
    }
  } else if constexpr (RADIAL) {
    if (active && st == PHOTON_LANDED) {
      const int k = radial_bin(sk, (double)p.x, (double)p.y);
      if (k >= 0) {
        const unsigned long long wf = radial_wfix((double)p.w);
        const unsigned long long tf = radial_tfix((double)p.w, p.t, sk.t_ref);
        // one branch per address space (no generic pointer)
        if (lds_acc) {
          atomicAdd(&lds_acc[k], 1ull);
          atomicAdd(&lds_acc[sk.n_bins + k], wf);
          atomicAdd(&lds_acc[2 * sk.n_bins + k], tf);
        } else {
          atomicAdd(&sk.rad_count[k], 1ull);
          atomicAdd(&sk.rad_w[k], wf);
          atomicAdd(&sk.rad_wt[k], tf);
        }
      } else {
        st = PHOTON_OFFGRID;
      }
    }
  } else if (!TEL_ONLY && !GRID_ONLY && sk.kind == PHOTON_SINK_PLANE) {
    if (active && slot_q < (uint64_t)sk.plane_capacity) {
      ((T*)sk.px)[slot_q] = p.x;
      ((T*)sk.py)[slot_q] = p.y;
      sk.pz[slot_q] = p.z;
      ((T*)sk.pux)[slot_q] = p.ux;
      ((T*)sk.puy)[slot_q] = p.uy;
      sk.puz[slot_q] = (double)p.uz;
      ((T*)sk.plam)[slot_q] = p.lambda;
      ((T*)sk.pw)[slot_q] = p.w;
      sk.pt[slot_q] = p.t;
      sk.ppath[slot_q] = p.path;
      sk.pseg[slot_q] = seg_row;
      sk.pj[slot_q] = j;
      sk.pstatus[slot_q] = p.status;
    }
  } else if (!GRID_ONLY && (TEL_ONLY || sk.kind == PHOTON_SINK_TELESCOPES)) {
    int k = -1;
    T s_hit = (T)0;
    if (active && st == PHOTON_LANDED) {
      uint32_t mask;
      if (-p.uz >= (T)kCapCos) {
        // cell indices rounded down (negative outside the grid on the low
        // side, so one unsigned comparison per axis bounds them)
        const T fx = (p.x - (T)sk.cand_x0) * (T)sk.cand_inv_cell;
        const T fy = (p.y - (T)sk.cand_y0) * (T)sk.cand_inv_cell;
        uint32_t ix, iy;
        if constexpr (sizeof(T) == 4) {
          ix = (uint32_t)__float2int_rd(fx);
          iy = (uint32_t)__float2int_rd(fy);
        } else {
          ix = (uint32_t)(int)floor(fmax(fmin(fx, 1e9), -1e9));
          iy = (uint32_t)(int)floor(fmax(fmin(fy, 1e9), -1e9));
        }
        const bool in = ix < (uint32_t)kCandCells && iy < (uint32_t)kCandCells;
        mask = in ? cand[__umul24(iy, (uint32_t)kCandCells) + ix] : 0u;
      } else {
        mask = sk.n_tel >= 32 ? 0xffffffffu : ((1u << sk.n_tel) - 1u);
      }
      if constexpr (sizeof(T) == 4)
        k = telescope_hit_masked_f(p, telf, (float)(p.z - sk.tel_hobs), mask, s_hit);
      else
        k = telescope_hit_masked<T>(p, tel, mask, s_hit);
    }
    const bool hit = k >= 0;
    const unsigned long long m = __ballot(hit);
    if (m) {
      HitRec r;
      if (hit) {
        r.seg = seg_row;
        r.j = j;
        r.tel = k;
        if constexpr (sizeof(T) == 4) {
          // the point on the sphere to float rounding (a few metres from the landing point)
          r.x = (double)(p.x + s_hit * p.ux);
          r.y = (double)(p.y + s_hit * p.uy);
          r.z = p.z + (double)(s_hit * p.uz);
          r.t = p.t + (double)(s_hit * (float)n_over_c);
        } else {
          r.x = p.x + s_hit * p.ux;
          r.y = p.y + s_hit * p.uy;
          r.z = p.z + s_hit * p.uz;
          r.t = p.t + n_over_c * s_hit;
        }
        r.ux = (float)p.ux;
        r.uy = (float)p.uy;
        r.uz = (float)p.uz;
        r.lam = (float)p.lambda;
        r.w = (float)p.w;
        st = PHOTON_HIT;
      }
      // one atomic per wave reserves the slots (in the block's LDS stage when
      // there is one, else in the output); lanes write at their rank
      const int leader = __ffsll((long long)m) - 1;
      const unsigned int nh = (unsigned int)__popcll(m);
      const unsigned int rank = lanes_below(m);
      unsigned long long base = 0;
      if (stage) {
        if (lane_id() == leader) base = atomicAdd(&stage->n, nh);
        base = lane_value(base, leader);
        if (hit) {
          if (base + rank < (unsigned long long)kHitStage) {
            stage->rec[base + rank] = r;
          } else {
            const unsigned long long slot = atomicAdd(sk.hits.count, 1ull);  // stage full
            if (slot < (unsigned long long)sk.hits.capacity) write_hit(sk.hits, slot, r);
          }
        }
      } else {
        if (lane_id() == leader) base = atomicAdd(sk.hits.count, (unsigned long long)nh);
        base = lane_value(base, leader);
        if (hit) {
          const unsigned long long slot = base + rank;
          if (slot < (unsigned long long)sk.hits.capacity) write_hit(sk.hits, slot, r);
        }
      }
    }
  } else if (GRID_ONLY || (!TEL_ONLY && sk.kind == PHOTON_SINK_GRID)) {
    if (active && st == PHOTON_LANDED) {
      const double fx = floor(((double)p.x - sk.x_min) / sk.cell);
      const double fy = floor(((double)p.y - sk.y_min) / sk.cell);
      if (fx >= 0.0 && fy >= 0.0 && fx < (double)sk.nx && fy < (double)sk.ny) {
        const int cell = (int)fy * sk.nx + (int)fx;
        atomicAdd(&sk.grid_count[cell], 1u);
        atomicAdd(&sk.grid_weight[cell], (unsigned long long)((double)p.w * 4294967296.0 + 0.5));
      } else {
        st = PHOTON_OFFGRID;
      }
    }
  }
  return st;
}

// Word k of the float telescope table (x, y, z - h_obs, R^2).
__device__ __forceinline__ float tel_float(const SinkDev& sk, int k) {
  const double v = (&sk.tel[0][0])[k];
  return (float)((k & 3) == 2 ? v - sk.tel_hobs : ((k & 3) == 3 ? v * v : v));
}

template <typename T>
__global__ __launch_bounds__(256) void k_collect(BlockView<T> b, int64_t n_ph, SinkDev sk, double n_obs) {
  const double n_over_c = n_obs * (1.0 / kC);  // ns per metre at the observation level
  __shared__ double s_tel[PHOTON_MAX_TELESCOPES][4];
  __shared__ __align__(16) float s_telf[PHOTON_MAX_TELESCOPES][4];
  __shared__ uint32_t s_cand[kCandCells * kCandCells];
  if (threadIdx.x < PHOTON_MAX_TELESCOPES * 4) {
    (&s_tel[0][0])[threadIdx.x] = (&sk.tel[0][0])[threadIdx.x];
    (&s_telf[0][0])[threadIdx.x] = tel_float(sk, threadIdx.x);
  }
  if (threadIdx.x < kCandCells * kCandCells) s_cand[threadIdx.x] = sk.cand_mask[threadIdx.x];
  __syncthreads();
  StatusCounter sc;
  sc.clear();
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = q < n_ph;
  Photon<T> p{};
  uint32_t s = 0, j = 0;
  if (active) {
    p.x = b.x[q];
    p.y = b.y[q];
    p.z = b.z[q];
    p.ux = b.ux[q];
    p.uy = b.uy[q];
    p.uzd = b.uz[q];
    p.uz = (T)p.uzd;
    p.lambda = b.lam[q];
    p.w = b.w[q];
    p.t = b.t[q];
    p.status = b.status[q];
    s = b.seg[q];
    j = b.j[q];
  }
  const int st = sk.kind == PHOTON_SINK_RADIAL
                     ? sink_photon<T, false, true>(sk, s_tel, s_telf, n_over_c, p, s, j, active, (uint64_t)q, nullptr,
                                                   nullptr, s_cand)
                     : sink_photon<T>(sk, s_tel, s_telf, n_over_c, p, s, j, active, (uint64_t)q, nullptr, nullptr,
                                      s_cand);
  if (active) sc.add(st);
  if (sk.totals) flush_status(sc, sk.totals);
}

// ------------------------------------------------------------ fused kernel --
constexpr int kWindow = 128;        // segments staged in LDS per piece of a work chunk
constexpr int kWindowSplat32 = 96;  // the same for the float splat (two blocks and their grids per CU)
// the float splat's launch: 768-thread blocks, two per CU (six waves per
// SIMD), chunks of eleven blocks' worth (about 70 segments, within the
// 96-segment window)
constexpr int kSplatBs32 = 768, kSplatChunk32 = 8448;
constexpr int kAdjSegWin = 64;      // segments staged in LDS per piece of a chunk of the adjoint
constexpr int kMaxChunk = 16384;     // photons per work chunk (the slot map's size)
constexpr int kMaxChunkSplat = 9216;
static_assert(kSplatChunk32 <= kMaxChunkSplat && 8192 <= kMaxChunkSplat, "splat chunks fit the slot map");

// Everything the fused kernels take, as one kernel argument.
struct FusedArgs {
  SegView seg;
  int64_t n_seg;
  AtmDev atm;
  GenParams g;
  uint32_t k0, k1;
  const uint64_t* offsets;
  int64_t n_ph;                       // < 0: offsets[n_seg]
  int64_t chunk;
  SinkDev sk;
  unsigned long long* cursor;         // work queue position
  unsigned long long* defer_counts;   // per block: near-horizon rays handed to the double pass
  uint2* defer_q;                     // their (segment row, j), defer_cap entries per block
  int64_t defer_cap;
  unsigned long long* defer_pref;     // exclusive prefix sums of the clamped counts (n_defer_blocks + 1)
  int32_t n_defer_blocks;             // blocks of the float kernel
};
static_assert(sizeof(FusedArgs) <= 4000, "fused kernel arguments must stay below 4 KB");

// Weight factor of segment s in the differentiable form: its Frank-Tamm mean
// at the current parameters over the frozen nominal mean (section 1.2).
template <typename T>
__device__ __forceinline__ T splat_wscale(const FusedArgs& A, int64_t s) {
  const double m0 = A.sk.mu0[s];
  const double mu = mean_cherenkov(A.seg, s, A.atm, A.g.K);
  return (T)(m0 > 0.0 ? mu / m0 : 0.0);
}

// Persistent kernel: blocks take chunks of the photon index space from an
// atomic queue; per chunk the segments it covers are found by two wave
// searches and their constants staged in LDS; every photon is generated,
// propagated and collected in registers. In the float form, rays near the
// horizon are appended to a queue for the double pass instead.
// Kernel instances (MODE bits): the sink of the differentiable form, the
// radial profile sink, the correction-table propagation, fluorescence
// emission (else Cherenkov). Each carries only its own code.
constexpr int kMSplat = 1, kMRadial = 2, kMTable = 4, kMFluo = 8, kMTel = 16, kMGrid = 32;

// Float instances are built for the waves per SIMD that their LDS allows:
// six of 256 threads (six blocks of under 26.6 KB per CU), four of 512.
// Double instances of 256 threads for two waves per SIMD (256 registers, no
// spills), that is two blocks per CU: one block's chunk set-up and barrier
// waits overlap the other's work (64-shower FP64 kernel 85.4 ms in 512-thread
// blocks, one per CU, 73.3 ms; three waves spill, 101 ms).
constexpr int fused_waves_per_eu(bool fp32, int mode, int bs) {
  // the float splat: two blocks per CU
  return (mode & kMSplat) ? (fp32 ? bs / 128 : 1)
                          : (!fp32 ? (bs == 256 ? 2 : 1) : (bs == 256 ? 6 : (bs >= 512 ? 4 : 1)));
}

template <typename T, int BS, int MODE = 0>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(fused_waves_per_eu(sizeof(T) == 4, MODE, BS))))
void k_fused(FusedArgs A) {
  constexpr bool SPLAT = (MODE & kMSplat) != 0;
  constexpr bool RADIAL = (MODE & kMRadial) != 0;
  constexpr bool TABLE = (MODE & kMTable) != 0;
  constexpr bool CHER = (MODE & kMFluo) == 0;
  // the telescope sink only (its instance carries no plane or grid code)
  constexpr bool TEL = (MODE & kMTel) != 0;
  constexpr bool GRIDS = (MODE & kMGrid) != 0;  // the grid sink only
  // float SPLAT: the block's grid in 32-bit LDS cells with carries into the
  // global grid, small enough for two blocks per CU
  constexpr bool SPLAT32 = SPLAT && sizeof(T) == 4;
  constexpr int kWin = SPLAT32 ? kWindowSplat32 : kWindow;
  // telescope tables only where a telescope sink can occur
  constexpr int kTel = (SPLAT || RADIAL) ? 1 : PHOTON_MAX_TELESCOPES;
  constexpr int kCand = (SPLAT || RADIAL) ? 1 : kCandCells * kCandCells;
  __shared__ SegConst<T> s_seg[kWin];
  __shared__ uint64_t s_off[kWin + 1];
  __shared__ uint64_t s_thr[PHOTON_MAX_LINES];
  __shared__ T s_lines[PHOTON_MAX_LINES];
  __shared__ double s_tel[kTel][4];
  __shared__ __align__(16) float s_telf[kTel][4];
  __shared__ unsigned long long s_c0;
  __shared__ int64_t s_lo, s_hi;
  __shared__ unsigned int s_dcount;
  __shared__ HitStageLds<SPLAT || RADIAL> s_hs;
  __shared__ T s_wsc[SPLAT ? kWin : 1];  // SPLAT: per-segment weight factors mu/mu0
  __shared__ AtmLane s_lane;
  __shared__ uint32_t s_cand[kCand];
  // slot map of a piece [cs, ce) of a chunk: bit i of s_bits is set where a
  // segment of the window starts at photon cs + i; s_pre holds the set bits
  // before each word and s_slot[r] the window slot of the r-th start (r = 0:
  // the segment holding cs)
  constexpr int kMapWords = (SPLAT ? kMaxChunkSplat : kMaxChunk) / 64;
  __shared__ unsigned long long s_bits[kMapWords];
  __shared__ uint32_t s_pre[kMapWords];
  __shared__ uint16_t s_slot[kWin];
  extern __shared__ unsigned long long s_splat[];  // dynamic: the block's fixed-point grid (SPLAT)
  // SPLAT: the waves share out each piece dynamically (photons in reach cost
  // more)
  constexpr bool DYN = SPLAT;
  constexpr bool LATE = sizeof(T) == 4 && CHER && !SPLAT;
  __shared__ unsigned int s_grab;
  // Isotropic fluorescence into a sink that records nothing for photons that
  // never land (grid, telescopes, radial bins): half the photons go up and
  // would leave their lanes idle beside the propagation of the others. Each
  // wave first draws its photons' direction words, whose top bit fixes the
  // sign of u_z, counts the up-going ones and passes the others on, 64 at a
  // time, through a ring of piece positions in LDS.
  constexpr bool FILT = !CHER && !SPLAT;
  constexpr int kRing = 2 * kWaveSize;
  const bool filt = FILT && !A.g.beam.on && A.sk.kind != PHOTON_SINK_PLANE;
  constexpr bool kDefer = sizeof(T) == 4;
  const bool stage_hits = !SPLAT && !RADIAL && A.sk.kind == PHOTON_SINK_TELESCOPES;
  // the block's LDS accumulator: the splat grid, or the radial bins
  unsigned long long* lds_acc = SPLAT ? (A.sk.splat_lds ? s_splat : nullptr) : (RADIAL ? s_splat : nullptr);
  const int n_cells = SPLAT ? A.sk.sg.nx * A.sk.sg.ny : 3 * A.sk.n_bins;

  const int tid = threadIdx.x;
  if (tid == 0) {
    s_dcount = 0u;
    if constexpr (!SPLAT && !RADIAL) s_hs.get()->n = 0u;
  }
  if (lds_acc) {
    if constexpr (SPLAT32)
      for (int k = tid; k < n_cells; k += BS) reinterpret_cast<uint32_t*>(lds_acc)[k] = 0u;
    else
      for (int k = tid; k < n_cells; k += BS) lds_acc[k] = 0ull;
  }
  if (tid < PHOTON_MAX_LINES) {
    s_thr[tid] = A.g.thr[tid];
    s_lines[tid] = (T)A.g.line_nm[tid];
  }
  if constexpr (!SPLAT && !RADIAL) {
    static_assert(kTel == PHOTON_MAX_TELESCOPES && kCand == kCandCells * kCandCells, "full telescope tables");
    for (int k = tid; k < PHOTON_MAX_TELESCOPES * 4; k += BS) {
      (&s_tel[0][0])[k] = (&A.sk.tel[0][0])[k];
      (&s_telf[0][0])[k] = tel_float(A.sk, k);
    }
    for (int k = tid; k < kCandCells * kCandCells; k += BS) s_cand[k] = A.sk.cand_mask[k];
  }
  atm_lane_fill(A.atm, &s_lane);
  constexpr bool cher = CHER;
  const int64_t n_seg = A.n_seg;
  const uint64_t* __restrict__ offsets = A.offsets;
  __shared__ unsigned long long s_stat[PHOTON_N_STATUS];  // the block's status totals
  if (tid < PHOTON_N_STATUS) s_stat[tid] = 0ull;
  uint64_t pk = 0;  // this lane's status counts in the current piece
  // Slots at or beyond offsets[n_seg] belong to no segment: counted INVALID.
  const uint64_t total = offsets[n_seg];
  const int64_t n_ph = A.n_ph < 0 ? (int64_t)total : A.n_ph;
  const uint64_t lim = min((uint64_t)n_ph, total);
  const double n_over_c = A.atm.n_obs * (1.0 / kC);  // ns per metre at the observation level

  for (;;) {
    if (tid == 0) s_c0 = atomicAdd(A.cursor, (unsigned long long)A.chunk);
    __syncthreads();
    const uint64_t c0 = s_c0;
    if (c0 >= (uint64_t)n_ph) break;
    const uint64_t c1 = min(c0 + (uint64_t)A.chunk, (uint64_t)n_ph);
    const uint64_t v1 = min(c1, lim);  // valid slots of this chunk: [c0, v1)
    const int wave = tid / kWaveSize;
    if (tid == 0 && c1 > max(c0, v1)) atomicAdd(&s_stat[PHOTON_INVALID], (unsigned long long)(c1 - max(c0, v1)));
    if (c0 >= v1) {
      __syncthreads();
      continue;
    }
    if (wave == (BS > kWaveSize ? 1 : 0)) {
      const int64_t sh = wave_upper_index(offsets, n_seg, v1 - 1);
      if (lane_id() == 0) s_hi = sh;
    }
    // the chunk in pieces [cs, ce) whose segments fit the LDS window (one
    // piece unless the chunk spans more than kWin segments)
    for (uint64_t cs = c0; cs < v1;) {
      if (wave == 0) {
        const int64_t sl = wave_upper_index(offsets, n_seg, cs);
        if (lane_id() == 0) s_lo = sl;
      }
      __syncthreads();
      // both ends lie in [0, n_seg) for offsets from the count call; the
      // clamps keep every index in bounds for any offsets array
      const int64_t lo = min(s_lo, n_seg - 1);
      const int64_t W_all = min(s_hi, n_seg - 1) - lo + 1;
      const int64_t W = min(W_all, (int64_t)kWin);
      // windows while the rest of the chunk has at least one photon per
      // segment; sparser chunks (mostly empty segments) look their photons'
      // segments up in global memory instead of staging every segment
      bool win = W >= 1 && (W_all <= (int64_t)kWin || (int64_t)(v1 - cs) >= W_all);
      if (win) {
        for (int t = tid; t < W; t += BS) {
          seg_const<T>(A.seg, lo + t, A.atm, cher, A.g.beam, s_seg[t]);
          if constexpr (SPLAT) s_wsc[t] = splat_wscale<T>(A, lo + t);
          s_off[t] = offsets[lo + t];
        }
        if (tid == 0) s_off[W] = offsets[lo + W];
      }
      if (DYN && tid == 0) s_grab = 0u;
      __syncthreads();
      // the piece ends where the first segment beyond the window starts
      uint64_t ce = win ? min(v1, (uint64_t)s_off[W]) : v1;
      if (!(ce > cs)) {
        ce = v1;
        win = false;
      }
      if (win) {
        const int nw = (int)((ce - cs + 63) >> 6);
        for (int k = tid; k < nw; k += BS) s_bits[k] = 0ull;
        __syncthreads();
        for (int t = tid + 1; t < W; t += BS) {
          const uint64_t st = s_off[t];
          if (st < ce && s_off[t + 1] > st) atomicOr(&s_bits[(st - cs) >> 6], 1ull << ((st - cs) & 63));
        }
        __syncthreads();
        if (wave == 0) {
          uint32_t carry = 0;
          for (int base = 0; base < nw; base += kWaveSize) {
            const int k = base + lane_id();
            const uint32_t cnt = k < nw ? (uint32_t)__popcll(s_bits[k]) : 0u;
            const uint32_t inc = (uint32_t)wave_incl_scan((unsigned long long)cnt);
            if (k < nw) s_pre[k] = carry + inc - cnt;
            carry += (uint32_t)__shfl(inc, kWaveSize - 1, kWaveSize);
          }
        }
        __syncthreads();
        if (tid == 0) s_slot[0] = 0;
        for (int t = tid + 1; t < W; t += BS) {
          const uint64_t st = s_off[t];
          if (st < ce && s_off[t + 1] > st) {
            const uint64_t i = st - cs;
            const uint32_t r = s_pre[i >> 6] + (uint32_t)__popcll(s_bits[i >> 6] & ((2ull << (i & 63)) - 1ull));
            s_slot[r] = (uint16_t)t;
          }
        }
        __syncthreads();
      }
      // filtered fluorescence: the wave's ring (head, length) and the next
      // block group of the piece whose directions are drawn; all wave-uniform
      uint32_t r_head = 0u, r_len = 0u, n_up = 0u;
      uint64_t q_draw = cs;
      // every lane of a wave runs the same number of iterations (the status
      // ballots); DYN: the waves take 64-photon groups of the piece from an
      // LDS counter, so that a wave slowed by its photons (splats) takes fewer
      for (uint32_t ng = 0;; ++ng) {
        uint64_t qb;
        if constexpr (DYN) {
          unsigned int g0 = 0u;
          if (lane_id() == 0) g0 = atomicAdd(&s_grab, (unsigned int)kWaveSize);
          qb = cs + (uint64_t)__shfl(g0, 0, kWaveSize);
        } else {
          qb = cs + (uint64_t)ng * BS;
        }
        uint64_t q_ring = 0;  // filtered fluorescence: the lane's photon from the ring, ce for none
        if constexpr (FILT) {
          if (filt) {
            __shared__ uint16_t s_ring[BS / kWaveSize][kRing];
            // draw directions group by group (the wave's slice of each block
            // group, as in the plain schedule) until the ring holds 64 photons
            while (r_len < (uint32_t)kWaveSize && q_draw < ce) {
              const uint64_t q = q_draw + (uint64_t)tid;
              const bool valid = q < ce;
              bool down = valid;
              if (valid && win) {
                const uint64_t i = q - cs;
                const int a = s_slot[s_pre[i >> 6] + (uint32_t)__popcll(s_bits[i >> 6] & ((2ull << (i & 63)) - 1ull))];
                const U4 r = philox((uint32_t)(q - s_off[a]), s_seg[a].idx, s_seg[a].shower, kDomFluo, A.k0, A.k1);
                down = (r.w[1] >> 31) != 0u;  // u_z = -(w1 - 2^31 + 1/2) 2^-31 < 0
              }
              const unsigned long long m = __ballot(down);
              n_up += (uint32_t)__popcll(__ballot(valid)) - (uint32_t)__popcll(m);
              if (down) s_ring[wave][(r_head + r_len + lanes_below(m)) & (kRing - 1)] = (uint16_t)(q - cs);
              r_len += (uint32_t)__popcll(m);
              q_draw += BS;
            }
            qb = r_len ? cs : ce;  // an empty ring ends the piece
            if (r_len) {
              // the lanes' ring writes before the reads of other lanes' entries
              __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
              const uint32_t take = min(r_len, (uint32_t)kWaveSize);
              q_ring = (uint32_t)lane_id() < take ? cs + s_ring[wave][(r_head + (uint32_t)lane_id()) & (kRing - 1)] : ce;
              // the reads before the next round's writes
              __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
              __builtin_amdgcn_wave_barrier();
              __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
              r_head += take;
              r_len -= take;
            }
          }
        }
        if (qb >= ce) break;
        const uint64_t q0 = (FILT && filt) ? q_ring : qb + (DYN ? (uint64_t)lane_id() : (uint64_t)tid);
        int st_out = -1;
        bool forced = false;
        // photon qq of the piece: its segment (from the window's slot map, or
        // looked up in global memory) and the photon itself
        auto fetch = [&](uint64_t qq, SegConst<T>& c, int64_t& s, uint32_t& j, T& wsc, Photon<T>& p) {
          uint64_t off_s;
          if (win) {
            // starts at or before qq, counted from the map
            const uint64_t i = qq - cs;
            const int a = s_slot[s_pre[i >> 6] + (uint32_t)__popcll(s_bits[i >> 6] & ((2ull << (i & 63)) - 1ull))];
            c = s_seg[a];
            if constexpr (SPLAT) wsc = s_wsc[a];
            off_s = s_off[a];
            // keeps the LDS load and the global one below apart (merged, they
            // would become one generic load through a selected pointer)
            asm volatile("" : "+v"(off_s));
            s = lo + a;
          } else {
            s = lane_upper_index(offsets, n_seg, qq);
            seg_const<T>(A.seg, s, A.atm, cher, A.g.beam, c);
            if constexpr (SPLAT) wsc = splat_wscale<T>(A, s);
            off_s = offsets[s];
          }
          j = (uint32_t)(qq - off_s);
          generate_kind<T, CHER>(c, j, A.g, A.k0, A.k1, s_thr, s_lines, p);
        };
        // its propagation and sink
        auto finish = [&](const SegConst<T>& c, int64_t s, uint32_t j, T wsc, Photon<T>& p, uint64_t qq) {
          propagate<T, kDefer, false, TABLE>(A.atm, s_lane, p, c.layer);
          if constexpr (SPLAT) p.w *= wsc;
          if (kDefer) {
            const bool defer = p.status == kDeferred;
            const unsigned long long m = __ballot(defer);
            if (m) {
              // the block's own queue: one LDS atomic per wave
              const int leader = __ffsll((long long)m) - 1;
              unsigned int base = 0;
              if (lane_id() == leader) base = atomicAdd(&s_dcount, (unsigned int)__popcll(m));
              base = lane_value(base, leader);
              if (defer) {
                const uint64_t slot = (uint64_t)base + lanes_below(m);
                if (slot < (uint64_t)A.defer_cap) {
                  A.defer_q[(uint64_t)blockIdx.x * (uint64_t)A.defer_cap + slot] = make_uint2((uint32_t)s, j);
                } else {
                  // queue full: this ray is evaluated here after all, in
                  // double as the photon-block path does
                  p.status = PHOTON_LANDED;
                  propagate<T>(A.atm, s_lane, p, c.layer);
                  forced = true;
                }
              }
            }
          }
          if (!kDefer || p.status != kDeferred) {
            if constexpr (SPLAT32) {
              st_out = p.status;
              if (st_out == PHOTON_LANDED) {
                const bool in = lds_acc ? splat_add32(A.sk.sg, (double)p.x, (double)p.y, (float)p.w,
                                                      reinterpret_cast<uint32_t*>(lds_acc), A.sk.splat_acc)
                                        : splat_add<float>(A.sk.sg, (double)p.x, (double)p.y, (float)p.w,
                                                           A.sk.splat_acc);
                if (!in) st_out = PHOTON_OFFGRID;
              }
            } else {
              st_out = sink_photon<T, SPLAT, RADIAL, TEL, GRIDS>(A.sk, s_tel, s_telf, n_over_c, p, (uint32_t)s, j, true, qq,
                                                     stage_hits ? s_hs.get() : nullptr, lds_acc, s_cand);
            }
          }
        };
        // Two arrangements of the same work, chosen by measurement: the
        // photon's state declared outside the lane's test and the two steps
        // as the calls above (LATE) make the float Cherenkov forms faster
        // (64-shower FP32 kernel 22.9 -> 21.3 ms) and the double ones and
        // the float splat slower (85.3 -> 92.0 ms; 3.39 -> 3.53 ms), which
        // keep the steps written out inside the test (the same statements as
        // fetch and finish).
        if constexpr (LATE) {
          uint64_t q = q0;
          bool have = q < ce;
          SegConst<T> c;
          int64_t s = 0;
          uint32_t j = 0;
          T wsc = (T)1;
          Photon<T> p;
          if (have) {
            fetch(q, c, s, j, wsc, p);
            finish(c, s, j, wsc, p, q);
          }
        } else {
          if (q0 < ce) {
            SegConst<T> c;
            int64_t s;
            uint32_t j;
            T wsc = (T)1;
            Photon<T> p;
            {
              const uint64_t qq = q0;
              uint64_t off_s;
              if (win) {
                // starts at or before qq, counted from the map
                const uint64_t i = qq - cs;
                const int a = s_slot[s_pre[i >> 6] + (uint32_t)__popcll(s_bits[i >> 6] & ((2ull << (i & 63)) - 1ull))];
                c = s_seg[a];
                if constexpr (SPLAT) wsc = s_wsc[a];
                off_s = s_off[a];
                // keeps the LDS load and the global one below apart (merged,
                // they would become one generic load through a selected pointer)
                asm volatile("" : "+v"(off_s));
                s = lo + a;
              } else {
                s = lane_upper_index(offsets, n_seg, qq);
                seg_const<T>(A.seg, s, A.atm, cher, A.g.beam, c);
                if constexpr (SPLAT) wsc = splat_wscale<T>(A, s);
                off_s = offsets[s];
              }
              j = (uint32_t)(qq - off_s);
              generate_kind<T, CHER>(c, j, A.g, A.k0, A.k1, s_thr, s_lines, p);
            }
            {
              const uint64_t qq = q0;
              propagate<T, kDefer, false, TABLE>(A.atm, s_lane, p, c.layer);
              if constexpr (SPLAT) p.w *= wsc;
              if (kDefer) {
                const bool defer = p.status == kDeferred;
                const unsigned long long m = __ballot(defer);
                if (m) {
                  // the block's own queue: one LDS atomic per wave
                  const int leader = __ffsll((long long)m) - 1;
                  unsigned int base = 0;
                  if (lane_id() == leader) base = atomicAdd(&s_dcount, (unsigned int)__popcll(m));
                  base = lane_value(base, leader);
                  if (defer) {
                    const uint64_t slot = (uint64_t)base + lanes_below(m);
                    if (slot < (uint64_t)A.defer_cap) {
                      A.defer_q[(uint64_t)blockIdx.x * (uint64_t)A.defer_cap + slot] = make_uint2((uint32_t)s, j);
                    } else {
                      // queue full: this ray is evaluated here after all, in
                      // double as the photon-block path does
                      p.status = PHOTON_LANDED;
                      propagate<T>(A.atm, s_lane, p, c.layer);
                      forced = true;
                    }
                  }
                }
              }
              if (!kDefer || p.status != kDeferred) {
                if constexpr (SPLAT32) {
                  st_out = p.status;
                  if (st_out == PHOTON_LANDED) {
                    const bool in = lds_acc ? splat_add32(A.sk.sg, (double)p.x, (double)p.y, (float)p.w,
                                                          reinterpret_cast<uint32_t*>(lds_acc), A.sk.splat_acc)
                                            : splat_add<float>(A.sk.sg, (double)p.x, (double)p.y, (float)p.w,
                                                               A.sk.splat_acc);
                    if (!in) st_out = PHOTON_OFFGRID;
                  }
                } else {
                  st_out = sink_photon<T, SPLAT, RADIAL, TEL, GRIDS>(A.sk, s_tel, s_telf, n_over_c, p, (uint32_t)s, j, true, qq,
                                                         stage_hits ? s_hs.get() : nullptr, lds_acc, s_cand);
                }
              }
            }
          }
        }
        pk += status_inc(st_out);
        if (kDefer && forced) pk += status_inc(PHOTON_HORIZON_FLOAT);
        if (DYN && (ng & 63u) == 63u) {
          // a lane's 8-bit counters hold 64 photons' increments
          flush_lane_status(pk, s_stat);
          pk = 0;
        }
      }
      // the per-lane 8-bit counters stay below 256 increments per piece
      flush_lane_status(pk, s_stat);
      pk = 0;
      if (FILT && n_up && lane_id() == 0) atomicAdd(&s_stat[PHOTON_UP], (unsigned long long)n_up);
      cs = ce;
      __syncthreads();  // the window is refilled for the next piece
    }
    if constexpr (!SPLAT && !RADIAL) {
      if (stage_hits) flush_hits(s_hs.get(), A.sk.hits);
    }
    __syncthreads();
  }
  if (kDefer && tid == 0) {
    const uint64_t nd = s_dcount;
    A.defer_counts[blockIdx.x] = nd < (uint64_t)A.defer_cap ? nd : (uint64_t)A.defer_cap;
  }
  if (lds_acc) {
    // the block's accumulator into the global one (the loop above ends with a barrier)
    if constexpr (SPLAT32) {
      for (int k = tid; k < n_cells; k += BS) {
        const uint32_t v = reinterpret_cast<const uint32_t*>(lds_acc)[k];
        if (v) atomicAdd(&A.sk.splat_acc[k], (unsigned long long)v);
      }
    } else if constexpr (SPLAT) {
      for (int k = tid; k < n_cells; k += BS) {
        const unsigned long long v = lds_acc[k];
        if (v) atomicAdd(&A.sk.splat_acc[k], v);
      }
    } else {
      const int nb = A.sk.n_bins;
      for (int k = tid; k < nb; k += BS) {
        const unsigned long long c = lds_acc[k];
        if (c) {
          atomicAdd(&A.sk.rad_count[k], c);
          atomicAdd(&A.sk.rad_w[k], lds_acc[nb + k]);
          atomicAdd(&A.sk.rad_wt[k], lds_acc[2 * nb + k]);
        }
      }
    }
  }
  // the block's status totals (the loop above ends with a barrier)
  if (A.sk.totals && tid < PHOTON_N_STATUS && s_stat[tid]) atomicAdd(&A.sk.totals[tid], s_stat[tid]);
}

// Exclusive prefix sums of the per-block queue lengths (each clamped to the
// queue capacity), pref[0..nb]; one block, nb <= 8192.
__global__ __launch_bounds__(1024) void k_defer_scan(const unsigned long long* __restrict__ counts, int nb,
                                                     int64_t cap, unsigned long long* __restrict__ pref) {
  __shared__ unsigned long long s_w[1024 / kWaveSize];
  constexpr int P = 8;
  const int t = threadIdx.x;
  unsigned long long v[P], sum = 0;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int i = t * P + k;
    const unsigned long long c = i < nb ? counts[i] : 0ull;
    v[k] = c < (unsigned long long)cap ? c : (unsigned long long)cap;
    sum += v[k];
  }
  const unsigned long long inc = wave_incl_scan(sum);
  if (lane_id() == kWaveSize - 1) s_w[t / kWaveSize] = inc;
  __syncthreads();
  if (t == 0) {
    unsigned long long run = 0;
    for (int w = 0; w < 1024 / kWaveSize; ++w) {
      const unsigned long long x = s_w[w];
      s_w[w] = run;
      run += x;
    }
  }
  __syncthreads();
  unsigned long long base = s_w[t / kWaveSize] + inc - sum;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int i = t * P + k;
    if (i < nb) pref[i] = base;
    base += v[k];
    if (i == nb - 1) pref[nb] = base;
  }
}

constexpr int kDeferOther = 0, kDeferSplat = 1, kDeferRadial = 2;

// Double pass over the near-horizon rays queued by the float kernel: each is
// regenerated in double from its counter-based random numbers and carried
// through propagation and collection in double. The queues of all blocks
// are taken as one list (numbered through defer_pref), spread evenly over
// the threads.
// Built for two waves per SIMD: the double evaluation needs more than 256
// registers, and at one wave per SIMD its latency is exposed.
// SINK: the sink class of the run (kDeferSplat, kDeferRadial, or
// kDeferOther for the plane, telescopes and grid), one instance each, so
// that each carries only its own sink's registers.
template <int BS, int SINK>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(2))) void k_fused_deferred(FusedArgs A) {
  __shared__ uint64_t s_thr[PHOTON_MAX_LINES];
  __shared__ double s_lines[PHOTON_MAX_LINES];
  __shared__ double s_tel[PHOTON_MAX_TELESCOPES][4];
  __shared__ __align__(16) float s_telf[PHOTON_MAX_TELESCOPES][4];
  __shared__ AtmLane s_lane;
  __shared__ uint32_t s_cand[kCandCells * kCandCells];
  const int tid = threadIdx.x;
  // blocks beyond the queued rays leave before staging their tables (the
  // grid is sized for the largest queue; usually a few blocks have work)
  if ((uint64_t)blockIdx.x * BS >= A.defer_pref[A.n_defer_blocks]) return;
  if (tid < PHOTON_MAX_LINES) {
    s_thr[tid] = A.g.thr[tid];
    s_lines[tid] = A.g.line_nm[tid];
  }
  for (int k = tid; k < PHOTON_MAX_TELESCOPES * 4; k += BS) {
    (&s_tel[0][0])[k] = (&A.sk.tel[0][0])[k];
    (&s_telf[0][0])[k] = tel_float(A.sk, k);
  }
  for (int k = tid; k < kCandCells * kCandCells; k += BS) s_cand[k] = A.sk.cand_mask[k];
  atm_lane_fill(A.atm, &s_lane);
  __syncthreads();
  const bool cher = A.g.kind == PHOTON_CHERENKOV;
  const double n_over_c = A.atm.n_obs * (1.0 / kC);
  StatusCounter sc;
  sc.clear();
  const unsigned long long* __restrict__ pref = A.defer_pref;
  const int nb = A.n_defer_blocks;
  const uint64_t total = pref[nb];
  for (uint64_t g = (uint64_t)blockIdx.x * BS + tid; g < total; g += (uint64_t)gridDim.x * BS) {
    int lo = 0, hi = nb;  // pref[lo] <= g < pref[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pref[mid] <= g) lo = mid; else hi = mid;
    }
    const uint2 e = A.defer_q[(uint64_t)lo * (uint64_t)A.defer_cap + (g - pref[lo])];
    const int64_t s = e.x < (uint32_t)A.n_seg ? (int64_t)e.x : A.n_seg - 1;
    SegConst<double> c;
    seg_const<double>(A.seg, s, A.atm, cher, A.g.beam, c);
    Photon<double> p;
    generate<double>(c, e.y, A.g, A.k0, A.k1, s_thr, s_lines, p);
    propagate<double>(A.atm, s_lane, p);
    constexpr bool splat = SINK == kDeferSplat;
    if (splat) p.w *= splat_wscale<double>(A, s);
    // collected in the run's precision (float)
    Photon<float> pf;
    pf.x = (float)p.x;
    pf.y = (float)p.y;
    pf.ux = (float)p.ux;
    pf.uy = (float)p.uy;
    pf.uz = (float)p.uz;
    pf.uzd = p.uzd;
    pf.lambda = (float)p.lambda;
    pf.w = (float)p.w;
    pf.z = p.z;
    pf.t = p.t;
    pf.path = p.path;
    pf.status = p.status;
    int st;
    if constexpr (SINK == kDeferSplat)
      st = sink_photon<float, true>(A.sk, s_tel, s_telf, n_over_c, pf, (uint32_t)s, e.y, true, 0, nullptr,
                                    nullptr, s_cand);
    else if constexpr (SINK == kDeferRadial)
      st = sink_photon<float, false, true>(A.sk, s_tel, s_telf, n_over_c, pf, (uint32_t)s, e.y, true, 0,
                                           nullptr, nullptr, s_cand);
    else
      st = sink_photon<float>(A.sk, s_tel, s_telf, n_over_c, pf, (uint32_t)s, e.y, true, A.offsets[s] + e.y,
                              nullptr, nullptr, s_cand);
    sc.add(st);
  }
  if (A.sk.totals) flush_status(sc, A.sk.totals);
}

// ---------------------------------------------- adjoint of the splatted density --
struct AdjArgs {
  SegView seg;
  int64_t n_seg;
  AtmDev atm;
  uint32_t k0, k1;
  double K, inv_l1, inv_dl;
  const uint64_t* offsets;   // frozen counts' offsets (n_seg + 1)
  int64_t chunk;
  const double* mu0;         // frozen nominal means
  SplatGeom sg;
  const void* grad;          // dL/dD, the run's precision
  double *gdx, *gdy, *gdz;   // per-segment direction gradients (accumulated)
  double* partials;          // kAdjWords per block (float form: then as many for the double pass)
  unsigned long long* cursor;
  unsigned long long* defer_counts;  // float form: per block, rays near the horizon left to the double pass
  uint2* defer_q;                    // their (segment row, j), defer_cap entries per block
  int64_t defer_cap;
  unsigned long long* defer_pref;    // exclusive prefix sums of the clamped counts (n_defer_blocks + 1)
  int32_t n_defer_blocks;
};

__device__ __forceinline__ SegRaw load_seg_raw(const AdjArgs& A, int64_t s) {
  SegRaw sg;
  sg.x0 = A.seg.x0[s];
  sg.y0 = A.seg.y0[s];
  sg.z0 = A.seg.z0[s];
  sg.dx = A.seg.dx[s];
  sg.dy = A.seg.dy[s];
  sg.dz = A.seg.dz[s];
  sg.len = A.seg.len[s];
  sg.beta = A.seg.beta[s];
  sg.zz = A.seg.charge ? (double)(A.seg.charge[s] * A.seg.charge[s]) : 1.0;
  sg.mu0 = A.mu0[s];
  sg.idx = seg_idx(A.seg, s);
  sg.shower = seg_shower(A.seg, s);
  return sg;
}

// Block sums of the lane-private accumulators, in thread order, into one
// row of partials (the caller has synchronised the block).
template <int BS>
__device__ __forceinline__ void adj_block_sums(const double* s_acc, double* row) {
  const int tid = threadIdx.x;
  if (tid < kAdjWords) {
    double t = 0.0;
    for (int i = 0; i < BS; ++i) t += s_acc[tid * BS + i];
    row[tid] = t;
  }
}

// Sums over each run of equal keys of a wave (keys nondecreasing over the
// lanes that hold a photon, negative and distinct in the others); the last
// lane of a run adds the run's sums to the outputs, one atomic per component.
__device__ __forceinline__ void seg_reduce_add(long long key, double v0, double v1, double v2, double* o0,
                                               double* o1, double* o2) {
  // nothing to add anywhere in the wave (every photon out of reach): done
  if (__ballot(v0 != 0.0 || v1 != 0.0 || v2 != 0.0) == 0ull) return;
  const int lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWaveSize; d <<= 1) {
    const long long ku = __shfl_up(key, d, kWaveSize);
    const double a0 = __shfl_up(v0, d, kWaveSize);
    const double a1 = __shfl_up(v1, d, kWaveSize);
    const double a2 = __shfl_up(v2, d, kWaveSize);
    if (lane >= d && ku == key) {
      v0 += a0;
      v1 += a1;
      v2 += a2;
    }
  }
  const long long kn = __shfl_down(key, 1, kWaveSize);
  const bool last = lane == kWaveSize - 1 || kn != key;
  if (last && key >= 0 && (v0 != 0.0 || v1 != 0.0 || v2 != 0.0)) {
    atomicAdd(&o0[key], v0);
    atomicAdd(&o1[key], v1);
    atomicAdd(&o2[key], v2);
  }
}

// Persistent like k_fused: chunks of the photon index space from an atomic
// queue, each taken in pieces of at most kAdjSegWin segments whose offsets
// and per-segment constants (adj_seg_setup) are staged in LDS once per piece
// (a piece starts at the segment of the first photon left, so runs of empty
// segments are skipped). Every photon is regenerated and carried forward and
// back (adjoint_photon); direction gradients are reduced per segment over the
// wave, the global sums per block into partials (summed in a fixed order by
// k_adj_finalize). The float form queues rays near the horizon for
// k_splat_adjoint_deferred.
template <typename T, int BS>
// Built for three waves per SIMD (float) or two (double): the spills this
// costs are cheaper than the latency two waves (one) leave exposed (FP32
// adjoint on the 1e6-segment workload 9.05 -> 7.70 ms, FP64 18.7 -> 12.7 ms;
// four float waves spill too much, 9.4 ms).
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 2))) void k_splat_adjoint(
    AdjArgs A) {
  __shared__ uint64_t s_off[kAdjSegWin + 1];
  __shared__ AdjSeg s_seg[kAdjSegWin];
  __shared__ unsigned int s_grab;
  __shared__ unsigned long long s_c0;
  __shared__ int64_t s_lo, s_hi;
  __shared__ double s_acc[kAdjWords * BS];  // lane-private sums: word k of thread t at k * BS + t
  __shared__ AtmLane s_lane;
  __shared__ unsigned int s_dcount;
  constexpr bool kDefer = sizeof(T) == 4;
  const int tid = threadIdx.x;
  if (tid == 0) s_dcount = 0u;
  atm_lane_fill(A.atm, &s_lane);
  const int64_t n_seg = A.n_seg;
  const uint64_t* __restrict__ offsets = A.offsets;
  const uint64_t total = offsets[n_seg];
  const T* G = (const T*)A.grad;
  for (int k = 0; k < kAdjWords; ++k) s_acc[k * BS + tid] = 0.0;
  // window entries not yet set up read as segments that emit nothing
  for (int t = tid; t < kAdjSegWin; t += BS) s_seg[t].ok = 0;
  const AdjAcc acc{&s_acc[tid], BS};
  for (;;) {
    if (tid == 0) s_c0 = atomicAdd(A.cursor, (unsigned long long)A.chunk);
    __syncthreads();  // also: the atmosphere record is filled
    const uint64_t c0 = s_c0;
    if (c0 >= total) break;
    const uint64_t v1 = min(c0 + (uint64_t)A.chunk, total);
    const int wave = tid / kWaveSize;
    if (wave == (BS > kWaveSize ? 1 : 0)) {
      const int64_t sh = wave_upper_index(offsets, n_seg, v1 - 1);
      if (lane_id() == 0) s_hi = sh;
    }
    for (uint64_t cs = c0; cs < v1;) {
      if (wave == 0) {
        const int64_t sl = wave_upper_index(offsets, n_seg, cs);
        if (lane_id() == 0) s_lo = sl;
      }
      __syncthreads();
      // both ends lie in [0, n_seg) for offsets from the count call; the
      // clamps keep every index in bounds for any offsets array
      const int64_t lo = min(s_lo, n_seg - 1);
      const int W = (int)max(min(min(s_hi, n_seg - 1) - lo + 1, (int64_t)kAdjSegWin), (int64_t)1);
      for (int t = tid; t <= W; t += BS) s_off[t] = offsets[lo + t];
      for (int t = tid; t < W; t += BS) {
        // segments without photons are never looked up
        if (offsets[lo + t + 1] > offsets[lo + t])
          adj_seg_setup(A.atm, s_lane, load_seg_raw(A, lo + t), seg_ok(A.seg, lo + t), A.K, s_seg[t]);
      }
      if (tid == 0) s_grab = 0u;
      __syncthreads();
      // the piece ends where the first segment beyond the window starts (for
      // offsets that do not increase, the rest of the chunk is one piece)
      uint64_t ce = min(v1, (uint64_t)s_off[W]);
      if (!(ce > cs)) ce = v1;
      // the waves take 64-photon groups of the piece from an LDS counter (a
      // wave slowed by photons in reach takes fewer)
      for (;;) {
        unsigned int g0 = 0u;
        if (lane_id() == 0) g0 = atomicAdd(&s_grab, (unsigned int)kWaveSize);
        const uint64_t qb = cs + (uint64_t)__shfl(g0, 0, kWaveSize);
        if (qb >= ce) break;
        const uint64_t q = qb + (uint64_t)lane_id();
        long long key = -1 - (long long)lane_id();
        double dd[3] = {0.0, 0.0, 0.0};
        if (q < ce) {
          int a = 0, b = W;  // s_off[a] <= q < s_off[b]
          while (b - a > 1) {
            const int mid = (a + b) >> 1;
            if (s_off[mid] <= q) a = mid; else b = mid;
          }
          const int64_t s = lo + a;
          key = s;
          const uint32_t j = (uint32_t)(q - s_off[a]);
          const AdjSeg& sg = s_seg[a];
          const int out = adjoint_photon<T, T>(A.atm, s_lane, sg, j, A.k0, A.k1, A.inv_l1, A.inv_dl, A.sg, G, acc, dd);
          if (kDefer) {
            const bool defer = out == kAdjDeferred;
            const unsigned long long m = __ballot(defer);
            if (m) {
              // the block's own queue: one LDS atomic per wave
              const int leader = __ffsll((long long)m) - 1;
              unsigned int base = 0;
              if (lane_id() == leader) base = atomicAdd(&s_dcount, (unsigned int)__popcll(m));
              base = lane_value(base, leader);
              if (defer) {
                const uint64_t slot = (uint64_t)base + lanes_below(m);
                if (slot < (uint64_t)A.defer_cap)
                  A.defer_q[(uint64_t)blockIdx.x * (uint64_t)A.defer_cap + slot] = make_uint2((uint32_t)s, j);
                else  // queue full: evaluated in float after all
                  adjoint_photon<T, T, true>(A.atm, s_lane, sg, j, A.k0, A.k1, A.inv_l1, A.inv_dl, A.sg, G, acc,
                                             dd);
              }
            }
          }
        }
        seg_reduce_add(key, dd[0], dd[1], dd[2], A.gdx, A.gdy, A.gdz);
      }
      cs = ce;
      __syncthreads();  // the window is refilled for the next piece
    }
  }
  if (kDefer && tid == 0) {
    const uint64_t nd = s_dcount;
    A.defer_counts[blockIdx.x] = nd < (uint64_t)A.defer_cap ? nd : (uint64_t)A.defer_cap;
  }
  adj_block_sums<BS>(s_acc, A.partials + (int64_t)blockIdx.x * kAdjWords);
}

// Double pass over the rays near the horizon queued by the float adjoint:
// the queues of all blocks are taken as one list (numbered through
// defer_pref) spread evenly over the threads; block b writes its sums to
// partial row row0 + b; direction gradients are added per photon.
template <int BS>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(2))) void k_splat_adjoint_deferred(
    AdjArgs A, int64_t row0) {
  __shared__ double s_acc[kAdjWords * BS];
  __shared__ AtmLane s_lane;
  const int tid = threadIdx.x;
  atm_lane_fill(A.atm, &s_lane);
  for (int k = 0; k < kAdjWords; ++k) s_acc[k * BS + tid] = 0.0;
  __syncthreads();
  const AdjAcc acc{&s_acc[tid], BS};
  const float* G = (const float*)A.grad;
  const unsigned long long* __restrict__ pref = A.defer_pref;
  const int nb = A.n_defer_blocks;
  const uint64_t total = pref[nb];
  for (uint64_t g = (uint64_t)blockIdx.x * BS + tid; g < total; g += (uint64_t)gridDim.x * BS) {
    int lo = 0, hi = nb;  // pref[lo] <= g < pref[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pref[mid] <= g) lo = mid; else hi = mid;
    }
    const uint2 e = A.defer_q[(uint64_t)lo * (uint64_t)A.defer_cap + (g - pref[lo])];
    const int64_t s = e.x < (uint32_t)A.n_seg ? (int64_t)e.x : A.n_seg - 1;
    AdjSeg sg;
    adj_seg_setup(A.atm, s_lane, load_seg_raw(A, s), true, A.K, sg);
    double dd[3] = {0.0, 0.0, 0.0};
    if (adjoint_photon<double, float>(A.atm, s_lane, sg, e.y, A.k0, A.k1, A.inv_l1, A.inv_dl, A.sg, G, acc, dd) ==
        kAdjDone) {
      atomicAdd(&A.gdx[s], dd[0]);
      atomicAdd(&A.gdy[s], dd[1]);
      atomicAdd(&A.gdz[s], dd[2]);
    }
  }
  __syncthreads();
  adj_block_sums<BS>(s_acc, A.partials + (row0 + (int64_t)blockIdx.x) * kAdjWords);
}

// Sums the block partials in block order and maps them to the parameters:
// dL/dH_k = direct part + sum over layers m > k of dL/d ln rb[m] times
// d ln rb[m]/dH_k = (hb[k+1] - hb[k])/H_k^2 (rb[m] is the product of
// exp(-(hb[i+1] - hb[i])/H_i) over i < m). Layers of infinite scale height get 0.
__global__ __launch_bounds__(64) void k_adj_finalize(const double* __restrict__ partials, int nb, AtmDev atm,
                                                     double* grad_H, double* grad_eta) {
  __shared__ double s[kAdjWords];
  const int k = threadIdx.x;
  if (k < kAdjWords) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += partials[(int64_t)b * kAdjWords + k];
    s[k] = t;
  }
  __syncthreads();
  if (k < atm.nl) {
    const bool homog = (atm.homog_mask >> k) & 1;
    double g = s[PHOTON_MAX_LAYERS + k];
    if (k + 1 < atm.nl) {
      const double f = (atm.hb[k + 1] - atm.hb[k]) * atm.invH[k] * atm.invH[k];
      for (int m = k + 1; m < atm.nl; ++m) g += s[m] * f;
    }
    grad_H[k] = homog ? 0.0 : g;
  }
  if (k == 0) *grad_eta = s[2 * PHOTON_MAX_LAYERS];
}

// Density from the fixed-point accumulator: D = norm * acc / splat_unit<T>().
template <typename T>
__global__ __launch_bounds__(256) void k_splat_finish(const unsigned long long* __restrict__ acc, int n, double norm,
                                                      T* __restrict__ D) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) D[i] = (T)((double)acc[i] * (norm / splat_unit<T>()));
}

// Per-segment means (section 1.2 Frank-Tamm, section 1.1 yield), the same
// evaluation as the count kernel's.
template <int KIND>
__global__ __launch_bounds__(256) void k_means(SegView seg, int64_t n, AtmDev atm, double K, CutDev cut,
                                               BeamDev beam, double* mean) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  mean[i] = KIND == PHOTON_CHERENKOV ? (passes_cut(seg, i, cut) ? mean_cherenkov(seg, i, atm, K) : 0.0)
                                     : beamed_mean(seg, i, beam, mean_fluor(seg, i, K));
}

// Radial profiles from the fixed-point sums, one thread per bin: density =
// weight / annulus area, mean time = t_ref + sum w (t - t_ref) / sum w.
__global__ __launch_bounds__(256) void k_radial_finish(SinkDev sk, double r_max, double* __restrict__ density,
                                                       double* __restrict__ mean_t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= sk.n_bins) return;
  const double n = (double)sk.n_bins;
  double r0, r1;
  if (sk.log_bins) {
    const double q = r_max / sk.r_min;
    r0 = sk.r_min * pow(q, (double)k / n);
    r1 = k + 1 == sk.n_bins ? r_max : sk.r_min * pow(q, (double)(k + 1) / n);
  } else {
    const double span = r_max - sk.r_min;
    r0 = sk.r_min + span * ((double)k / n);
    r1 = k + 1 == sk.n_bins ? r_max : sk.r_min + span * ((double)(k + 1) / n);
  }
  const double w = (double)sk.rad_w[k] * 0x1p-32;
  const double wt = (double)(long long)sk.rad_wt[k] * 0x1p-8;
  density[k] = w / (kPi * (r1 * r1 - r0 * r0));
  mean_t[k] = w > 0.0 ? sk.t_ref + wt / w : __builtin_nan("");
}

// Correction tables of the straight-line propagation, one thread per node:
// the exact integrals in double at (h_i, q_j) minus the straight line; the
// threads past the 2-D nodes fill the 1-D table of density and vertical
// column.
__global__ __launch_bounds__(256) void k_table_build(AtmDev a, int n_h, int n_q, int n_v, double h_max, double q_max,
                                                     float4* __restrict__ corr, float2* __restrict__ vert) {
  __shared__ AtmLane s_lane;
  atm_lane_fill(a, &s_lane);
  __syncthreads();
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n2 = (int64_t)n_h * n_q;
  const double span = h_max - a.hobs;
  double g0, pth, opt, col, ne, em, rb;
  if (idx < n2) {
    const int i = (int)(idx / n_q), j = (int)(idx % n_q);
    const double h = a.hobs + span * ((double)i / (double)(n_h - 1));
    const double dh = h - a.hobs;
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    if (dh > 0.0) {
      exact_ray_double(a, s_lane, h, 0.0, 1.0, g0, pth, opt, col, ne, em, rb);
      const double VX = col;
      const double pv = pth;
      // g at q = 0 is the limit, taken at q = 1e-4 q_max
      const double q = q_max * ((double)j / (double)(n_q - 1));
      const double qg = j == 0 ? 1e-4 * q_max : q;
      const double ce = 1.0 / sqrt(1.0 + qg * qg), se = qg * ce;
      exact_ray_double(a, s_lane, h, se, ce, g0, pth, opt, col, ne, em, rb);
      const double g = (ne * se * g0 - dh * qg) / qg;
      double dP, dX;
      if (j == 0) {
        dP = pv - dh;
        dX = 0.0;
      } else {
        const double sec = sqrt(1.0 + q * q);
        dP = pth - dh * sec;
        dX = col - sec * VX;
      }
      out = make_float4((float)g, (float)dP, (float)dX, 0.f);
    }
    corr[idx] = out;
  } else if (idx < n2 + n_v) {
    const int k = (int)(idx - n2);
    const double h = a.hobs + span * ((double)k / (double)(n_v - 1));
    exact_ray_double(a, s_lane, h, 0.0, 1.0, g0, pth, opt, col, ne, em, rb);
    vert[k] = make_float2((float)(rb * (1.0 + em)), (float)(h > a.hobs ? col : 0.0));
  }
}

// ------------------------------------------------------------ host helpers --
bool finite(double v) { return std::isfinite(v); }

// Fingerprint of what a correction table depends on (FNV-1a over the
// layers, scale heights, n0 - 1 and h_obs); never 0.
uint64_t atm_hash(const photon_atmosphere* a) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  mix(&a->n_layers, sizeof a->n_layers);
  mix(a->h_base, sizeof(double) * (size_t)a->n_layers);
  mix(a->scale_height, sizeof(double) * (size_t)a->n_layers);
  mix(&a->n0_minus_1, sizeof a->n0_minus_1);
  mix(&a->h_obs, sizeof a->h_obs);
  return h ? h : 1ull;
}

int check_table_shape(const photon_atmosphere* a, const photon_table* t) {
  if (t->n_h < 2 || t->n_h > 4096 || t->n_q < 2 || t->n_q > 4096 || t->n_v < 2 || t->n_v > 65536)
    return fail(PHOTON_EINVAL, "table nodes n_h = %d, n_q = %d, n_v = %d out of range", t->n_h, t->n_q, t->n_v);
  if (!std::isfinite(t->h_max) || !(t->h_max > a->h_obs)) return fail(PHOTON_EINVAL, "table h_max must exceed h_obs");
  if (!(t->q_max > 0.0) || !(t->q_max <= 1e3)) return fail(PHOTON_EINVAL, "table q_max must lie in (0, 1e3]");
  if (!t->corr || !t->vert) return fail(PHOTON_EINVAL, "table arrays are NULL");
  return PHOTON_OK;
}

int prep_atm(const photon_atmosphere* a, AtmDev* d) {
  if (!a) return fail(PHOTON_EINVAL, "atmosphere is NULL");
  if (a->n_layers < 1 || a->n_layers > PHOTON_MAX_LAYERS)
    return fail(PHOTON_EINVAL, "n_layers = %d outside 1..%d", a->n_layers, PHOTON_MAX_LAYERS);
  if (a->h_base[0] != 0.0) return fail(PHOTON_EINVAL, "h_base[0] must be 0");
  for (int i = 0; i < a->n_layers; ++i) {
    if (!finite(a->h_base[i])) return fail(PHOTON_EINVAL, "h_base[%d] not finite", i);
    if (i > 0 && !(a->h_base[i] > a->h_base[i - 1])) return fail(PHOTON_EINVAL, "h_base not strictly increasing at %d", i);
    if (!(a->scale_height[i] > 0.0)) return fail(PHOTON_EINVAL, "scale_height[%d] must be > 0", i);
  }
  if (!(a->n0_minus_1 >= 0.0) || !finite(a->n0_minus_1)) return fail(PHOTON_EINVAL, "n0_minus_1 must be finite and >= 0");
  if (!finite(a->h_obs)) return fail(PHOTON_EINVAL, "h_obs not finite");
  if (a->n_abs < 0 || a->n_abs > PHOTON_MAX_ABS) return fail(PHOTON_EINVAL, "n_abs = %d outside 0..%d", a->n_abs, PHOTON_MAX_ABS);
  for (int i = 0; i < a->n_abs; ++i) {
    if (!finite(a->abs_lambda_nm[i]) || !(a->abs_k_per_m[i] >= 0.0) || !finite(a->abs_k_per_m[i]))
      return fail(PHOTON_EINVAL, "absorption table entry %d invalid", i);
    if (i > 0 && !(a->abs_lambda_nm[i] > a->abs_lambda_nm[i - 1]))
      return fail(PHOTON_EINVAL, "abs_lambda_nm not strictly increasing at %d", i);
  }
  std::memset(d, 0, sizeof *d);
  d->nl = a->n_layers;
  d->n_abs = a->n_abs;
  d->hb[PHOTON_MAX_LAYERS] = HUGE_VAL;
  for (int i = 0; i < PHOTON_MAX_LAYERS; ++i) {
    const int k = i < a->n_layers ? i : a->n_layers - 1;
    // bases beyond the last layer are +inf: layer_of needs no layer count
    d->hb[i] = i < a->n_layers ? a->h_base[k] : HUGE_VAL;
    d->H[i] = a->scale_height[k];
    if (std::isinf(a->scale_height[k]) && i < a->n_layers) d->homog_mask |= 1 << i;
  }
  d->rb[0] = 1.0;
  for (int i = 0; i + 1 < a->n_layers; ++i)
    d->rb[i + 1] = d->rb[i] * exp_fixed(-(a->h_base[i + 1] - a->h_base[i]) / a->scale_height[i]);
  for (int i = a->n_layers; i < PHOTON_MAX_LAYERS; ++i) d->rb[i] = d->rb[a->n_layers - 1];
  d->eta0 = a->n0_minus_1;
  d->hobs = a->h_obs;
  int lo = 0;
  for (int k = 0; k < a->n_layers; ++k)
    if (a->h_base[k] <= a->h_obs) lo = k;
  d->l_obs = lo;
  d->rho_obs = d->rb[lo] * std::exp(-(a->h_obs - a->h_base[lo]) / a->scale_height[lo]);
  d->n_obs = 1.0 + a->n0_minus_1 * d->rho_obs;
  for (int i = 0; i < a->n_abs; ++i) {
    d->abs_l[i] = a->abs_lambda_nm[i];
    d->abs_k[i] = a->abs_k_per_m[i];
  }
  for (int i = 0; i < PHOTON_MAX_LAYERS; ++i) {
    d->invH[i] = 1.0 / d->H[i];
    d->em_full[i] = (i + 1 < a->n_layers) ? std::expm1(-(a->h_base[i + 1] - a->h_base[i]) / a->scale_height[i]) : 0.0;
  }
  d->em_obs = (lo + 1 < a->n_layers) ? std::expm1(-(a->h_base[lo + 1] - a->h_obs) / a->scale_height[lo]) : 0.0;
  d->abs_uniform = 0;
  if (a->n_abs >= 2) {
    const double step = (a->abs_lambda_nm[a->n_abs - 1] - a->abs_lambda_nm[0]) / (a->n_abs - 1);
    bool uni = step > 0.0;
    for (int i = 0; i + 1 < a->n_abs && uni; ++i)
      uni = std::fabs((a->abs_lambda_nm[i + 1] - a->abs_lambda_nm[i]) - step) <= 1e-9 * step;
    d->abs_uniform = uni ? 1 : 0;
    d->absf_l0 = (float)a->abs_lambda_nm[0];
    d->absf_inv_step = (float)(uni ? 1.0 / step : 0.0);
  }
  if (a->n_abs >= 1) {
    d->absf_l_lo = (float)d->abs_l[0];
    d->absf_k_lo = (float)d->abs_k[0];
    d->absf_l_hi = (float)d->abs_l[a->n_abs - 1];
    d->absf_k_hi = (float)d->abs_k[a->n_abs - 1];
  }
  if (a->table) {
    const photon_table* t = a->table;
    int rc = check_table_shape(a, t);
    if (rc) return rc;
    if (t->atm_hash != atm_hash(a)) return fail(PHOTON_EINVAL, "correction table not built for this atmosphere");
    d->tcorr = (const float4*)t->corr;
    d->tvert = (const float2*)t->vert;
    d->tn_h = t->n_h;
    d->tn_q = t->n_q;
    d->tn_v = t->n_v;
    d->t_hmax = t->h_max;
    d->t_qmax = t->q_max;
    d->t_fi = (double)(t->n_h - 1) / (t->h_max - a->h_obs);
    d->t_fj = (double)(t->n_q - 1) / t->q_max;
    d->t_fk = (double)(t->n_v - 1) / (t->h_max - a->h_obs);
  }
  return PHOTON_OK;
}

int prep_seg(const photon_segments* s, SegView* v, bool need_dedx) {
  if (!s) return fail(PHOTON_EINVAL, "segments is NULL");
  if (s->n < 0) return fail(PHOTON_EINVAL, "segment count n = %lld < 0", (long long)s->n);
  if (s->n > 0xffffffffll) return fail(PHOTON_EINVAL, "more than 2^32 - 1 segments");
  if (s->n > 0) {
    const void* req[] = {s->x0, s->y0, s->z0, s->dx, s->dy, s->dz, s->length, s->beta, s->t0};
    const char* nm[] = {"x0", "y0", "z0", "dx", "dy", "dz", "length", "beta", "t0"};
    for (int k = 0; k < 9; ++k)
      if (!req[k]) return fail(PHOTON_EINVAL, "segment field %s is NULL", nm[k]);
    if (need_dedx && !s->dedx) return fail(PHOTON_EINVAL, "segment field dedx is NULL (fluorescence)");
  }
  *v = SegView{s->x0, s->y0, s->z0, s->dx, s->dy, s->dz, s->length, s->beta, s->t0, s->dedx,
               s->charge, s->shower, s->index_in_shower};
  return PHOTON_OK;
}

int prep_cut(const photon_emission* em, CutDev* c) {
  std::memset(c, 0, sizeof *c);
  if (em->n_cut_points < 0 || em->n_cut_points > PHOTON_MAX_CUT_POINTS)
    return fail(PHOTON_EINVAL, "n_cut_points = %d outside 0..%d", em->n_cut_points, PHOTON_MAX_CUT_POINTS);
  if (em->n_cut_points == 0 || em->kind != PHOTON_CHERENKOV) return PHOTON_OK;
  if (!finite(em->cut_cos) || em->cut_cos < -1.0 || em->cut_cos > 1.0)
    return fail(PHOTON_EINVAL, "cut_cos must lie in [-1, 1]");
  c->n = em->n_cut_points;
  c->cos_cut = em->cut_cos;
  for (int k = 0; k < em->n_cut_points; ++k)
    for (int d = 0; d < 3; ++d) {
      if (!finite(em->cut_points[k][d])) return fail(PHOTON_EINVAL, "cut point %d not finite", k);
      c->pts[k][d] = em->cut_points[k][d];
    }
  return PHOTON_OK;
}

int prep_emission(const photon_emission* em, GenParams* g) {
  if (!em) return fail(PHOTON_EINVAL, "emission is NULL");
  std::memset(g, 0, sizeof *g);
  g->kind = em->kind;
  if (em->kind == PHOTON_CHERENKOV) {
    if (!(em->lambda_min_nm > 0.0) || !(em->lambda_max_nm > em->lambda_min_nm) || !finite(em->lambda_max_nm))
      return fail(PHOTON_EINVAL, "wavelength band must satisfy 0 < lambda_min < lambda_max");
    g->inv_l1 = 1.0 / em->lambda_min_nm;
    g->inv_dl = 1.0 / em->lambda_min_nm - 1.0 / em->lambda_max_nm;
    g->n_lines = 1;
    return PHOTON_OK;
  }
  if (em->kind != PHOTON_FLUORESCENCE) return fail(PHOTON_EINVAL, "unknown emission kind %d", em->kind);
  if (!(em->yield_per_MeV >= 0.0) || !finite(em->yield_per_MeV)) return fail(PHOTON_EINVAL, "yield_per_MeV must be >= 0");
  if (em->n_lines < 1 || em->n_lines > PHOTON_MAX_LINES)
    return fail(PHOTON_EINVAL, "n_lines = %d outside 1..%d", em->n_lines, PHOTON_MAX_LINES);
  double acc = 0.0, cdf[PHOTON_MAX_LINES];
  for (int k = 0; k < em->n_lines; ++k) {
    if (!(em->line_rel_yield[k] >= 0.0) || !finite(em->line_rel_yield[k]))
      return fail(PHOTON_EINVAL, "line_rel_yield[%d] must be >= 0", k);
    if (!(em->line_nm[k] > 0.0) || !finite(em->line_nm[k])) return fail(PHOTON_EINVAL, "line_nm[%d] must be > 0", k);
    acc = acc + em->line_rel_yield[k];
    cdf[k] = acc;
  }
  if (!(acc > 0.0)) return fail(PHOTON_EINVAL, "relative line yields are all zero");
  for (int k = 0; k < em->n_lines; ++k) cdf[k] = cdf[k] / acc;
  cdf[em->n_lines - 1] = 1.0;
  g->n_lines = em->n_lines;
  for (int k = 0; k < PHOTON_MAX_LINES; ++k) {
    const int kk = k < em->n_lines ? k : em->n_lines - 1;
    // u3 < cdf[k]  <=>  (w + 1/2) 2^-32 < cdf[k]  <=>  w < ceil(cdf[k] 2^32 - 1/2)
    g->thr[k] = (uint64_t)std::ceil(std::ldexp(cdf[kk], 32) - 0.5);
    g->line_nm[k] = em->line_nm[kk];
  }
  if (em->beam != 0) {
    if (em->beam != 1) return fail(PHOTON_EINVAL, "beam must be 0 or 1");
    for (int d = 0; d < 3; ++d)
      if (!finite(em->beam_center[d])) return fail(PHOTON_EINVAL, "beam_center not finite");
    if (!(em->beam_radius >= 0.0) || !finite(em->beam_radius))
      return fail(PHOTON_EINVAL, "beam_radius must be finite and >= 0");
    if (!(em->beam_margin_rad >= 0.0) || !(em->beam_margin_rad <= 0.5 * kPi))
      return fail(PHOTON_EINVAL, "beam_margin_rad must lie in [0, pi/2]");
    g->beam.on = 1;
    g->beam.cx = em->beam_center[0];
    g->beam.cy = em->beam_center[1];
    g->beam.cz = em->beam_center[2];
    g->beam.r = em->beam_radius;
    g->beam.cos_m = std::cos(em->beam_margin_rad);
    g->beam.sin_m = std::sin(em->beam_margin_rad);
  }
  return PHOTON_OK;
}

int prep_precision(int32_t p) {
  if (p != PHOTON_FP64 && p != PHOTON_FP32) return fail(PHOTON_EINVAL, "precision must be PHOTON_FP64 or PHOTON_FP32");
  return PHOTON_OK;
}

template <typename T>
int prep_block(const photon_block* b, BlockView<T>* v, bool need_cap) {
  if (!b) return fail(PHOTON_EINVAL, "photon block is NULL");
  if (b->n_photons < 0 || b->capacity < 0) return fail(PHOTON_EINVAL, "negative photon count or capacity");
  if (need_cap && b->n_photons > b->capacity)
    return fail(PHOTON_ECAPACITY, "n_photons = %lld exceeds capacity %lld", (long long)b->n_photons, (long long)b->capacity);
  if (b->n_photons > 0) {
    const void* req[] = {b->x, b->y, b->z, b->ux, b->uy, b->uz, b->wavelength_nm, b->weight, b->t_ns, b->path_m,
                         b->segment, b->j, b->status};
    for (int k = 0; k < 13; ++k)
      if (!req[k]) return fail(PHOTON_EINVAL, "photon block array %d is NULL", k);
  }
  *v = BlockView<T>{(T*)b->x,      (T*)b->y, (T*)b->ux, (T*)b->uy, (T*)b->wavelength_nm, (T*)b->weight,
                    b->uz,          b->z,     b->t_ns,   b->path_m, b->segment,           b->j,
                    b->status};
  return PHOTON_OK;
}

int check_block(const photon_block* b, int32_t precision) {
  if (precision == PHOTON_FP64) {
    BlockView<double> v;
    return prep_block<double>(b, &v, true);
  }
  BlockView<float> v;
  return prep_block<float>(b, &v, true);
}

void build_candidates(const photon_sink* s, double hobs, SinkDev* d) {
  const double tan_cap = std::sqrt(1.0 - kCapCos * kCapCos) / kCapCos;
  double reach[PHOTON_MAX_TELESCOPES];
  double x0 = 1e300, y0 = 1e300, x1 = -1e300, y1 = -1e300;
  for (int k = 0; k < s->n_tel; ++k) {
    reach[k] = s->tel[k][3] / kCapCos + std::fabs(s->tel[k][2] - hobs) * tan_cap;
    x0 = std::min(x0, s->tel[k][0] - reach[k]);
    x1 = std::max(x1, s->tel[k][0] + reach[k]);
    y0 = std::min(y0, s->tel[k][1] - reach[k]);
    y1 = std::max(y1, s->tel[k][1] + reach[k]);
  }
  const double cell = std::max(x1 - x0, y1 - y0) / kCandCells * (1.0 + 1e-9) + 1e-9;
  d->cand_x0 = (float)x0;
  d->cand_y0 = (float)y0;
  d->cand_inv_cell = (float)(1.0 / cell);
  d->tel_hobs = hobs;
  for (int iy = 0; iy < kCandCells; ++iy)
    for (int ix = 0; ix < kCandCells; ++ix) {
      uint32_t m = 0;
      const double cx0 = x0 + ix * cell, cy0 = y0 + iy * cell;
      for (int k = 0; k < s->n_tel; ++k) {
        // distance from the sphere centre to the cell square, with a margin
        const double dx = std::max(0.0, std::max(cx0 - s->tel[k][0], s->tel[k][0] - (cx0 + cell)));
        const double dy = std::max(0.0, std::max(cy0 - s->tel[k][1], s->tel[k][1] - (cy0 + cell)));
        // (1 mm more: the float form finds its cell to float rounding)
        const double rm = reach[k] * (1.0 + 1e-6) + 1e-3;
        if (dx * dx + dy * dy <= rm * rm) m |= 1u << k;
      }
      d->cand_mask[iy * kCandCells + ix] = m;
    }
}

// Radial profile geometry and accumulators of a sink.
int prep_radial(const photon_sink* s, SinkDev* d) {
  if (s->n_bins < 1 || s->n_bins > PHOTON_MAX_RADIAL_BINS)
    return fail(PHOTON_EINVAL, "n_bins = %d outside 1..%d", s->n_bins, PHOTON_MAX_RADIAL_BINS);
  if (s->log_bins != 0 && s->log_bins != 1) return fail(PHOTON_EINVAL, "log_bins must be 0 or 1");
  if (!finite(s->core_x) || !finite(s->core_y) || !finite(s->t_ref_ns))
    return fail(PHOTON_EINVAL, "radial core or t_ref not finite");
  if (!finite(s->r_min) || !finite(s->r_max) || !(s->r_min >= 0.0) || !(s->r_max > s->r_min))
    return fail(PHOTON_EINVAL, "radial range must satisfy 0 <= r_min < r_max");
  if (s->log_bins && !(s->r_min > 0.0)) return fail(PHOTON_EINVAL, "log bins need r_min > 0");
  if (!s->radial_count || !s->radial_weight || !s->radial_wt) return fail(PHOTON_EINVAL, "radial outputs are NULL");
  d->core_x = s->core_x;
  d->core_y = s->core_y;
  d->r_min = s->r_min;
  d->r_inv = s->log_bins ? (double)s->n_bins / std::log(s->r_max / s->r_min)
                         : (double)s->n_bins / (s->r_max - s->r_min);
  d->t_ref = s->t_ref_ns;
  d->n_bins = s->n_bins;
  d->log_bins = s->log_bins;
  d->rad_count = s->radial_count;
  d->rad_w = s->radial_weight;
  d->rad_wt = s->radial_wt;
  return PHOTON_OK;
}

int prep_sink(const photon_sink* s, SinkDev* d, double atm_hobs, int32_t precision) {
  if (!s) return fail(PHOTON_EINVAL, "sink is NULL");
  std::memset(d, 0, sizeof *d);
  d->kind = s->kind;
  d->totals = s->status_totals;
  if (s->kind == PHOTON_SINK_TELESCOPES) {
    if (s->n_tel < 1 || s->n_tel > PHOTON_MAX_TELESCOPES)
      return fail(PHOTON_EINVAL, "n_tel = %d outside 1..%d", s->n_tel, PHOTON_MAX_TELESCOPES);
    for (int k = 0; k < s->n_tel; ++k) {
      for (int c = 0; c < 4; ++c)
        if (!finite(s->tel[k][c])) return fail(PHOTON_EINVAL, "telescope %d not finite", k);
      if (!(s->tel[k][3] > 0.0)) return fail(PHOTON_EINVAL, "telescope %d radius must be > 0", k);
    }
    const photon_hits& h = s->hits;
    if (h.capacity < 0 || !h.count) return fail(PHOTON_EINVAL, "hits.count is NULL or capacity < 0");
    if (h.capacity > 0) {
      const void* req[] = {h.segment, h.j, h.telescope, h.x, h.y, h.z, h.t_ns, h.ux, h.uy, h.uz, h.wavelength_nm, h.weight};
      for (int k = 0; k < 12; ++k)
        if (!req[k]) return fail(PHOTON_EINVAL, "hit array %d is NULL", k);
    }
    d->n_tel = s->n_tel;
    std::memcpy(d->tel, s->tel, sizeof d->tel);
    d->hits = h;
    build_candidates(s, atm_hobs, d);
  } else if (s->kind == PHOTON_SINK_GRID) {
    if (s->nx < 1 || s->ny < 1 || (int64_t)s->nx * s->ny > (1 << 24))
      return fail(PHOTON_EINVAL, "grid shape %d x %d invalid", s->nx, s->ny);
    if (!(s->cell > 0.0) || !finite(s->x_min) || !finite(s->y_min) || !finite(s->cell))
      return fail(PHOTON_EINVAL, "grid origin/cell invalid");
    if (!s->grid_count || !s->grid_weight) return fail(PHOTON_EINVAL, "grid outputs are NULL");
    d->x_min = s->x_min;
    d->y_min = s->y_min;
    d->cell = s->cell;
    d->nx = s->nx;
    d->ny = s->ny;
    d->grid_count = s->grid_count;
    d->grid_weight = s->grid_weight;
  } else if (s->kind == PHOTON_SINK_PLANE) {
    const photon_block* b = s->plane;
    if (!b) return fail(PHOTON_EINVAL, "plane sink without a photon block");
    if (b->precision != precision) return fail(PHOTON_EINVAL, "plane block precision differs from the run's");
    if (b->capacity < 0) return fail(PHOTON_EINVAL, "plane capacity < 0");
    if (b->capacity > 0) {
      const void* req[] = {b->x, b->y, b->z, b->ux, b->uy, b->uz, b->wavelength_nm, b->weight, b->t_ns, b->path_m,
                           b->segment, b->j, b->status};
      for (int k = 0; k < 13; ++k)
        if (!req[k]) return fail(PHOTON_EINVAL, "plane array %d is NULL", k);
    }
    d->plane_capacity = b->capacity;
    d->px = b->x;
    d->py = b->y;
    d->pz = b->z;
    d->pux = b->ux;
    d->puy = b->uy;
    d->puz = b->uz;
    d->plam = b->wavelength_nm;
    d->pw = b->weight;
    d->pt = b->t_ns;
    d->ppath = b->path_m;
    d->pseg = b->segment;
    d->pj = b->j;
    d->pstatus = b->status;
  } else if (s->kind == PHOTON_SINK_RADIAL) {
    int rc = prep_radial(s, d);
    if (rc) return rc;
  } else if (s->kind != PHOTON_SINK_STATUS) {
    return fail(PHOTON_EINVAL, "unknown sink kind %d", s->kind);
  }
  return PHOTON_OK;
}

// ---------------------------------------------------------------- devices --
constexpr int64_t kDeferCap = 1 << 24;  // near-horizon rays queued per fused FP32 call
constexpr int kWorkWords = 8192;         // u64 words of the per-device work area
constexpr int kDeferCounts = 64;         // offset of the per-block deferred counts
constexpr int kMaxFusedGrid = kWorkWords - kDeferCounts;
static_assert(kScratchAreaWords == (size_t)kWorkWords, "the static scratch holds one work area");

// Device memory a fused run works in besides its inputs and outputs.
struct FusedScratch {
  unsigned long long* cursor = nullptr;        // work-queue position (one word)
  unsigned long long* defer_counts = nullptr;  // per block: queued near-horizon rays (kMaxFusedGrid words)
  unsigned long long* defer_pref = nullptr;    // their exclusive prefix sums (kMaxFusedGrid + 1 words)
  uint2* defer_q = nullptr;                    // the queue (float form only)
  int64_t defer_rays = 0;                      // its length
};

struct DeviceState {
  bool checked = false;
  bool ok = false;
  int cu = 0;
  size_t lds_per_block = 0;             // largest LDS allocation of one workgroup
  unsigned long long* work = nullptr;  // [0] = fused work cursor, [kDeferCounts..] per-block deferred counts
  uint2* defer_q = nullptr;            // deferred (segment row, j), defer_rays entries
  int64_t defer_rays = kDeferCap;      // length of the deferral queue (photon_set_defer_capacity)
  // calls working in this device's own scratch are ordered across streams:
  // the event recorded after the last one, and its stream
  hipEvent_t last_ev = nullptr;
  hipStream_t last_st = nullptr;
  bool last_valid = false;
  unsigned long long* defer_pref = nullptr;  // prefix sums of the per-block deferred counts
  struct OccEntry {
    const void* fn;
    size_t dyn;
    int occ;
  } occ_cache[96] = {};                     // fused blocks per CU by kernel instance and dynamic LDS
  int n_occ = 0;
  int occ_adj[2] = {0, 0};                  // adjoint blocks per CU by precision
  double* adj_part = nullptr;               // per-block partial sums of the adjoint
  unsigned long long* splat_acc = nullptr;  // fixed-point grid of the splat
  int64_t splat_cells = 0;
  // kernel timing (photon_kernel_timing): events around the last fused
  // kernel launched outside a stream capture
  bool timing = false, timed = false, timed_defer = false;
  hipEvent_t t_ev[3] = {nullptr, nullptr, nullptr};  // before and after the kernel, after the double pass
  unsigned long long* scratch_ptr = nullptr;  // this device's address of the static scratch
};
std::mutex g_mu;
DeviceState g_dev[64];

int current_device(DeviceState** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(PHOTON_ENODEV, "no HIP device");
  if (dev < 0 || dev >= 64) return fail(PHOTON_ENODEV, "device index %d unsupported", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceState& d = g_dev[dev];
  if (!d.checked) {
    d.checked = true;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(PHOTON_ENODEV, "hipGetDeviceProperties failed");
    d.ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    d.cu = prop.multiProcessorCount;
    d.lds_per_block = prop.sharedMemPerBlock;
  }
  if (!d.ok) return fail(PHOTON_ENODEV, "current device is not gfx950");
  *out = &d;
  return PHOTON_OK;
}

// The device's work area (work cursor, per-block deferral counts), allocated
// on first use (not inside a stream capture: photon_init and plan creation
// allocate it before capturing).
int ensure_work(DeviceState* dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev->work) return PHOTON_OK;
  if (hipMalloc(&dev->work, sizeof(unsigned long long) * kWorkWords) != hipSuccess) {
    dev->work = nullptr;
    return fail(PHOTON_EHIP, "work area allocation failed");
  }
  if (hipMemset(dev->work, 0, sizeof(unsigned long long) * kWorkWords) != hipSuccess) {
    (void)hipFree(dev->work);
    dev->work = nullptr;
    return fail(PHOTON_EHIP, "work area clear failed");
  }
  return PHOTON_OK;
}

// This device's address of the static scratch (looked up once per device,
// with the device current). Allocates nothing.
int static_scratch(DeviceState* dev, FusedScratch* ws) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!dev->scratch_ptr) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(PHOTON_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      dev->scratch_ptr = (unsigned long long*)p;
    }
  }
  unsigned long long* base = dev->scratch_ptr;
  ws->cursor = base;
  ws->defer_counts = base + kDeferCounts;
  ws->defer_pref = base + kScratchAreaWords;
  ws->defer_q = (uint2*)(base + 2 * kScratchAreaWords);
  ws->defer_rays = kScratchDeferRays;
  return PHOTON_OK;
}

int check_launch() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PHOTON_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
  return PHOTON_OK;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int count_and_scan(const SegView& sv, int64_t n, const AtmDev& atm, int kind, double K, const CutDev& cut,
                   const BeamDev& beam, uint64_t seed, uint32_t* counts, uint64_t* offsets, hipStream_t st) {
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  if (n == 0) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, (unsigned long long*)offsets, 1);
    return check_launch();
  }
  const int64_t nb = ceil_div(n, kScanBlock);
  if (nb <= kCountWideMaxBlocks) {
    if (kind == PHOTON_CHERENKOV)
      hipLaunchKernelGGL(k_count_wide<PHOTON_CHERENKOV>, dim3((unsigned)nb), dim3(kCountWide), 0, st, sv, n, atm, K,
                         k0, k1, cut, beam, counts, offsets);
    else
      hipLaunchKernelGGL(k_count_wide<PHOTON_FLUORESCENCE>, dim3((unsigned)nb), dim3(kCountWide), 0, st, sv, n, atm,
                         K, k0, k1, cut, beam, counts, offsets);
  } else if (kind == PHOTON_CHERENKOV) {
    hipLaunchKernelGGL(k_count<PHOTON_CHERENKOV>, dim3((unsigned)nb), dim3(kScanBlock), 0, st, sv, n, atm, K, k0, k1,
                       cut, beam, counts, offsets);
  } else {
    hipLaunchKernelGGL(k_count<PHOTON_FLUORESCENCE>, dim3((unsigned)nb), dim3(kScanBlock), 0, st, sv, n, atm, K, k0,
                       k1, cut, beam, counts, offsets);
  }
  hipLaunchKernelGGL(k_scan_tops, dim3(1), dim3(1024), 0, st, offsets, n, nb);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kScanBlock), 0, st, (const uint32_t*)counts, offsets, n);
  return check_launch();
}

template <typename T>
int launch_gen(const SegView& sv, int64_t n, const AtmDev& atm, const GenParams& g, uint64_t seed,
               const uint64_t* offsets, const photon_block* out, hipStream_t st) {
  BlockView<T> bv;
  int rc = prep_block<T>(out, &bv, true);
  if (rc) return rc;
  if (out->n_photons == 0) return PHOTON_OK;
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  hipLaunchKernelGGL(k_gen<T>, dim3((unsigned)ceil_div(out->n_photons, 256)), dim3(256), 0, st, sv, n, atm, g, k0, k1,
                     offsets, out->n_photons, bv);
  return check_launch();
}

int generate_common(const photon_segments* seg, const photon_atmosphere* atm, const photon_emission* em,
                    uint64_t seed, int32_t precision, uint32_t* counts, uint64_t* offsets, photon_block* out,
                    void* stream) {
  SegView sv;
  AtmDev ad;
  GenParams g;
  int rc;
  if ((rc = prep_seg(seg, &sv, em->kind == PHOTON_FLUORESCENCE))) return rc;
  if ((rc = prep_atm(atm, &ad))) return rc;
  if ((rc = prep_emission(em, &g))) return rc;
  CutDev cut;
  if ((rc = prep_cut(em, &cut))) return rc;
  if ((rc = prep_precision(precision))) return rc;
  if (!offsets) return fail(PHOTON_EINVAL, "offsets is NULL");
  if (!out && !counts) return fail(PHOTON_EINVAL, "counts is NULL");
  if (out && out->precision != precision) return fail(PHOTON_EINVAL, "photon block precision differs from the call's");
  if (out && (rc = check_block(out, precision))) return rc;
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (!out) {
    const double K = (em->kind == PHOTON_CHERENKOV)
                         ? (2.0 * kPi * kAlpha) * ((1e9 / em->lambda_min_nm) - (1e9 / em->lambda_max_nm))
                         : em->yield_per_MeV;
    return count_and_scan(sv, seg->n, ad, em->kind, K, cut, g.beam, seed, counts, offsets, st);
  }
  return precision == PHOTON_FP64 ? launch_gen<double>(sv, seg->n, ad, g, seed, offsets, out, st)
                                  : launch_gen<float>(sv, seg->n, ad, g, seed, offsets, out, st);
}

template <typename T>
int launch_propagate(photon_block* b, const AtmDev& atm, hipStream_t st) {
  BlockView<T> bv;
  int rc = prep_block<T>(b, &bv, true);
  if (rc) return rc;
  if (b->n_photons == 0) return PHOTON_OK;
  if (atm.tcorr)
    hipLaunchKernelGGL((k_propagate<T, true>), dim3((unsigned)ceil_div(b->n_photons, 256)), dim3(256), 0, st, atm,
                       bv, b->n_photons);
  else
    hipLaunchKernelGGL((k_propagate<T, false>), dim3((unsigned)ceil_div(b->n_photons, 256)), dim3(256), 0, st, atm,
                       bv, b->n_photons);
  return check_launch();
}

template <typename T>
int launch_collect(const photon_block* b, const AtmDev& atm, const SinkDev& sk, hipStream_t st) {
  BlockView<T> bv;
  int rc = prep_block<T>(b, &bv, true);
  if (rc) return rc;
  if (b->n_photons == 0) return PHOTON_OK;
  hipLaunchKernelGGL(k_collect<T>, dim3((unsigned)ceil_div(b->n_photons, 256)), dim3(256), 0, st, bv, b->n_photons,
                     sk, atm.n_obs);
  return check_launch();
}

// Blocks per CU of a kernel instance with a given dynamic LDS (cached).
int occupancy_of(DeviceState* dev, const void* fn, int bs, size_t dyn) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (int i = 0; i < dev->n_occ; ++i)
    if (dev->occ_cache[i].fn == fn && dev->occ_cache[i].dyn == dyn) return dev->occ_cache[i].occ;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, bs, dyn) != hipSuccess || occ < 1) occ = 1;
  if (dev->n_occ < 96) dev->occ_cache[dev->n_occ++] = {fn, dyn, occ};
  return occ;
}

// The fused kernel instance of a mode.
template <typename T, int BS>
const void* fused_instance(int mode) {
  // the float splat's own block size carries the splat instance only
  if constexpr (BS != 128 && BS != 256 && BS != 512) {
    return (const void*)k_fused<T, BS, kMSplat>;
  } else {
    switch (mode) {
      case kMSplat: return (const void*)k_fused<T, BS, kMSplat>;
      case kMRadial: return (const void*)k_fused<T, BS, kMRadial>;
      case kMTable: return (const void*)k_fused<T, BS, kMTable>;
      case kMRadial | kMTable: return (const void*)k_fused<T, BS, kMRadial | kMTable>;
      case kMFluo: return (const void*)k_fused<T, BS, kMFluo>;
      case kMFluo | kMRadial: return (const void*)k_fused<T, BS, kMFluo | kMRadial>;
      case kMFluo | kMTable: return (const void*)k_fused<T, BS, kMFluo | kMTable>;
      case kMFluo | kMRadial | kMTable: return (const void*)k_fused<T, BS, kMFluo | kMRadial | kMTable>;
      case kMTel: return (const void*)k_fused<T, BS, kMTel>;
      case kMTel | kMTable: return (const void*)k_fused<T, BS, kMTel | kMTable>;
      case kMTel | kMFluo: return (const void*)k_fused<T, BS, kMTel | kMFluo>;
      case kMTel | kMFluo | kMTable: return (const void*)k_fused<T, BS, kMTel | kMFluo | kMTable>;
      case kMGrid: return (const void*)k_fused<T, BS, kMGrid>;
      case kMGrid | kMTable: return (const void*)k_fused<T, BS, kMGrid | kMTable>;
      case kMGrid | kMFluo: return (const void*)k_fused<T, BS, kMGrid | kMFluo>;
      case kMGrid | kMFluo | kMTable: return (const void*)k_fused<T, BS, kMGrid | kMFluo | kMTable>;
      default: return (const void*)k_fused<T, BS, 0>;
    }
  }
}

void warm_occupancy(DeviceState* dev) {
  occupancy_of(dev, fused_instance<float, 256>(0), 256, 0);
  occupancy_of(dev, fused_instance<float, 512>(0), 512, 0);
  occupancy_of(dev, fused_instance<double, 256>(0), 256, 0);
  occupancy_of(dev, fused_instance<double, 512>(0), 512, 0);
  occupancy_of(dev, fused_instance<float, 256>(kMTel), 256, 0);
  occupancy_of(dev, fused_instance<float, 512>(kMTel), 512, 0);
  occupancy_of(dev, fused_instance<double, 256>(kMTel), 256, 0);
  occupancy_of(dev, fused_instance<double, 512>(kMTel), 512, 0);
}

// The deferral queue of the float form, allocated on first use (not inside
// a stream capture: plan creation allocates it before capturing).
int ensure_defer_queue(DeviceState* dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev->defer_q) return PHOTON_OK;
  if (hipMalloc(&dev->defer_q, sizeof(uint2) * dev->defer_rays) != hipSuccess) {
    dev->defer_q = nullptr;
    return fail(PHOTON_EHIP, "deferral queue allocation failed");
  }
  if (hipMalloc(&dev->defer_pref, sizeof(unsigned long long) * (kMaxFusedGrid + 1)) != hipSuccess) {
    (void)hipFree(dev->defer_q);
    dev->defer_q = nullptr;
    dev->defer_pref = nullptr;
    return fail(PHOTON_EHIP, "deferral queue allocation failed");
  }
  return PHOTON_OK;
}

// The device's own fused scratch: the work area and, for the float form, the
// deferral queue (2^24 rays unless resized), both allocated on first use.
int device_scratch(DeviceState* dev, bool defer, FusedScratch* ws) {
  int rc;
  if ((rc = ensure_work(dev))) return rc;
  if (defer && (rc = ensure_defer_queue(dev))) return rc;
  ws->cursor = dev->work;
  ws->defer_counts = dev->work + kDeferCounts;
  ws->defer_pref = dev->defer_pref;
  ws->defer_q = dev->defer_q;
  ws->defer_rays = defer ? dev->defer_rays : 0;
  return PHOTON_OK;
}

// Calls that work in the device's own scratch (work cursor, deferral queue,
// adjoint partial sums, splat accumulator) run one after another on the
// device whatever their streams: a call on another stream than the previous
// one first makes its stream wait for an event recorded after that call.
// Inside a stream capture neither the wait nor the record is made (a
// captured graph that uses the device's scratch must not be replayed beside
// other such calls).
int begin_device_scratch(DeviceState* dev, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return fail(PHOTON_EHIP, "stream capture query failed");
  if (cs != hipStreamCaptureStatusNone) return PHOTON_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev->last_valid && dev->last_st != st && hipStreamWaitEvent(st, dev->last_ev, 0) != hipSuccess)
    return fail(PHOTON_EHIP, "hipStreamWaitEvent failed");
  return PHOTON_OK;
}

int end_device_scratch(DeviceState* dev, hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess) return fail(PHOTON_EHIP, "stream capture query failed");
  if (cs != hipStreamCaptureStatusNone) return PHOTON_OK;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!dev->last_ev && hipEventCreateWithFlags(&dev->last_ev, hipEventDisableTiming) != hipSuccess) {
    dev->last_ev = nullptr;
    return fail(PHOTON_EHIP, "event creation failed");
  }
  if (hipEventRecord(dev->last_ev, st) != hipSuccess) return fail(PHOTON_EHIP, "event record failed");
  dev->last_st = st;
  dev->last_valid = true;
  return PHOTON_OK;
}

// Scratch owned by one captured plan: allocated before its capture, freed
// with it, so that plans replayed on different streams do not share a work
// cursor or a deferral queue.
struct OwnedScratch {
  unsigned long long* area = nullptr;  // cursor + per-block counts (kWorkWords), prefix sums (kWorkWords)
  uint2* queue = nullptr;
  int64_t rays = 0;
  FusedScratch view() const {
    FusedScratch w;
    w.cursor = area;
    w.defer_counts = area + kDeferCounts;
    w.defer_pref = area + kWorkWords;
    w.defer_q = queue;
    w.defer_rays = rays;
    return w;
  }
};

void free_scratch(OwnedScratch* o) {
  if (o->area) (void)hipFree(o->area);
  if (o->queue) (void)hipFree(o->queue);
  *o = OwnedScratch{};
}

int alloc_scratch(int64_t defer_rays, OwnedScratch* o) {
  if (hipMalloc(&o->area, sizeof(unsigned long long) * 2 * kWorkWords) != hipSuccess) {
    o->area = nullptr;
    return fail(PHOTON_EHIP, "plan scratch allocation failed");
  }
  if (hipMemset(o->area, 0, sizeof(unsigned long long) * 2 * kWorkWords) != hipSuccess) {
    free_scratch(o);
    return fail(PHOTON_EHIP, "plan scratch clear failed");
  }
  if (defer_rays > 0) {
    if (hipMalloc(&o->queue, sizeof(uint2) * defer_rays) != hipSuccess) {
      o->queue = nullptr;
      free_scratch(o);
      return fail(PHOTON_EHIP, "plan deferral queue allocation failed");
    }
    o->rays = defer_rays;
  }
  return PHOTON_OK;
}

// Launches the fused kernel (and, in the float form, the near-horizon double
// pass) working in `scratch`, or in the device's own scratch when it is NULL.
template <typename T, int BS, bool SPLAT = false>
int launch_fused_bs(const SegView& sv, int64_t n, const AtmDev& atm, const GenParams& g, uint64_t seed,
                    const uint64_t* offsets, int64_t n_ph, int64_t chunk, int bpc, const SinkDev& sk,
                    DeviceState* dev, hipStream_t st, size_t dyn_lds = 0, const ZeroList* pre = nullptr,
                    const FusedScratch* scratch_in = nullptr) {
  const bool radial = !SPLAT && sk.kind == PHOTON_SINK_RADIAL;
  const bool table = !SPLAT && atm.tcorr != nullptr;
  const bool tel = !SPLAT && sk.kind == PHOTON_SINK_TELESCOPES;
  const bool grid_only = !SPLAT && sk.kind == PHOTON_SINK_GRID;
  const int mode = SPLAT ? kMSplat
                         : ((radial ? kMRadial : 0) | (table ? kMTable : 0) |
                            (g.kind == PHOTON_FLUORESCENCE ? kMFluo : 0) | (tel ? kMTel : 0) |
                            (grid_only ? kMGrid : 0));
  // the slot map of a chunk's piece holds kMaxChunk (splat: kMaxChunkSplat) photons
  if (chunk < 1 || chunk > (SPLAT ? kMaxChunkSplat : kMaxChunk))
    return fail(PHOTON_EINVAL, "fused chunk %lld outside 1..%d", (long long)chunk, SPLAT ? kMaxChunkSplat : kMaxChunk);
  const void* kfn = fused_instance<T, BS>(mode);
  // the radial bins live in dynamic LDS: count, weight and w t per bin
  if (radial) dyn_lds = (size_t)3 * sizeof(unsigned long long) * (size_t)sk.n_bins;
  int occ = occupancy_of(dev, kfn, BS, dyn_lds);
  if (bpc > 0 && bpc < occ) occ = bpc;
  int64_t grid = (int64_t)dev->cu * occ;
  if (n_ph >= 0) {
    const int64_t chunks = ceil_div(n_ph, chunk);
    if (grid > chunks) grid = chunks;
  }
  if (grid > kMaxFusedGrid) grid = kMaxFusedGrid;
  const bool defer = sizeof(T) == 4;
  FusedScratch ws;
  if (scratch_in) {
    ws = *scratch_in;
  } else {
    int rc = device_scratch(dev, defer, &ws);
    if (rc) return rc;
    if ((rc = begin_device_scratch(dev, st))) return rc;
  }
  FusedArgs A;
  A.seg = sv;
  A.n_seg = n;
  A.atm = atm;
  A.g = g;
  A.k0 = (uint32_t)(seed & 0xffffffffu);
  A.k1 = (uint32_t)(seed >> 32);
  A.offsets = offsets;
  A.n_ph = n_ph;
  A.chunk = chunk;
  A.sk = sk;
  A.cursor = ws.cursor;
  A.defer_counts = ws.defer_counts;
  A.defer_q = ws.defer_q;
  A.defer_cap = defer ? ws.defer_rays / grid : 0;
  A.defer_pref = ws.defer_pref;
  A.n_defer_blocks = (int32_t)grid;
  // the work cursor, with whatever the caller asked to clear before the kernel
  ZeroList z = pre ? *pre : ZeroList{};
  z.add(ws.cursor, 1);
  launch_zero_list(z, st);
  void* kargs[] = {&A};
  bool timed = false;
  if (dev->timing) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return fail(PHOTON_EHIP, "stream capture query failed");
    timed = cs == hipStreamCaptureStatusNone;
    if (timed && hipEventRecord(dev->t_ev[0], st) != hipSuccess) return fail(PHOTON_EHIP, "event record failed");
  }
  if (hipLaunchKernel(kfn, dim3((unsigned)grid), dim3(BS), kargs, dyn_lds, st) != hipSuccess)
    return fail(PHOTON_EHIP, "fused kernel launch failed");
  if (timed) {
    if (hipEventRecord(dev->t_ev[1], st) != hipSuccess) return fail(PHOTON_EHIP, "event record failed");
    dev->timed = true;
    dev->timed_defer = false;
  }
  if (defer) {
    hipLaunchKernelGGL(k_defer_scan, dim3(1), dim3(1024), 0, st, (const unsigned long long*)A.defer_counts,
                       (int)grid, A.defer_cap, A.defer_pref);
    if (A.sk.kind == kSinkSplat)
      hipLaunchKernelGGL((k_fused_deferred<256, kDeferSplat>), dim3((unsigned)grid), dim3(256), 0, st, A);
    else if (A.sk.kind == PHOTON_SINK_RADIAL)
      hipLaunchKernelGGL((k_fused_deferred<256, kDeferRadial>), dim3((unsigned)grid), dim3(256), 0, st, A);
    else
      hipLaunchKernelGGL((k_fused_deferred<256, kDeferOther>), dim3((unsigned)grid), dim3(256), 0, st, A);
    if (timed) {
      if (hipEventRecord(dev->t_ev[2], st) != hipSuccess) return fail(PHOTON_EHIP, "event record failed");
      dev->timed_defer = true;
    }
  }
  const int rc = check_launch();
  if (rc) return rc;
  return scratch_in ? PHOTON_OK : end_device_scratch(dev, st);
}

template <typename T>
int launch_fused(const SegView& sv, int64_t n, const AtmDev& atm, const GenParams& g, uint64_t seed,
                 const uint64_t* offsets, int64_t n_ph, const photon_tuning* tun, const SinkDev& sk,
                 DeviceState* dev, hipStream_t st, const ZeroList* pre = nullptr,
                 const FusedScratch* ws = nullptr) {
  int bs = tun ? tun->block : 256;
  int64_t chunk = tun ? tun->chunk : 4096;
  int bpc = tun ? tun->blocks_per_cu : 0;
  if (bs != 128 && bs != 256 && bs != 512) return fail(PHOTON_EINVAL, "tuning.block must be 128, 256 or 512");
  if (chunk < bs || chunk % bs || chunk > kMaxChunk)
    return fail(PHOTON_EINVAL, "tuning.chunk must be a multiple of block, at most %d", kMaxChunk);
  if (bpc < 0) return fail(PHOTON_EINVAL, "tuning.blocks_per_cu must be >= 0");
  switch (bs) {
    case 128: return launch_fused_bs<T, 128>(sv, n, atm, g, seed, offsets, n_ph, chunk, bpc, sk, dev, st, 0, pre, ws);
    case 512: return launch_fused_bs<T, 512>(sv, n, atm, g, seed, offsets, n_ph, chunk, bpc, sk, dev, st, 0, pre, ws);
    default: return launch_fused_bs<T, 256>(sv, n, atm, g, seed, offsets, n_ph, chunk, bpc, sk, dev, st, 0, pre, ws);
  }
}

int validate_tuning(const photon_tuning* t) {
  if (!t) return PHOTON_OK;
  if (t->block != 128 && t->block != 256 && t->block != 512) return fail(PHOTON_EINVAL, "tuning.block must be 128, 256 or 512");
  if (t->chunk < t->block || t->chunk % t->block || t->chunk > kMaxChunk)
    return fail(PHOTON_EINVAL, "tuning.chunk must be a multiple of block, at most %d", kMaxChunk);
  if (t->blocks_per_cu < 0) return fail(PHOTON_EINVAL, "tuning.blocks_per_cu must be >= 0");
  return PHOTON_OK;
}

// Everything a fused step needs, validated.
struct StepArgs {
  SegView sv;
  int64_t n = 0;
  AtmDev ad;
  GenParams g;
  SinkDev sk;
  int kind = 0;
  double K = 0.0;
  CutDev cut;
  uint64_t seed = 0;
  int32_t precision = 0;
};

int prep_step(const photon_segments* seg, const photon_atmosphere* atm, const photon_emission* em, uint64_t seed,
              int32_t precision, const photon_sink* sink, const photon_tuning* tuning, StepArgs* a) {
  int rc;
  if (!em) return fail(PHOTON_EINVAL, "emission is NULL");
  if ((rc = prep_seg(seg, &a->sv, em->kind == PHOTON_FLUORESCENCE))) return rc;
  if ((rc = prep_atm(atm, &a->ad))) return rc;
  if ((rc = prep_emission(em, &a->g))) return rc;
  if ((rc = prep_cut(em, &a->cut))) return rc;
  if ((rc = prep_precision(precision))) return rc;
  if ((rc = prep_sink(sink, &a->sk, a->ad.hobs, precision))) return rc;
  if ((rc = validate_tuning(tuning))) return rc;
  a->n = seg->n;
  a->kind = em->kind;
  a->K = (em->kind == PHOTON_CHERENKOV) ? (2.0 * kPi * kAlpha) * ((1e9 / em->lambda_min_nm) - (1e9 / em->lambda_max_nm))
                                         : em->yield_per_MeV;
  a->seed = seed;
  a->precision = precision;
  return PHOTON_OK;
}

// The sink outputs a step clears before its fused kernel.
ZeroList sink_zero_list(const SinkDev& sk) {
  ZeroList z;
  if (sk.totals) z.add(sk.totals, PHOTON_N_STATUS);
  if (sk.kind == PHOTON_SINK_TELESCOPES) z.add(sk.hits.count, 1);
  if (sk.kind == PHOTON_SINK_GRID) {
    z.p32 = sk.grid_count;
    z.n32 = sk.nx * sk.ny;
    z.add(sk.grid_weight, sk.nx * sk.ny);
  }
  if (sk.kind == PHOTON_SINK_RADIAL) {
    z.add(sk.rad_count, sk.n_bins);
    z.add(sk.rad_w, sk.n_bins);
    z.add(sk.rad_wt, sk.n_bins);
  }
  return z;
}

int enqueue_fused(const StepArgs& a, const uint64_t* offsets, int64_t n_ph, const photon_tuning* tun,
                  DeviceState* dev, hipStream_t st, const ZeroList* pre = nullptr, const FusedScratch* ws = nullptr) {
  if (a.n == 0 || n_ph == 0) {
    if (pre) {
      launch_zero_list(*pre, st);
      return check_launch();
    }
    return PHOTON_OK;
  }
  return a.precision == PHOTON_FP64
             ? launch_fused<double>(a.sv, a.n, a.ad, a.g, a.seed, offsets, n_ph, tun, a.sk, dev, st, pre, ws)
             : launch_fused<float>(a.sv, a.n, a.ad, a.g, a.seed, offsets, n_ph, tun, a.sk, dev, st, pre, ws);
}

// One whole step: counts + offsets, cleared outputs, fused kernel.
int enqueue_step(const StepArgs& a, uint32_t* counts, uint64_t* offsets, const photon_tuning* tun,
                 DeviceState* dev, hipStream_t st, const FusedScratch* ws = nullptr) {
  int rc;
  if ((rc = count_and_scan(a.sv, a.n, a.ad, a.kind, a.K, a.cut, a.g.beam, a.seed, counts, offsets, st))) return rc;
  // the sink outputs are cleared by the launch that clears the work cursor
  const ZeroList z = sink_zero_list(a.sk);
  return enqueue_fused(a, offsets, -1, tun, dev, st, &z, ws);
}

// ------------------------------------------------------ differentiable form --
constexpr int64_t kAdjChunk = 4096;

int prep_splat_grid(const photon_splat_grid* gr, SplatGeom* g) {
  if (!gr) return fail(PHOTON_EINVAL, "splat grid is NULL");
  if (gr->nx < 1 || gr->ny < 1 || (int64_t)gr->nx * gr->ny > (1 << 22))
    return fail(PHOTON_EINVAL, "splat grid shape %d x %d invalid", gr->nx, gr->ny);
  if (!(gr->cell > 0.0) || !finite(gr->cell) || !finite(gr->x_min) || !finite(gr->y_min))
    return fail(PHOTON_EINVAL, "splat grid origin/cell invalid");
  if (!(gr->sigma > 0.0) || !finite(gr->sigma)) return fail(PHOTON_EINVAL, "splat sigma must be > 0");
  if (!(gr->trunc > 0.0) || !finite(gr->trunc) || gr->trunc * gr->sigma > 64.0 * gr->cell)
    return fail(PHOTON_EINVAL, "splat truncation must be > 0 and reach at most 64 cells");
  g->x_min = gr->x_min;
  g->y_min = gr->y_min;
  g->cell = gr->cell;
  g->inv_cell = 1.0 / gr->cell;
  g->nx = gr->nx;
  g->ny = gr->ny;
  g->reach = gr->trunc * gr->sigma;
  g->norm = 1.0 / (2.0 * kPi * gr->sigma * gr->sigma);
  g->inv_2s2 = 1.0 / (2.0 * gr->sigma * gr->sigma);
  g->q = std::exp(-(gr->cell * gr->cell) / (gr->sigma * gr->sigma));
  return PHOTON_OK;
}

struct SplatCall {
  SegView sv;
  int64_t n = 0;
  AtmDev ad;
  GenParams g;
  SplatGeom sg;
  uint64_t seed = 0;
  int32_t precision = 0;
};

int prep_splat_call(const photon_segments* seg, const photon_atmosphere* atm, double lambda_min_nm,
                    double lambda_max_nm, uint64_t seed, int32_t precision, const uint64_t* offsets,
                    const double* mean0, const photon_splat_grid* grid, SplatCall* c) {
  int rc;
  photon_emission em;
  std::memset(&em, 0, sizeof em);
  em.kind = PHOTON_CHERENKOV;
  em.lambda_min_nm = lambda_min_nm;
  em.lambda_max_nm = lambda_max_nm;
  if ((rc = prep_seg(seg, &c->sv, false))) return rc;
  if ((rc = prep_atm(atm, &c->ad))) return rc;
  if (c->ad.tcorr) return fail(PHOTON_EINVAL, "the differentiable form takes the exact propagation: atmosphere.table must be NULL");
  if ((rc = prep_emission(&em, &c->g))) return rc;
  if ((rc = prep_precision(precision))) return rc;
  if ((rc = prep_splat_grid(grid, &c->sg))) return rc;
  if (!offsets) return fail(PHOTON_EINVAL, "offsets is NULL");
  if (!mean0 && seg->n > 0) return fail(PHOTON_EINVAL, "mean0 is NULL");
  c->g.K = (2.0 * kPi * kAlpha) * ((1e9 / lambda_min_nm) - (1e9 / lambda_max_nm));
  c->n = seg->n;
  c->seed = seed;
  c->precision = precision;
  return PHOTON_OK;
}

int ensure_adj_partials(DeviceState* dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev->adj_part) return PHOTON_OK;
  if (hipMalloc(&dev->adj_part, sizeof(double) * kAdjWords * 2 * kMaxFusedGrid) != hipSuccess) {
    dev->adj_part = nullptr;
    return fail(PHOTON_EHIP, "adjoint partial-sum allocation failed");
  }
  return PHOTON_OK;
}

// The splat's global fixed-point grid, grown on demand (not inside a capture).
int ensure_splat_acc(DeviceState* dev, int64_t cells) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev->splat_cells >= cells) return PHOTON_OK;
  if (dev->splat_acc) (void)hipFree(dev->splat_acc);
  dev->splat_acc = nullptr;
  dev->splat_cells = 0;
  if (hipMalloc(&dev->splat_acc, sizeof(unsigned long long) * cells) != hipSuccess) {
    dev->splat_acc = nullptr;
    return fail(PHOTON_EHIP, "splat accumulator allocation failed");
  }
  dev->splat_cells = cells;
  return PHOTON_OK;
}

template <typename T>
int launch_adjoint(const SplatCall& c, const uint64_t* offsets, const double* mean0, const void* grad,
                   double* gH, double* geta, double* gdx, double* gdy, double* gdz, DeviceState* dev,
                   hipStream_t st) {
  constexpr int BS = 256;
  int& occ = dev->occ_adj[sizeof(T) == 8 ? 0 : 1];
  if (occ == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_splat_adjoint<T, BS>, BS, 0) != hipSuccess || occ < 1)
      occ = 1;
  }
  int64_t grid = (int64_t)dev->cu * occ;
  if (grid > kMaxFusedGrid) grid = kMaxFusedGrid;
  int rc;
  if ((rc = ensure_adj_partials(dev))) return rc;
  constexpr bool defer = sizeof(T) == 4;
  FusedScratch ws;
  if ((rc = device_scratch(dev, defer, &ws))) return rc;
  if ((rc = begin_device_scratch(dev, st))) return rc;
  if (c.n > 0) {
    const unsigned zb = (unsigned)std::min<int64_t>(ceil_div(c.n, 256), 4096);
    hipLaunchKernelGGL(k_zero64_n, dim3(zb), dim3(256), 0, st, (unsigned long long*)gdx, c.n);
    hipLaunchKernelGGL(k_zero64_n, dim3(zb), dim3(256), 0, st, (unsigned long long*)gdy, c.n);
    hipLaunchKernelGGL(k_zero64_n, dim3(zb), dim3(256), 0, st, (unsigned long long*)gdz, c.n);
  }
  int nb = 0;
  if (c.n > 0) {
    AdjArgs A;
    A.seg = c.sv;
    A.n_seg = c.n;
    A.atm = c.ad;
    A.k0 = (uint32_t)(c.seed & 0xffffffffu);
    A.k1 = (uint32_t)(c.seed >> 32);
    A.K = c.g.K;
    A.inv_l1 = c.g.inv_l1;
    A.inv_dl = c.g.inv_dl;
    A.offsets = offsets;
    A.chunk = kAdjChunk;
    A.mu0 = mean0;
    A.sg = c.sg;
    A.grad = grad;
    A.gdx = gdx;
    A.gdy = gdy;
    A.gdz = gdz;
    A.partials = dev->adj_part;
    A.cursor = ws.cursor;
    A.defer_counts = ws.defer_counts;
    A.defer_q = ws.defer_q;
    A.defer_cap = defer ? ws.defer_rays / grid : 0;
    A.defer_pref = ws.defer_pref;
    A.n_defer_blocks = (int32_t)grid;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, ws.cursor, 1);
    hipLaunchKernelGGL((k_splat_adjoint<T, BS>), dim3((unsigned)grid), dim3(BS), 0, st, A);
    nb = (int)grid;
    if (defer) {
      hipLaunchKernelGGL(k_defer_scan, dim3(1), dim3(1024), 0, st, (const unsigned long long*)A.defer_counts,
                         (int)grid, A.defer_cap, A.defer_pref);
      hipLaunchKernelGGL((k_splat_adjoint_deferred<256>), dim3((unsigned)grid), dim3(256), 0, st, A, grid);
      nb = 2 * (int)grid;
    }
  }
  hipLaunchKernelGGL(k_adj_finalize, dim3(1), dim3(64), 0, st, (const double*)dev->adj_part, nb, c.ad, gH, geta);
  if ((rc = check_launch())) return rc;
  return end_device_scratch(dev, st);
}

}  // namespace

struct photon_plan_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  OwnedScratch scratch;  // the plan's own work cursor and deferral queue
};

// ================================================================= C ABI ==
extern "C" {

#ifndef PHOTON_SOURCE_HASH
#define PHOTON_SOURCE_HASH "unknown"
#endif
const char* photon_version(void) { return "libphoton 0.2 (gfx950) source " PHOTON_SOURCE_HASH; }

const char* photon_last_error(void) { return g_err.c_str(); }

int photon_init(void) {
  DeviceState* d;
  int rc;
  if ((rc = current_device(&d))) return rc;
  if ((rc = ensure_work(d))) return rc;
  FusedScratch ws;
  return static_scratch(d, &ws);
}

int photon_gen_cherenkov(const photon_segments* seg, const photon_atmosphere* atm, double lambda_min_nm,
                         double lambda_max_nm, uint64_t seed, int32_t precision, uint32_t* counts, uint64_t* offsets,
                         photon_block* out, void* stream) {
  photon_emission em;
  std::memset(&em, 0, sizeof em);
  em.kind = PHOTON_CHERENKOV;
  em.lambda_min_nm = lambda_min_nm;
  em.lambda_max_nm = lambda_max_nm;
  return generate_common(seg, atm, &em, seed, precision, counts, offsets, out, stream);
}

int photon_gen_fluor(const photon_segments* seg, const photon_atmosphere* atm, const double* line_nm,
                     const double* line_rel_yield, int32_t n_lines, double yield_per_MeV, uint64_t seed,
                     int32_t precision, uint32_t* counts, uint64_t* offsets, photon_block* out, void* stream) {
  if (!line_nm || !line_rel_yield) return fail(PHOTON_EINVAL, "line tables are NULL");
  if (n_lines < 1 || n_lines > PHOTON_MAX_LINES)
    return fail(PHOTON_EINVAL, "n_lines = %d outside 1..%d", n_lines, PHOTON_MAX_LINES);
  photon_emission em;
  std::memset(&em, 0, sizeof em);
  em.kind = PHOTON_FLUORESCENCE;
  em.yield_per_MeV = yield_per_MeV;
  em.n_lines = n_lines;
  for (int k = 0; k < n_lines; ++k) {
    em.line_nm[k] = line_nm[k];
    em.line_rel_yield[k] = line_rel_yield[k];
  }
  return generate_common(seg, atm, &em, seed, precision, counts, offsets, out, stream);
}

int photon_propagate(photon_block* inout, const photon_atmosphere* atm, void* stream) {
  AtmDev ad;
  int rc;
  if (!inout) return fail(PHOTON_EINVAL, "photon block is NULL");
  if ((rc = prep_atm(atm, &ad))) return rc;
  if ((rc = prep_precision(inout->precision))) return rc;
  if ((rc = check_block(inout, inout->precision))) return rc;
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  hipStream_t st = (hipStream_t)stream;
  return inout->precision == PHOTON_FP64 ? launch_propagate<double>(inout, ad, st) : launch_propagate<float>(inout, ad, st);
}

int photon_collect(const photon_block* in, const photon_atmosphere* atm, const photon_sink* sink, void* stream) {
  AtmDev ad;
  SinkDev sk;
  int rc;
  if (!in) return fail(PHOTON_EINVAL, "photon block is NULL");
  if ((rc = prep_atm(atm, &ad))) return rc;
  if ((rc = prep_precision(in->precision))) return rc;
  if ((rc = prep_sink(sink, &sk, ad.hobs, in->precision))) return rc;
  if ((rc = check_block(in, in->precision))) return rc;
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  hipStream_t st = (hipStream_t)stream;
  return in->precision == PHOTON_FP64 ? launch_collect<double>(in, ad, sk, st) : launch_collect<float>(in, ad, sk, st);
}

int photon_run_fused(const photon_segments* seg, const photon_atmosphere* atm, const photon_emission* em, uint64_t seed,
                     int32_t precision, const uint64_t* offsets, int64_t n_photons, const photon_sink* sink,
                     const photon_tuning* tuning, void* stream) {
  StepArgs a;
  int rc;
  if ((rc = prep_step(seg, atm, em, seed, precision, sink, tuning, &a))) return rc;
  if (!offsets) return fail(PHOTON_EINVAL, "offsets is NULL");
  if (n_photons < -1) return fail(PHOTON_EINVAL, "n_photons must be >= 0, or -1 (total read on the device)");
  if (sink->kind == PHOTON_SINK_PLANE && n_photons > sink->plane->capacity)
    return fail(PHOTON_ECAPACITY, "n_photons = %lld exceeds the plane capacity %lld", (long long)n_photons,
                (long long)sink->plane->capacity);
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  return enqueue_fused(a, offsets, n_photons, tuning, dev, (hipStream_t)stream);
}

int photon_run_fused_noalloc(const photon_segments* seg, const photon_atmosphere* atm, const photon_emission* em,
                             uint64_t seed, int32_t precision, const uint64_t* offsets, int64_t n_photons,
                             const photon_sink* sink, const photon_tuning* tuning, void* stream) {
  StepArgs a;
  int rc;
  if ((rc = prep_step(seg, atm, em, seed, precision, sink, tuning, &a))) return rc;
  if (!offsets) return fail(PHOTON_EINVAL, "offsets is NULL");
  if (n_photons < -1) return fail(PHOTON_EINVAL, "n_photons must be >= 0, or -1 (total read on the device)");
  if (sink->kind == PHOTON_SINK_PLANE && n_photons > sink->plane->capacity)
    return fail(PHOTON_ECAPACITY, "n_photons = %lld exceeds the plane capacity %lld", (long long)n_photons,
                (long long)sink->plane->capacity);
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  FusedScratch ws;
  if ((rc = static_scratch(dev, &ws))) return rc;
  return enqueue_fused(a, offsets, n_photons, tuning, dev, (hipStream_t)stream, nullptr, &ws);
}

int photon_kernel_timing(int32_t on) {
  DeviceState* dev;
  int rc;
  if ((rc = current_device(&dev))) return rc;
  if (on && !dev->t_ev[0]) {
    for (hipEvent_t& e : dev->t_ev)
      if (hipEventCreate(&e) != hipSuccess) return fail(PHOTON_EHIP, "event creation failed");
  }
  dev->timing = on != 0;
  dev->timed = false;
  dev->timed_defer = false;
  return PHOTON_OK;
}

int photon_peak_run(int32_t kind, void* work, int64_t work_bytes, int32_t iters, double* ops, float* ms,
                    void* stream) {
  if (kind < 0 || kind > 7) return fail(PHOTON_EINVAL, "peak kind %d outside 0..7", kind);
  if (!work || !ops || !ms) return fail(PHOTON_EINVAL, "work/ops/ms is NULL");
  if (iters < 1 || iters > (1 << 20)) return fail(PHOTON_EINVAL, "iters %d outside 1..2^20", iters);
  DeviceState* dev;
  int rc;
  if ((rc = current_device(&dev))) return rc;
  // eight 256-thread blocks per CU: eight waves per SIMD
  const int64_t grid = (int64_t)dev->cu * 8;
  const int64_t threads = grid * peaks::kBlock;
  const int64_t out_bytes = threads * 8;
  constexpr int64_t kReadOffset = 1 << 16;
  if (kind != 5 && work_bytes < out_bytes)
    return fail(PHOTON_EINVAL, "work_bytes %lld below %lld", (long long)work_bytes, (long long)out_bytes);
  if (kind == 5 && (work_bytes < kReadOffset + (1 << 20) || grid * 4 > kReadOffset))
    return fail(PHOTON_EINVAL, "work_bytes %lld below 64 KiB + 1 MiB", (long long)work_bytes);
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(PHOTON_EHIP, "event creation failed");
  }
  (void)hipEventRecord(e0, st);
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(peaks::k_fma<float>, dim3((unsigned)grid), dim3(peaks::kBlock), 0, st, (float*)work, iters,
                         0.999f, 1e-4f);
      *ops = (double)threads * iters * peaks::kChains;
      break;
    case 1:
      hipLaunchKernelGGL(peaks::k_fma<double>, dim3((unsigned)grid), dim3(peaks::kBlock), 0, st, (double*)work, iters,
                         0.999, 1e-4);
      *ops = (double)threads * iters * peaks::kChains;
      break;
    case 2:
      hipLaunchKernelGGL(peaks::k_mad64, dim3((unsigned)grid), dim3(peaks::kBlock), 0, st, (uint64_t*)work, iters,
                         0xD2511F53u);
      *ops = (double)threads * iters * peaks::kChains;
      break;
    case 3:
      hipLaunchKernelGGL(peaks::k_exp2, dim3((unsigned)grid), dim3(peaks::kBlock), 0, st, (float*)work, iters);
      *ops = (double)threads * iters * peaks::kChains;
      break;
    case 4:
      hipLaunchKernelGGL(peaks::k_mix, dim3((unsigned)grid), dim3(peaks::kBlock), 0, st, (float*)work, iters, 0.999f,
                         1e-4f);
      *ops = (double)threads * iters * peaks::kChains;
      break;
    case 6:
      hipLaunchKernelGGL(peaks::k_lds_add32, dim3((unsigned)grid), dim3(peaks::kBlock), 0, st, (uint32_t*)work,
                         iters);
      *ops = (double)threads * iters * peaks::kChains;
      break;
    case 7:
      hipLaunchKernelGGL(peaks::k_lds_add64, dim3((unsigned)grid), dim3(peaks::kBlock), 0, st,
                         (unsigned long long*)work, iters);
      *ops = (double)threads * iters * peaks::kChains;
      break;
    default: {
      const int64_t n4 = (work_bytes - kReadOffset) / 16;
      hipLaunchKernelGGL(peaks::k_read, dim3((unsigned)grid), dim3(peaks::kBlock), 0, st,
                         (const float4*)((char*)work + kReadOffset), n4, (float*)work);
      *ops = (double)n4 * 16.0;
    }
  }
  (void)hipEventRecord(e1, st);
  rc = check_launch();
  if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess))
    rc = fail(PHOTON_EHIP, "event timing failed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int photon_fused_deferred_ms(float* ms) {
  if (!ms) return fail(PHOTON_EINVAL, "ms is NULL");
  DeviceState* dev;
  int rc;
  if ((rc = current_device(&dev))) return rc;
  if (!dev->timed) return fail(PHOTON_EINVAL, "no fused kernel timed on this device (photon_kernel_timing off?)");
  if (!dev->timed_defer) {
    *ms = 0.0f;
    return PHOTON_OK;
  }
  if (hipEventSynchronize(dev->t_ev[2]) != hipSuccess || hipEventElapsedTime(ms, dev->t_ev[1], dev->t_ev[2]) != hipSuccess)
    return fail(PHOTON_EHIP, "event timing failed");
  return PHOTON_OK;
}

int photon_fused_kernel_ms(float* ms) {
  if (!ms) return fail(PHOTON_EINVAL, "ms is NULL");
  DeviceState* dev;
  int rc;
  if ((rc = current_device(&dev))) return rc;
  if (!dev->timed) return fail(PHOTON_EINVAL, "no fused kernel timed on this device (photon_kernel_timing off?)");
  if (hipEventSynchronize(dev->t_ev[1]) != hipSuccess || hipEventElapsedTime(ms, dev->t_ev[0], dev->t_ev[1]) != hipSuccess)
    return fail(PHOTON_EHIP, "event timing failed");
  return PHOTON_OK;
}

int photon_plan_create(const photon_segments* seg, const photon_atmosphere* atm, const photon_emission* em,
                       uint64_t seed, int32_t precision, uint32_t* counts, uint64_t* offsets,
                       const photon_sink* sink, const photon_tuning* tuning, photon_plan* out) {
  if (!out) return fail(PHOTON_EINVAL, "plan output pointer is NULL");
  *out = nullptr;
  StepArgs a;
  int rc;
  if ((rc = prep_step(seg, atm, em, seed, precision, sink, tuning, &a))) return rc;
  if (!offsets || !counts) return fail(PHOTON_EINVAL, "counts/offsets are NULL");
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  warm_occupancy(dev);
  photon_plan_s* p = new photon_plan_s;
  if ((rc = alloc_scratch(precision == PHOTON_FP32 ? dev->defer_rays : 0, &p->scratch))) {
    delete p;
    return rc;
  }
  const FusedScratch ws = p->scratch.view();
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    free_scratch(&p->scratch);
    delete p;
    return fail(PHOTON_EHIP, "capture stream creation failed");
  }
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    free_scratch(&p->scratch);
    delete p;
    return fail(PHOTON_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  rc = enqueue_step(a, counts, offsets, tuning, dev, cs, &ws);
  e = hipStreamEndCapture(cs, &p->graph);
  (void)hipStreamDestroy(cs);
  if (rc || e != hipSuccess) {
    if (p->graph) (void)hipGraphDestroy(p->graph);
    free_scratch(&p->scratch);
    delete p;
    return rc ? rc : fail(PHOTON_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  }
  e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(p->graph);
    free_scratch(&p->scratch);
    delete p;
    return fail(PHOTON_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *out = p;
  return PHOTON_OK;
}

int photon_plan_launch(photon_plan plan, void* stream) {
  if (!plan || !plan->exec) return fail(PHOTON_EINVAL, "plan is NULL");
  HIP_TRY(hipGraphLaunch(plan->exec, (hipStream_t)stream));
  return PHOTON_OK;
}

int photon_plan_destroy(photon_plan plan) {
  if (!plan) return PHOTON_OK;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  free_scratch(&plan->scratch);
  delete plan;
  return PHOTON_OK;
}

int photon_set_defer_capacity(int64_t rays) {
  if (rays < 1 || rays > ((int64_t)1 << 28))
    return fail(PHOTON_EINVAL, "deferral capacity %lld outside 1..2^28", (long long)rays);
  DeviceState* dev;
  int rc;
  if ((rc = current_device(&dev))) return rc;
  HIP_TRY(hipDeviceSynchronize());
  std::lock_guard<std::mutex> lk(g_mu);
  if (dev->defer_q) (void)hipFree(dev->defer_q);
  if (dev->defer_pref) (void)hipFree(dev->defer_pref);
  dev->defer_q = nullptr;
  dev->defer_pref = nullptr;
  dev->defer_rays = rays;
  return PHOTON_OK;
}

int photon_autotune(const photon_segments* seg, const photon_atmosphere* atm, const photon_emission* em,
                    uint64_t seed, int32_t precision, const uint64_t* offsets, const photon_sink* sink,
                    const photon_tuning* candidates, int32_t n_candidates, int32_t reps, photon_tuning* best,
                    float* best_ms, void* stream) {
  StepArgs a;
  int rc;
  if ((rc = prep_step(seg, atm, em, seed, precision, sink, nullptr, &a))) return rc;
  if (!offsets) return fail(PHOTON_EINVAL, "offsets is NULL");
  if (!candidates || n_candidates < 1) return fail(PHOTON_EINVAL, "no candidate shapes");
  if (reps < 1) return fail(PHOTON_EINVAL, "reps must be >= 1");
  if (!best || !best_ms) return fail(PHOTON_EINVAL, "best/best_ms is NULL");
  for (int i = 0; i < n_candidates; ++i)
    if ((rc = validate_tuning(&candidates[i]))) return rc;
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best_t = 0.0f;
  int best_i = -1;
  // every run starts from cleared sink outputs, so that each candidate does
  // the same work (a full hit buffer would skip the stores of later runs)
  const ZeroList z = sink_zero_list(a.sk);
  for (int i = 0; i < n_candidates && rc == PHOTON_OK; ++i) {
    if ((rc = enqueue_fused(a, offsets, -1, &candidates[i], dev, st, &z))) break;
    float t[64];
    const int nr = reps < 64 ? reps : 64;
    for (int r = 0; r < nr; ++r) {
      (void)hipEventRecord(e0, st);
      if ((rc = enqueue_fused(a, offsets, -1, &candidates[i], dev, st, &z))) break;
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = fail(PHOTON_EHIP, "hipEventSynchronize failed");
        break;
      }
      (void)hipEventElapsedTime(&t[r], e0, e1);
    }
    if (rc) break;
    for (int x = 1; x < nr; ++x)  // insertion sort for the median
      for (int y = x; y > 0 && t[y] < t[y - 1]; --y) {
        const float tmp = t[y];
        t[y] = t[y - 1];
        t[y - 1] = tmp;
      }
    const float med = t[nr / 2];
    if (best_i < 0 || med < best_t) {
      best_t = med;
      best_i = i;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  launch_zero_list(z, st);
  if ((rc = check_launch())) return rc;
  *best = candidates[best_i];
  *best_ms = best_t;
  return PHOTON_OK;
}

int photon_count(const photon_segments* seg, const photon_atmosphere* atm, const photon_emission* em,
                 uint64_t seed, uint32_t* counts, uint64_t* offsets, void* stream) {
  if (!em) return fail(PHOTON_EINVAL, "emission is NULL");
  return generate_common(seg, atm, em, seed, PHOTON_FP64, counts, offsets, nullptr, stream);
}

int photon_table_build(const photon_atmosphere* atm, photon_table* table, void* stream) {
  if (!atm || !table) return fail(PHOTON_EINVAL, "atmosphere or table is NULL");
  photon_atmosphere a = *atm;
  a.table = nullptr;
  AtmDev ad;
  int rc;
  if ((rc = prep_atm(&a, &ad))) return rc;
  if ((rc = check_table_shape(&a, table))) return rc;
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  const int64_t n = (int64_t)table->n_h * table->n_q + table->n_v;
  hipLaunchKernelGGL(k_table_build, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, (hipStream_t)stream, ad,
                     table->n_h, table->n_q, table->n_v, table->h_max, table->q_max, (float4*)table->corr,
                     (float2*)table->vert);
  if ((rc = check_launch())) return rc;
  table->atm_hash = atm_hash(&a);
  return PHOTON_OK;
}

int photon_radial_profile(const photon_sink* sink, double* density, double* mean_t_ns, void* stream) {
  if (!sink) return fail(PHOTON_EINVAL, "sink is NULL");
  if (sink->kind != PHOTON_SINK_RADIAL) return fail(PHOTON_EINVAL, "sink is not RADIAL");
  SinkDev sk;
  std::memset(&sk, 0, sizeof sk);
  int rc;
  if ((rc = prep_radial(sink, &sk))) return rc;
  if (!density || !mean_t_ns) return fail(PHOTON_EINVAL, "profile outputs are NULL");
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_radial_finish, dim3((unsigned)ceil_div(sk.n_bins, 256)), dim3(256), 0, st, sk, sink->r_max,
                     density, mean_t_ns);
  return check_launch();
}

int photon_generate(const photon_segments* seg, const photon_atmosphere* atm, const photon_emission* em,
                    uint64_t seed, int32_t precision, const uint64_t* offsets, photon_block* out, void* stream) {
  if (!em) return fail(PHOTON_EINVAL, "emission is NULL");
  if (!out) return fail(PHOTON_EINVAL, "photon block is NULL");
  return generate_common(seg, atm, em, seed, precision, nullptr, const_cast<uint64_t*>(offsets), out, stream);
}

int photon_means(const photon_segments* seg, const photon_atmosphere* atm, const photon_emission* em, double* mean,
                 void* stream) {
  SegView sv;
  AtmDev ad;
  GenParams g;
  int rc;
  if (!em) return fail(PHOTON_EINVAL, "emission is NULL");
  if ((rc = prep_seg(seg, &sv, em->kind == PHOTON_FLUORESCENCE))) return rc;
  if ((rc = prep_atm(atm, &ad))) return rc;
  if ((rc = prep_emission(em, &g))) return rc;
  CutDev cut;
  if ((rc = prep_cut(em, &cut))) return rc;
  if (!mean && seg->n > 0) return fail(PHOTON_EINVAL, "mean is NULL");
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  if (seg->n == 0) return PHOTON_OK;
  hipStream_t st = (hipStream_t)stream;
  const unsigned nb = (unsigned)ceil_div(seg->n, 256);
  if (em->kind == PHOTON_CHERENKOV) {
    const double K = (2.0 * kPi * kAlpha) * ((1e9 / em->lambda_min_nm) - (1e9 / em->lambda_max_nm));
    hipLaunchKernelGGL(k_means<PHOTON_CHERENKOV>, dim3(nb), dim3(256), 0, st, sv, seg->n, ad, K, cut, g.beam, mean);
  } else {
    hipLaunchKernelGGL(k_means<PHOTON_FLUORESCENCE>, dim3(nb), dim3(256), 0, st, sv, seg->n, ad, em->yield_per_MeV, cut,
                       g.beam, mean);
  }
  return check_launch();
}

int photon_splat_forward(const photon_segments* seg, const photon_atmosphere* atm, double lambda_min_nm,
                         double lambda_max_nm, uint64_t seed, int32_t precision, const uint64_t* offsets,
                         const double* mean0, const photon_splat_grid* grid, void* density,
                         unsigned long long* status_totals, void* stream) {
  SplatCall c;
  int rc;
  if ((rc = prep_splat_call(seg, atm, lambda_min_nm, lambda_max_nm, seed, precision, offsets, mean0, grid, &c)))
    return rc;
  if (!density) return fail(PHOTON_EINVAL, "density is NULL");
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int cells = c.sg.nx * c.sg.ny;
  if ((rc = ensure_splat_acc(dev, cells))) return rc;
  if ((rc = begin_device_scratch(dev, st))) return rc;
  hipLaunchKernelGGL(k_zero64_n, dim3((unsigned)std::min<int64_t>(ceil_div(cells, 256), 4096)), dim3(256), 0, st,
                     dev->splat_acc, (int64_t)cells);
  if (status_totals) hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, status_totals, PHOTON_N_STATUS);
  if (c.n > 0) {
    SinkDev sk;
    std::memset(&sk, 0, sizeof sk);
    sk.kind = kSinkSplat;
    sk.totals = status_totals;
    sk.sg = c.sg;
    sk.splat_acc = dev->splat_acc;
    sk.mu0 = mean0;
    // each block accumulates the whole grid in LDS when it fits beside the
    // kernel's own LDS: 32-bit cells in the float form (splat_add32; two
    // 768-thread blocks per CU for a 128 x 128 grid), 64-bit cells in the
    // double form (one 512-thread block per CU)
    const size_t lds = (size_t)cells * (precision == PHOTON_FP32 ? sizeof(uint32_t) : sizeof(unsigned long long));
    hipFuncAttributes fa;
    const void* kf = precision == PHOTON_FP32 ? reinterpret_cast<const void*>(&k_fused<float, kSplatBs32, kMSplat>)
                                              : reinterpret_cast<const void*>(&k_fused<double, 512, kMSplat>);
    const bool fits = hipFuncGetAttributes(&fa, kf) == hipSuccess && fa.sharedSizeBytes + lds <= dev->lds_per_block;
    sk.splat_lds = fits ? 1 : 0;
    // large chunks: a block's serial set-up of a chunk (work cursor, segment
    // search, window) is hidden by few or no other blocks (1e6-segment
    // workload, FP64 4096 -> 8192 photons: 7.02 -> 6.55 ms; FP32 3072 -> 6144
    // -> 8448: 3.86 -> 3.52 -> ... -> 3.05 -> 2.84 ms)
    if (precision == PHOTON_FP32)
      rc = fits ? launch_fused_bs<float, kSplatBs32, true>(c.sv, c.n, c.ad, c.g, seed, offsets, -1, kSplatChunk32, 0, sk,
                                                           dev, st, lds)
                : launch_fused_bs<float, 256, true>(c.sv, c.n, c.ad, c.g, seed, offsets, -1, 4096, 0, sk, dev, st);
    else
      rc = fits ? launch_fused_bs<double, 512, true>(c.sv, c.n, c.ad, c.g, seed, offsets, -1, 8192, 0, sk, dev, st, lds)
                : launch_fused_bs<double, 256, true>(c.sv, c.n, c.ad, c.g, seed, offsets, -1, 4096, 0, sk, dev, st);
    if (rc) return rc;
  }
  const unsigned nb = (unsigned)ceil_div(cells, 256);
  if (precision == PHOTON_FP64)
    hipLaunchKernelGGL(k_splat_finish<double>, dim3(nb), dim3(256), 0, st, (const unsigned long long*)dev->splat_acc,
                       cells, c.sg.norm, (double*)density);
  else
    hipLaunchKernelGGL(k_splat_finish<float>, dim3(nb), dim3(256), 0, st, (const unsigned long long*)dev->splat_acc,
                       cells, c.sg.norm, (float*)density);
  if ((rc = check_launch())) return rc;
  return end_device_scratch(dev, st);
}

int photon_splat_backward(const photon_segments* seg, const photon_atmosphere* atm, double lambda_min_nm,
                          double lambda_max_nm, uint64_t seed, int32_t precision, const uint64_t* offsets,
                          const double* mean0, const photon_splat_grid* grid, const void* grad_density,
                          double* grad_scale_height, double* grad_n0_minus_1, double* grad_dx, double* grad_dy,
                          double* grad_dz, void* stream) {
  SplatCall c;
  int rc;
  if ((rc = prep_splat_call(seg, atm, lambda_min_nm, lambda_max_nm, seed, precision, offsets, mean0, grid, &c)))
    return rc;
  if (!grad_density) return fail(PHOTON_EINVAL, "grad_density is NULL");
  if (!grad_scale_height || !grad_n0_minus_1) return fail(PHOTON_EINVAL, "global gradient outputs are NULL");
  if (seg->n > 0 && (!grad_dx || !grad_dy || !grad_dz)) return fail(PHOTON_EINVAL, "direction gradient outputs are NULL");
  DeviceState* dev;
  if ((rc = current_device(&dev))) return rc;
  hipStream_t st = (hipStream_t)stream;
  return precision == PHOTON_FP64
             ? launch_adjoint<double>(c, offsets, mean0, grad_density, grad_scale_height, grad_n0_minus_1, grad_dx,
                                      grad_dy, grad_dz, dev, st)
             : launch_adjoint<float>(c, offsets, mean0, grad_density, grad_scale_height, grad_n0_minus_1, grad_dx,
                                     grad_dy, grad_dz, dev, st);
}

}  // extern "C"
