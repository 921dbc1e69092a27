// Micro-benchmarks of the device rates that bound the photon kernels: FP32
// and FP64 fused multiply-adds, the 32x32->64 integer multiply-add of the
// Philox rounds, the FP32 transcendental unit (exp2), FMAs and exp2
// interleaved (the two can issue side by side), HBM reads, and the LDS
// integer adds of the splat (32-bit returning the old value, 64-bit without).
// A measurement aid for the rooflines (their nominal peaks come from unit
// counts and clock); nothing on the photon path uses them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace peaks {

constexpr int kBlock = 256;
constexpr int kChains = 8;  // independent dependency chains per thread

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fma(T* __restrict__ out, int iters, T b, T c) {
  T a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = (T)(threadIdx.x + k) * (T)1e-3;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = __builtin_fma(a[k], b, c);
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

template <>
__global__ __launch_bounds__(kBlock) void k_fma<float>(float* __restrict__ out, int iters, float b, float c) {
  float a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = (float)(threadIdx.x + k) * 1e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = __builtin_fmaf(a[k], b, c);
  }
  float s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

// x <- lo32(x) * m + hi32(x): one 32x32->64 multiply-add per step
__global__ __launch_bounds__(kBlock) void k_mad64(uint64_t* __restrict__ out, int iters, uint32_t m) {
  uint64_t x[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) x[k] = (uint64_t)(threadIdx.x * 2654435761u + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = (uint64_t)(uint32_t)x[k] * m + (x[k] >> 32);
  }
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s ^= x[k];
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

// a <- exp2(-a): bounded (the iteration settles near 0.64), one hardware
// exp2 per step
__global__ __launch_bounds__(kBlock) void k_exp2(float* __restrict__ out, int iters) {
  float a[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) a[k] = (float)(threadIdx.x + k) * 1e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = __builtin_amdgcn_exp2f(-a[k]);
  }
  float s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += a[k];
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

// one FMA chain and one exp2 chain per pair, interleaved 1:1
__global__ __launch_bounds__(kBlock) void k_mix(float* __restrict__ out, int iters, float b, float c) {
  float a[kChains / 2], e[kChains / 2];
#pragma unroll
  for (int k = 0; k < kChains / 2; ++k) {
    a[k] = (float)(threadIdx.x + k) * 1e-3f;
    e[k] = (float)(threadIdx.x + 2 * k) * 1e-3f;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains / 2; ++k) {
      a[k] = __builtin_fmaf(a[k], b, c);
      e[k] = __builtin_amdgcn_exp2f(-e[k]);
    }
  }
  float s = 0;
#pragma unroll
  for (int k = 0; k < kChains / 2; ++k) s += a[k] + e[k];
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s;
}

// reads n float4 with a grid-stride loop, one sum per block written back
__global__ __launch_bounds__(kBlock) void k_read(const float4* __restrict__ in, int64_t n, float* __restrict__ out) {
  __shared__ float part[kBlock / 64];
  float s = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const float4 v = in[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (part[0] + part[1]) + (part[2] + part[3]);
}

// LDS integer adds in the splat's pattern along a row: the lanes of a wave
// add to consecutive words (no two lanes of a wave on one bank beyond what
// the word size implies), eight chains per thread. 32-bit: the float splat's
// cell update, which returns the old value (summed, so the adds stay live).
constexpr int kLdsWords32 = 4096;  // 16 KB per block
__global__ __launch_bounds__(kBlock) void k_lds_add32(uint32_t* __restrict__ out, int iters) {
  __shared__ uint32_t s[kLdsWords32];
  for (int k = threadIdx.x; k < kLdsWords32; k += kBlock) s[k] = 0u;
  __syncthreads();
  uint32_t acc = 0u;
  for (int i = 0; i < iters; ++i) {
    const int base = (int)threadIdx.x + (i & 1) * (kLdsWords32 / 2);
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc += atomicAdd(&s[(base + k * kBlock) & (kLdsWords32 - 1)], 1u + k);
  }
  __syncthreads();
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = acc + s[threadIdx.x];
}

// 64-bit adds without a returned value: the double splat's cell update.
constexpr int kLdsWords64 = 2048;  // 16 KB per block
__global__ __launch_bounds__(kBlock) void k_lds_add64(unsigned long long* __restrict__ out, int iters) {
  __shared__ unsigned long long s[kLdsWords64];
  for (int k = threadIdx.x; k < kLdsWords64; k += kBlock) s[k] = 0ull;
  __syncthreads();
  for (int i = 0; i < iters; ++i) {
    const int base = (int)threadIdx.x + (i & 1) * (kLdsWords64 / 2);
#pragma unroll
    for (int k = 0; k < kChains; ++k) atomicAdd(&s[(base + k * kBlock) & (kLdsWords64 - 1)], 1ull + k);
  }
  __syncthreads();
  out[(int64_t)blockIdx.x * kBlock + threadIdx.x] = s[threadIdx.x];
}

}  // namespace peaks
