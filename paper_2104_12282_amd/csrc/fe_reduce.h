// Deterministic block and grid reductions for float64 sums.
//
// Every workgroup reduces its values in a fixed order (wave64 butterfly, then
// the waves in index order), writes them to partials[v * blocks + block]
// and bumps an arrival counter; the workgroup that arrives last sums the
// partials in block order and runs the finaliser.  The result is independent
// of scheduling, so a solve is bitwise reproducible.
#pragma once
#include <hip/hip_runtime.h>

#include "fe_internal.h"

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Linear index and count of the workgroups of a (possibly 3-D) grid.
__device__ inline uint32_t block_id() {
  return blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
}
__device__ inline uint32_t block_count() { return gridDim.x * gridDim.y * gridDim.z; }

// Sum of v[0..NV) over the workgroup; the totals are valid in thread 0.
// Needs a barrier-free entry (all threads of the block call it).
template <int NV>
__device__ inline void block_sum(double (&v)[NV]) {
  __shared__ double sh[NV][FE_BLOCK / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = wave_sum(v[i]);
    if (lane == 0) sh[i][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < FE_BLOCK / 64; ++w) s += sh[i][w];
      v[i] = s;
    }
  }
  __syncthreads();
}

__device__ inline double block_max(double v) {
  __shared__ double sh[FE_BLOCK / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s = wave_max(v);
  if (lane == 0) sh[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < FE_BLOCK / 64; ++w) s = fmax(s, sh[w]);
    v = s;
  }
  __syncthreads();
  return v;
}

// Publishes the block sums and tells whether this block arrived last.  When it
// returns true, thread 0 holds in v[] the grid totals (fixed summation order).
template <int NV>
__device__ inline bool grid_sum(double (&v)[NV], double* partials, uint32_t* counter) {
  __shared__ int amlast;
  block_sum<NV>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[(size_t)i * block_count() + block_id()] = v[i];
    __threadfence();
    const uint32_t t = atomicAdd(counter, 1u);
    amlast = (t == block_count() - 1);
  }
  __syncthreads();
  if (!amlast) return false;
  __threadfence();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (uint32_t b = threadIdx.x; b < block_count(); b += FE_BLOCK)
      s += __builtin_nontemporal_load(&partials[(size_t)i * block_count() + b]);
    v[i] = s;
  }
  block_sum<NV>(v);
  if (threadIdx.x == 0) atomicExch(counter, 0u);
  return true;
}

__device__ inline bool grid_max(double& v, double* partials, uint32_t* counter) {
  __shared__ int amlast;
  v = block_max(v);
  if (threadIdx.x == 0) {
    partials[block_id()] = v;
    __threadfence();
    const uint32_t t = atomicAdd(counter, 1u);
    amlast = (t == block_count() - 1);
  }
  __syncthreads();
  if (!amlast) return false;
  __threadfence();
  double s = 0.0;
  for (uint32_t b = threadIdx.x; b < block_count(); b += FE_BLOCK)
    s = fmax(s, __builtin_nontemporal_load(&partials[b]));
  v = block_max(s);
  if (threadIdx.x == 0) atomicExch(counter, 0u);
  return true;
}

__device__ inline bool finite_d(double x) { return x - x == 0.0; }
