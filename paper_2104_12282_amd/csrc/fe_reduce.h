// Deterministic float64 reductions in two launches.
//
// A producing kernel reduces its values inside each workgroup in a fixed
// order (wave64 butterfly, then the four waves in index order) and stores
// one partial per workgroup: partials[slot * blocks + block].  A one-
// workgroup finalize kernel, launched right after on the same stream, sums
// the partials in block order and applies the scalar update.  The kernel
// boundary orders the two, so no workgroup ever fences the L2 (a device-scope
// fence per workgroup writes back and invalidates the L2 of its XCD, which
// costs more than the data pass itself).  Results are bitwise reproducible.
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

// Index and count of the workgroups of one problem: the x dimension of the
// grid (a batched launch runs one problem per y index, each with its own
// partials).
__device__ inline uint32_t block_id() { return blockIdx.x; }
__device__ inline uint32_t block_count() { return gridDim.x; }

// Sum of v[0..NV) over the workgroup (FE_BLOCK threads); totals valid in
// thread 0.  Every thread of the workgroup must call it.
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

// Producer side: one partial per workgroup and slot.
template <int NV>
__device__ inline void block_partials(double (&v)[NV], double* partials) {
  block_sum<NV>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[(size_t)i * block_count() + block_id()] = v[i];
  }
}

__device__ inline void block_partial_max(double v, double* partials) {
  v = block_max(v);
  if (threadIdx.x == 0) partials[block_id()] = v;
}

// Finalize side (one workgroup): totals of the nb partials of each slot, in
// thread 0.
template <int NV>
__device__ inline void reduce_partials(double (&v)[NV], const double* partials, int nb) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += FE_BLOCK) s += partials[(size_t)i * nb + b];
    v[i] = s;
  }
  block_sum<NV>(v);
}

__device__ inline double reduce_partials_max(const double* partials, int nb) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += FE_BLOCK) s = fmax(s, partials[b]);
  return block_max(s);
}

__device__ inline bool finite_d(double x) { return x - x == 0.0; }
