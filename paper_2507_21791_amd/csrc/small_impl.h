// Device code of the small kernels (fixed-order reduction of the Gram
// partials, fill, info reset): included by their launchers' sources and by
// the batched persistent kernel, which runs the same bodies as work items.
#pragma once

#include "common.h"

namespace bcgs {

// Sum of the G per-workgroup partials, entry by entry, in a fixed order:
// "wave" w of 16 adds partials w, w+16, ... into four interleaved running
// sums (so four loads are in flight), and the 16 wave sums are added in
// wave order.  Block `block` covers entries [64 block, 64 block + 64); a
// workgroup of fewer than 16 waves takes the 16 wave roles in turn, so the
// result depends only on G.  red: 16 x 64 doubles of LDS.
constexpr int kRedWaves = 16;

__device__ __forceinline__ void reduce_body(
    const double* __restrict__ partial, int G, int64_t elems,
    double* __restrict__ out, int32_t* syncs, double* red, int64_t block) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int nw = blockDim.x >> 6;
  const int64_t e = block * 64 + lane;
  for (int w = tid >> 6; w < kRedWaves; w += nw) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (e < elems) {
      int g = w;
      for (; g + 3 * kRedWaves < G; g += 4 * kRedWaves) {
        a0 += partial[(size_t)g * elems + e];
        a1 += partial[(size_t)(g + kRedWaves) * elems + e];
        a2 += partial[(size_t)(g + 2 * kRedWaves) * elems + e];
        a3 += partial[(size_t)(g + 3 * kRedWaves) * elems + e];
      }
      for (; g < G; g += kRedWaves) a0 += partial[(size_t)g * elems + e];
    }
    red[w * 64 + lane] = (a0 + a1) + (a2 + a3);
  }
  __syncthreads();
  if (tid < 64 && e < elems) {
    double t = red[lane];
#pragma unroll
    for (int i = 1; i < kRedWaves; ++i) t += red[i * 64 + lane];
    out[e] = t;
  }
  // one synchronization point completed (counted by one thread)
  if (syncs != nullptr && block == 0 && tid == 0) *syncs += 1;
}

// p(i, j) = value for i < rows, j < cols of a column-major matrix with
// leading dimension ld; block `block` of 256-element blocks
__device__ __forceinline__ void fill_body(double* p, int64_t rows,
                                          int64_t cols, int64_t ld, double v,
                                          int64_t block) {
  const int64_t i = block * 256 + (threadIdx.x & 255);
  if (threadIdx.x < 256 && i < rows * cols) p[(i / rows) * ld + i % rows] = v;
}

// reset of the info record; synchronization points are counted from zero
// by the reductions and TSQR roots that follow
__device__ __forceinline__ void info_init_body(bcgs_info* info) {
  if (threadIdx.x == 0) {
    info->status = BCGS_OK;
    info->block = -1;
    info->pivot = -1;
    info->stage = -1;
    info->syncs = 0;
    info->reserved = 0;
    info->value = 0.0;
  }
}

}  // namespace bcgs
