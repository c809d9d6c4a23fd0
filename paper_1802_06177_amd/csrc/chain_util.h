// Helpers shared by the segment-product kernels.
#pragma once
#include "common.h"
#include "launch.h"

namespace slmc {

static __device__ __forceinline__ const double* field_of(const FieldRef& f, int b) {
  return f.x + (f.xoff ? f.xoff[b] : (int64_t)b * f.xstride);
}

// v[q] = exp(-ldl x[l][q]) for q < N, 1 on padded sites.
static __device__ __forceinline__ void fill_v(double* v, const double* xb, int l, int N, int Np,
                                       double ldl) {
  for (int q = threadIdx.x; q < Np; q += blockDim.x)
    v[q] = q < N ? exp(-ldl * xb[(size_t)l * N + q]) : 1.0;
}

// Round-to-nearest-even float -> bf16 bit pattern, and back to double.
static __device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}
static __device__ __forceinline__ double bf16_to_d(uint16_t h) {
  return (double)__uint_as_float(((uint32_t)h) << 16);
}

}  // namespace slmc
