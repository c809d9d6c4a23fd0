// Shared device helpers for the gfx950 kernels: MFMA wrappers with their lane layouts,
// XCD-aware block remapping and small reductions.
//
// Matrix-core lane layouts on gfx950 (measured on the device, 64-lane wave, lane = c + 16 g,
// c = lane & 15, g = lane >> 4):
//   v_mfma_f64_16x16x4f64 : A[i][k] at lane i + 16 k;  B[k][j] at lane j + 16 k;
//                           D[i][j] at lane j + 16 (i % 4), register i / 4
//                           -> lane (g, c) holds rows g, g+4, g+8, g+12 of column c.
//   v_mfma_f32_16x16x4f32 : A, B as above; D[i][j] at lane j + 16 (i / 4), register i % 4
//                           -> lane (g, c) holds rows 4g .. 4g+3 of column c.
//   v_mfma_f32_16x16x32_bf16: A[i][k] at lane i + 16 (k / 8), element k % 8;
//                           B[k][j] at lane j + 16 (k / 8), element k % 8; D as f32 16x16x4.
// FP32 matrix-core accumulation rounds as it goes (1 + 0.75u + 0.75u returns 1), so long
// FP32 sums need promotion to FP64 for the accuracy target of the mixed path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slmc {

typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bfx8 __attribute__((ext_vector_type(8)));
typedef short sx8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ dx4 mfma64(double a, double b, dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fx4 mfma32(float a, float b, fx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fx4 mfmabf(bfx8 a, bfx8 b, fx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Row of the 16x16 accumulator block held by lane group g in register v.
__device__ __forceinline__ int drow64(int g, int v) { return g + 4 * v; }
__device__ __forceinline__ int drow32(int g, int v) { return 4 * g + v; }

// orders this wave's earlier LDS accesses before its later ones (lanes of one wave
// exchanging values through LDS)
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ dx4 zero4d() { dx4 z = {0.0, 0.0, 0.0, 0.0}; return z; }
__device__ __forceinline__ fx4 zero4f() { fx4 z = {0.f, 0.f, 0.f, 0.f}; return z; }

// Workgroups are dealt to the 8 XCDs round robin (block b runs on XCD b % 8).  This maps
// the hardware block id to a logical id so that consecutive logical ids (the tiles of one
// item) run on the same XCD and share its L2.  `count` is the number of logical blocks;
// the grid must be launched with xcd_grid(count) blocks; ids >= count return -1.
__host__ __device__ __forceinline__ int xcd_grid(int count) { return ((count + 7) / 8) * 8; }
__device__ __forceinline__ int xcd_remap(int bid, int count) {
  int per = (count + 7) / 8;
  int logical = (bid % 8) * per + bid / 8;
  return logical < count ? logical : -1;
}

// Row rotation of a double inside each 16-lane row (DPP row_ror:K).
template <int K>
__device__ __forceinline__ double ror16(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x120 + K, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x120 + K, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a row (lanes 16g .. 16g+15); every lane gets the total.
__device__ __forceinline__ double sum16(double v) {
  v += ror16<8>(v);
  v += ror16<4>(v);
  v += ror16<2>(v);
  v += ror16<1>(v);
  return v;
}
__device__ __forceinline__ double sum64(double v) {
  v = sum16(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}


}  // namespace slmc
