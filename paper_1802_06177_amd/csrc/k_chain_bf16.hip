// Segment products with split-bf16 matrix-core products (the "3 x BF16" precision form):
// every FP64 operand a is split as a = hi + lo (2 pieces, bf16x3: hi*hi + hi*lo + lo*hi)
// or a = hi + mid + lo (3 pieces, bf16x6: the six products of total order <= 2), the
// products run on v_mfma_f32_16x16x32_bf16 with FP32 accumulation inside each 32-wide
// k-block, and the k-block sums are promoted to FP64.  Structure otherwise as the FP64
// and FP32 segment kernels: one workgroup carries one column panel of one segment.
#include "common.h"
#include "launch.h"
#include "chain_util.h"

namespace slmc {

namespace {

// Split val into PIECES bf16 parts: each part is the bf16 rounding of what remains.
template <int PIECES>
__device__ __forceinline__ void split_bf(double val, uint16_t* out) {
  double r = val;
#pragma unroll
  for (int p = 0; p < PIECES; ++p) {
    uint16_t h = bf16_rne((float)r);
    out[p] = h;
    r -= bf16_to_d(h);
  }
}

// pairs (A piece, B piece) of the split product
template <int PIECES> struct Pairs;
template <> struct Pairs<2> {
  static constexpr int n = 3;
  __device__ static constexpr int a(int i) { return i == 2 ? 1 : 0; }
  __device__ static constexpr int b(int i) { return i == 1 ? 1 : 0; }
};
template <> struct Pairs<3> {
  static constexpr int n = 6;
  // (0,0) (0,1) (1,0) (0,2) (1,1) (2,0)
  __device__ static constexpr int a(int i) { return i == 2 ? 1 : (i == 4 ? 1 : (i == 5 ? 2 : 0)); }
  __device__ static constexpr int b(int i) { return i == 1 ? 1 : (i == 3 ? 2 : (i == 4 ? 1 : 0)); }
};

template <int RB, int CB, int PIECES>
__global__ __launch_bounds__(256) void seg_chain_bf(const double* __restrict__ E64,
                                                    const uint16_t* __restrict__ Ebf, FieldRef f,
                                                    int nb, int N, int Np, int Ltau, int n_s,
                                                    int m, int k0, int kc, double ldl, double* __restrict__ S,
                                                    double* __restrict__ snorm) {
  constexpr int W = 16 * CB;
  extern __shared__ double lds[];
  const int LDP = Np + 8;                                  // bf16 elements
  double* vbuf = lds;                                      // [2][Np]
  double* red = vbuf + 2 * Np;                             // [256]
  uint16_t* P = (uint16_t*)(red + 256);                    // [PIECES][W][LDP]
  const int npan = Np / W;
  const int id = xcd_remap(blockIdx.x, nb * kc * npan);
  if (id < 0) return;
  const int pan = id % npan, k = k0 + (id / npan) % kc, b = id / (npan * kc);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const int NRB = Np >> 4, NKB = Np >> 5, c0 = pan * W;
  const size_t plane = (size_t)W * LDP, eplane = (size_t)Np * Np;
  const double* xb = field_of(f, b);
  const int l0 = k * n_s, len = min(n_s, Ltau - l0);
  double* Sout = S + ((size_t)b * m + k) * Np * Np;
  double* nout = snorm + ((size_t)b * m + k) * Np;

  fill_v(vbuf, xb, l0, N, Np, ldl);
  if (len > 1) fill_v(vbuf + Np, xb, l0 + 1, N, Np, ldl);
  __syncthreads();
  if (len == 1) {
    const int j = tid % W, part = tid / W, nparts = 256 / W;
    double s2 = 0.0;
    for (int q = part; q < Np; q += nparts) {
      double val = E64[(size_t)q * Np + c0 + j] * vbuf[c0 + j];
      Sout[(size_t)q * Np + c0 + j] = val;
      s2 += val * val;
    }
    red[part * W + j] = s2;
    __syncthreads();
    if (tid < W) {
      double s = 0.0;
      for (int p = 0; p < nparts; ++p) s += red[p * W + tid];
      nout[c0 + tid] = s;
    }
    return;
  }
  for (int idx = tid; idx < W * Np; idx += 256) {
    int q = idx / W, j = idx - q * W;
    double val = vbuf[Np + q] * E64[(size_t)q * Np + c0 + j] * vbuf[c0 + j];
    uint16_t h[PIECES];
    split_bf<PIECES>(val, h);
#pragma unroll
    for (int p = 0; p < PIECES; ++p) P[p * plane + j * LDP + q] = h[p];
  }
  __syncthreads();

  for (int t = 1; t < len; ++t) {
    const bool last = (t == len - 1);
    double* vnext = vbuf + ((t + 1) & 1) * Np;
    if (!last) fill_v(vnext, xb, l0 + t + 1, N, Np, ldl);

    dx4 acc64[RB][CB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc64[r][cb] = zero4d();

    for (int kb = 0; kb < NKB; ++kb) {
      const int q0 = 32 * kb + 8 * g;
      sx8 av[RB][PIECES];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int rb = w + 4 * r;
        if (rb < NRB) {
#pragma unroll
          for (int p = 0; p < PIECES; ++p)
            av[r][p] = *(const sx8*)(Ebf + p * eplane + (size_t)(16 * rb + c) * Np + q0);
        }
      }
      sx8 bv[CB][PIECES];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int p = 0; p < PIECES; ++p)
          bv[cb][p] = *(const sx8*)(P + p * plane + (16 * cb + c) * LDP + q0);
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (w + 4 * r < NRB) {
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) {
            fx4 acc = zero4f();
#pragma unroll
            for (int i = Pairs<PIECES>::n - 1; i >= 0; --i)   // small products first
              acc = mfmabf(__builtin_bit_cast(bfx8, av[r][Pairs<PIECES>::a(i)]),
                           __builtin_bit_cast(bfx8, bv[cb][Pairs<PIECES>::b(i)]), acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[r][cb][v] += (double)acc[v];
          }
        }
    }
    __syncthreads();
    if (!last) {
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int rb = w + 4 * r;
        if (rb < NRB) {
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = 16 * rb + drow32(g, v);
              uint16_t h[PIECES];
              split_bf<PIECES>(vnext[row] * acc64[r][cb][v], h);
#pragma unroll
              for (int p = 0; p < PIECES; ++p) P[p * plane + (16 * cb + c) * LDP + row] = h[p];
            }
        }
      }
    } else {
      double s2[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) s2[cb] = 0.0;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int rb = w + 4 * r;
        if (rb < NRB) {
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = 16 * rb + drow32(g, v);
              const double val = acc64[r][cb][v];
              Sout[(size_t)row * Np + c0 + 16 * cb + c] = val;
              s2[cb] += val * val;
            }
        }
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        double sv = s2[cb];
        sv += __shfl_xor(sv, 16, 64);
        sv += __shfl_xor(sv, 32, 64);
        if (g == 0) red[w * W + 16 * cb + c] = sv;
      }
      __syncthreads();
      if (tid < W) nout[c0 + tid] = red[tid] + red[W + tid] + red[2 * W + tid] + red[3 * W + tid];
    }
    __syncthreads();
  }
}

template <int RB, int CB, int PIECES>
hipError_t run_bf(const double* E64, const uint16_t* Ebf, FieldRef f, int nb, int N, int Np,
                  int Ltau, int n_s, int m, int k0, int kc, double ldl, double* S, double* sn, hipStream_t st) {
  constexpr int W = 16 * CB;
  const int count = nb * kc * (Np / W);
  const size_t lds = (size_t)(2 * Np + 256) * sizeof(double) +
                     (size_t)PIECES * W * (Np + 8) * sizeof(uint16_t);
  hipLaunchKernelGGL((seg_chain_bf<RB, CB, PIECES>), dim3(xcd_grid(count)), dim3(256), lds, st,
                     E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, sn);
  return hipGetLastError();
}

template <int RB>
hipError_t pick_bf(int pieces, int CB, const double* E64, const uint16_t* Ebf, FieldRef f, int nb,
                   int N, int Np, int Ltau, int n_s, int m, int k0, int kc, double ldl, double* S, double* sn,
                   hipStream_t st) {
  if (pieces == 2) {
    if (CB == 2) return run_bf<RB, 2, 2>(E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, sn, st);
    return run_bf<RB, 1, 2>(E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, sn, st);
  }
  if (CB == 2) return run_bf<RB, 2, 3>(E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, sn, st);
  return run_bf<RB, 1, 3>(E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, sn, st);
}

}  // namespace

hipError_t launch_seg_bf16(int pieces, const double* E64, const uint16_t* Ebf, FieldRef f,
                           int nb, int N, int Np, int Ltau, int n_s, int m, int k0, int kc, double ldl,
                           double* S, double* snorm, hipStream_t st) {
  if (Np % 32 != 0) return hipErrorInvalidValue;   // k-blocks of 32
  const int NRB = Np / 16, RB = (NRB + 3) / 4;
  const int CB = (Np % 32 == 0) ? 2 : 1;
  switch (RB) {
    case 1: return pick_bf<1>(pieces, CB, E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
    case 2: return pick_bf<2>(pieces, CB, E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
    case 3: return pick_bf<3>(pieces, CB, E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
    case 4: return pick_bf<4>(pieces, CB, E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
    case 5: return pick_bf<5>(pieces, CB, E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
    case 6: return pick_bf<6>(pieces, CB, E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
    case 7: return pick_bf<7>(pieces, CB, E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
    default: return pick_bf<8>(pieces, CB, E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
  }
}

}  // namespace slmc
