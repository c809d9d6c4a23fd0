// Segment products of the slice-matrix chain (SM Eq. S2: M = I + B_L ... B_1 with
// B_l = e^{-dtau K} diag(e^{-dtau lam x_l})): S_k = B_{k n_s + len - 1} ... B_{k n_s}.
//
// Design: a workgroup owns a column panel S_k[:, c0 : c0 + 16 CB] of one (item, segment)
// and carries it through every slice of the segment without leaving the CU.  Column j of
// E (v ⊙ S) depends only on column j of S, so the panel lives in LDS between slices; the
// shared matrix E = e^{-dtau K} streams from L2 as the MFMA A-operand (each of the 4
// waves owns a disjoint set of 16-row blocks, so E is read once per slice per workgroup).
// The diagonal phonon factor of the next slice is applied to the panel rows as the
// matrix-core results are written back to LDS, so no separate scaling pass exists.
//
// This file holds the FP64 variant (v_mfma_f64_16x16x4f64) and the precision dispatch;
// the FP32 and split-bf16 variants live in k_chain_f32.hip and k_chain_bf16.hip.
#include "common.h"
#include "launch.h"
#include "chain_util.h"

namespace slmc {

namespace {

// Column panel of the first slice, E[:, c0+j] v_l0[c0+j], either scaled by v_next (rows)
// into the LDS panel (as TP), or written out with its column norms when the segment has
// a single slice.
template <typename TP>
__device__ void first_slice(const double* __restrict__ E, const double* vl0,
                            const double* vnext, TP* P, int LDP, int W, int c0, int Np,
                            bool single, double* __restrict__ Sout, double* red,
                            double* __restrict__ nout) {
  const int tid = threadIdx.x;
  if (!single) {
    for (int idx = tid; idx < W * Np; idx += blockDim.x) {
      int q = idx / W, j = idx - q * W;
      double val = E[(size_t)q * Np + c0 + j] * vl0[c0 + j];
      P[j * LDP + q] = (TP)(vnext[q] * val);
    }
  } else {
    // W divides 256: every thread keeps one column
    const int j = tid % W, part = tid / W, nparts = blockDim.x / W;
    double s2 = 0.0;
    for (int q = part; q < Np; q += nparts) {
      double val = E[(size_t)q * Np + c0 + j] * vl0[c0 + j];
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
  }
}

// ------------------------------------------------------------------------------ FP64

template <int RB, int CB>
__global__ __launch_bounds__(256) void seg_chain_f64(const double* __restrict__ E, FieldRef f,
                                                     int nb, int N, int Np, int Ltau, int n_s,
                                                     int m, int k0, int kc, double ldl,
                                                     double* __restrict__ S,
                                                     double* __restrict__ snorm) {
  constexpr int W = 16 * CB;
  extern __shared__ double lds[];
  const int LDP = Np + 2;
  double* P = lds;                      // [W][LDP] panel, k contiguous
  double* vbuf = P + W * LDP;           // [2][Np]
  double* red = vbuf + 2 * Np;          // [256] reduction scratch
  const int npan = Np / W;
  const int id = xcd_remap(blockIdx.x, nb * kc * npan);
  if (id < 0) return;
  const int pan = id % npan, k = k0 + (id / npan) % kc, b = id / (npan * kc);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const int NRB = Np >> 4, c0 = pan * W;
  const double* xb = field_of(f, b);
  const int l0 = k * n_s, len = min(n_s, Ltau - l0);
  double* Sout = S + ((size_t)b * m + k) * Np * Np;
  double* nout = snorm + ((size_t)b * m + k) * Np;

  fill_v(vbuf, xb, l0, N, Np, ldl);
  if (len > 1) fill_v(vbuf + Np, xb, l0 + 1, N, Np, ldl);
  __syncthreads();
  first_slice<double>(E, vbuf, vbuf + Np, P, LDP, W, c0, Np, len == 1, Sout, red, nout);
  if (len == 1) return;
  __syncthreads();

  for (int t = 1; t < len; ++t) {
    const bool last = (t == len - 1);
    double* vnext = vbuf + ((t + 1) & 1) * Np;   // v of slice l0+t+1 (unused when last)
    if (!last) fill_v(vnext, xb, l0 + t + 1, N, Np, ldl);

    dx4 acc[RB][CB];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[r][cb] = zero4d();

    double2 a0[RB], a1[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int rb = w + 4 * r;
      if (rb < NRB) {
        const double2* ep = (const double2*)(E + (size_t)(16 * rb + c) * Np + 4 * g);
        a0[r] = ep[0];
        a1[r] = ep[1];
      }
    }
    for (int kb = 0; kb < NRB; ++kb) {
      const int q0 = 16 * kb + 4 * g;
      double av[RB][4];
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        av[r][0] = a0[r].x; av[r][1] = a0[r].y; av[r][2] = a1[r].x; av[r][3] = a1[r].y;
      }
      if (kb + 1 < NRB) {   // prefetch the next k-block of E
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const int rb = w + 4 * r;
          if (rb < NRB) {
            const double2* ep = (const double2*)(E + (size_t)(16 * rb + c) * Np + q0 + 16);
            a0[r] = ep[0];
            a1[r] = ep[1];
          }
        }
      }
      double bv[CB][4];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const double2* pp = (const double2*)(P + (16 * cb + c) * LDP + q0);
        double2 b01 = pp[0], b23 = pp[1];
        bv[cb][0] = b01.x; bv[cb][1] = b01.y; bv[cb][2] = b23.x; bv[cb][3] = b23.y;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int r = 0; r < RB; ++r)
          if (w + 4 * r < NRB) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) acc[r][cb] = mfma64(av[r][s], bv[cb][s], acc[r][cb]);
          }
    }
    __syncthreads();   // every wave has finished reading the panel
    if (!last) {
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int rb = w + 4 * r;
        if (rb < NRB) {
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = 16 * rb + drow64(g, v);
              P[(16 * cb + c) * LDP + row] = vnext[row] * acc[r][cb][v];
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
              const int row = 16 * rb + drow64(g, v);
              const double val = acc[r][cb][v];
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

// ------------------------------------------------------------------------------ dispatch

template <int RB, int CB>
hipError_t run_f64(const double* E, FieldRef f, int nb, int N, int Np, int Ltau, int n_s, int m, int k0, int kc,
                   double ldl, double* S, double* sn, hipStream_t st) {
  constexpr int W = 16 * CB;
  const int count = nb * kc * (Np / W);
  const size_t lds = (size_t)(W * (Np + 2) + 2 * Np + 256) * sizeof(double);
  hipLaunchKernelGGL((seg_chain_f64<RB, CB>), dim3(xcd_grid(count)), dim3(256), lds, st, E, f,
                     nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, sn);
  return hipGetLastError();
}

template <int RB>
hipError_t pick_f64(int CB, const double* E, FieldRef f, int nb, int N, int Np, int Ltau,
                    int n_s, int m, int k0, int kc, double ldl, double* S, double* sn, hipStream_t st) {
  if (CB == 2) return run_f64<RB, 2>(E, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, sn, st);
  return run_f64<RB, 1>(E, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, sn, st);
}

// status[b] = 1 if any entry of item b's field is not finite, else 0 (one workgroup per
// item).  Every precision then reports such an item as non-finite, whatever its kernels
// make of the value (the int8 split, for one, cuts a NaN into finite digits).
__global__ __launch_bounds__(256) void field_status_k(FieldRef f, int nelem, int* __restrict__ status) {
  __shared__ int bad;
  const int b = blockIdx.x;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const double* xb = field_of(f, b);
  int mine = 0;
  for (int e = threadIdx.x; e < nelem; e += blockDim.x) mine |= !isfinite(xb[e]);
  if (mine) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0) status[b] = bad;
}

}  // namespace

hipError_t launch_field_status(FieldRef f, int nb, int nelem, int* status, hipStream_t st) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(field_status_k, dim3(nb), dim3(256), 0, st, f, nelem, status);
  return hipGetLastError();
}

hipError_t launch_seg_bf16(int pieces, const double* E64, const uint16_t* Ebf, FieldRef f,
                           int nb, int N, int Np, int Ltau, int n_s, int m, int k0, int kc, double ldl,
                           double* S, double* snorm, hipStream_t st);
hipError_t launch_seg_f32(int ecorr, int ch, const float* E32, const uint16_t* Elo,
                          const double* E64, FieldRef f, int nb, int N, int Np, int Ltau, int n_s,
                          int m, int k0, int kc, double ldl, double* S, double* snorm, hipStream_t st);

hipError_t launch_seg_i8(const int8_t* Eq, const double* Esc, const double* E64, FieldRef f,
                         int nb, int N, int Np, int Ltau, int n_s, int m, int k0, int kc,
                         double ldl, double* S, double* snorm, int trow, int seg_mode, int seg_cb,
                         hipStream_t st);

hipError_t launch_seg_chain(int prec, int acc_chunk, const double* E64, const float* E32,
                            const uint16_t* Elo, const uint16_t* Ebf, const int8_t* Eq,
                            const double* Esc, FieldRef f, int nb, int N, int Np, int Ltau,
                            int n_s, int m, int k0, int kc, double ldl, double* S, double* snorm,
                            int trow, hipStream_t st, int seg_mode, int seg_cb) {
  const int NRB = Np / 16;
  const int RB = (NRB + 3) / 4;
  if (RB < 1 || RB > 8) return hipErrorInvalidValue;
  if (prec == 0) {
    // panel width: 32 columns when it divides Np and the LDS panel stays small (seg_cb 1 or 2
    // forces 16 or 32 where 32 divides Np)
    int CB = (Np % 32 == 0 && Np <= 256) ? 2 : 1;
    if (seg_cb == 1) CB = 1;
    if (seg_cb == 2 && Np % 32 == 0) CB = 2;
    switch (RB) {
      case 1: return pick_f64<1>(CB, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
      case 2: return pick_f64<2>(CB, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
      case 3: return pick_f64<3>(CB, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
      case 4: return pick_f64<4>(CB, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
      case 5: return pick_f64<5>(CB, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
      case 6: return pick_f64<6>(CB, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
      case 7: return pick_f64<7>(CB, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
      default: return pick_f64<8>(CB, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
    }
  }
  if (prec == 1 || prec == 4)
    return launch_seg_f32(prec == 1, acc_chunk, E32, Elo, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S,
                          snorm, st);
  if (prec == 5)
    return launch_seg_i8(Eq, Esc, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, trow, seg_mode,
                         seg_cb, st);
  if (prec == 2 || prec == 3)
    return launch_seg_bf16(prec == 2 ? 2 : 3, E64, Ebf, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, st);
  return hipErrorInvalidValue;
}

}  // namespace slmc
