// Segment products (SM Eq. S2: B_l = e^{-dtau K} diag(e^{-dtau lam x_l})) on the int8
// matrix cores with exact integer accumulation.
//
// Every product E P is split into integer pieces: E is scaled per row by a power of two
// 2^{ea_i} (|E_ik 2^{-ea_i}| < 1/2) and cut into 5 slices of 7 bits each, rounded to
// nearest (|slice| <= 64), so E = 2^{ea} sum_p A_p 2^{-7p} up to 2^{-36} of the row
// maximum; the panel P is scaled per column by a power of two and rounded to nearest at
// 2^{-36} of that scale, then written as 5 signed 7-bit digits.  The products A_p B_q with
// p + q <= 6 (15 of the 25) are accumulated in int32 on v_mfma_i32_16x16x64_i8, exactly
// (|entries| <= 64 and K <= 448 keep every sum below 2^31), one accumulator per p + q,
// and recombined in FP64.  Relative to the row/column maxima the result carries an error
// of about 2^-36 per product, well below the FP32 matrix cores' rounding, and it is not
// biased (round-to-nearest slices).
//
// Workgroup (4 or 8 waves) = one (item, segment, 32- or 16-column panel), as in the FP64 kernel: the
// panel's int8 slices live in LDS, the E slices are the A operand, and the phonon factors
// of the next slice are applied when the FP64 result is recombined.
//
// E commutes with the lattice translations (nearest-neighbour hopping on a periodic
// lattice, SM Eq. S1), and the site order i = x + Lx y makes a translation by one lattice
// row an index shift by Lx: E[i + s][j + s] = E[i][j] (indices mod N) for every multiple
// s of Lx.  With N a multiple of 16 and trow = lcm(16, Lx), row block rb (16 rows) of E is
// base row block rb mod (trow/16), its columns rotated by 16 (rb - rb mod (trow/16)): the
// kernel keeps the slices of the first trow rows in LDS and reads every A operand there
// (tab mode), instead of streaming all of E from L2 once per slice product.  The host
// builds E from the displacement table, so the rotated rows are the same bytes and the
// result is bitwise that of the streaming mode.  The
// values are never stored in FP64 between slices: the new column scales come from a
// column-maximum pass over the accumulators, then the slices are cut from the same
// accumulators.
#include "common.h"
#include "launch.h"
#include "chain_util.h"

namespace slmc {

namespace {

typedef int ix4 __attribute__((ext_vector_type(4)));

constexpr int NSL = 5;          // slices per operand
constexpr int NDIAG = NSL;      // accumulators: p + q = 0 .. 4 (0-based slices)

__device__ __forceinline__ ix4 mfma_i8(ix4 a, ix4 b, ix4 c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

// FP64 value of one output element from its 5 diagonal sums (2^-14 .. 2^-42 weights).
// Each sum is below 2^24 in magnitude (K <= 448 terms of |a b| <= 2^12, at most 5 products
// per diagonal), so d0 128 + d1 and d2 128 + d3 are exact in int32.
__device__ __forceinline__ double recombine5(int d0, int d1, int d2, int d3, int d4) {
  const int hi = d0 * 128 + d1, mid = d2 * 128 + d3;
  return fma((double)hi, 0x1p-21, fma((double)mid, 0x1p-35, (double)d4 * 0x1p-42));
}

// 2^{e+1} with |m| < 2^e (frexp convention), so |value / scale| < 1/2; 1 for zero.
__device__ __forceinline__ double pow2_above(double m) {
  if (!(m > 0.0)) return 1.0;
  int e;
  (void)frexp(m, &e);
  return ldexp(1.0, e + 1);
}

// The 5 signed 7-bit digits (most significant first) of Y = RNE(v sc), |v sc| < 2^34,
// for 4 values: byte i of out[p] is digit p of value i, and Y = sum_p d_p 128^{4-p}.
// Adding 1.5 2^52 leaves Y in the low mantissa bits; adding C = 64 sum_p 128^p turns the
// signed digits into unsigned 7-bit fields of Y + C (0 <= Y + C < 2^36), which are cut by
// shifts and masks.  The top field gets 8 bits (digit range [-64, 64]); the others lose
// their offset byte-parallel: for u in [0, 127], u - 64 as a byte is w | (w & 0x40) << 1
// with w = u ^ 0x40.
__host__ __device__ __forceinline__ void slice4x5(const double (&v)[4], double sc,
                                                  uint32_t (&out)[NSL]) {
  uint32_t u[NSL] = {0u, 0u, 0u, 0u, 0u};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double t = fma(v[i], sc, 0x1.8p52);
    const uint64_t z = __builtin_bit_cast(uint64_t, t) + 0x408102040ull;
    u[0] |= (((uint32_t)(z >> 28) + 192u) & 255u) << (8 * i);
#pragma unroll
    for (int p = 1; p < NSL; ++p) u[p] |= ((uint32_t)(z >> (28 - 7 * p)) & 127u) << (8 * i);
  }
  out[0] = u[0];
#pragma unroll
  for (int p = 1; p < NSL; ++p) {
    const uint32_t w = u[p] ^ 0x40404040u;
    out[p] = w | ((w & 0x40404040u) << 1);
  }
}

// NW waves per workgroup, two waves per SIMD: 8 (one workgroup per CU) or 4 (two
// workgroups per CU, so that one slices its panel while the other is on the matrix cores)
template <int NW, int RB, int CB, bool TAB, bool REG>
__global__ __launch_bounds__(64 * NW, 8 / NW) void seg_chain_i8(const int8_t* __restrict__ Eq,
                                                    const double* __restrict__ Esc,
                                                    const double* __restrict__ E64, FieldRef f,
                                                    int nb, int N, int Np, int Npk, int Ltau,
                                                    int n_s, int m, int k0, int kc, double ldl,
                                                    double* __restrict__ S,
                                                    double* __restrict__ snorm, int trow,
                                                    int LDE) {
  constexpr int W = 16 * CB;
  extern __shared__ double lds[];
  constexpr int KBB = NSL * W * 64;             // bytes of one 64-row k block of slices
  double* vbuf = lds;                           // [2][Np]
  double* escs = vbuf + 2 * Np;                 // [Np] E's row scales
  double* red = escs + Np;                      // [NW][W]
  int8_t* Bsl = (int8_t*)(red + NW * W);  // [Npk/64][NSL][W][64]
  int8_t* E0 = Bsl + (Npk >> 6) * KBB;          // tab mode: [NSL][trow][LDE]
  const int npan = Np / W;
  const int id = xcd_remap(blockIdx.x, nb * kc * npan);
  if (id < 0) return;
  const int pan = id % npan, k = k0 + (id / npan) % kc, b = id / (npan * kc);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const int NRB = Np >> 4, c0 = pan * W;
  const bool full = NW * RB <= NRB;   // every wave's row blocks exist
  const double* xb = field_of(f, b);
  const int l0 = k * n_s, len = min(n_s, Ltau - l0);
  double* Sout = S + ((size_t)b * m + k) * Np * Np;
  double* nout = snorm + ((size_t)b * m + k) * Np;

  // v of the first two slices: both loads of a thread in flight before either is used
  for (int q = tid; q < Np; q += 64 * NW) {
    const double x0 = q < N ? xb[(size_t)l0 * N + q] : 0.0;
    const double x1 = (q < N && len > 1) ? xb[(size_t)(l0 + 1) * N + q] : 0.0;
    escs[q] = Esc[q];
    vbuf[q] = q < N ? exp(-ldl * x0) : 1.0;
    if (len > 1) vbuf[Np + q] = q < N ? exp(-ldl * x1) : 1.0;
  }
  // zero the k padding of the slices once (rows Np .. Npk-1 are never written later)
  for (int idx = tid; idx < NSL * W * (Npk - Np); idx += 64 * NW) {
    const int pc = idx / (Npk - Np), r = Np + idx - pc * (Npk - Np);
    Bsl[(r >> 6) * KBB + pc * 64 + (r & 63)] = 0;
  }
  if (TAB && len > 1) {
    // the slices of E's first trow rows, 16-byte chunks from the [row][k block][slice][64]
    // layout into [slice][row][LDE]
    const int nkb = Npk >> 6, nch = trow * nkb * NSL * 4;
    // 8 chunks per thread in flight, then stored
    for (int base = 0; base < nch; base += 8 * 64 * NW) {
      ix4 tmp[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + tid + u * 64 * NW;
        const int q4 = idx & 3, t = idx >> 2, p = t % NSL, kb = (t / NSL) % nkb, row = t / (NSL * nkb);
        if (idx < nch) tmp[u] = *(const ix4*)(Eq + (((size_t)row * nkb + kb) * NSL + p) * 64 + 16 * q4);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int idx = base + tid + u * 64 * NW;
        const int q4 = idx & 3, t = idx >> 2, p = t % NSL, kb = (t / NSL) % nkb, row = t / (NSL * nkb);
        if (idx < nch) *(ix4*)(E0 + (p * trow + row) * LDE + 64 * kb + 16 * q4) = tmp[u];
      }
    }
  }
  __syncthreads();

  if (len == 1) {
    // S_k = E diag(v_l0) on this panel's columns, and its column norms
    double s2[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) s2[cb] = 0.0;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int rb = w + NW * r;
      if (rb < NRB) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = 16 * rb + drow32(g, i), col = c0 + 16 * cb + c;
            const double val = E64[(size_t)row * Np + col] * vbuf[col];
            Sout[(size_t)row * Np + col] = val;
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
    if (tid < W) {
      double t2 = 0.0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) t2 += red[ww * W + tid];
      nout[c0 + tid] = t2;
    }
    return;
  }

  ix4 acc[RB][CB][NDIAG];
  double vals[RB][CB][4];   // the panel about to be sliced, in the accumulator layout
  double fcur[CB];          // column scales 2^f of the panel in Bsl (this lane's columns)

  // Cut the panel in vals into slices: column maxima over the waves, new scales, then
  // the bytes.  Ends with a barrier (slices ready).
  auto make_slices = [&]() {
    double mx[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) mx[cb] = 0.0;
#pragma unroll
    for (int r = 0; r < RB; ++r)
      if (w + NW * r < NRB) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) mx[cb] = fmax(mx[cb], fabs(vals[r][cb][i]));
      }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      double v = mx[cb];
      v = fmax(v, __shfl_xor(v, 16, 64));
      v = fmax(v, __shfl_xor(v, 32, 64));
      if (g == 0) red[w * W + 16 * cb + c] = v;
    }
    __syncthreads();
    double inv[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int col = 16 * cb + c;
      double v = 0.0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) v = fmax(v, red[ww * W + col]);
      fcur[cb] = pow2_above(v);
      inv[cb] = 0x1p35 / fcur[cb];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int rb = w + NW * r;
      if (rb < NRB) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
          uint32_t packed[NSL];
          slice4x5(vals[r][cb], inv[cb], packed);
#pragma unroll
          for (int p = 0; p < NSL; ++p)
            *(uint32_t*)(Bsl + (rb >> 2) * KBB + (p * W + 16 * cb + c) * 64 + 16 * (rb & 3) + 4 * g) = packed[p];
        }
      }
    }
    __syncthreads();
  };

  // first panel: v_{l0+1} E diag(v_l0); when every wave's row blocks exist the loads run
  // without a per-element branch, so all of them are in flight together
  if (full) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * (w + NW * r) + drow32(g, i), col = c0 + 16 * cb + c;
          vals[r][cb][i] = vbuf[Np + row] * E64[(size_t)row * Np + col] * vbuf[col];
        }
  } else {
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * (w + NW * r) + drow32(g, i), col = c0 + 16 * cb + c;
          vals[r][cb][i] = (w + NW * r < NRB) ? vbuf[Np + row] * E64[(size_t)row * Np + col] * vbuf[col] : 0.0;
        }
  }
  make_slices();

  const int nkb = Npk >> 6;
  // REG (base rows = one row block, 4 waves, Np a multiple of 64): the A operand of row
  // block w + 4 r and k block kb is chunk (4 (kb - r) + g - w) mod (Np / 16) of the base
  // rows, so a wave needs only RB distinct operands (by (kb - r) mod RB): loaded into
  // registers once, and the product loop reads only the panel's slices from LDS
  ix4 eA[REG ? RB : 1][NSL];
  if constexpr (REG) {
    const int Nc = Np >> 4;
#pragma unroll
    for (int e = 0; e < RB; ++e) {
      const int src = (4 * e + g - w + Nc) % Nc;
#pragma unroll
      for (int p = 0; p < NSL; ++p) eA[e][p] = *(const ix4*)(E0 + (p * 16 + c) * LDE + 16 * src);
    }
  }
  for (int t = 1; t < len; ++t) {
    const bool last = (t == len - 1);
    double* vnext = vbuf + ((t + 1) & 1) * Np;   // v of slice l0+t+1 (unused when last)
    // the field of slice l0+t+1 is loaded here and turned into vnext after the products,
    // so the load's latency hides behind them
    double xn[2] = {0.0, 0.0};
    if (!last) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int q = tid + 64 * NW * j;
        if (q < N) xn[j] = xb[(size_t)(l0 + t + 1) * N + q];
      }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
#pragma unroll
        for (int d = 0; d < NDIAG; ++d) acc[r][cb][d] = ix4{0, 0, 0, 0};
    if constexpr (REG) {
#pragma unroll
      for (int kb = 0; kb < RB; ++kb) {
        const int8_t* bk = Bsl + kb * KBB + 64 * c + 16 * g;
        ix4 bq[CB][NSL];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int q = 0; q < NSL; ++q) bq[cb][q] = *(const ix4*)(bk + (q * W + 16 * cb) * 64);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const int e = (kb - r + RB) % RB;
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int p = 0; p < NSL; ++p)
#pragma unroll
              for (int q = 0; q + p < NSL; ++q)
                acc[r][cb][p + q] = mfma_i8(eA[e][p], bq[cb][q], acc[r][cb][p + q]);
        }
      }
    } else if constexpr (TAB) {
      // A operands from the LDS copy of the base rows; the panel's slices stay in registers
      // across the row blocks
      const int Nc = Np >> 4, nbase = trow >> 4;
      for (int kb = 0; kb < nkb; ++kb) {
        const int8_t* bk = Bsl + kb * KBB + 64 * c + 16 * g;
        ix4 bq[CB][NSL];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int q = 0; q < NSL; ++q) bq[cb][q] = *(const ix4*)(bk + (q * W + 16 * cb) * 64);
        // this lane's 16-column chunk of k; chunks past N meet zero panel rows, any
        // in-range chunk serves them
        const int kap = min(4 * kb + g, Nc - 1);
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const int rb = w + NW * r;
          if (rb < NRB) {
            const int rb0 = rb % nbase, d = rb - rb0;
            const int src = kap - d < 0 ? kap - d + Nc : kap - d;
            const int8_t* ep = E0 + (16 * rb0 + c) * LDE + 16 * src;
            ix4 ap[NSL];
#pragma unroll
            for (int p = 0; p < NSL; ++p) ap[p] = *(const ix4*)(ep + p * trow * LDE);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
              for (int p = 0; p < NSL; ++p)
#pragma unroll
                for (int q = 0; q + p < NSL; ++q)
                  acc[r][cb][p + q] = mfma_i8(ap[p], bq[cb][q], acc[r][cb][p + q]);
          }
        }
      }
    } else {
      for (int kb = 0; kb < nkb; ++kb) {
        const int8_t* bk = Bsl + kb * KBB + 64 * c + 16 * g;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const int rb = w + NW * r;
          if (rb < NRB) {
            // E slices laid out [row][k block][slice][64 bytes]: one address per row block
            const int8_t* ep = Eq + ((size_t)(16 * rb + c) * nkb + kb) * (NSL * 64) + 16 * g;
            ix4 ap[NSL];
#pragma unroll
            for (int p = 0; p < NSL; ++p) ap[p] = *(const ix4*)(ep + 64 * p);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
              // the panel's slices are re-read from LDS per row block (registers are the
              // scarcer resource)
              ix4 bq[NSL];
#pragma unroll
              for (int q = 0; q < NSL; ++q) bq[q] = *(const ix4*)(bk + (q * W + 16 * cb) * 64);
#pragma unroll
              for (int p = 0; p < NSL; ++p)
#pragma unroll
                for (int q = 0; q + p < NSL; ++q)
                  acc[r][cb][p + q] = mfma_i8(ap[p], bq[q], acc[r][cb][p + q]);
            }
          }
        }
      }
    }
    if (!last) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int q = tid + 64 * NW * j;
        if (q < Np) vnext[q] = q < N ? exp(-ldl * xn[j]) : 1.0;
      }
    }
    __syncthreads();   // every wave is done with the slices; vnext is filled
    if (!last) {
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = 16 * (w + NW * r) + drow32(g, i);
            const double x = recombine5(acc[r][cb][0][i], acc[r][cb][1][i], acc[r][cb][2][i],
                                        acc[r][cb][3][i], acc[r][cb][4][i]);
            // branch-free when every row block exists (the LDS reads then overlap)
            if (full) vals[r][cb][i] = vnext[row] * (escs[row] * fcur[cb] * x);
            else vals[r][cb][i] = (w + NW * r < NRB) ? vnext[row] * (escs[row] * fcur[cb] * x) : 0.0;
          }
      make_slices();
    } else {
      double s2[CB];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) s2[cb] = 0.0;
      // opaque copies of the lane coordinates: the output addresses are formed here, not
      // hoisted to the start of the kernel (where they would be spilled)
      int go = g, co = c;
      __asm__ volatile("" : "+v"(go), "+v"(co));
      double* so = Sout + c0 + co;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int rb = w + NW * r;
        if (rb < NRB) {
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int row = 16 * rb + drow32(go, i);
              const double x = recombine5(acc[r][cb][0][i], acc[r][cb][1][i], acc[r][cb][2][i],
                                          acc[r][cb][3][i], acc[r][cb][4][i]);
              const double val = escs[row] * fcur[cb] * x;
              so[(size_t)row * Np + 16 * cb] = val;
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
      if (tid < W) {
        double t2 = 0.0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) t2 += red[ww * W + tid];
        nout[c0 + tid] = t2;
      }
    }
  }
}

template <int NW, int RB, int CB, bool TAB, bool REG>
hipError_t run_i8(const int8_t* Eq, const double* Esc, const double* E64, FieldRef f, int nb,
                  int N, int Np, int Ltau, int n_s, int m, int k0, int kc, double ldl, double* S,
                  double* sn, int trow, int LDE, hipStream_t st) {
  constexpr int W = 16 * CB;
  const int Npk = (Np + 63) / 64 * 64;
  const int count = nb * kc * (Np / W);
  const size_t lds = (size_t)(3 * Np + NW * W) * sizeof(double) + (size_t)NSL * W * Npk +
                     (TAB ? (size_t)NSL * trow * LDE : 0);
  hipLaunchKernelGGL((seg_chain_i8<NW, RB, CB, TAB, REG>), dim3(xcd_grid(count)), dim3(64 * NW), lds, st, Eq,
                     Esc, E64, f, nb, N, Np, Npk, Ltau, n_s, m, k0, kc, ldl, S, sn, trow, LDE);
  return hipGetLastError();
}

template <int NW, int RB, int CB>
hipError_t pick_tab(const int8_t* Eq, const double* Esc, const double* E64, FieldRef f, int nb,
                    int N, int Np, int Ltau, int n_s, int m, int k0, int kc, double ldl, double* S,
                    double* sn, int trow, int LDE, bool allow_reg, hipStream_t st) {
  // registers for the A operands when the base rows are one row block and the 4 waves'
  // row blocks cover Np in whole k blocks
  if (allow_reg && NW == 4 && trow == 16 && Np % 64 == 0 && Np / 64 == RB)
    return run_i8<NW, RB, CB, true, NW == 4>(Eq, Esc, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, sn, trow, LDE, st);
  if (trow > 0)
    return run_i8<NW, RB, CB, true, false>(Eq, Esc, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, sn, trow, LDE, st);
  return run_i8<NW, RB, CB, false, false>(Eq, Esc, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, sn, 0, 0, st);
}

}  // namespace

hipError_t launch_seg_i8(const int8_t* Eq, const double* Esc, const double* E64, FieldRef f,
                         int nb, int N, int Np, int Ltau, int n_s, int m, int k0, int kc,
                         double ldl, double* S, double* snorm, int trow, int seg_mode, int seg_cb,
                         hipStream_t st) {
  const int NRB = Np / 16;
  // tab mode when E repeats every trow rows (a multiple of 16, N unpadded) and the base
  // rows' slices fit in 64 KB of LDS; LDE = 16 mod 256 keeps the 16-row reads conflict free
  // (seg_mode 2: E streamed from memory; 1: no register operands)
  const int LDE = (N + 255) / 256 * 256 + 16;
  if (seg_mode == 2 ||
      !(trow > 0 && trow % 16 == 0 && trow <= N && N == Np && (size_t)NSL * trow * LDE <= 65536))
    trow = 0;
  const bool allow_reg = seg_mode == 0;
#define SEG_I8_ARGS Eq, Esc, E64, f, nb, N, Np, Ltau, n_s, m, k0, kc, ldl, S, snorm, trow, LDE, allow_reg, st
  if (NRB <= 16) {
    // 4 waves, up to 4 row blocks each; 32-column panels while RB <= 2 (seg_cb 1: 16 columns)
    const int RB = (NRB + 3) / 4;
    const bool cb2 = Np % 32 == 0 && RB <= 2 && seg_cb != 1;
    switch (RB) {
      case 1: return cb2 ? pick_tab<4, 1, 2>(SEG_I8_ARGS) : pick_tab<4, 1, 1>(SEG_I8_ARGS);
      case 2: return cb2 ? pick_tab<4, 2, 2>(SEG_I8_ARGS) : pick_tab<4, 2, 1>(SEG_I8_ARGS);
      case 3: return pick_tab<4, 3, 1>(SEG_I8_ARGS);
      default: return pick_tab<4, 4, 1>(SEG_I8_ARGS);
    }
  }
  // 8 waves, 3 or 4 row blocks each (Np <= 448 gives NRB <= 28)
  const int RB = (NRB + 7) / 8;
  if (RB == 3) return pick_tab<8, 3, 1>(SEG_I8_ARGS);
  if (RB == 4) return pick_tab<8, 4, 1>(SEG_I8_ARGS);
#undef SEG_I8_ARGS
  return hipErrorInvalidValue;
}

}  // namespace slmc
