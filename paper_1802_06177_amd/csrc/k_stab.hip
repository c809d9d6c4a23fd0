// FP64 stabilization of the slice-product chain (UDV form).  The paper gives the chain
// M = I + B_L ... B_1 and G = M^{-1} (SM Eqs. S2, S3) but not how to keep the product
// representable; the standard remedy used here refactors the running product every n_s
// slices:  A_k = S_k Q_{k-1} (Q_{k-1} from the previous factorization), columns ordered
// by the norms of A_k diag(D_{k-1}) (pre-pivoting), A_k P_k = Q_k R_k (Householder),
// D_k = |diag R_k| D_{k-1}[P_k], V_k = D_k^{-1} R_k diag(D_{k-1}[P_k]) P_k^T V_{k-1}.
// D is carried as log D, so no scale of the product is ever formed (no overflow).
//
// Kernels:
//   wy_apply : A = B Q with Q in compact-WY blocks, row panels across all CUs.
//   qr       : blocked Householder QR, one workgroup per item; the trailing update keeps
//              each 16-column block in the registers of one wave and runs on FP64 MFMA.
//   vupd     : V_k = F P^T V_{k-1}, an upper-triangular column-panel GEMM.
#include "common.h"
#include "launch.h"

namespace slmc {

namespace {

constexpr int LDY = 17;   // row stride of 16-column LDS panels (bank spread)

// Householder vector entry Y[r][i] of a panel whose rows/columns are local to the panel:
// unit diagonal, zero above, stored value below.
__device__ __forceinline__ double yval(const double* Pn, int r, int i) {
  return r > i ? Pn[r * LDY + i] : (r == i ? 1.0 : 0.0);
}

// ------------------------------------------------------------------------------ wy_apply

__global__ __launch_bounds__(256) void wy_apply_k(const double* __restrict__ Bsrc,
                                                  int64_t bstride,
                                                  const double* __restrict__ QRW,
                                                  const double* __restrict__ Tb,
                                                  double* __restrict__ A,
                                                  double* __restrict__ npart,
                                                  int transpose_out, int nb, int Np) {
  extern __shared__ double lds[];
  const int NRB = Np >> 4;
  const int LDB = Np + 2;
  double* Bp = lds;                 // [16][LDB]
  double* Wp = Bp + 16 * LDB;       // [4][16][LDY]
  double* Wf = Wp + 4 * 16 * LDY;   // [16][LDY]
  const int id = xcd_remap(blockIdx.x, nb * NRB);
  if (id < 0) return;
  const int rp = id % NRB, b = id / NRB, r0 = 16 * rp;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const double* Y = QRW + (size_t)b * Np * Np;
  const double* T = Tb + (size_t)b * NRB * 256;

  if (Bsrc) {
    const double* src = Bsrc + (size_t)b * bstride + (size_t)r0 * Np;
    for (int idx = tid; idx < 16 * Np; idx += 256) {
      int row = idx / Np, col = idx - row * Np;
      Bp[row * LDB + col] = src[idx];
    }
  } else {
    for (int idx = tid; idx < 16 * Np; idx += 256) {
      int row = idx / Np, col = idx - row * Np;
      Bp[row * LDB + col] = (r0 + row == col) ? 1.0 : 0.0;
    }
  }
  __syncthreads();

  for (int p = 0; p < NRB; ++p) {
    const int j0 = 16 * p;
    // (a) partial W = B[:, j0:] Y_p, k-blocks split over the waves
    dx4 acc = zero4d();
    for (int kb = p + w; kb < NRB; kb += 4) {
      const int q = 16 * kb + 4 * g;
      const double2* bp = (const double2*)(Bp + c * LDB + q);
      double2 a01 = bp[0], a23 = bp[1];
      double av[4] = {a01.x, a01.y, a23.x, a23.y};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double y = Y[(size_t)(q + s) * Np + j0 + c];
        if (kb == p) { const int kk = 4 * g + s; y = kk > c ? y : (kk == c ? 1.0 : 0.0); }
        acc = mfma64(av[s], y, acc);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Wp[(w * 16 + drow64(g, v)) * LDY + c] = acc[v];
    __syncthreads();
    // (b) W' = W T_p (one wave)
    if (w == 0) {
      dx4 a2 = zero4d();
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = 4 * g + s;
        double wv = Wp[(0 * 16 + c) * LDY + kk] + Wp[(1 * 16 + c) * LDY + kk] +
                    Wp[(2 * 16 + c) * LDY + kk] + Wp[(3 * 16 + c) * LDY + kk];
        double tv = T[(size_t)p * 256 + kk * 16 + c];
        a2 = mfma64(wv, tv, a2);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) Wf[drow64(g, v) * LDY + c] = a2[v];
    }
    __syncthreads();
    // (c) B[:, j0:] -= W' Y_p^T, column blocks split over the waves
    for (int cb = p + w; cb < NRB; cb += 4) {
      const double* yr = Y + (size_t)(16 * cb + c) * Np + j0 + 4 * g;
      const double2 y01 = ((const double2*)yr)[0], y23 = ((const double2*)yr)[1];
      double yv[4] = {y01.x, y01.y, y23.x, y23.y};
      if (cb == p) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int kk = 4 * g + s;
          yv[s] = c > kk ? yv[s] : (c == kk ? 1.0 : 0.0);
        }
      }
      dx4 d = zero4d();
#pragma unroll
      for (int s = 0; s < 4; ++s) d = mfma64(Wf[c * LDY + 4 * g + s], yv[s], d);
#pragma unroll
      for (int v = 0; v < 4; ++v) Bp[drow64(g, v) * LDB + 16 * cb + c] -= d[v];
    }
    __syncthreads();
  }

  double* out = A + (size_t)b * Np * Np;
  if (!transpose_out) {
    for (int idx = tid; idx < 16 * Np; idx += 256) {
      int row = idx / Np, col = idx - row * Np;
      out[(size_t)(r0 + row) * Np + col] = Bp[row * LDB + col];
    }
  } else {
    for (int idx = tid; idx < 16 * Np; idx += 256) {
      int col = idx >> 4, row = idx & 15;
      out[(size_t)col * Np + r0 + row] = Bp[row * LDB + col];
    }
  }
  if (npart) {
    double* np_ = npart + ((size_t)b * NRB + rp) * Np;
    for (int col = tid; col < Np; col += 256) {
      double s = 0.0;
#pragma unroll
      for (int row = 0; row < 16; ++row) { double v = Bp[row * LDB + col]; s += v * v; }
      np_[col] = s;
    }
  }
}

// ------------------------------------------------------------------------------ QR

template <int NRBMAX>
__global__ __launch_bounds__(256) void qr_k(const double* __restrict__ A, int64_t astride,
                                            const double* __restrict__ norm2, int64_t nstride,
                                            int nparts,
                                            const double* __restrict__ logDp,
                                            double* __restrict__ QRW, double* __restrict__ Tb,
                                            int* __restrict__ perm, double* __restrict__ logD,
                                            int* __restrict__ qsign, int* __restrict__ status,
                                            int Np) {
  extern __shared__ double lds[];
  const int b = blockIdx.x;
  const int NRB = Np >> 4;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  double* Pn0 = lds;                        // [2][Np][LDY]
  double* key = Pn0 + 2 * Np * LDY;         // [Np]
  double* beta = key + Np;                  // [Np]
  double* tauA = beta + Np;                 // [Np]
  double* Tl = tauA + Np;                   // [16][LDY]
  double* gram = Tl + 16 * LDY;             // [16][LDY]
  double* wsh = gram + 16 * LDY;            // [16]
  double* rc = wsh + 16;                    // [16]
  double* scl = rc + 16;                    // [16]
  int* iperm = (int*)(scl + 16);            // [Np]
  int* flag = iperm + Np;                   // [1]

  const double* Ab = A + (size_t)b * astride;
  double* Q = QRW + (size_t)b * Np * Np;
  double* Tg = Tb + (size_t)b * NRB * 256;
  if (tid == 0) flag[0] = 0;
  __syncthreads();

  // ---- pre-pivoting: order columns by log ||A e_j|| + log D_prev[j], descending
  for (int j = tid; j < Np; j += 256) {
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += norm2[(size_t)b * nstride + (size_t)p * Np + j];
    double kj = 0.5 * log(s) + (logDp ? logDp[(size_t)b * Np + j] : 0.0);
    if (kj != kj) { kj = -INFINITY; flag[0] = 1; }
    key[j] = kj;
  }
  __syncthreads();
  for (int j = tid; j < Np; j += 256) {
    const double kj = key[j];
    int r = 0;
    for (int jj = 0; jj < Np; ++jj) {
      const double kk = key[jj];
      r += (kk > kj) || (kk == kj && jj < j);
    }
    iperm[r] = j;
  }
  __syncthreads();
  // key now holds log D_prev in pivot order (the V-update factor needs it)
  for (int j = tid; j < Np; j += 256) key[j] = logDp ? logDp[(size_t)b * Np + iperm[j]] : 0.0;
  // panel 0 from A (gathered columns)
  for (int idx = tid; idx < Np * 16; idx += 256) {
    int r = idx >> 4, jj = idx & 15;
    Pn0[r * LDY + jj] = Ab[(size_t)r * Np + iperm[jj]];
  }
  __syncthreads();

  for (int p = 0; p < NRB; ++p) {
    const int j0 = 16 * p, K = Np - j0, nrbK = NRB - p;
    double* Pn = Pn0 + (p & 1) * Np * LDY;
    double* Pnx = Pn0 + ((p + 1) & 1) * Np * LDY;

    // ---- panel factorization (unblocked Householder on K x 16 in LDS)
    for (int cc = 0; cc < 16; ++cc) {
      {
        const int j = tid >> 4, part = tid & 15;
        double dj = 0.0, ss = 0.0;
        if (j >= cc) {
#pragma unroll 4
          for (int r = cc + 1 + part; r < K; r += 16) {
            const double a = Pn[r * LDY + cc];
            dj += a * Pn[r * LDY + j];
            ss += a * a;
          }
        }
        dj = sum16(dj);
        ss = sum16(ss);
        if (j >= cc && part == 0) {
          const double alpha = Pn[cc * LDY + cc];
          double tau, bt, sc;
          if (ss == 0.0) { tau = 0.0; bt = alpha; sc = 0.0; }
          else {
            bt = -copysign(sqrt(alpha * alpha + ss), alpha);
            tau = (bt - alpha) / bt;
            sc = 1.0 / (alpha - bt);
          }
          if (j == cc) { rc[cc] = bt; scl[cc] = sc; tauA[j0 + cc] = tau; beta[j0 + cc] = bt; }
          else {
            const double wj = Pn[cc * LDY + j] + sc * dj;
            wsh[j] = wj;
            rc[j] = Pn[cc * LDY + j] - tau * wj;
          }
        }
      }
      __syncthreads();
      {
        const double sc = scl[cc], tau = tauA[j0 + cc];
        double wv[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) wv[j] = (j > cc) ? wsh[j] : 0.0;
        for (int r = cc + 1 + tid; r < K; r += 256) {
          double* row = Pn + r * LDY;
          const double vr = row[cc] * sc;
          row[cc] = vr;
          const double tv = tau * vr;
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if (j > cc) row[j] -= tv * wv[j];
        }
        if (tid == 0)
          for (int j = cc; j < 16; ++j) Pn[cc * LDY + j] = rc[j];
      }
      __syncthreads();
    }

    // ---- T of the compact-WY form: Q_p = I - Y T Y^T (wave 0)
    if (w == 0) {
      dx4 ga[4] = {zero4d(), zero4d(), zero4d(), zero4d()};
      for (int rb = 0; rb < nrbK; ++rb) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int kr = 16 * rb + 4 * g + s;
          const double y = yval(Pn, kr, c);
          ga[s] = mfma64(y, y, ga[s]);
        }
      }
      const dx4 gacc = ga[0] + ga[1] + ga[2] + ga[3];
#pragma unroll
      for (int v = 0; v < 4; ++v) gram[drow64(g, v) * LDY + c] = gacc[v];
      // lanes 0..15: row j of T (kept in registers), built column by column
      if (lane < 16) {
        const int j = lane;
        double trow[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const double ti = tauA[j0 + i];
          double s = 0.0;
#pragma unroll
          for (int l = 0; l < i; ++l)
            if (l >= j) s += trow[l] * gram[l * LDY + i];
          trow[i] = (j < i) ? -ti * s : ((j == i) ? ti : 0.0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          Tl[j * LDY + i] = trow[i];
          Tg[(size_t)p * 256 + j * 16 + i] = trow[i];
        }
      }
    }
    __syncthreads();

    // ---- trailing update: each wave owns whole 16-column blocks in registers
    for (int cb = p + 1 + w; cb < NRB; cb += 4) {
      // opaque copies of the lane coordinates: keeps the per-row addresses from being
      // hoisted out of this loop (they would pin hundreds of registers)
      int c = lane & 15, g = lane >> 4;
      __asm__ volatile("" : "+v"(c), "+v"(g));
      dx4 blk[NRBMAX];
#pragma unroll
      for (int rb = 0; rb < NRBMAX; ++rb) {
        if (rb < nrbK) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = j0 + 16 * rb + drow64(g, v);
            blk[rb][v] = (p == 0) ? Ab[(size_t)row * Np + iperm[16 * cb + c]]
                                  : Q[(size_t)row * Np + 16 * cb + c];
          }
        }
      }
      dx4 aw[4] = {zero4d(), zero4d(), zero4d(), zero4d()};
#pragma unroll
      for (int rb = 0; rb < NRBMAX; ++rb) {
        if (rb < nrbK) {
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int kr = 16 * rb + drow64(g, s);
            aw[rb & 3] = mfma64(yval(Pn, kr, c), blk[rb][s], aw[rb & 3]);
          }
        }
      }
      dx4 W = aw[0] + aw[1] + aw[2] + aw[3];
      dx4 Wt = zero4d();
#pragma unroll
      for (int s = 0; s < 4; ++s) Wt = mfma64(Tl[drow64(g, s) * LDY + c], W[s], Wt);
#pragma unroll
      for (int rb = 0; rb < NRBMAX; ++rb) {
        if (rb < nrbK) {
#pragma unroll
          for (int s = 0; s < 4; ++s)
            blk[rb] = mfma64(-yval(Pn, 16 * rb + c, drow64(g, s)), Wt[s], blk[rb]);
        }
      }
#pragma unroll
      for (int rb = 0; rb < NRBMAX; ++rb) {
        if (rb < nrbK) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int lr = 16 * rb + drow64(g, v);
            Q[(size_t)(j0 + lr) * Np + 16 * cb + c] = blk[rb][v];
            if (cb == p + 1 && rb >= 1) Pnx[(lr - 16) * LDY + c] = blk[rb][v];
          }
        }
      }
    }
    // ---- the factored panel: R rows j0..j0+15 and Householder vectors below
    for (int idx = tid; idx < K * 16; idx += 256) {
      int r = idx >> 4, jj = idx & 15;
      Q[(size_t)(j0 + r) * Np + j0 + jj] = Pn[r * LDY + jj];
    }
    __threadfence_block();
    __syncthreads();
  }

  // ---- outputs: log D, det Q, perm, and the V-update factor in the upper triangle
  int ntau = 0;
  for (int i = tid; i < Np; i += 256) {
    logD[(size_t)b * Np + i] = log(fabs(beta[i])) + key[i];
    perm[(size_t)b * Np + i] = iperm[i];
    ntau += tauA[i] != 0.0;
  }
  for (int off = 32; off >= 1; off >>= 1) ntau += __shfl_xor(ntau, off, 64);
  double* nt = wsh;   // reuse: per-wave counts
  __syncthreads();
  if (lane == 0) nt[w] = (double)ntau;
  __syncthreads();
  if (tid == 0) {
    const int tot = (int)(nt[0] + nt[1] + nt[2] + nt[3]);
    qsign[b] = (tot & 1) ? -1 : 1;
    if (flag[0]) status[b] |= 1;
  }
  for (int idx = tid; idx < Np * Np; idx += 256) {
    const int i = idx / Np, j = idx - i * Np;
    if (j >= i) {
      const double bi = beta[i];
      double fv;
      if (j == i) fv = bi < 0.0 ? -1.0 : 1.0;
      else fv = Q[(size_t)i * Np + j] / fabs(bi) * exp(key[j] - key[i]);
      Q[(size_t)i * Np + j] = fv;
    }
  }
}

// ------------------------------------------------------------------------------ vupd

template <int RB, int CB>
__global__ __launch_bounds__(256) void vupd_k(const double* __restrict__ QRW,
                                              const int* __restrict__ perm,
                                              const double* __restrict__ Vo,
                                              double* __restrict__ Vn, int nb, int Np) {
  constexpr int W = 16 * CB;
  extern __shared__ double lds[];
  const int LDP = Np + 2;
  double* P = lds;   // [W][LDP]
  const int npan = Np / W, NRB = Np >> 4;
  const int id = xcd_remap(blockIdx.x, nb * npan);
  if (id < 0) return;
  const int pan = id % npan, b = id / npan, c0 = pan * W;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const double* F = QRW + (size_t)b * Np * Np;
  const int* pb = perm + (size_t)b * Np;
  for (int idx = tid; idx < W * Np; idx += 256) {
    const int q = idx / W, j = idx - q * W;
    const int src = pb[q];
    P[j * LDP + q] = Vo ? Vo[(size_t)b * Np * Np + (size_t)src * Np + c0 + j]
                        : (src == c0 + j ? 1.0 : 0.0);
  }
  __syncthreads();
  dx4 acc[RB][CB];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[r][cb] = zero4d();
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int rb = w + 4 * r;
    if (rb >= NRB) continue;
    for (int kb = rb; kb < NRB; ++kb) {
      const int q0 = 16 * kb + 4 * g;
      const double* fr = F + (size_t)(16 * rb + c) * Np + q0;
      const double2 f01 = ((const double2*)fr)[0], f23 = ((const double2*)fr)[1];
      double av[4] = {f01.x, f01.y, f23.x, f23.y};
      if (kb == rb) {
#pragma unroll
        for (int s = 0; s < 4; ++s) av[s] = (4 * g + s >= c) ? av[s] : 0.0;
      }
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const double2* pp = (const double2*)(P + (16 * cb + c) * LDP + q0);
        const double2 b01 = pp[0], b23 = pp[1];
        double bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[r][cb] = mfma64(av[s], bv[s], acc[r][cb]);
      }
    }
  }
  double* out = Vn + (size_t)b * Np * Np;
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int rb = w + 4 * r;
    if (rb >= NRB) continue;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(size_t)(16 * rb + drow64(g, v)) * Np + c0 + 16 * cb + c] = acc[r][cb][v];
  }
}

template <int NRBMAX>
hipError_t run_qr(const double* A, int64_t astride, const double* norm2, int64_t nstride, int nparts,
                  const double* logDp, double* QRW, double* Tb, int* perm, double* logD,
                  int* qsign, int* status, int nb, int Np, hipStream_t st) {
  const size_t lds = (size_t)(2 * Np * LDY + 3 * Np + 2 * 16 * LDY + 48) * sizeof(double) +
                     (size_t)(Np + 2) * sizeof(int);
  hipLaunchKernelGGL(qr_k<NRBMAX>, dim3(nb), dim3(256), lds, st, A, astride, norm2, nstride, nparts,
                     logDp, QRW, Tb, perm, logD, qsign, status, Np);
  return hipGetLastError();
}

template <int RB>
hipError_t run_vupd(const double* QRW, const int* perm, const double* Vo, double* Vn, int nb,
                    int Np, hipStream_t st) {
  constexpr int CB = 2;
  if (Np % 32 == 0) {
    const size_t lds = (size_t)(16 * CB) * (Np + 2) * sizeof(double);
    hipLaunchKernelGGL((vupd_k<RB, CB>), dim3(xcd_grid(nb * (Np / 32))), dim3(256), lds, st, QRW,
                       perm, Vo, Vn, nb, Np);
  } else {
    const size_t lds = (size_t)16 * (Np + 2) * sizeof(double);
    hipLaunchKernelGGL((vupd_k<RB, 1>), dim3(xcd_grid(nb * (Np / 16))), dim3(256), lds, st, QRW,
                       perm, Vo, Vn, nb, Np);
  }
  return hipGetLastError();
}

__global__ void fill_i32_k(int* dst, int n, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = value;
}

}  // namespace

hipError_t launch_fill_i32(int* dst, int n, int value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_k, dim3((n + 255) / 256), dim3(256), 0, st, dst, n, value);
  return hipGetLastError();
}

hipError_t launch_wy_apply(const double* Bsrc, int64_t bstride, const double* QRW,
                           const double* Tb, double* A, double* npart, int transpose_out,
                           int nb, int Np, hipStream_t st) {
  const int NRB = Np / 16;
  const size_t lds = (size_t)(16 * (Np + 2) + 5 * 16 * LDY) * sizeof(double);
  hipLaunchKernelGGL(wy_apply_k, dim3(xcd_grid(nb * NRB)), dim3(256), lds, st, Bsrc, bstride,
                     QRW, Tb, A, npart, transpose_out, nb, Np);
  return hipGetLastError();
}

hipError_t launch_qr(const double* A, int64_t astride, const double* norm2, int64_t nstride,
                     int nparts, const double* logDp, double* QRW, double* Tb, int* perm,
                     double* logD, int* qsign, int* status, int nb, int Np, hipStream_t st) {
  const int NRB = Np / 16;
  if (NRB <= 4) return run_qr<4>(A, astride, norm2, nstride, nparts, logDp, QRW, Tb, perm, logD, qsign, status, nb, Np, st);
  if (NRB <= 8) return run_qr<8>(A, astride, norm2, nstride, nparts, logDp, QRW, Tb, perm, logD, qsign, status, nb, Np, st);
  if (NRB <= 16) return run_qr<16>(A, astride, norm2, nstride, nparts, logDp, QRW, Tb, perm, logD, qsign, status, nb, Np, st);
  if (NRB <= 25) return run_qr<25>(A, astride, norm2, nstride, nparts, logDp, QRW, Tb, perm, logD, qsign, status, nb, Np, st);
  if (NRB <= 32) return run_qr<32>(A, astride, norm2, nstride, nparts, logDp, QRW, Tb, perm, logD, qsign, status, nb, Np, st);
  return hipErrorInvalidValue;
}

hipError_t launch_vupd(const double* QRW, const int* perm, const double* Vo, double* Vn, int nb,
                       int Np, hipStream_t st) {
  const int NRB = Np / 16, RB = (NRB + 3) / 4;
  switch (RB) {
    case 1: return run_vupd<1>(QRW, perm, Vo, Vn, nb, Np, st);
    case 2: return run_vupd<2>(QRW, perm, Vo, Vn, nb, Np, st);
    case 3: return run_vupd<3>(QRW, perm, Vo, Vn, nb, Np, st);
    case 4: return run_vupd<4>(QRW, perm, Vo, Vn, nb, Np, st);
    case 5: return run_vupd<5>(QRW, perm, Vo, Vn, nb, Np, st);
    case 6: return run_vupd<6>(QRW, perm, Vo, Vn, nb, Np, st);
    case 7: return run_vupd<7>(QRW, perm, Vo, Vn, nb, Np, st);
    case 8: return run_vupd<8>(QRW, perm, Vo, Vn, nb, Np, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace slmc
