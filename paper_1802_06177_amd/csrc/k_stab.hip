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

constexpr int LDY = 18;   // row stride of 16-column LDS panels (16-byte aligned rows)

// Householder vector entry Y[r][i] of a panel whose rows/columns are local to the panel:
// unit diagonal, zero above, stored value below.
// Arithmetic masking instead of a select: a select lets the compiler sink the LDS read
// into a divergent branch (one wait per matrix-core instruction); v*m + d keeps the read
// unconditional (the address is always inside the panel, whose entries are finite).
__device__ __forceinline__ double yval(const double* Pn, int r, int i) {
  const double v = Pn[r * LDY + i];
  return fma(v, (double)(r > i), (double)(r == i));
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

// Workgroup of 8 waves per item.  Wave 0 owns the panels: it updates the next panel's
// column block with the current reflectors first and then factors it on its own (no
// workgroup barrier per column), while waves 1-7 apply the current reflectors to the
// remaining column blocks (look-ahead by one panel).  One barrier per panel step.
constexpr int QR_THREADS = 512;
constexpr int QR_UPD_WAVES = QR_THREADS / 64 - 1;

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Unblocked Householder factorization (LAPACK convention: beta = -sign(alpha)||x||,
// v_0 = 1, tau = (beta - alpha)/beta) of the K x 16 panel Pn held in LDS, by one wave.
// Row r is handled by lane r mod 64; column sums go through a transposing LDS buffer.
// Branch-free: columns left of the pivot are masked, not skipped.  Must stay inlined so
// that Pn, red and dsum are addressed as LDS.
__device__ __forceinline__ void panel_factor_wave(double* Pn, int K, double* red, double* dsum,
                                                  double* tau_out, double* beta_out, int lane) {
  for (int cc = 0; cc < 16; ++cc) {
    double pj[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) pj[j] = 0.0;
    for (int r = lane; r < K; r += 64) {
      const double2* row2 = (const double2*)(Pn + r * LDY);
      double rv[16];
#pragma unroll
      for (int q = 0; q < 8; ++q) { const double2 t = row2[q]; rv[2 * q] = t.x; rv[2 * q + 1] = t.y; }
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j) a += rv[j] * (double)(j == cc);
      a *= (double)(r > cc);
#pragma unroll
      for (int j = 0; j < 16; ++j) pj[j] += a * rv[j];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) *(double2*)(red + lane * LDY + 2 * q) = make_double2(pj[2 * q], pj[2 * q + 1]);
    wave_fence();
    {
      const int jj = lane & 15, qq = lane >> 4;
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) s += red[(qq * 16 + i) * LDY + jj];
      s += __shfl_xor(s, 16, 64);
      s += __shfl_xor(s, 32, 64);
      if (qq == 0) dsum[jj] = s;
    }
    wave_fence();
    double dv[16], rc[16];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double2 t = ((const double2*)dsum)[q]; dv[2 * q] = t.x; dv[2 * q + 1] = t.y;
      const double2 u = ((const double2*)(Pn + cc * LDY))[q]; rc[2 * q] = u.x; rc[2 * q + 1] = u.y;
    }
    double alpha = 0.0, ss = 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) { alpha += rc[j] * (double)(j == cc); ss += dv[j] * (double)(j == cc); }
    double tau, bt, sc;
    if (ss == 0.0) { tau = 0.0; bt = alpha; sc = 0.0; }
    else {
      bt = -copysign(sqrt(alpha * alpha + ss), alpha);
      tau = (bt - alpha) / bt;
      sc = 1.0 / (alpha - bt);
    }
    double wv[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) wv[j] = (rc[j] + sc * dv[j]) * (double)(j > cc);
    for (int r = lane; r < K; r += 64) {
      double2* row2 = (double2*)(Pn + r * LDY);
      double rv[16];
#pragma unroll
      for (int q = 0; q < 8; ++q) { const double2 t = row2[q]; rv[2 * q] = t.x; rv[2 * q + 1] = t.y; }
      double x = 0.0;
#pragma unroll
      for (int j = 0; j < 16; ++j) x += rv[j] * (double)(j == cc);
      const double below = (double)(r > cc), piv = (double)(r == cc);
      const double v = x * sc * below + piv;
      const double tv = tau * v * (below + piv);
      const double nx = below * v + piv * bt + (1.0 - below - piv) * x;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double upd = rv[j] - tv * wv[j];
        rv[j] = (j == cc) ? nx : upd;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) row2[q] = make_double2(rv[2 * q], rv[2 * q + 1]);
    }
    if (lane == 0) { tau_out[cc] = tau; beta_out[cc] = bt; }
    wave_fence();
  }
}

template <int NRBMAX>
__device__ __forceinline__ void panel_factor(double* Pn, int K, double* red, double* dsum,
                                             double* tau_out, double* beta_out, int lane) {
  panel_factor_wave(Pn, K, red, dsum, tau_out, beta_out, lane);
}

// T of the compact-WY form I - Y T Y^T of a factored K x 16 panel (one wave): Gram
// Y^T Y on the matrix cores, then T column by column, row j of T in lane j's registers.
__device__ __forceinline__ void build_T(const double* Pn, int K, const double* tau, double* gram, double* Tl,
                        double* Tg, int lane) {
  const int g = lane >> 4, c = lane & 15;
  dx4 ga[4] = {zero4d(), zero4d(), zero4d(), zero4d()};
  for (int rb = 0; rb < (K >> 4); ++rb) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double y = yval(Pn, 16 * rb + 4 * g + s, c);
      ga[s] = mfma64(y, y, ga[s]);
    }
  }
  const dx4 gacc = ga[0] + ga[1] + ga[2] + ga[3];
#pragma unroll
  for (int v = 0; v < 4; ++v) gram[drow64(g, v) * LDY + c] = gacc[v];
  wave_fence();
  if (lane < 16) {
    const int j = lane;
    double trow[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const double ti = tau[i];
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < i; ++l) {
        s += trow[l] * gram[l * LDY + i] * (double)(l >= j);
      }
      trow[i] = (j < i) ? -ti * s : ((j == i) ? ti : 0.0);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      Tl[j * LDY + i] = trow[i];
      Tg[j * 16 + i] = trow[i];
    }
  }
  wave_fence();
}

// Rows j0.. of column block cb (16 columns), lane (g, c) register v = row g + 4v of each
// 16-row block; from A through the column permutation on the first panel step.
template <int NRBMAX>
__device__ __forceinline__ void load_block(dx4 (&blk)[NRBMAX], int nrbK, int j0, int cb,
                                           bool from_a, const double* Ab, const int* iperm,
                                           const double* Q, int Np, int g, int c) {
#pragma unroll
  for (int rb = 0; rb < NRBMAX; ++rb) {
    if (rb < nrbK) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = j0 + 16 * rb + drow64(g, v);
        blk[rb][v] = from_a ? Ab[(size_t)row * Np + iperm[16 * cb + c]]
                            : Q[(size_t)row * Np + 16 * cb + c];
      }
    }
  }
}

// blk <- (I - Y T Y^T)^T blk for the panel (Y in Pn, T in Tl).
template <int NRBMAX>
__device__ __forceinline__ void apply_panel(dx4 (&blk)[NRBMAX], int nrbK, const double* Pn,
                                            const double* Tl, int g, int c) {
  // W = Y^T blk: four independent accumulators (one per k-step) keep the pipe full
  dx4 aw[4] = {zero4d(), zero4d(), zero4d(), zero4d()};
#pragma unroll
  for (int rb = 0; rb < NRBMAX; ++rb) {
    if (rb < nrbK) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        aw[s] = mfma64(yval(Pn, 16 * rb + drow64(g, s), c), blk[rb][s], aw[s]);
    }
  }
  const dx4 W = aw[0] + aw[1] + aw[2] + aw[3];
  double tv[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) tv[s] = Tl[drow64(g, s) * LDY + c];
  dx4 Wt = zero4d();
#pragma unroll
  for (int s = 0; s < 4; ++s) Wt = mfma64(tv[s], W[s], Wt);
  // blk -= Y W': consecutive instructions go to different row blocks
#pragma unroll
  for (int s = 0; s < 4; ++s) {
#pragma unroll
    for (int rb = 0; rb < NRBMAX; ++rb) {
      if (rb < nrbK) blk[rb] = mfma64(-yval(Pn, 16 * rb + c, drow64(g, s)), Wt[s], blk[rb]);
    }
  }
}

// One column block of the trailing update, self-contained (load, apply, store) so that
// no block-sized register array lives across the panel/update branches of the kernel.
// Rows j0 .. j0+15 go to Q; rows below go to Q, or to the next panel buffer Px when given.
template <int NRBMAX>
__device__ __forceinline__ void update_block(int nrbK, int j0, int cb, int from_a,
                                          const double* __restrict__ Ab,
                                          const int* __restrict__ iperm, double* __restrict__ Q,
                                          int Np, const double* Pc, const double* Tc, double* Px,
                                          int lane) {
  int c = lane & 15, g = lane >> 4;
  __asm__ volatile("" : "+v"(c), "+v"(g));
  dx4 blk[NRBMAX];
  load_block<NRBMAX>(blk, nrbK, j0, cb, from_a != 0, Ab, iperm, Q, Np, g, c);
  apply_panel<NRBMAX>(blk, nrbK, Pc, Tc, g, c);
#pragma unroll
  for (int rb = 0; rb < NRBMAX; ++rb) {
    if (rb < nrbK) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = 16 * rb + drow64(g, v);
        if (Px && rb >= 1) Px[(lr - 16) * LDY + c] = blk[rb][v];
        else Q[(size_t)(j0 + lr) * Np + 16 * cb + c] = blk[rb][v];
      }
    }
  }
}

template <int NRBMAX>
__global__ __launch_bounds__(QR_THREADS) void qr_k(const double* __restrict__ A, int64_t astride,
                                                   const double* __restrict__ norm2,
                                                   int64_t nstride, int nparts,
                                                   const double* __restrict__ logDp,
                                                   double* __restrict__ QRW,
                                                   double* __restrict__ Tb,
                                                   int* __restrict__ perm,
                                                   double* __restrict__ logD,
                                                   int* __restrict__ qsign,
                                                   int* __restrict__ status, int Np) {
  extern __shared__ double lds[];
  const int b = blockIdx.x;
  const int NRB = Np >> 4;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  double* Pn0 = lds;                        // [2][Np][LDY] panel buffers
  double* Tl0 = Pn0 + 2 * Np * LDY;         // [2][16][LDY]
  double* gram = Tl0 + 2 * 16 * LDY;        // [16][LDY]
  double* red = gram + 16 * LDY;            // [64][LDY]
  double* dsum = red + 64 * LDY;            // [16]
  double* key = dsum + 16;                  // [Np]
  double* beta = key + Np;                  // [Np]
  double* tauA = beta + Np;                 // [Np]
  double* nt = tauA + Np;                   // [8]
  int* iperm = (int*)(nt + 8);              // [Np]
  int* flag = iperm + Np;                   // [1]

  const double* Ab = A + (size_t)b * astride;
  double* Q = QRW + (size_t)b * Np * Np;
  double* Tg = Tb + (size_t)b * NRB * 256;
  if (tid == 0) flag[0] = 0;
  __syncthreads();

  // ---- pre-pivoting: order columns by log ||A e_j|| + log D_prev[j], descending
  for (int j = tid; j < Np; j += QR_THREADS) {
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += norm2[(size_t)b * nstride + (size_t)p * Np + j];
    double kj = 0.5 * log(s) + (logDp ? logDp[(size_t)b * Np + j] : 0.0);
    if (kj != kj) { kj = -INFINITY; flag[0] = 1; }
    key[j] = kj;
  }
  __syncthreads();
  for (int j = tid; j < Np; j += QR_THREADS) {
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
  for (int j = tid; j < Np; j += QR_THREADS) key[j] = logDp ? logDp[(size_t)b * Np + iperm[j]] : 0.0;
  for (int idx = tid; idx < Np * 16; idx += QR_THREADS) {
    const int r = idx >> 4, jj = idx & 15;
    Pn0[r * LDY + jj] = Ab[(size_t)r * Np + iperm[jj]];
  }
  __syncthreads();
  if (w == 0) {
    panel_factor<NRBMAX>(Pn0, Np, red, dsum, tauA, beta, lane);
    build_T(Pn0, Np, tauA, gram, Tl0, Tg, lane);
  }
  __syncthreads();

  for (int p = 0; p < NRB; ++p) {
    const int j0 = 16 * p, K = Np - j0, nrbK = NRB - p;
    double* Pc = Pn0 + (p & 1) * Np * LDY;
    double* Px = Pn0 + ((p + 1) & 1) * Np * LDY;
    const double* Tc = Tl0 + (p & 1) * 16 * LDY;
    double* Tx = Tl0 + ((p + 1) & 1) * 16 * LDY;
    {
      // wave 0 updates only the next panel's block (into Px); waves 1-7 the rest
      const int cb0 = (w == 0) ? p + 1 : p + 2 + (w - 1);
      const int cbs = (w == 0) ? NRB : QR_UPD_WAVES;
      for (int cb = cb0; cb < NRB; cb += cbs)
        update_block<NRBMAX>(nrbK, j0, cb, p == 0, Ab, iperm, Q, Np, Pc, Tc,
                             cb == p + 1 ? Px : nullptr, lane);
    }
    if (w == 0) {
      if (p + 1 < NRB) {
        wave_fence();
        panel_factor<NRBMAX>(Px, K - 16, red, dsum, tauA + j0 + 16, beta + j0 + 16, lane);
        build_T(Px, K - 16, tauA + j0 + 16, gram, Tx, Tg + (size_t)(p + 1) * 256, lane);
      }
    } else {
      // the factored panel p: R rows j0..j0+15 and Householder vectors below
      for (int idx = tid - 64; idx < K * 16; idx += QR_THREADS - 64) {
        const int r = idx >> 4, jj = idx & 15;
        Q[(size_t)(j0 + r) * Np + j0 + jj] = Pc[r * LDY + jj];
      }
    }
    __threadfence_block();
    __syncthreads();
  }

  // ---- outputs: log D, det Q, perm, and the V-update factor in the upper triangle
  int ntau = 0;
  for (int i = tid; i < Np; i += QR_THREADS) {
    logD[(size_t)b * Np + i] = log(fabs(beta[i])) + key[i];
    perm[(size_t)b * Np + i] = iperm[i];
    ntau += tauA[i] != 0.0;
  }
  for (int off = 32; off >= 1; off >>= 1) ntau += __shfl_xor(ntau, off, 64);
  if (lane == 0) nt[w] = (double)ntau;
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (int k = 0; k < QR_THREADS / 64; ++k) tot += (int)nt[k];
    qsign[b] = (tot & 1) ? -1 : 1;
    if (flag[0]) status[b] |= 1;
  }
  for (int idx = tid; idx < Np * Np; idx += QR_THREADS) {
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
  const size_t lds = (size_t)(2 * Np * LDY + 3 * 16 * LDY + 64 * LDY + 16 + 3 * Np + 8) *
                         sizeof(double) + (size_t)(Np + 2) * sizeof(int);
  hipLaunchKernelGGL(qr_k<NRBMAX>, dim3(nb), dim3(QR_THREADS), lds, st, A, astride, norm2, nstride, nparts,
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
