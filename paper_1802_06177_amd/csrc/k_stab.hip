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
//   vupd     : V_k = F P^T V_{k-1}, an upper-triangular GEMM (register strips for Np <= 256).
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

// Workgroup of 8 waves per item.  Each 16-column panel is factored by waves 0-3 (one per
// SIMD), every thread holding one or two rows of the panel in registers; the column
// steps exchange their 16 sums through a wave reduce-scatter and an LDS-counter sync of
// those 4 waves.  Meanwhile waves 4-7 apply the previous panel to the trailing column
// blocks on the matrix cores (look-ahead by one panel); one workgroup barrier per panel.
constexpr int QR_THREADS = 512;
constexpr int QR_WAVES = QR_THREADS / 64;

template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// (x, y) <- lanes 32-63 of x exchanged with lanes 0-31 of y (v_permlane32_swap), and
// the same for odd/even 16-lane rows (v_permlane16_swap).
__device__ __forceinline__ void swap32(double& x, double& y) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
  x = __hiloint2double(hi[0], lo[0]);
  y = __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ void swap16(double& x, double& y) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
  x = __hiloint2double(hi[0], lo[0]);
  y = __hiloint2double(hi[1], lo[1]);
}

// Reduce-scatter of 16 values over the 64 lanes of a wave: on return lanes 4v .. 4v+3
// hold the wave total of value v.  Each halving stage pairs lanes that differ in one bit
// (5 and 4 by the permlane swaps, 3 and 2 by the row mirrors), the last two add quads.
__device__ __forceinline__ double reduce_scatter16(const double (&v)[16], int lane) {
  double a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double x = v[i], y = v[i + 8];
    swap32(x, y);
    a[i] = x + y;            // value i + 8 * bit5
  }
  double b[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double x = a[i], y = a[i + 4];
    swap16(x, y);
    b[i] = x + y;            // value ... + 4 * bit4
  }
  const bool h3 = (lane & 8) != 0, h2 = (lane & 4) != 0;
  double c[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double send = h3 ? b[i] : b[i + 2];
    const double keep = h3 ? b[i + 2] : b[i];
    c[i] = keep + dpp64<0x140>(send);    // row_mirror: partner 15 - l
  }
  const double send = h2 ? c[0] : c[1];
  double d = (h2 ? c[1] : c[0]) + dpp64<0x141>(send);   // row_half_mirror: partner 7 - l
  d += dpp64<0xB1>(d);                                 // quad_perm [1,0,3,2]
  d += dpp64<0x4E>(d);                                 // quad_perm [2,3,0,1]
  return d;
}

// Lane l's value of v, for a lane index that is the same in every lane.
__device__ __forceinline__ double readlane64(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Householder factorization (LAPACK convention: beta = -sign(alpha)||x||, v_0 = 1,
// tau = (beta - alpha)/beta) of the K x 16 panel held in registers by the first 4 waves
// (one per SIMD): thread t < 256 owns local rows t (row0) and t + 256 (row1, only when
// TWO); rows >= K are zero.  Column step cc needs P_j = sum_{r > cc} row_r[cc] row_r[j]
// for all 16 j: j = cc gives ||x||^2 below the pivot, j > cc the reflector's product with
// the remaining columns, and j < cc (the earlier Householder vectors) gives Y^T v, from
// which column cc of the compact-WY factor T follows (T_cc,cc = tau,
// T_l,cc = -tau sum_m T_l,m (Y^T v)_m); lane l & 15 keeps row l & 15 of T in trow and
// threads 0-15 store it to Tl.  The sums go through a wave reduce-scatter and one sync of
// the 4 panel waves per column (panel_sync); red [2][4][16] and prow [2][16] are
// double-buffered by column parity.
constexpr int QR_PANEL_WAVES = 4;
constexpr int QR_SPIN_LIMIT = 1 << 16;   // about 2 ms of s_sleep(1) polls
// Np from 272 to 400: the trailing update by pairs of waves, each with half of a column
// block in registers (update_block_pair); above, the chunked two-pass update of one wave
#define QR_PAIR_UPDATE(NRBMAX) ((NRBMAX) == 25)

// Arrive-and-wait among the 4 panel waves through a monotonically increasing LDS counter
// (the other waves keep working meanwhile).  The release on arrival orders the wave's
// earlier LDS writes before the count, the acquire on the wait orders later reads after
// it.  The wait is bounded: past the spin limit it sets *timeout and goes on, so every
// wave always reaches the end of the kernel.
__device__ __forceinline__ void panel_sync(int* cnt, int& epoch, int lane, int* timeout) {
  ++epoch;
  if (lane == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  const int target = QR_PANEL_WAVES * epoch;
  int spins = 0;
  while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
    // the first polls back to back (the other panel waves are usually a few hundred
    // cycles behind), then with a sleep between polls
    if (spins >= 16) __builtin_amdgcn_s_sleep(1);
    if (++spins > QR_SPIN_LIMIT) {
      *timeout = 1;
      break;
    }
  }
}

// 1 / d from the hardware reciprocal and two Newton steps (within an ulp; the Householder
// scalars need no correctly rounded quotient, and this is on the per-column critical path)
__device__ __forceinline__ double rcp_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  r = fma(fma(-d, r, 1.0), r, r);
  return r;
}

template <bool TWO>
__device__ __forceinline__ void panel_factor_all(double (&row0)[16], double (&row1)[16],
                                                 double (&trow)[16], int t, int K, double* red,
                                                 double* prow, double* Tl,
                                                 double* tau_out, double* beta_out, int* cnt,
                                                 int& epoch, int* timeout) {
  const int lane = t & 63, w = t >> 6, tl = lane & 15;
#pragma unroll
  for (int j = 0; j < 16; ++j) trow[j] = 0.0;
#pragma unroll
  for (int cc = 0; cc < 16; ++cc) {
    double* rb = red + (cc & 1) * QR_PANEL_WAVES * 16;
    double* pb = prow + (cc & 1) * 16;
    {
      const double am0 = row0[cc] * (double)(t > cc && t < K);
      const double am1 = TWO ? row1[cc] * (double)(t + 256 < K) : 0.0;
      double pj[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) pj[j] = TWO ? am0 * row0[j] + am1 * row1[j] : am0 * row0[j];
      if (t == cc) {
#pragma unroll
        for (int q = 0; q < 8; ++q) ((double2*)pb)[q] = make_double2(row0[2 * q], row0[2 * q + 1]);
      }
      const double ws = reduce_scatter16(pj, lane);
      if ((lane & 3) == 0) rb[w * 16 + (lane >> 2)] = ws;
    }
    panel_sync(cnt, epoch, lane, timeout);
    {
      // column totals: lane l adds the 4 wave partials of column l & 15 and reads the
      // pivot row's entry of that column; the wave-uniform scalars below are taken from
      // lane cc, and g_j from lane j, with readlane (no LDS round trip)
      double tot = 0.0;
#pragma unroll
      for (int ww = 0; ww < QR_PANEL_WAVES; ++ww) tot += rb[ww * 16 + tl];
      const double rcl = pb[tl];
      const double alpha = readlane64(rcl, cc), ss = readlane64(tot, cc);
      double tau, bt, sc;
      if (ss == 0.0) {
        tau = 0.0; bt = alpha; sc = 0.0;
      } else {
        bt = -copysign(sqrt(alpha * alpha + ss), alpha);
        tau = (bt - alpha) * rcp_nr(bt);
        sc = rcp_nr(alpha - bt);
      }
      // g_j = v^T row_j: Y^T v for j < cc, the reflector's product with column j for j > cc
      const double gl = rcl + sc * tot;
      double gv[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) gv[j] = readlane64(gl, j);
      double tp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int m = 0; m < cc; ++m) tp[m & 3] += trow[m] * gv[m];
      const double tl_cc = (tp[0] + tp[1]) + (tp[2] + tp[3]);
      trow[cc] = (tl < cc) ? -tau * tl_cc : (tl == cc ? tau : 0.0);
      // stored right away (a store cannot be postponed past the next sync, so the T
      // recurrence is not sunk to the end of the panel with all its operands kept live)
      if (t < 16) Tl[t * LDY + cc] = trow[cc];
      // apply the reflector to this thread's rows
      {
        const double a = row0[cc];
        const double v = (t > cc && t < K) ? sc * a : (t == cc ? 1.0 : 0.0);
        const double tv = tau * v;
#pragma unroll
        for (int j = cc + 1; j < 16; ++j) row0[j] -= tv * gv[j];
        row0[cc] = (t > cc) ? sc * a : (t == cc ? bt : a);
      }
      if (TWO) {
        const double a = row1[cc];
        const double tv = tau * sc * a;
#pragma unroll
        for (int j = cc + 1; j < 16; ++j) row1[j] -= tv * gv[j];
        row1[cc] = sc * a;
      }
      if (t == 0) { tau_out[cc] = tau; beta_out[cc] = bt; }
    }
  }
}

// Rows j0.. of one 16-column block, lane (g, c) register v = row g + 4v of each 16-row
// block; src points at row j0 of this lane's column (rows at stride Np).
template <int NRBMAX>
__device__ __forceinline__ void load_block(dx4 (&blk)[NRBMAX], int nrbK, const double* src,
                                           int Np, int g) {
#pragma unroll
  for (int rb = 0; rb < NRBMAX; ++rb) {
    if (rb < nrbK) {
#pragma unroll
      for (int v = 0; v < 4; ++v) blk[rb][v] = src[(16 * rb + drow64(g, v)) * Np];
    }
  }
}

// blk <- (I - Y T Y^T)^T blk for the panel (Y in Pn, T in Tl).  Only the top row block of
// Y needs the unit-lower masking; the Y values of the next row block (pair) are read from
// LDS while the current one's products issue, and the update runs over pairs of row
// blocks so that consecutive matrix-core instructions go to independent accumulators.
// Every accumulator sees its products in the same order as a plain loop would.
template <int NRBMAX>
__device__ __forceinline__ void apply_panel(dx4 (&blk)[NRBMAX], int nrbK, const double* Pn,
                                            const double* Tl, int g, int c) {
  // W = Y^T blk: four independent accumulators (one per k-step) keep the pipe full
  dx4 aw[4] = {zero4d(), zero4d(), zero4d(), zero4d()};
  double yn[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) yn[s] = yval(Pn, drow64(g, s), c);
#pragma unroll
  for (int rb = 0; rb < NRBMAX; ++rb) {
    if (rb < nrbK) {
      double yc[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) yc[s] = yn[s];
      if (rb + 1 < nrbK) {
#pragma unroll
        for (int s = 0; s < 4; ++s) yn[s] = Pn[(16 * (rb + 1) + drow64(g, s)) * LDY + c];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) aw[s] = mfma64(yc[s], blk[rb][s], aw[s]);
    }
  }
  const dx4 W = aw[0] + aw[1] + aw[2] + aw[3];
  double tv[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) tv[s] = Tl[drow64(g, s) * LDY + c];
  dx4 Wt = zero4d();
#pragma unroll
  for (int s = 0; s < 4; ++s) Wt = mfma64(tv[s], W[s], Wt);
  // blk -= Y W', row blocks in pairs: for each k-step s the two blocks' products in turn
  double qa[4], qb[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    qa[s] = -yval(Pn, c, drow64(g, s));
    qb[s] = 0.0;
    if (1 < nrbK) qb[s] = -Pn[(16 + c) * LDY + drow64(g, s)];
  }
#pragma unroll
  for (int rb = 0; rb < NRBMAX; rb += 2) {
    if (rb < nrbK) {
      double ca[4], cb[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) { ca[s] = qa[s]; cb[s] = qb[s]; }
      if (rb + 2 < nrbK) {
#pragma unroll
        for (int s = 0; s < 4; ++s) qa[s] = -Pn[(16 * (rb + 2) + c) * LDY + drow64(g, s)];
        if (rb + 3 < nrbK) {
#pragma unroll
          for (int s = 0; s < 4; ++s) qb[s] = -Pn[(16 * (rb + 3) + c) * LDY + drow64(g, s)];
        }
      }
      if (rb + 1 < nrbK) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          blk[rb] = mfma64(ca[s], Wt[s], blk[rb]);
          if (rb + 1 < NRBMAX) blk[rb + 1] = mfma64(cb[s], Wt[s], blk[rb + 1]);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) blk[rb] = mfma64(ca[s], Wt[s], blk[rb]);
      }
    }
  }
}

// One column block of the trailing update, self-contained (load, apply, store) so that
// no block-sized register array lives across the panel/update phases of the kernel.
// The block comes from A through the column order on the first panel step (from_a) and
// from Q after; rows j0 .. j0+15 go back to Q, rows below to Q or, for the next panel, to
// the LDS buffer Px.
template <int NRBMAX>
__device__ __forceinline__ void update_block(int nrbK, int j0, int cb, bool from_a,
                                             const double* __restrict__ Ab,
                                             const int* __restrict__ iperm, double* __restrict__ Q,
                                             int Np, const double* Pc, const double* Tc, double* Px,
                                             int lane) {
  int c = lane & 15, g = lane >> 4;
  __asm__ volatile("" : "+v"(c), "+v"(g));
  const int col = 16 * cb + c;
  const double* src = from_a ? Ab + iperm[col] : Q + (size_t)j0 * Np + col;
  double* dst = Q + (size_t)j0 * Np + col;
  dx4 blk[NRBMAX];
  load_block<NRBMAX>(blk, nrbK, src, Np, g);
  apply_panel<NRBMAX>(blk, nrbK, Pc, Tc, g, c);
  if (Px) {
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[drow64(g, v) * Np] = blk[0][v];
#pragma unroll
    for (int rb = 1; rb < NRBMAX; ++rb) {
      if (rb < nrbK) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Px[(16 * (rb - 1) + drow64(g, v)) * LDY + c] = blk[rb][v];
      }
    }
  } else {
#pragma unroll
    for (int rb = 0; rb < NRBMAX; ++rb) {
      if (rb < nrbK) {
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[(16 * rb + drow64(g, v)) * Np] = blk[rb][v];
      }
    }
  }
}

// update_block for large Np: the column block goes through registers CH row blocks at a
// time (all of it would not fit beside the other role's registers): one pass accumulates
// W = Y^T blk over all row blocks, a second reloads each chunk, applies the update and
// stores it.  The MFMA accumulation order is that of apply_panel, so the result is the same.
template <int CH>
__device__ __forceinline__ void update_block_chunked(int nrbK, int j0, int cb, bool from_a,
                                                     const double* __restrict__ Ab,
                                                     const int* __restrict__ iperm,
                                                     double* __restrict__ Q, int Np,
                                                     const double* Pc, const double* Tc, int lane) {
  int c = lane & 15, g = lane >> 4;
  __asm__ volatile("" : "+v"(c), "+v"(g));
  const int col = 16 * cb + c;
  const double* src = from_a ? Ab + iperm[col] : Q + (size_t)j0 * Np + col;
  double* dst = Q + (size_t)j0 * Np + col;
  dx4 aw[4] = {zero4d(), zero4d(), zero4d(), zero4d()};
  for (int r0 = 0; r0 < nrbK; r0 += CH) {
    dx4 blk[CH];
#pragma unroll
    for (int rb = 0; rb < CH; ++rb) {
      if (r0 + rb < nrbK) {
#pragma unroll
        for (int v = 0; v < 4; ++v) blk[rb][v] = src[(16 * (r0 + rb) + drow64(g, v)) * Np];
      }
    }
    double yn[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) yn[s] = yval(Pc, 16 * r0 + drow64(g, s), c);
#pragma unroll
    for (int rb = 0; rb < CH; ++rb) {
      if (r0 + rb < nrbK) {
        double yc[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) yc[s] = yn[s];
        if (rb + 1 < CH && r0 + rb + 1 < nrbK) {
#pragma unroll
          for (int s = 0; s < 4; ++s) yn[s] = Pc[(16 * (r0 + rb + 1) + drow64(g, s)) * LDY + c];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) aw[s] = mfma64(yc[s], blk[rb][s], aw[s]);
      }
    }
  }
  const dx4 W = aw[0] + aw[1] + aw[2] + aw[3];
  double tv[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) tv[s] = Tc[drow64(g, s) * LDY + c];
  dx4 Wt = zero4d();
#pragma unroll
  for (int s = 0; s < 4; ++s) Wt = mfma64(tv[s], W[s], Wt);
  for (int r0 = 0; r0 < nrbK; r0 += CH) {
    dx4 blk[CH];
#pragma unroll
    for (int rb = 0; rb < CH; ++rb) {
      if (r0 + rb < nrbK) {
#pragma unroll
        for (int v = 0; v < 4; ++v) blk[rb][v] = src[(16 * (r0 + rb) + drow64(g, v)) * Np];
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
#pragma unroll
      for (int rb = 0; rb < CH; ++rb) {
        if (r0 + rb < nrbK) blk[rb] = mfma64(-yval(Pc, 16 * (r0 + rb) + c, drow64(g, s)), Wt[s], blk[rb]);
      }
    }
#pragma unroll
    for (int rb = 0; rb < CH; ++rb) {
      if (r0 + rb < nrbK) {
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[(16 * (r0 + rb) + drow64(g, v)) * Np] = blk[rb][v];
      }
    }
  }
}

// Arrive-and-wait between the two waves of an update pair, as panel_sync does for the
// panel waves (bounded the same way).
__device__ __forceinline__ void pair_sync(int* cnt, int& epoch, int lane, int* timeout) {
  ++epoch;
  if (lane == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  const int target = 2 * epoch;
  int spins = 0;
  while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
    if (spins >= 16) __builtin_amdgcn_s_sleep(1);
    if (++spins > QR_SPIN_LIMIT) {
      *timeout = 1;
      break;
    }
  }
}

// update_block for large Np by a pair of waves: wave h holds one half of the column
// block's row blocks (the first ceil(nrbK / 2), or the rest) in registers, loaded once;
// the two partial products Y^T blk meet in LDS (wb: [2 halves][64 lanes][4]) behind a pair
// sync, both waves form the same W = W_0 + W_1, and each applies the update to its own
// half and stores it.  The caller alternates wb between two buffers from one column block
// to the next: a wave's arrival at the sync waits for its own earlier LDS reads, so the
// partner cannot overwrite a buffer that is still being read.
template <int HB>
__device__ __forceinline__ void update_block_pair(int nrbK, int j0, int cb, bool from_a,
                                                  const double* __restrict__ Ab,
                                                  const int* __restrict__ iperm,
                                                  double* __restrict__ Q, int Np, const double* Pc,
                                                  const double* Tc, double* wb, int h, int* pcnt,
                                                  int& pepoch, int lane, int* timeout) {
  int c = lane & 15, g = lane >> 4;
  __asm__ volatile("" : "+v"(c), "+v"(g));
  const int col = 16 * cb + c;
  const int n0 = (nrbK + 1) >> 1;
  const int r0 = h ? n0 : 0, nr = h ? nrbK - n0 : n0;
  const double* src = (from_a ? Ab + iperm[col] : Q + (size_t)j0 * Np + col) + (size_t)16 * r0 * Np;
  double* dst = Q + (size_t)(j0 + 16 * r0) * Np + col;
  const double* Ph = Pc + 16 * r0 * LDY;
  dx4 blk[HB];
#pragma unroll
  for (int rb = 0; rb < HB; ++rb) {
    if (rb < nr) {
#pragma unroll
      for (int v = 0; v < 4; ++v) blk[rb][v] = src[(16 * rb + drow64(g, v)) * Np];
    }
  }
  dx4 aw[4] = {zero4d(), zero4d(), zero4d(), zero4d()};
  double yn[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) yn[s] = yval(Pc, 16 * r0 + drow64(g, s), c);
#pragma unroll
  for (int rb = 0; rb < HB; ++rb) {
    if (rb < nr) {
      double yc[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) yc[s] = yn[s];
      // the next row block's Y values (unconditional, the row block clamped into the half:
      // below the diagonal block, so no masking)
      const int rn = min(rb + 1, nr - 1);
#pragma unroll
      for (int s = 0; s < 4; ++s) yn[s] = Ph[(16 * rn + drow64(g, s)) * LDY + c];
#pragma unroll
      for (int s = 0; s < 4; ++s) aw[s] = mfma64(yc[s], blk[rb][s], aw[s]);
    }
  }
  // every load of the half has been consumed by now; saying so spares the stores and the
  // products below the compiler's per-instruction waits on loads it cannot see completed
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  *(dx4*)(wb + (h * 64 + lane) * 4) = aw[0] + aw[1] + aw[2] + aw[3];
  pair_sync(pcnt, pepoch, lane, timeout);
  const dx4 W = *(const dx4*)(wb + lane * 4) + *(const dx4*)(wb + (64 + lane) * 4);
  double tv[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) tv[s] = Tc[drow64(g, s) * LDY + c];
  dx4 Wt = zero4d();
#pragma unroll
  for (int s = 0; s < 4; ++s) Wt = mfma64(tv[s], W[s], Wt);
  // blk -= Y W', row blocks in pairs (consecutive products go to independent accumulators);
  // the next pair's Y values are read while the current pair's products issue
  // (unconditionally, row blocks clamped into the half); every accumulator still sees
  // s = 0 .. 3 in order
  double qa[4], qb[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    qa[s] = -yval(Pc, 16 * r0 + c, drow64(g, s));
    qb[s] = -yval(Pc, 16 * (r0 + min(1, nr - 1)) + c, drow64(g, s));
  }
#pragma unroll
  for (int rb = 0; rb < HB; rb += 2) {
    if (rb < nr) {
      double ca[4], cb[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) { ca[s] = qa[s]; cb[s] = qb[s]; }
      const int ra = min(rb + 2, nr - 1), rbb = min(rb + 3, nr - 1);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        qa[s] = -yval(Pc, 16 * (r0 + ra) + c, drow64(g, s));
        qb[s] = -yval(Pc, 16 * (r0 + rbb) + c, drow64(g, s));
      }
      if (rb + 1 < nr) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          blk[rb] = mfma64(ca[s], Wt[s], blk[rb]);
          if (rb + 1 < HB) blk[rb + 1] = mfma64(cb[s], Wt[s], blk[rb + 1]);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) blk[rb] = mfma64(ca[s], Wt[s], blk[rb]);
      }
    }
  }
#pragma unroll
  for (int rb = 0; rb < HB; ++rb) {
    if (rb < nr) {
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[(16 * rb + drow64(g, v)) * Np] = blk[rb][v];
    }
  }
}

// Rows of a column block owned by panel wave w in the split update below (row blocks w,
// w+4, .. of the rows j0 ..), loaded ahead of use: from A through the column order on the
// first step (from_a), from Q after.
template <int RBQ>
__device__ __forceinline__ void prefetch_block(dx4 (&blk)[RBQ], int nrbK, int j0, int cb,
                                               bool from_a, const double* __restrict__ Ab,
                                               const int* __restrict__ iperm,
                                               const double* __restrict__ Q, int Np, int w,
                                               int lane) {
  const int c = lane & 15, g = lane >> 4, col = 16 * cb + c;
  const double* src = from_a ? Ab + iperm[col] : Q + (size_t)j0 * Np + col;
#pragma unroll
  for (int r = 0; r < RBQ; ++r) {
    const int rb = w + QR_PANEL_WAVES * r;
    if (rb < nrbK) {
#pragma unroll
      for (int v = 0; v < 4; ++v) blk[r][v] = src[(16 * rb + drow64(g, v)) * Np];
    }
  }
}

// The column block of the next panel, updated with the current panel by the 4 panel waves
// together: wave w holds the row blocks w, w+4, .. (prefetched); the partial products
// Y^T blk meet in LDS (wpart, [4][64 lanes][4]) behind one panel sync, then every wave
// finishes its rows.  Rows j0 .. j0+15 go to Q, the rows below to the next panel buffer Px.
template <int RBQ>
__device__ __forceinline__ void apply_block_split(dx4 (&blk)[RBQ], int nrbK, int j0, int cb,
                                                  double* __restrict__ Q, int Np, const double* Pc,
                                                  const double* Tc, double* Px, double* wpart,
                                                  int w, int lane, int* cnt, int& epoch,
                                                  int* timeout) {
  int c = lane & 15, g = lane >> 4;
  __asm__ volatile("" : "+v"(c), "+v"(g));
  double* dst = Q + (size_t)j0 * Np + 16 * cb + c;
  // (the Y values of the next row block are read from LDS while the current one's products
  // issue; same products, same order per accumulator)
  dx4 aw[4] = {zero4d(), zero4d(), zero4d(), zero4d()};
  double yn[4] = {0.0, 0.0, 0.0, 0.0};
  if (w < nrbK) {
#pragma unroll
    for (int s = 0; s < 4; ++s) yn[s] = yval(Pc, 16 * w + drow64(g, s), c);
  }
#pragma unroll
  for (int r = 0; r < RBQ; ++r) {
    const int rb = w + QR_PANEL_WAVES * r;
    if (rb < nrbK) {
      double yc[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) yc[s] = yn[s];
      if (rb + QR_PANEL_WAVES < nrbK) {
#pragma unroll
        for (int s = 0; s < 4; ++s) yn[s] = Pc[(16 * (rb + QR_PANEL_WAVES) + drow64(g, s)) * LDY + c];
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) aw[s] = mfma64(yc[s], blk[r][s], aw[s]);
    }
  }
  const dx4 Wp = aw[0] + aw[1] + aw[2] + aw[3];
  *(dx4*)(wpart + (w * 64 + lane) * 4) = Wp;
  panel_sync(cnt, epoch, lane, timeout);
  dx4 W = zero4d();
#pragma unroll
  for (int ww = 0; ww < QR_PANEL_WAVES; ++ww) W += *(const dx4*)(wpart + (ww * 64 + lane) * 4);
  double tv[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) tv[s] = Tc[drow64(g, s) * LDY + c];
  dx4 Wt = zero4d();
#pragma unroll
  for (int s = 0; s < 4; ++s) Wt = mfma64(tv[s], W[s], Wt);
  // blk -= Y W': this wave's row blocks, their Y values read up front
  double ya[RBQ][4];
#pragma unroll
  for (int r = 0; r < RBQ; ++r) {
    const int rb = w + QR_PANEL_WAVES * r;
    if (rb < nrbK) {
#pragma unroll
      for (int s = 0; s < 4; ++s) ya[r][s] = -yval(Pc, 16 * rb + c, drow64(g, s));
    }
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
#pragma unroll
    for (int r = 0; r < RBQ; ++r) {
      const int rb = w + QR_PANEL_WAVES * r;
      if (rb < nrbK) blk[r] = mfma64(ya[r][s], Wt[s], blk[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < RBQ; ++r) {
    const int rb = w + QR_PANEL_WAVES * r;
    if (rb < nrbK) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (rb == 0) dst[drow64(g, v) * Np] = blk[r][v];
        else Px[(16 * (rb - 1) + drow64(g, v)) * LDY + c] = blk[r][v];
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
                                                   double* __restrict__ keyo,
                                                   double* __restrict__ logD,
                                                   int* __restrict__ qsign,
                                                   int* __restrict__ status, int Np) {
  extern __shared__ double lds[];
  const int b = blockIdx.x;
  const int NRB = Np >> 4;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  double* Pn0 = lds;                        // [2][Np][LDY] Y of panel p / panel p+1
  double* Tl0 = Pn0 + 2 * Np * LDY;         // [2][16][LDY] T of panel p / panel p+1
  double* red = Tl0 + 2 * 16 * LDY;         // [2][4][16]
  double* prow = red + 2 * QR_PANEL_WAVES * 16;   // [2][16]
  double* wpart = prow + 32;                // [4][64][4] partial Y^T blk
  double* key = wpart + QR_PANEL_WAVES * 256;     // [Np]
  double* beta = key + Np;                  // [Np]
  double* tauA = beta + Np;                 // [Np]
  double* nt = tauA + Np;                   // [8]
  // [2 pairs][2 buffers][2 halves][64][4] partial Y^T blk of the update pairs (pair update only)
  double* wp2 = nt + 8;
  int* iperm = (int*)(wp2 + (QR_PAIR_UPDATE(NRBMAX) ? 2048 : 0));   // [Np]
  int* flag = iperm + Np;                   // [2]: non-finite input, sync timeout
  int* cnt = flag + 2;                      // [1] panel-wave sync counter
  int* blkrdy = cnt + 1;                    // [1] last step whose first trailing block is stored
  int* pcnt = blkrdy + 1;                   // [2] update-pair sync counters
  int* blkcnt = pcnt + 2;                   // [1] pair update: halves of first trailing blocks stored

  const double* Ab = A + (size_t)b * astride;
  double* Q = QRW + (size_t)b * Np * Np;
  double* Tg = Tb + (size_t)b * NRB * 256;
  if (tid == 0) { flag[0] = 0; flag[1] = 0; cnt[0] = 0; blkrdy[0] = -1; pcnt[0] = 0; pcnt[1] = 0; blkcnt[0] = 0; }
  __syncthreads();

  // ---- pre-pivoting: order columns by log ||A e_j|| + log D_prev[j], descending
  for (int j = tid; j < Np; j += QR_THREADS) {
    double s = 0.0;
#pragma unroll 4
    for (int p = 0; p < nparts; ++p) s += norm2[(size_t)b * nstride + (size_t)p * Np + j];
    double kj = 0.5 * log(s) + (logDp ? logDp[(size_t)b * Np + j] : 0.0);
    if (kj != kj) { kj = -INFINITY; flag[0] = 1; }
    key[j] = kj;
  }
  __syncthreads();
  for (int j = tid; j < Np; j += QR_THREADS) {
    const double kj = key[j];
    int r = 0;
#pragma unroll 8
    for (int jj = 0; jj < Np; ++jj) {
      const double kk = key[jj];
      r += (kk > kj) || (kk == kj && jj < j);
    }
    iperm[r] = j;
  }
  __syncthreads();
  // key now holds log D_prev in pivot order (the V-update factor needs it)
  for (int j = tid; j < Np; j += QR_THREADS) key[j] = logDp ? logDp[(size_t)b * Np + iperm[j]] : 0.0;

  // Panel waves (0-3) factor panel 0, then for every step p update column block p+1 with
  // panel p (split by row blocks) and factor it as panel p+1; waves 4-7 meanwhile apply
  // panel p to the column blocks p+2 ..  One workgroup barrier per step publishes panel p+1.
  constexpr bool TWO = NRBMAX > 16;
  constexpr int RBQ = (NRBMAX + QR_PANEL_WAVES - 1) / QR_PANEL_WAVES;
  // wave-uniform role (readfirstlane makes the branch on it a scalar one)
  const bool panel_wave = __builtin_amdgcn_readfirstlane(w) < QR_PANEL_WAVES;
  int epoch = 0;
  double row0[16], row1[16], trow[16];
  dx4 nblk[RBQ];   // this panel wave's rows of the next column block (prefetched)
  if (panel_wave) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      row0[j] = (tid < Np) ? Ab[(size_t)tid * Np + iperm[j]] : 0.0;
      row1[j] = (TWO && tid + 256 < Np) ? Ab[(size_t)(tid + 256) * Np + iperm[j]] : 0.0;
    }
  }
  // The two roles run separate loops (same number of workgroup barriers), so that the
  // registers of one role's data do not constrain the other's.
  if (panel_wave) {
    for (int p = -1; p < NRB - 1; ++p) {
      // this step factors panel q = p + 1; panel p (if any) is published in buffer p & 1
      const int q = p + 1, jq = 16 * q, Kq = Np - jq;
      double* Yq = Pn0 + (q & 1) * Np * LDY;
      double* Tq = Tl0 + (q & 1) * 16 * LDY;
      if (p >= 0) {
        // column block q (prefetched at the end of the previous step), updated with panel
        // p, lands in Yq (rows below its R part)
        apply_block_split<RBQ>(nblk, NRB - p, 16 * p, q, Q, Np, Pn0 + (p & 1) * Np * LDY,
                               Tl0 + (p & 1) * 16 * LDY, Yq, wpart, w, lane, cnt, epoch, flag + 1);
        panel_sync(cnt, epoch, lane, flag + 1);
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const double2 u = (tid < Kq) ? ((const double2*)(Yq + tid * LDY))[h] : make_double2(0.0, 0.0);
          row0[2 * h] = u.x;
          row0[2 * h + 1] = u.y;
          const double2 u1 = (TWO && tid + 256 < Kq) ? ((const double2*)(Yq + (tid + 256) * LDY))[h]
                                                     : make_double2(0.0, 0.0);
          row1[2 * h] = u1.x;
          row1[2 * h + 1] = u1.y;
        }
        // (no sync needed before the factored panel overwrites Yq: every panel wave uses its
        // rows in the first column step, before that step's sync, and a wave stores the
        // panel only after the last column's sync)
      }
      panel_factor_all<TWO>(row0, row1, trow, tid, Kq, red, prow, Tq, tauA + jq, beta + jq,
                            cnt, epoch, flag + 1);
      // the factored panel: R rows and Householder vectors to Q, Y to LDS; T (already in
      // LDS) to Q's T blocks
      if (tid < Kq) {
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const double2 u = make_double2(row0[2 * h], row0[2 * h + 1]);
          ((double2*)(Yq + tid * LDY))[h] = u;
          ((double2*)(Q + (size_t)(jq + tid) * Np + jq))[h] = u;
        }
      }
      if (TWO && tid + 256 < Kq) {
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const double2 u = make_double2(row1[2 * h], row1[2 * h + 1]);
          ((double2*)(Yq + (tid + 256) * LDY))[h] = u;
          ((double2*)(Q + (size_t)(jq + tid + 256) * Np + jq))[h] = u;
        }
      }
      if (tid < 16) {
#pragma unroll
        for (int j = 0; j < 16; ++j) Tg[(size_t)q * 256 + tid * 16 + j] = trow[j];
      }
      // prefetch the rows of column block q+1 for the next step: from A on the first step,
      // else from Q once wave 4 has stored it (its first block this step)
      if (q + 1 < NRB) {
        if (p >= 0) {
          // (pair update: both halves of block p + 2 of every step 0 .. p stored)
          int* const rdy = QR_PAIR_UPDATE(NRBMAX) ? blkcnt : blkrdy;
          const int want = QR_PAIR_UPDATE(NRBMAX) ? 2 * (p + 1) : p;
          int spins = 0;
          while (__hip_atomic_load(rdy, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < want) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > QR_SPIN_LIMIT) { flag[1] = 1; break; }
          }
        }
        prefetch_block<RBQ>(nblk, NRB - q, jq, q + 1, p < 0, Ab, iperm, Q, Np, w, lane);
      }
      __threadfence_block();
      __syncthreads();
    }
  } else if constexpr (QR_PAIR_UPDATE(NRBMAX)) {
    // two pairs of update waves, each pair one column block at a time (pair 0 starts with
    // block q+1, which the panel waves prefetch for the next step)
    // (wave-uniform: the half's row-block bounds become scalar branches)
    const int uw = __builtin_amdgcn_readfirstlane(w) - QR_PANEL_WAVES, pr = uw >> 1, h = uw & 1;
    int pepoch = 0, pbuf = 0;
    for (int p = -1; p < NRB - 1; ++p) {
      const int q = p + 1;
      if (p >= 0) {
        for (int cb = q + 1 + pr; cb < NRB; cb += 2) {
          update_block_pair<(NRBMAX + 1) / 2>(NRB - p, 16 * p, cb, p == 0, Ab, iperm, Q, Np,
                                              Pn0 + (p & 1) * Np * LDY, Tl0 + (p & 1) * 16 * LDY,
                                              wp2 + pr * 1024 + (pbuf & 1) * 512, h, pcnt + pr,
                                              pepoch, lane, flag + 1);
          ++pbuf;
          if (cb == q + 1) {
            __threadfence_block();
            if (lane == 0) __hip_atomic_fetch_add(blkcnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
      __threadfence_block();
      __syncthreads();
    }
  } else {
    for (int p = -1; p < NRB - 1; ++p) {
      const int q = p + 1;
      if (p >= 0) {
        // trailing column blocks q+1 .. with panel p; the first (wave 4) is announced to the
        // panel waves, which prefetch it for the next step
        for (int cb = q + 1 + (w - QR_PANEL_WAVES); cb < NRB; cb += QR_THREADS / 64 - QR_PANEL_WAVES) {
          if constexpr (NRBMAX > 16)
            update_block_chunked<13>(NRB - p, 16 * p, cb, p == 0, Ab, iperm, Q, Np,
                                     Pn0 + (p & 1) * Np * LDY, Tl0 + (p & 1) * 16 * LDY, lane);
          else
          update_block<NRBMAX>(NRB - p, 16 * p, cb, p == 0, Ab, iperm, Q, Np,
                               Pn0 + (p & 1) * Np * LDY, Tl0 + (p & 1) * 16 * LDY, nullptr, lane);
          if (cb == q + 1) {
            __threadfence_block();
            if (lane == 0) __hip_atomic_store(blkrdy, p, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
      }
      __threadfence_block();
      __syncthreads();
    }
  }

  // ---- outputs: log D, det Q, perm, and the two diagonal scalings of the V-update factor
  // F = S_r R S_c (S_c = e^(key_j - kref), S_r = e^(kref - key_i) / |R_ii|, with kref the
  // middle of the key range so that neither overflows before F itself would); the V update
  // applies them to its operand rows and output rows, off the chain's critical path
  int ntau = 0;
  double kmax = -INFINITY, kmin = INFINITY;
  for (int i = tid; i < Np; i += QR_THREADS) {
    logD[(size_t)b * Np + i] = log(fabs(beta[i])) + key[i];
    perm[(size_t)b * Np + i] = iperm[i];
    ntau += tauA[i] != 0.0;
    kmax = fmax(kmax, key[i]);
    kmin = fmin(kmin, key[i]);
  }
  for (int off = 32; off >= 1; off >>= 1) {
    ntau += __shfl_xor(ntau, off, 64);
    kmax = fmax(kmax, __shfl_xor(kmax, off, 64));
    kmin = fmin(kmin, __shfl_xor(kmin, off, 64));
  }
  if (lane == 0) {
    nt[w] = (double)ntau;
    red[w] = kmax;
    red[8 + w] = kmin;
  }
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (int k = 0; k < QR_THREADS / 64; ++k) tot += (int)nt[k];
    qsign[b] = (tot & 1) ? -1 : 1;
    if (flag[0]) status[b] |= 1;
    if (flag[1]) status[b] |= 8;
  }
  {
    double hi = red[0], lo = red[8];
    for (int k = 1; k < QR_THREADS / 64; ++k) {
      hi = fmax(hi, red[k]);
      lo = fmin(lo, red[8 + k]);
    }
    // (a non-finite key comes from a non-finite input, already flagged in status)
    const double kref = (isfinite(hi) && isfinite(lo)) ? 0.5 * (hi + lo) : 0.0;
    for (int i = tid; i < Np; i += QR_THREADS) {
      keyo[(size_t)b * 2 * Np + i] = exp(key[i] - kref);
      keyo[(size_t)b * 2 * Np + Np + i] = exp(kref - key[i]) / fabs(beta[i]);
    }
  }
}

// ------------------------------------------------------------------------------ vupd

template <int RB, int CB>
__global__ __launch_bounds__(256) void vupd_k(const double* __restrict__ QRW,
                                              const int* __restrict__ perm,
                                              const double* __restrict__ scales,
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
  const double* F = QRW + (size_t)b * Np * Np;   // R in the upper triangle
  const int* pb = perm + (size_t)b * Np;
  // the factor is S_r R S_c (diagonal scalings from the QR): P = S_c P^T V_old here, the
  // output rows scaled by S_r when stored
  const double* csc = scales + (size_t)b * 2 * Np;
  const double* rsc = csc + Np;
  for (int idx = tid; idx < W * Np; idx += 256) {
    const int q = idx / W, j = idx - q * W;
    const int src = pb[q];
    const double x = Vo ? Vo[(size_t)b * Np * Np + (size_t)src * Np + c0 + j]
                        : (src == c0 + j ? 1.0 : 0.0);
    P[j * LDP + q] = csc[q] * x;
  }
  __syncthreads();
  dx4 acc[RB][CB];
#pragma unroll
  for (int r = 0; r < RB; ++r)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[r][cb] = zero4d();
  // row blocks in zigzag order (w, 7 - w, 8 + w, ...): the triangle's rows are shared
  // evenly by the 4 waves; F's next 16-column slice is loaded while the current one is used
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int rb = (r & 1) ? 4 * r + 3 - w : 4 * r + w;
    if (rb >= NRB) continue;
    const double* frow = F + (size_t)(16 * rb + c) * Np + 4 * g;
    double2 n01 = ((const double2*)(frow + 16 * rb))[0], n23 = ((const double2*)(frow + 16 * rb))[1];
    for (int kb = rb; kb < NRB; ++kb) {
      const int q0 = 16 * kb + 4 * g;
      const double2 f01 = n01, f23 = n23;
      if (kb + 1 < NRB) {
        n01 = ((const double2*)(frow + 16 * (kb + 1)))[0];
        n23 = ((const double2*)(frow + 16 * (kb + 1)))[1];
      }
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
    const int rb = (r & 1) ? 4 * r + 3 - w : 4 * r + w;
    if (rb >= NRB) continue;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * rb + drow64(g, v);
        out[(size_t)row * Np + c0 + 16 * cb + c] = rsc[row] * acc[r][cb][v];
      }
  }
}

// A = B Q for Np <= 400: one wave per 16-row panel of B, the 4 panels of one item sharing
// a workgroup.  The panel lives in registers as the 16x16 tiles of B^T in the matrix-core
// accumulator layout (lane (g, c), register v: B^T[16t + g + 4v][c]), which is also the
// layout of a B operand (k = g + 4s for slice s).  With Y_p the block of Householder
// vectors and T_p its compact-WY factor,
//   W^T = Y_p^T B^T,  W'^T = T_p^T W^T,  B^T -= Y_p W'^T
// apply (I - Y_p T_p Y_p^T) from the right, block after block, without a transpose.
//
// Y_p and T_p are staged in LDS for the 4 waves, double-buffered: block p+1 is copied from
// global memory straight into LDS (global_load_lds_dwordx4, no registers) while block p is
// applied, so the registers go to the panel and to operand prefetch: each step's 4 LDS
// operands are read while the previous step's 4 matrix-core instructions issue.  Rows of a
// staged block sit at stride LYD doubles (even, so every 16-byte slot is aligned; the
// column reads of the update spread over the banks).  The unit-lower masking of the top
// 16 rows is applied in LDS by the threads whose copies wrote them.
constexpr int LDW = 18;   // row stride of the per-wave 16x16 transpose buffers
constexpr int LYD = 18;   // row stride of a staged Householder block

// 16 bytes from global memory into LDS: lane L of the wave writes bytes 16 L .. 16 L + 15
// from lds_base (the same in every lane)
__device__ __forceinline__ void lds_copy16(const double* src, double* lds_base) {
  __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                   (__attribute__((address_space(3))) void*)lds_base, 16, 0, 0);
}

// doubles of one staging buffer (at least the 4 per-wave transpose buffers, which alias
// the second one before the first copy into it and after the last)
__host__ __device__ constexpr int wy_ybuf(int Np) { return (Np > 64 ? Np : 64) * LYD; }

// Up to Np = 256 two workgroups share a CU (two waves per SIMD, 256 registers each); up to
// Np = 400 (25 tiles of the panel per wave) one workgroup per CU, whose waves then have
// the whole register file of their SIMD (the LDS staging buffers take 119 KB there).
template <int NRBMAX>
__global__ __launch_bounds__(256, NRBMAX > 16 ? 1 : 2) void wy_apply_reg_k(const double* __restrict__ Bsrc,
                                                      int64_t bstride,
                                                      const double* __restrict__ QRW,
                                                      const double* __restrict__ Tb,
                                                      double* __restrict__ A,
                                                      double* __restrict__ npart,
                                                      int transpose_out, int nb, int Np) {
  extern __shared__ double lds[];
  constexpr int NSLOT = (9 * 16 * NRBMAX + 255) / 256;   // copy instructions per block
  const int NRB = Np >> 4, npg = (NRB + 3) >> 2, YB = wy_ybuf(Np);
  // staging buffer k: Y block at lds + k YB ([K][LYD]: rows j0 .. Np-1, local), T block at
  // lds + 2 YB + 256 k (offsets from the shared array, so every access stays an LDS access)
  const int id = xcd_remap(blockIdx.x, nb * npg);
  if (id < 0) return;
  const int b = id / npg, tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4,
            c = lane & 15;
  double* wb = lds + YB + w * 16 * LDW;                  // [16][LDW] of this wave
  const int rp = 4 * (id % npg) + w, r0 = 16 * rp;
  const bool act = rp < NRB;
  const double* Y = QRW + (size_t)b * Np * Np;
  const double* T = Tb + (size_t)b * NRB * 256;

  // block p: 16-byte slot q = 9 r + m2 holds Y[j0 + r][j0 + 2 m2 ..], m2 = 8 is padding;
  // instruction i of wave w fills slots 256 i + 64 w .. + 63
  auto stage = [&](int p, int k) {
    double* yb = lds + k * YB;
    double* tb = lds + 2 * YB + 256 * k;
    const int j0 = 16 * p, nslot = 9 * (Np - j0);
    const double* Yp = Y + (size_t)j0 * Np + j0;
#pragma unroll
    for (int i = 0; i < NSLOT; ++i) {
      const int q = tid + 256 * i, r = q / 9, m2 = q - 9 * r;
      if (q < nslot && m2 < 8) lds_copy16(Yp + (size_t)r * Np + 2 * m2, yb + 2 * (256 * i + 64 * w));
    }
    if (tid < 128) lds_copy16(T + (size_t)p * 256 + 2 * tid, tb + 2 * 64 * w);
  };
  // after this thread's copies have landed: unit diagonal, zeros above, in the top rows
  auto mask_top = [&](int k) {
    double* yb = lds + k * YB;
    if (tid < 144) {
      const int r = tid / 9, m = 2 * (tid - 9 * (tid / 9));
      if (m < 16) {
        double* e = yb + r * LYD + m;
        const double y0 = e[0], y1 = e[1];
        e[0] = r > m ? y0 : (r == m ? 1.0 : 0.0);
        e[1] = r > m + 1 ? y1 : (r == m + 1 ? 1.0 : 0.0);
      }
    }
  };
  auto wait_copies = [] { __builtin_amdgcn_s_waitcnt(0x0F70); };   // vmcnt(0)

  // the panel's tiles: every row load is issued before the first one is turned around, so
  // the loads of all tiles are in flight together
  dx4 bt[NRBMAX];
#pragma unroll
  for (int t = 0; t < NRBMAX; ++t) {
    bt[t] = zero4d();
    if (t < NRB && act && Bsrc) {
      // lane: row lane >> 2 of the panel, columns 4 (lane & 3) .. + 3 of tile t
      const double* src = Bsrc + (size_t)b * bstride + (size_t)(r0 + (lane >> 2)) * Np + 16 * t +
                          4 * (lane & 3);
      const double2 x01 = ((const double2*)src)[0], x23 = ((const double2*)src)[1];
      bt[t][0] = x01.x;
      bt[t][1] = x01.y;
      bt[t][2] = x23.x;
      bt[t][3] = x23.y;
    }
  }
  stage(0, 0);
#pragma unroll
  for (int t = 0; t < NRBMAX; ++t) {
    if (t < NRB && act) {
      if (Bsrc) {
        // turned around in the wave's LDS buffer into the B^T tile layout
        double* d = wb + (lane >> 2) * LDW + 4 * (lane & 3);
        ((double2*)d)[0] = double2{bt[t][0], bt[t][1]};
        ((double2*)d)[1] = double2{bt[t][2], bt[t][3]};
        wave_lds_fence();
#pragma unroll
        for (int v = 0; v < 4; ++v) bt[t][v] = wb[c * LDW + g + 4 * v];
        wave_lds_fence();
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) bt[t][v] = (r0 + c == 16 * t + g + 4 * v) ? 1.0 : 0.0;
      }
    }
  }
  wait_copies();
  mask_top(0);
  __syncthreads();   // block 0 staged; the transpose buffers are free
  if (NRB > 1) stage(1, 1);

  for (int p = 0; p < NRB; ++p) {
    const double* Ys = lds + (p & 1) * YB;
    const double* Ts = lds + 2 * YB + 256 * (p & 1);
    if (act) {
      // operands ping-pong between two register sets by the parity of the (unrolled) step,
      // so a step's reads land while the previous step's products issue, with no copies
      double oa[4] = {0.0, 0.0, 0.0, 0.0}, ob[4] = {0.0, 0.0, 0.0, 0.0};
      // W^T = Y_p^T B^T: step kb reads rows 16 (kb - p) + 4 s + g of the block, column c
      if (p & 1) {
#pragma unroll
        for (int s = 0; s < 4; ++s) ob[s] = Ys[(4 * s + g) * LYD + c];
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) oa[s] = Ys[(4 * s + g) * LYD + c];
      }
      dx4 wt = zero4d();
#pragma unroll
      for (int kb = 0; kb < NRBMAX; ++kb) {
        if (kb >= p && kb < NRB) {
          double* cur = (kb & 1) ? ob : oa;
          double* nxt = (kb & 1) ? oa : ob;
          // the last step re-reads its own rows: an unconditional read keeps the wait
          // before the next step's products from covering this read
          const int kn = (kb + 1 < NRB ? kb + 1 : kb) - p;
#pragma unroll
          for (int s = 0; s < 4; ++s) nxt[s] = Ys[(16 * kn + 4 * s + g) * LYD + c];
#pragma unroll
          for (int s = 0; s < 4; ++s) wt = mfma64(cur[s], bt[kb][s], wt);
        }
      }
      dx4 wp = zero4d();
#pragma unroll
      for (int s = 0; s < 4; ++s) wp = mfma64(-Ts[(4 * s + g) * 16 + c], wt[s], wp);
      // wp holds -W'^T (negating T negates every product and sum exactly), so
      // B^T -= Y_p W'^T is B^T + Y_p wp: step cb reads row 16 (cb - p) + c of the block,
      // columns 4 s + g
      if (p & 1) {
#pragma unroll
        for (int s = 0; s < 4; ++s) ob[s] = Ys[c * LYD + 4 * s + g];
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) oa[s] = Ys[c * LYD + 4 * s + g];
      }
#pragma unroll
      for (int cb = 0; cb < NRBMAX; ++cb) {
        if (cb >= p && cb < NRB) {
          double* cur = (cb & 1) ? ob : oa;
          double* nxt = (cb & 1) ? oa : ob;
          const int kn = (cb + 1 < NRB ? cb + 1 : cb) - p;
#pragma unroll
          for (int s = 0; s < 4; ++s) nxt[s] = Ys[(16 * kn + c) * LYD + 4 * s + g];
#pragma unroll
          for (int s = 0; s < 4; ++s) bt[cb] = mfma64(cur[s], wp[s], bt[cb]);
        }
      }
    }
    if (p + 1 < NRB) {
      wait_copies();
      mask_top((p + 1) & 1);
    }
    __syncthreads();   // block p+1 staged and masked; every wave is done with block p
    if (p + 2 < NRB) stage(p + 2, p & 1);
  }

  if (!act) return;
  double* out = A + (size_t)b * Np * Np;
#pragma unroll
  for (int t = 0; t < NRBMAX; ++t) {
    if (t < NRB) {
      if (transpose_out) {
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(size_t)(16 * t + g + 4 * v) * Np + r0 + c] = bt[t][v];
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) wb[c * LDW + g + 4 * v] = bt[t][v];
        wave_lds_fence();
        const double* sp = wb + (lane >> 2) * LDW + 4 * (lane & 3);
        double* dst = out + (size_t)(r0 + (lane >> 2)) * Np + 16 * t + 4 * (lane & 3);
        ((double2*)dst)[0] = ((const double2*)sp)[0];
        ((double2*)dst)[1] = ((const double2*)sp)[1];
        wave_lds_fence();
      }
      if (npart) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double s2 = sum16(bt[t][v] * bt[t][v]);
          if (c == 0) npart[((size_t)b * NRB + rp) * Np + 16 * t + g + 4 * v] = s2;
        }
      }
    }
  }
}

// V_new = F P^T V_old for Np <= 256, each output strip split over k between two waves:
// the 4 strips of one item per workgroup of 8 waves; wave (strip w, parity h) holds the
// tiles of W = P^T V_old for the block rows kb = 2 i + h only (half the registers of one
// wave holding them all, so 4 waves per SIMD), and for every block row rb of F both waves
// of a strip sum their tiles kb >= rb.  One of them leaves its partial tile in LDS and the
// other adds it after the block row's barrier and stores the output tile; the two swap
// roles every block row, so a single partial buffer is never written before it is read.
// The 16 rows of F that block row rb needs (columns 16 rb .. Np-1) are copied from global
// memory straight into LDS (global_load_lds_dwordx4), double-buffered with the block row
// being applied, at row stride Np + 2 (even: 16-byte slots stay aligned).  The stored
// Householder vectors below the diagonal are masked to zero where they are read (only the
// diagonal block holds any), and each step's 4 LDS operands are read while the previous
// step's 4 matrix-core instructions issue.
template <int NRBMAX>
__global__ __launch_bounds__(512, 4) void vupd_split_k(const double* __restrict__ QRW,
                                                       const int* __restrict__ perm,
                                                       const double* __restrict__ scales,
                                                       const double* __restrict__ Vo,
                                                       double* __restrict__ Vn, int nb, int Np) {
  extern __shared__ double lds[];
  constexpr int NH = (NRBMAX + 1) / 2;
  const int LDF = Np + 2, FB = 16 * LDF;
  const int NRB = Np >> 4, npg = (NRB + 3) >> 2;
  const int id = xcd_remap(blockIdx.x, nb * npg);
  if (id < 0) return;
  const int b = id / npg, tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, g = lane >> 4,
            c = lane & 15;
  const int w = wv & 3, h = wv >> 2;
  const int cs = 4 * (id % npg) + w, col = 16 * cs + c;
  const bool act = cs < NRB;
  const double* F = QRW + (size_t)b * Np * Np;
  const int* pb = perm + (size_t)b * Np;
  double* part = lds + 2 * FB + (w * 64 + lane) * 4;   // [4 strips][64 lanes][4]
  double* rs = lds + 2 * FB + 1024;                     // [Np]: the output row scales

  // block row rb into buffer k: wave wv copies rows 2 wv and 2 wv + 1, 64 16-byte slots
  // (columns 2 j, 2 j + 1 for j = 64 u + lane) per instruction, the slots 8 rb <= j < Np / 2
  auto stage = [&](int rb, int k) {
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      const int r = 2 * wv + rr;
#pragma unroll
      for (int u = 0; u < (8 * NRBMAX + 63) / 64; ++u) {
        const int j = 64 * u + lane;
        if (j >= 8 * rb && 2 * j < Np)
          lds_copy16(F + (size_t)(16 * rb + r) * Np + 2 * j, lds + k * FB + r * LDF + 128 * u);
      }
    }
  };
  auto wait_copies = [] { __builtin_amdgcn_s_waitcnt(0x0F70); };   // vmcnt(0)
  stage(0, 0);

  // the factor is S_r R S_c (diagonal scalings from the QR): W = S_c P^T V_old here, the
  // output rows scaled by S_r when stored
  const double* csc = scales + (size_t)b * 2 * Np;
  for (int r = tid; r < Np; r += 512) rs[r] = csc[Np + r];
  // the gather in three passes (permutation, rows of V_old, scales) with every load of a
  // pass in flight together; rows and columns clamped into the item for unused tiles
  dx4 wt[NH];
  int src[NH][4];
  const int colc = act ? col : 0;
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    const int kb = 2 * i + h < NRB ? 2 * i + h : NRB - 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) src[i][v] = pb[16 * kb + g + 4 * v];
  }
  if (Vo) {
    const double* vb = Vo + (size_t)b * Np * Np + colc;
#pragma unroll
    for (int i = 0; i < NH; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) wt[i][v] = vb[(size_t)src[i][v] * Np];
  } else {
#pragma unroll
    for (int i = 0; i < NH; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) wt[i][v] = src[i][v] == col ? 1.0 : 0.0;
  }
#pragma unroll
  for (int i = 0; i < NH; ++i) {
    const int kb = 2 * i + h;
    const bool use = kb < NRB && act;
    const int kc = kb < NRB ? kb : NRB - 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double sc = csc[16 * kc + g + 4 * v];
      wt[i][v] = use ? sc * wt[i][v] : 0.0;
    }
  }
  wait_copies();
  __syncthreads();
  if (NRB > 1) stage(1, 1);
  double* out = Vn + (size_t)b * Np * Np;
  for (int rb = 0; rb < NRB; ++rb) {
    const bool fin = h == (rb & 1);   // this wave finishes the tile of block row rb
    dx4 acc = zero4d();
    if (act) {
      const double* Fs = lds + (rb & 1) * FB + c * LDF + g;
      // step i (kb = 2 i + h >= rb) reads F[16 rb + c][16 kb + 4 s + g]; the first step of
      // the finishing wave is the diagonal block, zero below the diagonal
      const int i0 = (rb - h + 1) >> 1;
      double oa[4] = {0.0, 0.0, 0.0, 0.0}, ob[4] = {0.0, 0.0, 0.0, 0.0};
      if (2 * i0 + h < NRB) {
        double f[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double v = Fs[16 * (2 * i0 + h) + 4 * s];
          f[s] = (fin && 4 * s + g < c) ? 0.0 : v;
        }
        if (i0 & 1) {
#pragma unroll
          for (int s = 0; s < 4; ++s) ob[s] = f[s];
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) oa[s] = f[s];
        }
      }
#pragma unroll
      for (int i = 0; i < NH; ++i) {
        const int kb = 2 * i + h;
        if (kb >= rb && kb < NRB) {
          double* cur = (i & 1) ? ob : oa;
          double* nxt = (i & 1) ? oa : ob;
          const int kn = kb + 2 < NRB ? kb + 2 : kb;
#pragma unroll
          for (int s = 0; s < 4; ++s) nxt[s] = Fs[16 * kn + 4 * s];
#pragma unroll
          for (int s = 0; s < 4; ++s) acc = mfma64(cur[s], wt[i][s], acc);
        }
      }
      if (!fin) *(dx4*)part = acc;
    }
    if (rb + 1 < NRB) wait_copies();
    __syncthreads();   // block row rb+1 staged; every wave is done with block row rb
    if (act && fin) {
      acc += *(const dx4*)part;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * rb + g + 4 * v;
        out[(size_t)row * Np + col] = rs[row] * acc[v];
      }
    }
    // issued after this step's LDS reads, which therefore wait for no copy
    if (rb + 2 < NRB) stage(rb + 2, rb & 1);
  }
}

template <int NRBMAX>
hipError_t run_qr(const double* A, int64_t astride, const double* norm2, int64_t nstride, int nparts,
                  const double* logDp, double* QRW, double* Tb, int* perm, double* key,
                  double* logD, int* qsign, int* status, int nb, int Np, hipStream_t st) {
  const size_t lds = (size_t)(2 * Np * LDY + 2 * 16 * LDY + 2 * QR_PANEL_WAVES * 16 + 32 +
                              QR_PANEL_WAVES * 256 + 3 * Np + 8 + (QR_PAIR_UPDATE(NRBMAX) ? 2048 : 0)) *
                         sizeof(double) + (size_t)(Np + 8) * sizeof(int);
  hipLaunchKernelGGL(qr_k<NRBMAX>, dim3(nb), dim3(QR_THREADS), lds, st, A, astride, norm2, nstride, nparts,
                     logDp, QRW, Tb, perm, key, logD, qsign, status, Np);
  return hipGetLastError();
}

template <int RB>
hipError_t run_vupd(const double* QRW, const int* perm, const double* scales, const double* Vo,
                    double* Vn, int nb, int Np, hipStream_t st) {
  constexpr int CB = 2;
  if (Np % 32 == 0) {
    const size_t lds = (size_t)(16 * CB) * (Np + 2) * sizeof(double);
    hipLaunchKernelGGL((vupd_k<RB, CB>), dim3(xcd_grid(nb * (Np / 32))), dim3(256), lds, st, QRW,
                       perm, scales, Vo, Vn, nb, Np);
  } else {
    const size_t lds = (size_t)16 * (Np + 2) * sizeof(double);
    hipLaunchKernelGGL((vupd_k<RB, 1>), dim3(xcd_grid(nb * (Np / 16))), dim3(256), lds, st, QRW,
                       perm, scales, Vo, Vn, nb, Np);
  }
  return hipGetLastError();
}

__global__ void fill_i32_k(int* dst, int n, int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = value;
}

__global__ void order_gate_k() {}

}  // namespace

hipError_t launch_order_gate(hipStream_t st) {
  hipLaunchKernelGGL(order_gate_k, dim3(1), dim3(64), 0, st);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* dst, int n, int value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_k, dim3((n + 255) / 256), dim3(256), 0, st, dst, n, value);
  return hipGetLastError();
}

hipError_t launch_wy_apply(const double* Bsrc, int64_t bstride, const double* QRW,
                           const double* Tb, double* A, double* npart, int transpose_out,
                           int nb, int Np, hipStream_t st) {
  const int NRB = Np / 16;
  if (NRB <= 25) {
    // register-resident panels (Np <= 400)
    const int npg = (NRB + 3) / 4;
    const size_t lds_r = (size_t)(2 * wy_ybuf(Np) + 512) * sizeof(double);
#define WY_REG(NR)                                                                              \
  hipLaunchKernelGGL(wy_apply_reg_k<NR>, dim3(xcd_grid(nb * npg)), dim3(256), lds_r, st, Bsrc,   \
                     bstride, QRW, Tb, A, npart, transpose_out, nb, Np)
    if (NRB <= 4) WY_REG(4);
    else if (NRB <= 8) WY_REG(8);
    else if (NRB <= 16) WY_REG(16);
    else WY_REG(25);
#undef WY_REG
    return hipGetLastError();
  }
  const size_t lds = (size_t)(16 * (Np + 2) + 5 * 16 * LDY) * sizeof(double);
  hipLaunchKernelGGL(wy_apply_k, dim3(xcd_grid(nb * NRB)), dim3(256), lds, st, Bsrc, bstride,
                     QRW, Tb, A, npart, transpose_out, nb, Np);
  return hipGetLastError();
}

hipError_t launch_qr(const double* A, int64_t astride, const double* norm2, int64_t nstride,
                     int nparts, const double* logDp, double* QRW, double* Tb, int* perm,
                     double* key, double* logD, int* qsign, int* status, int nb, int Np,
                     hipStream_t st) {
  const int NRB = Np / 16;
  if (NRB <= 4) return run_qr<4>(A, astride, norm2, nstride, nparts, logDp, QRW, Tb, perm, key, logD, qsign, status, nb, Np, st);
  if (NRB <= 8) return run_qr<8>(A, astride, norm2, nstride, nparts, logDp, QRW, Tb, perm, key, logD, qsign, status, nb, Np, st);
  if (NRB <= 16) return run_qr<16>(A, astride, norm2, nstride, nparts, logDp, QRW, Tb, perm, key, logD, qsign, status, nb, Np, st);
  if (NRB <= 25) return run_qr<25>(A, astride, norm2, nstride, nparts, logDp, QRW, Tb, perm, key, logD, qsign, status, nb, Np, st);
  if (NRB <= 32) return run_qr<32>(A, astride, norm2, nstride, nparts, logDp, QRW, Tb, perm, key, logD, qsign, status, nb, Np, st);
  return hipErrorInvalidValue;
}

hipError_t launch_vupd(const double* QRW, const int* perm, const double* key, const double* Vo,
                       double* Vn, int nb, int Np, hipStream_t st) {
  const int NRB = Np / 16, RB = (NRB + 3) / 4;
  if (NRB <= 16) {
    // register-resident strips (Np <= 256): two F block rows and the partial tiles in LDS
    const int npg = (NRB + 3) / 4;
    const size_t lds = ((size_t)2 * 16 * (Np + 2) + 4 * 64 * 4 + Np) * sizeof(double);
#define VUPD_SPLIT(NR)                                                                        \
  hipLaunchKernelGGL(vupd_split_k<NR>, dim3(xcd_grid(nb * npg)), dim3(512), lds, st, QRW, perm, \
                     key, Vo, Vn, nb, Np)
    if (NRB <= 4) VUPD_SPLIT(4);
    else if (NRB <= 8) VUPD_SPLIT(8);
    else VUPD_SPLIT(16);
#undef VUPD_SPLIT
    return hipGetLastError();
  }
  switch (RB) {
    case 1: return run_vupd<1>(QRW, perm, key, Vo, Vn, nb, Np, st);
    case 2: return run_vupd<2>(QRW, perm, key, Vo, Vn, nb, Np, st);
    case 3: return run_vupd<3>(QRW, perm, key, Vo, Vn, nb, Np, st);
    case 4: return run_vupd<4>(QRW, perm, key, Vo, Vn, nb, Np, st);
    case 5: return run_vupd<5>(QRW, perm, key, Vo, Vn, nb, Np, st);
    case 6: return run_vupd<6>(QRW, perm, key, Vo, Vn, nb, Np, st);
    case 7: return run_vupd<7>(QRW, perm, key, Vo, Vn, nb, Np, st);
    case 8: return run_vupd<8>(QRW, perm, key, Vo, Vn, nb, Np, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace slmc
