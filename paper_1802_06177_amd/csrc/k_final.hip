// Recombination of the stabilized product into log|det(I + U D V)|, its sign and
// G = (I + U D V)^{-1} (SM Eqs. S2, S3).
//
// With Db = max(D, 1) and Ds = min(D, 1) (both taken from log D, so neither overflows)
//   I + U D V = U Db X,   X = Db^{-1} U^T + Ds V,
//   log|det| = sum log Db + log|det X|,  sign = det U * sign det X,
//   G = X^{-1} (Db^{-1} U^T).
// X is factored by a blocked LU with partial pivoting (one workgroup per item, the pivot
// order kept as a row map so no row is moved in memory); the solve for G gives each wave
// one 16-column block of the right-hand side held in registers.  The FP64 residual step
// refines that solve: R = Db^{-1} U^T - X G (a tiled batched GEMM), G += X^{-1} R.
#include "common.h"
#include "launch.h"

namespace slmc {

namespace {

constexpr int LDY = 17;
constexpr double LN2 = 0.69314718055994530942;

// Pivot search key: the bits of |a| (monotonic for non-negative doubles) with the low 9
// mantissa bits replaced by 511 - slot, so the largest |a| wins and, among values equal to
// within 2^-43, the lowest slot.  Never 0 for a live row (slot < 448); NaN sorts above every
// number, so a NaN column becomes the pivot and is reported.
__device__ __forceinline__ uint64_t pivot_key(double a, int slot) {
  return ((uint64_t)__double_as_longlong(fabs(a)) & ~511ull) | (uint64_t)(511 - slot);
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// Maximum over the 64 lanes, returned to every lane: row rotations inside each 16-lane row
// (DPP row_ror 8, 4, 2, 1), then the permlane16 and permlane32 swaps of two copies, which
// leave lane l's partner (l ^ 16, then l ^ 32) in the second copy.
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  v = umax64(v, dpp_u64<0x128>(v));
  v = umax64(v, dpp_u64<0x124>(v));
  v = umax64(v, dpp_u64<0x122>(v));
  v = umax64(v, dpp_u64<0x121>(v));
  {
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)v, (uint32_t)v, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(v >> 32), (uint32_t)(v >> 32), false, false);
    v = umax64(((uint64_t)hi[0] << 32) | lo[0], ((uint64_t)hi[1] << 32) | lo[1]);
  }
  {
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)v, (uint32_t)v, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(v >> 32), (uint32_t)(v >> 32), false, false);
    v = umax64(((uint64_t)hi[0] << 32) | lo[0], ((uint64_t)hi[1] << 32) | lo[1]);
  }
  return v;
}

__device__ __forceinline__ double xval(const double* QT, const double* V, const double* dbi,
                                       const double* dsm, int Np, int r, int j) {
  return dbi[r] * QT[(size_t)r * Np + j] + dsm[r] * V[(size_t)r * Np + j];
}

// NT threads per item: 512 (8 waves, one panel row per thread) up to Np = 256, where the
// trailing update's registers fit two waves per SIMD and the second wave on each SIMD hides
// the first one's memory latency; 256 (4 waves, panel rows t and t + 256) above.
template <int NRBMAX, int NT>
__global__ __launch_bounds__(NT) void lu_k(const double* __restrict__ QT,
                                            const double* __restrict__ V,
                                            const double* __restrict__ logD,
                                            const int* __restrict__ qsign,
                                            const int* __restrict__ st_in,
                                            double* __restrict__ LU, int* __restrict__ prow_g,
                                            double* __restrict__ DI,
                                            const int* __restrict__ item_of,
                                            double* __restrict__ logdet_out,
                                            int8_t* __restrict__ sign_out,
                                            int32_t* __restrict__ status_out, int N, int Np) {
  extern __shared__ double lds[];
  constexpr int NW = NT / 64;
  constexpr bool TWO = NT < 448;           // a second panel row per thread (Np <= 448)
  const int b = blockIdx.x;
  const int NRB = Np >> 4;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  double* Pn0 = lds;                       // [2][Np][LDY]
  double* dbi = Pn0 + 2 * Np * LDY;        // [Np]
  double* dsm = dbi + Np;                  // [Np]
  double* ud = dsm + Np;                   // [Np] pivots (U diagonal)
  double* Li = ud + Np;                    // [16][LDY]
  double* Ui = Li + 16 * LDY;              // [16][LDY]
  double* redv = Ui + 16 * LDY;            // [2 NW]
  double* cand = redv + 2 * NW;            // [2][NW][17]: each wave's pivot candidate row + key
  int* prow = (int*)(cand + 2 * NW * 17);  // [Np]
  int* redi = prow + Np;                   // [NW]
  int* cnt = redi + NW;                    // [2]: swaps, singular
  int* phys = cnt + 2;                     // [Np] panel position -> slot
  int* posof = phys + Np;                  // [Np] slot -> panel position

  const double* QTb = QT + (size_t)b * Np * Np;
  const double* Vb = V + (size_t)b * Np * Np;
  double* L = LU + (size_t)b * Np * Np;
  double* DIb = DI + (size_t)b * NRB * 512;
  for (int i = tid; i < Np; i += NT) {
    const double ld = logD[(size_t)b * Np + i];
    dbi[i] = exp(-fmax(ld, 0.0));
    dsm[i] = exp(fmin(ld, 0.0));
    prow[i] = i;
  }
  if (tid == 0) { cnt[0] = 0; cnt[1] = 0; }
  __syncthreads();
  for (int idx = tid; idx < Np * 16; idx += NT) {
    const int r = idx >> 4, jj = idx & 15;
    Pn0[r * LDY + jj] = xval(QTb, Vb, dbi, dsm, Np, r, jj);
  }
  __syncthreads();

  for (int p = 0; p < NRB; ++p) {
    const int j0 = 16 * p, K = Np - j0, nrbK = NRB - p;
    double* Pn = Pn0 + (p & 1) * Np * LDY;
    double* Pnx = Pn0 + ((p + 1) & 1) * Np * LDY;
    // Panel (K rows x 16 columns): thread t keeps slot t (and t + NT) in registers.  Rows
    // never move: a row chosen as pivot leaves the search, and thread 0 keeps the
    // position <-> slot maps of the equivalent row exchanges (and their count).  One
    // barrier per column: every wave publishes its best candidate row, every thread then
    // takes the winner from LDS.
    const bool h0 = tid < K, h1 = TWO && tid + NT < K;
    double ra[16], rc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      ra[j] = h0 ? Pn[tid * LDY + j] : 0.0;
      rc[j] = h1 ? Pn[(tid + NT) * LDY + j] : 0.0;
    }
    for (int i = tid; i < K; i += NT) { phys[i] = i; posof[i] = i; }
    bool a0 = h0, a1 = h1;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      const uint64_t k0 = a0 ? pivot_key(ra[cc], tid) : 0ull;
      const uint64_t k1 = a1 ? pivot_key(rc[cc], tid + NT) : 0ull;
      const uint64_t mine = umax64(k0, k1);
      const uint64_t kw = wave_max_u64(mine);
      double* cd = cand + (cc & 1) * (NW * 17) + w * 17;
      if (kw != 0ull && mine == kw) {
        const bool second = (k1 == kw);
#pragma unroll
        for (int j = 0; j < 16; ++j) cd[j] = second ? rc[j] : ra[j];
        cd[16] = __longlong_as_double((long long)kw);
      }
      if (kw == 0ull && lane == 0) cd[16] = 0.0;
      __syncthreads();
      const double* c0 = cand + (cc & 1) * (NW * 17);
      uint64_t best = 0ull;
      int bw = 0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) {
        const uint64_t kk = (uint64_t)__double_as_longlong(c0[ww * 17 + 16]);
        if (kk > best) { best = kk; bw = ww; }
      }
      const int sp = 511 - (int)(best & 511ull);
      double pv[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) pv[j] = c0[bw * 17 + j];
      const double u = pv[cc];
      if (tid == 0) {
        const int q = posof[sp];
        if (q != cc) {
          const int s0 = phys[cc];
          phys[cc] = sp;
          phys[q] = s0;
          posof[sp] = cc;
          posof[s0] = q;
          cnt[0] += 1;
        }
        ud[j0 + cc] = u;
        if (u == 0.0 || u != u) cnt[1] = 1;
      }
      if (sp == tid) a0 = false;
      if (sp == tid + NT) a1 = false;
      const double ui = (u != 0.0) ? 1.0 / u : 0.0;
      if (a0) {
        const double l = ra[cc] * ui;
#pragma unroll
        for (int j = cc + 1; j < 16; ++j) ra[j] -= l * pv[j];
        ra[cc] = l;
      }
      if (a1) {
        const double l = rc[cc] * ui;
#pragma unroll
        for (int j = cc + 1; j < 16; ++j) rc[j] -= l * pv[j];
        rc[cc] = l;
      }
    }
    __syncthreads();   // the position maps are final
    // the panel back into LDS at its positions; the row map composed with the panel's
    int pr0 = 0, pr1 = 0;
    if (h0) {
      const int q = posof[tid];
#pragma unroll
      for (int j = 0; j < 16; ++j) Pn[q * LDY + j] = ra[j];
      pr0 = prow[j0 + phys[tid]];
    }
    if (h1) {
      const int q = posof[tid + NT];
#pragma unroll
      for (int j = 0; j < 16; ++j) Pn[q * LDY + j] = rc[j];
      pr1 = prow[j0 + phys[tid + NT]];
    }
    __syncthreads();
    if (h0) prow[j0 + tid] = pr0;
    if (h1) prow[j0 + tid + NT] = pr1;
    __syncthreads();
    // inverses of the unit-lower L11 (wave 0) and upper U11 (wave 1), one column per lane,
    // the column in registers (its zero entries add exact zeros to the sums, which keep the
    // order l = j .. i-1, resp. i+1 .. j, of the nonzero terms)
    if (w == 0 && lane < 16) {
      const int j = lane;
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < i; ++l) s += Pn[i * LDY + l] * x[l];
        x[i] = (i < j) ? 0.0 : (i == j ? 1.0 : -s);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) Li[i * LDY + j] = x[i];
    } else if (w == 1 && lane < 16) {
      const int j = lane;
      double x[16];
#pragma unroll
      for (int i = 15; i >= 0; --i) {
        double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
        for (int l = i + 1; l < 16; ++l) s -= Pn[i * LDY + l] * x[l];
        const double u = Pn[i * LDY + i];
        x[i] = (i > j) ? 0.0 : ((u != 0.0) ? s / u : 0.0);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) Ui[i * LDY + j] = x[i];
    }
    __syncthreads();
    for (int idx = tid; idx < 512; idx += NT) {
      const int which = idx >> 8, e = idx & 255, i = e >> 4, j = e & 15;
      DIb[(size_t)p * 512 + idx] = which ? Ui[i * LDY + j] : Li[i * LDY + j];
    }
    // trailing update: U12 = L11^-1 A12, A22 -= L21 U12
    for (int cb = p + 1 + w; cb < NRB; cb += NW) {
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
            const int pr = prow[j0 + 16 * rb + drow64(g, v)];
            blk[rb][v] = (p == 0) ? xval(QTb, Vb, dbi, dsm, Np, pr, 16 * cb + c)
                                  : L[(size_t)pr * Np + 16 * cb + c];
          }
        }
      }
      dx4 u12 = zero4d();
#pragma unroll
      for (int s = 0; s < 4; ++s) u12 = mfma64(Li[c * LDY + drow64(g, s)], blk[0][s], u12);
      blk[0] = u12;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int rb = 1; rb < NRBMAX; ++rb) {
          if (rb < nrbK) blk[rb] = mfma64(-Pn[(16 * rb + c) * LDY + drow64(g, s)], u12[s], blk[rb]);
        }
      }
#pragma unroll
      for (int rb = 0; rb < NRBMAX; ++rb) {
        if (rb < nrbK) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int lr = 16 * rb + drow64(g, v);
            L[(size_t)prow[j0 + lr] * Np + 16 * cb + c] = blk[rb][v];
            if (cb == p + 1 && rb >= 1) Pnx[(lr - 16) * LDY + c] = blk[rb][v];
          }
        }
      }
    }
    for (int idx = tid; idx < K * 16; idx += NT) {
      const int r = idx >> 4, jj = idx & 15;
      L[(size_t)prow[j0 + r] * Np + j0 + jj] = Pn[r * LDY + jj];
    }
    __threadfence_block();
    __syncthreads();
  }

  // log|det X|, sign, and the outputs
  double s = 0.0, sd = 0.0;
  int neg = 0;
  for (int i = tid; i < Np; i += NT) {
    const double u = ud[i];
    s += log(fabs(u));
    neg += u < 0.0;
    sd += fmax(logD[(size_t)b * Np + i], 0.0);
    prow_g[(size_t)b * Np + i] = prow[i];
  }
  s = sum64(s);
  sd = sum64(sd);
  for (int off = 32; off >= 1; off >>= 1) neg += __shfl_xor(neg, off, 64);
  if (lane == 0) { redv[w] = s; redv[NW + w] = sd; redi[w] = neg; }
  __syncthreads();
  if (tid == 0) {
    double lx = 0.0, lb = 0.0;
    int nn = 0;
    for (int k = 0; k < NW; ++k) {
      lx += redv[k];
      lb += redv[NW + k];
      nn += redi[k];
    }
    double ld = lb + lx - (double)(Np - N) * LN2;
    const int sgn = qsign[b] * (((nn + cnt[0]) & 1) ? -1 : 1);
    int stt = 0;
    if (st_in[b] != 0 || cnt[1] != 0 || !isfinite(ld)) {
      // bit 3 of the QR status: a bounded wait inside the QR ran out (device fault)
      stt = (st_in[b] & 8) ? 4 : 5;
      ld = __longlong_as_double(0x7ff8000000000000LL);
    }
    const int item = item_of ? item_of[b] : b;
    logdet_out[item] = ld;
    sign_out[item] = (int8_t)sgn;
    status_out[item] = stt;
  }
}

// Arrive-and-wait among the 4 panel waves of lu_la_k through a monotonically increasing LDS
// counter (the update waves keep working meanwhile); release on arrival, acquire on the
// wait.  Bounded: past the spin limit it sets *timeout (reported as a device fault) and
// goes on, so every wave reaches the end of the kernel.
constexpr int LU_PANEL_WAVES = 4;
constexpr int LU_SPIN_LIMIT = 1 << 16;

__device__ __forceinline__ void lu_panel_sync(int* cnt, int& epoch, int lane, int* timeout) {
  ++epoch;
  if (lane == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  const int target = LU_PANEL_WAVES * epoch;
  int spins = 0;
  while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
    if (spins >= 16) __builtin_amdgcn_s_sleep(1);
    if (++spins > LU_SPIN_LIMIT) {
      *timeout = 1;
      break;
    }
  }
}

// lu_k with look-ahead for Np <= 256 (512 threads; the panel rows, one per thread, all lie
// in waves 0-3).  Step p: waves 0-3 update column block q = p + 1 with panel p (each wave
// its row blocks w, w + 4, .. and, for U12, the top one) into the next panel buffer and
// factor it as panel q, with their own sync per column instead of a workgroup barrier;
// waves 4-7 meanwhile apply panel p to the column blocks p + 2 .. and store panel p's L
// columns.  Panel q's row map is composed after the step's barrier, once the update waves
// are done with panel p's.  The panel, its inverses and every product are those of lu_k, in
// the same order, so the factors are the same bit for bit.
template <int NRBMAX>
__global__ __launch_bounds__(512) void lu_la_k(const double* __restrict__ QT,
                                               const double* __restrict__ V,
                                               const double* __restrict__ logD,
                                               const int* __restrict__ qsign,
                                               const int* __restrict__ st_in,
                                               double* __restrict__ LU, int* __restrict__ prow_g,
                                               double* __restrict__ DI,
                                               const int* __restrict__ item_of,
                                               double* __restrict__ logdet_out,
                                               int8_t* __restrict__ sign_out,
                                               int32_t* __restrict__ status_out, int N, int Np) {
  extern __shared__ double lds[];
  constexpr int NT = 512, NW = NT / 64, NPW = LU_PANEL_WAVES;
  const int b = blockIdx.x;
  const int NRB = Np >> 4;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  double* Pn0 = lds;                       // [2][Np][LDY]
  double* dbi = Pn0 + 2 * Np * LDY;        // [Np]
  double* dsm = dbi + Np;                  // [Np]
  double* ud = dsm + Np;                   // [Np] pivots (U diagonal)
  double* Li0 = ud + Np;                   // [2][16][LDY] L11^-1 of panel p / p + 1
  double* Ui = Li0 + 2 * 16 * LDY;         // [16][LDY]
  double* redv = Ui + 16 * LDY;            // [2 NW]
  double* cand = redv + 2 * NW;            // [2][NPW][17]: each panel wave's candidate row + key
  int* prow = (int*)(cand + 2 * NPW * 17); // [Np]
  int* redi = prow + Np;                   // [NW]
  int* cnt = redi + NW;                    // [4]: swaps, singular, panel sync, sync timeout
  int* phys = cnt + 4;                     // [Np] panel position -> slot
  int* posof = phys + Np;                  // [Np] slot -> panel position

  const double* QTb = QT + (size_t)b * Np * Np;
  const double* Vb = V + (size_t)b * Np * Np;
  double* L = LU + (size_t)b * Np * Np;
  double* DIb = DI + (size_t)b * NRB * 512;
  for (int i = tid; i < Np; i += NT) {
    const double ld = logD[(size_t)b * Np + i];
    dbi[i] = exp(-fmax(ld, 0.0));
    dsm[i] = exp(fmin(ld, 0.0));
    prow[i] = i;
  }
  if (tid == 0) { cnt[0] = 0; cnt[1] = 0; cnt[2] = 0; cnt[3] = 0; }
  __syncthreads();
  for (int idx = tid; idx < Np * 16; idx += NT) {
    const int r = idx >> 4, jj = idx & 15;
    Pn0[r * LDY + jj] = xval(QTb, Vb, dbi, dsm, Np, r, jj);
  }
  __syncthreads();

  // The two roles run separate loops with the same barriers, so that the registers of one
  // role's data do not constrain the other's.
  if (__builtin_amdgcn_readfirstlane(w) < NPW) {
    int epoch = 0;
    for (int p = -1; p < NRB; ++p) {
      const int q = p + 1;
      int pr0 = 0;
      if (q < NRB) {
        const int jq = 16 * q, Kq = Np - jq;
        double* Pq = Pn0 + (q & 1) * Np * LDY;
        double* Lq = Li0 + (q & 1) * 16 * LDY;
        if (p >= 0) {
          // column block q with panel p: U12 = L11^-1 A12 (every panel wave computes it from
          // the top row block), A22 -= L21 U12 for this wave's row blocks, which go to Pq
          const int j0 = 16 * p, nrbK = NRB - p;
          const double* Pn = Pn0 + (p & 1) * Np * LDY;
          const double* Lip = Li0 + (p & 1) * 16 * LDY;
          int c = lane & 15, g = lane >> 4;
          __asm__ volatile("" : "+v"(c), "+v"(g));
          const int col = 16 * q + c;
          constexpr int RBQ = (NRBMAX + NPW - 1) / NPW;
          dx4 top, blk[RBQ];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int pr = prow[j0 + drow64(g, v)];
            top[v] = (p == 0) ? xval(QTb, Vb, dbi, dsm, Np, pr, col) : L[(size_t)pr * Np + col];
          }
#pragma unroll
          for (int r = 0; r < RBQ; ++r) {
            const int rb = w + NPW * r;
            if (rb >= 1 && rb < nrbK) {
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int pr = prow[j0 + 16 * rb + drow64(g, v)];
                blk[r][v] = (p == 0) ? xval(QTb, Vb, dbi, dsm, Np, pr, col) : L[(size_t)pr * Np + col];
              }
            }
          }
          dx4 u12 = zero4d();
#pragma unroll
          for (int s = 0; s < 4; ++s) u12 = mfma64(Lip[c * LDY + drow64(g, s)], top[s], u12);
          if (w == 0) {
#pragma unroll
            for (int v = 0; v < 4; ++v) L[(size_t)prow[j0 + drow64(g, v)] * Np + col] = u12[v];
          }
#pragma unroll
          for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int r = 0; r < RBQ; ++r) {
              const int rb = w + NPW * r;
              if (rb >= 1 && rb < nrbK) blk[r] = mfma64(-Pn[(16 * rb + c) * LDY + drow64(g, s)], u12[s], blk[r]);
            }
          }
#pragma unroll
          for (int r = 0; r < RBQ; ++r) {
            const int rb = w + NPW * r;
            if (rb >= 1 && rb < nrbK) {
#pragma unroll
              for (int v = 0; v < 4; ++v) Pq[(16 * (rb - 1) + drow64(g, v)) * LDY + c] = blk[r][v];
            }
          }
          lu_panel_sync(cnt + 2, epoch, lane, cnt + 3);
        }
        // panel q (Kq rows x 16 columns): thread t keeps slot t in registers; rows never move,
        // thread 0 keeps the position <-> slot maps of the equivalent row exchanges
        const bool h0 = tid < Kq;
        double ra[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) ra[j] = h0 ? Pq[tid * LDY + j] : 0.0;
        if (h0) { phys[tid] = tid; posof[tid] = tid; }
        bool a0 = h0;
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
          const uint64_t mine = a0 ? pivot_key(ra[cc], tid) : 0ull;
          const uint64_t kw = wave_max_u64(mine);
          double* cd = cand + (cc & 1) * (NPW * 17) + w * 17;
          if (kw != 0ull && mine == kw) {
#pragma unroll
            for (int j = 0; j < 16; ++j) cd[j] = ra[j];
            cd[16] = __longlong_as_double((long long)kw);
          }
          if (kw == 0ull && lane == 0) cd[16] = 0.0;
          lu_panel_sync(cnt + 2, epoch, lane, cnt + 3);
          const double* c0 = cand + (cc & 1) * (NPW * 17);
          uint64_t best = 0ull;
          int bw = 0;
#pragma unroll
          for (int ww = 0; ww < NPW; ++ww) {
            const uint64_t kk = (uint64_t)__double_as_longlong(c0[ww * 17 + 16]);
            if (kk > best) { best = kk; bw = ww; }
          }
          const int sp = 511 - (int)(best & 511ull);
          double pv[16];
#pragma unroll
          for (int j = 0; j < 16; ++j) pv[j] = c0[bw * 17 + j];
          const double u = pv[cc];
          if (tid == 0) {
            const int qq = posof[sp];
            if (qq != cc) {
              const int s0 = phys[cc];
              phys[cc] = sp;
              phys[qq] = s0;
              posof[sp] = cc;
              posof[s0] = qq;
              cnt[0] += 1;
            }
            ud[jq + cc] = u;
            if (u == 0.0 || u != u) cnt[1] = 1;
          }
          if (sp == tid) a0 = false;
          const double ui = (u != 0.0) ? 1.0 / u : 0.0;
          if (a0) {
            const double l = ra[cc] * ui;
#pragma unroll
            for (int j = cc + 1; j < 16; ++j) ra[j] -= l * pv[j];
            ra[cc] = l;
          }
        }
        lu_panel_sync(cnt + 2, epoch, lane, cnt + 3);   // the position maps are final
        if (h0) {
          const int qq = posof[tid];
#pragma unroll
          for (int j = 0; j < 16; ++j) Pq[qq * LDY + j] = ra[j];
          pr0 = prow[jq + phys[tid]];
        }
        lu_panel_sync(cnt + 2, epoch, lane, cnt + 3);   // the panel in position order
        // inverses of the unit-lower L11 (wave 0) and upper U11 (wave 1), one column per lane
        if (w == 0 && lane < 16) {
          const int j = lane;
          double x[16];
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < i; ++l) s += Pq[i * LDY + l] * x[l];
            x[i] = (i < j) ? 0.0 : (i == j ? 1.0 : -s);
          }
#pragma unroll
          for (int i = 0; i < 16; ++i) Lq[i * LDY + j] = x[i];
        } else if (w == 1 && lane < 16) {
          const int j = lane;
          double x[16];
#pragma unroll
          for (int i = 15; i >= 0; --i) {
            double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
            for (int l = i + 1; l < 16; ++l) s -= Pq[i * LDY + l] * x[l];
            const double u = Pq[i * LDY + i];
            x[i] = (i > j) ? 0.0 : ((u != 0.0) ? s / u : 0.0);
          }
#pragma unroll
          for (int i = 0; i < 16; ++i) Ui[i * LDY + j] = x[i];
        }
        lu_panel_sync(cnt + 2, epoch, lane, cnt + 3);
        for (int idx = tid; idx < 512; idx += NPW * 64) {
          const int which = idx >> 8, e = idx & 255, i = e >> 4, j = e & 15;
          DIb[(size_t)q * 512 + idx] = which ? Ui[i * LDY + j] : Lq[i * LDY + j];
        }
      }
      __threadfence_block();
      __syncthreads();
      // panel q's row map, composed now that no wave reads panel p's any more
      if (q < NRB && tid < Np - 16 * q) prow[16 * q + tid] = pr0;
      __syncthreads();
    }
  } else {
    for (int p = -1; p < NRB; ++p) {
      if (p >= 0) {
      // trailing update with panel p: U12 = L11^-1 A12, A22 -= L21 U12 for blocks p + 2 ..
      const int j0 = 16 * p, K = Np - j0, nrbK = NRB - p;
      const double* Pn = Pn0 + (p & 1) * Np * LDY;
      const double* Lip = Li0 + (p & 1) * 16 * LDY;
      for (int cb = p + 2 + (w - NPW); cb < NRB; cb += NW - NPW) {
        int c = lane & 15, g = lane >> 4;
        __asm__ volatile("" : "+v"(c), "+v"(g));
        dx4 blk[NRBMAX];
#pragma unroll
        for (int rb = 0; rb < NRBMAX; ++rb) {
          if (rb < nrbK) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int pr = prow[j0 + 16 * rb + drow64(g, v)];
              blk[rb][v] = (p == 0) ? xval(QTb, Vb, dbi, dsm, Np, pr, 16 * cb + c)
                                    : L[(size_t)pr * Np + 16 * cb + c];
            }
          }
        }
        dx4 u12 = zero4d();
#pragma unroll
        for (int s = 0; s < 4; ++s) u12 = mfma64(Lip[c * LDY + drow64(g, s)], blk[0][s], u12);
        blk[0] = u12;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
          for (int rb = 1; rb < NRBMAX; ++rb) {
            if (rb < nrbK) blk[rb] = mfma64(-Pn[(16 * rb + c) * LDY + drow64(g, s)], u12[s], blk[rb]);
          }
        }
#pragma unroll
        for (int rb = 0; rb < NRBMAX; ++rb) {
          if (rb < nrbK) {
#pragma unroll
            for (int v = 0; v < 4; ++v)
              L[(size_t)prow[j0 + 16 * rb + drow64(g, v)] * Np + 16 * cb + c] = blk[rb][v];
          }
        }
      }
      // panel p's L columns (and its U11 rows), at their rows through the row map
      for (int idx = tid - NPW * 64; idx < K * 16; idx += (NW - NPW) * 64) {
        const int r = idx >> 4, jj = idx & 15;
        L[(size_t)prow[j0 + r] * Np + j0 + jj] = Pn[r * LDY + jj];
      }
      }
      __threadfence_block();
      __syncthreads();
      __syncthreads();
    }
  }

  // log|det X|, sign, and the outputs
  double s = 0.0, sd = 0.0;
  int neg = 0;
  for (int i = tid; i < Np; i += NT) {
    const double u = ud[i];
    s += log(fabs(u));
    neg += u < 0.0;
    sd += fmax(logD[(size_t)b * Np + i], 0.0);
    prow_g[(size_t)b * Np + i] = prow[i];
  }
  s = sum64(s);
  sd = sum64(sd);
  for (int off = 32; off >= 1; off >>= 1) neg += __shfl_xor(neg, off, 64);
  if (lane == 0) { redv[w] = s; redv[NW + w] = sd; redi[w] = neg; }
  __syncthreads();
  if (tid == 0) {
    double lx = 0.0, lb = 0.0;
    int nn = 0;
    for (int k = 0; k < NW; ++k) {
      lx += redv[k];
      lb += redv[NW + k];
      nn += redi[k];
    }
    double ld = lb + lx - (double)(Np - N) * LN2;
    const int sgn = qsign[b] * (((nn + cnt[0]) & 1) ? -1 : 1);
    int stt = 0;
    if (st_in[b] != 0 || cnt[1] != 0 || cnt[3] != 0 || !isfinite(ld)) {
      // bit 3 of the QR status or this kernel's own sync timeout: a bounded wait ran out
      stt = ((st_in[b] & 8) || cnt[3]) ? 4 : 5;
      ld = __longlong_as_double(0x7ff8000000000000LL);
    }
    const int item = item_of ? item_of[b] : b;
    logdet_out[item] = ld;
    sign_out[item] = (int8_t)sgn;
    status_out[item] = stt;
  }
}

// X^{-1} applied to a right-hand side (mode 0: Db^{-1} U^T; mode 1: R): forward
// substitution with the unit lower factor, then backward with the upper one, using the
// 16x16 inverses of the diagonal blocks from the LU; one wave per (item, 16 columns), the
// right-hand-side strip in registers.
template <int NRBMAX>
__global__ __launch_bounds__(256) void lu_solve_k(int mode, const double* __restrict__ QT,
                                                  const double* __restrict__ logD,
                                                  const double* __restrict__ R,
                                                  const double* __restrict__ LU,
                                                  const int* __restrict__ prow,
                                                  const double* __restrict__ DI,
                                                  double* __restrict__ Gint, int accumulate,
                                                  double* __restrict__ Gout,
                                                  const int64_t* __restrict__ goff, int nb,
                                                  int N, int Np) {
  const int NRB = Np >> 4;
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= nb * NRB) return;
  const int cb = wid % NRB, b = wid / NRB;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const double* Lb = LU + (size_t)b * Np * Np;
  const int* pb = prow + (size_t)b * Np;
  const double* DIb = DI + (size_t)b * NRB * 512;
  const int col = 16 * cb + c;

  dx4 y[NRBMAX];
#pragma unroll
  for (int rb = 0; rb < NRBMAX; ++rb) {
    if (rb < NRB) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pr = pb[16 * rb + drow64(g, v)];
        if (mode == 0)
          y[rb][v] = exp(-fmax(logD[(size_t)b * Np + pr], 0.0)) * QT[(size_t)b * Np * Np + (size_t)pr * Np + col];
        else
          y[rb][v] = R[(size_t)b * Np * Np + (size_t)pr * Np + col];
      }
    }
  }
  // forward: L y = P rhs
#pragma unroll
  for (int rb = 0; rb < NRBMAX; ++rb) {
    if (rb < NRB) {
      dx4 t = y[rb];
      const double* lrow = Lb + (size_t)pb[16 * rb + c] * Np;
#pragma unroll
      for (int kb = 0; kb < rb; ++kb) {
#pragma unroll
        for (int s = 0; s < 4; ++s) t = mfma64(-lrow[16 * kb + drow64(g, s)], y[kb][s], t);
      }
      dx4 nv = zero4d();
#pragma unroll
      for (int s = 0; s < 4; ++s) nv = mfma64(DIb[(size_t)rb * 512 + c * 16 + drow64(g, s)], t[s], nv);
      y[rb] = nv;
    }
  }
  // backward: U x = y
#pragma unroll
  for (int rb = NRBMAX - 1; rb >= 0; --rb) {
    if (rb < NRB) {
      dx4 t = y[rb];
      const double* urow = Lb + (size_t)pb[16 * rb + c] * Np;
#pragma unroll
      for (int kb = rb + 1; kb < NRBMAX; ++kb) {
        if (kb < NRB) {
#pragma unroll
          for (int s = 0; s < 4; ++s) t = mfma64(-urow[16 * kb + drow64(g, s)], y[kb][s], t);
        }
      }
      dx4 nv = zero4d();
#pragma unroll
      for (int s = 0; s < 4; ++s)
        nv = mfma64(DIb[(size_t)rb * 512 + 256 + c * 16 + drow64(g, s)], t[s], nv);
      y[rb] = nv;
    }
  }
  double* Gi = Gint + (size_t)b * Np * Np;
  double* Go = Gout ? Gout + (goff ? goff[b] : (int64_t)b * N * N) : nullptr;
#pragma unroll
  for (int rb = 0; rb < NRBMAX; ++rb) {
    if (rb < NRB) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * rb + drow64(g, v);
        double val = y[rb][v];
        if (accumulate) val += Gi[(size_t)row * Np + col];
        Gi[(size_t)row * Np + col] = val;
        if (Go && row < N && col < N) Go[(size_t)row * N + col] = val;
      }
    }
  }
}

// The same solve for Np <= 256 with 4 right-hand-side strips of one item per workgroup:
// the 16 rows of L (forward) or U (backward) that block row rb needs are staged in LDS
// once for the 4 waves (rows gathered through the pivot map, each row read coalesced),
// double-buffered, the next block row loaded into registers while the current one is
// applied: one barrier per block row.
template <int NRBMAX>
__global__ __launch_bounds__(256, 2) void lu_solve_lds_k(int mode, const double* __restrict__ QT,
                                                         const double* __restrict__ logD,
                                                         const double* __restrict__ R,
                                                         const double* __restrict__ LU,
                                                         const int* __restrict__ prow,
                                                         const double* __restrict__ DI,
                                                         double* __restrict__ Gint, int accumulate,
                                                         double* __restrict__ Gout,
                                                         const int64_t* __restrict__ goff, int nb,
                                                         int N, int Np) {
  extern __shared__ double lds[];
  const int LDL = Np + 1;                  // odd row stride: the 16 rows of a slice spread over banks
  const int NRB = Np >> 4, npg = (NRB + 3) >> 2;
  const int id = xcd_remap(blockIdx.x, nb * npg);
  if (id < 0) return;
  const int b = id / npg, tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4,
            c = lane & 15;
  const int cb = 4 * (id % npg) + w;
  const bool act = cb < NRB;
  const double* Lb = LU + (size_t)b * Np * Np;
  const int* pb = prow + (size_t)b * Np;
  const double* DIb = DI + (size_t)b * NRB * 512;
  const int col = 16 * cb + c;
  // the pivot map in LDS: the gathers below take their row indices from there
  double* dbl = lds + 2 * 16 * LDL;        // [Np] Db^-1 (right-hand side of mode 0)
  int* pl = (int*)(dbl + Np);
  for (int i = tid; i < Np; i += 256) {
    pl[i] = pb[i];
    if (mode == 0) dbl[i] = exp(-fmax(logD[(size_t)b * Np + i], 0.0));
  }
  __syncthreads();

  // right-hand side through the pivot map: all loads of a thread issued before the first
  // is used
  dx4 y[NRBMAX];
  const int colc = act ? col : 0;
#pragma unroll
  for (int rb = 0; rb < NRBMAX; ++rb) {
    y[rb] = zero4d();
    if (rb < NRB) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pr = pl[16 * rb + drow64(g, v)];
        y[rb][v] = (mode == 0 ? QT : R)[(size_t)b * Np * Np + (size_t)pr * Np + colc];
      }
    }
  }
  if (mode == 0) {
#pragma unroll
    for (int rb = 0; rb < NRBMAX; ++rb) {
      if (rb < NRB) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          y[rb][v] = dbl[pl[16 * rb + drow64(g, v)]] * y[rb][v];
        }
      }
    }
  }

  // staging of block row rb: row i of the block (factor row pl[16 rb + i]), columns
  // [lo, hi): thread tid holds column tid of each of the 16 rows
  double st[16];
  auto sload = [&](int rb, int lo, int hi) {
    const bool in = tid >= lo && tid < hi;
    const int tc = in ? tid : 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) st[i] = Lb[(size_t)pl[16 * rb + i] * Np + tc];
  };
  auto sstore = [&](int buf, int lo, int hi) {
    double* Ls = lds + buf * 16 * LDL;
    if (tid >= lo && tid < hi) {
#pragma unroll
      for (int i = 0; i < 16; ++i) Ls[i * LDL + tid] = st[i];
    }
  };

  // forward: L y = P rhs (columns 0 .. 16 rb - 1 of block row rb); the inverse of the
  // diagonal block is read one block row ahead
  double di[4], din[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) di[s] = DIb[c * 16 + drow64(g, s)];
  sload(0, 0, 0);
  for (int rb = 0; rb < NRB; ++rb) {
    if (rb + 1 < NRB) sload(rb + 1, 0, 16 * (rb + 1));
    const int rn = rb + 1 < NRB ? rb + 1 : rb;
#pragma unroll
    for (int s = 0; s < 4; ++s) din[s] = DIb[(size_t)rn * 512 + c * 16 + drow64(g, s)];
    if (act) {
      const double* Ls = lds + (rb & 1) * 16 * LDL;
#pragma unroll
      for (int k = 0; k < NRBMAX; ++k) {
        if (k == rb) {
          dx4 t = y[k];
#pragma unroll
          for (int kb = 0; kb < k; ++kb) {
#pragma unroll
            for (int s = 0; s < 4; ++s) t = mfma64(-Ls[c * LDL + 16 * kb + drow64(g, s)], y[kb][s], t);
          }
          dx4 nv = zero4d();
#pragma unroll
          for (int s = 0; s < 4; ++s) nv = mfma64(di[s], t[s], nv);
          y[k] = nv;
        }
      }
    }
    if (rb + 1 < NRB) sstore((rb + 1) & 1, 0, 16 * (rb + 1));
#pragma unroll
    for (int s = 0; s < 4; ++s) di[s] = din[s];
    __syncthreads();
  }
  // backward: U x = y (columns 16 (rb + 1) .. Np - 1 of block row rb)
#pragma unroll
  for (int s = 0; s < 4; ++s) di[s] = DIb[(size_t)(NRB - 1) * 512 + 256 + c * 16 + drow64(g, s)];
  sload(NRB - 1, Np, Np);
  for (int rb = NRB - 1; rb >= 0; --rb) {
    const int buf = (NRB - 1 - rb) & 1;
    if (rb > 0) sload(rb - 1, 16 * rb, Np);
    const int rn = rb > 0 ? rb - 1 : rb;
#pragma unroll
    for (int s = 0; s < 4; ++s) din[s] = DIb[(size_t)rn * 512 + 256 + c * 16 + drow64(g, s)];
    if (act) {
      const double* Ls = lds + buf * 16 * LDL;
#pragma unroll
      for (int k = 0; k < NRBMAX; ++k) {
        if (k == rb) {
          dx4 t = y[k];
#pragma unroll
          for (int kb = k + 1; kb < NRBMAX; ++kb) {
            if (kb < NRB) {
#pragma unroll
              for (int s = 0; s < 4; ++s) t = mfma64(-Ls[c * LDL + 16 * kb + drow64(g, s)], y[kb][s], t);
            }
          }
          dx4 nv = zero4d();
#pragma unroll
          for (int s = 0; s < 4; ++s) nv = mfma64(di[s], t[s], nv);
          y[k] = nv;
        }
      }
    }
    if (rb > 0) sstore(buf ^ 1, 16 * rb, Np);
#pragma unroll
    for (int s = 0; s < 4; ++s) di[s] = din[s];
    __syncthreads();
  }

  if (!act) return;
  double* Gi = Gint + (size_t)b * Np * Np;
  double* Go = Gout ? Gout + (goff ? goff[b] : (int64_t)b * N * N) : nullptr;
  if (accumulate) {
    // the previous G, every load in flight before the first sum (straight-line when all
    // NRBMAX row blocks exist)
    if (NRB == NRBMAX) {
      // 4 row blocks (16 loads) at a time: the scheduling barriers keep the register
      // footprint of the loads in flight within the budget
#pragma unroll
      for (int rb = 0; rb < NRBMAX; ++rb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) y[rb][v] += Gi[(size_t)(16 * rb + drow64(g, v)) * Np + col];
        if ((rb & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int rb = 0; rb < NRBMAX; ++rb)
        if (rb < NRB) {
#pragma unroll
          for (int v = 0; v < 4; ++v) y[rb][v] += Gi[(size_t)(16 * rb + drow64(g, v)) * Np + col];
        }
    }
  }
#pragma unroll
  for (int rb = 0; rb < NRBMAX; ++rb) {
    if (rb < NRB) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * rb + drow64(g, v);
        const double val = y[rb][v];
        Gi[(size_t)row * Np + col] = val;
        if (Go && row < N && col < N) Go[(size_t)row * N + col] = val;
      }
    }
  }
}

// R = Db^{-1} U^T - X G for every item, X = Db^{-1} U^T + Ds V formed while the tiles are
// staged: a batched GEMM with 64 x 64 output tiles per workgroup (4 waves of 32 x 32) and
// k steps of 16 through LDS.
constexpr int RT = 64, RKS = 16;
__global__ __launch_bounds__(256) void residual_k(const double* __restrict__ QT,
                                                  const double* __restrict__ V,
                                                  const double* __restrict__ logD,
                                                  const double* __restrict__ Gint,
                                                  double* __restrict__ R, int nb, int Np) {
  __shared__ double As[RT][RKS + 2];
  __shared__ double Bs[RKS][RT + 2];
  __shared__ double dbs[RT], dss[RT];
  const int nt = (Np + RT - 1) / RT;
  const int id = xcd_remap(blockIdx.x, nb * nt * nt);
  if (id < 0) return;
  const int tj = id % nt, ti = (id / nt) % nt, b = id / (nt * nt);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const int i0 = RT * ti, j0 = RT * tj, ro = 32 * (w >> 1), co = 32 * (w & 1);
  const size_t off = (size_t)b * Np * Np;
  if (tid < RT) {
    const int row = i0 + tid;
    const double l = row < Np ? logD[(size_t)b * Np + row] : 0.0;
    dbs[tid] = exp(-fmax(l, 0.0));
    dss[tid] = exp(fmin(l, 0.0));
  }
  __syncthreads();
  dx4 acc[2][2] = {{zero4d(), zero4d()}, {zero4d(), zero4d()}};
  const int ar = tid >> 2, ak = 4 * (tid & 3);      // A tile element group
  const int bk = tid >> 4, bj = 4 * (tid & 15);     // B tile element group
  for (int k0 = 0; k0 < Np; k0 += RKS) {
    {
      const int row = i0 + ar;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = k0 + ak + e;
        As[ar][ak + e] = row < Np ? dbs[ar] * QT[off + (size_t)row * Np + k] +
                                        dss[ar] * V[off + (size_t)row * Np + k]
                                  : 0.0;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = j0 + bj + e;
        Bs[bk][bj + e] = j < Np ? Gint[off + (size_t)(k0 + bk) * Np + j] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      double a[2], bv[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        a[h] = As[ro + 16 * h + c][4 * kk + g];
        bv[h] = Bs[4 * kk + g][co + 16 * h + c];
      }
#pragma unroll
      for (int hi = 0; hi < 2; ++hi)
#pragma unroll
        for (int hj = 0; hj < 2; ++hj) acc[hi][hj] = mfma64(a[hi], bv[hj], acc[hi][hj]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int hi = 0; hi < 2; ++hi)
#pragma unroll
    for (int hj = 0; hj < 2; ++hj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rl = ro + 16 * hi + drow64(g, v);
        const int row = i0 + rl, col = j0 + co + 16 * hj + c;
        if (row < Np && col < Np)
          R[off + (size_t)row * Np + col] = dbs[rl] * QT[off + (size_t)row * Np + col] - acc[hi][hj][v];
      }
}

template <int NRBMAX>
hipError_t run_lu(const double* QT, const double* V, const double* logD, const int* qsign,
                  const int* st_in, double* LU, int* prow, double* DI, const int* item_of,
                  double* lo, int8_t* so, int32_t* sto, int nb, int N, int Np, hipStream_t st) {
  constexpr int NT = NRBMAX <= 16 ? 512 : 256;
  constexpr int NW = NT / 64;
  if constexpr (NRBMAX <= 16) {
    // look-ahead form (panel rows all in waves 0-3)
    const size_t lds = (size_t)(2 * Np * LDY + 3 * Np + 3 * 16 * LDY + 2 * NW + 2 * LU_PANEL_WAVES * 17) *
                           sizeof(double) + (size_t)(3 * Np + NW + 4) * sizeof(int);
    hipLaunchKernelGGL(lu_la_k<NRBMAX>, dim3(nb), dim3(NT), lds, st, QT, V, logD, qsign, st_in, LU,
                       prow, DI, item_of, lo, so, sto, N, Np);
    return hipGetLastError();
  }
  const size_t lds = (size_t)(2 * Np * LDY + 3 * Np + 2 * 16 * LDY + 2 * NW + 2 * NW * 17) * sizeof(double) +
                     (size_t)(3 * Np + NW + 2) * sizeof(int);
  hipLaunchKernelGGL((lu_k<NRBMAX, NT>), dim3(nb), dim3(NT), lds, st, QT, V, logD, qsign, st_in, LU,
                     prow, DI, item_of, lo, so, sto, N, Np);
  return hipGetLastError();
}

template <int NRBMAX>
hipError_t run_solve(int mode, const double* QT, const double* logD, const double* R,
                     const double* LU, const int* prow, const double* DI, double* Gint, int acc,
                     double* Gout, const int64_t* goff, int nb, int N, int Np, hipStream_t st) {
  if (NRBMAX <= 16) {
    const int npg = (Np / 16 + 3) / 4;
    const size_t lds = (size_t)(2 * 16 * (Np + 1) + Np) * sizeof(double) + (size_t)Np * sizeof(int);
    hipLaunchKernelGGL(lu_solve_lds_k<NRBMAX <= 16 ? NRBMAX : 16>, dim3(xcd_grid(nb * npg)), dim3(256), lds,
                       st, mode, QT, logD, R, LU, prow, DI, Gint, acc, Gout, goff, nb, N, Np);
    return hipGetLastError();
  }
  const int waves = nb * (Np / 16);
  hipLaunchKernelGGL(lu_solve_k<NRBMAX>, dim3((waves + 3) / 4), dim3(256), 0, st, mode, QT, logD,
                     R, LU, prow, DI, Gint, acc, Gout, goff, nb, N, Np);
  return hipGetLastError();
}

}  // namespace

#define SLMC_NRB_DISPATCH(FN, ...)                       \
  do {                                                   \
    const int NRB_ = Np / 16;                            \
    if (NRB_ <= 4) return FN<4>(__VA_ARGS__);            \
    if (NRB_ <= 8) return FN<8>(__VA_ARGS__);            \
    if (NRB_ <= 16) return FN<16>(__VA_ARGS__);          \
    if (NRB_ <= 25) return FN<25>(__VA_ARGS__);          \
    if (NRB_ <= 32) return FN<32>(__VA_ARGS__);          \
    return hipErrorInvalidValue;                         \
  } while (0)

hipError_t launch_lu(const double* QT, const double* V, const double* logD, const int* qsign,
                     const int* st_in, double* LU, int* prow, double* DI, const int* item_of,
                     double* logdet_out, int8_t* sign_out, int32_t* status_out, int nb, int N,
                     int Np, hipStream_t st) {
  SLMC_NRB_DISPATCH(run_lu, QT, V, logD, qsign, st_in, LU, prow, DI, item_of, logdet_out,
                    sign_out, status_out, nb, N, Np, st);
}

hipError_t launch_lu_solve(int mode, const double* QT, const double* logD, const double* R,
                           const double* LU, const int* prow, const double* DI, double* Gint,
                           int accumulate, double* Gout, const int64_t* goff, int nb, int N,
                           int Np, hipStream_t st) {
  SLMC_NRB_DISPATCH(run_solve, mode, QT, logD, R, LU, prow, DI, Gint, accumulate, Gout, goff, nb,
                    N, Np, st);
}

hipError_t launch_residual(const double* QT, const double* V, const double* logD,
                           const double* Gint, double* R, int nb, int Np, hipStream_t st) {
  const int nt = (Np + RT - 1) / RT;
  hipLaunchKernelGGL(residual_k, dim3(xcd_grid(nb * nt * nt)), dim3(256), 0, st, QT, V, logD, Gint,
                     R, nb, Np);
  return hipGetLastError();
}

}  // namespace slmc
