// DQMC comparison updates (SM Sec. I, Eqs. S4-S6): the local update of one phonon field
// with its O(1) determinant ratio and O(N^2) Sherman-Morrison update of the Green's
// function, and the block update that reflects a whole time column.
//
// With B_l = e^{-dtau K} diag(v_l) a change of x[l][i] multiplies B_l on the right by
// I + Delta (Delta_ii = expm1(-dtau lam dx)); with G = G after slice l-1 the spin ratio is
// R = 1 + (1 - G_ii) Delta_ii and the update is G' = G - (I - G) e_i (Delta_ii / R) e_i^T G.
// Both spins are equal: the fermion ratio is R^2.
//
// Local sweep design: one workgroup per chain walks the N sites of a slice in order (the
// updates do not commute); above N = 64 with delayed updates: the accepted sites are kept as a rank-m
// correction, G = G0 - sum_t a_t b_t^T (a_t = (e_i - G e_i) Delta_ii / R and b_t = G^T e_i
// of the current G when site t was accepted), in LDS, while G0 stays in device memory
// (cache-resident, 8 N^2 bytes per chain).  Per site thread 0 forms G_ii = G0_ii - sum_t
// a_t[i] b_t[i] (a sum kept per site as the rows are added), draws the move and decides; on accept every thread forms its entries of
// the column and row of site i from G0 (prefetched one site ahead) and the correction.
// Every KM accepts, and at the end of the slice, the correction is applied to G0 as one
// rank-KM product on the matrix cores.  One barrier per rejected site, two per accepted
// one, and 1/KM of the passes over G of rank-one updates.
#include "common.h"
#include "launch.h"
#include "philox.h"

namespace slmc {

namespace {

constexpr int DQ_THREADS = 1024;
constexpr int DQ_WAVES = DQ_THREADS / 64;

// Small lattices (N <= 64): the rank-one update of G right after each accepted site (G is
// 32 KB at most, four elements per thread): fewer steps per site than the delayed form.
__global__ __launch_bounds__(DQ_THREADS) void dqmc_slice_r1_k(double* __restrict__ G, int64_t sg,
                                                           double* __restrict__ x, int N, int Ltau, int l,
                                                           double dtau, double lam, double omega0,
                                                           double c_kin, double delta, uint32_t k0,
                                                           uint32_t k1, uint32_t sweep,
                                                           int64_t* __restrict__ nacc) {
  __shared__ double col[64], row[64];
  __shared__ double coef;
  __shared__ int take;
  const int ch = blockIdx.x, tid = threadIdx.x;
  double* Gc = G + (int64_t)ch * sg;
  double* xc = x + (int64_t)ch * N * Ltau;
  const int lp = l + 1 == Ltau ? 0 : l + 1, lm = l == 0 ? Ltau - 1 : l - 1;
  int64_t acc = 0;
  for (int i = 0; i < N; ++i) {
    if (tid == 0) {
      const U4 r = philox(U4{(uint32_t)(i + N * l), 0xC0000000u, sweep, (uint32_t)ch}, k0, k1);
      const double dx = delta * (2.0 * u01(r.x) - 1.0);
      const double xo = xc[(int64_t)l * N + i], xn = xo + dx;
      const double xp = xc[(int64_t)lp * N + i], xm = xc[(int64_t)lm * N + i];
      const double d = expm1(-dtau * lam * dx);
      const double R = 1.0 + (1.0 - Gc[(int64_t)i * N + i]) * d;
      const double pot = 0.5 * omega0 * omega0 * (xn * xn - xo * xo) - lam * (xn - xo);
      const double kin = (xp - xn) * (xp - xn) + (xn - xm) * (xn - xm) - (xp - xo) * (xp - xo) -
                         (xo - xm) * (xo - xm);
      const double log_r = 2.0 * log(fabs(R)) - dtau * (pot + c_kin * kin / (dtau * dtau));
      const int a = log(u01(r.y)) < log_r;
      take = a;
      coef = d / R;
      if (a) {
        xc[(int64_t)l * N + i] = xn;
        ++acc;
      }
    }
    __syncthreads();
    const int a = take;
    const double cf = coef;
    // every thread holds the decision before thread 0 may write the next one
    __syncthreads();
    if (!a) continue;
    for (int k = tid; k < N; k += DQ_THREADS) {
      col[k] = (k == i ? 1.0 : 0.0) - Gc[(int64_t)k * N + i];
      row[k] = Gc[(int64_t)i * N + k];
    }
    __syncthreads();
    for (int e = tid; e < N * N; e += DQ_THREADS) {
      const int k = e / N, j = e - k * N;
      Gc[e] -= (col[k] * row[j]) * cf;
    }
    __threadfence_block();
    __syncthreads();
  }
  if (tid == 0) nacc[ch] += acc;
}

template <int KM>
__global__ __launch_bounds__(DQ_THREADS) void dqmc_slice_k(double* __restrict__ G, int64_t sg,
                                                           double* __restrict__ x, int N, int Np,
                                                           int Ltau, int l, double dtau, double lam,
                                                           double omega0, double c_kin, double delta,
                                                           uint32_t k0, uint32_t k1, uint32_t sweep,
                                                           int64_t* __restrict__ nacc) {
  extern __shared__ double lds[];
  double* A = lds;                 // [KM][Np] a_t (rows >= m and columns >= N are zero)
  double* B = A + KM * Np;         // [KM][Np] b_t
  double* dg = B + KM * Np;        // [Np] diagonal of G0
  double* dgc = dg + Np;           // [Np] sum_t a_t[k] b_t[k], kept as the rows are added
  __shared__ double coef[2];
  __shared__ int take[2];
  const int ch = blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4,
            c = lane & 15;
  double* Gc = G + (int64_t)ch * sg;
  double* xc = x + (int64_t)ch * N * Ltau;
  const int lp = l + 1 == Ltau ? 0 : l + 1, lm = l == 0 ? Ltau - 1 : l - 1;
  for (int e = tid; e < 2 * KM * Np; e += DQ_THREADS) A[e] = 0.0;
  for (int k = tid; k < N; k += DQ_THREADS) {
    dg[k] = Gc[(int64_t)k * N + k];
    dgc[k] = 0.0;
  }
  __syncthreads();
  // G0 -= A^T B over the first m4 rows (m rounded up to 4; the rows beyond m are zero):
  // 16x16 output tiles, one wave per tile, k steps of 4 on v_mfma_f64_16x16x4f64; then the
  // diagonal of G0 is reloaded and the used rows of A and B cleared
  auto flush = [&](int m) {
    const int m4 = (m + 3) & ~3, nt = Np >> 4;
    for (int tile = w; tile < nt * nt; tile += DQ_WAVES) {
      const int r0 = 16 * (tile / nt), c0 = 16 * (tile - (tile / nt) * nt);
      dx4 acc = zero4d();
      for (int t0 = 0; t0 < m4; t0 += 4)
        acc = mfma64(A[(t0 + g) * Np + r0 + c], B[(t0 + g) * Np + c0 + c], acc);
      const int col = c0 + c;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + drow64(g, v);
        if (row < N && col < N) Gc[(int64_t)row * N + col] -= acc[v];
      }
    }
    __threadfence_block();
    __syncthreads();
    for (int k = tid; k < N; k += DQ_THREADS) {
      dg[k] = Gc[(int64_t)k * N + k];
      dgc[k] = 0.0;
    }
    for (int e = tid; e < m * Np; e += DQ_THREADS) { A[e] = 0.0; B[e] = 0.0; }
    __syncthreads();
  };
  int64_t acc = 0;
  int m = 0;
  // this thread's entries of column i and row i of G0, loaded one site ahead
  double pc = 0.0, pr = 0.0;
  if (tid < N) { pc = Gc[(int64_t)tid * N]; pr = Gc[tid]; }
  for (int i = 0; i < N; ++i) {
    if (tid == 0) {
      const double gii = dg[i] - dgc[i];
      const U4 r = philox(U4{(uint32_t)(i + N * l), 0xC0000000u, sweep, (uint32_t)ch}, k0, k1);
      const double dx = delta * (2.0 * u01(r.x) - 1.0);
      const double xo = xc[(int64_t)l * N + i], xn = xo + dx;
      const double xp = xc[(int64_t)lp * N + i], xm = xc[(int64_t)lm * N + i];
      const double d = expm1(-dtau * lam * dx);
      const double R = 1.0 + (1.0 - gii) * d;
      const double pot = 0.5 * omega0 * omega0 * (xn * xn - xo * xo) - lam * (xn - xo);
      const double kin = (xp - xn) * (xp - xn) + (xn - xm) * (xn - xm) - (xp - xo) * (xp - xo) -
                         (xo - xm) * (xo - xm);
      const double log_r = 2.0 * log(fabs(R)) - dtau * (pot + c_kin * kin / (dtau * dtau));
      const int a = log(u01(r.y)) < log_r;
      // slot i & 1: every thread has read slot i & 1 of site i - 2 before the barrier of
      // site i - 1, which thread 0 has passed
      take[i & 1] = a;
      coef[i & 1] = d / R;
      if (a) {
        xc[(int64_t)l * N + i] = xn;
        ++acc;
      }
    }
    __syncthreads();
    if (take[i & 1]) {
      const double cf = coef[i & 1];
      if (tid < N) {
        double sc = 0.0, sr = 0.0;
        for (int t = 0; t < m; ++t) {
          sc += A[t * Np + tid] * B[t * Np + i];
          sr += A[t * Np + i] * B[t * Np + tid];
        }
        const double av = ((tid == i ? 1.0 : 0.0) - (pc - sc)) * cf, bv = pr - sr;
        A[m * Np + tid] = av;
        B[m * Np + tid] = bv;
        dgc[tid] += av * bv;
      }
      ++m;
      __syncthreads();
      if (m == KM) {
        flush(m);
        m = 0;
      }
    }
    if (i + 1 < N && tid < N) {
      pc = Gc[(int64_t)tid * N + i + 1];
      pr = Gc[(int64_t)(i + 1) * N + tid];
    }
  }
  if (m > 0) flush(m);
  if (tid == 0) nacc[ch] += acc;
}

// x_prop = x_cur with column s negated; s = floor(r N / 2^32) from Philox word 0 at
// (0xFFFFFFFB, 0xFFFFFFFC, ctr, chain)
__global__ __launch_bounds__(256) void reflect_column_k(const double* __restrict__ x_cur,
                                                        double* __restrict__ x_prop, int N, int Ltau,
                                                        uint32_t k0, uint32_t k1, uint32_t ctr) {
  const int ch = blockIdx.x;
  const U4 r = philox(U4{0xFFFFFFFBu, 0xFFFFFFFCu, ctr, (uint32_t)ch}, k0, k1);
  const int s = (int)(((uint64_t)r.x * (uint64_t)N) >> 32);
  const int64_t n = (int64_t)N * Ltau, off = (int64_t)ch * n;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int i = (int)(e % N);
    const double v = x_cur[off + e];
    x_prop[off + e] = i == s ? -v : v;
  }
}

__global__ void fill_i64_k(int64_t* dst, int n, int64_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

__global__ void add_accepted_k(const uint8_t* __restrict__ a, int64_t* __restrict__ nacc, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) nacc[i] += a[i];
}

}  // namespace

hipError_t launch_dqmc_slice(double* G, int64_t sg, double* x, int nch, int N, int Ltau, int l,
                             double dtau, double lam, double omega0, double c_kin, double delta,
                             uint64_t seed, uint64_t sweep, int64_t* nacc, hipStream_t st) {
  if (N > 448) return hipErrorInvalidValue;
  const int Np = (N + 15) / 16 * 16;
  const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
  if (N <= 64) {
    hipLaunchKernelGGL(dqmc_slice_r1_k, dim3(nch), dim3(DQ_THREADS), 0, st, G, sg, x, N, Ltau, l, dtau, lam,
                       omega0, c_kin, delta, k0, k1, (uint32_t)(sweep & 0xFFFFFFFFu), nacc);
    return hipGetLastError();
  }
  // 32 delayed updates while A, B and the two diagonals fit in 140 KB of LDS, else 16
  if ((size_t)(2 * 32 + 2) * Np * sizeof(double) <= 140 * 1024) {
    const size_t lds = (size_t)(2 * 32 + 2) * Np * sizeof(double);
    hipLaunchKernelGGL(dqmc_slice_k<32>, dim3(nch), dim3(DQ_THREADS), lds, st, G, sg, x, N, Np, Ltau, l,
                       dtau, lam, omega0, c_kin, delta, k0, k1, (uint32_t)(sweep & 0xFFFFFFFFu), nacc);
  } else {
    const size_t lds = (size_t)(2 * 16 + 2) * Np * sizeof(double);
    hipLaunchKernelGGL(dqmc_slice_k<16>, dim3(nch), dim3(DQ_THREADS), lds, st, G, sg, x, N, Np, Ltau, l,
                       dtau, lam, omega0, c_kin, delta, k0, k1, (uint32_t)(sweep & 0xFFFFFFFFu), nacc);
  }
  return hipGetLastError();
}

hipError_t launch_reflect_column(const double* x_cur, double* x_prop, int nch, int N, int Ltau,
                                 uint64_t seed, uint32_t ctr, hipStream_t st) {
  const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
  hipLaunchKernelGGL(reflect_column_k, dim3(nch), dim3(256), 0, st, x_cur, x_prop, N, Ltau, k0, k1, ctr);
  return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t* dst, int n, int64_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i64_k, dim3((n + 255) / 256), dim3(256), 0, st, dst, n, v);
  return hipGetLastError();
}

hipError_t launch_add_accepted(const uint8_t* a, int64_t* nacc, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(add_accepted_k, dim3((n + 255) / 256), dim3(256), 0, st, a, nacc, n);
  return hipGetLastError();
}

}  // namespace slmc
