// Training the effective model (main text Eq. 5, SM Sec. III): the features of every
// configuration and the multi-linear regression of ln w onto them.
//
// E_eff is linear in its 8 coefficients, E_eff = sum_t J_t F_t(x) with
// F = (sum (x_{l+1}-x_l)^2, sum x^2, sum f4, sum f6, sum_NN x_i x_j, sum_NNN, sum_3rd,
// sum x_l x_{l+1}).  The fit solves the least-squares problem ln w ~ E0 - sum J_t F_t over
// the masked terms with a Householder QR of the tall design matrix (columns scaled to unit
// maximum first), in one workgroup: every column operation is a reduction over the
// configurations in a fixed order, so the result does not depend on scheduling.
#include "common.h"
#include "launch.h"

namespace slmc {

namespace {

constexpr int TR_THREADS = 1024;

__device__ __forceinline__ double tr_f4(double y, double a) { return 0.25 * y * y * y * y - 0.5 * a * a * y * y; }
__device__ __forceinline__ double tr_f6(double y, double a) {
  const double y2 = y * y;
  return y2 * y2 * y2 / 6.0 - 0.25 * a * a * y2 * y2;
}

// sum over the block in a fixed order (wave sums by xor butterflies, then waves in order)
__device__ __forceinline__ double tr_sum(double v, double* red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
  return s;
}

// F[c][t] for every configuration c (one workgroup each)
__global__ __launch_bounds__(TR_THREADS) void features_k(const double* __restrict__ x, int Lx, int Ly,
                                                         int Ltau, double a, double* __restrict__ F) {
  __shared__ double red[TR_THREADS / 64];
  const int c = blockIdx.x, N = Lx * Ly;
  const double* xc = x + (int64_t)c * N * Ltau;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int e = threadIdx.x; e < N * Ltau; e += TR_THREADS) {
    const int l = e / N, i = e - l * N, ix = i % Lx, iy = i / Lx;
    const double* xs = xc + (int64_t)l * N;
    const double y = xs[i], yn = xc[(int64_t)(l + 1 == Ltau ? 0 : l + 1) * N + i];
    const int xp = ix + 1 == Lx ? 0 : ix + 1, yp = iy + 1 == Ly ? 0 : iy + 1;
    const int ym = iy == 0 ? Ly - 1 : iy - 1;
    const int xp2 = (ix + 2) % Lx, yp2 = (iy + 2) % Ly;
    s[0] += (yn - y) * (yn - y);
    s[1] += y * y;
    s[2] += tr_f4(y, a);
    s[3] += tr_f6(y, a);
    s[4] += y * (xs[xp + Lx * iy] + xs[ix + Lx * yp]);
    s[5] += y * (xs[xp + Lx * yp] + xs[xp + Lx * ym]);
    s[6] += y * (xs[xp2 + Lx * iy] + xs[ix + Lx * yp2]);
    s[7] += y * yn;
  }
  for (int t = 0; t < 8; ++t) {
    const double v = tr_sum(s[t], red);
    if (threadIdx.x == 0) F[(int64_t)c * 8 + t] = v;
  }
}

// Least squares of y ~ A coef with A = [1, -F_t (t in mask)] (n x p, p <= 9), Householder QR.
// A is built column-major in Aw [p][n]; out[0] = E0, out[1 + t] = J_t (0 outside the mask).
__global__ __launch_bounds__(TR_THREADS) void fit_k(const double* __restrict__ F,
                                                    const double* __restrict__ logw, int n,
                                                    int mask, double* __restrict__ Aw,
                                                    double* __restrict__ yw, double* __restrict__ out) {
  __shared__ double red[TR_THREADS / 64];
  __shared__ double R[9][10], sc[9];
  __shared__ int col_t[9];
  __shared__ int p;
  const int tid = threadIdx.x;
  if (tid == 0) {
    int q = 1;
    col_t[0] = -1;
    for (int t = 0; t < 8; ++t)
      if (mask & (1 << t)) col_t[q++] = t;
    p = q;
  }
  __syncthreads();
  const int P = p;
  // columns and their scales (unit maximum)
  for (int j = 0; j < P; ++j) {
    double mx = 0.0;
    for (int c = tid; c < n; c += TR_THREADS) {
      const double v = col_t[j] < 0 ? 1.0 : -F[(int64_t)c * 8 + col_t[j]];
      Aw[(int64_t)j * n + c] = v;
      mx = fmax(mx, fabs(v));
    }
    for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int k = 0; k < TR_THREADS / 64; ++k) m = fmax(m, red[k]);
      sc[j] = m > 0.0 ? 1.0 / m : 1.0;
    }
    __syncthreads();
    for (int c = tid; c < n; c += TR_THREADS) Aw[(int64_t)j * n + c] *= sc[j];
  }
  for (int c = tid; c < n; c += TR_THREADS) yw[c] = logw[c];
  __threadfence_block();
  __syncthreads();
  // Householder: column k, rows k .. n-1
  for (int k = 0; k < P; ++k) {
    double* ak = Aw + (int64_t)k * n;
    double s2 = 0.0;
    for (int c = k + tid; c < n; c += TR_THREADS) s2 += ak[c] * ak[c];
    const double sig = tr_sum(s2, red);
    const double x1 = ak[k];
    const double alpha = x1 > 0.0 ? -sqrt(sig) : sqrt(sig);
    const double vtv = 2.0 * alpha * (alpha - x1);      // |x - alpha e1|^2
    __syncthreads();
    if (tid == 0) {
      ak[k] = x1 - alpha;                                // v, kept in the column
      R[k][k] = alpha;
    }
    __threadfence_block();
    __syncthreads();
    // apply H = I - 2 v v^T / v^T v to the later columns and to y
    for (int j = k + 1; j <= P; ++j) {
      double* aj = j < P ? Aw + (int64_t)j * n : yw;
      double d = 0.0;
      for (int c = k + tid; c < n; c += TR_THREADS) d += ak[c] * aj[c];
      const double w = tr_sum(d, red);
      const double f = vtv > 0.0 ? 2.0 * w / vtv : 0.0;
      for (int c = k + tid; c < n; c += TR_THREADS) aj[c] -= f * ak[c];
      __threadfence_block();
      __syncthreads();
      if (tid == 0) R[k][j] = aj[k];
      __syncthreads();
    }
  }
  if (tid == 0) {
    double coef[9];
    for (int k = P - 1; k >= 0; --k) {
      double s = R[k][P];
      for (int j = k + 1; j < P; ++j) s -= R[k][j] * coef[j];
      coef[k] = s / R[k][k];
    }
    for (int t = 0; t < 9; ++t) out[t] = 0.0;
    for (int j = 0; j < P; ++j) out[col_t[j] + 1] = coef[j] * sc[j];
  }
}

}  // namespace

hipError_t launch_features(const double* x, int n, int Lx, int Ly, int Ltau, double a, double* F,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(features_k, dim3(n), dim3(TR_THREADS), 0, st, x, Lx, Ly, Ltau, a, F);
  return hipGetLastError();
}

hipError_t launch_fit(const double* F, const double* logw, int n, int mask, double* Aw, double* yw,
                      double* out, hipStream_t st) {
  hipLaunchKernelGGL(fit_k, dim3(1), dim3(TR_THREADS), 0, st, F, logw, n, mask, Aw, yw, out);
  return hipGetLastError();
}

}  // namespace slmc
