// Symmetric effective boson model (Eq. 4 / S7 in the shifted frame, weight e^{-E_eff}),
// its checkerboard Metropolis sweeps (local updates of the cumulative proposal, main text
// "SLMC" and the last paragraph of SM Sec. IV), the full log-weight -dtau S_Bose + 2 log|det M| (SM Eq. S2)
// and the cumulative-update acceptance (Eq. 6).
//
// Sweep design: one workgroup per chain holds the chain's whole field in LDS when it fits
// (N Ltau doubles <= 144 KB; e.g. 12x12x120), otherwise works on it in place in global
// memory (L2-resident); every colour phase updates its sites in parallel (no two sites of
// a phase share a coupling) and a barrier separates phases.  Random numbers come from the
// Philox4x32-10 of philox.h.
#include "common.h"
#include "launch.h"
#include "philox.h"

namespace slmc {

namespace {

__device__ __forceinline__ int wrap(int a, int L) { a %= L; return a < 0 ? a + L : a; }
// periodic wrap of -L <= a < 2 L without a division
__device__ __forceinline__ int wrap1(int a, int L) { return a < 0 ? a + L : (a >= L ? a - L : a); }

__device__ __forceinline__ double f4(double y, double a) {
  return 0.25 * y * y * y * y - 0.5 * a * a * y * y;
}
__device__ __forceinline__ double f6(double y, double a) {
  const double y2 = y * y;
  return y2 * y2 * y2 / 6.0 - 0.25 * a * a * y2 * y2;
}

// sum over the bonds of range r touching site (ix, iy) of slice xs (both directions)
__device__ __forceinline__ double nbr_sum(const double* xs, int ix, int iy, int Lx, int Ly, int r) {
  int d[2][2];
  if (r == 0) { d[0][0] = 1; d[0][1] = 0; d[1][0] = 0; d[1][1] = 1; }
  else if (r == 1) { d[0][0] = 1; d[0][1] = 1; d[1][0] = 1; d[1][1] = -1; }
  else { d[0][0] = 2; d[0][1] = 0; d[1][0] = 0; d[1][1] = 2; }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    s += xs[wrap1(ix + d[k][0], Lx) + Lx * wrap1(iy + d[k][1], Ly)];
    s += xs[wrap1(ix - d[k][0], Lx) + Lx * wrap1(iy - d[k][1], Ly)];
  }
  return s;
}

// E_eff(x with x[l][i] -> xn) - E_eff(x): the terms touching (i, l)
__device__ __forceinline__ double local_delta(const double* x, int N, int Lx, int Ly, int Ltau,
                                              const EffParams& p, int ix, int iy, int l,
                                              double xn) {
  const int i = ix + Lx * iy;
  const double xo = x[l * N + i];
  const double xp = x[(l + 1 == Ltau ? 0 : l + 1) * N + i];
  const double xm = x[(l == 0 ? Ltau - 1 : l - 1) * N + i];
  const double d = xn - xo;
  double de = p.Jk * ((xp - xn) * (xp - xn) - (xp - xo) * (xp - xo) + (xn - xm) * (xn - xm) -
                      (xo - xm) * (xo - xm));
  de += p.J2 * (xn * xn - xo * xo);
  de += p.Jp * (f4(xn, p.a) - f4(xo, p.a));
  de += p.Jp6 * (f6(xn, p.a) - f6(xo, p.a));
  const double* xs = x + l * N;
  if (p.Js0 != 0.0) de += p.Js0 * d * nbr_sum(xs, ix, iy, Lx, Ly, 0);
  if (p.Js1 != 0.0) de += p.Js1 * d * nbr_sum(xs, ix, iy, Lx, Ly, 1);
  if (p.Js2 != 0.0) de += p.Js2 * d * nbr_sum(xs, ix, iy, Lx, Ly, 2);
  de += p.Jt * d * (xp + xm);
  return de;
}

// log(u01(r)) < z, decided as the FP64 comparison decides it: the FP32 logarithm (hardware
// log2, error below 4e-6 absolute for u >= 2^-32, plus 6e-8 from rounding u to FP32)
// settles every case farther than 1e-4 from the boundary, and only the rest takes the
// FP64 logarithm (a long software sequence, most of a site update's arithmetic otherwise).
__device__ __forceinline__ bool log_u_below(uint32_t r, double z) {
  const float lf = __logf((float)u01(r));
  if ((double)lf < z - 1e-4) return true;
  if ((double)lf > z + 1e-4) return false;
  return log(u01(r)) < z;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  T s = 0;
  for (int k = 0; k < nw; ++k) s += red[k];
  return s;
}

// ------------------------------------------------------------------------------ energy

// One workgroup of 1024 threads per chain (a fixed summation order, so the energy is
// reproducible); the neighbour offsets of every site come from tables in LDS and the
// (slice, site) pair of a thread advances by a constant step, so the loop does no integer
// division.
constexpr int EN_THREADS = 1024;
__global__ __launch_bounds__(EN_THREADS) void eff_energy_k(const double* __restrict__ x, int N, int Lx,
                                                           int Ly, int Ltau, EffParams p,
                                                           double* __restrict__ e) {
  __shared__ double red[16];
  __shared__ int nbr[6 * 448];   // +x, +y, +x+y, +x-y, +2x, +2y (N <= 448)
  const int ch = blockIdx.x;
  const double* xc = x + (size_t)ch * N * Ltau;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int ix = i % Lx, iy = i / Lx;
    nbr[6 * i + 0] = wrap(ix + 1, Lx) + Lx * iy;
    nbr[6 * i + 1] = ix + Lx * wrap(iy + 1, Ly);
    nbr[6 * i + 2] = wrap(ix + 1, Lx) + Lx * wrap(iy + 1, Ly);
    nbr[6 * i + 3] = wrap(ix + 1, Lx) + Lx * wrap(iy - 1, Ly);
    nbr[6 * i + 4] = wrap(ix + 2, Lx) + Lx * iy;
    nbr[6 * i + 5] = ix + Lx * wrap(iy + 2, Ly);
  }
  __syncthreads();
  const int dl = blockDim.x / N, di = blockDim.x - dl * N;
  int l = threadIdx.x / N, i = threadIdx.x - l * N;
  double s = 0.0;
#pragma unroll 4
  for (int idx = threadIdx.x; idx < N * Ltau; idx += blockDim.x) {
    const double* xs = xc + (size_t)l * N;
    const double y = xs[i];
    const double yn = xc[(size_t)(l + 1 == Ltau ? 0 : l + 1) * N + i];
    double t = p.Jk * (yn - y) * (yn - y) + p.J2 * y * y + p.Jp * f4(y, p.a) + p.Jp6 * f6(y, p.a);
    // bonds counted once: from site i in the + directions of each range
    if (p.Js0 != 0.0) t += p.Js0 * y * (xs[nbr[6 * i + 0]] + xs[nbr[6 * i + 1]]);
    if (p.Js1 != 0.0) t += p.Js1 * y * (xs[nbr[6 * i + 2]] + xs[nbr[6 * i + 3]]);
    if (p.Js2 != 0.0) t += p.Js2 * y * (xs[nbr[6 * i + 4]] + xs[nbr[6 * i + 5]]);
    t += p.Jt * y * yn;
    s += t;
    i += di;
    l += dl;
    if (i >= N) { i -= N; ++l; }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) e[ch] = s;
}

// ------------------------------------------------------------------------------ sweep

template <bool IN_LDS>
__global__ __launch_bounds__(1024) void eff_sweep_k(double* __restrict__ x, int N, int Lx, int Ly,
                                                    int Ltau, EffParams p, int mod, int n_sweeps,
                                                    uint32_t k0, uint32_t k1, uint32_t prop_arg,
                                                    const uint64_t* __restrict__ prop_dev,
                                                    int64_t* __restrict__ nacc) {
  // the proposal index comes from the argument, or from device memory (replayable graphs)
  const uint32_t prop = prop_dev ? (uint32_t)(*prop_dev & 0xFFFFFFFFu) : prop_arg;
  extern __shared__ double lds[];
  __shared__ int64_t redi[16];
  const int ch = blockIdx.x;
  const int n = N * Ltau;
  double* xg = x + (size_t)ch * n;
  double* xs = IN_LDS ? lds : xg;
  if (IN_LDS) {
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) xs[idx] = xg[idx];
    __syncthreads();
  }
  const int m2 = mod * mod, P = 2 * m2;
  const int nx = Lx / mod, ny = Ly / mod, per_l = nx * ny, cnt = (Ltau / 2) * per_l;
  const bool forward = proposal_forward(prop, (uint32_t)ch, k0, k1);
  // Work item t = lq per_l + ry nx + rx of a phase is the site (sx + mod rx, sy + mod ry) of
  // slice tc + 2 lq.  A thread's items are t0, t0 + blockDim, ..., the same in every phase:
  // their (lq, ry, rx) start from t0 and advance by blockDim's (dq, dry, drx) with carries,
  // so the site loop does no integer division.
  const int t0 = threadIdx.x, bd = blockDim.x;
  const int lq0 = t0 / per_l, ry0 = (t0 - lq0 * per_l) / nx, rx0 = t0 - lq0 * per_l - ry0 * nx;
  const int dq = bd / per_l, dry = (bd - dq * per_l) / nx, drx = bd - dq * per_l - dry * nx;
  int64_t acc = 0;
  for (int s = 0; s < n_sweeps; ++s) {
    for (int pi = 0; pi < P; ++pi) {
      const int ph = forward ? pi : P - 1 - pi;
      const int tc = ph / m2, sc = ph - tc * m2, sx = sc % mod, sy = sc / mod;
      int lq = lq0, ry = ry0, rx = rx0;
      for (int t = t0; t < cnt; t += bd) {
        const int l = tc + 2 * lq;
        const int ix = sx + mod * rx, iy = sy + mod * ry;
        const int i = ix + Lx * iy;
        const U4 r = philox(U4{(uint32_t)(i + N * l), (uint32_t)s, prop, (uint32_t)ch}, k0, k1);
        const double xo = xs[l * N + i];
        const double xn = xo + p.delta * (2.0 * u01(r.x) - 1.0);
        const double de = local_delta(xs, N, Lx, Ly, Ltau, p, ix, iy, l, xn);
        if (log_u_below(r.y, -de)) {
          xs[l * N + i] = xn;
          ++acc;
        }
        rx += drx;
        ry += dry;
        lq += dq;
        if (rx >= nx) { rx -= nx; ++ry; }
        if (ry >= ny) { ry -= ny; ++lq; }
      }
      if (!IN_LDS) __threadfence_block();
      __syncthreads();
    }
  }
  if (IN_LDS) {
    for (int idx = threadIdx.x; idx < n; idx += blockDim.x) xg[idx] = xs[idx];
  }
  acc = block_sum(acc, redi);
  if (threadIdx.x == 0) nacc[ch] = acc;
}

// ------------------------------------------------------------------------------ weight

__global__ __launch_bounds__(EN_THREADS) void log_weight_k(const double* __restrict__ x,
                                                    const double* __restrict__ logdet, int N,
                                                    int Ltau, double lam, double omega0,
                                                    double dtau, double c_kin,
                                                    double* __restrict__ logw) {
  __shared__ double red[16];
  const int ch = blockIdx.x;
  const double* xc = x + (size_t)ch * N * Ltau;
  double pot = 0.0, kin = 0.0;
  const int dl = blockDim.x / N, di = blockDim.x - dl * N;
  int l = threadIdx.x / N, i = threadIdx.x - l * N;
#pragma unroll 4
  for (int idx = threadIdx.x; idx < N * Ltau; idx += blockDim.x) {
    const double y = xc[idx];
    const double dy = xc[(size_t)(l + 1 == Ltau ? 0 : l + 1) * N + i] - y;
    pot += 0.5 * omega0 * omega0 * y * y - lam * y;
    kin += dy * dy;
    i += di;
    l += dl;
    if (i >= N) { i -= N; ++l; }
  }
  pot = block_sum(pot, red);
  kin = block_sum(kin, red);
  if (threadIdx.x == 0) {
    const double sb = pot + c_kin * kin / (dtau * dtau);
    logw[ch] = -dtau * sb + 2.0 * logdet[ch];
  }
}

__global__ __launch_bounds__(256) void accept_k(double* __restrict__ x_cur,
                                                const double* __restrict__ x_prop,
                                                double* __restrict__ logw_cur,
                                                double* __restrict__ eeff_cur,
                                                const double* __restrict__ logw_prop,
                                                const double* __restrict__ eeff_prop,
                                                int64_t nelem, uint32_t k0, uint32_t k1,
                                                uint32_t tag, uint32_t prop_arg,
                                                const uint64_t* __restrict__ prop_dev,
                                                uint8_t* __restrict__ accepted,
                                                double* __restrict__ log_ratio) {
  const uint32_t prop = prop_dev ? (uint32_t)(*prop_dev & 0xFFFFFFFFu) : prop_arg;
  __shared__ int dec;
  const int ch = blockIdx.x;
  if (threadIdx.x == 0) {
    const double lr = (logw_prop[ch] - logw_cur[ch]) + (eeff_prop[ch] - eeff_cur[ch]);
    const U4 r = philox(U4{0xFFFFFFFFu, tag, prop, (uint32_t)ch}, k0, k1);
    const int a = log(u01(r.x)) < lr;
    log_ratio[ch] = lr;
    accepted[ch] = (uint8_t)a;
    if (a) { logw_cur[ch] = logw_prop[ch]; eeff_cur[ch] = eeff_prop[ch]; }
    dec = a;
  }
  __syncthreads();
  if (dec) {
    const double* src = x_prop + (size_t)ch * nelem;
    double* dst = x_cur + (size_t)ch * nelem;
    for (int64_t e = threadIdx.x; e < nelem; e += blockDim.x) dst[e] = src[e];
  }
}

__global__ void incr_u64_k(uint64_t* c) {
  if (threadIdx.x == 0) *c += 1;
}

}  // namespace

hipError_t launch_incr_u64(uint64_t* c, hipStream_t st) {
  hipLaunchKernelGGL(incr_u64_k, dim3(1), dim3(64), 0, st, c);
  return hipGetLastError();
}

hipError_t launch_eff_energy(const double* x, int nch, int Lx, int Ly, int Ltau, EffParams p,
                             double* e, hipStream_t st) {
  hipLaunchKernelGGL(eff_energy_k, dim3(nch), dim3(EN_THREADS), 0, st, x, Lx * Ly, Lx, Ly, Ltau, p, e);
  return hipGetLastError();
}

hipError_t launch_eff_sweep(double* x, int nch, int Lx, int Ly, int Ltau, EffParams p, int mod,
                            int n_sweeps, uint64_t seed, uint64_t proposal, int64_t* nacc,
                            hipStream_t st, const uint64_t* prop_dev) {
  const int N = Lx * Ly;
  const size_t bytes = (size_t)N * Ltau * sizeof(double);
  const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
  const uint32_t pr = (uint32_t)(proposal & 0xFFFFFFFFu);
  if (bytes <= 144 * 1024) {
    hipLaunchKernelGGL(eff_sweep_k<true>, dim3(nch), dim3(1024), bytes, st, x, N, Lx, Ly, Ltau, p,
                       mod, n_sweeps, k0, k1, pr, prop_dev, nacc);
  } else {
    hipLaunchKernelGGL(eff_sweep_k<false>, dim3(nch), dim3(1024), 0, st, x, N, Lx, Ly, Ltau, p,
                       mod, n_sweeps, k0, k1, pr, prop_dev, nacc);
  }
  return hipGetLastError();
}

hipError_t launch_log_weight(const double* x, const double* logdet, int nch, int N, int Ltau,
                             double lam, double omega0, double dtau, double c_kin, double* logw,
                             hipStream_t st) {
  hipLaunchKernelGGL(log_weight_k, dim3(nch), dim3(EN_THREADS), 0, st, x, logdet, N, Ltau, lam, omega0,
                     dtau, c_kin, logw);
  return hipGetLastError();
}

hipError_t launch_accept(double* x_cur, const double* x_prop, double* logw_cur, double* eeff_cur,
                         const double* logw_prop, const double* eeff_prop, int nch,
                         int64_t nelem, uint64_t seed, uint64_t proposal, uint8_t* accepted,
                         double* log_ratio, hipStream_t st, uint32_t tag,
                         const uint64_t* prop_dev) {
  const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
  hipLaunchKernelGGL(accept_k, dim3(nch), dim3(256), 0, st, x_cur, x_prop, logw_cur, eeff_cur,
                     logw_prop, eeff_prop, nelem, k0, k1, tag, (uint32_t)(proposal & 0xFFFFFFFFu),
                     prop_dev, accepted, log_ratio);
  return hipGetLastError();
}

}  // namespace slmc
