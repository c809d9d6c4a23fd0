// Modified Wolff cluster moves of the symmetric effective model (SM Sec. IV, Eq. S8).
//
// A cluster lives in the spatial plane; each of its sites carries its whole imaginary-time
// column, and every field of the cluster is reflected about the symmetry axis (x -> -x in
// the shifted frame), which the Z2-even effective model accepts with probability one.
// Bond (i, t) joins site i to its neighbour at offset t (six offsets: (1,0), (0,1) with
// Js[0]; (1,1), (1,-1) with Js[1]; (2,0), (0,2) with Js[2]); its energy is
// e = J sum_tau x[tau][i] x[tau][j], and it is open with probability 1 - exp(min(0, 2 e)).
// The cluster is the connected component of the seed site in the graph of open bonds.
//
// Design: one workgroup per chain and cluster move.  The bond energies are column dot
// products over the field in place (L2-resident: 8 N Ltau bytes per chain), one thread per
// bond, slices in order; each open bond is decided by its own Philox draw, so the set of
// open bonds does not depend on the order of growth, and the component is grown by
// repeated parallel passes over the open bonds (monotone: a pass only adds sites) until a
// pass adds nothing, with one barrier per pass.  The reflection then negates the cluster's
// columns, coalesced over sites.
#include "common.h"
#include "launch.h"
#include "philox.h"

namespace slmc {

namespace {

constexpr int WF_THREADS = 1024;
constexpr int WF_MAXN = 448;

__global__ __launch_bounds__(WF_THREADS) void wolff_k(double* __restrict__ x, int N, int Lx, int Ly,
                                                      int Ltau, double J0, double J1, double J2,
                                                      int n_clusters, uint32_t k0, uint32_t k1,
                                                      uint32_t prop_arg,
                                                      const uint64_t* __restrict__ prop_dev,
                                                      int coin_mode, int* __restrict__ sizes) {
  const uint32_t prop = prop_dev ? (uint32_t)(*prop_dev & 0xFFFFFFFFu) : prop_arg;
  __shared__ int nbr[6 * WF_MAXN];             // neighbour of bond 6 i + t, -1: no bond
  __shared__ unsigned char open_b[6 * WF_MAXN];
  __shared__ unsigned char in_c[WF_MAXN];
  __shared__ int changed;
  __shared__ int red[WF_THREADS / 64];
  const int ch = blockIdx.x, tid = threadIdx.x, nb = 6 * N;
  // coin_mode 1: only chains whose proposal coin is forward, 2: only reverse ones
  if (coin_mode != 0) {
    const bool fwd = proposal_forward(prop, (uint32_t)ch, k0, k1);
    if ((coin_mode == 1) != fwd) return;
  }
  double* xc = x + (size_t)ch * N * Ltau;
  for (int b = tid; b < nb; b += WF_THREADS) {
    const int i = b / 6, t = b - 6 * i, ix = i % Lx, iy = i / Lx;
    const int dx = (t == 0 || t == 2 || t == 3) ? 1 : (t == 4 ? 2 : 0);
    const int dy = (t == 1 || t == 2) ? 1 : (t == 3 ? -1 : (t == 5 ? 2 : 0));
    const double J = t < 2 ? J0 : (t < 4 ? J1 : J2);
    const int j = (ix + dx) % Lx + Lx * ((iy + dy + Ly) % Ly);
    nbr[b] = (J != 0.0 && j != i) ? j : -1;
  }
  for (int w = 0; w < n_clusters; ++w) {
    __syncthreads();
    // bonds: energy over the columns, then the open/closed draw
    for (int b = tid; b < nb; b += WF_THREADS) {
      const int j = nbr[b];
      unsigned char o = 0;
      if (j >= 0) {
        const int i = b / 6, t = b - 6 * i;
        const double J = t < 2 ? J0 : (t < 4 ? J1 : J2);
        double s = 0.0;
        for (int l = 0; l < Ltau; ++l) s += xc[(size_t)l * N + i] * xc[(size_t)l * N + j];
        const double e = J * s;
        if (e < 0.0) {
          const U4 r = philox(U4{(uint32_t)b, 0x80000000u + (uint32_t)w, prop, (uint32_t)ch}, k0, k1);
          o = u01(r.x) < -expm1(2.0 * e);
        }
      }
      open_b[b] = o;
    }
    const U4 rs = philox(U4{0xFFFFFFFDu, 0x80000000u + (uint32_t)w, prop, (uint32_t)ch}, k0, k1);
    const int s0 = (int)(((uint64_t)rs.x * (uint64_t)N) >> 32);
    for (int i = tid; i < N; i += WF_THREADS) in_c[i] = (i == s0);
    __syncthreads();
    // grow the seed's component
    for (;;) {
      if (tid == 0) changed = 0;
      __syncthreads();
      int mine = 0;
      for (int b = tid; b < nb; b += WF_THREADS) {
        if (!open_b[b]) continue;
        const int i = b / 6, j = nbr[b];
        if (in_c[i] != in_c[j]) {
          in_c[i] = 1;
          in_c[j] = 1;
          mine = 1;
        }
      }
      if (mine) changed = 1;
      __syncthreads();
      if (!changed) break;
      __syncthreads();
    }
    // reflect the cluster's columns and count its sites
    for (int idx = tid; idx < N * Ltau; idx += WF_THREADS) {
      const int i = idx % N;
      if (in_c[i]) xc[idx] = -xc[idx];
    }
    int cnt = 0;
    for (int i = tid; i < N; i += WF_THREADS) cnt += in_c[i];
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = cnt;
    __threadfence_block();
    __syncthreads();
    if (tid == 0 && sizes) {
      int tot = 0;
      for (int k = 0; k < WF_THREADS / 64; ++k) tot += red[k];
      sizes[(size_t)ch * n_clusters + w] = tot;
    }
  }
}

}  // namespace

hipError_t launch_wolff(double* x, int nch, int Lx, int Ly, int Ltau, const double* Js,
                        int n_clusters, uint64_t seed, uint64_t proposal, int coin_mode,
                        int* sizes, hipStream_t st, const uint64_t* prop_dev) {
  if (nch <= 0 || n_clusters <= 0) return hipSuccess;
  if (Lx * Ly > WF_MAXN) return hipErrorInvalidValue;
  const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
  hipLaunchKernelGGL(wolff_k, dim3(nch), dim3(WF_THREADS), 0, st, x, Lx * Ly, Lx, Ly, Ltau, Js[0],
                     Js[1], Js[2], n_clusters, k0, k1, (uint32_t)(proposal & 0xFFFFFFFFu), prop_dev,
                     coin_mode, sizes);
  return hipGetLastError();
}

}  // namespace slmc
