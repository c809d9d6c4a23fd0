// Equal-time Green's function at every time slice (SM Eq. S3) and the CDW structure
// factor's per-field estimators (main text, "Results").
//
// G(l) after slice l is reached from an evaluated one by propagation,
// G(l+1) = B_{l+1} G(l) B_{l+1}^{-1} with B = e^{-dtau K} diag(v) and
// B^{-1} = diag(1/v) e^{+dtau K}: two FP64 matrix-core products per slice,
// T = (diag(v) G diag(1/v)) e^{dtau K} and G' = e^{-dtau K} T.  The evaluated slices come
// from the stabilized chain of a rotated field (the field's slices taken cyclically from
// slice r, whose product is B_{r-1} ... B_0 B_{Ltau-1} ... B_r), gathered here.
//
// The estimators need sum_i G_ii, sum_i p_i (1 - G_ii) and sum_ij p_i p_j G_ij G_ji
// (p_i = (-1)^(ix+iy)); the last pairs element (i, j) with its transpose, so a workgroup
// takes 16x16 tile pairs (I, J), (J, I), both read coalesced into LDS.
#include "common.h"
#include "launch.h"

namespace slmc {

namespace {

constexpr int MT = 64;    // output tile
constexpr int MK = 16;    // k step

// rotated fields: xr[b][k][i] = x[b][(k + r) mod Ltau][i]
__global__ __launch_bounds__(256) void rotate_k(const double* __restrict__ x, double* __restrict__ xr,
                                                int N, int Ltau, int r, int64_t total) {
  const int64_t per = (int64_t)N * Ltau;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / per, rem = e - b * per;
    const int k = (int)(rem / N), i = (int)(rem - (int64_t)k * N);
    int ks = k + r;
    if (ks >= Ltau) ks -= Ltau;
    xr[e] = x[b * per + (int64_t)ks * N + i];
  }
}

// C[b] = A[b] B[b] on N x N matrices (row-major, leading dimensions lda/ldb, ldc = N).
// STEP 0: A = diag(v) G diag(1/v) (G per item at A + b sa, v = exp(-ldl x[b][s][.])),
//         B = Bsh (shared, e^{+dtau K}).
// STEP 1: A = Ash (shared, e^{-dtau K}), B per item at B + b sb.
// 64 x 64 output tiles, four waves of 32 x 32 (2 x 2 blocks of 16 x 16 on
// v_mfma_f64_16x16x4f64), k steps of 16 through LDS; entries beyond N read as zero.
template <int STEP>
__global__ __launch_bounds__(256) void prop_gemm_k(const double* __restrict__ A, int64_t sa, int lda,
                                                   const double* __restrict__ B, int64_t sb, int ldb,
                                                   double* __restrict__ C, int64_t sc,
                                                   const double* __restrict__ x, int64_t sx, int s,
                                                   double ldl, int nb, int N) {
  __shared__ double As[MT][MK + 2];
  __shared__ double Bs[MK][MT + 2];
  __shared__ double vv[448], vi[448];
  const int nt = (N + MT - 1) / MT;
  const int id = xcd_remap(blockIdx.x, nb * nt * nt);
  if (id < 0) return;
  const int tj = id % nt, ti = (id / nt) % nt, b = id / (nt * nt);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
  const int i0 = MT * ti, j0 = MT * tj, ro = 32 * (w >> 1), co = 32 * (w & 1);
  const double* Ab = STEP == 0 ? A + b * sa : A;
  const double* Bb = STEP == 0 ? B : B + b * sb;
  if (STEP == 0) {
    const double* xs = x + b * sx + (int64_t)s * N;
    for (int q = tid; q < N; q += 256) {
      const double v = exp(-ldl * xs[q]);
      vv[q] = v;
      vi[q] = 1.0 / v;
    }
    __syncthreads();
  }
  dx4 acc[2][2] = {{zero4d(), zero4d()}, {zero4d(), zero4d()}};
  const int ar = tid >> 2, ak = 4 * (tid & 3);
  const int bk = tid >> 4, bj = 4 * (tid & 15);
  for (int k0 = 0; k0 < N; k0 += MK) {
    {
      const int row = i0 + ar;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = k0 + ak + e;
        double a = 0.0;
        if (row < N && k < N) {
          a = Ab[(int64_t)row * lda + k];
          if (STEP == 0) a = vv[row] * a * vi[k];
        }
        As[ar][ak + e] = a;
      }
      const int k = k0 + bk;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = j0 + bj + e;
        Bs[bk][bj + e] = (k < N && j < N) ? Bb[(int64_t)k * ldb + j] : 0.0;
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
  double* Cb = C + b * sc;
#pragma unroll
  for (int hi = 0; hi < 2; ++hi)
#pragma unroll
    for (int hj = 0; hj < 2; ++hj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i0 + ro + 16 * hi + drow64(g, v), col = j0 + co + 16 * hj + c;
        if (row < N && col < N) Cb[(int64_t)row * N + col] = acc[hi][hj][v];
      }
}

// Per (item, slice): s_nn = N m^2 + (2/N)(tr G - q), m = (2/N) sum_i p_i (1 - G_ii),
// q = sum_ij p_i p_j G_ij G_ji.  The 16x16 tile pairs (I, J >= I) are spread over
// ceil(nt/2) workgroups per item, workgroup k taking the tile rows I = k and I = nt-1-k
// (nt + 1 pairs each: balanced); each writes its three partial sums, reduced in a fixed
// order, and cdw_fin_k adds the partials of an item in order.
constexpr int CDW_MAXG = 14;   // workgroups per item: ceil(nt/2) for N <= 448

__global__ __launch_bounds__(256) void cdw_part_k(const double* __restrict__ G, int64_t sg, int Lx,
                                                  int N, double* __restrict__ part) {
  __shared__ double T1[16][17], T2[16][17];
  __shared__ double red[3][4];
  const int nt = (N + 15) / 16, ng = (nt + 1) / 2;
  const int b = blockIdx.x / ng, k = blockIdx.x - b * ng;
  const int tid = threadIdx.x, r = tid >> 4, cc = tid & 15;
  const double* Gb = G + b * sg;
  double q = 0.0, tr = 0.0, d = 0.0;
  for (int h = 0; h < 2; ++h) {
    const int I = h == 0 ? k : nt - 1 - k;
    if (h == 1 && I == k) break;
    for (int J = I; J < nt; ++J) {
      const int i = 16 * I + r, j = 16 * J + cc, i2 = 16 * J + r, j2 = 16 * I + cc;
      T1[r][cc] = (i < N && j < N) ? Gb[(int64_t)i * N + j] : 0.0;     // G[I-tile][J-tile]
      T2[r][cc] = (i2 < N && j2 < N) ? Gb[(int64_t)i2 * N + j2] : 0.0;  // G[J-tile][I-tile]
      __syncthreads();
      if (i < N && j < N) {
        // element (i, j) of the I,J tile with its transpose (j, i), held in T2[cc][r]
        const int pi = ((i % Lx) + (i / Lx)) & 1, pj = ((j % Lx) + (j / Lx)) & 1;
        const double t = T1[r][cc] * T2[cc][r];
        q += ((pi ^ pj) ? -t : t) * (I == J ? 1.0 : 2.0);
        if (I == J && r == cc) {
          const double gii = T1[r][cc];
          tr += gii;
          d += pi ? -(1.0 - gii) : (1.0 - gii);
        }
      }
      __syncthreads();
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    q += __shfl_xor(q, off, 64);
    tr += __shfl_xor(tr, off, 64);
    d += __shfl_xor(d, off, 64);
  }
  if ((tid & 63) == 0) { red[0][tid >> 6] = q; red[1][tid >> 6] = tr; red[2][tid >> 6] = d; }
  __syncthreads();
  if (tid < 3) {
    double* pp = part + ((int64_t)b * CDW_MAXG + k) * 3;
    pp[tid] = (red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]);
  }
}

__global__ __launch_bounds__(256) void cdw_fin_k(const double* __restrict__ part, int nb, int N,
                                                 double* __restrict__ s_nn, double* __restrict__ m_st,
                                                 int64_t so) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int ng = ((N + 15) / 16 + 1) / 2;
  const double* pp = part + (int64_t)b * CDW_MAXG * 3;
  double Q = 0.0, TR = 0.0, D = 0.0;
  for (int k = 0; k < ng; ++k) {
    Q += pp[3 * k];
    TR += pp[3 * k + 1];
    D += pp[3 * k + 2];
  }
  const double m = 2.0 * D / N;
  s_nn[b * so] = N * m * m + 2.0 * (TR - Q) / N;
  m_st[b * so] = m;
}

// dst[b sd + e] = src[b ss + e], e < n (batched copy with item strides)
__global__ __launch_bounds__(256) void copy_items_k(const double* __restrict__ src, int64_t ss,
                                                    double* __restrict__ dst, int64_t sd, int64_t n,
                                                    int nb) {
  const int64_t total = n * nb;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / n, k = e - b * n;
    dst[b * sd + k] = src[b * ss + k];
  }
}

__global__ void status_or_k(const int* __restrict__ a, int* __restrict__ out, int n, int first) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = first ? a[i] : (out[i] != 0 ? out[i] : a[i]);
}

}  // namespace

hipError_t launch_rotate_fields(const double* x, double* xr, int nb, int N, int Ltau, int r,
                                hipStream_t st) {
  const int64_t total = (int64_t)nb * N * Ltau;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(rotate_k, dim3(grid), dim3(256), 0, st, x, xr, N, Ltau, r, total);
  return hipGetLastError();
}

hipError_t launch_propagate(const double* Gin, int64_t sgin, double* Gout, int64_t sgout,
                            double* T, const double* E, const double* Einv, int ldE,
                            const double* x, int s, double ldl, int nb, int N, int Ltau,
                            hipStream_t st) {
  const int nt = (N + MT - 1) / MT;
  const dim3 grid(xcd_grid(nb * nt * nt));
  const int64_t sx = (int64_t)N * Ltau, nn = (int64_t)N * N;
  hipLaunchKernelGGL(prop_gemm_k<0>, grid, dim3(256), 0, st, Gin, sgin, N, Einv, (int64_t)0, ldE, T, nn, x,
                     sx, s, ldl, nb, N);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prop_gemm_k<1>, grid, dim3(256), 0, st, E, (int64_t)0, ldE, T, nn, N, Gout, sgout,
                     x, sx, s, ldl, nb, N);
  return hipGetLastError();
}

hipError_t launch_cdw(const double* G, int64_t sg, int nb, int Lx, int N, double* s_nn, double* m_st,
                      int64_t so, double* part, hipStream_t st) {
  const int ng = ((N + 15) / 16 + 1) / 2;
  if (ng > CDW_MAXG) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cdw_part_k, dim3(nb * ng), dim3(256), 0, st, G, sg, Lx, N, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cdw_fin_k, dim3((nb + 255) / 256), dim3(256), 0, st, part, nb, N, s_nn, m_st, so);
  return hipGetLastError();
}

hipError_t launch_copy_items(const double* src, int64_t ss, double* dst, int64_t sd, int64_t n, int nb,
                             hipStream_t st) {
  const int64_t total = n * nb;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(copy_items_k, dim3(grid), dim3(256), 0, st, src, ss, dst, sd, n, nb);
  return hipGetLastError();
}

hipError_t launch_status_or(const int* a, int* out, int n, int first, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(status_or_k, dim3((n + 255) / 256), dim3(256), 0, st, a, out, n, first);
  return hipGetLastError();
}

}  // namespace slmc
