// Host-side launchers of the device kernels (defined in the .hip files).  Every launcher
// enqueues on `st` and returns the hipError_t of the launch.  Sizes: N sites, Np = N
// rounded up to a multiple of 16 (the padded rows/columns carry an identity block, so the
// padded determinant is det * 2^(Np-N) and the padded G holds 1/2 on that block).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace slmc {

// Field of item b: x + (xoff ? xoff[b] : b * xstride), laid out [Ltau][N].
struct FieldRef {
  const double* x;
  const int64_t* xoff;   // device array or nullptr
  int64_t xstride;
};

// Segment products S_k = B_{k n_s + len-1} ... B_{k n_s}, B_l = E diag(exp(-ldl x_l)),
// for all items b < nb and segments k < m, into S[(b*m + k)][Np][Np] (FP64), and the
// squared column norms of every S_k into snorm[(b*m + k)][Np].  Only the segments
// k0 .. k0+kc-1 are computed (m stays the segment count of the S and snorm layout).
// prec: 0 FP64; 1 FP32 with the bf16 correction of E's FP32 rounding; 4 FP32 without it;
// (acc_chunk = k-steps of 4 per FP64 promotion of the FP32 sums, 0 = none); 2 bf16x3;
// 3 bf16x6; 5 int8 slices (5 per operand, 15 products, exact int32 sums).
// E64/E32/Elo/Ebf/Eq point at the padded exponential in each format (Elo: bf16 of
// E64 - E32; Ebf: [pieces][Np][Np] bf16 bit patterns; Eq/Esc: int8 slices and row scales).
// trow > 0: E[i + trow][j + trow] = E[i][j] (indices mod N), trow a multiple of 16; the
// int8 kernel then reads E's slices from an LDS copy of the first trow rows.  0: no such
// structure is used.
hipError_t launch_seg_chain(int prec, int acc_chunk, const double* E64, const float* E32,
                            const uint16_t* Elo, const uint16_t* Ebf, const int8_t* Eq,
                            const double* Esc, FieldRef f, int nb, int N, int Np, int Ltau,
                            int n_s, int m, int k0, int kc, double ldl, double* S, double* snorm,
                            int trow, hipStream_t st, int seg_mode = 0, int seg_cb = 0);
// seg_mode (int8 slices): 0 any (A operands in registers where the structure allows), 1 E's
// base rows in LDS but no register operands, 2 E streamed from memory.  seg_cb: 0 the
// default panel width, 1 16 columns, 2 32 columns where 32 divides Np (FP64; int8 with at
// most 2 row blocks per wave).  Every choice gives the same bits.

// A[b] = Bsrc[b] Q[b] (Q = H_0 ... H_{Np-1} in compact-WY blocks: Householder vectors
// in the strict lower triangle of QRW[b], T blocks in Tb[b][Np/16][16][16]).
// Bsrc == nullptr means the identity.  transpose_out: write A^T instead of A.
// npart != nullptr: squared column norms of each 16-row panel into npart[b][Np/16][Np].
hipError_t launch_wy_apply(const double* Bsrc, int64_t bstride, const double* QRW,
                           const double* Tb, double* A, double* npart, int transpose_out,
                           int nb, int Np, hipStream_t st);

// Column-pivoted (pre-sorted) blocked Householder QR of A[b] (one workgroup per item).
// Sort key of column j: 0.5 log(sum_p norm2[b*nstride + p*Np + j]) + logDp[b][j]; key[j] =
// logDp[b][perm j] (0 without logDp).  The V-update factor is F = S_r R S_c, F[i][j] =
// R[i][j]/|R[i][i]| exp(key[j] - key[i]) (j >= i).  Outputs: QRW[b] (strict lower:
// Householder vectors; upper incl. diagonal: R), scales[b][2 Np] = (S_c, S_r) =
// (e^(key_j - kref), e^(kref - key_i)/|R_ii|), Tb, perm[b][Np], logD[b][Np] = log|R_ii| +
// key[i], qsign[b] = det Q, status[b] |= 1 on NaN.
hipError_t launch_qr(const double* A, int64_t astride, const double* norm2, int64_t nstride,
                     int nparts, const double* logDp, double* QRW, double* Tb, int* perm,
                     double* scales, double* logD, int* qsign, int* status, int nb, int Np,
                     hipStream_t st);

// dst[0..n) = value (a plain kernel, safe inside captured graphs)
hipError_t launch_fill_i32(int* dst, int n, int value, hipStream_t st);
// status[b] = 1 if item b's field (nelem = Ltau N values) holds a non-finite value, else 0
// (a plain kernel, safe inside captured graphs)
hipError_t launch_field_status(FieldRef f, int nb, int nelem, int* status, hipStream_t st);
// One empty wave.  Enqueued on a side stream in front of work released at the same moment
// as a launch on another stream, its dispatch lets the other launch's workgroups reach the
// compute units first.
hipError_t launch_order_gate(hipStream_t st);

// Vn[b] = F[b] Vo[b][perm[b], :] with F = S_r R S_c the V-update factor of launch_qr, from R
// in the upper triangle of QRW[b] and scales[b] (Vo == nullptr: identity).
hipError_t launch_vupd(const double* QRW, const int* perm, const double* scales, const double* Vo,
                       double* Vn, int nb, int Np, hipStream_t st);

// LU with partial pivoting of X = Db^-1 QT + Ds V (Db = max(e^logD,1), Ds = min(e^logD,1))
// and logdet = sum max(logD, 0) + log|det X| - (Np-N) log 2, sign = qsign * sign det X.
// Writes LU[b], prow[b], diagonal-block inverses DI[b][Np/16][2][16][16] and, through
// the item map, logdet_out[item], sign_out[item], status_out[item].
hipError_t launch_lu(const double* QT, const double* V, const double* logD, const int* qsign,
                     const int* st_in, double* LU, int* prow, double* DI, const int* item_of,
                     double* logdet_out, int8_t* sign_out, int32_t* status_out, int nb,
                     int N, int Np, hipStream_t st);

// Solve X Y = RHS with the LU of launch_lu.  mode 0: RHS = Db^-1 QT; mode 1: RHS = R.
// accumulate: Gint += Y, else Gint = Y.  If Gout != nullptr also write the leading
// N x N block of Gint to Gout + goff[b] (or b*N*N).
hipError_t launch_lu_solve(int mode, const double* QT, const double* logD, const double* R,
                           const double* LU, const int* prow, const double* DI, double* Gint,
                           int accumulate, double* Gout, const int64_t* goff, int nb, int N,
                           int Np, hipStream_t st);

// R = Db^-1 QT - X Gint (residual of the recombination solve).
hipError_t launch_residual(const double* QT, const double* V, const double* logD,
                           const double* Gint, double* R, int nb, int Np, hipStream_t st);

// ---- effective model / accept ----
struct EffParams {
  double Jk, J2, Jp, Jp6, a, Js0, Js1, Js2, Jt, delta;
};

hipError_t launch_eff_energy(const double* x, int nch, int Lx, int Ly, int Ltau, EffParams p,
                             double* e, hipStream_t st);

// prop_dev (or nullptr): the proposal index is read from device memory instead of `proposal`
hipError_t launch_eff_sweep(double* x, int nch, int Lx, int Ly, int Ltau, EffParams p,
                            int mod, int n_sweeps, uint64_t seed, uint64_t proposal,
                            int64_t* nacc, hipStream_t st, const uint64_t* prop_dev = nullptr);
// *c += 1 (one thread)
hipError_t launch_incr_u64(uint64_t* c, hipStream_t st);

// n_clusters modified Wolff cluster moves of every chain (in place), bonds from the spatial
// couplings Js[3]; coin_mode 0: every chain, 1: only chains whose proposal coin picks the
// forward order, 2: only the reverse ones.  sizes (or nullptr): [nch][n_clusters].
hipError_t launch_wolff(double* x, int nch, int Lx, int Ly, int Ltau, const double* Js,
                        int n_clusters, uint64_t seed, uint64_t proposal, int coin_mode,
                        int* sizes, hipStream_t st, const uint64_t* prop_dev = nullptr);

// ---- G at every slice, CDW estimators ----
// xr[b][k] = x[b][(k + r) mod Ltau] (fields [nb][Ltau][N])
hipError_t launch_rotate_fields(const double* x, double* xr, int nb, int N, int Ltau, int r,
                                hipStream_t st);
// Gout[b] = B_s Gin[b] B_s^{-1}, B_s = E diag(exp(-ldl x[b][s])), via T[b] (scratch
// [nb][N][N]); E and Einv = e^{+dtau K} with leading dimension ldE; G strides sgin/sgout.
hipError_t launch_propagate(const double* Gin, int64_t sgin, double* Gout, int64_t sgout,
                            double* T, const double* E, const double* Einv, int ldE,
                            const double* x, int s, double ldl, int nb, int N, int Ltau,
                            hipStream_t st);
// s_nn[b so], m_st[b so] of G + b sg (N x N, row-major)
hipError_t launch_cdw(const double* G, int64_t sg, int nb, int Lx, int N, double* s_nn, double* m_st,
                      int64_t so, double* part, hipStream_t st);
// dst[b sd + e] = src[b ss + e] for e < n, b < nb
hipError_t launch_copy_items(const double* src, int64_t ss, double* dst, int64_t sd, int64_t n, int nb,
                             hipStream_t st);
// out[i] = a[i] (first) or the first nonzero of out[i], a[i]
hipError_t launch_status_or(const int* a, int* out, int n, int first, hipStream_t st);

// ---- effective-model regression ----
// F[c][8]: the effective model's terms with unit coefficients for every configuration
hipError_t launch_features(const double* x, int n, int Lx, int Ly, int Ltau, double a, double* F,
                           hipStream_t st);
// out[9] = (E0, J[8]): least squares of logw ~ E0 - sum_{t in mask} J_t F_t (Householder QR in
// one workgroup; Aw [9][n] and yw [n] scratch)
hipError_t launch_fit(const double* F, const double* logw, int n, int mask, double* Aw, double* yw,
                      double* out, hipStream_t st);

// log w = -dtau S_Bose + 2 logdet for every chain.
hipError_t launch_log_weight(const double* x, const double* logdet, int nch, int N, int Ltau,
                             double lam, double omega0, double dtau, double c_kin,
                             double* logw, hipStream_t st);

// Cumulative accept: log r = (logw' - logw) + (E' - E); accept iff log u < log r, u from
// Philox word 0 at counter (0xFFFFFFFF, tag, proposal mod 2^32, chain).
hipError_t launch_accept(double* x_cur, const double* x_prop, double* logw_cur,
                         double* eeff_cur, const double* logw_prop, const double* eeff_prop,
                         int nch, int64_t nelem, uint64_t seed, uint64_t proposal,
                         uint8_t* accepted, double* log_ratio, hipStream_t st,
                         uint32_t tag = 0xFFFFFFFFu, const uint64_t* prop_dev = nullptr);

// ---- DQMC comparison updates ----
// The N local updates of slice l of every chain, in order, with Sherman-Morrison updates
// of G (G after slice l-1 on entry, [nch] at stride sg); nacc[ch] += accepted moves.
hipError_t launch_dqmc_slice(double* G, int64_t sg, double* x, int nch, int N, int Ltau, int l,
                             double dtau, double lam, double omega0, double c_kin, double delta,
                             uint64_t seed, uint64_t sweep, int64_t* nacc, hipStream_t st);
// x_prop = x_cur with one column negated per chain (site from Philox at counter
// (0xFFFFFFFB, 0xFFFFFFFC, ctr, chain))
hipError_t launch_reflect_column(const double* x_cur, double* x_prop, int nch, int N, int Ltau,
                                 uint64_t seed, uint32_t ctr, hipStream_t st);
hipError_t launch_fill_i64(int64_t* dst, int n, int64_t v, hipStream_t st);
// nacc[i] += a[i]
hipError_t launch_add_accepted(const uint8_t* a, int64_t* nacc, int n, hipStream_t st);

}  // namespace slmc
