/*
 * slmc.h -- C ABI of the MI355X (gfx950) library for the hot path of symmetry-enforced
 * self-learning Monte Carlo on the 2D Holstein model (arXiv:1802.06177).
 *
 * What it computes
 *   For a phonon field x[l][i] (l = 0 .. Ltau-1 is the paper's slice l+1, i = ix + Lx*iy)
 *   the slice matrices are B_l = e^{-dtau K} diag(e^{-dtau*lambda*x[l][.]}) (SM Eq. S2 with
 *   the exponential of the hopping matrix K written first; both factor orders give the
 *   same |det|), and the library returns
 *     logdet = log|det(I + B_{Ltau-1} ... B_0)|   (one spin species; the weight squares it)
 *     sign   = sign det(I + B_{Ltau-1} ... B_0)
 *     G      = (I + B_{Ltau-1} ... B_0)^{-1}, G[i][j] = <c_i c_j^dagger>   (SM Eq. S3, l = L)
 *   stabilized by a column-pivoted QR (UDV form) every n_s slices; the symmetric
 *   effective-model energy and its checkerboard Metropolis sweeps (Eq. 4 / S7); and the
 *   cumulative-update acceptance (Eq. 6).
 *
 * Frame: x = X - alpha with alpha = -lambda/omega0^2 (the paper's g is `lambda` here, its
 *   Omega is `omega0`).  At half filling mu = 0 in this frame.  The bosonic action is
 *   S_Bose = sum_{i,l} [omega0^2/2 x^2 - lambda x + c_kin ((x_{l+1}-x_l)/dtau)^2] (time
 *   periodic) and the full log-weight is -dtau*S_Bose + 2*logdet.
 *
 * Conventions shared by every entry point
 *   - Data pointers named "device" are device (HBM) pointers owned by the caller; the
 *     library never frees or retains them.  Pointers named "host" are host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *     enqueued asynchronously on it; outputs are valid once the stream reaches the point
 *     of the call.
 *   - Argument validation is synchronous: a nonzero return means nothing was enqueued,
 *     and slmc_last_error() (thread-local) explains it.  No C++ exception crosses the ABI.
 *   - Per-item numerical failures (non-finite input or output) are reported in status[b]
 *     with logdet[b] = NaN; the call itself still returns SLMC_OK.  status[b] =
 *     SLMC_E_DEVICE marks an item whose QR workgroup hit the spin limit of its internal
 *     wait (a device fault, not expected in normal operation).
 *   - Doubles are IEEE binary64; x, G are row-major and packed per item.
 */
#ifndef SLMC_H
#define SLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum slmc_status {
  SLMC_OK = 0,
  SLMC_E_ARG = 1,         /* null pointer, out-of-range parameter                        */
  SLMC_E_SHAPE = 2,       /* lattice/time shape the operation does not support           */
  SLMC_E_WORKSPACE = 3,   /* workspace smaller than slmc_*_workspace_bytes()             */
  SLMC_E_DEVICE = 4,      /* HIP runtime error while enqueuing                           */
  SLMC_E_NONFINITE = 5,   /* per-item status: non-finite input or result                 */
  SLMC_E_UNSUPPORTED = 6  /* option combination not built                                */
};

/* Precision of the segment products B_{k n_s} ... B_{(k-1) n_s + 1} between
 * stabilizations.  The stabilization (QR/UDV), recombination, log-det accumulation and
 * the residual step are always FP64. */
enum slmc_precision {
  SLMC_FP64 = 0,       /* FP64 matrix cores                                           */
  SLMC_FP32 = 1,       /* FP32 matrix cores on fp32(E) and the FP32 panel, plus the
                          bf16 product (E - fp32(E)) * bf16(panel) that compensates the
                          fixed rounding of E; FP32 partial sums promoted to FP64 every
                          acc_chunk k-steps of 4 (acc_chunk = 0: never)                */
  SLMC_BF16X3 = 2,     /* two-piece bf16 split (hi + lo), three products, FP32 sums
                          promoted to FP64 per 32-wide k-block                        */
  SLMC_BF16X6 = 3,     /* three-piece bf16 split, six products, as above              */
  SLMC_FP32_PLAIN = 4, /* SLMC_FP32 without the compensation of E (error studies)     */
  SLMC_INT8X5 = 5      /* E and the panel each split into 5 int8 slices of 7 bits
                          (power-of-two scale per row of E / column of the panel,
                          round to nearest); the 15 slice products with exponent sum
                          <= 6 accumulate exactly in int32 on the int8 matrix cores and
                          are recombined in FP64 (about 2^-36 relative to the row and
                          column maxima per product)                                   */
};

/* One lattice model.  N = Lx*Ly sites, Ltau slices of width dtau (beta = Ltau*dtau),
 * stabilization every n_s slices (the last block may be shorter).
 * Limits: 2 <= Lx, Ly; N <= 448 (the QR workgroup keeps two N x 16 panels in LDS); 1 <= n_s <= Ltau. */
typedef struct {
  int32_t Lx, Ly, Ltau, n_s;
  double t;       /* nearest-neighbour hopping (Eq. 2)                                  */
  double mu;      /* chemical potential in the shifted frame (0 = half filling)         */
  double dtau;    /* Trotter step (SM Eq. S1)                                           */
  double lambda;  /* electron-phonon coupling (the paper's g)                           */
  double omega0;  /* phonon frequency (the paper's Omega), M = 1                         */
  double c_kin;   /* prefactor of sum((x_{l+1}-x_l)/dtau)^2 in S_Bose (1/2 or 1)        */
} slmc_model;

typedef struct {
  int32_t precision;       /* enum slmc_precision                                       */
  int32_t residual_steps;  /* FP64 refinement steps on G (0 or 1); ignored by logdet    */
  int32_t acc_chunk;       /* FP32 kinds: k-steps (of 4) per FP64 promotion: 0,1,2,4   */
  int32_t flags;           /* bit set of enum slmc_flags; other bits must be 0         */
} slmc_options;

/* Scheduling flags.  By default, when a model has more than one stabilization block, the
 * segment products and the V updates run on two streams the library owns (per device,
 * default priority, created on first use, destroyed by slmc_cache_clear), forked from and
 * joined back to the caller's stream with events, so that the sequential QR chain
 * overlaps the remaining segment products and the V updates (for SLMC_INT8X5 and
 * SLMC_BF16X3 released step by step into the time of each QR, otherwise queued up
 * front; the autotuner may choose otherwise per model, precision and batch size).  In a
 * packed call of several models, the model with the longest chain runs so on the caller's
 * stream while the other models run one after another in the serial schedule on a third
 * library stream beside it (also forked and joined with events).  Results are identical either way; calls from several host threads on one
 * device serialize while they enqueue.  A call can be captured into a HIP graph on the
 * caller's stream (the library's streams fork from it and join back through events; no
 * memset, no host synchronization) when the items of each model are contiguous and laid
 * out at a constant stride; a packed call whose items are not uploads its item tables
 * synchronously and cannot be captured. */
enum slmc_flags {
  SLMC_FLAG_SERIAL = 1,  /* run every kernel on the caller's stream, in order           */
  SLMC_FLAG_STREAM_E = 2 /* SLMC_INT8X5: read every E slice from device memory in each
                            product, even where E's translation symmetry lets the kernel
                            keep a few base rows in LDS instead (bitwise the same result;
                            for checking and measurement)                              */
};

/* A batch of items, possibly of different models (uneven sizes in one call).
 * model_idx, x_off, g_off are HOST arrays of n_items entries, or NULL:
 *   model_idx NULL -> every item uses model 0;
 *   x_off NULL     -> item b's field starts at x + b*Ltau*N (requires one model);
 *   g_off NULL     -> item b's G starts at G + b*N*N (requires one model).
 * Offsets are in elements (doubles). */
typedef struct {
  int32_t n_items;
  const int32_t* model_idx;
  const int64_t* x_off;
  const int64_t* g_off;
} slmc_batch;

/* Symmetric effective boson model (Eq. 4 / S7 in the shifted frame, weight e^{-E}):
 *   E = Jk sum (x_{i,l+1}-x_{i,l})^2 + J2 sum x^2 + Jp sum (x^4/4 - a^2 x^2/2)
 *     + Jp6 sum (x^6/6 - a^2 x^4/4) + sum_r Js[r] sum_{<ij>_r, l} x_{i,l} x_{j,l}
 *     + Jt sum x_{i,l} x_{i,l+1},
 * bonds counted once: r=0 offsets (1,0),(0,1); r=1 (1,1),(1,-1); r=2 (2,0),(0,2).
 * delta is the local move size: x -> x + delta*(2u-1). */
typedef struct {
  double Jk, J2, Jp, Jp6, a;
  double Js[3];
  double Jt, delta;
} slmc_eff;

/* Library version (major*10000 + minor*100 + patch). */
int slmc_version(void);

/* Thread-local text of the last synchronous error of this thread ("" if none). */
const char* slmc_last_error(void);

/* e^{-dtau K} of a model (SM Eq. S1), FP64, into E_host[N*N] (host, row-major), computed
 * on the host from the lattice's Fourier modes.  Returns SLMC_OK or SLMC_E_ARG. */
int slmc_expk(const slmc_model* model, double* E_host);

/* Device workspace, in bytes, that slmc_logdet / slmc_green need for this batch. */
size_t slmc_workspace_bytes(const slmc_model* models, int32_t n_models,
                            const slmc_batch* batch, const slmc_options* opt);

/* log|det(I + B...B)| and its sign for every item (SM Eq. S2).
 *   models[n_models]  host;  batch, opt host;
 *   x       device, fields (layout above);
 *   logdet  device [n_items] double;  sign device [n_items] int8 (+1/-1);
 *   status  device [n_items] int32 (SLMC_OK, SLMC_E_NONFINITE, or SLMC_E_DEVICE);
 *   ws      device workspace of ws_bytes >= slmc_workspace_bytes(). */
int slmc_logdet(const slmc_model* models, int32_t n_models, const slmc_batch* batch,
                const slmc_options* opt, const double* x, double* logdet, int8_t* sign,
                int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* As slmc_logdet, and also the equal-time Green's function (SM Eq. S3) into G (device,
 * N*N per item, row-major, G[i][j] = <c_i c_j^dagger>), refined by opt->residual_steps
 * FP64 residual-correction steps. */
int slmc_green(const slmc_model* models, int32_t n_models, const slmc_batch* batch,
               const slmc_options* opt, const double* x, double* logdet, int8_t* sign,
               double* G, int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* E_eff of every chain (Eq. 4 / S7).  x device [n_chains][Ltau][N]; e_eff device
 * [n_chains].  Needs Ltau >= 2. */
int slmc_eff_energy(const slmc_model* model, const slmc_eff* eff, int32_t n_chains,
                    const double* x, double* e_eff, void* stream);

/* n_sweeps checkerboard Metropolis sweeps of every chain, in place (main text "SLMC" and
 * the last paragraph of SM Sec. IV: local updates of the effective model).
 *   Colouring: spatial colour (ix mod m) + m (iy mod m), m = 2 when Js[2] == 0 (m = 3 if
 *   2 does not divide Lx, Ly), else m = 4 (or 3); temporal colour l mod 2; phase
 *   p = spatial colour + m*m*temporal colour, P = 2 m^2 phases; Ltau must be even.
 *   A per-proposal coin picks the forward (0..P-1) or reverse (P-1..0) phase order.
 *   Random numbers: Philox4x32-10, key (seed lo, seed hi); counter
 *   (i + N*l, sweep, proposal_idx mod 2^32, chain) -> u1 (word 0, move) and u2 (word 1,
 *   accept iff log u2 < -dE); coin counter (0xFFFFFFFF, 0xFFFFFFFE, proposal, chain)
 *   word 0, forward iff < 2^31; u = (r + 1/2) 2^-32.
 *   x device [n_chains][Ltau][N] in/out; n_accepted device [n_chains] int64 (set, not
 *   accumulated).  Returns SLMC_E_SHAPE if no colouring exists. */
int slmc_eff_sweep(const slmc_model* model, const slmc_eff* eff, int32_t n_chains,
                   double* x, int32_t n_sweeps, uint64_t seed, uint64_t proposal_idx,
                   int64_t* n_accepted, void* stream);

/* Device workspace, in bytes, of slmc_green_slices for n_items fields of one model. */
size_t slmc_slices_workspace_bytes(const slmc_model* model, int32_t n_items,
                                   const slmc_options* opt);

/* The equal-time Green's function after every time slice, G(l) = [I + B_l ... B_0
 * B_{Ltau-1} ... B_{l+1}]^{-1} for l = 0 .. Ltau-1 (SM Eq. S3; slice l = Ltau-1 is the G of
 * slmc_green), and per slice the CDW structure factor's estimators (main text, "Results";
 * two identical spin species, Wick's theorem):
 *   s_nn = N^-1 sum_ij p_i p_j <n_i n_j>,  <n_i n_j> = <n_i><n_j> + 2 (delta_ij - G_ji) G_ij,
 *   m_st = N^-1 sum_i p_i <n_i>,           <n_i> = 2 (1 - G_ii),   p_i = (-1)^(ix+iy);
 * over a Markov chain S_CDW = mean(s_nn) - N mean(m_st)^2.
 * Every n_wrap-th slice (l = n_wrap - 1, 2 n_wrap - 1, ..., and Ltau - 1) is evaluated by
 * the stabilized chain (precision opt->precision) of the field rotated to start after it;
 * the slices between are propagated from the last evaluated one, G(l+1) = B_{l+1} G(l)
 * B_{l+1}^{-1}, with FP64 matrix-core products (n_wrap = 1: every slice evaluated; the
 * propagation error grows at most by the condition number of B per slice).
 *   x device [n_items][Ltau][N]; G_all device [n_items][Ltau][N][N] or NULL (only the
 *   estimators); s_nn, m_st device [n_items][Ltau] double; status device [n_items] int32
 *   (the first non-OK status of the evaluations); ws device workspace of
 *   slmc_slices_workspace_bytes(). */
int slmc_green_slices(const slmc_model* model, const slmc_options* opt, int32_t n_items,
                      const double* x, int32_t n_wrap, double* G_all, double* s_nn, double* m_st,
                      int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Device workspace, in bytes, of slmc_dqmc_sweep and slmc_dqmc_block. */
size_t slmc_dqmc_workspace_bytes(const slmc_model* model, int32_t n_chains,
                                 const slmc_options* opt);

/* One DQMC local sweep of every chain, in place: the comparison method of the paper
 * (SM Sec. I, Eqs. S4-S6).  Slices l = 0 .. Ltau-1 in order, in each the sites i = 0 .. N-1
 * in order: move x[l][i] -> x + delta (2 u1 - 1), Delta = expm1(-dtau lambda dx), spin
 * ratio R = 1 + (1 - G_ii) Delta with G the Green's function after slice l-1 (the factor
 * order B_l = e^{-dtau K} diag(v_l) puts the change on the right of B_l), accept iff
 * log u2 < 2 log|R| - dtau dS_Bose; on accept G <- G - (I - G) e_i (Delta / R) e_i^T G
 * (Sherman-Morrison).  G after slice l-1 is evaluated by the stabilized chain
 * (opt->precision) of the rotated field at every slice l with l % n_rec == 0 and
 * propagated from the previous slice (FP64 products) otherwise.
 *   Random numbers: Philox4x32-10, key (seed lo, seed hi), counter (i + N l, 0xC0000000,
 *   sweep_idx mod 2^32, chain), words 0 (u1) and 1 (u2).
 *   x device [n_chains][Ltau][N] in/out; n_accepted device [n_chains] int64 (set);
 *   G_out device [n_chains][N][N] or NULL: the equal-time G of the final fields, evaluated;
 *   status device [n_chains] int32 (first non-OK status of the evaluations); ws of
 *   slmc_dqmc_workspace_bytes().  Each site update reads and writes all of G: O(N^2) per
 *   site, N^3 Ltau per sweep. */
int slmc_dqmc_sweep(const slmc_model* model, const slmc_options* opt, int32_t n_chains, double* x,
                    double delta, int32_t n_rec, uint64_t seed, uint64_t sweep_idx,
                    int64_t* n_accepted, double* G_out, int32_t* status, void* ws, size_t ws_bytes,
                    void* stream);

/* n_updates DQMC block updates of every chain (SM Sec. I, last paragraph; main text): the
 * column of one site is reflected, x[.][s] -> -x[.][s] (the reflection about the mean
 * displacement in the shifted frame), and accepted iff log u < log w(x') - log w(x), the
 * full weight ratio (log w = -dtau S_Bose + 2 logdet, logdet evaluated with
 * opt->precision).  Update u: site floor(r N / 2^32), r = Philox word 0 at counter
 * (0xFFFFFFFB, 0xFFFFFFFC, c, chain), u = word 0 at (0xFFFFFFFF, 0xFFFFFFFC, c, chain),
 * c = (sweep_idx n_updates + u) mod 2^32.  x in/out; logw device [n_chains] in/out (the
 * cached log weight of x, replaced on accept); n_accepted device [n_chains] int64 (set);
 * status as slmc_dqmc_sweep; ws of slmc_dqmc_workspace_bytes(). */
int slmc_dqmc_block(const slmc_model* model, const slmc_options* opt, int32_t n_chains, double* x,
                    double* logw, int32_t n_updates, uint64_t seed, uint64_t sweep_idx,
                    int64_t* n_accepted, int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Device workspace, in bytes, of slmc_eff_fit for n_configs configurations. */
size_t slmc_fit_workspace_bytes(int32_t n_configs);

/* Training of the effective model (main text Eq. 5, SM Sec. III): the multi-linear
 * regression of ln w onto the terms of the effective model over configurations (e.g. from
 * slmc_dqmc_sweep / slmc_log_weight).  E_eff is linear in its coefficients,
 * E_eff(x) = sum_t J_t F_t(x), with the features in the order of slmc_eff
 *   F = (sum (x_{l+1}-x_l)^2, sum x^2, sum f4(x; a), sum f6(x; a), sum over the bonds of
 *        Js[0], Js[1], Js[2] of x_i x_j, sum x_{i,l} x_{i,l+1})   (t = 0..7),
 * and the fit minimises sum_c (logw_c - E0 + sum_{t in mask} J_t F_ct)^2 by a Householder QR
 * of the design matrix [1, -F_mask] (columns scaled to unit maximum; FP64, one workgroup,
 * fixed reduction order).  mask: bit t selects term t; at most two of Jk, J2, Jt (bits 0,
 * 1, 7: they are linearly dependent) and the selected columns must have full rank.
 *   x device [n_configs][Ltau][N]; logw device [n_configs] (ln w of each configuration);
 *   features device [n_configs][8] or NULL; coef device [9] = (E0, Jk, J2, Jp, Jp6, Js0,
 *   Js1, Js2, Jt) (0 for terms outside the mask); a: the well position of f4, f6;
 *   ws of slmc_fit_workspace_bytes(). */
int slmc_eff_fit(const slmc_model* model, double a, int32_t n_configs, const double* x,
                 const double* logw, int32_t mask, double* features, double* coef, void* ws,
                 size_t ws_bytes, void* stream);

/* n_clusters modified Wolff cluster moves of every chain, in place (SM Sec. IV, Eq. S8):
 * a cluster grows in the spatial plane, each site carrying its whole time column; bond
 * (i, t) joins site i to its neighbour at offset t (t = 0..5: (1,0), (0,1) with Js[0];
 * (1,1), (1,-1) with Js[1]; (2,0), (0,2) with Js[2]; terms with J = 0 or whose ends
 * coincide are no bonds) and is open with probability 1 - exp(min(0, 2 e)),
 * e = J sum_l x[l][i] x[l][j]; the cluster (the seed's component of the open bonds) is
 * reflected, x -> -x on its columns, which the Z2-even effective model always accepts.
 *   Random numbers: Philox4x32-10, key (seed lo, seed hi); bond 6 i + t of cluster w:
 *   counter (6 i + t, 0x80000000 + w, proposal_idx mod 2^32, chain), word 0 -> u, open iff
 *   e < 0 and u < -expm1(2 e); seed site of cluster w: counter (0xFFFFFFFD, 0x80000000 + w,
 *   proposal, chain), word 0 -> r, site floor(r N / 2^32); u = (r + 1/2) 2^-32.
 *   x device [n_chains][Ltau][N] in/out; cluster_sizes device [n_chains][n_clusters] int32
 *   or NULL. */
int slmc_eff_wolff(const slmc_model* model, const slmc_eff* eff, int32_t n_chains, double* x,
                   int32_t n_clusters, uint64_t seed, uint64_t proposal_idx, int32_t* cluster_sizes,
                   void* stream);

/* The whole cumulative proposal of every chain, in place (SM Sec. IV, last paragraph:
 * local sweeps and cluster moves together): the proposal's coin (as in slmc_eff_sweep)
 * picks, per chain, either n_sweeps sweeps in forward phase order followed by n_clusters
 * cluster moves, or the cluster moves followed by the sweeps in reverse phase order; the
 * equal mixture of the two orders is reversible, so the acceptance of Eq. 6 stays exact.
 * Random numbers as slmc_eff_sweep and slmc_eff_wolff.  n_accepted device [n_chains]
 * int64 (local moves), cluster_sizes as slmc_eff_wolff.  Needs what slmc_eff_sweep needs. */
int slmc_eff_propose(const slmc_model* model, const slmc_eff* eff, int32_t n_chains, double* x,
                     int32_t n_sweeps, int32_t n_clusters, uint64_t seed, uint64_t proposal_idx,
                     int64_t* n_accepted, int32_t* cluster_sizes, void* stream);

/* Device workspace, in bytes, of slmc_cumulative_accept for n_chains chains. */
size_t slmc_accept_workspace_bytes(const slmc_model* model, int32_t n_chains,
                                   const slmc_options* opt);

/* Cumulative-update acceptance (Eq. 6) of one proposal per chain:
 *   log r = [log w(x') - log w(x)] + [E_eff(x') - E_eff(x)],
 *   log w = -dtau S_Bose + 2 logdet(x) (logdet with opt->precision),
 *   accept iff log u < log r with u = Philox word 0 at counter
 *   (0xFFFFFFFF, 0xFFFFFFFF, proposal_idx mod 2^32, chain).
 *   x_cur device [n_chains][Ltau][N] in/out (x_prop copied in on accept);
 *   x_prop device (same shape); logw_cur, eeff_cur device [n_chains] in/out (cached values
 *   of the current state, replaced on accept); accepted device [n_chains] uint8;
 *   log_ratio device [n_chains] double; G_prop device [n_chains][N][N] or NULL: the
 *   equal-time Green's function of every proposal (for measurements), computed by the
 *   same evaluation that gives its log-det; status device [n_chains] int32 or NULL: the
 *   status of each proposal's log-det evaluation (SLMC_OK, SLMC_E_NONFINITE for a
 *   non-finite field or result, SLMC_E_DEVICE for a QR wait that hit its spin limit).
 *   A proposal whose status is not SLMC_OK has log_ratio NaN and is rejected, so the
 *   chain keeps its state; status tells the caller which chains that happened to.
 *   ws device workspace. */
int slmc_cumulative_accept(const slmc_model* model, const slmc_eff* eff,
                           const slmc_options* opt, int32_t n_chains, double* x_cur,
                           const double* x_prop, double* logw_cur, double* eeff_cur,
                           uint64_t seed, uint64_t proposal_idx, uint8_t* accepted,
                           double* log_ratio, double* G_prop, int32_t* status, void* ws,
                           size_t ws_bytes, void* stream);

/* log w = -dtau S_Bose(x) + 2 logdet for every chain (seeds the cached logw_cur of
 * slmc_cumulative_accept).  status device [n_chains] int32 or NULL, as in
 * slmc_cumulative_accept (a chain with a non-OK status gets logw NaN, and a NaN cached
 * weight makes every later proposal of that chain be rejected).  Same workspace as
 * slmc_cumulative_accept. */
int slmc_log_weight(const slmc_model* model, const slmc_options* opt, int32_t n_chains,
                    const double* x, double* logw, int32_t* status, void* ws, size_t ws_bytes,
                    void* stream);

/* One whole SLMC step of every chain, as one call that a HIP graph can capture and replay
 * step after step: the proposal index is read from device memory (*proposal_counter) by
 * every kernel that draws random numbers and incremented by one at the end, so each replay
 * of a captured step makes the next proposal.  The step is
 *   x_prop = x_cur; the cumulative proposal of slmc_eff_propose (n_sweeps sweeps and
 *   n_clusters Wolff cluster moves in the order of the proposal's coin); the acceptance of
 *   slmc_cumulative_accept (Eq. 6) with its outputs accepted, log_ratio, G_prop (or NULL)
 *   and status (or NULL).
 * Random numbers as those calls with proposal_idx = *proposal_counter (mod 2^32).
 *   x_cur, x_prop device [n_chains][Ltau][N]; logw_cur, eeff_cur as slmc_cumulative_accept;
 *   proposal_counter device uint64 (read, then incremented on the stream);
 *   n_local_accepted device [n_chains] int64 (local moves of this proposal, set);
 *   ws of slmc_accept_workspace_bytes().  Capturable as slmc_green is (the model's
 *   constants must have been built by an earlier call outside the capture). */
int slmc_step(const slmc_model* model, const slmc_eff* eff, const slmc_options* opt,
              int32_t n_chains, double* x_cur, double* x_prop, double* logw_cur, double* eeff_cur,
              int32_t n_sweeps, int32_t n_clusters, uint64_t seed, uint64_t* proposal_counter,
              uint8_t* accepted, double* log_ratio, double* G_prop, int32_t* status,
              int64_t* n_local_accepted, void* ws, size_t ws_bytes, void* stream);

/* The schedule and tile choices of one model, precision and batch size (the batch size
 * rounded up to a power of two): schedule 0 the default per precision (step-by-step
 * release of the side work, "gated", for SLMC_INT8X5 and SLMC_BF16X3; everything queued
 * up front, "eager", otherwise), 1 eager, 2 gated, 3 serial (as SLMC_FLAG_SERIAL), 4 gated
 * with each V update queued behind the segment block on the same library stream; seg_ahead
 * 1-8 segment blocks released ahead of the chain (gated); gate 0/1 an empty kernel in front
 * of the gated side work; seg_mode (SLMC_INT8X5) 0 A operands in registers where E's
 * translation symmetry allows, 1 E's base rows in LDS only, 2 E streamed from memory;
 * seg_cb 0 the default panel width, 1 16 columns, 2 32 columns (FP64, and int8 panels of
 * at most two row blocks per wave); ms_per_call the tuned time of one logdet call.  Every
 * choice gives bitwise the same results. */
typedef struct {
  int32_t schedule, seg_ahead, gate, seg_mode, seg_cb;
  double ms_per_call;
} slmc_tuning;

/* The project's autotuner: times the candidate choices for logdet calls on the n_items
 * fields x (device [n_items][Ltau][N], one model) and keeps the fastest for this model,
 * precision and batch size; later slmc_logdet / slmc_green / accept calls that match use
 * it (calls on other batch sizes keep the defaults).  Candidates are tried coordinate by
 * coordinate: the segment kernel's variant under the default schedule (int8x5: seg_mode
 * x seg_cb; FP64: seg_cb), then the schedule (serial, eager, gated or gated with the V updates behind the
 * segment blocks, each with seg_ahead 1, 2, 3, 4, 6 or 8 and gate 0/1).  Each candidate's log-dets, signs and statuses are compared bitwise with the
 * default's before it is timed (one warm call, then 3 timed calls, HIP events on
 * `stream`); a candidate that differs is rejected.  The fastest is timed against the
 * default once more, alternating, and kept only if at least 2% faster.  Synchronous (it waits for `stream`).
 * With the environment variable SLMC_TUNE_CACHE naming a file, the choices are read from
 * it at first use and written back after each tuning.  ws: device workspace of at least
 * slmc_workspace_bytes(model, 1, {n_items}, opt) + 6 * roundup256(8 n_items) bytes.
 * chosen (host): the choice; n_tried, n_rejected (host, or NULL): candidates run and
 * rejected.  Not with SLMC_FLAG_SERIAL. */
int slmc_autotune(const slmc_model* model, const slmc_options* opt, int32_t n_items, const double* x,
                  void* ws, size_t ws_bytes, void* stream, slmc_tuning* chosen, int32_t* n_tried,
                  int32_t* n_rejected);

/* The choice in effect for this model, precision and batch size, into out (host);
 * *tuned (host) = 1 if the autotuner (or the cache file) provided it, 0 for the defaults. */
int slmc_tuning_lookup(const slmc_model* model, const slmc_options* opt, int32_t n_items,
                       slmc_tuning* out, int32_t* tuned);

/* Kernel timing with HIP events recorded around each launch on its stream (off by
 * default; costs two events per launch while on).  Classes: 0 seg_chain, 1 wy_apply,
 * 2 qr, 3 vupd, 4 lu, 5 lu_solve, 6 residual, 7 eff_sweep.  slmc_profile_read waits for
 * the recorded events and returns the accumulated milliseconds and launch count of one
 * class since the last slmc_profile_reset. */
int slmc_profile(int enable);
int slmc_profile_read(int32_t kernel_class, double* total_ms, int64_t* launches);
void slmc_profile_reset(void);
const char* slmc_profile_name(int32_t kernel_class);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): slmc_green (or slmc_logdet when G is
 * NULL) of n_items fields of ONE model laid out [n_items][Ltau][N] (G [n_items][N][N]),
 * that allocates nothing.  Its workspace and the model's constants (e^{-dtau K} in every
 * format) live in a static device array of 256 MiB that the library holds on each GPU it
 * runs on until the process ends; the workspace part is SLMC_NOALLOC_WORKSPACE_BYTES, and
 * a batch whose slmc_workspace_bytes() exceeds it is refused with SLMC_E_WORKSPACE (e.g.
 * at most 18 items of the 16x16, Ltau 160, n_s 8 model; 508 of the 8x8, Ltau 80 one).
 * It calls no hipMalloc, hipFree or allocating routine and creates no stream or event:
 * every kernel runs on `stream` in order (the serial schedule, bitwise the results of
 * slmc_green).  A call whose model differs from the previous call's on this GPU waits for
 * `stream` (host synchronization) and copies the new constants into the array first.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other host threads without ordering) race and must not be issued.  Arguments,
 * outputs and per-item status as slmc_green. */
#define SLMC_NOALLOC_WORKSPACE_BYTES ((size_t)248 << 20)
int slmc_green_noalloc(const slmc_model* model, const slmc_options* opt, int32_t n_items,
                       const double* x, double* logdet, int8_t* sign, double* G,
                       int32_t* status, void* stream);

/* Frees the library's device constant cache (e^{-dtau K} copies per model and device)
 * and its side streams (after waiting for them), and forgets the autotuner's choices (the
 * cache file, if any, stays and is read again at the next lookup).  Must not be called while work that
 * uses them is still queued on other streams. */
void slmc_cache_clear(void);

#ifdef __cplusplus
}
#endif
#endif /* SLMC_H */
