/*
 * tdagw.h -- C ABI of the MI355X (gfx950) TD-aGW propagation library.
 *
 * The library integrates the time-dependent adiabatic GW equation of motion
 * for the one-particle density matrix in the Bloch basis (paper Eq. tdagw):
 *
 *     i d rho_k/dt = [ H^QP_k + dSigma_k(t) - E(t) e.d_k , rho_k ],
 *     dSigma_{nm k} = sum_{n'm'k'} K_{(nmk),(n'm'k')} drho_{n'm'k'}   (Eq. sigma-from-k)
 *
 * with drho = rho - rho_eq, either with the dense kernel K or with the
 * compressed kernel K ~ K_diag + S V^H, S = U M (Eq. svd_diag_offdiag and
 * Eq. svd_acc), applied as K_diag o x + S (V^H x).
 *
 * Conventions shared by every call
 *   - Complex numbers are interleaved (re, im): c128 = 2 x double, c64 = 2 x float.
 *   - Matrices are row-major; "ld" is the row stride in elements.
 *   - Pair index: block ALL uses p = n*nb + m for every band pair (n, m);
 *     block EH uses p = (c - nv)*nv + v for conduction c >= nv and valence
 *     v < nv (the conduction-valence block).  Kernel index i = k*P + p,
 *     k = i1*nk2 + i2.  P = nb*nb (ALL) or (nb-nv)*nv (EH).
 *   - Every array argument is DEVICE memory owned by the caller, unless its
 *     comment says "host".  The library never frees caller memory; it owns
 *     only the workspace inside a context.
 *   - Calls enqueue work on the context's stream and return; results are
 *     valid after that stream is synchronised.  Host arrays passed in (field
 *     records) are copied when the call is queued and may be freed on return.
 *     Calls that wait for the stream: the three compressions,
 *     tdg_links_build, tdg_propagate_adjoint, tdg_check_numeric and
 *     tdg_profile_read; tdg_propagate only while it tunes a new shape (its
 *     first call for that shape) and when it checks a caller's rho(0).
 *   - Every call returns TDG_OK (0) or a negative TDG_E_* code and never
 *     aborts or throws; tdg_last_error() describes the last failure.
 *     Arguments are validated on the host before any device work is queued.
 */
#ifndef TDAGW_H
#define TDAGW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDG_OK 0
#define TDG_E_INVAL (-1)       /* bad argument: null pointer, shape, dtype, alignment */
#define TDG_E_HIP (-2)         /* a HIP runtime call or kernel launch failed */
#define TDG_E_NOMEM (-3)       /* workspace allocation failed */
#define TDG_E_UNSUPPORTED (-4) /* valid request the library does not implement */
#define TDG_E_NUMERIC (-5)     /* NaN / trace / Hermiticity drift found by tdg_check_numeric */
#define TDG_E_SOLVER (-6)      /* the eigensolver used by compression reported failure */

#define TDG_C128 0 /* complex double storage, FP64 arithmetic */
#define TDG_C64 1  /* complex float storage, FP32 arithmetic with FP32 accumulation */
/* BF16 split precision: a complex matrix [rows][ld] is stored as a plane of
 * bf16 (re, im) pairs holding hi = bf16(a), followed by a plane holding
 * lo = bf16(a - hi) (8 bytes per element, like TDG_C64; a ~ hi + lo to about
 * 16 significant bits).  Products run as A_hi x_hi + A_hi x_lo + A_lo x_hi on
 * the BF16 matrix cores with FP32 accumulation (x split the same way on the
 * fly).  Requires ld % 4 == 0.  Used by the batched propagation path only. */
#define TDG_BF16X2 2

#define TDG_BLOCK_ALL 0 /* every band pair (n, m) */
#define TDG_BLOCK_EH 1  /* conduction-valence block; dSigma_vc = conj(dSigma_cv) */

#define TDG_NB_MAX 8 /* largest number of bands per k point */

typedef struct tdg_ctx_s* tdg_ctx;

/* Library version as major*10000 + minor*100 + patch. */
int tdg_version(void);

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the device's default stream).  *out receives the
 * handle.  The context owns all library workspace on that device. */
int tdg_create(tdg_ctx* out, int device, void* hip_stream);
/* Release the context and its workspace (waits for its stream first). */
int tdg_destroy(tdg_ctx ctx);
/* Rebind the context to another stream of the same device.  Work queued on
 * the new stream after this call waits (through an event) for the work the
 * context queued on the old one, which may still be using the context's
 * workspace. */
int tdg_set_stream(tdg_ctx ctx, void* hip_stream);
/* Message describing the last failed call on ctx ("" if none); owned by ctx,
 * valid until the next call on ctx.  ctx may be NULL for tdg_create failures. */
const char* tdg_last_error(tdg_ctx ctx);

/* Band-structure input: quasiparticle energies, Bloch states, position and
 * velocity operators (paper Appendix A.1: H^QP and the dipole matrix r in a
 * smooth gauge; the velocity operator of the HHG current).  Device arrays:
 *   eps   double [nk][nb]          band energies (Ha), ascending per k
 *   evec  c128   [nk][nb][nb]      evec[k][alpha][n] = <alpha | n k>
 *   dip   c128   [2][nk][nb][nb]   interband position d^a_{nm k} (bohr), a = x, y
 *   vel   c128   [2][nk][nb][nb]   v^a_{nm k} (Ha bohr)
 *   links c128   [2][nk][nb][nb]   optional (NULL = none): parallel-transport links
 *                                  from tdg_links_build.  When set, the intraband
 *                                  part of r acts too: d rho_k/dt gains
 *                                  -E(t) e.(rho)_{;k} (see tdg_links_build).
 * nk = nk1*nk2 points of the uniform grid k = (2pi/a)((i + shift)/N - 1/2);
 * the lowest nv bands are occupied in rho_eq. */
typedef struct {
  int32_t nk1, nk2, nb, nv;
  double shift, a_bohr;
  const double* eps;
  const void* evec;
  const void* dip;
  const void* vel;
  const void* links;
} tdg_model;

/* Parallel-transport links for the intraband part of the position operator
 * (paper Eq. tdagw in the length gauge, r in the smooth gauge of Appendix
 * A.1; the paper gives no discretisation, this is the library's reading).
 * [r_intra, rho]_k = i (rho)_{;k}, discretised on the periodic grid as
 *   (rho)_{;a}(k) = [L_a(k) rho(k+b_a) L_a(k)^H - L_a(k-b_a)^H rho(k-b_a) L_a(k-b_a)] / (2|b_a|),
 * |b_a| = 2pi/(N_a a), a = x (index i1), y (index i2).  L_a(k) is block
 * diagonal: on the valence block (bands < nv) and on the conduction block it
 * is the unitary polar factor of that block of M = evec_k^H evec_{k+b_a}
 * (M_nm = <n k|m k+b_a>); zero between the blocks.  Writes links, device c128
 * [2][nk][nb][nb] row-major, caller-owned, 16-byte aligned (model->links is
 * ignored).  Synchronises the stream; TDG_E_NUMERIC names the first (axis, k)
 * whose block overlap is singular (neighbouring subspaces orthogonal: the
 * grid is too coarse for a transport) or whose polar iteration failed. */
int tdg_links_build(tdg_ctx ctx, const tdg_model* model, void* links);

/* Screened interaction for the kernel build: 2D Rytova-Keldysh
 * W(q) = 2pi / (q (1 + r0 q)); at q = 0 the average of W over the grid cell
 * [-h, h]^2, h = pi/(nk1 a), by nquad-point Gauss-Legendre (0 = 64). */
typedef struct {
  double r0_bohr;
  int32_t block; /* TDG_BLOCK_ALL or TDG_BLOCK_EH */
  int32_t nquad;
} tdg_coulomb;

/* Kernel dimension N = nk * P for a model and block (host call, no device work). */
int tdg_kernel_dim(const tdg_model* model, int32_t block, int64_t* n_out);

/* Build the direct electron-hole kernel of the lattice model (paper
 * Eq. sigma-from-k with the single-G limit of Eq. bse-direct-def):
 *   K_{(n m k),(n' m' k')} = -W(|fold(k - k')|) / (nk a^2) <n k|n' k'> <m' k'|m k>
 * into K (dtype TDG_C128, TDG_C64 or TDG_BF16X2, row-major [N][ld], ld >= N;
 * for C64 K must be 16-byte aligned and ld even, for BF16X2 ld % 4 == 0).
 * Overwrites the N x N block (BF16X2: and zero-fills columns N .. ld-1). */
int tdg_kernel_build(tdg_ctx ctx, const tdg_model* model, const tdg_coulomb* coulomb,
                     int32_t dtype, void* K, int64_t ld);

/* Rank rules for compression (paper Sec. SVD analysis): */
#define TDG_TRUNC_REL_CUT 0  /* keep singular values s_i > value * s_max */
#define TDG_TRUNC_FRACTION 1 /* keep round(value * N) singular values (at least 1) */
#define TDG_TRUNC_RANK 2     /* keep exactly value singular values */
#define TDG_TRUNC_R2 3       /* smallest rank with reconstruction R^2 >= value */
typedef struct {
  int32_t mode;
  int32_t pad;
  double value;
} tdg_trunc;
/* A rank never splits a group of singular values equal to within 1e-9 s_max:
 * it is raised to the end of the group, so the truncated kernel is unique. */

/* Output of compression.  The caller sets n, max_rank, dtype and the
 * pointers; the library fills rank and the norms.
 *   kdiag  device [n]               diagonal of K (dtype; TDG_C64 when dtype is TDG_BF16X2)
 *   us     device, n*max_rank elts  S = U diag(s), row-major [n][rank] (dtype);
 *                                   TDG_BF16X2: row stride ld_us = rank rounded up to a
 *                                   multiple of 4 (zero columns), capacity n*(max_rank+3)
 *   w      device, max_rank*n elts  V^H, row-major [rank][n] (dtype; BF16X2 needs n % 4 == 0)
 *   sigma  HOST double [n] or NULL  all singular values of K_off, descending
 * The output dtype may differ from the dtype of K. */
typedef struct {
  int64_t n, max_rank;
  int32_t dtype, pad;
  void* kdiag;
  void* us;
  void* w;
  double* sigma;
  int64_t rank;
  double tail_fro;  /* sqrt(sum_{i >= rank} s_i^2) = ||K_off - U S V^H||_F */
  double tail_spec; /* s_rank, the spectral norm of the discarded part */
} tdg_lowrank;

/* Split K = K_diag + K_off (K_diag the literal matrix diagonal) and replace
 * K_off by its rank-r truncated SVD (paper Eq. svd_diag_offdiag).  K is the
 * Hermitian kernel (dtype, [n][ld]); the SVD is computed in FP64 through the
 * Hermitian eigendecomposition K_off = Q L Q^H (s = |l|, U = Q sign(l),
 * V = Q).  Synchronises the stream.  Fails with TDG_E_INVAL if the chosen
 * rank exceeds max_rank (rank is still reported). */
int tdg_kernel_compress(tdg_ctx ctx, const void* K, int64_t ld, int32_t dtype,
                        const tdg_trunc* trunc, tdg_lowrank* out);

/* Same truncated factorisation as tdg_kernel_compress, for kernels too large
 * for an exact eigendecomposition (N in the tens of thousands).  Not the
 * paper's method: a randomized range finder with power iterations and a
 * Rayleigh-Ritz step on the Hermitian K_off (Halko, Martinsson, Tropp, SIAM
 * Review 53 (2011), Algs. 4.3/4.4 and 5.3), all in FP64 except the products
 * with K, which run in the precision of K:
 *   Y = K_off Omega; power_iters times { Q = qr(Y); Y = K_off Q };
 *   Q = qr(Y); T = Q^H K_off Q = W L W^H; keep the largest |l|;
 *   S = (Q W)_r L_r, V^H = (Q W)_r^H.
 *   K       device, dtype TDG_C128 or TDG_C64, row-major [n][ld], Hermitian
 *   omega   device c128, the n x l test matrix stored column by column
 *           (omega[j * n + i] = Omega_{ij}); the caller draws it
 *   l       number of test vectors, rank + oversampling, 1 <= l <= n
 * The rank rules read the l Ritz values |l| as singular values, with
 * ||K_off||_F and the mean of K_off computed exactly from K; a rule whose
 * rank is not reached within the l values fails with TDG_E_INVAL.
 * out->sigma (if not NULL) receives the l Ritz values, descending;
 * tail_fro = sqrt(max(0, ||K_off||_F^2 - sum_{i < rank} s_i^2)) and tail_spec
 * = s_rank are the corresponding estimates (exact when the range is; tail_spec
 * is NaN when rank == l < n).
 * Output dtypes and layouts as for tdg_kernel_compress.  Device workspace
 * about (3 n l + l^2) * 16 bytes, held by the context.  Synchronises the
 * stream. */
int tdg_kernel_compress_randomized(tdg_ctx ctx, const void* K, int64_t ld, int32_t dtype,
                                   const tdg_trunc* trunc, const void* omega, int64_t l,
                                   int32_t power_iters, tdg_lowrank* out);

/* Channel-wise compression (paper Eq. svd-channel-wise).  Channel (p, q) is
 * the nk x nk block K[k P + p][k' P + q] over k, k' (a transition between
 * band pairs p and q, Sec. "SVD analysis of electron-hole kernel").  Every
 * off-diagonal channel (p != q) is replaced by its own truncated SVD
 * S^{pq} V^{pq H} (S = U M), with the rank rule applied to that channel's nk
 * singular values (R^2 over its elements); the diagonal channels, close to
 * full rank in the paper, are kept whole.  The SVD of a channel A comes in
 * FP64 from the eigendecomposition of the Hermitian dilation [[0, A], [A^H, 0]]
 * (rocSOLVER heevd of order 2 nk).  The caller sets nk, npair, dtype, rmax
 * and the pointers:
 *   diag   device [P][nk][nk]              channel (p, p), row-major (dtype)
 *   s      device [nk P][(P - 1) rmax]     row k P + p: S^{pq}[k][0 .. rmax) for
 *                                          q != p in increasing q, zero past the rank
 *   w      device [P][P - 1][rmax][nk]     V^{pq H} rows, same order, zero past the rank
 *   ranks  HOST int64 [P][P] or NULL       kept rank per channel (nk on the diagonal)
 *   sigma  HOST double [P][P][nk] or NULL  singular values per off-diagonal channel
 * rmax is a multiple of 4 in [4, nk]; a channel needing more fails with
 * TDG_E_INVAL after the ranks before it are reported.  K is TDG_C128 or
 * TDG_C64 [nk P][ld]; dtype (of the outputs) TDG_C128 or TDG_C64.  Device
 * workspace 16 (2 nk)^2 bytes.  Synchronises the stream. */
typedef struct {
  int64_t nk;
  int32_t npair, dtype;
  int64_t rmax;
  void* diag;
  void* s;
  void* w;
  int64_t* ranks;
  double* sigma;
} tdg_channels;

int tdg_kernel_compress_channels(tdg_ctx ctx, const void* K, int64_t ld, int32_t dtype,
                                 const tdg_trunc* trunc, tdg_channels* out);

/* One driving-field instance (atomic units): a Gaussian-enveloped carrier
 * E(t) = e0 exp(-(t - t0)^2 / (2 tau^2)) cos(omega t) along (ex, ey), run for
 * nsteps RK4 steps.  64 bytes; arrays of it are HOST memory. */
typedef struct {
  double e0, omega, tau, t0, ex, ey;
  double nsteps; /* integral value stored as double */
  double pad;
} tdg_field;

#define TDG_OP_DENSE 0
#define TDG_OP_LOWRANK 1
#define TDG_OP_CHANNEL 2

/* The kernel operator applied each RK4 stage.  dtype selects arithmetic:
 * TDG_C128 -> FP64 contraction, TDG_C64 -> FP32 contraction with FP32
 * accumulation, TDG_BF16X2 -> BF16 split-precision products with FP32
 * accumulation (drho is formed in FP64 and rounded; dSigma is widened back
 * to FP64 before the commutator).  Dense: K [n][ld].  Low rank: kdiag [n],
 * us [n][rank], w [rank][n] as written by tdg_kernel_compress.  Channel-wise
 * (TDG_C128 or TDG_C64, one instance at a time): K = tdg_channels.diag,
 * us = tdg_channels.s, w = tdg_channels.w, rank = tdg_channels.rmax; kdiag
 * and ld unused. */
typedef struct {
  int32_t kind, dtype, block, pad;
  int64_t n;
  const void* K;
  int64_t ld;
  const void* kdiag;
  const void* us;
  const void* w;
  int64_t rank;
} tdg_operator;

/* Observable time series, device double arrays [batch][stride] (stride >=
 * max nsteps + 1); entry [b][n] is taken at t_n = n dt for n = 0..nsteps_b:
 *   P    (1/nk) sum_k Re Tr(e.d_k rho_k)        polarisation along e
 *   J    (1/nk) sum_k Re Tr(e.v_k rho_k)        current along e
 *   occ  (1/nk) sum_k Re rho_{c1 c1 k}          first conduction band
 *   tr   max_k |Tr rho_k - nv|                  diagnostic (may be NULL); with
 *        model links, |(1/nk) sum_k Tr rho_k - nv| (the drift moves charge
 *        between k points, only the total is conserved)
 *   herm max_k max_nm |rho_nm - conj rho_mn|    diagnostic (may be NULL) */
typedef struct {
  double* P;
  double* J;
  double* occ;
  double* tr;
  double* herm;
  int64_t stride;
} tdg_obs;

/* Integrate `batch` field instances with classical RK4 (fields evaluated at
 * t_n, t_n + dt/2 twice, t_n + dt; t_n = n dt), each for its own nsteps.
 * rho: device c128 [batch][nk][nb][nb], row n column m; on entry rho(0)
 * (ignored and replaced by rho_eq when init_eq != 0), on exit rho(T_b).
 * Every step of the path runs on the device; nothing is copied back.
 * With init_eq == 0, rho(0) is checked on the device first: if any
 * |rho_nm - conj rho_mn| exceeds 1e-12 (or is NaN) the call fails with
 * TDG_E_INVAL before anything is integrated; this check waits for its
 * one-number result. */
int tdg_propagate(tdg_ctx ctx, const tdg_operator* op, const tdg_model* model,
                  const tdg_field* fields, int32_t batch, double dt, void* rho,
                  int32_t init_eq, const tdg_obs* obs);

/* Size in bytes of the per-device scratch array of tdg_propagate_noalloc. */
#define TDG_NOALLOC_SCRATCH_BYTES 33554432 /* 32 MiB */

/* tdg_propagate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, integration and results, with every workspace buffer
 * (stage states, drho gathers, projections, observable partials, field
 * table) carved from a fixed device array of TDG_NOALLOC_SCRATCH_BYTES that
 * the library holds per GPU from tdg_create until the process ends.  It
 * calls no hipMalloc, hipFree or allocating library routine and creates no
 * events.  Differences from tdg_propagate:
 *   - every instance takes the per-instance path (each streams the operator;
 *     no matrix-core batching); BF16X2 operators fail with TDG_E_UNSUPPORTED;
 *   - the stage kernel is the one tdg_propagate tuned for this shape on the
 *     same context, else variant 0 (TDG_OPT_STAGE_VARIANT still forces one);
 *     nothing is timed; variants differ only in summation order;
 *   - a workspace larger than the array (it grows with batch * nk * nb^2 and
 *     batch * N) fails with TDG_E_INVAL before any work is queued; the
 *     observable partials are kept for fewer steps at a time to fit.
 * All calls on one GPU share its array, which keeps the last call's contents
 * (every byte a call reads it has written first): calls that may overlap on
 * one GPU (other streams or contexts) race and must be serialised by the
 * caller. */
int tdg_propagate_noalloc(tdg_ctx ctx, const tdg_operator* op, const tdg_model* model,
                          const tdg_field* fields, int32_t batch, double dt, void* rho,
                          int32_t init_eq, const tdg_obs* obs);

/* Reverse-mode derivative of tdg_propagate (not in the paper, which
 * integrates forward only): the exact gradient of the discrete RK4 scheme
 * for a real loss L given by its cotangents on the observable series,
 *   dL = sum_b sum_n gP[b][n] dP_b(t_n) + gJ[b][n] dJ_b(t_n) + gocc[b][n] docc_b(t_n),
 * device double arrays [batch][stride], stride >= nsteps + 1 (NULL = 0). */
typedef struct {
  const double* gP;
  const double* gJ;
  const double* gocc;
  int64_t stride;
} tdg_obs_grad;

/* Gradients, caller-owned device buffers, each NULL to skip.  Complex
 * gradients are dL/dRe Z + i dL/dIm Z.
 *   dfield  double [batch][4]          dL/d(e0, omega, tau, t0) of each instance
 *   dE      double [batch][nsteps][4]  dL/dE at the four stage times of each step
 *   drho0   c128 [batch][nk][nb][nb]   dL/drho(t_0)
 *   dus     c128 [n][rank]             dL/dS (low-rank operator only)
 *   dw      c128 [rank][n]             dL/dV^H (low-rank operator only) */
typedef struct {
  double* dfield;
  double* dE;
  void* drho0;
  void* dus;
  void* dw;
} tdg_grads;

/* Integrates forward from rho0 (device c128 [batch][nk][nb][nb]; NULL =
 * rho_eq) keeping rho every checkpoint_every (M) steps (M = nsteps under
 * TDG_OPT_ADJOINT_STASH 2 when the run fits; see there), then pulls the loss
 * back step by step, recomputing each segment from its checkpoint once and
 * keeping every step's stage states, products and gathers of the segment
 * (when those take at most 8 GiB; beyond that each backward step recomputes
 * its own forward step).  FP64 only: op->dtype must be TDG_C128 (dense or low
 * rank).  Every instance must have the same nsteps.  With model->links the
 * intraband term is differentiated too (its covariant difference is
 * anti-self-adjoint).  Device workspace about (nsteps / M + 4 M + 12) states
 * plus 12 M x n x batch complex128 values (without the stash: nsteps / M +
 * M + 15 states plus 4 (M for low rank) x 2 x n x batch values), 4 M x nk x
 * batch doubles of dE partials, and a transposed copy of the operator (n x n
 * dense, 2 x n x rank low rank), held by the context.  Synchronises the stream. */
int tdg_propagate_adjoint(tdg_ctx ctx, const tdg_operator* op, const tdg_model* model,
                          const tdg_field* fields, int32_t batch, double dt, const void* rho0,
                          int32_t checkpoint_every, const tdg_obs_grad* g, tdg_grads* out);

/* Observables of a given state: out device double [batch][5] =
 * (P, J, occ, tr, herm) as defined for tdg_obs, with e taken from fields
 * (host, batch entries). */
int tdg_observables(tdg_ctx ctx, const tdg_model* model, const void* rho, int32_t batch,
                    const tdg_field* fields, double* out);

/* Scan observable series for NaN/Inf and for trace or Hermiticity drift
 * beyond the given thresholds.  Synchronises; returns TDG_E_NUMERIC with the
 * first offending (instance, step) in tdg_last_error, else TDG_OK. */
int tdg_check_numeric(tdg_ctx ctx, const tdg_obs* obs, int32_t batch, const tdg_field* fields,
                      double tr_tol, double herm_tol);

/* Per-kernel timing with HIP events on the context stream, for measurement
 * only.  While enabled, every launch of the timed kernel classes is bracketed
 * by events; tdg_profile_read synchronises and returns the summed duration
 * (ms) and launch count of a class since the last reset. */
#define TDG_KCLASS_STAGE 0   /* fused contraction + commutator + RK4 stage kernel */
#define TDG_KCLASS_PROJECT 1 /* low-rank projection z = V^H x (single-instance path) */
#define TDG_KCLASS_GEMM 2    /* matrix-core products of the batched path */
#define TDG_KCLASS_INTRA 3   /* intraband covariant derivative launches (batched path, model links; the per-instance path forms it in the stage kernel) */
int tdg_profile_enable(tdg_ctx ctx, int32_t on);
int tdg_profile_read(tdg_ctx ctx, int32_t kclass, double* total_ms, int64_t* launches);

/* Launch-shape selection for the stage kernel.  The fused contraction +
 * commutator kernel exists in a few variants (threads per block, unroll
 * depth, occupancy target).  With autotuning on (the default), the first
 * tdg_propagate of a shape (operator kind, dtype, N, nk, batch, rank) times
 * each variant on the first RK4 stage (which leaves rho untouched), keeps the
 * fastest for the context and restarts the integration; variants differ only
 * in summation order. */
#define TDG_OPT_AUTOTUNE 0      /* 1 = tune on first use (default), 0 = use variant 0 */
#define TDG_OPT_STAGE_VARIANT 1 /* >= 0 forces that variant index, -1 = tuned/default */
/* Batched path: with a TDG_C64 operator and at least this many instances
 * (default 4), each stage contracts all running instances at once as complex
 * FP32 matrix products on the matrix cores (split-K partials summed by the
 * stage kernel); below it, every instance streams the operator itself. */
#define TDG_OPT_BATCHED_MIN 2
/* Tiling and split-K of the batched path's complex matrix-core products:
 * TDG_OPT_GEMM_VARIANT -1 (default) times, on the first use of each product
 * shape (M, K, instances), every tiling with each of a few split-K widths (the
 * default of about 1024 blocks, no split, twice the default, and about 256 j
 * blocks for 64-row tiles (j = 1..4) and for 128- and 256-row tiles (j = 1, 2),
 * in steps of 16 complex columns), each followed by one pass over the slices it
 * wrote, and keeps for the context the first pair (default split first) within
 * 2 % of the fastest.  FP32 tilings: 0 = 64-row tiles, 1 = 64-row tiles with
 * the next K tile prefetched into registers and two LDS buffers, 2 = 128-row
 * tiles; BF16X2 tilings 0 = 64-row tiles splitting X while staged, 1 = 128-row
 * tiles on X split once per product, 2 = 256-row tiles on X split once, both
 * operands copied straight to LDS three stages deep, 3 = 128-row tiles on X
 * split once with 64 real K per LDS stage, 4 = tiling 2 with 128-row tiles.
 * A value >= 0 forces that tiling (clamped to the last one) with the default
 * split (or the one TDG_OPT_GEMM_SLICES gives).  Tilings and splits differ
 * only in summation order.  TDG_OPT_GEMM_TILE 64 / 128 selects 0 / 2. */
#define TDG_OPT_GEMM_TILE 3
#define TDG_OPT_GEMM_VARIANT 4
/* 1 replays captured HIP graphs; 0 (default) launches every kernel directly.
 * Results are identical.  Batched path: one RK4 step (products, stage
 * kernels) per running instance count is captured on a private stream and
 * replayed on the context stream for every step in which no instance reaches
 * its final time (the stage kernels then read the step index from device
 * memory).  Per-instance path: every full observable chunk (up to 256 steps,
 * with its field table and observable reduction) in which no instance
 * reaches its final time is captured and replayed once; the host captures
 * the next chunk while the GPU runs the previous one.  tdg_propagate_noalloc
 * and profiled runs always launch directly. */
#define TDG_OPT_GRAPHS 5
/* Batched path: a value in [1, 4096] splits every matrix-core product's K
 * range into that many slices (clamped to twice the default count, the size of
 * the slice buffers) with the tiling the tuner or TDG_OPT_GEMM_VARIANT gives;
 * 0 (default) lets the tuner choose.  Other values: TDG_E_INVAL.  Results
 * differ only in summation order. */
#define TDG_OPT_GEMM_SLICES 6
/* tdg_propagate_adjoint: 2 (default) makes one segment of the whole run when
 * every step's stage data fits in 8 GiB and the device can hold it (no
 * checkpoint sweep; checkpoint_every is then unused), else acts as 1; 1 keeps
 * each segment's stage data when it fits (see there); 0 always recomputes
 * each backward step's forward step, for the smaller workspace.  0 and 1 give
 * identical results; 2 differs from them only in the summation order of the
 * factor gradients over segments.  tdg_last_variant names the plan a call
 * used.  Other values: TDG_E_INVAL. */
#define TDG_OPT_ADJOINT_STASH 7
int tdg_set_option(tdg_ctx ctx, int32_t option, int64_t value);
/* Name of the stage-kernel variant the last tdg_propagate used, or the
 * segment plan of the last tdg_propagate_adjoint ("" before any). */
const char* tdg_last_variant(tdg_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* TDAGW_H */
