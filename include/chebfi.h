/*
 * chebfi.h - C ABI of the MI355X Chebyshev-filter eigensolver hot path.
 *
 * The library finds the lowest M eigenpairs of a plane-wave Kohn-Sham
 * problem H psi = lambda S psi on an N x M block of wave functions kept in GPU
 * memory, as stated in arXiv 2604.11139, section "Problem setup".
 * H = 0.5|k+G|^2 (diagonal) + V_loc (applied on the FFT grid) + sum_R P_R D_R P_R^H
 * (section "Low-level operations").  S = I (norm-conserving), or, for PAW and
 * ultrasoft systems, the overlap S = I + sum_R P_R Q_R P_R^H with its inverse
 * applied by the Woodbury formula (sections "Introduction" and "Main
 * computational kernels").  The block is filtered by a Chebyshev polynomial of
 * S^-1 H (Algorithm "Parallel Chebyshev filtering of degree k"),
 * orthonormalised through the Cholesky factor of its S-Gram matrix (Algorithm
 * "S-ortho") and rotated by Rayleigh-Ritz (Algorithm "RR").  Only eigenvalues
 * and scalars come back to the host (section "Host-device memory transfers").
 *
 * Conventions shared by every call
 * --------------------------------
 * Blocks: device pointers to interleaved complex numbers (re, im), column-major
 *   npw x nband with leading dimension ld >= npw (one band per column; the
 *   band stride of section "Batch processing").  dtype ABI_C128 means double
 *   pairs (16 bytes per coefficient), ABI_C64 float pairs (8 bytes).  The row
 *   order is the library's sphere order (abi_get_gsphere): ascending FFT-box
 *   index i1 + n1*(i2 + n2*i3) with i_d = m_d mod n_d.
 * Ownership: the caller allocates and owns every block and output buffer; the
 *   library owns the handle and its tables and work buffers, frees them in
 *   abi_destroy, and keeps no caller pointer after the call's stream work.
 * Streams: `stream` is a hipStream_t (NULL = default stream).  Calls enqueue
 *   work and return; calls that return host values synchronise that stream.
 *   One handle must not be used from two host threads or streams at once.
 * Errors: every call returns ABI_OK (0) or a negative code; abi_last_error()
 *   gives the message of the calling thread's last failure.  On error nothing
 *   is guaranteed about output buffers.
 */
#ifndef CHEBFI_H
#define CHEBFI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t abi_status;

enum {
  ABI_OK = 0,
  ABI_ERR_ARG = -1,     /* null pointer, nband <= 0, ld < npw, degree < 1, b <= a, a0 > a ... */
  ABI_ERR_GRID = -2,    /* sphere does not fit the box, radix not in {2,3,5}, box too large */
  ABI_ERR_NOT_HPD = -3, /* Cholesky breakdown (pivot index in abi_last_error) */
  ABI_ERR_DEVICE = -4,  /* HIP runtime error */
  ABI_ERR_NOMEM = -5,   /* device allocation failed */
  ABI_ERR_STATE = -6    /* dtype or precision not allowed for this handle */
};

enum { ABI_C128 = 0, ABI_C64 = 1 };
enum { ABI_PREC_FP64 = 0, ABI_PREC_MIXED = 1 };

typedef struct abi_system_s *abi_system;

/* One Hamiltonian.  Host pointers are read during abi_set_system only. */
typedef struct {
  int32_t abi_version;   /* 1, or 2 to pass qij (version 1 callers omit the field) */
  double lattice[9];     /* rows a1, a2, a3 in bohr */
  double kpt_red[3];     /* k-point in reduced coordinates of the reciprocal basis */
  double ecut;           /* Ha; basis = {G : 0.5|k+G|^2 < ecut} (strict) */
  int32_t ngrid[3];      /* FFT box n1, n2, n3; each {2,3,5}-smooth and <= 96 */
  const double *vloc;    /* n1*n2*n3 reals, V_loc(r_i) with i1 fastest */
  int32_t natom;         /* >= 0; four projectors (s, px, py, pz) per atom */
  const double *tau_cart;/* natom*3 cartesian positions, bohr */
  double rc;             /* projector Gaussian width, bohr (> 0) */
  const double *dij;     /* natom*4*4 complex (re,im interleaved), row-major D_R[i][j], Hermitian */
  int32_t precision;     /* ABI_PREC_FP64 or ABI_PREC_MIXED */
  /* abi_version 2 only.  natom*4*4 complex (re,im interleaved), row-major Q_R[i][j],
   * Hermitian, or NULL: the overlap S = I + sum_R P_R Q_R P_R^H of PAW/ultrasoft
   * systems (NULL or natom = 0: S = I).  Q_R may be indefinite; S must be
   * positive definite (abi_set_system fails with ABI_ERR_NOT_HPD otherwise, and
   * when the projectors are linearly dependent). */
  const double *qij;
} abi_system_desc;

/* ---- host-only helpers (no GPU needed) ------------------------------------ */

/* Number of plane waves of the basis of `desc` (section "Low-level operations":
 * the cut-off fixes the grid and the data are moved into the FFT layout).
 * Fails with ABI_ERR_GRID if the sphere leaves the box window
 * [-n/2, n/2-1] (even n) / [-(n-1)/2, (n-1)/2] (odd n). */
abi_status abi_gsphere_count(const abi_system_desc *desc, int64_t *npw);

/* Fills host arrays of length npw (as returned by abi_gsphere_count):
 * miller (npw*3, m1 m2 m3 per plane wave), box_index (npw) and kinetic (npw,
 * 0.5|k+G|^2).  Any of the three may be NULL. */
abi_status abi_gsphere_build(const abi_system_desc *desc, int64_t npw, int32_t *miller,
                             int32_t *box_index, double *kinetic);

/* ---- handle ---------------------------------------------------------------- */

/* Builds the basis, the kinetic and projector tables and the FFT plans of one
 * Hamiltonian on the current HIP device and uploads V_loc and D.  The
 * projector matrix P (npw x 4*natom) has columns
 * p_s = g e^{-iG.R}/sqrt(Omega), p_c = rc q_c g e^{-iG.R}/sqrt(Omega),
 * q = k+G, g = exp(-|q|^2 rc^2/2) (section "Low-level operations").
 * Synchronises `stream`.  On success *out owns device memory until abi_destroy. */
abi_status abi_set_system(const abi_system_desc *desc, void *stream, abi_system *out);

abi_status abi_system_info(abi_system sys, int64_t *npw, int32_t *nproj, int32_t ngrid[3]);

/* Copies the basis maps to host arrays (npw*3 and npw int32). */
abi_status abi_get_gsphere(abi_system sys, int32_t *miller, int32_t *box_index);

/* Copies the FP64 projector matrix to a caller device buffer of npw*nproj
 * complex doubles, column-major with leading dimension npw.  Synchronises. */
abi_status abi_get_projectors(abi_system sys, void *P_out, void *stream);

abi_status abi_destroy(abi_system sys);

/* Overlap of the handle: *has_overlap = 1 when S != I, *s_min = the smallest
 * eigenvalue of S (1 when S = I).  Either pointer may be NULL.  With S != I,
 * abi_set_system forms B = P^H P, its Cholesky factor B = R^H R and the
 * eigen-decomposition R Q R^H = Z diag(mu) Z^H (FP64, on the device); S has
 * the eigenvalues 1 and 1 + mu_i, and S^-1 = I - P K P^H with
 * K = W diag(mu / (1 + mu)) W^H, W = R^-1 Z (the Woodbury formula of the Sinv
 * kernel, section "Main computational kernels"). */
abi_status abi_overlap_info(abi_system sys, int32_t *has_overlap, double *s_min);

/* ---- hot path ------------------------------------------------------------- */

/* HX = H X for nband columns (matrix-free H application of section "Main
 * computational kernels": kinetic diagonal, V_loc through batched 3D FFTs,
 * nonlocal through P^H X, D and P(...)).  X and HX must not overlap.
 * dtype ABI_C128: FP64 throughout.  dtype ABI_C64 (handles built with
 * ABI_PREC_MIXED only): complex64 blocks, FP32 FFT passes and recurrence,
 * FP32-accumulated MFMA projector products; D is applied in FP64. */
abi_status abi_apply_H(abi_system sys, const void *X, void *HX, int64_t nband, int64_t ld,
                       int32_t dtype, void *stream);

/* SX = S X and Y = S^-1 X (the HX_SX and Sinv kernels of section "Main
 * computational kernels"; S^-1 X = X - P (K (P^H X)), O(N_projs N) per band).
 * Blocks and dtype as for abi_apply_H; the output must not overlap X.  With
 * S = I both copy X.  The small product K (P^H X) is taken in FP64 for both
 * dtypes. */
abi_status abi_apply_S(abi_system sys, const void *X, void *SX, int64_t nband, int64_t ld,
                       int32_t dtype, void *stream);
abi_status abi_apply_Sinv(abi_system sys, const void *X, void *Y, int64_t nband, int64_t ld,
                          int32_t dtype, void *stream);

/* Bounds of the Chebyshev filter (Algorithm "Parallel Chebyshev filtering of
 * degree k", Rayleigh-quotient step): out[0] = a = max_i RQ_i,
 * out[2] = a0 = min_i RQ_i with RQ_i = Re(x_i^H H x_i)/Re(x_i^H S x_i), and
 * out[1] = b = theta_max(T) + beta_last from `nlanczos` (1..64) Lanczos steps
 * on S^-1 H with full reorthogonalisation in the S inner product u^H S v,
 * started from the device vector v0 (npw complex doubles, always FP64); the
 * run stops early with b = theta_max when beta_j <= 1e-12 max(1, |alpha_j|).
 * `out` is a host array of 3 doubles.  Synchronises `stream`. */
abi_status abi_spectral_bounds(abi_system sys, const void *X, int64_t nband, int64_t ld,
                               int32_t dtype, const void *v0, int32_t nlanczos, double *out,
                               void *stream);

/* Y = T_m((A - c)/e) X / T_m((a0 - c)/e), A = S^-1 H, e = (b-a)/2, c = (b+a)/2,
 * by the scaled three-term recurrence (the "axpy" recurrence of section
 * "Parallel implementation design"): Y_1 = (s_1/e)(A - c)X,
 * Y_{k+1} = (2 s_{k+1}/e)(A - c)Y_k - s_k s_{k+1} Y_{k-1}, s_1 = e/(a0 - c),
 * s_{k+1} = 1/(2/s_1 - s_k).  degree = m >= 1 applications of A; requires
 * b > a and a0 <= a.  X and Y (both npw x nband, leading dimension ld) must
 * not overlap; X is not modified.  dtype as for abi_apply_H.  With S != I each
 * step still projects and expands the block once: the projections P^H Y_k are
 * carried along (FP64) and the Woodbury correction is formed from them by
 * nproj x nproj products. */
abi_status abi_cheb_filter(abi_system sys, const void *X, void *Y, int64_t nband, int64_t ld,
                           int32_t dtype, int32_t degree, double a, double b, double a0,
                           void *stream);

/* abi_cheb_filter with H X supplied by the caller (HX: device, the dtype and
 * leading dimension of X, not overlapping X or Y; not modified): the first
 * step is then Y_1 = (s_1/e)(HX - c X), so the filter applies H degree - 1
 * times.  This is the reuse of the Rayleigh-quotient H X (or of the H Psi of
 * the last Rayleigh-Ritz step) behind the paper's count of k + 1 H
 * applications per cycle (section "Arithmetic intensity").  Equal to
 * abi_cheb_filter up to rounding when HX is H X.  S = I only (ABI_ERR_STATE
 * on a handle with an overlap). */
abi_status abi_cheb_filter_hx(abi_system sys, const void *X, const void *HX, void *Y,
                              int64_t nband, int64_t ld, int32_t dtype, int32_t degree, double a,
                              double b, double a0, void *stream);

/* Rayleigh-Ritz on the filtered block (Algorithms "S-ortho" and "RR"):
 * G = Y^H S Y = U^H U (Cholesky, FP64), H_s = Y^H (H Y),
 * U^-H H_s U^-1 = Z Lambda Z^H, Psi = Y U^-1 Z (S-orthonormal),
 * H Psi = (H Y) U^-1 Z, and the residual norms ||H psi_n - lambda_n S psi_n||
 * (Algorithm "Parallel Chebyshev filtering of degree k", last two steps).  By default computed
 * in FP64: a complex64 block (dtype ABI_C64, mixed handles) is promoted,
 * processed and rounded back, so the eigenvalues are those of the FP64 pencil
 * of the block (see flags for the split-BF16 form).
 * Y (npw x nband, ld): in: filtered block; out: Ritz vectors Psi.
 * HPsi: optional output of the same dtype and ld, or NULL.
 * eval: host, nband doubles, ascending.  resnorm: host, nband doubles, or NULL.
 * coef: device nband x nband complex doubles (ld nband) receiving C = U^-1 Z,
 *   so that Psi = Y_in C (the coefficients of the Ritz vectors), or NULL.
 * flags: host int32 in/out, or NULL.  In: ABI_RR_LOWPREC asks, for a complex64
 *   block on a mixed handle with S = I, for the split-BF16 form of the
 *   intermediate cycles of the mixed solver: columns scaled to unit norm
 *   (equilibration), G and H_s as split-BF16 MFMA products accumulated in
 *   FP32, Cholesky, reduction and eigensolve in FP64, the two rotations as
 *   split-BF16 products.  When the smallest squared pivot of the equilibrated
 *   Gram matrix's Cholesky factor U1 is below 0.5, the block is first
 *   orthonormalised (Q1 = Y E U1^-1, split-BF16) and the Gram matrix taken
 *   again on Q1 (CholeskyQR2), so the split products' ~2^-17 relative error
 *   is not magnified by the block's conditioning.  Ritz values then carry
 *   absolute errors of about 1e-5 max|lambda| and the Ritz vectors
 *   orthonormality errors of about 1e-5, which the next filter and a final
 *   FP64 Rayleigh-Ritz remove.  Out: ABI_RR_LOWPREC if that form ran (with
 *   ABI_RR_TWO_PASS when it took the second pass); ABI_RR_FELL_BACK if it was
 *   asked for but a squared pivot fell below 1e-4 (too ill-conditioned for
 *   the split products), in which case the FP64 form ran; 0 otherwise.
 * Fails with ABI_ERR_NOT_HPD if the Gram matrix is not positive definite.
 * Synchronises `stream`. */
enum { ABI_RR_FELL_BACK = 1, ABI_RR_LOWPREC = 2, ABI_RR_TWO_PASS = 4 };
abi_status abi_rayleigh_ritz(abi_system sys, void *Y, void *HPsi, int64_t nband, int64_t ld,
                             int32_t dtype, double *eval, double *resnorm, void *coef,
                             int32_t *flags, void *stream);

/* The eigensolver loop: cycles of spectral bounds (10 Lanczos steps from v0),
 * degree-m filter and Rayleigh-Ritz on the block X, the Ritz vectors of a cycle
 * being the next cycle's block (the subspace iteration of Algorithm "Parallel
 * Chebyshev filtering of degree k", repeated), until the residual norms of the
 * lowest nconv Ritz pairs are all <= tol or max_cycles cycles have run.  From
 * the second cycle on, the bounds take the Rayleigh quotients of the block from
 * the last Ritz values (they are equal for Ritz vectors) and keep the first
 * cycle's Lanczos upper bound (H is fixed), so they apply no H; and the filter
 * starts from the H Psi the last Rayleigh-Ritz step formed (abi_cheb_filter_hx;
 * S = I), so a cycle applies H degree times, the Rayleigh-Ritz's included.
 * X (in: start block; out: Ritz vectors, ascending Ritz values) is npw x nband
 * (ld) of `dtype`; v0: device, npw complex128.  With dtype ABI_C64 and
 * refine_degree > 0, the mixed cycles hand over to FP64 cycles of degree
 * refine_degree on the promoted block (a residual-driven refinement) when a
 * cycle improves the worst of those residuals by less than 10%, when they meet
 * tol, or after half of max_cycles; X then receives the complex64 rounding of
 * the FP64 Ritz vectors.  Those mixed cycles use the split-BF16 Rayleigh-Ritz
 * (ABI_RR_LOWPREC of abi_rayleigh_ritz); without refinement they use the FP64
 * one.  eval, resnorm (host, nband; resnorm may be NULL): the last cycle's
 * Ritz values and residual norms.  info (host, 4 entries, may be NULL): cycles
 * in the block's precision, FP64 refinement cycles, converged (0/1), 0.
 * Synchronises the stream.  Errors: those of the calls it makes; ABI_ERR_ARG
 * for nconv outside 1..nband, tol <= 0, refinement asked for a complex128
 * block. */
abi_status abi_chebfi_solve(abi_system sys, void *X, int64_t nband, int64_t ld, int32_t dtype,
                            const void *v0, int32_t degree, int32_t max_cycles, int32_t nconv,
                            double tol, int32_t refine_degree, double *eval, double *resnorm,
                            int32_t *info, void *stream);

/* Block LOBPCG, the solver the paper compares the Chebyshev filter with
 * (Algorithm "Parallel LOBPCG with b blocks and k line minimizations"), built on
 * the same kernels: passes over the nblocks blocks of nband/nblocks bands, each
 * block S-deflated against the blocks before it (X <- X - Q (Q^H S X)),
 * orthonormalised and rotated by Rayleigh-Ritz, then up to nline line
 * minimisations: W = (H - Lambda S) Psi (the block stops once all its residual
 * norms are <= tol), W <- K W with the Teter-Payne-Allan diagonal
 * K_G = p(x)/(p(x) + 16x^4), p = 27 + 18x + 12x^2 + 8x^3, x = 0.5|k+G|^2 / E_kin(psi),
 * S-deflation of W, H W and S W, columns of W and P scaled to unit S-norm,
 * S-ortho + Rayleigh-Ritz of [Psi, W] (first step) or [Psi, W, P] (falling
 * back to [Psi, W] when that Gram is not positive definite), P <- W C_W + P C_P,
 * Psi <- Psi C_Psi + P; with nblocks > 1 a global S-ortho + Rayleigh-Ritz ends the
 * pass.  Passes repeat until the lowest nconv residual norms are <= tol or
 * max_passes have run.  FP64 only: X (in: start block, out: Ritz vectors) is a
 * complex128 npw x nband block (ld).  eval, resnorm (host, nband; resnorm may be
 * NULL): the last pass's Ritz values (ascending) and ||H psi - lambda S psi||.
 * info (host, 4 entries, may be NULL): passes, line minimisations run (summed
 * over blocks and passes), converged (0/1), 0.  Synchronises the stream.
 * ABI_ERR_NOT_HPD if the Gram of a block or of [Psi, W] breaks down. */
abi_status abi_lobpcg_solve(abi_system sys, void *X, int64_t nband, int64_t ld, int32_t dtype,
                            int32_t nblocks, int32_t nline, int32_t max_passes, int32_t nconv,
                            double tol, double *eval, double *resnorm, int32_t *info,
                            void *stream);

/* Replaces V_loc (device, n1*n2*n3 doubles, i1 fastest) and/or D (device,
 * natom*16 complex doubles, row-major per atom); a NULL pointer keeps the old
 * table.  Stream-ordered; for differentiation and finite differences. */
abi_status abi_update_potential(abi_system sys, const double *vloc, const void *dij,
                                void *stream);

/* Copies the handle's V_loc (FP64, n1*n2*n3, i1 fastest) to a device array. */
abi_status abi_get_potential(abi_system sys, double *vloc, void *stream);

/* Adjoint of abi_cheb_filter (handles with S = I; ABI_ERR_STATE otherwise)
 * for the loss L = sum_n Re<W_n, Y_n>, Y = the
 * filter output (reverse mode of the filter recurrence; the paper's solver is
 * not differentiated, so this is the derivative of the operation
 * abi_cheb_filter computes).  With gamma_0 = s_1/e, gamma_k = 2 s_{k+1}/e and
 * delta_k = s_k s_{k+1}, the reverse recurrence A_m = W,
 * A_k += gamma_k (H - c) A_{k+1}, A_{k-1} -= delta_k A_{k+1} gives
 *   dX = A_0,
 *   dV(r) = sum_k gamma_k sum_n Re[conj(A~_{k+1,n}(r)) Y~_{k,n}(r)] / (n1 n2 n3),
 *   dD_R  = sum_k gamma_k (P_R^H A_{k+1}) (P_R^H Y_k)^H,
 * where ~ is the unnormalised inverse FFT of a sphere vector.  Gradients use
 * the convention dL/dRe + i dL/dIm (each D entry independent); the bounds are
 * held fixed.  Iterates are recomputed from (Y_{s-1}, Y_s) checkpoints taken
 * every ckpt_every steps (0 = one segment, all iterates kept).
 * X, W: npw x nband (ld), both of `dtype`: ABI_C128, or ABI_C64 on a handle
 * built with ABI_PREC_MIXED (then the iterates and adjoint iterates are
 * complex64, the FFT passes FP32 and the projector products split-BF16, as in
 * abi_cheb_filter; dV and dD are still accumulated in FP64).  Outputs (device,
 * overwritten): dV (n1*n2*n3 doubles), dD (natom*16 complex doubles; may be
 * NULL when natom = 0), dX (npw x nband, ld, of `dtype`) or NULL. */
abi_status abi_filter_backward(abi_system sys, const void *X, const void *W, int64_t nband,
                               int64_t ld, int32_t dtype, int32_t degree, double a, double b,
                               double a0, int32_t ckpt_every, double *dV, void *dD, void *dX,
                               void *stream);

/* Density of a block on the FFT grid: rho(r) = sum_n w_n |psi~_n(r)|^2 / (n1 n2 n3),
 * psi~ the unnormalised inverse FFT of the scattered sphere vector (so a unit
 * band integrates to 1 over the grid points).  The SCF loop builds the density
 * from the wave functions through FFTs (Algorithm "SCF", density step); with
 * unit weights on the lowest p Ritz vectors this is the Hellmann-Feynman
 * derivative of their eigenvalue sum with respect to V_loc(r).
 * Psi: npw x nband (ld), dtype as for abi_apply_H.  weights: device, nband
 * doubles, or NULL for unit weights.  rho: device, n1*n2*n3 doubles,
 * overwritten (FP64 accumulation in a fixed band order). */
abi_status abi_density(abi_system sys, const void *Psi, int64_t nband, int64_t ld, int32_t dtype,
                       const double *weights, double *rho, void *stream);

/* As abi_density, but adds to rho instead of overwriting it: the density of
 * several k-points (handles on the same FFT box) accumulated into one grid,
 * each call with its own weights (occupation times k-point weight). */
abi_status abi_density_add(abi_system sys, const void *Psi, int64_t nband, int64_t ld,
                           int32_t dtype, const double *weights, double *rho, void *stream);

/* ---- outer SCF step (Algorithm "Self-consistent field in DFT") ----------------
 * The paper computes the occupations from the eigenvalues on the host and the
 * density with FFTs on the GPU; the potential of the next iteration is the host
 * code's part and is defined here as V = V_ion + V_H[n] + v_x[n] with
 * n(r) = rho(r) n1 n2 n3 / Omega (rho the grid density of abi_density),
 * V_H(G) = 4 pi n(G) / |G|^2 (V_H(0) = 0, G in the box window of the sphere),
 * v_x = -(3 n / pi)^(1/3) (LDA exchange; 0 where n <= 0). */

/* Host only.  Fermi-Dirac occupations f_i = occ_max / (1 + exp((eval_i - mu)/kT))
 * of n states with mu found by bisection so that sum_i f_i = nelec (requires
 * kT > 0 and 0 <= nelec <= occ_max n).  f: host array of n; mu may be NULL. */
abi_status abi_occupations(int64_t n, const double *eval, double nelec, double kT, double occ_max,
                           double *f, double *mu);

/* vout = V_ion + V_H[n] + v_x[n] for the grid density rho (device arrays of
 * n1*n2*n3 doubles, i1 fastest; vout may alias neither input).  FP64 FFTs of
 * the whole box on the device.  Stream-ordered. */
abi_status abi_scf_potential(abi_system sys, const double *rho, const double *vion, double *vout,
                             void *stream);

/* SCF iterations at the handle's potential V_in (its current V_loc): cycles_per_iter
 * cycles of abi_chebfi_solve's loop on X (bounds from v0, degree-`degree` filter,
 * Rayleigh-Ritz), occupations of the nband Ritz values (occ_max 2, temperature
 * kT), the density, V_out = abi_scf_potential(rho, vion), then stop when
 * max_r |V_out - V_in| <= tol, else V_loc <- V_in + K (V_out - V_in) and repeat,
 * at most max_iter times.  K = alpha (linear mixing, q0 = 0) or, with q0 > 0,
 * Kerker's preconditioner K(G) = alpha |G|^2 / (|G|^2 + q0^2) (alpha at G = 0),
 * which damps the long-wavelength charge sloshing of large cells.  X, v0, dtype as for
 * abi_chebfi_solve (X keeps the Ritz vectors); vion: device, n1*n2*n3 doubles.
 * eval (host, nband): the last Ritz values.  rho_out (device, n1*n2*n3, or NULL):
 * the last density.  dv_out (host, or NULL): the last max |V_out - V_in|.
 * info (host, 4 entries, or NULL): iterations, converged (0/1), 0, 0.  On return
 * the handle's V_loc is the last V_in (the converged potential when converged).
 * Synchronises the stream. */
abi_status abi_scf_solve(abi_system sys, void *X, int64_t nband, int64_t ld, int32_t dtype,
                         const void *v0, const double *vion, double nelec, double kT,
                         double alpha, double q0, int32_t degree, int32_t cycles_per_iter,
                         int32_t max_iter, double tol, double *eval, double *rho_out,
                         double *dv_out, int32_t *info, void *stream);

/* ---- dense FP64 building blocks of the Rayleigh-Ritz step ---------------------
 * Column-major complex double matrices in device memory, leading dimension lda. */

/* In place: A (m x m Hermitian, upper triangle read) -> U upper with real
 * positive diagonal, A = U^H U; the strict lower triangle is zeroed
 * (Algorithm "S-ortho", potrf). */
abi_status abi_zpotrf_upper(int64_t m, void *A, int64_t lda, void *stream);

/* Eigen-decomposition of a Hermitian m x m matrix (upper and lower triangles
 * read as the average (A + A^H)/2): w (device, m doubles, ascending) and Z
 * (device, m x m, ldz) with A = Z diag(w) Z^H.  A is overwritten.  The hegvd
 * step of Algorithm "RR" after the Cholesky reduction.  1 <= m <= 8192
 * (ABI_ERR_ARG otherwise; 8192 is the paper's largest band count); allocates
 * and frees a device workspace of about 55 m^2 bytes per call (0.23 GB at
 * m = 2048), about 110 m^2 above m = 2560 (7.4 GB at m = 8192: the inverse
 * iteration of eigenvalue clusters then keeps its arrays in global memory
 * instead of LDS), and synchronises the stream. */
abi_status abi_zheev(int64_t m, void *A, int64_t lda, double *w, void *Z, int64_t ldz,
                     void *stream);

/* ---- batching: many systems in one set of launches ---------------------------
 * The paper applies the operator to a whole block of bands per call instead
 * of band by band (section "Batch processing"); a batch extends this across
 * independent systems (cells, k-points) of uneven plane-wave counts and FFT
 * boxes.  One filter step of every system of the batch is three launches for
 * the projector products (projection partial sums in tiles of 32 bands, their
 * reduction with D, the expansion P C' in tiles) and three FFT-pass launches per
 * group of boxes (the recurrence fused into the last), each a grid-stride loop
 * over the work items of all systems; the launches of a filter are captured
 * into a HIP graph on first use and replayed.  Limits: at most 1024 systems, at
 * most 256 atoms per system, FFT edges up to 96, S = I (no Q). */
typedef struct abi_batch_s *abi_batch;

/* Builds the nsys systems of `descs` (as abi_set_system; all with the same
 * precision) and the batch around them.  Errors: ABI_ERR_ARG (nsys out of
 * range, more than 256 atoms in a system, mixed precisions), and those of
 * abi_set_system. */
abi_status abi_set_system_batch(const abi_system_desc *descs, int32_t nsys, void *stream,
                                abi_batch *out);

/* The handle of system i (owned by the batch: valid until abi_destroy_batch,
 * never passed to abi_destroy); for abi_system_info, abi_get_gsphere, the
 * single-system calls and their parity checks. */
abi_status abi_batch_system(abi_batch batch, int32_t i, abi_system *out);

/* Y_i = the degree-m Chebyshev filter of X_i for every system i of the batch,
 * with its own bounds (a[i], b[i], a0[i]); the same result as abi_cheb_filter
 * on each system.  X, Y: host arrays of nsys device pointers (blocks npw_i x
 * nband[i], column stride ld[i], of `dtype`; Y_i separate from X_i).  nband,
 * ld, a, b, a0: host arrays of nsys entries.  Stream-ordered; does not
 * synchronise (it may capture a graph on the batch's own stream the first time
 * a configuration is seen). */
abi_status abi_cheb_filter_batch(abi_batch batch, const void *const *X, void *const *Y,
                                 const int64_t *nband, const int64_t *ld, int32_t dtype,
                                 int32_t degree, const double *a, const double *b,
                                 const double *a0, void *stream);

/* Times the launch variants of the batched filter on the caller's arguments
 * (same as abi_cheb_filter_batch; Y is overwritten; eager launches, best of
 * three filters per variant) and keeps the fastest:
 * FFT pass threads per workgroup (256 / 512 where the plans allow) and the
 * radix order of the FFT plans (ascending / descending).  choice (host, 4
 * entries, may be NULL) receives {fft threads, projection threads (256: the
 * tiled projector products), descending radix order (0/1), timed variants}.
 * Synchronises the stream. */
abi_status abi_batch_autotune(abi_batch batch, const void *const *X, void *const *Y,
                              const int64_t *nband, const int64_t *ld, int32_t dtype,
                              int32_t degree, const double *a, const double *b, const double *a0,
                              int32_t *choice, void *stream);

/* Graph capture on (1, default) or off (0: eager launches). */
abi_status abi_batch_use_graph(abi_batch batch, int32_t on);

/* Each filter step's projector products (P^H Y, D, P C') on a second stream of
 * the batch, beside the FFT passes A and B that do not need them, the last
 * pass waiting for them (1, default), or in line on the caller's stream (0).
 * The same kernels in either case: the results are bitwise the same.  The
 * second stream has the default priority. */
abi_status abi_batch_use_overlap(abi_batch batch, int32_t on);

abi_status abi_destroy_batch(abi_batch batch);

/* ---- no-allocation form ---------------------------------------------------------
 * For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same operation, arguments and results as abi_apply_H, but every work buffer
 * (split-K parts, D C, the projector part of the mixed form, the FFT box batch)
 * is a piece of one static 64 MiB scratch array per device, located when a
 * handle is first set up on that device; the call allocates nothing.  The FFT
 * passes take as many boxes per batch as fit.  Fails with ABI_ERR_NOMEM when
 * the work buffers of the call do not fit in 64 MiB (e.g. 22119 plane waves x
 * 512 bands in the mixed form: call it on fewer bands at a time), and with
 * ABI_ERR_STATE while timing (abi_profile_enable) is on.  All calls on one
 * device share its array: calls that overlap in time on one device (other
 * streams, other handles, other host threads) race and must not be issued. */
abi_status abi_apply_H_noalloc(abi_system sys, const void *X, void *HX, int64_t nband, int64_t ld,
                               int32_t dtype, void *stream);

/* ---- tuning --------------------------------------------------------------------
 * Launch choices of a handle's kernels.  Every choice computes the same
 * product; variants of one class agree to rounding (the split-BF16 ones are
 * bit for bit equal when they sum the same K chunks in the same order).
 *   ABI_TUNE_PROJ      split-BF16 projection P^H X: 0..3, 5..8 tile variants on
 *                      planes made by a split pass; 4 register-staged 128 x 128
 *                      reading the complex64 block; 9..14 direct-to-LDS tiles
 *                      reading the block (14, the default: eight waves with
 *                      scheduled fragment reads); 15, 16: the direct-to-LDS
 *                      tile of 14 (2 x 4 / 4 x 2 waves) on bf16 planes, which
 *                      inside a filter the previous step's last FFT pass writes
 *                      (a split pass makes them otherwise; a no-allocation call
 *                      uses 14)
 *   ABI_TUNE_EXPAND    split-BF16 expansion P C': 0..6 register-staged tiles,
 *                      7..14 direct-to-LDS tiles (see gemm.hip), 15 the persistent
 *                      direct-to-LDS 128 x 128 tile (default)
 *   ABI_TUNE_FFT_BATCH bands per FFT batch (1..4096)
 *   ABI_TUNE_OVERLAP   0/1: FFT passes on a second stream beside the projection
 *   ABI_TUNE_GENERIC_FFT 0/1: runtime-size FFT passes also for cubic boxes that
 *                      have compile-time specialised ones (for testing them)
 *   ABI_TUNE_MIXED_GEMM form of the mixed projector products: 0 split-BF16
 *                      (default), 1 FP32 MFMA, 2 split-BF16 single-buffered
 *                      64 x 64 tile (comparison forms)
 *   ABI_TUNE_FILTER_GRAPH 0/1 (default 0): abi_cheb_filter(_hx) records its
 *                      launches into a HIP graph on the first call with given
 *                      blocks, degree and launch choices (that call runs them
 *                      eagerly too), and replays the graph on the caller's stream
 *                      for later calls with the same blocks, degree and choices,
 *                      taking each step's coefficients from a device table
 *                      uploaded before the replay (so new bounds need no new
 *                      graph).  Bit for bit the eager result.  A reallocation
 *                      of any work buffer, the second stream, the profiler or
 *                      a no-allocation call make the filter run eagerly.  (On
 *                      one MI355X the kernels, not the launches, bound the
 *                      filter down to the smallest workload: replays gain
 *                      nothing there, so it is off by default.)
 * Fails with ABI_ERR_ARG for an unknown parameter or a value out of range, and
 * with ABI_ERR_STATE for a mixed-form parameter on an FP64 handle. */
enum {
  ABI_TUNE_PROJ = 0,
  ABI_TUNE_EXPAND = 1,
  ABI_TUNE_FFT_BATCH = 2,
  ABI_TUNE_OVERLAP = 3,
  ABI_TUNE_GENERIC_FFT = 4,
  ABI_TUNE_MIXED_GEMM = 5,
  ABI_TUNE_FILTER_GRAPH = 6
};
abi_status abi_set_tuning(abi_system sys, int32_t param, int32_t value);
abi_status abi_get_tuning(abi_system sys, int32_t param, int32_t *value);

/* Autotuner (section "Batch processing": FFT plans and tile shapes chosen per
 * problem).  Times filter steps on the `nband` bands of X (dtype; X is only
 * read; H X - X, so that the last FFT pass also reads a previous block as in
 * the filter's three-term recurrence) with the launch choices above, one coordinate at a time from the
 * current ones (projection tile 14 / 15 / 11 / 4 and expansion tile 15 / 13 /
 * 9 / 6 for complex64 blocks on a mixed handle, then the FFT batch halved /
 * doubled, then the second stream), best of five timed applications each; a
 * candidate replaces the current choice only when it is more than 1% faster.
 * With a cache file (cache_path, or if it is NULL the file named
 * by the environment variable ABI_AUTOTUNE_CACHE; no file: no cache) the
 * choice is first looked up under the key (GPU architecture, CU count, plane
 * waves, projectors, bands, FFT box, dtype) and applied without timing
 * (*from_cache = 1, may be NULL), else stored after tuning.  The cache is a
 * JSON object of one entry per line that this call reads and rewrites.
 * Synchronises the stream. */
abi_status abi_autotune(abi_system sys, const void *X, int64_t nband, int64_t ld, int32_t dtype,
                        const char *cache_path, int32_t *from_cache, void *stream);

/* ---- timing ------------------------------------------------------------------
 * Per-kernel-class timing with HIP events recorded on the stream of each call
 * (the method of the paper's section "Single-step benchmarks: GPU kernel
 * rooflines": time and algorithmic work aggregated per code section).
 * Classes: 0 projection GEMM P^H X, 1 expansion GEMM P C', 2-4 FFT passes
 * A/B/C, 5 split-K sum + D (classes 0-5 count the launches inside
 * abi_cheb_filter only), 6 Gram and subspace GEMMs, 7 Cholesky + inverse +
 * reduction, 8 eigensolver, 9 rotations (classes 6-9: abi_rayleigh_ritz),
 * 10 splitting of the block into bf16 hi/lo planes (mixed form; filter only).
 * `work` is the algorithmic flop count (GEMM, dense classes) or HBM byte count
 * (FFT passes, plane splitting) of the timed launches. */

/* Turns timing on or off and clears the accumulated figures. */
abi_status abi_profile_enable(abi_system sys, int32_t on);

/* Waits for the recorded events and returns, for classes 0..nclass-1, the
 * summed milliseconds, summed work and number of timed launches (host arrays of
 * nclass entries; classes past the last one read as zero). */
abi_status abi_profile_read(abi_system sys, int32_t nclass, double *total_ms, double *work,
                            int64_t *count);

const char *abi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CHEBFI_H */
