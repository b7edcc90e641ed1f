// Host-side launchers of the HIP kernels (one declaration per kernel family).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "internal.h"

namespace chebfi {

enum Op { OP_N = 0, OP_C = 1 };  // op(X) = X or X^H

// ---- fft.hip ----------------------------------------------------------------
// Out[:, b] = alpha * (V_loc Yk[:, b] + (kin - cshift) Yk[:, b]) - beta * Yprev[:, b]
// for b in [band0, band0 + nb); Yprev may be null (then beta is ignored).
// `box` holds nb boxes; V is double (T = double) or float (T = float).
// E (optional, ld lde): a block added to Out on the sphere (the projector part
// of H computed beforehand), with a plain rounded add after the local value.
// ypl (optional, T = float only): also write Out's bf16 planes there (the
// layout of split_planes: band b at b * ldpl, plane stride pspl; the padding
// rows are left as they are).
template <typename T>
void launch_local_potential(const abi_system_s *s, const void *Yk, int64_t ldk, const void *Yprev,
                            int64_t ldp, void *Out, int64_t ldo, int band0, int nb, void *box,
                            const void *V, double alpha, double cshift, double beta,
                            hipStream_t st, Profiler *prof = nullptr, const void *E = nullptr,
                            int64_t lde = 0, void *ypl = nullptr, int64_t ldpl = 0,
                            int64_t pspl = 0);

// Local part of one reverse step of the filter adjoint for bands
// [band0, band0+nb): dV += gamma/n^3 sum_b Re[conj(Ak1~) Yk~] and
// Ak = gamma (V_loc Ak1 + (kin - cshift) Ak1) (+ Ak when accumulate).
// box1/box2 hold nb boxes each.  Runtime-size passes (any grid).
template <typename T>
void launch_adjoint_local(const abi_system_s *s, const void *Ak1, int64_t lda1, const void *Yk,
                          int64_t ldy, void *Ak, int64_t ldak, bool accumulate, int band0, int nb,
                          void *box1, void *box2, const void *V, double gamma, double cshift,
                          double *dV, hipStream_t st);

// rho += sum_b w[band0+b] |psi~_b(r)|^2 / (n1 n2 n3) for bands [band0, band0+nb)
// (w may be null: unit weights).  box holds nb boxes.
template <typename T>
void launch_density(const abi_system_s *s, const void *Psi, int64_t ld, int band0, int nb,
                    void *box, const double *w, double *rho, hipStream_t st);

// ---- gemm.hip ---------------------------------------------------------------
// C = alpha op(A) op(B) + beta C, complex double, column-major.  When `part`
// is non-null the K range is split in `splits` chunks and chunk z writes its
// raw product to part + z*m*n (ld = m); C, alpha and beta are then unused.
void zgemm(Op opa, Op opb, int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
           const void *B, int64_t ldb, void *C, int64_t ldc, double2 alpha, double2 beta,
           hipStream_t st, void *part = nullptr, int splits = 1);

// Projector products of the H application (same kernels, own instantiations):
// part[z] = P^H X over K chunk z, and Out += P C'.
// fp32 = true: complex float operands and FP32 MFMA (mixed form).
void proj_gemm(int64_t nproj, int64_t nband, int64_t npw, const void *P, const void *X,
               int64_t ldx, void *part, int splits, hipStream_t st, bool fp32 = false);
void expand_gemm(int64_t npw, int64_t nband, int64_t nproj, const void *P, const void *Cp,
                 void *Out, int64_t ldo, hipStream_t st, bool fp32 = false);
// Split-BF16 forms (mixed precision): A holds four bf16 planes (Re hi, Im hi,
// Re lo, Im lo) of P^T (projection, rows = projectors, k = plane waves) or of P
// (expansion, rows = plane waves, k = projectors), row stride lda (a multiple
// of 8), plane stride pstride; blocks are complex float.
void proj_gemm_bf16x3(int64_t nproj, int64_t nband, int64_t npw, const void *Apl, int64_t lda,
                      int64_t pstride, const void *Y, int64_t ldy, void *part, int splits,
                      hipStream_t st);
void expand_gemm_bf16x3(int64_t npw, int64_t nband, int64_t nproj, const void *Apl, int64_t lda,
                        int64_t pstride, const void *Cp, void *Out, int64_t ldo, hipStream_t st);
// Planes x planes forms: the block operand is also given as bf16 planes
// (column j = band j, contraction index contiguous, stride ld, plane stride ps).
void split_planes(int64_t rows, int64_t cols, const void *X, int64_t ld, void *planes,
                  int64_t ldp, hipStream_t st);
// The transposed planes of a complex float block X (rows x cols, ld): plane p
// holds row i of X as its row i with the column index contiguous (stride ldp
// >= cols, zero from cols to ldp), plane stride ldp * rows: the A operand of
// the expansion-form product X W.
void split_planes_t(int64_t rows, int64_t cols, const void *X, int64_t ld, void *planes,
                    int64_t ldp, hipStream_t st);
// `variant` selects the tile shape (0..6, see gemm.hip); proj_planes_splits
// gives the K split count that fills the chip for that shape.
int proj_planes_splits(int variant, int64_t nproj, int64_t nband, int64_t npw);
void proj_gemm_planes(int64_t nproj, int64_t nband, int64_t npw, const void *Apl, int64_t lda,
                      int64_t psa, const void *Ypl, int64_t ldy, int64_t psy, void *part,
                      int splits, hipStream_t st, int variant);
// part[z] = P^H Y for a complex float block Y (ld ldy), split into bf16 planes
// inside the kernel while staged (the 128 x 128 double-buffered tile).
void proj_gemm_planes_f32(int64_t nproj, int64_t nband, int64_t npw, const void *Apl, int64_t lda,
                          int64_t psa, const void *Y, int64_t ldy, void *part, int splits,
                          hipStream_t st);
// part[z] = P^H Y by BF32 projection variant (0: register-staged 128 x 128,
// 1, 2: direct-to-LDS 128 x 128 with 2 x 2 / 1 x 4 waves; these need the planes
// of P zero up to the next multiple of 32 plane waves).
void proj_gemm_f32_variant(int variant, int64_t nproj, int64_t nband, int64_t npw,
                           const void *Apl, int64_t lda, int64_t psa, const void *Y, int64_t ldy,
                           void *part, int splits, hipStream_t st);
// Out += P C' (accumulate) or Out = P C'
void expand_gemm_planes(int64_t npw, int64_t nband, int64_t nproj, const void *Apl, int64_t lda,
                        int64_t psa, const void *Cpl, int64_t ldc_pl, int64_t psc, void *Out,
                        int64_t ldo, hipStream_t st, int variant, bool accumulate = true);
// Split-BF16 products of the Rayleigh-Ritz step (FP32 accumulation):
// part[z] = Y_pl^H Y over plane-wave chunk z (m x m per chunk; the planes of
// Y_pl zero-padded to a multiple of 32, ld lda, Y complex64 with ld ldy), and
// Out = A T from the transposed planes of A (npw x m, ld lda) and the planes of
// T (m x m, ld ldt), both zero-padded along m.
void rr_gram_f32(int64_t m, int64_t npw, const void *Apl, int64_t lda, const void *Y,
                 int64_t ldy, void *part, int splits, hipStream_t st);
void rr_rotate_planes(int64_t npw, int64_t m, const void *Apl, int64_t lda, const void *Tpl,
                      int64_t ldt, void *Out, int64_t ldo, hipStream_t st);
// Single-band forms: c = P^H x, out += P c.
void proj_gemv(int64_t npw, int nproj, const void *P, const void *x, void *c, hipStream_t st);
void expand_gemv(int64_t npw, int nproj, const void *P, const void *c, void *out, hipStream_t st);

// Number of K splits that fills the chip for an m x n output.
int zgemm_splits(int64_t m, int64_t n, int64_t k);
// C (m x m, ldc) = A^H B for a product known to be Hermitian (Gram matrices):
// only the 64 x 64 tiles on and above the diagonal are multiplied (split-K
// into `part`, splits x m x m), the lower triangle is the conjugate mirror.
int zgemm_herm_splits(int64_t m, int64_t k);
void zgemm_herm(int64_t m, int64_t k, const void *A, int64_t lda, const void *B, int64_t ldb,
                void *C, int64_t ldc, hipStream_t st, void *part, int splits);

// C = alpha * sum_z part[z] + beta C  (m x n, part ld = m)
void zsum_parts(int64_t m, int64_t n, const void *part, int splits, void *C, int64_t ldc,
                double2 alpha, double2 beta, hipStream_t st);

// ---- stream.hip -------------------------------------------------------------
// Cprime[4R+i, b] = alpha * sum_j D_R[i][j] * sum_z part[z][4R+j, b]
// (fp32: complex float partials and output, FP64 arithmetic inside)
void launch_dapply(int natom, int64_t nband, const void *part, int splits, const void *D,
                   double alpha, void *Cprime, hipStream_t st, bool fp32 = false,
                   const double *coef = nullptr);

// rq[b] = Re(x_b^H hx_b) / Re(x_b^H sx_b); sx_b = x_b when SX is null
void launch_rayleigh_quotients(int64_t npw, int64_t nband, const void *X, int64_t ldx,
                               const void *HX, int64_t ldh, double *rq, hipStream_t st,
                               bool fp32 = false, const void *SX = nullptr, int64_t lds = 0);
// Small-matrix part of a generalised filter step (m x n complex double, ld m):
// G = sum of the split partials of P^H Out (complex float with fp32),
// E += G / alpha + cshift Ck + (beta / alpha) Ckm1 (Ckm1 may be null), Cnext = G.
void launch_gen_combine(int64_t m, int64_t n, const void *part, int splits, bool fp32,
                        const void *Ck, const void *Ckm1, double alpha, double cshift,
                        double beta, void *E, void *Cnext, hipStream_t st);
// out (m x n complex double, contiguous) = sum of the split partials
void launch_parts_to_c128(int64_t m, int64_t n, const void *part, int splits, bool fp32,
                          void *out, hipStream_t st);
// out[:, j] = W[:, j] mu_j / (1 + mu_j)  (m x m complex double)
void launch_woodbury_scale(int64_t m, const void *W, int64_t ldw, const double *mu, void *out,
                           int64_t ldo, hipStream_t st);
// *out = sqrt(max(*in, 0))
void launch_sqrt_scalar(const double *in, double *out, hipStream_t st);
// LOBPCG block helpers (npw x m complex double blocks, one column per band):
// W = HX - lam_b SX with res[b] = ||W_b||;  W_b *= Teter-Payne-Allan diagonal of X_b;
// columns of W, HW (, SW) scaled to unit S-norm (SW null: S = I).
void launch_resid_block(int64_t npw, int64_t m, const void *HX, const void *SX, int64_t ld,
                        const double *lam, void *W, int64_t ldw, double *res, hipStream_t st);
void launch_tpa(int64_t npw, int64_t m, const double *kin, const void *X, int64_t ldx, void *W,
                int64_t ldw, hipStream_t st);
void launch_snorm_scale(int64_t npw, int64_t m, void *W, void *HW, void *SW, int64_t ld,
                        hipStream_t st);
// complex block precision conversions (round to nearest when narrowing)
void launch_c64_to_c128(int64_t rows, int64_t cols, const void *src, int64_t lds, void *dst,
                        int64_t ldd, hipStream_t st);
void launch_c128_to_c64(int64_t rows, int64_t cols, const void *src, int64_t lds, void *dst,
                        int64_t ldd, hipStream_t st);
// out[0] = max rq, out[2] = min rq
void launch_minmax(int64_t n, const double *rq, double *out, hipStream_t st);

// Lanczos helpers (vectors of npw complex doubles, scalars in device memory).
void launch_dot_re(int64_t npw, const void *x, const void *y, double *out, hipStream_t st);
void launch_axpy_dev(int64_t npw, const double *coef, double sign, const void *x, void *y,
                     hipStream_t st);  // y += sign * (*coef) * x
void launch_multi_dot(int64_t npw, int nvec, const void *V, int64_t ldv, const void *w,
                      void *h, hipStream_t st);  // h[j] = v_j^H w
void launch_multi_axpy(int64_t npw, int nvec, const void *V, int64_t ldv, const void *h,
                       void *w, hipStream_t st);  // w -= V h
void launch_norm(int64_t npw, const void *x, double *out, hipStream_t st);
void launch_scale_inv(int64_t npw, const double *s, const void *x, void *y, hipStream_t st);
// out[1] = theta_max(T(alpha, beta[0..k-2])) + (add_last ? beta[k-1] : 0)
void launch_tridiag_bound(int k, const double *alpha, const double *beta, int add_last,
                          double *out, hipStream_t st);

// dD[R][i][j] += gamma sum_b CA[4R+i, b] conj(CY[4R+j, b])  (raw projections,
// complex double or, with fp32, complex float; dD is complex double)
void launch_dd_accum(int natom, int64_t nband, const void *CA, const void *CY, double gamma,
                     void *dD, hipStream_t st, bool fp32 = false);
// out = -delta * in  (complex double or, with fp32, complex float blocks)
void launch_scale_neg(int64_t npw, int64_t nband, const void *in, int64_t ldi, double delta,
                      void *out, int64_t ldo, hipStream_t st, bool fp32 = false);
// out (m x n, contiguous) = sum over the `splits` partial products of a split-K GEMM
void launch_sum_parts(int64_t m, int64_t n, const void *part, int splits, void *out,
                      hipStream_t st, bool fp32);
void launch_fill_zero(int64_t count_doubles, double *p, hipStream_t st);
void launch_d2f(int64_t n, const double *src, float *dst, hipStream_t st);

// resnorm[b] = || HPsi[:, b] - eval[b] Psi[:, b] ||
void launch_residual_norms(int64_t npw, int64_t nband, const void *Psi, int64_t ldp,
                           const void *HPsi, int64_t ldh, const double *eval, double *res,
                           hipStream_t st);

// the same for complex float blocks (FP64 sums)
void launch_residual_norms_f(int64_t npw, int64_t nband, const void *Psi, int64_t ldp,
                             const void *HPsi, int64_t ldh, const double *eval, double *res,
                             hipStream_t st);
// nrm[b] = ||X[:, b]||, inv[b] = 1 / nrm[b] (0 for a zero column)
void launch_col_norms(int64_t npw, int64_t nband, const void *X, int64_t ldx, double *nrm,
                      double *inv, hipStream_t st, bool fp32);
// out = alpha (HX - c X): the filter's first step from a given H X
void launch_cheb_first(int64_t npw, int64_t nband, const void *X, int64_t ldx, const void *HX,
                       int64_t ldh, double alpha, double c, void *out, int64_t ldo, hipStream_t st,
                       bool fp32, const double *coef = nullptr);
// *out = min_i (Re A[i, i])^2 (m x m complex double, one workgroup)
void launch_diag_min_sq(int64_t m, const void *A, int64_t lda, double *out, hipStream_t st);
// out[:, b] = sc[b] X[:, b] (complex float blocks)
void launch_scale_cols_f(int64_t rows, int64_t cols, const void *X, int64_t ldx, const double *sc,
                         void *out, int64_t ldo, hipStream_t st);
// A[k, j] *= sc[k] (m x n complex double)
void launch_scale_rows(int64_t m, int64_t n, void *A, int64_t lda, const double *sc,
                       hipStream_t st);

// dense helpers (m x m complex double)
void launch_hermitize(int64_t m, void *A, int64_t lda, hipStream_t st);  // A = (A + A^H)/2
void launch_copy_block(int64_t rows, int64_t cols, const void *src, int64_t lds, void *dst,
                       int64_t ldd, hipStream_t st, bool fp32 = false);
void launch_zero_lower(int64_t m, void *A, int64_t lda, hipStream_t st);

// ---- dense.hip ----------------------------------------------------------------
// Cholesky A = U^H U in place (upper); returns the failing pivot (1-based) via
// *info_dev (0 = success).
void zpotrf_upper(int64_t m, void *A, int64_t lda, int *info_dev, void *work, hipStream_t st);
size_t zpotrf_work_bytes(int64_t m);
// Inverse of an upper triangular matrix in place.
void ztrtri_upper(int64_t m, void *A, int64_t lda, void *work, hipStream_t st);
size_t ztrtri_work_bytes(int64_t m);
// Hermitian eigensolver: A (m x m, overwritten) -> w ascending, Z.
void zheev(int64_t m, void *A, int64_t lda, double *w, void *Z, int64_t ldz, void *work,
           hipStream_t st);
size_t zheev_work_bytes(int64_t m);

// Threads per workgroup that one Stockham stage over npen pencils of the plan needs
// (at most 4 butterflies per thread; a multiple of 64).
int fft_stage_threads(const Plan1D &pl, int npen);

// ---- scf.hip --------------------------------------------------------------------
// vout = vion + V_H + v_x of the grid density rho (sum_r rho = N_el): density per
// volume n = rho n1 n2 n3 / Omega, V_H(G) = 4 pi n(G) / |G|^2 by FFTs of the whole
// box (box: n1 n2 n3 complex doubles of work space), v_x = -(3 n / pi)^(1/3).
void launch_scf_potential(const abi_system_s *s, const double *rho, const double *vion,
                          double *vout, void *box, hipStream_t st);
// vnext = vin + K (vout - vin) with K = alpha (q0 <= 0) or Kerker's
// alpha |G|^2 / (|G|^2 + q0^2) (alpha at G = 0) applied through box FFTs (box:
// n1 n2 n3 complex doubles of work space); *dv = max |vout - vin| (device scalar).
void launch_mix(const abi_system_s *s, const double *vin, const double *vout, double alpha,
                double q0, double *vnext, double *dv, void *box, hipStream_t st);

// ---- batch.hip ------------------------------------------------------------------
// One filter step (index j of the step table) of every system of a batch:
// projection + D, FFT passes A, B, C (with expansion and recurrence).
// side, fork, join (all null, or none): the projector products run on side,
// beside passes A and B on st, and pass C waits for them.
template <typename T>
void batch_step(const BatchLaunch &L, int j, hipStream_t st, hipStream_t side = nullptr,
                hipEvent_t fork = nullptr, hipEvent_t join = nullptr);
// True if batched systems on a cubic box of this edge get specialised passes.
bool batch_edge_specialised(int n);
// planes (slabs) of one band per work item of the specialised batched passes
int batch_item_planes(int n, bool fp32);
// Sets the dynamic LDS limits of the batched kernels (call outside graph capture).
template <typename T> void batch_prepare(const BatchLaunch &L);

}  // namespace chebfi
