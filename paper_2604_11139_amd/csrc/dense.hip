// Dense FP64 linear algebra of the Rayleigh-Ritz step on one GPU.
//
// The paper solves the M x M problems redundantly on each process with
// vendor potrf / trsm / hegvd calls (arXiv 2604.11139, Algorithms "S-ortho"
// and "RR", section "Parallel implementation design"), and names hegvd the
// main AMD bottleneck (section "Single-step benchmarks: GPU kernel
// rooflines").  Here every step is a hand-written kernel:
//
// * Cholesky A = U^H U: right-looking blocked, 32-column diagonal blocks
//   factored in LDS by one workgroup, the panel solved column-parallel and the
//   trailing matrix updated by the MFMA GEMM;
// * U^-1: blocked, diagonal blocks inverted in LDS, off-diagonal panels by GEMM;
// * Hermitian eigensolver: Householder reduction to real symmetric tridiagonal
//   form (reflectors H = I - tau u u^H with a real sub-diagonal, applied from
//   both sides as rank-2 updates gathered in panels of 32 columns: per column
//   a read-only product with the trailing matrix and a row-parallel finish,
//   per panel one GEMM update),
//   eigenvalues by Sturm-count multisection (one wave per eigenvalue, 64
//   points per round), eigenvectors of the tridiagonal by inverse iteration
//   with partial-pivoting LU (one lane per isolated eigenvalue; one workgroup
//   with modified Gram-Schmidt per cluster of (nearly) equal eigenvalues),
//   then the reflectors applied back in blocks (compact WY).  These are the
//   classical Householder / bisection / inverse-iteration methods (Wilkinson;
//   Golub & Van Loan, "Matrix Computations", chapter 8).
#include <cfloat>

#include "cplx.h"
#include "kernels.h"

namespace chebfi {

namespace {

constexpr int NB = 32;           // Cholesky / trtri block size
constexpr int kEigMaxM = 8192;   // eigensolver size limit
constexpr int kLdsInvitM = 2560; // clusters' inverse iteration in LDS up to this size
constexpr int kBtBlock = 64;     // reflectors per block of the back-transformation
constexpr int kBtMinM = 96;      // smaller problems apply the reflectors one at a time
constexpr int kBtSplits = 8;     // most K chunks of the V^H Z product
constexpr int kBtGSplits = 64;   // most K chunks of the V^H V product

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ double block_sum(double v, double *scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < nw; ++w) t += scratch[w];
  return t;
}

// Block sum of a pair (one set of barriers; scratch holds 32 doubles).
__device__ double2 block_sum2(double2 v, double *scratch) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    scratch[2 * wave] = v.x;
    scratch[2 * wave + 1] = v.y;
  }
  __syncthreads();
  double2 t{0, 0};
  for (int w = 0; w < nw; ++w) {
    t.x += scratch[2 * w];
    t.y += scratch[2 * w + 1];
  }
  return t;
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------- Cholesky --
// Factor the nb x nb diagonal block at (j0, j0) in LDS (upper, A = U^H U).
__global__ __launch_bounds__(256) void potrf_diag_kernel(int nb, double2 *__restrict__ A, int64_t lda, int64_t j0,
                                  int *__restrict__ info) {
  __shared__ double2 a[NB][NB + 1];  // a[i][j] = A(j0+i, j0+j)
  const int t = threadIdx.x;
  for (int idx = t; idx < NB * NB; idx += blockDim.x) {
    const int i = idx % NB, j = idx / NB;
    if (i < nb && j < nb) a[i][j] = A[(j0 + i) + (j0 + j) * lda];
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    const double dkk = a[k][k].x;
    const bool bad = !(dkk > 0.0);
    const double dk = bad ? 1.0 : sqrt(dkk);
    __syncthreads();
    if (t == 0) {
      if (bad && *info == 0) *info = (int)(j0 + k + 1);
      a[k][k] = double2{dk, 0.0};
    }
    for (int j = k + 1 + t; j < nb; j += blockDim.x) a[k][j] = cscale(a[k][j], 1.0 / dk);
    __syncthreads();
    for (int idx = t; idx < NB * NB; idx += blockDim.x) {
      const int i = idx % NB, j = idx / NB;
      if (i > k && j >= i && j < nb) {
        const double2 u = a[k][i], v = a[k][j];
        const double2 cu{u.x, -u.y};
        a[i][j] = csub(a[i][j], cmul(cu, v));
      }
    }
    __syncthreads();
  }
  for (int idx = t; idx < NB * NB; idx += blockDim.x) {
    const int i = idx % NB, j = idx / NB;
    if (i <= j && j < nb) A[(j0 + i) + (j0 + j) * lda] = a[i][j];
  }
}

// U12 = U11^-H A12 for the panel rows j0..j0+nb-1, columns j1..m-1.
__global__ __launch_bounds__(64) void potrf_panel_kernel(int nb, int64_t m, double2 *__restrict__ A, int64_t lda,
                                   int64_t j0) {
  __shared__ double2 u[NB][NB + 1];
  const int t = threadIdx.x;
  for (int idx = t; idx < nb * nb; idx += blockDim.x) {
    const int i = idx % nb, j = idx / nb;
    u[i][j] = A[(j0 + i) + (j0 + j) * lda];
  }
  __syncthreads();
  const int64_t col = j0 + nb + (int64_t)blockIdx.x * blockDim.x + t;
  if (col >= m) return;
  double2 x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) x[i] = (i < nb) ? A[(j0 + i) + col * lda] : double2{0, 0};
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i < nb) {
      double2 s = x[i];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (k < i) {
          const double2 cu{u[k][i].x, -u[k][i].y};
          s = csub(s, cmul(cu, x[k]));
        }
      }
      x[i] = cscale(s, 1.0 / u[i][i].x);
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i < nb) A[(j0 + i) + col * lda] = x[i];
}

__global__ void set_int_kernel(int *p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---------------------------------------------------------------- trtri ----
// Invert the nb x nb upper triangular diagonal block in place (LDS).
__global__ __launch_bounds__(256) void trtri_diag_kernel(int nb, double2 *__restrict__ A, int64_t lda, int64_t j0) {
  static_assert(NB == 32, "one lane group of 32 per column block");
  __shared__ double2 a[NB][NB + 1];
  __shared__ double2 r[NB][NB + 1];
  __shared__ double2 part[8][NB];
  const int t = threadIdx.x;
  for (int idx = t; idx < NB * NB; idx += blockDim.x) {
    const int i = idx % NB, j = idx / NB;
    if (i < nb && j < nb) a[i][j] = (i <= j) ? A[(j0 + i) + (j0 + j) * lda] : double2{0, 0};
  }
  __syncthreads();
  // rows of R = U^-1 from the bottom: R[i][j] = (delta_ij - sum_{i<k<=j} U[i][k] R[k][j]) / U[i][i]
  // for all j >= i at once; each column's sum is split over 8 groups of 32 threads
  const int j = t & 31, g = t >> 5;
  for (int i = nb - 1; i >= 0; --i) {
    double2 s{0, 0};
    if (j < nb && j > i)
      for (int k = i + 1 + g; k <= j; k += 8) s = cadd(s, cmul(a[i][k], r[k][j]));
    part[g][j] = s;
    __syncthreads();
    if (t < nb) {
      double2 v{0, 0};
      if (t >= i) {
        double2 sum{0, 0};
#pragma unroll
        for (int q = 0; q < 8; ++q) sum = cadd(sum, part[q][t]);
        v = csub((t == i) ? double2{1.0, 0.0} : double2{0, 0}, sum);
        const double2 d = a[i][i];
        const double den = d.x * d.x + d.y * d.y;
        v = double2{(v.x * d.x + v.y * d.y) / den, (v.y * d.x - v.x * d.y) / den};
      }
      r[i][t] = v;
    }
    __syncthreads();
  }
  for (int idx = t; idx < NB * NB; idx += blockDim.x) {
    const int i = idx % NB, jj = idx / NB;
    if (i < nb && jj < nb) A[(j0 + i) + (j0 + jj) * lda] = (i <= jj) ? r[i][jj] : double2{0, 0};
  }
}

// ------------------------------------------------------ tridiagonalisation --
// Column c of the reduction uses the reflector H_c = I - tau_c u_c u_c^H of
// the current column c below its subdiagonal (u_c[c+1] = 1, zero above), the
// product p_c = tau_c A22 u_c with the current trailing matrix A22 =
// A[c+1:, c+1:], a2_c = -tau_c (p_c^H u_c) / 2 and w_c = p_c + a2_c u_c; the
// two-sided application is the rank-2 update A22 -= u_c w_c^H + w_c u_c^H.
//
// The updates are applied in panels of kTriNB columns (the blocked form of
// the reduction, Golub & Van Loan section 8.3, as in LAPACK's hetrd/latrd):
// within a panel the stored matrix keeps its values from the panel's start,
// the current matrix being A - U W^H - W U^H over the panel's earlier columns
// (U holds their u, W their w).  So the product A22 u_c reads the stored
// matrix once, without writing it, and is corrected by the panel's small
// products, p_c = tau_c (A22 u_c - U (W^H u_c) - W (U^H u_c)); at the panel's
// end one GEMM applies A22 -= [U W] [W U]^H.  Each column takes two launches:
// tri_mv_kernel (the reflector of column c; one workgroup per trailing column
// for (A22 u_c)_i = (column i)^H u_c, A22 being Hermitian; and per block of 64
// rows the partial products U^H u_c and W^H u_c) and tri_fin_kernel (rows in
// blocks of 64: w_c, and the current column c+1 with the partial sums of
// squares of its entries below the subdiagonal).  The first column of a panel
// is copied by tri_start_kernel after the panel update.

constexpr int kTriNB = 32;     // columns per panel
constexpr int kTriRows = 64;   // rows per block
constexpr int kTriFinT = 512;  // threads of tri_fin_kernel: 8 groups share the panel columns

__device__ __forceinline__ double2 conj2(double2 a) { return double2{a.x, -a.y}; }

// Reflector of the current column (alpha = its entry on the subdiagonal,
// xnorm2 = the sum of squares below it): H^H (alpha, x) = (beta, 0) with beta
// real (LAPACK's larfg convention); u = (1, x * scal).
struct Reflector {
  double beta;
  double2 tau, scal;
};
__device__ Reflector make_reflector(double2 alpha, double xnorm2) {
  Reflector h;
  h.scal = double2{0.0, 0.0};
  if (xnorm2 == 0.0 && alpha.y == 0.0) {
    h.beta = alpha.x;
    h.tau = double2{0.0, 0.0};
    return h;
  }
  const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xnorm2);
  h.beta = (alpha.x >= 0.0) ? -nrm : nrm;
  h.tau = double2{(h.beta - alpha.x) / h.beta, -alpha.y / h.beta};
  const double2 den{alpha.x - h.beta, alpha.y};
  const double dd = den.x * den.x + den.y * den.y;
  h.scal = double2{den.x / dd, -den.y / dd};
  return h;
}

// Column c (rows c .. m-1) of the stored matrix as the current column (the
// first of a panel): x, d[c], and per block of 64 rows the sum of squares of
// the rows >= c + 2.  One wave per block.
__global__ __launch_bounds__(64) void tri_start_kernel(int64_t m, const double2 *__restrict__ A,
                                                       int64_t lda, int64_t c,
                                                       double2 *__restrict__ x,
                                                       double *__restrict__ d,
                                                       double *__restrict__ normpart) {
  const int64_t r = c + (int64_t)kTriRows * blockIdx.x + threadIdx.x;
  double s = 0.0;
  if (r < m) {
    const double2 a = A[r + c * lda];
    x[r] = a;
    if (r == c) d[c] = a.x;
    if (r >= c + 2) s = a.x * a.x + a.y * a.y;
  }
  s = wave_sum(s);
  if (threadIdx.x == 0) normpart[blockIdx.x] = s;
}

// Panel column k = c - j0, L = m - c - 1 trailing columns.  Workgroups
// 0 .. L-1: column i = c + 1 + blockIdx.x, y[i] = (column i)^H u_c over rows
// c+1 .. m-1 and yupart[blockIdx.x] = conj(y[i]) u_c[i].  Workgroups L .. L +
// nrb - 1: rows in blocks of 64, u_c stored into A (rows >= c + 2, read by the
// back-transformation), into column k of U in P1 = [U | W] (m x 2 kTriNB,
// ld m) and, conjugated, into Q = [W | U]^H (2 kTriNB x m, ld 2 kTriNB); and
// stpart[rb * 2 kTriNB + i] = U_i^H u_c (i < kTriNB), then W_i^H u_c, over
// the block's rows for the panel columns < k.
__global__ __launch_bounds__(256) void tri_mv_kernel(
    int64_t m, double2 *__restrict__ A, int64_t lda, int64_t c, int k,
    const double2 *__restrict__ x, const double *__restrict__ normpart, int nparts,
    double2 *__restrict__ P1, double2 *__restrict__ Q, double2 *__restrict__ y,
    double2 *__restrict__ yupart, double2 *__restrict__ stpart, double *__restrict__ e,
    double2 *__restrict__ tau) {
  __shared__ double scratch[32];
  __shared__ double2 urow[kTriRows];
  __shared__ double2 red[4][2 * kTriNB];
  const int t = threadIdx.x, lane = t & 63;
  const int64_t L = m - c - 1;
  // the reflector of column c (every wave computes it)
  double s = 0.0;
  for (int i = lane; i < nparts; i += 64) s += normpart[i];
  const Reflector h = make_reflector(x[c + 1], wave_sum(s));
  if (blockIdx.x == 0 && t == 0) {
    e[c] = h.beta;
    tau[c] = h.tau;
  }
  if (blockIdx.x < L) {
    const int64_t i = c + 1 + blockIdx.x;
    const double2 *col = A + i * lda;
    const double2 a1 = col[c + 1], xi = x[i];
    double2 acc{0.0, 0.0};  // (rows >= c + 2 of column i)^H x
    for (int64_t r = c + 2 + t; r < m; r += 256) {
      const double2 a = col[r], v = x[r];
      acc.x += a.x * v.x + a.y * v.y;
      acc.y += a.x * v.y - a.y * v.x;
    }
    const double2 dot = block_sum2(acc, scratch);
    if (t == 0) {
      const double2 yi = cadd(conj2(a1), cmul(h.scal, dot));  // u_c[c+1] = 1
      const double2 ui = (i == c + 1) ? double2{1.0, 0.0} : cmul(xi, h.scal);
      y[i] = yi;
      yupart[blockIdx.x] = cmul(conj2(yi), ui);
    }
    return;
  }
  const int64_t r0 = c + 1 + (int64_t)kTriRows * (blockIdx.x - L);
  if (t < kTriRows) {
    const int64_t r = r0 + t;
    double2 u{0.0, 0.0};
    if (r < m) {
      u = (r == c + 1) ? double2{1.0, 0.0} : cmul(x[r], h.scal);
      if (r >= c + 2) A[r + c * lda] = u;
      P1[r + (int64_t)k * m] = u;
      Q[(kTriNB + k) + r * 2 * kTriNB] = conj2(u);
    }
    urow[t] = u;
  }
  if (k == 0) return;
  __syncthreads();
  // thread (column i = t & 63, quarter q = t >> 6) sums 16 rows
  const int i = t & 63, q = t >> 6, ii = i & (kTriNB - 1);
  double2 dq{0.0, 0.0};
  if (ii < k) {
    const double2 *pc = P1 + (int64_t)(i < kTriNB ? ii : kTriNB + ii) * m;
    for (int l = 16 * q; l < 16 * q + 16; ++l) {
      const int64_t rl = r0 + l;
      if (rl < m) dq = cadd(dq, cmul(conj2(pc[rl]), urow[l]));
    }
  }
  red[q][i] = dq;
  __syncthreads();
  if (t < 2 * kTriNB)
    stpart[(int64_t)(blockIdx.x - L) * 2 * kTriNB + t] =
        cadd(cadd(red[0][t], red[1][t]), cadd(red[2][t], red[3][t]));
}

// Rows c+1 .. m-1 in blocks of 64 (thread: row lane = t & 63, group g = t >> 6
// of 8, the groups sharing the panel columns): w_c = tau_c (y - U s - W t) +
// a2_c u_c with s = W^H u_c, t = U^H u_c and a2_c = -|tau_c|^2 (u_c^H A22 u_c
// - s^H t - t^H s) / 2, stored as column k of W in P1 and Q.  With next != 0
// also the current column c+1: A[:, c+1] - [U u_c] [W w_c]^H[:, c+1] -
// [W w_c] [U u_c]^H[:, c+1] into x (rows c+1 .. m-1), d[c+1], and the
// per-block sums of squares of its rows >= c + 3.  nrb: the row blocks of
// tri_mv_kernel's partial products.
__global__ __launch_bounds__(kTriFinT) void tri_fin_kernel(
    int64_t m, const double2 *__restrict__ A, int64_t lda, int64_t c, int k, int next, int nrb,
    double2 *__restrict__ P1, double2 *__restrict__ Q, const double2 *__restrict__ y,
    const double2 *__restrict__ yupart, const double2 *__restrict__ stpart,
    const double2 *__restrict__ tau, double2 *__restrict__ x, double *__restrict__ d,
    double *__restrict__ normpart) {
  constexpr int NG = kTriFinT / 64, NJ = kTriNB / NG;
  __shared__ double2 st[2 * kTriNB];
  __shared__ double2 red[NG][kTriRows];
  __shared__ double2 red2[NG][kTriRows];
  __shared__ double sred[NG][6];
  const int t = threadIdx.x, lane = t & 63, g = t >> 6;
  const int64_t L = m - c - 1;
  const int64_t r = c + 1 + (int64_t)kTriRows * blockIdx.x + lane;
  const bool in = r < m;
  // loads that depend on nothing else: this row's panel entries (columns
  // i = g + NG j), row c+1's, this row's y, u and A[r, c+1], the partials
  double2 ur[NJ], wr[NJ], uc1[NJ], wc1r[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int i = g + NG * j;
    const bool ok = i < k;
    ur[j] = ok && in ? P1[r + (int64_t)i * m] : double2{0.0, 0.0};
    wr[j] = ok && in ? P1[r + (int64_t)(kTriNB + i) * m] : double2{0.0, 0.0};
    uc1[j] = ok ? P1[c + 1 + (int64_t)i * m] : double2{0.0, 0.0};
    wc1r[j] = ok ? P1[c + 1 + (int64_t)(kTriNB + i) * m] : double2{0.0, 0.0};
  }
  const double2 yr = in ? y[r] : double2{0.0, 0.0};
  const double2 u = in ? P1[r + (int64_t)k * m] : double2{0.0, 0.0};
  const double2 anext = (in && next) ? A[r + (c + 1) * lda] : double2{0.0, 0.0};
  const double2 yc1 = y[c + 1];
  const double2 tc = tau[c];
  double2 yu{0.0, 0.0};
  for (int64_t b = t; b < L; b += kTriFinT) yu = cadd(yu, yupart[b]);
  double2 stp{0.0, 0.0};
  if ((lane & (kTriNB - 1)) < k)
    for (int b = g; b < nrb; b += NG) stp = cadd(stp, stpart[(int64_t)b * 2 * kTriNB + lane]);
  // s and t
  red[g][lane] = stp;
  __syncthreads();
  if (t < 2 * kTriNB) {
    double2 v{0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NG; ++q) v = cadd(v, red[q][t]);
    st[t] = v;
  }
  __syncthreads();
  // one block reduction: u^H A22 u, s^H t + t^H s and row c+1's correction
  // (the last two from each group's panel columns, counted on its lane 0)
  double2 sht{0.0, 0.0}, cc1{0.0, 0.0}, corr{0.0, 0.0}, ncorr{0.0, 0.0};
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int i = g + NG * j;
    if (i < k) {
      const double2 ti = st[i], si = st[kTriNB + i];
      sht = cadd(sht, cadd(cmul(conj2(si), ti), cmul(conj2(ti), si)));
      cc1 = cadd(cc1, cadd(cmul(uc1[j], si), cmul(wc1r[j], ti)));
      corr = cadd(corr, cadd(cmul(ur[j], si), cmul(wr[j], ti)));
      ncorr = cadd(ncorr, cadd(cmul(ur[j], conj2(wc1r[j])), cmul(wr[j], conj2(uc1[j]))));
    }
  }
  if (lane != 0) {
    sht = double2{0.0, 0.0};
    cc1 = double2{0.0, 0.0};
  }
  double v6[6] = {yu.x, yu.y, sht.x, sht.y, cc1.x, cc1.y};
#pragma unroll
  for (int q = 0; q < 6; ++q) v6[q] = wave_sum(v6[q]);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 6; ++q) sred[g][q] = v6[q];
  red[g][lane] = corr;
  red2[g][lane] = ncorr;
  __syncthreads();
  if (g != 0) return;
  double tot[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < NG; ++q)
#pragma unroll
    for (int p = 0; p < 6; ++p) tot[p] += sred[q][p];
  const double tt = tc.x * tc.x + tc.y * tc.y;
  const double2 a2 = cscale(double2{tot[0] - tot[2], tot[1] - tot[3]}, -0.5 * tt);
  const double2 wc1 = cadd(cmul(tc, csub(yc1, double2{tot[4], tot[5]})), a2);  // u_c[c+1] = 1
  double s2 = 0.0;
  if (in) {
    double2 cs{0.0, 0.0}, ns{0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      cs = cadd(cs, red[q][lane]);
      ns = cadd(ns, red2[q][lane]);
    }
    const double2 w = (r == c + 1) ? wc1 : cadd(cmul(tc, csub(yr, cs)), cmul(a2, u));
    P1[r + (int64_t)(kTriNB + k) * m] = w;
    Q[k + r * 2 * kTriNB] = conj2(w);
    if (next) {
      // the panel's column k term: u[r] conj(w[c+1]) + w[r] conj(u[c+1]), u[c+1] = 1
      const double2 a = csub(csub(anext, ns), cadd(cmul(u, conj2(wc1)), w));
      x[r] = a;
      if (r == c + 1) d[c + 1] = a.x;
      if (r >= c + 3) s2 = a.x * a.x + a.y * a.y;
    }
  }
  if (next) {
    s2 = wave_sum(s2);
    if (lane == 0) normpart[blockIdx.x] = s2;
  }
}

// ---------------------------------------------------------------- bisection --
__device__ int sturm_less(int64_t m, const double *d, const double *e2, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++cnt;
  for (int64_t i = 1; i < m; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// The same count with d and e2 in LDS (the recurrence's operands are then a
// short LDS read away instead of a global one).
__device__ int sturm_less_lds(int64_t m, const double *d, const double *e2, double x,
                              double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++cnt;
#pragma unroll 4
  for (int64_t i = 1; i < m; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
  }
  return cnt;
}

__global__ __launch_bounds__(256) void tri_prep_kernel(int64_t m, const double *__restrict__ d,
                                const double *__restrict__ e, double *__restrict__ e2,
                                double *__restrict__ stats) {
  // stats[0] = Gershgorin lower, stats[1] = upper, stats[2] = |T| scale, stats[3] = pivmin
  __shared__ double slo[256], shi[256], smax[256];
  double lo = 1e300, hi = -1e300, mx = 0, emax2 = 0;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < m - 1 ? fabs(e[i]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    mx = fmax(mx, fmax(fabs(d[i] - r), fabs(d[i] + r)));
    if (i < m - 1) {
      e2[i] = e[i] * e[i];
      emax2 = fmax(emax2, e2[i]);
    }
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  smax[threadIdx.x] = fmax(mx, emax2);
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + s]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + s]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double scale = fmax(fmax(fabs(slo[0]), fabs(shi[0])), 1e-300);
    stats[0] = slo[0] - 2.0 * DBL_EPSILON * scale * (double)m - 1e-300;
    stats[1] = shi[0] + 2.0 * DBL_EPSILON * scale * (double)m + 1e-300;
    stats[2] = scale;
    stats[3] = fmax(DBL_MIN, DBL_MIN * smax[0]);
  }
}

// Eigenvalue i (ascending) by multisection: one wave per eigenvalue, its 64
// lanes take Sturm counts at 64 interior points of the bracket [lo, hi], which
// shrinks to the sub-interval where the count first reaches i + 1 (65 times
// narrower per round), until it is below the tolerance or no representable
// point is left inside.
// lds != 0: d and e2 are first copied into LDS (2 m doubles of dynamic LDS),
// which the Sturm recurrences of the workgroup's four waves then read
__global__ __launch_bounds__(256) void bisect_kernel(int64_t m, const double *__restrict__ d,
                                                     const double *__restrict__ e2,
                                                     const double *__restrict__ stats,
                                                     double *__restrict__ w, int lds) {
  extern __shared__ double sde[];
  if (lds) {
    for (int64_t j = threadIdx.x; j < m; j += blockDim.x) {
      sde[j] = d[j];
      sde[m + j] = j + 1 < m ? e2[j] : 0.0;
    }
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= m) return;  // uniform per wave
  double lo = stats[0], hi = stats[1];
  const double pivmin = stats[3];
  const double tol = 2.0 * DBL_EPSILON * stats[2];
  for (int it = 0; it < 64; ++it) {
    if (hi - lo <= tol) break;
    const double x = lo + (hi - lo) * ((double)(lane + 1) * (1.0 / 65.0));
    const bool inside = x > lo && x < hi;
    if (__ballot(inside) == 0ull) break;
    const bool above =
        inside ? (lds ? sturm_less_lds(m, sde, sde + m, x, pivmin) : sturm_less(m, d, e2, x, pivmin)) >=
                     i + 1
               : x >= hi;
    const unsigned long long mask = __ballot(above);
    const int k = mask ? __ffsll((long long)mask) - 1 : 64;
    const double xk = __shfl(x, k < 64 ? k : 63, 64), xk1 = __shfl(x, k > 0 ? k - 1 : 0, 64);
    const double nlo = k == 0 ? lo : xk1;
    const double nhi = k == 64 ? hi : xk;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) w[i] = 0.5 * (lo + hi);
}

// ------------------------------------------------------- inverse iteration --
__device__ __forceinline__ double hash_uniform(uint64_t a, uint64_t b) {
  // splitmix64 of (a, b) -> (-1, 1)
  uint64_t z = a * 0x9E3779B97F4A7C15ull + b + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return ((double)(z >> 11) * (1.0 / 9007199254740992.0)) * 2.0 - 1.0;
}

// Value of a wave-uniform lane k (k a compile-time constant in the unrolled
// sequential loops below).
__device__ __forceinline__ double lane_val(double v, int k) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, k);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Inverse iteration for the eigenvalues with no neighbour within the cluster
// gap (1e-6 |T|): one lane per eigenvalue, 64 per wave, each lane running the
// same steps as the workgroup form below without the Gram-Schmidt (LU with
// partial pivoting of T - lambda I, three solves from the same seeded start,
// each followed by scaling to max 1 and normalisation; sign of the largest
// component positive).  The factors and the iterate live in `work`, interleaved
// by lane (element i of lane l at i * 64 + l within the wave's slab), so that
// each sequential step of the 64 lanes is one coalesced access.
__global__ __launch_bounds__(64) void invit_lane_kernel(
    int64_t m, const double *__restrict__ d, const double *__restrict__ e,
    const double *__restrict__ w, const double *__restrict__ stats, double *__restrict__ S,
    int64_t lds, double *__restrict__ work, unsigned char *__restrict__ wswp) {
  const int lane = threadIdx.x;
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  const double scale = stats[2];
  const double gaptol = 1e-6 * scale;
  if (q >= m) return;
  if (q > 0 && w[q] - w[q - 1] <= gaptol) return;         // in a cluster
  if (q + 1 < m && w[q + 1] - w[q] <= gaptol) return;     // in a cluster
  const int64_t slab = m * 64, nb = gridDim.x, b = blockIdx.x;
  double *rud = work + (0 * nb + b) * slab + lane;
  double *u1 = work + (1 * nb + b) * slab + lane;
  double *u2 = work + (2 * nb + b) * slab + lane;
  double *lm = work + (3 * nb + b) * slab + lane;
  double *x = work + (4 * nb + b) * slab + lane;
  unsigned char *swp = wswp + b * slab + lane;
  const double tiny = DBL_EPSILON * scale;
  const double shift = w[q];
  // LU with partial pivoting of T - shift I
  double a = d[0] - shift;
  double cc = (m > 1) ? e[0] : 0.0;
  for (int64_t i = 0; i < m - 1; ++i) {
    const double bb = e[i], an = d[i + 1] - shift, cn = (i + 1 < m - 1) ? e[i + 1] : 0.0;
    const bool keep = fabs(a) >= fabs(bb);
    const double num = keep ? bb : a, den = keep ? a : bb;
    const double l = (den != 0.0) ? num / den : 0.0;
    double piv = den;
    if (fabs(piv) < tiny) piv = (piv < 0.0) ? -tiny : tiny;
    rud[i * 64] = 1.0 / piv;
    u1[i * 64] = keep ? cc : an;
    u2[i * 64] = keep ? 0.0 : cn;
    lm[i * 64] = l;
    swp[i * 64] = keep ? 0 : 1;
    const double na = keep ? an - l * cc : cc - l * an;
    cc = keep ? cn : -l * cn;
    a = na;
  }
  rud[(m - 1) * 64] = 1.0 / ((fabs(a) < tiny) ? ((a < 0.0) ? -tiny : tiny) : a);
  for (int64_t i = 0; i < m; ++i) x[i * 64] = hash_uniform(q, i);
  // the solves load the operands of kB steps into registers before running them
  // (one memory latency per block instead of per step)
  constexpr int kB = 32;
  for (int it = 0; it < 3; ++it) {
    double cur = x[0];
    int64_t i0 = 0;
    for (; i0 + kB <= m - 1; i0 += kB) {
      double nx[kB], l[kB];
      unsigned char sw[kB];
#pragma unroll
      for (int k = 0; k < kB; ++k) {
        nx[k] = x[(i0 + k + 1) * 64];
        l[k] = lm[(i0 + k) * 64];
        sw[k] = swp[(i0 + k) * 64];
      }
#pragma unroll
      for (int k = 0; k < kB; ++k) {
        const double c = sw[k] ? nx[k] : cur;
        const double n = (sw[k] ? cur : nx[k]) - l[k] * c;
        x[(i0 + k) * 64] = c;
        cur = n;
      }
    }
    for (int64_t i = i0; i < m - 1; ++i) {
      const double nx = x[(i + 1) * 64], l = lm[i * 64];
      const bool sw = swp[i * 64] != 0;
      const double c = sw ? nx : cur;
      const double n = (sw ? cur : nx) - l * c;
      x[i * 64] = c;
      cur = n;
    }
    double x1 = cur * rud[(m - 1) * 64], x2 = 0.0;
    x[(m - 1) * 64] = x1;
    double mx = fabs(x1);
    int64_t i1 = m - 2;
    for (; i1 - kB + 1 >= 0; i1 -= kB) {
      double xv[kB], a1[kB], a2[kB], r[kB];
#pragma unroll
      for (int k = 0; k < kB; ++k) {
        const int64_t i = i1 - k;
        xv[k] = x[i * 64];
        a1[k] = u1[i * 64];
        a2[k] = u2[i * 64];
        r[k] = rud[i * 64];
      }
#pragma unroll
      for (int k = 0; k < kB; ++k) {
        const double x0 = (xv[k] - a1[k] * x1 - a2[k] * x2) * r[k];
        x[(i1 - k) * 64] = x0;
        mx = fmax(mx, fabs(x0));
        x2 = x1;
        x1 = x0;
      }
    }
    for (int64_t i = i1; i >= 0; --i) {
      const double x0 = (x[i * 64] - u1[i * 64] * x1 - u2[i * 64] * x2) * rud[i * 64];
      x[i * 64] = x0;
      mx = fmax(mx, fabs(x0));
      x2 = x1;
      x1 = x0;
    }
    const double inv = (mx > 0) ? 1.0 / mx : 1.0;
    double nn = 0;
#pragma unroll 8
    for (int64_t i = 0; i < m; ++i) {
      const double v = x[i * 64] * inv;
      x[i * 64] = v;
      nn += v * v;
    }
    const double invn = (nn > 0) ? 1.0 / sqrt(nn) : 1.0;
#pragma unroll 8
    for (int64_t i = 0; i < m; ++i) x[i * 64] *= invn;
  }
  double best = -1.0;
  int64_t bi = 0;
  for (int64_t i = 0; i < m; ++i)
    if (fabs(x[i * 64]) > best) {
      best = fabs(x[i * 64]);
      bi = i;
    }
  const double sg = (x[bi * 64] < 0) ? -1.0 : 1.0;
  double *sq = S + q * lds;
  for (int64_t i = 0; i < m; ++i) sq[i] = sg * x[i * 64];
}

// One workgroup per cluster of eigenvalues closer than `gaptol`; the group
// leader (first index of the cluster) computes all members in order.
// S (m x m, real, column-major, lds) receives the tridiagonal eigenvectors.
// gws: NULL, or (m above kLdsInvitM) a global slab of `per` bytes for each
// cluster leader, which then holds the arrays kept in LDS otherwise.
__global__ __launch_bounds__(256) void invit_kernel(int64_t m, const double *__restrict__ d, const double *__restrict__ e,
                             const double *__restrict__ w, const double *__restrict__ stats,
                             double *__restrict__ S, int64_t lds, unsigned char *gws,
                             size_t per) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t c0 = blockIdx.x;
  const double scale = stats[2];
  const double gaptol = 1e-6 * scale;
  if (c0 > 0 && w[c0] - w[c0 - 1] <= gaptol) return;  // not a cluster leader
  int64_t c1 = c0 + 1;
  while (c1 < m && w[c1] - w[c1 - 1] <= gaptol) ++c1;
  if (c1 == c0 + 1) return;  // a lone eigenvalue: invit_lane_kernel

  double *sd = reinterpret_cast<double *>(gws ? gws + (size_t)c0 * per : smem_raw);
  double *se = sd + m;
  double *rud = se + m;  // reciprocals of U's diagonal
  double *u1 = rud + m;  // first superdiagonal
  double *u2 = u1 + m;   // second superdiagonal
  double *lm = u2 + m;   // multipliers
  double *x = lm + m;
  unsigned char *swp = reinterpret_cast<unsigned char *>(x + m);
  __shared__ double scratch[16];
  __shared__ int sh_idx[16];
  __shared__ double sh_coef;

  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    sd[i] = d[i];
    se[i] = (i < m - 1) ? e[i] : 0.0;
  }
  __syncthreads();
  const double tiny = DBL_EPSILON * scale;
  const double pert = 10.0 * DBL_EPSILON * scale;
  double shift_prev = 0.0;
  for (int64_t q = c0; q < c1; ++q) {
    double shift = w[q];
    if (q > c0 && shift - shift_prev < pert) shift = shift_prev + pert;
    shift_prev = shift;
    // LU with partial pivoting of T - shift I.  The recurrence is sequential:
    // wave 0 loads the operands of 64 steps at once (one per lane), runs the
    // 64 steps on lane-broadcast values in registers, and lane k keeps the
    // factors of step k; the reciprocal pivots follow in a parallel pass.
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      double a = sd[0] - shift;
      double cc = (m > 1) ? se[0] : 0.0;  // current superdiagonal of row i
      for (int64_t i0 = 0; i0 < m - 1; i0 += 64) {
        const int64_t ii = i0 + lane;
        const double Bv = (ii < m - 1) ? se[ii] : 0.0;        // subdiagonal (row i+1, col i)
        const double Dv = (ii + 1 < m) ? sd[ii + 1] : 0.0;    // diagonal of row i+1
        const double Ev = (ii + 1 < m - 1) ? se[ii + 1] : 0.0;  // superdiagonal of row i+1
        double P = 0.0, Lo = 0.0, V1 = 0.0, V2 = 0.0;
        int SW = 0;
#pragma unroll
        for (int k = 0; k < 64; ++k) {
          if (i0 + k >= m - 1) break;
          const double b = lane_val(Bv, k), an = lane_val(Dv, k) - shift, cn = lane_val(Ev, k);
          const bool keep = fabs(a) >= fabs(b);
          const double num = keep ? b : a, den = keep ? a : b;
          const double l = (den != 0.0) ? num / den : 0.0;
          const double na = keep ? an - l * cc : cc - l * an;
          const double ncc = keep ? cn : -l * cn;
          if (lane == k) {
            P = den;
            Lo = l;
            V1 = keep ? cc : an;
            V2 = keep ? 0.0 : cn;
            SW = keep ? 0 : 1;
          }
          a = na;
          cc = ncc;
        }
        if (ii < m - 1) {
          rud[ii] = (fabs(P) < tiny) ? ((P < 0.0) ? -tiny : tiny) : P;
          lm[ii] = Lo;
          u1[ii] = V1;
          u2[ii] = V2;
          swp[ii] = (unsigned char)SW;
        }
      }
      if (lane == 0) rud[m - 1] = (fabs(a) < tiny) ? ((a < 0.0) ? -tiny : tiny) : a;
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) rud[i] = 1.0 / rud[i];
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) x[i] = hash_uniform(q, i);
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
      if (threadIdx.x < 64) {
        // forward: row swaps and L, 64 steps per block as in the factorisation
        // (each block reads x[i0+1 .. i0+64] before writing x[i0 .. i0+63])
        const int lane = threadIdx.x;
        double cur = x[0];
        for (int64_t i0 = 0; i0 < m - 1; i0 += 64) {
          const int64_t ii = i0 + lane;
          const double Xv = (ii + 1 < m) ? x[ii + 1] : 0.0;
          const double Lv = (ii < m - 1) ? lm[ii] : 0.0;
          const int Sv = (ii < m - 1) ? (int)swp[ii] : 0;
          double out = 0.0;
#pragma unroll
          for (int k = 0; k < 64; ++k) {
            if (i0 + k >= m - 1) break;
            const double nx = lane_val(Xv, k), l = lane_val(Lv, k);
            const bool sw = __builtin_amdgcn_readlane(Sv, k) != 0;
            const double c = sw ? nx : cur;
            const double n = (sw ? cur : nx) - l * c;
            if (lane == k) out = c;
            cur = n;
          }
          if (ii < m - 1) x[ii] = out;
        }
        // backward: U with the reciprocal pivots, 64 rows per block from the bottom
        double x1 = cur * rud[m - 1], x2 = 0.0;
        if (lane == 0) x[m - 1] = x1;
        for (int64_t i1 = m - 2; i1 >= 0; i1 -= 64) {
          const int64_t ii = i1 - lane;
          const double Xv = (ii >= 0) ? x[ii] : 0.0, U1 = (ii >= 0) ? u1[ii] : 0.0;
          const double U2 = (ii >= 0) ? u2[ii] : 0.0, Rv = (ii >= 0) ? rud[ii] : 0.0;
          double out = 0.0;
#pragma unroll
          for (int k = 0; k < 64; ++k) {
            if (i1 - k < 0) break;
            const double x0 =
                (lane_val(Xv, k) - lane_val(U1, k) * x1 - lane_val(U2, k) * x2) * lane_val(Rv, k);
            if (lane == k) out = x0;
            x2 = x1;
            x1 = x0;
          }
          if (ii >= 0) x[ii] = out;
        }
      }
      __syncthreads();
      // scale to avoid overflow, then MGS against earlier members of the cluster
      double mx = 0;
      for (int64_t i = threadIdx.x; i < m; i += blockDim.x) mx = fmax(mx, fabs(x[i]));
      {
        // block max via sums of a one-hot is awkward; reuse scratch with max
        __syncthreads();
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
        if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = mx;
        __syncthreads();
        mx = 0;
        for (int wv = 0; wv < (int)((blockDim.x + 63) >> 6); ++wv) mx = fmax(mx, scratch[wv]);
        __syncthreads();
      }
      const double inv = (mx > 0) ? 1.0 / mx : 1.0;
      for (int64_t i = threadIdx.x; i < m; i += blockDim.x) x[i] *= inv;
      __syncthreads();
      for (int64_t r = c0; r < q; ++r) {
        const double *sr = S + r * lds;
        double s = 0;
        for (int64_t i = threadIdx.x; i < m; i += blockDim.x) s += sr[i] * x[i];
        s = block_sum(s, scratch);
        for (int64_t i = threadIdx.x; i < m; i += blockDim.x) x[i] -= s * sr[i];
        __syncthreads();
      }
      double nn = 0;
      for (int64_t i = threadIdx.x; i < m; i += blockDim.x) nn += x[i] * x[i];
      nn = block_sum(nn, scratch);
      const double invn = (nn > 0) ? 1.0 / sqrt(nn) : 1.0;
      for (int64_t i = threadIdx.x; i < m; i += blockDim.x) x[i] *= invn;
      __syncthreads();
    }
    // sign: largest-magnitude component (first on ties) made positive; the
    // first index of the maximum is found by a block reduction
    {
      double best = -1.0;
      int64_t bi = m;
      for (int64_t i = threadIdx.x; i < m; i += blockDim.x)
        if (fabs(x[i]) > best) {
          best = fabs(x[i]);
          bi = i;
        }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int64_t oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if ((threadIdx.x & 63) == 0) {
        scratch[threadIdx.x >> 6] = best;
        sh_idx[threadIdx.x >> 6] = (int)bi;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double b0 = scratch[0];
        int i0 = sh_idx[0];
        for (int wv = 1; wv < (int)((blockDim.x + 63) >> 6); ++wv)
          if (scratch[wv] > b0 || (scratch[wv] == b0 && sh_idx[wv] < i0)) {
            b0 = scratch[wv];
            i0 = sh_idx[wv];
          }
        sh_coef = (x[i0] < 0) ? -1.0 : 1.0;
      }
    }
    __syncthreads();
    const double sg = sh_coef;
    double *sq = S + q * lds;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) sq[i] = sg * x[i];
    __threadfence_block();
    __syncthreads();
  }
}

// Z = S as complex
__global__ __launch_bounds__(256) void real_to_complex_kernel(int64_t m, const double *__restrict__ S, int64_t lds,
                                       double2 *__restrict__ Z, int64_t ldz) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  const int64_t i = idx % m, j = idx / m;
  Z[i + j * ldz] = double2{S[i + j * lds], 0.0};
}

// wrow[c] = sum_{i>j} conj(u_i) Z[i, c]
__global__ __launch_bounds__(256) void bt_dot_kernel(int64_t m, int64_t j, const double2 *__restrict__ u,
                              const double2 *__restrict__ Z, int64_t ldz,
                              double2 *__restrict__ wrow) {
  __shared__ double scratch[16];
  const int64_t c = blockIdx.x;
  double sr = 0, si = 0;
  for (int64_t i = j + 1 + threadIdx.x; i < m; i += blockDim.x) {
    const double2 uv = u[i], z = Z[i + c * ldz];
    sr += uv.x * z.x + uv.y * z.y;
    si += uv.x * z.y - uv.y * z.x;
  }
  sr = block_sum(sr, scratch);
  si = block_sum(si, scratch);
  if (threadIdx.x == 0) wrow[c] = double2{sr, si};
}

// Z[i, c] -= tau u_i wrow[c]  for i > j
__global__ __launch_bounds__(256) void bt_update_kernel(int64_t m, int64_t j, const double2 *__restrict__ tau,
                                 const double2 *__restrict__ u, const double2 *__restrict__ wrow,
                                 double2 *__restrict__ Z, int64_t ldz) {
  const int64_t L = m - j - 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i >= L) return;
  const double2 t = cmul(tau[j], u[j + 1 + i]);
  double2 *p = Z + (j + 1 + i) + c * ldz;
  *p = csub(*p, cmul(t, wrow[c]));
}

// Householder vector u_j (with u_{j+1} = 1) restored from column j of A.
__global__ __launch_bounds__(256) void load_u_kernel(int64_t m, const double2 *__restrict__ A, int64_t lda, int64_t j,
                              double2 *__restrict__ u) {
  const int64_t i = j + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  u[i] = (i == j + 1) ? double2{1.0, 0.0} : A[i + j * lda];
}

// V (Lr x nb, ld Lr) of the reflectors j0 .. j0+nb-1 on rows j0+1 .. m-1:
// V[i, k] = 0 above row j0+k+1, 1 on it, A[r, j0+k] below (r = j0 + 1 + i).
__global__ __launch_bounds__(256) void build_v_kernel(int64_t m, const double2 *__restrict__ A,
                                                      int64_t lda, int64_t j0, int nb,
                                                      double2 *__restrict__ V) {
  const int64_t Lr = m - j0 - 1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Lr * nb) return;
  const int64_t i = idx % Lr, k = idx / Lr;
  const int64_t r = j0 + 1 + i, top = j0 + k + 1;
  V[idx] = r < top ? double2{0.0, 0.0} : (r == top ? double2{1.0, 0.0} : A[r + (j0 + k) * lda]);
}

// Upper triangular T with H_{j0} H_{j0+1} ... H_{j0+nb-1} = I - V T V^H (forward
// accumulation of the block reflector), from G = V^H V: T[k][k] = tau_k and
// T[i][k] = -tau_k sum_{l=i}^{k-1} T[i][l] G[l][k].  Row i depends only on
// itself and G; 16 lanes share a row (lane q sums the terms l = i + q (mod 16)
// and owns the entries T[i][k] with k = i + q (mod 16), the only ones it
// reads back), the sum completed by shuffles within the 16 lanes.
constexpr int kLarftLanes = 16;
__global__ __launch_bounds__(kBtBlock * kLarftLanes) void larft_kernel(
    int nb, const double2 *__restrict__ G, const double2 *__restrict__ tau,
    double2 *__restrict__ T) {
  __shared__ double2 Gs[kBtBlock * kBtBlock];  // column-major, ld nb
  __shared__ double2 Tr[kBtBlock * kBtBlock];  // row-major, ld kBtBlock
  __shared__ double2 taus[kBtBlock];
  const int t = threadIdx.x;
  for (int idx = t; idx < nb * nb; idx += blockDim.x) Gs[idx] = G[idx];
  if (t < nb) taus[t] = tau[t];
  for (int idx = t; idx < kBtBlock * kBtBlock; idx += blockDim.x) Tr[idx] = double2{0.0, 0.0};
  __syncthreads();
  const int i = t / kLarftLanes, q = t % kLarftLanes;
  double2 *row = Tr + i * kBtBlock;
  if (i < nb && q == 0) row[i] = taus[i];
  for (int k = 1; k < nb; ++k) {  // the same trip count on every lane (shuffles below)
    double2 acc{0.0, 0.0};
    if (i < k)
      for (int l = i + q; l < k; l += kLarftLanes) acc = cadd(acc, cmul(row[l], Gs[l + k * nb]));
    for (int off = kLarftLanes / 2; off > 0; off >>= 1) {
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
    }
    if (i < k && q == (k - i) % kLarftLanes) {
      const double2 v = cmul(taus[k], acc);
      row[k] = double2{-v.x, -v.y};
    }
  }
  __syncthreads();
  for (int idx = t; idx < nb * nb; idx += blockDim.x)
    T[idx] = Tr[(idx % nb) * kBtBlock + idx / nb];
}

}  // namespace

// ---------------------------------------------------------------- drivers ----
size_t zpotrf_work_bytes(int64_t) { return 0; }

void zpotrf_upper(int64_t m, void *Av, int64_t lda, int *info, void *, hipStream_t st) {
  double2 *A = (double2 *)Av;
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, st, info, 0);
  for (int64_t j0 = 0; j0 < m; j0 += NB) {
    const int nb = (int)std::min<int64_t>(NB, m - j0);
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, nb, A, lda, j0, info);
    CHEBFI_HIP(hipGetLastError());
    const int64_t rest = m - j0 - nb;
    if (rest > 0) {
      hipLaunchKernelGGL(potrf_panel_kernel, dim3(nblk(rest, 64)), dim3(64), 0, st, nb, m, A, lda,
                         j0);
      CHEBFI_HIP(hipGetLastError());
      double2 *U12 = A + j0 + (j0 + nb) * lda;
      double2 *A22 = A + (j0 + nb) + (j0 + nb) * lda;
      zgemm(OP_C, OP_N, rest, rest, nb, U12, lda, U12, lda, A22, lda, double2{-1.0, 0.0},
            double2{1.0, 0.0}, st);
    }
  }
  launch_zero_lower(m, A, lda, st);
}

size_t ztrtri_work_bytes(int64_t m) { return sizeof(double2) * (size_t)m * NB; }

void ztrtri_upper(int64_t m, void *Av, int64_t lda, void *work, hipStream_t st) {
  double2 *A = (double2 *)Av;
  double2 *T = (double2 *)work;  // m x NB
  for (int64_t j0 = 0; j0 < m; j0 += NB) {
    const int nb = (int)std::min<int64_t>(NB, m - j0);
    hipLaunchKernelGGL(trtri_diag_kernel, dim3(1), dim3(256), 0, st, nb, A, lda, j0);
    CHEBFI_HIP(hipGetLastError());
    if (j0 > 0) {
      // A[0:j0, j0:j0+nb] = -Uinv[0:j0,0:j0] * A[0:j0, j0:j0+nb] * Uinv_jj
      zgemm(OP_N, OP_N, j0, nb, j0, A, lda, A + j0 * lda, lda, T, j0, double2{1.0, 0.0},
            double2{0.0, 0.0}, st);
      zgemm(OP_N, OP_N, j0, nb, nb, T, j0, A + j0 + j0 * lda, lda, A + j0 * lda, lda,
            double2{-1.0, 0.0}, double2{0.0, 0.0}, st);
    }
  }
}

// bytes of one cluster's arrays in the inverse iteration (seven of m doubles,
// m pivot flags, 256-byte aligned)
static size_t invit_bytes(int64_t m) {
  return (sizeof(double) * 7 * (size_t)m + (size_t)m + 64 + 255) / 256 * 256;
}

size_t zheev_work_bytes(int64_t m) {
  // d, e, e2, w-tmp, stats, the norm partials, tau, u, wrow, the current
  // column, the reduction's panels P1, Q (m x 2 kTriNB each), y, its partial
  // sums, S (real m x m), the lane-interleaved inverse iteration's five
  // arrays and pivots (m x 64 per wave each), and the blocked
  // back-transformation's V (m x nb), G, T (nb x nb), W1, W2 (nb x m)
  const size_t nb = kBtBlock;
  const size_t tri = 4 * kTriNB * (size_t)m + 3 * (size_t)m + 2 * kTriNB * nblk(m, kTriRows);
  const size_t lane_slab = (size_t)m * 64 * (size_t)((m + 63) / 64);
  // (above kLdsInvitM the clusters' arrays take a global slab per possible leader)
  const size_t invit_slabs = m > kLdsInvitM ? (size_t)m * invit_bytes(m) : 0;
  return sizeof(double) * (size_t)(4 * m + 8) + sizeof(double2) * (size_t)(4 * m) +
         sizeof(double2) * tri +
         sizeof(double) * (size_t)m * m + (5 * sizeof(double) + 1) * lane_slab +
         sizeof(double2) * ((3 + kBtSplits) * nb * (size_t)m + 2 * nb * nb) + invit_slabs +
         28 * 256;  // each of the (at most 28) sub-buffers is rounded up to 256 bytes
}

void zheev(int64_t m, void *Av, int64_t lda, double *wout, void *Zv, int64_t ldz, void *work,
           hipStream_t st) {
  CHEBFI_REQUIRE(m >= 1 && m <= kEigMaxM, ABI_ERR_ARG, "eigensolver size out of range");
  double2 *A = (double2 *)Av;
  double2 *Z = (double2 *)Zv;
  char *wp = (char *)work;
  auto take = [&](size_t bytes) {
    void *p = wp;
    wp += (bytes + 255) / 256 * 256;
    return p;
  };
  double *d = (double *)take(sizeof(double) * m);
  double *e = (double *)take(sizeof(double) * m);
  double *e2 = (double *)take(sizeof(double) * m);
  double *stats = (double *)take(sizeof(double) * 8);
  double2 *tau = (double2 *)take(sizeof(double2) * m);
  double2 *u = (double2 *)take(sizeof(double2) * m);
  double2 *wrow = (double2 *)take(sizeof(double2) * m);
  // blocked reduction: P1 = [U W] (m x 2 kTriNB), Q = [W U]^H (2 kTriNB x m),
  // the current column, y = A22 u and the partial sums
  double2 *P1 = (double2 *)take(sizeof(double2) * 2 * kTriNB * (size_t)m);
  double2 *Q = (double2 *)take(sizeof(double2) * 2 * kTriNB * (size_t)m);
  double2 *xv = (double2 *)take(sizeof(double2) * m);
  double2 *yv = (double2 *)take(sizeof(double2) * m);
  double2 *yupart = (double2 *)take(sizeof(double2) * m);
  double *normpart = (double *)take(sizeof(double) * nblk(m, kTriRows));
  double2 *stpart = (double2 *)take(sizeof(double2) * 2 * kTriNB * (size_t)nblk(m, kTriRows));
  double *S = (double *)take(sizeof(double) * (size_t)m * m);
  const size_t lane_slab = (size_t)m * 64 * nblk(m, 64);  // per array, all waves
  double *lwork = (double *)take(sizeof(double) * 5 * lane_slab);
  unsigned char *lswp = (unsigned char *)take(lane_slab);

  launch_hermitize(m, A, lda, st);
  // reduction to tridiagonal form: two launches per column, and per panel of
  // kTriNB columns one GEMM update of the trailing matrix and one copy of the
  // next panel's first column
  hipLaunchKernelGGL(tri_start_kernel, dim3(nblk(m, kTriRows)), dim3(64), 0, st, m, A, lda,
                     int64_t{0}, xv, d, normpart);
  int64_t j0 = 0;
  auto panel_update = [&](int64_t c) {  // A[c:, c:] -= [U W] [W U]^H, then column c
    const int64_t L = m - c;
    zgemm(OP_N, OP_N, L, L, 2 * kTriNB, P1 + c, m, Q + c * 2 * kTriNB, 2 * kTriNB,
          A + c + c * lda, lda, double2{-1, 0}, double2{1, 0}, st);
    hipLaunchKernelGGL(tri_start_kernel, dim3(nblk(L, kTriRows)), dim3(64), 0, st, m, A, lda, c,
                       xv, d, normpart);
  };
  for (int64_t c = 0; c + 1 < m; ++c) {
    if (c == j0 + kTriNB) {
      panel_update(c);
      j0 = c;
    }
    const int k = (int)(c - j0);
    const int64_t L = m - c - 1;
    const int nrb = (int)nblk(L, kTriRows);
    hipLaunchKernelGGL(tri_mv_kernel, dim3((unsigned)(L + nrb)), dim3(256), 0, st, m, A, lda, c, k,
                       xv, normpart, (int)nblk(m - c, kTriRows), P1, Q, yv, yupart, stpart, e,
                       tau);
    const int next = (c + 1 < j0 + kTriNB) ? 1 : 0;
    hipLaunchKernelGGL(tri_fin_kernel, dim3(nrb), dim3(kTriFinT), 0, st, m, A, lda, c, k, next,
                       nrb, P1, Q, yv, yupart, stpart, tau, xv, d, normpart);
  }
  if (m >= 2 && m - 1 == j0 + kTriNB) panel_update(m - 1);  // the last diagonal entry
  CHEBFI_HIP(hipGetLastError());
  // eigenvalues of the tridiagonal
  hipLaunchKernelGGL(tri_prep_kernel, dim3(1), dim3(256), 0, st, m, d, e, e2, stats);
  {
    // d and e2 in LDS up to m = 4096 (64 KB)
    const int lds = m <= 4096 ? 1 : 0;
    const size_t lb = lds ? sizeof(double) * 2 * (size_t)m : 0;
    if (lds)
      CHEBFI_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(bisect_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lb));
    hipLaunchKernelGGL(bisect_kernel, dim3(nblk(m, 4)), dim3(256), lb, st, m, d, e2, stats, wout,
                       lds);
  }
  CHEBFI_HIP(hipGetLastError());
  // eigenvectors of the tridiagonal
  // clusters: arrays in LDS up to kLdsInvitM, else in a global slab per leader
  const bool in_lds = m <= kLdsInvitM;
  const size_t lds_bytes = in_lds ? sizeof(double) * 7 * (size_t)m + (size_t)m + 64 : 0;
  unsigned char *gws = in_lds ? nullptr : (unsigned char *)take((size_t)m * invit_bytes(m));
  if (in_lds)
    CHEBFI_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(invit_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
  hipLaunchKernelGGL(invit_lane_kernel, dim3(nblk(m, 64)), dim3(64), 0, st, m, d, e, wout, stats,
                     S, m, lwork, lswp);
  hipLaunchKernelGGL(invit_kernel, dim3((unsigned)m), dim3(256), lds_bytes, st, m, d, e, wout,
                     stats, S, m, gws, invit_bytes(m));
  CHEBFI_HIP(hipGetLastError());
  hipLaunchKernelGGL(real_to_complex_kernel, dim3(nblk(m * m, 256)), dim3(256), 0, st, m, S, m, Z,
                     ldz);
  // back-transformation Z = H_0 H_1 ... H_{m-2} S, in blocks of kBtBlock reflectors
  // from the last: Z <- (I - V T V^H) Z = Z - V (T (V^H Z)) on rows j0+1 .. m-1
  const int64_t nref = m - 1;
  const int64_t nb0 = std::min<int64_t>(kBtBlock, std::max<int64_t>(nref, 1));
  if (m >= kBtMinM) {
    double2 *V = (double2 *)take(sizeof(double2) * (size_t)m * nb0);
    double2 *G = (double2 *)take(sizeof(double2) * (size_t)nb0 * nb0);
    double2 *T = (double2 *)take(sizeof(double2) * (size_t)nb0 * nb0);
    double2 *W1 = (double2 *)take(sizeof(double2) * (size_t)nb0 * m);
    double2 *W2 = (double2 *)take(sizeof(double2) * (size_t)nb0 * m);
    double2 *Wp = (double2 *)take(sizeof(double2) * (size_t)kBtSplits * nb0 * m);
    for (int64_t jend = nref; jend > 0; jend -= nb0) {
      const int64_t j0 = std::max<int64_t>(0, jend - nb0);
      const int nb = (int)(jend - j0);
      const int64_t Lr = m - j0 - 1;
      double2 *Zr = Z + (j0 + 1);
      hipLaunchKernelGGL(build_v_kernel, dim3(nblk(Lr * nb, 256)), dim3(256), 0, st, m, A, lda, j0,
                         nb, V);
      // G = V^H V: a 64 x 64 product over Lr rows, split over K to fill the chip
      const int spg = (int)std::max<int64_t>(
          1, std::min<int64_t>({Lr / 64, kBtGSplits, (int64_t)kBtSplits * m / nb}));
      zgemm(OP_C, OP_N, nb, nb, Lr, V, Lr, V, Lr, nullptr, 0, double2{1, 0}, double2{0, 0}, st,
            Wp, spg);
      zsum_parts(nb, nb, Wp, spg, G, nb, double2{1, 0}, double2{0, 0}, st);
      hipLaunchKernelGGL(larft_kernel, dim3(1), dim3(kBtBlock * kLarftLanes), 0, st, nb, G,
                         tau + j0, T);
      const int sp = std::min(kBtSplits, zgemm_splits(nb, m, Lr));
      zgemm(OP_C, OP_N, nb, m, Lr, V, Lr, Zr, ldz, nullptr, 0, double2{1, 0}, double2{0, 0}, st, Wp,
            sp);
      zsum_parts(nb, m, Wp, sp, W1, nb, double2{1, 0}, double2{0, 0}, st);
      zgemm(OP_N, OP_N, nb, m, nb, T, nb, W1, nb, W2, nb, double2{1, 0}, double2{0, 0}, st);
      zgemm(OP_N, OP_N, Lr, m, nb, V, Lr, W2, nb, Zr, ldz, double2{-1, 0}, double2{1, 0}, st);
    }
  } else {
    for (int64_t j = m - 2; j >= 0; --j) {
      const int64_t L = m - j - 1;
      hipLaunchKernelGGL(load_u_kernel, dim3(nblk(L, 256)), dim3(256), 0, st, m, A, lda, j, u);
      hipLaunchKernelGGL(bt_dot_kernel, dim3((unsigned)m), dim3(256), 0, st, m, j, u, Z, ldz,
                         wrow);
      hipLaunchKernelGGL(bt_update_kernel, dim3(nblk(L, 256), (unsigned)m), dim3(256), 0, st, m, j,
                         tau, u, wrow, Z, ldz);
    }
  }
  CHEBFI_HIP(hipGetLastError());
}

}  // namespace chebfi
