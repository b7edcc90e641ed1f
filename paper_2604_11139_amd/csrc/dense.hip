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
//   both sides as a rank-2 update, applied lazily: two launches per column),
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
// Step j of the reduction uses the reflector H_j = I - tau_j u_j u_j^H of
// column j (u_j[j+1] = 1, zero above), the product p_j = tau_j A22 u_j with the
// trailing matrix A22 = A[j+1:, j+1:], a2_j = -tau_j (p_j^H u_j) / 2 and
// w_j = p_j + a2_j u_j; the two-sided application is the rank-2 update
// A22 -= u_j w_j^H + w_j u_j^H.  Each step is two launches: the rank-2 update
// of step j-1 is applied lazily, to column j in tri_col_kernel and to the
// columns right of it in tri_trail_kernel, which computes p_j from the updated
// values in the same pass.  u and p alternate between two buffers.

constexpr int kTriColThreads = 512;

__device__ __forceinline__ double2 conj2(double2 a) { return double2{a.x, -a.y}; }

// Column j, one workgroup.  For j >= 1: a2_{j-1} over rows j .. m-1, then
// column j (rows j .. m-1) receives step j-1's rank-2 update.  For j <= m-2:
// the Householder vector of column j below its subdiagonal (LAPACK-style
// larfg: H^H (alpha, x) = (beta, 0) with beta real, u = (1, x / (alpha - beta)));
// the scaled x is stored in A (the back-transformation reads it there) and in
// ucur.  d[j] takes the updated diagonal.
__global__ __launch_bounds__(kTriColThreads) void tri_col_kernel(
    int64_t m, double2 *__restrict__ A, int64_t lda, int64_t j, const double2 *__restrict__ uprev,
    const double2 *__restrict__ pprev, double2 *__restrict__ a2s, double *__restrict__ d,
    double *__restrict__ e, double2 *__restrict__ tau, double2 *__restrict__ ucur) {
  constexpr int NT = kTriColThreads, Q = (kEigMaxM + NT - 1) / NT;
  static_assert(NT >= 64 && NT % 64 == 0, "whole waves");
  __shared__ double scratch[32];
  __shared__ double2 sh_alpha;
  const int tid = threadIdx.x;
  double2 *col = A + j * lda;
  double2 c[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t r = j + tid + (int64_t)NT * q;
    c[q] = r < m ? col[r] : double2{0.0, 0.0};
  }
  if (j >= 1) {
    double sr = 0, si = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t r = j + tid + (int64_t)NT * q;
      if (r < m) {
        const double2 pv = pprev[r], uv = uprev[r];
        sr += pv.x * uv.x + pv.y * uv.y;  // conj(p) u
        si += pv.x * uv.y - pv.y * uv.x;
      }
    }
    const double2 dot = block_sum2(double2{sr, si}, scratch);
    const double2 a2 = cscale(cmul(tau[j - 1], dot), -0.5);
    const double2 uj = uprev[j];
    const double2 cwj = conj2(cadd(pprev[j], cmul(a2, uj))), cuj = conj2(uj);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t r = j + tid + (int64_t)NT * q;
      if (r < m) {
        const double2 ur = uprev[r], wr = cadd(pprev[r], cmul(a2, ur));
        c[q] = csub(c[q], cadd(cmul(ur, cwj), cmul(wr, cuj)));
      }
    }
    if (tid == 0) a2s[j - 1] = a2;
  }
  if (j + 1 >= m) {
    if (tid == 0) d[j] = c[0].x;
    return;
  }
  if (tid == 1) sh_alpha = c[0];  // row j + 1
  double s = 0;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t r = j + tid + (int64_t)NT * q;
    if (r >= j + 2 && r < m) s += c[q].x * c[q].x + c[q].y * c[q].y;
  }
  const double xnorm2 = block_sum(s, scratch);  // its barriers also publish sh_alpha
  const double2 alpha = sh_alpha;
  double beta, tr, ti;
  double2 scal{0, 0};
  if (xnorm2 == 0.0 && alpha.y == 0.0) {
    beta = alpha.x;
    tr = 0.0;
    ti = 0.0;
  } else {
    const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xnorm2);
    beta = (alpha.x >= 0.0) ? -nrm : nrm;
    tr = (beta - alpha.x) / beta;
    ti = -alpha.y / beta;
    const double2 den{alpha.x - beta, alpha.y};
    const double dd = den.x * den.x + den.y * den.y;
    scal = double2{den.x / dd, -den.y / dd};
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t r = j + tid + (int64_t)NT * q;
    if (r >= j + 2 && r < m) {
      const double2 v = cmul(c[q], scal);
      col[r] = v;
      ucur[r] = v;
    }
  }
  if (tid == 0) {
    ucur[j + 1] = double2{1.0, 0.0};
    d[j] = c[0].x;
    e[j] = beta;
    tau[j] = double2{tr, ti};
  }
}

// Columns j+1 .. m-1, one workgroup per column: for j >= 1, rows j+1 .. m-1
// of the column receive step j-1's rank-2 update and are stored; p_j[i] =
// tau_j times the conjugated (updated) column i dotted with u_j, which is row i
// of A22 u_j because A22 is Hermitian.  Row j of these columns is not
// updated: no later step reads it.
__global__ __launch_bounds__(256) void tri_trail_kernel(
    int64_t m, double2 *__restrict__ A, int64_t lda, int64_t j, const double2 *__restrict__ uprev,
    const double2 *__restrict__ pprev, const double2 *__restrict__ a2s,
    const double2 *__restrict__ ucur, const double2 *__restrict__ tau, double2 *__restrict__ pcur) {
  __shared__ double scratch[32];
  const int64_t ci = j + 1 + (int64_t)blockIdx.x;
  double2 *col = A + ci * lda;
  const bool upd = j >= 1;
  double2 a2{0, 0}, cwi{0, 0}, cui{0, 0};
  if (upd) {
    a2 = a2s[j - 1];
    const double2 ui = uprev[ci];
    cwi = conj2(cadd(pprev[ci], cmul(a2, ui)));
    cui = conj2(ui);
  }
  double sr = 0, si = 0;
  for (int64_t r = j + 1 + threadIdx.x; r < m; r += blockDim.x) {
    double2 a = col[r];
    if (upd) {
      const double2 ur = uprev[r], wr = cadd(pprev[r], cmul(a2, ur));
      a = csub(a, cadd(cmul(ur, cwi), cmul(wr, cui)));
      col[r] = a;
    }
    const double2 v = ucur[r];
    sr += a.x * v.x + a.y * v.y;  // conj(a) v
    si += a.x * v.y - a.y * v.x;
  }
  const double2 dot = block_sum2(double2{sr, si}, scratch);
  if (threadIdx.x == 0) pcur[ci] = cmul(tau[j], dot);
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
__global__ __launch_bounds__(256) void bisect_kernel(int64_t m, const double *__restrict__ d,
                                                     const double *__restrict__ e2,
                                                     const double *__restrict__ stats,
                                                     double *__restrict__ w) {
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
    const bool above = inside ? sturm_less(m, d, e2, x, pivmin) >= i + 1 : x >= hi;
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
// T[i][k] = -tau_k sum_{l=i}^{k-1} T[i][l] G[l][k].  Thread i owns row i.
__global__ __launch_bounds__(64) void larft_kernel(int nb, const double2 *__restrict__ G,
                                                   const double2 *__restrict__ tau,
                                                   double2 *__restrict__ T) {
  // row i of T depends only on row i and G: thread i runs its row's
  // recurrence with G and its row held in LDS (column-major, conflict-free)
  __shared__ double2 Gs[kBtBlock * kBtBlock];
  __shared__ double2 Ts[kBtBlock * kBtBlock];
  const int i = threadIdx.x;
  for (int idx = i; idx < nb * nb; idx += blockDim.x) {
    Gs[idx] = G[idx];
    Ts[idx] = double2{0.0, 0.0};
  }
  __syncthreads();
  if (i < nb) {
    Ts[i + i * nb] = tau[i];
    for (int k = i + 1; k < nb; ++k) {
      double2 acc{0.0, 0.0};
      for (int l = i; l < k; ++l) acc = cadd(acc, cmul(Ts[i + l * nb], Gs[l + k * nb]));
      const double2 t = cmul(tau[k], acc);
      Ts[i + k * nb] = double2{-t.x, -t.y};
    }
  }
  __syncthreads();
  for (int idx = i; idx < nb * nb; idx += blockDim.x) T[idx] = Ts[idx];
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
  // d, e, e2, w-tmp, stats, tau, u, wrow, two u and two p buffers, a2, S (real
  // m x m), the lane-interleaved inverse iteration's five arrays and pivots
  // (m x 64 per wave each), and the blocked back-transformation's V (m x nb),
  // G, T (nb x nb), W1, W2 (nb x m)
  const size_t nb = kBtBlock;
  const size_t lane_slab = (size_t)m * 64 * (size_t)((m + 63) / 64);
  // (above kLdsInvitM the clusters' arrays take a global slab per possible leader)
  const size_t invit_slabs = m > kLdsInvitM ? (size_t)m * invit_bytes(m) : 0;
  return sizeof(double) * (size_t)(4 * m + 8) + sizeof(double2) * (size_t)(8 * m) +
         sizeof(double) * (size_t)m * m + (5 * sizeof(double) + 1) * lane_slab +
         sizeof(double2) * ((3 + kBtSplits) * nb * (size_t)m + 2 * nb * nb) + invit_slabs +
         24 * 256;  // each of the (at most 24) sub-buffers is rounded up to 256 bytes
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
  double2 *ub = (double2 *)take(sizeof(double2) * 2 * m);
  double2 *pb = (double2 *)take(sizeof(double2) * 2 * m);
  double2 *a2s = (double2 *)take(sizeof(double2) * m);
  double *S = (double *)take(sizeof(double) * (size_t)m * m);
  const size_t lane_slab = (size_t)m * 64 * nblk(m, 64);  // per array, all waves
  double *lwork = (double *)take(sizeof(double) * 5 * lane_slab);
  unsigned char *lswp = (unsigned char *)take(lane_slab);

  launch_hermitize(m, A, lda, st);
  // reduction to tridiagonal form: two launches per column, then the last diagonal
  for (int64_t j = 0; j < m; ++j) {
    const int cur = (int)(j & 1), prev = cur ^ 1;
    hipLaunchKernelGGL(tri_col_kernel, dim3(1), dim3(kTriColThreads), 0, st, m, A, lda, j,
                       ub + prev * m, pb + prev * m, a2s, d, e, tau, ub + cur * m);
    const int64_t L = m - j - 1;
    if (L > 0)
      hipLaunchKernelGGL(tri_trail_kernel, dim3((unsigned)L), dim3(256), 0, st, m, A, lda, j,
                         ub + prev * m, pb + prev * m, a2s, ub + cur * m, tau, pb + cur * m);
  }
  CHEBFI_HIP(hipGetLastError());
  // eigenvalues of the tridiagonal
  hipLaunchKernelGGL(tri_prep_kernel, dim3(1), dim3(256), 0, st, m, d, e, e2, stats);
  hipLaunchKernelGGL(bisect_kernel, dim3(nblk(m, 4)), dim3(256), 0, st, m, d, e2, stats, wout);
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
      zgemm(OP_C, OP_N, nb, nb, Lr, V, Lr, V, Lr, G, nb, double2{1, 0}, double2{0, 0}, st);
      hipLaunchKernelGGL(larft_kernel, dim3(1), dim3(64), 0, st, nb, G, tau + j0, T);
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
