// Bandwidth-bound helper kernels of the path: the per-atom D application of
// the nonlocal operator, Rayleigh quotients and their extremes, the Lanczos
// vector operations, residual norms and small dense-matrix utilities.
//
// Paper (arXiv 2604.11139): D_ij^R couples the projections of one atom
// (section "Low-level operations"); the filter's bounds come from the minimum
// and maximum Rayleigh quotient (section "Parallel implementation design",
// Algorithm "Parallel Chebyshev filtering of degree k"); the cycle ends with
// W = (H - Lambda S) Psi and its column norms.  All reductions run in a fixed
// order inside one workgroup per result, so repeated runs agree bitwise.
#include "cplx.h"
#include "kernels.h"

namespace chebfi {

namespace {

constexpr int kRedThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the workgroup; every thread receives the total.
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

template <typename T>
__global__ void dapply_kernel(int natom, int64_t nband, const C2<T> *__restrict__ part,
                              int splits, const double2 *__restrict__ D, double alpha,
                              C2<T> *__restrict__ Cp, const double *__restrict__ coef) {
  if (coef) alpha = coef[0];  // (this step's alpha from device memory: captured filters)
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)natom * nband) return;
  const int64_t R = idx % natom, b = idx / natom;
  const int64_t nproj = 4 * (int64_t)natom;
  const int64_t mn = nproj * nband;
  double2 c[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double2 s{0, 0};
    for (int z = 0; z < splits; ++z) {
      const C2<T> v = part[(int64_t)z * mn + (4 * R + j) + b * nproj];
      s.x += (double)v.x;
      s.y += (double)v.y;
    }
    c[j] = s;
  }
  const double2 *d = D + 16 * R;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double2 s{0, 0};
#pragma unroll
    for (int j = 0; j < 4; ++j) s = cadd(s, cmul(d[4 * i + j], c[j]));
    Cp[(4 * R + i) + b * nproj] = C2<T>{(T)(alpha * s.x), (T)(alpha * s.y)};
  }
}

// rq[b] = Re(x^H hx) / Re(x^H sx), sx = x when SX is null (S = I)
template <typename T>
__global__ void rq_kernel(int64_t npw, const C2<T> *__restrict__ X, int64_t ldx,
                          const C2<T> *__restrict__ HX, int64_t ldh,
                          const C2<T> *__restrict__ SX, int64_t lds, double *__restrict__ rq) {
  __shared__ double scratch[16];
  const int64_t b = blockIdx.x;
  const C2<T> *x = X + b * ldx;
  const C2<T> *h = HX + b * ldh;
  const C2<T> *sx = SX ? SX + b * lds : x;
  double num = 0, den = 0;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const C2<T> xv = x[i], hv = h[i], sv = sx[i];
    num += (double)xv.x * hv.x + (double)xv.y * hv.y;
    den += (double)xv.x * sv.x + (double)xv.y * sv.y;
  }
  num = block_sum(num, scratch);
  den = block_sum(den, scratch);
  if (threadIdx.x == 0) rq[b] = num / den;
}

template <typename S, typename D>
__global__ void convert_block_kernel(int64_t rows, int64_t cols, const C2<S> *__restrict__ src,
                                     int64_t lds, C2<D> *__restrict__ dst, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx % rows, j = idx / rows;
  const C2<S> v = src[i + j * lds];
  dst[i + j * ldd] = C2<D>{(D)v.x, (D)v.y};
}

__global__ void minmax_kernel(int64_t n, const double *__restrict__ v, double *__restrict__ out) {
  __shared__ double smax[kRedThreads], smin[kRedThreads];
  double mx = -1.0 / 0.0, mn = 1.0 / 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    mx = fmax(mx, v[i]);
    mn = fmin(mn, v[i]);
  }
  smax[threadIdx.x] = mx;
  smin[threadIdx.x] = mn;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = smax[0];
    out[2] = smin[0];
  }
}

__global__ void dot_re_kernel(int64_t npw, const double2 *__restrict__ x,
                              const double2 *__restrict__ y, double *__restrict__ out) {
  __shared__ double scratch[16];
  double s = 0;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const double2 a = x[i], b = y[i];
    s += a.x * b.x + a.y * b.y;
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) *out = s;
}

__global__ void norm_kernel(int64_t npw, const double2 *__restrict__ x, double *__restrict__ out) {
  __shared__ double scratch[16];
  double s = 0;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const double2 a = x[i];
    s += a.x * a.x + a.y * a.y;
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) *out = sqrt(s);
}

__global__ void axpy_dev_kernel(int64_t npw, const double *__restrict__ coef, double sign,
                                const double2 *__restrict__ x, double2 *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npw) return;
  const double a = sign * (*coef);
  const double2 xv = x[i];
  double2 yv = y[i];
  yv.x += a * xv.x;
  yv.y += a * xv.y;
  y[i] = yv;
}

__global__ void scale_inv_kernel(int64_t npw, const double *__restrict__ s,
                                 const double2 *__restrict__ x, double2 *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npw) return;
  const double inv = 1.0 / (*s);
  y[i] = cscale(x[i], inv);
}

__global__ void multi_dot_kernel(int64_t npw, const double2 *__restrict__ V, int64_t ldv,
                                 const double2 *__restrict__ w, double2 *__restrict__ h) {
  __shared__ double scratch[16];
  const int j = blockIdx.x;
  const double2 *v = V + (int64_t)j * ldv;
  double re = 0, im = 0;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const double2 a = v[i], b = w[i];
    re += a.x * b.x + a.y * b.y;  // conj(a) * b
    im += a.x * b.y - a.y * b.x;
  }
  re = block_sum(re, scratch);
  im = block_sum(im, scratch);
  if (threadIdx.x == 0) h[j] = double2{re, im};
}

__global__ void multi_axpy_kernel(int64_t npw, int nvec, const double2 *__restrict__ V,
                                  int64_t ldv, const double2 *__restrict__ h,
                                  double2 *__restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npw) return;
  double2 s = w[i];
  for (int j = 0; j < nvec; ++j) s = csub(s, cmul(V[(int64_t)j * ldv + i], h[j]));
  w[i] = s;
}

// Number of eigenvalues of the symmetric tridiagonal (d, e) below x (Sturm count).
__device__ int sturm_count(int k, const double *d, const double *e, double x) {
  int cnt = 0;
  double q = 1.0;
  for (int i = 0; i < k; ++i) {
    const double e2 = (i > 0) ? e[i - 1] * e[i - 1] : 0.0;
    q = (d[i] - x) - ((i > 0) ? e2 / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

__global__ void tridiag_bound_kernel(int k, const double *__restrict__ alpha,
                                     const double *__restrict__ beta, int add_last,
                                     double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(beta[i - 1]) : 0.0) + (i < k - 1 ? fabs(beta[i]) : 0.0);
    lo = fmin(lo, alpha[i] - r);
    hi = fmax(hi, alpha[i] + r);
  }
  const double span = fmax(fabs(lo), fabs(hi));
  lo -= 1e-12 * span + 1e-300;
  hi += 1e-12 * span + 1e-300;
  for (int it = 0; it < 400; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(k, alpha, beta, mid) >= k)
      hi = mid;
    else
      lo = mid;
  }
  double theta = 0.5 * (lo + hi);
  if (k == 1) theta = alpha[0];
  out[1] = theta + (add_last ? beta[k - 1] : 0.0);
}

__global__ void residual_kernel(int64_t npw, const double2 *__restrict__ Psi, int64_t ldp,
                                const double2 *__restrict__ HPsi, int64_t ldh,
                                const double *__restrict__ eval, double *__restrict__ res) {
  __shared__ double scratch[16];
  const int64_t b = blockIdx.x;
  const double lam = eval[b];
  const double2 *p = Psi + b * ldp;
  const double2 *h = HPsi + b * ldh;
  double s = 0;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const double2 pv = p[i], hv = h[i];
    const double rx = hv.x - lam * pv.x, ry = hv.y - lam * pv.y;
    s += rx * rx + ry * ry;
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) res[b] = sqrt(s);
}

// residual norms of a complex float block (FP64 sums)
__global__ void residual_f_kernel(int64_t npw, const float2 *__restrict__ Psi, int64_t ldp,
                                  const float2 *__restrict__ HPsi, int64_t ldh,
                                  const double *__restrict__ eval, double *__restrict__ res) {
  __shared__ double scratch[16];
  const int64_t b = blockIdx.x;
  const double lam = eval[b];
  const float2 *p = Psi + b * ldp;
  const float2 *h = HPsi + b * ldh;
  double s = 0;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const float2 pv = p[i], hv = h[i];
    const double rx = (double)hv.x - lam * pv.x, ry = (double)hv.y - lam * pv.y;
    s += rx * rx + ry * ry;
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) res[b] = sqrt(s);
}

// nrm[b] = ||X[:, b]|| and inv[b] = 1 / nrm[b] (0 for a zero column), FP64 sums
template <typename V2>
__global__ void col_norms_kernel(int64_t npw, const V2 *__restrict__ X, int64_t ldx,
                                 double *__restrict__ nrm, double *__restrict__ inv) {
  __shared__ double scratch[16];
  const int64_t b = blockIdx.x;
  const V2 *x = X + b * ldx;
  double s = 0;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const double xr = x[i].x, xi = x[i].y;
    s += xr * xr + xi * xi;
  }
  s = block_sum(s, scratch);
  if (threadIdx.x == 0) {
    const double r = sqrt(s);
    nrm[b] = r;
    inv[b] = r > 0.0 ? 1.0 / r : 0.0;
  }
}

// First step of the filter from a given H X: out = alpha (HX - c X), in the
// block's precision (the arithmetic of the recurrence pass).
template <typename V2>
__global__ void cheb_first_kernel(int64_t npw, int64_t nband, const V2 *__restrict__ X,
                                  int64_t ldx, const V2 *__restrict__ HX, int64_t ldh,
                                  double alpha, double c, V2 *__restrict__ out, int64_t ldo,
                                  const double *__restrict__ coef) {
  typedef decltype(V2{}.x) R;
  if (coef) {  // (alpha, c) from device memory (captured filters)
    alpha = coef[0];
    c = coef[1];
  }
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npw * nband) return;
  const int64_t i = idx % npw, b = idx / npw;
  const V2 x = X[i + b * ldx], h = HX[i + b * ldh];
  const R a = (R)alpha, cc = (R)c;
  out[i + b * ldo] = V2{a * (h.x - cc * x.x), a * (h.y - cc * x.y)};
}

// *out = min_i (Re A[i, i])^2 over the diagonal of an m x m complex double matrix
// (one workgroup)
__global__ __launch_bounds__(kRedThreads) void diag_min_sq_kernel(int64_t m,
                                                                  const double2 *__restrict__ A,
                                                                  int64_t lda,
                                                                  double *__restrict__ out) {
  __shared__ double red[kRedThreads];
  double v = HUGE_VAL;
  for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
    const double d = A[i + i * lda].x;
    v = fmin(v, d * d);
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// out[:, b] = X[:, b] * sc[b] (complex float blocks, the scale rounded once)
__global__ void scale_cols_f_kernel(int64_t rows, int64_t cols, const float2 *__restrict__ X,
                                    int64_t ldx, const double *__restrict__ sc,
                                    float2 *__restrict__ out, int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx % rows, b = idx / rows;
  const double f = sc[b];
  const float2 v = X[i + b * ldx];
  out[i + b * ldo] = float2{(float)(v.x * f), (float)(v.y * f)};
}

// A[k, j] *= sc[k] (m x n complex double, ld lda): the rows of a coefficient matrix
__global__ void scale_rows_kernel(int64_t m, int64_t n, double2 *__restrict__ A, int64_t lda,
                                  const double *__restrict__ sc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * n) return;
  const int64_t k = idx % m, j = idx / m;
  double2 &a = A[k + j * lda];
  a.x *= sc[k];
  a.y *= sc[k];
}

__global__ void hermitize_kernel(int64_t m, double2 *__restrict__ A, int64_t lda) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  const int64_t i = idx % m, j = idx / m;
  if (i > j) return;
  if (i == j) {
    A[i + j * lda].y = 0.0;
    return;
  }
  const double2 a = A[i + j * lda], b = A[j + i * lda];
  const double2 v{0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
  A[i + j * lda] = v;
  A[j + i * lda] = double2{v.x, -v.y};
}

template <typename V2>
__global__ void copy_block_kernel(int64_t rows, int64_t cols, const V2 *__restrict__ src,
                                  int64_t lds, V2 *__restrict__ dst, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t i = idx % rows, j = idx / rows;
  dst[i + j * ldd] = src[i + j * lds];
}

__global__ void zero_lower_kernel(int64_t m, double2 *__restrict__ A, int64_t lda) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  const int64_t i = idx % m, j = idx / m;
  if (i > j) A[i + j * lda] = double2{0, 0};
}

// One workgroup per atom: 16 complex sums over the bands (in FP64).
template <typename T>
__global__ __launch_bounds__(256) void dd_accum_kernel(int natom, int64_t nband,
                                                       const C2<T> *__restrict__ CA,
                                                       const C2<T> *__restrict__ CY, double gamma,
                                                       double2 *__restrict__ dD) {
  __shared__ double scratch[16];
  const int R = blockIdx.x;
  const int64_t np = 4 * (int64_t)natom;
  double re[16], im[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) re[q] = im[q] = 0.0;
  for (int64_t b = threadIdx.x; b < nband; b += blockDim.x) {
    double2 a[4], y[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const C2<T> u = CA[(4 * R + i) + b * np], v = CY[(4 * R + i) + b * np];
      a[i] = double2{(double)u.x, (double)u.y};
      y[i] = double2{(double)v.x, (double)v.y};
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // a_i conj(y_j)
        re[4 * i + j] += a[i].x * y[j].x + a[i].y * y[j].y;
        im[4 * i + j] += a[i].y * y[j].x - a[i].x * y[j].y;
      }
  }
  for (int q = 0; q < 16; ++q) {
    const double sr = block_sum(re[q], scratch);
    const double si = block_sum(im[q], scratch);
    if (threadIdx.x == 0) {
      double2 d = dD[16 * R + q];
      d.x += gamma * sr;
      d.y += gamma * si;
      dD[16 * R + q] = d;
    }
  }
}

template <typename T>
__global__ void scale_neg_kernel(int64_t npw, int64_t nband, const C2<T> *__restrict__ in,
                                 int64_t ldi, double delta, C2<T> *__restrict__ out,
                                 int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npw * nband) return;
  const int64_t i = idx % npw, b = idx / npw;
  const C2<T> v = in[i + b * ldi];
  const T d = (T)delta;
  out[i + b * ldo] = C2<T>{-d * v.x, -d * v.y};
}

// out[i + j m] = sum_z part[z][i + j m] (summed in FP64, in z order).
template <typename T>
__global__ void sum_parts_kernel(int64_t mn, int splits, const C2<T> *__restrict__ part,
                                 C2<T> *__restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= mn) return;
  double sx = 0.0, sy = 0.0;
  for (int z = 0; z < splits; ++z) {
    const C2<T> v = part[(int64_t)z * mn + idx];
    sx += (double)v.x;
    sy += (double)v.y;
  }
  out[idx] = C2<T>{(T)sx, (T)sy};
}

__global__ void fill_zero_kernel(int64_t n, double *__restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void d2f_kernel(int64_t n, const double *__restrict__ s, float *__restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (float)s[i];
}

// Generalised filter step, small-matrix part (n projectors x nband, complex
// double, ld n): with G = sum_z part[z] = P^H Out (Out = alpha (T - c Y_k) -
// beta Y_{k-1} after the local passes, T the kinetic + local part of H Y_k),
// E += P^H T = G / alpha + c C_k + (beta / alpha) C_{k-1} and Cnext = G.
template <typename T>
__global__ void gen_combine_kernel(int64_t mn, int splits, const C2<T> *__restrict__ part,
                                   const double2 *__restrict__ Ck,
                                   const double2 *__restrict__ Ckm1, double alpha, double cshift,
                                   double beta, double2 *__restrict__ E,
                                   double2 *__restrict__ Cnext) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= mn) return;
  double gx = 0.0, gy = 0.0;
  for (int z = 0; z < splits; ++z) {
    const C2<T> v = part[(int64_t)z * mn + idx];
    gx += (double)v.x;
    gy += (double)v.y;
  }
  const double inv = 1.0 / alpha;
  const double2 ck = Ck[idx], e0 = E[idx];
  double ex = gx * inv + cshift * ck.x, ey = gy * inv + cshift * ck.y;
  if (Ckm1) {
    const double2 cp = Ckm1[idx];
    ex += beta * inv * cp.x;
    ey += beta * inv * cp.y;
  }
  E[idx] = double2{e0.x + ex, e0.y + ey};
  Cnext[idx] = double2{gx, gy};
}

// out = sum_z part[z] in complex double (partials complex float or double)
template <typename T>
__global__ void parts_to_c128_kernel(int64_t mn, int splits, const C2<T> *__restrict__ part,
                                     double2 *__restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= mn) return;
  double sx = 0.0, sy = 0.0;
  for (int z = 0; z < splits; ++z) {
    const C2<T> v = part[(int64_t)z * mn + idx];
    sx += (double)v.x;
    sy += (double)v.y;
  }
  out[idx] = double2{sx, sy};
}

// out[:, j] = W[:, j] * mu_j / (1 + mu_j)   (m x m, Woodbury kernel of S^-1)
__global__ void woodbury_scale_kernel(int64_t m, const double2 *__restrict__ W, int64_t ldw,
                                      const double *__restrict__ mu, double2 *__restrict__ out,
                                      int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  const int64_t i = idx % m, j = idx / m;
  const double f = mu[j] / (1.0 + mu[j]);
  out[i + j * ldo] = cscale(W[i + j * ldw], f);
}

__global__ void sqrt_scalar_kernel(const double *__restrict__ in, double *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = sqrt(fmax(*in, 0.0));
}

// LOBPCG block kernels (complex double, one workgroup per column b).
// W = HX - lam_b SX and res[b] = ||W_b||.
__global__ void resid_block_kernel(int64_t npw, const double2 *__restrict__ HX,
                                   const double2 *__restrict__ SX, int64_t ld,
                                   const double *__restrict__ lam, double2 *__restrict__ W,
                                   int64_t ldw, double *__restrict__ res) {
  __shared__ double scratch[16];
  const int64_t b = blockIdx.x;
  const double l = lam[b];
  const double2 *h = HX + b * ld;
  const double2 *sx = SX + b * ld;
  double2 *w = W + b * ldw;
  double acc = 0;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const double2 hv = h[i], sv = sx[i];
    const double2 r{hv.x - l * sv.x, hv.y - l * sv.y};
    w[i] = r;
    acc += r.x * r.x + r.y * r.y;
  }
  acc = block_sum(acc, scratch);
  if (threadIdx.x == 0) res[b] = sqrt(acc);
}

// Teter-Payne-Allan diagonal: W_b *= p(x) / (p(x) + 16 x^4), x = kin / E_kin(X_b),
// p(x) = 27 + 18 x + 12 x^2 + 8 x^3.
__global__ void tpa_kernel(int64_t npw, const double *__restrict__ kin,
                           const double2 *__restrict__ X, int64_t ldx, double2 *__restrict__ W,
                           int64_t ldw) {
  __shared__ double scratch[16];
  const int64_t b = blockIdx.x;
  const double2 *x = X + b * ldx;
  double2 *w = W + b * ldw;
  double num = 0, den = 0;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const double2 v = x[i];
    const double a2 = v.x * v.x + v.y * v.y;
    num += kin[i] * a2;
    den += a2;
  }
  num = block_sum(num, scratch);
  den = block_sum(den, scratch);
  const double inv_ek = den / num;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const double t = kin[i] * inv_ek;
    const double p = 27.0 + t * (18.0 + t * (12.0 + t * 8.0));
    const double t2 = t * t;
    w[i] = cscale(w[i], p / (p + 16.0 * t2 * t2));
  }
}

// Scales column b of W, HW (and SW when given) by 1 / sqrt(Re(w^H sw)), sw = w when
// SW is null.
__global__ void snorm_scale_kernel(int64_t npw, double2 *__restrict__ W, double2 *__restrict__ HW,
                                   double2 *__restrict__ SW, int64_t ld) {
  __shared__ double scratch[16];
  const int64_t b = blockIdx.x;
  double2 *w = W + b * ld;
  double2 *hw = HW + b * ld;
  double2 *sw = SW ? SW + b * ld : nullptr;
  double acc = 0;
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    const double2 a = w[i], c = sw ? sw[i] : a;
    acc += a.x * c.x + a.y * c.y;
  }
  acc = block_sum(acc, scratch);
  const double f = 1.0 / sqrt(acc);
  for (int64_t i = threadIdx.x; i < npw; i += blockDim.x) {
    w[i] = cscale(w[i], f);
    hw[i] = cscale(hw[i], f);
    if (sw) sw[i] = cscale(sw[i], f);
  }
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_dd_accum(int natom, int64_t nband, const void *CA, const void *CY, double gamma,
                     void *dD, hipStream_t st, bool fp32) {
  if (natom <= 0) return;
  if (fp32)
    hipLaunchKernelGGL(dd_accum_kernel<float>, dim3((unsigned)natom), dim3(256), 0, st, natom,
                       nband, (const float2 *)CA, (const float2 *)CY, gamma, (double2 *)dD);
  else
    hipLaunchKernelGGL(dd_accum_kernel<double>, dim3((unsigned)natom), dim3(256), 0, st, natom,
                       nband, (const double2 *)CA, (const double2 *)CY, gamma, (double2 *)dD);
  CHEBFI_HIP(hipGetLastError());
}

void launch_scale_neg(int64_t npw, int64_t nband, const void *in, int64_t ldi, double delta,
                      void *out, int64_t ldo, hipStream_t st, bool fp32) {
  if (fp32)
    hipLaunchKernelGGL(scale_neg_kernel<float>, dim3(nblk(npw * nband, 256)), dim3(256), 0, st,
                       npw, nband, (const float2 *)in, ldi, delta, (float2 *)out, ldo);
  else
    hipLaunchKernelGGL(scale_neg_kernel<double>, dim3(nblk(npw * nband, 256)), dim3(256), 0, st,
                       npw, nband, (const double2 *)in, ldi, delta, (double2 *)out, ldo);
  CHEBFI_HIP(hipGetLastError());
}

void launch_sum_parts(int64_t m, int64_t n, const void *part, int splits, void *out,
                      hipStream_t st, bool fp32) {
  const int64_t mn = m * n;
  if (mn <= 0) return;
  if (fp32)
    hipLaunchKernelGGL(sum_parts_kernel<float>, dim3(nblk(mn, 256)), dim3(256), 0, st, mn, splits,
                       (const float2 *)part, (float2 *)out);
  else
    hipLaunchKernelGGL(sum_parts_kernel<double>, dim3(nblk(mn, 256)), dim3(256), 0, st, mn,
                       splits, (const double2 *)part, (double2 *)out);
  CHEBFI_HIP(hipGetLastError());
}

void launch_fill_zero(int64_t n, double *p, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, n, p);
  CHEBFI_HIP(hipGetLastError());
}

void launch_d2f(int64_t n, const double *src, float *dst, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(d2f_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, n, src, dst);
  CHEBFI_HIP(hipGetLastError());
}

void launch_dapply(int natom, int64_t nband, const void *part, int splits, const void *D,
                   double alpha, void *Cprime, hipStream_t st, bool fp32, const double *coef) {
  const int64_t total = (int64_t)natom * nband;
  if (total <= 0) return;
  if (fp32)
    hipLaunchKernelGGL(dapply_kernel<float>, dim3(nblk(total, 256)), dim3(256), 0, st, natom,
                       nband, (const float2 *)part, splits, (const double2 *)D, alpha,
                       (float2 *)Cprime, coef);
  else
    hipLaunchKernelGGL(dapply_kernel<double>, dim3(nblk(total, 256)), dim3(256), 0, st, natom,
                       nband, (const double2 *)part, splits, (const double2 *)D, alpha,
                       (double2 *)Cprime, coef);
  CHEBFI_HIP(hipGetLastError());
}

void launch_rayleigh_quotients(int64_t npw, int64_t nband, const void *X, int64_t ldx,
                               const void *HX, int64_t ldh, double *rq, hipStream_t st,
                               bool fp32, const void *SX, int64_t lds) {
  if (fp32)
    hipLaunchKernelGGL(rq_kernel<float>, dim3((unsigned)nband), dim3(kRedThreads), 0, st, npw,
                       (const float2 *)X, ldx, (const float2 *)HX, ldh, (const float2 *)SX, lds,
                       rq);
  else
    hipLaunchKernelGGL(rq_kernel<double>, dim3((unsigned)nband), dim3(kRedThreads), 0, st, npw,
                       (const double2 *)X, ldx, (const double2 *)HX, ldh, (const double2 *)SX,
                       lds, rq);
  CHEBFI_HIP(hipGetLastError());
}

void launch_gen_combine(int64_t m, int64_t n, const void *part, int splits, bool fp32,
                        const void *Ck, const void *Ckm1, double alpha, double cshift,
                        double beta, void *E, void *Cnext, hipStream_t st) {
  const int64_t mn = m * n;
  if (mn <= 0) return;
  if (fp32)
    hipLaunchKernelGGL(gen_combine_kernel<float>, dim3(nblk(mn, 256)), dim3(256), 0, st, mn,
                       splits, (const float2 *)part, (const double2 *)Ck, (const double2 *)Ckm1,
                       alpha, cshift, beta, (double2 *)E, (double2 *)Cnext);
  else
    hipLaunchKernelGGL(gen_combine_kernel<double>, dim3(nblk(mn, 256)), dim3(256), 0, st, mn,
                       splits, (const double2 *)part, (const double2 *)Ck, (const double2 *)Ckm1,
                       alpha, cshift, beta, (double2 *)E, (double2 *)Cnext);
  CHEBFI_HIP(hipGetLastError());
}

void launch_parts_to_c128(int64_t m, int64_t n, const void *part, int splits, bool fp32,
                          void *out, hipStream_t st) {
  const int64_t mn = m * n;
  if (mn <= 0) return;
  if (fp32)
    hipLaunchKernelGGL(parts_to_c128_kernel<float>, dim3(nblk(mn, 256)), dim3(256), 0, st, mn,
                       splits, (const float2 *)part, (double2 *)out);
  else
    hipLaunchKernelGGL(parts_to_c128_kernel<double>, dim3(nblk(mn, 256)), dim3(256), 0, st, mn,
                       splits, (const double2 *)part, (double2 *)out);
  CHEBFI_HIP(hipGetLastError());
}

void launch_woodbury_scale(int64_t m, const void *W, int64_t ldw, const double *mu, void *out,
                           int64_t ldo, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(woodbury_scale_kernel, dim3(nblk(m * m, 256)), dim3(256), 0, st, m,
                     (const double2 *)W, ldw, mu, (double2 *)out, ldo);
  CHEBFI_HIP(hipGetLastError());
}

void launch_sqrt_scalar(const double *in, double *out, hipStream_t st) {
  hipLaunchKernelGGL(sqrt_scalar_kernel, dim3(1), dim3(64), 0, st, in, out);
  CHEBFI_HIP(hipGetLastError());
}

void launch_c64_to_c128(int64_t rows, int64_t cols, const void *src, int64_t lds, void *dst,
                        int64_t ldd, hipStream_t st) {
  if (rows * cols <= 0) return;
  hipLaunchKernelGGL((convert_block_kernel<float, double>), dim3(nblk(rows * cols, 256)),
                     dim3(256), 0, st, rows, cols, (const float2 *)src, lds, (double2 *)dst, ldd);
  CHEBFI_HIP(hipGetLastError());
}

void launch_c128_to_c64(int64_t rows, int64_t cols, const void *src, int64_t lds, void *dst,
                        int64_t ldd, hipStream_t st) {
  if (rows * cols <= 0) return;
  hipLaunchKernelGGL((convert_block_kernel<double, float>), dim3(nblk(rows * cols, 256)),
                     dim3(256), 0, st, rows, cols, (const double2 *)src, lds, (float2 *)dst, ldd);
  CHEBFI_HIP(hipGetLastError());
}

void launch_minmax(int64_t n, const double *rq, double *out, hipStream_t st) {
  hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(kRedThreads), 0, st, n, rq, out);
  CHEBFI_HIP(hipGetLastError());
}

void launch_dot_re(int64_t npw, const void *x, const void *y, double *out, hipStream_t st) {
  hipLaunchKernelGGL(dot_re_kernel, dim3(1), dim3(1024), 0, st, npw, (const double2 *)x,
                     (const double2 *)y, out);
  CHEBFI_HIP(hipGetLastError());
}

void launch_axpy_dev(int64_t npw, const double *coef, double sign, const void *x, void *y,
                     hipStream_t st) {
  hipLaunchKernelGGL(axpy_dev_kernel, dim3(nblk(npw, 256)), dim3(256), 0, st, npw, coef, sign,
                     (const double2 *)x, (double2 *)y);
  CHEBFI_HIP(hipGetLastError());
}

void launch_multi_dot(int64_t npw, int nvec, const void *V, int64_t ldv, const void *w, void *h,
                      hipStream_t st) {
  hipLaunchKernelGGL(multi_dot_kernel, dim3((unsigned)nvec), dim3(1024), 0, st, npw,
                     (const double2 *)V, ldv, (const double2 *)w, (double2 *)h);
  CHEBFI_HIP(hipGetLastError());
}

void launch_multi_axpy(int64_t npw, int nvec, const void *V, int64_t ldv, const void *h, void *w,
                       hipStream_t st) {
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(nblk(npw, 256)), dim3(256), 0, st, npw, nvec,
                     (const double2 *)V, ldv, (const double2 *)h, (double2 *)w);
  CHEBFI_HIP(hipGetLastError());
}

void launch_norm(int64_t npw, const void *x, double *out, hipStream_t st) {
  hipLaunchKernelGGL(norm_kernel, dim3(1), dim3(1024), 0, st, npw, (const double2 *)x, out);
  CHEBFI_HIP(hipGetLastError());
}

void launch_scale_inv(int64_t npw, const double *s, const void *x, void *y, hipStream_t st) {
  hipLaunchKernelGGL(scale_inv_kernel, dim3(nblk(npw, 256)), dim3(256), 0, st, npw, s,
                     (const double2 *)x, (double2 *)y);
  CHEBFI_HIP(hipGetLastError());
}

void launch_tridiag_bound(int k, const double *alpha, const double *beta, int add_last,
                          double *out, hipStream_t st) {
  hipLaunchKernelGGL(tridiag_bound_kernel, dim3(1), dim3(64), 0, st, k, alpha, beta, add_last,
                     out);
  CHEBFI_HIP(hipGetLastError());
}

void launch_residual_norms(int64_t npw, int64_t nband, const void *Psi, int64_t ldp,
                           const void *HPsi, int64_t ldh, const double *eval, double *res,
                           hipStream_t st) {
  hipLaunchKernelGGL(residual_kernel, dim3((unsigned)nband), dim3(kRedThreads), 0, st, npw,
                     (const double2 *)Psi, ldp, (const double2 *)HPsi, ldh, eval, res);
  CHEBFI_HIP(hipGetLastError());
}

void launch_residual_norms_f(int64_t npw, int64_t nband, const void *Psi, int64_t ldp,
                             const void *HPsi, int64_t ldh, const double *eval, double *res,
                             hipStream_t st) {
  hipLaunchKernelGGL(residual_f_kernel, dim3((unsigned)nband), dim3(kRedThreads), 0, st, npw,
                     (const float2 *)Psi, ldp, (const float2 *)HPsi, ldh, eval, res);
  CHEBFI_HIP(hipGetLastError());
}

void launch_col_norms(int64_t npw, int64_t nband, const void *X, int64_t ldx, double *nrm,
                      double *inv, hipStream_t st, bool fp32) {
  if (fp32)
    hipLaunchKernelGGL(col_norms_kernel<float2>, dim3((unsigned)nband), dim3(kRedThreads), 0, st,
                       npw, (const float2 *)X, ldx, nrm, inv);
  else
    hipLaunchKernelGGL(col_norms_kernel<double2>, dim3((unsigned)nband), dim3(kRedThreads), 0,
                       st, npw, (const double2 *)X, ldx, nrm, inv);
  CHEBFI_HIP(hipGetLastError());
}

void launch_cheb_first(int64_t npw, int64_t nband, const void *X, int64_t ldx, const void *HX,
                       int64_t ldh, double alpha, double c, void *out, int64_t ldo, hipStream_t st,
                       bool fp32, const double *coef) {
  const dim3 g(nblk(npw * nband, 256));
  if (fp32)
    hipLaunchKernelGGL(cheb_first_kernel<float2>, g, dim3(256), 0, st, npw, nband,
                       (const float2 *)X, ldx, (const float2 *)HX, ldh, alpha, c, (float2 *)out,
                       ldo, coef);
  else
    hipLaunchKernelGGL(cheb_first_kernel<double2>, g, dim3(256), 0, st, npw, nband,
                       (const double2 *)X, ldx, (const double2 *)HX, ldh, alpha, c,
                       (double2 *)out, ldo, coef);
  CHEBFI_HIP(hipGetLastError());
}

void launch_diag_min_sq(int64_t m, const void *A, int64_t lda, double *out, hipStream_t st) {
  hipLaunchKernelGGL(diag_min_sq_kernel, dim3(1), dim3(kRedThreads), 0, st, m, (const double2 *)A,
                     lda, out);
  CHEBFI_HIP(hipGetLastError());
}

void launch_scale_cols_f(int64_t rows, int64_t cols, const void *X, int64_t ldx, const double *sc,
                         void *out, int64_t ldo, hipStream_t st) {
  if (rows * cols <= 0) return;
  hipLaunchKernelGGL(scale_cols_f_kernel, dim3(nblk(rows * cols, 256)), dim3(256), 0, st, rows,
                     cols, (const float2 *)X, ldx, sc, (float2 *)out, ldo);
  CHEBFI_HIP(hipGetLastError());
}

void launch_scale_rows(int64_t m, int64_t n, void *A, int64_t lda, const double *sc,
                       hipStream_t st) {
  if (m * n <= 0) return;
  hipLaunchKernelGGL(scale_rows_kernel, dim3(nblk(m * n, 256)), dim3(256), 0, st, m, n,
                     (double2 *)A, lda, sc);
  CHEBFI_HIP(hipGetLastError());
}

void launch_hermitize(int64_t m, void *A, int64_t lda, hipStream_t st) {
  hipLaunchKernelGGL(hermitize_kernel, dim3(nblk(m * m, 256)), dim3(256), 0, st, m,
                     (double2 *)A, lda);
  CHEBFI_HIP(hipGetLastError());
}

void launch_copy_block(int64_t rows, int64_t cols, const void *src, int64_t lds, void *dst,
                       int64_t ldd, hipStream_t st, bool fp32) {
  if (rows * cols <= 0) return;
  if (fp32)
    hipLaunchKernelGGL(copy_block_kernel<float2>, dim3(nblk(rows * cols, 256)), dim3(256), 0, st,
                       rows, cols, (const float2 *)src, lds, (float2 *)dst, ldd);
  else
    hipLaunchKernelGGL(copy_block_kernel<double2>, dim3(nblk(rows * cols, 256)), dim3(256), 0, st,
                       rows, cols, (const double2 *)src, lds, (double2 *)dst, ldd);
  CHEBFI_HIP(hipGetLastError());
}

void launch_zero_lower(int64_t m, void *A, int64_t lda, hipStream_t st) {
  hipLaunchKernelGGL(zero_lower_kernel, dim3(nblk(m * m, 256)), dim3(256), 0, st, m,
                     (double2 *)A, lda);
  CHEBFI_HIP(hipGetLastError());
}

void launch_resid_block(int64_t npw, int64_t m, const void *HX, const void *SX, int64_t ld,
                        const double *lam, void *W, int64_t ldw, double *res, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(resid_block_kernel, dim3((unsigned)m), dim3(kRedThreads), 0, st, npw,
                     (const double2 *)HX, (const double2 *)SX, ld, lam, (double2 *)W, ldw, res);
  CHEBFI_HIP(hipGetLastError());
}

void launch_tpa(int64_t npw, int64_t m, const double *kin, const void *X, int64_t ldx, void *W,
                int64_t ldw, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(tpa_kernel, dim3((unsigned)m), dim3(kRedThreads), 0, st, npw, kin,
                     (const double2 *)X, ldx, (double2 *)W, ldw);
  CHEBFI_HIP(hipGetLastError());
}

void launch_snorm_scale(int64_t npw, int64_t m, void *W, void *HW, void *SW, int64_t ld,
                        hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(snorm_scale_kernel, dim3((unsigned)m), dim3(kRedThreads), 0, st, npw,
                     (double2 *)W, (double2 *)HW, (double2 *)SW, ld);
  CHEBFI_HIP(hipGetLastError());
}

}  // namespace chebfi
