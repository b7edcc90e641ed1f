// Outer SCF step on the FFT box: the Hartree + LDA-exchange potential of a grid
// density and the mixing of the potential (linear, or with Kerker's
// preconditioner K(G) = alpha |G|^2 / (|G|^2 + q0^2), Kerker 1981).
//
// Paper (arXiv 2604.11139): each SCF iteration solves the Kohn-Sham problem,
// computes the occupations on the host and accumulates the density from the
// occupations and wave functions with FFTs on the GPU (Algorithm "Self-consistent
// field in DFT").  The potential of the next iteration is the host code's part
// there; here: V = V_ion + V_H + v_x, V_H(G) = 4 pi n(G)/|G|^2 (V_H(0) = 0) by a
// complex FFT of the whole box, v_x = -(3 n / pi)^(1/3) (LDA exchange).
#include "fft_dev.h"
#include "kernels.h"

namespace chebfi {

namespace {

constexpr int kScfThreads = 256;

// box[r] = (rho[r] * scale, 0)
__global__ void rho_to_box_kernel(int64_t nbox, const double *__restrict__ rho, double scale,
                                  double2 *__restrict__ box) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nbox) box[i] = double2{rho[i] * scale, 0.0};
}

// 2D FFT of every z-plane (x then y), in place; sgn -1 forward, +1 inverse.
__global__ __launch_bounds__(512) void box_xy_kernel(double2 *__restrict__ box, BoxPlan plan,
                                                     const double2 *__restrict__ twg, int sgn) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2 *buf = reinterpret_cast<double2 *>(smem_raw);
  const int n1 = plan.d[0].n, n2 = plan.d[1].n;
  const int L1 = n1 + 1;  // rows padded to n1 + 1
  double2 *tw1 = buf + n2 * L1;
  double2 *tw2 = tw1 + n1;
  load_twiddles<double>(tw1, twg, n1);
  load_twiddles<double>(tw2, twg + kMaxN, n2);
  double2 *plane = box + (int64_t)blockIdx.x * n1 * n2;
  for (int i = threadIdx.x; i < n1 * n2; i += blockDim.x) buf[(i / n1) * L1 + i % n1] = plane[i];
  __syncthreads();
  lds_fft<double>(buf, plan.d[0], 1, n2, L1, tw1, sgn);
  lds_fft<double>(buf, plan.d[1], L1, n1, 1, tw2, sgn);
  for (int i = threadIdx.x; i < n1 * n2; i += blockDim.x) plane[i] = buf[(i / n1) * L1 + i % n1];
}

// 1D FFT along z of every x-z slab (fixed y), in place.
__global__ __launch_bounds__(512) void box_z_kernel(double2 *__restrict__ box, BoxPlan plan,
                                                    const double2 *__restrict__ twg, int sgn) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2 *buf = reinterpret_cast<double2 *>(smem_raw);
  const int n1 = plan.d[0].n, n2 = plan.d[1].n, n3 = plan.d[2].n;
  const int L1 = n1 + 1;
  double2 *tw3 = buf + n3 * L1;
  load_twiddles<double>(tw3, twg + 2 * kMaxN, n3);
  const int i2 = blockIdx.x;
  for (int i = threadIdx.x; i < n1 * n3; i += blockDim.x) {
    const int i1 = i % n1, i3 = i / n1;
    buf[i3 * L1 + i1] = box[i1 + (int64_t)n1 * (i2 + (int64_t)n2 * i3)];
  }
  __syncthreads();
  lds_fft<double>(buf, plan.d[2], L1, n1, 1, tw3, sgn);
  for (int i = threadIdx.x; i < n1 * n3; i += blockDim.x) {
    const int i1 = i % n1, i3 = i / n1;
    box[i1 + (int64_t)n1 * (i2 + (int64_t)n2 * i3)] = buf[i3 * L1 + i1];
  }
}

struct Recip {
  double b[9];  // rows b1, b2, b3 (2 pi included)
};

// box(G) *= 4 pi / |G|^2 * inv_n (G = 0 -> 0); m_d of index i_d in the box window
__global__ void hartree_kernel(int n1, int n2, int n3, Recip R, double inv_n,
                               double2 *__restrict__ box) {
  const int64_t nbox = (int64_t)n1 * n2 * n3;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbox) return;
  const int i1 = (int)(i % n1), i2 = (int)((i / n1) % n2), i3 = (int)(i / ((int64_t)n1 * n2));
  const int m1 = i1 < (n1 + 1) / 2 ? i1 : i1 - n1;
  const int m2 = i2 < (n2 + 1) / 2 ? i2 : i2 - n2;
  const int m3 = i3 < (n3 + 1) / 2 ? i3 : i3 - n3;
  double g2 = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double g = m1 * R.b[c] + m2 * R.b[3 + c] + m3 * R.b[6 + c];
    g2 += g * g;
  }
  const double f = g2 > 0.0 ? 4.0 * M_PI / g2 * inv_n : 0.0;
  box[i] = cscale(box[i], f);
}

// vout = vion + Re(box) + v_x(rho * scale)
__global__ void potential_kernel(int64_t nbox, const double *__restrict__ rho, double scale,
                                 const double *__restrict__ vion, const double2 *__restrict__ box,
                                 double *__restrict__ vout) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbox) return;
  const double n = rho[i] * scale;
  const double vx = n > 0.0 ? -cbrt(3.0 * n / M_PI) : 0.0;
  vout[i] = vion[i] + box[i].x + vx;
}

// vnext = vin + alpha (vout - vin); *dv = max |vout - vin| (one workgroup)
__global__ void mix_kernel(int64_t nbox, const double *__restrict__ vin,
                           const double *__restrict__ vout, double alpha,
                           double *__restrict__ vnext, double *__restrict__ dv) {
  __shared__ double smax[kScfThreads];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < nbox; i += blockDim.x) {
    const double d = vout[i] - vin[i];
    m = fmax(m, fabs(d));
    vnext[i] = vin[i] + alpha * d;
  }
  smax[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *dv = smax[0];
}

// box[r] = (vout[r] - vin[r], 0)
__global__ void diff_to_box_kernel(int64_t nbox, const double *__restrict__ vin,
                                   const double *__restrict__ vout, double2 *__restrict__ box) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nbox) box[i] = double2{vout[i] - vin[i], 0.0};
}

// box(G) *= K(G) * inv_n: Kerker's factor alpha |G|^2 / (|G|^2 + q0^2), alpha at G = 0
__global__ void kerker_kernel(int n1, int n2, int n3, Recip R, double alpha, double q0,
                              double inv_n, double2 *__restrict__ box) {
  const int64_t nbox = (int64_t)n1 * n2 * n3;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbox) return;
  const int i1 = (int)(i % n1), i2 = (int)((i / n1) % n2), i3 = (int)(i / ((int64_t)n1 * n2));
  const int m1 = i1 < (n1 + 1) / 2 ? i1 : i1 - n1;
  const int m2 = i2 < (n2 + 1) / 2 ? i2 : i2 - n2;
  const int m3 = i3 < (n3 + 1) / 2 ? i3 : i3 - n3;
  double g2 = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double g = m1 * R.b[c] + m2 * R.b[3 + c] + m3 * R.b[6 + c];
    g2 += g * g;
  }
  const double k = g2 > 0.0 ? alpha * g2 / (g2 + q0 * q0) : alpha;
  box[i] = cscale(box[i], k * inv_n);
}

// vnext = vin + Re(box)
__global__ void add_real_kernel(int64_t nbox, const double *__restrict__ vin,
                                const double2 *__restrict__ box, double *__restrict__ vnext) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nbox) vnext[i] = vin[i] + box[i].x;
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename F> void set_lds(F kernel, size_t bytes) {
  CHEBFI_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

}  // namespace

void launch_scf_potential(const abi_system_s *s, const double *rho, const double *vion,
                          double *vout, void *box, hipStream_t st) {
  const BoxPlan &plan = s->plan;
  const int n1 = plan.d[0].n, n2 = plan.d[1].n, n3 = plan.d[2].n;
  const int64_t nbox = (int64_t)n1 * n2 * n3;
  const double2 *tw = reinterpret_cast<const double2 *>(s->d_tw);
  double2 *bx = reinterpret_cast<double2 *>(box);
  double B[9];
  reciprocal(s->lattice, B);
  Recip R;
  for (int i = 0; i < 9; ++i) R.b[i] = B[i];
  const double omega = s->omega;
  const double scale = (double)nbox / omega;  // grid density -> electrons per bohr^3
  const int tXY = std::max(stage_threads(plan.d[0], n2), stage_threads(plan.d[1], n1));
  const int tZ = stage_threads(plan.d[2], n1);
  CHEBFI_REQUIRE(tXY <= 512 && tZ <= 512, ABI_ERR_GRID, "FFT plane too large for one workgroup");
  const size_t ldsXY = sizeof(double2) * (size_t)(n2 * (n1 + 1) + n1 + n2);
  const size_t ldsZ = sizeof(double2) * (size_t)(n3 * (n1 + 1) + n3);
  set_lds(box_xy_kernel, ldsXY);
  set_lds(box_z_kernel, ldsZ);
  hipLaunchKernelGGL(rho_to_box_kernel, dim3(nblk(nbox, kScfThreads)), dim3(kScfThreads), 0, st,
                     nbox, rho, scale, bx);
  hipLaunchKernelGGL(box_xy_kernel, dim3(n3), dim3(tXY), ldsXY, st, bx, plan, tw, -1);
  hipLaunchKernelGGL(box_z_kernel, dim3(n2), dim3(tZ), ldsZ, st, bx, plan, tw, -1);
  hipLaunchKernelGGL(hartree_kernel, dim3(nblk(nbox, kScfThreads)), dim3(kScfThreads), 0, st, n1,
                     n2, n3, R, 1.0 / (double)nbox, bx);
  hipLaunchKernelGGL(box_z_kernel, dim3(n2), dim3(tZ), ldsZ, st, bx, plan, tw, +1);
  hipLaunchKernelGGL(box_xy_kernel, dim3(n3), dim3(tXY), ldsXY, st, bx, plan, tw, +1);
  hipLaunchKernelGGL(potential_kernel, dim3(nblk(nbox, kScfThreads)), dim3(kScfThreads), 0, st,
                     nbox, rho, scale, vion, (const double2 *)bx, vout);
  CHEBFI_HIP(hipGetLastError());
}

void launch_mix(const abi_system_s *s, const double *vin, const double *vout, double alpha,
                double q0, double *vnext, double *dv, void *box, hipStream_t st) {
  const BoxPlan &plan = s->plan;
  const int n1 = plan.d[0].n, n2 = plan.d[1].n, n3 = plan.d[2].n;
  const int64_t nbox = (int64_t)n1 * n2 * n3;
  // linear mixing (and max |vout - vin|); Kerker's form then replaces vnext
  hipLaunchKernelGGL(mix_kernel, dim3(1), dim3(kScfThreads), 0, st, nbox, vin, vout, alpha, vnext,
                     dv);
  CHEBFI_HIP(hipGetLastError());
  if (q0 <= 0.0) return;
  const double2 *tw = reinterpret_cast<const double2 *>(s->d_tw);
  double2 *bx = reinterpret_cast<double2 *>(box);
  double B[9];
  reciprocal(s->lattice, B);
  Recip R;
  for (int i = 0; i < 9; ++i) R.b[i] = B[i];
  const int tXY = std::max(stage_threads(plan.d[0], n2), stage_threads(plan.d[1], n1));
  const int tZ = stage_threads(plan.d[2], n1);
  CHEBFI_REQUIRE(tXY <= 512 && tZ <= 512, ABI_ERR_GRID, "FFT plane too large for one workgroup");
  const size_t ldsXY = sizeof(double2) * (size_t)(n2 * (n1 + 1) + n1 + n2);
  const size_t ldsZ = sizeof(double2) * (size_t)(n3 * (n1 + 1) + n3);
  set_lds(box_xy_kernel, ldsXY);
  set_lds(box_z_kernel, ldsZ);
  hipLaunchKernelGGL(diff_to_box_kernel, dim3(nblk(nbox, kScfThreads)), dim3(kScfThreads), 0, st,
                     nbox, vin, vout, bx);
  hipLaunchKernelGGL(box_xy_kernel, dim3(n3), dim3(tXY), ldsXY, st, bx, plan, tw, -1);
  hipLaunchKernelGGL(box_z_kernel, dim3(n2), dim3(tZ), ldsZ, st, bx, plan, tw, -1);
  hipLaunchKernelGGL(kerker_kernel, dim3(nblk(nbox, kScfThreads)), dim3(kScfThreads), 0, st, n1,
                     n2, n3, R, alpha, q0, 1.0 / (double)nbox, bx);
  hipLaunchKernelGGL(box_z_kernel, dim3(n2), dim3(tZ), ldsZ, st, bx, plan, tw, +1);
  hipLaunchKernelGGL(box_xy_kernel, dim3(n3), dim3(tXY), ldsXY, st, bx, plan, tw, +1);
  hipLaunchKernelGGL(add_real_kernel, dim3(nblk(nbox, kScfThreads)), dim3(kScfThreads), 0, st,
                     nbox, vin, (const double2 *)bx, vnext);
  CHEBFI_HIP(hipGetLastError());
}

}  // namespace chebfi
