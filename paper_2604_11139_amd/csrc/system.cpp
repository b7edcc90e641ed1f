// Host-side setup of one Hamiltonian: basis sphere, FFT-box index map, kinetic
// diagonal, projector matrix and FFT plans.  Built with -ffp-contract=off so
// that every floating-point expression is evaluated exactly as written.
//
// The sphere is the plane-wave basis of a k-point cut at 0.5|k+G|^2 < E_cut;
// the paper moves these coefficients into the FFT-box layout before the batched
// transforms (arXiv 2604.11139, section "Low-level operations").  Maps:
// i_d = m_d mod n_d, box index i1 + n1*(i2 + n2*i3), basis sorted by box index.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.h"

namespace chebfi {

void reciprocal(const double A[9], double B[9]) {
  // Rows b_j = 2 pi (a_k x a_l) / (a_1 . (a_2 x a_3)) for cyclic (j, k, l).
  const double *a1 = A, *a2 = A + 3, *a3 = A + 6;
  double c23[3] = {a2[1] * a3[2] - a2[2] * a3[1], a2[2] * a3[0] - a2[0] * a3[2],
                   a2[0] * a3[1] - a2[1] * a3[0]};
  double c31[3] = {a3[1] * a1[2] - a3[2] * a1[1], a3[2] * a1[0] - a3[0] * a1[2],
                   a3[0] * a1[1] - a3[1] * a1[0]};
  double c12[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2],
                   a1[0] * a2[1] - a1[1] * a2[0]};
  double det = a1[0] * c23[0] + a1[1] * c23[1] + a1[2] * c23[2];
  const double twopi = 2.0 * M_PI;
  for (int c = 0; c < 3; ++c) {
    B[0 + c] = twopi * (c23[c] / det);
    B[3 + c] = twopi * (c31[c] / det);
    B[6 + c] = twopi * (c12[c] / det);
  }
}

static void window(int n, int *lo, int *hi) {
  if (n % 2 == 0) {
    *lo = -(n / 2);
    *hi = n / 2 - 1;
  } else {
    *lo = -((n - 1) / 2);
    *hi = (n - 1) / 2;
  }
}

abi_status build_sphere(const abi_system_desc *d, Sphere *out, std::string *err) {
  double B[9];
  reciprocal(d->lattice, B);
  const double *k = d->kpt_red;
  const double qmax = std::sqrt(2.0 * d->ecut);
  int reach[3];
  for (int c = 0; c < 3; ++c) {
    const double *a = d->lattice + 3 * c;
    double alen = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    reach[c] = (int)std::ceil(alen * qmax / (2.0 * M_PI) + std::fabs(k[c])) + 2;
  }
  const int n1 = d->ngrid[0], n2 = d->ngrid[1], n3 = d->ngrid[2];
  int lo[3], hi[3];
  window(n1, &lo[0], &hi[0]);
  window(n2, &lo[1], &hi[1]);
  window(n3, &lo[2], &hi[2]);
  struct Pt {
    int64_t box;
    int m[3];
    double e, q[3];
  };
  std::vector<Pt> pts;
  for (int m3 = -reach[2]; m3 <= reach[2]; ++m3)
    for (int m2 = -reach[1]; m2 <= reach[1]; ++m2)
      for (int m1 = -reach[0]; m1 <= reach[0]; ++m1) {
        double f1 = (double)m1 + k[0], f2 = (double)m2 + k[1], f3 = (double)m3 + k[2];
        double qx = f1 * B[0] + f2 * B[3] + f3 * B[6];
        double qy = f1 * B[1] + f2 * B[4] + f3 * B[7];
        double qz = f1 * B[2] + f2 * B[5] + f3 * B[8];
        double e = 0.5 * (qx * qx + qy * qy + qz * qz);
        if (!(e < d->ecut)) continue;
        if (m1 < lo[0] || m1 > hi[0] || m2 < lo[1] || m2 > hi[1] || m3 < lo[2] || m3 > hi[2]) {
          *err = "G-sphere does not fit the FFT box";
          return ABI_ERR_GRID;
        }
        int i1 = ((m1 % n1) + n1) % n1, i2 = ((m2 % n2) + n2) % n2, i3 = ((m3 % n3) + n3) % n3;
        Pt p;
        p.box = (int64_t)i1 + (int64_t)n1 * ((int64_t)i2 + (int64_t)n2 * (int64_t)i3);
        p.m[0] = m1;
        p.m[1] = m2;
        p.m[2] = m3;
        p.e = e;
        p.q[0] = qx;
        p.q[1] = qy;
        p.q[2] = qz;
        pts.push_back(p);
      }
  std::sort(pts.begin(), pts.end(), [](const Pt &a, const Pt &b) { return a.box < b.box; });
  const size_t npw = pts.size();
  out->miller.resize(npw * 3);
  out->box_index.resize(npw);
  out->kinetic.resize(npw);
  out->qcart.resize(npw * 3);
  out->gcart.resize(npw * 3);
  for (size_t i = 0; i < npw; ++i) {
    const Pt &p = pts[i];
    out->box_index[i] = (int32_t)p.box;
    out->kinetic[i] = p.e;
    for (int c = 0; c < 3; ++c) {
      out->miller[3 * i + c] = p.m[c];
      out->qcart[3 * i + c] = p.q[c];
      out->gcart[3 * i + c] =
          (double)p.m[0] * B[0 + c] + (double)p.m[1] * B[3 + c] + (double)p.m[2] * B[6 + c];
    }
  }
  return ABI_OK;
}

// P[g, 4R+i] (column-major, interleaved complex), four Gaussian projectors per
// atom: s = g e^{-iG.R}/sqrt(Omega), p_c = rc q_c g e^{-iG.R}/sqrt(Omega).
void build_projectors(const abi_system_desc *d, const Sphere &s, std::vector<double> *P) {
  const size_t npw = s.kinetic.size();
  const int nproj = 4 * d->natom;
  const double *A = d->lattice;
  double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
               A[2] * (A[3] * A[7] - A[4] * A[6]);
  const double inv_sqrt_omega = 1.0 / std::sqrt(std::fabs(det));
  const double rc = d->rc;
  P->assign(npw * (size_t)nproj * 2, 0.0);
  std::vector<double> g(npw);
  for (size_t i = 0; i < npw; ++i) {
    const double *q = &s.qcart[3 * i];
    g[i] = std::exp(-0.5 * (rc * rc) * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]));
  }
  for (int r = 0; r < d->natom; ++r) {
    const double *R = d->tau_cart + 3 * r;
    for (size_t i = 0; i < npw; ++i) {
      const double *G = &s.gcart[3 * i];
      const double ph = G[0] * R[0] + G[1] * R[1] + G[2] * R[2];
      const double cr = std::cos(ph) * inv_sqrt_omega, ci = -std::sin(ph) * inv_sqrt_omega;
      const double *q = &s.qcart[3 * i];
      const double amp[4] = {g[i], rc * q[0] * g[i], rc * q[1] * g[i], rc * q[2] * g[i]};
      for (int c = 0; c < 4; ++c) {
        double *dst = P->data() + 2 * ((size_t)(4 * r + c) * npw + i);
        dst[0] = amp[c] * cr;
        dst[1] = amp[c] * ci;
      }
    }
  }
}

bool make_plan(int n, Plan1D *p) {
  p->n = n;
  p->nstage = 0;
  int rem = n;
  // Radix 4 first (fewest LDS passes), then 2, 3, 5.
  const int order[4] = {4, 2, 3, 5};
  for (int oi = 0; oi < 4; ++oi) {
    const int r = order[oi];
    while (rem % r == 0) {
      if (p->nstage >= kMaxStages) return false;
      p->radix[p->nstage++] = r;
      rem /= r;
    }
  }
  return rem == 1 && n >= 2;
}

}  // namespace chebfi
