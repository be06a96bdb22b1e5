// Device-side helpers: enrichment functions, projector, quadrature geometry.
#pragma once

#include <hip/hip_runtime.h>

#include "efe_internal.h"

// Geometry of the uniform mesh passed by value to kernels.
struct MeshGeo {
  double lo[3], h[3];
  int ncell[3];
  int P, nloc, nq, nqp;
};

static inline MeshGeo mesh_geo(const efe_ctx *c) {
  MeshGeo g;
  for (int d = 0; d < 3; ++d) {
    g.lo[d] = c->lo[d];
    g.h[d] = c->h[d];
    g.ncell[d] = c->ncell[d];
  }
  g.P = c->P;
  g.nloc = c->nloc;
  g.nq = c->nq;
  g.nqp = c->nqp;
  return g;
}

// Position of Gauss point q of cell `cell`.
__device__ inline void quad_point(const MeshGeo &g, const double *__restrict__ xq1, int cell, int q,
                                  double x[3]) {
  int cx = cell % g.ncell[0], cy = (cell / g.ncell[0]) % g.ncell[1],
      cz = cell / (g.ncell[0] * g.ncell[1]);
  int qa = q % g.nq, qb = (q / g.nq) % g.nq, qc = q / (g.nq * g.nq);
  x[0] = g.lo[0] + cx * g.h[0] + (xq1[qa] + 1.0) * 0.5 * g.h[0];
  x[1] = g.lo[1] + cy * g.h[1] + (xq1[qb] + 1.0) * 0.5 * g.h[1];
  x[2] = g.lo[2] + cz * g.h[2] + (xq1[qc] + 1.0) * 0.5 * g.h[2];
}

// Enrichment functions: the Gaussian radial part exp(-alpha r^2) with one
// cutoff rc, or (tab != nullptr) tabulated radial parts f_l, f_l' on
// r = i dr (i < ntab; rows 2l and 2l+1 of tab) with a cutoff rcl[l] each.
struct EnrParam {
  int lmax, nf;
  double alpha, rc, t;
  const double *tab;
  int ntab;
  double dr, rcl[3];
};

static inline EnrParam enr_param(const efe_ctx *c) {
  EnrParam e;
  e.lmax = c->lmax;
  e.nf = c->nf;
  e.alpha = c->enr_alpha;
  e.rc = c->enr_rcut;
  e.t = c->enr_t;
  e.tab = c->ntab > 0 ? c->d_enr_tab : nullptr;
  e.ntab = c->ntab;
  e.dr = c->tab_dr;
  for (int l = 0; l < 3; ++l) e.rcl[l] = c->tab_rc[l];
  return e;
}

// Smooth cutoff h(r) = 1 (r <= r0), f(1-x)/(f(1-x)+f(x)) with f(y) = exp(-1/y),
// x = (r - r0)/(rc - r0), r0 = rc t/(1+t), and 0 beyond rc; also dh/dr.
__device__ inline void cutoff_fn(double r, double rc, double t, double &h, double &dh) {
  const double r0 = rc * t / (1.0 + t);
  const double x = (r - r0) / (rc - r0);
  if (x <= 0.0) {
    h = 1.0;
    dh = 0.0;
  } else if (x >= 1.0) {
    h = 0.0;
    dh = 0.0;
  } else {
    const double g = exp(-1.0 / (1.0 - x)), u = exp(-1.0 / x);
    const double s = g + u;
    h = g / s;
    dh = -g * u * (1.0 / ((1.0 - x) * (1.0 - x)) + 1.0 / (x * x)) / (s * s) / (rc - r0);
  }
}

// Cubic Hermite interpolation of a radial table (values f, slopes fp at
// r = i dr, i < n) at r: value and derivative, zero beyond the last point.
__device__ inline void hermite_fn(const double *__restrict__ f, const double *__restrict__ fp,
                                  int n, double dr, double r, double &v, double &dv) {
  const double s = r / dr;
  if (!(s <= (double)(n - 1))) {
    v = dv = 0.0;
    return;
  }
  int i = (int)floor(s);
  if (i > n - 2) i = n - 2;
  const double t = s - i, t2 = t * t, t3 = t2 * t;
  const double f0 = f[i], f1 = f[i + 1], m0 = fp[i] * dr, m1 = fp[i + 1] * dr;
  v = (2 * t3 - 3 * t2 + 1) * f0 + (t3 - 2 * t2 + t) * m0 + (-2 * t3 + 3 * t2) * f1 +
      (t3 - t2) * m1;
  dv = ((6 * t2 - 6 * t) * f0 + (3 * t2 - 4 * t + 1) * m0 + (-6 * t2 + 6 * t) * f1 +
        (3 * t2 - 2 * t) * m1) / dr;
}

// Unnormalized enrichment functions S_k(d) rad_l(r) at offset d from the
// atom, k in the order s | y z x | xy yz (3z^2-r^2) xz (x^2-y^2) (l = 0 | 1 |
// 2), rad_l = exp(-alpha r^2) h(r) or f_l(r) h_l(r); gradients when
// grad != nullptr (layout grad[3*k + axis]):
// grad phi_k = grad S_k rad_l + S_k (rad_l'(r) / r) d.
__device__ inline void enr_eval(const EnrParam &e, double dx, double dy, double dz, double *phi,
                                double *grad) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double r = sqrt(r2);
  double S[9], G[27];
  S[0] = 1.0;
  G[0] = G[1] = G[2] = 0.0;
  if (e.lmax >= 1) {
    S[1] = dy; G[3] = 0; G[4] = 1; G[5] = 0;
    S[2] = dz; G[6] = 0; G[7] = 0; G[8] = 1;
    S[3] = dx; G[9] = 1; G[10] = 0; G[11] = 0;
  }
  if (e.lmax >= 2) {
    S[4] = dx * dy;                   G[12] = dy;       G[13] = dx;       G[14] = 0;
    S[5] = dy * dz;                   G[15] = 0;        G[16] = dz;       G[17] = dy;
    S[6] = 2 * dz * dz - dx * dx - dy * dy;
                                      G[18] = -2 * dx;  G[19] = -2 * dy;  G[20] = 4 * dz;
    S[7] = dx * dz;                   G[21] = dz;       G[22] = 0;        G[23] = dx;
    S[8] = dx * dx - dy * dy;         G[24] = 2 * dx;   G[25] = -2 * dy;  G[26] = 0;
  }
  // radial parts per l and (radial derivative) / r
  double rad[3], drr[3];
  const double rs = r > 0.0 ? r : 1.0;
  if (e.tab) {
    for (int l = 0; l <= e.lmax; ++l) {
      double f, fp, h, dh;
      hermite_fn(e.tab + (int64_t)(2 * l) * e.ntab, e.tab + (int64_t)(2 * l + 1) * e.ntab, e.ntab,
                 e.dr, r, f, fp);
      cutoff_fn(r, e.rcl[l], e.t, h, dh);
      rad[l] = f * h;
      drr[l] = (fp * h + f * dh) / rs;
    }
  } else {
    double h, dh;
    cutoff_fn(r, e.rc, e.t, h, dh);
    const double ex = exp(-e.alpha * r2);
    const double eh = ex * h;
    const double d = eh * (-2.0 * e.alpha) + ex * dh / rs;
    for (int l = 0; l <= e.lmax; ++l) {
      rad[l] = eh;
      drr[l] = d;
    }
  }
  for (int k = 0; k < e.nf; ++k) {
    const int l = k == 0 ? 0 : (k < 4 ? 1 : 2);
    phi[k] = S[k] * rad[l];
    if (grad) {
      grad[3 * k + 0] = G[3 * k + 0] * rad[l] + S[k] * drr[l] * dx;
      grad[3 * k + 1] = G[3 * k + 1] * rad[l] + S[k] * drr[l] * dy;
      grad[3 * k + 2] = G[3 * k + 2] * rad[l] + S[k] * drr[l] * dz;
    }
  }
}

// PW92 LDA (unpolarized): energy per electron and potential
__device__ inline void lda_pw92(double rho, double &exc, double &vxc) {
  if (!(rho > 1e-14)) {
    exc = 0.0;
    vxc = 0.0;
    return;
  }
  const double ex = -0.75 * cbrt(3.0 / M_PI) * cbrt(rho);
  const double vx = 4.0 / 3.0 * ex;
  const double rs = cbrt(3.0 / (4.0 * M_PI * rho));
  const double A = 0.031091, a1 = 0.21370, b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
  const double srs = sqrt(rs);
  const double Q0 = -2.0 * A * (1.0 + a1 * rs);
  const double Q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs);
  const double Q1p = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs);
  const double L = log1p(1.0 / Q1);
  const double ec = Q0 * L;
  const double dec = -2.0 * A * a1 * L - Q0 * Q1p / (Q1 * Q1 + Q1);
  exc = ex + ec;
  vxc = vx + ec - rs / 3.0 * dec;
}

// Gaussian s projector with unit L2 norm, zero at r >= rcut.
__device__ inline double kb_beta(double r2, double w, double rcut) {
  if (r2 >= rcut * rcut) return 0.0;
  return pow(M_PI * w * w, -0.75) * exp(-r2 / (2.0 * w * w));
}
