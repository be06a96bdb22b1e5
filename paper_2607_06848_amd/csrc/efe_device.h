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

struct EnrParam {
  int lmax, nf;
  double alpha, rc, t;
};

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

// Unnormalized enrichment functions S_k(d) exp(-alpha r^2) h(r) at offset d
// from the atom, k in the order s | y z x | xy yz (3z^2-r^2) xz (x^2-y^2);
// gradients when grad != nullptr (layout grad[3*k + axis]).
__device__ inline void enr_eval(const EnrParam &e, double dx, double dy, double dz, double *phi,
                                double *grad) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double r = sqrt(r2);
  double h, dh;
  cutoff_fn(r, e.rc, e.t, h, dh);
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
  const double ex = exp(-e.alpha * r2);
  const double eh = ex * h;
  for (int k = 0; k < e.nf; ++k) phi[k] = S[k] * eh;
  if (grad) {
    const double rs = r > 0.0 ? r : 1.0;
    const double rad = eh * (-2.0 * e.alpha) + ex * dh / rs;   // multiplies d
    for (int k = 0; k < e.nf; ++k) {
      grad[3 * k + 0] = G[3 * k + 0] * eh + S[k] * rad * dx;
      grad[3 * k + 1] = G[3 * k + 1] * eh + S[k] * rad * dy;
      grad[3 * k + 2] = G[3 * k + 2] * eh + S[k] * rad * dz;
    }
  }
}

// Gaussian s projector with unit L2 norm, zero at r >= rcut.
__device__ inline double kb_beta(double r2, double w, double rcut) {
  if (r2 >= rcut * rcut) return 0.0;
  return pow(M_PI * w * w, -0.75) * exp(-r2 / (2.0 * w * w));
}
