// Radial Kohn-Sham problem of one isolated atom of the synthetic
// pseudopotential and the pristine enrichment tables built from it
// (Sec. II.B): single-atom Kohn-Sham eigenfunctions, a radial function times a
// real spherical harmonic, truncated at r0 chosen by three rules.
//
// u = r R on r_i = (i + 1) h (i = 0 .. n-1), zero at r = 0 and r = (n + 1) h;
// channel l is the symmetric tridiagonal T_l (three-point kinetic term,
// centrifugal term, v_eff), plus D q q^T in the s channel for the projector
// (q_i = sqrt(4 pi h) r_i beta(r_i), in the vector sqrt(h) u).  Levels by
// bisection on Sturm counts (multisection by a work-group), the rank-one term
// through the inertia of the bordered matrix: for A = T - sigma and D > 0,
// neg(A + D q q^T) = neg(A) - 1 + [q^T A^-1 q > -1/D], q^T A^-1 q from the
// same LDL^T sweep.  Vectors by inverse iteration (the s channel with the
// projector: (T - mu)^-1 q).  Hartree by the same three-point rule, PW92,
// Fermi occupations of the 2(2l+1)-fold levels, linear density mixing.  The
// converged density and the potential of the neutral atom (density plus the
// Gaussian smeared nuclear charge) are tabulated for the atomic fields of
// Sec. III.C.
#include <cmath>

#include "efe_device.h"

namespace {

struct RadArgs {
  int n, lmax, ns;
  double h, D;   // D = 0: no projector
};

__device__ inline double rgrid(const RadArgs &a, int i) { return (i + 1) * a.h; }

// diagonal of T_l at grid index i
__device__ inline double tdiag(const RadArgs &a, const double *__restrict__ v, int l, int i) {
  const double r = rgrid(a, i);
  return 1.0 / (a.h * a.h) + l * (l + 1) / (2.0 * r * r) + v[i];
}

// number of eigenvalues of channel l below sigma
__device__ int sturm_count(const RadArgs &a, const double *__restrict__ v,
                           const double *__restrict__ q, int l, double sigma) {
  const double e = -0.5 / (a.h * a.h), e2 = e * e;
  const double pivmin = 1e-300;
  const bool kb = l == 0 && a.D != 0.0;
  int neg = 0;
  double d = 0.0, y = 0.0, s = 0.0;
  for (int i = 0; i < a.n; ++i) {
    const double di = tdiag(a, v, l, i) - sigma;
    double lm = 0.0;
    if (i == 0) {
      d = di;
    } else {
      lm = e / d;
      d = di - e2 / d;
    }
    if (fabs(d) < pivmin) d = -pivmin;
    neg += d < 0.0;
    if (kb) {
      y = (i == 0 ? q[0] : q[i] - lm * y);
      s += y * y / d;
    }
  }
  if (kb) neg += (s > -1.0 / a.D ? 1 : 0) - 1;
  return neg;
}

// level k of channel l per work-group (blockIdx.x = l * ns + k): multisection
// with 256 probes per round until the bracket is a few ulps wide
__global__ __launch_bounds__(256) void k_rad_bisect(RadArgs a, const double *__restrict__ v,
                                                    const double *__restrict__ q,
                                                    double *__restrict__ eps) {
  __shared__ double lo_s[256], hi_s[256];
  __shared__ double bracket[2];
  const int l = blockIdx.x / a.ns, k = blockIdx.x % a.ns, t = threadIdx.x;
  // Gershgorin bracket (the rank-one term lies in [0, D |q|^2])
  if (t == 0) {
    const double e = 0.5 / (a.h * a.h);
    double lo = INFINITY, hi = -INFINITY, q2 = 0.0;
    for (int i = 0; i < a.n; ++i) {
      const double di = tdiag(a, v, l, i);
      const double rad = (i > 0 ? e : 0.0) + (i < a.n - 1 ? e : 0.0);
      lo = fmin(lo, di - rad);
      hi = fmax(hi, di + rad);
      if (l == 0 && a.D != 0.0) q2 += q[i] * q[i];
    }
    bracket[0] = lo - 1.0;
    bracket[1] = hi + a.D * q2 + 1.0;
  }
  __syncthreads();
  for (int round = 0; round < 16; ++round) {
    const double lo = bracket[0], hi = bracket[1];
    if (!(hi - lo > 4.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)))) break;
    const double sig = lo + (t + 1) * ((hi - lo) / 257.0);
    const int cnt = sturm_count(a, v, q, l, sig);
    lo_s[t] = cnt <= k ? sig : -INFINITY;   // below level k
    hi_s[t] = cnt >= k + 1 ? sig : INFINITY;  // at or above level k
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) {
        lo_s[t] = fmax(lo_s[t], lo_s[t + s]);
        hi_s[t] = fmin(hi_s[t], hi_s[t + s]);
      }
      __syncthreads();
    }
    if (t == 0) {
      if (lo_s[0] > bracket[0]) bracket[0] = lo_s[0];
      if (hi_s[0] < bracket[1]) bracket[1] = hi_s[0];
    }
    __syncthreads();
  }
  if (t == 0) eps[blockIdx.x] = 0.5 * (bracket[0] + bracket[1]);
}

// x = (T_l - mu)^-1 b in place (b in x), Gaussian elimination with partial
// pivoting on the tridiagonal (fill-in of one superdiagonal); work: 3 n
__device__ void tri_solve(const RadArgs &a, const double *__restrict__ v, int l, double mu,
                          double *__restrict__ x, double *__restrict__ w) {
  const int n = a.n;
  const double e = -0.5 / (a.h * a.h);
  double *U0 = w, *U1 = w + n, *U2 = w + 2 * n;   // rows of U: diag, +1, +2
  // current row's (diag, super) carried down the elimination
  double cd = tdiag(a, v, l, 0) - mu, cs = n > 1 ? e : 0.0;
  for (int i = 0; i < n - 1; ++i) {
    const double nd = tdiag(a, v, l, i + 1) - mu, ns = i + 2 < n ? e : 0.0;
    const double sub = e;   // the next row's entry below cd
    if (fabs(sub) > fabs(cd)) {
      // swap row i (cd, cs, 0) with row i+1 (sub, nd, ns)
      const double m = cd / sub;
      U0[i] = sub;
      U1[i] = nd;
      U2[i] = ns;
      const double xi = x[i];
      x[i] = x[i + 1];
      x[i + 1] = xi - m * x[i];
      cd = cs - m * nd;
      cs = -m * ns;
    } else {
      const double piv = cd != 0.0 ? cd : 1e-300;
      const double m = sub / piv;
      U0[i] = piv;
      U1[i] = cs;
      U2[i] = 0.0;
      x[i + 1] -= m * x[i];
      cd = nd - m * cs;
      cs = ns;
    }
  }
  U0[n - 1] = cd != 0.0 ? cd : 1e-300;
  x[n - 1] /= U0[n - 1];
  if (n > 1) x[n - 2] = (x[n - 2] - U1[n - 2] * x[n - 1]) / U0[n - 2];
  for (int i = n - 3; i >= 0; --i) x[i] = (x[i] - U1[i] * x[i + 1] - U2[i] * x[i + 2]) / U0[i];
}

// eigenvector of level (l, k) per work-group: one thread solves, the group
// normalizes (h sum u^2 = 1, largest |u| positive); u[(l ns + k) n + i]
__global__ __launch_bounds__(256) void k_rad_vectors(RadArgs a, const double *__restrict__ v,
                                                     const double *__restrict__ q,
                                                     const double *__restrict__ eps,
                                                     double *__restrict__ u,
                                                     double *__restrict__ work) {
  __shared__ double red[256];
  __shared__ int arg[256];
  const int lk = blockIdx.x, l = lk / a.ns, t = threadIdx.x;
  double *x = u + (int64_t)lk * a.n;
  double *w = work + (int64_t)lk * 3 * a.n;
  const double mu = eps[lk];
  if (t == 0) {
    if (l == 0 && a.D != 0.0) {
      for (int i = 0; i < a.n; ++i) x[i] = q[i];
      tri_solve(a, v, l, mu, x, w);
    } else {
      for (int i = 0; i < a.n; ++i) x[i] = 1.0;
      for (int it = 0; it < 3; ++it) {
        tri_solve(a, v, l, mu, x, w);
        double m = 0.0;
        for (int i = 0; i < a.n; ++i) m = fmax(m, fabs(x[i]));
        for (int i = 0; i < a.n; ++i) x[i] /= m;
      }
    }
  }
  __syncthreads();
  // the scaled vector sqrt(h) u has unit 2-norm: u = x / sqrt(h sum x^2)
  double s = 0.0, best = -1.0;
  int bi = 0;
  for (int i = t; i < a.n; i += 256) {
    s += x[i] * x[i];
    if (fabs(x[i]) > best) best = fabs(x[i]), bi = i;
  }
  red[t] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st) red[t] += red[t + st];
    __syncthreads();
  }
  const double nrm = sqrt(a.h * red[0]);
  __syncthreads();
  red[t] = best;
  arg[t] = bi;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st && (red[t + st] > red[t] || (red[t + st] == red[t] && arg[t + st] < arg[t]))) {
      red[t] = red[t + st];
      arg[t] = arg[t + st];
    }
    __syncthreads();
  }
  const double sg = x[arg[0]] > 0.0 ? 1.0 : -1.0;
  __syncthreads();
  for (int i = t; i < a.n; i += 256) x[i] *= sg / nrm;
}

// local pseudopotential, projector vector and the Gaussian start density
__global__ void k_rad_init(RadArgs a, double Z, double rc, double amp, double rg, double w,
                           double rcut, double a_rho, double *__restrict__ vloc,
                           double *__restrict__ q, double *__restrict__ rho) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const double r = rgrid(a, i);
  const double x = r / rc;
  const double eor = x < 1e-6 ? (2.0 / (rc * sqrt(M_PI))) * (1.0 - x * x / 3.0) : erf(x) / r;
  vloc[i] = -Z * eor + amp * exp(-(r / rg) * (r / rg));
  q[i] = w > 0.0 ? sqrt(4.0 * M_PI * a.h) * r * kb_beta(r * r, w, rcut) : 0.0;
  rho[i] = Z * pow(a_rho / M_PI, 1.5) * exp(-a_rho * r * r);
}

// v_eff = vloc + v_H + v_xc at rho_in; v_H = w / r with w'' = -4 pi r rho,
// w(0) = 0, w((n+1) h) = Q (the Thomas algorithm on the constant tridiagonal,
// one thread; the charge summed in index order)
__global__ void k_rad_veff(RadArgs a, const double *__restrict__ vloc,
                           const double *__restrict__ rho, double *__restrict__ v,
                           double *__restrict__ cp, double *__restrict__ dp) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int n = a.n;
  const double h = a.h;
  double Q = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = rgrid(a, i);
    Q += r * r * rho[i];
  }
  Q *= 4.0 * M_PI * h;
  // rows: w_{i-1} - 2 w_i + w_{i+1} = g_i
  for (int i = 0; i < n; ++i) {
    const double r = rgrid(a, i);
    double g = -4.0 * M_PI * h * h * r * rho[i];
    if (i == n - 1) g -= Q;
    if (i == 0) {
      cp[0] = 1.0 / -2.0;
      dp[0] = g / -2.0;
    } else {
      const double den = -2.0 - cp[i - 1];
      cp[i] = 1.0 / den;
      dp[i] = (g - dp[i - 1]) / den;
    }
  }
  double wn = dp[n - 1];
  v[n - 1] = wn;
  for (int i = n - 2; i >= 0; --i) {
    wn = dp[i] - cp[i] * wn;
    v[i] = wn;
  }
  for (int i = 0; i < n; ++i) {
    double exc, vxc;
    lda_pw92(rho[i], exc, vxc);
    v[i] = vloc[i] + v[i] / rgrid(a, i) + vxc;
  }
}

__device__ inline double expit(double x) {
  return x >= 0.0 ? 1.0 / (1.0 + exp(-x)) : exp(x) / (1.0 + exp(x));
}

// Fermi level of the 2(2l+1)-fold levels for Z electrons (bisection on the
// electron excess written as an integer count plus the Fermi tails, as the
// cluster solver does) and the occupations; one thread
__global__ void k_rad_occ(RadArgs a, double Z, double kT, const double *__restrict__ eps,
                          double *__restrict__ occ, double *__restrict__ mu_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int nl = (a.lmax + 1) * a.ns;
  double lo = INFINITY, hi = -INFINITY;
  for (int j = 0; j < nl; ++j) lo = fmin(lo, eps[j]), hi = fmax(hi, eps[j]);
  lo -= 50.0 * kT + 1.0;
  hi += 50.0 * kT + 1.0;
  for (int it = 0; it < 200; ++it) {
    const double mu = 0.5 * (lo + hi);
    double cnt = 0.0, tails = 0.0;
    for (int j = 0; j < nl; ++j) {
      const int l = j / a.ns;
      const double x = (eps[j] - mu) / kT;
      for (int m = 0; m < 2 * l + 1; ++m) {
        if (x <= 0.0) {
          cnt += 1.0;
          tails -= expit(x);
        } else {
          tails += expit(-x);
        }
      }
    }
    const double excess = (2.0 * cnt - Z) + 2.0 * tails;
    if (excess < 0.0) lo = mu;
    else hi = mu;
  }
  const double mu = 0.5 * (lo + hi);
  *mu_out = mu;
  for (int j = 0; j < nl; ++j) {
    const int l = j / a.ns;
    occ[j] = 2.0 * (2 * l + 1) * expit(-(eps[j] - mu) / kT);
  }
}

// rho_out = sum occ u^2 / (4 pi r^2); res = sqrt(4 pi h sum r^2 (rho_out -
// rho_in)^2); rho_next = rho_in + beta (rho_out - rho_in); one work-group
__global__ __launch_bounds__(256) void k_rad_density(RadArgs a, const double *__restrict__ u,
                                                     const double *__restrict__ occ,
                                                     const double *__restrict__ rho_in,
                                                     double beta, double *__restrict__ rho_out,
                                                     double *__restrict__ rho_next,
                                                     double *__restrict__ res) {
  __shared__ double red[256];
  const int t = threadIdx.x, nl = (a.lmax + 1) * a.ns;
  double s = 0.0;
  for (int i = t; i < a.n; i += 256) {
    const double r = rgrid(a, i);
    double acc = 0.0;
    for (int j = 0; j < nl; ++j) {
      const double x = u[(int64_t)j * a.n + i];
      acc += occ[j] * x * x;
    }
    const double ro = acc / (4.0 * M_PI * r * r);
    const double d = ro - rho_in[i];
    rho_out[i] = ro;
    rho_next[i] = rho_in[i] + beta * d;
    s += r * r * d * d;
  }
  red[t] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st) red[t] += red[t + st];
    __syncthreads();
  }
  if (t == 0) *res = sqrt(4.0 * M_PI * a.h * red[0]);
}

// per l: the table f_l = u / r^{l+1} of the lowest level (f_l(0) from the
// even expansion, slopes by central differences) and r0 by the three rules;
// one work-group per l.  tab rows 2l, 2l+1 of length n + 1.
__global__ __launch_bounds__(256) void k_rad_tables(RadArgs a, const double *__restrict__ u,
                                                    double t_cut, double r0_max, double norm_tol,
                                                    double slope_tol, double *__restrict__ tab,
                                                    double *__restrict__ r0_out) {
  __shared__ int best[256];
  __shared__ double rturn_s;
  const int l = blockIdx.x, t = threadIdx.x, n = a.n;
  const double h = a.h;
  const double *x = u + (int64_t)(l * a.ns) * n;   // lowest level of channel l
  double *f = tab + (int64_t)(2 * l) * (n + 1), *df = tab + (int64_t)(2 * l + 1) * (n + 1);
  for (int i = t; i < n; i += 256) f[i + 1] = x[i] / pow(rgrid(a, i), l + 1);
  __syncthreads();
  if (t == 0) {
    f[0] = (4.0 * f[1] - f[2]) / 3.0;
    // last interior extremum of u
    int last = -1;
    for (int i = 1; i < n - 1; ++i)
      if ((x[i + 1] - x[i]) * (x[i] - x[i - 1]) <= 0.0) last = i;
    rturn_s = last >= 0 ? rgrid(a, last) : 0.0;
  }
  __syncthreads();
  for (int i = t; i <= n; i += 256) {
    if (i == 0) df[0] = 0.0;
    else if (i == n) df[n] = (f[n] - f[n - 1]) / h;
    else df[i] = (f[i + 1] - f[i - 1]) / (2.0 * h);
  }
  // candidates: the smallest grid radius meeting the three rules
  int mine = INT32_MAX;
  for (int i = t; i < n; i += 256) {
    const double r = rgrid(a, i);
    if (r < rturn_s || r > r0_max) continue;
    // dR/dr with R = u / r: central differences, one-sided at the ends
    auto R = [&](int j) { return x[j] / rgrid(a, j); };
    const double dR = i == 0 ? (R(1) - R(0)) / h
                             : (i == n - 1 ? (R(n - 1) - R(n - 2)) / h
                                           : (R(i + 1) - R(i - 1)) / (2.0 * h));
    if (!(fabs(dR) < slope_tol)) continue;
    const double rc = r * (1.0 + 1.0 / t_cut);
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
      double hc, dh;
      cutoff_fn(rgrid(a, j), rc, t_cut, hc, dh);
      const double y = x[j] * hc;
      s += y * y;
    }
    if (1.0 - h * s <= norm_tol) mine = min(mine, i);
  }
  best[t] = mine;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st) best[t] = min(best[t], best[t + st]);
    __syncthreads();
  }
  if (t == 0) r0_out[l] = best[0] == INT32_MAX ? r0_max : rgrid(a, best[0]);
}

// atomic fields of the converged atom: rows rho, rho', phi, phi' at r = i h
// (i = 0..n), phi = v_H[rho] - Z erf(r/rb)/r with v_H by the same Thomas
// solve as k_rad_veff; values at r = 0 from (4 f(h) - f(2h))/3, slopes by
// central differences (one-sided at the end, 0 at r = 0); one thread
__global__ void k_rad_atab(RadArgs a, double Z, double rb, const double *__restrict__ rho,
                           double *__restrict__ cp, double *__restrict__ dp,
                           double *__restrict__ atab) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int n = a.n, m = n + 1;
  const double h = a.h;
  double Q = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = rgrid(a, i);
    Q += r * r * rho[i];
  }
  Q *= 4.0 * M_PI * h;
  for (int i = 0; i < n; ++i) {
    const double r = rgrid(a, i);
    double g = -4.0 * M_PI * h * h * r * rho[i];
    if (i == n - 1) g -= Q;
    if (i == 0) {
      cp[0] = 1.0 / -2.0;
      dp[0] = g / -2.0;
    } else {
      const double den = -2.0 - cp[i - 1];
      cp[i] = 1.0 / den;
      dp[i] = (g - dp[i - 1]) / den;
    }
  }
  double *fr = atab, *dfr = atab + m, *fp = atab + 2 * m, *dfp = atab + 3 * m;
  double w = dp[n - 1];
  for (int i = n - 1; i >= 0; --i) {
    if (i < n - 1) w = dp[i] - cp[i] * w;
    const double r = rgrid(a, i), x = r / rb;
    const double eor = x < 1e-6 ? (2.0 / (rb * sqrt(M_PI))) * (1.0 - x * x / 3.0) : erf(x) / r;
    fp[i + 1] = w / r - Z * eor;
    fr[i + 1] = rho[i];
  }
  fr[0] = (4.0 * fr[1] - fr[2]) / 3.0;
  fp[0] = (4.0 * fp[1] - fp[2]) / 3.0;
  for (int i = 0; i <= n; ++i) {
    if (i == 0) {
      dfr[0] = dfp[0] = 0.0;
    } else if (i == n) {
      dfr[n] = (fr[n] - fr[n - 1]) / h;
      dfp[n] = (fp[n] - fp[n - 1]) / h;
    } else {
      dfr[i] = (fr[i + 1] - fr[i - 1]) / (2.0 * h);
      dfp[i] = (fp[i + 1] - fp[i - 1]) / (2.0 * h);
    }
  }
}

}  // namespace

extern "C" efe_status efe_radial_atom(const efe_system_desc *sys, int32_t atom,
                                      const efe_radial_params *prm, void *stream, double *eps,
                                      double *u, double *occ, double *rho, double *r0,
                                      double *tab, double *atab, efe_radial_report *rep) {
  auto fail = [](efe_status st, const std::string &m) {
    efe_set_global_error("efe_radial_atom: " + m);
    return st;
  };
  if (!sys || !prm || !eps || !u || !occ || !rho || !r0 || !tab)
    return fail(EFE_EINVAL, "null argument");
  if (atom < 0 || atom >= sys->natoms || !sys->Z) return fail(EFE_EINVAL, "atom out of range");
  if (prm->n < 8 || !(prm->h > 0) || prm->lmax < 0 || prm->lmax > 2 || prm->nstates < 1 ||
      prm->nstates > 8 || !(prm->kT > 0) || !(prm->mix_beta > 0 && prm->mix_beta <= 1) ||
      !(prm->tol > 0) || prm->maxit < 1 || !(sys->enr_t > 0) || !(sys->loc_rc > 0) ||
      !(sys->loc_rg > 0) || !(sys->rho_alpha > 0) || (sys->kb_width > 0 && !(sys->kb_rcut > 0)))
    return fail(EFE_EINVAL, "bad parameters");
  hipStream_t st = (hipStream_t)stream;
  RadArgs a;
  a.n = prm->n;
  a.h = prm->h;
  a.lmax = prm->lmax;
  a.ns = prm->nstates;
  a.D = sys->kb_width > 0 ? sys->kb_D : 0.0;
  const int n = a.n, nl = (a.lmax + 1) * a.ns;
  const double Z = sys->Z[atom];
  // workspace: vloc, q, v, rho_in, rho_next, Thomas (2n), vectors' (3 n per level), scalars
  const size_t nw = (size_t)7 * n + (size_t)3 * n * nl + 4;
  double *wsp = nullptr;
  if (hipMalloc(&wsp, nw * 8) != hipSuccess) return fail(EFE_EHIP, "device allocation failed");
  double *vloc = wsp, *q = vloc + n, *v = q + n, *rin = v + n, *rnext = rin + n, *cp = rnext + n,
         *dp = cp + n, *vw = dp + n, *sc = vw + (size_t)3 * n * nl;
  efe_status out = EFE_OK;
  int it = 0;
  double res = INFINITY, mu = 0.0;
  k_rad_init<<<(n + 255) / 256, 256, 0, st>>>(a, Z, sys->loc_rc, sys->loc_amp, sys->loc_rg,
                                               sys->kb_width, sys->kb_rcut, sys->rho_alpha, vloc, q,
                                               rin);
  for (it = 1; it <= prm->maxit; ++it) {
    k_rad_veff<<<1, 64, 0, st>>>(a, vloc, rin, v, cp, dp);
    k_rad_bisect<<<nl, 256, 0, st>>>(a, v, q, eps);
    k_rad_vectors<<<nl, 256, 0, st>>>(a, v, q, eps, u, vw);
    k_rad_occ<<<1, 64, 0, st>>>(a, Z, prm->kT, eps, occ, sc + 1);
    k_rad_density<<<1, 256, 0, st>>>(a, u, occ, rin, prm->mix_beta, rho, rnext, sc);
    double hs[2];
    if (hipMemcpyAsync(hs, sc, 16, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      out = fail(EFE_EHIP, "HIP error in the radial SCF");
      break;
    }
    res = hs[0];
    mu = hs[1];
    if (!std::isfinite(res)) {
      out = fail(EFE_ENUMERIC, "radial SCF produced a non-finite density");
      break;
    }
    if (res < prm->tol) break;
    std::swap(rin, rnext);
  }
  if (!out && it > prm->maxit) it = prm->maxit;
  if (!out) {
    k_rad_tables<<<a.lmax + 1, 256, 0, st>>>(a, u, sys->enr_t, 10.0, 5e-3, 5e-3, tab, r0);
    if (atab) k_rad_atab<<<1, 64, 0, st>>>(a, Z, sys->loc_rc, rho, cp, dp, atab);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
      out = fail(EFE_EHIP, "HIP error in the radial tables");
  }
  (void)hipFree(wsp);
  if (rep) {
    rep->iterations = it;
    rep->residual = res;
    rep->mu = mu;
  }
  if (!out && !(res < prm->tol))
    return fail(EFE_ENOTCONV, "radial SCF did not reach the tolerance");
  return out;
}
