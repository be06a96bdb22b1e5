// Self-consistent field support (Sec. II.A, III.C; Fermi-Dirac smearing and
// Anderson mixing of Sec. IV):
//   rho_in -> Poisson for phi^rem (CFE stiffness, Jacobi CG) -> v_eff =
//   phi^at + phi^rem + v_short + v_xc(rho_in) -> operators -> Lanczos bound
//   -> residual-filter passes + Rayleigh-Ritz -> Fermi level -> rho_out ->
//   energies at rho_out -> Anderson update of rho_in.
// Energies at the output density:
//   E = 2 sum f eps - int rho_out v_in + E_xc[rho_out] + E_el[rho_out],
//   E_el = 1/2 sum_IJ <n_I, n_J> - E_self + dE_ZZ + int Drho phi^at
//          + 1/2 int Drho phi^rem[rho_out] + int rho_out v_short,
//   F = E - T S.  LDA is Perdew-Wang 1992 (unpolarized), zero for rho <= 1e-14.
#include <chrono>
#include <cmath>
#include <vector>

#include "efe_device.h"

#define KB_HA_PER_K 3.166811563e-6

// ------------------------------------------------------------------ state
struct ScfState {
  bool init = false;
  double *rho_at = nullptr, *phi_at = nullptr, *v_short = nullptr;   // [n_qpts]
  double *rho_in = nullptr, *rho_out = nullptr, *v_in = nullptr, *phiq = nullptr;
  double *phi_rem = nullptr, *phi_out = nullptr;                      // [n_nodes]
  double *Kdiag = nullptr;                                            // [n_nodes]
  double *cg = nullptr;                                               // r, z, p, Ap, b
  double *Ktile = nullptr;   // cell stiffness in the 16x16x4 MFMA operand layout
  double *part = nullptr;    // per-work-group partial sums of the CG reductions
  double *ycell = nullptr;   // K x cell by cell, before the gather to nodes
  double *hist = nullptr;                                             // Anderson X, F ring
  double *scal = nullptr;                                             // device scalars
  double *f = nullptr;                                                // occupations [N]
  double *kdiag_k = nullptr, *u_k = nullptr, *uq_k = nullptr;         // Kerker solve
  double kerker_k0 = -1.0;
  int32_t *cell_ptr = nullptr, *cell_atom = nullptr;                  // cell -> atoms
  double e_const = 0.0;
  int iter = 0, nhist = 0, hist_m = 0;
  double E_prev = 0.0;
  bool have_E = false;
};

static ScfState &S(efe_ctx *c) {
  static_assert(sizeof(void *) == 8, "64-bit only");
  if (!c->scf) c->scf = new ScfState();
  return *(ScfState *)c->scf;
}

void efe_scf_free(efe_ctx *c) {
  if (!c->scf) return;
  ScfState &s = *(ScfState *)c->scf;
  void *ptrs[] = {s.rho_at, s.phi_at, s.v_short, s.rho_in, s.rho_out, s.v_in, s.phiq,
                  s.phi_rem, s.phi_out, s.Kdiag, s.cg, s.hist, s.scal, s.f, s.cell_ptr,
                  s.cell_atom, s.Ktile, s.part, s.ycell, s.kdiag_k, s.u_k, s.uq_k};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete (ScfState *)c->scf;
  c->scf = nullptr;
}

// ------------------------------------------------------------------ kernels
__device__ inline double erf_over_r(double r, double a) {
  const double x = r / a;
  return x < 1e-6 ? (2.0 / (a * sqrt(M_PI))) * (1.0 - x * x / 3.0) : erf(x) / r;
}

// rho^(I), phi^(I) and v_short summed over atoms at every Gauss point:
// Gaussian forms, or (atab != nullptr) the tabulated radial solution (rows
// rho, rho', phi, phi' of natab points at r = i adr)
__global__ void k_atomic_fields(MeshGeo g, const double *__restrict__ xq1, int natoms,
                                const double *__restrict__ xyz, const double *__restrict__ Z,
                                double a_rho, double rb, double amp, double rg,
                                const double *__restrict__ atab, int natab, double adr,
                                double *__restrict__ rho_at, double *__restrict__ phi_at,
                                double *__restrict__ v_short) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nq = (int64_t)g.ncell[0] * g.ncell[1] * g.ncell[2] * g.nqp;
  if (idx >= nq) return;
  double x[3];
  quad_point(g, xq1, (int)(idx / g.nqp), (int)(idx % g.nqp), x);
  double ra = 0.0, pa = 0.0, vs = 0.0;
  const double norm = pow(a_rho / M_PI, 1.5);
  for (int I = 0; I < natoms; ++I) {
    const double dx = x[0] - xyz[3 * I], dy = x[1] - xyz[3 * I + 1], dz = x[2] - xyz[3 * I + 2];
    const double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
    if (atab) {
      double v, dv;
      hermite_fn(atab, atab + natab, natab, adr, r, v, dv);
      ra += v;
      hermite_fn(atab + 2 * natab, atab + 3 * natab, natab, adr, r, v, dv);
      pa += v;
    } else {
      ra += Z[I] * norm * exp(-a_rho * r2);
      pa += Z[I] * (erf_over_r(r, 1.0 / sqrt(a_rho)) - erf_over_r(r, rb));
    }
    vs += amp * exp(-(r / rg) * (r / rg));
  }
  rho_at[idx] = ra;
  phi_at[idx] = pa;
  v_short[idx] = vs;
}

// <n_I, n_J> of two tabulated neutral atoms at distance R (n = rho + b, b
// the Gaussian smeared charge -Z of width rb, phi the potential of n):
// 2 pi sum_k w_k r_k^2 n(r_k) sum_m u_m phi(d_km), d_km^2 = r_k^2 + R^2 -
// 2 r_k R mu_m, over the table points (trapezoid weights w) and the
// Gauss-Legendre nodes (mu, u).  One work-group per unordered pair i <= j;
// pe[pair] = the pair's share of 1/2 sum over ordered pairs.
__global__ __launch_bounds__(256) void k_pair_tab(int natoms, const double *__restrict__ xyz,
                                                  double Z, double rb,
                                                  const double *__restrict__ atab, int n,
                                                  double dr, const double *__restrict__ gl,
                                                  int nmu, double *__restrict__ pe) {
  __shared__ double red[256];
  int64_t p = blockIdx.x;
  int i = 0;
  while (p >= natoms - i) {
    p -= natoms - i;
    ++i;
  }
  const int j = i + (int)p;
  const double dx = xyz[3 * i] - xyz[3 * j], dy = xyz[3 * i + 1] - xyz[3 * j + 1],
               dz = xyz[3 * i + 2] - xyz[3 * j + 2];
  const double R = sqrt(dx * dx + dy * dy + dz * dz);
  const double bnorm = -Z / (pow(M_PI, 1.5) * rb * rb * rb);
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    const double r = k * dr;
    const double w = (k == 0 || k == n - 1) ? 0.5 * dr : dr;
    const double nr = atab[k] + bnorm * exp(-(r / rb) * (r / rb));
    double inner = 0.0;
    for (int m = 0; m < nmu; ++m) {
      const double d = sqrt(fmax(r * r + R * R - 2.0 * r * R * gl[m], 0.0));
      double v, dv;
      hermite_fn(atab + 2 * n, atab + 3 * n, n, dr, d, v, dv);
      inner += gl[nmu + m] * v;
    }
    acc += w * r * r * nr * inner;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) pe[blockIdx.x] = (i == j ? 0.5 : 1.0) * 2.0 * M_PI * red[0];
}

// out[0] += sum of the n values in index order (one work-group)
__global__ __launch_bounds__(256) void k_sum_fixed(int64_t n, const double *__restrict__ v,
                                                   double *__restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) acc += v[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += red[0];
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on the
// Legendre recurrence): x[0..n), w[0..n)
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      const double z1 = z;
      z = z1 - p1 / pp;
      if (fabs(z - z1) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

// <g_a, g_b>(R) for unit Gaussians with exponents a, b
__device__ inline double gauss_coulomb(double R, double a, double b) {
  const double mu = sqrt(a * b / (a + b));
  return erf_over_r(R, 1.0 / mu);
}

// 1/2 sum_IJ <n_I, n_J> - E_self + dE_ZZ (one thread per ordered pair);
// gauss_pairs = false leaves the <n_I, n_J> terms to k_pair_tab
__global__ void k_const_energy(int natoms, const double *__restrict__ xyz,
                               const double *__restrict__ Z, double a_rho, double rb,
                               bool gauss_pairs, double *__restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)natoms * natoms) return;
  const int i = t / natoms, j = t % natoms;
  const double dx = xyz[3 * i] - xyz[3 * j], dy = xyz[3 * i + 1] - xyz[3 * j + 1],
               dz = xyz[3 * i + 2] - xyz[3 * j + 2];
  const double R = sqrt(dx * dx + dy * dy + dz * dz);
  const double ab = 1.0 / (rb * rb);
  double e = gauss_pairs ? 0.5 * Z[i] * Z[j] *
                               (gauss_coulomb(R, a_rho, a_rho) - 2.0 * gauss_coulomb(R, a_rho, ab) +
                                gauss_coulomb(R, ab, ab))
                         : 0.0;
  if (i == j) e -= Z[i] * Z[i] / (sqrt(2.0 * M_PI) * rb);
  if (i < j) e += Z[i] * Z[j] * erfc(R / (sqrt(2.0) * rb)) / R;
  atomicAdd(out, e);
}

// diagonal of the assembled stiffness (1 on boundary nodes)
__global__ void k_kdiag(int64_t n_cells, int nloc, const int32_t *__restrict__ c2g,
                        const double *__restrict__ K, double *__restrict__ d) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n_cells * nloc) return;
  const int l = idx % nloc;
  atomicAdd(&d[c2g[idx]], K[(int64_t)l * nloc + l]);
}

__global__ void k_kdiag_fix(int64_t n, const double *__restrict__ minv, double *__restrict__ d) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && minv[i] == 0.0) d[i] = 1.0;
}

// f_j += 4 pi sum_q W fq N_l on interior nodes (one block per cell)
__global__ __launch_bounds__(256) void k_load_vector(int nloc, int nqp, const int32_t *__restrict__ c2g,
                                                     const double *__restrict__ N3,
                                                     const double *__restrict__ W3,
                                                     const double *__restrict__ fq,
                                                     const double *__restrict__ sub,
                                                     const double *__restrict__ minv,
                                                     double scale, double *__restrict__ out) {
  __shared__ double wf[EFE_MAXQ * EFE_MAXQ * EFE_MAXQ];
  const int64_t cell = blockIdx.x;
  for (int q = threadIdx.x; q < nqp; q += blockDim.x)
    wf[q] = W3[q] * (fq[cell * nqp + q] - (sub ? sub[cell * nqp + q] : 0.0));
  __syncthreads();
  for (int l = threadIdx.x; l < nloc; l += blockDim.x) {
    const int32_t node = c2g[cell * nloc + l];
    if (minv[node] == 0.0) continue;
    double acc = 0.0;
    for (int q = 0; q < nqp; ++q) acc += wf[q] * N3[(int64_t)q * nloc + l];
    atomicAdd(&out[node], scale * acc);
  }
}

typedef double v4d_s __attribute__((ext_vector_type(4)));

// Cell stiffness in the operand layout of v_mfma_f64_16x16x4:
// Kt[rb][ks][lane] = K[16 rb + lane%16][4 ks + lane/16] (zero past nloc)
__global__ void k_tile_K(int nloc, int RB, int KS, const double *__restrict__ K,
                         double *__restrict__ Kt) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)RB * KS * 64) return;
  const int l = (int)(idx % 64);
  const int ks = (int)((idx / 64) % KS), rb = (int)(idx / (64 * (int64_t)KS));
  const int row = 16 * rb + l % 16, col = 4 * ks + l / 16;
  Kt[idx] = (row < nloc && col < nloc) ? K[(int64_t)row * nloc + col] : 0.0;
}

// K x_c for every cell in one launch, on FP64 MFMA: a work-group takes 16
// cells, whose gathered x form the 16 columns of the B operand (in LDS,
// zero on boundary nodes and past nloc), and four row blocks of the shared
// cell stiffness (A operand, MFMA layout), one per wave; the products are
// written cell by cell and summed into the nodes by k_stiff_gather.
constexpr int STIFF_CELLS = 16;
__global__ __launch_bounds__(256) void k_stiff_apply_all(int64_t ncells, int nloc, int RB, int KS,
                                                         const int32_t *__restrict__ c2g,
                                                         const double *__restrict__ Kt,
                                                         const double *__restrict__ x,
                                                         const double *__restrict__ minv,
                                                         double *__restrict__ ycell,
                                                         const double *__restrict__ done) {
  extern __shared__ double xs[];   // [STIFF_CELLS][4 KS + 1]
  if (done && *done != 0.0) return;
  const int KP1 = 4 * KS + 1;      // odd row stride: the 16 cells hit different banks
  const int64_t c0 = (int64_t)blockIdx.x * STIFF_CELLS;
  const int ncb = (int)min<int64_t>(STIFF_CELLS, ncells - c0);
  for (int i = threadIdx.x; i < STIFF_CELLS * KP1; i += blockDim.x) {
    const int cc = i / KP1, l = i % KP1;
    double v = 0.0;
    if (cc < ncb && l < nloc) {
      const int32_t node = c2g[(c0 + cc) * nloc + l];
      if (minv[node] != 0.0) v = x[node];
    }
    xs[i] = v;
  }
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, li = lane % 16, lk = lane / 16;
  // one row block per wave; the work-groups of blockIdx.y share the gather
  const int rb = 4 * blockIdx.y + wave;
  if (rb < RB) {
    // four accumulators (k step mod 4) quarter the dependent MFMA chain; the
    // A fragments of eight k steps are loaded ahead of their MFMAs
    v4d_s acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
    const double *kt = Kt + (int64_t)rb * KS * 64 + lane;
    const double *xb = xs + li * KP1 + lk;
    int ks = 0;
    for (; ks + 7 < KS; ks += 8) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = kt[(int64_t)(ks + u) * 64];
#pragma unroll
      for (int u = 0; u < 8; u += 4) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], xb[4 * (ks + u)], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u + 1], xb[4 * (ks + u + 1)], acc1, 0, 0, 0);
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u + 2], xb[4 * (ks + u + 2)], acc2, 0, 0, 0);
        acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u + 3], xb[4 * (ks + u + 3)], acc3, 0, 0, 0);
      }
    }
    for (; ks < KS; ++ks)
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(kt[(int64_t)ks * 64], xb[4 * ks], acc0, 0, 0, 0);
    const v4d_s acc = (acc0 + acc1) + (acc2 + acc3);
    // accumulator v of lane l: local row 16 rb + 4 v + l/16 of cell l%16
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * rb + 4 * v + lk;
      if (li < ncb && row < nloc) ycell[(c0 + li) * nloc + row] = acc[v];
    }
  }
}

// y[node] = sum of ycell over the (up to 8) cells holding the node, in a
// fixed order (no atomics); zero on boundary nodes.  Node (i, j, k) lies in
// cells i/p - 1 and i/p along x when i is a multiple of p (inside the mesh),
// else in cell i/p only; likewise along y and z.  With part, the work-group
// also leaves its partial sum of x.y there (the p.Ap of CG).
struct GridDims {
  int64_t n1x, n1y, n1z;
  int ncx, ncy, ncz, p, P, nloc;
};
__global__ __launch_bounds__(256) void k_stiff_gather(GridDims d, const double *__restrict__ ycell,
                                                      const double *__restrict__ minv,
                                                      const double *__restrict__ x,
                                                      double *__restrict__ y,
                                                      double *__restrict__ part,
                                                      const double *__restrict__ done,
                                                      double shift,
                                                      const double *__restrict__ m) {
  __shared__ double red[256];
  if (done && *done != 0.0) return;
  const int64_t n = d.n1x * d.n1y * d.n1z;
  double acc = 0.0;
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < n;
       node += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    if (minv[node] != 0.0) {
      const int64_t gi = node % d.n1x, gj = (node / d.n1x) % d.n1y, gk = node / (d.n1x * d.n1y);
      int cs[3][2], ls[3][2], nc[3];
      const int64_t g3[3] = {gi, gj, gk};
      const int ncl[3] = {d.ncx, d.ncy, d.ncz};
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int cc = (int)(g3[t] / d.p), a = (int)(g3[t] % d.p);
        nc[t] = 0;
        if (a == 0 && cc > 0) {
          cs[t][nc[t]] = cc - 1;
          ls[t][nc[t]++] = d.p;
        }
        if (cc < ncl[t]) {
          cs[t][nc[t]] = cc;
          ls[t][nc[t]++] = a;
        }
      }
      for (int z = 0; z < nc[2]; ++z)
        for (int yy = 0; yy < nc[1]; ++yy)
          for (int xx = 0; xx < nc[0]; ++xx) {
            const int64_t cell = cs[0][xx] + (int64_t)d.ncx * (cs[1][yy] + (int64_t)d.ncy * cs[2][z]);
            const int l = ls[0][xx] + d.P * (ls[1][yy] + d.P * ls[2][z]);
            v += ycell[cell * d.nloc + l];
          }
      if (shift != 0.0) v += shift * m[node] * x[node];
    }
    y[node] = v;
    if (part) acc += x[node] * v;
  }
  if (part) {
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
  }
}

// nodal field -> Gauss points (one block per cell)
__global__ __launch_bounds__(256) void k_nodes_to_quad(int nloc, int nqp, const int32_t *__restrict__ c2g,
                                                       const double *__restrict__ N3,
                                                       const double *__restrict__ x,
                                                       const double *__restrict__ minv,
                                                       double *__restrict__ xq) {
  __shared__ double xs[EFE_MAXLOC];
  const int64_t cell = blockIdx.x;
  for (int l = threadIdx.x; l < nloc; l += blockDim.x) {
    const int32_t node = c2g[cell * nloc + l];
    xs[l] = minv[node] == 0.0 ? 0.0 : x[node];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nqp; q += blockDim.x) {
    const double *nr = N3 + (int64_t)q * nloc;
    double acc = 0.0;
    for (int l = 0; l < nloc; ++l) acc += nr[l] * xs[l];
    xq[cell * nqp + q] = acc;
  }
}

// v_in = phi_at + phi_rem(q) + v_short + v_xc(rho_in)
__global__ void k_veff(int64_t n, const double *__restrict__ rho, const double *__restrict__ phi_at,
                       const double *__restrict__ phiq, const double *__restrict__ vs,
                       double *__restrict__ v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double exc, vxc;
  lda_pw92(rho[i], exc, vxc);
  v[i] = phi_at[i] + phiq[i] + vs[i] + vxc;
}

// Fermi level by bisection: 2 sum f = Ne; writes mu, f, band, TS.  One
// work-group of 256 threads; every bisection step sums over the eigenvalues
// in a fixed tree order, so the result does not depend on timing.
__device__ __forceinline__ void fermi_reduce3(double *a, double *b, double *cc, double x, double y,
                                              double z) {
  const int t = threadIdx.x;
  a[t] = x;
  b[t] = y;
  cc[t] = z;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      a[t] += a[t + s];
      b[t] += b[t + s];
      cc[t] += cc[t + s];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_fermi(int N, const double *__restrict__ lam, double ne,
                                               double kT, double *__restrict__ f,
                                               double *__restrict__ out) {
  __shared__ double ra[256], rb[256], rc[256];
  const int t = threadIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  for (int i = t; i < N; i += 256) {
    lo = fmin(lo, lam[i]);
    hi = fmax(hi, lam[i]);
  }
  ra[t] = lo;
  rb[t] = hi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      ra[t] = fmin(ra[t], ra[t + s]);
      rb[t] = fmax(rb[t], rb[t + s]);
    }
    __syncthreads();
  }
  lo = ra[0] - (50.0 * kT + 1.0);
  hi = rb[0] + (50.0 * kT + 1.0);
  __syncthreads();
  // 2 sum f - N_e as the integer 2 #{lam <= mu} - N_e plus the Fermi tails
  // (f above mu, 1 - f below, each without cancellation), so that the sign
  // stays resolved inside a gap much wider than kT
  for (int it = 0; it < 200; ++it) {
    const double mu = 0.5 * (lo + hi);
    double up = 0.0, down = 0.0, nbelow = 0.0;
    for (int i = t; i < N; i += 256) {
      const double x = (lam[i] - mu) / kT;
      if (x <= 0.0) {
        nbelow += 1.0;
        down += 1.0 / (1.0 + exp(-x));
      } else {
        up += 1.0 / (1.0 + exp(x));
      }
    }
    fermi_reduce3(ra, rb, rc, up, down, nbelow);
    const double excess = (2.0 * rc[0] - ne) + 2.0 * (ra[0] - rb[0]);
    if (excess < 0.0) lo = mu;
    else hi = mu;
    __syncthreads();
  }
  const double mu = 0.5 * (lo + hi);
  double band = 0.0, ts = 0.0;
  for (int i = t; i < N; i += 256) {
    const double x = (lam[i] - mu) / kT;
    const double fi = x > 0 ? exp(-x) / (1.0 + exp(-x)) : 1.0 / (1.0 + exp(x));
    f[i] = fi;
    band += 2.0 * fi * lam[i];
    if (fi > 0.0 && fi < 1.0) ts += fi * log(fi) + (1.0 - fi) * log(1.0 - fi);
  }
  fermi_reduce3(ra, rb, rc, band, ts, 0.0);
  if (t == 0) {
    out[0] = mu;
    out[1] = ra[0];
    out[2] = -2.0 * kT * rb[0];
  }
}

// rho(q) = 2 sum_j f_j psi_j(q)^2, psi = N3 Xh_cell + sum_I phi_I(q) V^E_I
// (one block per cell; columns in chunks of 16, only the listed columns)
__global__ __launch_bounds__(256) void k_density(MeshGeo g, EnrParam e, const double *__restrict__ xq1,
                                                 const int32_t *__restrict__ c2g,
                                                 const double *__restrict__ N3,
                                                 const double *__restrict__ Xh, int64_t ldh,
                                                 const double *__restrict__ VE, int64_t lde,
                                                 const int32_t *__restrict__ cols, int ncols_occ,
                                                 const double *__restrict__ f,
                                                 const int32_t *__restrict__ cell_ptr,
                                                 const int32_t *__restrict__ cell_atom,
                                                 const double *__restrict__ xyz,
                                                 const double *__restrict__ nu,
                                                 double *__restrict__ rho, int accumulate) {
  __shared__ double xs[EFE_MAXLOC][16];
  __shared__ double ve[16][16 * 9];      // up to 16 atoms of the cell at a time
  const int64_t cell = blockIdx.x;
  const int nloc = g.nloc, nqp = g.nqp, nf = e.nf;
  const int a0 = cell_ptr[cell], a1 = cell_ptr[cell + 1];
  double racc[2] = {0.0, 0.0};
  for (int c0 = 0; c0 < ncols_occ; c0 += 16) {
    const int nc = min(16, ncols_occ - c0);
    for (int idx = threadIdx.x; idx < nloc * 16; idx += blockDim.x) {
      const int l = idx / 16, j = idx % 16;
      xs[l][j] = j < nc ? Xh[(int64_t)c2g[cell * nloc + l] * ldh + cols[c0 + j]] : 0.0;
    }
    __syncthreads();
    for (int r = 0; r < 2; ++r) {
      const int q = threadIdx.x + 256 * r;
      double psi[16];
      for (int j = 0; j < 16; ++j) psi[j] = 0.0;
      if (q < nqp) {
        const double *nr = N3 + (int64_t)q * nloc;
        for (int l = 0; l < nloc; ++l) {
          const double n = nr[l];
          for (int j = 0; j < 16; ++j) psi[j] += n * xs[l][j];
        }
      }
      // enrichment part, atoms of this cell in groups of 16
      for (int ab = a0; ab < a1; ab += 16) {
        const int na = min(16, a1 - ab);
        __syncthreads();
        for (int idx = threadIdx.x; idx < na * nf * 16; idx += blockDim.x) {
          const int ia = idx / (nf * 16), k = (idx / 16) % nf, j = idx % 16;
          const int I = cell_atom[ab + ia];
          ve[j][ia * nf + k] =
              j < nc ? nu[I * nf + k] * VE[(int64_t)(I * nf + k) * lde + cols[c0 + j]] : 0.0;
        }
        __syncthreads();
        if (q < nqp) {
          double x[3], phi[9];
          quad_point(g, xq1, (int)cell, q, x);
          for (int ia = 0; ia < na; ++ia) {
            const int I = cell_atom[ab + ia];
            enr_eval(e, x[0] - xyz[3 * I], x[1] - xyz[3 * I + 1], x[2] - xyz[3 * I + 2], phi,
                     nullptr);
            for (int k = 0; k < nf; ++k)
              for (int j = 0; j < 16; ++j) psi[j] += phi[k] * ve[j][ia * nf + k];
          }
        }
      }
      if (q < nqp)
        for (int j = 0; j < nc; ++j) racc[r] += 2.0 * f[cols[c0 + j]] * psi[j] * psi[j];
    }
    __syncthreads();
  }
  for (int r = 0; r < 2; ++r) {
    const int q = threadIdx.x + 256 * r;
    if (q < nqp) rho[cell * nqp + q] = (accumulate ? rho[cell * nqp + q] : 0.0) + racc[r];
  }
}

// energy integrals over the Gauss points:
// out[0] int rho v_in, [1] int rho eps_xc, [2] int Drho phi_at, [3] int Drho phiq,
// [4] int rho v_short, [5] int rho, [6] int (rho - rho_in)^2
__global__ void k_energy_sums(int64_t nq_tot, int nqp, const double *__restrict__ W3,
                              const double *__restrict__ rho, const double *__restrict__ v_in,
                              const double *__restrict__ rho_at, const double *__restrict__ phi_at,
                              const double *__restrict__ phiq, const double *__restrict__ vs,
                              const double *__restrict__ rho_in, double *__restrict__ out) {
  __shared__ double red[7][256];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nq_tot;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double w = W3[i % nqp], r = rho[i], dr = r - rho_at[i];
    double exc, vxc;
    lda_pw92(r, exc, vxc);
    const double d = r - rho_in[i];
    acc[0] += w * r * v_in[i];
    acc[1] += w * r * exc;
    acc[2] += w * dr * phi_at[i];
    acc[3] += w * dr * phiq[i];
    acc[4] += w * r * vs[i];
    acc[5] += w * r;
    acc[6] += w * d * d;
  }
  for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 7; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 7) atomicAdd(&out[threadIdx.x], red[threadIdx.x][0]);
}

// weighted dot of two vectors over the Gauss points: out += sum W a b
__global__ void k_wdot(int64_t n, int nqp, const double *__restrict__ W3,
                       const double *__restrict__ a, const double *__restrict__ b,
                       double *__restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += (W3 ? W3[i % nqp] : 1.0) * a[i] * b[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

// y = a x + b y (vectors)
__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b,
                        double *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

// z = r / d
__global__ void k_precond(int64_t n, const double *__restrict__ r, const double *__restrict__ d,
                          const double *__restrict__ minv, double *__restrict__ z) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) z[i] = minv[i] == 0.0 ? 0.0 : r[i] / d[i];
}

__global__ void k_sub(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                      double *__restrict__ c) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) c[i] = a[i] - b[i];
}

// ---- Poisson CG with its scalars on the device.  sc[0] r.z, sc[1] p.Ap,
// sc[2] r.r, sc[3] new r.z, sc[4] done flag, sc[5] iterations, sc[6] the
// squared stopping threshold, sc[7] beta.  Every kernel of an iteration
// returns at once when the flag is set, so the host can queue iterations in
// batches and still stop after the same iteration as a loop that tests r.r
// each time.  The reductions go through CG_NB per-work-group partial sums
// that are added in a fixed order (no atomics: the result does not depend
// on timing).
constexpr int CG_NB = 1024;

__device__ inline double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// sum of part[0 .. CG_NB) by one work-group of 256 threads, fixed order
__device__ inline double sum_parts(const double *__restrict__ part, double *red) {
  double a = 0.0;
  for (int i = threadIdx.x; i < CG_NB; i += 256) a += part[i];
  const double t = block_sum(a, red);
  __syncthreads();
  return t;
}

// alpha = r.z / p.Ap (every work-group adds the p.Ap partials itself, in the
// same order); phi += alpha p, r -= alpha Ap, z = r / diag (interior);
// partial sums of r.r and r.z
__global__ __launch_bounds__(256) void k_cg_update(int64_t n, const double *__restrict__ p,
                                                   const double *__restrict__ Ap,
                                                   const double *__restrict__ d,
                                                   const double *__restrict__ minv,
                                                   double *__restrict__ phi, double *__restrict__ r,
                                                   double *__restrict__ z, double *__restrict__ part,
                                                   const double *__restrict__ sc) {
  __shared__ double red[256];
  if (sc[4] != 0.0) return;
  const double alpha = sc[0] / sum_parts(part, red);
  double rr = 0.0, rz = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    phi[i] += alpha * p[i];
    const double ri = r[i] - alpha * Ap[i];
    r[i] = ri;
    const double zi = minv[i] == 0.0 ? 0.0 : ri / d[i];
    z[i] = zi;
    rr += ri * ri;
    rz += ri * zi;
  }
  const double t1 = block_sum(rr, red);
  __syncthreads();
  const double t2 = block_sum(rz, red);
  if (threadIdx.x == 0) {
    part[CG_NB + blockIdx.x] = t1;
    part[2 * CG_NB + blockIdx.x] = t2;
  }
}

// end of an iteration: r.r and the new r.z from their partials, the
// iteration count, the stopping test, beta, and r.z for the next iteration
__global__ __launch_bounds__(256) void k_cg_next(const double *__restrict__ part,
                                                 double *__restrict__ sc) {
  __shared__ double red[256];
  if (sc[4] != 0.0) return;
  const double rr = sum_parts(part + CG_NB, red);
  const double rz = sum_parts(part + 2 * CG_NB, red);
  if (threadIdx.x == 0) {
    sc[2] = rr;
    sc[3] = rz;
    sc[5] += 1.0;
    if (rr <= sc[6]) sc[4] = 1.0;
    sc[7] = rz / sc[0];
    sc[0] = rz;
  }
}

// p = z + beta p
__global__ void k_cg_pupdate(int64_t n, const double *__restrict__ z, double *__restrict__ p,
                             const double *__restrict__ sc) {
  if (sc[4] != 0.0) return;
  const double beta = sc[7];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + beta * p[i];
}

// slot j <- slot j + 1 for j < m, element by element (each thread reads a
// slot before it overwrites it, so the overlapping shift is safe)
__global__ void k_shift_history(int64_t n, int m, double *__restrict__ H) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = 0; j < m; ++j) H[(int64_t)j * n + i] = H[(int64_t)(j + 1) * n + i];
}

// Solve A g = r for the symmetric k x k matrix whose lower triangle is given
// (Gaussian elimination with partial pivoting).
__global__ void k_small_solve(int k, double *__restrict__ A, double *__restrict__ r,
                              double *__restrict__ g) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j) A[i * k + j] = A[j * k + i];
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int i = c + 1; i < k; ++i)
      if (fabs(A[i * k + c]) > fabs(A[piv * k + c])) piv = i;
    if (piv != c) {
      for (int j = 0; j < k; ++j) {
        double t = A[c * k + j];
        A[c * k + j] = A[piv * k + j];
        A[piv * k + j] = t;
      }
      double t = r[c];
      r[c] = r[piv];
      r[piv] = t;
    }
    const double d = A[c * k + c];
    for (int i = c + 1; i < k; ++i) {
      const double fct = d != 0.0 ? A[i * k + c] / d : 0.0;
      for (int j = c; j < k; ++j) A[i * k + j] -= fct * A[c * k + j];
      r[i] -= fct * r[c];
    }
  }
  for (int i = k - 1; i >= 0; --i) {
    double s = r[i];
    for (int j = i + 1; j < k; ++j) s -= A[i * k + j] * g[j];
    g[i] = A[i * k + i] != 0.0 ? s / A[i * k + i] : 0.0;
  }
}

// Anderson update: x_bar = X_k - sum g_i (X_{i+1} - X_i),
// F_bar = F_k - sum g_i (F_{i+1} - F_i); out = x_bar + beta F_bar, or, with
// Fb, out = x_bar and Fb = F_bar (to be preconditioned first)
__global__ void k_anderson_update(int64_t n, int k, const double *__restrict__ X,
                                  const double *__restrict__ F, int64_t stride,
                                  const double *__restrict__ g, double beta,
                                  double *__restrict__ out, double *__restrict__ Fb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = X[(int64_t)k * stride + i], fk = F[(int64_t)k * stride + i];
  for (int j = 0; j < k; ++j) {
    const double dx = X[(int64_t)(j + 1) * stride + i] - X[(int64_t)j * stride + i];
    const double df = F[(int64_t)(j + 1) * stride + i] - F[(int64_t)j * stride + i];
    x -= g[j] * dx;
    fk -= g[j] * df;
  }
  if (Fb) {
    out[i] = x;
    Fb[i] = fk;
  } else {
    out[i] = x + beta * fk;
  }
}

// y += a x
__global__ void k_axpy(int64_t n, double a, const double *__restrict__ x, double *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// ------------------------------------------------------------------ host
static efe_status scf_init(efe_ctx *c) {
  ScfState &s = S(c);
  if (s.init) return EFE_OK;
  efe_status st;
  const int64_t nq = c->n_qpts, nn = c->n_nodes;
  double **qs[] = {&s.rho_at, &s.phi_at, &s.v_short, &s.rho_in, &s.rho_out, &s.v_in, &s.phiq,
                   &s.uq_k};
  for (auto pp : qs)
    if ((st = efe_alloc(c, (void **)pp, nq * 8))) return st;
  double **ns[] = {&s.phi_rem, &s.phi_out, &s.Kdiag, &s.kdiag_k, &s.u_k};
  for (auto pp : ns)
    if ((st = efe_alloc(c, (void **)pp, nn * 8))) return st;
  if ((st = efe_alloc(c, (void **)&s.cg, 5 * nn * 8))) return st;
  if ((st = efe_alloc(c, (void **)&s.scal, 256 * 8))) return st;
  if ((st = efe_alloc(c, (void **)&s.part, 3 * CG_NB * 8))) return st;
  if ((st = efe_alloc(c, (void **)&s.ycell, (size_t)c->n_cells * c->nloc * 8))) return st;
  const int64_t kt = (int64_t)c->RB * c->KS * 64;
  if ((st = efe_alloc(c, (void **)&s.Ktile, kt * 8))) return st;
  k_tile_K<<<cdiv(kt, 256), 256, 0, c->stream>>>(c->nloc, c->RB, c->KS, c->d_K, s.Ktile);
  HIPCHK(c, hipMemsetAsync(s.phi_rem, 0, nn * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(s.Kdiag, 0, nn * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(s.scal, 0, 256 * 8, c->stream));
  const MeshGeo g = mesh_geo(c);
  const bool atab = c->natab > 0;
  k_atomic_fields<<<cdiv(nq, 256), 256, 0, c->stream>>>(
      g, c->d_xq1, c->natoms, c->d_xyz, c->d_Zs, c->rho_alpha, c->loc_rc, c->loc_amp, c->loc_rg,
      atab ? c->d_atom_tab : nullptr, c->natab, c->atab_dr, s.rho_at, s.phi_at, s.v_short);
  std::vector<double> glh;
  double *dgl = nullptr, *dpe = nullptr;
  if (c->natoms)
    k_const_energy<<<cdiv((int64_t)c->natoms * c->natoms, 256), 256, 0, c->stream>>>(
        c->natoms, c->d_xyz, c->d_Zs, c->rho_alpha, c->loc_rc, !atab, s.scal);
  if (c->natoms && atab) {
    // pair energies of the tabulated atoms, summed in pair order
    constexpr int NMU = 64;
    std::vector<double> gx, gw;
    gauss_legendre(NMU, gx, gw);
    glh = gx;
    glh.insert(glh.end(), gw.begin(), gw.end());
    const int64_t npr = (int64_t)c->natoms * (c->natoms + 1) / 2;
    if ((st = efe_ws(c, 35, (size_t)(2 * NMU + npr) * 8, (void **)&dgl))) return st;
    dpe = dgl + 2 * NMU;
    HIPCHK(c, hipMemcpyAsync(dgl, glh.data(), 2 * NMU * 8, hipMemcpyHostToDevice, c->stream));
    k_pair_tab<<<(unsigned)npr, 256, 0, c->stream>>>(c->natoms, c->d_xyz, c->Z[0], c->loc_rc,
                                                    c->d_atom_tab, c->natab, c->atab_dr, dgl, NMU,
                                                    dpe);
    k_sum_fixed<<<1, 256, 0, c->stream>>>(npr, dpe, s.scal);
  }
  k_kdiag<<<cdiv(c->n_cells * c->nloc, 256), 256, 0, c->stream>>>(c->n_cells, c->nloc, c->d_c2g,
                                                                   c->d_K, s.Kdiag);
  k_kdiag_fix<<<cdiv(nn, 256), 256, 0, c->stream>>>(nn, c->d_minv, s.Kdiag);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(&s.e_const, s.scal, 8, hipMemcpyDeviceToHost, c->stream));
  // cell -> atoms whose enrichment support holds the cell
  std::vector<int32_t> ptr(c->n_cells + 1, 0), lst;
  {
    std::vector<std::vector<int32_t>> per(c->n_cells);
    for (int I = 0; I < c->natoms; ++I)
      for (int32_t q = c->enr_ptr[I]; q < c->enr_ptr[I + 1]; ++q) per[c->enr_cells[q]].push_back(I);
    for (int64_t cc = 0; cc < c->n_cells; ++cc) {
      ptr[cc + 1] = ptr[cc] + (int32_t)per[cc].size();
      lst.insert(lst.end(), per[cc].begin(), per[cc].end());
    }
  }
  if ((st = efe_alloc(c, (void **)&s.cell_ptr, ptr.size() * 4))) return st;
  if ((st = efe_alloc(c, (void **)&s.cell_atom, std::max<size_t>(lst.size(), 1) * 4))) return st;
  HIPCHK(c, hipMemcpyAsync(s.cell_ptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice, c->stream));
  if (!lst.empty())
    HIPCHK(c, hipMemcpyAsync(s.cell_atom, lst.data(), lst.size() * 4, hipMemcpyHostToDevice,
                             c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // initial density: superposition of atomic densities
  HIPCHK(c, hipMemcpyAsync(s.rho_in, s.rho_at, nq * 8, hipMemcpyDeviceToDevice, c->stream));
  s.init = true;
  return EFE_OK;
}

// y = (K + shift diag(m)) x on interior nodes (sc: CG scalars whose done
// flag turns the launches into no-ops; part: also the per-work-group
// partials of x.y)
static efe_status stiff_apply(efe_ctx *c, const double *x, double *y, const double *sc = nullptr,
                              double *part = nullptr, double shift = 0.0) {
  ScfState &s = S(c);
  const size_t shm = (size_t)STIFF_CELLS * (4 * c->KS + 1) * 8;
  const dim3 grid((unsigned)cdiv(c->n_cells, STIFF_CELLS), (unsigned)cdiv(c->RB, 4));
  k_stiff_apply_all<<<grid, 256, shm, c->stream>>>(c->n_cells, c->nloc, c->RB, c->KS, c->d_c2g,
                                                   s.Ktile, x, c->d_minv, s.ycell,
                                                   sc ? sc + 4 : nullptr);
  const GridDims d{c->n1[0], c->n1[1], c->n1[2], c->ncell[0], c->ncell[1], c->ncell[2],
                   c->p,     c->P,     c->nloc};
  k_stiff_gather<<<CG_NB, 256, 0, c->stream>>>(d, s.ycell, c->d_minv, x, y, part,
                                               sc ? sc + 4 : nullptr, shift, c->d_m_int);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

static efe_status dot_host(efe_ctx *c, int64_t n, const double *a, const double *b, double *res) {
  ScfState &s = S(c);
  double *slot = s.scal + 64;
  HIPCHK(c, hipMemsetAsync(slot, 0, 8, c->stream));
  k_wdot<<<(unsigned)std::min<int64_t>(cdiv(n, 256), 1024), 256, 0, c->stream>>>(n, 1, nullptr, a,
                                                                                b, slot);
  HIPCHK(c, hipMemcpyAsync(res, slot, 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return EFE_OK;
}

// x (in/out, nodes): (K + shift diag(m)) x = scale int (fq - sub) N on the
// interior nodes, CG with the Jacobi preconditioner diag.  shift = 0,
// scale = 4 pi is the Poisson problem for phi^rem.
static efe_status cg_solve(efe_ctx *c, const double *fq, const double *sub, double scale,
                           double shift, const double *diag, double *phi, double rtol, int maxit,
                           int *iters) {
  ScfState &s = S(c);
  const int64_t nn = c->n_nodes;
  double *r = s.cg, *z = s.cg + nn, *p = s.cg + 2 * nn, *Ap = s.cg + 3 * nn, *b = s.cg + 4 * nn;
  efe_status st;
  const int T = 256;
  HIPCHK(c, hipMemsetAsync(b, 0, nn * 8, c->stream));
  k_load_vector<<<c->n_cells, 256, 0, c->stream>>>(c->nloc, c->nqp, c->d_c2g, c->d_N3, c->d_W3, fq,
                                                   sub, c->d_minv, scale, b);
  if ((st = stiff_apply(c, phi, Ap, nullptr, nullptr, shift))) return st;
  k_sub<<<cdiv(nn, T), T, 0, c->stream>>>(nn, b, Ap, r);
  k_precond<<<cdiv(nn, T), T, 0, c->stream>>>(nn, r, diag, c->d_minv, z);
  HIPCHK(c, hipMemcpyAsync(p, z, nn * 8, hipMemcpyDeviceToDevice, c->stream));
  double rz, bb, rr;
  if ((st = dot_host(c, nn, r, z, &rz))) return st;
  if ((st = dot_host(c, nn, b, b, &bb))) return st;
  if ((st = dot_host(c, nn, r, r, &rr))) return st;
  const double bn = sqrt(bb);
  int it = 0;
  if (bn == 0.0) {   // zero source: zero solution
    HIPCHK(c, hipMemsetAsync(phi, 0, nn * 8, c->stream));
    *iters = 0;
    return EFE_OK;
  }
  // iterations in batches of 16 with the scalars on the device; the loop
  // stops after the first iteration that meets sqrt(r.r) <= rtol |b|
  double *sc = s.scal + 96;
  const double init[8] = {rz, 0.0, 0.0, 0.0, sqrt(rr) > rtol * bn ? 0.0 : 1.0, 0.0,
                          (rtol * bn) * (rtol * bn), 0.0};   // read by the copy until the sync below
  HIPCHK(c, hipMemcpyAsync(sc, init, sizeof(init), hipMemcpyHostToDevice, c->stream));
  double hs[6] = {0, 0, 0, 0, 0, 0};
  while (it < maxit) {
    const int batch = std::min(16, maxit - it);
    for (int q = 0; q < batch; ++q) {
      if ((st = stiff_apply(c, p, Ap, sc, s.part, shift))) return st;   // Ap and the p.Ap partials
      k_cg_update<<<CG_NB, T, 0, c->stream>>>(nn, p, Ap, diag, c->d_minv, phi, r, z, s.part, sc);
      k_cg_next<<<1, T, 0, c->stream>>>(s.part, sc);
      k_cg_pupdate<<<cdiv(nn, T), T, 0, c->stream>>>(nn, z, p, sc);
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(hs, sc, 6 * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    it = (int)hs[5];
    if (hs[4] != 0.0) break;
  }
  *iters = it;
  if (hs[4] == 0.0) EFE_FAIL(c, EFE_ENOTCONV, "CG did not converge");
  return EFE_OK;
}

// phi (in/out, nodes): K phi = 4 pi int (fq - sub) N (Sec. III.C)
static efe_status poisson(efe_ctx *c, const double *fq, const double *sub, double *phi, double rtol,
                          int maxit, int *iters) {
  ScfState &s = S(c);
  return cg_solve(c, fq, sub, 4.0 * M_PI, 0.0, s.Kdiag, phi, rtol, maxit, iters);
}

// d = Kdiag + shift m on interior nodes (1 on the boundary)
__global__ void k_shift_diag(int64_t n, const double *__restrict__ kd, const double *__restrict__ m,
                             const double *__restrict__ minv, double shift,
                             double *__restrict__ d) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  d[i] = minv[i] == 0.0 ? 1.0 : kd[i] + shift * m[i];
}

// Kerker preconditioner of the mixing (a reading beyond the paper, which
// names Anderson mixing only): F <- F - u at the Gauss points, with u the CFE
// solution of (K + k0^2 diag(m)) u = k0^2 int F N.  In Fourier terms this
// multiplies F by q^2 / (q^2 + k0^2): long-wavelength charge sloshing is
// damped, short-wavelength components pass.
static efe_status kerker(efe_ctx *c, double k0, double *Fq, double rtol, int maxit, int *iters) {
  ScfState &s = S(c);
  efe_status st;
  const int64_t nn = c->n_nodes, nq = c->n_qpts;
  const double sh = k0 * k0;
  if (s.kerker_k0 != k0) {
    k_shift_diag<<<cdiv(nn, 256), 256, 0, c->stream>>>(nn, s.Kdiag, c->d_m_int, c->d_minv, sh,
                                                       s.kdiag_k);
    s.kerker_k0 = k0;
  }
  HIPCHK(c, hipMemsetAsync(s.u_k, 0, nn * 8, c->stream));
  if ((st = cg_solve(c, Fq, nullptr, sh, sh, s.kdiag_k, s.u_k, rtol, maxit, iters))) return st;
  k_nodes_to_quad<<<c->n_cells, 256, 0, c->stream>>>(c->nloc, c->nqp, c->d_c2g, c->d_N3, s.u_k,
                                                     c->d_minv, s.uq_k);
  k_sub<<<cdiv(nq, 256), 256, 0, c->stream>>>(nq, Fq, s.uq_k, Fq);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

static double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

extern "C" efe_status efe_set_density(efe_ctx *c, const double *rho) {
  if (!c) return EFE_EINVAL;
  if (!rho) EFE_FAIL(c, EFE_EINVAL, "null density");
  efe_status st;
  if ((st = scf_init(c))) return st;
  ScfState &s = S(c);
  HIPCHK(c, hipMemcpyAsync(s.rho_in, rho, c->n_qpts * 8, hipMemcpyDeviceToDevice, c->stream));
  s.nhist = 0;
  s.have_E = false;
  s.iter = 0;
  return EFE_OK;
}

extern "C" efe_status efe_get_density(efe_ctx *c, int32_t which, double *out) {
  if (!c) return EFE_EINVAL;
  if (!out || which < 0 || which > 2) EFE_FAIL(c, EFE_EINVAL, "bad arguments");
  efe_status st;
  if ((st = scf_init(c))) return st;
  ScfState &s = S(c);
  const double *src = which == 0 ? s.rho_in : which == 1 ? s.rho_out : s.rho_at;
  HIPCHK(c, hipMemcpyAsync(out, src, c->n_qpts * 8, hipMemcpyDeviceToDevice, c->stream));
  return EFE_OK;
}

extern "C" efe_status efe_scf_step(efe_ctx *c, double *V, int32_t N, int64_t ld, double *lambda,
                                   const double *v0, const efe_scf_params *prm,
                                   efe_scf_report *rep) {
  if (!c) return EFE_EINVAL;
  if (!V || !lambda || !v0 || !prm || !rep || N < 1 || ld < N)
    EFE_FAIL(c, EFE_EINVAL, "bad arguments");
  if (prm->degree < 1 || prm->passes < 1 || prm->passes_first < 1 || !(prm->kT > 0) ||
      prm->mix_history < 0 || prm->mix_history > 16 || !(prm->cg_rtol > 0) || prm->cg_maxit < 1 ||
      prm->lanczos_steps < 1 || !(prm->tau == prm->tau) || !(prm->kerker_k0 == prm->kerker_k0))
    EFE_FAIL(c, EFE_EINVAL, "bad SCF parameters");
  if (prm->prec != EFE_FP64 && prm->prec != EFE_FP32 && prm->prec != EFE_BF16)
    EFE_FAIL(c, EFE_EINVAL, "bad filter precision");
  if (prm->prec == EFE_BF16 && c->amplification > EFE_BF16_MAX_AMPLIFICATION)
    EFE_FAIL(c, EFE_EINVAL,
             "BF16 filter refused: enrichment amplification " + std::to_string(c->amplification) +
                 " exceeds " + std::to_string(EFE_BF16_MAX_AMPLIFICATION));
  if (N > 4096) EFE_FAIL(c, EFE_EINVAL, "more than 4096 vectors");
  efe_status st;
  if ((st = scf_init(c))) return st;
  ScfState &s = S(c);
  const int64_t nq = c->n_qpts;
  const int T = 256;
  auto t0 = std::chrono::steady_clock::now();
  double ne = 0.0;
  for (double z : c->Z) ne += z;
  // 1. potential of rho_in
  int cg_it = 0, cg_it2 = 0;
  if ((st = poisson(c, s.rho_in, s.rho_at, s.phi_rem, prm->cg_rtol, prm->cg_maxit, &cg_it)))
    return st;
  k_nodes_to_quad<<<c->n_cells, 256, 0, c->stream>>>(c->nloc, c->nqp, c->d_c2g, c->d_N3, s.phi_rem,
                                                     c->d_minv, s.phiq);
  k_veff<<<cdiv(nq, T), T, 0, c->stream>>>(nq, s.rho_in, s.phi_at, s.phiq, s.v_short, s.v_in);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double t_pois = ms_since(t0);
  auto tb = std::chrono::steady_clock::now();
  if ((st = efe_build_operators(c, s.v_in, prm->prec == EFE_FP64 ? 0 : (1 << prm->prec)))) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double t_ops = ms_since(tb);
  // 2. eigen-solve passes
  tb = std::chrono::steady_clock::now();
  double b;
  if ((st = efe_spectrum_upper_bound(c, v0, prm->lanczos_steps, &b))) return st;
  const double t_bound = ms_since(tb);
  double t_filter = 0.0, t_rr = 0.0;
  double *res;
  if ((st = efe_ws(c, 30, (size_t)N * 8, (void **)&res))) return st;
  if (!s.f && (st = efe_alloc(c, (void **)&s.f, 4096 * 8))) return st;
  double ne_d = ne;
  double *fo = s.scal + 8;   // mu, band, TS
  std::vector<double> fh(N), fermi(3), resh(N);
  // occupations at the current Ritz values and the largest residual among
  // the occupied states (f > 1e-14)
  auto occupied_residual = [&](double *out) -> efe_status {
    k_fermi<<<1, 256, 0, c->stream>>>(N, lambda, ne_d, prm->kT, s.f, fo);
    HIPCHK(c, hipMemcpyAsync(fh.data(), s.f, N * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(fermi.data(), fo, 3 * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(resh.data(), res, N * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double r = 0.0;
    for (int j = 0; j < N; ++j)
      if (fh[j] > 1e-14) r = std::max(r, resh[j]);
    *out = r;
    return EFE_OK;
  };
  if (s.iter == 0) {
    if ((st = efe_rayleigh_ritz(c, V, N, ld, lambda, res))) return st;
  }
  const int npass_min = s.iter == 0 ? prm->passes_first : prm->passes;
  const int npass_max = std::max(npass_min, prm->tau > 0.0 ? prm->max_passes : npass_min);
  std::vector<double> lh(N);
  int npass = 0;
  double max_occ_res = 0.0;
  for (int pss = 0; pss < npass_max; ++pss) {
    HIPCHK(c, hipMemcpyAsync(lh.data(), lambda, N * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    efe_cheb_params cp{prm->degree, lh[N - 1], b, lh[0], EFE_FILTER_RESIDUAL, prm->prec};
    auto ta = std::chrono::steady_clock::now();
    if ((st = efe_cheb_filter(c, V, lambda, N, ld, &cp))) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double tfl = ms_since(ta);
    t_filter += tfl;
    ta = std::chrono::steady_clock::now();
    if ((st = efe_rayleigh_ritz(c, V, N, ld, lambda, res))) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double trr = ms_since(ta);
    t_rr += trr;
    ++npass;
    if ((st = occupied_residual(&max_occ_res))) return st;
    if (prm->progress) prm->progress(pss, tfl, trr, prm->progress_user);
    if (npass >= npass_min && !(prm->tau > 0.0 && max_occ_res > prm->tau)) break;
  }
  auto t2 = std::chrono::steady_clock::now();
  // 3. occupations (from the last pass) and output density
  std::vector<int32_t> cols;
  for (int j = 0; j < N; ++j)
    if (fh[j] > 1e-14) cols.push_back(j);
  // output density, column chunk by column chunk (occupied columns only)
  int32_t *dcols;
  double *Xh;
  if ((st = efe_ws(c, 31, std::max<size_t>(cols.size(), 1) * 4, (void **)&dcols))) return st;
  if ((st = efe_ws(c, 0, (size_t)c->n_nodes * std::min<int32_t>(N, EFE_COL_CHUNK) * 8,
                   (void **)&Xh)))
    return st;
  std::vector<int32_t> rel(cols.size());   // read by async copies until the sync below
  {
    const MeshGeo g = mesh_geo(c);
    const EnrParam e = enr_param(c);
    size_t done = 0;
    bool first = true;
    for (int32_t j0 = 0; j0 < N; j0 += EFE_COL_CHUNK) {
      const int32_t nc = std::min<int32_t>(EFE_COL_CHUNK, N - j0);
      size_t k0 = done;
      while (done < cols.size() && cols[done] < j0 + nc) {
        rel[done] = cols[done] - j0;
        ++done;
      }
      const int nocc = (int)(done - k0);
      if (nocc == 0 && !first) continue;
      if (nocc)
        HIPCHK(c, hipMemcpyAsync(dcols + k0, rel.data() + k0, nocc * 4, hipMemcpyHostToDevice,
                                 c->stream));
      if ((st = efe_transform_cfe(c, V + j0, ld, Xh, nc, nc))) return st;
      k_density<<<c->n_cells, 256, 0, c->stream>>>(g, e, c->d_xq1, c->d_c2g, c->d_N3, Xh, nc,
                                                   V + c->n_nodes * ld + j0, ld, dcols + k0, nocc,
                                                   s.f + j0, s.cell_ptr, s.cell_atom, c->d_xyz,
                                                   c->d_nu, s.rho_out, first ? 0 : 1);
      HIPCHK(c, hipGetLastError());
      first = false;
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double t_dens = ms_since(t2);
  // 4. energies at rho_out
  tb = std::chrono::steady_clock::now();
  HIPCHK(c, hipMemcpyAsync(s.phi_out, s.phi_rem, c->n_nodes * 8, hipMemcpyDeviceToDevice, c->stream));
  if ((st = poisson(c, s.rho_out, s.rho_at, s.phi_out, prm->cg_rtol, prm->cg_maxit, &cg_it2)))
    return st;
  double *phiq_out;
  if ((st = efe_ws(c, 32, nq * 8, (void **)&phiq_out))) return st;
  k_nodes_to_quad<<<c->n_cells, 256, 0, c->stream>>>(c->nloc, c->nqp, c->d_c2g, c->d_N3, s.phi_out,
                                                     c->d_minv, phiq_out);
  double *sums = s.scal + 16;
  HIPCHK(c, hipMemsetAsync(sums, 0, 8 * 8, c->stream));
  k_energy_sums<<<1024, 256, 0, c->stream>>>(nq, c->nqp, c->d_W3, s.rho_out, s.v_in, s.rho_at,
                                             s.phi_at, phiq_out, s.v_short, s.rho_in, sums);
  std::vector<double> sh(7);
  HIPCHK(c, hipMemcpyAsync(sh.data(), sums, 7 * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  rep->t_energy_ms = ms_since(tb);
  const double E_el = s.e_const + sh[2] + 0.5 * sh[3] + sh[4];
  const double E = fermi[1] - sh[0] + sh[1] + E_el;
  rep->E = E;
  rep->F = E - fermi[2];
  rep->E_band = fermi[1];
  rep->E_xc = sh[1];
  rep->E_el = E_el;
  rep->mu = fermi[0];
  rep->n_el = sh[5];
  rep->drho = sqrt(sh[6]);
  rep->dE = s.have_E ? E - s.E_prev : 0.0;
  rep->max_occ_res = max_occ_res;
  rep->iter = s.iter;
  rep->passes = npass;
  rep->cg_iters = cg_it + cg_it2;
  rep->b = b;
  rep->t_poisson_ms = t_pois;
  rep->t_filter_ms = t_filter;
  rep->t_rr_ms = t_rr;
  rep->t_density_ms = t_dens;
  rep->t_operators_ms = t_ops;
  rep->t_bound_ms = t_bound;
  s.E_prev = E;
  s.have_E = true;
  // 5. Anderson mixing of rho_in
  auto t3 = std::chrono::steady_clock::now();
  const int m = prm->mix_history;
  if (!s.hist || s.hist_m != m) {
    if (s.hist) (void)hipFree(s.hist);
    s.hist = nullptr;
    if ((st = efe_alloc(c, (void **)&s.hist, (size_t)2 * (m + 1) * nq * 8))) return st;
    s.hist_m = m;
    s.nhist = 0;
  }
  double *HX = s.hist, *HF = s.hist + (int64_t)(m + 1) * nq;
  if (s.nhist == m + 1) {   // drop the oldest entry (the slots overlap: no memcpy)
    k_shift_history<<<cdiv(nq, T), T, 0, c->stream>>>(nq, m, HX);
    k_shift_history<<<cdiv(nq, T), T, 0, c->stream>>>(nq, m, HF);
    s.nhist = m;
  }
  const int k = s.nhist;
  HIPCHK(c, hipMemcpyAsync(HX + (int64_t)k * nq, s.rho_in, nq * 8, hipMemcpyDeviceToDevice, c->stream));
  k_sub<<<cdiv(nq, T), T, 0, c->stream>>>(nq, s.rho_out, s.rho_in, HF + (int64_t)k * nq);
  s.nhist = k + 1;
  double *gam = s.scal + 32;   // up to 16 coefficients
  double *A, *dfi, *dfj;
  if ((st = efe_ws(c, 33, (size_t)(16 * 16 + 16) * 8, (void **)&A))) return st;
  if ((st = efe_ws(c, 34, (size_t)2 * nq * 8, (void **)&dfi))) return st;
  dfj = dfi + nq;
  if (k > 0) {
    HIPCHK(c, hipMemsetAsync(A, 0, (16 * 16 + 16) * 8, c->stream));
    double *rhs = A + 16 * 16;
    const unsigned nb = (unsigned)std::min<int64_t>(cdiv(nq, 256), 1024);
    for (int i = 0; i < k; ++i) {
      k_sub<<<cdiv(nq, T), T, 0, c->stream>>>(nq, HF + (int64_t)(i + 1) * nq, HF + (int64_t)i * nq, dfi);
      k_wdot<<<nb, 256, 0, c->stream>>>(nq, c->nqp, c->d_W3, dfi, HF + (int64_t)k * nq, rhs + i);
      for (int j = 0; j <= i; ++j) {
        k_sub<<<cdiv(nq, T), T, 0, c->stream>>>(nq, HF + (int64_t)(j + 1) * nq, HF + (int64_t)j * nq,
                                                dfj);
        k_wdot<<<nb, 256, 0, c->stream>>>(nq, c->nqp, c->d_W3, dfi, dfj, A + i * k + j);
      }
    }
    k_small_solve<<<1, 1, 0, c->stream>>>(k, A, rhs, gam);
  }
  int kerker_it = 0;
  if (prm->kerker_k0 > 0.0) {
    // x_bar in rho_in, F_bar in dfi, then rho_in += beta P F_bar
    k_anderson_update<<<cdiv(nq, T), T, 0, c->stream>>>(nq, k, HX, HF, nq, gam, prm->mix_beta,
                                                        s.rho_in, dfi);
    if ((st = kerker(c, prm->kerker_k0, dfi, prm->cg_rtol, prm->cg_maxit, &kerker_it))) return st;
    k_axpy<<<cdiv(nq, T), T, 0, c->stream>>>(nq, prm->mix_beta, dfi, s.rho_in);
  } else {
    k_anderson_update<<<cdiv(nq, T), T, 0, c->stream>>>(nq, k, HX, HF, nq, gam, prm->mix_beta,
                                                        s.rho_in, nullptr);
  }
  rep->mix_cg_iters = kerker_it;
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  rep->t_other_ms = ms_since(t3);
  s.iter++;
  return EFE_OK;
}
