// Setup and per-potential operator kernels.
//
//  reference element   GLL/Gauss rules and 1-D Lagrange tables (host, a few
//                      numbers), 3-D basis/gradient tables, cell stiffness and
//                      lumped GLL mass on the GPU (Sec. III.A)
//  enrichment          normalization, b = int N phi, kinetic part of
//                      B = <phi| -1/2 Lap |N>, M^phiphi, kinetic H^phiphi,
//                      C = b diag(m)^-1, M^ee = M^phiphi - b diag(m)^-1 b^T and
//                      the inverses of its atom blocks (Sec. II.B, Eq.
//                      MEInvApprox)
//  projectors          P^C = int beta N, P^phi = int beta phi, D (Eq. KS)
//  potential           cell Hamiltonians 1/2 K + N^T diag(w v) N in the MFMA
//                      operand layout, B and H^phiphi potential parts
#include <cmath>
#include <vector>

#include "efe_device.h"

// ------------------------------------------------------------ 1-D rules
static void legendre(int n, double x, double &P, double &dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

static void gll_rule(int p, std::vector<double> &x, std::vector<double> &w) {
  x.assign(p + 1, 0.0);
  w.assign(p + 1, 0.0);
  x[0] = -1.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double t = -cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {   // Newton on P_p'
      double P, dP;
      legendre(p, t, P, dP);
      double d2P = (2 * t * dP - p * (p + 1) * P) / (1.0 - t * t);
      double dt = dP / d2P;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    x[i] = t;
  }
  for (int i = 0; i <= p; ++i) {
    double P, dP;
    legendre(p, x[i], P, dP);
    w[i] = 2.0 / (p * (p + 1) * P * P);
  }
}

static void gauss_rule(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = -cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, t, P, dP);
      double dt = P / dP;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    double P, dP;
    legendre(n, t, P, dP);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dP * dP);
  }
}

// ------------------------------------------------------------ kernels
// 3-D basis values and physical gradients at the Gauss points, weights.
__global__ void k_ref3d(int P, int nq, const double *__restrict__ N1, const double *__restrict__ D1,
                        const double *__restrict__ wq, double hx, double hy, double hz,
                        double *__restrict__ N3, double *__restrict__ G3, double *__restrict__ W3) {
  const int nloc = P * P * P, nqp = nq * nq * nq;
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nqp * nloc) return;
  int q = idx / nloc, l = idx % nloc;
  int a = l % P, b = (l / P) % P, c = l / (P * P);
  int qa = q % nq, qb = (q / nq) % nq, qc = q / (nq * nq);
  double na = N1[qa * P + a], nb = N1[qb * P + b], nc = N1[qc * P + c];
  double da = D1[qa * P + a], db = D1[qb * P + b], dc = D1[qc * P + c];
  N3[idx] = na * nb * nc;
  G3[idx] = da * nb * nc * (2.0 / hx);
  G3[(int64_t)nqp * nloc + idx] = na * db * nc * (2.0 / hy);
  G3[2 * (int64_t)nqp * nloc + idx] = na * nb * dc * (2.0 / hz);
  if (l == 0) W3[q] = wq[qa] * wq[qb] * wq[qc] * (hx * hy * hz / 8.0);
}

// K[l][l'] = sum_q W_q grad N_l . grad N_l'
__global__ void k_stiffness(int nloc, int nqp, const double *__restrict__ G3,
                            const double *__restrict__ W3, double *__restrict__ K) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nloc * nloc) return;
  int i = idx / nloc, j = idx % nloc;
  const int64_t s = (int64_t)nqp * nloc;
  double acc = 0.0;
  for (int q = 0; q < nqp; ++q) {
    const int64_t o = (int64_t)q * nloc;
    acc += W3[q] * (G3[o + i] * G3[o + j] + G3[s + o + i] * G3[s + o + j] +
                    G3[2 * s + o + i] * G3[2 * s + o + j]);
  }
  K[idx] = acc;
}

// Lumped GLL mass: product of 1-D lumped weights (shared nodes get both cells).
__global__ void k_lumped_mass(int64_t n1x, int64_t n1y, int64_t n1z, int p,
                              const double *__restrict__ wg, double hx, double hy, double hz,
                              double *__restrict__ m, double *__restrict__ minv,
                              double *__restrict__ m_int) {
  int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (n >= n1x * n1y * n1z) return;
  int64_t idx[3] = {n % n1x, (n / n1x) % n1y, n / (n1x * n1y)};
  int64_t nn[3] = {n1x, n1y, n1z};
  double hh[3] = {hx, hy, hz};
  double mm = 1.0;
  bool bnd = false;
  for (int d = 0; d < 3; ++d) {
    int64_t i = idx[d];
    int a = (int)(i % p);
    double w;
    if (a == 0 && i > 0 && i < nn[d] - 1) w = wg[0] + wg[p];
    else if (i == nn[d] - 1) w = wg[p];
    else w = wg[a];
    mm *= 0.5 * hh[d] * w;
    if (i == 0 || i == nn[d] - 1) bnd = true;
  }
  m[n] = mm;
  minv[n] = bnd ? 0.0 : 1.0 / mm;
  m_int[n] = bnd ? 0.0 : mm;
}

// sum_q W phi_raw^2 per enrichment function (one block per (atom, cell) pair)
__global__ void k_enr_norm(MeshGeo g, EnrParam e, const double *__restrict__ xq1,
                           const double *__restrict__ W3, const double *__restrict__ xyz,
                           const int32_t *__restrict__ pair_atom,
                           const int32_t *__restrict__ pair_cell, double *__restrict__ norm2) {
  __shared__ double red[256][9];
  const int pr = blockIdx.x;
  const int I = pair_atom[pr], cell = pair_cell[pr];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int q = threadIdx.x; q < g.nqp; q += blockDim.x) {
    double x[3], phi[9];
    quad_point(g, xq1, cell, q, x);
    enr_eval(e, x[0] - xyz[3 * I], x[1] - xyz[3 * I + 1], x[2] - xyz[3 * I + 2], phi, nullptr);
    for (int k = 0; k < e.nf; ++k) acc[k] += W3[q] * phi[k] * phi[k];
  }
  for (int k = 0; k < 9; ++k) red[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 9; ++k) red[threadIdx.x][k] += red[threadIdx.x + s][k];
    __syncthreads();
  }
  if (threadIdx.x < (unsigned)e.nf) atomicAdd(&norm2[I * e.nf + threadIdx.x], red[0][threadIdx.x]);
}

__global__ void k_inv_sqrt(int64_t n, double *__restrict__ x) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = 1.0 / sqrt(x[i]);
}

// Per pair: b[l][k] += sum_q W phi_k N_l ; Bkin[l][k] += 1/2 sum_q W grad phi_k . grad N_l
// (with_kin) or, for the potential part, Bv[l][k] += sum_q W v phi_k N_l.
template <bool KIN>
__global__ __launch_bounds__(256) void k_enr_pair_proj(
    MeshGeo g, EnrParam e, const double *__restrict__ xq1, const double *__restrict__ W3,
    const double *__restrict__ N3, const double *__restrict__ G3, const double *__restrict__ xyz,
    const double *__restrict__ nu, const int32_t *__restrict__ pair_atom,
    const int32_t *__restrict__ pair_cell, const int32_t *__restrict__ lmap,
    const double *__restrict__ vq, double *__restrict__ out_b, double *__restrict__ out_k,
    double *__restrict__ out_pair) {
  // weighted values at up to 64 quadrature points at a time
  __shared__ double sphi[9][64];
  __shared__ double sgrad[3][9][64];
  const int pr = blockIdx.x;
  const int I = pair_atom[pr], cell = pair_cell[pr];
  const int nf = e.nf, nloc = g.nloc, nqp = g.nqp;
  const int64_t s3 = (int64_t)nqp * nloc;
  // each thread owns outputs (l, k) with l = tid + 256 * r
  double accb[2][9], acck[2][9];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 9; ++k) accb[r][k] = acck[r][k] = 0.0;
  for (int q0 = 0; q0 < nqp; q0 += 64) {
    const int nqc = min(64, nqp - q0);
    if (threadIdx.x < (unsigned)nqc) {
      const int q = q0 + threadIdx.x;
      double x[3], phi[9], grad[27];
      quad_point(g, xq1, cell, q, x);
      enr_eval(e, x[0] - xyz[3 * I], x[1] - xyz[3 * I + 1], x[2] - xyz[3 * I + 2], phi,
               KIN ? grad : nullptr);
      const double w = W3[q] * (KIN ? 1.0 : vq[(int64_t)cell * nqp + q]);
      for (int k = 0; k < nf; ++k) {
        const double s = nu[I * nf + k];
        sphi[k][threadIdx.x] = w * s * phi[k];
        if (KIN)
          for (int d = 0; d < 3; ++d) sgrad[d][k][threadIdx.x] = 0.5 * w * s * grad[3 * k + d];
      }
    }
    __syncthreads();
    for (int r = 0; r < 2; ++r) {
      const int l = threadIdx.x + 256 * r;
      if (l >= nloc) continue;
      for (int qq = 0; qq < nqc; ++qq) {
        const int64_t o = (int64_t)(q0 + qq) * nloc + l;
        const double n = N3[o];
        for (int k = 0; k < nf; ++k) accb[r][k] += sphi[k][qq] * n;
        if (KIN) {
          const double gx = G3[o], gy = G3[s3 + o], gz = G3[2 * s3 + o];
          for (int k = 0; k < nf; ++k)
            acck[r][k] += sgrad[0][k][qq] * gx + sgrad[1][k][qq] * gy + sgrad[2][k][qq] * gz;
        }
      }
    }
    __syncthreads();
  }
  for (int r = 0; r < 2; ++r) {
    const int l = threadIdx.x + 256 * r;
    if (l >= nloc) continue;
    // the cell's own block (kinetic part), kept per pair for the coupling
    // E_c = B_c - C_c H_c of the orthogonalized basis
    if (KIN && out_pair)
      for (int k = 0; k < nf; ++k) out_pair[((int64_t)pr * nloc + l) * nf + k] = acck[r][k];
    const int32_t s = lmap[(int64_t)pr * nloc + l];
    if (s < 0) continue;
    for (int k = 0; k < nf; ++k) {
      atomicAdd(&out_b[(int64_t)s * nf + k], accb[r][k]);
      if (KIN) atomicAdd(&out_k[(int64_t)s * nf + k], acck[r][k]);
    }
  }
}

// Potential part of the same projections, on FP64 MFMA: for one (atom, cell)
// pair, out[l][k] += sum_q N[q][l] (w v s_k phi_k)(x_q), a 343 x 9 product
// over the cell's Gauss points.  The weighted enrichment values sit in LDS as
// the B operand (16 columns, zero past nf and past nqp); each wave takes row
// blocks of N^T (A operand, 16 consecutive entries of a row of N per load).
typedef double v4d_p __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_enr_pair_proj_v(
    MeshGeo g, EnrParam e, const double *__restrict__ xq1, const double *__restrict__ W3,
    const double *__restrict__ N3, const double *__restrict__ xyz, const double *__restrict__ nu,
    const int32_t *__restrict__ pair_atom, const int32_t *__restrict__ pair_cell,
    const int32_t *__restrict__ lmap, const double *__restrict__ vq, int KQ,
    double *__restrict__ out_b, const double *__restrict__ kin_pair,
    double *__restrict__ out_pair) {
  extern __shared__ double sphi[];   // [4 KQ][16]
  const int pr = blockIdx.x;
  const int I = pair_atom[pr], cell = pair_cell[pr];
  const int nf = e.nf, nloc = g.nloc, nqp = g.nqp;
  for (int q = threadIdx.x; q < 4 * KQ; q += blockDim.x) {
    double row[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) row[k] = 0.0;
    if (q < nqp) {
      double x[3], phi[9];
      quad_point(g, xq1, cell, q, x);
      enr_eval(e, x[0] - xyz[3 * I], x[1] - xyz[3 * I + 1], x[2] - xyz[3 * I + 2], phi, nullptr);
      const double w = W3[q] * vq[(int64_t)cell * nqp + q];
#pragma unroll
      for (int k = 0; k < 9; ++k)
        if (k < nf) row[k] = w * nu[I * nf + k] * phi[k];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) sphi[q * 16 + k] = row[k];
  }
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, li = lane % 16, lk = lane / 16;
  const int RB = (nloc + 15) / 16;
  for (int rb = wave; rb < RB; rb += 4) {
    const double *np = N3 + min(16 * rb + li, nloc - 1);
    v4d_p acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int ks = 0; ks < KQ; ++ks) {
      const int q = min(4 * ks + lk, nqp - 1);   // past nqp: zero rows of sphi
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(np[(int64_t)q * nloc],
                                                 sphi[(4 * ks + lk) * 16 + li], acc, 0, 0, 0);
    }
    // accumulator v of lane l: local node 16 rb + 4 v + l/16, function l%16
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int l = 16 * rb + 4 * v + lk;
      if (l < nloc && li < nf) {
        const int64_t o = ((int64_t)pr * nloc + l) * nf + li;
        if (out_pair) out_pair[o] = kin_pair[o] + acc[v];
        const int32_t sn = lmap[(int64_t)pr * nloc + l];
        if (sn >= 0) atomicAdd(&out_b[(int64_t)sn * nf + li], acc[v]);
      }
    }
  }
}

// C = b / m on support nodes
__global__ void k_scale_by_minv(int64_t n_snodes, int nf, const int32_t *__restrict__ snode,
                                const double *__restrict__ minv, const double *__restrict__ b,
                                double *__restrict__ C) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n_snodes * nf) return;
  C[i] = b[i] * minv[snode[i / nf]];
}

// node-major copy: dst[e*nf + k] = src[nm_src[e]*nf + k]
__global__ void k_to_node_major(int64_t nnz, int nf, const int32_t *__restrict__ nm_src,
                                const double *__restrict__ src, double *__restrict__ dst) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nnz * nf) return;
  dst[i] = src[(int64_t)nm_src[i / nf] * nf + i % nf];
}

// group-major copy: dst[(slot nf + k) 8 + n % 8] = src[nm_src[e] nf + k] for
// every node-major entry e of node n (slot = its atom's place in the union of
// the atoms of the 8-node group of n); entries not written stay zero
__global__ void k_to_group_major(int64_t n_nodes, int nf, const int32_t *__restrict__ nm_ptr,
                                 const int32_t *__restrict__ nm_src,
                                 const int32_t *__restrict__ nm_gslot,
                                 const double *__restrict__ src, double *__restrict__ dst) {
  const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (n >= n_nodes) return;
  const int j = (int)(n & 7);
  for (int32_t e = nm_ptr[n]; e < nm_ptr[n + 1]; ++e) {
    const int64_t slot = nm_gslot[e], s0 = (int64_t)nm_src[e] * nf;
    for (int k = 0; k < nf; ++k) dst[(slot * nf + k) * 8 + j] = src[s0 + k];
  }
}

// Per (cell, I, J): M[I k][J l] += sum_q W phi_Ik phi_Jl and, with KIN,
// H[I k][J l] += 1/2 sum_q W grad phi_Ik . grad phi_Jl; without KIN the
// weight carries the potential: H[I k][J l] += sum_q W v phi_Ik phi_Jl.
template <bool KIN>
__global__ __launch_bounds__(128) void k_enr_pp(MeshGeo g, EnrParam e, const double *__restrict__ xq1,
                                                const double *__restrict__ W3,
                                                const double *__restrict__ xyz,
                                                const double *__restrict__ nu,
                                                const int32_t *__restrict__ trip,
                                                const double *__restrict__ vq, int64_t n_enr,
                                                double *__restrict__ M, double *__restrict__ H) {
  __shared__ double pI[4][9][64], pJ[4][9][64];
  const int64_t t = blockIdx.x;
  const int cell = trip[3 * t], I = trip[3 * t + 1], J = trip[3 * t + 2];
  const int nf = e.nf, nqp = g.nqp;
  const int tid = threadIdx.x;
  const int k = tid / 9, l = tid % 9;          // 81 output pairs
  double am = 0.0, ah = 0.0;
  for (int q0 = 0; q0 < nqp; q0 += 64) {
    const int nqc = min(64, nqp - q0);
    if (tid < nqc) {
      const int q = q0 + tid;
      double x[3], phi[9], grad[27], phj[9], grj[27];
      quad_point(g, xq1, cell, q, x);
      enr_eval(e, x[0] - xyz[3 * I], x[1] - xyz[3 * I + 1], x[2] - xyz[3 * I + 2], phi,
               KIN ? grad : nullptr);
      enr_eval(e, x[0] - xyz[3 * J], x[1] - xyz[3 * J + 1], x[2] - xyz[3 * J + 2], phj,
               KIN ? grj : nullptr);
      const double w = W3[q] * (KIN ? 1.0 : vq[(int64_t)cell * nqp + q]);
      for (int a = 0; a < nf; ++a) {
        const double si = nu[I * nf + a], sj = nu[J * nf + a];
        pI[0][a][tid] = w * si * phi[a];
        pJ[0][a][tid] = sj * phj[a];
        if (KIN)
          for (int d = 0; d < 3; ++d) {
            pI[1 + d][a][tid] = 0.5 * w * si * grad[3 * a + d];
            pJ[1 + d][a][tid] = sj * grj[3 * a + d];
          }
      }
    }
    __syncthreads();
    if (k < nf && l < nf) {
      for (int qq = 0; qq < nqc; ++qq) {
        am += pI[0][k][qq] * pJ[0][l][qq];
        if (KIN)
          ah += pI[1][k][qq] * pJ[1][l][qq] + pI[2][k][qq] * pJ[2][l][qq] +
                pI[3][k][qq] * pJ[3][l][qq];
      }
    }
    __syncthreads();
  }
  if (k < nf && l < nf) {
    const int64_t o = (int64_t)(I * nf + k) * n_enr + J * nf + l;
    if (KIN) {
      atomicAdd(&M[o], am);
      atomicAdd(&H[o], ah);
    } else {
      atomicAdd(&H[o], am);
    }
  }
}

// Row f of b diag(m)^-1 b^T, subtracted from M^phiphi: Mee[f][:] = Mpp[f][:] - acc
__global__ __launch_bounds__(256) void k_mee_rows(int nf, int64_t n_enr, const int32_t *__restrict__ snode_ptr,
                                                  const int32_t *__restrict__ snode,
                                                  const int32_t *__restrict__ nm_ptr,
                                                  const int32_t *__restrict__ nm_atom,
                                                  const int32_t *__restrict__ nm_src,
                                                  const double *__restrict__ C_am,
                                                  const double *__restrict__ b_am,
                                                  const double *__restrict__ Mpp,
                                                  double *__restrict__ Mee) {
  extern __shared__ double acc[];
  const int64_t f = blockIdx.x;
  const int I = f / nf, k = f % nf;
  for (int64_t i = threadIdx.x; i < n_enr; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  for (int32_t s = snode_ptr[I] + threadIdx.x; s < snode_ptr[I + 1]; s += blockDim.x) {
    const int32_t j = snode[s];
    const double cf = C_am[(int64_t)s * nf + k];
    for (int32_t ee = nm_ptr[j]; ee < nm_ptr[j + 1]; ++ee) {
      const int J = nm_atom[ee];
      const int64_t src = nm_src[ee];
      for (int l = 0; l < nf; ++l) atomicAdd(&acc[J * nf + l], cf * b_am[src * nf + l]);
    }
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n_enr; i += blockDim.x)
    Mee[f * n_enr + i] = Mpp[f * n_enr + i] - acc[i];
}

// ------------------------------------------------------------ coupling
// The orthogonalized basis couples the enrichment rows to the CFE rows
// through H^ec = B - C H^cc (Sec. II.B: N^E = phi - C N^C).  Per cell,
// E_c = B_c - C_c H_c (n_e x nloc: the cell's enrichment functions against
// its nodes), formed here in FP64 so that the cancellation between B and
// C H happens before any rounding to a reduced precision.  One work-group
// takes a cell and 16 of its enrichment functions: C_c^T (nloc x 16) in LDS as
// the B operand, the cell Hamiltonian's MFMA tiles as the A operand, each wave
// a row block of H_c C_c^T.  The results go to both operand layouts of the
// apply (E_c^T rows = nodes, E_c rows = functions; zero padding included).
__global__ __launch_bounds__(256) void k_build_E(
    int nloc, int RB, int KS, int nf, int max_cb, const double *__restrict__ Ht,
    const int32_t *__restrict__ cell_eptr, const int32_t *__restrict__ cell_epair,
    const int64_t *__restrict__ cell_noff, const int32_t *__restrict__ lmap,
    const int32_t *__restrict__ spair, const double *__restrict__ C_am,
    const double *__restrict__ B_pair,
    double *__restrict__ Et, double *__restrict__ Ee, float *__restrict__ Et32,
    float *__restrict__ Ee32) {
  __shared__ double Cs[EFE_MAXLOC + 16][16];
  const int64_t cell = blockIdx.x / max_cb;
  const int cb = blockIdx.x % max_cb;
  const int32_t p0 = cell_eptr[cell];
  const int ne = (cell_eptr[cell + 1] - p0) * nf;
  if (16 * cb >= ne) return;
  const int nep = (ne + 15) / 16 * 16, kse_n = nep / 4;
  const int64_t noff = cell_noff[cell];
  for (int i = threadIdx.x; i < 4 * KS * 16; i += 256) {
    const int l = i / 16, j = i % 16, e = 16 * cb + j;
    double v = 0.0;
    if (l < nloc && e < ne) {
      const int32_t pr = cell_epair[p0 + e / nf];
      const int32_t sn = lmap[(int64_t)pr * nloc + l];
      if (sn >= 0) v = C_am[(int64_t)sn * nf + e % nf];
    }
    Cs[l][j] = v;
  }
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, li = lane % 16, lk = lane / 16;
  for (int rb = wave; rb < RB; rb += 4) {
    const double *hp = Ht + ((int64_t)cell * RB + rb) * KS * 64 + lane;
    v4d_p acc = {0.0, 0.0, 0.0, 0.0};
    for (int ks = 0; ks < KS; ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(hp[(int64_t)ks * 64], Cs[4 * ks + lk][li], acc,
                                                 0, 0, 0);
    // accumulator v of lane l: node row 16 rb + 4 v + l/16, function 16 cb + l%16
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int l = 16 * rb + 4 * v + lk, e = 16 * cb + li;
      double val = 0.0;
      if (l < nloc && e < ne) {
        const int32_t pr = cell_epair[p0 + e / nf], sp = spair[pr];
        // B_c vanishes on the layer of cells outside the support
        const double bv = sp >= 0 ? B_pair[((int64_t)sp * nloc + l) * nf + e % nf] : 0.0;
        val = bv - acc[v];
      }
      // E_c^T tile: row l (block rb), k index e
      const int64_t ot = 16 * (int64_t)RB * noff + ((int64_t)rb * kse_n + e / 4) * 64 +
                         (l % 16) + 16 * (e % 4);
      Et[ot] = val;
      if (Et32) Et32[ot] = (float)val;
      // E_c tile: row e (block e/16), k index l (k steps cover 4 KS nodes)
      if (l < 4 * KS) {
        const int64_t oe = 4 * (int64_t)KS * noff + ((int64_t)(e / 16) * KS + l / 4) * 64 +
                           (e % 16) + 16 * (l % 4);
        Ee[oe] = val;
        if (Ee32) Ee32[oe] = (float)val;
      }
    }
  }
}

// Rows of the enrichment block of the orthogonalized Hamiltonian without the
// projectors, H^E_ee = H^phiphi - C B^T - E C^T (the expansion of T^T Hhat T
// with E = B - C H^cc), first part: Hee = H^phiphi - C B^T, row f = (I, k)
// summed over the support nodes of atom I and, at each node, the atoms whose
// support holds it (B vanishes off the support).
__global__ __launch_bounds__(256) void k_hee_rows(int nf, int64_t n_enr,
                                                  const int32_t *__restrict__ snode_ptr,
                                                  const int32_t *__restrict__ snode,
                                                  const int32_t *__restrict__ nm_ptr,
                                                  const int32_t *__restrict__ nm_atom,
                                                  const int32_t *__restrict__ nm_src,
                                                  const double *__restrict__ C_am,
                                                  const double *__restrict__ B_am,
                                                  const double *__restrict__ Hpp,
                                                  double *__restrict__ Hee) {
  extern __shared__ double acc[];
  const int64_t f = blockIdx.x;
  const int I = f / nf, k = f % nf;
  for (int64_t i = threadIdx.x; i < n_enr; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  for (int32_t s = snode_ptr[I] + threadIdx.x; s < snode_ptr[I + 1]; s += blockDim.x) {
    const int32_t j = snode[s];
    const double cf = C_am[(int64_t)s * nf + k];
    for (int32_t ee = nm_ptr[j]; ee < nm_ptr[j + 1]; ++ee) {
      const int J = nm_atom[ee];
      const int64_t src = nm_src[ee];
      for (int l = 0; l < nf; ++l) atomicAdd(&acc[J * nf + l], cf * B_am[src * nf + l]);
    }
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n_enr; i += blockDim.x)
    Hee[f * n_enr + i] = Hpp[f * n_enr + i] - acc[i];
}

// Second part: Hee -= E C^T = sum over cells of E_c C_c^T (E is non-zero on
// the cells that hold an atom's support nodes, one layer beyond its support,
// so the product is taken cell by cell).  One work-group takes a cell and 16
// of its enrichment functions e2: C_c^T (nodes x 16) in LDS as the B operand,
// the E_c tiles as the A operand, each wave the row blocks e1 = wave + 4 i;
// every 16 x 16 block is added into Hee atomically.
__global__ __launch_bounds__(256) void k_hee_cells(
    int nloc, int KS, int nf, int max_cb, int64_t n_enr, const int32_t *__restrict__ cell_eptr,
    const int32_t *__restrict__ cell_epair, const int64_t *__restrict__ cell_noff,
    const int32_t *__restrict__ cpair_atom, const int32_t *__restrict__ lmap,
    const double *__restrict__ C_am, const double *__restrict__ Ee, double *__restrict__ Hee) {
  __shared__ double Cs[EFE_MAXLOC + 16][16];
  const int64_t cell = blockIdx.x / max_cb;
  const int cb = blockIdx.x % max_cb;
  const int32_t p0 = cell_eptr[cell];
  const int ne = (cell_eptr[cell + 1] - p0) * nf;
  if (16 * cb >= ne) return;
  const int RBE = (ne + 15) / 16;
  const int64_t noff = cell_noff[cell];
  for (int i = threadIdx.x; i < 4 * KS * 16; i += 256) {
    const int l = i / 16, j = i % 16, e = 16 * cb + j;
    double v = 0.0;
    if (l < nloc && e < ne) {
      const int32_t pr = cell_epair[p0 + e / nf];
      const int32_t sn = lmap[(int64_t)pr * nloc + l];
      if (sn >= 0) v = C_am[(int64_t)sn * nf + e % nf];
    }
    Cs[l][j] = v;
  }
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, li = lane % 16, lk = lane / 16;
  const int e2 = 16 * cb + li;
  const int64_t f2 = e2 < ne ? (int64_t)cpair_atom[cell_epair[p0 + e2 / nf]] * nf + e2 % nf : 0;
  for (int b1 = wave; b1 < RBE; b1 += 4) {
    const double *ap = Ee + 4 * (int64_t)KS * noff + (int64_t)b1 * KS * 64 + lane;
    v4d_p acc = {0.0, 0.0, 0.0, 0.0};
    for (int ks = 0; ks < KS; ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[(int64_t)ks * 64], Cs[4 * ks + lk][li], acc,
                                                 0, 0, 0);
    // accumulator v of lane l: function e1 = 16 b1 + 4 v + l/16, e2 = 16 cb + l%16
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int e1 = 16 * b1 + 4 * v + lk;
      if (e1 < ne && e2 < ne) {
        const int64_t f1 = (int64_t)cpair_atom[cell_epair[p0 + e1 / nf]] * nf + e1 % nf;
        atomicAdd(&Hee[f1 * n_enr + f2], -acc[v]);
      }
    }
  }
}

// Projector rows in the orthogonalized basis: P~^phi = P^phi - P^C C^T
// (beta . (phi - C N^C)), one work-group per projector.
__global__ __launch_bounds__(256) void k_ptilde(int nf, int64_t n_enr,
                                                const int32_t *__restrict__ kbnode_ptr,
                                                const int32_t *__restrict__ kbnode,
                                                const double *__restrict__ Pc_am,
                                                const int32_t *__restrict__ nm_ptr,
                                                const int32_t *__restrict__ nm_atom,
                                                const int32_t *__restrict__ nm_src,
                                                const double *__restrict__ C_am,
                                                const double *__restrict__ Pphi,
                                                double *__restrict__ Pt) {
  extern __shared__ double acc[];
  const int K = blockIdx.x;
  for (int64_t i = threadIdx.x; i < n_enr; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  for (int32_t s = kbnode_ptr[K] + threadIdx.x; s < kbnode_ptr[K + 1]; s += blockDim.x) {
    const int32_t j = kbnode[s];
    const double pc = Pc_am[s];
    for (int32_t ee = nm_ptr[j]; ee < nm_ptr[j + 1]; ++ee) {
      const int J = nm_atom[ee];
      const int64_t src = nm_src[ee];
      for (int l = 0; l < nf; ++l) atomicAdd(&acc[J * nf + l], pc * C_am[src * nf + l]);
    }
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n_enr; i += blockDim.x)
    Pt[(int64_t)K * n_enr + i] = Pphi[(int64_t)K * n_enr + i] - acc[i];
}

// Symmetrize a square matrix in place: A = (A + A^T)/2
__global__ void k_symmetrize(int64_t n, double *__restrict__ A) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  int64_t i = idx / n, j = idx % n;
  if (j <= i) return;
  double v = 0.5 * (A[i * n + j] + A[j * n + i]);
  A[i * n + j] = v;
  A[j * n + i] = v;
}

// Inverse of each atom-diagonal nf x nf block of M^ee (Gauss-Jordan, pivoted).
__global__ void k_block_inv(int natoms, int nf, int64_t n_enr, const double *__restrict__ Mee,
                            double *__restrict__ inv, int *__restrict__ fail) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= natoms) return;
  double a[9][18];
  for (int i = 0; i < nf; ++i)
    for (int j = 0; j < nf; ++j) {
      a[i][j] = Mee[(int64_t)(I * nf + i) * n_enr + I * nf + j];
      a[i][nf + j] = (i == j) ? 1.0 : 0.0;
    }
  for (int c = 0; c < nf; ++c) {
    int piv = c;
    for (int r = c + 1; r < nf; ++r)
      if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
    if (!(fabs(a[piv][c]) > 0.0)) {
      *fail = 1;
      return;
    }
    if (piv != c)
      for (int j = 0; j < 2 * nf; ++j) {
        double t = a[c][j];
        a[c][j] = a[piv][j];
        a[piv][j] = t;
      }
    double d = 1.0 / a[c][c];
    for (int j = 0; j < 2 * nf; ++j) a[c][j] *= d;
    for (int r = 0; r < nf; ++r)
      if (r != c) {
        double f = a[r][c];
        for (int j = 0; j < 2 * nf; ++j) a[r][j] -= f * a[c][j];
      }
  }
  for (int i = 0; i < nf; ++i)
    for (int j = 0; j < nf; ++j) inv[((int64_t)I * nf + i) * nf + j] = a[i][nf + j];
}

// amp[I] = ||M^phiphi_II||_F ||(M^ee_II)^-1||_F
__global__ void k_block_amp(int natoms, int nf, int64_t n_enr, const double *__restrict__ Mpp,
                            const double *__restrict__ inv, double *__restrict__ amp) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= natoms) return;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < nf; ++i)
    for (int j = 0; j < nf; ++j) {
      const double m = Mpp[(int64_t)(I * nf + i) * n_enr + I * nf + j];
      const double v = inv[((int64_t)I * nf + i) * nf + j];
      a += m * m;
      b += v * v;
    }
  amp[I] = sqrt(a) * sqrt(b);
}

// Projector: P^C[s] += sum_q W beta N_l (one block per (atom, cell) pair)
__global__ __launch_bounds__(256) void k_kb_pc(MeshGeo g, double w, double rcut,
                                               const double *__restrict__ xq1,
                                               const double *__restrict__ W3,
                                               const double *__restrict__ N3,
                                               const double *__restrict__ xyz,
                                               const int32_t *__restrict__ pair_atom,
                                               const int32_t *__restrict__ pair_cell,
                                               const int32_t *__restrict__ lmap,
                                               double *__restrict__ Pc) {
  __shared__ double sb[EFE_MAXQ * EFE_MAXQ * EFE_MAXQ];
  const int pr = blockIdx.x;
  const int I = pair_atom[pr], cell = pair_cell[pr];
  for (int q = threadIdx.x; q < g.nqp; q += blockDim.x) {
    double x[3];
    quad_point(g, xq1, cell, q, x);
    double dx = x[0] - xyz[3 * I], dy = x[1] - xyz[3 * I + 1], dz = x[2] - xyz[3 * I + 2];
    sb[q] = W3[q] * kb_beta(dx * dx + dy * dy + dz * dz, w, rcut);
  }
  __syncthreads();
  for (int l = threadIdx.x; l < g.nloc; l += blockDim.x) {
    const int32_t s = lmap[(int64_t)pr * g.nloc + l];
    if (s < 0) continue;
    double acc = 0.0;
    for (int q = 0; q < g.nqp; ++q) acc += sb[q] * N3[(int64_t)q * g.nloc + l];
    atomicAdd(&Pc[s], acc);
  }
}

// Projector-enrichment overlap: Pphi[I][J nf + l] += sum_q W beta_I phi_Jl
__global__ __launch_bounds__(256) void k_kb_pphi(MeshGeo g, EnrParam e, double w, double rcut,
                                                 const double *__restrict__ xq1,
                                                 const double *__restrict__ W3,
                                                 const double *__restrict__ xyz,
                                                 const double *__restrict__ nu,
                                                 const int32_t *__restrict__ trip, int64_t n_enr,
                                                 double *__restrict__ Pphi) {
  __shared__ double red[256][9];
  const int64_t t = blockIdx.x;
  const int cell = trip[3 * t], I = trip[3 * t + 1], J = trip[3 * t + 2];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int q = threadIdx.x; q < g.nqp; q += blockDim.x) {
    double x[3], phi[9];
    quad_point(g, xq1, cell, q, x);
    double dx = x[0] - xyz[3 * I], dy = x[1] - xyz[3 * I + 1], dz = x[2] - xyz[3 * I + 2];
    const double b = W3[q] * kb_beta(dx * dx + dy * dy + dz * dz, w, rcut);
    enr_eval(e, x[0] - xyz[3 * J], x[1] - xyz[3 * J + 1], x[2] - xyz[3 * J + 2], phi, nullptr);
    for (int k = 0; k < e.nf; ++k) acc[k] += b * phi[k];
  }
  for (int k = 0; k < 9; ++k) red[threadIdx.x][k] = acc[k];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < 9; ++k) red[threadIdx.x][k] += red[threadIdx.x + s][k];
    __syncthreads();
  }
  if (threadIdx.x < (unsigned)e.nf)
    atomicAdd(&Pphi[(int64_t)I * n_enr + J * e.nf + threadIdx.x],
              red[0][threadIdx.x] * nu[J * e.nf + threadIdx.x]);
}

// BF16 operand tiles of v_mfma_f32_16x16x32_bf16 from the FP64 tiles:
// out[cell][rb][ks32][lane][e] = H[16 rb + lane%16][32 ks32 + 8 (lane/16) + e]
__global__ void k_tile_bf16(int64_t n_cells, int RB, int KS, int KS32,
                            const double *__restrict__ H64, uint16_t *__restrict__ out) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t total = n_cells * RB * KS32 * 64 * 8;
  if (idx >= total) return;
  const int e = idx % 8;
  const int lane = (idx / 8) % 64;
  const int ks32 = (idx / 512) % KS32;
  const int64_t crb = idx / (512 * (int64_t)KS32);      // cell * RB + rb
  const int i = lane % 16;
  const int k = 32 * ks32 + 8 * (lane / 16) + e;
  double v = 0.0;
  if (k < 4 * KS) v = H64[(crb * KS + k / 4) * 64 + i + 16 * (k % 4)];
  const __bf16 hb = (__bf16)(float)v;
  out[idx] = *(const uint16_t *)&hb;
}

__global__ void k_fill(int64_t n, double v, double *__restrict__ x) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_copy(int64_t n, const double *__restrict__ a, double *__restrict__ b) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// Local pseudopotential at every Gauss point: sum_I -Z erf(r/rc)/r + A exp(-(r/rg)^2)
__global__ void k_local_potential(MeshGeo g, const double *__restrict__ xq1, int natoms,
                                  const double *__restrict__ xyz, const double *__restrict__ Z,
                                  double rc, double amp, double rg, double *__restrict__ vq) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nq = (int64_t)g.ncell[0] * g.ncell[1] * g.ncell[2] * g.nqp;
  if (idx >= nq) return;
  double x[3];
  quad_point(g, xq1, (int)(idx / g.nqp), (int)(idx % g.nqp), x);
  double v = 0.0;
  for (int I = 0; I < natoms; ++I) {
    double dx = x[0] - xyz[3 * I], dy = x[1] - xyz[3 * I + 1], dz = x[2] - xyz[3 * I + 2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    double s = r / rc;
    double eor = s < 1e-6 ? (2.0 / (rc * sqrt(M_PI))) * (1.0 - s * s / 3.0) : erf(s) / r;
    v += -Z[I] * eor + amp * exp(-(r / rg) * (r / rg));
  }
  vq[idx] = v;
}

// Cell Hamiltonians H_c = 1/2 K + N^T diag(w v_c) N (Eq. Hcell with the
// local potential at the Gauss points) on v_mfma_f64_16x16x4.  One work-group
// per (cell, 16-row block): the block's 16 columns of diag(w v_c) N sit in LDS,
// and each wave forms 16 x 16 tiles of the transposed product
// D'[j][i] = sum_q N[q][j] (w v N)[q][16 rb + i], whose accumulator layout
// (lane l of register v: j = j0 + 4 v + l/16, i = l % 16) is exactly the
// stored operand layout tile[cell][rb][j/4][i + 16 (j%4)] = base + 16 j + i,
// so every register is one contiguous 512-byte store.  Quadrature steps past
// nqp meet zero rows of the LDS strip.
typedef double v4d_b __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_build_hcell(int nloc, int nqp, int RB, int KS, int KQ8,
                                                     const double *__restrict__ N3,
                                                     const double *__restrict__ W3,
                                                     const double *__restrict__ K,
                                                     const double *__restrict__ vq,
                                                     double *__restrict__ H64,
                                                     float *__restrict__ H32) {
  extern __shared__ double bs[];   // [4 KQ8][16]: (w v N)[q][16 rb + i]
  const int cell = blockIdx.x / RB, rb = blockIdx.x % RB;
  for (int idx = threadIdx.x; idx < 64 * KQ8; idx += blockDim.x) {
    const int q = idx / 16, row = 16 * rb + idx % 16;
    bs[idx] = (q < nqp && row < nloc)
                  ? W3[q] * vq[(int64_t)cell * nqp + q] * N3[(int64_t)q * nloc + row]
                  : 0.0;
  }
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, li = lane % 16, lk = lane / 16;
  const int JT = (4 * KS + 15) / 16;
  const int64_t tbase = ((int64_t)cell * RB + rb) * KS * 64;
  for (int jt = wave; jt < JT; jt += 4) {
    const int j0 = 16 * jt;
    const double *np = N3 + min(j0 + li, nloc - 1);
    v4d_b acc = {0.0, 0.0, 0.0, 0.0};
    double a[8], na[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) a[s] = np[(int64_t)min(4 * s + lk, nqp - 1) * nloc];
    for (int k0 = 0; k0 < KQ8; k0 += 8) {
      // next batch of N^T fragments (clamped rows; they meet zero LDS rows)
#pragma unroll
      for (int s = 0; s < 8; ++s)
        na[s] = np[(int64_t)min(4 * (k0 + 8 + s) + lk, nqp - 1) * nloc];
#pragma unroll
      for (int s = 0; s < 8; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], bs[(4 * (k0 + s) + lk) * 16 + li], acc,
                                                   0, 0, 0);
#pragma unroll
      for (int s = 0; s < 8; ++s) a[s] = na[s];
    }
    const int row = 16 * rb + li;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = j0 + 4 * v + lk;
      if (j >= 4 * KS) continue;
      const double h =
          (row < nloc && j < nloc) ? 0.5 * K[(int64_t)row * nloc + j] + acc[v] : 0.0;
      H64[tbase + 16 * j + li] = h;
      if (H32) H32[tbase + 16 * j + li] = (float)h;
    }
  }
}

// ------------------------------------------------------------ host launchers
efe_status efe_build_reference(efe_ctx *c) {
  std::vector<double> xg, wg, xq, wq;
  gll_rule(c->p, xg, wg);
  gauss_rule(c->nq, xq, wq);
  std::vector<double> N1(c->nq * c->P), D1(c->nq * c->P);
  for (int q = 0; q < c->nq; ++q)
    for (int a = 0; a < c->P; ++a) {
      double v = 1.0, d = 0.0;
      for (int b = 0; b < c->P; ++b)
        if (b != a) v *= (xq[q] - xg[b]) / (xg[a] - xg[b]);
      for (int b = 0; b < c->P; ++b) {
        if (b == a) continue;
        double t = 1.0 / (xg[a] - xg[b]);
        for (int cc = 0; cc < c->P; ++cc)
          if (cc != a && cc != b) t *= (xq[q] - xg[cc]) / (xg[a] - xg[cc]);
        d += t;
      }
      N1[q * c->P + a] = v;
      D1[q * c->P + a] = d;
    }
  double *dN1, *dD1, *dwq, *dwg;
  efe_status s;
  if ((s = efe_alloc(c, (void **)&dN1, N1.size() * 8))) return s;
  if ((s = efe_alloc(c, (void **)&dD1, D1.size() * 8))) return s;
  if ((s = efe_alloc(c, (void **)&dwq, wq.size() * 8))) return s;
  if ((s = efe_alloc(c, (void **)&dwg, wg.size() * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_xq1, xq.size() * 8))) return s;
  HIPCHK(c, hipMemcpyAsync(dN1, N1.data(), N1.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(dD1, D1.data(), D1.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(dwq, wq.data(), wq.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(dwg, wg.data(), wg.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_xq1, xq.data(), xq.size() * 8, hipMemcpyHostToDevice, c->stream));
  const int64_t nt = (int64_t)c->nqp * c->nloc;
  if ((s = efe_alloc(c, (void **)&c->d_N3, nt * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_G3, 3 * nt * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_W3, c->nqp * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_K, (int64_t)c->nloc * c->nloc * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_m, c->n_nodes * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_minv, c->n_nodes * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_m_int, c->n_nodes * 8))) return s;
  k_ref3d<<<cdiv(nt, 256), 256, 0, c->stream>>>(c->P, c->nq, dN1, dD1, dwq, c->h[0], c->h[1],
                                                c->h[2], c->d_N3, c->d_G3, c->d_W3);
  k_stiffness<<<cdiv((int64_t)c->nloc * c->nloc, 256), 256, 0, c->stream>>>(c->nloc, c->nqp,
                                                                             c->d_G3, c->d_W3, c->d_K);
  k_lumped_mass<<<cdiv(c->n_nodes, 256), 256, 0, c->stream>>>(
      c->n1[0], c->n1[1], c->n1[2], c->p, dwg, c->h[0], c->h[1], c->h[2], c->d_m, c->d_minv, c->d_m_int);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  (void)hipFree(dN1);
  (void)hipFree(dD1);
  (void)hipFree(dwq);
  (void)hipFree(dwg);
  // MFMA tile geometry of the cell GEMM
  c->KP = (int)cdiv(c->nloc, 4) * 4;
  c->KS = c->KP / 4;
  c->RB = (int)cdiv(c->nloc, 16);
  c->KS32 = (int)cdiv(c->nloc, 32);
  return EFE_OK;
}

efe_status efe_build_enrichment(efe_ctx *c) {
  efe_status s;
  const MeshGeo g = mesh_geo(c);
  const EnrParam e = enr_param(c);
  const int nf = c->nf;
  const int64_t ne = c->n_enr;
  const int64_t ns = c->n_snodes * nf;
  if ((s = efe_alloc(c, (void **)&c->d_nu, ne * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_b_am, ns * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_C_am, ns * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_Bkin_am, ns * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_B_am, ns * 8))) return s;
  const int64_t ng = c->n_gslots * nf * 8;
  if ((s = efe_alloc(c, (void **)&c->d_Cg, ng * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_Bg, ng * 8))) return s;
  if (ng) {
    HIPCHK(c, hipMemsetAsync(c->d_Cg, 0, ng * 8, c->stream));
    HIPCHK(c, hipMemsetAsync(c->d_Bg, 0, ng * 8, c->stream));
  }
  if ((s = efe_alloc(c, (void **)&c->d_Mpp, ne * ne * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_Mee, ne * ne * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_Hpp_kin, ne * ne * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_Hpp, ne * ne * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_Mee_inv, (int64_t)c->natoms * nf * nf * 8))) return s;
  HIPCHK(c, hipMemsetAsync(c->d_nu, 0, ne * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_b_am, 0, ns * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_Bkin_am, 0, ns * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_Mpp, 0, ne * ne * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_Hpp_kin, 0, ne * ne * 8, c->stream));
  if (nf > 0 && c->npairs > 0) {
    k_enr_norm<<<c->npairs, 256, 0, c->stream>>>(g, e, c->d_xq1, c->d_W3, c->d_xyz,
                                                 c->d_pair_atom, c->d_pair_cell, c->d_nu);
    k_inv_sqrt<<<cdiv(ne, 256), 256, 0, c->stream>>>(ne, c->d_nu);
    if ((s = efe_alloc(c, (void **)&c->d_Bkin_pair, (size_t)c->npairs * c->nloc * nf * 8)))
      return s;
    k_enr_pair_proj<true><<<c->npairs, 256, 0, c->stream>>>(
        g, e, c->d_xq1, c->d_W3, c->d_N3, c->d_G3, c->d_xyz, c->d_nu, c->d_pair_atom,
        c->d_pair_cell, c->d_pair_lmap, nullptr, c->d_b_am, c->d_Bkin_am, c->d_Bkin_pair);
    k_scale_by_minv<<<cdiv(ns, 256), 256, 0, c->stream>>>(c->n_snodes, nf, c->d_snode, c->d_minv,
                                                          c->d_b_am, c->d_C_am);
    k_to_group_major<<<cdiv(c->n_nodes, 256), 256, 0, c->stream>>>(
        c->n_nodes, nf, c->d_nm_ptr, c->d_nm_src, c->d_nm_gslot, c->d_C_am, c->d_Cg);
    if (c->ntrip > 0)
      k_enr_pp<true><<<c->ntrip, 128, 0, c->stream>>>(g, e, c->d_xq1, c->d_W3, c->d_xyz, c->d_nu,
                                                      c->d_trip, nullptr, ne, c->d_Mpp,
                                                      c->d_Hpp_kin);
    k_symmetrize<<<cdiv(ne * ne, 256), 256, 0, c->stream>>>(ne, c->d_Mpp);
    k_symmetrize<<<cdiv(ne * ne, 256), 256, 0, c->stream>>>(ne, c->d_Hpp_kin);
    if (ne * 8 > 150 * 1024) EFE_FAIL(c, EFE_EINVAL, "too many enrichment functions for M^ee rows");
    k_mee_rows<<<ne, 256, ne * 8, c->stream>>>(nf, ne, c->d_snode_ptr, c->d_snode, c->d_nm_ptr,
                                               c->d_nm_atom, c->d_nm_src, c->d_C_am, c->d_b_am,
                                               c->d_Mpp, c->d_Mee);
    k_symmetrize<<<cdiv(ne * ne, 256), 256, 0, c->stream>>>(ne, c->d_Mee);
    int *dfail;
    if ((s = efe_alloc(c, (void **)&dfail, sizeof(int)))) return s;
    HIPCHK(c, hipMemsetAsync(dfail, 0, sizeof(int), c->stream));
    k_block_inv<<<cdiv(c->natoms, 64), 64, 0, c->stream>>>(c->natoms, nf, ne, c->d_Mee,
                                                           c->d_Mee_inv, dfail);
    int hfail = 0;
    HIPCHK(c, hipMemcpyAsync(&hfail, dfail, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    (void)hipFree(dfail);
    if (hfail) EFE_FAIL(c, EFE_ENUMERIC, "singular atom block of M^ee");
    double *damp;
    if ((s = efe_alloc(c, (void **)&damp, (size_t)c->natoms * 8))) return s;
    k_block_amp<<<cdiv(c->natoms, 64), 64, 0, c->stream>>>(c->natoms, nf, ne, c->d_Mpp,
                                                           c->d_Mee_inv, damp);
    std::vector<double> amp(c->natoms);
    HIPCHK(c, hipMemcpyAsync(amp.data(), damp, (size_t)c->natoms * 8, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    (void)hipFree(damp);
    c->amplification = 1.0;
    for (double a : amp) c->amplification = std::max(c->amplification, a);
  }
  // projectors
  const int np = c->nproj;
  if ((s = efe_alloc(c, (void **)&c->d_Pc_am, c->n_kbnodes * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_Pc_nm, c->nnz_kbnm * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_Pphi, (int64_t)np * ne * 8))) return s;
  if ((s = efe_alloc(c, (void **)&c->d_D, np * 8))) return s;
  HIPCHK(c, hipMemsetAsync(c->d_Pc_am, 0, c->n_kbnodes * 8, c->stream));
  HIPCHK(c, hipMemsetAsync(c->d_Pphi, 0, (int64_t)np * ne * 8, c->stream));
  if (np > 0) {
    k_fill<<<cdiv(np, 256), 256, 0, c->stream>>>(np, c->kb_D, c->d_D);
    k_kb_pc<<<c->nkbpairs, 256, 0, c->stream>>>(g, c->kb_width, c->kb_rcut, c->d_xq1, c->d_W3,
                                                c->d_N3, c->d_xyz, c->d_kbpair_atom,
                                                c->d_kbpair_cell, c->d_kbpair_lmap, c->d_Pc_am);
    k_to_node_major<<<cdiv(c->nnz_kbnm, 256), 256, 0, c->stream>>>(c->nnz_kbnm, 1, c->d_kbnm_src,
                                                                   c->d_Pc_am, c->d_Pc_nm);
    if (c->nkbtrip > 0)
      k_kb_pphi<<<c->nkbtrip, 256, 0, c->stream>>>(g, e, c->kb_width, c->kb_rcut, c->d_xq1,
                                                   c->d_W3, c->d_xyz, c->d_nu, c->d_kbtrip, ne,
                                                   c->d_Pphi);
  }
  // projector rows in the orthogonalized basis
  if ((s = efe_alloc(c, (void **)&c->d_Ptil, (int64_t)np * ne * 8))) return s;
  if (np > 0 && ne > 0)
    k_ptilde<<<np, 256, ne * 8, c->stream>>>(nf, ne, c->d_kbnode_ptr, c->d_kbnode, c->d_Pc_am,
                                             c->d_nm_ptr, c->d_nm_atom, c->d_nm_src, c->d_C_am,
                                             c->d_Pphi, c->d_Ptil);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

efe_status efe_launch_local_potential(efe_ctx *c, double *vq) {
  const MeshGeo g = mesh_geo(c);
  k_local_potential<<<cdiv(c->n_qpts, 256), 256, 0, c->stream>>>(
      g, c->d_xq1, c->natoms, c->d_xyz, c->d_Zs, c->loc_rc, c->loc_amp, c->loc_rg, vq);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

efe_status efe_build_operators(efe_ctx *c, const double *vq, int precisions) {
  efe_status s;
  const MeshGeo g = mesh_geo(c);
  const EnrParam e = enr_param(c);
  const int nf = c->nf;
  const int64_t ne = c->n_enr;
  const int64_t tiles = c->n_cells * c->RB * c->KS * 64;
  if (!c->d_vq && (s = efe_alloc(c, (void **)&c->d_vq, c->n_qpts * 8))) return s;
  k_copy<<<cdiv(c->n_qpts, 256), 256, 0, c->stream>>>(c->n_qpts, vq, c->d_vq);
  if (!c->d_Htile64 && (s = efe_alloc(c, (void **)&c->d_Htile64, tiles * 8))) return s;
  const bool want32 = precisions & (1 << EFE_FP32);
  const bool want16 = precisions & (1 << EFE_BF16);
  if (want32 && !c->d_Htile32 && (s = efe_alloc(c, (void **)&c->d_Htile32, tiles * 4))) return s;
  const int64_t tiles16 = c->n_cells * c->RB * c->KS32 * 64 * 8;
  if (want16 && !c->d_Htile16 && (s = efe_alloc(c, (void **)&c->d_Htile16, tiles16 * 2))) return s;
  const int KQ8 = (int)cdiv(cdiv(c->nqp, 4), 8) * 8;   // quadrature k steps, padded
  const size_t shm = (size_t)KQ8 * 64 * 8;
  if (shm > 64 * 1024) EFE_FAIL(c, EFE_EINVAL, "too many Gauss points per cell");
  k_build_hcell<<<c->n_cells * c->RB, 256, shm, c->stream>>>(
      c->nloc, c->nqp, c->RB, c->KS, KQ8, c->d_N3, c->d_W3, c->d_K, c->d_vq, c->d_Htile64,
      want32 ? c->d_Htile32 : nullptr);
  if (want16)
    k_tile_bf16<<<cdiv(tiles16, 256), 256, 0, c->stream>>>(c->n_cells, c->RB, c->KS, c->KS32,
                                                           c->d_Htile64, c->d_Htile16);
  c->have32 = want32;
  c->have16 = want16;
  if (nf > 0 && c->npairs > 0) {
    const int64_t ns = c->n_snodes * nf;
    const size_t pb = (size_t)c->npairs * c->nloc * nf * 8;   // support pairs
    if (!c->d_B_pair && (s = efe_alloc(c, (void **)&c->d_B_pair, pb))) return s;
    if (!c->d_Hee && (s = efe_alloc(c, (void **)&c->d_Hee, ne * ne * 8))) return s;
    const int64_t tT = 16 * (int64_t)c->RB * c->n_epad, tE = 4 * (int64_t)c->KS * c->n_epad;
    if (!c->d_Et64 && (s = efe_alloc(c, (void **)&c->d_Et64, tT * 8))) return s;
    if (!c->d_Ee64 && (s = efe_alloc(c, (void **)&c->d_Ee64, tE * 8))) return s;
    if (want32 && !c->d_Et32 && (s = efe_alloc(c, (void **)&c->d_Et32, tT * 4))) return s;
    if (want32 && !c->d_Ee32 && (s = efe_alloc(c, (void **)&c->d_Ee32, tE * 4))) return s;
    k_copy<<<cdiv(ns, 256), 256, 0, c->stream>>>(ns, c->d_Bkin_am, c->d_B_am);
    const int KQ = (int)cdiv(c->nqp, 4);
    k_enr_pair_proj_v<<<c->npairs, 256, (size_t)KQ * 64 * 8, c->stream>>>(
        g, e, c->d_xq1, c->d_W3, c->d_N3, c->d_xyz, c->d_nu, c->d_pair_atom, c->d_pair_cell,
        c->d_pair_lmap, c->d_vq, KQ, c->d_B_am, c->d_Bkin_pair, c->d_B_pair);
    k_copy<<<cdiv(ne * ne, 256), 256, 0, c->stream>>>(ne * ne, c->d_Hpp_kin, c->d_Hpp);
    if (c->ntrip > 0)
      k_enr_pp<false><<<c->ntrip, 128, 0, c->stream>>>(g, e, c->d_xq1, c->d_W3, c->d_xyz,
                                                       c->d_nu, c->d_trip, c->d_vq, ne, nullptr,
                                                       c->d_Hpp);
    k_symmetrize<<<cdiv(ne * ne, 256), 256, 0, c->stream>>>(ne, c->d_Hpp);
    // coupling of the orthogonalized basis: E_c per cell, then
    // H^E_ee = H^phiphi - C B^T - sum_c E_c C_c^T
    k_build_E<<<c->n_cells * c->max_rbe, 256, 0, c->stream>>>(
        c->nloc, c->RB, c->KS, nf, c->max_rbe, c->d_Htile64, c->d_cell_eptr, c->d_cell_epair,
        c->d_cell_noff, c->d_cpair_lmap, c->d_cpair_spair, c->d_C_am, c->d_B_pair, c->d_Et64,
        c->d_Ee64, want32 ? c->d_Et32 : nullptr, want32 ? c->d_Ee32 : nullptr);
    k_hee_rows<<<ne, 256, ne * 8, c->stream>>>(nf, ne, c->d_snode_ptr, c->d_snode, c->d_nm_ptr,
                                               c->d_nm_atom, c->d_nm_src, c->d_C_am, c->d_B_am,
                                               c->d_Hpp, c->d_Hee);
    k_hee_cells<<<c->n_cells * c->max_rbe, 256, 0, c->stream>>>(
        c->nloc, c->KS, nf, c->max_rbe, ne, c->d_cell_eptr, c->d_cell_epair, c->d_cell_noff,
        c->d_cpair_atom, c->d_cpair_lmap, c->d_C_am, c->d_Ee64, c->d_Hee);
    k_symmetrize<<<cdiv(ne * ne, 256), 256, 0, c->stream>>>(ne, c->d_Hee);
  }
  HIPCHK(c, hipGetLastError());
  c->have_potential = true;
  return EFE_OK;
}
