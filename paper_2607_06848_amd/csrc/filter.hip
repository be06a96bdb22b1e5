// Chebyshev filtering (Sec. III.B) and the Lanczos spectrum bound.
//
// Residual filter (Eqs. residual, residualapprox, with the coefficients that
// follow from inserting Eq. ChebyRecur into the definition of Z_k):
//   G   = H V - M V Lambda
//   Z_1 = (s_1/e) G,  Z_0 = 0
//   Z_k = (2 s_k/e) H M~^-1 Z_{k-1} - (2 c s_k/e) Z_{k-1} - s_{k-1} s_k Z_{k-2}
//         + (2 s_k/e) G C_{k-1}(Lambda)
//   V  <- M~^-1 Z_m + V C_m(Lambda)
// The CFE part of M~^-1 (1/m) is folded into the gather of the H apply; the
// enrichment part is a batched nf x nf block product.  Z_k overwrites Z_{k-2}.
#include <cmath>
#include <vector>

#include "efe_device.h"

// sigma_1 = e / (a_min - c), sigma_k = 1 / (2 / sigma_1 - sigma_{k-1})
__global__ void k_sigma_table(int m, double a, double b, double a_min, double *__restrict__ sig) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double cc = 0.5 * (a + b), e = 0.5 * (b - a);
  sig[0] = 0.0;
  sig[1] = e / (a_min - cc);
  for (int k = 2; k <= m; ++k) sig[k] = 1.0 / (2.0 / sig[1] - sig[k - 1]);
}

// C_k(lambda_j), k = 0..m, by the scalar recurrence (one thread per column)
__global__ void k_cheb_table(int m, int ncols, const double *__restrict__ lam, double c, double e,
                             const double *__restrict__ sig, double *__restrict__ T) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= ncols) return;
  const double x = lam[j];
  double cm2 = 1.0, cm1 = sig[1] * (x - c) / e;
  T[j] = 1.0;
  if (m >= 1) T[ncols + j] = cm1;
  for (int k = 2; k <= m; ++k) {
    const double ck = (2.0 * sig[k] / e) * (x - c) * cm1 - sig[k - 1] * sig[k] * cm2;
    T[(int64_t)k * ncols + j] = ck;
    cm2 = cm1;
    cm1 = ck;
  }
}

// G = W - MV diag(lam) over all rows (ld of G, W, MV = ncols); Z = s G
// (MV and Zp may be the same buffer)
__global__ void k_residual_init(int64_t rows, int ncols, const double *__restrict__ W,
                                const double *MV, const double *__restrict__ lam, double s1e,
                                double *__restrict__ G, double *__restrict__ Z, double *Zp) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= rows * ncols) return;
  const double mv = MV[idx];
  const double g = W[idx] - mv * lam[idx % ncols];
  G[idx] = g;
  Z[idx] = s1e * g;
  Zp[idx] = 0.0;
}

// V <- w_r Z + V Cl on CFE rows (w = 1/m), enrichment rows use ZE = M~ee^-1 Z^E
__global__ void k_vout(int64_t n_nodes, int64_t rows, int ncols, const double *__restrict__ minv,
                       const double *__restrict__ Z, const double *__restrict__ ZE,
                       const double *__restrict__ Cl, double *__restrict__ V, int64_t ld) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= rows * ncols) return;
  const int64_t r = idx / ncols;
  const int j = idx % ncols;
  const double y = r < n_nodes ? minv[r] * Z[idx] : ZE[(r - n_nodes) * ncols + j];
  double v = V[r * ld + j] * Cl[j];
  if (r < n_nodes && minv[r] == 0.0) v = 0.0;
  V[r * ld + j] = y + v;
}

// standard filter step on A = M~^-1 H:
// Yn = a (AY - c Y) + gam Yp with AY = (1/m) W on CFE rows, WE on enrichment rows
__global__ void k_std_step(int64_t n_nodes, int64_t rows, int ncols, double a, double cc,
                           double gam, const double *__restrict__ minv,
                           const double *__restrict__ W, const double *__restrict__ WE,
                           const double *__restrict__ Y, const double *Yp, double *Yn) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= rows * ncols) return;
  const int64_t r = idx / ncols;
  const double ay = r < n_nodes ? minv[r] * W[idx] : WE[idx - n_nodes * ncols];
  const double yp = Yp ? Yp[idx] : 0.0;
  Yn[idx] = a * (ay - cc * Y[idx]) + gam * yp;
}

__global__ void k_copy_in(int64_t rows, int ncols, const double *__restrict__ src, int64_t lds,
                          double *__restrict__ dst, int64_t ldd) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= rows * ncols) return;
  const int64_t r = idx / ncols;
  const int j = idx % ncols;
  dst[r * ldd + j] = src[r * lds + j];
}

// ------------------------------------------------------------------ filter
// One column chunk of the filter (the filter acts on every column on its own,
// so chunks of a wide block give the same result as one pass over it).
static efe_status filter_chunk(efe_ctx *c, double *V, const double *lambda, int32_t ncols,
                               int64_t ld, const efe_cheb_params *prm) {
  efe_status s;
  const int m = prm->degree;
  const double cc = 0.5 * (prm->a + prm->b), e = 0.5 * (prm->b - prm->a);
  std::vector<double> sig(m + 1, 0.0);
  sig[1] = e / (prm->a_min - cc);
  for (int k = 2; k <= m; ++k) sig[k] = 1.0 / (2.0 / sig[1] - sig[k - 1]);
  const int64_t rows = c->rows, nn = c->n_nodes;
  const int64_t blk = rows * ncols;
  double *G, *Za, *Zb, *W, *XE, *Cl, *dsig;
  if ((s = efe_ws(c, 2, blk * 8, (void **)&G))) return s;
  if ((s = efe_ws(c, 3, blk * 8, (void **)&Za))) return s;
  if ((s = efe_ws(c, 4, blk * 8, (void **)&Zb))) return s;
  if ((s = efe_ws(c, 5, blk * 8, (void **)&W))) return s;
  if ((s = efe_ws(c, 6, (size_t)std::max<int64_t>(c->n_enr, 1) * ncols * 8, (void **)&XE))) return s;
  if ((s = efe_ws(c, 7, (size_t)(m + 1) * ncols * 8, (void **)&Cl))) return s;
  if ((s = efe_ws(c, 8, (size_t)(m + 1) * 8, (void **)&dsig))) return s;
  // the same table on the device (the same IEEE operations in the same order
  // as the host's, so both hold identical values)
  k_sigma_table<<<1, 1, 0, c->stream>>>(m, prm->a, prm->b, prm->a_min, dsig);
  const int T = 256;
  const int64_t nb = cdiv(blk, T);

  if (prm->mode == EFE_FILTER_STANDARD) {
    // Y_0 = V (copied to Za), Y_1 = (s1/e)(A V - c V), Y_k = (2 s_k/e)(A - c) Y_{k-1} - s s Y_{k-2}
    k_copy_in<<<nb, T, 0, c->stream>>>(rows, ncols, V, ld, Za, ncols);
    double *Yp = nullptr, *Yc = Za, *Yn = Zb;
    for (int k = 1; k <= m; ++k) {
      if ((s = efe_apply_H_internal(c, Yc, ncols, nullptr, Yc + nn * ncols, ncols, W, ncols, ncols,
                                    prm->prec)))
        return s;
      if ((s = efe_enr_block_inv(c, W + nn * ncols, ncols, XE, ncols, ncols))) return s;
      const double a = (k == 1 ? 1.0 : 2.0) * sig[k] / e;
      const double gam = k == 1 ? 0.0 : -sig[k - 1] * sig[k];
      k_std_step<<<nb, T, 0, c->stream>>>(nn, rows, ncols, a, cc, gam, c->d_minv, W, XE, Yc,
                                          k == 1 ? nullptr : Yp, Yn);
      double *t = Yp ? Yp : G;
      Yp = Yc;
      Yc = Yn;
      Yn = t;
    }
    k_copy_in<<<nb, T, 0, c->stream>>>(rows, ncols, Yc, ncols, V, ld);
    HIPCHK(c, hipGetLastError());
    return EFE_OK;
  }

  k_cheb_table<<<cdiv(ncols, 64), 64, 0, c->stream>>>(m, ncols, lambda, cc, e, dsig, Cl);
  // G = H V - M V Lambda (MV staged in Zb)
  if ((s = efe_apply_H_internal(c, V, ld, nullptr, V + nn * ld, ld, W, ncols, ncols, EFE_FP64)))
    return s;
  if ((s = efe_apply_M_internal(c, V, ld, Zb, ncols, ncols))) return s;
  double *Zc = Za, *Zp = Zb;
  k_residual_init<<<nb, T, 0, c->stream>>>(rows, ncols, W, Zb, lambda, sig[1] / e, G, Zc, Zp);
  for (int k = 2; k <= m; ++k) {
    if ((s = efe_enr_block_inv(c, Zc + nn * ncols, ncols, XE, ncols, ncols))) return s;
    // the recurrence's H applies run in the requested precision (G stays
    // FP64); its three affine terms enter the assembly itself: Z_k is
    // written in place of Z_{k-2}, starting from the terms and accumulating
    // alpha H M~^-1 Z_{k-1} over the colour passes
    ApplyEpilogue ep;
    ep.alpha = 2.0 * sig[k] / e;
    ep.beta = -cc * ep.alpha;
    ep.gamma = -sig[k - 1] * sig[k];
    ep.Z1 = Zc;
    ep.Z2 = Zp;
    ep.G = G;
    ep.Cl = Cl + (int64_t)(k - 1) * ncols;
    const int t = efe_timer_begin(c, EFE_T_RECUR);
    if ((s = efe_apply_H_internal(c, Zc, ncols, c->d_minv, XE, ncols, Zp, ncols, ncols, prm->prec,
                                  &ep)))
      return s;
    efe_timer_end(c, EFE_T_RECUR, t);
    std::swap(Zc, Zp);
  }
  if ((s = efe_enr_block_inv(c, Zc + nn * ncols, ncols, XE, ncols, ncols))) return s;
  k_vout<<<nb, T, 0, c->stream>>>(nn, rows, ncols, c->d_minv, Zc, XE, Cl + (int64_t)m * ncols, V, ld);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

efe_status efe_filter_check(efe_ctx *c, double *V, const double *lambda, int32_t ncols,
                            int64_t ld, const efe_cheb_params *prm) {
  if (!c) return EFE_EINVAL;
  if (!V || !prm || ncols < 0 || ld < ncols || ld < 1) EFE_FAIL(c, EFE_EINVAL, "bad arguments");
  if (prm->degree < 1) EFE_FAIL(c, EFE_EINVAL, "degree must be >= 1");
  if (!(prm->a < prm->b) || !(prm->a_min < prm->a)) EFE_FAIL(c, EFE_EINVAL, "need a_min < a < b");
  if (prm->mode != EFE_FILTER_RESIDUAL && prm->mode != EFE_FILTER_STANDARD)
    EFE_FAIL(c, EFE_EINVAL, "bad filter mode");
  if (prm->prec != EFE_FP64 && prm->prec != EFE_FP32 && prm->prec != EFE_BF16)
    EFE_FAIL(c, EFE_EINVAL, "bad filter precision");
  if (prm->mode == EFE_FILTER_RESIDUAL && !lambda) EFE_FAIL(c, EFE_EINVAL, "residual mode needs lambda");
  if (prm->prec == EFE_BF16 && c->amplification > EFE_BF16_MAX_AMPLIFICATION)
    EFE_FAIL(c, EFE_EINVAL,
             "BF16 filter refused: enrichment amplification " + std::to_string(c->amplification) +
                 " exceeds " + std::to_string(EFE_BF16_MAX_AMPLIFICATION));
  if (!c->have_potential) EFE_FAIL(c, EFE_ESTATE, "no potential set");
  return EFE_OK;
}

efe_status efe_filter_run(efe_ctx *c, double *V, const double *lambda, int32_t ncols, int64_t ld,
                          const efe_cheb_params *prm) {
  efe_status s;
  for (int32_t j0 = 0; j0 < ncols; j0 += EFE_COL_CHUNK) {
    const int32_t nc = std::min<int32_t>(EFE_COL_CHUNK, ncols - j0);
    if ((s = filter_chunk(c, V + j0, lambda ? lambda + j0 : nullptr, nc, ld, prm))) return s;
  }
  return EFE_OK;
}

extern "C" efe_status efe_cheb_filter(efe_ctx *c, double *V, const double *lambda, int32_t ncols,
                                      int64_t ld, const efe_cheb_params *prm) {
  efe_status s = efe_filter_check(c, V, lambda, ncols, ld, prm);
  if (s) return s;
  return efe_filter_run(c, V, lambda, ncols, ld, prm);
}

// ------------------------------------------------------------------ Lanczos
// out[0] = sum_r x_r y_r ; out[1] = x^T M~ x (CFE: m x^2, enrichment blocks)
__global__ void k_dot(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                      const double *__restrict__ w, double *__restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += x[i] * y[i] * (w ? w[i] : 1.0);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

// sum over atoms of x_I^T Mee_II y_I
__global__ void k_enr_block_dot(int natoms, int nf, int64_t n_enr, const double *__restrict__ Mee,
                                const double *__restrict__ x, const double *__restrict__ y,
                                double *__restrict__ out) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= natoms) return;
  double acc = 0.0;
  for (int k = 0; k < nf; ++k)
    for (int l = 0; l < nf; ++l)
      acc += x[I * nf + k] * Mee[(int64_t)(I * nf + k) * n_enr + I * nf + l] * y[I * nf + l];
  atomicAdd(out, acc);
}

// Lanczos vector update: w = u - alpha v - beta_prev v_prev; scalars on device
// sc = [alpha_j, beta_j, beta_{j-1}, ...]: out = (u - a v - b vp)
__global__ void k_lanczos_update(int64_t n, const double *__restrict__ u,
                                 const double *__restrict__ v, const double *__restrict__ vp,
                                 const double *__restrict__ alpha, const double *__restrict__ bprev,
                                 double *__restrict__ w) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  w[i] = u[i] - (*alpha) * v[i] - (bprev ? *bprev : 0.0) * vp[i];
}

__global__ void k_mask_copy(int64_t n_nodes, int64_t rows, const double *__restrict__ minv,
                            const double *__restrict__ x, double *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= rows) return;
  y[i] = (i < n_nodes && minv[i] == 0.0) ? 0.0 : x[i];
}

__global__ void k_scale_by_inv_sqrt(int64_t n, const double *__restrict__ nrm2,
                                    const double *__restrict__ x, double *__restrict__ y,
                                    double *__restrict__ beta_out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const double b = sqrt(*nrm2);
  if (i == 0 && beta_out) *beta_out = b;
  if (i < n) y[i] = x[i] / b;
}

// theta_max of the k x k tridiagonal (alpha, beta) by Sturm bisection, plus |beta_k|
__global__ void k_tridiag_bound(int k, const double *__restrict__ alpha,
                                const double *__restrict__ beta, double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < k; ++i) {
    double r = (i > 0 ? fabs(beta[i - 1]) : 0.0) + (i < k - 1 ? fabs(beta[i]) : 0.0);
    lo = fmin(lo, alpha[i] - r);
    hi = fmax(hi, alpha[i] + r);
  }
  // number of eigenvalues below x
  for (int it = 0; it < 200; ++it) {
    const double x = 0.5 * (lo + hi);
    if (!(x > lo && x < hi)) break;
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
      const double b2 = i > 0 ? beta[i - 1] * beta[i - 1] : 0.0;
      d = alpha[i] - x - (i > 0 ? b2 / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++cnt;
    }
    if (cnt >= k) hi = x;   // all eigenvalues below x
    else lo = x;
  }
  out[0] = hi + fabs(beta[k - 1]);
}

// w -= sum_{i <= j} c_i V_i (classical Gram-Schmidt against the Lanczos basis)
__global__ void k_reorth(int64_t n, int j, const double *__restrict__ V, int64_t ldv,
                         const double *__restrict__ c, double *__restrict__ w) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc = 0.0;
  for (int i = 0; i <= j; ++i) acc += c[i] * V[(int64_t)i * ldv + r];
  w[r] -= acc;
}

extern "C" efe_status efe_spectrum_upper_bound(efe_ctx *c, const double *v0, int32_t steps,
                                               double *b_out) {
  if (!c) return EFE_EINVAL;
  if (!v0 || !b_out || steps < 1 || steps > 1000) EFE_FAIL(c, EFE_EINVAL, "bad arguments");
  if (!c->have_potential) EFE_FAIL(c, EFE_ESTATE, "no potential set");
  efe_status s;
  const int64_t rows = c->rows, nn = c->n_nodes, ne = c->n_enr;
  double *buf, *sc;
  // the Lanczos basis V_0 .. V_{steps-1}, then u (= H v), w, x (= M~^-1 u)
  if ((s = efe_ws(c, 20, (size_t)rows * (steps + 3) * 8, (void **)&buf))) return s;
  const size_t nsc = (size_t)steps * steps + 4 * (size_t)steps + 8;
  if ((s = efe_ws(c, 21, nsc * 8, (void **)&sc))) return s;
  double *Vb = buf, *u = buf + (int64_t)steps * rows, *w = u + rows, *x = w + rows;
  double *alpha = sc, *beta = sc + steps, *nrm = sc + 2 * steps;   // nrm: steps + 1 slots
  double *coef = sc + 4 * steps + 8;                               // steps x steps
  HIPCHK(c, hipMemsetAsync(sc, 0, nsc * 8, c->stream));
  const int T = 256;
  const int nbk = (int)std::min<int64_t>(cdiv(rows, T), 1024);
  // copy of v0 without its boundary rows
  k_mask_copy<<<cdiv(rows, T), T, 0, c->stream>>>(nn, rows, c->d_minv, v0, u);
  // inner product of the M~ norm: m x y on CFE rows + atom blocks
  auto mdot = [&](const double *a, const double *b, double *out) -> efe_status {
    k_dot<<<nbk, T, 0, c->stream>>>(nn, a, b, c->d_m_int, out);
    if (ne) k_enr_block_dot<<<cdiv(c->natoms, 64), 64, 0, c->stream>>>(c->natoms, c->nf, ne, c->d_Mee,
                                                                       a + nn, b + nn, out);
    HIPCHK(c, hipGetLastError());
    return EFE_OK;
  };
  if ((s = mdot(u, u, &nrm[steps]))) return s;
  k_scale_by_inv_sqrt<<<cdiv(rows, T), T, 0, c->stream>>>(rows, &nrm[steps], u, Vb, nullptr);
  for (int j = 0; j < steps; ++j) {
    double *v = Vb + (int64_t)j * rows;
    if ((s = efe_apply_H_internal(c, v, 1, nullptr, v + nn, 1, u, 1, 1, EFE_FP64))) return s;
    // alpha_j = v^T H v
    k_dot<<<nbk, T, 0, c->stream>>>(rows, v, u, nullptr, &alpha[j]);
    if ((s = efe_apply_Minv_internal(c, u, 1, x, 1, 1))) return s;
    k_lanczos_update<<<cdiv(rows, T), T, 0, c->stream>>>(
        rows, x, v, j > 0 ? v - rows : v, &alpha[j], j > 0 ? &beta[j - 1] : nullptr, w);
    // once more against the whole basis
    double *cj = coef + (int64_t)j * steps;
    for (int i = 0; i <= j; ++i)
      if ((s = mdot(Vb + (int64_t)i * rows, w, &cj[i]))) return s;
    k_reorth<<<cdiv(rows, T), T, 0, c->stream>>>(rows, j, Vb, rows, cj, w);
    if ((s = mdot(w, w, &nrm[j]))) return s;
    // v_{j+1} = w / beta_j (the last one is not kept)
    double *vn = j + 1 < steps ? Vb + (int64_t)(j + 1) * rows : x;
    k_scale_by_inv_sqrt<<<cdiv(rows, T), T, 0, c->stream>>>(rows, &nrm[j], w, vn, &beta[j]);
  }
  double *res = sc + 4 * steps + 4;
  k_tridiag_bound<<<1, 1, 0, c->stream>>>(steps, alpha, beta, res);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(b_out, res, 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return EFE_OK;
}
