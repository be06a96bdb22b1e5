// Rayleigh-Ritz in FP64 (Eq. projectedKSEig) with the exact overlap M^E
// (Sec. III.B: the approximate inverse is used only inside the filter).
//
//   W  = H V                      (column chunks of the cell GEMM's width)
//   S  = V^T M V  (lumped mass on CFE rows, M^ee on enrichment rows)
//   Hp = V^T W
//   S = L L^T, A = L^-1 Hp L^-T, A = Q Lambda Q^T (block Jacobi), R = L^-T Q:
//   Hp R = S R Lambda, R^T S R = I, ascending Lambda
//   V <- V R, W <- W R (row blocks, in place),
//   resnorm_j = ||W e_j - lambda_j M V e_j||
// Every product runs on the FP64 matrix cores (dense.hip).
#include <cmath>

#include "efe_device.h"

__global__ void k_resnorm(int64_t n_nodes, int64_t rows, int N, const double *__restrict__ W,
                          const double *__restrict__ V, int64_t ldv,
                          const double *__restrict__ m_int,
                          const double *__restrict__ MVE, const double *__restrict__ lam,
                          double *__restrict__ out) {
  __shared__ double red[4][64];
  const int j = blockIdx.y * 64 + threadIdx.x;
  double acc = 0.0;
  if (j < N) {
    for (int64_t r = blockIdx.x * 4 + threadIdx.y; r < rows; r += (int64_t)gridDim.x * 4) {
      const double mv = r < n_nodes ? m_int[r] * V[r * ldv + j] : MVE[(r - n_nodes) * N + j];
      const double w = (r < n_nodes && m_int[r] == 0.0) ? 0.0 : W[r * N + j];
      const double d = w - lam[j] * mv;
      acc += d * d;
    }
  }
  red[threadIdx.y][threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.y == 0 && j < N)
    atomicAdd(&out[j], red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                           red[3][threadIdx.x]);
}

__global__ void k_sqrt_inplace(int n, double *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = sqrt(x[i]);
}

// V[r0 + r][j] <- T[r][j] (boundary rows zero)
__global__ void k_copy_masked(int64_t r0, int64_t n_nodes, int64_t nr, int N,
                              const double *__restrict__ minv, const double *__restrict__ T,
                              double *__restrict__ V, int64_t ld) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= nr * N) return;
  const int64_t r = idx / N, g = r0 + r;
  const int j = idx % N;
  V[r * ld + j] = (g < n_nodes && minv[g] == 0.0) ? 0.0 : T[idx];
}

// rows of the in-place rotation per pass
static int64_t rot_rows(int32_t N) { return std::max<int64_t>(64, (int64_t)(256 << 20) / (8 * N)); }

extern "C" efe_status efe_rayleigh_ritz(efe_ctx *c, double *V, int32_t N, int64_t ld,
                                        double *lambda, double *resnorm) {
  if (!c) return EFE_EINVAL;
  if (!V || !lambda || N < 1 || ld < N) EFE_FAIL(c, EFE_EINVAL, "bad arguments");
  if (!c->have_potential) EFE_FAIL(c, EFE_ESTATE, "no potential set");
  efe_status s;
  const int64_t rows = c->rows, nn = c->n_nodes, ne = c->n_enr;
  const int64_t rb = std::min<int64_t>(rows, rot_rows(N));
  const int64_t N2 = (int64_t)N * N;
  double *W, *T, *MVE, *S, *Hp, *Li, *T1, *Qe, *R, *work;
  int *iwork, *flag;
  if ((s = efe_ws(c, 5, (size_t)rows * N * 8, (void **)&W))) return s;
  if ((s = efe_ws(c, 3, (size_t)rb * N * 8, (void **)&T))) return s;
  if ((s = efe_ws(c, 6, (size_t)std::max<int64_t>(ne, 1) * N * 8, (void **)&MVE))) return s;
  if ((s = efe_ws(c, 10, (size_t)6 * N2 * 8 + 256, (void **)&S))) return s;
  Hp = S + N2;
  Li = Hp + N2;
  T1 = Li + N2;
  Qe = T1 + N2;
  R = Qe + N2;
  flag = (int *)(R + N2);
  if ((s = efe_ws(c, 13, efe_syev_work(N) * 8, (void **)&work))) return s;
  if ((s = efe_ws(c, 14, efe_syev_iwork(N) * sizeof(int), (void **)&iwork))) return s;
  const int t_rr = efe_timer_begin(c, EFE_T_RR);
  // W = H V, chunk by chunk
  for (int32_t j0 = 0; j0 < N; j0 += EFE_COL_CHUNK) {
    const int32_t nc = std::min<int32_t>(EFE_COL_CHUNK, N - j0);
    if ((s = efe_apply_H_internal(c, V + j0, ld, nullptr, V + nn * ld + j0, ld, W + j0, N, nc,
                                  EFE_FP64)))
      return s;
  }
  // S = V^T M V, Hp = V^T W: tall-skinny products (N x N from all rows), the
  // sum over rows split across work-groups so that the launch fills the
  // chip; both are symmetric (H^E is), so only the upper triangle is formed
  HIPCHK(c, hipMemsetAsync(S, 0, (size_t)2 * N2 * 8, c->stream));
  if ((s = efe_gram_sym(c, N, nn, V, ld, V, ld, S, N, c->d_m_int))) return s;
  if (ne) {
    if ((s = efe_dgemm(c, false, false, ne, N, ne, 1.0, c->d_Mee, ne, V + nn * ld, ld, 0.0, MVE,
                       N)))
      return s;
    if ((s = efe_gram_sym(c, N, ne, V + nn * ld, ld, MVE, N, S, N))) return s;
  }
  if ((s = efe_gram_sym(c, N, nn, V, ld, W, N, Hp, N))) return s;
  if (ne && (s = efe_gram_sym(c, N, ne, V + nn * ld, ld, W + nn * N, N, Hp, N))) return s;
  if ((s = efe_mirror_upper(c, N, S, N)) || (s = efe_mirror_upper(c, N, Hp, N))) return s;
  // S = L L^T; Hp <- L^-1 Hp L^-T
  HIPCHK(c, hipMemsetAsync(flag, 0, sizeof(int), c->stream));
  if ((s = efe_potrf(c, N, S, N, flag))) return s;
  int hflag = 0;
  HIPCHK(c, hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (hflag) EFE_FAIL(c, EFE_ENUMERIC, "overlap of the block is not positive definite");
  if ((s = efe_trtri_lower(c, N, S, N, Li, N))) return s;
  if ((s = efe_dgemm(c, false, false, N, N, N, 1.0, Li, N, Hp, N, 0.0, T1, N))) return s;
  if ((s = efe_dgemm(c, false, true, N, N, N, 1.0, T1, N, Li, N, 0.0, Hp, N))) return s;
  // Hp = Q Lambda Q^T; R = L^-T Q
  if ((s = efe_syev_jacobi(c, N, Hp, N, lambda, Qe, work, iwork, &c->rr_sweeps))) return s;
  if ((s = efe_dgemm(c, true, false, N, N, N, 1.0, Li, N, Qe, N, 0.0, R, N))) return s;
  // V <- V R, W <- W R, row block by row block through T
  for (int64_t r0 = 0; r0 < rows; r0 += rb) {
    const int64_t nr = std::min<int64_t>(rb, rows - r0);
    if ((s = efe_dgemm(c, false, false, nr, N, N, 1.0, V + r0 * ld, ld, R, N, 0.0, T, N))) return s;
    k_copy_masked<<<cdiv(nr * N, 256), 256, 0, c->stream>>>(r0, nn, nr, N, c->d_minv, T, V + r0 * ld,
                                                           ld);
    if (resnorm) {
      if ((s = efe_dgemm(c, false, false, nr, N, N, 1.0, W + r0 * N, N, R, N, 0.0, T, N))) return s;
      k_copy_masked<<<cdiv(nr * N, 256), 256, 0, c->stream>>>(r0, nn, nr, N, c->d_minv, T,
                                                             W + r0 * N, N);
    }
  }
  if (resnorm) {
    if (ne && (s = efe_dgemm(c, false, false, ne, N, ne, 1.0, c->d_Mee, ne, V + nn * ld, ld, 0.0,
                             MVE, N)))
      return s;
    HIPCHK(c, hipMemsetAsync(resnorm, 0, N * 8, c->stream));
    dim3 blkd(64, 4), grd((unsigned)std::min<int64_t>(cdiv(rows, 4), 4096), cdiv(N, 64));
    k_resnorm<<<grd, blkd, 0, c->stream>>>(nn, rows, N, W, V, ld, c->d_m_int, MVE, lambda, resnorm);
    k_sqrt_inplace<<<cdiv(N, 256), 256, 0, c->stream>>>(N, resnorm);
  }
  efe_timer_end(c, EFE_T_RR, t_rr);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}
