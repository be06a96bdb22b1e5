// Rayleigh-Ritz in FP64 (Eq. projectedKSEig) with the exact overlap M^E
// (Sec. III.B: the approximate inverse is used only inside the filter).
//
//   W  = H V
//   S  = V^T M V  (lumped mass on CFE rows, M^ee on enrichment rows)
//   Hp = V^T W
//   S = L L^T (Cholesky), Hh = L^-1 Hp L^-T, Hh = Q Lambda Q^T (cyclic Jacobi),
//   R = L^-T Q (ascending Lambda),  V <- V R,  resnorm_j = ||W R e_j - lambda_j M V R e_j||
// The small dense steps run in one work-group on matrices held in global
// memory (they are O(N^3) with N the block width and stay in L2).
#include <cmath>

#include "efe_device.h"

__device__ inline void block_sync() { __syncthreads(); }

// One work-group: Cholesky of S (lower, in place), Hh = L^-1 Hp L^-T (in T),
// Jacobi on Hh with eigenvectors in Q, sort, R = L^-T Q_sorted (in R).
__global__ __launch_bounds__(1024) void k_rr_small(int N, double *__restrict__ S,
                                                   double *__restrict__ Hp, double *__restrict__ T,
                                                   double *__restrict__ Q, double *__restrict__ R,
                                                   double *__restrict__ lam, int *__restrict__ info,
                                                   int max_sweeps) {
  __shared__ int s_fail;
  __shared__ double red[1024], red2[1024];
  __shared__ double cs_c[1024], cs_s[1024];
  __shared__ int cs_p[1024], cs_q[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  if (tid == 0) s_fail = 0;
  block_sync();
  // ---- Cholesky S = L L^T (lower triangle)
  for (int k = 0; k < N; ++k) {
    if (tid == 0) {
      const double d = S[(int64_t)k * N + k];
      if (!(d > 0.0) || !isfinite(d)) s_fail = 1;
      else S[(int64_t)k * N + k] = sqrt(d);
    }
    block_sync();
    if (s_fail) {
      if (tid == 0) *info = 1 + k;
      return;
    }
    const double lkk = S[(int64_t)k * N + k];
    for (int i = k + 1 + tid; i < N; i += nt) S[(int64_t)i * N + k] /= lkk;
    block_sync();
    const int m = N - k - 1;
    for (int64_t idx = tid; idx < (int64_t)m * m; idx += nt) {
      const int i = k + 1 + (int)(idx / m), j = k + 1 + (int)(idx % m);
      if (j <= i) S[(int64_t)i * N + j] -= S[(int64_t)i * N + k] * S[(int64_t)j * N + k];
    }
    block_sync();
  }
  // ---- X = L^-1 Hp, column-parallel forward substitution (X overwrites Hp)
  for (int j = tid; j < N; j += nt)
    for (int i = 0; i < N; ++i) {
      double acc = Hp[(int64_t)i * N + j];
      for (int k = 0; k < i; ++k) acc -= S[(int64_t)i * N + k] * Hp[(int64_t)k * N + j];
      Hp[(int64_t)i * N + j] = acc / S[(int64_t)i * N + i];
    }
  block_sync();
  // T = X^T, then T <- L^-1 T
  for (int64_t idx = tid; idx < (int64_t)N * N; idx += nt) {
    const int i = idx / N, j = idx % N;
    T[idx] = Hp[(int64_t)j * N + i];
  }
  block_sync();
  for (int j = tid; j < N; j += nt)
    for (int i = 0; i < N; ++i) {
      double acc = T[(int64_t)i * N + j];
      for (int k = 0; k < i; ++k) acc -= S[(int64_t)i * N + k] * T[(int64_t)k * N + j];
      T[(int64_t)i * N + j] = acc / S[(int64_t)i * N + i];
    }
  block_sync();
  for (int64_t idx = tid; idx < (int64_t)N * N; idx += nt) {
    const int i = idx / N, j = idx % N;
    if (j > i) {
      const double v = 0.5 * (T[(int64_t)i * N + j] + T[(int64_t)j * N + i]);
      T[(int64_t)i * N + j] = v;
      T[(int64_t)j * N + i] = v;
    }
    Q[idx] = (i == j) ? 1.0 : 0.0;
  }
  block_sync();
  // ---- cyclic Jacobi, round-robin pairing (Np even, index >= N is a dummy)
  const int Np = N + (N & 1);
  const int npair = Np / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int r = 0; r < Np - 1; ++r) {
      for (int i = tid; i < npair; i += nt) {
        const int top = (i == 0) ? 0 : 1 + (i - 1 + r) % (Np - 1);
        const int bot = 1 + (Np - 2 - i + r) % (Np - 1);
        int p = min(top, bot), q = max(top, bot);
        double c = 1.0, s = 0.0;
        if (q < N) {
          const double app = T[(int64_t)p * N + p], aqq = T[(int64_t)q * N + q],
                       apq = T[(int64_t)p * N + q];
          if (apq != 0.0) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        } else {
          q = -1;
        }
        cs_c[i] = c;
        cs_s[i] = s;
        cs_p[i] = p;
        cs_q[i] = q;
      }
      block_sync();
      // rows p, q of T
      for (int64_t idx = tid; idx < (int64_t)npair * N; idx += nt) {
        const int i = idx / N, j = idx % N;
        const int p = cs_p[i], q = cs_q[i];
        if (q < 0 || cs_s[i] == 0.0) continue;
        const double c = cs_c[i], s = cs_s[i];
        const double ap = T[(int64_t)p * N + j], aq = T[(int64_t)q * N + j];
        T[(int64_t)p * N + j] = c * ap - s * aq;
        T[(int64_t)q * N + j] = s * ap + c * aq;
      }
      block_sync();
      // columns p, q of T and Q
      for (int64_t idx = tid; idx < (int64_t)npair * N; idx += nt) {
        const int i = idx / N, j = idx % N;
        const int p = cs_p[i], q = cs_q[i];
        if (q < 0 || cs_s[i] == 0.0) continue;
        const double c = cs_c[i], s = cs_s[i];
        double ap = T[(int64_t)j * N + p], aq = T[(int64_t)j * N + q];
        T[(int64_t)j * N + p] = c * ap - s * aq;
        T[(int64_t)j * N + q] = s * ap + c * aq;
        ap = Q[(int64_t)j * N + p];
        aq = Q[(int64_t)j * N + q];
        Q[(int64_t)j * N + p] = c * ap - s * aq;
        Q[(int64_t)j * N + q] = s * ap + c * aq;
      }
      block_sync();
    }
    // convergence: off-diagonal mass against the total
    double off = 0.0, tot = 0.0;
    for (int64_t idx = tid; idx < (int64_t)N * N; idx += nt) {
      const double v = T[idx] * T[idx];
      tot += v;
      if (idx / N != idx % N) off += v;
    }
    red[tid] = off;
    red2[tid] = tot;
    block_sync();
    for (int st = nt / 2; st > 0; st >>= 1) {
      if (tid < st) {
        red[tid] += red[tid + st];
        red2[tid] += red2[tid + st];
      }
      block_sync();
    }
    const bool done = red[0] <= 1e-30 * red2[0];
    block_sync();
    if (done) break;
  }
  // ---- sort eigenvalues ascending (rank by value, ties by index)
  for (int i = tid; i < N; i += nt) {
    const double li = T[(int64_t)i * N + i];
    int rank = 0;
    for (int j = 0; j < N; ++j) {
      const double lj = T[(int64_t)j * N + j];
      if (lj < li || (lj == li && j < i)) ++rank;
    }
    lam[rank] = li;
    for (int k = 0; k < N; ++k) Hp[(int64_t)k * N + rank] = Q[(int64_t)k * N + i];
  }
  block_sync();
  // ---- R = L^-T Qs (back substitution, column-parallel)
  for (int j = tid; j < N; j += nt)
    for (int i = N - 1; i >= 0; --i) {
      double acc = Hp[(int64_t)i * N + j];
      for (int k = i + 1; k < N; ++k) acc -= S[(int64_t)k * N + i] * R[(int64_t)k * N + j];
      R[(int64_t)i * N + j] = acc / S[(int64_t)i * N + i];
    }
  if (tid == 0) *info = 0;
}

// column sums of squares of W - lam_j MV (CFE rows: MV = m V), enrichment rows
// use MVE (n_enr x N)
__global__ void k_resnorm(int64_t n_nodes, int64_t rows, int N, const double *__restrict__ W,
                          const double *__restrict__ V, const double *__restrict__ m_int,
                          const double *__restrict__ MVE, const double *__restrict__ lam,
                          double *__restrict__ out) {
  __shared__ double red[4][64];
  const int j = blockIdx.y * 64 + threadIdx.x;
  double acc = 0.0;
  if (j < N) {
    for (int64_t r = blockIdx.x * 4 + threadIdx.y; r < rows; r += (int64_t)gridDim.x * 4) {
      const double mv = r < n_nodes ? m_int[r] * V[r * N + j] : MVE[(r - n_nodes) * N + j];
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

// V[r][j] <- Vn[r][j] (boundary rows zero)
__global__ void k_copy_masked(int64_t n_nodes, int64_t rows, int N, const double *__restrict__ minv,
                              const double *__restrict__ Vn, double *__restrict__ V, int64_t ld) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= rows * N) return;
  const int64_t r = idx / N;
  const int j = idx % N;
  V[r * ld + j] = (r < n_nodes && minv[r] == 0.0) ? 0.0 : Vn[idx];
}

extern "C" efe_status efe_rayleigh_ritz(efe_ctx *c, double *V, int32_t N, int64_t ld,
                                        double *lambda, double *resnorm) {
  if (!c) return EFE_EINVAL;
  if (!V || !lambda || N < 1 || ld < N) EFE_FAIL(c, EFE_EINVAL, "bad arguments");
  if (N > 2048) EFE_FAIL(c, EFE_EINVAL, "block wider than 2048 columns");
  if (!c->have_potential) EFE_FAIL(c, EFE_ESTATE, "no potential set");
  efe_status s;
  const int64_t rows = c->rows, nn = c->n_nodes, ne = c->n_enr;
  const int64_t blk = rows * N;
  double *W, *Vn, *Wn, *MVE, *S, *Hp, *T, *Q, *R;
  int *info;
  if ((s = efe_ws(c, 5, blk * 8, (void **)&W))) return s;
  if ((s = efe_ws(c, 3, blk * 8, (void **)&Vn))) return s;
  if ((s = efe_ws(c, 4, blk * 8, (void **)&Wn))) return s;
  if ((s = efe_ws(c, 6, (size_t)std::max<int64_t>(ne, 1) * N * 8, (void **)&MVE))) return s;
  if ((s = efe_ws(c, 10, (size_t)5 * N * N * 8 + 64, (void **)&S))) return s;
  Hp = S + (int64_t)N * N;
  T = Hp + (int64_t)N * N;
  Q = T + (int64_t)N * N;
  R = Q + (int64_t)N * N;
  info = (int *)(R + (int64_t)N * N);
  const int t_rr = efe_timer_begin(c, EFE_T_RR);
  // W = H V
  if ((s = efe_apply_H_internal(c, V, ld, nullptr, V + nn * ld, ld, W, N, N, EFE_FP64))) return s;
  // S = V^T M V, Hp = V^T W
  HIPCHK(c, hipMemsetAsync(S, 0, (size_t)2 * N * N * 8, c->stream));
  if ((s = efe_gram(c, N, N, nn, 1.0, V, ld, V, ld, c->d_m_int, S, N))) return s;
  if (ne) {
    if ((s = efe_gemm(c, false, false, ne, N, ne, 1.0, c->d_Mee, ne, V + nn * ld, ld, 0.0, MVE, N)))
      return s;
    if ((s = efe_gram(c, N, N, ne, 1.0, V + nn * ld, ld, MVE, N, nullptr, S, N))) return s;
  }
  if ((s = efe_gram(c, N, N, nn, 1.0, V, ld, W, N, nullptr, Hp, N))) return s;
  if (ne && (s = efe_gram(c, N, N, ne, 1.0, V + nn * ld, ld, W + nn * N, N, nullptr, Hp, N)))
    return s;
  k_rr_small<<<1, 1024, 0, c->stream>>>(N, S, Hp, T, Q, R, lambda, info, 40);
  HIPCHK(c, hipGetLastError());
  int hinfo = 0;
  HIPCHK(c, hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (hinfo) EFE_FAIL(c, EFE_ENUMERIC, "overlap of the block is not positive definite");
  // V <- V R, W <- W R
  if ((s = efe_gemm(c, false, false, rows, N, N, 1.0, V, ld, R, N, 0.0, Vn, N))) return s;
  if (resnorm) {
    if ((s = efe_gemm(c, false, false, rows, N, N, 1.0, W, N, R, N, 0.0, Wn, N))) return s;
    if (ne && (s = efe_gemm(c, false, false, ne, N, ne, 1.0, c->d_Mee, ne, Vn + nn * N, N, 0.0,
                            MVE, N)))
      return s;
    HIPCHK(c, hipMemsetAsync(resnorm, 0, N * 8, c->stream));
    dim3 blkd(64, 4), grd((unsigned)std::min<int64_t>(cdiv(rows, 4), 4096), cdiv(N, 64));
    k_resnorm<<<grd, blkd, 0, c->stream>>>(nn, rows, N, Wn, Vn, c->d_m_int, MVE, lambda, resnorm);
    k_sqrt_inplace<<<cdiv(N, 256), 256, 0, c->stream>>>(N, resnorm);
  }
  k_copy_masked<<<cdiv(blk, 256), 256, 0, c->stream>>>(nn, rows, N, c->d_minv, Vn, V, ld);
  efe_timer_end(c, EFE_T_RR, t_rr);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}
