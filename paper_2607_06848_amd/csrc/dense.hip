// Dense FP64 linear algebra of Rayleigh-Ritz (Eq. projectedKSEig) on the
// matrix cores: a tiled GEMM (v_mfma_f64_16x16x4, optionally split over the
// summation index with atomic accumulation, for the tall-skinny Grams), a
// blocked Cholesky factorization, the inverse of a triangular factor and a
// two-sided block Jacobi eigensolver for the projected N x N problem.
#include <algorithm>
#include <cmath>

#include "efe_internal.h"

typedef double v4d_g __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ GEMM
// C[M x N] = alpha op(A) op(B) (+ beta C), row-major; op(A) = A (M x K, lda)
// or A^T (A stored K x M); op(B) = B (K x N) or B^T (B stored N x K); wK
// (optional) weights the sum over k.  A work-group computes a 128 x 128 tile:
// four waves of 64 x 64 (4 x 4 MFMA blocks of 16 x 16), 16-deep k slices
// staged through LDS, the next slice loaded into registers while the current
// one is multiplied.  An operand stored with its output index contiguous
// (A^T, B) sits in LDS as [k][m] rows of 144 doubles; one stored with k
// contiguous (A, B^T) as [m][k] rows of 17 doubles: either way a half-wave's
// MFMA operand read touches 32 distinct banks.  SPLIT: C += the product over
// the k range of the work-group's split (atomic adds).  TRI (square C, split
// only): only tiles on or above the diagonal; the caller mirrors them.
// Consecutive logical work-groups (the tiles of one k range, or the column
// tiles of one row panel) run on one XCD, which then reads the shared panel
// from its own L2.
constexpr int GT = 128, GK = 16, LDM = GT + 16, LDK = GK + 1;

struct GemmArgs {
  int64_t M, N, K;
  double alpha, beta;
  const double *A, *B, *wK;
  double *C;
  int64_t lda, ldb, ldc, kchunk;
  int tm, tn, nsplit;
  int64_t ntiles, nblk;
  bool tri, vec, atomic;
};

// one operand's 16 x 128 slice: 8 values per thread as 4 pairs; MC: the
// output index is contiguous in memory (pairs along it), else k is
// contiguous (pairs along k)
template <bool MC>
struct Slice {
  double2 r[4];
  __device__ __forceinline__ void load(const double *__restrict__ P, int64_t ld, int64_t o0,
                                       int64_t olim, int64_t k0, int64_t klim, bool fast,
                                       const double *__restrict__ w) {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = t + 256 * q;
      int kk, oo;
      if (MC) {
        kk = p >> 6;
        oo = (p & 63) * 2;
      } else {
        oo = p >> 3;
        kk = (p & 7) * 2;
      }
      const int64_t gk = k0 + kk, go = o0 + oo;
      const double *src = MC ? P + gk * ld + go : P + go * ld + gk;
      double2 v;
      if (fast) {
        v = *(const double2 *)src;
      } else if (MC) {
        const bool kin = gk < klim;
        v.x = kin && go < olim ? src[0] : 0.0;
        v.y = kin && go + 1 < olim ? src[1] : 0.0;
      } else {
        const bool oin = go < olim;
        v.x = oin && gk < klim ? src[0] : 0.0;
        v.y = oin && gk + 1 < klim ? src[1] : 0.0;
      }
      if (w) {
        if (MC) {
          const double wk = gk < klim ? w[gk] : 0.0;
          v.x *= wk;
          v.y *= wk;
        } else {
          v.x *= gk < klim ? w[gk] : 0.0;
          v.y *= gk + 1 < klim ? w[gk + 1] : 0.0;
        }
      }
      r[q] = v;
    }
  }
  __device__ __forceinline__ void store(double *S) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int p = t + 256 * q;
      if (MC) {
        *(double2 *)&S[(p >> 6) * LDM + (p & 63) * 2] = r[q];
      } else {
        const int oo = p >> 3, kk = (p & 7) * 2;
        S[oo * LDK + kk] = r[q].x;
        S[oo * LDK + kk + 1] = r[q].y;
      }
    }
  }
};

// operand value of MFMA lane (li, lk) at output index o, k index k
template <bool MC>
__device__ __forceinline__ double lds_at(const double *S, int o, int k) {
  return MC ? S[k * LDM + o] : S[o * LDK + k];
}

template <bool TA, bool TB, bool SPLIT>
__global__ __launch_bounds__(256, 2) void k_dgemm(GemmArgs g) {
  __shared__ __align__(16) double As[GK * LDM > GT * LDK ? GK * LDM : GT * LDK];
  __shared__ __align__(16) double Bs[GK * LDM > GT * LDK ? GK * LDM : GT * LDK];
  const int t = threadIdx.x, wave = t / 64, lane = t % 64, li = lane % 16, lk = lane / 16;
  int64_t logical = blockIdx.x;
  if (g.nblk % 8 == 0) logical = (int64_t)(blockIdx.x % 8) * (g.nblk / 8) + blockIdx.x / 8;
  const int64_t split = logical / g.ntiles;
  int64_t tile = logical % g.ntiles;
  int ti, tj;
  if (g.tri) {
    ti = 0;
    while (tile >= g.tn - ti) {
      tile -= g.tn - ti;
      ++ti;
    }
    tj = ti + (int)tile;
  } else {
    ti = (int)(tile / g.tn);
    tj = (int)(tile % g.tn);
  }
  const int64_t m0 = (int64_t)ti * GT, n0 = (int64_t)tj * GT;
  const int64_t kb = split * g.kchunk, ke = min(g.K, kb + g.kchunk);
  const int wm = (wave / 2) * 64, wn = (wave % 2) * 64;
  v4d_g acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (v4d_g){0.0, 0.0, 0.0, 0.0};
  const bool tile_in = g.vec && m0 + GT <= g.M && n0 + GT <= g.N;
  Slice<TA> sa;
  Slice<!TB> sb;
  if (kb < ke) {
    sa.load(g.A, g.lda, m0, g.M, kb, ke, tile_in && kb + GK <= ke, g.wK);
    sb.load(g.B, g.ldb, n0, g.N, kb, ke, tile_in && kb + GK <= ke, nullptr);
    for (int64_t k0 = kb; k0 < ke; k0 += GK) {
      __syncthreads();
      sa.store(As);
      sb.store(Bs);
      __syncthreads();
      const int64_t k1 = k0 + GK;
      if (k1 < ke) {
        const bool fast = tile_in && k1 + GK <= ke;
        sa.load(g.A, g.lda, m0, g.M, k1, ke, fast, g.wK);
        sb.load(g.B, g.ldb, n0, g.N, k1, ke, fast, nullptr);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = lds_at<TA>(As, wm + 16 * i + li, 4 * s + lk);
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = lds_at<!TB>(Bs, wn + 16 * j + li, 4 * s + lk);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
  }
  // accumulator v of lane l: row 4 v + l/16, column l%16 of the 16 x 16 block
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gm = m0 + wm + 16 * i + 4 * v + lk, gn = n0 + wn + 16 * j + li;
        if (gm < g.M && gn < g.N) {
          double *cp = g.C + gm * g.ldc + gn;
          if (SPLIT) atomicAdd(cp, g.alpha * acc[i][j][v]);
          else *cp = g.alpha * acc[i][j][v] + (g.beta == 0.0 ? 0.0 : g.beta * *cp);
        }
      }
}

// C[j][i] = C[i][j] for j > i (n x n)
__global__ void k_mirror_upper(int64_t n, double *__restrict__ C, int64_t ldc) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t r = e / n, c = e % n;
  if (r > c) C[r * ldc + c] = C[c * ldc + r];
}

static bool aligned16(const void *p) { return (uintptr_t)p % 16 == 0; }

static efe_status dgemm_launch(efe_ctx *c, bool ta, bool tb, const GemmArgs &g) {
  if (g.nblk > 0x7fffffffLL) EFE_FAIL(c, EFE_EINVAL, "dgemm grid too large");
  const unsigned nb = (unsigned)g.nblk;
#define GL(a, b, sp) k_dgemm<a, b, sp><<<nb, 256, 0, c->stream>>>(g)
  if (g.atomic) {
    if (!ta && !tb) GL(false, false, true);
    else if (ta && !tb) GL(true, false, true);
    else if (!ta && tb) GL(false, true, true);
    else GL(true, true, true);
  } else {
    if (!ta && !tb) GL(false, false, false);
    else if (ta && !tb) GL(true, false, false);
    else if (!ta && tb) GL(false, true, false);
    else GL(true, true, false);
  }
#undef GL
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

static GemmArgs gemm_args(int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                          int64_t lda, const double *B, int64_t ldb, double beta, double *C,
                          int64_t ldc, const double *wK) {
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = alpha;
  g.beta = beta;
  g.A = A;
  g.B = B;
  g.wK = wK;
  g.C = C;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.tm = (int)cdiv(M, GT);
  g.tn = (int)cdiv(N, GT);
  g.vec = lda % 2 == 0 && ldb % 2 == 0 && aligned16(A) && aligned16(B);
  return g;
}

efe_status efe_dgemm(efe_ctx *c, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                     const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                     double *C, int64_t ldc, const double *wK, bool split) {
  if (M <= 0 || N <= 0) return EFE_OK;
  if (K <= 0) EFE_FAIL(c, EFE_EINVAL, "efe_dgemm with K = 0");
  GemmArgs g = gemm_args(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, wK);
  g.ntiles = (int64_t)g.tm * g.tn;
  g.nsplit = 1;
  g.kchunk = K;
  if (split) {
    // enough work-groups to fill the chip twice over, in a multiple of the
    // XCD count; C must already hold the value to add to
    int64_t ns = std::max<int64_t>(1, std::min<int64_t>(cdiv(4096, g.ntiles), cdiv(K, 256)));
    g.kchunk = cdiv(cdiv(K, ns), GK) * GK;
    g.nsplit = (int)cdiv(K, g.kchunk);
    g.atomic = true;
  }
  g.nblk = g.ntiles * g.nsplit;
  return dgemm_launch(c, ta, tb, g);
}

efe_status efe_gram_sym(efe_ctx *c, int64_t N, int64_t K, const double *A, int64_t lda,
                        const double *B, int64_t ldb, double *C, int64_t ldc, const double *wK) {
  if (N <= 0 || K <= 0) return EFE_OK;
  GemmArgs g = gemm_args(N, N, K, 1.0, A, lda, B, ldb, 0.0, C, ldc, wK);
  g.tri = true;
  g.atomic = true;
  g.ntiles = (int64_t)g.tn * (g.tn + 1) / 2;
  int64_t ns = std::max<int64_t>(1, std::min<int64_t>(cdiv(4096, g.ntiles), cdiv(K, 256)));
  ns = cdiv(ns, 8) * 8;
  g.kchunk = cdiv(cdiv(K, ns), GK) * GK;
  g.nsplit = (int)cdiv(K, g.kchunk);
  g.nblk = g.ntiles * g.nsplit;
  return dgemm_launch(c, true, false, g);
}

efe_status efe_mirror_upper(efe_ctx *c, int64_t n, double *C, int64_t ldc) {
  k_mirror_upper<<<cdiv(n * n, 256), 256, 0, c->stream>>>(n, C, ldc);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

// ------------------------------------------------------------------ Cholesky
// Blocked right-looking Cholesky A = L L^T of a symmetric positive definite
// n x n matrix (row-major, lower triangle used and overwritten, upper zeroed):
// per 64-column panel, the diagonal block is factored by one work-group in
// LDS, the rows below solve against it, and the trailing matrix takes the
// rank-64 update on the matrix cores.
constexpr int CB = 64;

// factor the nb x nb diagonal block at (j, j) in LDS; flag[0] = 1 when a
// pivot is not positive
__global__ __launch_bounds__(256) void k_potrf_diag(int64_t n, int64_t j, int nb,
                                                    double *__restrict__ A, int64_t lda,
                                                    int *__restrict__ flag) {
  __shared__ double L[CB][CB + 1];
  const int t = threadIdx.x;
  for (int e = t; e < nb * nb; e += 256) {
    const int r = e / nb, q = e % nb;
    L[r][q] = A[(j + r) * lda + j + q];
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    if (t == 0) {
      const double d = L[k][k];
      if (!(d > 0.0)) *flag = 1;
      L[k][k] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double dk = L[k][k];
    for (int r = k + 1 + t; r < nb; r += 256) L[r][k] /= dk;
    __syncthreads();
    // rank-1 update of the trailing lower triangle
    for (int e = t; e < (nb - k - 1) * (nb - k - 1); e += 256) {
      const int r = k + 1 + e / (nb - k - 1), q = k + 1 + e % (nb - k - 1);
      if (q <= r) L[r][q] -= L[r][k] * L[q][k];
    }
    __syncthreads();
  }
  for (int e = t; e < nb * nb; e += 256) {
    const int r = e / nb, q = e % nb;
    A[(j + r) * lda + j + q] = q <= r ? L[r][q] : 0.0;
  }
}

// rows i >= j + nb of the panel: x L_jj^T = a, one thread per row
__global__ __launch_bounds__(64) void k_trsm_panel(int64_t n, int64_t j, int nb,
                                                   double *__restrict__ A, int64_t lda) {
  __shared__ double L[CB][CB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 64) {
    const int r = e / nb, q = e % nb;
    L[r][q] = A[(j + r) * lda + j + q];
  }
  __syncthreads();
  const int64_t i = j + nb + (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (i >= n) return;
  double x[CB];
  for (int q = 0; q < nb; ++q) x[q] = A[i * lda + j + q];
  for (int q = 0; q < nb; ++q) {
    double s = x[q];
    for (int p = 0; p < q; ++p) s -= x[p] * L[q][p];
    x[q] = s / L[q][q];
  }
  for (int q = 0; q < nb; ++q) A[i * lda + j + q] = x[q];
}

efe_status efe_potrf(efe_ctx *c, int64_t n, double *A, int64_t lda, int *dflag) {
  for (int64_t j = 0; j < n; j += CB) {
    const int nb = (int)std::min<int64_t>(CB, n - j);
    k_potrf_diag<<<1, 256, 0, c->stream>>>(n, j, nb, A, lda, dflag);
    const int64_t rest = n - j - nb;
    if (rest > 0) {
      k_trsm_panel<<<cdiv(rest, 64), 64, 0, c->stream>>>(n, j, nb, A, lda);
      efe_status s;
      // A[j+nb:, j+nb:] -= P P^T with P = A[j+nb:, j:j+nb]
      if ((s = efe_dgemm(c, false, true, rest, rest, nb, -1.0, A + (j + nb) * lda + j, lda,
                         A + (j + nb) * lda + j, lda, 1.0, A + (j + nb) * lda + j + nb, lda,
                         nullptr, false)))
        return s;
    }
  }
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

// ------------------------------------------------------------------ L^-1
// X = L^-1 (lower triangular, n x n) by blocked forward substitution on the
// identity: per row panel i, B = I_i - L[i, :i] X[:i, :] (matrix cores), then
// X_i = L_ii^-1 B with one thread per column.
__global__ __launch_bounds__(256) void k_eye(int64_t n, double *__restrict__ X, int64_t ldx) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  X[(e / n) * ldx + e % n] = (e / n == e % n) ? 1.0 : 0.0;
}

__global__ __launch_bounds__(256) void k_trsv_block(int64_t n, int64_t i0, int nb,
                                                    const double *__restrict__ L, int64_t ldl,
                                                    double *__restrict__ X, int64_t ldx) {
  __shared__ double D[CB][CB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int r = e / nb, q = e % nb;
    D[r][q] = L[(i0 + r) * ldl + i0 + q];
  }
  __syncthreads();
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= n) return;
  double x[CB];
  for (int r = 0; r < nb; ++r) {
    double s = X[(i0 + r) * ldx + col];
    for (int p = 0; p < r; ++p) s -= D[r][p] * x[p];
    x[r] = s / D[r][r];
  }
  for (int r = 0; r < nb; ++r) X[(i0 + r) * ldx + col] = x[r];
}

efe_status efe_trtri_lower(efe_ctx *c, int64_t n, const double *L, int64_t ldl, double *X,
                           int64_t ldx) {
  k_eye<<<cdiv(n * n, 256), 256, 0, c->stream>>>(n, X, ldx);
  efe_status s;
  for (int64_t i0 = 0; i0 < n; i0 += CB) {
    const int nb = (int)std::min<int64_t>(CB, n - i0);
    if (i0 > 0 && (s = efe_dgemm(c, false, false, nb, n, i0, -1.0, L + i0 * ldl, ldl, X, ldx, 1.0,
                                 X + i0 * ldx, ldx, nullptr, false)))
      return s;
    k_trsv_block<<<cdiv(n, 256), 256, 0, c->stream>>>(n, i0, nb, L, ldl, X, ldx);
  }
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

// ------------------------------------------------------------------ Jacobi
// Two-sided block Jacobi for a symmetric n x n matrix A (row-major, padded
// to np = nb * JB rows and columns, nb even): in every round the nb blocks of
// JB indices are paired (round-robin ordering, nb - 1 rounds per sweep), and
// for every pair (p, q) one work-group diagonalizes the 2 JB x 2 JB
// submatrix by cyclic scalar Jacobi in LDS (until its off-diagonal part is
// below thr in squared Frobenius norm), giving U_pq.  Then
// A <- U^T A U and V <- V U with U block-diagonal in the paired blocks (two
// passes on the matrix cores: rows, then columns).  Sweeps repeat until the
// off-diagonal part is below tol of the whole.
constexpr int JB = 32, J2 = 2 * JB;

// the pairs of every round of a sweep: round r, position k -> (p, q), by
// the circle method (block 0 stays, blocks 1 .. nb-1 rotate one place per
// round; position k meets position nb-1-k)
__global__ void k_round_pairs(int nb, int *__restrict__ pairs) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int npair = nb / 2, m = nb - 1;
  if (e >= m * npair) return;
  const int r = e / npair, k = e % npair;
  const int a = k == 0 ? 0 : 1 + (r + k - 1) % m;
  const int b = k == 0 ? 1 + (r + m - 1) % m : 1 + (r + m - k - 1) % m;
  pairs[2 * e] = min(a, b);
  pairs[2 * e + 1] = max(a, b);
}

// the 2 JB x 2 JB subproblem of pair k: eigenvectors into U[k] (row-major
// 64 x 64), by cyclic Jacobi sweeps with a parallel (round-robin) ordering of
// the 32 index pairs of each step
__global__ __launch_bounds__(256) void k_jacobi_sub(int64_t np, const double *__restrict__ A,
                                                    int64_t lda, const int *__restrict__ pairs,
                                                    double *__restrict__ U, int max_sweeps,
                                                    double thr) {
  __shared__ double S[J2][J2 + 1], Q[J2][J2 + 1];
  __shared__ double cs[J2 / 2], sn[J2 / 2];
  __shared__ int ip[J2 / 2], jp[J2 / 2];
  __shared__ double red[256];
  const int k = blockIdx.x, t = threadIdx.x;
  const int p = pairs[2 * k], q = pairs[2 * k + 1];
  for (int e = t; e < J2 * J2; e += 256) {
    const int r = e / J2, cc = e % J2;
    const int64_t gr = r < JB ? (int64_t)p * JB + r : (int64_t)q * JB + r - JB;
    const int64_t gc = cc < JB ? (int64_t)p * JB + cc : (int64_t)q * JB + cc - JB;
    S[r][cc] = A[gr * lda + gc];
    Q[r][cc] = r == cc ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sw = 0; sw < max_sweeps; ++sw) {
    // off-diagonal size of S
    double off = 0.0;
    for (int e = t; e < J2 * J2; e += 256) {
      const double v = S[e / J2][e % J2];
      if (e / J2 != e % J2) off += v * v;
    }
    red[t] = off;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (t < s) red[t] += red[t + s];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    if (!(offs > thr)) break;
    for (int step = 0; step < J2 - 1; ++step) {
      if (t < J2 / 2) {
        // round-robin pairing of 64 indices: index 0 fixed
        const int m = J2 - 1;
        int a = t == 0 ? 0 : 1 + (step + t - 1) % m;
        int b = t == 0 ? 1 + (step + m - 1) % m : 1 + (step + m - t - 1) % m;
        const int i = min(a, b), j = max(a, b);
        ip[t] = i;
        jp[t] = j;
        const double aij = S[i][j], aii = S[i][i], ajj = S[j][j];
        double c = 1.0, s = 0.0;
        if (aij != 0.0) {
          const double tau = (ajj - aii) / (2.0 * aij);
          const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
        }
        cs[t] = c;
        sn[t] = s;
      }
      __syncthreads();
      // rows i, j of S
      for (int e = t; e < (J2 / 2) * J2; e += 256) {
        const int w = e / J2, col = e % J2;
        const int i = ip[w], j = jp[w];
        const double c = cs[w], s = sn[w];
        const double si = S[i][col], sj = S[j][col];
        S[i][col] = c * si - s * sj;
        S[j][col] = s * si + c * sj;
      }
      __syncthreads();
      // columns i, j of S and of Q
      for (int e = t; e < (J2 / 2) * J2; e += 256) {
        const int w = e / J2, row = e % J2;
        const int i = ip[w], j = jp[w];
        const double c = cs[w], s = sn[w];
        const double si = S[row][i], sj = S[row][j];
        S[row][i] = c * si - s * sj;
        S[row][j] = s * si + c * sj;
        const double qi = Q[row][i], qj = Q[row][j];
        Q[row][i] = c * qi - s * qj;
        Q[row][j] = s * qi + c * qj;
      }
      __syncthreads();
    }
  }
  for (int e = t; e < J2 * J2; e += 256) U[(int64_t)k * J2 * J2 + e] = Q[e / J2][e % J2];
}

// B[rows of pair k] = U_k^T A[rows of pair k] (all columns): one work-group
// per (pair, 64 columns), one thread per column, the 64 x 64 U_k in LDS
__global__ __launch_bounds__(64) void k_jacobi_rows(int64_t np, const double *__restrict__ A,
                                                    int64_t lda, const int *__restrict__ pairs,
                                                    const double *__restrict__ U,
                                                    double *__restrict__ B) {
  __shared__ double Us[J2][J2 + 1];
  const int k = blockIdx.y;
  const int p = pairs[2 * k], q = pairs[2 * k + 1];
  for (int e = threadIdx.x; e < J2 * J2; e += 64) Us[e / J2][e % J2] = U[(int64_t)k * J2 * J2 + e];
  __syncthreads();
  const int64_t col = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (col >= np) return;
  double a[J2];
  for (int r = 0; r < J2; ++r) {
    const int64_t gr = r < JB ? (int64_t)p * JB + r : (int64_t)q * JB + r - JB;
    a[r] = A[gr * lda + col];
  }
  for (int r = 0; r < J2; ++r) {
    double s = 0.0;
    for (int m = 0; m < J2; ++m) s += Us[m][r] * a[m];
    const int64_t gr = r < JB ? (int64_t)p * JB + r : (int64_t)q * JB + r - JB;
    B[gr * lda + col] = s;
  }
}

// X[:, cols of pair k] = B[:, cols of pair k] U_k, one thread per row
__global__ __launch_bounds__(64) void k_jacobi_cols(int64_t nrows, const double *__restrict__ B,
                                                    int64_t ldb, const int *__restrict__ pairs,
                                                    const double *__restrict__ U,
                                                    double *__restrict__ X, int64_t ldx) {
  __shared__ double Us[J2][J2 + 1];
  const int k = blockIdx.y;
  const int p = pairs[2 * k], q = pairs[2 * k + 1];
  for (int e = threadIdx.x; e < J2 * J2; e += 64) Us[e / J2][e % J2] = U[(int64_t)k * J2 * J2 + e];
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (row >= nrows) return;
  double b[J2];
  for (int cc = 0; cc < J2; ++cc) {
    const int64_t gc = cc < JB ? (int64_t)p * JB + cc : (int64_t)q * JB + cc - JB;
    b[cc] = B[row * ldb + gc];
  }
  for (int cc = 0; cc < J2; ++cc) {
    double s = 0.0;
    for (int m = 0; m < J2; ++m) s += b[m] * Us[m][cc];
    const int64_t gc = cc < JB ? (int64_t)p * JB + cc : (int64_t)q * JB + cc - JB;
    X[row * ldx + gc] = s;
  }
}

// off[0] += sum of squares off the diagonal, off[1] += on it
__global__ __launch_bounds__(256) void k_offnorm(int64_t np, const double *__restrict__ A,
                                                 int64_t lda, double *__restrict__ out) {
  __shared__ double r0[256], r1[256];
  double a = 0.0, d = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np * np;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = A[(e / np) * lda + e % np];
    if (e / np == e % np) d += v * v;
    else a += v * v;
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = d;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r0[threadIdx.x] += r0[threadIdx.x + s];
      r1[threadIdx.x] += r1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&out[0], r0[0]);
    atomicAdd(&out[1], r1[0]);
  }
}

// copy the n x n matrix into the padded np x np one; the padding is diagonal
// with distinct values above every eigenvalue (pad[i] = top + i), so it never
// couples and sorts last
__global__ void k_pad_sym(int64_t n, int64_t np, const double *__restrict__ H, int64_t ldh,
                          double top, double *__restrict__ A) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= np * np) return;
  const int64_t r = e / np, cc = e % np;
  double v;
  if (r < n && cc < n) v = 0.5 * (H[r * ldh + cc] + H[cc * ldh + r]);
  else v = r == cc ? top + (double)r : 0.0;
  A[e] = v;
}

// ascending order of the diagonal of the np x np A (ties by index): the
// first n values into w, their indices into ord
__global__ void k_sort_diag(int64_t np, const double *__restrict__ A, int64_t n,
                            double *__restrict__ w, int *__restrict__ ord) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= np) return;
  const double di = A[i * (np + 1)];
  int64_t rank = 0;
  for (int64_t j = 0; j < np; ++j) {
    const double dj = A[j * (np + 1)];
    rank += (dj < di) || (dj == di && j < i);
  }
  if (rank < n) {
    w[rank] = di;
    ord[rank] = (int)i;
  }
}

// Q[r][i] = V[r][ord[i]] for r, i < n
__global__ void k_gather_cols(int64_t n, const double *__restrict__ V, int64_t ldv,
                              const int *__restrict__ ord, double *__restrict__ Q, int64_t ldq) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t r = e / n, i = e % n;
  Q[r * ldq + i] = V[r * ldv + ord[i]];
}

// number of index blocks of the padded problem (even, at least 2)
static int jacobi_blocks(int64_t n) {
  int nb = (int)cdiv(n, JB);
  nb += nb % 2;
  return std::max(nb, 2);
}

size_t efe_syev_work(int64_t n) {
  const int64_t np = (int64_t)jacobi_blocks(n) * JB;
  return (size_t)(3 * np * np + (np / J2) * J2 * J2 + 2);
}

size_t efe_syev_iwork(int64_t n) {
  const int nb = jacobi_blocks(n);
  return (size_t)((int64_t)(nb - 1) * nb + n);
}

// Eigen-decomposition H = Q diag(w) Q^T of the symmetric n x n matrix H.
// Converged when the off-diagonal part of the rotated matrix is below 1e-14
// of ||H||_F (the eigenvalues are then exact to that much of ||H||_F), or
// when it stops falling once below 1e-11 ||H||_F (rounding has then reached
// it: about sqrt(n) eps ||H||_F).
efe_status efe_syev_jacobi(efe_ctx *c, int64_t n, const double *H, int64_t ldh, double *w,
                           double *Q, double *work, int *iwork, int *sweeps_out) {
  if (n < 1) EFE_FAIL(c, EFE_EINVAL, "eigensolve of an empty matrix");
  const int nb = jacobi_blocks(n);
  const int64_t np = (int64_t)nb * JB;
  const int npair = nb / 2;
  double *A = work, *B = A + np * np, *V = B + np * np, *U = V + np * np;
  double *off = U + (int64_t)npair * J2 * J2;
  // a bound above every eigenvalue (Gershgorin through the Frobenius norm)
  HIPCHK(c, hipMemsetAsync(off, 0, 2 * 8, c->stream));
  k_offnorm<<<std::min<int64_t>(cdiv(n * n, 256), 1024), 256, 0, c->stream>>>(n, H, ldh, off);
  double h2[2];
  HIPCHK(c, hipMemcpyAsync(h2, off, 16, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double hn2 = h2[0] + h2[1];
  if (!std::isfinite(hn2)) EFE_FAIL(c, EFE_ENUMERIC, "eigensolve of a matrix with non-finite entries");
  const double top = 2.0 * sqrt(hn2) + 1.0;
  k_pad_sym<<<cdiv(np * np, 256), 256, 0, c->stream>>>(n, np, H, ldh, top, A);
  k_eye<<<cdiv(np * np, 256), 256, 0, c->stream>>>(np, V, np);
  // the pair lists of all rounds of a sweep
  k_round_pairs<<<cdiv((int64_t)(nb - 1) * npair, 256), 256, 0, c->stream>>>(nb, iwork);
  int sw = 0;
  double prev = INFINITY;
  for (;; ++sw) {
    HIPCHK(c, hipMemsetAsync(off, 0, 2 * 8, c->stream));
    k_offnorm<<<std::min<int64_t>(cdiv(np * np, 256), 1024), 256, 0, c->stream>>>(np, A, np, off);
    HIPCHK(c, hipMemcpyAsync(h2, off, 16, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!std::isfinite(h2[0])) EFE_FAIL(c, EFE_ENUMERIC, "block Jacobi diverged");
    if (!(h2[0] > 1e-28 * hn2)) break;
    if (h2[0] <= 1e-22 * hn2 && h2[0] > 0.25 * prev) break;
    if (sw == 40) EFE_FAIL(c, EFE_ENOTCONV, "block Jacobi did not converge in 40 sweeps");
    prev = h2[0];
    for (int r = 0; r < nb - 1; ++r) {
      const int *pr = iwork + (int64_t)r * 2 * npair;
      k_jacobi_sub<<<npair, 256, 0, c->stream>>>(np, A, np, pr, U, 8, 1e-30 * hn2);
      // B = U^T A on the paired rows (every row belongs to one pair)
      k_jacobi_rows<<<dim3((unsigned)cdiv(np, 64), npair), 64, 0, c->stream>>>(np, A, np, pr, U, B);
      // A = B U, V = V U on the paired columns
      k_jacobi_cols<<<dim3((unsigned)cdiv(np, 64), npair), 64, 0, c->stream>>>(np, B, np, pr, U, A,
                                                                              np);
      k_jacobi_cols<<<dim3((unsigned)cdiv(np, 64), npair), 64, 0, c->stream>>>(np, V, np, pr, U, B,
                                                                              np);
      std::swap(V, B);
    }
  }
  if (sweeps_out) *sweeps_out = sw;
  // eigenvalues: the diagonal in ascending order; Q[:, i] = V[:n, ord[i]]
  int *ord = iwork + (int64_t)(nb - 1) * 2 * npair;
  k_sort_diag<<<cdiv(np, 256), 256, 0, c->stream>>>(np, A, n, w, ord);
  k_gather_cols<<<cdiv(n * n, 256), 256, 0, c->stream>>>(n, V, np, ord, Q, n);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}
