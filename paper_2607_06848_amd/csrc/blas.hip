// FP64 dense products around the hot path: a tiled kernel for plain and
// weighted products, split over the summation index (partial sums added
// atomically) for the enrichment blocks of the apply and the tall-skinny
// weighted Grams V^T M V of Rayleigh-Ritz.
#include "efe_internal.h"

// C = alpha op(A) op(B) (+ beta C), row-major, 64x64 tiles, 16-deep k steps;
// thread (ty, tx) owns rows ty + 16 i and columns tx + 16 j (i, j < 4).
// With ATOMIC the result is added to C with atomics (split-K over blockIdx.z).
template <bool TA, bool TB, bool ATOMIC>
__global__ __launch_bounds__(256) void k_gemm(int64_t M, int64_t N, int64_t K, double alpha,
                                              const double *__restrict__ A, int64_t lda,
                                              const double *__restrict__ B, int64_t ldb,
                                              double beta, double *__restrict__ C, int64_t ldc,
                                              const double *__restrict__ wK, int64_t kchunk) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int t = threadIdx.x;
  const int tx = t % 16, ty = t / 16;
  const int64_t m0 = (int64_t)blockIdx.y * 64, n0 = (int64_t)blockIdx.x * 64;
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = min(K, kb + kchunk);
  double acc[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t k0 = kb; k0 < ke; k0 += 16) {
    for (int r = 0; r < 4; ++r) {
      int kk, mm;
      if (!TA) {
        kk = t % 16;
        mm = t / 16 + 16 * r;
      } else {
        mm = t % 64;
        kk = t / 64 + 4 * r;
      }
      const int64_t gk = k0 + kk, gm = m0 + mm;
      double v = 0.0;
      if (gk < ke && gm < M) {
        v = TA ? A[gk * lda + gm] : A[gm * lda + gk];
        if (wK) v *= wK[gk];
      }
      As[kk][mm] = v;
      int nn;
      if (!TB) {
        nn = t % 64;
        kk = t / 64 + 4 * r;
      } else {
        kk = t % 16;
        nn = t / 16 + 16 * r;
      }
      const int64_t gk2 = k0 + kk, gn = n0 + nn;
      double w = 0.0;
      if (gk2 < ke && gn < N) w = TB ? B[gn * ldb + gk2] : B[gk2 * ldb + gn];
      Bs[kk][nn] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      const int64_t gm = m0 + ty + 16 * i, gn = n0 + tx + 16 * j;
      if (gm < M && gn < N) {
        if (ATOMIC) atomicAdd(&C[gm * ldc + gn], alpha * acc[i][j]);
        else C[gm * ldc + gn] = alpha * acc[i][j] + (beta == 0.0 ? 0.0 : beta * C[gm * ldc + gn]);
      }
    }
}

efe_status efe_gemm(efe_ctx *ctx, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                    const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                    double *C, int64_t ldc, const double *wK) {
  if (M <= 0 || N <= 0) return EFE_OK;
  if (K <= 0) {
    EFE_FAIL(ctx, EFE_EINVAL, "efe_gemm with K = 0");
  }
  dim3 grid(cdiv(N, 64), cdiv(M, 64), 1);
  if (grid.y > 65535u * 32u) EFE_FAIL(ctx, EFE_EINVAL, "gemm grid too large");
#define GL(a, b) \
  k_gemm<a, b, false><<<grid, 256, 0, ctx->stream>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, wK, K)
  if (!ta && !tb) GL(false, false);
  else if (ta && !tb) GL(true, false);
  else if (!ta && tb) GL(false, true);
  else GL(true, true);
#undef GL
  HIPCHK(ctx, hipGetLastError());
  return EFE_OK;
}

efe_status efe_gemm_acc(efe_ctx *ctx, bool ta, int64_t M, int64_t N, int64_t K, double alpha,
                        const double *A, int64_t lda, const double *B, int64_t ldb, double *C,
                        int64_t ldc) {
  if (M <= 0 || N <= 0 || K <= 0) return EFE_OK;
  // split the sum over K so that the launch fills the chip; partial sums
  // meet in C by atomic adds
  const int64_t tiles = cdiv(M, 64) * cdiv(N, 64);
  int64_t nsplit = std::max<int64_t>(1, cdiv(1024, tiles));
  int64_t kchunk = std::max<int64_t>(64, cdiv(cdiv(K, nsplit), 16) * 16);
  nsplit = cdiv(K, kchunk);
  dim3 grid(cdiv(N, 64), cdiv(M, 64), nsplit);
  if (ta)
    k_gemm<true, false, true><<<grid, 256, 0, ctx->stream>>>(M, N, K, alpha, A, lda, B, ldb, 0.0,
                                                             C, ldc, nullptr, kchunk);
  else
    k_gemm<false, false, true><<<grid, 256, 0, ctx->stream>>>(M, N, K, alpha, A, lda, B, ldb, 0.0,
                                                              C, ldc, nullptr, kchunk);
  HIPCHK(ctx, hipGetLastError());
  return EFE_OK;
}

efe_status efe_gram(efe_ctx *ctx, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                    int64_t lda, const double *B, int64_t ldb, const double *w, double *C,
                    int64_t ldc) {
  if (M <= 0 || N <= 0 || K <= 0) return EFE_OK;
  const int64_t tiles = cdiv(M, 64) * cdiv(N, 64);
  int64_t nsplit = cdiv(2048, tiles);
  int64_t kchunk = cdiv(cdiv(K, nsplit), 16) * 16;
  if (kchunk < 256) kchunk = 256;
  nsplit = cdiv(K, kchunk);
  dim3 grid(cdiv(N, 64), cdiv(M, 64), nsplit);
  k_gemm<true, false, true><<<grid, 256, 0, ctx->stream>>>(M, N, K, alpha, A, lda, B, ldb, 0.0, C,
                                                           ldc, w, kchunk);
  HIPCHK(ctx, hipGetLastError());
  return EFE_OK;
}
