// Learned initial density: quadrature export, atom-centred descriptors, the
// density MLP (forward, backward, loss gradient, Adam) and the guess
// ρ_0 = max(ρ_SAD + Δρ, 0) renormalized to the electron count, with the
// superposition of atomic densities as fallback.  All MLP arithmetic is FP32;
// descriptors are formed in FP64 and stored in FP32.
#include <cmath>

#include "efe_device.h"

// positions and weights (reference weight times cell Jacobian) of every
// Gauss point, cell by cell
__global__ void k_quadrature(MeshGeo g, const double *__restrict__ xq1,
                             const double *__restrict__ W3, double *__restrict__ xq,
                             double *__restrict__ wq) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nq = (int64_t)g.ncell[0] * g.ncell[1] * g.ncell[2] * g.nqp;
  if (idx >= nq) return;
  const int q = (int)(idx % g.nqp);
  if (xq) {
    double x[3];
    quad_point(g, xq1, (int)(idx / g.nqp), q, x);
    xq[3 * idx] = x[0];
    xq[3 * idx + 1] = x[1];
    xq[3 * idx + 2] = x[2];
  }
  if (wq) wq[idx] = W3[q];
}

extern "C" efe_status efe_get_quadrature(efe_ctx *c, double *xq, double *wq) {
  if (!c) return EFE_EINVAL;
  if (!xq && !wq) EFE_FAIL(c, EFE_EINVAL, "both outputs null");
  const MeshGeo g = mesh_geo(c);
  k_quadrature<<<cdiv(c->n_qpts, 256), 256, 0, c->stream>>>(g, c->d_xq1, c->d_W3, xq, wq);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

// ------------------------------------------------------------------ descriptors
namespace {
constexpr int KNEAR = 16;   // nearest atoms per point
constexpr int NRAD = 8;     // radial Gaussians exp(-(d - n)^2 / 2), n = 0..7
constexpr int MLP_IN = 25;  // 8 x 3 power-spectrum entries + log rho_SAD
constexpr int MLP_H = 128;
// flat parameter layout: W1 [128][25], b1, W2 [128][128], b2, W3, b3, W4 [128], b4
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + MLP_H * MLP_IN, OFF_W2 = OFF_B1 + MLP_H,
              OFF_B2 = OFF_W2 + MLP_H * MLP_H, OFF_W3 = OFF_B2 + MLP_H,
              OFF_B3 = OFF_W3 + MLP_H * MLP_H, OFF_W4 = OFF_B3 + MLP_H, OFF_B4 = OFF_W4 + MLP_H,
              N_PARAMS = OFF_B4 + 1;
constexpr double RHO_FLOOR = 1e-12;
constexpr int TP = 64;      // points per work-group tile of the MLP kernels
constexpr int WLD = 132;    // LDS row stride of the transposed weights (float4 aligned)
}  // namespace

__device__ inline double dist2_nofma(double x0, double x1, double x2, const double *a) {
#pragma clang fp contract(off)
  const double dx = x0 - a[0], dy = x1 - a[1], dz = x2 - a[2];
  return (dx * dx + dy * dy) + dz * dz;
}

// One thread per point: the 16 nearest atoms (ties by lower index, kept in
// registers by an unrolled insertion), then for every radial Gaussian n the
// sums A_lm = sum_I g_n(d_I) Y_lm(u_I) and the power spectrum per l.
__global__ __launch_bounds__(256) void k_descriptors(int64_t npts, const double *__restrict__ pts,
                                                     int natoms, const double *__restrict__ xyz,
                                                     const double *__restrict__ rho_sad,
                                                     const float *__restrict__ shift,
                                                     const float *__restrict__ scale,
                                                     float *__restrict__ feat) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const double x0 = pts[3 * p], x1 = pts[3 * p + 1], x2 = pts[3 * p + 2];
  double kd[KNEAR];
  int ki[KNEAR];
#pragma unroll
  for (int j = 0; j < KNEAR; ++j) {
    kd[j] = INFINITY;
    ki[j] = -1;
  }
  for (int I = 0; I < natoms; ++I) {
    const double d2 = dist2_nofma(x0, x1, x2, xyz + 3 * I);
    if (d2 < kd[KNEAR - 1]) {
#pragma unroll
      for (int j = KNEAR - 1; j > 0; --j) {
        const bool up = kd[j - 1] > d2;
        const bool here = !up && kd[j] > d2;
        kd[j] = up ? kd[j - 1] : (here ? d2 : kd[j]);
        ki[j] = up ? ki[j - 1] : (here ? I : ki[j]);
      }
      if (kd[0] > d2) {
        kd[0] = d2;
        ki[0] = I;
      }
    }
  }
  const double c0 = 0.5 / sqrt(M_PI), c1 = sqrt(3.0 / (4.0 * M_PI)), c2 = 0.5 * sqrt(15.0 / M_PI),
               c20 = 0.25 * sqrt(5.0 / M_PI), c22 = 0.25 * sqrt(15.0 / M_PI);
  float *f = feat + p * MLP_IN;
  for (int n = 0; n < NRAD; ++n) {
    double A[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) A[m] = 0.0;
#pragma unroll
    for (int j = 0; j < KNEAR; ++j) {
      if (ki[j] >= 0) {
        const double *a = xyz + 3 * ki[j];
        const double vx = x0 - a[0], vy = x1 - a[1], vz = x2 - a[2];
        const double d = sqrt(kd[j]);
        const double g = exp(-0.5 * (d - n) * (d - n));
        A[0] += g * c0;
        if (d > 0.0) {
          const double ux = vx / d, uy = vy / d, uz = vz / d;
          A[1] += g * c1 * uy;
          A[2] += g * c1 * uz;
          A[3] += g * c1 * ux;
          A[4] += g * c2 * ux * uy;
          A[5] += g * c2 * uy * uz;
          A[6] += g * c20 * (3.0 * uz * uz - 1.0);
          A[7] += g * c2 * ux * uz;
          A[8] += g * c22 * (ux * ux - uy * uy);
        }
      }
    }
    const double P[3] = {A[0] * A[0], A[1] * A[1] + A[2] * A[2] + A[3] * A[3],
                         A[4] * A[4] + A[5] * A[5] + A[6] * A[6] + A[7] * A[7] + A[8] * A[8]};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const int i = 3 * n + l;
      f[i] = shift ? (float)((P[l] - (double)shift[i]) / (double)scale[i]) : (float)P[l];
    }
  }
  const double lr = log(fmax(rho_sad[p], RHO_FLOOR));
  f[24] = shift ? (float)((lr - (double)shift[24]) / (double)scale[24]) : (float)lr;
}

// ------------------------------------------------------------------ MLP
__device__ inline float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }

// Fused forward pass of a 64-point tile: activations stay in LDS (transposed,
// [neuron][point]); each layer's W^T is staged in LDS; every thread owns 4
// neurons x 8 points.  acts (optional) receives the pre-activations z1..z3.
__global__ __launch_bounds__(256) void k_mlp_fwd(int64_t npts, const float *__restrict__ prm,
                                                 const float *__restrict__ X,
                                                 float *__restrict__ y, float *__restrict__ acts) {
  extern __shared__ float sm[];
  float *Wt = sm;                 // [128][WLD]
  float *Ht = sm + MLP_H * WLD;   // [128][TP]
  const int t = threadIdx.x;
  const int64_t p0 = blockIdx.x * (int64_t)TP;
  const int np = (int)min<int64_t>(TP, npts - p0);
  for (int i = t; i < TP * MLP_IN; i += 256) {
    const int p = i / MLP_IN, k = i % MLP_IN;
    Ht[k * TP + p] = p < np ? X[p0 * MLP_IN + i] : 0.0f;
  }
  const int jg = t & 31, pg = t >> 5;
  for (int l = 0; l < 3; ++l) {
    const int K = l == 0 ? MLP_IN : MLP_H;
    const float *W = prm + (l == 0 ? OFF_W1 : l == 1 ? OFF_W2 : OFF_W3);
    const float *b = prm + (l == 0 ? OFF_B1 : l == 1 ? OFF_B2 : OFF_B3);
    for (int i = t; i < MLP_H * K; i += 256) {
      const int j = i / K, k = i % K;
      Wt[k * WLD + j] = W[i];
    }
    __syncthreads();
    float acc[8][4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const float bj = b[4 * jg + jj];
#pragma unroll
      for (int p = 0; p < 8; ++p) acc[p][jj] = bj;
    }
    for (int k = 0; k < K; ++k) {
      const float4 w = *(const float4 *)&Wt[k * WLD + 4 * jg];
      const float4 ha = *(const float4 *)&Ht[k * TP + 8 * pg];
      const float4 hb = *(const float4 *)&Ht[k * TP + 8 * pg + 4];
      const float h[8] = {ha.x, ha.y, ha.z, ha.w, hb.x, hb.y, hb.z, hb.w};
      const float wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[p][jj] = fmaf(h[p], wv[jj], acc[p][jj]);
    }
    __syncthreads();
    if (acts) {
#pragma unroll
      for (int p = 0; p < 8; ++p)
        if (8 * pg + p < np)
          *(float4 *)&acts[(int64_t)l * npts * MLP_H + (p0 + 8 * pg + p) * MLP_H + 4 * jg] =
              make_float4(acc[p][0], acc[p][1], acc[p][2], acc[p][3]);
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      float s[8];
#pragma unroll
      for (int p = 0; p < 8; ++p) s[p] = acc[p][jj] * sigm(acc[p][jj]);
      *(float4 *)&Ht[(4 * jg + jj) * TP + 8 * pg] = make_float4(s[0], s[1], s[2], s[3]);
      *(float4 *)&Ht[(4 * jg + jj) * TP + 8 * pg + 4] = make_float4(s[4], s[5], s[6], s[7]);
    }
    __syncthreads();
  }
  if (t < np) {
    float s = prm[OFF_B4];
    for (int k = 0; k < MLP_H; ++k) s = fmaf(prm[OFF_W4 + k], Ht[k * TP + t], s);
    y[p0 + t] = s;
  }
}

// Output layer backward: dz3 = dy W4 silu'(z3); gW4 += dy silu(z3), gb4 += dy.
__global__ __launch_bounds__(256) void k_mlp_bwd_head(int64_t npts, const float *__restrict__ prm,
                                                      const float *__restrict__ dy,
                                                      const float *__restrict__ z3,
                                                      float *__restrict__ dz3,
                                                      float *__restrict__ grads) {
  const int t = threadIdx.x, k = t & (MLP_H - 1), half = t >> 7;
  const float w4 = prm[OFF_W4 + k];
  float gw = 0.0f, gb = 0.0f;
  for (int64_t p = blockIdx.x * 2 + half; p < npts; p += (int64_t)gridDim.x * 2) {
    const float d = dy[p], z = z3[p * MLP_H + k];
    const float s = sigm(z);
    gw = fmaf(d, z * s, gw);
    dz3[p * MLP_H + k] = d * w4 * (s * (1.0f + z * (1.0f - s)));
    if (k == 0) gb += d;
  }
  atomicAdd(&grads[OFF_W4 + k], gw);
  if (k == 0) atomicAdd(&grads[OFF_B4], gb);
}

// Backward of one hidden layer z = W h + b over 64-point tiles (grid-stride):
// gW += dz^T h and gb += sum dz accumulate in registers and are added to
// grads once per work-group; for KIN = 128 also dz_prev = (dz W) silu'(z_prev).
// hin is the standardized input X (KIN = 25) or z_prev (KIN = 128).
template <int KIN>
__global__ __launch_bounds__(256) void k_mlp_bwd_layer(int64_t npts, const float *__restrict__ prm,
                                                       int offW, int offB,
                                                       const float *__restrict__ dz,
                                                       const float *__restrict__ hin,
                                                       float *__restrict__ dzprev,
                                                       float *__restrict__ grads) {
  extern __shared__ float sm[];
  constexpr bool PREV = KIN == MLP_H;
  float *Ws = sm;                                // [128][128] row-major (PREV only)
  float *Ds = sm + (PREV ? MLP_H * MLP_H : 0);   // [TP][128]
  float *Hs = Ds + TP * MLP_H;                   // [TP][128], zero beyond KIN
  const int t = threadIdx.x;
  if (PREV)
    for (int i = t; i < MLP_H * MLP_H; i += 256) Ws[i] = prm[offW + i];
  const int jg = t >> 4, kg = t & 15;            // gW block: j 8jg.., k 8kg..
  float gw[8][8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int c = 0; c < 8; ++c) gw[a][c] = 0.0f;
  float gb = 0.0f;
  const int64_t ntiles = (npts + TP - 1) / TP;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t p0 = tile * TP;
    const int np = (int)min<int64_t>(TP, npts - p0);
    __syncthreads();
    for (int i = t; i < TP * MLP_H; i += 256) {
      const int p = i >> 7, k = i & (MLP_H - 1);
      Ds[i] = p < np ? dz[(p0 + p) * MLP_H + k] : 0.0f;
      float h = 0.0f;
      if (p < np && k < KIN) {
        const float v = hin[(p0 + p) * KIN + k];
        h = PREV ? v * sigm(v) : v;
      }
      Hs[i] = h;
    }
    __syncthreads();
    for (int p = 0; p < np; ++p) {
      const float4 da = *(const float4 *)&Ds[p * MLP_H + 8 * jg];
      const float4 db = *(const float4 *)&Ds[p * MLP_H + 8 * jg + 4];
      const float4 ha = *(const float4 *)&Hs[p * MLP_H + 8 * kg];
      const float4 hb = *(const float4 *)&Hs[p * MLP_H + 8 * kg + 4];
      const float dv[8] = {da.x, da.y, da.z, da.w, db.x, db.y, db.z, db.w};
      const float hv[8] = {ha.x, ha.y, ha.z, ha.w, hb.x, hb.y, hb.z, hb.w};
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int c = 0; c < 8; ++c) gw[a][c] = fmaf(dv[a], hv[c], gw[a][c]);
    }
    if (t < MLP_H)
      for (int p = 0; p < np; ++p) gb += Ds[p * MLP_H + t];
    if (PREV) {
      const int pg = t >> 5, kq = t & 31;          // 8 points x 4 inputs
      float acc[8][4];
#pragma unroll
      for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[p][c] = 0.0f;
      for (int j = 0; j < MLP_H; ++j) {
        const float4 w = *(const float4 *)&Ws[j * MLP_H + 4 * kq];
        const float wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int p = 0; p < 8; ++p) {
          const float d = Ds[(8 * pg + p) * MLP_H + j];
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[p][c] = fmaf(d, wv[c], acc[p][c]);
        }
      }
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        if (8 * pg + p < np) {
          const int64_t o = (p0 + 8 * pg + p) * MLP_H + 4 * kq;
          const float4 z = *(const float4 *)&hin[o];
          const float zv[4] = {z.x, z.y, z.z, z.w};
          float r[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float s = sigm(zv[c]);
            r[c] = acc[p][c] * (s * (1.0f + zv[c] * (1.0f - s)));
          }
          *(float4 *)&dzprev[o] = make_float4(r[0], r[1], r[2], r[3]);
        }
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int k = 8 * kg + c;
      if (k < KIN) atomicAdd(&grads[offW + (8 * jg + a) * KIN + k], gw[a][c]);
    }
  if (t < MLP_H) atomicAdd(&grads[offB + t], gb);
}

// sums[0] += sum w, sums[1] += sum w (y - t)^2 (FP64)
__global__ __launch_bounds__(256) void k_loss_sums(int64_t n, const float *__restrict__ y,
                                                   const float *__restrict__ tg,
                                                   const float *__restrict__ w,
                                                   double *__restrict__ sums) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double r = (double)y[i] - (double)tg[i];
    a += w[i];
    b += w[i] * r * r;
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s0[threadIdx.x] += s0[threadIdx.x + s];
      s1[threadIdx.x] += s1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&sums[0], s0[0]);
    atomicAdd(&sums[1], s1[0]);
  }
}

__global__ void k_loss_grad(int64_t n, const float *__restrict__ y, const float *__restrict__ tg,
                            const float *__restrict__ w, const double *__restrict__ sums,
                            float *__restrict__ dy) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dy[i] = (float)(2.0 * (double)w[i] * ((double)y[i] - (double)tg[i]) / sums[0]);
}

__global__ void k_fill_f32(int64_t n, float *__restrict__ x, float v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_fill_f64(int64_t n, double *__restrict__ x, double v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_adam(int64_t n, float *__restrict__ prm, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  prm[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// rho0 = max(rho_SAD + s_t y, 0); sums[0] += int rho0, sums[1] counts non-finite values
__global__ __launch_bounds__(256) void k_guess(int64_t n, const double *__restrict__ sad,
                                               const float *__restrict__ y, double st,
                                               const double *__restrict__ wq,
                                               double *__restrict__ rho,
                                               double *__restrict__ sums) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double r = sad[i] + st * (double)y[i];
    if (!isfinite(r)) {
      b += 1.0;
      rho[i] = 0.0;
    } else {
      const double c = fmax(r, 0.0);
      rho[i] = c;
      a += wq[i] * c;
    }
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s0[threadIdx.x] += s0[threadIdx.x + s];
      s1[threadIdx.x] += s1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&sums[0], s0[0]);
    atomicAdd(&sums[1], s1[0]);
  }
}

__global__ void k_scale_f64(int64_t n, double *__restrict__ x, double f) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] *= f;
}

// ------------------------------------------------------------------ C ABI
namespace {
efe_status gfail(efe_status code, const std::string &msg) {
  efe_set_global_error(msg);
  return code;
}
#define GCHK(call)                                                                   \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return gfail(EFE_EHIP, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t FWD_LDS = (size_t)(MLP_H * WLD + MLP_H * TP) * sizeof(float);
constexpr size_t BWD_LDS_128 = (size_t)(MLP_H * MLP_H + 2 * TP * MLP_H) * sizeof(float);
constexpr size_t BWD_LDS_25 = (size_t)(2 * TP * MLP_H) * sizeof(float);

efe_status lds_attrs() {
  static bool done = false;
  if (done) return EFE_OK;
  GCHK(hipFuncSetAttribute((const void *)k_mlp_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                           (int)FWD_LDS));
  GCHK(hipFuncSetAttribute((const void *)k_mlp_bwd_layer<MLP_H>,
                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)BWD_LDS_128));
  GCHK(hipFuncSetAttribute((const void *)k_mlp_bwd_layer<MLP_IN>,
                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)BWD_LDS_25));
  done = true;
  return EFE_OK;
}

efe_status mlp_forward(hipStream_t s, const float *prm, const float *feat, int64_t npts, float *out,
                       float *acts) {
  efe_status st;
  if ((st = lds_attrs())) return st;
  if (npts == 0) return EFE_OK;
  k_mlp_fwd<<<cdiv(npts, TP), 256, FWD_LDS, s>>>(npts, prm, feat, out, acts);
  GCHK(hipGetLastError());
  return EFE_OK;
}
}  // namespace

extern "C" efe_status efe_descriptors(void *stream, const double *pts, int64_t npts,
                                      const double *xyz, int32_t natoms, const double *rho_sad,
                                      const float *shift, const float *scale, float *feat) {
  if (npts < 0 || natoms < 0 || (npts && (!pts || !rho_sad || !feat)) || (natoms && !xyz) ||
      (!shift) != (!scale))
    return gfail(EFE_EINVAL, "efe_descriptors: bad arguments");
  if (npts == 0) return EFE_OK;
  k_descriptors<<<cdiv(npts, 256), 256, 0, (hipStream_t)stream>>>(npts, pts, natoms, xyz, rho_sad,
                                                                  shift, scale, feat);
  GCHK(hipGetLastError());
  return EFE_OK;
}

extern "C" efe_status efe_mlp_forward(void *stream, const float *params, const float *feat,
                                      int64_t npts, float *out, float *acts) {
  if (npts < 0 || (npts && (!params || !feat || !out)))
    return gfail(EFE_EINVAL, "efe_mlp_forward: bad arguments");
  return mlp_forward((hipStream_t)stream, params, feat, npts, out, acts);
}

extern "C" efe_status efe_mlp_loss_grad(void *stream, const float *out, const float *target,
                                        const float *weight, int64_t npts, float *dout,
                                        double *sums) {
  if (npts <= 0 || !out || !target || !weight || !dout || !sums)
    return gfail(EFE_EINVAL, "efe_mlp_loss_grad: bad arguments");
  hipStream_t s = (hipStream_t)stream;
  k_fill_f64<<<1, 64, 0, s>>>(2, sums, 0.0);
  k_loss_sums<<<(int)std::min<int64_t>(cdiv(npts, 256), 1024), 256, 0, s>>>(npts, out, target,
                                                                            weight, sums);
  k_loss_grad<<<cdiv(npts, 256), 256, 0, s>>>(npts, out, target, weight, sums, dout);
  GCHK(hipGetLastError());
  return EFE_OK;
}

extern "C" efe_status efe_mlp_backward(void *stream, const float *params, const float *feat,
                                       const float *acts, const float *dout, int64_t npts,
                                       float *grads, float *work) {
  if (npts <= 0 || !params || !feat || !acts || !dout || !grads || !work)
    return gfail(EFE_EINVAL, "efe_mlp_backward: bad arguments");
  efe_status st;
  if ((st = lds_attrs())) return st;
  hipStream_t s = (hipStream_t)stream;
  const int64_t zs = npts * MLP_H;
  const float *z1 = acts, *z2 = acts + zs, *z3 = acts + 2 * zs;
  float *A = work, *B = work + zs;
  k_fill_f32<<<cdiv(N_PARAMS, 256), 256, 0, s>>>(N_PARAMS, grads, 0.0f);
  const int gh = (int)std::min<int64_t>(cdiv(npts, 2), 512);
  k_mlp_bwd_head<<<gh, 256, 0, s>>>(npts, params, dout, z3, A, grads);
  const int gl = (int)std::min<int64_t>(cdiv(npts, TP), 256);
  k_mlp_bwd_layer<MLP_H><<<gl, 256, BWD_LDS_128, s>>>(npts, params, OFF_W3, OFF_B3, A, z2, B, grads);
  k_mlp_bwd_layer<MLP_H><<<gl, 256, BWD_LDS_128, s>>>(npts, params, OFF_W2, OFF_B2, B, z1, A, grads);
  k_mlp_bwd_layer<MLP_IN><<<gl, 256, BWD_LDS_25, s>>>(npts, params, OFF_W1, OFF_B1, A, feat, nullptr,
                                                      grads);
  GCHK(hipGetLastError());
  return EFE_OK;
}

extern "C" efe_status efe_mlp_adam(void *stream, float *params, const float *grads, float *m,
                                   float *v, int64_t n, double lr, double beta1, double beta2,
                                   double eps, int64_t step) {
  if (n <= 0 || !params || !grads || !m || !v || step < 1 || !(lr > 0) || !(beta1 >= 0) ||
      !(beta1 < 1) || !(beta2 >= 0) || !(beta2 < 1) || !(eps > 0))
    return gfail(EFE_EINVAL, "efe_mlp_adam: bad arguments");
  const double c1 = 1.0 / (1.0 - pow(beta1, (double)step));
  const double c2 = 1.0 / (1.0 - pow(beta2, (double)step));
  k_adam<<<cdiv(n, 256), 256, 0, (hipStream_t)stream>>>(n, params, grads, m, v, (float)lr,
                                                        (float)beta1, (float)beta2, (float)eps,
                                                        (float)c1, (float)c2);
  GCHK(hipGetLastError());
  return EFE_OK;
}

extern "C" int64_t efe_mlp_num_params(void) { return N_PARAMS; }

extern "C" efe_status efe_density_guess(efe_ctx *c, const float *params, const float *norm,
                                        int32_t *used_fallback, double *factor) {
  if (!c) return EFE_EINVAL;
  if (!used_fallback || !factor || (params && !norm))
    EFE_FAIL(c, EFE_EINVAL, "efe_density_guess: bad arguments");
  const int64_t nq = c->n_qpts;
  efe_status st;
  double *sad, *rho, *xq, *wq, *sums;
  float *feat, *y, *dnorm;
  if ((st = efe_ws(c, 40, nq * 8, (void **)&sad))) return st;
  if ((st = efe_get_density(c, 2, sad))) return st;
  *used_fallback = 1;
  *factor = 1.0;
  if (!params) return efe_set_density(c, sad);
  if ((st = efe_ws(c, 41, nq * 8, (void **)&rho))) return st;
  if ((st = efe_ws(c, 42, nq * 24, (void **)&xq))) return st;
  if ((st = efe_ws(c, 43, nq * 8, (void **)&wq))) return st;
  if ((st = efe_ws(c, 44, nq * (MLP_IN + 1) * 4, (void **)&feat))) return st;
  if ((st = efe_ws(c, 45, 256, (void **)&sums))) return st;
  if ((st = efe_ws(c, 46, 64 * 4, (void **)&dnorm))) return st;
  y = feat + nq * MLP_IN;
  if ((st = efe_get_quadrature(c, xq, wq))) return st;
  HIPCHK(c, hipMemcpyAsync(dnorm, norm, 2 * MLP_IN * sizeof(float), hipMemcpyHostToDevice,
                           c->stream));
  k_descriptors<<<cdiv(nq, 256), 256, 0, c->stream>>>(nq, xq, c->natoms, c->d_xyz, sad, dnorm,
                                                      dnorm + MLP_IN, feat);
  HIPCHK(c, hipGetLastError());
  if ((st = mlp_forward(c->stream, params, feat, nq, y, nullptr))) {
    c->err = efe_last_error(nullptr);
    return st;
  }
  k_fill_f64<<<1, 64, 0, c->stream>>>(2, sums, 0.0);
  k_guess<<<(int)std::min<int64_t>(cdiv(nq, 256), 2048), 256, 0, c->stream>>>(
      nq, sad, y, (double)norm[2 * MLP_IN], wq, rho, sums);
  HIPCHK(c, hipGetLastError());
  double h[2];
  HIPCHK(c, hipMemcpyAsync(h, sums, 16, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double n_el = 0.0;
  for (double z : c->Z) n_el += z;
  const double f = h[0] > 0.0 ? n_el / h[0] : INFINITY;
  *factor = f;
  if (h[1] != 0.0 || !std::isfinite(f) || f < 0.9 || f > 1.1) {
    if (h[1] != 0.0) *factor = NAN;
    return efe_set_density(c, sad);
  }
  k_scale_f64<<<cdiv(nq, 256), 256, 0, c->stream>>>(nq, rho, f);
  HIPCHK(c, hipGetLastError());
  *used_fallback = 0;
  return efe_set_density(c, rho);
}
