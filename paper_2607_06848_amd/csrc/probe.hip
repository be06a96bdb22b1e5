// Operand/accumulator layout check of the MFMA instructions used by the cell
// GEMMs: one wave multiplies a 16 x K and a K x 16 matrix with the lane
// mappings the kernels assume and writes the 16 x 16 product row-major.
#include "efe_internal.h"

typedef double v4d_p __attribute__((ext_vector_type(4)));
typedef float v4f_p __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf_p __attribute__((ext_vector_type(8)));

__global__ void k_probe(int which, const double *__restrict__ A, const double *__restrict__ B,
                        double *__restrict__ D) {
  const int lane = threadIdx.x;
  const int li = lane % 16, lk = lane / 16;
  if (which == 0) {   // v_mfma_f64_16x16x4: D row 4 v + l/16
    v4d_p acc = {0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(A[li * 4 + lk], B[lk * 16 + li], acc, 0, 0, 0);
    for (int v = 0; v < 4; ++v) D[(4 * v + lk) * 16 + li] = acc[v];
  } else if (which == 1) {   // v_mfma_f32_16x16x4: D row 4 (l/16) + v
    v4f_p acc = {0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32((float)A[li * 4 + lk], (float)B[lk * 16 + li], acc,
                                               0, 0, 0);
    for (int v = 0; v < 4; ++v) D[(4 * lk + v) * 16 + li] = acc[v];
  } else {   // v_mfma_f32_16x16x32_bf16: k = 8 (l/16) + e for A and B, D row 4 (l/16) + v
    v8bf_p a, b;
    for (int e = 0; e < 8; ++e) {
      a[e] = (__bf16)(float)A[li * 32 + 8 * lk + e];
      b[e] = (__bf16)(float)B[(8 * lk + e) * 16 + li];
    }
    v4f_p acc = {0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    for (int v = 0; v < 4; ++v) D[(4 * lk + v) * 16 + li] = acc[v];
  }
}

extern "C" efe_status efe_probe_mfma(int32_t which, const double *A, const double *B, double *D) {
  if (which < 0 || which > 2 || !A || !B || !D) return EFE_EINVAL;
  k_probe<<<1, 64>>>(which, A, B, D);
  if (hipGetLastError() != hipSuccess) return EFE_EHIP;
  if (hipDeviceSynchronize() != hipSuccess) return EFE_EHIP;
  return EFE_OK;
}
