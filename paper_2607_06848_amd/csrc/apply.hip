// Application of the EFE Hamiltonian H^E = T^T Hhat T (Sec. II.B, Eq.
// Discrete_Eig_Gen_H), the exact overlap M^E and its approximate inverse
// (Eq. MEInvApprox) to a block of node-major vectors.
//
// With T = [[I, -C^T], [0, I]] the apply of Y = H^E X runs as
//   pre        Xh = s X^C - C^T X^E,  Y^C = B^T X^E       (node-major lists)
//   project    W  = D (P^C Xh + P^phi X^E)                 (projector rows)
//   cell       Y^C += sum_c P_c^T H_c P_c Xh               (MFMA cell GEMM,
//              eight colour passes, no two cells of a pass share a node)
//   expand     Y^C += P^C^T W
//   enrichment Y^E  = H^phiphi X^E + P^phi^T W + B Xh - C Y^C
// where s = 1, or 1/m when the caller folds the CFE part of (M~^E)^-1 in.
#include <algorithm>

#include "efe_device.h"

typedef double v4d __attribute__((ext_vector_type(4)));

// columns per lane (x 64) of the row-reduction kernels
constexpr int POST_Q = 3;

// value of v in lane l (l wave-uniform), for every lane: two readlanes
__device__ inline double lane_bcast(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// block index of the calling work-group under an XcdSplit, or -1
__device__ inline int64_t xcd_block(const XcdSplit &x) {
  const int xcd = blockIdx.x % 8;
  const int64_t i = x.off[xcd] + blockIdx.x / 8;
  return i < x.off[xcd + 1] ? i : -1;
}

// ------------------------------------------------------------------ pre
// One wave per group of 8 consecutive nodes, one lane per column (up to 192
// columns per pass, three per lane).  For every atom of the group's union
// the nine X^E rows are read once and applied to all eight nodes with the
// group-major coefficients (uniform over the wave, so they come through the
// scalar cache): Xh = s X^C - C^T X^E and Y^C = B^T X^E.
constexpr int PRE_Q = 3;
__global__ __launch_bounds__(256) void k_pre(int64_t n_nodes, int ncols, const double *__restrict__ XC,
                                             int64_t ldx, const double *__restrict__ scale,
                                             const double *__restrict__ minv,
                                             const double *__restrict__ XE, int64_t lde,
                                             const int32_t *__restrict__ g_ptr,
                                             const int32_t *__restrict__ g_atom,
                                             const double *__restrict__ Cg,
                                             const double *__restrict__ Bg, int nf,
                                             double *__restrict__ Xh, int64_t ldh,
                                             double *Y, int64_t ldy) {
  const int64_t grp =
      (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
  const int lane = threadIdx.x % 64;
  const int64_t n0 = grp * 8;
  if (n0 >= n_nodes) return;
  const int nn = (int)min<int64_t>(8, n_nodes - n0);
  double s[8];
  bool inner[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    inner[j] = j < nn && minv[n0 + j] != 0.0;
    s[j] = j < nn ? (scale ? scale[n0 + j] : 1.0) : 0.0;
  }
  const int32_t a0 = g_ptr[grp], a1 = g_ptr[grp + 1];
  for (int c0 = 0; c0 < ncols; c0 += 64 * PRE_Q) {
    double xh[PRE_Q][8], y[PRE_Q][8];
#pragma unroll
    for (int q = 0; q < PRE_Q; ++q) {
      const int col = c0 + 64 * q + lane;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        // unconditional loads at clamped addresses keep every load of the
        // group in flight at once; the select drops what they brought in
        const double xv = XC[(n0 + min(j, nn - 1)) * ldx + min(col, ncols - 1)];
        xh[q][j] = (inner[j] && col < ncols) ? s[j] * xv : 0.0;
        y[q][j] = 0.0;
      }
    }
    for (int32_t a = a0; a < a1; ++a) {
      const double *xe = XE + (int64_t)g_atom[a] * nf * lde;
      const double *cg = Cg + (int64_t)a * nf * 8, *bg = Bg + (int64_t)a * nf * 8;
      for (int k = 0; k < nf; ++k) {
        double v[PRE_Q];
#pragma unroll
        for (int q = 0; q < PRE_Q; ++q) {
          const int col = c0 + 64 * q + lane;
          v[q] = xe[(int64_t)k * lde + min(col, ncols - 1)];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const double cj = cg[k * 8 + j], bj = bg[k * 8 + j];
#pragma unroll
          for (int q = 0; q < PRE_Q; ++q) {
            xh[q][j] -= cj * v[q];
            y[q][j] += bj * v[q];
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < PRE_Q; ++q) {
      const int col = c0 + 64 * q + lane;
      if (col >= ncols) continue;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        if (j >= nn) continue;
        Xh[(n0 + j) * ldh + col] = inner[j] ? xh[q][j] : 0.0;
        if (Y) Y[(n0 + j) * ldy + col] = inner[j] ? y[q][j] : 0.0;
      }
    }
  }
}

// ------------------------------------------------------------------ cell GEMM
// Cell GEMM, second form: one work-group = one cell of the colour and a
// part of its row blocks, all (up to 160) columns.  Each wave keeps RBW row
// blocks x CBM column blocks of accumulators, so every cell-matrix fragment
// loaded from memory feeds CBM MFMAs.  The gathered block of Xh streams
// through LDS in 16-row chunks, double buffered; the cell-matrix fragments
// of the next chunk are loaded into registers while the current chunk is
// multiplied.  T = double (v_mfma_f64_16x16x4) or float
// (v_mfma_f32_16x16x4, FP32 accumulation).
template <typename T>
struct CellMfma;
template <>
struct CellMfma<double> {
  typedef v4d acc_t;
  // LDS row stride for NC columns: the two 16-lane rows of a half-wave read
  // hit disjoint banks
  static constexpr int ncp(int NC) { return NC == 16 ? 16 : NC + 16; }
  __device__ static inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator register v of lane l holds row 4 v + l/16
  __device__ static inline int row(int v, int lk) { return 4 * v + lk; }
};
typedef float v4f __attribute__((ext_vector_type(4)));
template <>
struct CellMfma<float> {
  typedef v4f acc_t;
  // LDS row stride for NC columns: the four 16-lane rows of a wave read hit
  // disjoint banks
  static constexpr int ncp(int NC) { return NC == 16 ? 16 : NC + 48; }
  __device__ static inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator register v of lane l holds row 4 (l/16) + v
  __device__ static inline int row(int v, int lk) { return 4 * lk + v; }
};

// waves per SIMD the wide tiles are compiled for: the FP64 accumulators of
// one row block x ten column blocks leave room for three, the FP32 ones for four
template <typename T, int CBM>
constexpr int cell_waves() {
  return CBM == 1 ? 1 : (sizeof(T) == 8 ? 3 : 4);
}

template <typename T, int RBW, int CBM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(cell_waves<T, CBM>()))) void k_cell2(int ncells, int nparts,
                                               const int32_t *__restrict__ cells,
                                               const int32_t *__restrict__ c2g, int nloc, int RB,
                                               int KS, const T *__restrict__ Ht,
                                               const double *__restrict__ Xh, int64_t ldx,
                                               double *__restrict__ Y, int64_t ldy,
                                               const double *__restrict__ minv, int ncols) {
  typedef CellMfma<T> M;
  typedef typename M::acc_t acc_t;
  constexpr int NC = CBM * 16, KC = 16, EPT = KC * NC / 256;
  __shared__ T Xs[2][KC][M::ncp(NC)];
  __shared__ int32_t gs[EFE_MAXLOC];   // the cell's node numbers
  const int b = blockIdx.x;
  const int xcd = b % 8, slot = b / 8;
  const int ci = (slot / nparts) * 8 + xcd;
  const int part = slot % nparts;
  if (ci >= ncells) return;
  const int cell = cells[ci];
  const int32_t *g = c2g + (int64_t)cell * nloc;
  const int t = threadIdx.x, wave = t / 64, lane = t % 64, li = lane % 16, lk = lane / 16;
  for (int l = t; l < nloc; l += 256) gs[l] = g[l];
  __syncthreads();
  const int rbase = (part * 4 + wave) * RBW;
  const int CB = (ncols + 15) / 16;
  const int NCH = (KS + 3) / 4;
  const T *hp = Ht + ((int64_t)cell * RB) * KS * 64 + lane;

  T a0[4][RBW], a1[4][RBW];
  acc_t acc[RBW][CBM];
#pragma unroll
  for (int r = 0; r < RBW; ++r)
#pragma unroll
    for (int cb = 0; cb < CBM; ++cb) acc[r][cb] = (acc_t){0, 0, 0, 0};

  // Loads are unconditional, at clamped addresses, and nothing consumes a
  // loaded value before it is needed, so the compiler waits only for the
  // current chunk's operands and the next chunk's loads stay in flight.
  // Out-of-range X rows and columns are zeroed when they are written to LDS;
  // a clamped A fragment then multiplies zero rows of Xs (k past the end) or
  // feeds accumulators that are never stored (row blocks past the end).
  // wide tiles read the gathered rows as pairs of doubles (ldx even, so the
  // pairs never cross a row) with 32-bit element offsets (the host checks
  // n_nodes * ldx < 2^31)
  constexpr bool PAIRS = NC >= 32;
  constexpr int NP = PAIRS ? NC / 2 : NC, EPT2 = PAIRS ? KC * NP / 256 : EPT;
  static_assert(KC * NP % 256 == 0, "the gather must cover the chunk exactly");
  const int NPV = (ncols + 1) / 2;
  double2 xr[EPT2];
  auto stage_load = [&](int ch) {
#pragma unroll
    for (int j = 0; j < EPT2; ++j) {
      const int idx = t + 256 * j, r = idx / NP, cp = idx % NP, k = ch * KC + r;
      if constexpr (PAIRS) {
        const uint32_t off = (uint32_t)gs[min(k, nloc - 1)] * (uint32_t)ldx +
                             2u * (uint32_t)min(cp, NPV - 1);
        xr[j] = *reinterpret_cast<const double2 *>(Xh + off);
      } else {
        xr[j].x = Xh[(int64_t)gs[min(k, nloc - 1)] * ldx + min(cp, ncols - 1)];
      }
    }
  };
  auto stage_store = [&](int buf, int ch) {
#pragma unroll
    for (int j = 0; j < EPT2; ++j) {
      const int idx = t + 256 * j, r = idx / NP, cp = idx % NP, k = ch * KC + r;
      const bool kr = k < nloc;
      if constexpr (PAIRS) {
        Xs[buf][r][2 * cp] = (kr && 2 * cp < ncols) ? (T)xr[j].x : (T)0;
        Xs[buf][r][2 * cp + 1] = (kr && 2 * cp + 1 < ncols) ? (T)xr[j].y : (T)0;
      } else {
        Xs[buf][r][cp] = (kr && cp < ncols) ? (T)xr[j].x : (T)0;
      }
    }
  };
  auto a_load = [&](int ch, T (&dst)[4][RBW]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int r = 0; r < RBW; ++r)
        dst[s][r] = hp[((int64_t)min(rbase + r, RB - 1) * KS + min(ch * 4 + s, KS - 1)) * 64];
  };
  // k steps past the end meet zero rows of Xs and zero A fragments, and
  // column blocks past the end zero columns: all MFMAs run unconditionally
  auto compute = [&](int buf, const T (&src)[4][RBW]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      T bv[CBM];
#pragma unroll
      for (int cb = 0; cb < CBM; ++cb) bv[cb] = Xs[buf][s * 4 + lk][cb * 16 + li];
#pragma unroll
      for (int r = 0; r < RBW; ++r)
#pragma unroll
        for (int cb = 0; cb < CBM; ++cb) acc[r][cb] = M::op(src[s][r], bv[cb], acc[r][cb]);
    }
  };
  auto step = [&](int ch, const T (&cur)[4][RBW], T (&nxt)[4][RBW], int buf) {
    const bool more = ch + 1 < NCH;
    if (more) {
      stage_load(ch + 1);
      a_load(ch + 1, nxt);
    }
    compute(buf, cur);
    if (more) stage_store(buf ^ 1, ch + 1);
    __syncthreads();
  };

  stage_load(0);
  a_load(0, a0);
  stage_store(0, 0);
  __syncthreads();
  for (int ch = 0; ch < NCH; ch += 2) {
    step(ch, a0, a1, 0);
    if (ch + 1 < NCH) step(ch + 1, a1, a0, 1);
  }
  // scatter: per row block, all reads of Y first, then all writes, so the
  // reads overlap instead of each waiting for the one before
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rb = rbase + r;
    if (rb >= RB) continue;
    int64_t node[4];
    bool ok[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rb * 16 + M::row(v, lk);
      node[v] = gs[min(row, nloc - 1)];
      ok[v] = row < nloc;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) ok[v] = ok[v] && minv[node[v]] != 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double yv[CBM];
#pragma unroll
      for (int cb = 0; cb < CBM; ++cb) yv[cb] = Y[node[v] * ldy + min(cb * 16 + li, ncols - 1)];
#pragma unroll
      for (int cb = 0; cb < CBM; ++cb) {
        const int col = cb * 16 + li;
        if (ok[v] && cb < CB && col < ncols) Y[node[v] * ldy + col] = yv[cb] + (double)acc[r][cb][v];
      }
    }
  }
}

// BF16 variant: v_mfma_f32_16x16x32_bf16, FP32 accumulation.  A operand tile
// [cell][rb][ks32][lane][8]: lane l holds H[16 rb + l%16][32 ks + 8 (l/16) + e];
// the gathered block is kept transposed in LDS (XT[col][k]) so that the eight
// k values of a B operand are one 16-byte read.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ inline __bf16 to_bf16(double x) { return (__bf16)(float)x; }

template <int NT>
__global__ __launch_bounds__(256) void k_cell_bf16(int ncells, int ntiles,
                                                   const int32_t *__restrict__ cells,
                                                   const int32_t *__restrict__ c2g, int nloc,
                                                   int RB, int KS32, const v8bf *__restrict__ Ht,
                                                   const double *__restrict__ Xh, int64_t ldx,
                                                   double *__restrict__ Y, int64_t ldy,
                                                   const double *__restrict__ minv, int ncols) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int KP = KS32 * 32;
  const int SK = KP + 8;                   // row stride of XT in bf16 elements
  __bf16 *XT = (__bf16 *)smem;             // [NT][SK]
  const int b = blockIdx.x;
  const int xcd = b % 8, slot = b / 8;
  const int ci = (slot / ntiles) * 8 + xcd;
  const int tile = slot % ntiles;
  if (ci >= ncells) return;
  const int cell = cells[ci];
  const int col0 = tile * NT;
  const int32_t *g = c2g + (int64_t)cell * nloc;
  for (int idx = threadIdx.x; idx < KP * NT; idx += 256) {
    const int r = idx / NT, cc = idx % NT;
    double v = 0.0;
    if (r < nloc && col0 + cc < ncols) v = Xh[(int64_t)g[r] * ldx + col0 + cc];
    XT[cc * SK + r] = to_bf16(v);
  }
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int li = lane % 16, lk = lane / 16;
  for (int rb = wave; rb < RB; rb += 4) {
    v4f acc[NT / 16];
    for (int cb = 0; cb < NT / 16; ++cb) acc[cb] = (v4f){0.f, 0.f, 0.f, 0.f};
    const v8bf *hp = Ht + (((int64_t)cell * RB + rb) * KS32) * 64 + lane;
    for (int ks = 0; ks < KS32; ++ks) {
      const v8bf a = hp[(int64_t)ks * 64];
#pragma unroll
      for (int cb = 0; cb < NT / 16; ++cb) {
        const v8bf bv = *(const v8bf *)(XT + (cb * 16 + li) * SK + ks * 32 + lk * 8);
        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv, acc[cb], 0, 0, 0);
      }
    }
    for (int v = 0; v < 4; ++v) {
      const int row = rb * 16 + 4 * lk + v;
      if (row >= nloc) continue;
      const int64_t node = g[row];
      if (minv[node] == 0.0) continue;
#pragma unroll
      for (int cb = 0; cb < NT / 16; ++cb) {
        const int col = col0 + cb * 16 + li;
        if (col < ncols) Y[node * ldy + col] += (double)acc[cb][v];
      }
    }
  }
}

// ------------------------------------------------------------------ projectors
// W[I] += D_I sum_s P^C_s Xh[node_s] over one work item (atom, support-list
// range); the items of a node region run back to back, so the rows of Xh
// they read are shared through the caches.  Waves take one support node at a
// time (wave-uniform) for up to 192 columns, three per lane.
__global__ __launch_bounds__(256) void k_kb_project(int ncols, const int32_t *__restrict__ items,
                                                    XcdSplit xs,
                                                    const int32_t *__restrict__ kbnode,
                                                    const double *__restrict__ Pc,
                                                    const double *__restrict__ Xh, int64_t ldh,
                                                    const double *__restrict__ D,
                                                    double *__restrict__ W) {
  __shared__ double red[3][64 * POST_Q];
  const int64_t item = xcd_block(xs);
  if (item < 0) return;
  const int32_t *it = items + 3 * item;
  const int I = it[0];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
  const int lane = threadIdx.x % 64;
  const int c0 = blockIdx.y * 64 * POST_Q;
  double acc[POST_Q] = {0.0, 0.0, 0.0};
  // entries it[1] + wave + 4 i: node numbers and coefficients come in 64 at
  // a time by vector loads and reach the wave by readlane; clamped columns
  // keep the row loads unconditional (their sums are not stored)
  const int32_t s0 = it[1], s1 = it[2];
  for (int32_t sb = s0 + wave; sb < s1; sb += 256) {
    const int cnt = min(64, (s1 - sb + 3) / 4);
    const int32_t sl = min(sb + 4 * lane, s1 - 1);
    const int32_t nodes = kbnode[sl];
    const double pv = Pc[sl];
    for (int i = 0; i < cnt; ++i) {
      const int64_t node = __builtin_amdgcn_readlane(nodes, i);
      const double p = lane_bcast(pv, i);
#pragma unroll
      for (int q = 0; q < POST_Q; ++q)
        acc[q] += p * Xh[node * ldh + min(c0 + 64 * q + lane, ncols - 1)];
    }
  }
  if (wave > 0)
#pragma unroll
    for (int q = 0; q < POST_Q; ++q) red[wave - 1][64 * q + lane] = acc[q];
  __syncthreads();
  if (wave == 0)
#pragma unroll
    for (int q = 0; q < POST_Q; ++q) {
      const int col = c0 + 64 * q + lane;
      if (col < ncols)
        atomicAdd(&W[(int64_t)I * ncols + col],
                  D[I] * (acc[q] + red[0][64 * q + lane] + red[1][64 * q + lane] +
                          red[2][64 * q + lane]));
    }
}

// W[I] = D_I sum_f P^phi_If XE_f (first term of the projector coefficients):
// one work-group per (projector, 64 columns); the four waves take every
// fourth f and their sums meet in LDS in a fixed order
__global__ __launch_bounds__(256) void k_kb_w_pphi(int ncols, int64_t n_enr,
                                                   const double *__restrict__ Pphi,
                                                   const double *__restrict__ XE, int64_t lde,
                                                   const double *__restrict__ D,
                                                   double *__restrict__ W) {
  __shared__ double red[4][64];
  const int I = blockIdx.x;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int col = blockIdx.y * 64 + lane;
  const int cc = min(col, ncols - 1);
  const double *p = Pphi + (int64_t)I * n_enr;
  double acc = 0.0;
  for (int64_t f = wave; f < n_enr; f += 4) acc += p[f] * XE[f * lde + cc];
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && col < ncols)
    W[(int64_t)I * ncols + col] = D[I] * (((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]);
}

// Y^C[node] += sum_e P^C_e W[atom_e] over the node's projector entries.  One
// wave per 8 consecutive nodes, three columns per lane.  The nodes' entry
// pointers and (when the group has at most 64 entries, as usual) their
// entries, contiguous for consecutive nodes, come in by vector loads and
// reach the wave by readlane.
__global__ __launch_bounds__(256) void k_kb_expand(int64_t n_nodes, int ncols,
                                                   const int32_t *__restrict__ kbnm_ptr,
                                                   const int32_t *__restrict__ kbnm_atom,
                                                   const double *__restrict__ Pc_nm,
                                                   const double *__restrict__ W,
                                                   double *__restrict__ Y, int64_t ldy) {
  const int64_t grp =
      (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
  const int64_t n0 = grp * 8;
  if (n0 >= n_nodes) return;
  const int lane = threadIdx.x % 64;
  const int nn = (int)min<int64_t>(8, n_nodes - n0);
  const int32_t pv = kbnm_ptr[n0 + min(lane, nn)];   // pointers of nodes n0 .. n0 + nn
  const int32_t eb = __builtin_amdgcn_readlane(pv, 0), ee = __builtin_amdgcn_readlane(pv, nn);
  if (eb == ee) return;
  const bool vec = ee - eb <= 64;
  const int32_t el = min(eb + lane, ee - 1);
  const int32_t av = kbnm_atom[el];
  const double cv = Pc_nm[el];
  for (int c0 = 0; c0 < ncols; c0 += 64 * POST_Q) {
    for (int j = 0; j < nn; ++j) {
      const int32_t e0 = __builtin_amdgcn_readlane(pv, j);
      const int32_t e1 = __builtin_amdgcn_readlane(pv, j + 1);
      if (e0 == e1) continue;
      double acc[POST_Q] = {0.0, 0.0, 0.0};
      for (int32_t e = e0; e < e1; ++e) {
        const int32_t atom = vec ? __builtin_amdgcn_readlane(av, e - eb) : kbnm_atom[e];
        const double p = vec ? lane_bcast(cv, e - eb) : Pc_nm[e];
        const double *w = W + (int64_t)atom * ncols;
#pragma unroll
        for (int q = 0; q < POST_Q; ++q) acc[q] += p * w[min(c0 + 64 * q + lane, ncols - 1)];
      }
      double *y = Y + (n0 + j) * ldy;
#pragma unroll
      for (int q = 0; q < POST_Q; ++q) {
        const int col = c0 + 64 * q + lane;
        if (col < ncols) y[col] += acc[q];
      }
    }
  }
}

// Y^E[I] += sum_s (B_s Xh[node_s] - C_s Y[node_s]) over one work item
// (atom I, range of its support list).  Each wave takes one support node at a
// time (wave-uniform, so the 2 x nf coefficients come through the scalar
// cache) for up to 192 columns, three per lane; the four waves' sums meet in
// LDS and are added to Y^E once per item.
__global__ __launch_bounds__(256) void k_enr_post(int nf, int ncols,
                                                  const int32_t *__restrict__ items, XcdSplit xs,
                                                  const int32_t *__restrict__ snode,
                                                  const double *__restrict__ B_am,
                                                  const double *__restrict__ C_am,
                                                  const double *__restrict__ Xh, int64_t ldh,
                                                  const double *__restrict__ Y, int64_t ldy,
                                                  double *__restrict__ YE, int64_t lde) {
  __shared__ double red[3][9][64 * POST_Q];
  const int64_t item = xcd_block(xs);
  if (item < 0) return;
  const int32_t *it = items + 3 * item;
  const int I = it[0];
  const int32_t s0 = it[1], s1 = it[2];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
  const int lane = threadIdx.x % 64;
  const int c0 = blockIdx.y * 64 * POST_Q;
  double acc[POST_Q][9];
#pragma unroll
  for (int q = 0; q < POST_Q; ++q)
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[q][k] = 0.0;
  // This wave takes support entries s0 + wave + 4 i.  Their node numbers
  // come in 64 at a time by one vector load, and the 2 nf coefficients of an
  // entry by one vector load (lane k: B_k, lane 16 + k: C_k) one entry ahead
  // of their use; readlane hands both to the wave.  Columns are clamped, so
  // every load is unconditional; the sums of clamped columns are not stored.
  const int kl = lane & 15;
  const double *csrc = lane < 16 ? B_am : C_am;
  auto cload = [&](int32_t s) -> double {
    return csrc[(int64_t)min(s, s1 - 1) * nf + min(kl, nf - 1)];
  };
  for (int32_t sb = s0 + wave; sb < s1; sb += 256) {
    const int cnt = min(64, (s1 - sb + 3) / 4);
    const int32_t nodes = snode[min(sb + 4 * lane, s1 - 1)];
    double cv = cload(sb);
    for (int i = 0; i < cnt; ++i) {
      const int32_t s = sb + 4 * i;
      const int64_t node = __builtin_amdgcn_readlane(nodes, i);
      const double cn = cload(s + 4);
      double xh[POST_Q], y[POST_Q];
#pragma unroll
      for (int q = 0; q < POST_Q; ++q) {
        const int col = min(c0 + 64 * q + lane, ncols - 1);
        xh[q] = Xh[node * ldh + col];
        y[q] = Y[node * ldy + col];
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const double b = k < nf ? lane_bcast(cv, k) : 0.0;
        const double c = k < nf ? lane_bcast(cv, 16 + k) : 0.0;
#pragma unroll
        for (int q = 0; q < POST_Q; ++q) acc[q][k] += b * xh[q] - c * y[q];
      }
      cv = cn;
    }
  }
  if (wave > 0)
#pragma unroll
    for (int q = 0; q < POST_Q; ++q)
#pragma unroll
      for (int k = 0; k < 9; ++k) red[wave - 1][k][64 * q + lane] = acc[q][k];
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < POST_Q; ++q) {
      const int col = c0 + 64 * q + lane;
      if (col >= ncols) continue;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const double v = acc[q][k] + red[0][k][64 * q + lane] + red[1][k][64 * q + lane] +
                         red[2][k][64 * q + lane];
        if (k < nf) atomicAdd(&YE[(int64_t)(I * nf + k) * lde + col], v);
      }
    }
  }
}

// ------------------------------------------------------------- one column
// Single-vector forms of the four row kernels (the Lanczos bound applies
// H^E to one vector): threads run over nodes or support entries instead of
// columns, so no lane idles.  Same sums, same order within each node.

// sum of x over the work-group (256 threads), in a fixed order
__device__ inline double block_sum256(double x, double *red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = x;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(256) void k_pre1(int64_t n_nodes, const double *__restrict__ XC,
                                              int64_t ldx, const double *__restrict__ scale,
                                              const double *__restrict__ minv,
                                              const double *__restrict__ XE, int64_t lde,
                                              const int32_t *__restrict__ g_ptr,
                                              const int32_t *__restrict__ g_atom,
                                              const double *__restrict__ Cg,
                                              const double *__restrict__ Bg, int nf,
                                              double *__restrict__ Xh, int64_t ldh, double *Y,
                                              int64_t ldy) {
  const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (n >= n_nodes) return;
  const int64_t grp = n / 8;
  const int j = (int)(n % 8);
  const bool inner = minv[n] != 0.0;
  double xh = inner ? (scale ? scale[n] : 1.0) * XC[n * ldx] : 0.0, y = 0.0;
  for (int32_t a = g_ptr[grp]; a < g_ptr[grp + 1]; ++a) {
    const double *xe = XE + (int64_t)g_atom[a] * nf * lde;
    for (int k = 0; k < nf; ++k) {
      const double v = xe[(int64_t)k * lde];
      xh -= Cg[((int64_t)a * nf + k) * 8 + j] * v;
      y += Bg[((int64_t)a * nf + k) * 8 + j] * v;
    }
  }
  Xh[n * ldh] = inner ? xh : 0.0;
  if (Y) Y[n * ldy] = inner ? y : 0.0;
}

// W[I] += D_I sum_s P^C_s Xh[node_s] over one work item, threads over entries
__global__ __launch_bounds__(256) void k_kb_project1(const int32_t *__restrict__ items,
                                                     const int32_t *__restrict__ kbnode,
                                                     const double *__restrict__ Pc,
                                                     const double *__restrict__ Xh, int64_t ldh,
                                                     const double *__restrict__ D,
                                                     double *__restrict__ W) {
  __shared__ double red[4];
  const int32_t *it = items + 3 * (int64_t)blockIdx.x;
  const int I = it[0];
  double acc = 0.0;
  for (int32_t s = it[1] + threadIdx.x; s < it[2]; s += 256) acc += Pc[s] * Xh[(int64_t)kbnode[s] * ldh];
  const double t = block_sum256(acc, red);
  if (threadIdx.x == 0) atomicAdd(&W[I], D[I] * t);
}

// Y^C[node] += sum_e P^C_e W[atom_e], one thread per node
__global__ __launch_bounds__(256) void k_kb_expand1(int64_t n_nodes,
                                                    const int32_t *__restrict__ kbnm_ptr,
                                                    const int32_t *__restrict__ kbnm_atom,
                                                    const double *__restrict__ Pc_nm,
                                                    const double *__restrict__ W,
                                                    double *__restrict__ Y, int64_t ldy) {
  const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (n >= n_nodes) return;
  const int32_t e0 = kbnm_ptr[n], e1 = kbnm_ptr[n + 1];
  if (e0 == e1) return;
  double acc = 0.0;
  for (int32_t e = e0; e < e1; ++e) acc += Pc_nm[e] * W[kbnm_atom[e]];
  Y[n * ldy] += acc;
}

// Y^E[I] += sum_s (B_s Xh[node_s] - C_s Y[node_s]) over one work item, threads
// over entries, one work-group sum per enrichment function
__global__ __launch_bounds__(256) void k_enr_post1(int nf, const int32_t *__restrict__ items,
                                                   const int32_t *__restrict__ snode,
                                                   const double *__restrict__ B_am,
                                                   const double *__restrict__ C_am,
                                                   const double *__restrict__ Xh, int64_t ldh,
                                                   const double *__restrict__ Y, int64_t ldy,
                                                   double *__restrict__ YE, int64_t lde) {
  __shared__ double red[4];
  const int32_t *it = items + 3 * (int64_t)blockIdx.x;
  const int I = it[0];
  const int32_t s0 = it[1], s1 = it[2];
  double acc[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) acc[k] = 0.0;
  for (int32_t s = s0 + threadIdx.x; s < s1; s += 256) {
    const int64_t node = snode[s];
    const double x = Xh[node * ldh], y = Y[node * ldy];
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k < nf) acc[k] += B_am[(int64_t)s * nf + k] * x - C_am[(int64_t)s * nf + k] * y;
  }
  for (int k = 0; k < nf; ++k) {
    const double t = block_sum256(acc[k], red);
    if (threadIdx.x == 0) atomicAdd(&YE[(int64_t)(I * nf + k) * lde], t);
  }
}

// ------------------------------------------------------------------ overlap
// CFE rows: Y = w X (w = m or 1/m, zero on the boundary)
__global__ void k_rowscale(int64_t n, int ncols, const double *__restrict__ w,
                           const double *__restrict__ X, int64_t ldx, double *__restrict__ Y,
                           int64_t ldy) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * ncols) return;
  const int64_t r = idx / ncols, c = idx % ncols;
  Y[r * ldy + c] = w[r] * X[r * ldx + c];
}

// Enrichment rows: Y_I = inv_I X_I for each atom block
__global__ void k_enr_block_apply(int natoms, int nf, int ncols, const double *__restrict__ inv,
                                  const double *__restrict__ X, int64_t ldx,
                                  double *__restrict__ Y, int64_t ldy) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)natoms * nf * ncols) return;
  const int c = idx % ncols;
  const int64_t f = idx / ncols;
  const int I = f / nf, k = f % nf;
  const double *a = inv + ((int64_t)I * nf + k) * nf;
  double acc = 0.0;
  for (int l = 0; l < nf; ++l) acc += a[l] * X[((int64_t)I * nf + l) * ldx + c];
  Y[f * ldy + c] = acc;
}

// ------------------------------------------------------------------ launchers
// Colour passes of the cell GEMM in column chunks of 16 CBM.
template <typename T, int RBW, int CBM>
static void launch_cell2(efe_ctx *c, const T *Ht, const double *Xh, int64_t ldh, double *Y,
                         int64_t ldy, int ncols) {
  const int nparts = (int)cdiv(c->RB, 4 * RBW);
  for (int col0 = 0; col0 < ncols; col0 += 16 * CBM) {
    const int nch = std::min(16 * CBM, ncols - col0);
    for (int col = 0; col < 8; ++col) {
      const int nc = c->colour_offsets[col + 1] - c->colour_offsets[col];
      if (nc == 0) continue;
      const int64_t nblk = cdiv(nc, 8) * 8 * nparts;
      const int t = efe_timer_begin(c, CBM == 1 ? EFE_T_CELL_NARROW : EFE_T_CELL);
      k_cell2<T, RBW, CBM><<<nblk, 256, 0, c->stream>>>(
          nc, nparts, c->d_colour_order + c->colour_offsets[col], c->d_c2g, c->nloc, c->RB, c->KS,
          Ht, Xh + col0, ldh, Y + col0, ldy, c->d_minv, nch);
      efe_timer_end(c, CBM == 1 ? EFE_T_CELL_NARROW : EFE_T_CELL, t);
    }
  }
}

efe_status efe_apply_H_internal(efe_ctx *c, const double *XC, int64_t ldx, const double *scale,
                                const double *XE, int64_t lde, double *Y, int64_t ldy, int ncols,
                                int prec) {
  if (!c->have_potential) EFE_FAIL(c, EFE_ESTATE, "no potential set");
  if (ncols <= 0) return EFE_OK;
  if ((prec == EFE_FP32 && !c->have32) || (prec == EFE_BF16 && !c->have16))
    EFE_FAIL(c, EFE_ESTATE, "reduced-precision cell matrices were not built by efe_set_potential");
  efe_status s;
  double *Xh, *W = nullptr;
  // even row length: the cell GEMM reads X^ in pairs of doubles
  const int64_t ldh = (ncols + 1) & ~1;
  if (c->nf > 16) EFE_FAIL(c, EFE_EINVAL, "more than 16 enrichment functions per atom");
  if (c->n_nodes * ldh >= (1ll << 31))
    EFE_FAIL(c, EFE_EINVAL, "n_nodes x columns exceeds the 32-bit offsets of the cell GEMM");
  if ((s = efe_ws(c, 0, (size_t)c->n_nodes * ldh * 8, (void **)&Xh))) return s;
  if (c->nproj && (s = efe_ws(c, 1, (size_t)c->nproj * ncols * 8, (void **)&W))) return s;
  const int nf = c->nf;
  double *YE = Y + c->n_nodes * ldy;
  const int t_cls = ncols <= 16 ? EFE_T_APPLY_NARROW : EFE_T_APPLY;
  const int t_apply = efe_timer_begin(c, t_cls);
  // pre: Xh and Y^C = B^T X^E
  {
    const int t = efe_timer_begin(c, EFE_T_PRE);
    if (ncols == 1)
      k_pre1<<<cdiv(c->n_nodes, 256), 256, 0, c->stream>>>(c->n_nodes, XC, ldx, scale, c->d_minv,
                                                           XE, lde, c->d_g_ptr, c->d_g_atom,
                                                           c->d_Cg, c->d_Bg, nf, Xh, ldh, Y, ldy);
    else
      k_pre<<<cdiv(c->n_nodes, 32), 256, 0, c->stream>>>(c->n_nodes, ncols, XC, ldx, scale,
                                                         c->d_minv, XE, lde, c->d_g_ptr,
                                                         c->d_g_atom, c->d_Cg, c->d_Bg, nf, Xh, ldh,
                                                         Y, ldy);
    efe_timer_end(c, EFE_T_PRE, t);
  }
  // projector coefficients
  if (c->nproj) {
    k_kb_w_pphi<<<dim3(c->nproj, cdiv(ncols, 64)), 256, 0, c->stream>>>(ncols, c->n_enr, c->d_Pphi,
                                                                        XE, lde, c->d_D, W);
    if (c->n_kb_items) {
      XcdSplit xs;
      for (int i = 0; i <= 8; ++i) xs.off[i] = c->kb_items_off[i];
      dim3 grd(8 * xs.max_len(), cdiv(ncols, 64 * POST_Q));
      if (ncols == 1)
        k_kb_project1<<<c->n_kb_items, 256, 0, c->stream>>>(c->d_kb_items, c->d_kbnode, c->d_Pc_am,
                                                            Xh, ldh, c->d_D, W);
      else
        k_kb_project<<<grd, 256, 0, c->stream>>>(ncols, c->d_kb_items, xs, c->d_kbnode,
                                                 c->d_Pc_am, Xh, ldh, c->d_D, W);
    }
  }
  // cell GEMM, colour by colour
  // 160-column register tiles; a single 16-column tile (six row blocks per
  // wave, one part per cell) for narrow blocks such as the Lanczos vector
  if (prec == EFE_FP64 && ncols <= 16) {
    launch_cell2<double, 6, 1>(c, c->d_Htile64, Xh, ldh, Y, ldy, ncols);
  } else if (prec == EFE_FP64) {
    launch_cell2<double, 1, 10>(c, c->d_Htile64, Xh, ldh, Y, ldy, ncols);
  } else if (prec == EFE_FP32 && ncols <= 16) {
    launch_cell2<float, 6, 1>(c, c->d_Htile32, Xh, ldh, Y, ldy, ncols);
  } else if (prec == EFE_FP32) {
    launch_cell2<float, 1, 10>(c, c->d_Htile32, Xh, ldh, Y, ldy, ncols);
  } else {
    const int NT = 32;
    const int ntiles = (int)cdiv(ncols, NT);
    const size_t shm = (size_t)NT * (c->KS32 * 32 + 8) * 2;
    for (int col = 0; col < 8; ++col) {
      const int nc = c->colour_offsets[col + 1] - c->colour_offsets[col];
      if (nc == 0) continue;
      const int64_t nblk = cdiv(nc, 8) * 8 * ntiles;
      const int t = efe_timer_begin(c, EFE_T_CELL);
      k_cell_bf16<32><<<nblk, 256, shm, c->stream>>>(
            nc, ntiles, c->d_colour_order + c->colour_offsets[col], c->d_c2g, c->nloc, c->RB,
            c->KS32, (const v8bf *)c->d_Htile16, Xh, ldh, Y, ldy, c->d_minv, ncols);
      efe_timer_end(c, EFE_T_CELL, t);
    }
  }
  if (c->nproj) {
    if (ncols == 1)
      k_kb_expand1<<<cdiv(c->n_nodes, 256), 256, 0, c->stream>>>(c->n_nodes, c->d_kbnm_ptr,
                                                                 c->d_kbnm_atom, c->d_Pc_nm, W, Y,
                                                                 ldy);
    else
      k_kb_expand<<<cdiv(c->n_nodes, 32), 256, 0, c->stream>>>(c->n_nodes, ncols, c->d_kbnm_ptr,
                                                              c->d_kbnm_atom, c->d_Pc_nm, W, Y, ldy);
  }
  // enrichment rows
  const int t_post = efe_timer_begin(c, EFE_T_POST);
  if (c->n_enr) {
    if ((s = efe_gemm(c, false, false, c->n_enr, ncols, c->n_enr, 1.0, c->d_Hpp, c->n_enr, XE, lde,
                      0.0, YE, ldy)))
      return s;
    if (c->nproj &&
        (s = efe_gemm(c, true, false, c->n_enr, ncols, c->nproj, 1.0, c->d_Pphi, c->n_enr, W, ncols,
                      1.0, YE, ldy)))
      return s;
    if (c->n_enr_items) {
      XcdSplit xs;
      for (int i = 0; i <= 8; ++i) xs.off[i] = c->enr_items_off[i];
      dim3 grd(8 * xs.max_len(), cdiv(ncols, 64 * POST_Q));
      if (ncols == 1)
        k_enr_post1<<<c->n_enr_items, 256, 0, c->stream>>>(nf, c->d_enr_items, c->d_snode,
                                                           c->d_B_am, c->d_C_am, Xh, ldh, Y, ldy,
                                                           YE, ldy);
      else
        k_enr_post<<<grd, 256, 0, c->stream>>>(nf, ncols, c->d_enr_items, xs, c->d_snode,
                                               c->d_B_am, c->d_C_am, Xh, ldh, Y, ldy, YE, ldy);
    }
  }
  efe_timer_end(c, EFE_T_POST, t_post);
  efe_timer_end(c, t_cls, t_apply);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

efe_status efe_transform_cfe(efe_ctx *c, const double *X, int64_t ldx, double *Xh, int64_t ldh,
                             int ncols) {
  if (ncols <= 0) return EFE_OK;
  k_pre<<<cdiv(c->n_nodes, 32), 256, 0, c->stream>>>(c->n_nodes, ncols, X, ldx, nullptr, c->d_minv,
                                                     X + c->n_nodes * ldx, ldx, c->d_g_ptr,
                                                     c->d_g_atom, c->d_Cg, c->d_Bg, c->nf, Xh, ldh,
                                                     nullptr, 0);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

efe_status efe_apply_M_internal(efe_ctx *c, const double *X, int64_t ldx, double *Y, int64_t ldy,
                                int ncols) {
  if (ncols <= 0) return EFE_OK;
  k_rowscale<<<cdiv(c->n_nodes * ncols, 256), 256, 0, c->stream>>>(c->n_nodes, ncols, c->d_m_int,
                                                                   X, ldx, Y, ldy);
  HIPCHK(c, hipGetLastError());
  if (c->n_enr)
    return efe_gemm(c, false, false, c->n_enr, ncols, c->n_enr, 1.0, c->d_Mee, c->n_enr,
                    X + c->n_nodes * ldx, ldx, 0.0, Y + c->n_nodes * ldy, ldy);
  return EFE_OK;
}

efe_status efe_enr_block_inv(efe_ctx *c, const double *XE, int64_t ldx, double *YE, int64_t ldy,
                             int ncols) {
  if (!c->n_enr || ncols <= 0) return EFE_OK;
  const int64_t n = c->n_enr * ncols;
  k_enr_block_apply<<<cdiv(n, 256), 256, 0, c->stream>>>(c->natoms, c->nf, ncols, c->d_Mee_inv, XE,
                                                         ldx, YE, ldy);
  HIPCHK(c, hipGetLastError());
  return EFE_OK;
}

efe_status efe_apply_Minv_internal(efe_ctx *c, const double *X, int64_t ldx, double *Y,
                                   int64_t ldy, int ncols) {
  if (ncols <= 0) return EFE_OK;
  k_rowscale<<<cdiv(c->n_nodes * ncols, 256), 256, 0, c->stream>>>(c->n_nodes, ncols, c->d_minv, X,
                                                                   ldx, Y, ldy);
  HIPCHK(c, hipGetLastError());
  return efe_enr_block_inv(c, X + c->n_nodes * ldx, ldx, Y + c->n_nodes * ldy, ldy, ncols);
}

// ------------------------------------------------------------------ C ABI
static efe_status check_block(efe_ctx *c, const void *X, const void *Y, int ncols, int64_t ld) {
  if (!c) return EFE_EINVAL;
  if (!X || !Y || ncols < 0 || ld < ncols || ld < 1) EFE_FAIL(c, EFE_EINVAL, "bad block arguments");
  if (X == Y) EFE_FAIL(c, EFE_EINVAL, "input and output blocks must differ");
  return EFE_OK;
}

extern "C" efe_status efe_local_potential(efe_ctx *c, double *vq) {
  if (!c) return EFE_EINVAL;
  if (!vq) EFE_FAIL(c, EFE_EINVAL, "null vq");
  return efe_launch_local_potential(c, vq);
}

extern "C" efe_status efe_set_potential(efe_ctx *c, const double *vq, int32_t precisions) {
  if (!c) return EFE_EINVAL;
  if (!vq) EFE_FAIL(c, EFE_EINVAL, "null vq");
  if (precisions & ~((1 << EFE_FP32) | (1 << EFE_BF16))) EFE_FAIL(c, EFE_EINVAL, "bad precision mask");
  return efe_build_operators(c, vq, precisions);
}

// wide blocks go through the apply in column chunks of the cell GEMM's
// register tile, so its workspaces stay n_nodes x 160
static efe_status apply_H_chunked(efe_ctx *c, const double *X, double *Y, int32_t ncols,
                                  int64_t ld, int prec) {
  efe_status s;
  for (int32_t j0 = 0; j0 < ncols; j0 += EFE_COL_CHUNK) {
    const int32_t nc = std::min<int32_t>(EFE_COL_CHUNK, ncols - j0);
    if ((s = efe_apply_H_internal(c, X + j0, ld, nullptr, X + c->n_nodes * ld + j0, ld, Y + j0, ld,
                                  nc, prec)))
      return s;
  }
  return EFE_OK;
}

extern "C" efe_status efe_apply_H(efe_ctx *c, const double *X, double *Y, int32_t ncols,
                                  int64_t ld) {
  efe_status s = check_block(c, X, Y, ncols, ld);
  if (s) return s;
  return apply_H_chunked(c, X, Y, ncols, ld, EFE_FP64);
}

extern "C" efe_status efe_apply_H_prec(efe_ctx *c, const double *X, double *Y, int32_t ncols,
                                       int64_t ld, int32_t prec) {
  efe_status s = check_block(c, X, Y, ncols, ld);
  if (s) return s;
  if (prec != EFE_FP64 && prec != EFE_FP32 && prec != EFE_BF16)
    EFE_FAIL(c, EFE_EINVAL, "bad precision");
  return apply_H_chunked(c, X, Y, ncols, ld, prec);
}

extern "C" efe_status efe_apply_M(efe_ctx *c, const double *X, double *Y, int32_t ncols,
                                  int64_t ld) {
  efe_status s = check_block(c, X, Y, ncols, ld);
  if (s) return s;
  return efe_apply_M_internal(c, X, ld, Y, ld, ncols);
}

extern "C" efe_status efe_apply_Minv_approx(efe_ctx *c, const double *X, double *Y, int32_t ncols,
                                            int64_t ld) {
  efe_status s = check_block(c, X, Y, ncols, ld);
  if (s) return s;
  return efe_apply_Minv_internal(c, X, ld, Y, ld, ncols);
}
