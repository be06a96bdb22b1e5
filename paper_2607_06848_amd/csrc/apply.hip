// Application of the EFE Hamiltonian H^E = T^T Hhat T (Sec. II.B, Eq.
// Discrete_Eig_Gen_H), the exact overlap M^E and its approximate inverse
// (Eq. MEInvApprox) to a block of node-major vectors.
//
// T = [[I, -C^T], [0, I]] is applied when the operator is built: per cell the
// coupling of the orthogonalized basis E_c = B_c - C_c H_c, the enrichment
// block H^E_ee = H^phiphi - C B^T - E C^T and the projector rows
// P~^phi = P^phi - P^C C^T are formed in FP64 (setup.hip).  The apply of
// Y = alpha H^E X (+ the terms of the Chebyshev recurrence) then runs as
//   project    W   = D (P^C s X^C + P~^phi X^E)
//   init       Y^C = alpha P^C^T W + beta Z1 + gamma Z2 + alpha G Cl
//   cell       Y^C += alpha sum_c P_c^T [H_c | E_c^T] [s X^C_c ; X^E_c]
//              Yp_c = E_c s X^C_c       (MFMA cell GEMM, eight colour passes,
//                                        no two cells of a pass share a node)
//   reduce     Y^E = alpha (sum_c Yp_c + H^E_ee X^E + P~^phi^T W) + ...
// where s = 1, or 1/m when the caller folds the CFE part of (M~^E)^-1 in.
#include <algorithm>

#include "efe_device.h"

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

// Streams that a launch reads or writes once and that are far larger than the
// caches (cell matrices, the recurrence blocks, Y of a colour pass, the
// enrichment partial rows) go with the non-temporal hint, so that they do not
// evict what is re-read through L2 (the gathered cell rows, the projector
// support rows).  The hint changes cache policy only, not the values.
template <typename T>
__device__ inline T ld_nt(const T *p) {
  return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ inline void st_nt(T v, T *p) {
  __builtin_nontemporal_store(v, p);
}
__device__ inline double2 ld_nt2(const double *p) {
  const v2d t = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(p));
  return make_double2(t.x, t.y);
}
__device__ inline void st_nt2(double2 v, double *p) {
  const v2d t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<v2d *>(p));
}

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
// Matrix-core operations of the cell GEMM per element type: the operand
// fragments and accumulator layout of v_mfma_f64_16x16x4 (double) and
// v_mfma_f32_16x16x4 (float, FP32 accumulation), and the LDS row strides of
// the gathered block.
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

template <typename T>
struct CellOps {
  int ncells, nparts_c, nparts_e;
  const int32_t *cells, *c2g;
  int nloc, RB, KS, nf, ncols;
  const T *Ht, *Et, *Ee;           // cell Hamiltonians, E_c^T and E_c tiles
  const double *X;                 // CFE rows (even ld, 16-byte aligned)
  int64_t ldx;
  const double *scale, *minv;      // row scale of X (NULL: 1), 1/m (0 on the boundary)
  const double *XE;                // enrichment rows
  int64_t lde;
  double *Y;                       // CFE rows, read-modify-write
  int64_t ldy;
  double alpha;
  double *Yp;                      // enrichment partial rows, one row block per (cell, atom)
  int64_t ldp;
  const int32_t *cell_eptr, *cell_epair, *pair_atom;
  const int64_t *cell_noff;
};

// waves per SIMD the wide tiles are compiled for: the FP64 accumulators of
// one row block x ten column blocks, or the FP32 ones of two, leave room for
// three; the FP32 ones of one row block for four
template <typename T, int RBW, int CBM>
constexpr int cell_waves() {
  return CBM == 1 ? 1 : (sizeof(T) == 8 || RBW > 1 ? 3 : 4);
}

// Cell GEMM of one colour pass of H^E = T^T Hhat T written per cell in the
// orthogonalized basis: with X_c = [s X^C_c ; X^E_c] (the cell's nodes, scaled
// by s, then the rows of its enrichment atoms),
//   Y^C_c += alpha [H_c | E_c^T] X_c          (parts 0 .. nparts_c - 1)
//   Yp_c   = E_c (s X^C_c)                      (parts nparts_c ..: the cell's
//                                               enrichment rows, summed over
//                                               cells afterwards)
// One work-group = one cell of the colour and a part of its row blocks, all
// (up to 160) columns.  Each wave keeps RBW row blocks x CBM column blocks of
// accumulators, so every matrix fragment loaded from memory feeds CBM MFMAs.
// The gathered rows stream through LDS in 16-row chunks, double buffered; the
// matrix fragments of the next chunk are loaded into registers while the
// current chunk is multiplied.  T = double (v_mfma_f64_16x16x4) or float
// (v_mfma_f32_16x16x4, FP32 accumulation).  ENR = false: plain CFE.
template <typename T, int RBW, int CBM, bool ENR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(cell_waves<T, RBW, CBM>())))
void k_cell3(CellOps<T> a) {
  typedef CellMfma<T> M;
  typedef typename M::acc_t acc_t;
  constexpr int NC = CBM * 16, KC = 16;
  __shared__ T Xs[2][KC][M::ncp(NC)];
  // rows of the gathered block: the cell's nodes (CFE chunks, with their row
  // scales), then the rows of its enrichment atoms (padding rows read row 0:
  // the E_c^T tiles are zero in their columns)
  __shared__ int32_t gs[16 * ((EFE_MAXLOC + 15) / 16) + (ENR ? EFE_MAX_CELL_ENR : 0)];
  __shared__ double gsc[16 * ((EFE_MAXLOC + 15) / 16)];
  const int b = blockIdx.x;
  const int nparts = a.nparts_c + a.nparts_e;
  const int xcd = b % 8, slot = b / 8;
  const int ci = (slot / nparts) * 8 + xcd;
  const int part = slot % nparts;
  if (ci >= a.ncells) return;
  const int cell = a.cells[ci];
  const int nloc = a.nloc, ncols = a.ncols;
  const int t = threadIdx.x, wave = t / 64, lane = t % 64, li = lane % 16, lk = lane / 16;
  const bool erole = part >= a.nparts_c;
  int ne = 0, nep = 0;
  int32_t p0 = 0;
  int64_t noff = 0;
  if (ENR) {
    p0 = a.cell_eptr[cell];
    ne = (a.cell_eptr[cell + 1] - p0) * a.nf;
    nep = (ne + 15) / 16 * 16;
    noff = a.cell_noff[cell];
  }
  const int RBE = nep / 16;
  // enrichment-row parts beyond the cell's rows (uniform over the work-group)
  if (erole && (!ENR || (part - a.nparts_c) * 4 * RBW >= RBE)) return;
  const int NCHc = (a.KS + 3) / 4;
  const int KCF = NCHc * 16;                 // CFE rows of the gathered block, padded
  const int32_t *g = a.c2g + (int64_t)cell * nloc;
  for (int l = t; l < KCF; l += 256) {
    const int32_t node = g[min(l, nloc - 1)];
    gs[l] = node;
    gsc[l] = (l >= nloc || a.minv[node] == 0.0) ? 0.0 : (a.scale ? a.scale[node] : 1.0);
  }
  if (ENR && !erole)
    for (int r = t; r < nep; r += 256)
      gs[KCF + r] = r < ne ? a.pair_atom[a.cell_epair[p0 + r / a.nf]] * a.nf + r % a.nf : 0;
  __syncthreads();
  const int nrb = erole ? RBE : a.RB;
  const int rbase = ((erole ? part - a.nparts_c : part) * 4 + wave) * RBW;
  const int CB = (ncols + 15) / 16;
  const int NCH = NCHc + ((ENR && !erole) ? RBE : 0);
  const int kse_n = nep / 4;
  const T *hp = erole ? a.Ee + 4 * (int64_t)a.KS * noff + lane
                      : a.Ht + ((int64_t)cell * a.RB) * a.KS * 64 + lane;
  const T *tp = ENR ? a.Et + 16 * (int64_t)a.RB * noff + lane : hp;

  T a0[4][RBW], a1[4][RBW];
  acc_t acc[RBW][CBM];
#pragma unroll
  for (int r = 0; r < RBW; ++r)
#pragma unroll
    for (int cb = 0; cb < CBM; ++cb) acc[r][cb] = (acc_t){0, 0, 0, 0};

  // Loads are unconditional, at clamped addresses, and nothing consumes a
  // loaded value before it is needed, so the compiler waits only for the
  // current chunk's operands and the next chunk's loads stay in flight.
  // Out-of-range rows and columns are zeroed when they are written to LDS
  // (row scale 0); a clamped A fragment then multiplies zero rows of Xs (k
  // past the end) or feeds accumulators that are never stored (row blocks
  // past the end).  Wide tiles read the rows as pairs of doubles with 32-bit
  // element offsets (even leading dimensions; the host checks the offsets fit).
  constexpr bool PAIRS = NC >= 32;
  constexpr int NP = PAIRS ? NC / 2 : NC, EPT2 = KC * NP / 256;
  static_assert(KC * NP % 256 == 0, "the gather must cover the chunk exactly");
  const int NPV = (ncols + 1) / 2;
  double2 xr[EPT2];
  // chunk ch reads rows ch*16 .. of the gathered block: CFE rows from X,
  // enrichment rows from XE (a uniform choice per chunk)
  auto stage_load = [&](int ch) {
    const bool ce = ENR && ch >= NCHc;
    const double *base = ce ? a.XE : a.X;
    const uint32_t ld = (uint32_t)(ce ? a.lde : a.ldx);
#pragma unroll
    for (int j = 0; j < EPT2; ++j) {
      const int idx = t + 256 * j, r = idx / NP, cp = idx % NP;
      const uint32_t row = (uint32_t)gs[ch * KC + r];
      if constexpr (PAIRS) {
        xr[j] = *reinterpret_cast<const double2 *>(base + row * ld +
                                                   2u * (uint32_t)min(cp, NPV - 1));
      } else {
        xr[j].x = base[(int64_t)row * ld + min(cp, ncols - 1)];
      }
    }
  };
  auto stage_store = [&](int buf, int ch) {
    const bool ce = ENR && ch >= NCHc;
#pragma unroll
    for (int j = 0; j < EPT2; ++j) {
      const int idx = t + 256 * j, r = idx / NP, cp = idx % NP;
      const double s = ce ? 1.0 : gsc[ch * KC + r];
      if constexpr (PAIRS) {
        Xs[buf][r][2 * cp] = 2 * cp < ncols ? (T)(s * xr[j].x) : (T)0;
        Xs[buf][r][2 * cp + 1] = 2 * cp + 1 < ncols ? (T)(s * xr[j].y) : (T)0;
      } else {
        Xs[buf][r][cp] = cp < ncols ? (T)(s * xr[j].x) : (T)0;
      }
    }
  };
  // A fragments of chunk ch: cell Hamiltonian (or E_c) tiles, then E_c^T tiles
  auto a_load = [&](int ch, T (&dst)[4][RBW]) {
    const bool ce = ENR && ch >= NCHc;
    const T *ap = ce ? tp : hp;
    const int64_t rs = ce ? kse_n : a.KS;
    const int k0 = ce ? (ch - NCHc) * 4 : ch * 4;
    const int kmax = ce ? kse_n - 1 : a.KS - 1;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int r = 0; r < RBW; ++r) {
        const int64_t rb = min(rbase + r, nrb - 1);
        dst[s][r] = ld_nt(&ap[(rb * rs + min(k0 + s, kmax)) * 64]);
      }
  };
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
  if (erole) {
    // the cell's enrichment rows: partial sums of E_c (s X^C_c)
#pragma unroll
    for (int r = 0; r < RBW; ++r) {
      const int rb = rbase + r;
      if (rb >= RBE) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int e = rb * 16 + M::row(v, lk);
        if (e >= ne) continue;
        double *yp = a.Yp + ((int64_t)a.nf * p0 + e) * a.ldp;
#pragma unroll
        for (int cb = 0; cb < CBM; ++cb) {
          const int col = cb * 16 + li;
          if (cb < CB && col < ncols) st_nt((double)acc[r][cb][v], &yp[col]);
        }
      }
    }
    return;
  }
  // scatter: per row block, all reads of Y first, then all writes, so the
  // reads overlap instead of each waiting for the one before; the wide tiles
  // stream Y non-temporally (the narrow ones, whose rows are a 128-byte
  // piece, measured slower that way)
  constexpr bool YNT = CBM > 1;
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rb = rbase + r;
    if (rb >= a.RB) continue;
    int64_t node[4];
    bool ok[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rb * 16 + M::row(v, lk);
      node[v] = gs[min(row, nloc - 1)];
      ok[v] = row < nloc;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) ok[v] = ok[v] && a.minv[node[v]] != 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double yv[CBM];
#pragma unroll
      for (int cb = 0; cb < CBM; ++cb) {
        const int64_t o = node[v] * a.ldy + min(cb * 16 + li, ncols - 1);
        yv[cb] = YNT ? ld_nt(&a.Y[o]) : a.Y[o];
      }
#pragma unroll
      for (int cb = 0; cb < CBM; ++cb) {
        const int col = cb * 16 + li;
        if (ok[v] && cb < CB && col < ncols) {
          const double y = yv[cb] + a.alpha * (double)acc[r][cb][v];
          if (YNT)
            st_nt(y, &a.Y[node[v] * a.ldy + col]);
          else
            a.Y[node[v] * a.ldy + col] = y;
        }
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
                                                   const double *__restrict__ scale,
                                                   double *__restrict__ Y, int64_t ldy,
                                                   const double *__restrict__ minv, int ncols,
                                                   double alpha) {
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
    if (r < nloc && col0 + cc < ncols) {
      const int64_t node = g[r];
      const double s = minv[node] == 0.0 ? 0.0 : (scale ? scale[node] : 1.0);
      v = s * Xh[node * ldx + col0 + cc];
    }
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
        if (col < ncols) Y[node * ldy + col] += alpha * (double)acc[cb][v];
      }
    }
  }
}


// Affine epilogue of an apply (device copy of ApplyEpilogue)
struct EpiArgs {
  double alpha, beta, gamma;
  const double *Z1, *Z2, *G, *Cl;
};
// ------------------------------------------------------------------ projectors
// W[I] += D_I sum_s P^C_s s_node X[node_s] over one work item (atom, support-list
// range); the items of a node region run back to back, so the rows of X they
// read are shared through the caches.  Waves take one support node at a time
// (wave-uniform); a lane owns two column pairs (256 columns per work-group
// column block), read as 16-byte pairs with 32-bit offsets (X has an even
// leading dimension, 16-byte aligned, n_nodes x ld < 2^31: the apply ensures
// it), and four entries' rows are in flight at a time.
constexpr int KBP = 2;   // column pairs per lane

__global__ __launch_bounds__(256) void k_kb_project(int ncols, const int32_t *__restrict__ items,
                                                    XcdSplit xs,
                                                    const int32_t *__restrict__ kbnode,
                                                    const double *__restrict__ Pc,
                                                    const double *__restrict__ X, int64_t ldx,
                                                    const double *__restrict__ scale,
                                                    const double *__restrict__ D,
                                                    double *__restrict__ W) {
  __shared__ double2 red[3][64 * KBP];
  const int64_t item = xcd_block(xs);
  if (item < 0) return;
  const int32_t *it = items + 3 * item;
  const int I = it[0];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / 64));
  const int lane = threadIdx.x % 64;
  const int c0 = blockIdx.y * 128 * KBP;
  const int npv = (min(ncols - c0, 128 * KBP) + 1) / 2;   // column pairs of this block
  int pofs[KBP];
#pragma unroll
  for (int q = 0; q < KBP; ++q) pofs[q] = c0 + 2 * min(lane + 64 * q, npv - 1);
  double2 acc[KBP];
#pragma unroll
  for (int q = 0; q < KBP; ++q) acc[q] = make_double2(0.0, 0.0);
  // entries it[1] + wave + 4 i: node numbers and coefficients (times the row
  // scale) come in 64 at a time by vector loads and reach the wave by
  // readlane; clamped pairs keep the row loads unconditional (their sums are
  // not stored)
  const int32_t s0 = it[1], s1 = it[2];
  const uint32_t ld = (uint32_t)ldx;
  for (int32_t sb = s0 + wave; sb < s1; sb += 256) {
    const int cnt = min(64, (s1 - sb + 3) / 4);
    const int32_t sl = min(sb + 4 * lane, s1 - 1);
    const int32_t nodes = kbnode[sl];
    const double pv = Pc[sl] * (scale ? scale[nodes] : 1.0);
    for (int i = 0; i < cnt; i += 4) {
      double2 xv[4][KBP];
      double pj[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int ii = min(i + j, cnt - 1);
        const uint32_t node = (uint32_t)__builtin_amdgcn_readlane(nodes, ii);
        const double pb = lane_bcast(pv, ii);
        pj[j] = i + j < cnt ? pb : 0.0;
#pragma unroll
        for (int q = 0; q < KBP; ++q)
          xv[j][q] = *reinterpret_cast<const double2 *>(X + (node * ld + (uint32_t)pofs[q]));
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < KBP; ++q) {
          acc[q].x += pj[j] * xv[j][q].x;
          acc[q].y += pj[j] * xv[j][q].y;
        }
    }
  }
  if (wave > 0)
#pragma unroll
    for (int q = 0; q < KBP; ++q) red[wave - 1][64 * q + lane] = acc[q];
  __syncthreads();
  if (wave == 0)
#pragma unroll
    for (int q = 0; q < KBP; ++q) {
      const int pp = lane + 64 * q;
      if (pp >= npv) continue;
      const int col = c0 + 2 * pp;
      const double2 r0 = red[0][64 * q + lane], r1 = red[1][64 * q + lane],
                    r2 = red[2][64 * q + lane];
      atomicAdd(&W[(int64_t)I * ncols + col], D[I] * (acc[q].x + r0.x + r1.x + r2.x));
      if (col + 1 < ncols)
        atomicAdd(&W[(int64_t)I * ncols + col + 1], D[I] * (acc[q].y + r0.y + r1.y + r2.y));
    }
}

// sum of x over the work-group (256 threads), in a fixed order
__device__ inline double block_sum256(double x, double *red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = x;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

// the same for one column: threads over the item's entries
__global__ __launch_bounds__(256) void k_kb_project1(const int32_t *__restrict__ items,
                                                     const int32_t *__restrict__ kbnode,
                                                     const double *__restrict__ Pc,
                                                     const double *__restrict__ X, int64_t ldx,
                                                     const double *__restrict__ scale,
                                                     const double *__restrict__ D,
                                                     double *__restrict__ W) {
  __shared__ double red[4];
  const int32_t *it = items + 3 * (int64_t)blockIdx.x;
  const int I = it[0];
  double acc = 0.0;
  for (int32_t s = it[1] + threadIdx.x; s < it[2]; s += 256) {
    const int64_t node = kbnode[s];
    acc += Pc[s] * (scale ? scale[node] : 1.0) * X[node * ldx];
  }
  const double t = block_sum256(acc, red);
  if (threadIdx.x == 0) atomicAdd(&W[I], D[I] * t);
}

// W[I] = D_I sum_f P~^phi_If XE_f (the enrichment part of the projector
// coefficients): one work-group per (projector, 64 columns); the four waves
// take every fourth f and their sums meet in LDS in a fixed order
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

// Affine epilogue terms of one element: beta Z1 + gamma Z2 + alpha G Cl
__device__ inline double epi_terms(const EpiArgs &e, int64_t o, int col) {
  double v = 0.0;
  if (e.Z1) v += e.beta * e.Z1[o];
  if (e.Z2) v += e.gamma * e.Z2[o];
  if (e.G) v += e.alpha * e.G[o] * e.Cl[col];
  return v;
}

// Y^C[node] = alpha sum_e P^C_e W[atom_e] + epilogue terms on every interior
// node (boundary rows 0): the projector expansion, and the start value of the
// colour passes' read-modify-write.  Flat over (node, column pair): a thread
// takes two adjacent columns of one node, so every array is read and written
// in coalesced 16-byte pieces, and the threads of a wave share one or two
// nodes, whose projector entries they loop over together.  Even ld (the host
// checks it) keeps the pairs aligned.
constexpr int EXP_P = 2;   // column pairs per thread of k_expand_init

__global__ __launch_bounds__(256) void k_expand_init(int64_t n_nodes, int ncols,
                                                     const int32_t *__restrict__ kbnm_ptr,
                                                     const int32_t *__restrict__ kbnm_atom,
                                                     const double *__restrict__ Pc_nm,
                                                     const double *__restrict__ W,
                                                     const double *__restrict__ minv,
                                                     EpiArgs e, double *Y, int64_t ldy,
                                                     bool vec) {
  const int npr = (ncols + 1) / 2;             // column pairs of a node
  const int nth = (npr + EXP_P - 1) / EXP_P;   // threads of a node
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n_nodes * nth) return;
  int64_t node;
  int j;
  if (n_nodes * nth < (1ll << 31)) {          // 32-bit division where it fits
    node = (uint32_t)idx / (uint32_t)nth;
    j = (int)((uint32_t)idx - (uint32_t)node * (uint32_t)nth);
  } else {
    node = idx / nth;
    j = (int)(idx % nth);
  }
  // this thread's pairs: j, j + nth, ... (adjacent threads, adjacent pairs)
  int c0[EXP_P];
  bool has[EXP_P], two[EXP_P];
#pragma unroll
  for (int q = 0; q < EXP_P; ++q) {
    c0[q] = 2 * (j + q * nth);
    has[q] = c0[q] < ncols;
    two[q] = c0[q] + 1 < ncols;
  }
  const int64_t rowo = node * ldy;
  // pairs by 16-byte accesses when the layout allows it (vec: even ld,
  // aligned arrays), else element by element
  auto ld2 = [&](const double *p, int q) -> double2 {
    const int64_t o = rowo + c0[q];
    if (vec && two[q]) return ld_nt2(p + o);
    double2 r;
    r.x = has[q] ? p[o] : 0.0;
    r.y = two[q] ? p[o + 1] : 0.0;
    return r;
  };
  // the streamed rows first, so that they are in flight while the
  // projector entries (two dependent loads each) come in
  double2 z1[EXP_P], z2[EXP_P], g[EXP_P], cl[EXP_P];
#pragma unroll
  for (int q = 0; q < EXP_P; ++q) {
    z1[q] = z2[q] = g[q] = cl[q] = make_double2(0.0, 0.0);
    if (e.Z1) z1[q] = ld2(e.Z1, q);
    if (e.Z2) z2[q] = ld2(e.Z2, q);
    if (e.G) {
      g[q] = ld2(e.G, q);
      cl[q].x = has[q] ? e.Cl[c0[q]] : 0.0;
      cl[q].y = two[q] ? e.Cl[c0[q] + 1] : 0.0;
    }
  }
  const bool inner = minv[node] != 0.0;
  double2 a[EXP_P];
#pragma unroll
  for (int q = 0; q < EXP_P; ++q) a[q] = make_double2(0.0, 0.0);
  if (kbnm_ptr) {
    const int32_t e0 = kbnm_ptr[node], e1 = kbnm_ptr[node + 1];
    for (int32_t en = e0; en < e1; ++en) {
      const double p = Pc_nm[en];
      const double *w = W + (int64_t)kbnm_atom[en] * ncols;
#pragma unroll
      for (int q = 0; q < EXP_P; ++q) {
        if (has[q]) a[q].x += p * w[c0[q]];
        if (two[q]) a[q].y += p * w[c0[q] + 1];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < EXP_P; ++q) {
    if (!has[q]) continue;
    double2 v;
    v.x = e.alpha * (a[q].x + g[q].x * cl[q].x);
    v.y = e.alpha * (a[q].y + g[q].y * cl[q].y);
    if (e.Z1) {
      v.x += e.beta * z1[q].x;
      v.y += e.beta * z1[q].y;
    }
    if (e.Z2) {
      v.x += e.gamma * z2[q].x;
      v.y += e.gamma * z2[q].y;
    }
    if (!inner) v.x = v.y = 0.0;
    const int64_t o = rowo + c0[q];
    if (vec && two[q]) {
      st_nt2(v, Y + o);
    } else {
      Y[o] = v.x;
      if (two[q]) Y[o + 1] = v.y;
    }
  }
}

// Y^E[I] = alpha (sum over the cells of atom I of their partial rows + TE[I])
// + epilogue terms, the partial rows added in cell order (fixed).  One
// work-group per (atom, 64 columns); the four waves take every fourth function.
__global__ __launch_bounds__(576) void k_enr_reduce(int nf, int ncols,
                                                    const int32_t *__restrict__ cpair_ptr,
                                                    const int32_t *__restrict__ cpair_cpos,
                                                    const double *__restrict__ Yp, int64_t ldp,
                                                    const double *__restrict__ TE,
                                                    EpiArgs e, double *YE, int64_t ldy) {
  const int I = blockIdx.x;
  const int k = threadIdx.x / 64, lane = threadIdx.x % 64;   // one wave per function
  const int col = blockIdx.y * 64 + lane;
  const int colc = min(col, ncols - 1);      // every lane runs: the readlanes below
  const int32_t q0 = cpair_ptr[I], q1 = cpair_ptr[I + 1];
  // four partial sums over the atom's pairs (pair q into sum q mod 4), added
  // in a fixed order; pair positions come 64 at a time by one vector load
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int32_t qb = q0; qb < q1; qb += 64) {
    const int cnt = min(64, q1 - qb);
    const int32_t cpv = cpair_cpos[min(qb + lane, q1 - 1)];
    for (int i = 0; i < cnt; i += 4) {
      double v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t cp = __builtin_amdgcn_readlane(cpv, min(i + j, cnt - 1));
        v[j] = ld_nt(&Yp[((int64_t)nf * cp + k) * ldp + colc]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (i + j < cnt) a[j] += v[j];
    }
  }
  if (col >= ncols) return;
  const int64_t f = (int64_t)I * nf + k;
  const double acc = (a[0] + a[1]) + (a[2] + a[3]) + TE[f * ncols + col];
  const int64_t o = f * ldy + col;
  YE[o] = e.alpha * acc + epi_terms(e, o, col);
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
static void launch_cell3(efe_ctx *c, const T *Ht, const T *Et, const T *Ee, const double *X,
                         int64_t ldx, const double *scale, const double *XE, int64_t lde,
                         double *Y, int64_t ldy, double alpha, double *Yp, int64_t ldp,
                         int ncols) {
  const bool enr = c->n_enr > 0 && c->ncpairs > 0;
  CellOps<T> a;
  a.nparts_c = (int)cdiv(c->RB, 4 * RBW);
  a.nparts_e = enr ? (int)cdiv(c->max_rbe, 4 * RBW) : 0;
  a.c2g = c->d_c2g;
  a.nloc = c->nloc;
  a.RB = c->RB;
  a.KS = c->KS;
  a.nf = c->nf;
  a.Ht = Ht;
  a.Et = Et;
  a.Ee = Ee;
  a.ldx = ldx;
  a.scale = scale;
  a.minv = c->d_minv;
  a.lde = lde;
  a.ldy = ldy;
  a.alpha = alpha;
  a.ldp = ldp;
  a.cell_eptr = c->d_cell_eptr;
  a.cell_epair = c->d_cell_epair;
  a.pair_atom = c->d_cpair_atom;
  a.cell_noff = c->d_cell_noff;
  const int nparts = a.nparts_c + a.nparts_e;
  for (int col0 = 0; col0 < ncols; col0 += 16 * CBM) {
    a.ncols = std::min(16 * CBM, ncols - col0);
    a.X = X + col0;
    a.XE = XE + col0;
    a.Y = Y + col0;
    a.Yp = Yp + col0;
    for (int col = 0; col < 8; ++col) {
      const int nc = c->colour_offsets[col + 1] - c->colour_offsets[col];
      if (nc == 0) continue;
      a.ncells = nc;
      a.cells = c->d_colour_order + c->colour_offsets[col];
      const int64_t nblk = cdiv(nc, 8) * 8 * nparts;
      const int t = efe_timer_begin(c, CBM == 1 ? EFE_T_CELL_NARROW : EFE_T_CELL);
      if (enr)
        k_cell3<T, RBW, CBM, true><<<nblk, 256, 0, c->stream>>>(a);
      else
        k_cell3<T, RBW, CBM, false><<<nblk, 256, 0, c->stream>>>(a);
      efe_timer_end(c, CBM == 1 ? EFE_T_CELL_NARROW : EFE_T_CELL, t);
    }
  }
}

__global__ void k_fill_zero(int64_t n, double *__restrict__ x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// X -> Xc with an even leading dimension (the cell GEMM's paired gathers)
__global__ void k_copy_cols(int64_t rows, int ncols, const double *__restrict__ X, int64_t ldx,
                            double *__restrict__ Y, int64_t ldy) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= rows * ncols) return;
  const int64_t r = idx / ncols;
  const int j = (int)(idx % ncols);
  Y[r * ldy + j] = X[r * ldx + j];
}

efe_status efe_apply_H_internal(efe_ctx *c, const double *XC, int64_t ldx, const double *scale,
                                const double *XE, int64_t lde, double *Y, int64_t ldy, int ncols,
                                int prec, const ApplyEpilogue *epi) {
  if (!c->have_potential) EFE_FAIL(c, EFE_ESTATE, "no potential set");
  if (ncols <= 0) return EFE_OK;
  if (ncols > EFE_COL_CHUNK) EFE_FAIL(c, EFE_EINVAL, "apply chunk wider than 160 columns");
  if ((prec == EFE_FP32 && !c->have32) || (prec == EFE_BF16 && !c->have16))
    EFE_FAIL(c, EFE_ESTATE, "reduced-precision cell matrices were not built by efe_set_potential");
  if (prec == EFE_BF16 && c->n_enr > 0)
    EFE_FAIL(c, EFE_EINVAL, "the BF16 cell GEMM takes plain CFE systems only");
  efe_status s;
  const int nf = c->nf;
  const int64_t nn = c->n_nodes, ne = c->n_enr;
  ApplyEpilogue E0;
  const ApplyEpilogue &ep = epi ? *epi : E0;
  // the cell GEMM reads the CFE rows in pairs with 32-bit offsets: other
  // layouts are copied to an even leading dimension first
  const bool pairs_ok = (ldx % 2 == 0) && ((uintptr_t)XC % 16 == 0) && nn * ldx < (1ll << 31);
  if (!pairs_ok) {
    const int64_t ldc = (ncols + 1) & ~1;
    double *Xc;
    if (nn * ldc >= (1ll << 31))
      EFE_FAIL(c, EFE_EINVAL, "n_nodes x columns exceeds the 32-bit offsets of the cell GEMM");
    if ((s = efe_ws(c, 0, (size_t)nn * ldc * 8, (void **)&Xc))) return s;
    k_copy_cols<<<cdiv(nn * ncols, 256), 256, 0, c->stream>>>(nn, ncols, XC, ldx, Xc, ldc);
    XC = Xc;
    ldx = ldc;
  }
  if (ne && ((lde % 2) || ((uintptr_t)XE % 16) || ne * lde >= (1ll << 31))) {
    const int64_t ldc = (ncols + 1) & ~1;
    double *Xc;
    if ((s = efe_ws(c, 12, (size_t)ne * ldc * 8, (void **)&Xc))) return s;
    k_copy_cols<<<cdiv(ne * ncols, 256), 256, 0, c->stream>>>(ne, ncols, XE, lde, Xc, ldc);
    XE = Xc;
    lde = ldc;
  }
  double *W = nullptr, *Yp = nullptr, *TE = nullptr;
  if (c->nproj && (s = efe_ws(c, 1, (size_t)c->nproj * ncols * 8, (void **)&W))) return s;
  if (ne) {
    if ((s = efe_ws(c, 9, (size_t)nf * std::max<int64_t>(c->ncpairs, 1) * ncols * 8, (void **)&Yp)))
      return s;
    if ((s = efe_ws(c, 11, (size_t)ne * ncols * 8, (void **)&TE))) return s;
  }
  EpiArgs ec{ep.alpha, ep.beta, ep.gamma, ep.Z1, ep.Z2, ep.G, ep.Cl};
  const int t_cls = ncols <= 16 ? EFE_T_APPLY_NARROW : EFE_T_APPLY;
  const int t_apply = efe_timer_begin(c, t_cls);
  // 1. projector coefficients W = D (P^C s X^C + P~^phi X^E), then Y^C =
  //    alpha P^C^T W + epilogue terms on every node
  {
    const int t = efe_timer_begin(c, EFE_T_PRE);
    if (c->nproj) {
      // (without enrichment this writes W = 0)
      k_kb_w_pphi<<<dim3(c->nproj, cdiv(ncols, 64)), 256, 0, c->stream>>>(
          ncols, ne, c->d_Ptil, XE, lde, c->d_D, W);
      if (c->n_kb_items) {
        XcdSplit xs;
        for (int i = 0; i <= 8; ++i) xs.off[i] = c->kb_items_off[i];
        if (ncols == 1)
          k_kb_project1<<<c->n_kb_items, 256, 0, c->stream>>>(c->d_kb_items, c->d_kbnode,
                                                              c->d_Pc_am, XC, ldx, scale, c->d_D, W);
        else
          k_kb_project<<<dim3(8 * xs.max_len(), cdiv(ncols, 128 * KBP)), 256, 0, c->stream>>>(
              ncols, c->d_kb_items, xs, c->d_kbnode, c->d_Pc_am, XC, ldx, scale, c->d_D, W);
      }
    }
    auto al = [](const double *p) { return p == nullptr || (uintptr_t)p % 16 == 0; };
    const bool vec = ldy % 2 == 0 && al(Y) && al(ep.Z1) && al(ep.Z2) && al(ep.G);
    k_expand_init<<<cdiv(nn * (((ncols + 1) / 2 + EXP_P - 1) / EXP_P), 256), 256, 0, c->stream>>>(
        nn, ncols, c->nproj ? c->d_kbnm_ptr : nullptr, c->d_kbnm_atom, c->d_Pc_nm, W, c->d_minv,
        ec, Y, ldy, vec);
    efe_timer_end(c, EFE_T_PRE, t);
  }
  // 2. cell GEMM, colour by colour: 160-column register tiles; a single
  //    16-column tile (six row blocks per wave) for narrow blocks such as the
  //    Lanczos vector
  if (prec == EFE_FP64 && ncols <= 16)
    launch_cell3<double, 6, 1>(c, c->d_Htile64, c->d_Et64, c->d_Ee64, XC, ldx, scale, XE, lde, Y,
                               ldy, ep.alpha, Yp, ncols, ncols);
  else if (prec == EFE_FP64)
    launch_cell3<double, 1, 10>(c, c->d_Htile64, c->d_Et64, c->d_Ee64, XC, ldx, scale, XE, lde, Y,
                                ldy, ep.alpha, Yp, ncols, ncols);
  else if (prec == EFE_FP32 && ncols <= 16)
    launch_cell3<float, 6, 1>(c, c->d_Htile32, c->d_Et32, c->d_Ee32, XC, ldx, scale, XE, lde, Y,
                              ldy, ep.alpha, Yp, ncols, ncols);
  else if (prec == EFE_FP32)
    launch_cell3<float, 2, 10>(c, c->d_Htile32, c->d_Et32, c->d_Ee32, XC, ldx, scale, XE, lde, Y,
                               ldy, ep.alpha, Yp, ncols, ncols);
  else {
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
          c->KS32, (const v8bf *)c->d_Htile16, XC, ldx, scale, Y, ldy, c->d_minv, ncols,
          ep.alpha);
      efe_timer_end(c, EFE_T_CELL, t);
    }
  }
  // 3. enrichment rows: Y^E = alpha (sum of the cells' partial rows
  //    + H^E_ee X^E + P~^phi^T W) + epilogue terms
  const int t_post = efe_timer_begin(c, EFE_T_POST);
  if (ne) {
    k_fill_zero<<<cdiv(ne * ncols, 256), 256, 0, c->stream>>>(ne * ncols, TE);
    if ((s = efe_dgemm(c, false, false, ne, ncols, ne, 1.0, c->d_Hee, ne, XE, lde, 1.0, TE, ncols,
                               nullptr, true)))
      return s;
    if (c->nproj &&
        (s = efe_dgemm(c, true, false, ne, ncols, c->nproj, 1.0, c->d_Ptil, ne, W, ncols, 1.0, TE,
                            ncols, nullptr, true)))
      return s;
    EpiArgs ee = ec;
    if (ee.Z1) ee.Z1 += nn * ldy;
    if (ee.Z2) ee.Z2 += nn * ldy;
    if (ee.G) ee.G += nn * ldy;
    k_enr_reduce<<<dim3(c->natoms, cdiv(ncols, 64)), 64 * nf, 0, c->stream>>>(
        nf, ncols, c->d_cpair_ptr, c->d_cpair_cpos, Yp, ncols, TE, ee, Y + nn * ldy, ldy);
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
    return efe_dgemm(c, false, false, c->n_enr, ncols, c->n_enr, 1.0, c->d_Mee, c->n_enr,
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
