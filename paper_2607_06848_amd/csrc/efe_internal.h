// Internal declarations of the EFE library: context layout, error helpers
// and the host-side launchers shared between translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/efe.h"

#define EFE_MAXP 6
#define EFE_MAXQ 7
#define EFE_MAXLOC ((EFE_MAXP + 1) * (EFE_MAXP + 1) * (EFE_MAXP + 1))
// enrichment functions that may couple to one cell (padded to 16): 85 atoms
// of 9 (the cell GEMM keeps their row numbers in LDS)
#define EFE_MAX_CELL_ENR 768

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

struct efe_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;

  // ---------------------------------------------------------------- mesh
  double lo[3], hi[3], h[3];
  int ncell[3], p, P, nloc, nq, nqp;
  int64_t n1[3];
  int64_t n_nodes = 0, n_cells = 0, n_qpts = 0, rows = 0, n_dof = 0, n_enr = 0;
  std::vector<int32_t> c2g, colour_order, boundary_i;
  int32_t colour_offsets[9];
  std::vector<uint8_t> boundary;

  // ---------------------------------------------------------------- system
  int natoms = 0, nf = 0, lmax = -1, nproj = 0;
  std::vector<double> xyz, Z;
  double loc_rc, loc_amp, loc_rg, kb_width, kb_D, kb_rcut, enr_alpha, enr_rcut, enr_t,
      rho_alpha;
  // tabulated radial enrichment (ntab = 0: Gaussian)
  int ntab = 0;
  double tab_dr = 0.0, tab_rc[3] = {0.0, 0.0, 0.0};
  double *d_enr_tab = nullptr;
  std::vector<double> tab_host;
  // tabulated atomic density and potential (natab = 0: Gaussian forms)
  int natab = 0;
  double atab_dr = 0.0;
  double *d_atom_tab = nullptr;
  std::vector<double> atab_host;

  // support tables (host copies kept for efe_get_support)
  std::vector<int32_t> enr_ptr, enr_cells, kb_ptr, kb_cells;

  // ---------------------------------------------------------------- device
  int32_t *d_c2g = nullptr, *d_colour_order = nullptr;
  double *d_m = nullptr, *d_minv = nullptr;            // lumped mass, 1/m (0 on boundary)
  double *d_m_int = nullptr;                           // lumped mass, 0 on boundary
  double *d_N3 = nullptr, *d_G3 = nullptr;             // [nqp][nloc], [3][nqp][nloc]
  double *d_W3 = nullptr, *d_K = nullptr;              // [nqp] (times Jacobian), [nloc][nloc]
  double *d_xq1 = nullptr;                             // 1-D Gauss abscissae (nq)
  double *d_xyz = nullptr, *d_Zs = nullptr;

  // enrichment: (atom, cell) pairs sorted by atom then cell
  int64_t npairs = 0;
  int32_t *d_pair_atom = nullptr, *d_pair_cell = nullptr, *d_pair_lmap = nullptr;
  int64_t n_snodes = 0;                                // sum over atoms of support nodes
  int32_t *d_snode_ptr = nullptr, *d_snode = nullptr;
  std::vector<int32_t> snode_ptr_h;
  double *d_nu = nullptr;                              // normalization per function
  double *d_b_am = nullptr, *d_C_am = nullptr, *d_Bkin_am = nullptr, *d_B_am = nullptr;
  // node-major copy: per node the list of (atom, support-node index)
  int64_t nnz_nm = 0;
  int32_t *d_nm_ptr = nullptr, *d_nm_atom = nullptr, *d_nm_src = nullptr;
  // groups of 8 consecutive nodes: per group the union of the atoms whose
  // support holds one of its nodes (slots), and C, B per slot as [slot][k][8]
  int64_t n_gslots = 0;
  int32_t *d_g_ptr = nullptr, *d_g_atom = nullptr, *d_nm_gslot = nullptr;
  double *d_Cg = nullptr, *d_Bg = nullptr;
  // coupling pairs (atom, cell): every cell holding one of the atom's support
  // nodes (atom-major, by cell), with the support pair of the cell (-1 for
  // the layer outside the support) and the local-to-support map; their
  // cell-major view: per cell its pairs (ascending atom), per pair its
  // cell-major position, per cell the prefix of its padded enrichment row
  // count (functions x atoms rounded up to 16), which places its tiles
  int64_t ncpairs = 0;
  int32_t *d_cpair_atom = nullptr, *d_cpair_spair = nullptr, *d_cpair_lmap = nullptr;
  int32_t *d_cpair_ptr = nullptr, *d_cpair_cpos = nullptr;
  int32_t *d_cell_eptr = nullptr, *d_cell_epair = nullptr;
  int64_t *d_cell_noff = nullptr;
  int max_rbe = 0;                                     // max padded rows / 16 over cells
  int64_t n_epad = 0;                                  // sum of padded rows
  // per-pair cell blocks [pair][l][k]: kinetic part of B (setup), B (per potential)
  double *d_Bkin_pair = nullptr, *d_B_pair = nullptr;
  // coupling of the orthogonalized basis per cell, E_c = B_c - C_c H_c, in the
  // MFMA operand layouts: Et = E_c^T tiles (rows: cell nodes, k: the cell's
  // enrichment functions), Ee = E_c tiles (rows: enrichment functions, k: nodes)
  double *d_Et64 = nullptr, *d_Ee64 = nullptr;
  float *d_Et32 = nullptr, *d_Ee32 = nullptr;
  double *d_Hee = nullptr;                             // H^E_ee without projectors
  double *d_Ptil = nullptr;                            // P^phi - P^C C^T, [nproj][n_enr]
  // (cell, I, J) triples of atoms sharing a support cell
  int64_t ntrip = 0;
  int32_t *d_trip = nullptr;
  double *d_Mpp = nullptr, *d_Mee = nullptr, *d_Hpp_kin = nullptr, *d_Hpp = nullptr;
  double *d_Mee_inv = nullptr;                         // [natoms][nf][nf]
  double amplification = 1.0;                          // efe_enrichment_amplification
  // (atom, first, end) work items over the support lists, ordered by node region
  int64_t n_enr_items = 0, n_kb_items = 0;
  int64_t enr_items_off[9] = {0}, kb_items_off[9] = {0};   // per-XCD ranges
  int32_t *d_enr_items = nullptr, *d_kb_items = nullptr;

  // Kleinman-Bylander projectors (one per atom)
  int64_t nkbpairs = 0;
  int32_t *d_kbpair_atom = nullptr, *d_kbpair_cell = nullptr, *d_kbpair_lmap = nullptr;
  int64_t n_kbnodes = 0;
  int32_t *d_kbnode_ptr = nullptr, *d_kbnode = nullptr;
  double *d_Pc_am = nullptr;
  int64_t nnz_kbnm = 0;
  int32_t *d_kbnm_ptr = nullptr, *d_kbnm_atom = nullptr, *d_kbnm_src = nullptr;
  double *d_Pc_nm = nullptr;
  int64_t nkbtrip = 0;
  int32_t *d_kbtrip = nullptr;                         // (cell, I_kb, J_enr)
  double *d_Pphi = nullptr, *d_D = nullptr;            // [nproj][n_enr], [nproj]

  // potential-dependent operators
  bool have_potential = false;
  double *d_vq = nullptr;
  double *d_Htile64 = nullptr;                         // MFMA-tiled cell Hamiltonians
  float *d_Htile32 = nullptr;
  uint16_t *d_Htile16 = nullptr;
  int RB = 0, KS = 0, KP = 0;                          // tile geometry of the cell GEMM
  int KS32 = 0;                                        // 32-wide k steps of the BF16 tiles
  bool have32 = false, have16 = false;                 // reduced-precision tiles built

  // workspaces (grown on demand)
  std::vector<DevBuf> ws;
  // while an entry point that allocates nothing runs, workspace slots are
  // carved out of the caller-fixed region [arena, arena + arena_cap) instead
  // (slot -> offset, bytes; reset for every call)
  char *arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  static constexpr int kArenaSlots = 64;
  size_t arena_off[kArenaSlots] = {0}, arena_len[kArenaSlots] = {0};

  // SCF state (scf.hip)
  void *scf = nullptr;
  // rocBLAS handle of the dense eigensolver (created on first use)
  int rr_sweeps = 0;          // block Jacobi sweeps of the last Rayleigh-Ritz

  // event timing (efe_timing)
  bool timing = false;
  std::vector<hipEvent_t> tev[8];   // start/stop pairs per kernel class
  int64_t tused[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

// ------------------------------------------------------------------ helpers
#define EFE_FAIL(ctx, code, msg)       \
  do {                                 \
    (ctx)->err = (msg);                \
    return (code);                     \
  } while (0)

#define HIPCHK(ctx, call)                                                          \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      (ctx)->err = std::string(#call) + " failed: " + hipGetErrorString(e_);        \
      return EFE_EHIP;                                                             \
    }                                                                              \
  } while (0)

efe_status efe_alloc(efe_ctx *ctx, void **p, size_t bytes);
// per-device address of the static scratch region of efe_cheb_filter_noalloc
// (noalloc.hip), taken once per device at context setup
efe_status efe_scratch_attach(efe_ctx *ctx);
// rocBLAS handle bound to the context's stream (rr.hip)
// message returned by efe_last_error(NULL) (calls that take no context)
void efe_set_global_error(const std::string &msg);
// workspace slot `slot` of at least `bytes` bytes (kept across calls)
efe_status efe_ws(efe_ctx *ctx, int slot, size_t bytes, void **p);

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Work-groups are dealt round-robin over the eight XCDs (block b runs on XCD
// b % 8).  XcdSplit maps a block to (XCD, slot) and a per-XCD range of work
// items, so that a chosen set of items runs on one XCD and shares its L2.
struct XcdSplit {
  int64_t off[9];
  __host__ __device__ int64_t max_len() const {
    int64_t m = 0;
    for (int x = 0; x < 8; ++x) m = off[x + 1] - off[x] > m ? off[x + 1] - off[x] : m;
    return m;
  }
};

// Column chunk of the wide-block passes (filter, Rayleigh-Ritz H V, density):
// the cell GEMM's column tile, and the width the per-pass workspaces are
// sized for.
constexpr int32_t EFE_COL_CHUNK = 160;

// ------------------------------------------------------------------ launchers
// setup / operators (setup.hip)
efe_status efe_build_reference(efe_ctx *ctx);
efe_status efe_build_enrichment(efe_ctx *ctx);
efe_status efe_build_operators(efe_ctx *ctx, const double *vq, int precisions);
efe_status efe_launch_local_potential(efe_ctx *ctx, double *vq);

// dense FP64 linear algebra on the matrix cores (dense.hip)
// C[M x N] = alpha op(A) op(B) + beta C, row-major; op(A) = A (M x K, lda)
// or A^T (A stored K x M); op(B) = B (K x N) or B^T (B stored N x K); wK
// (may be NULL) weights the sum over k.  split: the sum over K is spread over
// work-groups whose partial products are added to C atomically, C += alpha
// op(A) op(B) (beta ignored; for tall-skinny Grams and short outputs).
efe_status efe_dgemm(efe_ctx *ctx, bool transA, bool transB, int64_t M, int64_t N, int64_t K,
                     double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                     double beta, double *C, int64_t ldc, const double *wK = nullptr,
                     bool split = false);
// C += A^T diag(wK) B (N x N from K rows; A, B stored K x N) on the tiles on
// and above the diagonal only; efe_mirror_upper then copies the upper
// triangle into the lower
efe_status efe_gram_sym(efe_ctx *ctx, int64_t N, int64_t K, const double *A, int64_t lda,
                        const double *B, int64_t ldb, double *C, int64_t ldc,
                        const double *wK = nullptr);
efe_status efe_mirror_upper(efe_ctx *ctx, int64_t n, double *C, int64_t ldc);
// A = L L^T in place (lower triangle of the symmetric positive definite n x n
// A; the upper triangle outside the diagonal blocks is left undefined);
// *dflag (device) is set to 1 when a pivot is not positive
efe_status efe_potrf(efe_ctx *ctx, int64_t n, double *A, int64_t lda, int *dflag);
// X = L^-1 for the lower triangular L (n x n; X full, zero above the diagonal)
efe_status efe_trtri_lower(efe_ctx *ctx, int64_t n, const double *L, int64_t ldl, double *X,
                           int64_t ldx);
// H = Q diag(w) Q^T for the symmetric n x n H (both triangles read and
// averaged): w ascending (device, n), Q row-major n x n with the eigenvectors
// as columns.  work: efe_syev_work(n) doubles; iwork: efe_syev_iwork(n) ints.
efe_status efe_syev_jacobi(efe_ctx *ctx, int64_t n, const double *H, int64_t ldh, double *w,
                           double *Q, double *work, int *iwork, int *sweeps);
size_t efe_syev_work(int64_t n);
size_t efe_syev_iwork(int64_t n);

// operator applications (apply.hip)
// Affine epilogue of an H apply (the Chebyshev recurrence fused into the
// assembly): Y = alpha H X + beta Z1 + gamma Z2 + alpha G diag(Cl), with Z1,
// Z2, G in the layout of Y (Y may be Z2).  alpha = 1 and null terms: Y = H X.
struct ApplyEpilogue {
  double alpha = 1.0, beta = 0.0, gamma = 0.0;
  const double *Z1 = nullptr, *Z2 = nullptr, *G = nullptr, *Cl = nullptr;
};
// Y = H^E X with X given as (XC scaled row-wise by `scale` if non-NULL, XE);
// prec selects the cell GEMM precision; epi (may be NULL) the epilogue.
efe_status efe_apply_H_internal(efe_ctx *ctx, const double *XC, int64_t ldx, const double *scale,
                                const double *XE, int64_t lde, double *Y, int64_t ldy, int ncols,
                                int prec, const ApplyEpilogue *epi = nullptr);
efe_status efe_apply_M_internal(efe_ctx *ctx, const double *X, int64_t ldx, double *Y,
                                int64_t ldy, int ncols);
efe_status efe_apply_Minv_internal(efe_ctx *ctx, const double *X, int64_t ldx, double *Y,
                                   int64_t ldy, int ncols);
// Xh = X^C - C^T X^E on interior CFE rows (0 on the boundary)
efe_status efe_transform_cfe(efe_ctx *ctx, const double *X, int64_t ldx, double *Xh, int64_t ldh,
                             int ncols);
void efe_scf_free(efe_ctx *ctx);
// argument checks and the column-chunk loop of efe_cheb_filter (filter.hip)
efe_status efe_filter_check(efe_ctx *ctx, double *V, const double *lambda, int32_t ncols,
                            int64_t ld, const efe_cheb_params *prm);
efe_status efe_filter_run(efe_ctx *ctx, double *V, const double *lambda, int32_t ncols,
                          int64_t ld, const efe_cheb_params *prm);
efe_status efe_enr_block_inv(efe_ctx *ctx, const double *XE, int64_t ldx, double *YE,
                             int64_t ldy, int ncols);

// ------------------------------------------------------------------ timing
// Optional HIP-event timing of the hot-path kernels (efe_timing).
#define EFE_T_CELL 0     // one colour pass of the cell GEMM
#define EFE_T_PRE 1      // projector pass and Y^C initialization of an H apply
#define EFE_T_POST 2     // enrichment rows of an H apply (reduction and dense blocks)
#define EFE_T_RECUR 3    // residual recurrence update
#define EFE_T_APPLY 4    // a whole H apply
#define EFE_T_RR 5       // a whole Rayleigh-Ritz
#define EFE_T_CELL_NARROW 6    // colour pass of a block of <= 16 vectors
#define EFE_T_APPLY_NARROW 7   // H apply of a block of <= 16 vectors
#define EFE_T_N 8
int efe_timer_begin(efe_ctx *ctx, int which);
void efe_timer_end(efe_ctx *ctx, int which, int slot);
