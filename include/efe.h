/*
 * efe.h -- C ABI of the MI355X enriched-finite-element (EFE) eigensolver.
 *
 * The library solves the generalized Kohn-Sham eigenproblem H^E x = eps M^E x
 * of the orthogonalized EFE basis (Sec. II.B, Eqs. lineigensolveghep,
 * Discrete_Eig_Gen_H, Discrete_Eig_Gen_M) by residual Chebyshev-filtered
 * subspace iteration (Sec. III.B, Eqs. ChebyRecur, residual, residualapprox)
 * followed by Rayleigh-Ritz (Eq. projectedKSEig), and runs the SCF pieces
 * around it (Sec. II.A, III.C).  All compute runs in HIP kernels on the GPU
 * selected when the context is created.
 *
 * Conventions shared by every entry point
 *   Blocks of vectors are device arrays, row-major, one row per DoF and the
 *   vectors of a row contiguous ("node-major"): element (r, j) at ptr[r*ld+j],
 *   ld >= ncols.  Row order: the (ncell*p+1)^3 CFE nodes of the full grid
 *   first (node (i,j,k) -> i + n1x*(j + n1y*k)), boundary nodes included and
 *   held at zero (homogeneous Dirichlet), then the enrichment rows, atom after
 *   atom, n_f = (lmax+1)^2 functions per atom (Sec. II.B: M = n_h + sum n_I).
 *   The caller owns every block and device array it passes; the library owns
 *   its context and workspaces and frees them in efe_destroy.
 *   All work is ordered on the stream given to efe_setup_mesh; calls that
 *   return values in host memory synchronize that stream.
 *   Errors: every call returns an efe_status; arguments are checked before any
 *   launch; the message of the last failure is kept for efe_last_error.
 *   One context per host thread.
 */
#ifndef EFE_H
#define EFE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t efe_status;
#define EFE_OK        0
#define EFE_EINVAL   -1   /* bad argument (null pointer, size, range)       */
#define EFE_ENOMEM   -2   /* device allocation failed                        */
#define EFE_EHIP     -3   /* a HIP runtime call failed                       */
#define EFE_ENOTCONV -4   /* an iteration did not converge                    */
#define EFE_ENUMERIC -5   /* numerical breakdown (Cholesky, non-finite data) */
#define EFE_ESTATE   -6   /* call out of order (e.g. no potential set)       */

/* Precision of the filter's cell GEMMs and projector updates (Sec. III.B runs
 * in FP64; FP32 and BF16 keep FP64 eigen-residual, output and Rayleigh-Ritz). */
#define EFE_FP64 0
#define EFE_FP32 1
#define EFE_BF16 2

#define EFE_FILTER_RESIDUAL 0   /* Eqs. residual, residualapprox             */
#define EFE_FILTER_STANDARD 1   /* Eq. ChebyRecur on (M~^E)^-1 H^E           */

typedef struct efe_ctx efe_ctx;

/* Uniform hexahedral mesh of spectral elements of order p (GLL nodes) on the
 * box [lo, hi]; nq Gauss points per axis for integrals with a potential, a
 * gradient, an enrichment function or a projector (Sec. III.A). */
typedef struct {
  double lo[3], hi[3];
  int32_t ncell[3];
  int32_t p;    /* 1 <= p <= 6 */
  int32_t nq;   /* 1 <= nq <= 7 */
} efe_mesh_desc;

/* Atoms and the synthetic pseudopotential / enrichment parameters.
 *   local part   v(r) = -Z erf(r/loc_rc)/r + loc_amp exp(-(r/loc_rg)^2)
 *   projector    beta(r) = (pi w^2)^(-3/4) exp(-r^2/(2 w^2)), r < kb_rcut,
 *                one per atom with coupling kb_D (kb_width <= 0: none)
 *   enrichment   S_lm(x-R) exp(-enr_alpha r^2) h(r), l <= enr_lmax, smooth
 *                cutoff h ending at enr_rcut with smoothness enr_t
 *                (Eq. eqnCutoffProperties); enr_lmax < 0: plain CFE
 *   rho_alpha    exponent of the Gaussian isolated-atom density (Sec. III.C)
 *   enr_tab_n    > 0: pristine enrichment (Sec. II.B) instead of the Gaussian:
 *                S_lm(x-R) f_l(r) h(r) with f_l = R_l / r^l of the isolated
 *                atom's lowest level of angular momentum l (efe_radial_atom),
 *                tabulated at r = i enr_tab_dr, i < enr_tab_n, as
 *                enr_tab[(2 l) n + i] = f_l, enr_tab[(2 l + 1) n + i] = f_l'
 *                (l <= enr_lmax), cubic Hermite interpolation, zero beyond
 *                the table; h ends at enr_tab_rc[l] with smoothness enr_t;
 *                enr_rcut (the support radius) must cover every enr_tab_rc[l]
 *   atom_tab_n   > 0: atomic densities and potentials (Sec. III.C) from the
 *                isolated atom's radial solution instead of the Gaussian
 *                forms (rho_alpha unused): rows of atom_tab, each of
 *                atom_tab_n values at r = i atom_tab_dr: rho^(I), its slope,
 *                phi^(I) (the potential of rho^(I) + the Gaussian smeared
 *                charge of width loc_rc), its slope (efe_radial_atom); cubic
 *                Hermite interpolation, zero beyond the table; one species
 *                (every Z equal); the pair energies <n_I, n_J> by
 *                radial-angular quadrature over the table points
 * xyz, Z, enr_tab and atom_tab are host arrays read during efe_setup_mesh
 * only. */
typedef struct {
  int32_t natoms;
  const double *xyz;
  const double *Z;
  double loc_rc, loc_amp, loc_rg;
  double kb_width, kb_D, kb_rcut;
  int32_t enr_lmax;
  double enr_alpha, enr_rcut, enr_t;
  double rho_alpha;
  int32_t enr_tab_n;
  double enr_tab_dr;
  const double *enr_tab;
  double enr_tab_rc[3];
  int32_t atom_tab_n;
  double atom_tab_dr;
  const double *atom_tab;
} efe_system_desc;

/* Build the mesh tables, the enrichment and projector data and the overlap
 * blocks (Sec. II.B, III.A): lumped CFE mass, C = b diag(m)^-1, M^ee and the
 * inverses of its atom-diagonal blocks (Eq. MEInvApprox).  `stream` is a
 * hipStream_t (NULL: default stream).  On success *out owns device memory. */
efe_status efe_setup_mesh(const efe_mesh_desc *mesh, const efe_system_desc *sys,
                          void *stream, efe_ctx **out);

/* Radial Kohn-Sham problem of one isolated atom of the synthetic
 * pseudopotential (Sec. II.B: the pristine enrichment functions are the
 * isolated atom's eigenfunctions, a radial part from a 1-D problem times a
 * real spherical harmonic).  u = r R on r_i = i h (i = 1 .. n), zero at 0 and
 * (n+1) h; channel l: -(u_{i+1} - 2u_i + u_{i-1})/(2h^2) + (l(l+1)/(2r^2) +
 * v_eff) u, plus the s projector D |beta><beta| in channel 0; v_eff = local
 * pseudopotential + Hartree (same three-point rule, w = r v_H, w'' = -4 pi r
 * rho) + PW92; Fermi occupations (kT) of the 2(2l+1)-fold levels for Z[atom]
 * electrons; rho_in <- rho_in + mix_beta (rho_out - rho_in) from the Gaussian
 * atomic density until sqrt(4 pi h sum r^2 (rho_out - rho_in)^2) < tol.
 * Then, per l, the lowest level's table f_l = R/r^l and r0 by the three rules
 * of Sec. II.B (at or beyond the last turning point of u, truncated norm
 * within 5e-3 of one, |dR/dr| < 5e-3; at most 10 bohr) with the cutoff's
 * smoothness sys->enr_t.  Outputs (device, written on `stream`):
 *   eps[(lmax+1) nstates], occ[...] (electrons per level, with 2(2l+1)),
 *   u[(l nstates + k) n + i] (h sum u^2 = 1, largest |u| positive),
 *   rho[n] (the last output density), r0[lmax+1],
 *   tab[2(lmax+1)][n+1]: rows 2l, 2l+1 = f_l, f_l' at r = i h (i = 0..n),
 *   the layout of efe_system_desc.enr_tab (cutoff radius r0 (1 + 1/t)),
 *   atab[4][n+1] (may be NULL): rho of the last output density, its slope,
 *   the potential of rho + the Gaussian smeared charge (width loc_rc) with
 *   v_H by the same three-point rule, its slope, at r = i h (values at 0
 *   from (4 f(h) - f(2h))/3, slopes by central differences), the layout of
 *   efe_system_desc.atom_tab.
 * Allocates and frees its own device workspace; reads sys on the host.
 * EFE_ENOTCONV when maxit iterations do not reach tol (outputs are those of
 * the last iteration); messages through efe_last_error(NULL). */
typedef struct {
  int32_t n;          /* grid points */
  double h;           /* spacing (bohr) */
  int32_t lmax;       /* channels 0..lmax, lmax <= 2 */
  int32_t nstates;    /* levels per channel, 1..8 */
  double kT, mix_beta, tol;
  int32_t maxit;
} efe_radial_params;

typedef struct {
  int32_t iterations;
  double residual;    /* last density residual */
  double mu;          /* Fermi level */
} efe_radial_report;

efe_status efe_radial_atom(const efe_system_desc *sys, int32_t atom,
                           const efe_radial_params *prm, void *stream, double *eps, double *u,
                           double *occ, double *rho, double *r0, double *tab, double *atab,
                           efe_radial_report *rep);

/* sizes[0..7] = rows, n_nodes, n_dof (interior nodes + enrichment), n_enr,
 * n_cells, n_qpts (n_cells * nq^3), natoms, nloc ((p+1)^3).  Host array. */
efe_status efe_get_sizes(const efe_ctx *ctx, int64_t *sizes);

/* Coupling of the orthogonalized enrichment to the cells (Sec. II.B, N^E =
 * phi - C N^C): *ncpairs = number of (atom, cell) pairs whose coupling block
 * E_c = B_c - C_c H_c is non-zero (every cell holding one of the atom's
 * support nodes), *max_cell = largest number of enrichment functions coupled
 * to one cell.  Host outputs (either may be NULL). */
efe_status efe_get_coupling(const efe_ctx *ctx, int64_t *ncpairs, int64_t *max_cell);

/* Integer mesh tables in host memory (any pointer may be NULL):
 * cell_to_global[n_cells*nloc], colour_order[n_cells] (cells sorted by colour
 * (cx&1)+2(cy&1)+4(cz&1), then id), colour_offsets[9], boundary[n_nodes]. */
efe_status efe_get_tables(const efe_ctx *ctx, int32_t *cell_to_global, int32_t *colour_order,
                          int32_t *colour_offsets, uint8_t *boundary);

/* Per-atom support cells (which = 0: enrichment, radius enr_rcut; 1: projector,
 * radius kb_rcut).  A cell belongs when its box distance to the atom is below
 * the radius.  *npairs receives the total; ptr[natoms+1] and cells[*npairs]
 * (ascending per atom) are filled when non-NULL.  Host arrays. */
efe_status efe_get_support(const efe_ctx *ctx, int32_t which, int64_t *npairs,
                           int32_t *ptr, int32_t *cells);

/* vq[n_qpts] (device) = sum over atoms of the local pseudopotential at the
 * Gauss points, cell-major (Sec. II.A, Eq. Eel). */
efe_status efe_local_potential(efe_ctx *ctx, double *vq);

/* Set the local Kohn-Sham potential at the Gauss points (device, n_qpts) and
 * rebuild the potential-dependent blocks: per-cell Hamiltonians
 * 1/2 K_cell + V_cell, the enrichment coupling B and H^phiphi (Eq. KS,
 * Discrete_Eig_Gen_H).  `precisions` is a bit mask of (1 << EFE_FP32) and
 * (1 << EFE_BF16) for the reduced-precision cell matrices to keep as well. */
efe_status efe_set_potential(efe_ctx *ctx, const double *vq, int32_t precisions);

/* Y = H^E X for ncols vectors (device blocks, rows x ld).  Blocks wider than
 * 160 vectors are applied 160 columns at a time.  The apply runs the per-cell
 * form of T^T Hhat T: the cell GEMM takes [H_c | E_c^T] on the cell's nodes
 * and enrichment rows, E_c on its nodes for the enrichment rows.  EFE_EINVAL
 * if n_nodes x 160 reaches 2^31 (32-bit offsets of the cell GEMM's gathers);
 * efe_setup_mesh refuses systems with more than 768 enrichment functions
 * coupled to one cell. */
efe_status efe_apply_H(efe_ctx *ctx, const double *X, double *Y, int32_t ncols, int64_t ld);
/* Y = H^E X with the cell GEMMs in the given precision (EFE_FP64, or EFE_FP32
 * / EFE_BF16 with FP32 accumulation; the matrices must have been built by
 * efe_set_potential).  The coupling blocks E_c are formed in FP64 and rounded
 * with the cell matrices; projector and enrichment-block products stay FP64.
 * EFE_BF16 takes plain CFE systems only (EFE_EINVAL with enrichment). */
efe_status efe_apply_H_prec(efe_ctx *ctx, const double *X, double *Y, int32_t ncols, int64_t ld,
                            int32_t prec);
/* Y = M^E X (exact overlap: diag(m) on CFE rows, M^ee on enrichment rows). */
efe_status efe_apply_M(efe_ctx *ctx, const double *X, double *Y, int32_t ncols, int64_t ld);
/* Y = (M~^E)^-1 X (Eq. MEInvApprox). */
efe_status efe_apply_Minv_approx(efe_ctx *ctx, const double *X, double *Y, int32_t ncols,
                                 int64_t ld);

/* Upper bound of the spectrum of (M~^E)^-1 H^E by `steps` Lanczos steps in
 * the M~ inner product from the device start vector v0 (rows):
 * theta_max(T) + |beta_last|.  Result in host memory. */
efe_status efe_spectrum_upper_bound(efe_ctx *ctx, const double *v0, int32_t steps,
                                    double *b_out);

typedef struct {
  int32_t degree;     /* m >= 1 */
  double a, b, a_min; /* unwanted interval (a, b); a_min <= lowest eigenvalue < a */
  int32_t mode;       /* EFE_FILTER_RESIDUAL or EFE_FILTER_STANDARD */
  int32_t prec;       /* EFE_FP64, EFE_FP32, EFE_BF16: operands of the cell GEMMs of
                       * the recurrence; projectors, enrichment rows, G and
                       * V_out stay FP64 */
} efe_cheb_params;

/* Round-off amplification of (M~^E)^-1, set when the context is built:
 * A = max over atoms of ||M^phiphi_II||_F ||(M^ee_II)^-1||_F (an upper bound
 * of ||M^phiphi_II||_2 / lambda_min(M^ee_II); 1 without enrichment).  M^ee is
 * the difference of two terms of the size of M^phiphi, so when an enrichment
 * function lies close to the CFE space the inverse magnifies the rounding of
 * anything it is applied to by up to A.  Host output. */
efe_status efe_enrichment_amplification(const efe_ctx *ctx, double *amp);

/* Largest amplification for which the filter accepts EFE_BF16: the BF16 unit
 * round-off 2^-8 times A must stay below 1, i.e. A <= 256.  Beyond it the
 * rounding of the cell GEMM operands, magnified by (M~^E)^-1, is as large as
 * the filtered residual itself and the filter output carries no digits. */
#define EFE_BF16_MAX_AMPLIFICATION 256.0

/* Chebyshev filter of ncols vectors in place (Sec. III.B).  Residual mode
 * needs the Ritz values `lambda` (device, ncols) paired with V:
 *   G = H V - M V Lambda, Z_1 = (s1/e) G,
 *   Z_k = (2 s_k/e) H M~^-1 Z_{k-1} - (2 c s_k/e) Z_{k-1} - s_{k-1} s_k Z_{k-2}
 *         + (2 s_k/e) G C_{k-1}(Lambda),
 *   V <- M~^-1 Z_m + V C_m(Lambda).
 * Standard mode ignores lambda and applies C_m((M~^E)^-1 H^E) to V.
 * Blocks wider than 160 vectors are filtered 160 columns at a time (every
 * column is filtered on its own).  EFE_EINVAL for EFE_BF16 when the context's
 * amplification exceeds EFE_BF16_MAX_AMPLIFICATION (efe_enrichment_amplification). */
efe_status efe_cheb_filter(efe_ctx *ctx, double *V, const double *lambda, int32_t ncols,
                           int64_t ld, const efe_cheb_params *prm);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * filter as efe_cheb_filter with every workspace taken from a fixed region of
 * EFE_NOALLOC_SCRATCH_BYTES of device memory that the library holds on each
 * GPU it runs on until the process ends (its address on a device is taken
 * when the first context on that device is set up).  No device memory is
 * allocated or freed.  EFE_EINVAL when the call's workspaces (about
 * 4 x rows x min(ncols, 160) doubles plus the apply's) exceed the region;
 * EFE_ESTATE if the region is unavailable on the context's device.  Every call
 * on a GPU shares that GPU's region and leaves its contents behind: calls that
 * overlap on one GPU (other streams, other host threads) race and must not
 * be issued. */
#define EFE_NOALLOC_SCRATCH_BYTES (64u << 20)
efe_status efe_cheb_filter_noalloc(efe_ctx *ctx, double *V, const double *lambda, int32_t ncols,
                                   int64_t ld, const efe_cheb_params *prm);

/* Rayleigh-Ritz in FP64 (Eq. projectedKSEig): S = V^T M V, Hp = V^T H V,
 * Hp R = S R Lambda with R^T S R = I (dense generalized eigensolve on the
 * GPU: Cholesky of S, reduction, divide and conquer), V <- V R.
 * lambda (device, ncols) ascending; resnorm (device, ncols, may be NULL)
 * = ||H v_j - lambda_j M v_j||_2.  Boundary rows of V are set to zero.
 * Any block width: H V is formed in column chunks, the rotation in row
 * blocks in place.  Returns EFE_ENUMERIC if S is not positive definite or
 * the dense eigensolve does not converge. */
efe_status efe_rayleigh_ritz(efe_ctx *ctx, double *V, int32_t ncols, int64_t ld,
                             double *lambda, double *resnorm);

/* ---------------------------------------------------------------- SCF
 * Self-consistent field around the eigensolver (Sec. II.A, III.C): LDA
 * (Perdew-Wang 1992), phi = phi^at + phi^rem with phi^rem from a CFE Poisson
 * problem for rho - sum_I rho^(I) (homogeneous Dirichlet, Jacobi CG),
 * Fermi-Dirac occupations, Anderson mixing of rho at the Gauss points. */
typedef struct {
  int32_t passes_first;  /* filter + Rayleigh-Ritz passes in the first step (minimum) */
  int32_t passes;        /* passes in later steps (minimum) */
  int32_t degree;        /* Chebyshev degree */
  int32_t prec;          /* filter precision (EFE_FP64 / EFE_FP32 / EFE_BF16); EFE_BF16 is
                          * refused as in efe_cheb_filter */
  double kT;             /* smearing temperature in Ha */
  double mix_beta;       /* Anderson damping */
  int32_t mix_history;   /* Anderson history depth, 0..16 */
  double cg_rtol;        /* Poisson CG relative residual (also the Kerker solve) */
  int32_t cg_maxit;
  int32_t lanczos_steps; /* spectrum bound per step */
  /* optional: called on the host after every filter + Rayleigh-Ritz pass with
   * the pass index, the pass's filter and Rayleigh-Ritz times (ms) and
   * `progress_user` (progress reports of long steps); NULL: none */
  void (*progress)(int32_t pass, double filter_ms, double rr_ms, void *user);
  void *progress_user;
  /* Sec. III.B: after the minimum number of passes, further passes run while
   * the largest residual ||H v_j - lambda_j M v_j||_2 of the occupied states
   * (f_j > 1e-14 at the current Ritz values) exceeds tau, up to max_passes
   * passes in the step.  tau <= 0: the minimum only. */
  double tau;
  int32_t max_passes;
  /* Kerker preconditioning of the Anderson update (not in the paper, which
   * names Anderson mixing only): the mixed residual is multiplied by
   * q^2 / (q^2 + k0^2), realized on the CFE mesh as F - u with
   * (K + k0^2 diag(m)) u = k0^2 int F N.  kerker_k0 <= 0: plain Anderson. */
  double kerker_k0;
} efe_scf_params;

typedef struct {
  double E, F, E_band, E_xc, E_el; /* energies at the output density (Ha)      */
  double mu, n_el, drho, dE;       /* Fermi level, int rho_out, ||rho_out - rho_in||, E - E_prev */
  double max_occ_res, b;           /* largest residual of occupied states, bound */
  /* wall times (ms): Poisson solve for rho_in; filter passes; Rayleigh-Ritz;
   * occupied-state density; Anderson mixing; operator rebuild for the new
   * potential; Lanczos bound; Poisson solve and energy sums at rho_out */
  double t_poisson_ms, t_filter_ms, t_rr_ms, t_density_ms, t_other_ms;
  double t_operators_ms, t_bound_ms, t_energy_ms;
  /* passes: filter + Rayleigh-Ritz passes run; cg_iters: Poisson CG
   * iterations (both solves); mix_cg_iters: iterations of the Kerker solve */
  int32_t iter, passes, cg_iters, mix_cg_iters;
} efe_scf_report;

/* Input density of the next SCF step (device, n_qpts, Gauss points cell by
 * cell); resets the mixing history.  Without a call the first step starts
 * from the superposition of atomic densities. */
efe_status efe_set_density(efe_ctx *ctx, const double *rho_q);
/* Copy a density (device, n_qpts): which = 0 input of the next step, 1 output
 * of the last step, 2 superposition of atomic densities. */
efe_status efe_get_density(efe_ctx *ctx, int32_t which, double *out);
/* Gauss points of the mesh (Sec. III.A: n_q-point rule per cell), in the
 * order every per-point array uses (cell by cell, x fastest inside a cell):
 * xq (device, n_qpts x 3) positions, wq (device, n_qpts) weights including the
 * cell Jacobian.  Either output may be NULL, not both (EFE_EINVAL). */
efe_status efe_get_quadrature(efe_ctx *ctx, double *xq, double *wq);

/* ---------------------------------------------------------------------------
 * Learned initial density.  The paper starts the SCF from atomic densities
 * (Sec. IV); this component proposes a corrected start and leaves the
 * converged answer to the SCF.  A point's 25 features are the power spectrum
 * P_nl = sum_m (sum_I g_n(d_I) Y_lm(u_I))^2 of its 16 nearest atoms (ties by
 * the lower atom index; g_n(d) = exp(-(d - n)^2 / 2), n = 0..7; real spherical
 * harmonics l = 0..2; feature 3n + l) and log(max(rho_SAD, 1e-12)) (feature
 * 24), standardized as (f - shift) / scale.  The network is
 * 25 -> 128 -> 128 -> 128 -> 1 with SiLU, FP32, parameters in one flat array
 * of efe_mlp_num_params() floats: W1 [128][25], b1 [128], W2 [128][128], b2,
 * W3 [128][128], b3, W4 [128], b4 [1], row-major.  These calls take no
 * context: `stream` is a hipStream_t (NULL: the default stream), all arrays
 * are device arrays owned by the caller, and errors are reported by status
 * with the message in efe_last_error(NULL).  EFE_EINVAL is returned for
 * negative sizes or missing arrays before any launch.
 * ------------------------------------------------------------------------- */
int64_t efe_mlp_num_params(void);
/* feat (npts x 25, FP32, row per point) of the points pts (npts x 3) around
 * the atoms xyz (natoms x 3) with SAD densities rho_sad (npts).  shift and
 * scale (25 each) are both NULL (raw features) or both given. */
efe_status efe_descriptors(void *stream, const double *pts, int64_t npts, const double *xyz,
                           int32_t natoms, const double *rho_sad, const float *shift,
                           const float *scale, float *feat);
/* out (npts) = network(feat).  acts (3 x npts x 128, optional) receives the
 * pre-activations of the three hidden layers for efe_mlp_backward. */
efe_status efe_mlp_forward(void *stream, const float *params, const float *feat, int64_t npts,
                           float *out, float *acts);
/* Quadrature-weighted squared error L = sum w (out - target)^2 / sum w:
 * dout = dL/dout, sums (2 doubles) = {sum w, sum w (out - target)^2}. */
efe_status efe_mlp_loss_grad(void *stream, const float *out, const float *target,
                             const float *weight, int64_t npts, float *dout, double *sums);
/* grads (efe_mlp_num_params floats, overwritten) = d(sum dout * out)/dparams
 * for the batch whose forward pass stored acts; work: 2 x npts x 128 floats. */
efe_status efe_mlp_backward(void *stream, const float *params, const float *feat,
                            const float *acts, const float *dout, int64_t npts, float *grads,
                            float *work);
/* One Adam step (step counts from 1) on n parameters with moments m, v:
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * params -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps). */
efe_status efe_mlp_adam(void *stream, float *params, const float *grads, float *m, float *v,
                        int64_t n, double lr, double beta1, double beta2, double eps, int64_t step);
/* Set the next SCF step's input density to the learned guess
 * rho_0 = max(rho_SAD + s_t * network, 0) scaled to the electron count
 * sum_I Z_I, on the context's Gauss points; resets the mixing history.
 * norm (host, 51 floats) = shift[25], scale[25], s_t.  Falls back to rho_SAD
 * (and reports *used_fallback = 1) when params is NULL, a value is not
 * finite, or the scale factor leaves [0.9, 1.1]; *factor (host) is that
 * factor (NaN for non-finite values).  Synchronizes the stream. */
efe_status efe_density_guess(efe_ctx *ctx, const float *params, const float *norm,
                             int32_t *used_fallback, double *factor);
/* One SCF step.  V (rows x ld, device) holds the N-vector subspace: any block
 * before the first step (it is Rayleigh-Ritz orthonormalized first), the Ritz
 * vectors after each step; lambda (device, N) their values; v0 (device, rows)
 * the Lanczos start vector.  The report (host) carries the energies of the
 * step and max_occ_res, the largest occupied-state residual after its last
 * pass.  Convergence is decided by the caller (e.g. |dE| / N_atoms < tol).
 * EFE_EINVAL for a bad precision or parameter before any work is done. */
efe_status efe_scf_step(efe_ctx *ctx, double *V, int32_t ncols, int64_t ld, double *lambda,
                        const double *v0, const efe_scf_params *prm, efe_scf_report *rep);

/* Kernel timing.  enable != 0 clears earlier records and starts recording HIP
 * events on the context's stream around the tracked launches; 0 stops.
 * efe_timing_get returns, for a kernel class, the number of recorded launches
 * and their summed duration in milliseconds (synchronizes the stream):
 *   0 one colour pass of the cell GEMM
 *   1 projector coefficients and the Y^C start values of an H apply
 *   2 enrichment rows of an H apply (partial sums and dense blocks)
 *   3 whole H apply of a recurrence step (the recurrence fused into it)
 *   4 whole H apply                      5 whole Rayleigh-Ritz
 *   6 colour pass, blocks of <= 16 vectors (e.g. the Lanczos vector)
 *   7 whole H apply, blocks of <= 16 vectors
 * Classes 0 and 4 count blocks wider than 16 vectors only. */
efe_status efe_timing(efe_ctx *ctx, int32_t enable);
efe_status efe_timing_get(efe_ctx *ctx, int32_t which, int64_t *launches, double *total_ms);

/* Layout check of the matrix-core instructions the cell GEMMs use (test
 * support): one wave forms D = A B with A 16 x K, B K x 16 (device, FP64,
 * row-major; K = 4 for which = 0 FP64 and 1 FP32, K = 32 for 2 BF16) through
 * the lane mappings of the kernels, D 16 x 16 row-major (device). */
efe_status efe_probe_mfma(int32_t which, const double *A, const double *B, double *D);

/* Message of the last failure on this context ("" if none); with ctx == NULL
 * the message of the last failed efe_setup_mesh on the calling thread. */
const char *efe_last_error(const efe_ctx *ctx);

/* Free the context and everything it owns (NULL is ignored). */
void efe_destroy(efe_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* EFE_H */
