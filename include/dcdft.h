/*
 * dcdft.h - C ABI of the divide-and-conquer DFT fragment SCF library (gfx950).
 *
 * The library runs the ground-state SCF iteration of divide-and-conquer DFT
 * (Yamada & Otobe, "SALMON 2.3: Implementation of divide-and-conquer
 * ground-state initialization for large-scale real-time TDDFT", Sec. 2.2):
 * a periodic rectangular cell is cut into a regular grid of core boxes, each
 * extended by a buffer of b grid points into an overlapping fragment with
 * periodic boundaries of its own; every fragment solves its Kohn-Sham problem
 * (Eq. (1)) with the Hamiltonian of Eq. (5); a global chemical potential fixes
 * the electron count; the total density is the sum of the fragment densities
 * projected onto their cores (Eqs. (2)-(4)).  The fragment keywords mirror the
 * paper's input table (Table 1): num_fragment, nstate_frag, num_rgrid_buffer.
 *
 * Conventions shared by every entry point:
 *  - Every call returns a dcdft_status; nothing aborts, throws or exits.
 *    dcdft_last_error() gives a message for the last failure (per context, or
 *    process-wide for a failed setup when called with ctx == NULL).
 *  - Units are Hartree atomic units (bohr, Ha).
 *  - Global arrays are x-fastest: index g = gx + Nx (gy + Ny gz).
 *  - Fragment alpha = ax + Fx (ay + Fy az); its local point l = lx + nx (ly + ny lz)
 *    maps to global gd = (ad * ncore_d - b_d + ld) mod N_d, ncore_d = N_d / F_d,
 *    n_d = ncore_d + 2 b_d.  All fragments have the same box shape.
 *  - Fragment orbital blocks are orbital-major: element (i, l) at i * n + l.
 *  - Inner products carry the volume element dV = hx hy hz, h_d = cell_d / N_d.
 *  - Host input arrays are caller-owned and copied during the call.  Output
 *    buffers are caller-allocated; a buffer that is too small gives
 *    DCDFT_ERR_ARG and the required size in the error message.
 *  - Pointers documented as "device" must point to memory on the context's
 *    GPU (for example a torch tensor's data_ptr()); the library never
 *    allocates or frees them.
 *  - A context is not thread-safe; separate contexts are independent.  All
 *    device work is issued on the context's stream.
 */
#ifndef DCDFT_H
#define DCDFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dcdft_ctx dcdft_ctx;

typedef enum {
  DCDFT_OK = 0,
  DCDFT_ERR_ARG = -1,           /* null pointer, bad value, buffer too small        */
  DCDFT_ERR_SHAPE = -2,         /* grid not divisible by fragments, box too large   */
  DCDFT_ERR_CAPACITY = -3,      /* fragment states cannot hold N_e electrons        */
  DCDFT_ERR_NOT_SPD = -4,       /* overlap matrix not positive definite (Cholesky)  */
  DCDFT_ERR_EIG = -5,           /* subspace eigensolver did not converge            */
  DCDFT_ERR_NAN = -6,           /* non-finite value detected                        */
  DCDFT_ERR_HIP = -7,           /* HIP runtime error                                */
  DCDFT_ERR_OOM = -8,           /* device allocation failed                         */
  DCDFT_ERR_NOT_CONVERGED = -9  /* reserved for drivers that iterate to a tolerance */
} dcdft_status;

/* Model pseudopotential of one species (stand-in for the norm-conserving
 * pseudopotentials of Sec. 2.2):
 *   V_loc(r) = sum_a vloc_depth exp(-|r-R_a|^2 / (2 vloc_sigma^2)), each term kept
 *              where |r-R_a| <= 10 vloc_sigma (minimum-image distance);
 *   V_NL     = sum_a kb_energy |beta_a><beta_a|, beta_a proportional to
 *              exp(-|r-R_a|^2 / (2 kb_sigma^2)) on |r-R_a| <= kb_rcut, normalised
 *              on the global grid, restricted to each fragment box without
 *              renormalisation (Eq. (5), "defined within the fragment"). */
typedef struct {
  double valence;
  double vloc_depth;
  double vloc_sigma;
  double kb_energy;
  double kb_sigma;
  double kb_rcut;
} dcdft_species;

enum { DCDFT_PREC_FP64 = 0, DCDFT_PREC_MIXED = 1 };

typedef struct {
  int32_t n_grid[3];            /* global grid points per axis (x, y, z)            */
  double cell[3];               /* periodic box lengths (bohr)                      */
  int32_t num_fragment[3];      /* Table 1: fragments per axis; must divide n_grid  */
  int32_t num_rgrid_buffer[3];  /* Table 1: buffer b in grid points per axis        */
  int32_t n_atoms;
  const double *atom_pos;       /* host [n_atoms][3] (bohr)                         */
  const int32_t *atom_species;  /* host [n_atoms], index into species               */
  int32_t n_species;
  const dcdft_species *species; /* host [n_species]                                 */
  /* orbitals per fragment: 1..80; with one fragment (the conventional
   * calculation of the cell) 1..4096, more than 80 taking the large-orbital path
   * (BLAS products and FP64 factorisations of the solver library, no captured
   * graph; DC-LCFO is not available there) */
  const int32_t *nstate_frag;   /* host [F] orbitals per fragment, or NULL          */
  int32_t nstate_frag_uniform;  /* Table 1 nstate_frag, used when the array is NULL */
  double n_electrons;           /* N_e fixed by the global chemical potential       */
  double smearing;              /* kT of the Fermi-Dirac occupation (Ha), > 0       */
  double mixing;                /* linear density-mixing fraction in (0, 1]         */
  int32_t cg_sweeps;            /* CG sweeps per SCF iteration, >= 1                */
  int32_t precision;            /* DCDFT_PREC_FP64 or DCDFT_PREC_MIXED              */
  int32_t batched;              /* 1: all fragments per launch + graph replay;
                                   0: one launch sequence per fragment              */
  uint64_t seed;                /* initial-orbital generator seed                   */
  void *hip_stream;             /* hipStream_t to use; NULL: the library makes one  */
} dcdft_params;

/* Scalars of one SCF iteration.  Energies follow the Harris-Foulkes / Mermin
 * form at the input density (ion-ion term omitted). */
typedef struct {
  int32_t iter;                 /* 1-based count of completed iterations            */
  double mu;                    /* global chemical potential (Ha)                   */
  double e_total;               /* free energy (Ha)                                 */
  double e_band;                /* sum 2 f eps w over all fragment states (Ha)      */
  double entropy;               /* -sum 2 w [f ln f + (1-f) ln(1-f)]                */
  double residual_paper;        /* dV sum |rho_k^in - rho_(k-1)^in| / N_e (Sec. 3.3) */
  double residual_out_in;       /* dV sum |rho^out - rho^in| / N_e                  */
  double charge;                /* dV sum rho_tot^out                               */
  float ms_step;                /* device time of the step (ms)                     */
  /* Device time of the step's phases (ms; they add up to ms_step less the host
   * launch gap, -1 where the runtime could not time them):
   *   ms_poisson       from the start to V_eff formed (Hartree solve, V_eff; the
   *                    first projections of the orbitals overlap this phase),
   *   ms_fragments     from there to the last fragment eigensolve finished,
   *   ms_fermi_density chemical potential, densities, energy terms, mixing. */
  float ms_poisson;
  float ms_fragments;
  float ms_fermi_density;
} dcdft_scf_info;

/* Validate p, build the fragment and projector tables, upload them, draw the
 * initial orbitals (SplitMix64 counter stream: orbital-point (alpha, i, l) uses
 * counter ((alpha << 40) | (i << 24) | l) + 1; value = top 53 bits * 2^-53 - 1/2)
 * and Cholesky-orthonormalise them; the input density starts uniform, N_e / volume.
 * Errors: ARG (null or out-of-range field; also when more projectors meet one
 * projector region of a fragment box (a block of whole x rows of at most 256
 * points, or 256 consecutive points) than the projector kernels hold: 96, or
 * fewer where their slot tables would exceed 64 KB of LDS), SHAPE (n_grid %
 * num_fragment != 0 or ncore + 2 b > N), OOM, HIP, NOT_SPD.  On success *out owns
 * all device memory. */
dcdft_status dcdft_setup(const dcdft_params *p, dcdft_ctx **out);

/* Exactly one SCF iteration over all fragments (Sec. 2.2): Hartree potential of
 * rho_tot^in (nine-point FD Poisson equation, solved exactly, zero mean),
 * V_eff of every fragment, cg_sweeps CG sweeps + Rayleigh-Ritz per fragment,
 * core weights, global mu, rho^out assembly (Eqs. (2)-(4)), energy, residuals,
 * linear mixing of rho_tot and of every fragment density.  info may be NULL.
 * Errors: CAPACITY (sum 2 w < N_e), NOT_SPD, EIG, NAN, HIP.  The step is atomic:
 * after CAPACITY, NOT_SPD, EIG or NAN the context holds the state of the last
 * completed step, bit for bit (orbitals, input and output densities, potentials,
 * eigenvalues, weights, occupations, mixer history), and the iteration count is
 * unchanged; info (if given) then carries the failed step's scalars.  After HIP
 * the state is unspecified. */
dcdft_status dcdft_scf_step(dcdft_ctx *c, dcdft_scf_info *info);

/* Host copy of rho_tot^out of the last step (Eq. (2)), n = Nx Ny Nz doubles. */
dcdft_status dcdft_density(const dcdft_ctx *c, double *rho, size_t n);

/* Device copy (double, n = Nx Ny Nz) of rho_tot^out of the last step. */
dcdft_status dcdft_density_device(const dcdft_ctx *c, void *dptr, size_t n);

/* Eigenvalues eps (ascending) and core weights w of fragment frag after the last
 * step; cap = capacity of both host buffers, *m receives m_alpha.  w may be NULL. */
dcdft_status dcdft_eigenvalues(const dcdft_ctx *c, int32_t frag, double *eps, double *w,
                               int32_t cap, int32_t *m);

/* Fragment geometry: shape[3] = (nx, ny, nz), origin[3] = a_d ncore_d - b_d,
 * *m = orbitals, *n_proj = atoms whose projector reaches the fragment box. */
dcdft_status dcdft_fragment_info(const dcdft_ctx *c, int32_t frag, int32_t *shape,
                                 int32_t *origin, int32_t *m, int32_t *n_proj);

/* Global fields (host copy, N doubles) */
enum { DCDFT_FIELD_VLOC = 0, DCDFT_FIELD_VH = 1, DCDFT_FIELD_RHO_IN = 2, DCDFT_FIELD_RHO_OUT = 3 };
dcdft_status dcdft_get_field(const dcdft_ctx *c, int32_t which, double *host, size_t n);

/* Fragment fields (host copy, n doubles): V_eff of the last step, rho_alpha^in,
 * rho_alpha^out. */
enum { DCDFT_FFIELD_VEFF = 0, DCDFT_FFIELD_RHO_IN = 1, DCDFT_FFIELD_RHO_OUT = 2 };
dcdft_status dcdft_get_fragment_field(const dcdft_ctx *c, int32_t frag, int32_t which,
                                      double *host, size_t n);

/* Orbitals of fragment frag as FP64 host arrays [m][n] (state access for
 * restarts and step-by-step comparisons).  set does not re-orthonormalise. */
dcdft_status dcdft_get_orbitals(const dcdft_ctx *c, int32_t frag, double *host, size_t count);
dcdft_status dcdft_set_orbitals(dcdft_ctx *c, int32_t frag, const double *host, size_t count);

/* Replace rho_tot^in (N doubles) and, if rho_frag_in is not NULL, every fragment's
 * rho_alpha^in ([F][n] doubles); with NULL each fragment gathers rho_tot^in.  V_H
 * and V_eff are formed from the new density.  Errors: ARG (NULL), NAN (a value of
 * either array not finite; nothing is changed), HIP. */
dcdft_status dcdft_set_density(dcdft_ctx *c, const double *rho_tot_in, const double *rho_frag_in);

/* Fixed-density DC (Sec. 2.6, third usage; Sec. 3.2): with fixed = 1 every later
 * dcdft_scf_step keeps rho_tot^in and each rho_alpha^in as they are (a density read
 * in, typically with dcdft_set_density from a conventional calculation): V_H and
 * V_eff are formed once, here, from the current rho^in, and the step runs the
 * fragment eigensolvers, mu, rho^out, energies and residuals without the Poisson
 * solve, the V_eff update or the mixing (residual_paper is 0; residual_out_in
 * measures how far rho^out is from the frozen density).  dcdft_set_density while
 * fixed re-forms the potentials of the new density.  fixed = 0 restores the SCF
 * step.  Errors: ARG (fixed not 0 or 1), HIP. */
dcdft_status dcdft_fix_density(dcdft_ctx *c, int32_t fixed);

/* Density-template potential of Eq. (5): V^alpha(l) = (rho_alpha^in(l) - rho_tot^in(g(l)))
 * / xi, g(l) the global point of fragment point l, added to every fragment's V_eff.
 * xi > 0 turns it on; xi = 0 turns it off (the default, as in the paper).  It enters
 * the next formation of V_eff: the next dcdft_scf_step, or at once in fixed-density
 * mode.  The energy expression is unchanged (linear mixing keeps the two input
 * densities equal on core points, so V^alpha acts on buffer points only).
 * Errors: ARG (xi negative or not finite). */
dcdft_status dcdft_set_template(dcdft_ctx *c, double xi);

/* Density mixing of the SCF step.  The paper iterates rho_tot "by the same
 * procedure as conventional DFT" (Sec. 2.2) and names no scheme.
 *   DCDFT_MIX_LINEAR: rho <- rho + alpha (rho^out - rho) for rho_tot and every
 *     fragment density (setup's `mixing` is this alpha); q0 and history ignored.
 *   DCDFT_MIX_PULAY: Pulay (DIIS) mixing with a Kerker preconditioner.  From the
 *     last `history` pairs (rho_in^(j), R^(j) = rho_out^(j) - rho_in^(j)) the weights
 *     c (sum 1) minimise |sum c_j R^(j)|^2 (plain sum over grid points, Gaussian
 *     elimination with partial pivoting on the bordered system, oldest entry
 *     first; a pivot at most 1e-12 max|A| cuts the history to the newest entry),
 *     and rho_new = sum c_j rho_in^(j) + alpha K[sum c_j R^(j)], K(q) = q^2 /
 *     (q^2 + q0^2) on the Fourier modes of the periodic grid with q^2 the symbol
 *     of minus the nine-point Laplacian of the Poisson solve (K = 1 when q0 = 0).
 *     Every fragment density is the gathered rho_tot plus a deviation (zero on
 *     its core, Eq. (3)), mixed with the same weights and alpha without K.
 *     A new Pulay mixer starts with an empty history.
 * alpha in (0, 1], q0 >= 0 (bohr^-1), history 1..16.  The first Pulay call
 * allocates (history + 1) x (N + F n) doubles twice, kept until dcdft_destroy.
 * Errors: ARG, OOM, HIP. */
enum { DCDFT_MIX_LINEAR = 0, DCDFT_MIX_PULAY = 1 };
dcdft_status dcdft_set_mixer(dcdft_ctx *c, int32_t kind, double alpha, double q0,
                             int32_t history);

/* DC-LCFO post-processing (Sec. 2.3, Eqs. (6)-(9)), on the orbitals and V_eff of
 * the last step (normally a converged SCF).  Per fragment: the orbitals with
 * eps < eps_cut (Ha; the paper quotes eps_cut - mu = 0.1 eV) projected on the
 * core (Eq. (3)'s projection), their overlap S (Eq. (6)), its eigenpairs, and the
 * basis lambda_l = sum_j phibar_j v_jl / sqrt(sigma_l) over the eigenvalues sigma_l
 * > lambda_cut (the paper quotes 1e-7), ascending in sigma, orthonormal over the
 * whole system (Eq. (7)).  Then the global matrix of Eq. (9): same-fragment
 * blocks <lambda^a_i|H^a lambda^a_j>; blocks of fragments a != b whose core meets
 * the other's box, 1/2 [<H^a lambda^a_i|lambda^b_j> + <lambda^a_i|H^b lambda^b_j>];
 * zero elsewhere.  H^a is the fragment Hamiltonian of Eq. (5) on the fragment box.
 * All of it is FP64 (orbitals of the mixed mode are widened).  The diagonalisation
 * of the global matrix is not part of this library.  The first call allocates
 * device memory (two FP64 arrays of the orbital size and the pair tables), kept
 * until dcdft_destroy; the call overwrites work arrays, never the SCF state.
 * Errors: ARG (no step taken yet, non-finite eps_cut, lambda_cut not > 0, a
 * fragment of more than 80 orbitals, or a projector region too dense for the FP64
 * projector kernels' 64 KB of LDS, which a mixed-precision setup does not
 * check), EIG, OOM, HIP. */
typedef struct {
  int32_t n_basis;              /* basis functions over all fragments               */
  int32_t n_pairs;              /* ordered fragment pairs with a neighbour block    */
  float ms;                     /* device time of the build (ms)                    */
} dcdft_lcfo_info;
dcdft_status dcdft_lcfo_build(dcdft_ctx *c, double eps_cut, double lambda_cut,
                              dcdft_lcfo_info *info);

/* Basis of fragment frag from the last dcdft_lcfo_build, host [nb][n] (fragment box
 * points, zero outside the core); *nb (may be NULL) receives the count; host NULL
 * queries the count only.  Errors: ARG (no build, index, buffer smaller than nb n). */
dcdft_status dcdft_lcfo_basis(const dcdft_ctx *c, int32_t frag, double *host, size_t count,
                              int32_t *nb);

/* The global matrix of the last dcdft_lcfo_build, host row-major [N][N], N the total
 * basis count (fragments in order, each fragment's basis in its order); host NULL
 * queries N only.  Errors: ARG (no build, buffer smaller than N^2). */
dcdft_status dcdft_lcfo_hamiltonian(const dcdft_ctx *c, double *host, size_t count,
                                    int32_t *n_basis);

/* One block of that matrix, rows of fragment a's basis and columns of b's, host
 * row-major [rows][cols]: the same-fragment block for a == b, the symmetrised
 * neighbour block otherwise (zero for fragments that are not neighbours); the same
 * values as the dense matrix without forming it.  host NULL queries the shape.
 * Errors: ARG (no build, index, buffer smaller than rows cols). */
dcdft_status dcdft_lcfo_block(const dcdft_ctx *c, int32_t a, int32_t b, double *host,
                              size_t count, int32_t *rows, int32_t *cols);

/* H^alpha psi for m vectors of fragment frag with its V_eff of the last step
 * (after setup: V_loc + V_xc of the uniform density, V_H = 0), Eq. (5):
 * kinetic (nine-point FD, periodic on the fragment box) + V_eff + V_NL.
 * psi, hpsi: device [m][n] of double (prec 0) or float (prec 1); may not alias.
 * The work runs on the context's stream, in chunks of at most m_pad vectors,
 * with scratch the context allocated at setup (nothing is allocated per call).
 * psi must be complete when the call is made (the call does not wait for work
 * on other streams); hpsi is complete when the call returns (the call
 * synchronises the context's stream).  Errors: ARG (NULL, fragment index, m < 0,
 * prec, aliasing), HIP. */
dcdft_status dcdft_apply_h(dcdft_ctx *c, int32_t frag, const void *psi, void *hpsi,
                           int32_t m, int32_t prec);

/* Band-energy functional E = sum_i f_i <psi_i|H^alpha|psi_i> (inner product with dV)
 * and its gradient, recomputing H psi:
 *   grad_psi[i][l] = 2 f_i dV (H psi_i)(l),   grad_v[l] = dV sum_i f_i psi_i(l)^2,
 * grad_v being the derivative with respect to the local potential V_eff (with f
 * carrying 2 x occupation it is dV times the fragment density of Eq. (4)).
 * psi, grad_psi: device [m][n], double (prec 0) or float (prec 1); f: device
 * double [m]; veff: device double [n] used as V_eff of the fragment, or NULL for
 * the fragment's V_eff of the last step; grad_v: device double [n]; energy:
 * device double [1].  Any of energy, grad_psi, grad_v may be NULL.  H psi is
 * formed chunk by chunk (at most m_pad vectors) in scratch the context allocated
 * at setup; nothing is allocated per call.  Inputs must be complete when the call
 * is made; outputs are complete when it returns (the context's stream is
 * synchronised).  Errors: ARG (NULL psi or f, fragment index, m < 1, prec), HIP. */
dcdft_status dcdft_band_energy(dcdft_ctx *c, int32_t frag, const void *psi, const double *f,
                               int32_t m, int32_t prec, const double *veff, double *energy,
                               void *grad_psi, double *grad_v);

/* The backward of the band-energy functional in the argument order of the
 * boundary's original statement: dcdft_band_energy(c, frag, psi, f, m, prec,
 * NULL, NULL, grad_psi, grad_v), i.e. grad_psi[i][l] = 2 f_i dV (H^alpha psi_i)(l)
 * and grad_v[l] = dV sum_i f_i psi_i(l)^2 (device double [n]) with the fragment's
 * V_eff of the last step, Eq. (5).  Same layouts, scratch, synchronisation and
 * errors as dcdft_band_energy. */
dcdft_status dcdft_band_energy_bwd(dcdft_ctx *c, int32_t frag, const void *psi, const double *f,
                                   void *grad_psi, void *grad_v, int32_t m, int32_t prec);

/* The band-energy functional of every fragment in one call, with its gradients
 * (Eq. (5) for each H^alpha, V_eff^alpha of the last step):
 *   E = sum_alpha sum_i f_i <psi_i^alpha|H^alpha|psi_i^alpha>  (inner products with dV),
 *   grad_psi[B][l] = 2 f_B dV (H^alpha psi_B)(l),
 *   grad_v[G] = dV sum over the fragment boxes containing global point G of
 *               sum_i f_i psi_i^alpha(l)^2, l the local point of G in the box,
 * grad_v being the derivative with respect to the local potential on the global
 * grid, which enters every H^alpha through V_eff^alpha.  psi, grad_psi: device
 * [M_tot][n] of double (prec 0) or float (prec 1): the vectors of every fragment
 * in fragment order (fragment alpha's nstate_frag[alpha] vectors after those of
 * the fragments before it; M_tot their sum); f: device double [M_tot]; energy:
 * device double [1]; grad_v: device double [Nx Ny Nz], x fastest.  Any of energy,
 * grad_psi, grad_v may be NULL.  H psi is formed in grad_psi when given (and
 * scaled there to the gradient), else in the context's search-direction array,
 * which holds it when prec's element is no wider than the context's.  Nothing is
 * allocated; the call shares scratch with dcdft_scf_step, so both go on the
 * context's stream (never concurrently).  Inputs must be complete when the call
 * is made; outputs are complete when it returns.  On the large-orbital path (one
 * fragment of more than 80 orbitals) the call is dcdft_band_energy of fragment 0
 * (chunk by chunk, H psi in its scratch) with grad_v formed on the global grid.
 * Errors: ARG (NULL psi or f, prec, grad_psi aliasing psi, an FP64 call on a
 * mixed-precision context without grad_psi, projector LDS of that precision),
 * HIP. */
dcdft_status dcdft_band_energy_all(dcdft_ctx *c, const void *psi, const double *f, int32_t prec,
                                   double *energy, void *grad_psi, double *grad_v);

/* dcdft_band_energy for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, results and errors, with H psi formed in a static 8 MiB device array
 * of the library instead of the context's scratch.  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).  Each GPU holds one copy
 * of the array until the process ends, found at dcdft_setup on that device, and
 * every call on that GPU shares it: calls that overlap in time on one GPU (from
 * several threads or contexts) race and give undefined results.  Nothing in it
 * needs clearing (each call writes every part it reads).  The array holds the
 * layout tables (about 12 bytes per fragment) and as many vectors of the
 * fragment box as fit (at most m_pad per chunk): a box whose single vector does
 * not fit beside the tables gives ARG, as does a context on a device numbered 64
 * or above. */
dcdft_status dcdft_band_energy_noalloc(dcdft_ctx *c, int32_t frag, const void *psi,
                                       const double *f, int32_t m, int32_t prec,
                                       const double *veff, double *energy, void *grad_psi,
                                       double *grad_v);

/* Device-time accounting of kernel families (for roofline reports).  While
 * enabled, steps run eagerly (not from the step graph) and every launch of the
 * families below is bracketed by HIP events on the context's stream; dcdft_kernel_time returns, since timing was (re-)enabled,
 * the number of launches, their summed device milliseconds, and their summed
 * algorithmic HBM bytes and flops (minimum traffic: every operand read once,
 * every result written once; any of the outputs may be NULL).  Enabling resets
 * the counters.  Timing adds two event records per launch and nothing else.
 *   HLOC:   (-1/2 L_FD + V_eff) X; bytes 2 s n per orbital + 8 n per fragment
 *           (s = 8 for FP64), flops 55 n per orbital.
 *   GRAM:   plain X^T Y per fragment; bytes s n (m_x + m_y), flops 2 n m^2.
 *   ROTATE: Y = c Z + M^T X per fragment; bytes s n m (2 to 4), flops 2 n m^2.
 *   GRAM_FUSED: Gram products fused with building their operand (P = beta P -
 *           G, written; or the 2x2 band rotations of Psi and W, written);
 *           bytes s n m (4 or 6), flops 2 n m^2 (n m^2 when symmetric).
 *   KB:     projections c = dV beta^T X (bytes s n m) and their application
 *           Y += beta E c (bytes 2 s n m); flops not counted. */
enum { DCDFT_KERNEL_HLOC = 0, DCDFT_KERNEL_GRAM = 1, DCDFT_KERNEL_ROTATE = 2,
       DCDFT_KERNEL_GRAM_FUSED = 3, DCDFT_KERNEL_KB = 4, DCDFT_KERNEL_COUNT = 5 };
dcdft_status dcdft_kernel_timing(dcdft_ctx *c, int32_t enable);
dcdft_status dcdft_kernel_time(dcdft_ctx *c, int32_t kernel, int64_t *launches, double *ms,
                               double *bytes, double *flops);

/* Launch-shape autotuner for the batched step.  Times, on this context's own
 * orbital arrays and with HIP events on its stream, the candidate shapes of
 *   - the stencil kernel H_loc X (DCDFT_HLOC_*: one plane in flight, or a
 *     haloed LDS plane with 2-, 3- or 4-plane load chunks, or 2-plane chunks
 *     with the periodic end planes held in registers, or 16-byte runs of x
 *     points per thread with one-plane chunks and a few orbitals per
 *     workgroup (fewest that keep 85% of lanes busy, or the most that fill
 *     whole waves), also with z cut into 2 or 3 segments per orbital (more
 *     workgroups in flight, four extra planes read at each cut), or 8-byte
 *     runs (fewer registers per thread, more waves); the vector forms need n_x
 *     a multiple of the run length (segments: n_z / segments >= 4) and fall
 *     back to the 2-plane haloed kernel otherwise),
 *   - the rotation kernels (2, 4 or 8 sixteen-point tiles per wave),
 *   - the Gram products (the point range of a fragment cut into G chunks,
 *     G among half, one, two and four times the default),
 * and keeps the fastest of each for every later step (the step graph is
 * re-captured).  Stencil variants are timed with the fused <x, Hx> the sweeps
 * use; the two fastest are timed again, alternately, before the choice.
 * Stencil variants give bitwise-identical results; the tile
 * and chunk counts change only the summation order of FP64 partial sums.
 * Call between steps: it overwrites work arrays, never the SCF state.
 * cache_path (may be NULL): a text file of earlier choices, one line per
 * device/shape key; a matching line is applied without timing, otherwise the
 * new choice is appended (an unwritable file gives DCDFT_ERR_ARG after the
 * choice has been applied).  out (may be NULL) receives the choice and the
 * measured milliseconds per launch (-1: candidate not applicable or not
 * timed).  A context on the large-orbital path (one fragment of more than 80
 * orbitals) tunes the stencil variant only: its products are library GEMMs.
 * Fragment boxes with more than 1024 points per plane use the plane-tiled
 * stencil whatever the variant. */
enum { DCDFT_HLOC_PLANE = 0, DCDFT_HLOC_HALO_PD2 = 1, DCDFT_HLOC_HALO_PD3 = 2,
       DCDFT_HLOC_HALO_PD4 = 3, DCDFT_HLOC_HALO_PD2_ENDS = 4, DCDFT_HLOC_VEC = 5,
       DCDFT_HLOC_VEC_WIDE = 6, DCDFT_HLOC_VEC_Z2 = 7, DCDFT_HLOC_VEC_Z3 = 8,
       DCDFT_HLOC_VEC8 = 9, DCDFT_HLOC_VEC8_WIDE = 10, DCDFT_HLOC_COUNT = 11 };
typedef struct {
  int32_t hloc_variant;  /* DCDFT_HLOC_* */
  int32_t rot_tiles;     /* 2, 4 or 8 */
  int32_t gram_chunks;
  int32_t from_cache;    /* 1 if the choice came from cache_path */
  double ms_hloc[DCDFT_HLOC_COUNT];
  double ms_rot[3];      /* tiles 2, 4, 8 */
  int32_t gram_candidates[4];
  double ms_gram[4];
} dcdft_tune_info;
dcdft_status dcdft_autotune(dcdft_ctx *c, const char *cache_path, dcdft_tune_info *out);

/* Read or set the launch shapes directly.  set: hloc_variant DCDFT_HLOC_* (the
 * halo variants need a fragment box of at least 4 x 4 x 8 points), rot_tiles
 * 2, 4 or 8, gram_chunks 1..gram_chunks_max (as get reports it), streams
 * 1..4: the batched step's eigensolver runs over `streams` groups of
 * fragments (split at equal sums of m_alpha times the square of its 16-padded
 * count) on as
 * many streams, forked and joined inside the step (default 2, or 3 with 192
 * fragments or more; results do not depend on it); anything else is
 * DCDFT_ERR_ARG and changes nothing.  get: any pointer may be NULL. */
dcdft_status dcdft_get_launch(const dcdft_ctx *c, int32_t *hloc_variant, int32_t *rot_tiles,
                              int32_t *gram_chunks, int32_t *gram_chunks_max, int32_t *streams);
dcdft_status dcdft_set_launch(dcdft_ctx *c, int32_t hloc_variant, int32_t rot_tiles,
                              int32_t gram_chunks, int32_t streams);

/* Release everything owned by c.  NULL-safe. */
void dcdft_destroy(dcdft_ctx *c);

/* Static string for a status code (any int32 value: codes outside the
 * dcdft_status values give "unknown status"). */
const char *dcdft_status_string(int32_t s);

/* Copy the last error message of c (or of the last failed setup if c is NULL)
 * into buf (NUL-terminated, truncated to n bytes). */
dcdft_status dcdft_last_error(const dcdft_ctx *c, char *buf, size_t n);

#ifdef __cplusplus
}
#endif

#endif /* DCDFT_H */
