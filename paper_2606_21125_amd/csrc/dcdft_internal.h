// Internal declarations of the DC-DFT fragment SCF library: context layout,
// device helpers and the host launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dcdft.h"

namespace dcdft {

constexpr int kWave = 64;
constexpr int kMaxTiles = 5;        // m_pad <= 80 orbitals per fragment (16-wide MFMA tiles)
constexpr int kMaxOrb = 16 * kMaxTiles;
// one fragment (the conventional calculation of a cell) may hold more: its
// subspace algebra then runs on rocBLAS / rocSOLVER (the large-orbital path)
constexpr int kMaxOrbLarge = 4096;
constexpr int kLargeGramParts = 64;  // Gram products: chunks of points summed in FP64

// Device-side status flags (bit mask, read back once per step).
enum : int { FLAG_NOT_SPD = 1, FLAG_EIG = 2, FLAG_CAPACITY = 4, FLAG_NAN = 8 };

// Slots of the device scalar block.
enum : int {
  SC_MU = 0, SC_EBAND, SC_ENTROPY, SC_CAPACITY,
  SC_HXC, SC_EH, SC_EXC, SC_CHARGE, SC_RES_OUT_IN, SC_RES_PAPER,
  SC_COUNT
};

// Geometry shared by all kernels (passed by value).
struct Geo {
  int N[3];       // global grid
  int nl[3];      // fragment box (nx, ny, nz)
  int nc[3];      // core size per axis
  int b[3];       // buffer per axis
  int F[3];       // fragments per axis
  int n;          // points per fragment
  long long Ng;   // global points
  double h[3];
  double dv;
  // kinetic stencil coefficients -1/2 c_k / h_d^2: [0] centre (all axes), then
  // x k=1..4, y k=1..4, z k=1..4 (set once at setup, uniform in every kernel)
  double kc[13];
  // launch choices (set at setup, possibly replaced by the autotuner)
  int hloc_variant;  // HLOC_*
  int rot_tiles;     // 16-point tiles per wave of the rotation kernels: 2, 4 or 8
};

// stencil kernel variants; all compute the same sums in the same order
enum {
  HLOC_PLANE = DCDFT_HLOC_PLANE,                  // one plane in flight
  HLOC_HALO_PD2 = DCDFT_HLOC_HALO_PD2,            // haloed LDS plane, 2-plane load chunks
  HLOC_HALO_PD3 = DCDFT_HLOC_HALO_PD3,            // ... 3-plane chunks
  HLOC_HALO_PD4 = DCDFT_HLOC_HALO_PD4,            // ... 4-plane chunks
  HLOC_HALO_PD2_ENDS = DCDFT_HLOC_HALO_PD2_ENDS,  // 2-plane chunks, end planes in registers
  HLOC_VEC = DCDFT_HLOC_VEC,                      // 16-byte x runs per thread, few orbitals/WG
  HLOC_VEC_WIDE = DCDFT_HLOC_VEC_WIDE,            // ... whole-wave orbital groups
  HLOC_VEC_Z2 = DCDFT_HLOC_VEC_Z2,                // HLOC_VEC with z cut into 2 segments
  HLOC_VEC_Z3 = DCDFT_HLOC_VEC_Z3,                // ... 3 segments
  HLOC_VEC8 = DCDFT_HLOC_VEC8,                    // 8-byte x runs, few orbitals/WG
  HLOC_VEC8_WIDE = DCDFT_HLOC_VEC8_WIDE,          // ... whole-wave orbital groups
  HLOC_NVARIANT = DCDFT_HLOC_COUNT
};
bool hloc_halo_ok(const Geo &g);
// LDS bytes a projector kernel needs (slot tables plus the (E C)^T block of apply
// or the partial sums of project) for KS slots, rr region rows and tiles 16-orbital
// tiles
size_t kb_lds_bytes(const Geo &g, int KS, int rr, int rp, int tiles, size_t elem, bool apply);

// Fragments are launched in an order sorted by their count of 16-orbital tiles
// (launch order; the identity when every fragment has the same count): kernels
// tiled by fragment take a range [f0, f1) of launch positions and the fragment at
// position p is perm[p].  Bands are laid out in launch order, so a launch range
// covers a contiguous range of bands.
struct LargeBlas;         // rocBLAS state of the large-orbital path (k_large.hip)

struct OrbSet {           // flattened orbital layout [M_tot][n]
  int nfrag;
  int m_pad;              // multiple of 16, >= max m (stride of the small matrices)
  int tiles;              // 16-orbital tiles the launched kernels are compiled for
  long long M_tot;
  const int *m;           // [F] orbitals of each fragment
  const long long *moff;  // [F] first band of each fragment
  const int *band_frag;   // [M_tot]
  const int *perm;        // [F] fragment at each launch position
  const long long *h_moff;  // host [F + 1]: first band of each launch position (ranges)
  const int *h_m;           // host copy of m
  // 1: the arrays hold m_pad spare rows after the last band, so a kernel may
  // read any padded row of a fragment (context arrays); 0: rows past a
  // fragment's m must not be read (caller-provided arrays)
  int row_pad;
  long long b0(int p) const { return h_moff[p]; }
  long long nb(int p0, int p1) const { return h_moff[p1] - h_moff[p0]; }
};

// Projector regions: each fragment's points are cut into regions of at most
// kRegion points, each listing the KS (padded) fragment atoms whose support
// meets it.  Block regions (RY > 0) are RX x-points (a multiple of 4 dividing
// nx) times RY rows times RZ planes (RP = RX RY RZ points, a multiple of 64),
// shaped to meet as few atoms as possible; otherwise (RY = 0) a region is
// kRegion consecutive points.  The beta values are not stored: the kernels
// evaluate beta_a(l) = sc_a exp(-r2 / (2 sigma_a^2)) on r2 <= rcut_a^2, with
// r2 = (dz^2 + dy^2) + dx^2 taken from per-pair tables of squared offsets, as
// the product of per-row and per-x exponential factors staged per region.
constexpr int kRegion = 256;
constexpr int kBlockRegionMax = 512;   // points of a block region, at most
constexpr int kMaxSlotTiles = 6;    // KS_max <= 96 slots per region
// local rows (runs of nl[0] points) a region can touch
__host__ __device__ constexpr int region_rows(int nx) { return (kRegion - 1) / nx + 2; }

struct KBTables {
  int A_max;
  int NR;                            // regions per fragment
  int KS;                            // slots per region (multiple of 16)
  int RX, RY, RZ;                    // block regions: x points, rows, planes (RY = 0: linear)
  int RP;                            // points per region
  const int *reg_atom;               // [F][NR][KS] local atom index or -1
  const int *reg_nt;                 // [F][NR] slot tiles in use (16 slots each)
  const long long *ar_ptr;           // [F * A_max + 1] into (region, slot) lists
  const int *ar_reg;                 // region of each entry
  const int *ar_slot;                // slot of each entry
  int n_pairs;                       // total (fragment, atom) pairs
  const int *A;                      // [F] atoms per fragment
  const int *pair_first;             // [F + 1] pair of local atom a of f: pair_first[f] + a
  const double *pr_sq;               // [n_pairs][nl0 + nl1 + nl2] squared axis offsets (inf: outside)
  const double *pr_par;              // [n_pairs][3] sc, 1 / (2 sigma^2), rcut^2
  const double *E;                   // [F][A_max]
};

void fail_hip(hipError_t e, const char *what);

// Pulay mixing with a Kerker preconditioner: history of at most H entries in
// S = H + 1 ring slots (the step writes the free one), device-side bookkeeping
// st = {entries in use, newest slot}, residual Gram A [S][S] by slot, weights c [S].
constexpr int kMixMaxSlots = 17;    // H <= 16
struct MixState {
  int S = 0, H = 0, nblk = 0;
  double alpha = 0.3, q0 = 0.0;
  int *st = nullptr;                 // [2]
  double *A = nullptr, *c = nullptr; // [S * S], [S]
  double *part = nullptr;            // [nblk * kMixMaxSlots] block partials
  double *hrho = nullptr, *hres = nullptr;   // [S][N_g]: rho_in^(j), R^(j)
  double *hdin = nullptr, *hdres = nullptr;  // [S][F n]: fragment deviations
  double *rbar = nullptr, *kres = nullptr;   // [N_g]: sum c rho_in, K sum c R
};

}  // namespace dcdft

struct dcdft_ctx {
  dcdft::Geo geo;
  int nF = 0;
  std::vector<int> m;
  std::vector<long long> moff;       // [F + 1] first band of each fragment (moff[F] = M_tot)
  std::vector<int> perm, inv_perm;   // launch order: fragment at each position, and back
  std::vector<long long> pmoff;      // [F + 1] first band of each launch position
  // runs of launch positions whose fragments use the same number of 16-orbital tiles
  struct TileClass {
    int p0, p1, tiles;
  };
  std::vector<TileClass> classes;
  int m_pad = 0, tiles = 0;
  long long M_tot = 0;
  double ne = 0, smearing = 0, mixing = 0;
  int sweeps = 0, precision = 0, batched = 1;
  uint64_t seed = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;                  // the HIP device current at setup
  // Concurrent fragment groups of the batched step: the eigensolver runs over
  // `streams` groups of fragments (split at equal padded matrix-core work), group g on
  // stream g (group 0 on the context's stream), forked and joined by events
  // inside the captured step.  xs is the stream the eigensolver helpers issue
  // to (null: the context's stream).
  static constexpr int kMaxStreams = 4;
  int streams = 2;                // set at setup from the fragment count
  hipStream_t xstreams[kMaxStreams] = {};  // [0] unused (the context's stream)
  hipEvent_t ev_fork = nullptr, ev_join[kMaxStreams] = {};
  bool pre_projected = false;    // the step's first projections were issued before V_eff
  hipStream_t xs = nullptr;
  int iter = 0;
  int gram_chunks = 1;
  int gram_chunks_max = 1;

  // fragment -> host copies
  std::vector<int> A;                // projectors per fragment
  std::vector<int> pair_first;       // [F + 1] first (fragment, atom) pair of each fragment
  int A_max = 0;

  // device allocations (freed in destroy)
  std::vector<void *> allocs;

  // tables
  int *d_m = nullptr, *d_perm = nullptr;
  long long *d_moff = nullptr;
  int *d_band_frag = nullptr;
  // the same tables in fragment order (bands of fragment f after those of the
  // fragments before it), for calls on caller arrays of every fragment
  std::vector<long long> nmoff;      // [F + 1]
  long long *d_nmoff = nullptr;
  int *d_nband = nullptr, *d_ident = nullptr;
  double *d_eb_all = nullptr;        // [M_tot] per-band energy terms
  // KB
  int n_pairs = 0;
  int *d_A = nullptr, *d_pair_first = nullptr;
  double *d_pr_sq = nullptr, *d_pr_par = nullptr, *d_E = nullptr;
  double *d_C = nullptr;             // [F][A_max][m_pad] projections
  int NR = 0, KS = 0, RX = 0, RY = 0, RZ = 0, RP = 256;
  int *d_reg_atom = nullptr, *d_reg_nt = nullptr, *d_ar_reg = nullptr, *d_ar_slot = nullptr;
  long long *d_ar_ptr = nullptr;
  double *d_cpart = nullptr;         // region projection partials [F][NR][KS][m_pad]

  // orbital arrays [M_tot][n], element type double (FP64) or float (mixed).
  // The orbitals live in two buffers: d_psi holds the state of the last
  // completed step; a step reads it and writes its new orbitals into
  // d_psi_next, and the two swap only when the step succeeds.
  void *d_psi = nullptr, *d_psi_next = nullptr, *d_w = nullptr, *d_p = nullptr, *d_q = nullptr;
  void *psi_first = nullptr;    // the buffer d_psi pointed to after setup (graph slot 0)
  size_t elem = sizeof(double);

  // fields
  double *d_vloc = nullptr, *d_vh = nullptr, *d_rho_in = nullptr, *d_rho_out = nullptr;
  double *d_fft_a = nullptr, *d_fft_b = nullptr;   // Poisson work arrays
  double *d_qf[3] = {nullptr, nullptr, nullptr};   // forward basis per axis [N][N]
  double *d_qi[3] = {nullptr, nullptr, nullptr};   // inverse basis per axis
  double *d_lam[3] = {nullptr, nullptr, nullptr};  // per-axis FD eigenvalue of each basis column
  double *d_veff = nullptr, *d_rhof_in = nullptr, *d_rhof_out = nullptr;
  float *d_veff32 = nullptr;  // FP32 rounding of d_veff (read by the FP32 stencil)
  double *d_hdot = nullptr;   // stencil dot partials [kHlocZsMax][M_tot]

  // small matrices [F][m_pad][m_pad]
  double *d_gpart = nullptr;         // Gram partials [F][chunks][m_pad][m_pad]
  double *d_gpart2 = nullptr;        // second product of a fused Gram, same layout
  double *d_gtmp = nullptr;          // Gram result when only the symmetric part is kept
  double *d_dpart = nullptr;         // per-workgroup band partials [F][wpf][2][m_pad]
  double *d_hs_full = nullptr, *d_hs = nullptr, *d_x = nullptr, *d_s = nullptr, *d_lin = nullptr,
         *d_u = nullptr, *d_bmat = nullptr;

  // per-band [M_tot]
  double *d_gamma = nullptr, *d_gamma_prev = nullptr, *d_beta = nullptr, *d_nu = nullptr,
         *d_inv = nullptr, *d_a = nullptr, *d_bb = nullptr, *d_cc = nullptr, *d_cos = nullptr,
         *d_sin = nullptr, *d_eps = nullptr, *d_wcore = nullptr, *d_occ = nullptr;
  double *d_scal = nullptr;          // [SC_COUNT]
  double *d_part = nullptr;          // reduction partials
  int n_part = 0;
  int *d_flags = nullptr;
  double *d_info_host = nullptr;     // pinned host mirror of scalars

  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::string last_error;


  // kernel-family timing (dcdft_kernel_timing)
  struct PendingTimer {
    hipEvent_t a, b;
    int kind;
    double bytes, flops;
  };
  bool timing = false;
  std::vector<PendingTimer> pending;
  std::vector<hipEvent_t> event_pool;
  long long k_launches[DCDFT_KERNEL_COUNT] = {};
  double k_ms[DCDFT_KERNEL_COUNT] = {}, k_bytes[DCDFT_KERNEL_COUNT] = {},
         k_flops[DCDFT_KERNEL_COUNT] = {};

  // graphs of the three phases of one batched SCF step (captured on first use,
  // replayed after), one set per orbital buffer holding the current state
  hipGraph_t graph[2][3] = {};
  hipGraphExec_t graph_exec[2][3] = {};
  // State that a step overwrites in place, copied aside at the start of every step
  // and copied back when the step fails (densities, potentials, eigenpairs,
  // occupations, scalars, mixer history)
  struct Backup {
    void *live;
    void *save;
    size_t bytes;
  };
  std::vector<Backup> backups;
  // Scratch of the calls on caller-provided vectors (apply_h, band_energy):
  // single-fragment layout tables, H psi of one chunk of vectors, per-band terms
  struct ExtScratch {
    int *m = nullptr;             // [F]
    long long *moff = nullptr;    // [F + 1]
    int *band = nullptr;          // [chunk]
    void *hp = nullptr;           // [chunk][n] of double or float
    double *eb = nullptr;         // [chunk]
    int chunk = 0;                // vectors per chunk (<= m_pad)
  };
  ExtScratch ext;
  std::vector<int> ext_h_m;           // host copies of the layout tables (launch ranges)
  std::vector<long long> ext_h_moff;  // [F + 1] in launch order
  // phase boundaries of a step: start, V_eff formed, fragment eigensolvers
  // joined, end (recorded between the phases' graph launches)
  hipEvent_t ev_ph[4] = {nullptr, nullptr, nullptr, nullptr};
  bool use_graph = true;
  double template_xi = 0.0;    // xi of the density-template potential; 0: off
  int mix_kind = DCDFT_MIX_LINEAR;
  dcdft::MixState mix;
  // DC-LCFO post-processing (built on request; FP64 arrays in the orbital layout)
  double *d_lcfo_lam = nullptr, *d_lcfo_hlam = nullptr;  // basis, H^alpha basis [M_tot + m_pad][n]
  double *d_lcfo_sig = nullptr, *d_lcfo_w = nullptr;  // overlap eigenvalues, core weights [M_tot]
  int *d_lcfo_k = nullptr, *d_lcfo_nb = nullptr;      // selected orbitals, basis size [F]
  int *d_lcfo_pairs = nullptr;                        // [P][8] neighbour pairs
  int2 *d_lcfo_axes = nullptr;                        // per-axis overlap coordinates
  double *d_lcfo_x = nullptr;                         // [P][m_pad][m_pad] cross products
  int lcfo_pairs = -1;                                // -1: tables not built
  std::vector<int> lcfo_nb;                           // basis functions per fragment
  std::vector<double> lcfo_same;                      // [F][m_pad][m_pad] same-fragment blocks
  std::vector<double> lcfo_cross;                     // [P][m_pad][m_pad] neighbour products
  std::vector<int> lcfo_pair_of;                      // [F][F] pair index of (a, b), -1: none
  bool lcfo_ready = false;
  bool fixed_density = false;  // rho^in frozen: no Poisson, V_eff or mixing update in the step
  // large-orbital path: one fragment with more than kMaxOrb orbitals; tiles is
  // then kMaxTiles (the chunk of the stencil and projector launches) and m_pad
  // the padded orbital count
  bool large = false;
  dcdft::LargeBlas *blas = nullptr;
  void *d_lpart = nullptr;           // Gram chunk products [(parts + 1)][m_pad][m_pad], orbital type
  void *d_lrot = nullptr;            // rotation matrix in the orbital type [m_pad][m_pad]
  int *d_linfo = nullptr;            // rocSOLVER info words [4]
  double *d_le = nullptr;            // eigensolver work [m_pad]
  int large_status = 0;              // first failed library call of the step (0: none)
  std::string large_error;

  dcdft::OrbSet orbset(int f0, int f1) const;
  dcdft::KBTables kb() const;
};

namespace dcdft {

// ---- launchers (all asynchronous on the given stream) -------------------------------------
// Orbital arrays are [M_tot][n] of T = double (FP64 path) or float (mixed path);
// small matrices, per-band scalars and fields are FP64.

// Y = (-1/2 L_FD + V_eff) X for every orbital of fragments [f0, f1); dot (if not
// null) receives dV <x_B, y_B> per band.  veffT is V_eff in the storage type
// (the FP32 rounding for float; may be null, which rules out the variants that
// read it).
// dot_part: kHlocZsMax x (bands of the launch) doubles of scratch for the
// z-segmented variants (null: those variants fall back when dot is wanted).
constexpr int kHlocZsMax = 3;
template <typename T>
void launch_hloc(const Geo &g, const OrbSet &o, int f0, int f1, const double *veff,
                 const T *veffT, const T *x, T *y, hipStream_t s, double *dot = nullptr,
                 int vbase = 0, double *dot_part = nullptr);
// C[f][a][i] = dV sum beta_a(l) X_i(l) (region partials in part)
template <typename T>
void launch_kb_project(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1,
                       const T *x, double *C, double *part, hipStream_t s);
// Y_i(l) += sum_a beta_a(l) E_a C[f][a][i]
template <typename T>
void launch_kb_apply(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1,
                     const double *C, T *y, hipStream_t s);
template <typename T>
void launch_init_orbitals(const Geo &g, const OrbSet &o, uint64_t seed, T *psi, hipStream_t s);
// band energy of nb bands: eb[B] = f_B <psi_B|H psi_B>, energy = sum eb (or
// energy += sum eb with accumulate; energy may be null), grad_psi = 2 f dV H psi
// (may be null)
template <typename T>
void launch_band_energy_terms(const Geo &g, int nb, const T *psi, const T *hpsi, const double *f,
                              double *eb, double *energy, int accumulate, T *grad_psi,
                              hipStream_t s);
// grad_v(l) = dV sum_B f_B psi_B(l)^2 over nb bands
// Per-band terms of the band energy with H psi given in hg (replaced in place by
// 2 f dV H psi when scale is set); energy = sum of the band terms in band order.
template <typename T>
void launch_band_terms_inplace(const Geo &g, int nb, const T *psi, T *hg, const double *f,
                               double *eb, double *energy, int scale, hipStream_t s);
// dE/dV_loc on the global grid [Ng] for bands in fragment order (moff, m).
template <typename T>
void launch_grad_v_all(const Geo &g, const long long *moff, const int *m, const T *psi,
                       const double *f, double *grad_v, hipStream_t s);
template <typename T>
void launch_grad_v(const Geo &g, int nb, const T *psi, const double *f, double *grad_v,
                   hipStream_t s);
// device layout tables of mm vectors of fragment frag alone (m [nf], moff [nf + 1],
// band_frag [mm])
void launch_single_layout(int nf, int frag, int mm, int *m, long long *moff, int *band_frag,
                          hipStream_t s);

// Gram partials of X^T Y (row form G_ij = sum_l X_i(l) Y_j(l)); X == Y is symmetric
template <typename T>
void launch_gram(const Geo &g, const OrbSet &o, int f0, int f1, int chunks, const T *x,
                 const T *y, double *part, hipStream_t s);
// P = beta P - G (in place over P), Gram partials of Psi^T P; beta_zero: beta is
// zero for every band (P_prev is not read)
template <typename T>
void launch_gram_direction(const Geo &g, const OrbSet &o, int f0, int f1, int chunks,
                           const T *psi, const T *gres, T *p, const double *beta, double *part,
                           hipStream_t s, bool beta_zero = false);
// Psi_out <- cs Psi + sn P (psi_out may be psi), W <- cs W + sn Q (in place),
// symmetric Gram partials of Psi_out; with part_m also the partials of the full
// product <Psi_out, W> (same layout), and then store_w = false leaves W unwritten
// (only its product is needed)
template <typename T>
void launch_gram_update(const Geo &g, const OrbSet &o, int f0, int f1, int chunks,
                        const T *psi, T *psi_out, const T *p, T *w, const T *q, const double *cs,
                        const double *sn, double *part, hipStream_t s, double *part_m = nullptr,
                        bool store_w = true);
// G = dV sum of chunk partials (sym: X == Y, lower tiles mirrored); Gs = sym(G) if
// not null; diag -> per-band (may be null)
void launch_gram_reduce(const Geo &g, const OrbSet &o, int f0, int f1, int chunks, int sym,
                        const double *part, double *G, double *Gs, double *diag, hipStream_t s);
// both reductions of a fused update: S (symmetric partials) and M (full)
void launch_gram_reduce_pair(const Geo &g, const OrbSet &o, int f0, int f1, int chunks,
                             const double *part_s, double *S, const double *part_m, double *M,
                             hipStream_t s);
// Fused rotations (per-band reductions go through dpart, one partial per
// rotation workgroup, then a band reduction).
int rot_wpf(const Geo &g);
// G = W - Hs Psi into gout, gamma = dV |G|^2; with gamma_prev also the
// Fletcher-Reeves beta = gamma / gamma_prev (0 when first), then gamma_prev = gamma
template <typename T>
void launch_rot_residual(const Geo &g, const OrbSet &o, int f0, int f1, const double *Hs,
                         const T *psi, const T *w, T *gout, double *dpart, double *gamma,
                         hipStream_t s, int first = 0, double *gamma_prev = nullptr,
                         double *beta = nullptr);
// P <- P - X^T Psi, nu = dV |P|^2, pw = dV <P, W>; with inv also inv = 1/sqrt(nu)
template <typename T>
void launch_rot_project_out(const Geo &g, const OrbSet &o, int f0, int f1, const double *X,
                            const T *psi, T *p, const T *w, double *dpart, double *nu,
                            double *pw, hipStream_t s, double *inv = nullptr);
// Psi <- Linv Psi and, if w is not null, W <- Linv W (Linv lower triangular)
template <typename T>
void launch_rot_cholesky(const Geo &g, const OrbSet &o, int f0, int f1, const double *Linv,
                         T *psi, T *w, hipStream_t s);
// Psi <- U^T Psi (Ritz vectors), wcore = dV sum_core psi^2
template <typename T>
void launch_rot_ritz(const Geo &g, const OrbSet &o, int f0, int f1, const double *U, T *psi,
                     double *dpart, double *wcore, hipStream_t s);

// cp[B] += sum_a E_a C[f][a][i]^2, then the 2x2 CG step: theta = atan2(-2 inv bp,
// inv^2 cp - a) / 2 -> cs = cos(theta), sn = inv sin(theta)
void launch_kb_quad_theta(const OrbSet &o, int f0, int f1, const KBTables &kb, const double *C,
                          double *cp, const double *a, const double *bp, const double *inv,
                          double *cs, double *sn, hipStream_t s);
// Psi <- Linv Psi', W <- Linv W' (in place) and G = W - Bm Psi' into gout, with
// gamma = dV |g|^2 (Bm = Hs Linv from launch_cholinv)
template <typename T>
void launch_rot_cholres(const Geo &g, const OrbSet &o, int f0, int f1, const double *Linv,
                        const double *Bm, T *psi, T *w, T *gout, double *dpart, double *gamma,
                        hipStream_t s, double *gamma_prev = nullptr, double *beta = nullptr);
// S -> Linv (row-major lower-triangular inverse of the Cholesky factor), FP64;
// with M = <Psi', W'> also Hs = sym(Linv M Linv^T), its diagonal and Bm = Hs Linv
void launch_cholinv(const OrbSet &o, int f0, int f1, const double *S, double *Linv, int *flags,
                    hipStream_t s, const double *M = nullptr, double *Hs = nullptr,
                    double *adiag = nullptr, double *Bm = nullptr);
// Hs -> U (eigenvectors as columns), eps (ascending), FP64 Jacobi
// C = L^-T U per fragment (one rotation by C of the arrays before
// re-orthonormalisation gives the Ritz vectors)
void launch_ritz_combine(const OrbSet &o, int f0, int f1, const double *Linv, const double *U,
                         double *C, hipStream_t s);
void launch_syev(const OrbSet &o, int f0, int f1, const double *Hs, double *U, double *eps,
                 int *flags, hipStream_t s);
// DC-LCFO: core projection of the first k_sel[f] orbitals of every fragment into
// FP64 arrays; basis coefficients from the overlap eigenpairs (nb[f] functions);
// products between a fragment's H lambda and its neighbours' lambda on the
// overlap of core b with box a
template <typename T>
void launch_lcfo_gather(const Geo &g, const OrbSet &o, const int *band_frag, const int *k_sel,
                        const T *psi, double *phi, hipStream_t s);
void launch_lcfo_coeffs(const OrbSet &o, const double *U, const double *sigma, double lambda_cut,
                        double *Cm, int *nb, hipStream_t s);
void launch_lcfo_cross(const Geo &g, const OrbSet &o, int n_pairs, const int *pairs,
                       const int2 *axes, const int *nb, const double *hlam, const double *lam,
                       double *X, hipStream_t s);
// global chemical potential, occupations, band energy, entropy (one workgroup)
void launch_fermi(const OrbSet &o, const double *eps, const double *w, double ne, double sigma,
                  double *occ, double *scal, int *flags, hipStream_t s);
// rho_alpha^out and the core scatter into rho_tot^out
template <typename T>
void launch_density(const Geo &g, const OrbSet &o, int f0, int f1, const T *psi,
                    const double *occ, double *rhof_out, double *rho_out, hipStream_t s);
// V_eff^alpha = V_loc + V_H (gathered) + V_xc(rho_alpha^in)
// (and, if veff32 is not null, its FP32 rounding)
void launch_veff(const Geo &g, int f0, int f1, const double *vloc, const double *vh,
                 const double *rhof_in, const double *rho_tot_in, double xi, double *veff,
                 float *veff32, hipStream_t s);
// Energy terms, residuals and mixing on the global grid; fragment mixing
void launch_global_terms(const Geo &g, double *rho_in, const double *rho_out, const double *vh,
                         double mixing, double *part, int n_part, double *scal, hipStream_t s,
                         double ne, double sigma);
void launch_frag_mix(const Geo &g, int nfrag, double *rhof_in, const double *rhof_out,
                     double mixing, hipStream_t s);
// Pulay-Kerker mixing of rho_in (with the paper's residual into scal) and of every
// fragment density (gathered total density plus the mixed deviation)
void launch_pulay_mix(const Geo &g, int nfrag, const MixState &m, const double *rho_out,
                      const double *rhof_out, double *rho_in, double *rhof_in, double ne,
                      double *const qf[3], double *const qi[3], double *const lam[3],
                      double *wa, double *wb, double *scal, hipStream_t s);
// Poisson: V_H from rho (exact FD solution, zero mean)
void launch_poisson(const Geo &g, const double *rho, double *vh, double *wa, double *wb,
                    double *const qf[3], double *const qi[3], double *const lam[3],
                    hipStream_t s);
void launch_fill(double *p, long long n, double v, hipStream_t s);

// ---- large-orbital path (one fragment, m > kMaxOrb): k_large.hip -------------------------
// Orbital arrays: m rows of n points; small matrices FP64 column-major with
// leading dimension ld >= m.  The int results are rocBLAS statuses (0: success).
LargeBlas *large_create(hipStream_t s, std::string *err);
void large_destroy(LargeBlas *b);
const char *large_status_string(int st);
int large_gram_parts(int n);
// out = dv X Y^T (out[i + j ld] = dv <x_i, y_j>): products over
// large_gram_parts(n) chunks of points into part ((parts + 1) ld^2 values of the
// orbital type), summed in FP64 in chunk order
int large_gram(LargeBlas *b, int n, int m, int ld, const double *x, const double *y, double dv,
               double *out, void *part, hipStream_t s);
int large_gram(LargeBlas *b, int n, int m, int ld, const float *x, const float *y, double dv,
               double *out, void *part, hipStream_t s);
// out_i = alpha sum_j R'_ij x_j + beta out_i with R' = R^T (trans_r false) or R
// (trans_r true); FP32 arrays use rt (ld^2 floats) for the rounded R
int large_rotate(LargeBlas *b, int n, int m, int ld, const double *x, const double *r,
                 bool trans_r, double alpha, double beta, double *out, double *rt, hipStream_t s);
int large_rotate(LargeBlas *b, int n, int m, int ld, const float *x, const double *r,
                 bool trans_r, double alpha, double beta, float *out, float *rt, hipStream_t s);
// s (S on entry) <- L^-1 with S = L L^T, strict upper part zeroed; info[0..1]
// device ints; FLAG_NOT_SPD raised when S is not positive definite (s is then
// the identity)
int large_chol_inverse(LargeBlas *b, int m, int ld, double *s, int *info, int *flags,
                       hipStream_t st);
// a (symmetric on entry) <- eigenvectors (columns, ascending eigenvalues in eps,
// each with its largest entry positive); e_work: m doubles; info: two device
// ints; FLAG_EIG on failure, FLAG_NAN (and the identity solved instead) for a
// non-finite or overflowing a
int large_eigh(LargeBlas *b, int m, int ld, double *a, double *eps, double *e_work, int *info,
               int *flags, hipStream_t st);
template <typename T>
void launch_large_row_dots(const Geo &g, int m, const T *x, const T *y, const T *z, double *oy,
                           double *oz, bool core, hipStream_t s);
template <typename T>
void launch_large_direction(const Geo &g, int m, const T *gbuf, const T *pprev, T *pout,
                            const double *gamma, const double *gamma_prev, bool first,
                            hipStream_t s);
void launch_large_theta(int m, int ld, const double *hs_full, const double *nu, const double *bb,
                        const double *cc, double *cs, double *sn, double *inv, hipStream_t s);
template <typename T>
void launch_large_band_update(const Geo &g, int m, const T *psi_in, T *psi_out, T *w, const T *p,
                              const T *q, const double *cs, const double *sn, const double *inv,
                              hipStream_t s);
void launch_large_sym(int m, int ld, const double *a, double *s_out, double *diag, hipStream_t s);
void launch_fill_int(int *p, long long n, int v, hipStream_t s);
void launch_nan_check(const double *p, long long n, int *flags, hipStream_t s);
void launch_convert(const double *a, float *b, long long n, hipStream_t s);
void launch_convert(const float *a, double *b, long long n, hipStream_t s);

}  // namespace dcdft
