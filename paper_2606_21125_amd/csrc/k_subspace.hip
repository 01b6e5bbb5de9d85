// Subspace kernels of the fragment eigensolver: Gram matrices and subspace
// rotations on MFMA (the dense contractions that dominate ground-state cost,
// Sec. 2.2), with FP64 or FP32 orbital arrays (template T) and FP64 results;
// the FP64 Cholesky factor inverse for re-orthonormalisation, the FP64 Jacobi
// eigensolver of the Rayleigh-Ritz step (Eq. (1) in the subspace), and the
// per-band CG scalar updates.
#include "device_common.h"

namespace dcdft {

namespace {

// Fused rotation: y = cz z + cm R^T x (and, with RF_TWO, y2 = cm R^T x2 with the
// same R), with optional per-band reductions of the stored values v over the
// workgroup's points: RF_DOT_SELF sums v^2, RF_DOT_W sums v * wdot, RF_CORE
// restricts both to core points; RF_Z says z is given; RF_TRI says R^T is lower
// triangular (y_j needs inputs i <= j only, so the products of input orbitals
// past an output tile are skipped).  R = M^T (trans 0) or M (trans 1) is staged
// in LDS once per workgroup, transposed and with the inputs of one matrix-core
// step side by side (kpos), so that the R values one lane feeds to the matrix
// cores for an output tile are contiguous; step s takes the input orbitals
// 4s .. 4s + 3, one per lane group; each wave
// handles NT tiles of 16 points and every output orbital, so y may alias x or
// z.  Per tile a wave issues the
// loads of the next tile's operand rows before its own matrix-core products
// (and the z / wdot rows of its own outputs), so one tile of loads is always in
// flight.  Loads are unconditional (indices clamped into the arrays, values
// masked after): a load under a branch makes the compiler drain every
// outstanding load where the paths merge.  The per-band sums of a tile are
// reduced over the 16 point lanes with row-local DPP moves and added into a
// per-wave LDS row by one lane, then the waves are added in order: one FP64
// partial per workgroup, dpart[(f * wpf + wg) * 2 * m_pad + k * m_pad + j],
// k = 0 (self), 1 (wdot).
enum { RF_DOT_SELF = 1, RF_DOT_W = 2, RF_CORE = 4, RF_TWO = 8, RF_Z = 32, RF_TRI = 64 };

// LDS column of input orbital i in a staged rotation matrix: matrix-core step s
// of lane group kk takes input i = 4 s + kk, and a lane's values for one output
// tile sit contiguously at kk * NS + s.
template <int NS>
__device__ inline int kpos(int i) { return (i & 3) * NS + (i >> 2); }

// n consecutive values from 16-byte aligned LDS
template <typename T, int N>
__device__ inline void lds_read_vec(const T *p, T *d) {
  static_assert((N * sizeof(T)) % 16 == 0, "whole 16-byte vectors");
  typedef T v16 __attribute__((ext_vector_type(16 / sizeof(T))));
  constexpr int V = 16 / sizeof(T);
#pragma unroll
  for (int q = 0; q < N / V; ++q) {
    const v16 v = reinterpret_cast<const v16 *>(p)[q];
#pragma unroll
    for (int i = 0; i < V; ++i) d[q * V + i] = v[i];
  }
}

template <int CTRL>
__device__ inline double dpp_double(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 16 lanes of a DPP row (rotate by 8, by 4, then quad swaps);
// every lane of the row gets a sum of all 16 values in a fixed order.
__device__ inline double row16_sum(double v) {
  v += dpp_double<0x128>(v);  // row_ror:8
  v += dpp_double<0x124>(v);  // row_ror:4
  v += dpp_double<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_double<0xB1>(v);   // quad_perm [1,0,3,2]
  return v;
}

template <typename T, int TM, int NT, int FL>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && TM < 5 ? 4 : 2, 8)))
k_rot_fused(Geo g, OrbSet o, int f0, int wpf, const double *__restrict__ M, int trans,
            const T *x, const T *z, double cz, double cm, T *y, const T *x2, T *y2,
            const T *wdot, double *__restrict__ dpart) {
  typedef Mfma<T> MM;
  constexpr int MP = 16 * TM;
  constexpr int NS = 4 * TM;                     // MFMA steps over the input orbitals
  constexpr int S2 = MP + 16 / (int)sizeof(T);   // row stride of R^T in LDS (16-byte rows)
  constexpr bool DOTS = (FL & (RF_DOT_SELF | RF_DOT_W)) != 0;
  constexpr int NARR = (FL & RF_TWO) ? 2 : 1;
  constexpr int NITEM = NT * NARR;
  static_assert(!(FL & RF_TWO) || !(FL & (RF_Z | RF_DOT_SELF | RF_DOT_W)),
                "the second array is rotated without z or reductions");
  __shared__ __attribute__((aligned(16))) T RtT[MP * S2];
  __shared__ double red[4][2][MP];
  const int f = o.perm[f0 + blockIdx.x / wpf];
  const int wg = blockIdx.x % wpf;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int mf = o.m[f], mp = o.m_pad;
  // 16-orbital tiles this fragment uses (wave-uniform); the rest are neither
  // loaded from memory nor multiplied
  const int tf = __builtin_amdgcn_readfirstlane((mf + 15) >> 4);
  const double *Mf = M + (long long)f * mp * mp;
  // R^T with output orbital j as the row: RtT[j][kpos(i)] = R[i][j]
  for (int e = threadIdx.x; e < MP * MP; e += blockDim.x) {
    const int i = e / MP, j = e % MP;
    double v = 0.0;
    if (i < mf && j < mf) v = trans ? Mf[j * mp + i] : Mf[i * mp + j];
    RtT[j * S2 + kpos<NS>(i)] = (T)v;
  }
  if (DOTS)
    for (int e = lane; e < 2 * MP; e += 64) red[wave][e / MP][e % MP] = 0.0;
  __syncthreads();
  const long long base = o.moff[f] * (long long)g.n;
  const int jl = lane & 15, kk = lane >> 4;
  const T tcm = (T)cm, tcz = (T)cz;
  // Tile u of wave w covers points (wg*NT*4 + u*4 + w)*16 .. +15: at each tile
  // step the four waves cover 64 consecutive points, so the two 16-point halves
  // of a 128-byte FP32 line are requested together (by neighbouring waves)
  // rather than one tile step apart.
  auto tile_p0 = [&](int u) { return ((wg * NT + u) * 4 + wave) * 16; };
  // Addresses split into a wave-uniform row part and one lane offset (rows up
  // to the padded count exist: the arrays carry m_pad spare rows).
  // Input orbital of MFMA step s in lane group kk: i = 4 s + kk (a lane's R
  // values for one output tile are contiguous in LDS: 16-byte reads).
  // operand rows i of item it at the lane's point:
  auto load_rows = [&](int it, T *bx) {
    const int u = it / NARR, arr = it % NARR;
    const int pc = tile_p0(u) + jl;
    const bool pin = pc < g.n;
    const int lo = kk * g.n + (pin ? pc : g.n - 1);
    const T *xs = (arr ? x2 : x) + base;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      // rows past the fragment's tiles repeat the first step's address (a cache
      // hit, no memory traffic); their values are masked
      const int sr = s < 4 * tf ? s : 0;
      const T v = (xs + (long long)(4 * sr) * g.n)[lo];
      bx[s] = (4 * s + kk < mf && pin) ? v : (T)0;
    }
  };
  T bx[NS];
  load_rows(0, bx);
  for (int it = 0; it < NITEM; ++it) {
    const int u = it / NARR, arr = it % NARR;
    const int p0 = tile_p0(u);
    if (p0 >= g.n) break;
    const int pc = p0 + jl;
    const bool pin = pc < g.n;
    const bool core = (FL & RF_CORE) ? is_core_point(g, pc) : true;
    // output rows j = jt*16 + row_u(rr) + row_l(kk) of this lane
    const int lo_out = MM::row_l(kk) * g.n + (pin ? pc : g.n - 1);
    T zv[TM][4], wv[TM][4];
    if (FL & RF_Z) {
#pragma unroll
      for (int jt = 0; jt < TM; ++jt)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          zv[jt][rr] = (z + base + (long long)((jt < tf ? jt : 0) * 16 + MM::row_u(rr)) * g.n)[lo_out];
    }
    if (FL & RF_DOT_W) {
#pragma unroll
      for (int jt = 0; jt < TM; ++jt)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          wv[jt][rr] = (wdot + base + (long long)((jt < tf ? jt : 0) * 16 + MM::row_u(rr)) * g.n)[lo_out];
    }
    T bn[NS];
    load_rows(it + 1 < NITEM ? it + 1 : it, bn);  // unconditional (see above)
    typename MM::acc_t acc[TM];
#pragma unroll
    for (int jt = 0; jt < TM; ++jt) acc[jt] = MM::zero();
#pragma unroll
    for (int jt = 0; jt < TM; ++jt) {
      if (jt >= tf) continue;
      T a[NS];
      lds_read_vec<T, NS>(RtT + (jt * 16 + jl) * S2 + kk * NS, a);
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if ((!(FL & RF_TRI) || s < 4 * jt + 4) && s < 4 * tf)
          acc[jt] = MM::mma(a[s], bx[s], acc[jt]);
      // keep later operand reads from being hoisted (register pressure)
      __builtin_amdgcn_sched_barrier(0);
    }
    T *ys = arr ? y2 : y;
#pragma unroll
    for (int jt = 0; jt < TM; ++jt)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int j = jt * 16 + MM::row(kk, rr);
        const bool ok = j < mf && pin;
        T v = tcm * acc[jt][rr];
        if (FL & RF_Z) v += tcz * zv[jt][rr];
        if (ok) (ys + base + (long long)(jt * 16 + MM::row_u(rr)) * g.n)[lo_out] = v;
        if (DOTS) {
          const bool use = ok && core;
          if (FL & RF_DOT_SELF) {
            const double d = row16_sum(use ? (double)v * (double)v : 0.0);
            if (jl == 0) red[wave][0][j] += d;
          }
          if (FL & RF_DOT_W) {
            const double d = row16_sum(use ? (double)v * (double)wv[jt][rr] : 0.0);
            if (jl == 0) red[wave][1][j] += d;
          }
        }
      }
#pragma unroll
    for (int s = 0; s < NS; ++s) bx[s] = bn[s];
  }
  if (DOTS) {
    __syncthreads();
    double *out = dpart + ((long long)f * wpf + wg) * 2 * mp;
    for (int e = threadIdx.x; e < 2 * MP; e += blockDim.x) {
      const int k = e / MP, j = e % MP;
      out[k * mp + j] = red[0][k][j] + red[1][k][j] + red[2][k][j] + red[3][k][j];
    }
  }
}

// Cholesky re-orthonormalisation fused with the next sweep's residual: from
// Psi' and W' (in place), Psi = L^-1 Psi', W = L^-1 W' and G = W - B Psi' with
// B = Hs L^-1 (so G = W - Hs Psi), with the per-band sums |g|^2 as one FP64
// partial per workgroup in dpart[(f * wpf + wg) * 2 * m_pad + j].  Same tiling,
// LDS layout and load pipeline as k_rot_fused, with both matrices staged.
template <typename T, int TM, int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_rot_cholres(Geo g, OrbSet o, int f0, int wpf, const double *__restrict__ Linv,
              const double *__restrict__ Bm, T *psi, T *w, T *gout,
              double *__restrict__ dpart) {
  typedef Mfma<T> MM;
  constexpr int MP = 16 * TM;
  constexpr int NS = 4 * TM;
  constexpr int S2 = MP + 16 / (int)sizeof(T);
  constexpr bool PF = sizeof(T) == 4;   // FP32: load the next tile during this one
  __shared__ __attribute__((aligned(16))) T R1[MP * S2];
  __shared__ __attribute__((aligned(16))) T R2[MP * S2];
  __shared__ double red[4][MP];
  const int f = o.perm[f0 + blockIdx.x / wpf];
  const int wg = blockIdx.x % wpf;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int mf = o.m[f], mp = o.m_pad;
  const int tf = __builtin_amdgcn_readfirstlane((mf + 15) >> 4);   // tiles in use
  const double *Lf = Linv + (long long)f * mp * mp, *Bf = Bm + (long long)f * mp * mp;
  for (int e = threadIdx.x; e < MP * MP; e += blockDim.x) {
    const int j = e / MP, i = e % MP;
    const bool in = i < mf && j < mf;
    R1[j * S2 + kpos<NS>(i)] = in ? (T)Lf[j * mp + i] : (T)0;
    R2[j * S2 + kpos<NS>(i)] = in ? (T)Bf[j * mp + i] : (T)0;
  }
  for (int e = lane; e < MP; e += 64) red[wave][e] = 0.0;
  __syncthreads();
  const long long base = o.moff[f] * (long long)g.n;
  const int jl = lane & 15, kk = lane >> 4;
  auto tile_p0 = [&](int u) { return ((wg * NT + u) * 4 + wave) * 16; };
  auto load_rows = [&](int u, const T *xs, T *bx) {
    const int pc = tile_p0(u) + jl;
    const bool pin = pc < g.n;
    const int lo = kk * g.n + (pin ? pc : g.n - 1);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int sr = s < 4 * tf ? s : 0;   // past the fragment's tiles: a cache hit
      const T v = (xs + base + (long long)(4 * sr) * g.n)[lo];
      bx[s] = (4 * s + kk < mf && pin) ? v : (T)0;
    }
  };
  T bx[NS], bw[NS];
  load_rows(0, psi, bx);
  load_rows(0, w, bw);
  for (int u = 0; u < NT; ++u) {
    const int p0 = tile_p0(u);
    if (p0 >= g.n) break;
    const int pc = p0 + jl;
    const bool pin = pc < g.n;
    const int lo_out = MM::row_l(kk) * g.n + (pin ? pc : g.n - 1);
    T bxn[PF ? NS : 1], bwn[PF ? NS : 1];
    if (PF) {
      load_rows(u + 1 < NT ? u + 1 : u, psi, bxn);
      load_rows(u + 1 < NT ? u + 1 : u, w, bwn);
    }
    typename MM::acc_t ap[TM], aw[TM], ab[TM];
#pragma unroll
    for (int jt = 0; jt < TM; ++jt) {
      ap[jt] = MM::zero();
      aw[jt] = MM::zero();
      ab[jt] = MM::zero();
      if (jt >= tf) continue;
      T a[NS];
      lds_read_vec<T, NS>(R1 + (jt * 16 + jl) * S2 + kk * NS, a);
      // L^-1 is lower triangular: inputs past the output tile contribute nothing
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s < 4 * jt + 4) {
          ap[jt] = MM::mma(a[s], bx[s], ap[jt]);
          aw[jt] = MM::mma(a[s], bw[s], aw[jt]);
        }
      __builtin_amdgcn_sched_barrier(0);
      lds_read_vec<T, NS>(R2 + (jt * 16 + jl) * S2 + kk * NS, a);
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s < 4 * tf) ab[jt] = MM::mma(a[s], bx[s], ab[jt]);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int jt = 0; jt < TM; ++jt)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int j = jt * 16 + MM::row(kk, rr);
        const bool ok = j < mf && pin;
        const long long ro = base + (long long)(jt * 16 + MM::row_u(rr)) * g.n;
        const T vg = aw[jt][rr] - ab[jt][rr];
        if (ok) {
          (psi + ro)[lo_out] = ap[jt][rr];
          (w + ro)[lo_out] = aw[jt][rr];
          (gout + ro)[lo_out] = vg;
        }
        const double d = row16_sum(ok ? (double)vg * (double)vg : 0.0);
        if (jl == 0) red[wave][j] += d;
      }
    if (PF) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        bx[s] = bxn[s];
        bw[s] = bwn[s];
      }
    } else if (u + 1 < NT) {
      load_rows(u + 1, psi, bx);
      load_rows(u + 1, w, bw);
    }
  }
  __syncthreads();
  double *out = dpart + ((long long)f * wpf + wg) * 2 * mp;
  for (int j = threadIdx.x; j < MP; j += blockDim.x)
    out[j] = red[0][j] + red[1][j] + red[2][j] + red[3][j];
}

// CG scalar steps of one band (every reduction is FP64):
// Fletcher-Reeves beta = gamma / gamma_prev (0 on the first sweep or a zero
// gamma_prev), the inverse norm of the search direction, and the exact
// minimiser theta = atan2(-2b, c - a) / 2 of the 2x2 Rayleigh quotient for the
// normalised direction p_hat = inv p (b = inv <p, w>, c = inv^2 <p, H p>),
// returned as cos(theta) and inv sin(theta).
__device__ inline double cg_beta_of(double gamma, double gamma_prev, int first) {
  return (first || !(gamma_prev > 0.0)) ? 0.0 : gamma / gamma_prev;
}
__device__ inline double cg_inv_of(double nu) { return (nu > 1e-300) ? 1.0 / sqrt(nu) : 0.0; }
__device__ inline void cg_theta_of(double a, double b, double c, double inv, double &cs,
                                   double &sn) {
  double th = 0.0;
  if (inv != 0.0) th = 0.5 * atan2(-2.0 * inv * b, inv * inv * c - a);
  cs = cos(th);
  sn = inv * sin(th);
}

// Tail applied to the first band sum: BT_BETA takes it as gamma (x0 = gamma_prev,
// updated; x1 = beta), BT_INV as nu (x0 = 1 / sqrt(nu)).
enum { BT_NONE = 0, BT_BETA = 1, BT_INV = 2 };

// out_k[B] = dV sum over the workgroup partials of band B (k = 0, 1; null skips):
// one wave per band, lanes over the partials, fixed-order wave sum; then the
// tail (see above).
__global__ void __launch_bounds__(256) k_band_reduce(Geo g, OrbSet o, long long b0, long long nb,
                                                     int wpf, const double *__restrict__ dpart,
                                                     double *__restrict__ out0,
                                                     double *__restrict__ out1, int tail,
                                                     int first, double *__restrict__ x0,
                                                     double *__restrict__ x1) {
  const long long t = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= nb) return;  // wave-uniform
  const long long B = b0 + t;
  const int f = o.band_frag[B];
  const int i = (int)(B - o.moff[f]);
  const int mp = o.m_pad;
  double s0 = 0.0, s1 = 0.0;
  for (int wg = lane; wg < wpf; wg += 64) {
    const double *pp = dpart + ((long long)f * wpf + wg) * 2 * mp;
    s0 += pp[i];
    if (out1) s1 += pp[mp + i];
  }
  s0 = wave_sum(s0);
  if (out1) s1 = wave_sum(s1);
  if (lane == 0) {
    const double v0 = g.dv * s0;
    if (out0) out0[B] = v0;
    if (out1) out1[B] = g.dv * s1;
    if (tail == BT_BETA) {
      x1[B] = cg_beta_of(v0, x0[B], first);
      x0[B] = v0;
    } else if (tail == BT_INV) {
      x0[B] = cg_inv_of(v0);
    }
  }
}

// Gram products.  Workgroup = (fragment, chunk of points).  Per step of KT = 32
// points the workgroup loads the operand rows cooperatively into LDS (rows
// padded by 16 bytes), and each wave accumulates its share of the output
// tiles.  The second operand can be built during the load:
//   GM_PLAIN:  Y given (SYM when X == Y: upper tiles only, one operand).
//   GM_DIR:    Y = P = beta P_prev - G, written over P_prev.
//   GM_UPDATE: X = Psi' = c Psi + s P, written to xo (which may be X itself), and
//              W' = c W + s Q, written in place; symmetric product of Psi'.
//   GM_UPDATE_M: as GM_UPDATE, and also the full product <Psi', W'> (into part2).
// Partials are written in FP64 (one per workgroup).
enum { GM_PLAIN = 0, GM_DIR = 1, GM_UPDATE = 2, GM_UPDATE_M = 3 };
constexpr int kGramKT = 32;
// LDS row stride: rows stay 16-byte aligned for vector reads, with a 16-byte skew
template <typename T>
constexpr int gram_ld() { return kGramKT + 16 / (int)sizeof(T); }


template <typename T>
struct Vec4Load;
template <>
struct Vec4Load<double> {
  __device__ static inline void load(const double *p, double *d) {
    const double2 a = *reinterpret_cast<const double2 *>(p);
    const double2 b = *reinterpret_cast<const double2 *>(p + 2);
    d[0] = a.x; d[1] = a.y; d[2] = b.x; d[3] = b.y;
  }
  __device__ static inline void store(double *p, const double *d) {
    *reinterpret_cast<double2 *>(p) = double2{d[0], d[1]};
    *reinterpret_cast<double2 *>(p + 2) = double2{d[2], d[3]};
  }
};
template <>
struct Vec4Load<float> {
  __device__ static inline void load(const float *p, float *d) {
    const float4 a = *reinterpret_cast<const float4 *>(p);
    d[0] = a.x; d[1] = a.y; d[2] = a.z; d[3] = a.w;
  }
  __device__ static inline void store(float *p, const float *d) {
    *reinterpret_cast<float4 *>(p) = float4{d[0], d[1], d[2], d[3]};
  }
};

template <typename T, int TM, int MODE, bool SYM, bool VEC>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(MODE == GM_UPDATE_M ? 3 : (sizeof(T) == 4 || TM < 5 ? 4 : 2), 8)))
k_gram3(Geo g, OrbSet o, int f0, int chunks, int kchunk, const T *x, T *xo, T *a1,
        const T *a2, T *a3, const T *a4, const double *__restrict__ c1, const double *__restrict__ c2,
        double *__restrict__ part, double *__restrict__ part2, int store_w) {
  typedef Mfma<T> MM;
  constexpr int MP = 16 * TM;
  constexpr bool UPM = MODE == GM_UPDATE_M;   // second (full) product X^T Y into part2
  constexpr int NTS = SYM ? TM * (TM + 1) / 2 : TM * TM;
  constexpr int NTILE = NTS + (UPM ? TM * TM : 0);
  constexpr int PER_WAVE = (NTILE + 3) / 4;
  // operand items of one step: MP rows x KT/4 runs of 4 points, over 256 threads
  constexpr int NI = (MP * (kGramKT / 4) + 255) / 256;
  // arrays read per item: PLAIN x (and y), DIR x, G, P_prev, UPDATE Psi, P, W, Q
  constexpr int NA = MODE == GM_PLAIN ? (SYM ? 1 : 2) : (MODE == GM_DIR ? 3 : 4);
  constexpr int LD = gram_ld<T>();
  __shared__ __attribute__((aligned(16))) T Xs[MP * LD];
  __shared__ __attribute__((aligned(16))) T Ys[SYM && !UPM ? 4 : MP * LD];
  const int f = o.perm[f0 + blockIdx.x / chunks];
  const int c = blockIdx.x % chunks;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int mf = o.m[f];
  const int mp = o.m_pad;
  // 16-orbital tiles this fragment uses (wave-uniform): rows past them are not
  // read from memory and their output tiles are not multiplied (they stay zero)
  const int tf = __builtin_amdgcn_readfirstlane((mf + 15) >> 4);
  const long long base = o.moff[f] * (long long)g.n;
  const int p_begin = c * kchunk;
  const int p_end = min(p_begin + kchunk, g.n);
  // tiles of this wave: the (wave + 4 k)-th output tile in row order (upper
  // triangle only when SYM), then (UPM) the tiles of X^T Y; fixed indexing
  // keeps the table in registers
  int tI[PER_WAVE], tJ[PER_WAVE], tW[PER_WAVE];
#pragma unroll
  for (int k = 0; k < PER_WAVE; ++k) {
    const int q = wave + 4 * k;
    tI[k] = -1;
    tJ[k] = -1;
    tW[k] = 0;
    int idx = 0;
#pragma unroll
    for (int ti = 0; ti < TM; ++ti)
#pragma unroll
      for (int tj = 0; tj < TM; ++tj) {
        if (SYM && ti > tj) continue;
        if (idx == q) {
          tI[k] = ti;
          tJ[k] = tj;
        }
        ++idx;
      }
    if (UPM)
#pragma unroll
      for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TM; ++tj) {
          if (idx == q) {
            tI[k] = ti;
            tJ[k] = tj;
            tW[k] = 1;
          }
          ++idx;
        }
  }
  // FP32 products: each step's 32-point sums leave the matrix cores in FP32 and
  // are added into FP64 accumulators (the chunk sum of up to thousands of
  // points would otherwise accumulate in FP32); FP64 products accumulate in the
  // matrix cores directly.
  constexpr bool ACC64 = sizeof(T) == 4;
  typename MM::acc_t acc[PER_WAVE];
  double acc64[ACC64 ? PER_WAVE : 1][4];
#pragma unroll
  for (int k = 0; k < PER_WAVE; ++k) acc[k] = MM::zero();
#pragma unroll
  for (int k = 0; k < (ACC64 ? PER_WAVE : 1); ++k)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) acc64[k][rr] = 0.0;
  const T *Yl = SYM ? Xs : Ys;
  // GM_DIR reads P_prev from a1 unless a3 is given (a3 = G when beta is zero
  // for every band: the read then hits the lines just loaded for G)
  auto src = [&](int a) -> const T * {
    return a == 0 ? x
                  : (a == 1 ? (MODE == GM_DIR ? a2 : a1)
                            : (a == 2 ? (MODE == GM_DIR ? (a3 ? a3 : a1) : a3) : a4));
  };
  // Raw operand values of one step, loaded a step ahead of their use.  Rows up
  // to MP exist in the arrays (m_pad spare rows at the end), points outside
  // the chunk are read at a clamped index; both are masked at commit.
  // (prefetch only while the raw values fit in 48 registers per lane)
  constexpr bool PF = NI * NA * 4 * sizeof(T) <= 192;
  T raw[NI][NA][4];
  auto load_item = [&](int k, int p0) {
    {
      const int it = threadIdx.x + 256 * k;
      const int row0 = it / (kGramKT / 4) < MP ? it / (kGramKT / 4) : MP - 1;
      // rows past the fragment's tiles repeat a row of the first tile (a cache
      // hit); their values are masked at commit
      const int row = row0 < 16 * tf ? row0 : (row0 & 15);
      const int p = p0 + (it % (kGramKT / 4)) * 4;
      const int lo = row * g.n;  // lane offset (fits: m_pad n < 2^31)
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const T *rp = src(a) + base;  // wave-uniform
        if (VEC) {
          Vec4Load<T>::load(rp + (lo + (p < p_end ? p : p_begin)), raw[k][a]);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) raw[k][a][t] = rp[lo + (p + t < p_end ? p + t : p_begin)];
        }
      }
    }
  };
  auto load_step = [&](int p0) {
#pragma unroll
    for (int k = 0; k < NI; ++k) load_item(k, p0);
  };
  if (PF) load_step(p_begin);
  for (int p0 = p_begin; p0 < p_end; p0 += kGramKT) {
    __syncthreads();  // the previous step's products are done with the LDS rows
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      if (!PF) load_item(k, p0);
      const int it = threadIdx.x + 256 * k;
      const int row = it / (kGramKT / 4);
      const int pq = (it % (kGramKT / 4)) * 4;
      const int p = p0 + pq;
      if (row >= MP) continue;
      const bool rin = row < mf;
      T xv[4], yv[4];
      if (MODE == GM_PLAIN) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          xv[t] = raw[k][0][t];
          yv[t] = SYM ? (T)0 : raw[k][NA - 1][t];
        }
      } else if (MODE == GM_DIR) {
        // P = beta P_prev - G (beta = 0: P = -G without reading P_prev's value)
        const T b = (T)c1[o.moff[f] + (rin ? row : 0)];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          xv[t] = raw[k][0][t];
          yv[t] = b != (T)0 ? b * raw[k][2][t] - raw[k][1][t] : -raw[k][1][t];
        }
      } else {
        const T cs = (T)c1[o.moff[f] + (rin ? row : 0)];
        const T sn = (T)c2[o.moff[f] + (rin ? row : 0)];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          xv[t] = cs * raw[k][0][t] + sn * raw[k][1][t];
          yv[t] = cs * raw[k][2][t] + sn * raw[k][3][t];
        }
      }
      if (MODE != GM_PLAIN && rin) {
        const long long ro = base + (long long)row * g.n;
        T *d0 = MODE == GM_DIR ? a1 : xo;
        const T *v0 = MODE == GM_DIR ? yv : xv;
        if (VEC && p + 3 < p_end) {
          Vec4Load<T>::store(d0 + ro + p, v0);
          if (MODE >= GM_UPDATE && store_w) Vec4Load<T>::store(a3 + ro + p, yv);
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (p + t < p_end) {
              d0[ro + p + t] = v0[t];
              if (MODE >= GM_UPDATE && store_w) a3[ro + p + t] = yv[t];
            }
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool ok = rin && p + t < p_end;
        Xs[row * LD + pq + t] = ok ? xv[t] : (T)0;
        if (!SYM || UPM) Ys[row * LD + pq + t] = ok ? yv[t] : (T)0;
      }
    }
    __syncthreads();
    // unconditional: past the chunk the point index is clamped inside load_step
    if (PF) load_step(p0 + kGramKT);
    // lane (r, kk) takes the step's points kk*KQ .. kk*KQ + KQ - 1 (any
    // assignment of points to the K slots gives the same sum up to rounding):
    // contiguous in LDS, so a tile's operands come in 16-byte reads
    const int r = lane & 15, kk = lane >> 4;
    constexpr int KQ = kGramKT / 4;
#pragma unroll
    for (int k = 0; k < PER_WAVE; ++k) {
      if (tI[k] < 0 || tI[k] >= tf || tJ[k] >= tf) continue;
      T av[KQ], bv[KQ];
      lds_read_vec<T, KQ>(Xs + (tI[k] * 16 + r) * LD + kk * KQ, av);
      lds_read_vec<T, KQ>((UPM && tW[k] ? Ys : Yl) + (tJ[k] * 16 + r) * LD + kk * KQ, bv);
      if (ACC64) acc[k] = MM::zero();
#pragma unroll
      for (int t = 0; t < KQ; ++t) acc[k] = MM::mma(av[t], bv[t], acc[k]);
      if (ACC64) {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) acc64[k][rr] += (double)acc[k][rr];
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  const long long po = (long long)blockIdx.x * mp * mp;   // (launch-local fragment, chunk)
#pragma unroll
  for (int k = 0; k < PER_WAVE; ++k) {
    if (tI[k] < 0) continue;
    double *out = (UPM && tW[k] ? part2 : part) + po;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int row = tI[k] * 16 + MM::row(lane >> 4, rr);
      const int col = tJ[k] * 16 + (lane & 15);
      out[row * mp + col] = ACC64 ? acc64[k][rr] : (double)acc[k][rr];
    }
  }
}

// G = dV sum over chunk partials, element-parallel; for symmetric products the
// tiles below the diagonal are taken from their mirror.
// A second product (part2 -> G2, not symmetric) may ride in the same launch:
// indices past the first product's total handle it.
__global__ void __launch_bounds__(256) k_gram_reduce2(Geo g, OrbSet o, int f0, int nf, int chunks,
                                                      int sym, const double *__restrict__ part,
                                                      double *__restrict__ G,
                                                      double *__restrict__ diag,
                                                      const double *__restrict__ part2,
                                                      double *__restrict__ G2) {
  const int mp = o.m_pad;
  const long long total = (long long)nf * mp * mp;
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) {
    if (!part2 || idx >= 2 * total) return;
    idx -= total;
    part = part2;
    G = G2;
    sym = 0;
    diag = nullptr;
  }
  const int fl = (int)(idx / (mp * mp));
  const int e = (int)(idx % (mp * mp));
  const int f = o.perm[f0 + fl];
  int i = e / mp, j = e % mp;
  const int mf = o.m[f];
  double s = 0.0;
  if (i < mf && j < mf) {
    int si = i, sj = j;
    if (sym && (i / 16) > (j / 16)) {
      si = j;
      sj = i;
    }
    const double *pf = part + (long long)fl * chunks * mp * mp + si * mp + sj;
    // eight partials in flight at a time, added in chunk order
    int q = 0;
    for (; q + 8 <= chunks; q += 8) {
      double v[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = pf[(long long)(q + t) * mp * mp];
#pragma unroll
      for (int t = 0; t < 8; ++t) s += v[t];
    }
    for (; q < chunks; ++q) s += pf[(long long)q * mp * mp];
  }
  const double v = g.dv * s;
  G[(long long)f * mp * mp + e] = v;
  if (diag && i == j && i < mf) diag[o.moff[f] + i] = v;
}

__global__ void __launch_bounds__(256) k_symmetrize(OrbSet o, int f0, int nf,
                                                    const double *__restrict__ G,
                                                    double *__restrict__ Gs) {
  const int mp = o.m_pad;
  const long long total = (long long)nf * mp * mp;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int f = o.perm[f0 + (int)(idx / (mp * mp))];
  const int e = (int)(idx % (mp * mp));
  const int i = e / mp, j = e % mp;
  const double *Gf = G + (long long)f * mp * mp;
  Gs[(long long)f * mp * mp + e] = 0.5 * (Gf[i * mp + j] + Gf[j * mp + i]);
}

// C = P Q (QT: C = P Q^T) for nt x nt tiles of 16 x 16 LDS matrices (row
// stride ld, entries past the fragment's size zero) on the FP64 matrix cores;
// wave w takes the 16-row bands w, w + 4, ... of C and hands every entry to
// out(row, column, value).
template <bool QT, typename F>
__device__ inline void lds_gemm_f64(const double *P, const double *Q, int ld, int nt, F out) {
  typedef Mfma<double> MM;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, kk = lane >> 4;
  for (int rt = wave; rt < nt; rt += (int)(blockDim.x >> 6)) {
    MM::acc_t acc[kMaxTiles];
#pragma unroll
    for (int ct = 0; ct < kMaxTiles; ++ct) acc[ct] = MM::zero();
    for (int k = 0; k < 16 * nt; k += 4) {
      const double a = P[(rt * 16 + r) * ld + k + kk];
#pragma unroll
      for (int ct = 0; ct < kMaxTiles; ++ct)
        if (ct < nt) {
          const double b = QT ? Q[(ct * 16 + r) * ld + k + kk] : Q[(k + kk) * ld + ct * 16 + r];
          acc[ct] = MM::mma(a, b, acc[ct]);
        }
    }
#pragma unroll
    for (int ct = 0; ct < kMaxTiles; ++ct)
      if (ct < nt)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) out(rt * 16 + MM::row(kk, rr), ct * 16 + r, acc[ct][rr]);
  }
}

// Cholesky S = L L^T and the rows of L^-1 (row-major, lower triangular), with
// the matrix in registers: thread (ty, tx) of a 16 x 16 grid holds the entries
// (ty + 16 a, tx + 16 b).  At elimination step k the owners of column k of S
// and of row k of L^-1 publish them to LDS (two buffers, one barrier a step),
// and every thread scales and applies them to its own entries; L^-1 comes from
// the same elimination applied to the identity.
// With M = <Psi', W'> (the raw Gram of the arrays before re-orthonormalisation)
// the kernel also forms, for Psi = L^-1 Psi' and W = L^-1 W',
//   Hs = sym(L^-1 M L^-T) = sym(<Psi, W>)  -> Hs (and its diagonal into adiag),
//   B  = Hs L^-1                          -> Bm,
// so that G = W - Hs Psi = L^-1 W' - B Psi' needs no second pass.
// NT: 16-row tiles of the padded size (register blocks per thread are NT x NT)
template <int NT>
__global__ void __launch_bounds__(256) k_cholinv(OrbSet o, int f0, const double *__restrict__ S,
                                                 double *__restrict__ Linv, int *flags,
                                                 const double *__restrict__ M,
                                                 double *__restrict__ Hs,
                                                 double *__restrict__ adiag,
                                                 double *__restrict__ Bm) {
  constexpr int MTS = 16 * NT;   // staging sized for the tile count
  __shared__ double colb[2][MTS], xrowb[2][MTS];
  __shared__ double B0[MTS * (MTS + 1)];
  __shared__ double B1[MTS * (MTS + 1)];
  __shared__ double B2[MTS * (MTS + 1)];
  __shared__ int bad;
  const int f = o.perm[f0 + blockIdx.x];
  const int mf = o.m[f], mp = o.m_pad;
  const double *Sf = S + (long long)f * mp * mp;
  double *Lf = Linv + (long long)f * mp * mp;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  if (threadIdx.x == 0) bad = 0;
  double a[NT][NT], x[NT][NT];
#pragma unroll
  for (int ai = 0; ai < NT; ++ai)
#pragma unroll
    for (int bj = 0; bj < NT; ++bj) {
      const int i = ty + 16 * ai, j = tx + 16 * bj;
      const bool in = i < mf && j < mf;
      a[ai][bj] = in ? 0.5 * (Sf[i * mp + j] + Sf[j * mp + i]) : 0.0;
      x[ai][bj] = (in && i == j) ? 1.0 : 0.0;
    }
#pragma unroll
  for (int kb = 0; kb < NT; ++kb) {
    if (kb * 16 >= mf) break;
    for (int kr = 0; kr < 16; ++kr) {
      const int k = kb * 16 + kr;
      if (k >= mf) break;
      const int buf = k & 1;
      if (tx == kr)
#pragma unroll
        for (int ai = 0; ai < NT; ++ai) colb[buf][ty + 16 * ai] = a[ai][kb];
      if (ty == kr)
#pragma unroll
        for (int bj = 0; bj < NT; ++bj) xrowb[buf][tx + 16 * bj] = x[kb][bj];
      __syncthreads();
      double d = colb[buf][k];
      if (!(d > 0.0)) {
        if (threadIdx.x == 0) bad = 1;
        d = 1.0;
      }
      const double rdk = rsqrt_f64(d);
      double li[NT], lj[NT], xk[NT];
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        li[q] = colb[buf][ty + 16 * q] * rdk;
        lj[q] = colb[buf][tx + 16 * q] * rdk;
        xk[q] = xrowb[buf][tx + 16 * q] * rdk;
      }
      // S_ij -= L_ik L_jk below and right of the pivot; row k of L^-1 is row k
      // of the running matrix divided by L_kk, and L_ik times it leaves the
      // rows below
#pragma unroll
      for (int ai = 0; ai < NT; ++ai)
#pragma unroll
        for (int bj = 0; bj < NT; ++bj) {
          const int i = ty + 16 * ai, j = tx + 16 * bj;
          if (i > k && j > k) a[ai][bj] -= li[ai] * lj[bj];
          if (j <= k) {
            if (i > k) x[ai][bj] -= li[ai] * xk[bj];
            else if (i == k) x[ai][bj] = xk[bj];
          }
        }
    }
  }
#pragma unroll
  for (int ai = 0; ai < NT; ++ai)
#pragma unroll
    for (int bj = 0; bj < NT; ++bj) {
      const int r = ty + 16 * ai, c = tx + 16 * bj;
      if (r < mp && c < mp) Lf[r * mp + c] = (r < mf && c < mf && r >= c) ? x[ai][bj] : 0.0;
    }
  __syncthreads();
  if (threadIdx.x == 0 && bad) atomicOr(flags, FLAG_NOT_SPD);
  if (!M) return;
  const double *Mf = M + (long long)f * mp * mp;
  double *Hf = Hs + (long long)f * mp * mp, *Bf = Bm + (long long)f * mp * mp;
  const int nt = (mf + 15) / 16, mt = 16 * nt;
  const int ld = mt + 1;
  // B0 = L^-1, B1 = M (zero past the fragment's size)
#pragma unroll
  for (int ai = 0; ai < NT; ++ai)
#pragma unroll
    for (int bj = 0; bj < NT; ++bj) {
      const int i = ty + 16 * ai, j = tx + 16 * bj;
      if (i < mt && j < mt) {
        const bool in = i < mf && j < mf;
        B0[i * ld + j] = in ? x[ai][bj] : 0.0;
        B1[i * ld + j] = in ? Mf[i * mp + j] : 0.0;
      }
    }
  __syncthreads();
  // B2 = T = L^-1 M
  lds_gemm_f64<false>(B0, B1, ld, nt, [&](int r, int c, double v) { B2[r * ld + c] = v; });
  __syncthreads();
  // B1 = T L^-T
  lds_gemm_f64<true>(B2, B0, ld, nt, [&](int r, int c, double v) { B1[r * ld + c] = v; });
  __syncthreads();
  // B2 = Hs = sym(B1)
#pragma unroll
  for (int ai = 0; ai < NT; ++ai)
#pragma unroll
    for (int bj = 0; bj < NT; ++bj) {
      const int i = ty + 16 * ai, j = tx + 16 * bj;
      if (i < mp && j < mp) {
        const bool in = i < mf && j < mf;
        const double h = in ? 0.5 * (B1[i * ld + j] + B1[j * ld + i]) : 0.0;
        if (i < mt && j < mt) B2[i * ld + j] = h;
        Hf[i * mp + j] = h;
        if (in && i == j) adiag[o.moff[f] + i] = h;
        if (i >= mt || j >= mt) Bf[i * mp + j] = 0.0;
      }
    }
  __syncthreads();
  // B = Hs L^-1
  lds_gemm_f64<false>(B2, B0, ld, nt, [&](int r, int c, double v) {
    if (r < mp && c < mp) Bf[r * mp + c] = (r < mf && c < mf) ? v : 0.0;
  });
}

// C = L^-T U for the closing rotation of the re-orthonormalisation and the
// Rayleigh-Ritz step together: with Psi = L^-1 Psi' the Ritz vectors are
// U^T Psi = (L^-T U)^T Psi', so one rotation of Psi' by C replaces two.  One
// workgroup per fragment, FP64 matrix cores; LDS sized for NT 16-orbital tiles.
template <int NT>
__global__ void __launch_bounds__(256) k_ritz_combine(OrbSet o, int f0,
                                                      const double *__restrict__ Linv,
                                                      const double *__restrict__ U,
                                                      double *__restrict__ C) {
  constexpr int MT = 16 * NT;
  __shared__ double P[MT * (MT + 1)];
  __shared__ double Q[MT * (MT + 1)];
  const int f = o.perm[f0 + blockIdx.x];
  const int mf = o.m[f], mp = o.m_pad;
  const int nt = (mf + 15) / 16, mt = 16 * nt, ld = mt + 1;
  const double *Lf = Linv + (long long)f * mp * mp, *Uf = U + (long long)f * mp * mp;
  double *Cf = C + (long long)f * mp * mp;
  // P = L^-T, Q = U (zero past the fragment's size)
  for (int e = threadIdx.x; e < mt * mt; e += blockDim.x) {
    const int i = e / mt, j = e % mt;
    const bool in = i < mf && j < mf;
    P[i * ld + j] = in ? Lf[j * mp + i] : 0.0;
    Q[i * ld + j] = in ? Uf[i * mp + j] : 0.0;
  }
  for (int e = threadIdx.x; e < mp * mp; e += blockDim.x) {
    const int i = e / mp, j = e % mp;
    if (i >= mt || j >= mt) Cf[e] = 0.0;
  }
  __syncthreads();
  lds_gemm_f64<false>(P, Q, ld, nt, [&](int r, int c, double v) {
    if (r < mp && c < mp) Cf[r * mp + c] = (r < mf && c < mf) ? v : 0.0;
  });
}

// Round-robin (circle) pairing: in round r of mm - 1, pair k.
__device__ inline void rr_pair(int mm, int r, int k, int &p, int &q) {
  if (k == 0) {
    p = mm - 1;
    q = r;
  } else {
    p = (r + k) % (mm - 1);
    q = (r - k + (mm - 1)) % (mm - 1);
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// Parallel cyclic Jacobi: each round rotates mm/2 disjoint (p, q) planes at once.
// A and V in LDS sized for NT 16-orbital tiles (launched per tile class, so that
// the workgroups of small fragments fit several to a compute unit).
template <int NT>
__global__ void __launch_bounds__(1024) k_syev(OrbSet o, int f0, const double *__restrict__ H,
                                              double *__restrict__ U, double *__restrict__ eps,
                                              int *flags) {
  constexpr int MT = 16 * NT;
  __shared__ double A[MT * (MT + 1)];
  __shared__ double V[MT * (MT + 1)];
  // rotations of two consecutive rounds: round r is applied while round r + 1's
  // angles are formed
  // (p, q) and (c, s) of each pair packed: one LDS read each
  __shared__ int2 pq_of[2][MT / 2 + 1];
  __shared__ double2 cs_of[2][MT / 2 + 1];
  __shared__ double red[32];
  __shared__ int rank_of[MT];
  const int f = o.perm[f0 + blockIdx.x];
  const int mf = o.m[f], mp = o.m_pad;
  const int ld = mf | 1;   // odd row stride: column walks hit distinct banks
  const double *Hf = H + (long long)f * mp * mp;
  // 32 x 32 thread grid (no runtime division in the index arithmetic)
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int i = ty; i < mf; i += 32)
    for (int j = tx; j < mf; j += 32) {
      A[i * ld + j] = 0.5 * (Hf[i * mp + j] + Hf[j * mp + i]);
      V[i * ld + j] = (i == j) ? 1.0 : 0.0;
    }
  const int mm = (mf % 2) ? mf + 1 : mf;   // an odd size gets one idle index
  const int npair = mm / 2;
  // rotation angles of round r from the current A into buffer b (first wave)
  auto angles = [&](int r, int b) {
    for (int k = threadIdx.x; k < npair; k += 64) {
      int p, q;
      rr_pair(mm, r, k, p, q);
      double c = 1.0, s = 0.0;
      if (q < mf) {
        const double apq = A[p * ld + q];
        if (apq != 0.0) {
          // t = sign(tau) / (|tau| + sqrt(1 + tau^2)), c = 1 / sqrt(1 + t^2), s = t c
          // (|tau| > 1e100: t = 1 / (2 tau), where 1 + tau^2 would overflow)
          const double tau = (A[q * ld + q] - A[p * ld + p]) * rcp_f64(2.0 * apq);
          const double x = fma(tau, tau, 1.0);
          const double t = fabs(tau) > 1e100
                               ? 0.5 * rcp_f64(tau)
                               : (tau >= 0.0 ? 1.0 : -1.0) * rcp_f64(fabs(tau) + x * rsqrt_f64(x));
          c = rsqrt_f64(fma(t, t, 1.0));
          s = t * c;
        }
      }
      pq_of[b][k] = make_int2(p, q);
      cs_of[b][k] = make_double2(c, s);
    }
  };
  bool converged = (mf <= 1);
  double prev_off = 1e300;
  for (int sweep = 0; sweep < 60 && !converged; ++sweep) {
    __syncthreads();
    // convergence: max |off-diagonal| against the largest diagonal magnitude
    double off = 0.0, dia = 0.0;
    for (int i = ty; i < mf; i += 32)
      for (int j = tx; j < mf; j += 32) {
        const double v = fabs(A[i * ld + j]);
        if (i == j) dia = fmax(dia, v);
        else off = fmax(off, v);
      }
    for (int s = 32; s > 0; s >>= 1) {
      off = fmax(off, __shfl_xor(off, s, 64));
      dia = fmax(dia, __shfl_xor(dia, s, 64));
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x >> 6] = off;
      red[16 + (threadIdx.x >> 6)] = dia;
    }
    __syncthreads();
    double offm = 0.0, diam = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      offm = fmax(offm, red[w]);
      diam = fmax(diam, red[16 + w]);
    }
    // converged at 1e-13 of the largest diagonal entry, or at the rounding floor
    // (no further halving once below 1e-11 of it)
    if (offm <= 1e-13 * diam || offm == 0.0 || (offm < 1e-11 * diam && offm > 0.5 * prev_off)) {
      converged = true;
      break;
    }
    prev_off = offm;
    if (threadIdx.x < 64) angles(0, 0);
    for (int r = 0; r < mm - 1; ++r) {
      const int b = r & 1;
      __syncthreads();
      // A <- J^T A J as 2x2 blocks (rows of pair k1, columns of pair k2: the
      // blocks are disjoint, so one pass with no intermediate barrier).  The idle
      // index of an odd size (q = mf) is neither read nor written.
      for (int k1 = ty; k1 < npair; k1 += 32)
      for (int k2 = tx; k2 < npair; k2 += 32) {
        const int2 pq1 = pq_of[b][k1], pq2 = pq_of[b][k2];
        const double2 cs1 = cs_of[b][k1], cs2 = cs_of[b][k2];
        const int p1 = pq1.x, q1 = pq1.y, p2 = pq2.x, q2 = pq2.y;
        const bool h1 = q1 < mf, h2 = q2 < mf;
        const double c1 = cs1.x, s1 = cs1.y, c2 = cs2.x, s2 = cs2.y;
        const double app = A[p1 * ld + p2];
        const double apq = h2 ? A[p1 * ld + q2] : 0.0;
        const double aqp = h1 ? A[q1 * ld + p2] : 0.0;
        const double aqq = (h1 && h2) ? A[q1 * ld + q2] : 0.0;
        // rows (pair k1), then columns (pair k2)
        const double rpp = c1 * app - s1 * aqp, rpq = c1 * apq - s1 * aqq;
        const double rqp = s1 * app + c1 * aqp, rqq = s1 * apq + c1 * aqq;
        A[p1 * ld + p2] = c2 * rpp - s2 * rpq;
        if (h2) A[p1 * ld + q2] = s2 * rpp + c2 * rpq;
        if (h1) A[q1 * ld + p2] = c2 * rqp - s2 * rqq;
        if (h1 && h2) A[q1 * ld + q2] = s2 * rqp + c2 * rqq;
      }
      __syncthreads();
      // the first wave forms the next round's angles from the updated A while
      // the other waves apply this round's rotations to V (V <- V J)
      if (threadIdx.x < 64) {
        if (r + 1 < mm - 1) angles(r + 1, b ^ 1);
      } else {
        for (int k = ty - 2; k < npair; k += 30)
        for (int i = tx; i < mf; i += 32) {
          const int2 pq = pq_of[b][k];
          const int p = pq.x, q = pq.y;
          if (q >= mf) continue;
          const double2 cq = cs_of[b][k];
          const double c = cq.x, s = cq.y;
          const double vp = V[i * ld + p], vq = V[i * ld + q];
          V[i * ld + p] = c * vp - s * vq;
          V[i * ld + q] = s * vp + c * vq;
        }
      }
    }
  }
  __syncthreads();
  // ascending order (ties by index), then canonical column signs
  for (int i = threadIdx.x; i < mf; i += blockDim.x) {
    const double ai = A[i * ld + i];
    int rk = 0;
    for (int j = 0; j < mf; ++j) {
      const double aj = A[j * ld + j];
      if (aj < ai || (aj == ai && j < i)) ++rk;
    }
    rank_of[i] = rk;
  }
  __syncthreads();
  double *Uf = U + (long long)f * mp * mp;
  for (int i = threadIdx.x; i < mf; i += blockDim.x) {
    const int col = rank_of[i];
    int best = 0;
    double bv = -1.0;
    for (int r = 0; r < mf; ++r) {
      const double v = fabs(V[r * ld + i]);
      if (v > bv) {
        bv = v;
        best = r;
      }
    }
    const double sg = V[best * ld + i] < 0.0 ? -1.0 : 1.0;
    for (int r = 0; r < mp; ++r) Uf[r * mp + col] = (r < mf) ? sg * V[r * ld + i] : 0.0;
    eps[o.moff[f] + col] = A[i * ld + i];
  }
  for (int e = threadIdx.x; e < mp * mp; e += blockDim.x) {
    const int c = e % mp;
    if (c >= mf) Uf[e] = 0.0;
  }
  if (threadIdx.x == 0 && !converged) atomicOr(flags, FLAG_EIG);
}

// cp[B] += sum_a E_a C[f][a][i]^2 (the projector part of <p, H p>): one wave
// per band, lanes over the fragment's atoms, fixed-order wave sum; then theta
// of the 2x2 problem from a, bp, cp and inv (cg_theta_of).
__global__ void __launch_bounds__(256) k_kb_quad_theta(long long b0, long long nb,
                                                       const int *__restrict__ band_frag,
                                                       const long long *__restrict__ moff,
                                                       const int *__restrict__ A, int A_max,
                                                       int m_pad, const double *__restrict__ E,
                                                       const double *__restrict__ C,
                                                       double *__restrict__ cp,
                                                       const double *__restrict__ a,
                                                       const double *__restrict__ bp,
                                                       const double *__restrict__ inv,
                                                       double *__restrict__ cs,
                                                       double *__restrict__ sn) {
  const long long t = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= nb) return;  // wave-uniform
  const long long B = b0 + t;
  const int f = band_frag[B];
  const int i = (int)(B - moff[f]);
  double s = 0.0;
  for (int a = lane; a < A[f]; a += 64) {
    const double v = C[((long long)f * A_max + a) * m_pad + i];
    s += E[(long long)f * A_max + a] * v * v;
  }
  s = wave_sum(s);
  if (lane == 0) {
    const double c = cp[B] + s;
    cp[B] = c;
    cg_theta_of(a[B], bp[B], c, inv[B], cs[B], sn[B]);
  }
}

template <typename T, int TM, int MODE, bool SYM>
void gram3_t(const Geo &g, const OrbSet &o, int f0, int f1, int chunks, int kchunk, const T *x,
             T *xo, T *a1, const T *a2, T *a3, const T *a4, const double *c1, const double *c2, double *part,
             double *part2, int store_w, hipStream_t s) {
  const dim3 grid((f1 - f0) * chunks), block(256);
  if ((g.n % 4) == 0)
    hipLaunchKernelGGL((k_gram3<T, TM, MODE, SYM, true>), grid, block, 0, s, g, o, f0, chunks,
                       kchunk, x, xo, a1, a2, a3, a4, c1, c2, part, part2, store_w);
  else
    hipLaunchKernelGGL((k_gram3<T, TM, MODE, SYM, false>), grid, block, 0, s, g, o, f0, chunks,
                       kchunk, x, xo, a1, a2, a3, a4, c1, c2, part, part2, store_w);
}

template <typename T, int MODE, bool SYM>
void gram3_tm(const Geo &g, const OrbSet &o, int f0, int f1, int chunks, const T *x, T *xo, T *a1,
              const T *a2, T *a3, const T *a4, const double *c1, const double *c2, double *part,
              hipStream_t s, double *part2 = nullptr, int store_w = 1) {
  if (f1 <= f0) return;
  int kc = (g.n + chunks - 1) / chunks;
  kc = ((kc + kGramKT - 1) / kGramKT) * kGramKT;
  switch (o.tiles) {
    case 1: gram3_t<T, 1, MODE, SYM>(g, o, f0, f1, chunks, kc, x, xo, a1, a2, a3, a4, c1, c2, part, part2, store_w, s); break;
    case 2: gram3_t<T, 2, MODE, SYM>(g, o, f0, f1, chunks, kc, x, xo, a1, a2, a3, a4, c1, c2, part, part2, store_w, s); break;
    case 3: gram3_t<T, 3, MODE, SYM>(g, o, f0, f1, chunks, kc, x, xo, a1, a2, a3, a4, c1, c2, part, part2, store_w, s); break;
    case 4: gram3_t<T, 4, MODE, SYM>(g, o, f0, f1, chunks, kc, x, xo, a1, a2, a3, a4, c1, c2, part, part2, store_w, s); break;
    default: gram3_t<T, 5, MODE, SYM>(g, o, f0, f1, chunks, kc, x, xo, a1, a2, a3, a4, c1, c2, part, part2, store_w, s); break;
  }
}

template <typename T, int FL>
void rot_fused_tm(const Geo &g, const OrbSet &o, int f0, int f1, int wpf, const double *M,
                  int trans, const T *x, const T *z, double cz, double cm, T *y, const T *x2,
                  T *y2, const T *wdot, double *dpart, hipStream_t s) {
  if (f1 <= f0) return;
  const dim3 grid((f1 - f0) * wpf), block(256);
#define DCDFT_ROT_NT(TMV, NT)                                                                  \
  hipLaunchKernelGGL((k_rot_fused<T, TMV, NT, FL>), grid, block, 0, s, g, o, f0, wpf, M, trans, \
                     x, z, cz, cm, y, x2, y2, wdot, dpart)
#define DCDFT_ROT(TMV)                                   \
  do {                                                   \
    if (g.rot_tiles == 2) DCDFT_ROT_NT(TMV, 2);          \
    else if (g.rot_tiles == 8) DCDFT_ROT_NT(TMV, 8);     \
    else DCDFT_ROT_NT(TMV, 4);                           \
  } while (0)
  switch (o.tiles) {
    case 1: DCDFT_ROT(1); break;
    case 2: DCDFT_ROT(2); break;
    case 3: DCDFT_ROT(3); break;
    case 4: DCDFT_ROT(4); break;
    default: DCDFT_ROT(5); break;
  }
#undef DCDFT_ROT
#undef DCDFT_ROT_NT
}

void band_reduce(const Geo &g, const OrbSet &o, int f0, int f1, int wpf, const double *dpart,
                 double *out0, double *out1, hipStream_t s, int tail = BT_NONE, int first = 0,
                 double *x0 = nullptr, double *x1 = nullptr) {
  const long long nb = o.nb(f0, f1);
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_band_reduce, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, s, g, o,
                     o.b0(f0), nb, wpf, dpart, out0, out1, tail, first, x0, x1);
}

}  // namespace

int rot_wpf(const Geo &g) {
  const int nt = (g.rot_tiles == 2 || g.rot_tiles == 8) ? g.rot_tiles : 4;
  const int per_wg = 4 * nt * 16;
  return (g.n + per_wg - 1) / per_wg;
}

template <typename T>
void launch_gram(const Geo &g, const OrbSet &o, int f0, int f1, int chunks, const T *x,
                 const T *y, double *part, hipStream_t s) {
  T *xx = const_cast<T *>(x), *yy = const_cast<T *>(y);
  if (x == y)
    gram3_tm<T, GM_PLAIN, true>(g, o, f0, f1, chunks, xx, xx, xx, nullptr, nullptr, nullptr,
                                nullptr, nullptr, part, s);
  else
    gram3_tm<T, GM_PLAIN, false>(g, o, f0, f1, chunks, xx, xx, yy, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, part, s);
}

template <typename T>
void launch_gram_direction(const Geo &g, const OrbSet &o, int f0, int f1, int chunks,
                           const T *psi, const T *gres, T *p, const double *beta, double *part,
                           hipStream_t s, bool beta_zero) {
  gram3_tm<T, GM_DIR, false>(g, o, f0, f1, chunks, psi, const_cast<T *>(psi), p, gres,
                             beta_zero ? const_cast<T *>(gres) : nullptr, nullptr, beta, nullptr,
                             part, s);
}

template <typename T>
void launch_gram_update(const Geo &g, const OrbSet &o, int f0, int f1, int chunks,
                        const T *psi, T *psi_out, const T *p, T *w, const T *q, const double *cs,
                        const double *sn, double *part, hipStream_t s, double *part_m,
                        bool store_w) {
  if (part_m)
    gram3_tm<T, GM_UPDATE_M, true>(g, o, f0, f1, chunks, psi, psi_out, const_cast<T *>(p),
                                   nullptr, w, q, cs, sn, part, s, part_m, store_w ? 1 : 0);
  else
    gram3_tm<T, GM_UPDATE, true>(g, o, f0, f1, chunks, psi, psi_out, const_cast<T *>(p), nullptr,
                                 w, q, cs, sn, part, s);
}

template <typename T>
void launch_rot_residual(const Geo &g, const OrbSet &o, int f0, int f1, const double *Hs,
                         const T *psi, const T *w, T *gout, double *dpart, double *gamma,
                         hipStream_t s, int first, double *gamma_prev, double *beta) {
  const int wpf = rot_wpf(g);
  rot_fused_tm<T, RF_DOT_SELF | RF_Z>(g, o, f0, f1, wpf, Hs, 0, psi, w, 1.0, -1.0, gout, nullptr,
                               nullptr, nullptr, dpart, s);
  band_reduce(g, o, f0, f1, wpf, dpart, gamma, nullptr, s, gamma_prev ? BT_BETA : BT_NONE, first,
              gamma_prev, beta);
}

template <typename T>
void launch_rot_project_out(const Geo &g, const OrbSet &o, int f0, int f1, const double *X,
                            const T *psi, T *p, const T *w, double *dpart, double *nu,
                            double *pw, hipStream_t s, double *inv) {
  const int wpf = rot_wpf(g);
  rot_fused_tm<T, RF_DOT_SELF | RF_DOT_W | RF_Z>(g, o, f0, f1, wpf, X, 0, psi, p, 1.0, -1.0, p,
                                                 nullptr,
                                          nullptr, w, dpart, s);
  band_reduce(g, o, f0, f1, wpf, dpart, nu, pw, s, inv ? BT_INV : BT_NONE, 0, inv);
}

template <typename T>
void launch_rot_cholesky(const Geo &g, const OrbSet &o, int f0, int f1, const double *Linv,
                         T *psi, T *w, hipStream_t s) {
  const int wpf = rot_wpf(g);
  if (w)
    rot_fused_tm<T, RF_TWO | RF_TRI>(g, o, f0, f1, wpf, Linv, 1, psi, nullptr, 0.0, 1.0, psi, w,
                                     w, nullptr, nullptr, s);
  else
    rot_fused_tm<T, RF_TRI>(g, o, f0, f1, wpf, Linv, 1, psi, nullptr, 0.0, 1.0, psi, nullptr,
                            nullptr, nullptr, nullptr, s);
}

template <typename T>
void launch_rot_cholres(const Geo &g, const OrbSet &o, int f0, int f1, const double *Linv,
                        const double *Bm, T *psi, T *w, T *gout, double *dpart, double *gamma,
                        hipStream_t s, double *gamma_prev, double *beta) {
  if (f1 <= f0) return;
  const int wpf = rot_wpf(g);
  const dim3 grid((f1 - f0) * wpf), block(256);
#define DCDFT_CR(TMV)                                                                         \
  do {                                                                                        \
    if (g.rot_tiles == 2)                                                                     \
      hipLaunchKernelGGL((k_rot_cholres<T, TMV, 2>), grid, block, 0, s, g, o, f0, wpf, Linv, Bm, \
                         psi, w, gout, dpart);                                                \
    else if (g.rot_tiles == 8)                                                                \
      hipLaunchKernelGGL((k_rot_cholres<T, TMV, 8>), grid, block, 0, s, g, o, f0, wpf, Linv, Bm, \
                         psi, w, gout, dpart);                                                \
    else                                                                                      \
      hipLaunchKernelGGL((k_rot_cholres<T, TMV, 4>), grid, block, 0, s, g, o, f0, wpf, Linv, Bm, \
                         psi, w, gout, dpart);                                                \
  } while (0)
  switch (o.tiles) {
    case 1: DCDFT_CR(1); break;
    case 2: DCDFT_CR(2); break;
    case 3: DCDFT_CR(3); break;
    case 4: DCDFT_CR(4); break;
    default: DCDFT_CR(5); break;
  }
#undef DCDFT_CR
  band_reduce(g, o, f0, f1, wpf, dpart, gamma, nullptr, s, gamma_prev ? BT_BETA : BT_NONE, 0,
              gamma_prev, beta);
}

template <typename T>
void launch_rot_ritz(const Geo &g, const OrbSet &o, int f0, int f1, const double *U, T *psi,
                     double *dpart, double *wcore, hipStream_t s) {
  const int wpf = rot_wpf(g);
  rot_fused_tm<T, RF_DOT_SELF | RF_CORE>(g, o, f0, f1, wpf, U, 0, psi, nullptr, 0.0, 1.0, psi,
                                         nullptr, nullptr, nullptr, dpart, s);
  band_reduce(g, o, f0, f1, wpf, dpart, wcore, nullptr, s);
}

#define DCDFT_INSTANTIATE(T)                                                                    \
  template void launch_gram<T>(const Geo &, const OrbSet &, int, int, int, const T *, const T *, \
                               double *, hipStream_t);                                        \
  template void launch_gram_direction<T>(const Geo &, const OrbSet &, int, int, int, const T *,  \
                                         const T *, T *, const double *, double *, hipStream_t,  \
                                         bool);                                                \
  template void launch_gram_update<T>(const Geo &, const OrbSet &, int, int, int, const T *, T *, \
                                      const T *, T *, const T *, const double *, const double *, \
                                      double *, hipStream_t, double *, bool);                 \
  template void launch_rot_residual<T>(const Geo &, const OrbSet &, int, int, const double *,    \
                                       const T *, const T *, T *, double *, double *,            \
                                       hipStream_t, int, double *, double *);                 \
  template void launch_rot_project_out<T>(const Geo &, const OrbSet &, int, int, const double *, \
                                          const T *, T *, const T *, double *, double *,         \
                                          double *, hipStream_t, double *);                     \
  template void launch_rot_cholesky<T>(const Geo &, const OrbSet &, int, int, const double *, T *, \
                                       T *, hipStream_t);                                       \
  template void launch_rot_ritz<T>(const Geo &, const OrbSet &, int, int, const double *, T *,   \
                                   double *, double *, hipStream_t);                          \
  template void launch_rot_cholres<T>(const Geo &, const OrbSet &, int, int, const double *,     \
                                      const double *, T *, T *, T *, double *, double *,         \
                                      hipStream_t, double *, double *);
DCDFT_INSTANTIATE(double)
DCDFT_INSTANTIATE(float)
#undef DCDFT_INSTANTIATE

void launch_gram_reduce(const Geo &g, const OrbSet &o, int f0, int f1, int chunks, int sym,
                        const double *part, double *G, double *Gs, double *diag, hipStream_t s) {
  if (f1 <= f0) return;
  const long long total = (long long)(f1 - f0) * o.m_pad * o.m_pad;
  const unsigned nb = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL(k_gram_reduce2, dim3(nb), dim3(256), 0, s, g, o, f0, f1 - f0, chunks, sym,
                     part, G, diag, (const double *)nullptr, (double *)nullptr);
  if (Gs) hipLaunchKernelGGL(k_symmetrize, dim3(nb), dim3(256), 0, s, o, f0, f1 - f0, G, Gs);
}

void launch_gram_reduce_pair(const Geo &g, const OrbSet &o, int f0, int f1, int chunks,
                             const double *part_s, double *S, const double *part_m, double *M,
                             hipStream_t s) {
  if (f1 <= f0) return;
  const long long total = (long long)(f1 - f0) * o.m_pad * o.m_pad;
  const unsigned nb = (unsigned)((2 * total + 255) / 256);
  hipLaunchKernelGGL(k_gram_reduce2, dim3(nb), dim3(256), 0, s, g, o, f0, f1 - f0, chunks, 1,
                     part_s, S, (double *)nullptr, part_m, M);
}

void launch_cholinv(const OrbSet &o, int f0, int f1, const double *S, double *Linv, int *flags,
                    hipStream_t s, const double *M, double *Hs, double *adiag, double *Bm) {
  if (f1 <= f0) return;
  switch (o.tiles) {
#define DCDFT_CHOLINV(NT)                                                                       \
  hipLaunchKernelGGL(k_cholinv<NT>, dim3(f1 - f0), dim3(256), 0, s, o, f0, S, Linv, flags, M, Hs, \
                     adiag, Bm);                                                                \
  break
    case 1: DCDFT_CHOLINV(1);
    case 2: DCDFT_CHOLINV(2);
    case 3: DCDFT_CHOLINV(3);
    case 4: DCDFT_CHOLINV(4);
    default: DCDFT_CHOLINV(5);
#undef DCDFT_CHOLINV
  }
}

void launch_ritz_combine(const OrbSet &o, int f0, int f1, const double *Linv, const double *U,
                         double *C, hipStream_t s) {
  if (f1 <= f0) return;
  switch (o.tiles) {
#define DCDFT_RITZ(NT)                                                                          \
  hipLaunchKernelGGL(k_ritz_combine<NT>, dim3(f1 - f0), dim3(256), 0, s, o, f0, Linv, U, C);   \
  break
    case 1: DCDFT_RITZ(1);
    case 2: DCDFT_RITZ(2);
    case 3: DCDFT_RITZ(3);
    case 4: DCDFT_RITZ(4);
    default: DCDFT_RITZ(5);
#undef DCDFT_RITZ
  }
}

void launch_syev(const OrbSet &o, int f0, int f1, const double *Hs, double *U, double *eps,
                 int *flags, hipStream_t s) {
  if (f1 <= f0) return;
  switch (o.tiles) {
#define DCDFT_SYEV(NT)                                                                          \
  hipLaunchKernelGGL(k_syev<NT>, dim3(f1 - f0), dim3(1024), 0, s, o, f0, Hs, U, eps, flags);   \
  break
    case 1: DCDFT_SYEV(1);
    case 2: DCDFT_SYEV(2);
    case 3: DCDFT_SYEV(3);
    case 4: DCDFT_SYEV(4);
    default: DCDFT_SYEV(5);
#undef DCDFT_SYEV
  }
}

void launch_kb_quad_theta(const OrbSet &o, int f0, int f1, const KBTables &kb, const double *C,
                          double *cp, const double *a, const double *bp, const double *inv,
                          double *cs, double *sn, hipStream_t s) {
  const long long nb = o.nb(f0, f1);
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_kb_quad_theta, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, s, o.b0(f0),
                     nb, o.band_frag, o.moff, kb.A, kb.A_max, o.m_pad, kb.E, C, cp, a, bp, inv,
                     cs, sn);
}

}  // namespace dcdft
