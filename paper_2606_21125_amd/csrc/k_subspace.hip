// Subspace kernels of the fragment eigensolver: Gram matrices and subspace
// rotations on FP64 MFMA (the dense contractions that dominate ground-state
// cost, Sec. 2.2), the FP64 Cholesky factor inverse for re-orthonormalisation,
// the FP64 Jacobi eigensolver of the Rayleigh-Ritz step (Eq. (1) restricted to
// the subspace), and the per-band CG scalar updates.
#include "dcdft_internal.h"

namespace dcdft {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 lane layout on gfx950 (checked on the device):
//   A (16x4): lane l holds A[l % 16][l / 16]
//   B (4x16): lane l holds B[l / 16][l % 16]
//   D (16x16): lane l, register r holds D[l / 16 + 4 r][l % 16]
__device__ inline dbl4 mfma16x16x4(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// LDS row stride for an m_pad-wide operand block: the smallest S >= m_pad with
// S = 16 (mod 32), so the four 16-lane groups of an MFMA operand read land on
// different bank halves.
__host__ __device__ constexpr int lds_stride(int mp) { return mp + ((16 - mp % 32) + 32) % 32; }

// Gram partials, version 2.  Workgroup = (fragment, chunk of kchunk points); each
// of the 4 waves accumulates every output tile over a quarter of the chunk (the
// upper-triangle tiles only when X == Y), then the 4 wave results are summed in
// LDS and one partial per workgroup is written.  With VEC each lane fetches its 4
// consecutive points as two 16-byte loads (rows are 32-byte aligned when n % 4 == 0).
template <int TM, bool SYM, bool VEC>
__global__ void __launch_bounds__(256) k_gram2(Geo g, OrbSet o, int f0, int chunks, int kchunk,
                                               const double *__restrict__ x,
                                               const double *__restrict__ y,
                                               double *__restrict__ part) {
  __shared__ double red[kMaxOrb * kMaxOrb];
  const int f = f0 + blockIdx.x / chunks;
  const int c = blockIdx.x % chunks;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int mf = o.m[f];
  const int mp = o.m_pad;
  const long long base = o.moff[f] * (long long)g.n;
  const int sub = kchunk / 4;
  const int p_begin = c * kchunk + wave * sub;
  const int p_end = min(p_begin + sub, g.n);
  const int r = lane & 15, kk = lane >> 4;
  dbl4 acc[TM][TM];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int p0 = p_begin; p0 < p_end; p0 += 16) {
    double xa[TM][4], yb[TM][4];
    const int pl = p0 + 4 * kk;
#pragma unroll
    for (int ti = 0; ti < TM; ++ti) {
      const int row = ti * 16 + r;
      const bool rok = row < mf;
      const double *xr = x + base + (long long)row * g.n;
      const double *yr = y + base + (long long)row * g.n;
      if (VEC && rok && pl + 3 < p_end) {
        const double2 a0 = *reinterpret_cast<const double2 *>(xr + pl);
        const double2 a1 = *reinterpret_cast<const double2 *>(xr + pl + 2);
        xa[ti][0] = a0.x; xa[ti][1] = a0.y; xa[ti][2] = a1.x; xa[ti][3] = a1.y;
        if (!SYM) {
          const double2 b0 = *reinterpret_cast<const double2 *>(yr + pl);
          const double2 b1 = *reinterpret_cast<const double2 *>(yr + pl + 2);
          yb[ti][0] = b0.x; yb[ti][1] = b0.y; yb[ti][2] = b1.x; yb[ti][3] = b1.y;
        }
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const bool ok = rok && pl + t < p_end;
          xa[ti][t] = ok ? xr[pl + t] : 0.0;
          if (!SYM) yb[ti][t] = ok ? yr[pl + t] : 0.0;
        }
      }
      if (SYM) {
#pragma unroll
        for (int t = 0; t < 4; ++t) yb[ti][t] = xa[ti][t];
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TM; ++tj)
          if (!SYM || ti <= tj) acc[ti][tj] = mfma16x16x4(xa[ti][t], yb[tj][t], acc[ti][tj]);
  }
  // sum the four wave partials in LDS (fixed order: wave 0, 1, 2, 3)
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int ti = 0; ti < TM; ++ti)
#pragma unroll
        for (int tj = 0; tj < TM; ++tj) {
          if (SYM && ti > tj) continue;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int row = ti * 16 + (lane >> 4) + 4 * rr;
            const int col = tj * 16 + (lane & 15);
            const double v = acc[ti][tj][rr];
            red[row * mp + col] = (w == 0) ? v : red[row * mp + col] + v;
          }
        }
    }
    __syncthreads();
  }
  double *out = part + ((long long)(f - f0) * chunks + c) * mp * mp;
  for (int e = threadIdx.x; e < mp * mp; e += blockDim.x) {
    const int i = e / mp, j = e % mp;
    double v = 0.0;
    if (!SYM || (i / 16) <= (j / 16)) v = red[e];
    out[e] = v;
  }
}

// G = dV sum over chunk partials, element-parallel; for symmetric products the
// tiles below the diagonal are taken from their mirror.
__global__ void __launch_bounds__(256) k_gram_reduce2(Geo g, OrbSet o, int f0, int nf, int chunks,
                                                      int sym, const double *__restrict__ part,
                                                      double *__restrict__ G,
                                                      double *__restrict__ diag) {
  const int mp = o.m_pad;
  const long long total = (long long)nf * mp * mp;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int fl = (int)(idx / (mp * mp));
  const int e = (int)(idx % (mp * mp));
  const int f = f0 + fl;
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
    for (int q = 0; q < chunks; ++q) s += pf[(long long)q * mp * mp];
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
  const int f = f0 + (int)(idx / (mp * mp));
  const int e = (int)(idx % (mp * mp));
  const int i = e / mp, j = e % mp;
  const double *Gf = G + (long long)f * mp * mp;
  Gs[(long long)f * mp * mp + e] = 0.5 * (Gf[i * mp + j] + Gf[j * mp + i]);
}

// Rotation, version 2: R^T (as Rt[i][j] = R[j][i]) staged once per workgroup in
// LDS; each wave handles NT tiles of 16 points and all output orbitals; the
// X column of a tile (m_pad/4 doubles per lane) is fetched in one burst before
// its MFMA chain.  Y may alias X or Z (each wave reads its points fully first).
template <int TM, int NT>
__global__ void __launch_bounds__(256) k_rotate2(Geo g, OrbSet o, int f0, int wpf,
                                                 const double *__restrict__ M, int trans,
                                                 const double *x, const double *z, double cz,
                                                 double cm, double *y) {
  constexpr int MP = 16 * TM;
  constexpr int S = lds_stride(MP);
  __shared__ double Rt[MP * S];
  const int f = f0 + blockIdx.x / wpf;
  const int wg = blockIdx.x % wpf;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int mf = o.m[f], mp = o.m_pad;
  const double *Mf = M + (long long)f * mp * mp;
  for (int e = threadIdx.x; e < MP * MP; e += blockDim.x) {
    const int i = e / MP, j = e % MP;
    double v = 0.0;
    if (i < mf && j < mf) v = trans ? Mf[j * mp + i] : Mf[i * mp + j];
    Rt[i * S + j] = v;
  }
  __syncthreads();
  const long long base = o.moff[f] * (long long)g.n;
  const int jl = lane & 15, kk = lane >> 4;
  for (int u = 0; u < NT; ++u) {
    const int p0 = ((wg * 4 + wave) * NT + u) * 16;
    if (p0 >= g.n) break;
    const int pc = p0 + jl;
    const bool pin = pc < g.n;
    double bx[TM * 4];
#pragma unroll
    for (int s = 0; s < TM * 4; ++s) {
      const int i = 4 * s + kk;
      bx[s] = (i < mf && pin) ? x[base + (long long)i * g.n + pc] : 0.0;
    }
    dbl4 acc[TM];
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[j] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < TM * 4; ++s) {
      const double *rrow = Rt + (4 * s + kk) * S + jl;
#pragma unroll
      for (int jt = 0; jt < TM; ++jt) acc[jt] = mfma16x16x4(rrow[jt * 16], bx[s], acc[jt]);
    }
#pragma unroll
    for (int jt = 0; jt < TM; ++jt)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int j = jt * 16 + kk + 4 * rr;
        if (j < mf && pin) {
          const long long e = base + (long long)j * g.n + pc;
          double v = cm * acc[jt][rr];
          if (z) v += cz * z[e];
          y[e] = v;
        }
      }
  }
}

// Cholesky S = L L^T in LDS and the rows of L^-1 (row-major, lower triangular).
__global__ void __launch_bounds__(256) k_cholinv(OrbSet o, int f0, const double *__restrict__ S,
                                                 double *__restrict__ Linv, int *flags) {
  __shared__ double A[kMaxOrb * (kMaxOrb + 1)];
  __shared__ double X[kMaxOrb * (kMaxOrb + 1)];
  __shared__ int bad;
  const int f = f0 + blockIdx.x;
  const int mf = o.m[f], mp = o.m_pad;
  const int ld = mf + 1;   // odd row stride: column walks hit distinct banks
  const double *Sf = S + (long long)f * mp * mp;
  double *Lf = Linv + (long long)f * mp * mp;
  if (threadIdx.x == 0) bad = 0;
  for (int e = threadIdx.x; e < mf * mf; e += blockDim.x)
    A[(e / mf) * ld + e % mf] = 0.5 * (Sf[(e / mf) * mp + e % mf] + Sf[(e % mf) * mp + e / mf]);
  for (int k = 0; k < mf; ++k) {
    __syncthreads();
    if (threadIdx.x == 0) {
      double d = A[k * ld + k];
      if (!(d > 0.0)) {
        bad = 1;
        d = 1.0;
      }
      A[k * ld + k] = sqrt(d);
    }
    __syncthreads();
    const double dk = A[k * ld + k];
    for (int i = k + 1 + threadIdx.x; i < mf; i += blockDim.x) A[i * ld + k] /= dk;
    __syncthreads();
    const int w = mf - k - 1;
    for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
      const int i = k + 1 + e / w, j = k + 1 + e % w;
      if (j <= i) A[i * ld + j] -= A[i * ld + k] * A[j * ld + k];
    }
  }
  __syncthreads();
  // column c of L^-1 by forward substitution in LDS, then stored as Lf[r][c]
  for (int c = threadIdx.x; c < mf; c += blockDim.x) {
    for (int r = c; r < mf; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int q = c; q < r; ++q) s -= A[r * ld + q] * X[q * ld + c];
      X[r * ld + c] = s / A[r * ld + r];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < mp * mp; e += blockDim.x) {
    const int r = e / mp, c = e % mp;
    Lf[e] = (r < mf && c < mf && r >= c) ? X[r * ld + c] : 0.0;
  }
  if (threadIdx.x == 0 && bad) atomicOr(flags, FLAG_NOT_SPD);
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
__global__ void __launch_bounds__(256) k_syev(OrbSet o, int f0, const double *__restrict__ H,
                                              double *__restrict__ U, double *__restrict__ eps,
                                              int *flags) {
  __shared__ double A[kMaxOrb * (kMaxOrb + 1)];
  __shared__ double V[kMaxOrb * (kMaxOrb + 1)];
  __shared__ double cs[kMaxOrb / 2 + 1], sn[kMaxOrb / 2 + 1];
  __shared__ int pp[kMaxOrb / 2 + 1], qq[kMaxOrb / 2 + 1];
  __shared__ double red[16];
  __shared__ int rank_of[kMaxOrb];
  const int f = f0 + blockIdx.x;
  const int mf = o.m[f], mp = o.m_pad;
  const int ld = mf + 1;   // odd row stride: column walks hit distinct banks
  const double *Hf = H + (long long)f * mp * mp;
  for (int e = threadIdx.x; e < mf * mf; e += blockDim.x) {
    const int i = e / mf, j = e % mf;
    A[i * ld + j] = 0.5 * (Hf[i * mp + j] + Hf[j * mp + i]);
    V[i * ld + j] = (i == j) ? 1.0 : 0.0;
  }
  const int mm = (mf % 2) ? mf + 1 : mf;   // an odd size gets one idle index
  const int npair = mm / 2;
  bool converged = (mf <= 1);
  for (int sweep = 0; sweep < 60 && !converged; ++sweep) {
    __syncthreads();
    // convergence: max |off-diagonal| against the largest diagonal magnitude
    double off = 0.0, dia = 0.0;
    for (int e = threadIdx.x; e < mf * mf; e += blockDim.x) {
      const int i = e / mf, j = e % mf;
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
      red[8 + (threadIdx.x >> 6)] = dia;
    }
    __syncthreads();
    double offm = 0.0, diam = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      offm = fmax(offm, red[w]);
      diam = fmax(diam, red[8 + w]);
    }
    if (offm <= 1e-14 * diam || offm == 0.0) {
      converged = true;
      break;
    }
    for (int r = 0; r < mm - 1; ++r) {
      __syncthreads();
      for (int k = threadIdx.x; k < npair; k += blockDim.x) {
        int p, q;
        rr_pair(mm, r, k, p, q);
        double c = 1.0, s = 0.0;
        if (q < mf) {
          const double apq = A[p * ld + q];
          if (apq != 0.0) {
            const double tau = (A[q * ld + q] - A[p * ld + p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pp[k] = p;
        qq[k] = q;
        cs[k] = c;
        sn[k] = s;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int e = threadIdx.x; e < npair * mf; e += blockDim.x) {
        const int k = e / mf, j = e % mf;
        const int p = pp[k], q = qq[k];
        if (q >= mf) continue;
        const double c = cs[k], s = sn[k];
        const double ap = A[p * ld + j], aq = A[q * ld + j];
        A[p * ld + j] = c * ap - s * aq;
        A[q * ld + j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int e = threadIdx.x; e < npair * mf; e += blockDim.x) {
        const int k = e / mf, i = e % mf;
        const int p = pp[k], q = qq[k];
        if (q >= mf) continue;
        const double c = cs[k], s = sn[k];
        const double ap = A[i * ld + p], aq = A[i * ld + q];
        A[i * ld + p] = c * ap - s * aq;
        A[i * ld + q] = s * ap + c * aq;
        const double vp = V[i * ld + p], vq = V[i * ld + q];
        V[i * ld + p] = c * vp - s * vq;
        V[i * ld + q] = s * vp + c * vq;
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

__global__ void k_cg_beta(long long b0, long long nb, int first, const double *__restrict__ gamma,
                          const double *__restrict__ gamma_prev, double *__restrict__ beta) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const long long B = b0 + i;
  const double gp = gamma_prev[B];
  beta[B] = (first || !(gp > 0.0)) ? 0.0 : gamma[B] / gp;
}

__global__ void k_cg_norm(long long b0, long long nb, const double *__restrict__ nu,
                          double *__restrict__ inv) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const long long B = b0 + i;
  const double v = nu[B];
  inv[B] = (v > 1e-300) ? 1.0 / sqrt(v) : 0.0;
}

// theta = atan2(-2b, c - a) / 2 with b, c taken for the normalised direction
__global__ void k_cg_theta(long long b0, long long nb, const double *__restrict__ a,
                           const double *__restrict__ b, const double *__restrict__ c,
                           const double *__restrict__ inv, double *__restrict__ cs,
                           double *__restrict__ sn) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const long long B = b0 + i;
  double th = 0.0;
  if (inv[B] != 0.0) th = 0.5 * atan2(-2.0 * b[B], c[B] - a[B]);
  cs[B] = cos(th);
  sn[B] = sin(th);
}

__global__ void k_copy(long long b0, long long nb, const double *__restrict__ src,
                       double *__restrict__ dst) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  dst[b0 + i] = src[b0 + i];
}

template <int TM>
void gram_t(const Geo &g, const OrbSet &o, int f0, int f1, int chunks, int kchunk,
            const double *x, const double *y, double *part, hipStream_t s) {
  const bool sym = (x == y);
  const bool vec = (g.n % 4) == 0;
  const dim3 grid((f1 - f0) * chunks), block(256);
  if (sym && vec)
    hipLaunchKernelGGL((k_gram2<TM, true, true>), grid, block, 0, s, g, o, f0, chunks, kchunk, x,
                       y, part);
  else if (sym)
    hipLaunchKernelGGL((k_gram2<TM, true, false>), grid, block, 0, s, g, o, f0, chunks, kchunk, x,
                       y, part);
  else if (vec)
    hipLaunchKernelGGL((k_gram2<TM, false, true>), grid, block, 0, s, g, o, f0, chunks, kchunk, x,
                       y, part);
  else
    hipLaunchKernelGGL((k_gram2<TM, false, false>), grid, block, 0, s, g, o, f0, chunks, kchunk,
                       x, y, part);
}

constexpr int kRotTiles = 4;   // 16-point tiles per wave in k_rotate2

template <int TM>
void rotate_t(const Geo &g, const OrbSet &o, int f0, int f1, const double *M, int trans,
              const double *x, const double *z, double cz, double cm, double *y, hipStream_t s) {
  const int per_wg = 4 * kRotTiles * 16;
  const int wpf = (g.n + per_wg - 1) / per_wg;
  hipLaunchKernelGGL((k_rotate2<TM, kRotTiles>), dim3((f1 - f0) * wpf), dim3(256), 0, s, g, o, f0,
                     wpf, M, trans, x, z, cz, cm, y);
}

}  // namespace

int gram_kchunk(const Geo &g, int chunks) {
  int k = (g.n + chunks - 1) / chunks;
  return ((k + 63) / 64) * 64;
}

void launch_gram(const Geo &g, const OrbSet &o, int f0, int f1, int chunks, const double *x,
                 const double *y, double *part, hipStream_t s) {
  if (f1 <= f0) return;
  const int kc = gram_kchunk(g, chunks);
  switch (o.tiles) {
    case 1: gram_t<1>(g, o, f0, f1, chunks, kc, x, y, part, s); break;
    case 2: gram_t<2>(g, o, f0, f1, chunks, kc, x, y, part, s); break;
    case 3: gram_t<3>(g, o, f0, f1, chunks, kc, x, y, part, s); break;
    case 4: gram_t<4>(g, o, f0, f1, chunks, kc, x, y, part, s); break;
    default: gram_t<5>(g, o, f0, f1, chunks, kc, x, y, part, s); break;
  }
}

void launch_gram_reduce(const Geo &g, const OrbSet &o, int f0, int f1, int chunks, int sym,
                        const double *part, double *G, double *Gs, double *diag, hipStream_t s) {
  if (f1 <= f0) return;
  const long long total = (long long)(f1 - f0) * o.m_pad * o.m_pad;
  const unsigned nb = (unsigned)((total + 255) / 256);
  hipLaunchKernelGGL(k_gram_reduce2, dim3(nb), dim3(256), 0, s, g, o, f0, f1 - f0, chunks, sym,
                     part, G, diag);
  if (Gs) hipLaunchKernelGGL(k_symmetrize, dim3(nb), dim3(256), 0, s, o, f0, f1 - f0, G, Gs);
}

void launch_rotate(const Geo &g, const OrbSet &o, int f0, int f1, const double *M, int trans,
                   const double *x, const double *z, double cz, double cm, double *y,
                   hipStream_t s) {
  if (f1 <= f0) return;
  switch (o.tiles) {
    case 1: rotate_t<1>(g, o, f0, f1, M, trans, x, z, cz, cm, y, s); break;
    case 2: rotate_t<2>(g, o, f0, f1, M, trans, x, z, cz, cm, y, s); break;
    case 3: rotate_t<3>(g, o, f0, f1, M, trans, x, z, cz, cm, y, s); break;
    case 4: rotate_t<4>(g, o, f0, f1, M, trans, x, z, cz, cm, y, s); break;
    default: rotate_t<5>(g, o, f0, f1, M, trans, x, z, cz, cm, y, s); break;
  }
}

void launch_cholinv(const OrbSet &o, int f0, int f1, const double *S, double *Linv, int *flags,
                    hipStream_t s) {
  if (f1 <= f0) return;
  hipLaunchKernelGGL(k_cholinv, dim3(f1 - f0), dim3(256), 0, s, o, f0, S, Linv, flags);
}

void launch_syev(const OrbSet &o, int f0, int f1, const double *Hs, double *U, double *eps,
                 int *flags, hipStream_t s) {
  if (f1 <= f0) return;
  hipLaunchKernelGGL(k_syev, dim3(f1 - f0), dim3(256), 0, s, o, f0, Hs, U, eps, flags);
}

void launch_cg_beta(const OrbSet &o, int f0, int f1, int first, const double *gamma,
                    const double *gamma_prev, double *beta, hipStream_t s) {
  const long long nb = o.nb(f0, f1);
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_cg_beta, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, o.b0(f0), nb,
                     first, gamma, gamma_prev, beta);
}

void launch_cg_norm(const OrbSet &o, int f0, int f1, const double *nu, double *inv,
                    hipStream_t s) {
  const long long nb = o.nb(f0, f1);
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_cg_norm, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, o.b0(f0), nb,
                     nu, inv);
}

void launch_cg_theta(const OrbSet &o, int f0, int f1, const double *a, const double *b,
                     const double *c, const double *inv, double *cs, double *sn, hipStream_t s) {
  const long long nb = o.nb(f0, f1);
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_cg_theta, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, o.b0(f0), nb,
                     a, b, c, inv, cs, sn);
}

void launch_copy_band(const OrbSet &o, int f0, int f1, const double *src, double *dst,
                      hipStream_t s) {
  const long long nb = o.nb(f0, f1);
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, o.b0(f0), nb,
                     src, dst);
}

}  // namespace dcdft
