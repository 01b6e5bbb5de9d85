// Orbital-array kernels: the local part of the fragment Hamiltonian (Eq. (5):
// nine-point FD kinetic operator, periodic on the fragment box, plus V_eff),
// the Kleinman-Bylander projection and application, per-band reductions and
// updates, and the initial-orbital generator.
#include "dcdft_internal.h"

namespace dcdft {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block sum (fixed shuffle tree, waves combined in index order).
__device__ inline double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += red[w];
  return t;
}

// One workgroup per orbital; thread (x, y) of the plane marches along z with a
// nine-plane register window; x/y neighbours come from the current plane in LDS.
__global__ void __launch_bounds__(1024) k_hloc(Geo g, const int *__restrict__ band_frag,
                                               long long b0, const double *__restrict__ veff,
                                               const double *__restrict__ x,
                                               double *__restrict__ y, double *__restrict__ dot) {
  extern __shared__ double lds[];
  __shared__ double red[16];
  double dacc = 0.0;
  const long long B = b0 + blockIdx.x;
  const int f = band_frag[B];
  const int nx = g.nl[0], ny = g.nl[1], nz = g.nl[2];
  const int plane = nx * ny;
  const int t = threadIdx.x;
  const int ix = t % nx, iy = t / nx;
  const double *xb = x + B * (long long)g.n;
  double *yb = y + B * (long long)g.n;
  const double *vb = veff + (long long)f * g.n;
  const double c0 = g.kc[0];
  const double *ax = g.kc + 1, *ay = g.kc + 5, *az = g.kc + 9;
  int ox[8], oy[8];
#pragma unroll
  for (int k = 1; k <= 4; ++k) {
    ox[2 * (k - 1)] = ((ix + k) % nx) + iy * nx;
    ox[2 * (k - 1) + 1] = ((ix - k) % nx + nx) % nx + iy * nx;
    oy[2 * (k - 1)] = ix + ((iy + k) % ny) * nx;
    oy[2 * (k - 1) + 1] = ix + (((iy - k) % ny + ny) % ny) * nx;
  }
  double win[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int zz = ((k - 4) % nz + nz) % nz;
    win[k] = xb[(long long)zz * plane + t];
  }
  // V_eff two planes ahead of use, so its load latency overlaps the stencil
  double v0 = vb[t], v1 = (nz > 1) ? vb[plane + t] : 0.0;
  for (int z = 0; z < nz; ++z) {
    double *pl = lds + (z & 1) * plane;
    pl[t] = win[4];
    __syncthreads();
    double acc = c0 * win[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      acc += ax[k] * (pl[ox[2 * k]] + pl[ox[2 * k + 1]]);
      acc += ay[k] * (pl[oy[2 * k]] + pl[oy[2 * k + 1]]);
      acc += az[k] * (win[5 + k] + win[3 - k]);
    }
    const long long e = (long long)z * plane + t;
    acc += v0 * win[4];
    yb[e] = acc;
    dacc += win[4] * acc;
    v0 = v1;
    if (z + 2 < nz) v1 = vb[e + 2 * plane];
#pragma unroll
    for (int k = 0; k < 8; ++k) win[k] = win[k + 1];
    const int zn = (z + 5) % nz;
    win[8] = xb[(long long)zn * plane + t];
  }
  if (dot) {
    dacc = block_sum(dacc, red);
    if (t == 0) dot[B] = g.dv * dacc;
  }
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 (gfx950 lane layout: A[l%16][l/16], B[l/16][l%16],
// D[l/16 + 4r][l%16]).
__device__ inline dbl4 mfma16x16x4(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Region partials of the projections: part[(f, region)][slot][i] =
// sum_{l in region} beta_slot(l) X_i(l), as MFMA products of the dense region
// block (slots x points) with the region's orbital columns.  Wave w takes the
// orbital tiles w, w + 4; the K index walks points as u*16 + 4 (lane/16) + t so
// that every lane reads 32 contiguous bytes of both operands.
template <int TM, int KT>
__global__ void __launch_bounds__(256) k_kb_project2(Geo g, OrbSet o, KBTables kb, int f0,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ part) {
  const int f = f0 + blockIdx.x / kb.NR;
  const int reg = blockIdx.x % kb.NR;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int mf = o.m[f];
  const int pbase = reg * kRegion;
  const long long base = o.moff[f] * (long long)g.n;
  const double *blk = kb.reg_beta + ((long long)f * kb.NR + reg) * kb.KS * kRegion;
  const int r = lane & 15, kk = lane >> 4;
  constexpr int JW = (TM + 3) / 4;   // orbital tiles per wave
  dbl4 acc[KT][JW];
#pragma unroll
  for (int a = 0; a < KT; ++a)
#pragma unroll
    for (int b = 0; b < JW; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int u = 0; u < kRegion / 16; ++u) {
    const int pu = pbase + u * 16 + 4 * kk;
    double bx[JW][4];
#pragma unroll
    for (int q = 0; q < JW; ++q) {
      const int jt = wave + 4 * q;
      const int orb = jt * 16 + r;
      const bool ok = jt < TM && orb < mf;
#pragma unroll
      for (int t = 0; t < 4; ++t)
        bx[q][t] = (ok && pu + t < g.n) ? x[base + (long long)orb * g.n + pu + t] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int st = 0; st < KT; ++st) {
        const double av = blk[(st * 16 + r) * kRegion + u * 16 + 4 * kk + t];
#pragma unroll
        for (int q = 0; q < JW; ++q) acc[st][q] = mfma16x16x4(av, bx[q][t], acc[st][q]);
      }
    }
  }
  double *out = part + ((long long)f * kb.NR + reg) * kb.KS * o.m_pad;
#pragma unroll
  for (int q = 0; q < JW; ++q) {
    const int jt = wave + 4 * q;
    if (jt >= TM) continue;
#pragma unroll
    for (int st = 0; st < KT; ++st)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int slot = st * 16 + kk + 4 * rr;
        const int orb = jt * 16 + r;
        out[slot * o.m_pad + orb] = acc[st][q][rr];
      }
  }
}

// C[f][a][i] = dV sum over the (region, slot) entries of atom a.
__global__ void __launch_bounds__(256) k_kb_reduce(Geo g, OrbSet o, KBTables kb, int f0, int nf,
                                                   const double *__restrict__ part,
                                                   double *__restrict__ C) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)nf * kb.A_max * o.m_pad;
  if (idx >= total) return;
  const int i = (int)(idx % o.m_pad);
  const long long fa = (long long)f0 * kb.A_max + idx / o.m_pad;
  const int f = (int)(fa / kb.A_max);
  double s = 0.0;
  for (long long e = kb.ar_ptr[fa]; e < kb.ar_ptr[fa + 1]; ++e) {
    const long long q = ((long long)f * kb.NR + kb.ar_reg[e]) * kb.KS + kb.ar_slot[e];
    s += part[q * o.m_pad + i];
  }
  C[fa * o.m_pad + i] = g.dv * s;
}

// Y_i(l) += sum_slot beta_slot(l) E_slot C[f][slot atom][i] per region, as MFMA
// products of (E C)^T (orbitals x slots, staged in LDS) with the dense region
// block (slots x points); wave w takes the 16-point tiles w, w + 4, ...
template <int TM, int KT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) k_kb_apply2(Geo g, OrbSet o, KBTables kb, int f0,
                                                   const double *__restrict__ C,
                                                   double *__restrict__ y) {
  constexpr int MP = 16 * TM;
  constexpr int LD = MP + ((16 - MP % 32) + 32) % 32;
  constexpr int KSM = 16 * KT;
  __shared__ double ec[KSM * LD];
  const int f = f0 + blockIdx.x / kb.NR;
  const int reg = blockIdx.x % kb.NR;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int mf = o.m[f];
  const int *ra = kb.reg_atom + ((long long)f * kb.NR + reg) * kb.KS;
  const double *Cf = C + (long long)f * kb.A_max * o.m_pad;
  const double *Ef = kb.E + (long long)f * kb.A_max;
  for (int e = threadIdx.x; e < KSM * MP; e += blockDim.x) {
    const int slot = e / MP, i = e % MP;
    const int a = (slot < kb.KS) ? ra[slot] : -1;
    ec[slot * LD + i] = (a >= 0 && i < mf) ? Ef[a] * Cf[(long long)a * o.m_pad + i] : 0.0;
  }
  __syncthreads();
  const double *blk = kb.reg_beta + ((long long)f * kb.NR + reg) * kb.KS * kRegion;
  const long long base = o.moff[f] * (long long)g.n;
  const int c = lane & 15, kk = lane >> 4;
  for (int u = wave; u < kRegion / 16; u += 4) {
    const int p = reg * kRegion + u * 16 + c;
    dbl4 acc[TM];
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[j] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < KT * 4; ++st) {
      const double bv = blk[(4 * st + kk) * kRegion + u * 16 + c];
#pragma unroll
      for (int jt = 0; jt < TM; ++jt)
        acc[jt] = mfma16x16x4(ec[(4 * st + kk) * LD + jt * 16 + c], bv, acc[jt]);
      if ((st & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    if (p < g.n) {
#pragma unroll
      for (int jt = 0; jt < TM; ++jt)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int orb = jt * 16 + kk + 4 * rr;
          if (orb < mf) y[base + (long long)orb * g.n + p] += acc[jt][rr];
        }
    }
  }
}

__device__ inline bool is_core(const Geo &g, int l) {
  const int lx = l % g.nl[0];
  const int ly = (l / g.nl[0]) % g.nl[1];
  const int lz = l / (g.nl[0] * g.nl[1]);
  return lx >= g.b[0] && lx < g.b[0] + g.nc[0] && ly >= g.b[1] && ly < g.b[1] + g.nc[1] &&
         lz >= g.b[2] && lz < g.b[2] + g.nc[2];
}

__global__ void __launch_bounds__(256) k_band_dot(Geo g, long long b0, const double *__restrict__ x,
                                                  const double *__restrict__ y, int core,
                                                  double *__restrict__ out) {
  __shared__ double red[16];
  const long long B = b0 + blockIdx.x;
  const double *xb = x + B * (long long)g.n;
  const double *yb = y + B * (long long)g.n;
  double acc = 0.0;
  if (core) {
    for (int l = threadIdx.x; l < g.n; l += blockDim.x)
      if (is_core(g, l)) acc += xb[l] * yb[l];
  } else {
    for (int l = threadIdx.x; l < g.n; l += blockDim.x) acc += xb[l] * yb[l];
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) out[B] = g.dv * acc;
}

__global__ void __launch_bounds__(256) k_band_axpby(Geo g, long long b0, long long nb,
                                                    const double *__restrict__ a, double a_const,
                                                    const double *__restrict__ b, double b_const,
                                                    const double *__restrict__ x,
                                                    double *__restrict__ y) {
  const long long total = nb * (long long)g.n;
  const long long base = b0 * (long long)g.n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long B = b0 + e / g.n;
    const double ca = a ? a[B] : a_const;
    const double cb = b ? b[B] : b_const;
    const double yv = (a || a_const != 0.0) ? ca * y[base + e] : 0.0;
    y[base + e] = yv + cb * x[base + e];
  }
}

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator.
__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) k_init_orbitals(Geo g, const int *__restrict__ band_frag,
                                                       const long long *__restrict__ moff,
                                                       long long M_tot, uint64_t seed,
                                                       double *__restrict__ psi) {
  const long long total = M_tot * (long long)g.n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long B = e / g.n;
    const uint64_t l = (uint64_t)(e % g.n);
    const int f = band_frag[B];
    const uint64_t i = (uint64_t)(B - moff[f]);
    const uint64_t key = ((uint64_t)f << 40) | (i << 24) | l;
    const uint64_t z = splitmix64(seed, key + 1);
    psi[e] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
  }
}

// E = sum_i f_i dV sum_l psi_i H psi_i (one block per band then host-side sum in a
// second pass), grad_psi = 2 f dV H psi, grad_v = dV sum f psi^2.
__global__ void __launch_bounds__(256) k_band_energy_terms(Geo g, const double *__restrict__ psi,
                                                           const double *__restrict__ hpsi,
                                                           const double *__restrict__ f,
                                                           double *__restrict__ eb,
                                                           double *__restrict__ grad_psi) {
  __shared__ double red[16];
  const long long B = blockIdx.x;
  const double *pb = psi + B * (long long)g.n;
  const double *hb = hpsi + B * (long long)g.n;
  double acc = 0.0;
  const double s = 2.0 * f[B] * g.dv;
  for (int l = threadIdx.x; l < g.n; l += blockDim.x) {
    acc += pb[l] * hb[l];
    if (grad_psi) grad_psi[B * (long long)g.n + l] = s * hb[l];
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) eb[B] = f[B] * g.dv * acc;
}

__global__ void __launch_bounds__(256) k_band_energy_sum(int nb, const double *__restrict__ eb,
                                                         double *__restrict__ energy) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += eb[i];
    energy[0] = s;
  }
}

__global__ void __launch_bounds__(256) k_grad_v(Geo g, int nb, const double *__restrict__ psi,
                                                const double *__restrict__ f,
                                                double *__restrict__ grad_v) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= g.n) return;
  double acc = 0.0;
  for (int i = 0; i < nb; ++i) {
    const double v = psi[(long long)i * g.n + l];
    acc += f[i] * v * v;
  }
  grad_v[l] = g.dv * acc;
}

inline int grid_for(long long n, int block) {
  long long b = (n + block - 1) / block;
  if (b > 65536 * 4) b = 65536 * 4;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

void launch_hloc(const Geo &g, const OrbSet &o, int f0, int f1, const double *veff,
                 const double *x, double *y, hipStream_t s, double *dot) {
  const long long nb = o.nb(f0, f1);
  if (nb <= 0) return;
  const int plane = g.nl[0] * g.nl[1];
  hipLaunchKernelGGL(k_hloc, dim3((unsigned)nb), dim3(plane), 2 * plane * sizeof(double), s, g,
                     o.band_frag, o.b0(f0), veff, x, y, dot);
}

template <int TM, int KT>
void kb_t(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1, const double *x,
          double *C, double *part, double *y, hipStream_t s) {
  const dim3 grid((f1 - f0) * kb.NR), block(256);
  if (x) {
    hipLaunchKernelGGL((k_kb_project2<TM, KT>), grid, block, 0, s, g, o, kb, f0, x, part);
    const long long total = (long long)(f1 - f0) * kb.A_max * o.m_pad;
    hipLaunchKernelGGL(k_kb_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g, o,
                       kb, f0, f1 - f0, part, C);
  } else {
    hipLaunchKernelGGL((k_kb_apply2<TM, KT>), grid, block, 0, s, g, o, kb, f0, C, y);
  }
}

template <int TM>
void kb_tm(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1, const double *x,
           double *C, double *part, double *y, hipStream_t s) {
  switch (kb.KS / 16) {
    case 1: kb_t<TM, 1>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 2: kb_t<TM, 2>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 3: kb_t<TM, 3>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 4: kb_t<TM, 4>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 5: kb_t<TM, 5>(g, o, kb, f0, f1, x, C, part, y, s); break;
    default: kb_t<TM, 6>(g, o, kb, f0, f1, x, C, part, y, s); break;
  }
}

void kb_dispatch(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1,
                 const double *x, double *C, double *part, double *y, hipStream_t s) {
  if (f1 <= f0) return;
  switch (o.tiles) {
    case 1: kb_tm<1>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 2: kb_tm<2>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 3: kb_tm<3>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 4: kb_tm<4>(g, o, kb, f0, f1, x, C, part, y, s); break;
    default: kb_tm<5>(g, o, kb, f0, f1, x, C, part, y, s); break;
  }
}

void launch_kb_project(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1,
                       const double *x, double *C, double *part, hipStream_t s) {
  kb_dispatch(g, o, kb, f0, f1, x, C, part, nullptr, s);
}

void launch_kb_apply(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1,
                     const double *C, double *y, hipStream_t s) {
  kb_dispatch(g, o, kb, f0, f1, nullptr, const_cast<double *>(C), nullptr, y, s);
}

void launch_band_dot(const Geo &g, const OrbSet &o, int f0, int f1, const double *x,
                     const double *y, int core, double *out, hipStream_t s) {
  const long long nb = o.nb(f0, f1);
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_band_dot, dim3((unsigned)nb), dim3(256), 0, s, g, o.b0(f0), x, y, core,
                     out);
}

void launch_band_axpby(const Geo &g, const OrbSet &o, int f0, int f1, const double *a,
                       double a_const, const double *b, double b_const, const double *x,
                       double *y, hipStream_t s) {
  const long long nb = o.nb(f0, f1);
  if (nb <= 0) return;
  const long long total = nb * g.n;
  hipLaunchKernelGGL(k_band_axpby, dim3(grid_for(total, 256)), dim3(256), 0, s, g, o.b0(f0), nb,
                     a, a_const, b, b_const, x, y);
}

void launch_init_orbitals(const Geo &g, const OrbSet &o, uint64_t seed, double *psi,
                          hipStream_t s) {
  const long long total = o.M_tot * g.n;
  hipLaunchKernelGGL(k_init_orbitals, dim3(grid_for(total, 256)), dim3(256), 0, s, g,
                     o.band_frag, o.moff, o.M_tot, seed, psi);
}

void launch_band_energy(const Geo &g, int nb, const double *psi, const double *hpsi,
                        const double *f, double *eb, double *energy, double *grad_psi,
                        double *grad_v, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_band_energy_terms, dim3(nb), dim3(256), 0, s, g, psi, hpsi, f, eb,
                     grad_psi);
  if (energy) hipLaunchKernelGGL(k_band_energy_sum, dim3(1), dim3(64), 0, s, nb, eb, energy);
  if (grad_v)
    hipLaunchKernelGGL(k_grad_v, dim3((g.n + 255) / 256), dim3(256), 0, s, g, nb, psi, f, grad_v);
}

}  // namespace dcdft
