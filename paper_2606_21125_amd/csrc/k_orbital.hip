// Orbital-array kernels: the local part of the fragment Hamiltonian (Eq. (5):
// nine-point FD kinetic operator, periodic on the fragment box, plus V_eff),
// the Kleinman-Bylander projection and application, the initial-orbital
// generator and the band-energy functional with its gradient.  Orbital arrays
// are FP64 or FP32 (template T); reductions accumulate in FP64.
#include <algorithm>
#include <type_traits>

#include "device_common.h"

namespace dcdft {

namespace {

// One workgroup per orbital; thread (x, y) of the plane marches along z with a
// nine-plane register window; x/y neighbours come from the current plane in LDS.
// V_eff of fragment f starts at veff + (f - vbase) n.  dot (if not null)
// receives dV <x, y> for the orbital.
template <typename T>
__global__ void __launch_bounds__(1024) k_hloc(Geo g, const int *__restrict__ band_frag,
                                               long long b0, int vbase,
                                               const double *__restrict__ veff,
                                               const T *__restrict__ x, T *__restrict__ y,
                                               double *__restrict__ dot) {
  extern __shared__ char lds_raw[];
  T *lds = reinterpret_cast<T *>(lds_raw);
  __shared__ double red[16];
  double dacc = 0.0;
  const long long B = b0 + xcd_ordered(blockIdx.x, gridDim.x);
  const int f = band_frag[B];
  const int nx = g.nl[0], ny = g.nl[1], nz = g.nl[2];
  const int plane = nx * ny;
  const int t = threadIdx.x;
  const int ix = t % nx, iy = t / nx;
  const T *xb = x + B * (long long)g.n;
  T *yb = y + B * (long long)g.n;
  const double *vb = veff + (long long)(f - vbase) * g.n;
  const T c0 = (T)g.kc[0];
  T ax[4], ay[4], az[4];
  int ox[8], oy[8];
#pragma unroll
  for (int k = 1; k <= 4; ++k) {
    ax[k - 1] = (T)g.kc[k];
    ay[k - 1] = (T)g.kc[4 + k];
    az[k - 1] = (T)g.kc[8 + k];
    ox[2 * (k - 1)] = ((ix + k) % nx) + iy * nx;
    ox[2 * (k - 1) + 1] = ((ix - k) % nx + nx) % nx + iy * nx;
    oy[2 * (k - 1)] = ix + ((iy + k) % ny) * nx;
    oy[2 * (k - 1) + 1] = ix + (((iy - k) % ny + ny) % ny) * nx;
  }
  T win[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int zz = ((k - 4) % nz + nz) % nz;
    win[k] = xb[(long long)zz * plane + t];
  }
  // V_eff two planes ahead of use
  double v0 = vb[t], v1 = (nz > 1) ? vb[plane + t] : 0.0;
  for (int z = 0; z < nz; ++z) {
    T *pl = lds + (z & 1) * plane;
    pl[t] = win[4];
    __syncthreads();
    T acc = c0 * win[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      acc += ax[k] * (pl[ox[2 * k]] + pl[ox[2 * k + 1]]);
      acc += ay[k] * (pl[oy[2 * k]] + pl[oy[2 * k + 1]]);
      acc += az[k] * (win[5 + k] + win[3 - k]);
    }
    const long long e = (long long)z * plane + t;
    acc += (T)v0 * win[4];
    yb[e] = acc;
    dacc += (double)win[4] * (double)acc;
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

// Same operator for boxes with nx, ny >= 4, built for memory-level
// parallelism: the plane sits in LDS with a four-point periodic halo on both
// axes (row stride SX = nx + 32, so consecutive rows continue the bank sequence
// of an unpadded plane), which turns every neighbour read into a fixed offset
// from one address; the planes entering the window are loaded a chunk of PD
// iterations ahead, so PD..2PD plane loads of a workgroup are in flight; and
// the four planes at each end of the periodic z range stay in registers, so
// every plane of the orbital is read from memory once.  NX > 0 fixes nx at
// compile time (immediate LDS offsets); NX = 0 takes it from the geometry.
template <typename T, int NX, int PD, bool HT>
__global__ void __launch_bounds__(1024) k_hloc_halo(Geo g, const int *__restrict__ band_frag,
                                                    long long b0, int vbase,
                                                    const double *__restrict__ veff,
                                                    const T *__restrict__ x, T *__restrict__ y,
                                                    double *__restrict__ dot) {
  extern __shared__ char lds_raw[];
  T *lds = reinterpret_cast<T *>(lds_raw);
  __shared__ double red[16];
  const long long B = b0 + xcd_ordered(blockIdx.x, gridDim.x);
  const int f = band_frag[B];
  const int nx = NX > 0 ? NX : g.nl[0];
  const int ny = g.nl[1], nz = g.nl[2];
  const int SX = nx + 32;
  const int plane = nx * ny;
  const int lplane = (ny + 8) * SX;
  const int t = threadIdx.x;
  const int ix = t % nx, iy = t / nx;
  const int tp = (iy + 4) * SX + ix + 4;
  // periodic copies this thread also writes: into the high halo (ix < 4) and
  // into the low halo (ix >= nx - 4), both when nx < 8; likewise along y
  const bool xh = ix < 4, xl = ix >= nx - 4, yh = iy < 4, yl = iy >= ny - 4;
  const T *xb = x + B * (long long)g.n;
  T *yb = y + B * (long long)g.n;
  const double *vb = veff + (long long)(f - vbase) * g.n;
  const T c0 = (T)g.kc[0];
  T ax[4], ay[4], az[4];
#pragma unroll
  for (int k = 1; k <= 4; ++k) {
    ax[k - 1] = (T)g.kc[k];
    ay[k - 1] = (T)g.kc[4 + k];
    az[k - 1] = (T)g.kc[8 + k];
  }
  // head = planes 0..3, tail = planes nz-4..nz-1 (nz >= 8), window = z-4..z+4
  T head[HT ? 4 : 1], tail[HT ? 4 : 1], win[9];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    win[k] = xb[(long long)(nz - 4 + k) * plane + t];
    win[4 + k] = xb[(long long)k * plane + t];
    if (HT) {
      head[k] = win[4 + k];
      tail[k] = win[k];
    }
  }
  win[8] = xb[4LL * plane + t];
  // Planes 5, 6, ... come through the prefetch chunks.  Every load below is
  // unconditional, with its plane index wrapped or clamped into the box: a
  // load on one side of a branch makes the compiler drain all outstanding
  // loads where the paths merge, which would undo the prefetch.
  auto chunk_plane = [&](int pz) {
    if (HT) return pz < nz - 4 ? pz : nz - 5;  // end planes come from registers
    pz = pz < nz ? pz : pz - nz;               // pz <= nz + 2 PD + 3 < 3 nz
    return pz < nz ? pz : pz - nz;
  };
  // V_eff goes through the same chunks (a load needed one iteration after it
  // was issued would make every older load wait too).
  auto v_plane = [&](int pz) { return pz < nz ? pz : nz - 1; };
  T nxt[PD];
  double vn[PD];
#pragma unroll
  for (int j = 0; j < PD; ++j) nxt[j] = xb[(long long)chunk_plane(5 + j) * plane + t];
#pragma unroll
  for (int j = 0; j < PD; ++j) vn[j] = vb[(long long)v_plane(j) * plane + t];
  double dacc = 0.0;
  for (int z0 = 0; z0 < nz; z0 += PD) {
    T fut[PD];
    double vfut[PD];
#pragma unroll
    for (int j = 0; j < PD; ++j)
      fut[j] = xb[(long long)chunk_plane(z0 + 5 + PD + j) * plane + t];
#pragma unroll
    for (int j = 0; j < PD; ++j) vfut[j] = vb[(long long)v_plane(z0 + PD + j) * plane + t];
#pragma unroll
    for (int j = 0; j < PD; ++j) {
      const int z = z0 + j;
      if (z >= nz) break;
      const double v0 = vn[j];
      T *pl = lds + (z & 1) * lplane;
      const T c = win[4];
      pl[tp] = c;
      if (xh) pl[tp + nx] = c;
      if (xl) pl[tp - nx] = c;
      if (yh) pl[tp + ny * SX] = c;
      if (yl) pl[tp - ny * SX] = c;
      __syncthreads();
      T acc = c0 * c;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        acc += ax[k] * (pl[tp + k + 1] + pl[tp - k - 1]);
        acc += ay[k] * (pl[tp + (k + 1) * SX] + pl[tp - (k + 1) * SX]);
        acc += az[k] * (win[5 + k] + win[3 - k]);
      }
      acc += (T)v0 * c;
      yb[(long long)z * plane + t] = acc;
      dacc += (double)c * (double)acc;
#pragma unroll
      for (int k = 0; k < 8; ++k) win[k] = win[k + 1];
      // plane z + 5 enters the window
      const int pz = z + 5;
      T w8 = nxt[j];
      if (HT && pz > nz - 5) {
        const int ht = pz >= nz ? pz - nz : pz - (nz - 4);
        const T *src = pz >= nz ? head : tail;
        w8 = ht == 0 ? src[0] : (ht == 1 ? src[1] : (ht == 2 ? src[2] : src[3]));
      }
      win[8] = w8;
    }
#pragma unroll
    for (int j = 0; j < PD; ++j) {
      nxt[j] = fut[j];
      vn[j] = vfut[j];
    }
  }
  if (dot) {
    dacc = block_sum(dacc, red);
    if (t == 0) dot[B] = g.dv * dacc;
  }
}

// Vector form of the haloed-plane kernel: each thread owns a run of
// RX = VB / sizeof(T) consecutive x points (one VB-byte load, store and LDS
// access per plane for the run; the x neighbours come from the two runs beside
// it), opw orbitals share a workgroup (tpo = nx / RX * ny threads each), and
// V_eff is read in the storage type (its FP32 rounding on the mixed path, which
// is what the FP32 product uses anyway).  Same sums in the same order as the
// other variants.  Needs nx % RX == 0, nx, ny >= 4, nz >= 8 and 16-byte
// aligned arrays.  Bands past the batch are computed as duplicates of the last
// band (identical values to identical addresses) so every load stays
// unconditional; only the per-band dot is masked.
template <typename T, int PD, int VB>
__global__ void __launch_bounds__(1024) k_hloc_vec(Geo g, const int *__restrict__ band_frag,
                                                   long long b0, long long nbands, int opw,
                                                   int zs, int vbase, const T *__restrict__ veff,
                                                   const T *__restrict__ x, T *__restrict__ y,
                                                   double *__restrict__ dot,
                                                   double *__restrict__ dot_part) {
  constexpr int RX = VB / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(RX)));
  extern __shared__ __attribute__((aligned(16))) char lds_vec[];
  const int nx = g.nl[0], ny = g.nl[1], nz = g.nl[2];
  const int bx = nx / RX, tpo = bx * ny;
  const int SX = nx + 32, lplane = (ny + 8) * SX;  // rows continue the bank sequence
  const int ol = threadIdx.x / tpo, tt = threadIdx.x % tpo;
  // z segments of one orbital group are consecutive work items
  const unsigned wi = xcd_ordered(blockIdx.x, gridDim.x);
  const int seg = wi % zs;
  const int zlen = (nz + zs - 1) / zs;
  const int zb = seg * zlen, ze = zb + zlen < nz ? zb + zlen : nz;
  long long B = b0 + (long long)(wi / zs) * opw + ol;
  const bool valid = B < b0 + nbands;
  if (!valid) B = b0 + nbands - 1;
  const int f = band_frag[B];
  const int ix = (tt % bx) * RX, iy = tt / bx;
  T *lds = reinterpret_cast<T *>(lds_vec) + (size_t)ol * 2 * lplane;
  const int tp = (iy + 4) * SX + ix + 4;
  const int pvec = bx * ny;  // vectors per plane
  const vec *xb = reinterpret_cast<const vec *>(x + B * (long long)g.n) + tt;
  vec *yb = reinterpret_cast<vec *>(y + B * (long long)g.n) + tt;
  const vec *vb = reinterpret_cast<const vec *>(veff + (long long)(f - vbase) * g.n) + tt;
  const bool xh = ix < 4, xl = ix >= nx - 4, yh = iy < 4, yl = iy >= ny - 4;
  const T c0 = (T)g.kc[0];
  T ax[4], ay[4], az[4];
#pragma unroll
  for (int k = 1; k <= 4; ++k) {
    ax[k - 1] = (T)g.kc[k];
    ay[k - 1] = (T)g.kc[4 + k];
    az[k - 1] = (T)g.kc[8 + k];
  }
  auto wrap = [&](int pz) {  // pz < 3 nz
    pz = pz < nz ? pz : pz - nz;
    return pz < nz ? pz : pz - nz;
  };
  auto clampz = [&](int pz) { return pz < nz ? pz : nz - 1; };
  vec win[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) win[k] = xb[(long long)wrap(zb + nz - 4 + k) * pvec];
  vec nxt[PD], vn[PD];
#pragma unroll
  for (int j = 0; j < PD; ++j) nxt[j] = xb[(long long)wrap(zb + 5 + j) * pvec];
#pragma unroll
  for (int j = 0; j < PD; ++j) vn[j] = vb[(long long)clampz(zb + j) * pvec];
  double dacc = 0.0;
  for (int z0 = zb; z0 < ze; z0 += PD) {
    vec fut[PD], vfut[PD];
#pragma unroll
    for (int j = 0; j < PD; ++j) fut[j] = xb[(long long)wrap(z0 + 5 + PD + j) * pvec];
#pragma unroll
    for (int j = 0; j < PD; ++j) vfut[j] = vb[(long long)clampz(z0 + PD + j) * pvec];
#pragma unroll
    for (int j = 0; j < PD; ++j) {
      const int z = z0 + j;
      if (z >= ze) break;
      T *pl = lds + (z & 1) * lplane;
      const vec c = win[4];
      *reinterpret_cast<vec *>(pl + tp) = c;
      if (xh) *reinterpret_cast<vec *>(pl + tp + nx) = c;
      if (xl) *reinterpret_cast<vec *>(pl + tp - nx) = c;
      if (yh) *reinterpret_cast<vec *>(pl + tp + ny * SX) = c;
      if (yl) *reinterpret_cast<vec *>(pl + tp - ny * SX) = c;
      __syncthreads();
      // e[q] = value at x - 4 + q, q = 0 .. RX + 7
      T e[RX + 8];
#pragma unroll
      for (int q = 0; q < 4 / RX; ++q) {
        const vec a = *reinterpret_cast<const vec *>(pl + tp - 4 + q * RX);
        const vec b = *reinterpret_cast<const vec *>(pl + tp + RX + q * RX);
#pragma unroll
        for (int i = 0; i < RX; ++i) {
          e[q * RX + i] = a[i];
          e[4 + RX + q * RX + i] = b[i];
        }
      }
#pragma unroll
      for (int i = 0; i < RX; ++i) e[4 + i] = c[i];
      T acc[RX];
#pragma unroll
      for (int i = 0; i < RX; ++i) acc[i] = c0 * c[i];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const vec yp = *reinterpret_cast<const vec *>(pl + tp + (k + 1) * SX);
        const vec ym = *reinterpret_cast<const vec *>(pl + tp - (k + 1) * SX);
#pragma unroll
        for (int i = 0; i < RX; ++i) {
          acc[i] += ax[k] * (e[4 + i + k + 1] + e[4 + i - k - 1]);
          acc[i] += ay[k] * (yp[i] + ym[i]);
          acc[i] += az[k] * (win[5 + k][i] + win[3 - k][i]);
        }
      }
      vec out;
#pragma unroll
      for (int i = 0; i < RX; ++i) {
        acc[i] += vn[j][i] * c[i];
        out[i] = acc[i];
        dacc += (double)c[i] * (double)acc[i];
      }
      yb[(long long)z * pvec] = out;
#pragma unroll
      for (int k = 0; k < 8; ++k) win[k] = win[k + 1];
      win[8] = nxt[j];
    }
#pragma unroll
    for (int j = 0; j < PD; ++j) {
      nxt[j] = fut[j];
      vn[j] = vfut[j];
    }
  }
  if (dot) {
    // per-orbital tree over the orbital's threads (fixed order), in the
    // (no longer needed) plane area
    double *red = reinterpret_cast<double *>(lds_vec) + (size_t)ol * tpo;
    __syncthreads();
    red[tt] = dacc;
    __syncthreads();
    int p2 = 1;
    while (p2 < tpo) p2 <<= 1;
    for (int sft = p2 >> 1; sft > 0; sft >>= 1) {
      if (tt < sft && tt + sft < tpo) red[tt] += red[tt + sft];
      __syncthreads();
    }
    if (tt == 0 && valid) {
      if (zs == 1)
        dot[B] = g.dv * red[0];
      else
        dot_part[(long long)seg * nbands + (B - b0)] = red[0];
    }
  }
}

// dot[b0 + i] = dV sum over segments (in order) of the segment partials
__global__ void __launch_bounds__(256) k_dot_segments(Geo g, long long b0, long long nbands,
                                                      int zs, const double *__restrict__ part,
                                                      double *__restrict__ dot) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nbands) return;
  double sum = 0.0;
  for (int q = 0; q < zs; ++q) sum += part[(long long)q * nbands + i];
  dot[b0 + i] = g.dv * sum;
}

// Four consecutive values from 16-byte aligned LDS.
template <typename T>
__device__ inline void lds_read4(const T *p, T *d) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  if (sizeof(T) == 4) {
    const v4 v = *reinterpret_cast<const v4 *>(p);
    d[0] = v[0]; d[1] = v[1]; d[2] = v[2]; d[3] = v[3];
  } else {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 a = reinterpret_cast<const v2 *>(p)[0], b = reinterpret_cast<const v2 *>(p)[1];
    d[0] = a[0]; d[1] = a[1]; d[2] = b[0]; d[3] = b[1];
  }
}

template <typename T>
__device__ inline void load4_aligned(const T *p, T *d);
template <>
__device__ inline void load4_aligned<float>(const float *p, float *d) {
  const float4 v = *reinterpret_cast<const float4 *>(p);
  d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
}
template <>
__device__ inline void load4_aligned<double>(const double *p, double *d) {
  const double2 a = reinterpret_cast<const double2 *>(p)[0];
  const double2 b = reinterpret_cast<const double2 *>(p)[1];
  d[0] = a.x; d[1] = a.y; d[2] = b.x; d[3] = b.y;
}

// Rows (runs of nx points) of a projector region.
__device__ inline int region_nrows(const Geo &g, const KBTables &kb) {
  return kb.RY ? kb.RY * kb.RZ : region_rows(g.nl[0]);
}
// (ly, lz) of row rr of region reg (rows past the box of the last linear
// region map to a valid row; their points are masked)
__device__ inline void region_row(const Geo &g, const KBTables &kb, int reg, int rr, int &ly,
                                  int &lz) {
  const int ny = g.nl[1];
  if (kb.RY) {
    const int b = reg / (g.nl[0] / kb.RX);   // (row block, plane block) of the region
    const int nyr = ny / kb.RY;
    ly = (b % nyr) * kb.RY + rr % kb.RY;
    lz = (b / nyr) * kb.RZ + rr / kb.RY;
  } else {
    const int row = reg * kRegion / g.nl[0] + rr;
    ly = row % ny;
    lz = min(row / ny, g.nl[2] - 1);
  }
}
// Local point of region-local index q, with its x and region row (q < RP;
// linear regions: the result may pass the box, x and row are then clamped)
__device__ inline int region_point(const Geo &g, const KBTables &kb, int reg, int q, int &lx,
                                   int &rr) {
  const int nx = g.nl[0];
  if (kb.RY) {
    lx = (reg % (nx / kb.RX)) * kb.RX + q % kb.RX;
    rr = q / kb.RX;
    int ly, lz;
    region_row(g, kb, reg, rr, ly, lz);
    return lx + nx * (ly + g.nl[1] * lz);
  }
  const int l = reg * kRegion + q;
  const int lc = l < g.n ? l : g.n - 1;
  lx = lc % nx;
  rr = lc / nx - reg * kRegion / nx;
  return l;
}

// Tables of one projector region in LDS, built once per workgroup (byte
// offsets from kb_tab): the region's points pts[q] = (local point l, x | row
// << 16); per slot s the separable factors of the Gaussian, ex[s][x] =
// exp(-c2 dx^2) and eyz[s][row] = sc exp(-c2 (dz^2 + dy^2)); and the support
// of the slot as bit masks over x, msk[s][row][x / 32], bit set where
// r2 = (dz^2 + dy^2) + dx^2 <= rcut^2 in FP64 (the test of the definition).
// An empty slot has no support bits.  The FP64 squared offsets are staged in
// tmp (the kernel's own area, free until the tables are built).
struct KbTab {
  int nxs, rrs;                     // row strides of ex and of eyz / msk (bank spread)
  int msk, eyz, ex, pts, area;
};
__host__ __device__ inline int kb_align16(int b) { return (b + 15) & ~15; }
__host__ __device__ inline KbTab kb_tab(int KS, int nx, int RR, int RP, int elem) {
  KbTab t;
  t.nxs = nx + 16 / elem;           // 16-byte rows when 16 bytes hold whole x runs
  t.rrs = RR | 1;
  t.msk = 0;
  t.eyz = kb_align16(KS * t.rrs * ((nx + 31) >> 5) * 4);
  t.ex = kb_align16(t.eyz + KS * t.rrs * elem);
  t.pts = kb_align16(t.ex + KS * t.nxs * elem);
  t.area = kb_align16(t.pts + RP * 8);
  return t;
}

template <typename T>
__device__ inline void stage_region(const Geo &g, const KBTables &kb, const KbTab &tb, int f,
                                    int reg, unsigned *msk, T *eyz, T *ex, int2 *pts,
                                    double *tmp) {
  const int nx = g.nl[0], ny = g.nl[1], nls = g.nl[0] + g.nl[1] + g.nl[2];
  const int RR = region_nrows(g, kb), NWD = (nx + 31) >> 5, KS = kb.KS;
  const int *ra = kb.reg_atom + ((long long)f * kb.NR + reg) * KS;
  const int pf = kb.pair_first[f];
  double *tsx = tmp, *tsyz = tmp + KS * nx;
  for (int q = threadIdx.x; q < kb.RP; q += blockDim.x) {
    int lx, rr;
    const int l = region_point(g, kb, reg, q, lx, rr);
    pts[q] = make_int2(l, lx | (rr << 16));
  }
  for (int e = threadIdx.x; e < KS * nx; e += blockDim.x) {
    const int a = ra[e / nx];
    double v = 0.0, c2 = 0.0;
    if (a >= 0) {
      v = kb.pr_sq[(long long)(pf + a) * nls + e % nx];
      c2 = kb.pr_par[(long long)(pf + a) * 3 + 1];
    }
    tsx[e] = v;
    ex[(e / nx) * tb.nxs + e % nx] = (T)exp(-v * c2);
  }
  for (int e = threadIdx.x; e < KS * RR; e += blockDim.x) {
    const int a = ra[e / RR];
    int ly, lz;
    region_row(g, kb, reg, e % RR, ly, lz);
    double v = 0.0, w = 0.0;
    if (a >= 0) {
      const double *q = kb.pr_sq + (long long)(pf + a) * nls;
      const double *par = kb.pr_par + (long long)(pf + a) * 3;
      v = q[nx + ny + lz] + q[nx + ly];
      w = par[0] * exp(-v * par[1]);
    }
    tsyz[e] = v;
    eyz[(e / RR) * tb.rrs + e % RR] = (T)w;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < KS * RR * NWD; e += blockDim.x) {
    const int sl = e / (RR * NWD), row = (e / NWD) % RR, w = e % NWD;
    const int a = ra[sl];
    unsigned m = 0u;
    if (a >= 0) {
      const double rc2 = kb.pr_par[(long long)(pf + a) * 3 + 2], yz = tsyz[sl * RR + row];
      const double *sx = tsx + sl * nx + 32 * w;
      const int nb = min(32, nx - 32 * w);
      for (int b = 0; b < nb; ++b)
        if (!(yz + sx[b] > rc2)) m |= 1u << b;
    }
    msk[(sl * tb.rrs + row) * NWD + w] = m;
  }
}

// beta of slot s at the point (lx, region row rr): eyz ex on the support, else 0
template <typename T>
__device__ inline T beta_at(const KbTab &tb, const unsigned *msk, const T *eyz, const T *ex,
                            int NWD, int s, int lx, int rr) {
  const int sr = s * tb.rrs + rr;
  const unsigned m = msk[sr * NWD + (lx >> 5)];
  const T v = eyz[sr] * ex[s * tb.nxs + lx];
  return ((m >> (lx & 31)) & 1u) ? v : (T)0;
}

// Points per load step of the projection.
template <typename T>
constexpr int kb_chunk() { return sizeof(T) == 4 ? 64 : 32; }

// Region partials of the projections: part[(f, region)][slot][i] =
// sum_{l in region} beta_slot(l) X_i(l), as MFMA products of the region's beta
// block (slots x points) with its orbital columns.  Wave w takes orbital tile w
// over every point, and with five tiles the fifth goes to wave (workgroup index
// mod 4), so that no SIMD always takes the heavier wave; tiles at or beyond the
// fragment's orbital count are skipped (their partials stay zero).  The K index
// walks the points of a 16-point step as 4 (lane/16) + t, so every lane reads
// runs of 4 contiguous orbital values (16-byte loads when VEC: n % 4 == 0 and
// nx % 4 == 0).  Each wave forms its own beta operand in registers from the
// region tables: with VEC a lane's 4 points lie in one x run, so one 16-byte
// read of ex, one eyz value and one mask word give all four.  The main loop
// has no barrier; the orbital values of the next step are loaded before the
// products of the current one (unconditional loads, rows and points clamped,
// values masked).
template <typename T, int TM, int KT, bool VEC>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? (TM < 5 ? 4 : 3) : 1, 8))) k_kb_project(Geo g, OrbSet o, KBTables kb, int f0,
                                                    const T *__restrict__ x,
                                                    double *__restrict__ part) {
  typedef Mfma<T> MM;
  constexpr int MP = 16 * TM;
  constexpr int CH = kb_chunk<T>();
  constexpr int NS = CH / 16;                  // 16-point steps per load step
  constexpr int JW = (TM + 3) / 4;             // orbital tile items per wave
  static_assert(JW <= 2, "at most eight orbital tiles");
  extern __shared__ __attribute__((aligned(16))) double kb_lds[];
  const int nx = g.nl[0], RR = region_nrows(g, kb), NWD = (nx + 31) >> 5;
  const int NCH = kb.RP / CH;
  const KbTab tb = kb_tab(kb.KS, nx, RR, kb.RP, (int)sizeof(T));
  char *lds = reinterpret_cast<char *>(kb_lds);
  unsigned *msk = reinterpret_cast<unsigned *>(lds + tb.msk);
  T *eyz = reinterpret_cast<T *>(lds + tb.eyz), *ex = reinterpret_cast<T *>(lds + tb.ex);
  int2 *pts = reinterpret_cast<int2 *>(lds + tb.pts);
  const int f = o.perm[f0 + blockIdx.x / kb.NR];
  const int reg = blockIdx.x % kb.NR;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, kk = lane >> 4;
  const int mf = o.m[f];
  const int rmax = o.row_pad ? MP - 1 : mf - 1;
  const long long base = o.moff[f] * (long long)g.n;
  // orbital tile of item q of this wave (TM when the item has none) and whether
  // it holds orbitals of the fragment (uniform over the wave)
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  int jts[JW];
  bool live[JW];
#pragma unroll
  for (int q = 0; q < JW; ++q) {
    jts[q] = q == 0 ? wv : (wv == (int)(blockIdx.x & 3) ? 4 * q : TM);
    if (jts[q] > TM) jts[q] = TM;
    live[q] = jts[q] < TM && jts[q] * 16 < mf;
  }
  // (the first step's loads are issued before the point table exists)
  auto load_x = [&](int ch, T (*bx)[NS][4], bool direct) {
#pragma unroll
    for (int q = 0; q < JW; ++q) {
      const int jt = jts[q];
      const int orb = jt * 16 + r;
      const bool ok = live[q] && orb < mf;
      if (!live[q]) {
#pragma unroll
        for (int u = 0; u < NS; ++u)
#pragma unroll
          for (int t = 0; t < 4; ++t) bx[q][u][t] = (T)0;
        continue;
      }
      const T *row = x + base + (long long)(orb < rmax ? orb : rmax) * g.n;
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int qu = ch * CH + u * 16 + 4 * kk;
        int pu;
        if (direct) {
          int lx0, rr0;
          pu = region_point(g, kb, reg, qu, lx0, rr0);
        } else {
          pu = pts[qu].x;
        }
        if (VEC) {
          // four consecutive region points are consecutive local points of one
          // x run, wholly inside or outside the box
          const int pc = pu < g.n ? pu : g.n - 4;
          T v[4];
          load4_aligned(row + pc, v);
#pragma unroll
          for (int t = 0; t < 4; ++t) bx[q][u][t] = (ok && pu < g.n) ? v[t] : (T)0;
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int pt = direct ? pu + t : pts[qu + t].x;
            const T v = row[pt < g.n ? pt : g.n - 1];
            bx[q][u][t] = (ok && pt < g.n) ? v : (T)0;
          }
        }
      }
    }
  };
  // beta of slot tile st (slot st * 16 + r) at the lane's four points of region
  // index q0 .. q0 + 3
  auto beta4 = [&](int st, int q0, T *av) {
    const int sl = st * 16 + r;
    if (VEC) {
      const int2 pq = pts[q0];
      const int lx = (pq.y & 0xFFFF) & ~3, rr = pq.y >> 16;
      const int sr = sl * tb.rrs + rr;
      const unsigned m = msk[sr * NWD + (lx >> 5)] >> (lx & 31);
      const T e = eyz[sr];
      T xv[4];
      lds_read4(ex + sl * tb.nxs + lx, xv);
#pragma unroll
      for (int t = 0; t < 4; ++t) av[t] = (pq.x < g.n && ((m >> t) & 1u)) ? e * xv[t] : (T)0;
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int2 pq = pts[q0 + t];
        const T v = beta_at<T>(tb, msk, eyz, ex, NWD, sl, pq.y & 0xFFFF, pq.y >> 16);
        av[t] = pq.x < g.n ? v : (T)0;
      }
    }
  };
  // slot tiles that hold atoms in this region (the rest are skipped)
  const int nt = kb.reg_nt[(long long)f * kb.NR + reg];
  T bx[JW][NS][4];
  load_x(0, bx, true);
  stage_region<T>(g, kb, tb, f, reg, msk, eyz, ex, pts, reinterpret_cast<double *>(lds + tb.area));
  __syncthreads();
  typename MM::acc_t acc[KT][JW];
#pragma unroll
  for (int st = 0; st < KT; ++st)
#pragma unroll
    for (int q = 0; q < JW; ++q) acc[st][q] = MM::zero();
  for (int ch = 0; ch < NCH; ++ch) {
    T bn[JW][NS][4];
    load_x(ch + 1 < NCH ? ch + 1 : ch, bn, false);
    // products of the slot tiles in use (nt is uniform: a compile-time count each)
    auto products = [&](auto kte) {
      constexpr int KTE = decltype(kte)::value;
#pragma unroll
      for (int u = 0; u < NS; ++u)
#pragma unroll
        for (int st = 0; st < KTE; ++st) {
          T av[4];
          beta4(st, ch * CH + u * 16 + 4 * kk, av);
#pragma unroll
          for (int q = 0; q < JW; ++q)
            if (live[q])
#pragma unroll
              for (int t = 0; t < 4; ++t) acc[st][q] = MM::mma(av[t], bx[q][u][t], acc[st][q]);
        }
    };
    if (nt <= 1)
      products(std::integral_constant<int, 1>());
    else if (nt == 2)
      products(std::integral_constant<int, (KT < 2 ? KT : 2)>());
    else
      products(std::integral_constant<int, KT>());
#pragma unroll
    for (int q = 0; q < JW; ++q)
#pragma unroll
      for (int u = 0; u < NS; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) bx[q][u][t] = bn[q][u][t];
  }
  // partials in the accumulation type (FP32 sums are stored exactly as FP32)
  T *out = reinterpret_cast<T *>(part) + ((long long)f * kb.NR + reg) * kb.KS * o.m_pad;
#pragma unroll
  for (int q = 0; q < JW; ++q) {
    const int jt = jts[q];
    if (jt >= TM) continue;
#pragma unroll
    for (int st = 0; st < KT; ++st)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr)
        out[(st * 16 + MM::row(kk, rr)) * o.m_pad + jt * 16 + r] = acc[st][q][rr];
  }
}

// C[f][a][i] = dV sum over the (region, slot) entries of atom a (region partials
// of type T, summed in FP64).
template <typename T>
__global__ void __launch_bounds__(256) k_kb_reduce(Geo g, OrbSet o, KBTables kb, int f0, int nf,
                                                   const T *__restrict__ part,
                                                   double *__restrict__ C) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)nf * kb.A_max * o.m_pad;
  if (idx >= total) return;
  const int i = (int)(idx % o.m_pad);
  const long long la = idx / o.m_pad;   // (launch-local fragment, atom)
  const int f = o.perm[f0 + (int)(la / kb.A_max)];
  const long long fa = (long long)f * kb.A_max + la % kb.A_max;
  double s = 0.0;
  // four entries in flight at a time, added in entry order
  long long e = kb.ar_ptr[fa];
  const long long e1 = kb.ar_ptr[fa + 1];
  for (; e + 4 <= e1; e += 4) {
    double v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const long long q = ((long long)f * kb.NR + kb.ar_reg[e + t]) * kb.KS + kb.ar_slot[e + t];
      v[t] = (double)part[q * o.m_pad + i];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) s += v[t];
  }
  for (; e < e1; ++e) {
    const long long q = ((long long)f * kb.NR + kb.ar_reg[e]) * kb.KS + kb.ar_slot[e];
    s += (double)part[q * o.m_pad + i];
  }
  C[fa * o.m_pad + i] = g.dv * s;
}

// Y_i(l) += sum_slot beta_slot(l) E_slot C[f][slot atom][i] per region, as MFMA
// products of (E C)^T (orbitals x slots, staged in LDS) with the region's beta
// block (slots x points, evaluated in registers from the staged slot tables);
// wave w takes the 16-point tiles w, w + 4, ... so the four waves cover 64
// consecutive points at a time.  The old Y values of the next tile are loaded
// before the products of the current one (unconditional loads, rows and points
// clamped, stores masked).
template <typename T, int TM, int KT, bool RP>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2, 8)))
k_kb_apply(Geo g, OrbSet o, KBTables kb, int f0, const double *__restrict__ C,
           T *__restrict__ y) {
  typedef Mfma<T> MM;
  constexpr int MP = 16 * TM;
  constexpr int LD = lds_stride(MP);
  constexpr int KSM = 16 * KT;
  extern __shared__ __attribute__((aligned(16))) double kb_lds[];
  const int nx = g.nl[0], RR = region_nrows(g, kb), NWD = (nx + 31) >> 5;
  const int NU = kb.RP / 16 / 4;  // tiles per wave
  const KbTab tb = kb_tab(kb.KS, nx, RR, kb.RP, (int)sizeof(T));
  char *lds = reinterpret_cast<char *>(kb_lds);
  unsigned *msk = reinterpret_cast<unsigned *>(lds + tb.msk);
  T *eyz = reinterpret_cast<T *>(lds + tb.eyz), *ex = reinterpret_cast<T *>(lds + tb.ex);
  int2 *pts = reinterpret_cast<int2 *>(lds + tb.pts);
  T *ec = reinterpret_cast<T *>(lds + tb.area);   // [KSM][LD]
  const int f = o.perm[f0 + blockIdx.x / kb.NR];
  const int reg = blockIdx.x % kb.NR;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int mf = o.m[f];
  const int rmax = o.row_pad ? MP - 1 : mf - 1;
  // 16-orbital tiles this fragment uses (wave-uniform): the rest are not loaded
  // (their addresses repeat the first tile's) nor multiplied
  const int tf = __builtin_amdgcn_readfirstlane((mf + 15) >> 4);
  const int *ra = kb.reg_atom + ((long long)f * kb.NR + reg) * kb.KS;
  const int nt = kb.reg_nt[(long long)f * kb.NR + reg];   // slot tiles in use
  const double *Cf = C + (long long)f * kb.A_max * o.m_pad;
  const double *Ef = kb.E + (long long)f * kb.A_max;
  // the tables first: their FP64 staging shares the area of (E C)^T
  stage_region<T>(g, kb, tb, f, reg, msk, eyz, ex, pts, reinterpret_cast<double *>(lds + tb.area));
  __syncthreads();
  for (int e = threadIdx.x; e < KSM * MP; e += blockDim.x) {
    const int slot = e / MP, i = e % MP;
    const int a = (slot < kb.KS) ? ra[slot] : -1;
    ec[slot * LD + i] = (a >= 0 && i < mf) ? (T)(Ef[a] * Cf[(long long)a * o.m_pad + i]) : (T)0;
  }
  __syncthreads();
  const long long base = o.moff[f] * (long long)g.n;
  const int c = lane & 15, kk = lane >> 4;
  // Y row orb = jt*16 + row_u(rr) + row_l(kk): with padded arrays (RP) the
  // address is a wave-uniform row part plus one lane offset; otherwise rows are
  // clamped per lane to the fragment's last band
  auto yaddr = [&](int jt, int rr, int pc) -> T * {
    if (RP)
      return y + base + (long long)(jt * 16 + MM::row_u(rr)) * g.n + (MM::row_l(kk) * g.n + pc);
    const int orb = jt * 16 + MM::row(kk, rr);
    return y + base + (long long)(orb < rmax ? orb : rmax) * g.n + pc;
  };
  auto load_y = [&](int k, T (*yv)[4]) {
    const int p = pts[(wave + 4 * k) * 16 + c].x;
    const int pc = p < g.n ? p : g.n - 1;
#pragma unroll
    for (int jt = 0; jt < TM; ++jt)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) yv[jt][rr] = *yaddr(jt < tf ? jt : 0, rr, pc);
  };
  T yv[TM][4];
  load_y(0, yv);
  for (int k = 0; k < NU; ++k) {
    T yn[TM][4];
    load_y(k + 1 < NU ? k + 1 : k, yn);
    const int2 pq = pts[(wave + 4 * k) * 16 + c];
    const int p = pq.x, lx = pq.y & 0xFFFF, rr0 = pq.y >> 16;
    typename MM::acc_t acc[TM];
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[j] = MM::zero();
    // beta of slots 4 st + kk at the lane's point and the products, over the
    // slot tiles in use (nt is uniform: a compile-time count each)
    auto products = [&](auto kte) {
      constexpr int KTE = decltype(kte)::value;
      T bv[KTE * 4];
#pragma unroll
      for (int st = 0; st < KTE * 4; ++st) {
        const T v = beta_at<T>(tb, msk, eyz, ex, NWD, 4 * st + kk, lx, rr0);
        bv[st] = p < g.n ? v : (T)0;
      }
#pragma unroll
      for (int st = 0; st < KTE * 4; ++st) {
#pragma unroll
        for (int jt = 0; jt < TM; ++jt)
          if (jt < tf) acc[jt] = MM::mma(ec[(4 * st + kk) * LD + jt * 16 + c], bv[st], acc[jt]);
        if ((st & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    };
    if (nt <= 1)
      products(std::integral_constant<int, 1>());
    else if (nt == 2)
      products(std::integral_constant<int, (KT < 2 ? KT : 2)>());
    else
      products(std::integral_constant<int, KT>());
#pragma unroll
    for (int jt = 0; jt < TM; ++jt)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int orb = jt * 16 + MM::row(kk, rr);
        if (orb < mf && p < g.n) *yaddr(jt, rr, p) = yv[jt][rr] + acc[jt][rr];
      }
#pragma unroll
    for (int jt = 0; jt < TM; ++jt)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) yv[jt][rr] = yn[jt][rr];
  }
}

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator.
__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ void __launch_bounds__(256) k_init_orbitals(Geo g, const int *__restrict__ band_frag,
                                                       const long long *__restrict__ moff,
                                                       long long M_tot, uint64_t seed,
                                                       T *__restrict__ psi) {
  const long long total = M_tot * (long long)g.n;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long B = e / g.n;
    const uint64_t l = (uint64_t)(e % g.n);
    const int f = band_frag[B];
    const uint64_t i = (uint64_t)(B - moff[f]);
    const uint64_t key = ((uint64_t)f << 40) | (i << 24) | l;
    const uint64_t z = splitmix64(seed, key + 1);
    psi[e] = (T)((double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5);
  }
}

// Band energy per band eb[B] = f_B dV <psi_B, H psi_B>, grad_psi = 2 f dV H psi.
template <typename T>
__global__ void __launch_bounds__(256) k_band_energy_terms(Geo g, const T *__restrict__ psi,
                                                           const T *__restrict__ hpsi,
                                                           const double *__restrict__ f,
                                                           double *__restrict__ eb,
                                                           T *__restrict__ grad_psi) {
  __shared__ double red[16];
  const long long B = blockIdx.x;
  const T *pb = psi + B * (long long)g.n;
  const T *hb = hpsi + B * (long long)g.n;
  double acc = 0.0;
  const double s = 2.0 * f[B] * g.dv;
  for (int l = threadIdx.x; l < g.n; l += blockDim.x) {
    acc += (double)pb[l] * (double)hb[l];
    if (grad_psi) grad_psi[B * (long long)g.n + l] = (T)(s * (double)hb[l]);
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) eb[B] = f[B] * g.dv * acc;
}

// The same per band with H psi given in hg and, when scale is set, replaced in
// place by the gradient 2 f_B dV H psi_B (each value read, then written, by the
// same thread).
template <typename T>
__global__ void __launch_bounds__(256) k_band_terms_inplace(Geo g, const T *__restrict__ psi,
                                                            T *hg, const double *__restrict__ f,
                                                            double *__restrict__ eb, int scale) {
  __shared__ double red[16];
  const long long B = blockIdx.x;
  const T *pb = psi + B * (long long)g.n;
  T *hb = hg + B * (long long)g.n;
  double acc = 0.0;
  const double s = 2.0 * f[B] * g.dv;
  for (int l = threadIdx.x; l < g.n; l += blockDim.x) {
    const double h = (double)hb[l];
    acc += (double)pb[l] * h;
    if (scale) hb[l] = (T)(s * h);
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) eb[B] = f[B] * g.dv * acc;
}

// dE/dV_loc on the global grid for the orbitals of every fragment: at global
// point G, dV sum over the fragment boxes that contain G (fragments in z, y, x
// order of their indices along each axis) of sum_i f_i psi_i(l)^2, l the local
// point of G in that box.  moff, m: band offsets and counts in fragment order.
template <typename T>
__global__ void __launch_bounds__(256) k_grad_v_all(Geo g, const long long *__restrict__ moff,
                                                    const int *__restrict__ m,
                                                    const T *__restrict__ psi,
                                                    const double *__restrict__ f,
                                                    double *__restrict__ gv) {
  const long long G = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (G >= g.Ng) return;
  const int gc[3] = {(int)(G % g.N[0]), (int)((G / g.N[0]) % g.N[1]),
                     (int)(G / ((long long)g.N[0] * g.N[1]))};
  // per axis: the fragment indices whose box covers the coordinate, and the local
  // coordinate in each (a box holds a point once: n_core + 2 b <= N)
  int fa[3][7], la[3][7], na[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    na[d] = 0;
    const int kmax = min(3, (g.b[d] + g.nc[d] - 1) / g.nc[d]);
    const int a0 = gc[d] / g.nc[d];
    for (int da = -kmax; da <= kmax; ++da) {
      int a = (a0 + da) % g.F[d];
      if (a < 0) a += g.F[d];
      bool dup = false;
      for (int k = 0; k < na[d]; ++k) dup |= fa[d][k] == a;
      if (dup) continue;
      int l = (gc[d] - (a * g.nc[d] - g.b[d])) % g.N[d];
      if (l < 0) l += g.N[d];
      if (l < g.nl[d]) {
        fa[d][na[d]] = a;
        la[d][na[d]] = l;
        ++na[d];
      }
    }
  }
  double acc = 0.0;
  for (int kz = 0; kz < na[2]; ++kz)
    for (int ky = 0; ky < na[1]; ++ky)
      for (int kx = 0; kx < na[0]; ++kx) {
        const int fr = fa[0][kx] + g.F[0] * (fa[1][ky] + g.F[1] * fa[2][kz]);
        const int l = la[0][kx] + g.nl[0] * (la[1][ky] + g.nl[1] * la[2][kz]);
        const long long b0 = moff[fr], b1 = b0 + m[fr];
        double s = 0.0;
        for (long long B = b0; B < b1; ++B) {
          const double v = (double)psi[B * g.n + l];
          s += f[B] * v * v;
        }
        acc += s;
      }
  gv[G] = g.dv * acc;
}

// energy = sum eb (accumulate: energy += sum eb, for a later chunk of bands)
__global__ void __launch_bounds__(64) k_band_energy_sum(int nb, const double *__restrict__ eb,
                                                        double *__restrict__ energy,
                                                        int accumulate) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = accumulate ? energy[0] : 0.0;
    for (int i = 0; i < nb; ++i) s += eb[i];
    energy[0] = s;
  }
}

// Orbital layout of mm vectors of fragment frag alone (every other fragment
// empty): m[f], moff[f] for f < nf and moff[nf], band_frag[B] for B < mm.
__global__ void __launch_bounds__(256) k_single_layout(int nf, int frag, int mm,
                                                       int *__restrict__ m,
                                                       long long *__restrict__ moff,
                                                       int *__restrict__ band_frag) {
  for (int f = blockIdx.x * blockDim.x + threadIdx.x; f <= nf; f += gridDim.x * blockDim.x) {
    if (f < nf) m[f] = f == frag ? mm : 0;
    moff[f] = f > frag ? mm : 0;
    if (f < mm) band_frag[f] = frag;
  }
  for (int B = nf + 1 + blockIdx.x * blockDim.x + threadIdx.x; B < mm;
       B += gridDim.x * blockDim.x)
    band_frag[B] = frag;
}

// grad_v(l) = dV sum_i f_i psi_i(l)^2
template <typename T>
__global__ void __launch_bounds__(256) k_grad_v(Geo g, int nb, const T *__restrict__ psi,
                                                const double *__restrict__ f,
                                                double *__restrict__ grad_v) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= g.n) return;
  double acc = 0.0;
  for (int i = 0; i < nb; ++i) {
    const double v = (double)psi[(long long)i * g.n + l];
    acc += f[i] * v * v;
  }
  grad_v[l] = g.dv * acc;
}

inline int grid_for(long long n, int block) {
  long long b = (n + block - 1) / block;
  if (b > 65536 * 4) b = 65536 * 4;
  return (int)(b < 1 ? 1 : b);
}

template <typename T, int TM, int KT>
void kb_t(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1, const T *x,
          double *C, double *part, T *y, hipStream_t s) {
  const dim3 grid((f1 - f0) * kb.NR), block(256);
  if (x) {
    const size_t lds = kb_lds_bytes(g, kb.KS, kb.RY ? kb.RY * kb.RZ : region_rows(g.nl[0]), kb.RP, TM,
                                    sizeof(T), false);
    // 16-byte runs of one x run need n % 4 == 0, nx % 4 == 0 and an aligned array
    if (g.n % 4 == 0 && g.nl[0] % 4 == 0 && (uintptr_t)x % 16 == 0)
      hipLaunchKernelGGL((k_kb_project<T, TM, KT, true>), grid, block, lds, s, g, o, kb, f0, x,
                         part);
    else
      hipLaunchKernelGGL((k_kb_project<T, TM, KT, false>), grid, block, lds, s, g, o, kb, f0, x,
                         part);
    const long long total = (long long)(f1 - f0) * kb.A_max * o.m_pad;
    hipLaunchKernelGGL(k_kb_reduce<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g,
                       o, kb, f0, f1 - f0, reinterpret_cast<const T *>(part), C);
  } else {
    const size_t lds = kb_lds_bytes(g, kb.KS, kb.RY ? kb.RY * kb.RZ : region_rows(g.nl[0]), kb.RP, TM,
                                    sizeof(T), true);
    if (o.row_pad)
      hipLaunchKernelGGL((k_kb_apply<T, TM, KT, true>), grid, block, lds, s, g, o, kb, f0, C, y);
    else
      hipLaunchKernelGGL((k_kb_apply<T, TM, KT, false>), grid, block, lds, s, g, o, kb, f0, C, y);
  }
}

template <typename T, int TM>
void kb_tm(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1, const T *x,
           double *C, double *part, T *y, hipStream_t s) {
  switch (kb.KS / 16) {
    case 1: kb_t<T, TM, 1>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 2: kb_t<T, TM, 2>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 3: kb_t<T, TM, 3>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 4: kb_t<T, TM, 4>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 5: kb_t<T, TM, 5>(g, o, kb, f0, f1, x, C, part, y, s); break;
    default: kb_t<T, TM, 6>(g, o, kb, f0, f1, x, C, part, y, s); break;
  }
}

template <typename T>
void kb_dispatch(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1, const T *x,
                 double *C, double *part, T *y, hipStream_t s) {
  if (f1 <= f0) return;
  switch (o.tiles) {
    case 1: kb_tm<T, 1>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 2: kb_tm<T, 2>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 3: kb_tm<T, 3>(g, o, kb, f0, f1, x, C, part, y, s); break;
    case 4: kb_tm<T, 4>(g, o, kb, f0, f1, x, C, part, y, s); break;
    default: kb_tm<T, 5>(g, o, kb, f0, f1, x, C, part, y, s); break;
  }
}

template <typename T, int PD, bool HT>
void launch_halo(const Geo &g, long long nb, const OrbSet &o, int f0, const double *veff,
                 const T *x, T *y, hipStream_t s, double *dot, int vbase) {
  const int plane = g.nl[0] * g.nl[1];
  const size_t lds = 2 * (size_t)(g.nl[1] + 8) * (g.nl[0] + 32) * sizeof(T);
  if (g.nl[0] == 24)
    hipLaunchKernelGGL((k_hloc_halo<T, 24, PD, HT>), dim3((unsigned)nb), dim3(plane), lds, s, g,
                       o.band_frag, o.b0(f0), vbase, veff, x, y, dot);
  else if (g.nl[0] == 32)
    hipLaunchKernelGGL((k_hloc_halo<T, 32, PD, HT>), dim3((unsigned)nb), dim3(plane), lds, s, g,
                       o.band_frag, o.b0(f0), vbase, veff, x, y, dot);
  else
    hipLaunchKernelGGL((k_hloc_halo<T, 0, PD, HT>), dim3((unsigned)nb), dim3(plane), lds, s, g,
                       o.band_frag, o.b0(f0), vbase, veff, x, y, dot);
}

// Orbitals per workgroup of the vector kernel (0: not applicable): wide = the
// largest count whose thread total is a whole number of waves, otherwise the
// smallest count that keeps at least 85% of the lanes busy.
template <typename T, int VB>
int vec_opw(const Geo &g, bool wide) {
  constexpr int RX = VB / sizeof(T) > 0 ? VB / sizeof(T) : 1;
  if (g.nl[0] % RX || !hloc_halo_ok(g)) return 0;
  const int tpo = g.nl[0] / RX * g.nl[1];
  if (tpo > 1024) return 0;
  const size_t lds1 = 2 * (size_t)(g.nl[1] + 8) * (g.nl[0] + 32) * sizeof(T);
  const int top = std::min(4, 1024 / tpo);
  if (wide) {
    for (int opw = top; opw >= 1; --opw)
      if (opw * lds1 <= 65536 && (opw * tpo) % 64 == 0) return opw;
  }
  for (int opw = 1; opw <= top; ++opw) {
    if (opw * lds1 > 65536) break;
    const int threads = opw * tpo, lanes = (threads + 63) / 64 * 64;
    if (threads >= 0.85 * lanes) return opw;
  }
  return lds1 <= 65536 ? 1 : 0;
}

template <typename T, int PD, int VB>
void launch_vec(const Geo &g, long long nb, int opw, int zs, const OrbSet &o, int f0,
                const T *veffT, const T *x, T *y, hipStream_t s, double *dot, double *dot_part,
                int vbase) {
  const int tpo = g.nl[0] / (VB / (int)sizeof(T)) * g.nl[1];
  const size_t lds = (size_t)opw * 2 * (g.nl[1] + 8) * (g.nl[0] + 32) * sizeof(T);
  const unsigned grid = (unsigned)((nb + opw - 1) / opw * zs);
  hipLaunchKernelGGL((k_hloc_vec<T, PD, VB>), dim3(grid), dim3(opw * tpo), lds, s, g, o.band_frag,
                     o.b0(f0), nb, opw, zs, vbase, veffT, x, y, dot, dot_part);
  if (dot && zs > 1)
    hipLaunchKernelGGL(k_dot_segments, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, g,
                       o.b0(f0), nb, zs, dot_part, dot);
}

}  // namespace

// LDS bytes of the projector kernels: the region tables, then an area that
// holds the FP64 staging of the tables (and afterwards, in the application,
// the (E C)^T block of the widest orbital count)
size_t kb_lds_bytes(const Geo &g, int KS, int rr, int rp, int tiles, size_t elem, bool apply) {
  const KbTab t = kb_tab(KS, g.nl[0], rr, rp, (int)elem);
  const size_t tmp = (size_t)KS * (g.nl[0] + rr) * sizeof(double);
  const int MP = 16 * tiles;
  const size_t own = apply ? (size_t)KS * lds_stride(MP) * elem : 0;
  return (size_t)t.area + std::max(own, tmp);
}

// Planes of more than 1024 points (one workgroup cannot hold a thread per
// point): one workgroup per (kTileX x kTileY tile of the plane, orbital).  The
// tile with a four-point periodic halo of the current plane is staged in LDS
// (double-buffered, one barrier per plane); its entries are loaded kTilePD
// planes ahead into registers (each thread holds kTilePer entries of each plane
// in flight, at offsets computed once).  Each thread's own column marches along
// z with the nine-plane register window.  The terms are added in the order of
// k_hloc, so both give the same values.
constexpr int kTileX = 32, kTileY = 16, kTileNT = kTileX * kTileY, kTilePD = 4;
constexpr int kTileLX = kTileX + 8, kTileLY = kTileY + 8;
constexpr int kTilePer = (kTileLX * kTileLY + kTileNT - 1) / kTileNT;

template <typename T>
__global__ void __launch_bounds__(kTileNT)
    k_hloc_tile(Geo g, const int *__restrict__ band_frag, long long b0, int vbase,
                const double *__restrict__ veff, const T *__restrict__ x, T *__restrict__ y) {
  constexpr int LX = kTileLX, LY = kTileLY;
  __shared__ T lds[2][LY * LX];
  const int nx = g.nl[0], ny = g.nl[1], nz = g.nl[2];
  const int ntx = (nx + kTileX - 1) / kTileX;
  // the tiles of one orbital are consecutive work items
  const unsigned wi = xcd_ordered(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
  const int tile = wi % gridDim.x;
  const int tx0 = (tile % ntx) * kTileX, ty0 = (tile / ntx) * kTileY;
  const long long B = b0 + wi / gridDim.x;
  const int f = band_frag[B];
  const long long plane = (long long)nx * ny;
  const int t = threadIdx.x, lx = t % kTileX, ly = t / kTileX;
  const int ix = tx0 + lx, iy = ty0 + ly;
  const bool own = ix < nx && iy < ny;
  const long long pt = own ? ix + (long long)iy * nx : 0;   // idle lanes read point 0
  const T *xb = x + B * (long long)g.n;
  T *yb = y + B * (long long)g.n;
  const double *vb = veff + (long long)(f - vbase) * g.n;
  const T c0 = (T)g.kc[0];
  T ax[4], ay[4], az[4];
#pragma unroll
  for (int k = 1; k <= 4; ++k) {
    ax[k - 1] = (T)g.kc[k];
    ay[k - 1] = (T)g.kc[4 + k];
    az[k - 1] = (T)g.kc[8 + k];
  }
  // this thread's tile entries: plane offset (periodic wrap) and LDS slot;
  // entries past the tile repeat the last slot (loaded and stored like it)
  int off[kTilePer], slot[kTilePer];
#pragma unroll
  for (int j = 0; j < kTilePer; ++j) {
    const int e = min(t + j * kTileNT, LX * LY - 1);
    const int ex = e % LX, ey = e / LX;
    const int gx = ((tx0 - 4 + ex) % nx + nx) % nx;
    const int gy = ((ty0 - 4 + ey) % ny + ny) % ny;
    off[j] = gx + gy * nx;
    slot[j] = e;
  }
  // planes z .. z + kTilePD - 1 in flight (plane indices clamped into the box:
  // loads past the last plane are issued but never stored)
  T pre[kTilePD][kTilePer];
#pragma unroll
  for (int k = 0; k < kTilePD; ++k) {
    const long long zz = min(k, nz - 1);
#pragma unroll
    for (int j = 0; j < kTilePer; ++j) pre[k][j] = xb[zz * plane + off[j]];
  }
  T win[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int zz = ((k - 4) % nz + nz) % nz;
    win[k] = xb[zz * plane + pt];
  }
  double v0 = vb[pt], v1 = (nz > 1) ? vb[plane + pt] : 0.0;
  for (int z0 = 0; z0 < nz; z0 += kTilePD) {
#pragma unroll
    for (int k = 0; k < kTilePD; ++k) {
      const int z = z0 + k;
      if (z < nz) {   // uniform over the workgroup
        T *pl = lds[z & 1];
#pragma unroll
        for (int j = 0; j < kTilePer; ++j) pl[slot[j]] = pre[k][j];
        __syncthreads();
        const long long zn = min(z + kTilePD, nz - 1);
#pragma unroll
        for (int j = 0; j < kTilePer; ++j) pre[k][j] = xb[zn * plane + off[j]];
        if (own) {
          const int c = (ly + 4) * LX + lx + 4;
          T acc = c0 * win[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            acc += ax[q] * (pl[c + q + 1] + pl[c - q - 1]);
            acc += ay[q] * (pl[c + (q + 1) * LX] + pl[c - (q + 1) * LX]);
            acc += az[q] * (win[5 + q] + win[3 - q]);
          }
          acc += (T)v0 * win[4];
          yb[z * plane + pt] = acc;
        }
        v0 = v1;
        if (z + 2 < nz) v1 = vb[(z + 2) * plane + pt];
#pragma unroll
        for (int q = 0; q < 8; ++q) win[q] = win[q + 1];
        win[8] = xb[(long long)((z + 5) % nz) * plane + pt];
      }
    }
  }
}

// dot[B] = dV <x_B, y_B> for nb bands from b0 (the stencil's fused dot, for the
// tiled stencil); one workgroup per band
template <typename T>
__global__ void __launch_bounds__(256) k_band_dot(Geo g, long long b0, const T *__restrict__ x,
                                                  const T *__restrict__ y,
                                                  double *__restrict__ dot) {
  __shared__ double red[4];
  const long long B = b0 + blockIdx.x;
  const T *xb = x + B * (long long)g.n, *yb = y + B * (long long)g.n;
  double acc = 0.0;
  for (int l = threadIdx.x; l < g.n; l += blockDim.x) acc += (double)xb[l] * (double)yb[l];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) dot[B] = g.dv * acc;
}

bool hloc_halo_ok(const Geo &g) {
  // halo copies need nx, ny >= 4; the held end planes need nz >= 8; the padded
  // double plane must fit the 64 KB LDS a workgroup may address
  // (and a thread per point of the plane)
  return g.nl[0] >= 4 && g.nl[1] >= 4 && g.nl[2] >= 8 && g.nl[0] * g.nl[1] <= 1024 &&
         2 * (size_t)(g.nl[1] + 8) * (g.nl[0] + 32) * sizeof(double) <= 65536;
}

template <typename T>
void launch_hloc(const Geo &g, const OrbSet &o, int f0, int f1, const double *veff,
                 const T *veffT, const T *x, T *y, hipStream_t s, double *dot, int vbase,
                 double *dot_part) {
  const long long nb = o.nb(f0, f1);
  if (nb <= 0) return;
  const int plane = g.nl[0] * g.nl[1];
  if (plane > 1024) {
    // tiled plane (every variant); the dot in a pass of its own
    const unsigned tiles = (unsigned)(((g.nl[0] + kTileX - 1) / kTileX) *
                                      ((g.nl[1] + kTileY - 1) / kTileY));
    for (long long j0 = 0; j0 < nb; j0 += 65535) {
      const unsigned nj = (unsigned)std::min<long long>(65535, nb - j0);
      hipLaunchKernelGGL(k_hloc_tile<T>, dim3(tiles, nj), dim3(kTileNT), 0, s, g,
                         o.band_frag, o.b0(f0) + j0, vbase, veff, x, y);
    }
    if (dot)
      hipLaunchKernelGGL(k_band_dot<T>, dim3((unsigned)nb), dim3(256), 0, s, g, o.b0(f0), x, y,
                         dot);
    return;
  }
  int hv = g.hloc_variant;
  if (hv == HLOC_VEC || hv == HLOC_VEC_WIDE || hv == HLOC_VEC_Z2 || hv == HLOC_VEC_Z3 ||
      hv == HLOC_VEC8 || hv == HLOC_VEC8_WIDE) {
    const bool v8 = hv == HLOC_VEC8 || hv == HLOC_VEC8_WIDE;
    const bool wide = hv == HLOC_VEC_WIDE || hv == HLOC_VEC8_WIDE;
    const int opw = v8 ? vec_opw<T, 8>(g, wide) : vec_opw<T, 16>(g, wide);
    const int zs = hv == HLOC_VEC_Z2 ? 2 : (hv == HLOC_VEC_Z3 ? 3 : 1);
    const int vb = v8 ? 8 : 16;
    const bool aligned = ((uintptr_t)x % vb == 0) && ((uintptr_t)y % vb == 0) && veffT &&
                         ((uintptr_t)veffT % vb == 0);
    // z segments need nz / zs >= 4 and, with a dot, a partial buffer of
    // kHlocZsMax x nb doubles
    const bool zs_ok = zs == 1 || (g.nl[2] / zs >= 4 && (!dot || dot_part));
    if (opw > 0 && aligned && zs_ok) {
      if (v8)
        launch_vec<T, 1, 8>(g, nb, opw, zs, o, f0, veffT, x, y, s, dot, dot_part, vbase);
      else
        launch_vec<T, 1, 16>(g, nb, opw, zs, o, f0, veffT, x, y, s, dot, dot_part, vbase);
      return;
    }
    hv = HLOC_HALO_PD2;  // same results
  }
  if (hloc_halo_ok(g)) {
    switch (hv) {
      case HLOC_HALO_PD2: launch_halo<T, 2, false>(g, nb, o, f0, veff, x, y, s, dot, vbase); return;
      case HLOC_HALO_PD3: launch_halo<T, 3, false>(g, nb, o, f0, veff, x, y, s, dot, vbase); return;
      case HLOC_HALO_PD4: launch_halo<T, 4, false>(g, nb, o, f0, veff, x, y, s, dot, vbase); return;
      case HLOC_HALO_PD2_ENDS:
        launch_halo<T, 2, true>(g, nb, o, f0, veff, x, y, s, dot, vbase);
        return;
      default: break;
    }
  }
  hipLaunchKernelGGL(k_hloc<T>, dim3((unsigned)nb), dim3(plane), 2 * plane * sizeof(T), s, g,
                     o.band_frag, o.b0(f0), vbase, veff, x, y, dot);
}

template <typename T>
void launch_kb_project(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1,
                       const T *x, double *C, double *part, hipStream_t s) {
  kb_dispatch<T>(g, o, kb, f0, f1, x, C, part, nullptr, s);
}

template <typename T>
void launch_kb_apply(const Geo &g, const OrbSet &o, const KBTables &kb, int f0, int f1,
                     const double *C, T *y, hipStream_t s) {
  kb_dispatch<T>(g, o, kb, f0, f1, nullptr, const_cast<double *>(C), nullptr, y, s);
}

template <typename T>
void launch_init_orbitals(const Geo &g, const OrbSet &o, uint64_t seed, T *psi, hipStream_t s) {
  const long long total = o.M_tot * g.n;
  hipLaunchKernelGGL(k_init_orbitals<T>, dim3(grid_for(total, 256)), dim3(256), 0, s, g,
                     o.band_frag, o.moff, o.M_tot, seed, psi);
}

template <typename T>
void launch_band_energy_terms(const Geo &g, int nb, const T *psi, const T *hpsi, const double *f,
                              double *eb, double *energy, int accumulate, T *grad_psi,
                              hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_band_energy_terms<T>, dim3(nb), dim3(256), 0, s, g, psi, hpsi, f, eb,
                     grad_psi);
  if (energy)
    hipLaunchKernelGGL(k_band_energy_sum, dim3(1), dim3(64), 0, s, nb, eb, energy, accumulate);
}

template <typename T>
void launch_band_terms_inplace(const Geo &g, int nb, const T *psi, T *hg, const double *f,
                               double *eb, double *energy, int scale, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_band_terms_inplace<T>, dim3(nb), dim3(256), 0, s, g, psi, hg, f, eb,
                     scale);
  if (energy)
    hipLaunchKernelGGL(k_band_energy_sum, dim3(1), dim3(64), 0, s, nb, eb, energy, 0);
}

template <typename T>
void launch_grad_v_all(const Geo &g, const long long *moff, const int *m, const T *psi,
                       const double *f, double *grad_v, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_v_all<T>, dim3((unsigned)((g.Ng + 255) / 256)), dim3(256), 0, s, g,
                     moff, m, psi, f, grad_v);
}

template <typename T>
void launch_grad_v(const Geo &g, int nb, const T *psi, const double *f, double *grad_v,
                   hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_grad_v<T>, dim3((g.n + 255) / 256), dim3(256), 0, s, g, nb, psi, f,
                     grad_v);
}

void launch_single_layout(int nf, int frag, int mm, int *m, long long *moff, int *band_frag,
                          hipStream_t s) {
  const int n = std::max(nf + 1, mm);
  hipLaunchKernelGGL(k_single_layout, dim3((n + 255) / 256), dim3(256), 0, s, nf, frag, mm, m,
                     moff, band_frag);
}

#define DCDFT_INSTANTIATE(T)                                                                   \
  template void launch_hloc<T>(const Geo &, const OrbSet &, int, int, const double *,        \
                               const T *, const T *, T *, hipStream_t, double *, int,        \
                               double *);                                                    \
  template void launch_kb_project<T>(const Geo &, const OrbSet &, const KBTables &, int, int, \
                                     const T *, double *, double *, hipStream_t);            \
  template void launch_kb_apply<T>(const Geo &, const OrbSet &, const KBTables &, int, int,   \
                                   const double *, T *, hipStream_t);                        \
  template void launch_init_orbitals<T>(const Geo &, const OrbSet &, uint64_t, T *,           \
                                        hipStream_t);                                        \
  template void launch_band_energy_terms<T>(const Geo &, int, const T *, const T *,            \
                                            const double *, double *, double *, int, T *,     \
                                            hipStream_t);                                     \
  template void launch_grad_v<T>(const Geo &, int, const T *, const double *, double *,       \
                                 hipStream_t);                                                \
  template void launch_band_terms_inplace<T>(const Geo &, int, const T *, T *, const double *, \
                                             double *, double *, int, hipStream_t);           \
  template void launch_grad_v_all<T>(const Geo &, const long long *, const int *, const T *,   \
                                     const double *, double *, hipStream_t);
DCDFT_INSTANTIATE(double)
DCDFT_INSTANTIATE(float)
#undef DCDFT_INSTANTIATE

}  // namespace dcdft
