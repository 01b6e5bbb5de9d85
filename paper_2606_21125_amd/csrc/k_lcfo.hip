// DC-LCFO post-processing kernels (Sec. 2.3, Eqs. (6)-(9)): core projection of the
// selected fragment orbitals, the basis coefficients from the overlap eigenpairs,
// and the inner products between neighbouring fragments.  The overlap and
// same-fragment products, the overlap eigensolve, the rotation into the basis and
// the Hamiltonian application reuse the SCF kernels on FP64 arrays in the
// orbital layout [M_tot][n].
#include "dcdft_internal.h"
#include "device_common.h"

#include <type_traits>

namespace dcdft {
namespace {

// phibar[B][l] = psi[B][l] on core points of band B's fragment when B is among the
// fragment's first k_sel orbitals (eigenvalues ascending: those below eps_cut),
// 0 otherwise.
template <typename T>
__global__ void __launch_bounds__(256) k_lcfo_gather(Geo g, const int *__restrict__ band_frag,
                                                     const long long *__restrict__ moff,
                                                     const int *__restrict__ k_sel,
                                                     long long total, const T *__restrict__ psi,
                                                     double *__restrict__ phi) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const long long B = idx / g.n;
  const int l = (int)(idx - B * g.n);
  const int f = band_frag[B];
  const int i = (int)(B - moff[f]);
  const int lx = l % g.nl[0], ly = (l / g.nl[0]) % g.nl[1], lz = l / (g.nl[0] * g.nl[1]);
  const bool core = lx >= g.b[0] && lx < g.b[0] + g.nc[0] && ly >= g.b[1] &&
                    ly < g.b[1] + g.nc[1] && lz >= g.b[2] && lz < g.b[2] + g.nc[2];
  phi[idx] = (i < k_sel[f] && core) ? (double)psi[idx] : 0.0;
}

// The same for four consecutive points per thread (n and n_x multiples of 4: the
// four lie in one x row of one band; the core's x edges need not be multiples of
// 4, so the core test is taken per point).
template <typename T>
__global__ void __launch_bounds__(256) k_lcfo_gather4(Geo g, const int *__restrict__ band_frag,
                                                      const long long *__restrict__ moff,
                                                      const int *__restrict__ k_sel,
                                                      long long quads, const T *__restrict__ psi,
                                                      double *__restrict__ phi) {
  const long long qd = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (qd >= quads) return;
  const long long idx = 4 * qd;
  const long long B = idx / g.n;
  const int l = (int)(idx - B * g.n);
  const int f = band_frag[B];
  const bool sel = (int)(B - moff[f]) < k_sel[f];
  const int lx = l % g.nl[0], ly = (l / g.nl[0]) % g.nl[1], lz = l / (g.nl[0] * g.nl[1]);
  const bool row = ly >= g.b[1] && ly < g.b[1] + g.nc[1] && lz >= g.b[2] &&
                   lz < g.b[2] + g.nc[2];
  double v[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const bool core = row && lx + t >= g.b[0] && lx + t < g.b[0] + g.nc[0];
    v[t] = (sel && core) ? (double)psi[idx + t] : 0.0;
  }
  double2 *dst = reinterpret_cast<double2 *>(phi + idx);
  dst[0] = make_double2(v[0], v[1]);
  dst[1] = make_double2(v[2], v[3]);
}

// Basis coefficients of fragment f from the overlap eigenpairs (U columns,
// sigma ascending): the eigenvalues above lambda_cut are a suffix of the sorted
// list; column t of Cm is U[:, m - nb + t] / sqrt(sigma), t < nb, zero otherwise.
__global__ void __launch_bounds__(256) k_lcfo_coeffs(OrbSet o, const double *__restrict__ U,
                                                     const double *__restrict__ sigma,
                                                     double lambda_cut, double *__restrict__ Cm,
                                                     int *__restrict__ nb_out) {
  const int f = blockIdx.x;
  const int mf = o.m[f], mp = o.m_pad;
  const double *sg = sigma + o.moff[f];
  int nb = 0;
  for (int l = 0; l < mf; ++l) nb += sg[l] > lambda_cut ? 1 : 0;
  const double *Uf = U + (long long)f * mp * mp;
  double *Cf = Cm + (long long)f * mp * mp;
  for (int e = threadIdx.x; e < mp * mp; e += blockDim.x) {
    const int j = e / mp, t = e % mp;
    double v = 0.0;
    if (t < nb && j < mf) {
      const int l = mf - nb + t;
      v = Uf[j * mp + l] / sqrt(sg[l]);
    }
    Cf[e] = v;
  }
  if (threadIdx.x == 0) nb_out[f] = nb;
}

// X[p][i][j] = dV sum over the points of core b inside the box of a of
// (H^a lambda^a_i)(l_a) lambda^b_j(l_b), pair p = (a, b).  pairs[p] = {a, b,
// cx, cy, cz, ox, oy, oz}: per axis c* overlapping coordinates listed from o*
// in axes as (local coordinate in a's box, local coordinate in b's box).
// 16 x 16 threads, each holding up to a 5 x 5 block of the (at most 80 x 80)
// result (only the 16-row tiles the two bases use are loaded and multiplied);
// the points pass through LDS 32 at a time.
__global__ void __launch_bounds__(256) k_lcfo_cross(Geo g, OrbSet o, const int *__restrict__ pairs,
                                                    const int2 *__restrict__ axes,
                                                    const int *__restrict__ nbasis,
                                                    const double *__restrict__ hlam,
                                                    const double *__restrict__ lam,
                                                    double *__restrict__ X) {
  constexpr int R = kMaxOrb / 16;
  __shared__ double HA[kMaxOrb][33];
  __shared__ double LB[kMaxOrb][33];
  const int *pr = pairs + 8LL * blockIdx.x;
  const int a = pr[0], b = pr[1], cx = pr[2], cy = pr[3], cz = pr[4];
  const int ox = pr[5], oy = pr[6], oz = pr[7];
  const int na = nbasis[a], nbb = nbasis[b];
  const long long ra = o.moff[a] * (long long)g.n, rb = o.moff[b] * (long long)g.n;
  const int npts = cx * cy * cz;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  // 16-row tiles holding basis functions of a and of b (uniform over the block)
  const int ta = (na + 15) / 16, tb = (nbb + 15) / 16;
  const int rows = 16 * (ta > tb ? ta : tb);
  double acc[R][R];
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < R; ++j) acc[i][j] = 0.0;
  // the values of one 32-point chunk, loaded into registers a chunk ahead of
  // their use: thread item k holds row e >> 5 and point e & 31, e = tid + 256 k
  constexpr int NE = kMaxOrb * 32 / 256;
  double va[NE], vb[NE];
  // every item of a thread has the same point (256 k is a multiple of 32), so
  // its local indices are formed once per chunk
  auto gather = [&](int q0) {
    const int q = q0 + (threadIdx.x & 31);
    int la = 0, lb = 0;
    if (q < npts) {
      const int ix = q % cx, iy = (q / cx) % cy, iz = q / (cx * cy);
      const int2 px = axes[ox + ix], py = axes[oy + iy], pz = axes[oz + iz];
      la = px.x + g.nl[0] * (py.x + g.nl[1] * pz.x);
      lb = px.y + g.nl[0] * (py.y + g.nl[1] * pz.y);
    }
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int r = (threadIdx.x + 256 * k) >> 5;
      va[k] = (q < npts && r < na) ? hlam[ra + (long long)r * g.n + la] : 0.0;
      vb[k] = (q < npts && r < nbb) ? lam[rb + (long long)r * g.n + lb] : 0.0;
    }
  };
  gather(0);
  for (int q0 = 0; q0 < npts; q0 += 32) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = threadIdx.x + 256 * k;
      if ((e >> 5) < rows) {
        HA[e >> 5][e & 31] = va[k];
        LB[e >> 5][e & 31] = vb[k];
      }
    }
    __syncthreads();
    if (q0 + 32 < npts) gather(q0 + 32);
    auto products = [&](auto ca, auto cb) {   // compile-time tile counts
      constexpr int RA = decltype(ca)::value, RB = decltype(cb)::value;
      for (int pt = 0; pt < 32; ++pt) {
        double x[RA], y[RB];
#pragma unroll
        for (int i = 0; i < RA; ++i) x[i] = HA[ty + 16 * i][pt];
#pragma unroll
        for (int j = 0; j < RB; ++j) y[j] = LB[tx + 16 * j][pt];
#pragma unroll
        for (int i = 0; i < RA; ++i)
#pragma unroll
          for (int j = 0; j < RB; ++j) acc[i][j] = fma(x[i], y[j], acc[i][j]);
      }
    };
    const int tm = ta > tb ? ta : tb;
    if (tm <= 1) products(std::integral_constant<int, 1>(), std::integral_constant<int, 1>());
    else if (tm == 2) products(std::integral_constant<int, 2>(), std::integral_constant<int, 2>());
    else if (tm == 3) products(std::integral_constant<int, 3>(), std::integral_constant<int, 3>());
    else if (tm == 4) products(std::integral_constant<int, 4>(), std::integral_constant<int, 4>());
    else products(std::integral_constant<int, R>(), std::integral_constant<int, R>());
  }
  const int mp = o.m_pad;
  double *Xp = X + (long long)blockIdx.x * mp * mp;
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < R; ++j) {
      const int l = ty + 16 * i, l2 = tx + 16 * j;
      if (l < mp && l2 < mp) Xp[l * mp + l2] = g.dv * acc[i][j];
    }
}

}  // namespace

template <typename T>
void launch_lcfo_gather(const Geo &g, const OrbSet &o, const int *band_frag, const int *k_sel,
                        const T *psi, double *phi, hipStream_t s) {
  const long long total = o.M_tot * (long long)g.n;
  if (total <= 0) return;
  if (g.n % 4 == 0 && g.nl[0] % 4 == 0) {
    const long long quads = total / 4;
    hipLaunchKernelGGL(k_lcfo_gather4<T>, dim3((unsigned)((quads + 255) / 256)), dim3(256), 0, s,
                       g, band_frag, o.moff, k_sel, quads, psi, phi);
    return;
  }
  hipLaunchKernelGGL(k_lcfo_gather<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g,
                     band_frag, o.moff, k_sel, total, psi, phi);
}
template void launch_lcfo_gather<double>(const Geo &, const OrbSet &, const int *, const int *,
                                         const double *, double *, hipStream_t);
template void launch_lcfo_gather<float>(const Geo &, const OrbSet &, const int *, const int *,
                                        const float *, double *, hipStream_t);

void launch_lcfo_coeffs(const OrbSet &o, const double *U, const double *sigma, double lambda_cut,
                        double *Cm, int *nb, hipStream_t s) {
  if (o.nfrag <= 0) return;
  hipLaunchKernelGGL(k_lcfo_coeffs, dim3(o.nfrag), dim3(256), 0, s, o, U, sigma, lambda_cut, Cm,
                     nb);
}

void launch_lcfo_cross(const Geo &g, const OrbSet &o, int n_pairs, const int *pairs,
                       const int2 *axes, const int *nb, const double *hlam, const double *lam,
                       double *X, hipStream_t s) {
  if (n_pairs <= 0) return;
  hipLaunchKernelGGL(k_lcfo_cross, dim3(n_pairs), dim3(256), 0, s, g, o, pairs, axes, nb, hlam,
                     lam, X);
}

}  // namespace dcdft
