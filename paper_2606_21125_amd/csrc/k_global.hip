// Global-grid and fragment-field kernels of the SCF iteration: the global
// chemical potential (Sec. 2.2), fragment and total densities (Eqs. (2)-(4)),
// the fragment effective potential (Eq. (5)), the Hartree potential of the
// total density, the LDA exchange-correlation (Perdew-Zunger 1981), the
// energy terms, residuals and linear mixing.
#include "device_common.h"

namespace dcdft {

namespace {

__device__ inline double block_min(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = red[0];
  for (int w = 1; w < nw; ++w) t = fmin(t, red[w]);
  return t;
}

// Fermi-Dirac occupation 1 / (1 + e^x) without overflow.
__device__ inline double fermi(double x) {
  if (x >= 0.0) {
    const double t = exp(-x);
    return t / (1.0 + t);
  }
  return 1.0 / (1.0 + exp(x));
}

// Perdew-Zunger 1981 unpolarised LDA: eps_xc and v_xc, zero below rho = 1e-20.
__device__ inline void pz81(double rho, double &exc, double &vxc) {
  if (!(rho >= 1e-20)) {
    exc = 0.0;
    vxc = 0.0;
    return;
  }
  const double pi = 3.14159265358979323846;
  const double rs = cbrt(3.0 / (4.0 * pi * rho));
  const double cx = (3.0 / (4.0 * pi)) * cbrt(9.0 * pi / 4.0);
  const double ex = -cx / rs;
  const double vx = 4.0 / 3.0 * ex;
  double ec, vc;
  if (rs >= 1.0) {
    const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
    const double sq = sqrt(rs);
    const double den = 1.0 + b1 * sq + b2 * rs;
    ec = g / den;
    vc = ec * (1.0 + 7.0 / 6.0 * b1 * sq + 4.0 / 3.0 * b2 * rs) / den;
  } else {
    const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
    const double ln = log(rs);
    ec = A * ln + B + C * rs * ln + D * rs;
    vc = A * ln + (B - A / 3.0) + 2.0 / 3.0 * C * rs * ln + (2.0 * D - C) / 3.0 * rs;
  }
  exc = ex + ec;
  vxc = vx + vc;
}

__device__ inline long long global_of_local(const Geo &g, int f, int l) {
  const int ax = f % g.F[0], ay = (f / g.F[0]) % g.F[1], az = f / (g.F[0] * g.F[1]);
  const int lx = l % g.nl[0], ly = (l / g.nl[0]) % g.nl[1], lz = l / (g.nl[0] * g.nl[1]);
  int gx = (ax * g.nc[0] - g.b[0] + lx) % g.N[0];
  int gy = (ay * g.nc[1] - g.b[1] + ly) % g.N[1];
  int gz = (az * g.nc[2] - g.b[2] + lz) % g.N[2];
  if (gx < 0) gx += g.N[0];
  if (gy < 0) gy += g.N[1];
  if (gz < 0) gz += g.N[2];
  return gx + (long long)g.N[0] * (gy + (long long)g.N[1] * gz);
}

// Two block sums with one exchange: each value is summed exactly as block_sum
// sums it (wave sums, then the waves in order).  red holds 32 doubles.
__device__ inline void block_sum2(double &a, double &b, double *red) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    red[wave] = a;
    red[16 + wave] = b;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0;
  for (int w = 0; w < nw; ++w) {
    ta += red[w];
    tb += red[16 + w];
  }
  a = ta;
  b = tb;
}

// N(mu) = sum 2 f((eps - mu) / sigma) w by bisection over the bracket
// [min eps - 50 sigma, max eps + 50 sigma], one workgroup.
__global__ void __launch_bounds__(1024) k_fermi(long long nb, const double *__restrict__ eps,
                                                const double *__restrict__ w, double ne,
                                                double sigma, double *__restrict__ occ,
                                                double *__restrict__ scal, int *flags) {
  __shared__ double red[32];
  double cap = 0.0, lo = 1e300, hi = 1e300;
  for (long long i = threadIdx.x; i < nb; i += blockDim.x) {
    cap += 2.0 * w[i];
    lo = fmin(lo, eps[i]);
    hi = fmin(hi, -eps[i]);
  }
  cap = block_sum(cap, red);
  lo = block_min(lo, red) - 50.0 * sigma;
  hi = -block_min(hi, red) + 50.0 * sigma;
  const bool ok = cap >= ne * (1.0 - 1e-12);
  // N(mu) is increasing: keep a bracket lo < mu* <= hi and take Newton steps
  // (N' = sum 2 w f (1 - f) / sigma) from the previous step's mu when they
  // stay inside it, bisection otherwise; stop when N(mu) = N_e to 1e-14
  // relative, the Newton step is below 1e-15 |mu|, or the bracket cannot be
  // halved any more.
  double mu = scal[SC_MU];
  if (!(mu > lo && mu < hi)) mu = 0.5 * (lo + hi);
  for (int it = 0; it < 200 && ok; ++it) {
    double cnt = 0.0, der = 0.0;
    for (long long i = threadIdx.x; i < nb; i += blockDim.x) {
      const double fo = fermi((eps[i] - mu) / sigma);
      cnt += 2.0 * fo * w[i];
      der += 2.0 * fo * (1.0 - fo) * w[i];
    }
    block_sum2(cnt, der, red);
    der = der / sigma;
    if (fabs(cnt - ne) <= 1e-14 * ne) break;
    if (cnt < ne) lo = mu;
    else hi = mu;
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    const double step = (der > 0.0) ? (ne - cnt) / der : 0.0;
    const double nt = mu + step;
    if (der > 0.0 && nt > lo && nt < hi) {
      if (fabs(step) <= 1e-15 * fmax(1.0, fabs(mu))) {
        mu = nt;
        break;
      }
      mu = nt;
    } else {
      mu = mid;
    }
  }
  double eb = 0.0, ent = 0.0;
  for (long long i = threadIdx.x; i < nb; i += blockDim.x) {
    const double fo = fermi((eps[i] - mu) / sigma);
    occ[i] = fo;
    eb += 2.0 * fo * eps[i] * w[i];
    double t = 0.0;
    if (fo > 0.0) t += fo * log(fo);
    if (fo < 1.0) t += (1.0 - fo) * log(1.0 - fo);
    ent += -2.0 * w[i] * t;
  }
  block_sum2(eb, ent, red);
  if (threadIdx.x == 0) {
    scal[SC_MU] = mu;
    scal[SC_EBAND] = eb;
    scal[SC_ENTROPY] = ent;
    scal[SC_CAPACITY] = cap;
    if (!ok) atomicOr(flags, FLAG_CAPACITY);
  }
}

// rho_alpha^out(l) = sum_i 2 f_i psi_i(l)^2; core points also written to rho_tot^out.
template <typename T>
__global__ void __launch_bounds__(256) k_density(Geo g, const long long *__restrict__ moff,
                                                 const int *__restrict__ mcount,
                                                 int f0, int f1, const T *__restrict__ psi,
                                                 const double *__restrict__ occ,
                                                 double *__restrict__ rhof_out,
                                                 double *__restrict__ rho_out) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)(f1 - f0) * g.n) return;
  const int f = f0 + (int)(idx / g.n);
  const int l = (int)(idx % g.n);
  const long long b1 = moff[f] + mcount[f];
  const T *p = psi + l;
  double acc = 0.0;
  long long B = moff[f];
  // eight loads in flight, then the terms added in band order (the same sums as
  // one band at a time)
  for (; B + 8 <= b1; B += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (double)p[(B + k) * g.n];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += 2.0 * occ[B + k] * v[k] * v[k];
  }
  for (; B < b1; ++B) {
    const double v = (double)p[B * g.n];
    acc += 2.0 * occ[B] * v * v;
  }
  rhof_out[(long long)f * g.n + l] = acc;
  if (is_core_point(g, l)) rho_out[global_of_local(g, f, l)] = acc;
}

// V_eff of Eq. (5); with xi > 0 (rho_tot_in not NULL) the density-template
// potential (rho_alpha^in - rho_tot^in) / xi is added.
__global__ void __launch_bounds__(256) k_veff(Geo g, int f0, int f1, const double *__restrict__ vloc,
                                              const double *__restrict__ vh,
                                              const double *__restrict__ rhof_in,
                                              const double *__restrict__ rho_tot_in, double xi,
                                              double *__restrict__ veff,
                                              float *__restrict__ veff32) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)(f1 - f0) * g.n) return;
  const int f = f0 + (int)(idx / g.n);
  const int l = (int)(idx % g.n);
  const long long gi = global_of_local(g, f, l);
  const double rf = rhof_in[(long long)f * g.n + l];
  double exc, vxc;
  pz81(rf, exc, vxc);
  double v = vloc[gi] + vh[gi] + vxc;
  if (rho_tot_in) v = v + (rf - rho_tot_in[gi]) / xi;
  veff[(long long)f * g.n + l] = v;
  if (veff32) veff32[(long long)f * g.n + l] = (float)v;
}

// Energy terms on rho^in, charge and residuals, then linear mixing of rho_tot.
// part[block][6]: sum rho_in (V_H + V_xc), sum rho_in V_H, sum rho_in eps_xc,
// sum rho_out, sum |rho_out - rho_in|, sum |rho_new - rho_in|.
__global__ void __launch_bounds__(256) k_global_terms(Geo g, double *__restrict__ rho_in,
                                                      const double *__restrict__ rho_out,
                                                      const double *__restrict__ vh, double mixing,
                                                      double *__restrict__ part) {
  __shared__ double red[16];
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.Ng;
       i += (long long)gridDim.x * blockDim.x) {
    const double ri = rho_in[i], ro = rho_out[i], v = vh[i];
    double exc, vxc;
    pz81(ri, exc, vxc);
    s[0] += ri * (v + vxc);
    s[1] += ri * v;
    s[2] += ri * exc;
    s[3] += ro;
    s[4] += fabs(ro - ri);
    const double rn = ri + mixing * (ro - ri);
    s[5] += fabs(rn - ri);
    rho_in[i] = rn;
  }
  for (int k = 0; k < 6; ++k) {
    const double t = block_sum(s[k], red);
    if (threadIdx.x == 0) part[blockIdx.x * 6 + k] = t;
  }
}

__global__ void __launch_bounds__(256) k_global_final(Geo g, int nblk, double ne, double sigma,
                                                      const double *__restrict__ part,
                                                      double *__restrict__ scal) {
  __shared__ double red[16];
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
    for (int k = 0; k < 6; ++k) s[k] += part[b * 6 + k];
  for (int k = 0; k < 6; ++k) s[k] = block_sum(s[k], red);
  if (threadIdx.x != 0) return;
  const double dv = g.dv;
  scal[SC_HXC] = dv * s[0];
  scal[SC_EH] = 0.5 * dv * s[1];
  scal[SC_EXC] = dv * s[2];
  scal[SC_CHARGE] = dv * s[3];
  scal[SC_RES_OUT_IN] = dv * s[4] / ne;
  scal[SC_RES_PAPER] = dv * s[5] / ne;
  (void)sigma;
}

__global__ void __launch_bounds__(256) k_frag_mix(long long total, double *__restrict__ rin,
                                                  const double *__restrict__ rout, double mixing) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x)
    rin[i] = rin[i] + mixing * (rout[i] - rin[i]);
}

// out[a][k][c] = sum_j in[a][j][c] Q[j][k]   (axis of length n, inner stride C)
__global__ void __launch_bounds__(256) k_axis_transform(long long total, int n, long long C,
                                                        const double *__restrict__ in,
                                                        const double *__restrict__ Q,
                                                        double *__restrict__ out) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long c = e % C;
    const long long ak = e / C;
    const int k = (int)(ak % n);
    const long long a = ak / n;
    const double *src = in + a * n * C + c;
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc += src[(long long)j * C] * Q[(long long)j * n + k];
    out[e] = acc;
  }
}

// The same contraction on the FP64 matrix cores, for n % 16 == 0 and C % 16 == 0
// (or C == 1 with A % 16 == 0): one wave per 16 x 16 output tile.  C > 1: tile
// (a, k0, c0) of Out_a = Q^T In_a with In_a = in[a][.][.] (n x C); C == 1: tile
// (a0, k0) of Out = In Q with In = in[.][.] (A x n).  Each step takes 4 of the n
// contracted indices, one per lane group.
__global__ void __launch_bounds__(256) k_axis_mfma(long long A, int n, long long C,
                                                   const double *__restrict__ in,
                                                   const double *__restrict__ Q,
                                                   double *__restrict__ out) {
  typedef Mfma<double> MM;
  const long long tile = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, r = lane & 15, kk = lane >> 4;
  const long long nkt = n / 16;
  const long long ntc = C > 1 ? C / 16 : A / 16;   // column tiles (C > 1) or row tiles
  if (tile >= nkt * ntc * (C > 1 ? A : 1)) return;  // wave-uniform
  MM::acc_t acc = MM::zero();
  if (C > 1) {
    const long long a = tile / (nkt * ntc);
    const long long rem = tile % (nkt * ntc);
    const int k0 = (int)(rem / ntc) * 16;
    const long long c0 = (rem % ntc) * 16;
    const double *ia = in + a * n * C + c0 + r;
    for (int j = 0; j < n; j += 4) {
      // A = Q^T (16 k x 4 j), B = In_a (4 j x 16 c)
      acc = MM::mma(Q[(long long)(j + kk) * n + k0 + r], ia[(long long)(j + kk) * C], acc);
    }
    double *oa = out + a * n * C + c0 + r;
#pragma unroll
    for (int q = 0; q < 4; ++q) oa[(long long)(k0 + MM::row(kk, q)) * C] = acc[q];
  } else {
    const long long a0 = (tile / nkt) * 16;
    const int k0 = (int)(tile % nkt) * 16;
    for (int j = 0; j < n; j += 4) {
      // A = In (16 a x 4 j), B = Q (4 j x 16 k)
      acc = MM::mma(in[(a0 + r) * n + j + kk], Q[(long long)(j + kk) * n + k0 + r], acc);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) out[(a0 + MM::row(kk, q)) * n + k0 + r] = acc[q];
  }
}

// V_hat = -4 pi rho_hat / (lx + ly + lz), zero for the constant mode
__global__ void __launch_bounds__(256) k_poisson_scale(Geo g, const double *__restrict__ lx,
                                                       const double *__restrict__ ly,
                                                       const double *__restrict__ lz,
                                                       double *__restrict__ v) {
  const double pi = 3.14159265358979323846;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < g.Ng;
       e += (long long)gridDim.x * blockDim.x) {
    const int kx = (int)(e % g.N[0]);
    const int ky = (int)((e / g.N[0]) % g.N[1]);
    const int kz = (int)(e / ((long long)g.N[0] * g.N[1]));
    const double lam = lx[kx] + ly[ky] + lz[kz];
    v[e] = (kx == 0 && ky == 0 && kz == 0) ? 0.0 : -4.0 * pi * v[e] / lam;
  }
}

__global__ void k_fill(double *p, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_int(int *p, long long n, int v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_nan_check(const double *p, long long n, int *flags) {
  bool bad = false;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    if (!isfinite(p[i])) bad = true;
  if (bad) atomicOr(flags, FLAG_NAN);
}

// ---- Pulay mixing with a Kerker preconditioner ----------------------------------
// History slots: S = H + 1 ring slots of rho_in, R = rho_out - rho_in (global) and
// of the fragment deviations delta_in, delta_R (fragment boxes); at most H are in
// use, so the slot a step writes never holds an entry of the history it mixes.
// st[0] = entries in use, st[1] = newest slot (-1: none yet).
// A[i * S + j] = sum_g R_i(g) R_j(g) by slot; c[slot] = Pulay weight.

// Record the step in the free slot s = st[1] + 1 (mod S) and form the partial
// dot products of its residual with every slot's: part[block][j], j < S.
__global__ void __launch_bounds__(256) k_mix_record(Geo g, int S, const int *__restrict__ st,
                                                    const double *__restrict__ rho_in,
                                                    const double *__restrict__ rho_out,
                                                    double *__restrict__ hrho,
                                                    double *__restrict__ hres,
                                                    double *__restrict__ part) {
  __shared__ double red[16];
  const int s = (st[1] + 1) % S;
  double acc[kMixMaxSlots];
#pragma unroll
  for (int j = 0; j < kMixMaxSlots; ++j) acc[j] = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.Ng;
       i += (long long)gridDim.x * blockDim.x) {
    const double ri = rho_in[i];
    const double r = rho_out[i] - ri;
    hrho[(long long)s * g.Ng + i] = ri;
    hres[(long long)s * g.Ng + i] = r;
#pragma unroll
    for (int j = 0; j < kMixMaxSlots; ++j)
      if (j < S) acc[j] += r * (j == s ? r : hres[(long long)j * g.Ng + i]);
  }
  for (int j = 0; j < S; ++j) {
    const double t = block_sum(acc[j], red);
    if (threadIdx.x == 0) part[blockIdx.x * kMixMaxSlots + j] = t;
  }
}

// Fragment deviations of the step into slot s: delta_in = rho_alpha^in - rho_in(g(l)),
// delta_R = (rho_alpha^out - rho_out(g(l))) - delta_in.
__global__ void __launch_bounds__(256) k_mix_record_frag(Geo g, int nfrag, int S,
                                                         const int *__restrict__ st,
                                                         const double *__restrict__ rho_in,
                                                         const double *__restrict__ rho_out,
                                                         const double *__restrict__ rhof_in,
                                                         const double *__restrict__ rhof_out,
                                                         double *__restrict__ hdin,
                                                         double *__restrict__ hdres) {
  const int s = (st[1] + 1) % S;
  const long long total = (long long)nfrag * g.n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const int f = (int)(i / g.n), l = (int)(i % g.n);
    const long long gi = global_of_local(g, f, l);
    const double din = rhof_in[i] - rho_in[gi];
    hdin[(long long)s * total + i] = din;
    hdres[(long long)s * total + i] = (rhof_out[i] - rho_out[gi]) - din;
  }
}

// One thread: the new row of A from the partials, the history advanced by one,
// and the Pulay weights from the bordered system [[A, 1], [1^T, 0]] [c; l] = [0; 1]
// over the entries in use, oldest first, by Gaussian elimination with partial
// pivoting; a pivot at most 1e-12 max|A| cuts the history to the newest entry.
__global__ void __launch_bounds__(64) k_mix_solve(int S, int H, int nblk, int *__restrict__ st,
                                                  const double *__restrict__ part,
                                                  double *__restrict__ A,
                                                  double *__restrict__ c) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int s = (st[1] + 1) % S;
  for (int j = 0; j < S; ++j) {
    double t = 0.0;
    for (int b = 0; b < nblk; ++b) t += part[b * kMixMaxSlots + j];
    A[s * S + j] = t;
    A[j * S + s] = t;
  }
  int k = st[0] + 1 > H ? H : st[0] + 1;
  st[0] = k;
  st[1] = s;
  int slot[kMixMaxSlots];
  for (int q = 0; q < k; ++q) slot[q] = ((s - (k - 1) + q) % S + S) % S;
  double m[kMixMaxSlots + 1][kMixMaxSlots + 2];
  double amax = 0.0;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      m[i][j] = A[slot[i] * S + slot[j]];
      amax = fmax(amax, fabs(m[i][j]));
    }
  for (int i = 0; i < k; ++i) {
    m[i][k] = 1.0;
    m[k][i] = 1.0;
    m[i][k + 1] = 0.0;
  }
  m[k][k] = 0.0;
  m[k][k + 1] = 1.0;
  const double tiny = 1e-12 * amax;
  bool ok = true;
  for (int col = 0; col <= k && ok; ++col) {
    int piv = col;
    for (int r = col + 1; r <= k; ++r)
      if (fabs(m[r][col]) > fabs(m[piv][col])) piv = r;
    if (!(fabs(m[piv][col]) > tiny)) {
      ok = false;
      break;
    }
    if (piv != col)
      for (int j = 0; j <= k + 1; ++j) {
        const double t = m[col][j];
        m[col][j] = m[piv][j];
        m[piv][j] = t;
      }
    for (int r = col + 1; r <= k; ++r) {
      const double fr = m[r][col] / m[col][col];
      for (int j = col; j <= k + 1; ++j) m[r][j] -= fr * m[col][j];
    }
  }
  for (int j = 0; j < S; ++j) c[j] = 0.0;
  if (!ok) {
    st[0] = 1;
    c[s] = 1.0;
    return;
  }
  double x[kMixMaxSlots + 1];
  for (int r = k; r >= 0; --r) {
    double t = 0.0;
    for (int j = r + 1; j <= k; ++j) t += m[r][j] * x[j];
    x[r] = (m[r][k + 1] - t) / m[r][r];
  }
  for (int q = 0; q < k; ++q) c[slot[q]] = x[q];
}

// rho_bar = sum_j c_j rho_j into rbar, R_bar = sum_j c_j R_j into res (slots in use,
// oldest first)
__global__ void __launch_bounds__(256) k_mix_combine(Geo g, int S, const int *__restrict__ st,
                                                     const double *__restrict__ c,
                                                     const double *__restrict__ hrho,
                                                     const double *__restrict__ hres,
                                                     double *__restrict__ rbar,
                                                     double *__restrict__ res) {
  const int k = st[0], s = st[1];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.Ng;
       i += (long long)gridDim.x * blockDim.x) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < k; ++q) {
      const int j = ((s - (k - 1) + q) % S + S) % S;
      a += c[j] * hrho[(long long)j * g.Ng + i];
      b += c[j] * hres[(long long)j * g.Ng + i];
    }
    rbar[i] = a;
    res[i] = b;
  }
}

// Kerker filter in the real Fourier basis: v <- q^2 / (q^2 + q0^2) v, q^2 = -(lx + ly
// + lz), zero for the constant mode
__global__ void __launch_bounds__(256) k_kerker_scale(Geo g, const double *__restrict__ lx,
                                                      const double *__restrict__ ly,
                                                      const double *__restrict__ lz, double q02,
                                                      double *__restrict__ v) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < g.Ng;
       e += (long long)gridDim.x * blockDim.x) {
    const int kx = (int)(e % g.N[0]);
    const int ky = (int)((e / g.N[0]) % g.N[1]);
    const int kz = (int)(e / ((long long)g.N[0] * g.N[1]));
    const double q2 = -(lx[kx] + ly[ky] + lz[kz]);
    v[e] = (kx == 0 && ky == 0 && kz == 0) ? 0.0 : q2 / (q2 + q02) * v[e];
  }
}

// rho_in <- rho_bar + a K[R_bar], with partial sums of |rho_new - rho_in^(newest)|
// (the input density of this step) per block in part[block]
__global__ void __launch_bounds__(256) k_mix_update(Geo g, int S, const int *__restrict__ st,
                                                    const double *__restrict__ hrho,
                                                    const double *__restrict__ rbar,
                                                    const double *__restrict__ kres, double a,
                                                    double *__restrict__ rho_in,
                                                    double *__restrict__ part) {
  __shared__ double red[16];
  const int s = st[1];
  double d = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.Ng;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = rbar[i] + a * kres[i];
    d += fabs(v - hrho[(long long)s * g.Ng + i]);
    rho_in[i] = v;
  }
  const double t = block_sum(d, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// rho_alpha^in = rho_new(g(l)) + sum_j c_j delta_in^(j) + a sum_j c_j delta_R^(j)
__global__ void __launch_bounds__(256) k_mix_update_frag(Geo g, int nfrag, int S,
                                                         const int *__restrict__ st,
                                                         const double *__restrict__ c,
                                                         const double *__restrict__ hdin,
                                                         const double *__restrict__ hdres,
                                                         const double *__restrict__ rho_new,
                                                         double a, double *__restrict__ rhof_in) {
  const int k = st[0], s = st[1];
  const long long total = (long long)nfrag * g.n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    double di = 0.0, dr = 0.0;
    for (int q = 0; q < k; ++q) {
      const int j = ((s - (k - 1) + q) % S + S) % S;
      di += c[j] * hdin[(long long)j * total + i];
      dr += c[j] * hdres[(long long)j * total + i];
    }
    const int f = (int)(i / g.n), l = (int)(i % g.n);
    rhof_in[i] = rho_new[global_of_local(g, f, l)] + (di + a * dr);
  }
}

// scal[SC_RES_PAPER] = dV sum of the block partials / N_e
__global__ void __launch_bounds__(256) k_mix_residual(Geo g, int nblk, double ne,
                                                      const double *__restrict__ part,
                                                      double *__restrict__ scal) {
  __shared__ double red[16];
  double t = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) t += part[b];
  t = block_sum(t, red);
  if (threadIdx.x == 0) scal[SC_RES_PAPER] = g.dv * t / ne;
}

inline int grid_for(long long n, int block) {
  long long b = (n + block - 1) / block;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

void launch_fermi(const OrbSet &o, const double *eps, const double *w, double ne, double sigma,
                  double *occ, double *scal, int *flags, hipStream_t s) {
  hipLaunchKernelGGL(k_fermi, dim3(1), dim3(1024), 0, s, o.M_tot, eps, w, ne, sigma, occ, scal,
                     flags);
}

template <typename T>
void launch_density(const Geo &g, const OrbSet &o, int f0, int f1, const T *psi,
                    const double *occ, double *rhof_out, double *rho_out, hipStream_t s) {
  const long long total = (long long)(f1 - f0) * g.n;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_density<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g,
                     o.moff, o.m, f0, f1, psi, occ, rhof_out, rho_out);
}
template void launch_density<double>(const Geo &, const OrbSet &, int, int, const double *,
                                     const double *, double *, double *, hipStream_t);
template void launch_density<float>(const Geo &, const OrbSet &, int, int, const float *,
                                    const double *, double *, double *, hipStream_t);

__global__ void k_to_float(const double *__restrict__ a, float *__restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

__global__ void k_to_double(const float *__restrict__ a, double *__restrict__ b, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = (double)a[i];
}

void launch_convert(const double *a, float *b, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_to_float, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, n);
}

void launch_convert(const float *a, double *b, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_to_double, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, n);
}

void launch_veff(const Geo &g, int f0, int f1, const double *vloc, const double *vh,
                 const double *rhof_in, const double *rho_tot_in, double xi, double *veff,
                 float *veff32, hipStream_t s) {
  const long long total = (long long)(f1 - f0) * g.n;
  if (total <= 0) return;
  if (!(xi > 0.0)) rho_tot_in = nullptr;
  hipLaunchKernelGGL(k_veff, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g, f0, f1,
                     vloc, vh, rhof_in, rho_tot_in, xi, veff, veff32);
}

void launch_global_terms(const Geo &g, double *rho_in, const double *rho_out, const double *vh,
                         double mixing, double *part, int n_part, double *scal, hipStream_t s,
                         double ne, double sigma) {
  hipLaunchKernelGGL(k_global_terms, dim3(n_part), dim3(256), 0, s, g, rho_in, rho_out, vh,
                     mixing, part);
  hipLaunchKernelGGL(k_global_final, dim3(1), dim3(256), 0, s, g, n_part, ne, sigma, part, scal);
}

void launch_frag_mix(const Geo &g, int nfrag, double *rhof_in, const double *rhof_out,
                     double mixing, hipStream_t s) {
  const long long total = (long long)nfrag * g.n;
  hipLaunchKernelGGL(k_frag_mix, dim3(grid_for(total, 256)), dim3(256), 0, s, total, rhof_in,
                     rhof_out, mixing);
}

// out = in contracted with Q (n x n) along the axis of stride C; matrix cores
// when the shape allows it.
static void axis_transform(long long Ng, int n, long long C, const double *in, const double *Q,
                           double *out, hipStream_t s) {
  const long long A = Ng / ((long long)n * C);
  const bool tiles = n % 16 == 0 && (C > 1 ? C % 16 == 0 : A % 16 == 0);
  if (tiles) {
    const long long nt = (long long)(n / 16) * (C > 1 ? A * (C / 16) : A / 16);
    hipLaunchKernelGGL(k_axis_mfma, dim3((unsigned)((nt + 3) / 4)), dim3(256), 0, s, A, n, C, in,
                       Q, out);
  } else {
    hipLaunchKernelGGL(k_axis_transform, dim3(grid_for(Ng, 256)), dim3(256), 0, s, Ng, n, C, in,
                       Q, out);
  }
}

void launch_poisson(const Geo &g, const double *rho, double *vh, double *wa, double *wb,
                    double *const qf[3], double *const qi[3], double *const lam[3],
                    hipStream_t s) {
  const long long Ng = g.Ng;
  const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
  const int gb = grid_for(Ng, 256);
  // forward: x (C = 1), y (C = Nx), z (C = Nx Ny)
  axis_transform(Ng, Nx, 1LL, rho, qf[0], wa, s);
  axis_transform(Ng, Ny, (long long)Nx, wa, qf[1], wb, s);
  axis_transform(Ng, Nz, (long long)Nx * Ny, wb, qf[2], wa, s);
  hipLaunchKernelGGL(k_poisson_scale, dim3(gb), dim3(256), 0, s, g, lam[0], lam[1], lam[2], wa);
  axis_transform(Ng, Nz, (long long)Nx * Ny, wa, qi[2], wb, s);
  axis_transform(Ng, Ny, (long long)Nx, wb, qi[1], wa, s);
  axis_transform(Ng, Nx, 1LL, wa, qi[0], vh, s);
}

void launch_fill(double *p, long long n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
}

void launch_fill_int(int *p, long long n, int v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_int, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
}

void launch_nan_check(const double *p, long long n, int *flags, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_nan_check, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, flags);
}

void launch_pulay_mix(const Geo &g, int nfrag, const MixState &m, const double *rho_out,
                      const double *rhof_out, double *rho_in, double *rhof_in, double ne,
                      double *const qf[3], double *const qi[3], double *const lam[3],
                      double *wa, double *wb, double *scal, hipStream_t s) {
  const int nblk = m.nblk;
  const long long fn = (long long)nfrag * g.n;
  hipLaunchKernelGGL(k_mix_record, dim3(nblk), dim3(256), 0, s, g, m.S, m.st, rho_in, rho_out,
                     m.hrho, m.hres, m.part);
  hipLaunchKernelGGL(k_mix_record_frag, dim3(grid_for(fn, 256)), dim3(256), 0, s, g, nfrag,
                     m.S, m.st, rho_in, rho_out, rhof_in, rhof_out, m.hdin, m.hdres);
  hipLaunchKernelGGL(k_mix_solve, dim3(1), dim3(64), 0, s, m.S, m.H, nblk, m.st, m.part, m.A,
                     m.c);
  hipLaunchKernelGGL(k_mix_combine, dim3(grid_for(g.Ng, 256)), dim3(256), 0, s, g, m.S, m.st,
                     m.c, m.hrho, m.hres, m.rbar, m.kres);
  if (m.q0 > 0.0) {
    // K R_bar through the real Fourier basis of the Poisson solve
    const long long Ng = g.Ng;
    const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
    axis_transform(Ng, Nx, 1LL, m.kres, qf[0], wa, s);
    axis_transform(Ng, Ny, (long long)Nx, wa, qf[1], wb, s);
    axis_transform(Ng, Nz, (long long)Nx * Ny, wb, qf[2], wa, s);
    hipLaunchKernelGGL(k_kerker_scale, dim3(grid_for(Ng, 256)), dim3(256), 0, s, g, lam[0],
                       lam[1], lam[2], m.q0 * m.q0, wa);
    axis_transform(Ng, Nz, (long long)Nx * Ny, wa, qi[2], wb, s);
    axis_transform(Ng, Ny, (long long)Nx, wb, qi[1], wa, s);
    axis_transform(Ng, Nx, 1LL, wa, qi[0], m.kres, s);
  }
  hipLaunchKernelGGL(k_mix_update, dim3(nblk), dim3(256), 0, s, g, m.S, m.st, m.hrho, m.rbar,
                     m.kres, m.alpha, rho_in, m.part);
  hipLaunchKernelGGL(k_mix_update_frag, dim3(grid_for(fn, 256)), dim3(256), 0, s, g, nfrag,
                     m.S, m.st, m.c, m.hdin, m.hdres, rho_in, m.alpha, rhof_in);
  hipLaunchKernelGGL(k_mix_residual, dim3(1), dim3(256), 0, s, g, nblk, ne, m.part, scal);
}

}  // namespace dcdft
