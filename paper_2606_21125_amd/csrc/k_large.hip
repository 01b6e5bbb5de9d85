// Subspace algebra for one fragment with more orbitals than the register- and
// LDS-tiled kernels take (the conventional calculation of a cell, Sec. 3.1's
// comparison): the same CG band update and Rayleigh-Ritz step (Sec. 2.2), with
// the products over the fragment's points as rocBLAS GEMMs, the FP64 Cholesky
// factor, its inverse and the symmetric eigensolve as rocSOLVER routines, and
// the per-band steps (norms, the Fletcher-Reeves direction, the 2x2 minimiser,
// the band rotations) as the kernels below.
//
// Layouts: an orbital array holds m rows of n points (row i contiguous), which
// is the column-major n x m matrix of the BLAS calls with leading dimension n.
// Small matrices are FP64, column-major with leading dimension ld >= m.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "device_common.h"

namespace dcdft {

struct LargeBlas {
  rocblas_handle h = nullptr;
};

namespace {

constexpr int kRowBlock = 256;

// oy[i] = dV <x_i, y_i> and (z not null) oz[i] = dV <x_i, z_i>; core: only the
// fragment's core points count.  One workgroup per row, FP64 sums.
template <typename T>
__global__ void __launch_bounds__(kRowBlock)
    k_large_row_dots(Geo g, const T *__restrict__ x, const T *__restrict__ y,
                     const T *__restrict__ z, double *__restrict__ oy, double *__restrict__ oz,
                     int core) {
  __shared__ double red[kRowBlock / 64];
  const long long base = (long long)blockIdx.x * g.n;
  double ay = 0.0, az = 0.0;
  for (int l = threadIdx.x; l < g.n; l += kRowBlock) {
    if (core && !is_core_point(g, l)) continue;
    const double xv = (double)x[base + l];
    ay += xv * (double)y[base + l];
    if (z) az += xv * (double)z[base + l];
  }
  ay = block_sum(ay, red);
  if (z) az = block_sum(az, red);
  if (threadIdx.x == 0) {
    oy[blockIdx.x] = g.dv * ay;
    if (z) oz[blockIdx.x] = g.dv * az;
  }
}

// P_i = -G_i + beta_i P_prev_i with the Fletcher-Reeves beta_i = gamma_i /
// gamma_prev_i (0 in the first sweep or when gamma_prev_i = 0); pout may be gbuf.
template <typename T>
__global__ void __launch_bounds__(256)
    k_large_direction(int n, const T *gbuf, const T *__restrict__ pprev, T *pout,
                      const double *__restrict__ gamma, const double *__restrict__ gamma_prev,
                      int first) {
  const int i = blockIdx.y;
  const double gp = gamma_prev[i];
  const double beta = (first || !(gp > 0.0)) ? 0.0 : gamma[i] / gp;
  const long long base = (long long)i * n;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n; l += gridDim.x * blockDim.x) {
    const double gv = (double)gbuf[base + l];
    pout[base + l] = (T)(beta == 0.0 ? -gv : -gv + beta * (double)pprev[base + l]);
  }
}

// The exact minimiser of the 2x2 Rayleigh quotient on span(psi_i, p_i / |p_i|):
// a = <psi_i, H psi_i> (diagonal of the unsymmetrised <Psi, W>), b = <p, w> / |p|,
// c = <p, H p> / |p|^2, theta = atan2(-2 b, c - a) / 2; a vanishing direction
// (|p|^2 <= 1e-300) leaves the band as it is.
__global__ void k_large_theta(int m, int ld, const double *__restrict__ hs_full,
                              const double *__restrict__ nu, const double *__restrict__ bb,
                              const double *__restrict__ cc, double *__restrict__ cs,
                              double *__restrict__ sn, double *__restrict__ inv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const bool live = nu[i] > 1e-300;
  const double r = live ? 1.0 / sqrt(nu[i]) : 0.0;
  const double a = hs_full[(long long)i * ld + i];
  const double th = live ? 0.5 * atan2(-2.0 * bb[i] * r, cc[i] * r * r - a) : 0.0;
  cs[i] = cos(th);
  sn[i] = sin(th);
  inv[i] = r;
}

// psi_out = cos psi_in + sin p / |p|, w <- cos w + sin q / |p| (psi_out may be
// psi_in)
template <typename T>
__global__ void __launch_bounds__(256)
    k_large_band_update(int n, const T *psi_in, T *psi_out, T *w, const T *__restrict__ p,
                        const T *__restrict__ q, const double *__restrict__ cs,
                        const double *__restrict__ sn, const double *__restrict__ inv) {
  const int i = blockIdx.y;
  const double c = cs[i], s = sn[i] * inv[i];
  const long long base = (long long)i * n;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n; l += gridDim.x * blockDim.x) {
    const long long e = base + l;
    const double pv = (double)p[e], qv = (double)q[e];
    psi_out[e] = (T)(c * (double)psi_in[e] + s * pv);
    w[e] = (T)(c * (double)w[e] + s * qv);
  }
}

// s = (a + a^T) / 2 on the leading m x m block; diag (not null) = diagonal of a
__global__ void k_large_sym(int m, int ld, const double *__restrict__ a, double *__restrict__ s,
                            double *__restrict__ diag) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)m * m) return;
  const int i = (int)(e % m), j = (int)(e / m);
  s[(long long)j * ld + i] = 0.5 * (a[(long long)j * ld + i] + a[(long long)i * ld + j]);
  if (diag && i == j) diag[i] = a[(long long)i * ld + i];
}

// out = scale * sum_k part_k on the leading m x m block (parts in order, FP64),
// zero in the padding
template <typename P>
__global__ void k_large_reduce_parts(int m, int ld, int nparts, const P *__restrict__ part,
                                     double scale, double *__restrict__ out) {
  const long long mm = (long long)ld * ld;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mm) return;
  const int i = (int)(e % ld), j = (int)(e / ld);
  double acc = 0.0;
  if (i < m && j < m)
    for (int k = 0; k < nparts; ++k) acc += (double)part[k * mm + e];
  out[e] = scale * acc;
}

// Lower triangle kept (the inverse factor), strict upper part and padding zeroed.
// A nonzero info of the factorisation or the inversion raises flag and puts the
// identity in its place, so that the rest of the failed step (whose results are
// discarded) stays finite.
__global__ void k_large_tril(int m, int ld, double *__restrict__ l, const int *__restrict__ info,
                             int *__restrict__ flags, int flag) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool failed = info[0] != 0 || info[1] != 0;
  if (e == 0 && failed) atomicOr(flags, flag);
  if (e >= (long long)ld * ld) return;
  const int i = (int)(e % ld), j = (int)(e / ld);
  if (failed) l[e] = (i == j && i < m) ? 1.0 : 0.0;
  else if (i < j || i >= m || j >= m) l[e] = 0.0;
}

// The eigensolver is iterative: a matrix with a non-finite or overflowing entry
// (|a| > 1e150) raises flag and is replaced by the identity before it.  Scan:
// any workgroup that finds such an entry sets *bad (cleared by the caller);
// fill: with *bad set, the identity and the flag.
__global__ void __launch_bounds__(256)
    k_large_finite_scan(int m, int ld, const double *__restrict__ a, int *__restrict__ bad) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)m * m) return;
  if (!(fabs(a[(e / m) * ld + e % m]) <= 1e150)) atomicOr(bad, 1);
}
__global__ void __launch_bounds__(256)
    k_large_finite_fill(int m, int ld, double *__restrict__ a, const int *__restrict__ bad,
                        int *__restrict__ flags, int flag) {
  if (!*bad) return;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) atomicOr(flags, flag);
  if (e >= (long long)m * m) return;
  const long long i = e % m, j = e / m;
  a[j * ld + i] = i == j ? 1.0 : 0.0;
}

// Each eigenvector (column) flipped so that its largest-magnitude entry, the
// first one on ties, is positive; a nonzero info of the eigensolver raises flag
__global__ void __launch_bounds__(256)
    k_large_signs(int m, int ld, double *__restrict__ u, const int *__restrict__ info,
                  int *__restrict__ flags, int flag) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int j = blockIdx.x;
  if (j == 0 && threadIdx.x == 0 && info[0] != 0) atomicOr(flags, flag);
  double *col = u + (long long)j * ld;
  double best = -1.0;
  int at = m;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double v = fabs(col[i]);
    if (v > best) {   // rows ascend per thread: the first maximum is kept
      best = v;
      at = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = at;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double v = bv[threadIdx.x + off];
      const int k = bi[threadIdx.x + off];
      if (v > bv[threadIdx.x] || (v == bv[threadIdx.x] && k < bi[threadIdx.x])) {
        bv[threadIdx.x] = v;
        bi[threadIdx.x] = k;
      }
    }
    __syncthreads();
  }
  const int k = bi[0];
  const bool flip = k < m && col[k] < 0.0;
  __syncthreads();
  if (flip)
    for (int i = threadIdx.x; i < m; i += blockDim.x) col[i] = -col[i];
}

__global__ void k_large_fill_int(int *p, int v) { *p = v; }

__global__ void k_large_to_float(long long n, const double *__restrict__ a, float *__restrict__ b) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = (float)a[e];
}

inline unsigned blocks_for(long long n, int block) {
  return (unsigned)((n + block - 1) / block);
}

// workgroups along the points of a row for the elementwise kernels
inline dim3 row_grid(int n, int m) {
  const int bx = (int)std::min<long long>(blocks_for(n, 256), 64);
  return dim3((unsigned)bx, (unsigned)m);
}

int gemm(LargeBlas *b, rocblas_operation ta, rocblas_operation tb, int M, int N, int K,
         double alpha, const double *A, int lda, const double *B, int ldb, double beta,
         double *C, int ldc) {
  return (int)rocblas_dgemm(b->h, ta, tb, M, N, K, &alpha, A, lda, B, ldb, &beta, C, ldc);
}
int gemm(LargeBlas *b, rocblas_operation ta, rocblas_operation tb, int M, int N, int K,
         double alpha, const float *A, int lda, const float *B, int ldb, double beta, float *C,
         int ldc) {
  const float af = (float)alpha, bf = (float)beta;
  return (int)rocblas_sgemm(b->h, ta, tb, M, N, K, &af, A, lda, B, ldb, &bf, C, ldc);
}

}  // namespace

LargeBlas *large_create(hipStream_t s, std::string *err) {
  LargeBlas *b = new (std::nothrow) LargeBlas();
  if (!b) {
    *err = "host allocation failed";
    return nullptr;
  }
  rocblas_status st = rocblas_create_handle(&b->h);
  if (st == rocblas_status_success) st = rocblas_set_stream(b->h, s);
  if (st == rocblas_status_success) st = rocblas_set_pointer_mode(b->h, rocblas_pointer_mode_host);
  // no split-K kernels that sum with atomics: every product is reproducible bit
  // for bit (a step repeated from the same state gives the same result)
  if (st == rocblas_status_success) st = rocblas_set_atomics_mode(b->h, rocblas_atomics_not_allowed);
  if (st != rocblas_status_success) {
    *err = std::string("rocBLAS handle: ") + rocblas_status_to_string(st);
    large_destroy(b);
    return nullptr;
  }
  return b;
}

void large_destroy(LargeBlas *b) {
  if (!b) return;
  if (b->h) rocblas_destroy_handle(b->h);
  delete b;
}

const char *large_status_string(int st) {
  return rocblas_status_to_string((rocblas_status)st);
}

int large_gram_parts(int n) { return std::min(kLargeGramParts, std::max(1, n)); }

namespace {

rocblas_status gemm_batched(LargeBlas *b, int M, int N, int K, const double *x, int lx,
                            long long sx, const double *y, int ly, long long sy, double *c,
                            int ldc, long long sc, int batch) {
  const double one = 1.0, zero = 0.0;
  return rocblas_dgemm_strided_batched(b->h, rocblas_operation_transpose, rocblas_operation_none,
                                       M, N, K, &one, x, lx, sx, y, ly, sy, &zero, c, ldc, sc,
                                       batch);
}
rocblas_status gemm_batched(LargeBlas *b, int M, int N, int K, const float *x, int lx,
                            long long sx, const float *y, int ly, long long sy, float *c,
                            int ldc, long long sc, int batch) {
  const float one = 1.0f, zero = 0.0f;
  return rocblas_sgemm_strided_batched(b->h, rocblas_operation_transpose, rocblas_operation_none,
                                       M, N, K, &one, x, lx, sx, y, ly, sy, &zero, c, ldc, sc,
                                       batch);
}

// The products over chunks of the points (one batched GEMM, the remainder in a
// second call), summed in FP64 in chunk order: a Gram product has an m x m
// result and n-long sums, and without split-K kernels (atomics are off) an
// unchunked GEMM would run on a handful of workgroups
template <typename T>
int gram_chunked(LargeBlas *b, int n, int m, int ld, const T *x, const T *y, double dv,
                 double *out, T *part, hipStream_t s) {
  const int parts = large_gram_parts(n);
  const int kc = (n + parts - 1) / parts;
  const int full = n / kc, tail = n - full * kc;
  const long long mm = (long long)ld * ld;
  rocblas_status st = gemm_batched(b, m, m, kc, x, n, kc, y, n, kc, part, ld, mm, full);
  if (st != rocblas_status_success) return (int)st;
  if (tail > 0) {
    st = gemm_batched(b, m, m, tail, x + (long long)full * kc, n, 0, y + (long long)full * kc, n,
                      0, part + full * mm, ld, 0, 1);
    if (st != rocblas_status_success) return (int)st;
  }
  hipLaunchKernelGGL(k_large_reduce_parts<T>, dim3(blocks_for(mm, 256)), dim3(256), 0, s, m, ld,
                     full + (tail > 0 ? 1 : 0), part, dv, out);
  return 0;
}

}  // namespace

int large_gram(LargeBlas *b, int n, int m, int ld, const double *x, const double *y, double dv,
               double *out, void *part, hipStream_t s) {
  return gram_chunked<double>(b, n, m, ld, x, y, dv, out, static_cast<double *>(part), s);
}

int large_gram(LargeBlas *b, int n, int m, int ld, const float *x, const float *y, double dv,
               double *out, void *part, hipStream_t s) {
  return gram_chunked<float>(b, n, m, ld, x, y, dv, out, static_cast<float *>(part), s);
}

int large_rotate(LargeBlas *b, int n, int m, int ld, const double *x, const double *r,
                 bool trans_r, double alpha, double beta, double *out, double *, hipStream_t) {
  return gemm(b, rocblas_operation_none,
              trans_r ? rocblas_operation_transpose : rocblas_operation_none, n, m, m, alpha, x,
              n, r, ld, beta, out, n);
}

int large_rotate(LargeBlas *b, int n, int m, int ld, const float *x, const double *r,
                 bool trans_r, double alpha, double beta, float *out, float *rt, hipStream_t s) {
  const long long mm = (long long)ld * ld;
  hipLaunchKernelGGL(k_large_to_float, dim3(blocks_for(mm, 256)), dim3(256), 0, s, mm, r, rt);
  return gemm(b, rocblas_operation_none,
              trans_r ? rocblas_operation_transpose : rocblas_operation_none, n, m, m, alpha, x,
              n, rt, ld, beta, out, n);
}

int large_chol_inverse(LargeBlas *b, int m, int ld, double *s, int *info, int *flags,
                       hipStream_t st) {
  rocblas_status e = rocsolver_dpotrf(b->h, rocblas_fill_lower, m, s, ld, info);
  if (e == rocblas_status_success)
    e = rocsolver_dtrtri(b->h, rocblas_fill_lower, rocblas_diagonal_non_unit, m, s, ld, info + 1);
  if (e != rocblas_status_success) return (int)e;
  const long long mm = (long long)ld * ld;
  hipLaunchKernelGGL(k_large_tril, dim3(blocks_for(mm, 256)), dim3(256), 0, st, m, ld, s, info,
                     flags, (int)FLAG_NOT_SPD);
  return 0;
}

int large_eigh(LargeBlas *b, int m, int ld, double *a, double *eps, double *e_work, int *info,
               int *flags, hipStream_t st) {
  // info[1] holds the scan's finding (info[0] is the eigensolver's)
  const unsigned nb = blocks_for((long long)m * m, 256);
  hipLaunchKernelGGL(k_large_fill_int, dim3(1), dim3(1), 0, st, info + 1, 0);
  hipLaunchKernelGGL(k_large_finite_scan, dim3(nb), dim3(256), 0, st, m, ld, a, info + 1);
  hipLaunchKernelGGL(k_large_finite_fill, dim3(nb), dim3(256), 0, st, m, ld, a, info + 1, flags,
                     (int)FLAG_NAN);
  rocblas_status e = rocsolver_dsyevd(b->h, rocblas_evect_original, rocblas_fill_lower, m, a, ld,
                                      eps, e_work, info);
  if (e != rocblas_status_success) return (int)e;
  hipLaunchKernelGGL(k_large_signs, dim3((unsigned)m), dim3(256), 0, st, m, ld, a, info, flags,
                     (int)FLAG_EIG);
  return 0;
}

template <typename T>
void launch_large_row_dots(const Geo &g, int m, const T *x, const T *y, const T *z, double *oy,
                           double *oz, bool core, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_large_row_dots<T>, dim3((unsigned)m), dim3(kRowBlock), 0, s, g, x, y, z,
                     oy, oz, core ? 1 : 0);
}

template <typename T>
void launch_large_direction(const Geo &g, int m, const T *gbuf, const T *pprev, T *pout,
                            const double *gamma, const double *gamma_prev, bool first,
                            hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_large_direction<T>, row_grid(g.n, m), dim3(256), 0, s, g.n, gbuf, pprev,
                     pout, gamma, gamma_prev, first ? 1 : 0);
}

void launch_large_theta(int m, int ld, const double *hs_full, const double *nu, const double *bb,
                        const double *cc, double *cs, double *sn, double *inv, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_large_theta, dim3(blocks_for(m, 256)), dim3(256), 0, s, m, ld, hs_full, nu,
                     bb, cc, cs, sn, inv);
}

template <typename T>
void launch_large_band_update(const Geo &g, int m, const T *psi_in, T *psi_out, T *w, const T *p,
                              const T *q, const double *cs, const double *sn, const double *inv,
                              hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_large_band_update<T>, row_grid(g.n, m), dim3(256), 0, s, g.n, psi_in,
                     psi_out, w, p, q, cs, sn, inv);
}

void launch_large_sym(int m, int ld, const double *a, double *s_out, double *diag, hipStream_t s) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_large_sym, dim3(blocks_for((long long)m * m, 256)), dim3(256), 0, s, m, ld,
                     a, s_out, diag);
}

#define DCDFT_LARGE_INST(T)                                                                    \
  template void launch_large_row_dots<T>(const Geo &, int, const T *, const T *, const T *,      \
                                         double *, double *, bool, hipStream_t);               \
  template void launch_large_direction<T>(const Geo &, int, const T *, const T *, T *,           \
                                          const double *, const double *, bool, hipStream_t);  \
  template void launch_large_band_update<T>(const Geo &, int, const T *, T *, T *, const T *,    \
                                            const T *, const double *, const double *,         \
                                            const double *, hipStream_t);
DCDFT_LARGE_INST(double)
DCDFT_LARGE_INST(float)
#undef DCDFT_LARGE_INST

}  // namespace dcdft
