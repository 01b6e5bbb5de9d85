// Device helpers shared by the kernel files: deterministic reductions and the
// MFMA 16x16x4 operations for the two storage precisions of orbital arrays.
#pragma once

#include "dcdft_internal.h"

namespace dcdft {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// 1/x and 1/sqrt(x) in FP64: the hardware estimate refined by two Newton steps
// (each doubles the correct bits; the result is within about an ulp).  For
// finite nonzero x; rsqrt_f64 needs x > 0.
__device__ inline double rcp_f64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}
__device__ inline double rsqrt_f64(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = r * fma(-h * r, r, 1.5);
  return r * fma(-h * r, r, 1.5);
}

// Workgroups are dealt to the eight XCDs in turn (linear id mod 8), and each XCD
// has its own L2.  xcd_ordered(b, n) is the work item workgroup b of n takes so
// that every XCD works through one contiguous range of items (a bijection on
// [0, n)): neighbouring items, which read the same inputs (the orbitals of one
// fragment read its V_eff), are then cached in one L2 instead of eight.
__device__ inline unsigned xcd_ordered(unsigned b, unsigned n) {
  constexpr unsigned kXcd = 8;
  const unsigned q = n / kXcd, r = n % kXcd, x = b % kXcd;
  return x * q + (x < r ? x : r) + b / kXcd;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block sum (fixed shuffle tree, waves combined in index order);
// red must hold one double per wave.  Every thread receives the total.
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

// 16x16x4 matrix-core products on gfx950.  For both precisions the operand lanes
// are A[l % 16][l / 16] and B[l / 16][l % 16] (one value per lane); the result
// rows differ (checked on the device):
//   f64: lane l, register r holds D[l / 16 + 4 r][l % 16]
//   f32: lane l, register r holds D[4 (l / 16) + r][l % 16]
template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef dbl4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int kk, int r) { return kk + 4 * r; }
  // row(kk, r) = row_u(r) + row_l(kk): wave-uniform and lane parts
  __device__ static inline int row_u(int r) { return 4 * r; }
  __device__ static inline int row_l(int kk) { return kk; }
};

template <>
struct Mfma<float> {
  typedef flt4 acc_t;
  __device__ static inline acc_t zero() { return acc_t{0.0f, 0.0f, 0.0f, 0.0f}; }
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int kk, int r) { return 4 * kk + r; }
  __device__ static inline int row_u(int r) { return r; }
  __device__ static inline int row_l(int kk) { return 4 * kk; }
};

// LDS row stride for an MP-wide operand block: the smallest S >= MP with
// S = 16 (mod 32) elements, so the four 16-lane groups of an operand read fall
// on different bank ranges.
__host__ __device__ constexpr int lds_stride(int mp) { return mp + ((16 - mp % 32) + 32) % 32; }

__device__ inline bool is_core_point(const Geo &g, int l) {
  const int lx = l % g.nl[0], ly = (l / g.nl[0]) % g.nl[1], lz = l / (g.nl[0] * g.nl[1]);
  return lx >= g.b[0] && lx < g.b[0] + g.nc[0] && ly >= g.b[1] && ly < g.b[1] + g.nc[1] &&
         lz >= g.b[2] && lz < g.b[2] + g.nc[2];
}

}  // namespace dcdft
