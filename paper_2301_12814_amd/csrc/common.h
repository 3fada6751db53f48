// Device-side helpers shared by the gfx950 kernels of libgbsmpo.
//
// Charges.  A bond charge is the pair (n, n') of ket and bra photons to the
// right of the bond (App. D).  It is packed into one int as (n << 16) | n',
// so that the integer order is the lexicographic order of (n, n'); bonds are
// stored sorted by this key, which makes every charge window
// {n in [a, b], n' in [c, e]} a union of at most (b - a + 1) contiguous runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GBS_WAVE 64

namespace gbs {

// 16-byte aligned so that one lane moves a whole element with one 128-bit
// access (two 64-bit halves at a 16-byte lane stride hit every LDS bank twice).
struct __attribute__((aligned(16))) cd {
  double re, im;
};

__host__ __device__ inline cd cmk(double r, double i) { return cd{r, i}; }
__host__ __device__ inline cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cd csub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cd cmul(cd a, cd b) {
  return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
__host__ __device__ inline cd cmulc(cd a, cd b) {
  return cd{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__host__ __device__ inline cd cconj(cd a) { return cd{a.re, -a.im}; }
__host__ __device__ inline cd cscale(cd a, double s) { return cd{a.re * s, a.im * s}; }
__host__ __device__ inline double cabs2(cd a) { return a.re * a.re + a.im * a.im; }
// acc += a * b
__host__ __device__ inline void cfma(cd &acc, cd a, cd b) {
  acc.re = fma(a.re, b.re, fma(-a.im, b.im, acc.re));
  acc.im = fma(a.re, b.im, fma(a.im, b.re, acc.im));
}

// Single-precision complex (the mixed-precision Jacobi's LDS operand).
struct __attribute__((aligned(8))) cf {
  float re, im;
};

__host__ __device__ inline cf cfmk(float r, float i) { return cf{r, i}; }
__host__ __device__ inline cf cadd(cf a, cf b) { return cf{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cf csub(cf a, cf b) { return cf{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cf cmul(cf a, cf b) {
  return cf{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cf cconj(cf a) { return cf{a.re, -a.im}; }
__host__ __device__ inline cf cscale(cf a, float s) { return cf{a.re * s, a.im * s}; }
__host__ __device__ inline float cabs2(cf a) { return a.re * a.re + a.im * a.im; }

// Conversions between the two precisions (the global operands stay FP64).
template <typename T> __host__ __device__ inline T to_c(cd a);
template <> __host__ __device__ inline cd to_c<cd>(cd a) { return a; }
template <> __host__ __device__ inline cf to_c<cf>(cd a) { return cf{(float)a.re, (float)a.im}; }
__host__ __device__ inline cd to_cd(cd a) { return a; }
__host__ __device__ inline cd to_cd(cf a) { return cd{(double)a.re, (double)a.im}; }

// Real scalar type of a complex type.
template <typename T> struct real_of;
template <> struct real_of<cd> { using type = double; };
template <> struct real_of<cf> { using type = float; };

__host__ __device__ inline int pack_charge(int n, int np) { return (n << 16) | np; }
__host__ __device__ inline int charge_n(int c) { return c >> 16; }
__host__ __device__ inline int charge_np(int c) { return c & 0xffff; }

// Sentinel stored past the end of a bond: larger than every real charge.
constexpr int CHARGE_NONE = 0x7fffffff;

// First index in sorted c[0, D) whose value is >= key.
__device__ inline int lower_bound(const int *c, int D, int key) {
  int lo = 0, hi = D;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (c[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Device error bits, latched in the handle and reported by the next
// synchronising call.
enum : int {
  ERR_SVD_NOT_CONVERGED = 1,
  ERR_NONFINITE = 2,
  ERR_BOX_OVERFLOW = 4,
  ERR_TIE_OVERFLOW = 8,
  ERR_WORKSPACE = 16,
};

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, GBS_WAVE);
  return v;
}

}  // namespace gbs
