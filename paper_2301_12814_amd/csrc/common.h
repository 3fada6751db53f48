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

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, false);
  const int h2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(h2, l2);
}
template <int CTRL>
__device__ __forceinline__ float dpp_d(float v) {
  const int x = __float_as_int(v);
  return __int_as_float(__builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false));
}

// v plus the value of the lane 16 (ROW16) or 32 lanes away, through the
// gfx950 lane swaps (VALU ops, no LDS crossbar round trip).  Swapping v with
// itself leaves in the first result, in every lane, the value of the lower
// row (half) of its pair and in the second the value of the upper one, so the
// sum is the same expression in both lanes of a pair.
template <bool ROW16>
__device__ __forceinline__ double swap_sum(double v) {
  const unsigned lo = __double2loint(v), hi = __double2hiint(v);
  if (ROW16) {
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
  }
}
template <bool ROW16>
__device__ __forceinline__ float swap_sum(float v) {
  const unsigned x = __float_as_uint(v);
  if (ROW16) {
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
}

// Sum over a group of L lanes: xor 1 and xor 2 inside each quad, the row
// mirror (quad q with quad 3 - q), the half-row mirror (quad 0 with 1, 2
// with 3), then across rows (16 lanes) and halves (32 lanes).  Every step
// adds two values in an order-independent way, so all lanes of the group end
// with bitwise the same sum (the callers branch on it).
template <int L, typename R>
__device__ __forceinline__ R group_sum(R v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x140>(v);
  v += dpp_d<0x141>(v);
  if (L >= 32) v = swap_sum<true>(v);
  if (L >= 64) v = swap_sum<false>(v);
  return v;
}

// Sum over the 64 lanes of a wave (every lane active), the same in every lane.
__device__ inline double wave_sum(double v) { return group_sum<64>(v); }

}  // namespace gbs
