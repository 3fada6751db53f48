// Workgroup-wide primitives: exclusive scan and the size-weighted top-chi
// radix select used by the truncation rule.
#pragma once

#include "common.h"

namespace gbs {

// Exclusive scan of one value per thread over the whole workgroup
// (blockDim.x a multiple of 64, at most 1024).  s_tmp needs 17 slots.
template <typename T>
__device__ inline T block_exclusive_scan(T v, T *s_tmp, T &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  T x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_tmp[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    T acc = 0;
    for (int w = 0; w < nw; ++w) {
      T t = s_tmp[w];
      s_tmp[w] = acc;
      acc += t;
    }
    s_tmp[16] = acc;
  }
  __syncthreads();
  T res = s_tmp[wave] + x - v;
  total = s_tmp[16];
  __syncthreads();
  return res;
}

// Result of the truncation select: a unit u is kept iff
//   bits(u) > vb  or  (bits(u) == vb and key(u) <= kstar).
struct SelectResult {
  unsigned long long vb;
  unsigned long long kstar;
};

constexpr int TIE_CAP = 1024;

// Size-weighted selection of the first units, in the order
// (value descending, key ascending), whose running size stays <= chi; the first
// unit that does not fit ends the selection.  Units with value bits 0 never
// exist (values are >= the rank cut > 0).  Runs on the whole workgroup.
// uval/ukey/usize: U units in global memory.
__device__ inline SelectResult topk_select(const unsigned long long *uval,
                                           const unsigned long long *ukey, const int *usize,
                                           int U, int chi, int *err) {
  __shared__ int s_hist[256];
  __shared__ unsigned long long s_prefix, s_mask;
  __shared__ int s_taken, s_state;  // state: 0 searching, 1 all fit
  __shared__ int s_ntie;
  __shared__ unsigned long long s_tkey[TIE_CAP];
  __shared__ int s_tsize[TIE_CAP];
  __shared__ unsigned long long s_kstar;
  if (threadIdx.x == 0) {
    s_prefix = 0;
    s_mask = 0;
    s_taken = 0;
    s_state = 0;
    s_ntie = 0;
  }
  __syncthreads();
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    for (int i = threadIdx.x; i < 256; i += blockDim.x) s_hist[i] = 0;
    __syncthreads();
    const unsigned long long pre = s_prefix, msk = s_mask;
    for (int u = threadIdx.x; u < U; u += blockDim.x) {
      unsigned long long v = uval[u];
      if ((v & msk) == pre) atomicAdd(&s_hist[(v >> shift) & 255], usize[u]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int taken = s_taken;
      int found = -1;
      for (int dg = 255; dg >= 0; --dg) {
        if (taken + s_hist[dg] > chi) {
          found = dg;
          break;
        }
        taken += s_hist[dg];
      }
      if (found < 0) {
        // Everything inside the current prefix fits.  In pass 0 this means all
        // units fit; later it cannot happen (the bucket chosen before overflowed).
        s_state = 1;
      } else {
        s_prefix = pre | ((unsigned long long)found << shift);
        s_mask = msk | (255ull << shift);
        s_taken = taken;
      }
    }
    __syncthreads();
    if (s_state == 1) break;
  }
  SelectResult res;
  if (s_state == 1) {
    res.vb = 0;
    res.kstar = ~0ull;
    return res;
  }
  // ties at the boundary value: keep them in key order while they fit
  const unsigned long long vb = s_prefix;
  for (int u = threadIdx.x; u < U; u += blockDim.x) {
    if (uval[u] == vb) {
      int slot = atomicAdd(&s_ntie, 1);
      if (slot < TIE_CAP) {
        s_tkey[slot] = ukey[u];
        s_tsize[slot] = usize[u];
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nt = s_ntie;
    if (nt > TIE_CAP) {
      atomicOr(err, ERR_TIE_OVERFLOW);
      nt = TIE_CAP;
    }
    // insertion sort by key (tie counts are tiny)
    for (int i = 1; i < nt; ++i) {
      unsigned long long k = s_tkey[i];
      int sz = s_tsize[i];
      int j = i - 1;
      while (j >= 0 && s_tkey[j] > k) {
        s_tkey[j + 1] = s_tkey[j];
        s_tsize[j + 1] = s_tsize[j];
        --j;
      }
      s_tkey[j + 1] = k;
      s_tsize[j + 1] = sz;
    }
    int taken = s_taken;
    unsigned long long kstar = 0;
    bool any = false;
    for (int i = 0; i < nt; ++i) {
      if (taken + s_tsize[i] > chi) break;
      taken += s_tsize[i];
      kstar = s_tkey[i];
      any = true;
    }
    // kstar = 0 with no kept tie: keys are > 0 by construction (see callers)
    s_kstar = any ? kstar : 0ull;
  }
  __syncthreads();
  res.vb = vb;
  res.kstar = s_kstar;
  return res;
}

__device__ inline bool unit_kept(const SelectResult &sr, unsigned long long v,
                                 unsigned long long key) {
  return v > sr.vb || (v == sr.vb && key <= sr.kstar);
}

}  // namespace gbs
