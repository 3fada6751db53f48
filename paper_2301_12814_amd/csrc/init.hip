// Initial lossy squeezed product state in U(1) Vidal form.
//
// Per mode (App. C input wavefunction; App. B pure-loss Kraus channel):
//   psi[2n] = tanh(r)^n sqrt((2n)!) / (2^n n!) / sqrt(cosh r),
//   rho[m][m'] = sum_l k(m,l) k(m',l) psi[m+l] psi[m'+l],
//   k(m,l) = sqrt(binom(m+l, m) eta^m (1-eta)^l),
// evaluated in an internal Fock space of nint levels, then cropped to [0,d)^2.
//
// Product state with the auxiliary total-charge leg (App. D charges; App. A:
// the leftmost bond's charge counts every photon): every bond has one Schmidt
// vector per right charge q, with
//   lam_b[q] = A_b sqrt(w_b(q)),  A_b = prod_{j<b} ||rho_j||_F,
//   w_b = |rho_b|^2 (*) w_{b+1}   (2-D convolution, w_M = delta_0),
//   Gamma_j[q', q] = rho_j[q' - q] A_j / (A_{j+1} lam_j[q']).
// Every bond keeps its top-chi charges under the mirror-pair rule.
//
// Total photon cap K (App. A reading in which the cutoff bounds the total
// photon number): the state is projected onto at most K photons in ket and
// in bra, i.e. the aux charge Q = p + q (p: photons left of the bond, q: right)
// stays <= K.  The left factor A_b^2 becomes V_b(q) = sum_{p <= K - q} u_b(p),
// u_b the 2-D convolution of |rho_j|^2 over j < b (u_0 = delta_0), so
//   lam_b[q] = sqrt(w_b(q) V_b(q))  (q <= K),
//   Gamma_j[q', q] = rho_j[q' - q] sqrt(V_j(q')) / (sqrt(V_{j+1}(q)) lam_j[q']).
#include "blockops.h"
#include "internal.h"

namespace gbs {

__global__ void k_init_rho(const double *r, const int *nint, double eta, int d, double *rho) {
  const int j = blockIdx.x;
  const double rj = r[j];
  const int N = nint[j];
  const double t = tanh(rj);
  const double lt = (t > 0.0) ? log(t) : 0.0;
  const double lch = log(cosh(rj));
  const double le = log(eta);
  const double l1e = (eta < 1.0) ? log1p(-eta) : 0.0;
  for (int idx = threadIdx.x; idx < d * d; idx += blockDim.x) {
    const int m = idx / d, mp = idx % d;
    double acc = 0.0;
    if (((m - mp) & 1) == 0) {
      for (int l = 0; m + l < N && mp + l < N; ++l) {
        const int a = m + l, b = mp + l;
        if (a & 1) continue;                      // psi vanishes on odd levels
        if (l > 0 && eta >= 1.0) break;           // no loss: only l = 0
        if (t == 0.0 && (a > 0 || b > 0)) continue;
        const int na = a / 2, nb = b / 2;
        const double lpa = (t > 0.0 ? na * lt : 0.0) + 0.5 * lgamma(a + 1.0) - na * M_LN2 -
                           lgamma(na + 1.0) - 0.5 * lch;
        const double lpb = (t > 0.0 ? nb * lt : 0.0) + 0.5 * lgamma(b + 1.0) - nb * M_LN2 -
                           lgamma(nb + 1.0) - 0.5 * lch;
        const double lka = 0.5 * (lgamma(a + 1.0) - lgamma(m + 1.0) - lgamma(l + 1.0) +
                                  (m > 0 ? m * le : 0.0) + (l > 0 ? l * l1e : 0.0));
        const double lkb = 0.5 * (lgamma(b + 1.0) - lgamma(mp + 1.0) - lgamma(l + 1.0) +
                                  (mp > 0 ? mp * le : 0.0) + (l > 0 ? l * l1e : 0.0));
        // sign of psi[2n] is sign(tanh r)^n = + for r >= 0; the two factors are
        // grouped so that rho[m][m'] and rho[m'][m] round identically
        acc += exp((lka + lpa) + (lkb + lpb));
      }
    }
    rho[(size_t)j * d * d + idx] = acc;
  }
}

hipError_t launch_init_rho(const double *r, const int *nint, double eta, int M, int d,
                           double *rho, hipStream_t s) {
  hipLaunchKernelGGL(k_init_rho, dim3(M), dim3(256), 0, s, r, nint, eta, d, rho);
  return hipGetLastError();
}

__global__ void k_init_norms(const double *rho, int M, int d, double *A) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double acc = 1.0;
  A[0] = 1.0;
  for (int j = 0; j < M; ++j) {
    double f = 0.0;
    for (int i = 0; i < d * d; ++i) f += rho[(size_t)j * d * d + i] * rho[(size_t)j * d * d + i];
    acc *= sqrt(f);
    A[j + 1] = acc;
  }
}

hipError_t launch_init_norms(const double *rho, int M, int d, double *A, hipStream_t s) {
  hipLaunchKernelGGL(k_init_norms, dim3(1), dim3(64), 0, s, rho, M, d, A);
  return hipGetLastError();
}

// w_b[q0][q1] = sum_{m,m'} w_{b+1}[q0-m][q1-m'] rho_b[m][m']^2 on a W_b x W_b grid,
// W_b = (M-b)(d-1)+1.  rho_b is symmetric, so w_b is; each canonical cell
// q0 <= q1 is computed once and written to both mirror cells, which keeps the
// mirror charges' Schmidt values bitwise equal.
__global__ void k_init_conv(const double *rho, int M, int d, int b, const long long *woff,
                            double *w) {
  const int Wb = (M - b) * (d - 1) + 1;
  const int Wn = (M - b - 1) * (d - 1) + 1;
  const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= (long long)Wb * Wb) return;
  const int q0 = (int)(cell / Wb), q1 = (int)(cell % Wb);
  if (q0 > q1) return;
  const double *wn = w + woff[b + 1];
  const double *rb = rho + (size_t)b * d * d;
  double acc = 0.0;
  for (int m = 0; m < d; ++m) {
    const int p0 = q0 - m;
    if (p0 < 0 || p0 >= Wn) continue;
    for (int mp = 0; mp < d; ++mp) {
      const int p1 = q1 - mp;
      if (p1 < 0 || p1 >= Wn) continue;
      const double x = rb[m * d + mp];
      acc = fma(wn[(long long)p0 * Wn + p1], x * x, acc);
    }
  }
  w[woff[b] + cell] = acc;
  w[woff[b] + (long long)q1 * Wb + q0] = acc;
}

hipError_t launch_init_conv(const double *rho, int M, int d, int b, const long long *woff,
                            double *w, hipStream_t s) {
  const long long Wb = (long long)(M - b) * (d - 1) + 1;
  const long long n = Wb * Wb;
  hipLaunchKernelGGL(k_init_conv, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rho, M, d,
                     b, woff, w);
  return hipGetLastError();
}

// Left weights of the total cap K: V[b][x0][x1] = sum_{p <= (K - x0, K - x1)}
// u_b(p) for every bond b, on the (K+1)^2 grid (indexed by x = K - q).  One
// workgroup walks the bonds; each canonical cell (x0 <= x1) is computed once
// and copied to its mirror, so mirror charges get bitwise equal values.
__global__ __launch_bounds__(256) void k_init_left(const double *rho, int M, int d, int K,
                                                   double *V) {
  const int W = K + 1;
  __shared__ double s_u[2][16 * 16];
  for (int c = threadIdx.x; c < W * W; c += blockDim.x) s_u[0][c] = c == 0 ? 1.0 : 0.0;
  __syncthreads();
  for (int b = 0; b <= M; ++b) {
    const double *u = s_u[b & 1];
    double *Vb = V + (size_t)b * W * W;
    for (int c = threadIdx.x; c < W * W; c += blockDim.x) {
      const int x0 = c / W, x1 = c % W;
      if (x0 > x1) continue;
      // q = (K - x0, K - x1); admissible left charges p <= (x0, x1)
      double acc = 0.0;
      for (int p0 = 0; p0 <= x0; ++p0)
        for (int p1 = 0; p1 <= x1; ++p1) acc += u[p0 * W + p1];
      Vb[x0 * W + x1] = acc;
      Vb[x1 * W + x0] = acc;
    }
    if (b == M) break;
    double *un = s_u[(b + 1) & 1];
    const double *rb = rho + (size_t)b * d * d;
    for (int c = threadIdx.x; c < W * W; c += blockDim.x) {
      const int p0 = c / W, p1 = c % W;
      if (p0 > p1) continue;
      double acc = 0.0;
      for (int m = 0; m < d && m <= p0; ++m)
        for (int mp = 0; mp < d && mp <= p1; ++mp) {
          const double x = rb[m * d + mp];
          acc = fma(u[(p0 - m) * W + (p1 - mp)], x * x, acc);
        }
      un[p0 * W + p1] = acc;
      un[p1 * W + p0] = acc;
    }
    __syncthreads();
  }
}

hipError_t launch_init_left(const double *rho, int M, int d, int K, double *V, hipStream_t s) {
  if (K < 0 || K > 15) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_init_left, dim3(1), dim3(256), 0, s, rho, M, d, K, V);
  return hipGetLastError();
}

// Schmidt value of cell c = (q0, q1) of bond b: A_b sqrt(w_b(q)) without a
// cap, sqrt(w_b(q) V_b(q)) with the total cap K (0 above the cap).
__device__ inline double init_value(const double *wb, long long c, int Wb, double Ab,
                                    const double *Vb, int K) {
  if (K < 0) return Ab * sqrt(wb[c]);
  const int q0 = (int)(c / Wb), q1 = (int)(c % Wb);
  if (q0 > K || q1 > K) return 0.0;
  return sqrt(wb[c] * Vb[(K - q0) * (K + 1) + (K - q1)]);
}

// One workgroup per bond: keep the top-chi charges (mirror-pair rule) and
// write the sorted bond.  Units are the canonical cells q0 <= q1.
__global__ __launch_bounds__(1024) void k_init_select(State st, const double *w,
                                                      const long long *woff, const double *A,
                                                      unsigned long long *uval,
                                                      unsigned long long *ukey, int *usize,
                                                      long long ucap, const double *V, int K) {
  const int b = blockIdx.x;
  const int M = st.M, d = st.d, chi = st.chi;
  const int Wb = (M - b) * (d - 1) + 1;
  const long long ncell = (long long)Wb * Wb;
  const double *wb = w + woff[b];
  const double Ab = A[b];
  const double *Vb = K >= 0 ? V + (size_t)b * (K + 1) * (K + 1) : nullptr;
  unsigned long long *uv = uval + (long long)b * ucap;
  unsigned long long *uk = ukey + (long long)b * ucap;
  int *us = usize + (long long)b * ucap;
  __shared__ double s_max;
  __shared__ long long s_scan[17];
  // largest Schmidt value of the bond
  double lmax = 0.0;
  for (long long c = threadIdx.x; c < ncell; c += blockDim.x)
    lmax = fmax(lmax, init_value(wb, c, Wb, Ab, Vb, K));
  if (threadIdx.x == 0) s_max = 0.0;
  __syncthreads();
  atomicMax((unsigned long long *)&s_max, (unsigned long long)__double_as_longlong(lmax));
  __syncthreads();
  const double cut = 1e-14 * s_max;
  // units, one per canonical cell with a member above the cut (cell order)
  long long base = 0;
  for (long long c0 = 0; c0 < ncell; c0 += blockDim.x) {
    const long long c = c0 + threadIdx.x;
    long long flag = 0;
    double vq = 0.0, vm = 0.0;
    int q0 = 0, q1 = 0;
    if (c < ncell) {
      q0 = (int)(c / Wb);
      q1 = (int)(c % Wb);
      if (q0 <= q1) {
        vq = init_value(wb, c, Wb, Ab, Vb, K);
        vm = init_value(wb, (long long)q1 * Wb + q0, Wb, Ab, Vb, K);
        const int sz = (vq >= cut && vq > 0.0) + ((q0 != q1) && vm >= cut && vm > 0.0);
        flag = sz > 0;
      }
    }
    long long tot;
    const long long pos = base + block_exclusive_scan<long long>(flag, s_scan, tot);
    if (flag) {
      const bool okq = vq >= cut && vq > 0.0;
      const bool okm = (q0 != q1) && vm >= cut && vm > 0.0;
      const double v = fmax(okq ? vq : 0.0, okm ? vm : 0.0);
      uv[pos] = (unsigned long long)__double_as_longlong(v);
      uk[pos] = ((unsigned long long)(pack_charge(q0, q1) + 1) << 20);
      us[pos] = (int)okq + (int)okm;
    }
    base += tot;
  }
  __syncthreads();
  const int U = (int)base;
  const SelectResult sr = topk_select(uv, uk, us, U, chi, st.err);
  // keep flags per cell, compaction in charge order
  int *chg = st.chg + (size_t)b * chi;
  double *lam = st.lam + (size_t)b * chi;
  long long outb = 0;
  for (long long c0 = 0; c0 < ncell; c0 += blockDim.x) {
    const long long c = c0 + threadIdx.x;
    long long flag = 0;
    double v = 0.0;
    int q0 = 0, q1 = 0;
    if (c < ncell) {
      q0 = (int)(c / Wb);
      q1 = (int)(c % Wb);
      v = init_value(wb, c, Wb, Ab, Vb, K);
      if (v >= cut && v > 0.0) {
        const int c0m = min(q0, q1), c1m = max(q0, q1);
        const double vo = init_value(wb, (long long)q1 * Wb + q0, Wb, Ab, Vb, K);
        const bool oko = (q0 != q1) && vo >= cut && vo > 0.0;
        const double uvv = fmax(v, oko ? vo : 0.0);
        const unsigned long long key = ((unsigned long long)(pack_charge(c0m, c1m) + 1) << 20);
        flag = unit_kept(sr, (unsigned long long)__double_as_longlong(uvv), key);
      }
    }
    long long tot;
    const long long pos = outb + block_exclusive_scan<long long>(flag, s_scan, tot);
    if (flag && pos < chi) {
      chg[pos] = pack_charge(q0, q1);
      lam[pos] = v;
    }
    outb += tot;
  }
  __syncthreads();
  const int D = (int)min(outb, (long long)chi);
  for (int i = D + threadIdx.x; i < chi; i += blockDim.x) {
    chg[i] = CHARGE_NONE;
    lam[i] = 0.0;
  }
  if (threadIdx.x == 0) st.dim[b] = D;
}

hipError_t launch_init_select(State st, const double *w, const long long *woff, const double *A,
                              unsigned long long *uval, unsigned long long *ukey, int *usize,
                              long long ucap, const double *V, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_init_select, dim3(st.M + 1), dim3(1024), 0, s, st, w, woff, A, uval, ukey,
                     usize, ucap, V, K);
  return hipGetLastError();
}

// Gamma_j[a][b] = rho_j[c_a - c_b] A_j / (A_{j+1} lam_j[a]) when the charge
// difference is a valid local pair, else 0 (padding included); with the total
// cap K the factor A_j / A_{j+1} is sqrt(V_j(c_a)) / sqrt(V_{j+1}(c_b)).
__global__ void k_init_gamma(State st, const double *rho, const double *A, const double *V,
                             int K) {
  const int j = blockIdx.y;
  const int chi = st.chi, d = st.d;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)chi * chi) return;
  const int a = (int)(idx / chi), b = (int)(idx % chi);
  const int Dl = st.dim[j], Dr = st.dim[j + 1];
  cd v = cmk(0.0, 0.0);
  if (a < Dl && b < Dr) {
    const int ca = st.chg[(size_t)j * chi + a], cb = st.chg[(size_t)(j + 1) * chi + b];
    const int m = charge_n(ca) - charge_n(cb), mp = charge_np(ca) - charge_np(cb);
    if (m >= 0 && m < d && mp >= 0 && mp < d) {
      const double x = rho[(size_t)j * d * d + m * d + mp];
      const double la = st.lam[(size_t)j * chi + a];
      if (K < 0) {
        v.re = x * A[j] / (A[j + 1] * la);
      } else {
        const int W = K + 1;
        const double va = V[(size_t)j * W * W + (K - charge_n(ca)) * W + (K - charge_np(ca))];
        const double vb =
            V[(size_t)(j + 1) * W * W + (K - charge_n(cb)) * W + (K - charge_np(cb))];
        v.re = x * sqrt(va) / (sqrt(vb) * la);
      }
    }
  }
  st.gam[(size_t)j * chi * chi + idx] = v;
}

hipError_t launch_init_gamma(State st, const double *rho, const double *A, const double *V, int K,
                             hipStream_t s) {
  const long long n = (long long)st.chi * st.chi;
  hipLaunchKernelGGL(k_init_gamma, dim3((unsigned)((n + 255) / 256), st.M), dim3(256), 0, s, st,
                     rho, A, V, K);
  return hipGetLastError();
}

}  // namespace gbs
