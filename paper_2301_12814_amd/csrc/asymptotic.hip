// Renyi entropies of the bonds (Sec. III.B) and the single-mode asymptotic
// estimate of the operator entanglement entropy (App. C).
//
// Renyi-alpha of a bond: S_alpha = log2(sum p^alpha) / (1 - alpha) with
// p = lam^2 / sum lam^2 (the EE's normalised spectrum); alpha = 1 is the EE.
//
// Asymptotic estimate (App. C).  One squeezed input mode, truncated to photon
// numbers 0..n_max together with the pure-loss Kraus operators (App. C input
// wavefunction, App. B Kraus operators), is split by the basis transform of
// App. B (Eq. transform): |n> -> sum_k sqrt(binom(n, k)) c^k s^(n-k)
// |k>_u |n-k>_d, c = cos theta, s = sin theta.  The vectorised output operator
// grouped as X[(k_u, k'_u), (k_d, k'_d)] = rho_out[k_u, k_d; k'_u, k'_d] is a
// real (n_max+1)^2 square matrix; the eigenvalues of the reduced operator
// tr_u |rho>><<rho| are its squared singular values, found here by a one-sided
// (Hestenes) Jacobi in one workgroup.  The estimate is the entropy of the
// normalised spectrum times the number of squeezed inputs (App. B: the output
// is a product over inputs, so the entropy is additive).
#include <math.h>

#include "internal.h"

namespace gbs {

// ---------------------------------------------------------------- Renyi
__global__ __launch_bounds__(256) void k_renyi(State st, double alpha, double *out) {
  const int b = blockIdx.x + 1;
  const int D = st.dim[b];
  const double *lam = st.lam + (size_t)b * st.chi;
  __shared__ double s_a[4], s_b[4];
  double n2 = 0.0;
  for (int i = threadIdx.x; i < D; i += blockDim.x) n2 += lam[i] * lam[i];
  n2 = wave_sum(n2);
  if ((threadIdx.x & 63) == 0) s_a[threadIdx.x >> 6] = n2;
  __syncthreads();
  const double tot = s_a[0] + s_a[1] + s_a[2] + s_a[3];
  double acc = 0.0;
  for (int i = threadIdx.x; i < D; i += blockDim.x) {
    const double p = lam[i] * lam[i] / tot;
    if (p > 0.0) acc += alpha == 1.0 ? -p * log2(p) : (alpha == 0.0 ? 1.0 : pow(p, alpha));
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_b[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double S = s_b[0] + s_b[1] + s_b[2] + s_b[3];
    out[b - 1] = alpha == 1.0 ? S : log2(S) / (1.0 - alpha);
  }
}

hipError_t launch_renyi(State st, double alpha, double *out, hipStream_t s) {
  if (st.M < 2) return hipSuccess;
  hipLaunchKernelGGL(k_renyi, dim3(st.M - 1), dim3(256), 0, s, st, alpha, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- App. C estimate
constexpr int ASYM_THREADS = 1024;
constexpr int ASYM_WAVES = ASYM_THREADS / 64;

// log of binom(n, k)
__device__ inline double log_binom(int n, int k) {
  return lgamma(n + 1.0) - lgamma(k + 1.0) - lgamma((double)(n - k) + 1.0);
}

// Block-wide sum (1024 threads), the same value in every thread.
__device__ inline double asym_block_sum(double v, double *s_red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < ASYM_WAVES; ++w) t += s_red[w];
  return t;
}

// out[0] = n_inputs * S_alpha of the normalised spectrum, spec[D] = the
// normalised spectrum (column order), X: D x D column-major workspace.
__global__ __launch_bounds__(ASYM_THREADS) void k_asym(double r, double mu, int nmax,
                                                       double theta, int n_inputs,
                                                       double alpha, double *X, double *spec,
                                                       double *out, int *err) {
  const int L = nmax + 1, D = L * L;
  __shared__ double s_psi[32], s_rho[32 * 32], s_T[32 * 32], s_red[ASYM_WAVES];
  __shared__ int s_rot;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // squeezed vacuum amplitudes on 0..nmax (App. C)
  if (tid < L) {
    double v = 0.0;
    if ((tid & 1) == 0) {
      const int k = tid >> 1;
      if (r == 0.0) {
        v = k == 0 ? 1.0 : 0.0;
      } else {
        v = exp(k * log(tanh(r)) + 0.5 * lgamma(2.0 * k + 1.0) - k * log(2.0) - lgamma(k + 1.0)) /
            sqrt(cosh(r));
      }
    }
    s_psi[tid] = v;
  }
  __syncthreads();
  // pure loss with both the state and the Kraus operators on 0..nmax (App. B):
  // rho[a][b] = sum_l k_l(a) psi[a+l] psi[b+l] k_l(b),
  // k_l(a) = sqrt(binom(a+l, a) mu^a (1-mu)^l)
  for (int idx = tid; idx < L * L; idx += blockDim.x) {
    const int a = idx / L, b = idx % L;
    double acc = 0.0;
    for (int l = 0; a + l <= nmax && b + l <= nmax; ++l) {
      const double ll = l > 0 ? l * log1p(-mu) : 0.0;
      const double ka = exp(0.5 * (log_binom(a + l, a) + (a > 0 ? a * log(mu) : 0.0) + ll));
      const double kb = exp(0.5 * (log_binom(b + l, b) + (b > 0 ? b * log(mu) : 0.0) + ll));
      acc += ka * s_psi[a + l] * s_psi[b + l] * kb;
    }
    s_rho[a * 32 + b] = acc;
  }
  // split amplitudes <k_u, k_d | U | k_u + k_d> (App. B, Eq. kun)
  const double c = cos(theta), s = sin(theta);
  for (int idx = tid; idx < L * L; idx += blockDim.x) {
    const int ku = idx / L, kd = idx % L;
    s_T[ku * 32 + kd] =
        ku + kd <= nmax ? sqrt(exp(log_binom(ku + kd, ku))) * pow(c, (double)ku) * pow(s, (double)kd)
                        : 0.0;
  }
  __syncthreads();
  // X[(ku, ku'), (kd, kd')], column-major
  double f2 = 0.0;
  for (long long idx = tid; idx < (long long)D * D; idx += blockDim.x) {
    const int col = (int)(idx / D), row = (int)(idx % D);
    const int ku = row / L, kup = row % L, kd = col / L, kdp = col % L;
    double v = 0.0;
    if (ku + kd <= nmax && kup + kdp <= nmax)
      v = s_T[ku * 32 + kd] * s_T[kup * 32 + kdp] * s_rho[(ku + kd) * 32 + (kup + kdp)];
    X[idx] = v;
    f2 += v * v;
  }
  f2 = asym_block_sum(f2, s_red);
  // one-sided Jacobi on the columns: round-robin tournament of column pairs,
  // one wavefront per pair; pairs with a column at the rounding floor are
  // left alone (their values lie far below every value that matters)
  const double tol = 1e-14;
  const double floor2 = 16.0 * D * 1.2e-32 * f2;
  const int Dp = D + (D & 1);
  int sweep = 0;
  for (; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int round = 0; round < Dp - 1; ++round) {
      for (int k = wave; k < Dp / 2; k += ASYM_WAVES) {
        int I, J;
        if (k == 0) {
          I = round;
          J = Dp - 1;
        } else {
          I = (round + k) % (Dp - 1);
          J = (round - k + Dp - 1) % (Dp - 1);
        }
        if (I >= D || J >= D) continue;
        double *x = X + (size_t)I * D, *y = X + (size_t)J * D;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < D; i += 64) {
          const double xi = x[i], yi = y[i];
          al += xi * xi;
          be += yi * yi;
          ga += xi * yi;
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (al <= floor2 || be <= floor2 || !(fabs(ga) > tol * sqrt(al * be))) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cr = 1.0 / sqrt(1.0 + t * t), sr = cr * t;
        for (int i = lane; i < D; i += 64) {
          const double xi = x[i], yi = y[i];
          x[i] = cr * xi - sr * yi;
          y[i] = sr * xi + cr * yi;
        }
        if (lane == 0) s_rot = 1;
      }
      __syncthreads();
    }
    const int any = s_rot;
    __syncthreads();
    if (!any) break;
  }
  if (sweep == JACOBI_MAX_SWEEPS && tid == 0) atomicOr(err, ERR_SVD_NOT_CONVERGED);
  // squared column norms = eigenvalues of the reduced operator
  for (int col = wave; col < D; col += ASYM_WAVES) {
    double a = 0.0;
    for (int i = lane; i < D; i += 64) a += X[(size_t)col * D + i] * X[(size_t)col * D + i];
    a = wave_sum(a);
    if (lane == 0) spec[col] = a;
  }
  __syncthreads();
  double tot = 0.0;
  for (int i = tid; i < D; i += blockDim.x) tot += spec[i];
  tot = asym_block_sum(tot, s_red);
  double acc = 0.0;
  for (int i = tid; i < D; i += blockDim.x) {
    const double p = spec[i] / tot;
    if (p > 0.0) acc += alpha == 1.0 ? -p * log2(p) : (alpha == 0.0 ? 1.0 : pow(p, alpha));
  }
  acc = asym_block_sum(acc, s_red);
  for (int i = tid; i < D; i += blockDim.x) spec[i] /= tot;
  if (tid == 0) {
    const double S1 = alpha == 1.0 ? acc : log2(acc) / (1.0 - alpha);
    out[0] = n_inputs * S1;
    if (!isfinite(S1)) atomicOr(err, ERR_NONFINITE);
  }
}

hipError_t launch_asym(double r, double mu, int nmax, double theta, int n_inputs, double alpha,
                       double *X, double *spec, double *out, int *err, hipStream_t s) {
  hipLaunchKernelGGL(k_asym, dim3(1), dim3(ASYM_THREADS), 0, s, r, mu, nmax, theta, n_inputs,
                     alpha, X, spec, out, err);
  return hipGetLastError();
}

}  // namespace gbs
