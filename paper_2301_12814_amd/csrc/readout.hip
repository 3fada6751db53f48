// Readouts of the U(1) Vidal MPO: output phase screen, trace and photon
// marginals (the trace deficit 1 - Tr rho is the paper's error proxy,
// Sec. III and App. A).
//
// With the auxiliary total-charge leg contracted with the all-ones vector and
// every site with the identity (local ket = bra), the trace is a chain of
// matrix-vector products over the diagonal-compatible entries of each site
// matrix (c_a - c_b = (n, n), 0 <= n < d):
//   E_M = 1,  E_j[a] = sum_b Gamma_j[a, b] lam_{j+1}[b] E_{j+1}[b],
//   L_0 = 1,  L_{j+1}[b] = sum_a L_j[a] lam_j[a] Gamma_j[a, b],
//   Tr rho = sum_a lam_0[a] E_0[a],
//   Tr(rho Pi_{j,n}) = sum_{c_a - c_b = (n,n)} L_j[a] lam_j[a] Gamma_j[a,b] lam_{j+1}[b] E_{j+1}[b].
#include <mutex>

#include "internal.h"

namespace gbs {

__device__ inline int diag_photons(int ca, int cb, int d) {
  const int m = charge_n(ca) - charge_n(cb), mp = charge_np(ca) - charge_np(cb);
  return (m == mp && m >= 0 && m < d) ? m : -1;
}

// one wavefront per row a of site j
__global__ __launch_bounds__(256) void k_env_right(State st, int j, cd *E) {
  const int chi = st.chi, d = st.d;
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int Dl = st.dim[j], Dr = st.dim[j + 1];
  if (a >= Dl) return;
  const int ca = st.chg[(size_t)j * chi + a];
  const cd *G = st.gam + (size_t)j * chi * chi + (size_t)a * chi;
  const cd *En = E + (size_t)(j + 1) * chi;
  const double *lr = st.lam + (size_t)(j + 1) * chi;
  const int *cr = st.chg + (size_t)(j + 1) * chi;
  double re = 0.0, im = 0.0;
  for (int b = lane; b < Dr; b += 64) {
    if (diag_photons(ca, cr[b], d) < 0) continue;
    const cd x = cscale(cmul(G[b], En[b]), lr[b]);
    re += x.re;
    im += x.im;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) E[(size_t)j * chi + a] = cmk(re, im);
}

// one thread per column b of site j
__global__ __launch_bounds__(256) void k_env_left(State st, int j, cd *L) {
  const int chi = st.chi, d = st.d;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int Dl = st.dim[j], Dr = st.dim[j + 1];
  if (b >= Dr) return;
  const int cb = st.chg[(size_t)(j + 1) * chi + b];
  const cd *G = st.gam + (size_t)j * chi * chi + b;
  const cd *Lp = L + (size_t)j * chi;
  const double *ll = st.lam + (size_t)j * chi;
  const int *cl = st.chg + (size_t)j * chi;
  cd acc = cmk(0.0, 0.0);
  for (int a = 0; a < Dl; ++a) {
    if (diag_photons(cl[a], cb, d) < 0) continue;
    cfma(acc, cscale(Lp[a], ll[a]), G[(size_t)a * chi]);
  }
  L[(size_t)(j + 1) * chi + b] = acc;
}

__global__ void k_env_init(State st, cd *L, cd *E) {
  const int chi = st.chi;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < chi; i += gridDim.x * blockDim.x) {
    L[i] = cmk(1.0, 0.0);
    E[(size_t)st.M * chi + i] = cmk(i == 0 ? 1.0 : 0.0, 0.0);
  }
}

// one wavefront per row a of site j = blockIdx.y; each workgroup writes its
// per-n partial sums to part[(j * gridDim.x + blockIdx.x) * d + n] (summed in a
// fixed order by k_marg_reduce, so the result does not depend on scheduling)
__global__ __launch_bounds__(256) void k_marg(State st, const cd *L, const cd *E, double *part) {
  const int chi = st.chi, d = st.d;
  const int j = blockIdx.y;
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  __shared__ double s_bin[4][16];
  for (int i = threadIdx.x; i < 64; i += blockDim.x) (&s_bin[0][0])[i] = 0.0;
  __syncthreads();
  const int Dl = st.dim[j], Dr = st.dim[j + 1];
  if (a < Dl) {
    const int ca = st.chg[(size_t)j * chi + a];
    const cd la = cscale(L[(size_t)j * chi + a], st.lam[(size_t)j * chi + a]);
    const cd *G = st.gam + (size_t)j * chi * chi + (size_t)a * chi;
    const cd *En = E + (size_t)(j + 1) * chi;
    const double *lr = st.lam + (size_t)(j + 1) * chi;
    const int *cr = st.chg + (size_t)(j + 1) * chi;
    for (int n = 0; n < d; ++n) {
      double re = 0.0;
      for (int b = lane; b < Dr; b += 64) {
        if (diag_photons(ca, cr[b], d) != n) continue;
        const cd x = cmul(cmul(la, G[b]), cscale(En[b], lr[b]));
        re += x.re;
      }
      re = wave_sum(re);
      if (lane == 0) s_bin[threadIdx.x >> 6][n] = re;
    }
  }
  __syncthreads();
  if (threadIdx.x < d) {
    const double v = s_bin[0][threadIdx.x] + s_bin[1][threadIdx.x] + s_bin[2][threadIdx.x] +
                     s_bin[3][threadIdx.x];
    part[((size_t)j * gridDim.x + blockIdx.x) * d + threadIdx.x] = v;
  }
}

// P[j][n] = sum over the row groups of site j, in order.
__global__ void k_marg_reduce(State st, const double *part, int nx, double *P) {
  const int j = blockIdx.x, d = st.d;
  for (int n = threadIdx.x; n < d; n += blockDim.x) {
    double acc = 0.0;
    for (int x = 0; x < nx; ++x) acc += part[((size_t)j * nx + x) * d + n];
    P[j * d + n] = acc;
  }
}

__global__ void k_trace(State st, const cd *E, double *trace) {
  __shared__ double s[4];
  double acc = 0.0;
  for (int a = threadIdx.x; a < st.dim[0]; a += blockDim.x) acc += st.lam[a] * E[a].re;
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *trace = s[0] + s[1] + s[2] + s[3];
}

size_t marginals_scratch(int M, int d, int chi) { return (size_t)M * d * ((chi + 3) / 4); }

hipError_t launch_marginals(State st, cd *envL, cd *envR, double *part, double *P,
                            double *trace, hipStream_t s) {
  const int chi = st.chi;
  const int nx = (chi + 3) / 4;
  hipLaunchKernelGGL(k_env_init, dim3((chi + 255) / 256), dim3(256), 0, s, st, envL, envR);
  for (int j = st.M - 1; j >= 0; --j)
    hipLaunchKernelGGL(k_env_right, dim3((chi + 3) / 4), dim3(256), 0, s, st, j, envR);
  for (int j = 0; j < st.M; ++j)
    hipLaunchKernelGGL(k_env_left, dim3((chi + 255) / 256), dim3(256), 0, s, st, j, envL);
  hipLaunchKernelGGL(k_marg, dim3(nx, st.M), dim3(256), 0, s, st, envL, envR, part);
  hipLaunchKernelGGL(k_marg_reduce, dim3(st.M), dim3(64), 0, s, st, part, nx, P);
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(256), 0, s, st, envR, trace);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Marginals without allocation.  The trace environments, the per-workgroup
// partial sums, the raw marginals and the trace live in one file-scope device
// array of NOALLOC_SCRATCH_BYTES (each GPU holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel: its
// device address is looked up once per device with hipGetSymbolAddress and
// kept in g_scratch_ptr.  Every call on a device shares that device's array,
// so calls that overlap on one GPU race.
// ----------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

size_t marginals_noalloc_bytes(int M, int d, int chi) {
  const size_t env = align256(sizeof(cd) * (size_t)(M + 1) * chi);
  const size_t part = align256(sizeof(double) * marginals_scratch(M, d, chi));
  const size_t P = align256(sizeof(double) * (size_t)M * d);
  return 2 * env + part + P + align256(sizeof(double));
}

hipError_t noalloc_scratch_init() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void *ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = ptr;
  return hipSuccess;
}

hipError_t launch_marginals_noalloc(State st, double **P, double **trace, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = g_scratch_ptr[dev];
  }
  if (!base) {
    e = noalloc_scratch_init();
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = g_scratch_ptr[dev];
  }
  if (marginals_noalloc_bytes(st.M, st.d, st.chi) > (size_t)NOALLOC_SCRATCH_BYTES)
    return hipErrorInvalidValue;
  unsigned char *p = static_cast<unsigned char *>(base);
  const size_t env = align256(sizeof(cd) * (size_t)(st.M + 1) * st.chi);
  cd *envL = reinterpret_cast<cd *>(p);
  cd *envR = reinterpret_cast<cd *>(p + env);
  double *part = reinterpret_cast<double *>(p + 2 * env);
  double *dP = reinterpret_cast<double *>(
      p + 2 * env + align256(sizeof(double) * marginals_scratch(st.M, st.d, st.chi)));
  double *dT = reinterpret_cast<double *>(reinterpret_cast<unsigned char *>(dP) +
                                          align256(sizeof(double) * (size_t)st.M * st.d));
  *P = dP;
  *trace = dT;
  return launch_marginals(st, envL, envR, part, dP, dT, s);
}

// Output phase screen: Gamma_j[a, b] *= e^{i phase_j (m - m')}, (m, m') = c_a - c_b.
__global__ void k_phases(State st, const double *phase) {
  const int j = blockIdx.y;
  const int chi = st.chi;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)chi * chi) return;
  const int a = (int)(idx / chi), b = (int)(idx % chi);
  if (a >= st.dim[j] || b >= st.dim[j + 1]) return;
  const int ca = st.chg[(size_t)j * chi + a], cb = st.chg[(size_t)(j + 1) * chi + b];
  const int dm = (charge_n(ca) - charge_n(cb)) - (charge_np(ca) - charge_np(cb));
  const double ang = phase[j] * dm;
  cd *G = st.gam + (size_t)j * chi * chi + idx;
  *G = cmul(*G, cmk(cos(ang), sin(ang)));
}

hipError_t launch_phases(State st, const double *phase, hipStream_t s) {
  const long long n = (long long)st.chi * st.chi;
  hipLaunchKernelGGL(k_phases, dim3((unsigned)((n + 255) / 256), st.M), dim3(256), 0, s, st,
                     phase);
  return hipGetLastError();
}

}  // namespace gbs
