// C ABI of libgbsmpo: handle, validation, device memory, layer orchestration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gbs_mpo.h"
#include "internal.h"

using namespace gbs;

static thread_local std::string g_err;

static int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      return fail(MPO_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));       \
  } while (0)

struct gbs_mpo {
  State st{};
  Layer ly{};
  int precision = MPO_FP64;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int max_gates = 0;
  long long capA = 0;
  int capBig = 0;
  int *h_active = nullptr;
  GateParam *h_gates = nullptr;
  GateTot *h_tot = nullptr;
  GateBase *h_base = nullptr;
  int *h_err = nullptr;
  cd *envL = nullptr, *envR = nullptr;
  double *dP = nullptr, *dTrace = nullptr, *dPhase = nullptr;
  long long stats[6] = {0, 0, 0, 0, 0, -1};
  int latched = 0;
  // profiling: HIP events around each phase of a layer, read at the next sync
  static constexpr int NPH = 8;
  bool prof = false;
  bool prof_pending = false;
  hipEvent_t ev[2 * NPH] = {};
  double ph_ms[NPH] = {};
  long long ph_n[NPH] = {};
  double work[4] = {};      // svd flops, sector elements, candidates, layers
  std::vector<void *> allocs;
};

namespace {

template <typename T>
hipError_t dalloc(gbs_mpo *h, T **p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)p, sizeof(T) * count);
  if (e == hipSuccess) h->allocs.push_back((void *)*p);
  return e;
}

void dfree(gbs_mpo *h, void *p) {
  if (!p) return;
  hipFree(p);
  h->allocs.erase(std::remove(h->allocs.begin(), h->allocs.end(), p), h->allocs.end());
}

// Internal Fock dimension of the squeezed vacuum: smallest even size whose
// neglected tail |psi_{2n}|^2 is below 1e-20 and that covers the cutoff d.
int internal_levels(double r, int d) {
  if (r == 0.0) return std::max(d, 2);
  const double lt2 = std::log(std::tanh(r) * std::tanh(r));
  for (int n = 0;; ++n) {
    const double lp = n * lt2 + std::lgamma(2.0 * n + 1.0) - 2.0 * n * std::log(2.0) -
                      2.0 * std::lgamma(n + 1.0) - std::log(std::cosh(r));
    if (2 * n + 1 >= d && lp < std::log(1e-20)) return 2 * n + 2;
  }
}

int check_latched(gbs_mpo *h) {
  if (h->latched) {
    const int e = h->latched;
    std::string msg = "device error latched:";
    if (e & ERR_SVD_NOT_CONVERGED) msg += " Jacobi SVD did not converge;";
    if (e & ERR_NONFINITE) msg += " non-finite value;";
    if (e & ERR_BOX_OVERFLOW) msg += " charge box exceeds workspace;";
    if (e & ERR_TIE_OVERFLOW) msg += " too many tied singular values;";
    if (e & ERR_WORKSPACE) msg += " sector workspace overflow;";
    return fail(MPO_ENUMERIC, msg);
  }
  return MPO_OK;
}

// Read the elapsed times of the previous layer's phase events (its work has
// completed once the stream was synchronised).
void prof_collect(gbs_mpo *h) {
  if (!h->prof || !h->prof_pending) return;
  for (int p = 0; p < gbs_mpo::NPH; ++p) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev[2 * p], h->ev[2 * p + 1]) == hipSuccess) {
      h->ph_ms[p] += ms;
      h->ph_n[p] += 1;
    }
  }
  h->prof_pending = false;
}

void prof_mark(gbs_mpo *h, int phase, int edge) {
  if (h->prof) hipEventRecord(h->ev[2 * phase + edge], h->stream);
}

int sync_and_check(gbs_mpo *h) {
  HIPCHK(hipMemcpyAsync(h->h_err, h->st.err, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->latched |= *h->h_err;
  prof_collect(h);
  return check_latched(h);
}

}  // namespace

extern "C" const char *mpo_last_error(void) { return g_err.c_str(); }

extern "C" void mpo_free(gbs_mpo *h) {
  if (!h) return;
  if (h->stream) hipStreamSynchronize(h->stream);
  for (void *p : h->allocs) hipFree(p);
  if (h->h_gates) hipHostFree(h->h_gates);
  if (h->h_tot) hipHostFree(h->h_tot);
  if (h->h_base) hipHostFree(h->h_base);
  if (h->h_err) hipHostFree(h->h_err);
  if (h->h_active) hipHostFree(h->h_active);
  for (int i = 0; i < 2 * gbs_mpo::NPH; ++i)
    if (h->ev[i]) hipEventDestroy(h->ev[i]);
  if (h->own_stream && h->stream) hipStreamDestroy(h->stream);
  delete h;
}

extern "C" int mpo_init_lossy_squeezed(int M, const double *r, double eta, int d, int chi,
                                       int precision, void *hip_stream, gbs_mpo **out) {
  if (!out) return fail(MPO_EINVAL, "out is NULL");
  *out = nullptr;
  if (M < 2 || M > 4096) return fail(MPO_EINVAL, "M must be in [2, 4096]");
  if (!r) return fail(MPO_EINVAL, "r is NULL");
  for (int j = 0; j < M; ++j)
    if (!(r[j] >= 0.0) || !std::isfinite(r[j]) || r[j] > 20.0)
      return fail(MPO_EINVAL, "r[j] must be finite and in [0, 20]");
  if (!(eta > 0.0 && eta <= 1.0)) return fail(MPO_EINVAL, "eta must be in (0, 1]");
  if (d < 2 || d > 16) return fail(MPO_EINVAL, "d must be in [2, 16]");
  if (chi < 1 || chi > 4096) return fail(MPO_EINVAL, "chi must be in [1, 4096]");
  if (precision != MPO_FP64 && precision != MPO_MIXED)
    return fail(MPO_EINVAL, "precision must be MPO_FP64 or MPO_MIXED");
  if ((long long)M * (d - 1) + 1 > 32767) return fail(MPO_EINVAL, "charges exceed 15 bits");

  // projected footprint: state + per-layer workspace (sector pools start small)
  const long long W0 = (long long)M * (d - 1) + 1;
  const int max_gates = M / 2;
  const long long cap_g = (long long)d * d * chi;
  long long need = (long long)M * chi * chi * 16 + (long long)(M + 1) * chi * 12 +
                   (long long)max_gates * (cap_g * (4 + 4 + 4 + 8 + 4 + 8 + 8 + 4) +
                                           cap_g * (long long)sizeof(BlkDesc));
  long long init_need = (long long)(M + 1) * W0 * W0 * 28;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess)
    return fail(MPO_EDEVICE, "hipMemGetInfo failed");
  if ((double)(need + init_need) > 0.9 * (double)free_b)
    return fail(MPO_ENOMEM, "projected device memory exceeds the free HBM");

  gbs_mpo *h = new gbs_mpo();
  h->precision = precision;
  h->max_gates = max_gates;
  int rc = MPO_OK;
  auto bail = [&](int code) {
    mpo_free(h);
    return code;
  };
#define TRY(x)                                                                        \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      rc = fail(e_ == hipErrorOutOfMemory ? MPO_ENOMEM : MPO_EDEVICE,                 \
                std::string(#x) + ": " + hipGetErrorString(e_));                      \
      return bail(rc);                                                                \
    }                                                                                 \
  } while (0)
  if (hip_stream) {
    h->stream = (hipStream_t)hip_stream;
  } else {
    TRY(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    h->own_stream = true;
  }
  State &st = h->st;
  st.M = M;
  st.d = d;
  st.chi = chi;
  TRY(dalloc(h, &st.gam, (size_t)M * chi * chi));
  TRY(dalloc(h, &st.lam, (size_t)(M + 1) * chi));
  TRY(dalloc(h, &st.chg, (size_t)(M + 1) * chi));
  TRY(dalloc(h, &st.dim, (size_t)(M + 1)));
  TRY(dalloc(h, &st.ee, (size_t)(M + 1)));
  TRY(dalloc(h, &st.ee_max, 1));
  TRY(dalloc(h, &st.err, 1));
  TRY(hipMemsetAsync(st.ee, 0, sizeof(double) * (M + 1), h->stream));
  TRY(hipMemsetAsync(st.ee_max, 0, sizeof(unsigned long long), h->stream));
  TRY(hipMemsetAsync(st.err, 0, sizeof(int), h->stream));

  Layer &ly = h->ly;
  ly.max_blk = (int)cap_g;
  ly.box_cap = (int)std::min<long long>(W0 * W0, 1LL << 30);
  TRY(dalloc(h, &ly.gates, max_gates));
  TRY(dalloc(h, &ly.fock, (size_t)max_gates * (2 * d - 1) * d * d));
  TRY(dalloc(h, &ly.blk, (size_t)max_gates * cap_g));
  TRY(dalloc(h, &ly.tot, max_gates));
  TRY(dalloc(h, &ly.base, max_gates));
  TRY(dalloc(h, &ly.bigl, (size_t)max_gates * cap_g));
  TRY(dalloc(h, &ly.active, 1));
  h->capBig = 4096;
  TRY(dalloc(h, &ly.rotf, (size_t)4 * h->capBig));
  TRY(dalloc(h, &ly.mirL, (size_t)max_gates * chi));
  TRY(dalloc(h, &ly.mirR, (size_t)max_gates * chi));
  TRY(dalloc(h, &ly.rows, (size_t)max_gates * cap_g));
  TRY(dalloc(h, &ly.cols, (size_t)max_gates * cap_g));
  TRY(dalloc(h, &ly.sv, (size_t)max_gates * cap_g));
  TRY(dalloc(h, &ly.perm, (size_t)max_gates * cap_g));
  TRY(dalloc(h, &ly.uval, (size_t)max_gates * cap_g));
  TRY(dalloc(h, &ly.ukey, (size_t)max_gates * cap_g));
  TRY(dalloc(h, &ly.usize, (size_t)max_gates * cap_g));
  h->capA = std::max<long long>(1 << 20, (long long)chi * chi * 4);
  TRY(dalloc(h, &ly.A, (size_t)h->capA));
  TRY(dalloc(h, &ly.A0, (size_t)h->capA));
  TRY(hipHostMalloc((void **)&h->h_gates, sizeof(GateParam) * std::max(max_gates, 1)));
  TRY(hipHostMalloc((void **)&h->h_tot, sizeof(GateTot) * std::max(max_gates, 1)));
  TRY(hipHostMalloc((void **)&h->h_base, sizeof(GateBase) * std::max(max_gates, 1)));
  TRY(hipHostMalloc((void **)&h->h_err, sizeof(int)));
  TRY(hipHostMalloc((void **)&h->h_active, sizeof(int)));
  TRY(dalloc(h, &h->envL, (size_t)(M + 1) * chi));
  TRY(dalloc(h, &h->envR, (size_t)(M + 1) * chi));
  TRY(dalloc(h, &h->dP, (size_t)M * d));
  TRY(dalloc(h, &h->dTrace, 1));
  TRY(dalloc(h, &h->dPhase, (size_t)M));

  // ---- initial state ----
  std::vector<int> nint(M);
  for (int j = 0; j < M; ++j) nint[j] = internal_levels(r[j], d);
  std::vector<long long> woff(M + 2, 0);
  // lay the grids out from bond M upwards
  {
    long long acc = 0;
    for (int b = M; b >= 0; --b) {
      const long long Wb = (long long)(M - b) * (d - 1) + 1;
      woff[b] = acc;
      acc += Wb * Wb;
    }
    woff[M + 1] = acc;
  }
  double *d_r = nullptr, *d_rho = nullptr, *d_A = nullptr, *d_w = nullptr;
  int *d_nint = nullptr;
  long long *d_woff = nullptr;
  unsigned long long *d_uv = nullptr, *d_uk = nullptr;
  int *d_us = nullptr;
  const long long ucap = W0 * W0;
  TRY(dalloc(h, &d_r, M));
  TRY(dalloc(h, &d_nint, M));
  TRY(dalloc(h, &d_rho, (size_t)M * d * d));
  TRY(dalloc(h, &d_A, M + 1));
  TRY(dalloc(h, &d_w, (size_t)woff[M + 1]));
  TRY(dalloc(h, &d_woff, M + 2));
  TRY(dalloc(h, &d_uv, (size_t)ucap * (M + 1)));
  TRY(dalloc(h, &d_uk, (size_t)ucap * (M + 1)));
  TRY(dalloc(h, &d_us, (size_t)ucap * (M + 1)));
  TRY(hipMemcpyAsync(d_r, r, sizeof(double) * M, hipMemcpyHostToDevice, h->stream));
  TRY(hipMemcpyAsync(d_nint, nint.data(), sizeof(int) * M, hipMemcpyHostToDevice, h->stream));
  TRY(hipMemcpyAsync(d_woff, woff.data(), sizeof(long long) * (M + 2), hipMemcpyHostToDevice,
                     h->stream));
  const double one = 1.0;
  TRY(hipMemcpyAsync(d_w + woff[M], &one, sizeof(double), hipMemcpyHostToDevice, h->stream));
  TRY(launch_init_rho(d_r, d_nint, eta, M, d, d_rho, h->stream));
  TRY(launch_init_norms(d_rho, M, d, d_A, h->stream));
  for (int b = M - 1; b >= 0; --b) TRY(launch_init_conv(d_rho, M, d, b, d_woff, d_w, h->stream));
  TRY(launch_init_select(st, d_w, d_woff, d_A, d_uv, d_uk, d_us, ucap, h->stream));
  TRY(launch_init_gamma(st, d_rho, d_A, h->stream));
  TRY(launch_entropy_all(st, h->stream));
  TRY(hipStreamSynchronize(h->stream));
  for (void *p : std::vector<void *>{d_r, d_nint, d_rho, d_A, d_w, d_woff, d_uv, d_uk, d_us})
    dfree(h, p);
  rc = sync_and_check(h);
  if (rc != MPO_OK) return bail(rc);
  *out = h;
  return MPO_OK;
#undef TRY
}

extern "C" int mpo_apply_bs_layer(gbs_mpo *h, int n_gates, const int *left_site,
                                  const double *theta, const double *phi) {
  if (!h) return fail(MPO_EINVAL, "handle is NULL");
  int rc = check_latched(h);
  if (rc != MPO_OK) return rc;
  const int M = h->st.M;
  if (n_gates < 0 || n_gates > h->max_gates) return fail(MPO_EINVAL, "n_gates out of range");
  if (n_gates == 0) return MPO_OK;
  if (!left_site || !theta || !phi) return fail(MPO_EINVAL, "NULL gate array");
  std::vector<char> used(M, 0);
  for (int g = 0; g < n_gates; ++g) {
    const int k = left_site[g];
    if (k < 0 || k > M - 2) return fail(MPO_EINVAL, "left_site out of range");
    if (used[k] || used[k + 1]) return fail(MPO_EINVAL, "gates of a layer must be disjoint");
    if (!std::isfinite(theta[g]) || !std::isfinite(phi[g]))
      return fail(MPO_EINVAL, "non-finite gate angle");
    used[k] = used[k + 1] = 1;
  }
  State &st = h->st;
  Layer &ly = h->ly;
  for (int g = 0; g < n_gates; ++g) h->h_gates[g] = GateParam{left_site[g], 0, theta[g], phi[g]};
  ly.ngates = n_gates;
  HIPCHK(hipMemcpyAsync(ly.gates, h->h_gates, sizeof(GateParam) * n_gates,
                        hipMemcpyHostToDevice, h->stream));
  prof_mark(h, 0, 0);
  HIPCHK(launch_fock(ly, st.d, h->stream));
  prof_mark(h, 0, 1);
  prof_mark(h, 1, 0);
  HIPCHK(launch_plan(st, ly, h->stream));
  prof_mark(h, 1, 1);
  HIPCHK(hipMemcpyAsync(h->h_tot, ly.tot, sizeof(GateTot) * n_gates, hipMemcpyDeviceToHost,
                        h->stream));
  rc = sync_and_check(h);
  if (rc != MPO_OK) return rc;
  // global offsets of the sector pools
  long long e = 0, ch = 0;
  int blkb = 0, bigb = 0, maxpp = 0;
  long long st_blk = 0, st_el = 0, st_sv = 0, st_mr = 0, st_mc = 0;
  double st_fl = 0.0;
  for (int g = 0; g < n_gates; ++g) {
    const GateTot &t = h->h_tot[g];
    h->h_base[g] = GateBase{e, blkb, bigb, ch};
    e += t.elems;
    ch += t.chunks;
    blkb += t.nblk;
    bigb += t.nbig;
    maxpp = std::max(maxpp, t.maxpp);
    st_blk += t.nblk;
    st_el += t.elems;
    st_sv += t.sv;
    st_mr = std::max<long long>(st_mr, t.maxr);
    st_mc = std::max<long long>(st_mc, t.maxc);
    st_fl += t.svd_flops;
  }
  h->stats[0] = st_blk;
  h->stats[1] = st_el;
  h->stats[2] = st_sv;
  h->stats[3] = st_mr;
  h->stats[4] = st_mc;
  h->stats[5] = -1;
  if (h->prof) {
    h->work[0] += st_fl;
    h->work[1] += (double)st_el;
    h->work[2] += (double)st_sv;
    h->work[3] += 1.0;
  }
  if (e > h->capA) {
    const long long cap = std::max(e, h->capA * 2);
    dfree(h, ly.A);
    dfree(h, ly.A0);
    ly.A = ly.A0 = nullptr;
    if (dalloc(h, &ly.A, (size_t)cap) != hipSuccess || dalloc(h, &ly.A0, (size_t)cap) != hipSuccess)
      return fail(MPO_ENOMEM, "sector operand pool allocation failed");
    h->capA = cap;
  }
  if (bigb > h->capBig) {
    const int cap = std::max(bigb, h->capBig * 2);
    dfree(h, ly.rotf);
    ly.rotf = nullptr;
    if (dalloc(h, &ly.rotf, (size_t)4 * cap) != hipSuccess)
      return fail(MPO_ENOMEM, "flag allocation failed");
    h->capBig = cap;
  }
  ly.total_chunks = ch;
  ly.total_blocks = blkb;
  ly.total_big = bigb;
  ly.maxpp = maxpp;
  HIPCHK(hipMemcpyAsync(ly.base, h->h_base, sizeof(GateBase) * n_gates, hipMemcpyHostToDevice,
                        h->stream));
  prof_mark(h, 2, 0);
  HIPCHK(launch_contract(st, ly, h->stream));
  prof_mark(h, 2, 1);
  prof_mark(h, 3, 0);
  HIPCHK(launch_svd_small(st, ly, h->stream));
  int sweeps_run = 0;
  if (bigb > 0) {
    // panel rounds of the big blocks; convergence is read back every 3 sweeps
    HIPCHK(launch_svd_big_prep(st, ly, h->stream));
    const int kMaxSweeps = 60;
    for (int s = 0; s < kMaxSweeps; ++s) {
      for (int r = 0; r < maxpp - 1; ++r) HIPCHK(launch_svd_panel_round(st, ly, r, s, h->stream));
      sweeps_run = s + 1;
      if (s % 3 == 2 || s == kMaxSweeps - 1) {
        HIPCHK(launch_svd_count(st, ly, s, h->stream));
        HIPCHK(hipMemcpyAsync(h->h_active, ly.active, sizeof(int), hipMemcpyDeviceToHost,
                              h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (*h->h_active == 0) break;
      }
    }
    HIPCHK(launch_svd_big_finish(st, ly, sweeps_run, h->stream));
  }
  h->stats[5] = sweeps_run;
  prof_mark(h, 3, 1);
  prof_mark(h, 4, 0);
  HIPCHK(launch_select(st, ly, h->stream));
  prof_mark(h, 4, 1);
  prof_mark(h, 5, 0);
  HIPCHK(launch_scatter(st, ly, h->stream));
  prof_mark(h, 5, 1);
  prof_mark(h, 6, 0);
  HIPCHK(launch_entropy_layer(st, ly, h->stream));
  prof_mark(h, 6, 1);
  prof_mark(h, 7, 0);
  prof_mark(h, 7, 1);
  if (h->prof) h->prof_pending = true;
  return MPO_OK;
}

extern "C" int mpo_apply_phases(gbs_mpo *h, const double *phase) {
  if (!h || !phase) return fail(MPO_EINVAL, "NULL argument");
  int rc = check_latched(h);
  if (rc != MPO_OK) return rc;
  for (int j = 0; j < h->st.M; ++j)
    if (!std::isfinite(phase[j])) return fail(MPO_EINVAL, "non-finite phase");
  HIPCHK(hipMemcpyAsync(h->dPhase, phase, sizeof(double) * h->st.M, hipMemcpyHostToDevice,
                        h->stream));
  HIPCHK(launch_phases(h->st, h->dPhase, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return MPO_OK;
}

extern "C" int mpo_sync(gbs_mpo *h) {
  if (!h) return fail(MPO_EINVAL, "handle is NULL");
  return sync_and_check(h);
}

extern "C" int mpo_entropy(gbs_mpo *h, double *S, double *S_max_so_far) {
  if (!h || !S) return fail(MPO_EINVAL, "NULL argument");
  const int M = h->st.M;
  std::vector<double> ee(M + 1);
  unsigned long long mx = 0;
  HIPCHK(hipMemcpyAsync(ee.data(), h->st.ee, sizeof(double) * (M + 1), hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipMemcpyAsync(&mx, h->st.ee_max, sizeof(mx), hipMemcpyDeviceToHost, h->stream));
  int rc = sync_and_check(h);
  if (rc != MPO_OK) return rc;
  for (int b = 1; b < M; ++b) S[b - 1] = ee[b];
  if (S_max_so_far) {
    double m;
    std::memcpy(&m, &mx, sizeof(m));
    for (int b = 1; b < M; ++b) m = std::max(m, ee[b]);
    *S_max_so_far = m;
  }
  return MPO_OK;
}

extern "C" int mpo_photon_marginals(gbs_mpo *h, double *P, double *trace) {
  if (!h || !P) return fail(MPO_EINVAL, "NULL argument");
  int rc = check_latched(h);
  if (rc != MPO_OK) return rc;
  const int M = h->st.M, d = h->st.d;
  HIPCHK(launch_marginals(h->st, h->envL, h->envR, h->dP, h->dTrace, h->stream));
  std::vector<double> raw((size_t)M * d);
  double tr = 0.0;
  HIPCHK(hipMemcpyAsync(raw.data(), h->dP, sizeof(double) * M * d, hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipMemcpyAsync(&tr, h->dTrace, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  rc = sync_and_check(h);
  if (rc != MPO_OK) return rc;
  if (!(tr > 0.0) || !std::isfinite(tr)) return fail(MPO_ENUMERIC, "non-positive trace");
  for (size_t i = 0; i < raw.size(); ++i) P[i] = raw[i] / tr;
  if (trace) *trace = tr;
  return MPO_OK;
}

extern "C" int mpo_get_bond(gbs_mpo *h, int b, int *dim, double *lam, int *charges) {
  if (!h || !dim) return fail(MPO_EINVAL, "NULL argument");
  const int M = h->st.M, chi = h->st.chi;
  if (b < 0 || b > M) return fail(MPO_EINVAL, "bond out of range");
  int D = 0;
  HIPCHK(hipMemcpyAsync(&D, h->st.dim + b, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  *dim = D;
  if (D > 0 && lam)
    HIPCHK(hipMemcpy(lam, h->st.lam + (size_t)b * chi, sizeof(double) * D,
                     hipMemcpyDeviceToHost));
  if (D > 0 && charges) {
    std::vector<int> c(D);
    HIPCHK(hipMemcpy(c.data(), h->st.chg + (size_t)b * chi, sizeof(int) * D,
                     hipMemcpyDeviceToHost));
    for (int i = 0; i < D; ++i) {
      charges[2 * i] = charge_n(c[i]);
      charges[2 * i + 1] = charge_np(c[i]);
    }
  }
  return sync_and_check(h);
}

extern "C" int mpo_get_site(gbs_mpo *h, int j, double *G) {
  if (!h || !G) return fail(MPO_EINVAL, "NULL argument");
  const int M = h->st.M, chi = h->st.chi;
  if (j < 0 || j >= M) return fail(MPO_EINVAL, "site out of range");
  int D[2];
  HIPCHK(hipMemcpyAsync(D, h->st.dim + j, sizeof(int) * 2, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  std::vector<cd> tmp((size_t)chi * chi);
  HIPCHK(hipMemcpy(tmp.data(), h->st.gam + (size_t)j * chi * chi, sizeof(cd) * chi * chi,
                   hipMemcpyDeviceToHost));
  for (int a = 0; a < D[0]; ++a)
    for (int b = 0; b < D[1]; ++b) {
      G[2 * ((size_t)a * D[1] + b)] = tmp[(size_t)a * chi + b].re;
      G[2 * ((size_t)a * D[1] + b) + 1] = tmp[(size_t)a * chi + b].im;
    }
  return sync_and_check(h);
}

extern "C" int mpo_layer_stats(gbs_mpo *h, long long *stats) {
  if (!h || !stats) return fail(MPO_EINVAL, "NULL argument");
  int rc = sync_and_check(h);
  if (rc != MPO_OK) return rc;
  for (int i = 0; i < 6; ++i) stats[i] = h->stats[i];
  return MPO_OK;
}

extern "C" int mpo_set_profiling(gbs_mpo *h, int enable) {
  if (!h) return fail(MPO_EINVAL, "handle is NULL");
  int rc = sync_and_check(h);
  if (rc != MPO_OK) return rc;
  if (enable) {
    for (int i = 0; i < 2 * gbs_mpo::NPH; ++i)
      if (!h->ev[i]) HIPCHK(hipEventCreate(&h->ev[i]));
  }
  h->prof = enable != 0;
  h->prof_pending = false;
  for (int p = 0; p < gbs_mpo::NPH; ++p) {
    h->ph_ms[p] = 0.0;
    h->ph_n[p] = 0;
  }
  for (double &x : h->work) x = 0.0;
  return MPO_OK;
}

extern "C" int mpo_get_profile(gbs_mpo *h, double *phase_ms, long long *phase_launches,
                               double *work) {
  if (!h) return fail(MPO_EINVAL, "handle is NULL");
  int rc = sync_and_check(h);
  if (rc != MPO_OK) return rc;
  for (int p = 0; p < gbs_mpo::NPH; ++p) {
    if (phase_ms) phase_ms[p] = h->ph_ms[p];
    if (phase_launches) phase_launches[p] = h->ph_n[p];
  }
  if (work)
    for (int i = 0; i < 4; ++i) work[i] = h->work[i];
  return MPO_OK;
}

extern "C" int mpo_layer_blocks(gbs_mpo *h, int max_blocks, int *out) {
  if (!h || max_blocks < 0 || (max_blocks > 0 && !out)) return fail(MPO_EINVAL, "bad argument");
  int rc = sync_and_check(h);
  if (rc != MPO_OK) return rc;
  const Layer &ly = h->ly;
  int total = 0;
  std::vector<BlkDesc> tmp;
  for (int g = 0; g < ly.ngates; ++g) {
    const int nb = h->h_tot[g].nblk;
    tmp.resize(nb);
    if (nb > 0)
      HIPCHK(hipMemcpy(tmp.data(), ly.blk + (size_t)g * ly.max_blk, sizeof(BlkDesc) * nb,
                       hipMemcpyDeviceToHost));
    for (int i = 0; i < nb; ++i, ++total) {
      if (total >= max_blocks) continue;
      int *o = out + (size_t)8 * total;
      o[0] = g;
      o[1] = charge_n(tmp[i].q);
      o[2] = charge_np(tmp[i].q);
      o[3] = tmp[i].r;
      o[4] = tmp[i].s;
      o[5] = tmp[i].comp;
      o[6] = tmp[i].sweeps;
      o[7] = tmp[i].kq;
    }
  }
  return total;
}
