// C ABI of libgbsmpo: validation, device memory, and the engine that applies
// one layer of beam splitters to one or many simulations in one batched
// launch sequence.
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

int gbs::set_error(int code, const char *msg) { return fail(code, msg); }

#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      return fail(e_ == hipErrorOutOfMemory ? MPO_ENOMEM : MPO_EDEVICE,               \
                  std::string(#x) + ": " + hipGetErrorString(e_));                    \
  } while (0)

namespace {

// Growable device buffer.
template <typename T>
struct DBuf {
  T *p = nullptr;
  size_t cap = 0;
  // Grows to at least n (by half again, capped at `limit` when that is >= n).
  hipError_t ensure(size_t n, size_t limit = ~(size_t)0) {
    if (n <= cap && p) return hipSuccess;
    size_t nc = std::max<size_t>(n, cap * 3 / 2 + 1);
    if (limit >= n) nc = std::min(nc, limit);
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc((void **)&p, sizeof(T) * std::max<size_t>(nc, 1));
    if (e == hipSuccess) cap = nc;
    return e;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

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

std::string err_text(int e) {
  std::string msg = "device error latched:";
  if (e & ERR_SVD_NOT_CONVERGED) msg += " Jacobi SVD did not converge;";
  if (e & ERR_NONFINITE) msg += " non-finite value;";
  if (e & ERR_BOX_OVERFLOW) msg += " charge box too large;";
  if (e & ERR_TIE_OVERFLOW) msg += " too many tied singular values;";
  if (e & ERR_WORKSPACE) msg += " sector workspace overflow;";
  return msg;
}

}  // namespace

// One simulation resident on the device.
struct Instance {
  int id = -1;
  bool live = false;
  State st{};                      // device pointers; st.err points into the engine's table
  std::vector<void *> allocs;
  cd *envL = nullptr, *envR = nullptr;
  double *dP = nullptr, *dTrace = nullptr, *dPhase = nullptr, *dPart = nullptr;
  // schedule of beam-splitter layers (engine mode)
  std::vector<int> lptr, site;
  std::vector<double> theta, phi;
  int next_layer = 0;
  bool done = false;
  long long bytes = 0;
  // results of a retired simulation
  double smax = 0.0, trace = 0.0;
  std::vector<double> P;
  int status = MPO_OK;
  std::string msg;                 // error text of a failed simulation
};

struct Engine {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int precision = MPO_FP64;
  long long budget = 0;            // admission budget (bytes)
  long long committed = 0;         // projected bytes of live simulations
  std::vector<Instance> inst;      // slots
  int next_id = 0;
  // state table
  DBuf<State> d_states;
  int *d_errs = nullptr;           // one error word per slot
  size_t errs_cap = 0;
  int *h_errs = nullptr;
  bool states_dirty = true;
  // gate-level workspace
  DBuf<GateParam> d_gates;
  DBuf<GateTot> d_tot;
  DBuf<GateBase> d_base;
  DBuf<cd> d_fock;
  DBuf<int> d_mirL, d_mirR, d_ctab, d_runs;
  GateParam *h_gates = nullptr;
  GateTot *h_tot = nullptr;
  GateBase *h_base = nullptr;
  size_t h_cap = 0;
  // chunk-level workspace
  DBuf<BlkDesc> d_blk;
  DBuf<int> d_rows, d_cols, d_bigl, d_perm, d_usize, d_piv;
  DBuf<double> d_sv;
  DBuf<unsigned long long> d_uval, d_ukey;
  DBuf<cd> d_A, d_A0, d_R, d_U, d_V, d_tau;
  DBuf<int> d_rotf, d_tasks, d_qord, d_bord, d_pver;
  DBuf<int> d_active;
  DBuf<int> d_eng_err;
  int *h_small = nullptr;          // pinned: [1] engine error word, [2..3] rotating blocks / tasks
  long long pool_budget = 0;       // sector operand elements per chunk
  // profiling
  static constexpr int NPH = 8;
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  size_t ev_next = 0;
  double ph_ms[NPH] = {};
  long long ph_n[NPH] = {};
  double work[4] = {};
  double contr_flops = 0.0;        // algorithmic contraction flops while profiling
  long long stats[6] = {0, 0, 0, 0, 0, -1};
  // sector histogram of the last layer, read from d_blk only when asked for
  // (valid while the layer ran as one chunk and no later layer overwrote it)
  bool last_blk_valid = false;
  std::vector<long long> last_blk0;   // per gate: first descriptor in d_blk
  std::vector<int> last_nblk;         // per gate: descriptors
};

struct gbs_mpo {
  Engine eng;
  int slot = 0;
};

struct gbs_engine {
  Engine eng;
};

namespace {

// ------------------------------------------------------------------ profiling
hipEvent_t next_event(Engine &E) {
  if (E.ev_next == E.ev_pool.size()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    E.ev_pool.push_back(ev);
  }
  return E.ev_pool[E.ev_next++];
}

// HIP events around one phase on the engine's stream; read at the next sync.
struct PhaseMark {
  Engine &E;
  int ph;
  hipEvent_t a = nullptr;
  PhaseMark(Engine &e, int p) : E(e), ph(p) {
    if (E.prof) {
      a = next_event(E);
      if (a) hipEventRecord(a, E.stream);
    }
  }
  ~PhaseMark() {
    if (E.prof && a) {
      hipEvent_t b = next_event(E);
      if (b) {
        hipEventRecord(b, E.stream);
        E.pending.push_back({ph, {a, b}});
      }
    }
  }
};

void prof_collect(Engine &E) {
  for (auto &pe : E.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
      E.ph_ms[pe.first] += ms;
      E.ph_n[pe.first] += 1;
    }
  }
  E.pending.clear();
  E.ev_next = 0;
}

// ------------------------------------------------------------------ errors
// Synchronises the stream and reads every slot's error word into h_errs.  With
// check_instances, a latched error of any live simulation is returned.
int sync_and_check(Engine &E, bool check_instances = true) {
  const int n = (int)E.inst.size();
  HIPCHK(hipStreamSynchronize(E.stream));
  if (n > 0) HIPCHK(hipMemcpy(E.h_errs, E.d_errs, sizeof(int) * n, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(E.h_small + 1, E.d_eng_err.p, sizeof(int), hipMemcpyDeviceToHost));
  prof_collect(E);
  int any = E.h_small[1];
  if (check_instances)
    for (int i = 0; i < n; ++i)
      if (E.inst[i].live) any |= E.h_errs[i];
  if (any) return fail(MPO_ENUMERIC, err_text(any));
  return MPO_OK;
}

// ------------------------------------------------------------------ engine setup
int engine_init(Engine &E, void *hip_stream, int precision, long long budget) {
  E.precision = precision;
  if (hip_stream) {
    E.stream = (hipStream_t)hip_stream;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&E.stream, hipStreamNonBlocking));
    E.own_stream = true;
  }
  size_t fb = 0, tb = 0;
  HIPCHK(hipMemGetInfo(&fb, &tb));
  E.budget = budget > 0 ? budget : (long long)(0.85 * (double)fb);
  // sector operand pools per chunk (A and A0): at most a quarter of the budget each
  E.pool_budget = std::max<long long>(1LL << 22, E.budget / 4 / (long long)sizeof(cd));
  HIPCHK(hipHostMalloc((void **)&E.h_small, sizeof(int) * 4));
  HIPCHK(E.d_active.ensure(2));
  HIPCHK(E.d_eng_err.ensure(1));
  HIPCHK(hipMemsetAsync(E.d_eng_err.p, 0, sizeof(int), E.stream));
  HIPCHK(hipStreamSynchronize(E.stream));
  return MPO_OK;
}

void engine_destroy(Engine &E) {
  if (E.stream) hipStreamSynchronize(E.stream);
  for (auto &I : E.inst)
    for (void *p : I.allocs) hipFree(p);
  E.d_states.release();
  if (E.d_errs) hipFree(E.d_errs);
  E.d_gates.release();
  E.d_tot.release();
  E.d_base.release();
  E.d_fock.release();
  E.d_mirL.release();
  E.d_mirR.release();
  E.d_ctab.release();
  E.d_runs.release();
  E.d_blk.release();
  E.d_rows.release();
  E.d_cols.release();
  E.d_bigl.release();
  E.d_perm.release();
  E.d_piv.release();
  E.d_usize.release();
  E.d_sv.release();
  E.d_uval.release();
  E.d_ukey.release();
  E.d_A.release();
  E.d_A0.release();
  E.d_R.release();
  E.d_U.release();
  E.d_V.release();
  E.d_tau.release();
  E.d_rotf.release();
  E.d_tasks.release();
  E.d_qord.release();
  E.d_bord.release();
  E.d_pver.release();
  E.d_active.release();
  E.d_eng_err.release();
  if (E.h_errs) hipHostFree(E.h_errs);
  if (E.h_gates) hipHostFree(E.h_gates);
  if (E.h_tot) hipHostFree(E.h_tot);
  if (E.h_base) hipHostFree(E.h_base);
  if (E.h_small) hipHostFree(E.h_small);
  for (hipEvent_t ev : E.ev_pool) hipEventDestroy(ev);
  if (E.own_stream && E.stream) hipStreamDestroy(E.stream);
}

template <typename T>
hipError_t ialloc(Instance &I, T **p, size_t count) {
  *p = nullptr;
  hipError_t e = hipMalloc((void **)p, sizeof(T) * std::max<size_t>(count, 1));
  if (e == hipSuccess) I.allocs.push_back((void *)*p);
  return e;
}

// Projected device bytes of one simulation: the state, its readout scratch,
// and the larger of the one-off initial-state scratch and its share of the
// per-layer sector workspace (operand, pristine copy, left vectors and R
// factors: about 2.5 chi^2 elements per gate for each, plus the per-gate lists).
long long projected_bytes(int M, int d, int chi) {
  const long long W0 = (long long)M * (d - 1) + 1;
  const long long state = (long long)M * chi * chi * 16 + (long long)(M + 1) * chi * 60 +
                          (long long)M * d * ((chi + 3) / 4) * 8;
  const long long init = (long long)(M + 1) * W0 * W0 * 28;
  const long long layer = (long long)(M / 2) * (long long)(2.5 * chi * chi) * 56 +
                          (long long)(M / 2) * d * d * chi * 48;
  return state + std::max(init, layer);
}

int validate_args(int M, const double *r, double eta, int d, int chi, int precision) {
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
  return MPO_OK;
}

int upload_states(Engine &E) {
  if (!E.states_dirty) return MPO_OK;
  const int n = (int)E.inst.size();
  std::vector<State> tab(std::max(n, 1));
  for (int i = 0; i < n; ++i) tab[i] = E.inst[i].st;
  HIPCHK(E.d_states.ensure(std::max(n, 1)));
  HIPCHK(hipMemcpyAsync(E.d_states.p, tab.data(), sizeof(State) * std::max(n, 1),
                        hipMemcpyHostToDevice, E.stream));
  HIPCHK(hipStreamSynchronize(E.stream));
  E.states_dirty = false;
  return MPO_OK;
}

// A free slot for a new simulation (the error-word table grows by copy).
int engine_reserve_slot(Engine &E) {
  for (size_t i = 0; i < E.inst.size(); ++i)
    if (!E.inst[i].live && E.inst[i].id < 0) return (int)i;
  const size_t n = E.inst.size() + 1;
  if (E.errs_cap < n) {
    const size_t nc = std::max<size_t>(n * 2, 16);
    int *np = nullptr;
    if (hipMalloc((void **)&np, sizeof(int) * nc) != hipSuccess) return -1;
    if (hipMemsetAsync(np, 0, sizeof(int) * nc, E.stream) != hipSuccess) return -1;
    if (E.d_errs)
      hipMemcpyAsync(np, E.d_errs, sizeof(int) * E.errs_cap, hipMemcpyDeviceToDevice, E.stream);
    hipStreamSynchronize(E.stream);
    if (E.d_errs) hipFree(E.d_errs);
    E.d_errs = np;
    E.errs_cap = nc;
    for (size_t s = 0; s < E.inst.size(); ++s)
      if (E.inst[s].live) E.inst[s].st.err = np + s;
    if (E.h_errs) hipHostFree(E.h_errs);
    E.h_errs = nullptr;
    if (hipHostMalloc((void **)&E.h_errs, sizeof(int) * nc) != hipSuccess) return -1;
    E.states_dirty = true;
  }
  E.inst.resize(n);
  return (int)n - 1;
}

// Allocates and builds the initial state of a new simulation in `slot`
// (total_cap >= 0: projected onto at most total_cap photons in ket and bra).
int instance_create(Engine &E, int slot, int M, const double *r, double eta, int d, int chi,
                    int total_cap = -1) {
  Instance &I = E.inst[slot];
  I = Instance();
  I.live = true;
  State &st = I.st;
  st.M = M;
  st.d = d;
  st.chi = chi;
  st.max_sweeps = JACOBI_MAX_SWEEPS;
  HIPCHK(ialloc(I, &st.gam, (size_t)M * chi * chi));
  HIPCHK(ialloc(I, &st.lam, (size_t)(M + 1) * chi));
  HIPCHK(ialloc(I, &st.chg, (size_t)(M + 1) * chi));
  HIPCHK(ialloc(I, &st.dim, (size_t)(M + 1)));
  HIPCHK(ialloc(I, &st.ee, (size_t)(M + 1)));
  HIPCHK(ialloc(I, &st.ee_max, 1));
  HIPCHK(ialloc(I, &I.envL, (size_t)(M + 1) * chi));
  HIPCHK(ialloc(I, &I.envR, (size_t)(M + 1) * chi));
  HIPCHK(ialloc(I, &I.dP, (size_t)M * d));
  HIPCHK(ialloc(I, &I.dTrace, 1));
  HIPCHK(ialloc(I, &I.dPhase, (size_t)M));
  HIPCHK(ialloc(I, &I.dPart, marginals_scratch(M, d, chi)));
  st.err = E.d_errs + slot;
  HIPCHK(hipMemsetAsync(st.ee, 0, sizeof(double) * (M + 1), E.stream));
  HIPCHK(hipMemsetAsync(st.ee_max, 0, sizeof(unsigned long long), E.stream));
  HIPCHK(hipMemsetAsync(st.err, 0, sizeof(int), E.stream));
  // initial state
  std::vector<int> nint(M);
  for (int j = 0; j < M; ++j) nint[j] = internal_levels(r[j], d);
  std::vector<long long> woff(M + 2, 0);
  long long acc = 0;
  for (int b = M; b >= 0; --b) {
    const long long Wb = (long long)(M - b) * (d - 1) + 1;
    woff[b] = acc;
    acc += Wb * Wb;
  }
  woff[M + 1] = acc;
  const long long W0 = (long long)M * (d - 1) + 1;
  const long long ucap = W0 * W0;
  double *d_r = nullptr, *d_rho = nullptr, *d_A = nullptr, *d_w = nullptr, *d_V = nullptr;
  int *d_nint = nullptr, *d_us = nullptr;
  long long *d_woff = nullptr;
  unsigned long long *d_uv = nullptr, *d_uk = nullptr;
  std::vector<void *> tmp;
  auto cleanup = [&]() {
    hipStreamSynchronize(E.stream);
    for (void *p : tmp) hipFree(p);
    tmp.clear();
  };
  hipError_t e = hipSuccess;
#define TALLOC(p, count)                                                              \
  if (e == hipSuccess) {                                                              \
    e = hipMalloc((void **)&p, sizeof(*p) * std::max<size_t>((size_t)(count), 1));    \
    if (e == hipSuccess) tmp.push_back((void *)p);                                    \
  }
  TALLOC(d_r, M);
  TALLOC(d_nint, M);
  TALLOC(d_rho, (size_t)M * d * d);
  TALLOC(d_A, M + 1);
  TALLOC(d_w, acc);
  TALLOC(d_woff, M + 2);
  TALLOC(d_uv, (size_t)ucap * (M + 1));
  TALLOC(d_uk, (size_t)ucap * (M + 1));
  TALLOC(d_us, (size_t)ucap * (M + 1));
  if (total_cap >= 0) TALLOC(d_V, (size_t)(M + 1) * (total_cap + 1) * (total_cap + 1));
#undef TALLOC
  if (e != hipSuccess) {
    cleanup();
    return fail(e == hipErrorOutOfMemory ? MPO_ENOMEM : MPO_EDEVICE,
                std::string("initial-state scratch: ") + hipGetErrorString(e));
  }
  const double one = 1.0;
  if (e == hipSuccess) e = hipMemcpyAsync(d_r, r, sizeof(double) * M, hipMemcpyHostToDevice, E.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_nint, nint.data(), sizeof(int) * M, hipMemcpyHostToDevice, E.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_woff, woff.data(), sizeof(long long) * (M + 2), hipMemcpyHostToDevice,
                       E.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_w + woff[M], &one, sizeof(double), hipMemcpyHostToDevice, E.stream);
  if (e == hipSuccess) e = launch_init_rho(d_r, d_nint, eta, M, d, d_rho, E.stream);
  if (e == hipSuccess) e = launch_init_norms(d_rho, M, d, d_A, E.stream);
  for (int b = M - 1; b >= 0 && e == hipSuccess; --b)
    e = launch_init_conv(d_rho, M, d, b, d_woff, d_w, E.stream);
  if (e == hipSuccess && total_cap >= 0)
    e = launch_init_left(d_rho, M, d, total_cap, d_V, E.stream);
  if (e == hipSuccess)
    e = launch_init_select(st, d_w, d_woff, d_A, d_uv, d_uk, d_us, ucap, d_V, total_cap, E.stream);
  if (e == hipSuccess) e = launch_init_gamma(st, d_rho, d_A, d_V, total_cap, E.stream);
  if (e == hipSuccess) e = launch_entropy_all(st, E.stream);
  cleanup();
  if (e != hipSuccess) return fail(MPO_EDEVICE, hipGetErrorString(e));
  I.bytes = projected_bytes(M, d, chi);
  E.states_dirty = true;
  return MPO_OK;
}

// Frees a simulation's device memory (its results stay in the slot).
void instance_release(Engine &E, int slot) {
  Instance &I = E.inst[slot];
  hipStreamSynchronize(E.stream);
  for (void *p : I.allocs) hipFree(p);
  I.allocs.clear();
  if (I.live) E.committed -= I.bytes;
  I.live = false;
  I.bytes = 0;
  E.states_dirty = true;
}

// ------------------------------------------------------------------ one batched layer
int ensure_host(Engine &E, size_t n) {
  if (n <= E.h_cap) return MPO_OK;
  const size_t nc = std::max(n, E.h_cap * 2 + 16);
  if (E.h_gates) hipHostFree(E.h_gates);
  if (E.h_tot) hipHostFree(E.h_tot);
  if (E.h_base) hipHostFree(E.h_base);
  E.h_gates = nullptr;
  E.h_tot = nullptr;
  E.h_base = nullptr;
  HIPCHK(hipHostMalloc((void **)&E.h_gates, sizeof(GateParam) * nc));
  HIPCHK(hipHostMalloc((void **)&E.h_tot, sizeof(GateTot) * nc));
  HIPCHK(hipHostMalloc((void **)&E.h_base, sizeof(GateBase) * nc));
  E.h_cap = nc;
  return MPO_OK;
}

// Applies one batched layer: the gates (disjoint inside each simulation) of
// any number of simulations.  Fock tables and the count pass run for all
// gates at once; the rest runs in chunks of consecutive gates whose sector
// operands fit the pool budget.  With check_instances, an error latched by
// any live simulation fails the call; otherwise per-simulation errors are
// left to the caller (the engine retires the failing simulations only).
int engine_apply(Engine &E, const std::vector<GateParam> &gates, bool check_instances) {
  const int n = (int)gates.size();
  if (n == 0) return MPO_OK;
  int rc = upload_states(E);
  if (rc != MPO_OK) return rc;
  rc = ensure_host(E, n);
  if (rc != MPO_OK) return rc;
  long long fk = 0, mr = 0;
  int max_chi = 1, max_d = 2;
  for (int g = 0; g < n; ++g) {
    GateParam gp = gates[g];
    const State &st = E.inst[gp.inst].st;
    gp.fock0 = fk;
    gp.mir0 = mr;
    gp.blk0 = 0;
    gp.lst0 = 0;
    fk += (long long)(2 * st.d - 1) * st.d * st.d;
    mr += st.chi;
    max_chi = std::max(max_chi, st.chi);
    max_d = std::max(max_d, st.d);
    E.h_gates[g] = gp;
  }
  HIPCHK(E.d_gates.ensure(n));
  HIPCHK(E.d_tot.ensure(n));
  HIPCHK(E.d_base.ensure(n));
  HIPCHK(E.d_fock.ensure(fk));
  HIPCHK(E.d_mirL.ensure(mr));
  HIPCHK(E.d_mirR.ensure(mr));
  HIPCHK(hipMemcpyAsync(E.d_gates.p, E.h_gates, sizeof(GateParam) * n, hipMemcpyHostToDevice,
                        E.stream));
  Layer L{};
  L.states = E.d_states.p;
  L.fock = E.d_fock.p;
  L.mirL = E.d_mirL.p;
  L.mirR = E.d_mirR.p;
  L.ngates = n;
  L.gates = E.d_gates.p;
  L.tot = E.d_tot.p;
  L.base = E.d_base.p;
  L.panel_lds = panel_lds_bytes(max_chi);
  L.mixed = E.precision == MPO_MIXED ? 1 : 0;
  L.esz = L.mixed ? 8 : 16;
  {
    PhaseMark pm(E, 0);
    HIPCHK(launch_fock(L, E.stream));
  }
  {
    PhaseMark pm(E, 1);
    HIPCHK(launch_plan_count(L, E.stream));
  }
  HIPCHK(hipMemcpyAsync(E.h_tot, E.d_tot.p, sizeof(GateTot) * n, hipMemcpyDeviceToHost,
                        E.stream));
  rc = sync_and_check(E, check_instances);
  if (rc != MPO_OK) return rc;
  long long st_blk = 0, st_el = 0, st_sv = 0, st_mr = 0, st_mc = 0;
  double st_fl = 0.0, st_cf = 0.0;
  for (int g = 0; g < n; ++g) {
    const GateTot &t = E.h_tot[g];
    st_blk += t.nblk;
    st_el += t.elems;
    st_sv += t.sv;
    st_mr = std::max<long long>(st_mr, t.maxr);
    st_mc = std::max<long long>(st_mc, t.maxc);
    st_fl += t.svd_flops;
    st_cf += t.contr_flops;
  }
  if (E.prof) {
    E.work[0] += st_fl;
    E.work[1] += (double)st_el;
    E.work[2] += (double)st_sv;
    E.work[3] += 1.0;
    E.contr_flops += st_cf;
  }
  // centre-bond run tables of every gate
  long long ct = 0;
  for (int g = 0; g < n; ++g) {
    const GateTot &t = E.h_tot[g];
    E.h_gates[g].ct0 = ct;
    if (t.c1hi >= 0) ct += (long long)(t.c0hi - t.c0lo + 2) * (t.c1hi + 2);
  }
  HIPCHK(E.d_ctab.ensure(std::max(ct, 1LL)));
  HIPCHK(hipMemcpyAsync(E.d_gates.p, E.h_gates, sizeof(GateParam) * n, hipMemcpyHostToDevice,
                        E.stream));
  L.ctab = E.d_ctab.p;
  HIPCHK(launch_ctab(L, E.stream));
  E.last_blk_valid = false;
  // Every chunk is planned and every pool sized before the first chunk's
  // kernels run, so that a size limit or an allocation failure returns with
  // the state untouched (no chunk has scattered new tensors yet).
  struct Chunk {
    int c0, c1, blkb, bigb, maxpp;
    long long blk0, lst0, e, re;
  };
  std::vector<Chunk> chunks;
  std::vector<GateBase> bases(n);
  Chunk need{0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int c0 = 0; c0 < n;) {
    int c1 = c0;
    long long el = 0;
    while (c1 < n && (c1 == c0 || el + E.h_tot[c1].elems + E.h_tot[c1].relems <= E.pool_budget)) {
      el += E.h_tot[c1].elems + E.h_tot[c1].relems;
      ++c1;
    }
    Chunk ch{c0, c1, 0, 0, 0, 0, 0, 0, 0};
    for (int g = c0; g < c1; ++g) {
      const GateTot &t = E.h_tot[g];
      GateParam &gp = E.h_gates[g];
      gp.blk0 = ch.blk0;
      gp.lst0 = ch.lst0;
      ch.blk0 += std::max(t.nblk, 1);
      ch.lst0 += std::max(std::max(t.rows, t.cols), std::max(t.sv, 1));
      bases[g] = GateBase{ch.e, ch.blkb, ch.bigb, ch.re};
      ch.e += t.elems;
      ch.re += t.relems;
      ch.blkb += t.nblk;
      ch.bigb += t.nbig;
      ch.maxpp = std::max(ch.maxpp, t.maxpp);
    }
    if (ch.bigb > 65535 || ch.maxpp / 2 > 65535)
      return fail(MPO_EINVAL, "too many large sectors in one layer chunk");
    need.blk0 = std::max(need.blk0, ch.blk0);
    need.lst0 = std::max(need.lst0, ch.lst0);
    need.e = std::max(need.e, ch.e);
    need.re = std::max(need.re, ch.re);
    need.bigb = std::max(need.bigb, ch.bigb);
    chunks.push_back(ch);
    c0 = c1;
  }
  HIPCHK(E.d_blk.ensure(need.blk0));
  HIPCHK(E.d_runs.ensure((size_t)need.blk0 * 64));
  HIPCHK(E.d_rows.ensure(need.lst0));
  HIPCHK(E.d_cols.ensure(need.lst0));
  HIPCHK(E.d_bigl.ensure(need.lst0));
  HIPCHK(E.d_perm.ensure(need.lst0));
  HIPCHK(E.d_usize.ensure(need.lst0));
  HIPCHK(E.d_sv.ensure(need.lst0));
  HIPCHK(E.d_uval.ensure(need.lst0));
  HIPCHK(E.d_ukey.ensure(need.lst0));
  HIPCHK(E.d_A.ensure(std::max(need.e, 1LL), (size_t)E.pool_budget));
  HIPCHK(E.d_A0.ensure(std::max(need.e, 1LL), (size_t)E.pool_budget));
  HIPCHK(E.d_U.ensure(std::max(need.e, 1LL), (size_t)E.pool_budget));
  HIPCHK(E.d_R.ensure(std::max(need.re, 1LL), (size_t)E.pool_budget));
  HIPCHK(E.d_V.ensure(std::max(need.re, 1LL), (size_t)E.pool_budget));
  HIPCHK(E.d_tau.ensure(need.lst0));
  HIPCHK(E.d_piv.ensure(need.lst0));
  HIPCHK(E.d_rotf.ensure((size_t)4 * std::max(need.bigb, 1)));
  HIPCHK(E.d_tasks.ensure((size_t)2 * std::max(need.bigb, 1) + 1));
  long long max_blkb = 1;
  for (const Chunk &chk : chunks) max_blkb = std::max<long long>(max_blkb, chk.blkb);
  HIPCHK(E.d_qord.ensure((size_t)max_blkb));
  HIPCHK(E.d_bord.ensure((size_t)std::max(need.bigb, 1)));
  HIPCHK(E.d_pver.ensure((size_t)panel_version_ints() * std::max(need.bigb, 1)));
  for (const Chunk &chk : chunks) {
    const int c0 = chk.c0, c1 = chk.c1, ng = c1 - c0;
    const long long blk0 = chk.blk0;
    const int blkb = chk.blkb, bigb = chk.bigb, maxpp = chk.maxpp;
    for (int g = c0; g < c1; ++g) E.h_base[g - c0] = bases[g];
    HIPCHK(hipMemcpyAsync(E.d_gates.p + c0, E.h_gates + c0, sizeof(GateParam) * ng,
                          hipMemcpyHostToDevice, E.stream));
    HIPCHK(hipMemcpyAsync(E.d_base.p, E.h_base, sizeof(GateBase) * ng, hipMemcpyHostToDevice,
                          E.stream));
    Layer C = L;
    C.ngates = ng;
    C.gates = E.d_gates.p + c0;
    C.tot = E.d_tot.p + c0;
    C.base = E.d_base.p;
    C.blk = E.d_blk.p;
    C.runs = E.d_runs.p;
    C.rows = E.d_rows.p;
    C.cols = E.d_cols.p;
    C.bigl = E.d_bigl.p;
    C.perm = E.d_perm.p;
    C.usize = E.d_usize.p;
    C.sv = E.d_sv.p;
    C.uval = E.d_uval.p;
    C.ukey = E.d_ukey.p;
    C.A = E.d_A.p;
    C.A0 = E.d_A0.p;
    C.R = E.d_R.p;
    C.U = E.d_U.p;
    C.V = E.d_V.p;
    C.tau = E.d_tau.p;
    C.piv = E.d_piv.p;
    C.qr_order = E.d_qord.p;
    C.big_order = E.d_bord.p;
    C.pver = E.d_pver.p;
    C.rotf = E.d_rotf.p;
    C.active = E.d_active.p;
    C.task_blk = E.d_tasks.p;
    C.task_pre = E.d_tasks.p + std::max(bigb, 1);
    C.nact = 0;
    C.ntask = 0;
    C.total_blocks = blkb;
    C.total_big = bigb;
    C.maxpp = maxpp;
    {
      PhaseMark pm(E, 1);
      HIPCHK(launch_plan_fill(C, E.stream));
    }
    {
      PhaseMark pm(E, 2);
      HIPCHK(launch_contract(C, max_chi, max_d, E.stream));
    }
    int sweeps_run = 0;
    {
      PhaseMark pm(E, 3);
      HIPCHK(launch_qr(C, max_chi, E.stream));
      HIPCHK(launch_svd_small(C, E.stream));
      if (bigb > 0) {
        // panel rounds of the big blocks (each block at its own sweep); the
        // still-rotating blocks are compacted into the launch's task list and
        // counted every 16 launches
        HIPCHK(launch_svd_big_prep(C, E.stream));
        const int tmax = svd_max_steps(C);
        auto check = [&](int last, int next_step) -> int {
          HIPCHK(launch_svd_count(C, last, next_step, E.stream));
          HIPCHK(hipMemcpyAsync(E.h_small + 2, E.d_active.p, 2 * sizeof(int),
                                hipMemcpyDeviceToHost, E.stream));
          HIPCHK(hipStreamSynchronize(E.stream));
          C.nact = E.h_small[2];
          C.ntask = E.h_small[3];
          return MPO_OK;
        };
        int crc = check(0, 0);
        if (crc != MPO_OK) return crc;
        for (int t = 0; t < tmax && C.nact > 0; ++t) {
          HIPCHK(launch_svd_panel_step(C, t, E.stream));
          sweeps_run = t + 1;
          const bool last = t == tmax - 1;
          if ((t & 15) == 15 || last) {
            crc = check(last ? 1 : 0, t + 1);
            if (crc != MPO_OK) return crc;
          }
        }
        HIPCHK(launch_svd_big_finish(C, sweeps_run, max_chi, E.stream));
      }
    }
    (void)sweeps_run;
    {
      PhaseMark pm(E, 4);
      HIPCHK(launch_select(C, E.stream));
    }
    {
      PhaseMark pm(E, 5);
      HIPCHK(launch_leftvec(C, max_chi, E.stream));
      HIPCHK(launch_scatter(C, max_chi, E.stream));
    }
    {
      PhaseMark pm(E, 6);
      HIPCHK(launch_entropy_layer(C, E.stream));
    }
    if (c0 == 0 && c1 == n) {
      // the sector histogram of a single-chunk layer stays in d_blk; it is
      // copied to the host only by mpo_layer_blocks / mpo_layer_stats
      E.last_blk_valid = true;
      E.last_blk0.assign(n, 0);
      E.last_nblk.assign(n, 0);
      for (int g = 0; g < n; ++g) {
        E.last_blk0[g] = E.h_gates[g].blk0;
        E.last_nblk[g] = E.h_tot[g].nblk;
      }
      (void)blk0;
    }
  }
  E.stats[0] = st_blk;
  E.stats[1] = st_el;
  E.stats[2] = st_sv;
  E.stats[3] = st_mr;
  E.stats[4] = st_mc;
  E.stats[5] = -1;              // slowest block's sweeps: read lazily from d_blk
  return MPO_OK;
}

int readout_marginals(Engine &E, Instance &I, double *P, double *trace) {
  const int M = I.st.M, d = I.st.d;
  HIPCHK(launch_marginals(I.st, I.envL, I.envR, I.dPart, I.dP, I.dTrace, E.stream));
  std::vector<double> raw((size_t)M * d);
  double tr = 0.0;
  HIPCHK(hipMemcpyAsync(raw.data(), I.dP, sizeof(double) * M * d, hipMemcpyDeviceToHost,
                        E.stream));
  HIPCHK(hipMemcpyAsync(&tr, I.dTrace, sizeof(double), hipMemcpyDeviceToHost, E.stream));
  HIPCHK(hipStreamSynchronize(E.stream));
  // A truncated MPO need not be positive: at very small chi its trace can
  // reach zero or below; the marginals are then reported unnormalised.
  if (!std::isfinite(tr)) return fail(MPO_ENUMERIC, "non-finite trace");
  if (P)
    for (size_t i = 0; i < raw.size(); ++i) P[i] = tr != 0.0 ? raw[i] / tr : raw[i];
  if (trace) *trace = tr;
  return MPO_OK;
}

int readout_entropy(Engine &E, Instance &I, double *S, double *S_max) {
  const int M = I.st.M;
  std::vector<double> ee(M + 1);
  unsigned long long mx = 0;
  HIPCHK(hipMemcpyAsync(ee.data(), I.st.ee, sizeof(double) * (M + 1), hipMemcpyDeviceToHost,
                        E.stream));
  HIPCHK(hipMemcpyAsync(&mx, I.st.ee_max, sizeof(mx), hipMemcpyDeviceToHost, E.stream));
  HIPCHK(hipStreamSynchronize(E.stream));
  if (S)
    for (int b = 1; b < M; ++b) S[b - 1] = ee[b];
  if (S_max) {
    double m;
    std::memcpy(&m, &mx, sizeof(m));
    for (int b = 1; b < M; ++b) m = std::max(m, ee[b]);
    *S_max = m;
  }
  return MPO_OK;
}

bool valid_layer(int M, int n_gates, const int *left_site, const double *theta,
                 const double *phi) {
  std::vector<char> used(M, 0);
  for (int g = 0; g < n_gates; ++g) {
    const int k = left_site[g];
    if (k < 0 || k > M - 2) return false;
    if (used[k] || used[k + 1]) return false;
    if (!std::isfinite(theta[g]) || !std::isfinite(phi[g])) return false;
    used[k] = used[k + 1] = 1;
  }
  return true;
}

}  // namespace

// ============================================================================
// single-simulation C ABI
// ============================================================================
extern "C" const char *mpo_last_error(void) { return g_err.c_str(); }

extern "C" int gbs_device_memory(long long *free_bytes, long long *total_bytes) {
  if (!free_bytes || !total_bytes) return fail(MPO_EINVAL, "NULL argument");
  size_t fb = 0, tb = 0;
  HIPCHK(hipMemGetInfo(&fb, &tb));
  *free_bytes = (long long)fb;
  *total_bytes = (long long)tb;
  return MPO_OK;
}

extern "C" int gbs_set_svd_route(int lds_limit_bytes, int qr_enable) {
  if (lds_limit_bytes < 0) return fail(MPO_EINVAL, "LDS limit must be >= 0");
  set_svd_route(lds_limit_bytes, qr_enable);
  return MPO_OK;
}

extern "C" void mpo_free(gbs_mpo *h) {
  if (!h) return;
  engine_destroy(h->eng);
  delete h;
}

static int init_handle(int M, const double *r, double eta, int d, int chi, int precision,
                       void *hip_stream, gbs_mpo **out, int total_cap) {
  if (!out) return fail(MPO_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_args(M, r, eta, d, chi, precision);
  if (rc != MPO_OK) return rc;
  size_t fb = 0, tb = 0;
  if (hipMemGetInfo(&fb, &tb) != hipSuccess) return fail(MPO_EDEVICE, "hipMemGetInfo failed");
  if ((double)projected_bytes(M, d, chi) > 0.9 * (double)fb)
    return fail(MPO_ENOMEM, "projected device memory exceeds the free HBM");
  gbs_mpo *h = new gbs_mpo();
  rc = engine_init(h->eng, hip_stream, precision, 0);
  if (rc == MPO_OK && noalloc_scratch_init() != hipSuccess)
    rc = fail(MPO_EDEVICE, "device address of the static scratch array not found");
  if (rc == MPO_OK) {
    h->slot = engine_reserve_slot(h->eng);
    if (h->slot < 0) rc = fail(MPO_ENOMEM, "state table allocation failed");
  }
  if (rc == MPO_OK) rc = instance_create(h->eng, h->slot, M, r, eta, d, chi, total_cap);
  if (rc == MPO_OK) rc = upload_states(h->eng);
  if (rc == MPO_OK) rc = sync_and_check(h->eng);
  if (rc != MPO_OK) {
    mpo_free(h);
    return rc;
  }
  h->eng.inst[h->slot].id = 0;
  h->eng.committed += h->eng.inst[h->slot].bytes;
  *out = h;
  return MPO_OK;
}

extern "C" int mpo_init_lossy_squeezed(int M, const double *r, double eta, int d, int chi,
                                       int precision, void *hip_stream, gbs_mpo **out) {
  return init_handle(M, r, eta, d, chi, precision, hip_stream, out, -1);
}

extern "C" int mpo_init_lossy_squeezed_total_cap(int M, const double *r, double eta, int d,
                                                 int chi, int precision, void *hip_stream,
                                                 gbs_mpo **out) {
  return init_handle(M, r, eta, d, chi, precision, hip_stream, out, d - 1);
}

extern "C" int mpo_apply_bs_layer(gbs_mpo *h, int n_gates, const int *left_site,
                                  const double *theta, const double *phi) {
  if (!h) return fail(MPO_EINVAL, "handle is NULL");
  Instance &I = h->eng.inst[h->slot];
  const int M = I.st.M;
  if (n_gates < 0 || n_gates > M / 2) return fail(MPO_EINVAL, "n_gates out of range");
  if (n_gates == 0) return MPO_OK;
  if (!left_site || !theta || !phi) return fail(MPO_EINVAL, "NULL gate array");
  if (!valid_layer(M, n_gates, left_site, theta, phi))
    return fail(MPO_EINVAL, "gates must be disjoint, in range and finite");
  std::vector<GateParam> gates(n_gates);
  for (int g = 0; g < n_gates; ++g) {
    gates[g] = GateParam{};
    gates[g].site = left_site[g];
    gates[g].inst = h->slot;
    gates[g].theta = theta[g];
    gates[g].phi = phi[g];
  }
  return engine_apply(h->eng, gates, true);
}

extern "C" int mpo_apply_phases(gbs_mpo *h, const double *phase) {
  if (!h || !phase) return fail(MPO_EINVAL, "NULL argument");
  Instance &I = h->eng.inst[h->slot];
  for (int j = 0; j < I.st.M; ++j)
    if (!std::isfinite(phase[j])) return fail(MPO_EINVAL, "non-finite phase");
  HIPCHK(hipMemcpyAsync(I.dPhase, phase, sizeof(double) * I.st.M, hipMemcpyHostToDevice,
                        h->eng.stream));
  HIPCHK(launch_phases(I.st, I.dPhase, h->eng.stream));
  return sync_and_check(h->eng);
}

extern "C" int mpo_photon_marginals_noalloc(gbs_mpo *h, double *P, double *trace) {
  if (!h || !P) return fail(MPO_EINVAL, "NULL argument");
  const State &st = h->eng.inst[h->slot].st;
  if (marginals_noalloc_bytes(st.M, st.d, st.chi) > NOALLOC_SCRATCH_BYTES)
    return fail(MPO_EINVAL, "state too large for the static scratch array (needs " +
                                std::to_string(marginals_noalloc_bytes(st.M, st.d, st.chi)) +
                                " bytes, limit " + std::to_string(NOALLOC_SCRATCH_BYTES) + ")");
  int rc = sync_and_check(h->eng);
  if (rc != MPO_OK) return rc;
  double *dP = nullptr, *dT = nullptr;
  HIPCHK(launch_marginals_noalloc(st, &dP, &dT, h->eng.stream));
  double tr = 0.0;
  const int n = st.M * st.d;
  HIPCHK(hipMemcpyAsync(P, dP, sizeof(double) * n, hipMemcpyDeviceToHost, h->eng.stream));
  HIPCHK(hipMemcpyAsync(&tr, dT, sizeof(double), hipMemcpyDeviceToHost, h->eng.stream));
  HIPCHK(hipStreamSynchronize(h->eng.stream));
  if (!std::isfinite(tr)) return fail(MPO_ENUMERIC, "non-finite trace");
  if (tr != 0.0)
    for (int i = 0; i < n; ++i) P[i] /= tr;
  if (trace) *trace = tr;
  return MPO_OK;
}

extern "C" int mpo_sync(gbs_mpo *h) {
  if (!h) return fail(MPO_EINVAL, "handle is NULL");
  return sync_and_check(h->eng);
}

extern "C" int mpo_entropy(gbs_mpo *h, double *S, double *S_max_so_far) {
  if (!h || !S) return fail(MPO_EINVAL, "NULL argument");
  int rc = sync_and_check(h->eng);
  if (rc != MPO_OK) return rc;
  return readout_entropy(h->eng, h->eng.inst[h->slot], S, S_max_so_far);
}

extern "C" int mpo_photon_marginals(gbs_mpo *h, double *P, double *trace) {
  if (!h || !P) return fail(MPO_EINVAL, "NULL argument");
  int rc = sync_and_check(h->eng);
  if (rc != MPO_OK) return rc;
  return readout_marginals(h->eng, h->eng.inst[h->slot], P, trace);
}

extern "C" int mpo_renyi(gbs_mpo *h, double alpha, double *S) {
  if (!h || !S) return fail(MPO_EINVAL, "NULL argument");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(MPO_EINVAL, "alpha must be finite and >= 0");
  int rc = sync_and_check(h->eng);
  if (rc != MPO_OK) return rc;
  Instance &I = h->eng.inst[h->slot];
  const int M = I.st.M;
  // the marginals' output buffer (M * d doubles) holds the M - 1 values
  HIPCHK(launch_renyi(I.st, alpha, I.dP, h->eng.stream));
  HIPCHK(hipMemcpyAsync(S, I.dP, sizeof(double) * (M - 1), hipMemcpyDeviceToHost, h->eng.stream));
  HIPCHK(hipStreamSynchronize(h->eng.stream));
  return MPO_OK;
}

extern "C" int gbs_asymptotic_ee(double r, double mu, int n_max, double theta, int n_inputs,
                                 double alpha, double *S, double *spectrum) {
  if (!S) return fail(MPO_EINVAL, "S is NULL");
  if (!(r >= 0.0 && r <= 20.0)) return fail(MPO_EINVAL, "r must be in [0, 20]");
  if (!(mu > 0.0 && mu <= 1.0)) return fail(MPO_EINVAL, "mu must be in (0, 1]");
  if (n_max < 1 || n_max > 31) return fail(MPO_EINVAL, "n_max must be in [1, 31]");
  if (n_inputs < 0) return fail(MPO_EINVAL, "n_inputs must be >= 0");
  if (!std::isfinite(theta)) return fail(MPO_EINVAL, "theta must be finite");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(MPO_EINVAL, "alpha must be finite and >= 0");
  const int D = (n_max + 1) * (n_max + 1);
  double *X = nullptr, *spec = nullptr, *out = nullptr;
  int *err = nullptr;
  hipStream_t s = nullptr;
  auto release = [&]() {
    if (s) hipStreamSynchronize(s);
    if (X) hipFree(X);
    if (spec) hipFree(spec);
    if (out) hipFree(out);
    if (err) hipFree(err);
    if (s) hipStreamDestroy(s);
  };
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc((void **)&X, sizeof(double) * (size_t)D * D);
  if (e == hipSuccess) e = hipMalloc((void **)&spec, sizeof(double) * D);
  if (e == hipSuccess) e = hipMalloc((void **)&out, sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void **)&err, sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(err, 0, sizeof(int), s);
  if (e == hipSuccess) e = launch_asym(r, mu, n_max, theta, n_inputs, alpha, X, spec, out, err, s);
  int herr = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(S, out, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && spectrum)
    e = hipMemcpyAsync(spectrum, spec, sizeof(double) * D, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  release();
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? MPO_ENOMEM : MPO_EDEVICE, hipGetErrorString(e));
  if (herr) return fail(MPO_ENUMERIC, err_text(herr));
  return MPO_OK;
}

extern "C" int mpo_get_bond(gbs_mpo *h, int b, int *dim, double *lam, int *charges) {
  if (!h || !dim) return fail(MPO_EINVAL, "NULL argument");
  const State &st = h->eng.inst[h->slot].st;
  if (b < 0 || b > st.M) return fail(MPO_EINVAL, "bond out of range");
  int rc = sync_and_check(h->eng);
  if (rc != MPO_OK) return rc;
  int D = 0;
  HIPCHK(hipMemcpy(&D, st.dim + b, sizeof(int), hipMemcpyDeviceToHost));
  *dim = D;
  if (D > 0 && lam)
    HIPCHK(hipMemcpy(lam, st.lam + (size_t)b * st.chi, sizeof(double) * D,
                     hipMemcpyDeviceToHost));
  if (D > 0 && charges) {
    std::vector<int> c(D);
    HIPCHK(hipMemcpy(c.data(), st.chg + (size_t)b * st.chi, sizeof(int) * D,
                     hipMemcpyDeviceToHost));
    for (int i = 0; i < D; ++i) {
      charges[2 * i] = charge_n(c[i]);
      charges[2 * i + 1] = charge_np(c[i]);
    }
  }
  return MPO_OK;
}

extern "C" int mpo_get_site(gbs_mpo *h, int j, double *G) {
  if (!h || !G) return fail(MPO_EINVAL, "NULL argument");
  const State &st = h->eng.inst[h->slot].st;
  if (j < 0 || j >= st.M) return fail(MPO_EINVAL, "site out of range");
  int rc = sync_and_check(h->eng);
  if (rc != MPO_OK) return rc;
  int D[2];
  HIPCHK(hipMemcpy(D, st.dim + j, sizeof(int) * 2, hipMemcpyDeviceToHost));
  std::vector<cd> tmp((size_t)st.chi * st.chi);
  HIPCHK(hipMemcpy(tmp.data(), st.gam + (size_t)j * st.chi * st.chi,
                   sizeof(cd) * st.chi * st.chi, hipMemcpyDeviceToHost));
  for (int a = 0; a < D[0]; ++a)
    for (int b = 0; b < D[1]; ++b) {
      G[2 * ((size_t)a * D[1] + b)] = tmp[(size_t)a * st.chi + b].re;
      G[2 * ((size_t)a * D[1] + b) + 1] = tmp[(size_t)a * st.chi + b].im;
    }
  return MPO_OK;
}

// Sector histogram of the last layer (descriptors in layer order), copied
// from the device on demand; empty when the layer ran in several chunks.
static int last_blocks(Engine &E, std::vector<BlkDesc> &blk, std::vector<int> &gate) {
  blk.clear();
  gate.clear();
  if (!E.last_blk_valid) return MPO_OK;
  long long total = 0;
  for (size_t g = 0; g < E.last_blk0.size(); ++g)
    total = std::max(total, E.last_blk0[g] + std::max(E.last_nblk[g], 1));
  std::vector<BlkDesc> tmp((size_t)total);
  if (total > 0) {
    HIPCHK(hipMemcpyAsync(tmp.data(), E.d_blk.p, sizeof(BlkDesc) * total, hipMemcpyDeviceToHost,
                          E.stream));
    HIPCHK(hipStreamSynchronize(E.stream));
  }
  for (size_t g = 0; g < E.last_blk0.size(); ++g)
    for (int b = 0; b < E.last_nblk[g]; ++b) {
      blk.push_back(tmp[E.last_blk0[g] + b]);
      gate.push_back((int)g);
    }
  return MPO_OK;
}

extern "C" int mpo_layer_stats(gbs_mpo *h, long long *stats) {
  if (!h || !stats) return fail(MPO_EINVAL, "NULL argument");
  int rc = sync_and_check(h->eng);
  if (rc != MPO_OK) return rc;
  std::vector<BlkDesc> blk;
  std::vector<int> gate;
  rc = last_blocks(h->eng, blk, gate);
  if (rc != MPO_OK) return rc;
  long long sw = blk.empty() ? -1 : 0;
  for (const BlkDesc &B : blk)
    if (B.comp) sw = std::max<long long>(sw, B.sweeps);
  for (int i = 0; i < 5; ++i) stats[i] = h->eng.stats[i];
  stats[5] = sw;
  return MPO_OK;
}

extern "C" int mpo_layer_blocks(gbs_mpo *h, int max_blocks, int *out) {
  if (!h || max_blocks < 0 || (max_blocks > 0 && !out)) return fail(MPO_EINVAL, "bad argument");
  int rc = sync_and_check(h->eng, false);   // diagnostics stay readable after a numeric error
  if (rc != MPO_OK) return rc;
  std::vector<BlkDesc> blk;
  std::vector<int> gate;
  rc = last_blocks(h->eng, blk, gate);
  if (rc != MPO_OK) return rc;
  const int total = (int)blk.size();
  for (int i = 0; i < total && i < max_blocks; ++i) {
    const BlkDesc &B = blk[i];
    int *o = out + (size_t)8 * i;
    o[0] = gate[i];
    o[1] = charge_n(B.q);
    o[2] = charge_np(B.q);
    o[3] = B.r;
    o[4] = B.s;
    o[5] = B.comp;
    o[6] = B.sweeps;
    o[7] = B.kq;
  }
  return total;
}

static int set_profiling(Engine &E, int enable) {
  int rc = sync_and_check(E);
  if (rc != MPO_OK) return rc;
  E.prof = enable != 0;
  for (int p = 0; p < Engine::NPH; ++p) {
    E.ph_ms[p] = 0.0;
    E.ph_n[p] = 0;
  }
  for (double &x : E.work) x = 0.0;
  E.contr_flops = 0.0;
  return MPO_OK;
}

static int get_profile(Engine &E, double *phase_ms, long long *phase_launches, double *work) {
  int rc = sync_and_check(E);
  if (rc != MPO_OK) return rc;
  for (int p = 0; p < Engine::NPH; ++p) {
    if (phase_ms) phase_ms[p] = E.ph_ms[p];
    if (phase_launches) phase_launches[p] = E.ph_n[p];
  }
  if (work)
    for (int i = 0; i < 4; ++i) work[i] = E.work[i];
  return MPO_OK;
}

extern "C" int mpo_get_contraction_work(gbs_mpo *h, double *flops) {
  if (!h || !flops) return fail(MPO_EINVAL, "NULL argument");
  int rc = sync_and_check(h->eng);
  if (rc != MPO_OK) return rc;
  *flops = h->eng.contr_flops;
  return MPO_OK;
}

extern "C" int mpo_set_profiling(gbs_mpo *h, int enable) {
  if (!h) return fail(MPO_EINVAL, "handle is NULL");
  return set_profiling(h->eng, enable);
}

extern "C" int mpo_get_profile(gbs_mpo *h, double *phase_ms, long long *phase_launches,
                               double *work) {
  if (!h) return fail(MPO_EINVAL, "handle is NULL");
  return get_profile(h->eng, phase_ms, phase_launches, work);
}

// ============================================================================
// batched / continuous-batching engine C ABI
// ============================================================================
extern "C" long long mpo_engine_projected_bytes(int M, int d, int chi) {
  if (M < 2 || d < 2 || chi < 1) return -1;
  return projected_bytes(M, d, chi);
}

extern "C" int mpo_engine_create(void *hip_stream, int precision, long long budget_bytes,
                                 gbs_engine **out) {
  if (!out) return fail(MPO_EINVAL, "out is NULL");
  *out = nullptr;
  if (precision != MPO_FP64 && precision != MPO_MIXED)
    return fail(MPO_EINVAL, "precision must be MPO_FP64 or MPO_MIXED");
  if (budget_bytes < 0) return fail(MPO_EINVAL, "budget must be >= 0");
  gbs_engine *e = new gbs_engine();
  int rc = engine_init(e->eng, hip_stream, precision, budget_bytes);
  if (rc != MPO_OK) {
    engine_destroy(e->eng);
    delete e;
    return rc;
  }
  *out = e;
  return MPO_OK;
}

extern "C" void mpo_engine_free(gbs_engine *e) {
  if (!e) return;
  engine_destroy(e->eng);
  delete e;
}

extern "C" int mpo_engine_add(gbs_engine *e, int M, const double *r, double eta, int d, int chi,
                              const double *U_reim, int *id) {
  if (!e || !id || !U_reim) return fail(MPO_EINVAL, "NULL argument");
  Engine &E = e->eng;
  int rc = validate_args(M, r, eta, d, chi, E.precision);
  if (rc != MPO_OK) return rc;
  const long long need = projected_bytes(M, d, chi);
  if (E.committed + need > E.budget)
    return fail(MPO_ENOMEM, "projected memory of the request exceeds the free budget");
  const int G = M * (M - 1) / 2;
  std::vector<int> lptr(M + 1), site(std::max(G, 1));
  std::vector<double> theta(std::max(G, 1)), phi(std::max(G, 1)), phase(M);
  const int nl = gbs_clements_decompose(M, U_reim, lptr.data(), site.data(), theta.data(),
                                        phi.data(), phase.data());
  if (nl < 0) return fail(MPO_EINVAL, "interferometer is not unitary");
  lptr.resize(nl + 1);
  const int slot = engine_reserve_slot(E);
  if (slot < 0) return fail(MPO_ENOMEM, "state table allocation failed");
  rc = instance_create(E, slot, M, r, eta, d, chi);
  if (rc != MPO_OK) {
    Instance &I = E.inst[slot];
    for (void *p : I.allocs) hipFree(p);
    I = Instance();
    E.states_dirty = true;
    return rc;
  }
  Instance &I = E.inst[slot];
  I.lptr = std::move(lptr);
  I.site = std::move(site);
  I.theta = std::move(theta);
  I.phi = std::move(phi);
  I.next_layer = 0;
  I.id = E.next_id++;
  E.committed += I.bytes;
  if (nl == 0) {
    I.done = true;
    I.P.assign((size_t)M * d, 0.0);
    int rr = readout_entropy(E, I, nullptr, &I.smax);
    if (rr == MPO_OK) rr = readout_marginals(E, I, I.P.data(), &I.trace);
    I.status = rr;
    instance_release(E, slot);
  }
  *id = I.id;
  return MPO_OK;
}

// Applies the next layer of every live, unfinished simulation in one batched
// launch sequence; simulations whose last layer was applied are retired
// (readouts taken, device memory released).
extern "C" int mpo_engine_step(gbs_engine *e, int *n_active) {
  if (!e) return fail(MPO_EINVAL, "engine is NULL");
  Engine &E = e->eng;
  std::vector<GateParam> gates;
  std::vector<int> stepped;
  for (size_t s = 0; s < E.inst.size(); ++s) {
    Instance &I = E.inst[s];
    if (!I.live || I.done) continue;
    const int l = I.next_layer;
    for (int g = I.lptr[l]; g < I.lptr[l + 1]; ++g) {
      GateParam gp{};
      gp.site = I.site[g];
      gp.inst = (int)s;
      gp.theta = I.theta[g];
      gp.phi = I.phi[g];
      gates.push_back(gp);
    }
    stepped.push_back((int)s);
  }
  int rc = engine_apply(E, gates, false);
  if (rc != MPO_OK) return rc;
  rc = sync_and_check(E, false);
  if (rc != MPO_OK) return rc;
  int active = 0;
  for (int s : stepped) {
    Instance &I = E.inst[s];
    ++I.next_layer;
    const int err = E.h_errs[s];
    if (err || I.next_layer + 1 >= (int)I.lptr.size()) {
      // finished, or failed on the device: retire (a failure stays in status)
      I.done = true;
      I.P.assign((size_t)I.st.M * I.st.d, 0.0);
      int rr = err ? fail(MPO_ENUMERIC, err_text(err)) : MPO_OK;
      if (rr == MPO_OK) rr = readout_entropy(E, I, nullptr, &I.smax);
      if (rr == MPO_OK) rr = readout_marginals(E, I, I.P.data(), &I.trace);
      I.status = rr;
      if (rr != MPO_OK) I.msg = g_err;
      instance_release(E, s);
    } else {
      ++active;
    }
  }
  if (n_active) *n_active = active;
  return MPO_OK;
}

extern "C" int mpo_engine_result(gbs_engine *e, int id, int *done, double *S_max, double *trace,
                                 double *P) {
  if (!e || !done) return fail(MPO_EINVAL, "NULL argument");
  Engine &E = e->eng;
  for (auto &I : E.inst) {
    if (I.id != id) continue;
    *done = (I.done && !I.live) ? 1 : 0;
    if (*done) {
      if (I.status != MPO_OK) return fail(I.status, "simulation failed: " + I.msg);
      if (S_max) *S_max = I.smax;
      if (trace) *trace = I.trace;
      if (P) std::copy(I.P.begin(), I.P.end(), P);
    }
    return MPO_OK;
  }
  return fail(MPO_EINVAL, "unknown simulation id");
}

extern "C" int mpo_engine_release(gbs_engine *e, int id) {
  if (!e) return fail(MPO_EINVAL, "engine is NULL");
  Engine &E = e->eng;
  for (size_t s = 0; s < E.inst.size(); ++s) {
    Instance &I = E.inst[s];
    if (I.id != id) continue;
    if (I.live) return fail(MPO_EBUSY, "simulation still running");
    I = Instance();
    return MPO_OK;
  }
  return fail(MPO_EINVAL, "unknown simulation id");
}

extern "C" int mpo_engine_set_sweep_limit(gbs_engine *e, int id, int max_sweeps) {
  if (!e) return fail(MPO_EINVAL, "engine is NULL");
  if (max_sweeps < 1 || max_sweeps > JACOBI_MAX_SWEEPS)
    return fail(MPO_EINVAL, "sweep limit must be in [1, 60]");
  Engine &E = e->eng;
  for (auto &I : E.inst) {
    if (I.id != id) continue;
    if (!I.live || I.done) return fail(MPO_EINVAL, "simulation is not running");
    I.st.max_sweeps = max_sweeps;
    E.states_dirty = true;
    return MPO_OK;
  }
  return fail(MPO_EINVAL, "unknown simulation id");
}

extern "C" int mpo_engine_set_profiling(gbs_engine *e, int enable) {
  if (!e) return fail(MPO_EINVAL, "engine is NULL");
  return set_profiling(e->eng, enable);
}

extern "C" int mpo_engine_get_profile(gbs_engine *e, double *phase_ms, long long *phase_launches,
                                      double *work) {
  if (!e) return fail(MPO_EINVAL, "engine is NULL");
  return get_profile(e->eng, phase_ms, phase_launches, work);
}
