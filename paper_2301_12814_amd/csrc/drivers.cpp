// Experiment drivers of App. A on top of the library's own C ABI: the
// EE-saturation stop rule and the fixed-accuracy bond-dimension search.
// Host orchestration only; every gate, SVD and readout runs in the library's
// kernels through the calls declared in gbs_mpo.h.
#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/gbs_mpo.h"
#include "internal.h"

namespace {

// An EE "increase" must exceed the best value so far by more than this many
// bits (the paper gives no threshold; rounding must not count).
constexpr double kEeEps = 1e-12;

struct Circuit {
  int M = 0, nl = 0;
  std::vector<int> ptr, site;
  std::vector<double> theta, phi, phase;
};

int decompose(int M, const double *U_reim, Circuit &c) {
  const int G = M * (M - 1) / 2;
  c.M = M;
  c.ptr.assign(M + 1, 0);
  c.site.assign(std::max(G, 1), 0);
  c.theta.assign(std::max(G, 1), 0.0);
  c.phi.assign(std::max(G, 1), 0.0);
  c.phase.assign(M, 0.0);
  if (M < 2 || M > 4096) return gbs::set_error(MPO_EINVAL, "M must be in [2, 4096]");
  c.nl = gbs_clements_decompose(M, U_reim, c.ptr.data(), c.site.data(), c.theta.data(),
                                c.phi.data(), c.phase.data());
  return c.nl < 0 ? gbs::set_error(c.nl, "interferometer is not unitary") : MPO_OK;
}

int apply_layer(gbs_mpo *h, const Circuit &c, int l) {
  const int g0 = c.ptr[l], n = c.ptr[l + 1] - c.ptr[l];
  return mpo_apply_bs_layer(h, n, c.site.data() + g0, c.theta.data() + g0, c.phi.data() + g0);
}

// 1 - Tr rho after the whole circuit at bond dimension chi.
int error_at(int M, const double *r, double eta, int d, int chi, int precision, const Circuit &c,
             double *err) {
  gbs_mpo *h = nullptr;
  int rc = mpo_init_lossy_squeezed(M, r, eta, d, chi, precision, nullptr, &h);
  for (int l = 0; rc == MPO_OK && l < c.nl; ++l) rc = apply_layer(h, c, l);
  std::vector<double> P((size_t)M * d);
  double tr = 0.0;
  if (rc == MPO_OK) rc = mpo_photon_marginals(h, P.data(), &tr);
  mpo_free(h);
  if (rc == MPO_OK) *err = 1.0 - tr;
  return rc;
}

}  // namespace

extern "C" int gbs_run_until_saturation(int M, const double *r, double eta, int d, int chi,
                                        int precision, const double *U_reim, int patience,
                                        int *layers_used, double *S_max, int *layer_of_max,
                                        double *trace) {
  if (!U_reim || !layers_used || !S_max || !layer_of_max || patience < 1)
    return gbs::set_error(MPO_EINVAL, "NULL output or patience < 1");
  Circuit c;
  int rc = decompose(M, U_reim, c);
  if (rc != MPO_OK) return rc;
  gbs_mpo *h = nullptr;
  rc = mpo_init_lossy_squeezed(M, r, eta, d, chi, precision, nullptr, &h);
  if (rc != MPO_OK) return rc;
  std::vector<double> S(std::max(M - 1, 1));
  double best = 0.0;
  bool have = false;
  int at = 0, since = 0, used = 0;
  for (int l = 0; l < c.nl; ++l) {
    rc = apply_layer(h, c, l);
    if (rc == MPO_OK) rc = mpo_entropy(h, S.data(), nullptr);
    if (rc != MPO_OK) break;
    ++used;
    const double s = *std::max_element(S.begin(), S.begin() + (M - 1));
    if (!have || s > best + kEeEps) {
      best = s;
      at = used;
      since = 0;
      have = true;
    } else if (++since >= patience) {
      break;
    }
  }
  if (rc == MPO_OK && trace) {
    std::vector<double> P((size_t)M * d);
    rc = mpo_photon_marginals(h, P.data(), trace);
  }
  mpo_free(h);
  if (rc != MPO_OK) return rc;
  *layers_used = used;
  *S_max = best;
  *layer_of_max = at;
  return MPO_OK;
}

extern "C" int gbs_chi_search(int M, const double *r, double eta, int d, int precision,
                              const double *U_reim, int chi0, int chi_max, double target,
                              int refine, int *chi_found, double *err_found, int max_trials,
                              int *n_trials, int *trial_chi, double *trial_err) {
  if (!U_reim || !chi_found || !err_found || chi0 < 1 || chi_max < chi0 || refine < 0 ||
      !(target >= 0.0) || max_trials < 0 || (max_trials > 0 && (!trial_chi || !trial_err)))
    return gbs::set_error(MPO_EINVAL, "bad chi range, target, refine count or trial buffers");
  Circuit c;
  int rc = decompose(M, U_reim, c);
  if (rc != MPO_OK) return rc;
  int nt = 0;
  auto err = [&](int chi, double *e) -> int {
    int rr = error_at(M, r, eta, d, chi, precision, c, e);
    if (rr != MPO_OK) return rr;
    if (nt < max_trials) {
      trial_chi[nt] = chi;
      trial_err[nt] = *e;
    }
    ++nt;
    return MPO_OK;
  };
  // doubling until the target is met, then bisection between the last
  // failing and the first passing bond dimension (App. A)
  int lo = -1, chi = chi0;
  double e = 0.0;
  if ((rc = err(chi, &e)) != MPO_OK) return rc;
  bool found = true;
  while (e > target) {
    if (chi >= chi_max) {
      found = false;
      break;
    }
    lo = chi;
    chi = std::min(2 * chi, chi_max);
    if ((rc = err(chi, &e)) != MPO_OK) return rc;
  }
  int hi = chi;
  double ehi = e;
  if (found)
    for (int k = 0; k < refine && lo >= 0 && hi - lo > 1; ++k) {
      const int mid = (lo + hi) / 2;
      double em = 0.0;
      if ((rc = err(mid, &em)) != MPO_OK) return rc;
      if (em <= target) {
        hi = mid;
        ehi = em;
      } else {
        lo = mid;
      }
    }
  *chi_found = found ? hi : -1;
  *err_found = ehi;
  if (n_trials) *n_trials = nt;
  return MPO_OK;
}
