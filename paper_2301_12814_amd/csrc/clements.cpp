// Host-only helper: rectangular (Clements et al., Optica 3, 1460 (2016))
// decomposition of an interferometer into nearest-neighbour beam splitters,
// the M-layer array the paper uses for its Haar-random interferometers
// (App. A).  Elements null the lower triangle alternately from the right
// (T^dag on columns) and from the left (T on rows); the left elements are then
// moved through the remaining diagonal, L^dag D = D' T(theta, phi').
#include <cmath>
#include <complex>
#include <string>
#include <vector>

#include "../../include/gbs_mpo.h"

namespace {

using cplx = std::complex<double>;

struct Elem {
  int m;
  double theta, phi;
};

double wrap_angle(double x) {
  double y = std::remainder(x, 2.0 * M_PI);
  return (y == -M_PI) ? M_PI : y;
}

// entries of T(theta, phi)
void t_entries(double th, double ph, cplx &t11, cplx &t12, cplx &t21, cplx &t22) {
  const cplx e = std::polar(1.0, ph);
  t11 = e * std::cos(th);
  t12 = -std::sin(th);
  t21 = e * std::sin(th);
  t22 = std::cos(th);
}

}  // namespace

extern "C" int gbs_clements_decompose(int M, const double *U_reim, int *layer_ptr, int *left_site,
                                      double *theta, double *phi, double *phase) {
  if (M < 2 || !U_reim || !layer_ptr || !left_site || !theta || !phi || !phase)
    return MPO_EINVAL;
  std::vector<cplx> V((size_t)M * M);
  for (int i = 0; i < M * M; ++i) V[i] = cplx(U_reim[2 * i], U_reim[2 * i + 1]);
  // unitarity check
  for (int i = 0; i < M; ++i)
    for (int k = 0; k < M; ++k) {
      cplx acc = 0.0;
      for (int j = 0; j < M; ++j) acc += V[(size_t)i * M + j] * std::conj(V[(size_t)k * M + j]);
      if (std::abs(acc - (i == k ? 1.0 : 0.0)) > 1e-10) return MPO_EINVAL;
    }
  auto at = [&](int i, int j) -> cplx & { return V[(size_t)i * M + j]; };
  std::vector<Elem> right, left;
  for (int i = 0; i < M - 1; ++i) {
    if (i % 2 == 0) {
      for (int j = 0; j <= i; ++j) {
        const int row = M - 1 - j, col = i - j;
        const cplx a = at(row, col), b = at(row, col + 1);
        const double th = std::atan2(std::abs(a), std::abs(b));
        const double ph = (a == 0.0 || b == 0.0) ? 0.0 : wrap_angle(std::arg(a) - std::arg(b));
        cplx t11, t12, t21, t22;
        t_entries(th, ph, t11, t12, t21, t22);
        // V <- V T^dag on columns (col, col+1)
        for (int r = 0; r < M; ++r) {
          const cplx x = at(r, col), y = at(r, col + 1);
          at(r, col) = x * std::conj(t11) + y * std::conj(t12);
          at(r, col + 1) = x * std::conj(t21) + y * std::conj(t22);
        }
        right.push_back({col, th, ph});
      }
    } else {
      for (int j = 0; j <= i; ++j) {
        const int row = M - 1 - i + j, col = j;
        const cplx a = at(row - 1, col), b = at(row, col);
        const double th = std::atan2(std::abs(b), std::abs(a));
        const double ph =
            (a == 0.0 || b == 0.0) ? 0.0 : wrap_angle(M_PI + std::arg(b) - std::arg(a));
        cplx t11, t12, t21, t22;
        t_entries(th, ph, t11, t12, t21, t22);
        // V <- T V on rows (row-1, row)
        for (int c = 0; c < M; ++c) {
          const cplx x = at(row - 1, c), y = at(row, c);
          at(row - 1, c) = t11 * x + t12 * y;
          at(row, c) = t21 * x + t22 * y;
        }
        left.push_back({row - 1, th, ph});
      }
    }
  }
  std::vector<cplx> dg(M);
  for (int i = 0; i < M; ++i) dg[i] = at(i, i);
  std::vector<Elem> gates = right;
  for (int k = (int)left.size() - 1; k >= 0; --k) {
    const Elem L = left[k];
    const cplx d1 = dg[L.m], d2 = dg[L.m + 1];
    const double ph_new = wrap_angle(std::arg(-d1 / d2));
    dg[L.m] = -std::polar(1.0, -L.phi) * d2;
    gates.push_back({L.m, L.theta, ph_new});
  }
  // as-soon-as-possible layering of disjoint pairs
  std::vector<int> last(M, 0), layer_of(gates.size());
  int nlayers = 0;
  for (size_t g = 0; g < gates.size(); ++g) {
    const int m = gates[g].m;
    const int Lg = std::max(last[m], last[m + 1]);
    layer_of[g] = Lg;
    last[m] = last[m + 1] = Lg + 1;
    nlayers = std::max(nlayers, Lg + 1);
  }
  int pos = 0;
  for (int l = 0; l < nlayers; ++l) {
    layer_ptr[l] = pos;
    for (size_t g = 0; g < gates.size(); ++g)
      if (layer_of[g] == l) {
        left_site[pos] = gates[g].m;
        theta[pos] = gates[g].theta;
        phi[pos] = gates[g].phi;
        ++pos;
      }
  }
  layer_ptr[nlayers] = pos;
  for (int i = 0; i < M; ++i) phase[i] = std::arg(dg[i]);
  return nlayers;
}
