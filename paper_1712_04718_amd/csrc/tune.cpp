// Ewald and SE parameters from an error tolerance (host code only).
//
// Truncation estimates of Kolafa and Perram (section 2.1, eqs. 2.1-2.2), their
// inversions for xi and k_inf (eqs. 2.3-2.4), the SE approximation-error
// estimates (sections 5.1-5.3), and a runtime model of the section 7 form
// whose minimum over the cutoff picks (rc, xi, M, P).
#include <cmath>
#include <cstdio>

#include "sekspace.h"

namespace sek {
se_status report(se_status s, const char *msg);
int tile_edge_of(const se_params &p);
int rs_reach(double L, double rc, long long N);
int rs_cells_per_side(double L, double rc, int reach);
}

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kDefaultC = 0.95;
constexpr int kPMin = 4, kPMax = 16;     // Gaussian supports the kernels are built for
constexpr int kMMin = 8, kMMax = 512;    // grid sizes se_plan_create accepts
// Largest eta the selection takes.  The approximation estimate of section 5
// is derived at M = 2 k_inf ~ 4 xi L, where eta = P / (16 pi c^2) <= 0.36 for
// P <= 16; measured errors stay under it up to eta ~ 0.5 and exceed it
// several-fold as eta approaches 1.
constexpr double kEtaMax = 0.5;

bool pos(double v) { return std::isfinite(v) && v > 0.0; }

se_status bad(const char *what) { return sek::report(SE_ERR_ARG, what); }

// Principal branch of Lambert W at z = e^y (z > 0), i.e. the root w > 0 of
// f(w) = w + ln w - y.  f is increasing and concave, so Newton's method from a
// start below the root climbs to it monotonically.  Starts below the root:
// z/(1+z) <= W(z) for z <= e, and y - ln y <= W(e^y) for y > 1.
double lambert_w_exp(double y) {
  if (y < -700.0) return std::exp(y);  // W(z) = z (1 - z + ...) below double's resolution
  double w;
  if (y > 1.0) {
    w = y - std::log(y);
  } else {
    const double z = std::exp(y);
    w = z / (1.0 + z);
  }
  for (int it = 0; it < 100; ++it) {
    const double f = w + std::log(w) - y;
    const double step = f / (1.0 + 1.0 / w);
    const double wn = w - step;
    if (!(wn > 0.0)) break;  // cannot happen from below the root; guards NaN input
    if (std::fabs(wn - w) <= 1e-16 * wn) {
      w = wn;
      break;
    }
    w = wn;
  }
  return w;
}

bool kind_ok(int k) { return k == SE_EST_POTENTIAL || k == SE_EST_ENERGY || k == SE_EST_FORCE; }

double real_err(int kind, double Q, double L, double xi, double rc) {
  const double g = std::exp(-(rc * xi) * (rc * xi));
  const double L3 = L * L * L;
  switch (kind) {
    case SE_EST_POTENTIAL: return std::sqrt(Q * rc / (2.0 * L3)) / ((xi * rc) * (xi * rc)) * g;
    case SE_EST_ENERGY: return Q * std::sqrt(rc / (2.0 * L3)) / ((xi * rc) * (xi * rc)) * g;
    default: return 2.0 * Q * std::sqrt(1.0 / (rc * L3)) * g;
  }
}

double fourier_err(int kind, double Q, double L, double xi, double kinf) {
  const double t = kPi * kinf / (xi * L);
  const double g = std::exp(-t * t);
  switch (kind) {
    case SE_EST_POTENTIAL: return xi / (kPi * kPi) * std::pow(kinf, -1.5) * std::sqrt(Q) * g;
    case SE_EST_ENERGY: return xi / (kPi * kPi) * std::pow(kinf, -1.5) * Q * g;
    default: return xi / (L * kPi) * std::sqrt(8.0 / kinf) * Q * g;
  }
}

// xi solving real_err = eps; false when the force form has no solution.
bool xi_of(int kind, double eps, double Q, double L, double rc, double *xi) {
  const double L3 = L * L * L;
  double s;  // (xi rc)^2
  switch (kind) {
    case SE_EST_POTENTIAL:  // (xi rc)^2 e^{(xi rc)^2} = sqrt(Q rc / 2 L^3) / eps
      s = lambert_w_exp(0.5 * std::log(Q * rc / (2.0 * L3)) - std::log(eps));
      break;
    case SE_EST_ENERGY:
      s = lambert_w_exp(std::log(Q) + 0.5 * std::log(rc / (2.0 * L3)) - std::log(eps));
      break;
    default:
      s = std::log(2.0 * Q / eps) - 0.5 * std::log(rc * L3);
      if (!(s > 0.0)) return false;
  }
  *xi = std::sqrt(s) / rc;
  return true;
}

// k_inf solving fourier_err = eps, with the W argument formed in logarithms.
double kinf_of(int kind, double eps, double Q, double L, double xi) {
  if (kind == SE_EST_FORCE) {  // W(2^8 xi^2 Q^4 / (eps^4 L^6 pi^2))
    const double y = 8.0 * std::log(2.0) + 2.0 * std::log(xi) + 4.0 * std::log(Q) -
                     4.0 * std::log(eps) - 6.0 * std::log(L) - 2.0 * std::log(kPi);
    return L * xi / (2.0 * kPi) * std::sqrt(lambert_w_exp(y));
  }
  // W(4/(3 L^2) (Q^a / (pi xi eps^2))^{2/3}), a = 1 (potential) or 2 (energy)
  const double a = kind == SE_EST_ENERGY ? 2.0 : 1.0;
  const double y = std::log(4.0 / 3.0) - 2.0 * std::log(L) +
                   (2.0 / 3.0) * (a * std::log(Q) - std::log(kPi * xi) - 2.0 * std::log(eps));
  return std::sqrt(3.0) * L * xi / (2.0 * kPi) * std::sqrt(lambert_w_exp(y));
}

double se_amp(int kind, double Q, double L, double xi) {
  switch (kind) {
    case SE_EST_POTENTIAL: return std::sqrt(Q * xi * L) / L;
    case SE_EST_ENERGY: return Q * std::sqrt(xi * L) / L;
    default: return 4.0 * kPi * Q * std::sqrt(xi * xi * xi / L);
  }
}

double se_err(int kind, double Q, double L, double xi, int P, double c) {
  return se_amp(kind, Q, L, xi) * std::exp(-kPi * P * c * c / 2.0);
}

int support_of(int kind, double eps, double Q, double L, double xi, double c) {
  for (int P = 2; P <= 64; P += 2)
    if (se_err(kind, Q, L, xi, P, c) <= eps) return P;
  return 0;
}

bool only_235(int m) {
  for (int f : {2, 3, 5})
    while (m % f == 0) m /= f;
  return m == 1;
}

// Real-space work-groups resident at once on a 256-CU device: FP32 four per
// CU (five with the smaller stage it takes above 1024 cells), FP64 two.
inline double rs_resident(int dtype, double ncells) {
  if (dtype == SE_FP64) return 512.0;
  return ncells > 1024.0 ? 1280.0 : 1024.0;
}

// The runtime model (terms as documented with se_cost_model); false when no
// tile edge fits (M, P) in this precision.
bool predict(const se_cost_model &cm, int dtype, int N, double L, double rc, int M, int P,
             double *t_real, double *t_k) {
  const int reach = sek::rs_reach(L, rc, N);
  const double nc = sek::rs_cells_per_side(L, rc, reach);
  const double ncells = nc * nc * nc;
  const double cs = L / nc;
  const double L3 = L * L * L;
  const double w = 2.0 * reach + 1.0;  // neighbour cells searched per side
  const double ntest = w * w * w * cs * cs * cs * N / L3;
  const double res = rs_resident(dtype, ncells);
  const double q = std::ceil(ncells / res) * res / ncells;
  const double nbar = 4.0 / 3.0 * kPi * rc * rc * rc * N / L3;
  se_params prm{};
  prm.M = M;
  prm.P = P;
  prm.L = L;
  prm.xi = 1.0;
  prm.c = kDefaultC;
  prm.window = SE_WINDOW_GAUSSIAN;
  prm.dtype = dtype;
  const int T = sek::tile_edge_of(prm);
  if (T == 0) return false;
  const double nt = std::ceil(static_cast<double>(M) / T);
  const double blk = static_cast<double>(T + P - 1);
  const double M3 = static_cast<double>(M) * M * M;
  *t_real = cm.real_fixed + cm.real_atom * N + cm.real_pair * N * nbar + cm.real_cell * ncells +
            cm.real_test * N * ntest * q;
  *t_k = cm.k_fixed + cm.k_atom * N + cm.k_window * N * std::pow(P, 3) +
         cm.k_block * nt * nt * nt * blk * blk * blk + cm.k_grid * M3 +
         cm.k_fft * (M3 / 2.0) * std::log(M3 / 2.0);
  return true;
}

}  // namespace

extern "C" {

se_status se_est_real_error(int kind, double Q, double L, double xi, double rc, double *err) {
  if (!kind_ok(kind)) return bad("unknown estimate kind");
  if (!pos(Q) || !pos(L) || !pos(xi) || !pos(rc)) return bad("Q, L, xi and rc must be finite and > 0");
  if (!err) return bad("err is NULL");
  *err = real_err(kind, Q, L, xi, rc);
  return SE_OK;
}

se_status se_est_fourier_error(int kind, double Q, double L, double xi, double kinf,
                               double *err) {
  if (!kind_ok(kind)) return bad("unknown estimate kind");
  if (!pos(Q) || !pos(L) || !pos(xi) || !pos(kinf))
    return bad("Q, L, xi and kinf must be finite and > 0");
  if (!err) return bad("err is NULL");
  *err = fourier_err(kind, Q, L, xi, kinf);
  return SE_OK;
}

se_status se_est_xi(int kind, double eps, double Q, double L, double rc, double *xi) {
  if (!kind_ok(kind)) return bad("unknown estimate kind");
  if (!pos(eps) || !pos(Q) || !pos(L) || !pos(rc))
    return bad("eps, Q, L and rc must be finite and > 0");
  if (!xi) return bad("xi is NULL");
  double v;
  if (!xi_of(kind, eps, Q, L, rc, &v))
    return bad("eps is above the real-space force estimate at xi = 0: any xi meets it");
  *xi = v;
  return SE_OK;
}

se_status se_est_kinf(int kind, double eps, double Q, double L, double xi, double *kinf) {
  if (!kind_ok(kind)) return bad("unknown estimate kind");
  if (!pos(eps) || !pos(Q) || !pos(L) || !pos(xi))
    return bad("eps, Q, L and xi must be finite and > 0");
  if (!kinf) return bad("kinf is NULL");
  *kinf = kinf_of(kind, eps, Q, L, xi);
  return SE_OK;
}

se_status se_est_se_error(int kind, double Q, double L, double xi, int P, double c,
                          double *err) {
  if (!kind_ok(kind)) return bad("unknown estimate kind");
  if (!pos(Q) || !pos(L) || !pos(xi) || P < 1 || !std::isfinite(c))
    return bad("Q, L, xi must be finite and > 0, P >= 1, c finite");
  if (!err) return bad("err is NULL");
  *err = se_err(kind, Q, L, xi, P, c > 0.0 ? c : kDefaultC);
  return SE_OK;
}

se_status se_est_se_support(int kind, double eps, double Q, double L, double xi, double c,
                            int *P) {
  if (!kind_ok(kind)) return bad("unknown estimate kind");
  if (!pos(eps) || !pos(Q) || !pos(L) || !pos(xi) || !std::isfinite(c))
    return bad("eps, Q, L, xi must be finite and > 0, c finite");
  if (!P) return bad("P is NULL");
  const int v = support_of(kind, eps, Q, L, xi, c > 0.0 ? c : kDefaultC);
  if (v == 0) return bad("no even support up to 64 meets eps");
  *P = v;
  return SE_OK;
}

se_status se_cost_model_mi355x(int dtype, se_cost_model *m) {
  if (!m) return bad("model is NULL");
  // Non-negative least-squares fits of the model to se_kspace and se_rs_eval
  // times on an MI355X (calibrate.py of this package; 60 k-space and 15
  // real-space configurations per precision).
  // Largest relative deviation of the fit: 27% (FP32), 23% (FP64).
  if (dtype == SE_FP32) {
    *m = se_cost_model{2.6945e-05, 3.2147e-11, 1.2664e-12, 4.2873e-09, 7.6776e-13,
                       3.8105e-05, 9.0256e-11, 3.0490e-13, 2.4347e-12, 0.0, 1.4182e-12};
  } else if (dtype == SE_FP64) {
    *m = se_cost_model{3.3205e-05, 0.0, 7.5893e-12, 1.3672e-08, 2.1569e-12,
                       3.6594e-05, 1.3720e-10, 4.4701e-13, 6.3684e-12, 0.0, 1.9237e-12};
  } else {
    return bad("unknown dtype");
  }
  return SE_OK;
}

se_status se_cost_predict(const se_cost_model *model, int dtype, int N, double L, double rc,
                          int M, int P, double *t_real, double *t_kspace) {
  if (!model) return bad("model is NULL");
  if (dtype != SE_FP32 && dtype != SE_FP64) return bad("unknown dtype");
  if (N < 0 || !pos(L) || !pos(rc) || M < 1 || P < 1)
    return bad("need N >= 0, L and rc finite and > 0, M and P >= 1");
  double tr, tk;
  if (!predict(*model, dtype, N, L, rc, M, P, &tr, &tk))
    return sek::report(SE_ERR_UNSUPPORTED, "no tile edge fits this support and precision");
  if (t_real) *t_real = tr;
  if (t_kspace) *t_kspace = tk;
  return SE_OK;
}

se_status se_choose_params(int kind, double eps, int N, double Q, double L, double rc_min,
                           double rc_max, int n_rc, double c, int dtype,
                           const se_cost_model *model, se_choice *out) {
  if (!kind_ok(kind)) return bad("unknown estimate kind");
  if (!pos(eps) || !pos(Q) || !pos(L)) return bad("eps, Q and L must be finite and > 0");
  if (N < 1) return bad("N must be >= 1");
  if (!pos(rc_min) || !std::isfinite(rc_max) || rc_max < rc_min || n_rc < 1)
    return bad("need 0 < rc_min <= rc_max and n_rc >= 1");
  if (!std::isfinite(c)) return bad("c must be finite");
  if (dtype != SE_FP32 && dtype != SE_FP64) return bad("unknown dtype");
  if (!model || !out) return bad("model or out is NULL");
  if (c <= 0.0) c = kDefaultC;
  const se_cost_model &cm = *model;
  bool found = false;
  se_choice best{};
  const double step = n_rc > 1 ? (rc_max - rc_min) / (n_rc - 1) : 0.0;
  for (int i = 0; i < n_rc; ++i) {
    const double rc = i == n_rc - 1 && n_rc > 1 ? rc_max : rc_min + i * step;
    if (3.0 * rc > L) continue;
    double xi;
    if (!xi_of(kind, eps, Q, L, rc, &xi)) continue;
    const double kinf = kinf_of(kind, eps, Q, L, xi);
    int P = support_of(kind, eps, Q, L, xi, c);
    if (P == 0 || P > kPMax) continue;
    if (P < kPMin) P = kPMin;
    int M = 0;
    double eta = 0.0;
    for (int m = kMMin; m <= kMMax; m += 2) {
      if (!only_235(m) || m < 2.0 * kinf) continue;
      eta = P * L * L * xi * xi / (c * c * kPi * m * m);
      if (eta <= kEtaMax) {
        M = m;
        break;
      }
    }
    if (M == 0) continue;
    double t_real, t_k;
    if (!predict(cm, dtype, N, L, rc, M, P, &t_real, &t_k)) continue;
    if (!found || t_real + t_k < best.t_real + best.t_kspace) {
      found = true;
      best.rc = rc;
      best.xi = xi;
      best.kinf = kinf;
      best.M = M;
      best.P = P;
      best.eta = eta;
      best.t_real = t_real;
      best.t_kspace = t_k;
      best.est_real = real_err(kind, Q, L, xi, rc);
      best.est_fourier = fourier_err(kind, Q, L, xi, M / 2.0);
      best.est_approx = se_err(kind, Q, L, xi, P, c);
    }
  }
  if (!found)
    return sek::report(SE_ERR_UNSUPPORTED,
                       "no cutoff in the range meets the tolerance with M <= 512, P <= 16, rc <= L/3");
  *out = best;
  return SE_OK;
}

}  // extern "C"
