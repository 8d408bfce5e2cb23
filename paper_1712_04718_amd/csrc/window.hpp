// Per-axis window factors of the two methods, evaluated for one particle by
// the lanes of the spreading and gathering kernels that use them.  Grid
// units: a particle with anchor floor(x/h) = i0 and offset d = x/h - i0 in
// [0,1) touches the S grid points i0 + OFF + j, j = 0..S-1.
//
// SE (section 4): truncated Gaussian, OFF = -(P/2 - 1).  Per axis
//   g_j = beta exp(-cg t_j^2),  t_j = j + OFF - d   (= (x_j - x)/h),
// with cg = a h^2, a = 2 xi^2 / eta and beta = h sqrt(a/pi), so that the
// product over three axes is the h^3-weighted Gaussian of eq. (4.5).  The
// FP64 factors follow the fast Gaussian gridding recurrence of eqs.
// (4.10)-(4.11): g_{j+1} = g_j r_j with r_j = exp(-cg (2 t_j + 1)) and
// r_{j+1} = r_j exp(-2 cg), i.e. two exponentials per axis instead of P.
// FP32 factors are evaluated directly near the centre and by a short
// recurrence in the tail (see window_axis).  The derivative
// factor used for forces is the derivative with respect to the particle
// coordinate, d/dx_m W(x_j - x_m) = 2 a (x_j - x_m) W, i.e. per axis
// dg_j = 2 a h t_j g_j.
//
// SPME (section 6): cardinal B-spline of order p, OFF = -(p - 1),
//   g_j = M_p(d + p - 1 - j),  dg_j = (1/h) M_p'(d + p - 1 - j),
// with M_p built by the recursion of section 6.1 from M_2 and
// M_p' (u) = M_{p-1}(u) - M_{p-1}(u - 1).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace sek {

constexpr int kGauss = 0;
constexpr int kBspline = 1;

template <int WIN, int S> struct Stencil {
  static constexpr int OFF = (WIN == kGauss) ? -(S / 2 - 1) : -(S - 1);
};

constexpr int kMaxHalfSupport = 8;  // S / 2 for the largest Gaussian support

struct WindowConsts {
  double cg;     // Gaussian exponent in grid units (SE)
  double beta;   // per-axis Gaussian normalisation (SE)
  double kap;    // exp(-2 cg), ratio of successive recurrence factors (SE)
  double dcoef;  // SE: 2 a h; SPME: 1/h   (derivative scale)
  float rk[kMaxHalfSupport + 1];  // exp(-cg (2m + 1)), m = 0..S/2 (SE, FP32)
  double cgl2;   // cg log2(e): FP32 factors as beta 2^{-cgl2 t^2} (SE)
  // kt[i]: the largest value factor i of an axis takes over d in [0, 1),
  // without the Gaussian's beta (the spread's tile bound; window_bounds)
  double kt[2 * kMaxHalfSupport];
};

// e^{-cg t^2} in FP32 as 2^{-cgl2 t^2} with the hardware base-2 exponential
// (v_exp_f32: within 0.8 ulp, mean error -3e-9 relative, over [-12, 4)).
__device__ inline float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// One FP32 Gaussian factor beta e^{-cg t^2} at t = k - d (k an integer
// offset, d in [0,1)): t, t^2 and the exponent are formed in FP64 (t exact,
// two roundings of 1e-16), the exponent is rounded once to FP32, then the
// hardware exp2.  The error is about one ulp of the factor plus its
// exponent's rounding, 6e-8 |ln g|, smallest where the factors are largest.
__device__ inline float gauss_factor(float beta, double cgl2, int k, float d) {
  const double t = static_cast<double>(k) - static_cast<double>(d);
  return beta * exp2_fast(static_cast<float>(-cgl2 * t * t));
}

inline WindowConsts window_consts(double cg, double beta, double dcoef) {
  WindowConsts wc{cg, beta, std::exp(-2.0 * cg), dcoef, {}, cg * M_LOG2E, {}};
  for (int m = 0; m <= kMaxHalfSupport; ++m)
    wc.rk[m] = static_cast<float>(std::exp(-cg * (2.0 * m + 1.0)));
  return wc;
}

// Cardinal B-spline M_n(u) (section 6.1): M_2(u) = 1 - |u - 1| on [0, 2],
// M_n(u) = (u M_{n-1}(u) + (n - u) M_{n-1}(u - 1)) / (n - 1).
inline double bspline_value(int n, double u) {
  if (u <= 0.0 || u >= n) return 0.0;
  if (n == 2) return 1.0 - std::fabs(u - 1.0);
  return (u * bspline_value(n - 1, u) + (n - u) * bspline_value(n - 1, u - 1.0)) / (n - 1);
}

// wc.kt for a support of S points: Gaussian factor i is e^{-cg t^2} at
// t = i + OFF - d, largest where t is nearest 0 (distance of i + OFF from
// [0, 1]); B-spline factor i is M_S(d + S - 1 - i), and M_S, symmetric
// and unimodal about S/2, is largest at the point of [S - 1 - i, S - i]
// nearest S/2.
inline void window_bounds(WindowConsts &wc, int window, int S) {
  for (int i = 0; i < S && i < 2 * kMaxHalfSupport; ++i) {
    if (window == kGauss) {
      const int t = i - (S / 2 - 1);
      const double dist = t < 0 ? -t : (t > 1 ? t - 1 : 0);
      wc.kt[i] = std::exp(-wc.cg * dist * dist);
    } else {
      const double lo = S - 1 - i, hi = S - i, mid = 0.5 * S;
      wc.kt[i] = bspline_value(S, mid < lo ? lo : (mid > hi ? hi : mid));
    }
  }
}

// All S factors of one axis (and optionally their derivatives).
//
// FP32 evaluates the four central Gaussian factors directly and builds the
// tail outward from them (six exponentials per axis for any support, and
// rounding grows only towards the small tail factors): the recurrence of
// eqs. (4.10)-(4.11) started at the stencil end would pass the relative
// rounding of its first, smallest factor on to the large central ones.
// FP64 uses that recurrence, whose accumulated rounding stays near 1e-15.
template <typename R, int WIN, int S, bool DERIV>
__device__ inline void window_axis(R d, const WindowConsts &wc, R (&g)[S], R (&dg)[S]) {
  if constexpr (WIN == kGauss) {
    constexpr int OFF = Stencil<WIN, S>::OFF;
    const R cg = static_cast<R>(wc.cg);
    const R beta = static_cast<R>(wc.beta);
    if constexpr (sizeof(R) == 4) {
      // With k = j + OFF (k = 0 at the anchor) and t_k = k - d, the four
      // factors nearest the centre (k = -1..2), which carry most of the
      // weight, are evaluated directly by gauss_factor; the rest outward by
      //   g_{k+1} = g_k B e^{-cg (2k + 1)}   (k >= 2),
      //   g_{k-1} = g_k B^{-1} e^{-cg (1 - 2k)}   (k <= -1),   B = e^{2 cg d},
      // two roundings per step on factors below e^{-cg 4}.  Rounding in a
      // product of separately rounded exponentials (beta e^{-cg d^2} B^k
      // e^{-cg k^2}) costs about twice the error of the direct form at
      // k = 1, where that form's intermediate exponents are largest.
      constexpr int J0 = -OFF;  // index of the anchor point
#pragma unroll
      for (int k = -1; k <= 2; ++k)
        if (J0 + k >= 0 && J0 + k < S) g[J0 + k] = gauss_factor(beta, wc.cgl2, k, d);
      const float eb = static_cast<float>(2.0 * wc.cgl2 * static_cast<double>(d));
      if constexpr (J0 + 3 < S) {
        const R Bu = exp2_fast(eb);
#pragma unroll
        for (int k = 2; J0 + k + 1 < S; ++k) g[J0 + k + 1] = g[J0 + k] * Bu * wc.rk[k];
      }
      if constexpr (J0 - 2 >= 0) {
        const R Bd = exp2_fast(-eb);
#pragma unroll
        for (int m = 1; J0 - m - 1 >= 0; ++m) g[J0 - m - 1] = g[J0 - m] * Bd * wc.rk[m];
      }
      if constexpr (DERIV) {
#pragma unroll
        for (int j = 0; j < S; ++j) dg[j] = static_cast<R>(wc.dcoef) * (static_cast<R>(OFF + j) - d) * g[j];
      }
    } else {
      const R t0 = static_cast<R>(OFF) - d;
      R gj = beta * exp(-cg * t0 * t0);
      R rj = exp(-cg * (R(2) * t0 + R(1)));
      const R kap = static_cast<R>(wc.kap);
#pragma unroll
      for (int j = 0; j < S; ++j) {
        g[j] = gj;
        if constexpr (DERIV) dg[j] = static_cast<R>(wc.dcoef) * (t0 + R(j)) * gj;
        gj *= rj;
        rj *= kap;
      }
    }
  } else {
    // v[i] = M_n(d + i), i = 0..n-1, built up from n = 2.
    R v[S];
#pragma unroll
    for (int i = 0; i < S; ++i) v[i] = R(0);
    v[0] = d;
    v[1] = R(1) - d;
#pragma unroll
    for (int n = 2; n < S; ++n) {
      // order n -> n + 1:
      // M_{n+1}(d+i) = ((d+i) M_n(d+i) + (n+1-d-i) M_n(d+i-1)) / n
      if (n == S - 1 && DERIV) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
          const int i = S - 1 - j;  // dg_j = (1/h)(M_{S-1}(d+i) - M_{S-1}(d+i-1))
          const R hi = (i <= S - 2) ? v[i] : R(0);
          const R lo = (i >= 1) ? v[i - 1] : R(0);
          dg[j] = static_cast<R>(wc.dcoef) * (hi - lo);
        }
      }
      const R inv = R(1) / static_cast<R>(n);
#pragma unroll
      for (int i = n; i >= 0; --i) {
        const R cur = (i <= n - 1) ? v[i] : R(0);
        const R prev = (i >= 1) ? v[i - 1] : R(0);
        v[i] = ((d + R(i)) * cur + (R(n + 1) - d - R(i)) * prev) * inv;
      }
    }
#pragma unroll
    for (int j = 0; j < S; ++j) g[j] = v[S - 1 - j];
  }
}

}  // namespace sek
