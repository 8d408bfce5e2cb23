// Gaussian supports P = 18..24 in FP64: the high-accuracy end of the SE
// method (the approximation error e^{-pi P c^2/2} of section 5 falls below
// 1e-12 from P = 20 and to 1.7e-15 at P = 24).  A tile block of (T+P-1)^3
// doubles no longer fits the 160 KB of LDS of a CU at a tile edge that keeps
// the ghost blocks small, so this path has no tiles:
//   prep   : per particle the anchor floor(x/h) mod M and the offsets
//            d = x/h - anchor (as the binning writes them), in input order,
//            and per-block sums of q^2 for the self energy;
//   spread : the grid is cleared by a fill kernel, then one thread per
//            (particle, z row) adds its P^2 products into the grid with FP64
//            atomics (eq. 4.5);
//   gather : one wave per particle reads its P^3 stencil from the grid (L2)
//            and reduces phi and the three derivative sums across the wave
//            (eqs. 4.9 and 4.12).
// The FFT and scaling passes are the ones of the tiled path.
#include "se_common.hpp"
#include "window.hpp"

namespace sek {
namespace {

constexpr int kDirectWaves = 4;  // particles per gather work-group

template <typename R>
__global__ void __launch_bounds__(kThreads)
k_direct_prep(int N, const R *__restrict__ x, const R *__restrict__ q, double h, int M,
              SortedParticle<R> *__restrict__ out, int2 *__restrict__ meta,
              double *__restrict__ qsq_part) {
  const int n = blockIdx.x * kThreads + threadIdx.x;
  double qq = 0.0;
  if (n < N) {
    int a[3];
    R d[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      double frac;
      a[ax] = anchor_mod(static_cast<double>(x[3 * n + ax]) / h, M, &frac);
      d[ax] = static_cast<R>(frac);
    }
    const R qn = q[n];
    out[n] = SortedParticle<R>{d[0], d[1], d[2], qn};
    meta[n] = make_int2(a[0] | (a[1] << 10) | (a[2] << 20), n);
    qq = static_cast<double>(qn) * static_cast<double>(qn);
  }
  for (int o = 32; o > 0; o >>= 1) qq += __shfl_xor(qq, o);
  __shared__ double red[kThreads / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = qq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
    qsq_part[blockIdx.x] = s;
  }
}

template <typename R>
__global__ void __launch_bounds__(kThreads) k_direct_zero(R *__restrict__ grid, long long n) {
  const long long i = static_cast<long long>(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) grid[i] = R(0);
}

__device__ inline int wrap_mod(int v, int M) {
  v %= M;
  return v < 0 ? v + M : v;
}

template <int S>
__global__ void __launch_bounds__(kThreads)
k_direct_spread(int N, const SortedParticle<double> *__restrict__ pts,
                const int2 *__restrict__ meta, int M, WindowConsts wc,
                double *__restrict__ grid) {
  constexpr int OFF = Stencil<kGauss, S>::OFF;
  const long long t = static_cast<long long>(blockIdx.x) * kThreads + threadIdx.x;
  if (t >= static_cast<long long>(N) * S) return;
  const int n = static_cast<int>(t / S), jz = static_cast<int>(t % S);
  const SortedParticle<double> p = pts[n];
  const int packed = meta[n].x;
  const int ax = packed & 1023, ay = (packed >> 10) & 1023, az = (packed >> 20) & 1023;
  double gx[S], gy[S], unused[S];
  window_axis<double, kGauss, S, false>(p.dx, wc, gx, unused);
  window_axis<double, kGauss, S, false>(p.dy, wc, gy, unused);
  const double tz = static_cast<double>(jz + OFF) - p.dz;  // this thread's z factor, directly
  const double qz = p.q * wc.beta * exp(-wc.cg * tz * tz);
  const int z = wrap_mod(az + OFF + jz, M);
  int xs[S];
#pragma unroll
  for (int j = 0; j < S; ++j) xs[j] = wrap_mod(ax + OFF + j, M);
  for (int jy = 0; jy < S; ++jy) {
    const int y = wrap_mod(ay + OFF + jy, M);
    double *row = grid + (static_cast<long long>(z) * M + y) * M;
    const double qyz = qz * gy[jy];
#pragma unroll
    for (int jx = 0; jx < S; ++jx) atomicAdd(&row[xs[jx]], qyz * gx[jx]);
  }
}

template <int S>
__global__ void __launch_bounds__(64 * kDirectWaves)
k_direct_gather(int N, const SortedParticle<double> *__restrict__ pts,
                const int2 *__restrict__ meta, const double *__restrict__ grid, int M,
                WindowConsts wc, const double *__restrict__ gscale, int mode, double self_coef,
                double *__restrict__ out_pot, double *__restrict__ out_vec) {
  constexpr int OFF = Stencil<kGauss, S>::OFF;
  const int lane = threadIdx.x & 63;
  const int n = blockIdx.x * kDirectWaves + (threadIdx.x >> 6);
  if (n >= N) return;  // uniform across the wave
  const SortedParticle<double> p = pts[n];
  const int2 mt = meta[n];
  const int ax = mt.x & 1023, ay = (mt.x >> 10) & 1023, az = (mt.x >> 20) & 1023;
  double gx[S], dgx[S];
  window_axis<double, kGauss, S, true>(p.dx, wc, gx, dgx);
  int xs[S];
#pragma unroll
  for (int j = 0; j < S; ++j) xs[j] = wrap_mod(ax + OFF + j, M);
  double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;  // phi, and F / (-q) along x, y, z
  for (int r = lane; r < S * S; r += 64) {
    const int jy = r / S, jz = r - (r / S) * S;
    const int y = wrap_mod(ay + OFF + jy, M), z = wrap_mod(az + OFF + jz, M);
    const double *row = grid + (static_cast<long long>(z) * M + y) * M;
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int jx = 0; jx < S; ++jx) {
      const double v = row[xs[jx]];
      a += v * gx[jx];
      b += v * dgx[jx];
    }
    // this lane's y and z factors and derivatives, evaluated directly
    // (jy and jz differ across lanes)
    const double ty = static_cast<double>(jy + OFF) - p.dy, tz = static_cast<double>(jz + OFF) - p.dz;
    const double fy = wc.beta * exp(-wc.cg * ty * ty), fz = wc.beta * exp(-wc.cg * tz * tz);
    const double dfy = wc.dcoef * ty * fy, dfz = wc.dcoef * tz * fz;
    t0 += fy * fz * a;
    t1 += fy * fz * b;
    t2 += dfy * fz * a;
    t3 += fy * dfz * a;
  }
  for (int o = 32; o > 0; o >>= 1) {
    t0 += __shfl_xor(t0, o);
    t1 += __shfl_xor(t1, o);
    t2 += __shfl_xor(t2, o);
    t3 += __shfl_xor(t3, o);
  }
  if (lane == 0) {
    const double scale = gscale ? *gscale : 1.0;
    const int orig = mt.y;
    // potential-force mode: F = -q (t1, t2, t3); adjoint: -gE F = gE q (t1, t2, t3)
    const double fq = (mode == kGatherPotentialForce) ? -scale * p.q : scale * p.q;
    if (out_pot) out_pot[orig] = scale * (t0 + self_coef * p.q);
    if (out_vec) {
      out_vec[3 * orig + 0] = fq * t1;
      out_vec[3 * orig + 1] = fq * t2;
      out_vec[3 * orig + 2] = fq * t3;
    }
  }
}

template <int S>
hipError_t direct_spread_S(se_plan &p, int N) {
  const WindowConsts wc = window_consts(p.cg, p.beta, 0.0);
  const long long threads = static_cast<long long>(N) * S;
  launch_on(&p, k_direct_spread<S>, static_cast<unsigned>((threads + kThreads - 1) / kThreads), kThreads, 0,
                       p.stream, N, static_cast<const SortedParticle<double> *>(p.buf.sorted),
                                   p.buf.meta, p.prm.M, wc, static_cast<double *>(p.buf.grid));
  return hipGetLastError();
}

template <int S>
hipError_t direct_gather_S(se_plan &p, int N, const void *pts, const int2 *meta,
                           const double *gscale, int mode, double self, void *pot, void *vec) {
  const WindowConsts wc = window_consts(p.cg, p.beta, 2.0 * p.a * p.h);
  launch_on(&p, k_direct_gather<S>, (N + kDirectWaves - 1) / kDirectWaves, 64 * kDirectWaves, 0, p.stream, 
      N, static_cast<const SortedParticle<double> *>(pts), meta,
      static_cast<const double *>(p.buf.grid), p.prm.M, wc, gscale, mode, self,
      static_cast<double *>(pot), static_cast<double *>(vec));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_direct_prep(se_plan &p, int N, const void *x, const void *q, void *pts,
                              int2 *meta, double *qsq_part, int *parts) {
  const int blocks = (N + kThreads - 1) / kThreads;
  if (parts) *parts = blocks;
  if (N == 0) return hipSuccess;
  launch_on(&p, k_direct_prep<double>, blocks, kThreads, 0, p.stream, 
      N, static_cast<const double *>(x), static_cast<const double *>(q), p.h, p.prm.M,
      static_cast<SortedParticle<double> *>(pts), meta, qsq_part);
  return hipGetLastError();
}

hipError_t launch_direct_forward(se_plan &p, int N, const void *x, const void *q) {
  hipError_t e = launch_direct_prep(p, N, x, q, p.buf.sorted, p.buf.meta, p.buf.part,
                                    &p.bin_parts);
  if (e != hipSuccess) return e;
  stage_begin(p, SE_STAGE_SPREAD);
  const long long ngrid = static_cast<long long>(p.prm.M) * p.prm.M * p.prm.M;
  launch_on(&p, k_direct_zero<double>, static_cast<unsigned>((ngrid + kThreads - 1) / kThreads), kThreads, 0,
                          p.stream, static_cast<double *>(p.buf.grid), ngrid);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (N > 0) {
    switch (p.prm.P) {
      case 18: e = direct_spread_S<18>(p, N); break;
      case 20: e = direct_spread_S<20>(p, N); break;
      case 22: e = direct_spread_S<22>(p, N); break;
      case 24: e = direct_spread_S<24>(p, N); break;
      default: e = hipErrorInvalidValue; break;
    }
  }
  stage_end(p, SE_STAGE_SPREAD);
  return e;
}

hipError_t launch_direct_gather(se_plan &p, int N, const double *gscale, int mode, void *pot,
                                void *vec) {
  if (N == 0 || (!pot && !vec)) return hipSuccess;
  const bool tgt = mode == kGatherTargets;
  const double self =
      (!tgt && (p.prm.flags & SE_FLAG_ADD_SELF)) ? -2.0 * p.prm.xi / sqrt(M_PI) : 0.0;
  const void *pts = tgt ? p.tgt.sorted : p.buf.sorted;
  const int2 *meta = tgt ? p.tgt.meta : p.buf.meta;
  const int kmode = tgt ? kGatherPotentialForce : mode;
  if (!tgt) stage_begin(p, SE_STAGE_GATHER);
  hipError_t e;
  switch (p.prm.P) {
    case 18: e = direct_gather_S<18>(p, N, pts, meta, gscale, kmode, self, pot, vec); break;
    case 20: e = direct_gather_S<20>(p, N, pts, meta, gscale, kmode, self, pot, vec); break;
    case 22: e = direct_gather_S<22>(p, N, pts, meta, gscale, kmode, self, pot, vec); break;
    case 24: e = direct_gather_S<24>(p, N, pts, meta, gscale, kmode, self, pot, vec); break;
    default: e = hipErrorInvalidValue; break;
  }
  if (!tgt) stage_end(p, SE_STAGE_GATHER);
  return e;
}

}  // namespace sek
