// Step 2 of Algorithm 1: spread the charges onto the grid (SE eq. 4.5 or
// SPME eq. 6.1), with neither global atomics nor floating-point atomics.
//
// One work-group per tile of T^3 anchor points.  The particles anchored in
// the tile touch a (T+S-1)^3 block of the grid, accumulated in LDS and then
// stored, with plain coalesced 16-byte stores, as the tile's own block of a
// "ghost" array (blocks ghost_stride values apart); a fold kernel then adds
// the overlapping blocks that cover each grid point, so no grid zeroing and
// no global atomics are needed.
//
// LDS accumulation in fixed point, with a per-tile scale 2^B / bound, where
// bound is at least every partial sum the tile's block can hold: B = 30 in
// 32-bit integers (FP32) and B = 50 in 64-bit integers (FP64, where every
// contribution then lies below 2^51 and rounds to an integer with one FP64
// add, round_to_int64).  The bound is the tile's charge histogram over
// (y, z) anchors convolved with the window's largest values (tile_bound_yz),
// about ten times tighter than wmax * sum_tile |q| on a water-like system,
// so the fixed-point quantum stays below the rest of each precision's
// rounding.  No partial sum can leave (-2^(B+1), 2^(B+1)), each contribution
// is rounded once, and the result does not depend on the order of the
// additions, so both precisions are bitwise reproducible.  (Integer LDS
// atomics run far faster than floating-point ones on this chip.)  An FP32
// contribution has 24 significant bits while the fixed point spans 30, so
// exact halves are common: they round to even, which keeps the sum unbiased
// (rounding halves up would not).
// Work split (k_spread_lane, both windows): each wave holds 64/S particle
// groups of S lanes; lane (group, jx) owns the x-offset jx of one particle,
// evaluates the factors it needs itself (Gaussian: its x factor and all S
// factors along y and z, each to about one FP32 rounding; B-spline: the
// order-S recursion of section 6.1 along the three axes) and adds its S^2
// (jy, jz) products.  The factor arithmetic runs in the shadow of the LDS
// atomics, whose issue rate bounds the kernel, and no factor table or
// barrier sits between the particles and their atomics.
#include "se_common.hpp"
#include "window.hpp"

namespace sek {
namespace {

extern __shared__ __align__(16) unsigned char g_smem[];

// v rounded to the nearest integer, ties to even, as a 64-bit two's
// complement value, for |v| < 2^51: adding 1.5 2^52 leaves v's rounded
// integer in the low bits of a double in [2^52, 2^53), whose bit pattern
// grows by one per unit there.
__device__ inline unsigned long long round_to_int64(double v) {
  constexpr double kMagic = 6755399441055744.0;  // 1.5 2^52
  return static_cast<unsigned long long>(__double_as_longlong(v + kMagic)) -
         static_cast<unsigned long long>(__double_as_longlong(kMagic));
}

template <typename R> struct Acc;
template <> struct Acc<float> { using T = int; };      // fixed point
template <> struct Acc<double> { using T = long long; };  // fixed point

// Bound on every partial sum the tile's block can hold, for the
// fixed-point scale, independent of the order of the tile's particles (that
// order comes from atomics).  A particle with anchor (ax, ay, az) in the tile
// adds to block point (jx, jy, jz) the value q g_x g_y g_z with
//   0 <= g_d <= wmax^(1/3) k(j_d - a_d),  k(i) = the largest value factor i
//   takes over d in [0, 1) (wc.kt: e^{-cg dist(i + OFF, [0,1])^2} for the
//   Gaussian, whose factors carry beta = wmax^(1/3); M_S at the point of its
//   interval nearest S/2 for the B-spline, wmax = 1),
// and g_x <= wmax^(1/3), so every partial sum at (jx, jy, jz) is at most
//   wmax sum_n |q_n| k(jy - ay_n) k(jz - az_n),
// the tile's (y, z) anchor histogram of |q| convolved with k along y and z.
// To be order-free the histogram holds integers: u = ceil(|q| / qmax 2^20)
// >= |q| / qmax 2^20 per particle (qmax = max |q| is exact), added with
// 64-bit integer atomics; the convolutions run in a fixed order (along y in
// FP64 into an FP32 buffer, then along z in FP64), and the result is raised
// by 1e-5 for the roundings of the buffer, of the k table and of the FP32
// factors.  On the 100k-atom water workload this bound is 11x tighter than
// wmax sum |q| (the partial sums there stay far below the charge a tile
// holds), which takes the FP32 fixed-point rounding of the forces from
// 1.4e-6 to 1.3e-7 (and keeps the 50-bit FP64 quantum near 1e-13).  LDS: U
// (T^2 integers), C (TS x T floats), red (2 NWAVES doubles).  A non-finite
// charge weighs 0 (the integer conversion stays defined).  Returns the bound
// divided by wmax (0 for a tile without charge).
template <typename R, int S, int T, int NWAVES>
__device__ inline double tile_bound_yz(const SortedParticle<R> *__restrict__ sorted,
                                       const int2 *__restrict__ meta, int start, int end,
                                       const WindowConsts &wc, unsigned long long *U, float *C,
                                       double *red) {
  constexpr int TS = T + S - 1;
  const double *kt = wc.kt;  // k(i), from the host (window_bounds)
  const int tid = threadIdx.x;
  // the first KB particles of each thread stay in registers for the
  // histogram pass (one read of them instead of two)
  constexpr int KB = 4;
  R qv[KB];
  int pv[KB];
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int p = start + tid + k * kTileThreads;
    qv[k] = R(0);
    pv[k] = 0;
    if (p < end) {
      qv[k] = sorted[p].q;
      pv[k] = meta[p].x;
    }
  }
  for (int i = tid; i < T * T; i += kTileThreads) U[i] = 0ull;
  double m = 0.0;
#pragma unroll
  for (int k = 0; k < KB; ++k) m = fmax(m, fabs(static_cast<double>(qv[k])));
  for (int p = start + tid + KB * kTileThreads; p < end; p += kTileThreads)
    m = fmax(m, fabs(static_cast<double>(sorted[p].q)));
  m = wave_reduce0(m, [](double a, double b) { return fmax(a, b); });
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  double qmax = 0.0;
  for (int w = 0; w < NWAVES; ++w) qmax = fmax(qmax, red[w]);
  if (!(qmax > 0.0)) return 0.0;  // uniform across the work-group
  // |q| 2^20 / qmax through a reciprocal: u falls short of it by at most
  // two FP64 roundings (4e-16 relative), far inside the margin below
  const double inv = 1048576.0 / qmax;
  const auto add = [&](R q, int packed) {
    const double aq = fabs(static_cast<double>(q));
    const double w = fmin(ceil(aq * inv), 1048576.0);
    const int ay = (packed >> 8) & 0xff, az = (packed >> 16) & 0xff;
    if (aq <= qmax) atomicAdd(&U[ay * T + az], static_cast<unsigned long long>(w));
  };
#pragma unroll
  for (int k = 0; k < KB; ++k)
    if (start + tid + k * kTileThreads < end) add(qv[k], pv[k]);
  for (int p = start + tid + KB * kTileThreads; p < end; p += kTileThreads)
    add(sorted[p].q, meta[p].x);
  __syncthreads();
  // C(jy, az) = sum_ay U(ay, az) k(jy - ay)
  for (int i = tid; i < TS * T; i += kTileThreads) {
    const int jy = i / T, az = i - jy * T;
    double c = 0.0;
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int ay = jy - t;
      if (ay >= 0 && ay < T) c += static_cast<double>(U[ay * T + az]) * kt[t];
    }
    C[i] = static_cast<float>(c);
  }
  __syncthreads();
  // max over (jy, jz) of sum_az C(jy, az) k(jz - az)
  double bmax = 0.0;
  for (int i = tid; i < TS * TS; i += kTileThreads) {
    const int jy = i / TS, jz = i - jy * TS;
    double b = 0.0;
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int az = jz - t;
      if (az >= 0 && az < T) b += static_cast<double>(C[jy * T + az]) * kt[t];
    }
    bmax = fmax(bmax, b);
  }
  bmax = wave_reduce0(bmax, [](double a, double b) { return fmax(a, b); });
  if ((tid & 63) == 0) red[NWAVES + (tid >> 6)] = bmax;
  __syncthreads();
  double bm = 0.0;
  for (int w = 0; w < NWAVES; ++w) bm = fmax(bm, red[NWAVES + w]);
  return qmax * (bm / 1048576.0) * (1.0 + 1e-5);
}

// LDS of k_spread_lane: the fixed-point block (ghost_stride values), then
// the bound's histogram U (T^2 64-bit integers) and C (TS x T floats,
// rounded up to 8 bytes), then 128 bytes of reduction slots.
constexpr size_t spread_lane_bound_lds(int S, int T) {
  return 8 * static_cast<size_t>(T * T) + ((4 * static_cast<size_t>((T + S - 1) * T) + 7) & ~size_t(7));
}
constexpr size_t spread_lane_lds(int real_size, int S, int T) {
  const size_t acc = real_size == 4 ? 4 : 8;
  return acc * static_cast<size_t>(ghost_stride(T + S - 1)) + spread_lane_bound_lds(S, T) + 128;
}

// The factors are evaluated by the lanes that use them (see the file
// comment).  Gaussian, per lane: its x factor g_jx = beta e^{-cg t^2}
// (t = jx + OFF - dx) directly (gauss_factor in FP32), and the S factors
// along y and z with window_axis (the central ones directly as well).
// B-spline: every lane runs the order-S recursion of window_axis for the
// three axes of its particle and keeps entry jx along x.
template <typename R, int WIN, int S, int T>
__global__ void __launch_bounds__(kTileThreads)
k_spread_lane(const SortedParticle<R> *__restrict__ sorted, const int2 *__restrict__ meta,
              const int *__restrict__ offsets, int *__restrict__ counts, WindowConsts wc,
              double wmax, R *__restrict__ ghost) {
  using A = typename Acc<R>::T;
  constexpr int TS = T + S - 1, TSB = ghost_stride(TS);
  constexpr int GROUPS = 64 / S;
  constexpr int NWAVES = kTileThreads / 64;
  constexpr int OFF = Stencil<WIN, S>::OFF;
  // the block is cleared and stored 16 bytes per lane
  constexpr int NV = 16 / sizeof(R);
  using VA = A __attribute__((ext_vector_type(NV)));
  using VR = R __attribute__((ext_vector_type(NV)));
  static_assert(TSB % NV == 0, "whole 16-byte vectors per block");
  constexpr double kFix = sizeof(R) == 4 ? 1073741824.0 : 1125899906842624.0;  // 2^30, 2^50
  static_assert(2 * NWAVES * 8 <= 128, "reduction slots");
  static_assert(T <= 256, "local anchors are packed in 8 bits");

  const int tile = xcd_local(blockIdx.x, gridDim.x);
  const int start = offsets[tile], end = offsets[tile + 1];
  const int tid = threadIdx.x;
  // the binning left this tile's count for its consumer to reset
  if (tid == 0) counts[tile * kCountStride] = 0;
  R *out = ghost + static_cast<long long>(tile) * TSB;
  if (start == end) {  // uniform across the work-group
    for (int i = tid; i < TSB / NV; i += kTileThreads) reinterpret_cast<VR *>(out)[i] = VR(0);
    return;
  }
  A *blk = reinterpret_cast<A *>(g_smem);
  unsigned char *bnd = g_smem + sizeof(A) * TSB;
  unsigned long long *U = reinterpret_cast<unsigned long long *>(bnd);
  float *C = reinterpret_cast<float *>(bnd + 8 * T * T);
  double *red = reinterpret_cast<double *>(bnd + spread_lane_bound_lds(S, T));

  const int wave = tid >> 6, lane = tid & 63;
  const int grp = lane / S, jx = lane - grp * S;
  const bool active = grp < GROUPS;
  constexpr int STRIDE = NWAVES * GROUPS;
  int c = start + wave * GROUPS + grp;
  // this group's first particle is requested before the block is cleared
  // and the bound reduced
  SortedParticle<R> sp{};
  int packed = 0;
  if (active && c < end) {
    sp = sorted[c];
    packed = meta[c].x;
  }
  for (int i = tid; i < TSB / NV; i += kTileThreads) reinterpret_cast<VA *>(blk)[i] = VA(0);
  const double bound =
      wmax * tile_bound_yz<R, S, T, NWAVES>(sorted, meta, start, end, wc, U, C, red);
  const double scale = bound > 0.0 ? kFix / bound : 1.0;
  const double inv_scale = bound > 0.0 ? bound / kFix : 1.0;  // the barriers of the bound also
                                                              // order the clearing of blk

  const R cg = static_cast<R>(wc.cg), beta = static_cast<R>(wc.beta);
  for (; active && c < end; c += STRIDE) {
    const int cn = c + STRIDE;
    SortedParticle<R> nsp{};
    int npacked = 0;
    if (cn < end) {  // the next particle is requested before this one's atomics
      nsp = sorted[cn];
      npacked = meta[cn].x;
    }
    R gy[S], gz[S], unused[S];
    window_axis<R, WIN, S, false>(sp.dy, wc, gy, unused);
    window_axis<R, WIN, S, false>(sp.dz, wc, gz, unused);
    R gx;
    if constexpr (WIN == kBspline) {
      R gxs[S];
      window_axis<R, WIN, S, false>(sp.dx, wc, gxs, unused);
      gx = gxs[0];
#pragma unroll
      for (int j = 1; j < S; ++j) gx = j == jx ? gxs[j] : gx;
    } else if constexpr (sizeof(R) == 4) {
      gx = gauss_factor(beta, wc.cgl2, jx + OFF, sp.dx);
    } else {
      const R t = static_cast<R>(jx + OFF) - sp.dx;
      gx = beta * exp(-cg * t * t);
    }
    const int ax = packed & 0xff, ay = (packed >> 8) & 0xff, az = (packed >> 16) & 0xff;
    A *row = blk + (az * TS + ay) * TS + ax + jx;
    // the charge in fixed-point units times this lane's x factor
    const R wq = static_cast<R>(static_cast<double>(sp.q) * scale) * gx;
#pragma unroll
    for (int jz = 0; jz < S; ++jz) {
      const R wz = wq * gz[jz];
#pragma unroll
      for (int jy = 0; jy < S; ++jy) {
        if constexpr (sizeof(R) == 4)
          atomicAdd(row + (jz * TS + jy) * TS, __float2int_rn(wz * gy[jy]));
        else  // two's complement: the unsigned add is the signed one
          atomicAdd(reinterpret_cast<unsigned long long *>(row + (jz * TS + jy) * TS),
                    round_to_int64(wz * gy[jy]));
      }
    }
    sp = nsp;
    packed = npacked;
  }
  __syncthreads();
  // (the block's last TSB - TS^3 values are zeros that no fold reads)
  for (int i = tid; i < TSB / NV; i += kTileThreads) {
    const VA a = reinterpret_cast<const VA *>(blk)[i];
    VR o;
#pragma unroll
    for (int k = 0; k < NV; ++k) o[k] = static_cast<R>(static_cast<double>(a[k]) * inv_scale);
    reinterpret_cast<VR *>(out)[i] = o;
  }
}

// ------------------------------------------------------------------ fold
// The spread grid is the sum of the tile blocks that cover each point.

// General case: per grid point, tables of the covering (tile, local index)
// pairs along each axis (packed as tile * 64 + local index).
template <typename R>
__global__ void __launch_bounds__(kThreads)
k_fold(const R *__restrict__ ghost, FoldTables ft, int M, R *__restrict__ grid) {
  const long long n = static_cast<long long>(M) * M * M;
  const long long i = static_cast<long long>(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= n) return;
  const int x = static_cast<int>(i % M);
  const long long zy = i / M;
  const int y = static_cast<int>(zy % M), z = static_cast<int>(zy / M);
  const int TS = ft.TS, TSB = ghost_stride(TS), KC = ft.KC;
  R s = R(0);
  const int nz = ft.count[z], ny = ft.count[y], nx = ft.count[x];
  for (int iz = 0; iz < nz; ++iz) {
    const int cz = ft.cover[z * KC + iz];
    for (int iy = 0; iy < ny; ++iy) {
      const int cy = ft.cover[y * KC + iy];
      const long long base =
          static_cast<long long>(((cz >> 6) * ft.ntx + (cy >> 6)) * ft.ntx) * TSB +
          ((cz & 63) * TS + (cy & 63)) * TS;
      for (int ix = 0; ix < nx; ++ix) {
        const int cx = ft.cover[x * KC + ix];
        s += ghost[base + static_cast<long long>(cx >> 6) * TSB + (cx & 63)];
      }
    }
  }
  grid[i] = s;
}

// Tiles partition the grid (M = ntx T) and no block wraps onto itself
// (T + S - 1 <= M): tile t owns the T^3 points starting at t T + OFF.
// Along each axis a point with local index l gets block t at l, block t-1 at
// l + T, block t-2 at l + 2T, while the local index stays inside the block.
// One work-group per tile, one thread per owned (x, y) column walking its
// T points along z, ZU planes at a time: only the candidates inside a block
// are loaded, all of a group of planes' loads are issued before the first
// is used, and each work-group reads its blocks plane after plane.  (A
// work-group per plane of a tile took 28 instead of 18 us at 10^6 ions.)
template <typename R, int WIN, int S, int T>
__global__ void __launch_bounds__(kThreads)
k_fold_tiles(const R *__restrict__ ghost, int M, int ntx, R *__restrict__ grid) {
  constexpr int TS = T + S - 1, TSB = ghost_stride(TS);
  constexpr int MAXK = (TS + T - 1) / T;
  constexpr int OFF = Stencil<WIN, S>::OFF;
  // z planes whose loads are issued together (at M = 432, 16-point tiles:
  // 244 us with two, 253 with four; at 12-point tiles four beat two)
  constexpr int ZU = T >= 16 ? 2 : 4;
  static_assert(T * T <= kThreads, "one thread per (x, y) column of a tile");
  const int i = static_cast<int>(threadIdx.x);
  if (i >= T * T) return;
  const int tile = xcd_local(blockIdx.x, gridDim.x);
  const int tz = tile / (ntx * ntx), ty = (tile / ntx) % ntx, tx = tile % ntx;
  const int ly = i / T, lx = i % T;
  int gy = ty * T + OFF + ly, gx = tx * T + OFF + lx;
  gy += gy < 0 ? M : 0;
  gx += gx < 0 ? M : 0;
  for (int lz0 = 0; lz0 < T; lz0 += ZU) {
    R v[ZU][MAXK][MAXK][MAXK];
#pragma unroll
    for (int u = 0; u < ZU; ++u) {
      const int lz = lz0 + u;
#pragma unroll
      for (int kz = 0; kz < MAXK; ++kz)
#pragma unroll
        for (int ky = 0; ky < MAXK; ++ky)
#pragma unroll
          for (int kx = 0; kx < MAXK; ++kx) {
            v[u][kz][ky][kx] = R(0);
            const int cz = lz + kz * T, cy = ly + ky * T, cx = lx + kx * T;
            if (lz < T && cz < TS && cy < TS && cx < TS) {
              const int sz = tz - kz + (tz < kz ? ntx : 0), sy = ty - ky + (ty < ky ? ntx : 0);
              const int sx = tx - kx + (tx < kx ? ntx : 0);
              v[u][kz][ky][kx] = ghost[static_cast<long long>((sz * ntx + sy) * ntx + sx) * TSB +
                                       (cz * TS + cy) * TS + cx];
            }
          }
    }
#pragma unroll
    for (int u = 0; u < ZU; ++u) {
      const int lz = lz0 + u;
      if (lz >= T) break;
      R s = R(0);
#pragma unroll
      for (int kz = 0; kz < MAXK; ++kz)
#pragma unroll
        for (int ky = 0; ky < MAXK; ++ky)
#pragma unroll
          for (int kx = 0; kx < MAXK; ++kx) s += v[u][kz][ky][kx];
      int gz = tz * T + OFF + lz;
      gz += gz < 0 ? M : 0;
      grid[(static_cast<long long>(gz) * M + gy) * M + gx] = s;
    }
  }
}

template <typename R, int WIN, int S, int T>
hipError_t spread_one(se_plan &p) {
  const size_t lds = spread_lane_lds(sizeof(R), S, T);
  WindowConsts wc = window_consts(p.cg, p.beta, 0.0);
  window_bounds(wc, WIN, S);
  const double wmax = (WIN == kGauss) ? p.beta * p.beta * p.beta : 1.0;
  const void *kern = reinterpret_cast<const void *>(&k_spread_lane<R, WIN, S, T>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  stage_begin(p, SE_STAGE_SPREAD);
  launch_on(&p, k_spread_lane<R, WIN, S, T>, p.ntiles, kTileThreads, lds, p.stream,
            static_cast<const SortedParticle<R> *>(p.buf.sorted), p.buf.meta, p.buf.offsets,
            p.buf.counts, wc, wmax, static_cast<R *>(p.buf.ghost));
  stage_end(p, SE_STAGE_SPREAD);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int M = p.prm.M;
  stage_begin(p, SE_STAGE_FOLD);
  if (p.fold_by_tiles) {
    launch_on(&p, k_fold_tiles<R, WIN, S, T>, p.ntiles, (T * T + 63) / 64 * 64, 0, p.stream, 
        static_cast<const R *>(p.buf.ghost), M, p.ntx, static_cast<R *>(p.buf.grid));
  } else {
    const long long ngrid = static_cast<long long>(M) * M * M;
    launch_on(&p, k_fold<R>, static_cast<unsigned>((ngrid + kThreads - 1) / kThreads), kThreads, 0,
                p.stream, static_cast<const R *>(p.buf.ghost), p.fold, M,
                            static_cast<R *>(p.buf.grid));
  }
  stage_end(p, SE_STAGE_FOLD);
  return hipGetLastError();
}

template <typename R, int WIN, int T>
hipError_t spread_dispatch_S(se_plan &p) {
  switch (p.prm.P) {
    case 3: if constexpr (WIN == kBspline) return spread_one<R, WIN, 3, T>(p); break;
    case 4: return spread_one<R, WIN, 4, T>(p);
    case 5: if constexpr (WIN == kBspline) return spread_one<R, WIN, 5, T>(p); break;
    case 6: return spread_one<R, WIN, 6, T>(p);
    case 7: if constexpr (WIN == kBspline) return spread_one<R, WIN, 7, T>(p); break;
    case 8: return spread_one<R, WIN, 8, T>(p);
    case 10: if constexpr (WIN == kGauss) return spread_one<R, WIN, 10, T>(p); break;
    case 12: if constexpr (WIN == kGauss) return spread_one<R, WIN, 12, T>(p); break;
    case 14: if constexpr (WIN == kGauss) return spread_one<R, WIN, 14, T>(p); break;
    case 16: if constexpr (WIN == kGauss) return spread_one<R, WIN, 16, T>(p); break;
    default: break;
  }
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t spread_dispatch(se_plan &p) {
  const bool gauss = p.prm.window == SE_WINDOW_GAUSSIAN;
  if (p.T == 16)
    return gauss ? spread_dispatch_S<R, kGauss, 16>(p) : spread_dispatch_S<R, kBspline, 16>(p);
  if (p.T == 12)
    return gauss ? spread_dispatch_S<R, kGauss, 12>(p) : spread_dispatch_S<R, kBspline, 12>(p);
  return gauss ? spread_dispatch_S<R, kGauss, 8>(p) : spread_dispatch_S<R, kBspline, 8>(p);
}

}  // namespace

size_t spread_lds_bytes(int real_size, int window, int S, int T) {
  (void)window;
  return spread_lane_lds(real_size, S, T);
}

hipError_t launch_spread(se_plan &plan) {
  return plan.prm.dtype == SE_FP64 ? spread_dispatch<double>(plan)
                                   : spread_dispatch<float>(plan);
}

}  // namespace sek
