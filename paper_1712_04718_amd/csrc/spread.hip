// Step 2 of Algorithm 1: spread the charges onto the grid (SE eq. 4.5 or
// SPME eq. 6.1) without global atomics on the hot loop.
//
// One work-group per tile of T^3 anchor points.  The particles anchored in
// the tile touch a (T+S-1)^3 block of the grid, which is accumulated in LDS
// with LDS atomics and then added to the global grid once (coalesced rows).
// Each wave takes the tile's particles in chunks:
//   phase A: one lane per particle computes its 3S separable window factors
//            (charge folded into the x factors) into the wave's LDS area;
//   phase B: the wave holds 64/S particle groups of S lanes; lane
//            (group, jx) owns the x-offset jx of one particle and adds its
//            S^2 (jy, jz) products, so one LDS instruction touches S
//            consecutive addresses per particle.
#include "se_common.hpp"
#include "window.hpp"

namespace sek {
namespace {

extern __shared__ __align__(16) unsigned char g_smem[];

template <typename R, int S, int T> struct SpreadLds {
  static constexpr int TS = T + S - 1;
  static constexpr int CH = Chunk<S>::CH;
  static constexpr int REC = 3 * S;                         // factors per particle
  static constexpr size_t BLK = sizeof(R) * TS * TS * TS;
  static constexpr size_t FAC = sizeof(R) * CH * REC;       // per wave
  static constexpr size_t ANC = sizeof(int) * CH;           // per wave
  static constexpr size_t TOTAL = BLK + (kThreads / 64) * (FAC + ANC);
};

template <typename R, int WIN, int S, int T>
__global__ void __launch_bounds__(kThreads)
k_spread(const SortedParticle<R> *__restrict__ sorted, const int2 *__restrict__ meta,
         const int *__restrict__ offsets, int M, int ntx, WindowConsts wc,
         R *__restrict__ grid) {
  using L = SpreadLds<R, S, T>;
  constexpr int TS = L::TS, CH = L::CH, REC = L::REC;
  constexpr int GROUPS = Chunk<S>::GROUPS;
  constexpr int OFF = Stencil<WIN, S>::OFF;
  constexpr int NWAVES = kThreads / 64;

  const int tile = blockIdx.x;
  const int start = offsets[tile], end = offsets[tile + 1];
  if (start == end) return;  // uniform across the work-group

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  R *blk = reinterpret_cast<R *>(g_smem);
  R *fac = reinterpret_cast<R *>(g_smem + L::BLK + wave * (L::FAC + L::ANC));
  int *anc = reinterpret_cast<int *>(reinterpret_cast<unsigned char *>(fac) + L::FAC);

  for (int i = tid; i < TS * TS * TS; i += kThreads) blk[i] = R(0);
  __syncthreads();

  const int grp = lane / S, jx = lane - grp * S;
  for (int base = start + wave * CH; base < end; base += NWAVES * CH) {
    const int nval = min(CH, end - base);
    // phase A: factors of particle base + lane
    if (lane < nval) {
      const SortedParticle<R> sp = sorted[base + lane];
      R g[S], unused[S];
      R *f = fac + lane * REC;
      window_axis<R, WIN, S, false>(sp.dx, wc, g, unused);
#pragma unroll
      for (int j = 0; j < S; ++j) f[j] = sp.q * g[j];
      window_axis<R, WIN, S, false>(sp.dy, wc, g, unused);
#pragma unroll
      for (int j = 0; j < S; ++j) f[S + j] = g[j];
      window_axis<R, WIN, S, false>(sp.dz, wc, g, unused);
#pragma unroll
      for (int j = 0; j < S; ++j) f[2 * S + j] = g[j];
      anc[lane] = meta[base + lane].x;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // phase B: accumulate into the tile block
    if (grp < GROUPS) {
      for (int c = grp; c < nval; c += GROUPS) {
        const R *f = fac + c * REC;
        const int packed = anc[c];
        const int ax = packed & 0xff, ay = (packed >> 8) & 0xff, az = (packed >> 16) & 0xff;
        const R wq = f[jx];
        R gy[S], gz[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
          gy[j] = f[S + j];
          gz[j] = f[2 * S + j];
        }
        R *row = blk + (az * TS + ay) * TS + ax + jx;
#pragma unroll
        for (int jz = 0; jz < S; ++jz) {
          const R wz = wq * gz[jz];
#pragma unroll
          for (int jy = 0; jy < S; ++jy)
            unsafeAtomicAdd(row + (jz * TS + jy) * TS, wz * gy[jy]);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();

  // add the block to the global grid (periodic wrap of the halo)
  const int tz = tile / (ntx * ntx), ty = (tile / ntx) % ntx, tx = tile % ntx;
  const int bz = tz * T + OFF, by = ty * T + OFF, bx = tx * T + OFF;
  for (int i = tid; i < TS * TS * TS; i += kThreads) {
    const R v = blk[i];
    if (v == R(0)) continue;
    const int lz = i / (TS * TS), ly = (i / TS) % TS, lx = i % TS;
    int gz = (bz + lz) % M, gy = (by + ly) % M, gx = (bx + lx) % M;
    gz += gz < 0 ? M : 0;
    gy += gy < 0 ? M : 0;
    gx += gx < 0 ? M : 0;
    unsafeAtomicAdd(grid + (static_cast<long long>(gz) * M + gy) * M + gx, v);
  }
}

template <typename R, int WIN, int S, int T>
hipError_t spread_one(se_plan &p) {
  const size_t lds = SpreadLds<R, S, T>::TOTAL;
  WindowConsts wc{p.cg, p.beta, exp(-2.0 * p.cg), 0.0};
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_spread<R, WIN, S, T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  stage_begin(p, SE_STAGE_SPREAD);
  k_spread<R, WIN, S, T><<<p.ntiles, kThreads, lds, p.stream>>>(
      static_cast<const SortedParticle<R> *>(p.buf.sorted), p.buf.meta, p.buf.offsets,
      p.prm.M, p.ntx, wc, static_cast<R *>(p.buf.grid));
  stage_end(p, SE_STAGE_SPREAD);
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
  return gauss ? spread_dispatch_S<R, kGauss, 8>(p) : spread_dispatch_S<R, kBspline, 8>(p);
}

}  // namespace

size_t spread_lds_bytes(int real_size, int S, int T) {
  const size_t ts = T + S - 1;
  const size_t groups = 64 / S, ch = groups * ((32 + groups - 1) / groups);
  return real_size * ts * ts * ts + (kThreads / 64) * (real_size * ch * 3 * S + 4 * ch);
}

hipError_t launch_spread(se_plan &plan, int N) {
  if (N == 0) return hipSuccess;
  return plan.prm.dtype == SE_FP64 ? spread_dispatch<double>(plan)
                                   : spread_dispatch<float>(plan);
}

}  // namespace sek
