// Step 6 of Algorithm 1: gather the potential (SE eq. 4.9, SPME eq. 6.3)
// and the force by analytic differentiation of the window (section 3.1;
// eq. 4.12 read as F = -dE/dx):
//   phi_m = sum_j Phi_j W_j(x_m),
//   F_m   = -q_m sum_j Phi_j dW_j(x_m)/dx_m .
// The same kernel serves the adjoint used for reverse-mode differentiation:
// grad_q = gE phi and grad_x = -gE F, with gE read from device memory.
//
// One work-group per tile: the (T+S-1)^3 block of the scaled grid Phi that
// the tile's particles touch is staged in LDS.  Lane (group, jx) of a wave's
// 64/S particle groups owns the x-offset jx of one particle and sums over
// the S^2 (jy, jz) offsets, its sums over jy compensated (Kahan); the S
// lanes of a particle are then combined with DPP lane moves, without the
// LDS (for S = 4, 8, 16 a tree of row moves; otherwise the group's first
// lane adds the S values in lane order, compensated).
// After the block barrier the waves take the tile's particles in a strided
// loop with no further block barrier (k_gather_lane):
//   Gaussian window: each lane evaluates three factors (x, y, z at its own
//     offset) and shares the y and z ones with its group through a per-wave
//     LDS slot; the derivative sums are rearranged around the stencil centre;
//   B-spline window: lanes 0, 1 and 2 of a group run the order-p recursion
//     (section 6.1) for x, y and z with its derivatives and share all of
//     them through the slot.
#include "se_common.hpp"
#include "window.hpp"

namespace sek {
namespace {

extern __shared__ __align__(16) unsigned char h_smem[];

template <typename R> struct Kahan {
  R s = R(0), c = R(0);
  __device__ inline void add(R v) {
    const R y = v - c;
    const R t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ inline R value() const { return s - c; }
};

// Work-group size of k_gather_lane: 12 waves in FP32, so that the two
// work-groups a CU holds at the 12-point tiles of a 96^3 grid give each SIMD
// six waves (what the kernel's registers allow) to hide the latency of its
// LDS reads; 8 waves in FP64, whose registers allow five.
constexpr int gather_threads(int real_size) { return real_size == 4 ? 768 : 512; }

// LDS of k_gather_lane: the block of Phi, then one region that holds the
// staging tables (row and column offsets) until the block barrier and the
// groups' factor slots after it (sharing it keeps two FP32 work-groups at
// 16-point tiles within a CU's LDS).
constexpr int gather_slot(int window, int S) { return window == kGauss ? 2 * S : 6 * S; }
constexpr size_t gather_lane_lds(int real_size, int window, int S, int T) {
  const size_t TS = T + S - 1;
  const size_t wf = static_cast<size_t>(real_size) * (gather_threads(real_size) / 64) * (64 / S) *
                    gather_slot(window, S);
  const size_t tables = 4 * (TS * TS + TS);
  return real_size * ((TS * TS * TS + 3) & ~static_cast<size_t>(3)) +
         (wf > tables ? wf : tables);
}

// Sum of the S lanes of a group (S = 2..16, a power of two; groups start at
// multiples of S) in the group's first lane: partial sums at lane distances
// S/2, ..., 2, 1, each lane adding the value of the lane that distance above
// it (row shifts by 8 and 4, then quad permutations that swap pairs and
// neighbours).
template <int S, typename R> __device__ inline R group_sum_first(R v) {
  static_assert(S >= 2 && S <= 16 && (S & (S - 1)) == 0, "a power-of-two group within a row");
  if constexpr (S >= 16) v += dpp_move<0x108>(v);  // row_shl:8, lane i + 8
  if constexpr (S >= 8) v += dpp_move<0x104>(v);   // row_shl:4, lane i + 4
  if constexpr (S >= 4) v += dpp_move<0x4e>(v);    // quad_perm [2,3,0,1], lane i ^ 2
  v += dpp_move<0xb1>(v);                          // quad_perm [1,0,3,2], lane i ^ 1
  return v;
}

// The block of Phi is staged first; then each wave takes particle groups in
// a strided loop without block barriers.  Gaussian: lane (group, jx)
// evaluates three factors of its particle directly, g = beta e^{-cg t^2} at
// t = jx + OFF - d along x, y and z, keeps its x factor and shares the y and
// z ones with the group through the wave's LDS slot, so each lane computes
// three exponentials per particle (instead of one thread computing all 3S in
// a phase of its own between barriers).  B-spline: three lanes of the group
// run the recursion, one axis each, and share factors and derivatives.
template <typename R, int WIN, int S, int T>
__global__ void __launch_bounds__(gather_threads(sizeof(R)))
k_gather_lane(const R *__restrict__ phi_grid, const SortedParticle<R> *__restrict__ sorted,
              const int2 *__restrict__ meta, const int *__restrict__ offsets, int M, int ntx,
              WindowConsts wc, const double *__restrict__ gscale, int mode, R self_coef,
              R *__restrict__ out_pot, R *__restrict__ out_vec) {
  constexpr int TS = T + S - 1, TS3 = TS * TS * TS;
  constexpr int GROUPS = 64 / S;
  constexpr int OFF = Stencil<WIN, S>::OFF;
  constexpr int SLOT = gather_slot(WIN, S);
  constexpr int GTH = gather_threads(sizeof(R));
  constexpr int NWAVES = GTH / 64;
  constexpr bool POW2 = (S & (S - 1)) == 0;
  constexpr size_t BLK = sizeof(R) * ((TS3 + 3) & ~3);

  const int tile = xcd_local(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  R *blk = reinterpret_cast<R *>(h_smem);
  // the staging tables and the factor slots share one region: the tables
  // are last read before the block barrier, the slots first written after it
  R *wfac = reinterpret_cast<R *>(h_smem + BLK);
  int *rowtab = reinterpret_cast<int *>(h_smem + BLK), *xtab = rowtab + TS * TS;

  // Stage the block (batched loads into registers, then LDS stores; grid
  // offsets from row and column tables).
  const int tz = tile / (ntx * ntx), ty = (tile / ntx) % ntx, tx = tile % ntx;
  const int bz = tz * T + OFF, by = ty * T + OFF, bx = tx * T + OFF;
  constexpr int NST = (TS3 + GTH - 1) / GTH;  // elements per thread
  constexpr int BATCH = sizeof(R) == 4 ? 16 : 8;
  const int start = offsets[tile], end = offsets[tile + 1];
  if (start == end) return;  // uniform across the work-group
  for (int r = tid; r < TS * TS; r += GTH) {
    const int lz = r / TS, ly = r - lz * TS;
    rowtab[r] = (wrap_near(bz + lz, M) * M + wrap_near(by + ly, M)) * M;
  }
  if (tid < TS) xtab[tid] = wrap_near(bx + tid, M);
  __syncthreads();
  const int grp = lane / S, jx = lane - grp * S;
  const bool active = grp < GROUPS;
  constexpr int STRIDE = NWAVES * GROUPS;
  int c = start + wave * GROUPS + grp;
  // this group's first particle is requested while the block is staged
  SortedParticle<R> sp{};
  int2 mt = make_int2(0, 0);
  if (active && c < end) {
    sp = sorted[c];
    mt = meta[c];
  }
#pragma unroll
  for (int k0 = 0; k0 < NST; k0 += BATCH) {
    R v[BATCH];
#pragma unroll
    for (int k = 0; k < BATCH; ++k) {
      const int i = tid + (k0 + k) * GTH;
      if (k0 + k < NST && i < TS3) {
        const int r = i / TS, lx = i - r * TS;
        // byte offset from the grid's base in 32 bits (grids stay below 4 GB)
        const unsigned off =
            static_cast<unsigned>(rowtab[r] + xtab[lx]) * static_cast<unsigned>(sizeof(R));
        v[k] = *reinterpret_cast<const R *>(reinterpret_cast<const char *>(phi_grid) + off);
      }
    }
#pragma unroll
    for (int k = 0; k < BATCH; ++k) {
      const int i = tid + (k0 + k) * GTH;
      if (k0 + k < NST && i < TS3) blk[i] = v[k];
    }
  }
  __syncthreads();

  const R scale = gscale ? static_cast<R>(*gscale) : R(1);
  const R cg = static_cast<R>(wc.cg), beta = static_cast<R>(wc.beta);
  const R dc = static_cast<R>(wc.dcoef);
  R *gslot = wfac + (wave * GROUPS + grp) * SLOT;  // this group's shared factors
  for (; active && c < end; c += STRIDE) {
    const int cn = c + STRIDE;
    SortedParticle<R> nsp{};
    int2 nmt = make_int2(0, 0);
    if (cn < end) {  // the next particle is requested before this one's sums
      nsp = sorted[cn];
      nmt = meta[cn];
    }
    const R kj = static_cast<R>(jx + OFF);
    const R tx0 = kj - sp.dx, ty0 = kj - sp.dy, tz0 = kj - sp.dz;
    R gx, dgx = R(0);
    if constexpr (WIN == kBspline) {
      // lanes 0, 1, 2 of the group run the recursion for x, y, z and share
      // the factors and derivatives: slot [g_x | dg_x | g_y | dg_y | g_z | dg_z]
      if (jx < 3) {
        R g[S], dg[S];
        window_axis<R, WIN, S, true>(jx == 0 ? sp.dx : (jx == 1 ? sp.dy : sp.dz), wc, g, dg);
#pragma unroll
        for (int j = 0; j < S; ++j) {
          gslot[2 * S * jx + j] = g[j];
          gslot[2 * S * jx + S + j] = dg[j];
        }
      }
    } else if constexpr (sizeof(R) == 4) {
      gx = gauss_factor(beta, wc.cgl2, jx + OFF, sp.dx);
      gslot[jx] = gauss_factor(beta, wc.cgl2, jx + OFF, sp.dy);
      gslot[S + jx] = gauss_factor(beta, wc.cgl2, jx + OFF, sp.dz);
    } else {
      gx = beta * exp(-cg * tx0 * tx0);
      gslot[jx] = beta * exp(-cg * ty0 * ty0);
      gslot[S + jx] = beta * exp(-cg * tz0 * tz0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // Gaussian: d/dx_m of a factor is dc (j + OFF - d) g_j.  With the
    // centred weights c_j = j + OFF - 1/2 and e = d - 1/2 (|e| <= 1/2):
    //   sum_j (j + OFF - d) g_j a_j = sum_j c_j g_j a_j - e sum_j g_j a_j,
    // so the derivative needs one extra weighted sum per axis.  B-spline:
    // cy, cz are the derivatives themselves.
    R gy[S], gz[S], cy[S], cz[S];
#pragma unroll
    for (int j = 0; j < S; ++j) {
      if constexpr (WIN == kBspline) {
        gy[j] = gslot[2 * S + j];
        cy[j] = gslot[3 * S + j];
        gz[j] = gslot[4 * S + j];
        cz[j] = gslot[5 * S + j];
      } else {
        gy[j] = gslot[j];
        gz[j] = gslot[S + j];
        cy[j] = (static_cast<R>(j + OFF) - R(0.5)) * gy[j];
        cz[j] = (static_cast<R>(j + OFF) - R(0.5)) * gz[j];
      }
    }
    if constexpr (WIN == kBspline) {
      gx = gslot[jx];
      dgx = gslot[S + jx];
    }
    const int packed = mt.x;
    const int ax = packed & 0xff, ay = (packed >> 8) & 0xff, az = (packed >> 16) & 0xff;
    const R *col = blk + (az * TS + ay) * TS + ax + jx;
    Kahan<R> k0, k1, k2;
#pragma unroll
    for (int jy = 0; jy < S; ++jy) {
      R a0 = R(0), b1 = R(0);
#pragma unroll
      for (int jz = 0; jz < S; ++jz) {
        const R v = col[(jz * TS + jy) * TS];
        a0 += v * gz[jz];
        b1 += v * cz[jz];
      }
      k0.add(gy[jy] * a0);  // sum g_y g_z Phi
      k1.add(cy[jy] * a0);  // sum c_y g_y g_z Phi
      k2.add(gy[jy] * b1);  // sum g_y c_z g_z Phi
    }
    const R s0 = k0.value(), s1 = k1.value(), s2 = k2.value();
    R t0, t1, t2, t3;
    if constexpr (WIN == kBspline) {
      t0 = gx * s0;
      t1 = dgx * s0;
      t2 = gx * s1;
      t3 = gx * s2;
    } else {
      const R ey = sp.dy - R(0.5), ez = sp.dz - R(0.5);
      dgx = dc * tx0 * gx;
      t0 = gx * s0;
      t1 = dgx * s0;
      t2 = dc * gx * (s1 - ey * s0);
      t3 = dc * gx * (s2 - ez * s0);
    }
    // the group's slot is rewritten only after every lane has read it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if constexpr (POW2) {
      t0 = group_sum_first<S>(t0);
      t1 = group_sum_first<S>(t1);
      t2 = group_sum_first<S>(t2);
      t3 = group_sum_first<S>(t3);
    } else {
      // the group's first lane adds the S lane values in lane order,
      // compensated, the values moving down one lane per step
      Kahan<R> k0, k1, k2, k3;
      k0.add(t0);
      k1.add(t1);
      k2.add(t2);
      k3.add(t3);
#pragma unroll
      for (int l = 1; l < S; ++l) {
        t0 = dpp_move<0x130>(t0);  // wave_shl:1, lane i + 1
        t1 = dpp_move<0x130>(t1);
        t2 = dpp_move<0x130>(t2);
        t3 = dpp_move<0x130>(t3);
        k0.add(t0);
        k1.add(t1);
        k2.add(t2);
        k3.add(t3);
      }
      t0 = k0.value();
      t1 = k1.value();
      t2 = k2.value();
      t3 = k3.value();
    }
    if (jx == 0) {
      const R q = sp.q;
      const int orig = mt.y;
      if (mode >= kGatherIkX) {
        out_vec[3 * orig + (mode - kGatherIkX)] = scale * q * t0;
      } else {
        const R pot = t0 + self_coef * q;
        const R fq = (mode == kGatherPotentialForce) ? -scale * q : scale * q;
        if (out_pot) out_pot[orig] = scale * pot;
        if (out_vec) {
          out_vec[3 * orig + 0] = fq * t1;
          out_vec[3 * orig + 1] = fq * t2;
          out_vec[3 * orig + 2] = fq * t3;
        }
      }
    }
    sp = nsp;
    mt = nmt;
  }
}

// One gather launch over the grid `grid`: the plan's particles, or with
// `tgt` its evaluation points (unit test charges, no self term).
template <typename R, int WIN, int S, int T>
hipError_t gather_one(se_plan &p, const void *grid, bool tgt, const double *gscale, int mode,
                      void *pot, void *vec) {
  const size_t lds = gather_lane_lds(sizeof(R), WIN, S, T);
  const double dcoef = (WIN == kGauss) ? 2.0 * p.a * p.h : 1.0 / p.h;
  const WindowConsts wc = window_consts(p.cg, p.beta, dcoef);
  const double self =
      (!tgt && (p.prm.flags & SE_FLAG_ADD_SELF)) ? -2.0 * p.prm.xi / sqrt(M_PI) : 0.0;
  const void *sorted = tgt ? p.tgt.sorted : p.buf.sorted;
  const int2 *meta = tgt ? p.tgt.meta : p.buf.meta;
  const int *offsets = tgt ? p.tgt.offsets : p.buf.offsets;
  const void *kern = reinterpret_cast<const void *>(&k_gather_lane<R, WIN, S, T>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  if (!tgt) stage_begin(p, SE_STAGE_GATHER);
  launch_on(&p, k_gather_lane<R, WIN, S, T>, p.ntiles, gather_threads(sizeof(R)), lds, p.stream,
            static_cast<const R *>(grid), static_cast<const SortedParticle<R> *>(sorted), meta,
            offsets, p.prm.M, p.ntx, wc, gscale, mode, static_cast<R>(self), static_cast<R *>(pot),
            static_cast<R *>(vec));
  if (!tgt) stage_end(p, SE_STAGE_GATHER);
  return hipGetLastError();
}

struct GatherCall {
  const void *grid;
  bool tgt;
  const double *gscale;
  int mode;
  void *pot, *vec;
};

template <typename R, int WIN, int T>
hipError_t gather_dispatch_S(se_plan &p, const GatherCall &g) {
  switch (p.prm.P) {
#define SE_GATHER_CASE(S) return gather_one<R, WIN, S, T>(p, g.grid, g.tgt, g.gscale, g.mode, g.pot, g.vec)
    case 3: if constexpr (WIN == kBspline) SE_GATHER_CASE(3); break;
    case 4: SE_GATHER_CASE(4);
    case 5: if constexpr (WIN == kBspline) SE_GATHER_CASE(5); break;
    case 6: SE_GATHER_CASE(6);
    case 7: if constexpr (WIN == kBspline) SE_GATHER_CASE(7); break;
    case 8: SE_GATHER_CASE(8);
    case 10: if constexpr (WIN == kGauss) SE_GATHER_CASE(10); break;
    case 12: if constexpr (WIN == kGauss) SE_GATHER_CASE(12); break;
    case 14: if constexpr (WIN == kGauss) SE_GATHER_CASE(14); break;
    case 16: if constexpr (WIN == kGauss) SE_GATHER_CASE(16); break;
#undef SE_GATHER_CASE
    default: break;
  }
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t gather_dispatch(se_plan &p, const GatherCall &g) {
  const bool gauss = p.prm.window == SE_WINDOW_GAUSSIAN;
  if (p.T == 16)
    return gauss ? gather_dispatch_S<R, kGauss, 16>(p, g) : gather_dispatch_S<R, kBspline, 16>(p, g);
  if (p.T == 12)
    return gauss ? gather_dispatch_S<R, kGauss, 12>(p, g) : gather_dispatch_S<R, kBspline, 12>(p, g);
  return gauss ? gather_dispatch_S<R, kGauss, 8>(p, g) : gather_dispatch_S<R, kBspline, 8>(p, g);
}

hipError_t gather_call(se_plan &p, const GatherCall &g) {
  return p.prm.dtype == SE_FP64 ? gather_dispatch<double>(p, g) : gather_dispatch<float>(p, g);
}

}  // namespace

size_t gather_lds_bytes(int real_size, int window, int S, int T) {
  return gather_lane_lds(real_size, window == SE_WINDOW_GAUSSIAN ? kGauss : kBspline, S, T);
}

hipError_t launch_gather(se_plan &plan, int N, const double *gscale, int mode, void *out_pot,
                         void *out_vec) {
  if (N == 0 || (!out_pot && !out_vec)) return hipSuccess;
  if (plan.direct) return launch_direct_gather(plan, N, gscale, mode, out_pot, out_vec);
  const bool tgt = mode == kGatherTargets;
  const int kmode = tgt ? kGatherPotentialForce : mode;
  // ik forces: the potential from Phi, each force component from its field
  // grid; the adjoint stays the analytic derivative of the window
  const bool ik = (plan.prm.flags & SE_FLAG_IK_FORCE) && mode != kGatherAdjoint && out_vec;
  if (!ik) return gather_call(plan, {plan.buf.grid, tgt, gscale, kmode, out_pot, out_vec});
  hipError_t e = hipSuccess;
  if (out_pot) e = gather_call(plan, {plan.buf.grid, tgt, gscale, kmode, out_pot, nullptr});
  const size_t rs = plan.prm.dtype == SE_FP64 ? 8 : 4;
  const size_t m3 = static_cast<size_t>(plan.prm.M) * plan.prm.M * plan.prm.M;
  for (int d = 0; d < 3 && e == hipSuccess; ++d)
    e = gather_call(plan, {static_cast<const char *>(plan.buf.field) + d * m3 * rs, tgt, gscale,
                           kGatherIkX + d, nullptr, out_vec});
  return e;
}

}  // namespace sek
