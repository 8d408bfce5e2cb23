// Real-space part of the Ewald sums (section 1, eqs. 1.5-1.7), truncated at
// a cutoff rc (section 2.1):
//   phi_m = sum_{n != m, |r| < rc} q_n erfc(xi r) / r,
//   F_m   = q_m sum_{n != m, |r| < rc} q_n (2 xi / sqrt(pi) e^{-xi^2 r^2}
//                                          + erfc(xi r) / r) r_vec / r^2,
//   E     = 1/2 sum_m q_m phi_m,
// with r_vec = x_m - x_n over the nearest periodic image (rc <= L/3, so at
// most one image of a pair lies within rc).  Together with the k-space part
// and the self terms this is the total Ewald sum.
//
// Cell list: nc = min(floor(L / rc), 64) >= 3 cells per side of edge
// cs = L / nc >= rc,
// so every pair within rc lies in one of the 27 cells around a particle's
// own.  Particles are put in cell order by the binning kernels (cell edge =
// one point of an nc^3 grid); their stored offsets from the cell corner
// give distances without the rounding of absolute coordinates.  One
// work-group per cell stages the 27 neighbour cells in LDS and evaluates
// every pair of a home particle with them (k_rs_pairs).
#include <cmath>
#include <cstdio>
#include <new>

#include "se_common.hpp"

struct se_rs_plan {
  double L, xi, rc;
  int dtype;
  int n_max;
  hipStream_t stream;
  int nc_max;    // cells per side the buffers hold
  // the current call's cell list
  int nc;        // cells per side
  int reach;     // neighbour cells searched on each side (1 or 2)
  int cus;       // compute units of the plan's device
  int ncells;
  double cs;     // cell edge
  int bin_blocks;
  int *counts = nullptr;
  int *offsets = nullptr;
  int2 *key = nullptr;
  int2 *meta = nullptr;
  void *sorted = nullptr;
  double *part = nullptr;  // q^2 partials of binning (unused), then energy partials
};

namespace sek {

int rs_reach(double L, double rc, long long N);
int rs_cells_per_side(double L, double rc, int reach);

namespace {

constexpr int kRsThreads = 256;
// Pair queue entries per thread (a template argument of the pair kernel):
// FP32 takes 16 with the 1024-particle stage, keeping the work-group's LDS at
// about 37 KB so that four share a CU (a 32-entry queue, 53 KB and three per
// CU, made water_L100 459 us instead of 352), and 12 with the 512-particle
// stage (10^6 ions: 2.44 instead of 2.61 ms).  FP64 keeps 32 (a shorter
// queue flushed more often and was slower there).
constexpr int kBatch = 8;    // LDS reads issued together in the test and evaluation loops

template <typename R> struct alignas(4 * sizeof(R)) Staged {
  R x, y, z, q;  // position relative to the home cell's corner (length units), charge
};

// Staged neighbours per pass (CAP): 1024 (16 KB of LDS in FP32, 32 KB in
// FP64); FP32 takes 512 when the cells outnumber four work-groups per CU, so
// that more share a CU (10^6 ions: 2.61 instead of 2.83 ms with a 16-entry
// queue), and keeps 1024, fewer staging passes, when every cell already runs
// at once.

// FP32 erfc(x) for x >= 0 from e2 = e^{-x^2}: e2 t sum a_i t^i, t = 1/(1 + p x)
// (the form of Abramowitz-Stegun 7.1.26 with eight terms fitted for relative
// accuracy 5.7e-8 on [0, 8]; coefficients printed by csrc/erfc_fit.py).
__device__ inline float erfc_from_exp(float x, float e2) {
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * x);
  float s = -1.445127714e-01f;
  s = fmaf(s, t, 5.111943020e-01f);
  s = fmaf(s, t, -4.318033468e-01f);
  s = fmaf(s, t, 4.781717052e-01f);
  s = fmaf(s, t, 1.147496118e-02f);
  s = fmaf(s, t, 2.104277537e-01f);
  s = fmaf(s, t, 1.799369890e-01f);
  s = fmaf(s, t, 1.851103503e-01f);
  return e2 * t * s;
}

// One pair in range: adds q_n erfc(xi r)/r to ph and
// q_n (2 xi/sqrt(pi) e^{-xi^2 r^2} + erfc(xi r)/r) r_vec / r^2 to f.
__device__ inline void pair_term(float rx, float ry, float rz, float r2, float qn, float xi,
                                 float c2, float &ph, float &fx, float &fy, float &fz) {
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float x = xi * r2 * rinv;
  const float e2 = __expf(-x * x);
  const float ec = erfc_from_exp(x, e2) * rinv;
  ph = fmaf(qn, ec, ph);
  const float fr = qn * fmaf(c2, e2, ec) * rinv * rinv;
  fx = fmaf(fr, rx, fx);
  fy = fmaf(fr, ry, fy);
  fz = fmaf(fr, rz, fz);
}

// FP64 erfc(x) for x >= 0 from e2 = e^{-x^2}, the same form with seventeen
// terms (relative accuracy 3.1e-15 on [0, 6.5]; past 6.5 the sum stays in
// [0.18, 0.27], so the absolute error stays below 1e-19; coefficients
// printed by csrc/erfc_fit.py).  t comes from the hardware reciprocal and
// two Newton steps.
__device__ inline double erfc_from_exp(double x, double e2) {
  const double d = fma(0.3275911, x, 1.0);
  double t = __builtin_amdgcn_rcp(d);
  t = fma(t, fma(-d, t, 1.0), t);
  t = fma(t, fma(-d, t, 1.0), t);
  double s = 4.43316889962291991e-03;
  s = fma(s, t, -5.31251213997580851e-02);
  s = fma(s, t, 2.86756754026755822e-01);
  s = fma(s, t, -9.16781273041880396e-01);
  s = fma(s, t, 1.92458234028409003e+00);
  s = fma(s, t, -2.80197466275800489e+00);
  s = fma(s, t, 2.96517744131502781e+00);
  s = fma(s, t, -2.40169469331875085e+00);
  s = fma(s, t, 1.49703442398298314e+00);
  s = fma(s, t, -6.91707206481767534e-01);
  s = fma(s, t, 3.31178847928336517e-01);
  s = fma(s, t, 1.47299983323466166e-02);
  s = fma(s, t, 1.44269557494913714e-01);
  s = fma(s, t, 1.52276933253771785e-01);
  s = fma(s, t, 1.75217196070903275e-01);
  s = fma(s, t, 1.84802126744575718e-01);
  s = fma(s, t, 1.84824168666835043e-01);
  return e2 * t * s;
}

// FP64 pair term: 1/r from the hardware reciprocal square root and two
// Newton steps on e = 1 - r^2 y^2 (y <- y + y e/2, quadratic convergence
// from its 2^-22 start), and one exponential shared by erfc and the force.
__device__ inline void pair_term(double rx, double ry, double rz, double r2, double qn, double xi,
                                 double c2, double &ph, double &fx, double &fy, double &fz) {
  double rinv = __builtin_amdgcn_rsq(r2);
  rinv = fma(0.5 * rinv, fma(-r2 * rinv, rinv, 1.0), rinv);
  rinv = fma(0.5 * rinv, fma(-r2 * rinv, rinv, 1.0), rinv);
  const double x = xi * r2 * rinv;
  const double e2 = exp(-x * x);
  const double ec = erfc_from_exp(x, e2) * rinv;
  ph = fma(qn, ec, ph);
  const double fr = qn * fma(c2, e2, ec) * rinv * rinv;
  fx = fma(fr, rx, fx);
  fy = fma(fr, ry, fy);
  fz = fma(fr, rz, fz);
}

// One work-group per cell.  The particles of the 27 neighbour cells (home
// cell included) are staged in LDS, in passes of CAP.  Home particles
// take nhp = min(nh, 256) lanes, and the other lanes take the same home
// particles again: G = 256 / nhp slices of the staged range per home particle,
// summed at the end.  Each thread first tests its candidates (distance only)
// and queues the indices of the pairs in range in LDS; the wave evaluates the
// queued pairs together once some lane's queue could overflow, so the erfc and
// exp run on full waves instead of on every tested pair under a mask.
template <typename R, int CAP, int QN, int RCH>
__global__ void __launch_bounds__(kRsThreads)
k_rs_pairs(const SortedParticle<R> *__restrict__ sorted, const int2 *__restrict__ meta,
           const int *__restrict__ offsets, int nc, R cs, R xi, R rc2, R *__restrict__ phi,
           R *__restrict__ F, double *__restrict__ epart) {
  // a batch of tests appends at most kBatch entries after a flush check that
  // left at most QN - kBatch, so qn never exceeds QN
  static_assert(QN >= kBatch, "a batch of tests must fit the queue");
  constexpr int W = 2 * RCH + 1, NB = W * W * W;  // neighbour cells, home at NB / 2
  static_assert(NB <= 128, "the prefix sum takes two neighbour cells per lane of one wave");
  __shared__ Staged<R> stage[CAP];
  __shared__ int queue[QN * kRsThreads];  // entry m of thread t at m * 256 + t
  __shared__ int nb_src[NB], nb_pre[NB + 1];
  __shared__ R red[4][kRsThreads];
  __shared__ double ered[kRsThreads / 64];
  const int tid = threadIdx.x;
  const int cell = xcd_local(blockIdx.x, gridDim.x);
  const int cz = cell / (nc * nc), cy = (cell / nc) % nc, cx = cell % nc;
  if (tid < NB) {
    const int oz = tid / (W * W) - RCH, oy = (tid / W) % W - RCH, ox = tid % W - RCH;
    const int nz = cz + oz < 0 ? cz + oz + nc : (cz + oz >= nc ? cz + oz - nc : cz + oz);
    const int ny = cy + oy < 0 ? cy + oy + nc : (cy + oy >= nc ? cy + oy - nc : cy + oy);
    const int nx = cx + ox < 0 ? cx + ox + nc : (cx + ox >= nc ? cx + ox - nc : cx + ox);
    const int nb = (nz * nc + ny) * nc + nx;
    nb_src[tid] = offsets[nb];
    nb_pre[tid + 1] = offsets[nb + 1] - offsets[nb];
  }
  __syncthreads();
  if (tid < 64) {
    // inclusive prefix sum of the counts nb_pre[1..NB], two per lane
    const int i1 = 2 * tid + 1, i2 = 2 * tid + 2;
    const int a = i1 <= NB ? nb_pre[i1] : 0, b = i2 <= NB ? nb_pre[i2] : 0;
    const int v = wave_inclusive_scan(a + b);
    const int before = v - a - b;
    if (i1 <= NB) nb_pre[i1] = before + a;
    if (i2 <= NB) nb_pre[i2] = v;
    if (tid == 0) nb_pre[0] = 0;
  }
  __syncthreads();
  const int S = nb_pre[NB];
  const int home0 = nb_pre[NB / 2];  // home cell (offset 0,0,0) in the staged order
  const int nh = nb_pre[NB / 2 + 1] - home0;
  const int hsrc = nb_src[NB / 2];
  const R c2 = static_cast<R>(1.1283791670955126) * xi;  // 2 xi / sqrt(pi)
  double e = 0.0;

  for (int hb = 0; hb < nh; hb += kRsThreads) {  // uniform across the work-group
    const int nhp = min(kRsThreads, nh - hb);
    const int G = kRsThreads / nhp;
    const int hi = tid % nhp, sl = tid / nhp;
    const bool active = sl < G;
    const SortedParticle<R> pi = sorted[hsrc + hb + hi];
    const R px = pi.dx * cs, py = pi.dy * cs, pz = pi.dz * cs;
    const int self = home0 + hb + hi;
    R ph = R(0), fx = R(0), fy = R(0), fz = R(0);
    for (int c0 = 0; c0 < S; c0 += CAP) {
      const int cn = min(CAP, S - c0);
      __syncthreads();  // previous pass consumed
      {
        // stage this pass: all loads issued before the first LDS store
        constexpr int PER = CAP / kRsThreads;
        SortedParticle<R> buf[PER];
        int kk[PER];
        int k = 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int j = c0 + tid + u * kRsThreads;
          kk[u] = -1;
          if (j < c0 + cn) {
            if constexpr (RCH > 1) {
              // neighbour cell of staged particle j: the last k with nb_pre[k] <= j
              int lo_k = k, hi_k = NB - 1;
              while (lo_k < hi_k) {
                const int mid = (lo_k + hi_k + 1) >> 1;
                if (nb_pre[mid] <= j) lo_k = mid; else hi_k = mid - 1;
              }
              k = lo_k;
            }
            while (nb_pre[k + 1] <= j) ++k;
            kk[u] = k;
            buf[u] = sorted[nb_src[k] + (j - nb_pre[k])];
          }
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          if (kk[u] >= 0) {
            const int kc = kk[u];
            stage[tid + u * kRsThreads] =
                Staged<R>{(static_cast<R>(kc % W - RCH) + buf[u].dx) * cs,
                          (static_cast<R>((kc / W) % W - RCH) + buf[u].dy) * cs,
                          (static_cast<R>(kc / (W * W) - RCH) + buf[u].dz) * cs, buf[u].q};
          }
        }
      }
      __syncthreads();
      // this thread's slice of the pass
      const int lo = active ? sl * cn / G : 0, hi_end = active ? (sl + 1) * cn / G : 0;
      const int self_l = self - c0;
      int qn = 0;
      auto flush = [&]() {
        for (int m0 = 0; __any(m0 < qn); m0 += kBatch) {
          // rows past the queue (QN need not be a multiple of kBatch) are
          // not read; such entries are beyond qn <= QN and masked below
          int idx[kBatch];
#pragma unroll
          for (int u = 0; u < kBatch; ++u)
            idx[u] = m0 + u < QN ? queue[(m0 + u) * kRsThreads + tid] : 0;
          Staged<R> c[kBatch];
#pragma unroll
          for (int u = 0; u < kBatch; ++u) c[u] = stage[min(static_cast<unsigned>(idx[u]),
                                                            static_cast<unsigned>(cn - 1))];
#pragma unroll
          for (int u = 0; u < kBatch; ++u) {
            if (m0 + u < qn) {
              const R rx = px - c[u].x, ry = py - c[u].y, rz = pz - c[u].z;
              pair_term(rx, ry, rz, rx * rx + ry * ry + rz * rz, c[u].q, xi, c2, ph, fx, fy, fz);
            }
          }
        }
        qn = 0;
      };
      for (int k0 = lo; __any(k0 < hi_end); k0 += kBatch) {
        Staged<R> c[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) c[u] = stage[min(k0 + u, cn - 1)];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const int idx = k0 + u;
          const R rx = px - c[u].x, ry = py - c[u].y, rz = pz - c[u].z;
          const R r2 = rx * rx + ry * ry + rz * rz;
          const bool hit = idx < hi_end && r2 < rc2 && idx != self_l;
          // the free slot qn is written either way; only a hit keeps it
          queue[qn * kRsThreads + tid] = idx;
          qn += hit ? 1 : 0;
        }
        if (__any(qn > QN - kBatch)) flush();
      }
      flush();
    }
    // sum the slices of each home particle
    __syncthreads();
    red[0][tid] = ph;
    red[1][tid] = fx;
    red[2][tid] = fy;
    red[3][tid] = fz;
    __syncthreads();
    if (sl == 0) {
      for (int g = 1; g < G; ++g) {
        ph += red[0][g * nhp + hi];
        fx += red[1][g * nhp + hi];
        fy += red[2][g * nhp + hi];
        fz += red[3][g * nhp + hi];
      }
      const int orig = meta[hsrc + hb + hi].y;
      if (phi) phi[orig] = ph;
      if (F) {
        F[3 * orig + 0] = pi.q * fx;
        F[3 * orig + 1] = pi.q * fy;
        F[3 * orig + 2] = pi.q * fz;
      }
      e += 0.5 * static_cast<double>(pi.q) * static_cast<double>(ph);
    }
  }
  // energy partial of this cell (fixed order)
  e = wave_reduce0(e, [](double a, double b) { return a + b; });
  if ((tid & 63) == 0) ered[tid >> 6] = e;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < kRsThreads / 64; ++w) s += ered[w];
    epart[cell] = s;
  }
}

// E = sum of the cell partials in a fixed order (one work-group).
__global__ void __launch_bounds__(kRsThreads)
k_rs_energy(const double *__restrict__ epart, int n, double *__restrict__ E) {
  __shared__ double red[kRsThreads / 64];
  // each thread sums its strided share in index order, loads issued eight
  // at a time (the cell count reaches 64^3)
  constexpr int U = 8;
  double s = 0.0;
  for (int i0 = threadIdx.x; i0 < n; i0 += U * kRsThreads) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * kRsThreads;
      v[u] = i < n ? epart[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  s = wave_reduce0(s, [](double a, double b) { return a + b; });
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kRsThreads / 64; ++w) t += red[w];
    *E = t;
  }
}

template <typename R>
hipError_t rs_eval(se_rs_plan &p, int N, const void *x, const void *q, double *E, void *phi,
                   void *F) {
  p.reach = rs_reach(p.L, p.rc, N);
  p.nc = rs_cells_per_side(p.L, p.rc, p.reach);
  p.ncells = p.nc * p.nc * p.nc;
  p.cs = p.L / p.nc;
  if (p.nc > p.nc_max) return hipErrorInvalidValue;
  BinJob j;
  j.N = N;
  j.x = x;
  j.q = q;
  j.fp64 = sizeof(R) == 8;
  j.h = p.cs;
  j.M = p.nc;
  j.T = 1;
  j.ntx = p.nc;
  j.ncells = p.ncells;
  j.counts = p.counts;
  j.key = p.key;
  j.offsets = p.offsets;
  j.sorted = p.sorted;
  j.meta = p.meta;
  j.qsq_part = p.part;
  j.stream = p.stream;
  hipError_t e = launch_bin_job(j, nullptr);
  if (e != hipSuccess) return e;
  double *epart = p.part + p.bin_blocks;
  const auto sorted = static_cast<const SortedParticle<R> *>(p.sorted);
  const R cs = static_cast<R>(p.cs), xi = static_cast<R>(p.xi), rc2 = static_cast<R>(p.rc * p.rc);
  const auto run = [&](auto kernel) {
    kernel<<<p.ncells, kRsThreads, 0, p.stream>>>(sorted, p.meta, p.offsets, p.nc, cs, xi, rc2,
                                                  static_cast<R *>(phi), static_cast<R *>(F),
                                                  epart);
  };
  bool small_stage = false;
  if constexpr (sizeof(R) == 4) {
    small_stage = p.ncells > 4 * p.cus;
    if (small_stage) {
      if (p.reach == 2)
        run(k_rs_pairs<R, 512, 12, 2>);
      else
        run(k_rs_pairs<R, 512, 12, 1>);
    }
  }
  if (!small_stage) {
    if (p.reach == 2)
      run(k_rs_pairs<R, 1024, sizeof(R) == 4 ? 16 : 32, 2>);
    else
      run(k_rs_pairs<R, 1024, sizeof(R) == 4 ? 16 : 32, 1>);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_rs_energy<<<1, kRsThreads, 0, p.stream>>>(epart, p.ncells, E);
  return hipGetLastError();
}

se_status rs_fail(se_status s, const char *fmt, double a, double b) {
  char buf[256];
  snprintf(buf, sizeof(buf), fmt, a, b);
  return report(s, buf);
}

void rs_free(se_rs_plan &p) {
  void *ptrs[] = {p.counts, p.offsets, p.key, p.meta, p.sorted, p.part};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
}

}  // namespace

// Cell list of the real-space sum of N particles, box edge L, cutoff
// rc <= L/3: cells of edge >= rc searched one cell to each side (3^3
// neighbour cells, which test 27 cs^3 / ((4/3) pi rc^3) >= 6.4 times the
// pairs in range), or cells of edge >= rc / 2 searched two to each side
// (5^3 cells, 3.7 times).  The finer list pays a fixed cost per cell (125
// neighbour ranges to find and stage) and wins only where its cells are
// populated: MI355X times (FP32 and FP64, 20k-400k particles, rc 4-12 at
// 0.1 per unit volume) favour it from 10 particles per cell, and from 5
// when the coarse list has fewer than 1024 cells (four work-groups per CU);
// below 3 per cell it took 1.7 to 8 times as long.  At most 64 cells per
// side (the counters take a cache line each); larger cells stay correct.
int rs_reach(double L, double rc, long long N) {
  const double nc1 = std::floor(L / rc);
  if (nc1 >= 64.0) return 1;
  const double nc2 = std::fmin(std::floor(2.0 * L / rc), 64.0);
  const double occ = static_cast<double>(N) / (nc2 * nc2 * nc2);
  return (occ >= 10.0 || (occ >= 5.0 && nc1 * nc1 * nc1 < 1024.0)) ? 2 : 1;
}
int rs_cells_per_side(double L, double rc, int reach) {
  return static_cast<int>(std::fmin(std::floor(reach * L / rc), 64.0));
}

}  // namespace sek

extern "C" {

se_status se_rs_plan_create(double L, double xi, double rc, int dtype, int n_max,
                            void *hip_stream, se_rs_plan **out) {
  using sek::rs_fail;
  if (!out) return sek::report(SE_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!(L > 0.0) || !std::isfinite(L) || !(xi > 0.0) || !std::isfinite(xi))
    return rs_fail(SE_ERR_ARG, "L and xi must be finite and > 0 (got %g, %g)", L, xi);
  if (!(rc > 0.0) || !(3.0 * rc <= L))
    return rs_fail(SE_ERR_ARG, "cutoff rc = %g must lie in (0, L/3], L = %g", rc, L);
  if (dtype != SE_FP32 && dtype != SE_FP64) return sek::report(SE_ERR_ARG, "unknown dtype");
  if (n_max < 1) return sek::report(SE_ERR_ARG, "n_max must be >= 1");
  // the cell list of each call follows its N (sek::rs_reach); the buffers
  // hold the finer of the two
  const int nc = sek::rs_cells_per_side(L, rc, std::floor(L / rc) >= 64.0 ? 1 : 2);
  se_rs_plan *p = new (std::nothrow) se_rs_plan{};
  if (!p) return sek::report(SE_ERR_WORKSPACE, "host allocation failed");
  p->L = L;
  p->xi = xi;
  p->rc = rc;
  p->dtype = dtype;
  p->n_max = n_max;
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->nc_max = nc;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    p->cus = cus;
  }
  p->bin_blocks = (n_max + sek::kThreads - 1) / sek::kThreads;
  const size_t cells_max = static_cast<size_t>(nc) * nc * nc;
  const size_t rs = dtype == SE_FP64 ? 8 : 4;
  struct { void **ptr; size_t n; } allocs[] = {
      {reinterpret_cast<void **>(&p->counts), cells_max * sek::kCountStride * 4},
      {reinterpret_cast<void **>(&p->offsets),
       (cells_max + 1 + static_cast<size_t>(sek::scan_chunks(static_cast<int>(cells_max)))) * 4},
      {reinterpret_cast<void **>(&p->key), static_cast<size_t>(n_max) * 8},
      {reinterpret_cast<void **>(&p->meta), static_cast<size_t>(n_max) * 8},
      {&p->sorted, static_cast<size_t>(n_max) * 4 * rs},
      {reinterpret_cast<void **>(&p->part), (p->bin_blocks + cells_max) * 8}};
  for (auto &a : allocs) {
    hipError_t e = hipMalloc(a.ptr, a.n);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      sek::rs_free(*p);
      delete p;
      return sek::report(SE_ERR_WORKSPACE, "hipMalloc failed for the real-space workspace");
    }
  }
  hipError_t e = hipMemset(p->counts, 0, cells_max * sek::kCountStride * 4);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    sek::rs_free(*p);
    delete p;
    return sek::report(SE_ERR_HIP, hipGetErrorString(e));
  }
  *out = p;
  return SE_OK;
}

se_status se_rs_plan_set_stream(se_rs_plan *plan, void *hip_stream) {
  if (!plan) return sek::report(SE_ERR_ARG, "plan is NULL");
  plan->stream = static_cast<hipStream_t>(hip_stream);
  return SE_OK;
}

se_status se_rs_eval(se_rs_plan *plan, int N, const void *x, const void *q, double *E_dev,
                     void *phi, void *F) {
  if (!plan) return sek::report(SE_ERR_ARG, "plan is NULL");
  if (N < 0 || N > plan->n_max) return sek::report(SE_ERR_ARG, "N outside [0, n_max]");
  if (N > 0 && (!x || !q)) return sek::report(SE_ERR_ARG, "x or q is NULL");
  if (!E_dev) return sek::report(SE_ERR_ARG, "E_dev is NULL");
  const hipError_t e = plan->dtype == SE_FP64
                           ? sek::rs_eval<double>(*plan, N, x, q, E_dev, phi, F)
                           : sek::rs_eval<float>(*plan, N, x, q, E_dev, phi, F);
  if (e != hipSuccess) return sek::report(SE_ERR_HIP, hipGetErrorString(e));
  return SE_OK;
}

se_status se_rs_plan_destroy(se_rs_plan *plan) {
  if (!plan) return SE_OK;
  const hipError_t e = hipStreamSynchronize(plan->stream);
  sek::rs_free(*plan);
  delete plan;
  return e == hipSuccess ? SE_OK : sek::report(SE_ERR_HIP, hipGetErrorString(e));
}

}  // extern "C"
