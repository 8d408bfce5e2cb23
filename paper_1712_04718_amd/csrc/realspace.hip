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
// one point of an nc^3 grid); their stored offsets from the cell corner (in
// units of cs) give distances without the rounding of absolute coordinates.
// One work-group per cell: each thread holds one particle of the cell and
// the 27 neighbour cells are staged in LDS in turn.
#include <cmath>
#include <cstdio>
#include <new>

#include "se_common.hpp"

struct se_rs_plan {
  double L, xi, rc;
  int dtype;
  int n_max;
  hipStream_t stream;
  int nc;        // cells per side
  int ncells;
  double cs;     // cell edge
  int bin_blocks;
  int *counts = nullptr;
  int *offsets = nullptr;
  int2 *key = nullptr;
  int2 *meta = nullptr;
  void *sorted = nullptr;
  double *part = nullptr;  // q^2 partials of binning (unused), then energy partials
  int last_N = -1;
};

namespace sek {
namespace {

constexpr int kRsThreads = 256;

template <typename R> struct alignas(4 * sizeof(R)) Staged {
  R x, y, z, q;  // position relative to the home cell's corner (cell units), charge
};

template <typename R> __device__ inline R erfc_r(R v);
template <> __device__ inline float erfc_r<float>(float v) { return erfcf(v); }
template <> __device__ inline double erfc_r<double>(double v) { return erfc(v); }
template <typename R> __device__ inline R exp_r(R v);
template <> __device__ inline float exp_r<float>(float v) { return expf(v); }
template <> __device__ inline double exp_r<double>(double v) { return exp(v); }

template <typename R>
__global__ void __launch_bounds__(kRsThreads)
k_rs_pairs(const SortedParticle<R> *__restrict__ sorted, const int2 *__restrict__ meta,
           const int *__restrict__ offsets, int nc, R cs, R xi, R rc2, R *__restrict__ phi,
           R *__restrict__ F, double *__restrict__ epart) {
  __shared__ Staged<R> stage[kRsThreads];
  const int tid = threadIdx.x;
  const int cell = xcd_local(blockIdx.x, gridDim.x);
  const int cz = cell / (nc * nc), cy = (cell / nc) % nc, cx = cell % nc;
  const int h0 = offsets[cell], h1 = offsets[cell + 1];
  const R c2 = static_cast<R>(1.1283791670955126) * xi;  // 2 xi / sqrt(pi)
  double e = 0.0;
  for (int hb = h0; hb < h1; hb += kRsThreads) {  // uniform across the work-group
    const int i = hb + tid;
    const bool mine = i < h1;
    SortedParticle<R> pi{};
    if (mine) pi = sorted[i];
    R ph = R(0), fx = R(0), fy = R(0), fz = R(0);
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int nz = cz + oz < 0 ? cz + oz + nc : (cz + oz >= nc ? cz + oz - nc : cz + oz);
          const int ny = cy + oy < 0 ? cy + oy + nc : (cy + oy >= nc ? cy + oy - nc : cy + oy);
          const int nx = cx + ox < 0 ? cx + ox + nc : (cx + ox >= nc ? cx + ox - nc : cx + ox);
          const int nb = (nz * nc + ny) * nc + nx;
          const int n0 = offsets[nb], n1 = offsets[nb + 1];
          const bool home = oz == 0 && oy == 0 && ox == 0;
          for (int nbb = n0; nbb < n1; nbb += kRsThreads) {
            __syncthreads();  // previous batch consumed
            const int j = nbb + tid;
            if (j < n1) {
              const SortedParticle<R> sj = sorted[j];
              stage[tid] = Staged<R>{static_cast<R>(ox) + sj.dx, static_cast<R>(oy) + sj.dy,
                                     static_cast<R>(oz) + sj.dz, sj.q};
            }
            __syncthreads();
            const int cnt = min(kRsThreads, n1 - nbb);
            if (mine) {
              for (int k = 0; k < cnt; ++k) {
                const Staged<R> s = stage[k];
                const R rx = (pi.dx - s.x) * cs, ry = (pi.dy - s.y) * cs, rz = (pi.dz - s.z) * cs;
                const R r2 = rx * rx + ry * ry + rz * rz;
                if (r2 < rc2 && !(home && nbb + k == i)) {
                  const R r = sqrt(r2);
                  const R ec = erfc_r(xi * r) / r;
                  ph += s.q * ec;
                  const R fr = s.q * (c2 * exp_r(-xi * xi * r2) + ec) / r2;
                  fx += fr * rx;
                  fy += fr * ry;
                  fz += fr * rz;
                }
              }
            }
          }
        }
    if (mine) {
      const int orig = meta[i].y;
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
  for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
  __shared__ double red[kRsThreads / 64];
  if ((tid & 63) == 0) red[tid >> 6] = e;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < kRsThreads / 64; ++w) s += red[w];
    epart[cell] = s;
  }
}

// E = sum of the cell partials in a fixed order (one work-group).
__global__ void __launch_bounds__(kRsThreads)
k_rs_energy(const double *__restrict__ epart, int n, double *__restrict__ E) {
  __shared__ double red[kRsThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kRsThreads) s += epart[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = kRsThreads / 2; st > 0; st >>= 1) {
    if (static_cast<int>(threadIdx.x) < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *E = red[0];
}

template <typename R>
hipError_t rs_eval(se_rs_plan &p, int N, const void *x, const void *q, double *E, void *phi,
                   void *F) {
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
  k_rs_pairs<R><<<p.ncells, kRsThreads, 0, p.stream>>>(
      static_cast<const SortedParticle<R> *>(p.sorted), p.meta, p.offsets, p.nc,
      static_cast<R>(p.cs), static_cast<R>(p.xi), static_cast<R>(p.rc * p.rc),
      static_cast<R *>(phi), static_cast<R *>(F), epart);
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
  // cells of edge L / nc >= rc; at most 64 per side (the counters take a
  // cache line each), larger cells are still correct
  const int nc = static_cast<int>(std::fmin(std::floor(L / rc), 64.0));
  se_rs_plan *p = new (std::nothrow) se_rs_plan{};
  if (!p) return sek::report(SE_ERR_WORKSPACE, "host allocation failed");
  p->L = L;
  p->xi = xi;
  p->rc = rc;
  p->dtype = dtype;
  p->n_max = n_max;
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->nc = nc;
  p->ncells = nc * nc * nc;
  p->cs = L / nc;
  p->bin_blocks = (n_max + sek::kThreads - 1) / sek::kThreads;
  const size_t rs = dtype == SE_FP64 ? 8 : 4;
  struct { void **ptr; size_t n; } allocs[] = {
      {reinterpret_cast<void **>(&p->counts), static_cast<size_t>(p->ncells) * sek::kCountStride * 4},
      {reinterpret_cast<void **>(&p->offsets), static_cast<size_t>(p->ncells + 1) * 4},
      {reinterpret_cast<void **>(&p->key), static_cast<size_t>(n_max) * 8},
      {reinterpret_cast<void **>(&p->meta), static_cast<size_t>(n_max) * 8},
      {&p->sorted, static_cast<size_t>(n_max) * 4 * rs},
      {reinterpret_cast<void **>(&p->part), static_cast<size_t>(p->bin_blocks + p->ncells) * 8}};
  for (auto &a : allocs) {
    hipError_t e = hipMalloc(a.ptr, a.n);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      sek::rs_free(*p);
      delete p;
      return sek::report(SE_ERR_WORKSPACE, "hipMalloc failed for the real-space workspace");
    }
  }
  hipError_t e = hipMemset(p->counts, 0, static_cast<size_t>(p->ncells) * sek::kCountStride * 4);
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
  plan->last_N = N;
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
