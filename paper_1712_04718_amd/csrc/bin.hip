// Step 1 of the k-space evaluation: sort particles into T^3 tiles of the grid.
//
// A particle's anchor is the grid point floor(x/h) (taken modulo M); its
// truncated window (Gaussian, section 4; or B-spline, section 6) covers a
// fixed stencil relative to that anchor, so all particles anchored in one
// tile touch one (T+S-1)^3 block of the grid.  Spreading and gathering then
// run one work-group per tile with that block staged in LDS.
//
// k_bin_count: each particle's tile and its rank inside the tile (atomic
//   counter), and per-block sums of q^2;
// k_bin_scan: one work-group turns the tile counts into offsets (exclusive
//   scan), resets the counts for the next call and totals q^2;
// k_bin_scatter: write the particles in tile order as (offsets from the
//   anchor in grid units, q) plus (packed local anchor, original index).
#include "se_common.hpp"

namespace sek {
namespace {

__device__ inline long long floor_div_mod(double u, int M, double *frac) {
  double fl = floor(u);
  *frac = u - fl;
  long long i = static_cast<long long>(fl) % M;
  return i < 0 ? i + M : i;
}

template <typename R>
__global__ void __launch_bounds__(kThreads)
k_bin_count(int N, const R *__restrict__ x, const R *__restrict__ q, double h, int M, int T,
            int ntx, int *__restrict__ counts, int2 *__restrict__ key,
            double *__restrict__ qsq_part) {
  const int tid = threadIdx.x;
  const int n = blockIdx.x * blockDim.x + tid;
  double qq = 0.0;
  int tile = -1;
  if (n < N) {
    double frac;
    const int ax = static_cast<int>(floor_div_mod(static_cast<double>(x[3 * n + 0]) / h, M, &frac));
    const int ay = static_cast<int>(floor_div_mod(static_cast<double>(x[3 * n + 1]) / h, M, &frac));
    const int az = static_cast<int>(floor_div_mod(static_cast<double>(x[3 * n + 2]) / h, M, &frac));
    tile = ((az / T) * ntx + ay / T) * ntx + ax / T;
    const double qn = static_cast<double>(q[n]);
    qq = qn * qn;
  }
  // Runs of equal tiles among neighbouring lanes (the atoms of a molecule are
  // usually adjacent in the input) take one atomic per run.
  const int lane = tid & 63;
  const int prev = __shfl_up(tile, 1);
  const bool head = lane == 0 || tile != prev;
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1);
  const int run0 = 63 - __clzll(heads & upto);            // first lane of my run
  const unsigned long long after = heads & ~upto;
  const int run_end = after ? __ffsll(after) - 1 : 64;    // first lane of the next run
  int base = 0;
  if (head && tile >= 0) base = atomicAdd(&counts[tile * kCountStride], run_end - lane);
  base = __shfl(base, run0);
  if (tile >= 0) key[n] = make_int2(tile, base + lane - run0);
  for (int o = 32; o > 0; o >>= 1) qq += __shfl_xor(qq, o);
  __shared__ double red[kThreads / 64];
  if ((tid & 63) == 0) red[tid >> 6] = qq;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) s += red[w];
    qsq_part[blockIdx.x] = s;
  }
}

// One work-group: exclusive scan of the tile counts into offsets, counts reset
// for the next call, and the total of q^2 (fixed order, deterministic).
__global__ void __launch_bounds__(kThreads)
k_bin_scan(int *__restrict__ counts, int *__restrict__ offsets, int ntiles,
           const double *__restrict__ qsq_part, int nparts, double *__restrict__ qsq_total) {
  const int tid = threadIdx.x;
  const int chunk = (ntiles + kThreads - 1) / kThreads;
  const int lo = min(tid * chunk, ntiles), hi = min(lo + chunk, ntiles);
  int local = 0;
  for (int t = lo; t < hi; ++t) local += counts[t * kCountStride];
  __shared__ int scan[kThreads];
  scan[tid] = local;
  __syncthreads();
  for (int s = 1; s < kThreads; s <<= 1) {  // inclusive Hillis-Steele scan
    const int v = tid >= s ? scan[tid - s] : 0;
    __syncthreads();
    scan[tid] += v;
    __syncthreads();
  }
  int run = scan[tid] - local;
  for (int t = lo; t < hi; ++t) {
    const int c = counts[t * kCountStride];
    offsets[t] = run;
    run += c;
    counts[t * kCountStride] = 0;
  }
  if (tid == kThreads - 1) offsets[ntiles] = scan[kThreads - 1];

  __shared__ double red[kThreads];
  double s = 0.0;
  for (int b = tid; b < nparts; b += kThreads) s += qsq_part[b];
  red[tid] = s;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) *qsq_total = red[0];
}

template <typename R>
__global__ void __launch_bounds__(kThreads)
k_bin_scatter(int N, const R *__restrict__ x, const R *__restrict__ q, double h,
              int M, int T, const int2 *__restrict__ key,
              const int *__restrict__ offsets,
              SortedParticle<R> *__restrict__ sorted, int2 *__restrict__ meta) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int2 k = key[n];
  const int dst = offsets[k.x] + k.y;
  double fx, fy, fz;
  const int ax = static_cast<int>(floor_div_mod(static_cast<double>(x[3 * n + 0]) / h, M, &fx));
  const int ay = static_cast<int>(floor_div_mod(static_cast<double>(x[3 * n + 1]) / h, M, &fy));
  const int az = static_cast<int>(floor_div_mod(static_cast<double>(x[3 * n + 2]) / h, M, &fz));
  SortedParticle<R> s;
  s.dx = static_cast<R>(fx);
  s.dy = static_cast<R>(fy);
  s.dz = static_cast<R>(fz);
  s.q = q[n];
  sorted[dst] = s;
  meta[dst] = make_int2((ax % T) | ((ay % T) << 8) | ((az % T) << 16), n);
}

template <typename R>
hipError_t bin_impl(se_plan &p, int N, const void *x, const void *q) {
  const int M = p.prm.M;
  const int blocks = N > 0 ? (N + kThreads - 1) / kThreads : 0;
  hipError_t e = hipSuccess;
  stage_begin(p, SE_STAGE_BIN_COUNT);
  if (blocks > 0) {
    k_bin_count<R><<<blocks, kThreads, 0, p.stream>>>(
        N, static_cast<const R *>(x), static_cast<const R *>(q), p.h, M, p.T, p.ntx,
        p.buf.counts, p.buf.key, p.buf.part);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    k_bin_scan<<<1, kThreads, 0, p.stream>>>(p.buf.counts, p.buf.offsets, p.ntiles, p.buf.part,
                                           blocks, p.buf.qsq);
    e = hipGetLastError();
  }
  stage_end(p, SE_STAGE_BIN_COUNT);
  if (e != hipSuccess || N == 0) return e;
  stage_begin(p, SE_STAGE_BIN_SCATTER);
  k_bin_scatter<R><<<blocks, kThreads, 0, p.stream>>>(
      N, static_cast<const R *>(x), static_cast<const R *>(q), p.h, M, p.T,
      p.buf.key, p.buf.offsets, static_cast<SortedParticle<R> *>(p.buf.sorted),
      p.buf.meta);
  stage_end(p, SE_STAGE_BIN_SCATTER);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bin(se_plan &plan, int N, const void *x, const void *q) {
  return plan.prm.dtype == SE_FP64 ? bin_impl<double>(plan, N, x, q)
                                   : bin_impl<float>(plan, N, x, q);
}

}  // namespace sek
