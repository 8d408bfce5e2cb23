// Step 1 of the k-space evaluation: sort particles into T^3 tiles of the grid.
//
// A particle's anchor is the grid point floor(x/h) (taken modulo M); its
// truncated window (Gaussian, section 4; or B-spline, section 6) covers a
// fixed stencil relative to that anchor, so all particles anchored in one
// tile touch one (T+S-1)^3 block of the grid.  Spreading and gathering then
// run one work-group per tile with that block staged in LDS.
//
// k_bin_count: zero the spread grid, compute each particle's tile and its
//   rank inside the tile (atomic counter), and the per-block sums of q^2;
//   the last block to finish turns the tile counts into offsets (exclusive
//   scan), resets the counts for the next call and totals q^2.
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
k_bin_count(int N, const R *__restrict__ x, const R *__restrict__ q, double h,
            int M, int T, int ntx, int *__restrict__ counts,
            int2 *__restrict__ key, double *__restrict__ qsq_part,
            unsigned *__restrict__ done, int *__restrict__ offsets, int ntiles,
            double *__restrict__ qsq_total, R *__restrict__ grid,
            long long ngrid) {
  const int tid = threadIdx.x;
  // zero the spread grid (accumulated with atomics by the spreading kernel)
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + tid; i < ngrid;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    grid[i] = R(0);

  const int n = blockIdx.x * blockDim.x + tid;
  double qq = 0.0;
  if (n < N) {
    double frac;
    const int ax = static_cast<int>(floor_div_mod(static_cast<double>(x[3 * n + 0]) / h, M, &frac));
    const int ay = static_cast<int>(floor_div_mod(static_cast<double>(x[3 * n + 1]) / h, M, &frac));
    const int az = static_cast<int>(floor_div_mod(static_cast<double>(x[3 * n + 2]) / h, M, &frac));
    const int tile = ((az / T) * ntx + ay / T) * ntx + ax / T;
    const int rank = atomicAdd(&counts[tile], 1);
    key[n] = make_int2(tile, rank);
    const double qn = static_cast<double>(q[n]);
    qq = qn * qn;
  }

  __shared__ double red[kThreads];
  red[tid] = qq;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) qsq_part[blockIdx.x] = red[0];

  // Last-arriving block: exclusive scan of the tile counts.
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (tid == 0) is_last = (atomicAdd(done, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!is_last) return;
  __threadfence();

  const int chunk = (ntiles + kThreads - 1) / kThreads;
  const int lo = min(tid * chunk, ntiles), hi = min(lo + chunk, ntiles);
  int local = 0;
  for (int t = lo; t < hi; ++t)
    local += __hip_atomic_load(&counts[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __shared__ int scan[kThreads];
  scan[tid] = local;
  __syncthreads();
  for (int s = 1; s < kThreads; s <<= 1) {  // inclusive Hillis-Steele scan
    const int v = tid >= s ? scan[tid - s] : 0;
    __syncthreads();
    scan[tid] += v;
    __syncthreads();
  }
  int run = scan[tid] - local;  // exclusive prefix of this chunk
  for (int t = lo; t < hi; ++t) {
    const int c = __hip_atomic_load(&counts[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    offsets[t] = run;
    run += c;
    counts[t] = 0;  // ready for the next call
  }
  if (tid == kThreads - 1) offsets[ntiles] = scan[kThreads - 1];

  // total of q^2 in a fixed order (deterministic)
  double s = 0.0;
  for (int b = tid; b < static_cast<int>(gridDim.x); b += kThreads)
    s += __hip_atomic_load(&qsq_part[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  red[tid] = s;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (tid < st) red[tid] += red[tid + st];
    __syncthreads();
  }
  if (tid == 0) {
    *qsq_total = red[0];
    *done = 0u;
  }
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
  const long long ngrid = static_cast<long long>(M) * M * M;
  const int blocks = N > 0 ? (N + kThreads - 1) / kThreads : 1;
  stage_begin(p, SE_STAGE_BIN_COUNT);
  k_bin_count<R><<<blocks, kThreads, 0, p.stream>>>(
      N, static_cast<const R *>(x), static_cast<const R *>(q), p.h, M, p.T, p.ntx,
      p.buf.counts, p.buf.key, p.buf.part, p.buf.done, p.buf.offsets, p.ntiles,
      p.buf.qsq, static_cast<R *>(p.buf.grid), ngrid);
  stage_end(p, SE_STAGE_BIN_COUNT);
  hipError_t e = hipGetLastError();
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
