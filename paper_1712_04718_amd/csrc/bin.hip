// Step 1 of the k-space evaluation: sort particles into T^3 tiles of the grid.
//
// A particle's anchor is the grid point floor(x/h) (taken modulo M); its
// truncated window (Gaussian, section 4; or B-spline, section 6) covers a
// fixed stencil relative to that anchor, so all particles anchored in one
// tile touch one (T+S-1)^3 block of the grid.  Spreading and gathering then
// run one work-group per tile with that block staged in LDS.
//
// Counting: each particle gets its tile and its rank among the particles of
// that tile from an atomic add on the tile's counter (one cache line per
// counter).  Returning global atomics are the cost here, so they are
// aggregated:
//   k_bin_count_lds: a work-group takes its particles (256 threads x 1, or
//     1024 x 8 when tiles hold many particles), ranks them per tile with
//     LDS atomics, then adds each touched tile's count to the global
//     counter once and hands the returned base to its particles;
//   k_bin_count_run: for grids with more tiles than the LDS tables hold,
//     one atomic per run of equal tiles among neighbouring lanes of a wave
//     (the atoms of a molecule are usually adjacent in the input).
// Both also write per-block sums of q^2 (for the self energy).
// k_bin_scan: one work-group turns the tile counts into offsets (exclusive
//   scan) and resets the counts for the next call; above 2048 cells
//   k_bin_scan_sums and k_bin_scan_apply do it over chunks of 2048 cells on
//   as many work-groups (the real-space cell lists reach 85k cells);
// k_bin_scatter: write the particles in tile order as (offsets from the
//   anchor in grid units, q) plus (packed local anchor, original index);
// k_bin_scatter_scan: the two in one launch when tiles x work-groups is at
//   most 2^20 (each work-group scans the counts itself); the counts are
//   then reset by the kernel that consumes the tiles (the k-space spread).
#include "se_common.hpp"

namespace sek {
namespace {

constexpr int kLdsTilesMax = 8192;  // tiles the LDS tables of k_bin_count_lds hold

__device__ inline long long floor_div_mod(double u, int M, double *frac) {
  return anchor_mod(u, M, frac);
}

// Tile of a particle at (x0, x1, x2).
template <typename R>
__device__ inline int tile_of(R x0, R x1, R x2, double h, int M, int T, int ntx) {
  double frac;
  const int ax = static_cast<int>(floor_div_mod(static_cast<double>(x0) / h, M, &frac));
  const int ay = static_cast<int>(floor_div_mod(static_cast<double>(x1) / h, M, &frac));
  const int az = static_cast<int>(floor_div_mod(static_cast<double>(x2) / h, M, &frac));
  return ((az / T) * ntx + ay / T) * ntx + ax / T;
}

// Tile of particle n (and q_n^2).
template <typename R>
__device__ inline int particle_tile(const R *__restrict__ x, const R *__restrict__ q, int n,
                                    double h, int M, int T, int ntx, double *qq) {
  const double qn = static_cast<double>(q[n]);
  *qq = qn * qn;
  return tile_of(x[3 * n + 0], x[3 * n + 1], x[3 * n + 2], h, M, T, ntx);
}

// Sum of a per-thread double over a work-group of NTHR threads, written by
// thread 0.
template <int NTHR = kThreads>
__device__ inline void block_sum_to(double v, double *out) {
  v = wave_reduce0(v, [](double a, double b) { return a + b; });
  __shared__ double red[NTHR / 64];
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < NTHR / 64; ++w) s += red[w];
    *out = s;
  }
}

// NTHR threads per work-group, PPT particles per thread: the work-group's
// NTHR PPT particles are ranked per tile in LDS, then each touched tile's
// count is added to its global counter once.  Device-scope atomics are the
// cost (about 20 per ns over the chip), so where tiles hold many particles
// the work-groups are large (1024 threads x 8: a quarter of the atomics of
// 256 x 8 with the same loads in flight).
template <typename R, int PPT, int NTHR>
__global__ void __launch_bounds__(NTHR)
k_bin_count_lds(int N, const R *__restrict__ x, const R *__restrict__ q, double h, int M,
                int T, int ntx, int ntiles, int *__restrict__ counts, int2 *__restrict__ key,
                double *__restrict__ qsq_part) {
  extern __shared__ int lds_tiles[];
  int *lcnt = lds_tiles, *lbase = lds_tiles + ntiles;
  const int tid = threadIdx.x;
  const int n0 = blockIdx.x * (NTHR * PPT);
  for (int t = tid; t < ntiles; t += NTHR) lcnt[t] = 0;
  // all PPT particles are read before the first is used (the index is
  // clamped into [0, N), N >= 1, so the loads need no branch)
  R px[PPT][3], pq[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int nc = min(n0 + k * NTHR + tid, N - 1);  // consecutive threads, consecutive particles
    px[k][0] = x[3 * nc + 0];
    px[k][1] = x[3 * nc + 1];
    px[k][2] = x[3 * nc + 2];
    pq[k] = q[nc];
  }
  int tile[PPT], rank[PPT];
  double qq = 0.0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int n = n0 + k * NTHR + tid;
    tile[k] = -1;
    rank[k] = 0;
    if (n < N) {
      tile[k] = tile_of(px[k][0], px[k][1], px[k][2], h, M, T, ntx);
      qq += static_cast<double>(pq[k]) * static_cast<double>(pq[k]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PPT; ++k)
    if (tile[k] >= 0) rank[k] = atomicAdd(&lcnt[tile[k]], 1);
  __syncthreads();
  // one global atomic per touched tile; a thread issues a batch of them
  // before it needs any of the returned bases
  constexpr int kAtomicBatch = 8;
  for (int t0 = tid; t0 < ntiles; t0 += NTHR * kAtomicBatch) {
    int c[kAtomicBatch], b[kAtomicBatch];
#pragma unroll
    for (int k = 0; k < kAtomicBatch; ++k) {
      const int t = t0 + k * NTHR;
      c[k] = t < ntiles ? lcnt[t] : 0;
    }
#pragma unroll
    for (int k = 0; k < kAtomicBatch; ++k)
      b[k] = c[k] > 0 ? atomicAdd(&counts[(t0 + k * NTHR) * kCountStride], c[k]) : 0;
#pragma unroll
    for (int k = 0; k < kAtomicBatch; ++k) {
      const int t = t0 + k * NTHR;
      if (t < ntiles) lbase[t] = b[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int n = n0 + k * NTHR + tid;
    if (tile[k] >= 0) key[n] = make_int2(tile[k], lbase[tile[k]] + rank[k]);
  }
  block_sum_to<NTHR>(qq, &qsq_part[blockIdx.x]);
}

template <typename R>
__global__ void __launch_bounds__(kThreads)
k_bin_count_run(int N, const R *__restrict__ x, const R *__restrict__ q, double h, int M, int T,
                int ntx, int *__restrict__ counts, int2 *__restrict__ key,
                double *__restrict__ qsq_part) {
  const int tid = threadIdx.x;
  const int n = blockIdx.x * kThreads + tid;
  double qq = 0.0;
  int tile = -1;
  if (n < N) tile = particle_tile(x, q, n, h, M, T, ntx, &qq);
  // one atomic per run of equal tiles among neighbouring lanes
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
  block_sum_to(qq, &qsq_part[blockIdx.x]);
}

// One work-group: exclusive scan of the tile counts into offsets, and the
// counts reset for the next call.  Each thread takes a contiguous chunk of
// tiles and requests all its counts before using any; the chunk sums are
// scanned within each wave by DPP row moves and across the waves through LDS
// (one barrier).
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 32;  // counts per thread held in registers
__global__ void __launch_bounds__(kScanThreads)
k_bin_scan(int *__restrict__ counts, int *__restrict__ offsets, int ntiles) {
  const int tid = threadIdx.x;
  const int chunk = (ntiles + kScanThreads - 1) / kScanThreads;
  const int lo = min(tid * chunk, ntiles), hi = min(lo + chunk, ntiles);
  int v[kScanPer];
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) v[k] = (lo + k < hi) ? counts[(lo + k) * kCountStride] : 0;
  int local = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) local += v[k];
  // more than 32K tiles: the rest in blocks of kScanPer loads issued together
  for (int t0 = lo + kScanPer; t0 < hi; t0 += kScanPer) {
    int w[kScanPer];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) w[k] = (t0 + k < hi) ? counts[(t0 + k) * kCountStride] : 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) local += w[k];
  }
  const int lane = tid & 63, wave = tid >> 6;
  const int incl = wave_inclusive_scan(local);  // over the lanes of the wave
  __shared__ int wsum[kScanThreads / 64];
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wave; ++w) base += wsum[w];
  int run = base + incl - local;
  const auto emit = [&](int t, int c) {
    offsets[t] = run;
    run += c;
    counts[t * kCountStride] = 0;
  };
#pragma unroll
  for (int k = 0; k < kScanPer; ++k)
    if (lo + k < hi) emit(lo + k, v[k]);
  for (int t0 = lo + kScanPer; t0 < hi; t0 += kScanPer) {
    int w[kScanPer];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) w[k] = (t0 + k < hi) ? counts[(t0 + k) * kCountStride] : 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k)
      if (t0 + k < hi) emit(t0 + k, w[k]);
  }
  if (tid == kScanThreads - 1) offsets[ntiles] = base + incl;
}

// Two-level exclusive scan of the cell counts for many cells (k_bin_scan is
// one work-group): k_bin_scan_sums writes the sum of each chunk of
// kScanChunk counts; k_bin_scan_apply then scans each chunk on its own
// work-group, starting from the sum of the chunk sums before it, writes the
// offsets and resets the counts.  Counts are requested kScanChunk/kThreads
// per thread before any is used.
constexpr int kScanPerThread = kScanChunk / kThreads;
static_assert(kScanChunk % kThreads == 0, "whole chunks per work-group");

__device__ inline int block_sum_int(int v, int *red) {
  v = wave_reduce0(v, [](int a, int b) { return a + b; });
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  int s = 0;
  for (int w = 0; w < kThreads / 64; ++w) s += red[w];
  return s;
}

__global__ void __launch_bounds__(kThreads)
k_bin_scan_sums(const int *__restrict__ counts, int ncells, int *__restrict__ sums) {
  __shared__ int red[kThreads / 64];
  const int lo = blockIdx.x * kScanChunk + threadIdx.x * kScanPerThread;
  int v = 0;
#pragma unroll
  for (int k = 0; k < kScanPerThread; ++k)
    v += lo + k < ncells ? counts[(lo + k) * kCountStride] : 0;
  const int s = block_sum_int(v, red);
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads)
k_bin_scan_apply(int *__restrict__ counts, int *__restrict__ offsets, int ncells,
                 const int *__restrict__ sums) {
  __shared__ int red[kThreads / 64];
  __shared__ int wsum[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lo = blockIdx.x * kScanChunk + tid * kScanPerThread;
  int v[kScanPerThread];
#pragma unroll
  for (int k = 0; k < kScanPerThread; ++k) v[k] = lo + k < ncells ? counts[(lo + k) * kCountStride] : 0;
  int before = 0;  // the chunk sums of the work-groups before this one
  for (int b = tid; b < static_cast<int>(blockIdx.x); b += kThreads) before += sums[b];
  const int base = block_sum_int(before, red);
  int local = 0;
#pragma unroll
  for (int k = 0; k < kScanPerThread; ++k) local += v[k];
  const int incl = wave_inclusive_scan(local);  // over the lanes of the wave
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int run = base + incl - local;
  for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
  for (int k = 0; k < kScanPerThread; ++k)
    if (lo + k < ncells) {
      offsets[lo + k] = run;
      run += v[k];
      counts[(lo + k) * kCountStride] = 0;
    }
  if (lo < ncells && lo + kScanPerThread >= ncells) offsets[ncells] = run;  // the last cell's thread
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

// k_bin_scatter with the scan folded in: every work-group scans the tile
// counts into LDS itself (a chunk of counts per thread, DPP prefix sums
// within the waves, one barrier across them), work-group 0 also publishes
// the offsets, and the counts are left for the consumer of the tiles to
// reset.  Saves the
// one-work-group scan launch between counting and scattering.
template <typename R>
__global__ void __launch_bounds__(kThreads)
k_bin_scatter_scan(int N, const R *__restrict__ x, const R *__restrict__ q, double h, int M,
                   int T, const int2 *__restrict__ key, const int *__restrict__ counts,
                   int ntiles, int *__restrict__ offsets, SortedParticle<R> *__restrict__ sorted,
                   int2 *__restrict__ meta) {
  extern __shared__ int soff[];  // ntiles + 1 offsets
  const int tid = threadIdx.x;
  const int n = blockIdx.x * blockDim.x + tid;
  // the particle's inputs are requested before the scan
  int2 kk = make_int2(0, 0);
  R px = R(0), py = R(0), pz = R(0), pq = R(0);
  if (n < N) {
    kk = key[n];
    px = x[3 * n + 0];
    py = x[3 * n + 1];
    pz = x[3 * n + 2];
    pq = q[n];
  }
  const int chunk = (ntiles + kThreads - 1) / kThreads;
  const int lo = min(tid * chunk, ntiles), hi = min(lo + chunk, ntiles);
  constexpr int kPer = 32;  // counts per thread held in registers (ntiles <= 8192)
  int v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) v[k] = (lo + k < hi) ? counts[(lo + k) * kCountStride] : 0;
  int local = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) local += v[k];
  const int lane = tid & 63, wave = tid >> 6;
  const int incl = wave_inclusive_scan(local);  // over the lanes of the wave
  __shared__ int wsum[kThreads / 64];
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int run = incl - local;
  for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
  for (int k = 0; k < kPer; ++k)
    if (lo + k < hi) {
      soff[lo + k] = run;
      if (blockIdx.x == 0) offsets[lo + k] = run;
      run += v[k];
    }
  if (tid == kThreads - 1) {
    soff[ntiles] = run;
    if (blockIdx.x == 0) offsets[ntiles] = run;
  }
  __syncthreads();
  if (n >= N) return;
  const int dst = soff[kk.x] + kk.y;
  double fx, fy, fz;
  const int ax = static_cast<int>(floor_div_mod(static_cast<double>(px) / h, M, &fx));
  const int ay = static_cast<int>(floor_div_mod(static_cast<double>(py) / h, M, &fy));
  const int az = static_cast<int>(floor_div_mod(static_cast<double>(pz) / h, M, &fz));
  SortedParticle<R> sp;
  sp.dx = static_cast<R>(fx);
  sp.dy = static_cast<R>(fy);
  sp.dz = static_cast<R>(fz);
  sp.q = pq;
  sorted[dst] = sp;
  meta[dst] = make_int2((ax % T) | ((ay % T) << 8) | ((az % T) << 16), n);
}

template <typename R>
hipError_t bin_impl(const BinJob &j, se_plan *timing) {
  const R *xr = static_cast<const R *>(j.x), *qr = static_cast<const R *>(j.q);
  const int N = j.N;
  const int blocks1 = N > 0 ? (N + kThreads - 1) / kThreads : 0;
  hipError_t e = hipSuccess;
  if (timing) stage_begin(*timing, SE_STAGE_BIN_COUNT);
  int parts = 0;
  if (N > 0) {
    if (j.ncells <= kLdsTilesMax) {
      const size_t lds = sizeof(int) * 2 * static_cast<size_t>(j.ncells);
      if (static_cast<long long>(N) >= 256LL * j.ncells) {
        constexpr int PPT = 8, NTHR = 1024;
        parts = (N + NTHR * PPT - 1) / (NTHR * PPT);
        launch_on(timing, k_bin_count_lds<R, PPT, NTHR>, parts, NTHR, lds, j.stream, N, xr, qr,
                  j.h, j.M, j.T, j.ntx, j.ncells, j.counts, j.key, j.qsq_part);
      } else {
        parts = blocks1;
        launch_on(timing, k_bin_count_lds<R, 1, kThreads>, parts, kThreads, lds, j.stream, N, xr,
                  qr, j.h, j.M, j.T, j.ntx, j.ncells, j.counts, j.key, j.qsq_part);
      }
    } else {
      parts = blocks1;
      launch_on(timing, k_bin_count_run<R>, parts, kThreads, 0, j.stream, 
          N, xr, qr, j.h, j.M, j.T, j.ntx, j.counts, j.key, j.qsq_part);
    }
    e = hipGetLastError();
  }
  if (j.qsq_parts) *j.qsq_parts = parts;
  if (timing) stage_end(*timing, SE_STAGE_BIN_COUNT);
  if (e != hipSuccess) return e;
  // every scatter work-group reads all the (line-spaced) counts: worth it
  // while that stays small against the separate scan's launch
  const long long scan_reads = static_cast<long long>(j.ncells) * max(blocks1, 1);
  if (j.fused_scan && j.ncells <= kLdsTilesMax && scan_reads <= (1LL << 20)) {
    // the consumer of the tiles resets the counts
    if (timing) stage_begin(*timing, SE_STAGE_BIN_SCATTER);
    launch_on(timing, k_bin_scatter_scan<R>, max(blocks1, 1), kThreads, sizeof(int) * (j.ncells + 1), j.stream, 
        N, xr, qr, j.h, j.M, j.T, j.key, j.counts, j.ncells, j.offsets,
        static_cast<SortedParticle<R> *>(j.sorted), j.meta);
    if (timing) stage_end(*timing, SE_STAGE_BIN_SCATTER);
    return hipGetLastError();
  }
  if (timing) stage_begin(*timing, SE_STAGE_BIN_SCAN);
  if (j.ncells <= kScanOneGroupMax) {
    launch_on(timing, k_bin_scan, 1, kScanThreads, 0, j.stream, j.counts, j.offsets, j.ncells);
  } else {
    const int chunks = scan_chunks(j.ncells);
    int *sums = j.offsets + j.ncells + 1;
    launch_on(timing, k_bin_scan_sums, chunks, kThreads, 0, j.stream, j.counts, j.ncells, sums);
    launch_on(timing, k_bin_scan_apply, chunks, kThreads, 0, j.stream, j.counts, j.offsets,
              j.ncells, sums);
  }
  if (timing) stage_end(*timing, SE_STAGE_BIN_SCAN);
  if ((e = hipGetLastError()) != hipSuccess || N == 0) return e;
  if (timing) stage_begin(*timing, SE_STAGE_BIN_SCATTER);
  launch_on(timing, k_bin_scatter<R>, blocks1, kThreads, 0, j.stream, 
      N, xr, qr, j.h, j.M, j.T, j.key, j.offsets, static_cast<SortedParticle<R> *>(j.sorted),
      j.meta);
  if (timing) stage_end(*timing, SE_STAGE_BIN_SCATTER);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_bin_job(const BinJob &job, se_plan *timing) {
  return job.fp64 ? bin_impl<double>(job, timing) : bin_impl<float>(job, timing);
}

hipError_t launch_bin(se_plan &plan, int N, const void *x, const void *q) {
  BinJob j;
  j.N = N;
  j.x = x;
  j.q = q;
  j.fp64 = plan.prm.dtype == SE_FP64;
  j.h = plan.h;
  j.M = plan.prm.M;
  j.T = plan.T;
  j.ntx = plan.ntx;
  j.ncells = plan.ntiles;
  j.counts = plan.buf.counts;
  j.key = plan.buf.key;
  j.offsets = plan.buf.offsets;
  j.sorted = plan.buf.sorted;
  j.meta = plan.buf.meta;
  j.qsq_part = plan.buf.part;
  j.qsq_parts = &plan.bin_parts;
  j.stream = plan.stream;
  j.fused_scan = true;  // the spread resets the tile counts
  return launch_bin_job(j, &plan);
}

}  // namespace sek
