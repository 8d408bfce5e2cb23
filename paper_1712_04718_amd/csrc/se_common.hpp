// Internal declarations shared by the translation units of libsekspace.so.
// Not part of the public ABI (that is include/sekspace.h).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "sekspace.h"

namespace sek {

// ---------------------------------------------------------------- numerics

template <typename R> struct Cplx;
template <> struct Cplx<float> { using T = float2; };
template <> struct Cplx<double> { using T = double2; };
template <typename R> using cplx_t = typename Cplx<R>::T;

// A particle after sorting: offsets (grid units, in [0,1)) of the particle
// from its anchor grid point floor(x/h), and its charge.
template <typename R> struct alignas(4 * sizeof(R)) SortedParticle {
  R dx, dy, dz, q;
};

// ----------------------------------------------------------------- the plan

constexpr int kMaxRadixStages = 16;

// Division by a runtime constant d <= 1024 of a numerator n with
// n * (magic * d - 2^32) < 2^32 (true for every index below): the high half
// of n * magic, magic = ceil(2^32 / d).
__host__ __device__ inline unsigned div_magic(unsigned d) {
  return d <= 1 ? 0u : static_cast<unsigned>(((1ull << 32) + d - 1) / d);
}
__device__ inline int fast_div(int n, unsigned magic) {
  return static_cast<int>(__umulhi(static_cast<unsigned>(n), magic));
}

// Work-groups are dealt to the 8 XCDs round-robin (work-group b runs on XCD
// b mod 8), and each XCD has its own L2.  Renumbering b so that every XCD
// gets a contiguous range of work items keeps neighbouring tiles and
// pencils, which share cache lines and halo data, in one L2.  Bijective on
// [0, G): the first 8 floor(G/8) work-groups are permuted, the rest keep
// their number.
constexpr int kXcds = 8;
__device__ inline int xcd_local(int b, int G) {
  const int q = G / kXcds;
  return b < q * kXcds ? (b % kXcds) * q + b / kXcds : b;
}

// The value v of the lane that the DPP control CTRL selects (a row move
// stays within the lane's row of 16 lanes, a wave shift moves by one lane),
// 0 where that lane does not exist.
template <int CTRL> __device__ inline int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true);
}
template <int CTRL> __device__ inline float dpp_move(float v) {
  return __int_as_float(dpp_move<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ inline double dpp_move(double v) {
  return __hiloint2double(dpp_move<CTRL>(__double2hiint(v)), dpp_move<CTRL>(__double2loint(v)));
}
template <int CTRL> __device__ inline long long dpp_move(long long v) {
  const int lo = dpp_move<CTRL>(static_cast<int>(v & 0xffffffffLL));
  const int hi = dpp_move<CTRL>(static_cast<int>(v >> 32));
  return (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo);
}
// v of lane L (a wave-uniform value)
template <int L> __device__ inline int read_lane(int v) { return __builtin_amdgcn_readlane(v, L); }
template <int L> __device__ inline double read_lane(double v) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), L),
                          __builtin_amdgcn_readlane(__double2loint(v), L));
}
template <int L> __device__ inline long long read_lane(long long v) {
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(v & 0xffffffffLL), L);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(v >> 32), L);
  return (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo);
}
// v combined by op (associative and commutative, with 0 as a neutral value
// for the lanes' values: a sum, or a maximum of non-negative values) over
// the 64 lanes of the wave, valid in lane 0: DPP row moves reduce each row
// of 16 lanes into its first lane, which lane 0 then reads.  Every lane of
// the wave must be active.
template <typename T, typename Op> __device__ inline T wave_reduce0(T v, Op op) {
  v = op(v, dpp_move<0x108>(v));  // row_shl:8, lane i + 8
  v = op(v, dpp_move<0x104>(v));  // row_shl:4, lane i + 4
  v = op(v, dpp_move<0x4e>(v));   // quad_perm [2,3,0,1], lane i ^ 2
  v = op(v, dpp_move<0xb1>(v));   // quad_perm [1,0,3,2], lane i ^ 1
  return op(op(v, read_lane<16>(v)), op(read_lane<32>(v), read_lane<48>(v)));
}

// Inclusive prefix sum of v over the 64 lanes of the wave (exact integer
// arithmetic, so its order does not matter): DPP row shifts by 1, 2, 4, 8
// scan each row of 16 lanes, then each row adds the totals of the rows
// before it, read from their last lanes.  Every lane of the wave must be
// active.
__device__ inline int wave_inclusive_scan(int v) {
  v += dpp_move<0x111>(v);  // row_shr:1, lane i - 1
  v += dpp_move<0x112>(v);  // row_shr:2
  v += dpp_move<0x114>(v);  // row_shr:4
  v += dpp_move<0x118>(v);  // row_shr:8
  const int lane = static_cast<int>(threadIdx.x) & 63;
  const int r0 = read_lane<15>(v), r1 = read_lane<31>(v), r2 = read_lane<47>(v);
  return v + (lane >= 16 ? r0 : 0) + (lane >= 32 ? r1 : 0) + (lane >= 48 ? r2 : 0);
}

// Anchor of a coordinate u in grid units: floor(u) reduced mod M into
// [0, M), and the offset u - floor(u).  A non-finite u (or one beyond the
// integer range) takes anchor 0 while its offset stays NaN, so the outputs
// show the bad input and no index derived from it leaves the grid.
__device__ inline int anchor_mod(double u, int M, double *frac) {
  double fl = floor(u);
  *frac = u - fl;
  if (!(fabs(fl) < 4.0e18)) {
    fl = 0.0;
    *frac = __builtin_nan("");
  }
  const long long i = static_cast<long long>(fl) % M;
  return static_cast<int>(i < 0 ? i + M : i);
}

// v mod M for v in [-M, 3M), branch-free.  Every grid index of a staged tile
// block lies in [-(S-1), M + T + S - 3], inside that range whenever S <= M and
// T + S - 3 < 2M (the plan checks both).
__device__ inline int wrap_near(int v, int M) {
  v = v < 0 ? v + M : v;
  v = v >= M ? v - M : v;
  return v >= M ? v - M : v;
}

struct FftPlan {
  int M;                        // transform length
  int nstages;                  // number of radix stages
  int radix[kMaxRadixStages];   // radices in stage order (2, 3, 4, 5, 8)
  int ns[kMaxRadixStages];      // product of the radices of the earlier stages
  unsigned ns_magic[kMaxRadixStages];  // div_magic(ns[s])
  int tstep[kMaxRadixStages];   // M / (ns[s] * radix[s]): twiddle index step
  unsigned m_magic;             // div_magic(M)
};

// Which tile blocks of the ghost array cover each grid index along one axis
// (the same along all three axes of the cubic grid).
struct FoldTables {
  const int *cover;  // [M][KC]: tile * 64 + index inside the tile block
  const int *count;  // [M]: entries used in cover[g]
  int KC;            // entries per grid index
  int TS;            // tile block edge T + S - 1
  int ntx;           // tiles per axis
};

// Event pairs around the launches of one stage (plans with SE_FLAG_TIMING).
// A ring of kTimingSlots pairs: when it is full, the oldest pair is waited for
// and its duration added to sum_ms before the pair is reused, so every launch
// is counted while up to kTimingSlots launches stay in flight.
constexpr int kTimingSlots = 16;
struct StageTimer {
  hipEvent_t begin[kTimingSlots] = {};
  hipEvent_t end[kTimingSlots] = {};
  long long issued = 0;     // launches recorded
  long long harvested = 0;  // launches whose duration is in sum_ms
  double sum_ms = 0.0;      // durations harvested since the last read
  long long count = 0;      // launches in sum_ms
};

// Wait for the oldest unharvested launch of a stage and add its duration.
inline hipError_t harvest_oldest(StageTimer &t) {
  const int slot = static_cast<int>(t.harvested % kTimingSlots);
  hipError_t e = hipEventSynchronize(t.end[slot]);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.begin[slot], t.end[slot]);
  ++t.harvested;
  if (e == hipSuccess) {
    t.sum_ms += ms;
    ++t.count;
  }
  return e;
}

// Binning workspace for evaluation points that are not sources
// (se_eval_targets): cap points, sorted into the plan's tiles.
struct TargetBuffers {
  int cap = 0;
  int *counts = nullptr;   // ntiles counters, kCountStride ints apart
  int *offsets = nullptr;  // ntiles + 1
  int2 *key = nullptr;     // cap
  int2 *meta = nullptr;    // cap
  void *sorted = nullptr;  // cap SortedParticle<R>
  double *part = nullptr;  // binning partials (unused)
  void *ones = nullptr;    // cap unit charges
};

struct DeviceBuffers {
  void *grid = nullptr;       // M^3 real: the scaled grid Phi (input of gathering)
  void *ghost = nullptr;      // ntiles * ghost_stride(T+S-1) real: spread tile blocks
  int *cover = nullptr;       // fold tables (FoldTables)
  int *cover_count = nullptr;
  void *spec = nullptr;       // M*M*(M/2+1) complex half spectrum
  void *spec2 = nullptr;      // SE_FLAG_IK_FORCE: half spectrum of one field component
  void *field = nullptr;      // SE_FLAG_IK_FORCE: 3 M^3 real, the field grids -dPhi/dx_d
  void *sorted = nullptr;     // n_max SortedParticle<R>
  int2 *meta = nullptr;       // n_max (packed local anchor, original index)
  int2 *key = nullptr;        // n_max (tile, rank within tile)
  int *counts = nullptr;      // ntiles counters, kCountStride ints apart (own cache line)
  int *offsets = nullptr;     // ntiles + 1: first sorted index of each tile, then N
  double *part = nullptr;     // per-block partial sums: bin_blocks of q^2, then energy
  void *twiddle = nullptr;    // M complex: e^{-2 pi i j / M}
  void *axis_f = nullptr;     // M real: per-axis factor of the influence function
  void *axis_k2 = nullptr;    // M real: k_n^2 per axis
  size_t bytes = 0;
};

}  // namespace sek

struct se_plan {
  se_params prm;
  int n_max;
  hipStream_t stream;
  int device;

  // derived parameters (section 4, eq. 5.2)
  double h;        // grid spacing L/M
  double eta;      // Gaussian shape (0 for B-splines)
  double a;        // 2 xi^2 / eta: Gaussian exponent in physical units
  double cg;       // a h^2: Gaussian exponent in grid units
  double beta;     // h sqrt(a/pi): per-axis window normalisation
  double wscale;   // 4 pi / L^3

  // tiling of the grid for spreading and gathering
  int T;           // tile edge (grid points)
  int ntx;         // tiles per axis, ceil(M/T)
  int ntiles;      // ntx^3
  int bin_blocks;  // blocks of the binning kernel for n_max
  int bin_parts;   // q^2 partials written by the last binning (its block count)
  int zfft_blocks; // blocks of the z-pass (energy partials)
  int fft_lgb[3];  // log2 pencils per FFT work-group of the x, y and z passes
  int fft_threads; // threads per FFT work-group

  sek::FftPlan fft;
  sek::DeviceBuffers buf;  // pieces of one workspace (owned, or the caller's)
  void *owned = nullptr;   // the workspace the plan allocated itself, if any
  bool touched = false;    // device work or memory exists (destroy synchronises)
  sek::TargetBuffers tgt;
  sek::FoldTables fold;
  bool fold_by_tiles;  // tiles partition the grid: tile-structured fold
  bool direct;         // FP64 Gaussian with P > 16: untiled spread and gather (direct.hip)

  int last_N;      // particles of the last se_forward, -1 before the first

  // optional per-kernel timing (SE_FLAG_TIMING)
  bool timing;
  sek::StageTimer timers[SE_NUM_STAGES];
  int armed_stage = -1;      // stage whose event pair the next launches carry
  bool armed_first = false;  // no launch has carried it yet
};

namespace sek {

// Binning of N particles into cells of a regular grid: cell edge T points
// of spacing h on an M^3 grid with ntx cells per axis (the k-space tiles, or
// T = 1 for the real-space cell list).  Produces per-cell offsets (ncells +
// 1), particles in cell order (offsets from their grid point in units of h,
// and q) and (packed local grid point, original index); counts must be zero
// on entry and are left zero.
struct BinJob {
  int N = 0;
  const void *x = nullptr, *q = nullptr;
  bool fp64 = false;
  double h = 0.0;
  int M = 0, T = 1, ntx = 0, ncells = 0;
  int *counts = nullptr;
  int2 *key = nullptr;
  int *offsets = nullptr;
  void *sorted = nullptr;
  int2 *meta = nullptr;
  double *qsq_part = nullptr;  // per-block q^2 sums (at least ceil(N/256) entries)
  int *qsq_parts = nullptr;    // out: number of partials written
  hipStream_t stream = nullptr;
  // scan inside the scatter kernel (up to 8192 tiles); the counts are then
  // left for the consumer of the tiles to reset before the next binning
  bool fused_scan = false;
};
hipError_t launch_bin_job(const BinJob &job, se_plan *timing);

// Record msg as the calling thread's last error (se_last_error) and return s.
se_status report(se_status s, const char *msg);

// Launch wrappers (one per translation unit); each enqueues on plan.stream
// and returns the launch status.
hipError_t launch_bin(se_plan &plan, int N, const void *x, const void *q);
hipError_t launch_spread(se_plan &plan);
// Untiled path (FP64 Gaussian, P = 18..24): anchors and offsets in input
// order (with q^2 block sums), spread with FP64 atomics, gather per wave.
hipError_t launch_direct_prep(se_plan &p, int N, const void *x, const void *q, void *pts,
                              int2 *meta, double *qsq_part, int *parts);
hipError_t launch_direct_forward(se_plan &p, int N, const void *x, const void *q);
hipError_t launch_direct_gather(se_plan &p, int N, const double *gscale, int mode, void *pot,
                                void *vec);
hipError_t launch_fft_forward_scale_inverse(se_plan &plan, double *E_dev);
hipError_t launch_gather(se_plan &plan, int N, const double *gscale, int mode,
                         void *out_pot, void *out_vec);

// Per-stage timing of plans with SE_FLAG_TIMING.  stage_begin arms the
// stage's next event pair; every launch_on inside the stage carries the pair
// (hipExtLaunchKernelGGL timestamps exactly that dispatch, as a profiler's
// kernel trace does): the first launch sets the start, each launch the stop,
// so a stage of several launches spans them all; stage_end counts the pair
// if a launch used it.
inline void stage_begin(se_plan &p, int stage) {
  if (!p.timing) return;
  StageTimer &t = p.timers[stage];
  if (t.issued - t.harvested == kTimingSlots) (void)harvest_oldest(t);
  p.armed_stage = stage;
  p.armed_first = true;
}
inline void stage_end(se_plan &p, int stage) {
  if (!p.timing) return;
  if (p.armed_stage == stage && !p.armed_first) ++p.timers[stage].issued;
  p.armed_stage = -1;
}

// Launch a kernel (<<<grid, block, lds, stream>>>), with the armed stage's
// event pair when tp is a timing plan inside stage_begin/stage_end.
template <typename... KArgs, typename... Args>
inline void launch_on(se_plan *tp, void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t lds,
                      hipStream_t stream, Args... args) {
  if (tp && tp->timing && tp->armed_stage >= 0) {
    StageTimer &t = tp->timers[tp->armed_stage];
    const int slot = static_cast<int>(t.issued % kTimingSlots);
    hipExtLaunchKernelGGL(kernel, grid, block, static_cast<std::uint32_t>(lds), stream,
                          tp->armed_first ? t.begin[slot] : nullptr, t.end[slot], 0u,
                          static_cast<KArgs>(args)...);
    tp->armed_first = false;
  } else {
    kernel<<<grid, block, lds, stream>>>(static_cast<KArgs>(args)...);
  }
}

// LDS bytes a spreading / gathering work-group needs (tile edge T, support S).
size_t spread_lds_bytes(int real_size, int window, int S, int T);
size_t gather_lds_bytes(int real_size, int window, int S, int T);
constexpr size_t kMaxLds = 160 * 1024;

// Values per tile block in the ghost array: the (T+S-1)^3 block rounded up
// to a multiple of four, so that every block starts on 16 bytes and the
// spread stores it 16 bytes per lane.
__host__ __device__ constexpr int ghost_stride(int TS) { return (TS * TS * TS + 3) & ~3; }

// gather modes
constexpr int kGatherPotentialForce = 0;  // out_pot = phi, out_vec = F
constexpr int kGatherAdjoint = 1;         // out_pot = gE phi, out_vec = -gE F
constexpr int kGatherTargets = 2;         // points of plan.tgt: phi (no self term), -grad phi
constexpr int kGatherIkX = 3;             // +d (d = 0, 1, 2): out_vec[3 n + d] = scale q * (field d at n)

constexpr int kMaxSplineOrder = 8;  // largest SPME order built
constexpr int kThreads = 256;      // work-group size of the binning, fold and FFT kernels (the
                                   // five-pass FFT at M >= 384 widens some passes to 512)
constexpr int kTileThreads = 512;  // work-group size of the tile spread kernel (the gather's
                                   // depends on the precision)

// Most pencils per FFT work-group, per pass.  Lanes run over the B pencils
// fastest, so a wave reads 64 / B consecutive elements of each pencil: the
// y pencils are contiguous and B = 4 gives whole 128-byte lines with many
// work-groups in flight.  x rows take B = 4 as well (at M = 192 the FP32 x
// pass took 13.4 instead of 15.9 us, at M = 432 164 instead of 220 us, the
// inverse x pass 212 instead of 308 us); FP32 z columns take B = 8 (22.5
// against 24.6 us at M = 192), FP64 ones B = 4 (33.6 against 41.6 us, the
// LDS per work-group halved).  (Measured with two pencil buffers; with the
// one buffer of the compiled sizes, 16 FP32 z columns were slower again.)
enum FftPass { kPassX = 0, kPassY = 1, kPassZ = 2 };
constexpr int fft_batch_cap(int pass, int real_size) {
  return pass == kPassZ && real_size == 4 ? 8 : 4;
}

// Grid sizes whose FFT kernels are compiled for their M (the others run
// the run-time plan's kernels).
constexpr int kCompiledM[] = {16,  24,  32,  40,  48,  64,  80,  96,  120, 128, 144,
                              160, 192, 216, 240, 256, 288, 320, 384, 432, 480, 512};
constexpr bool fft_compiled(int M) {
  for (int m : kCompiledM)
    if (m == M) return true;
  return false;
}

// Pencils per FFT work-group of one pass, as log2: B a power of two, at most
// fft_batch_cap(pass, real_size), with M * B <= 16 * kThreads (elements per thread when
// loading) and the LDS buffers of M x B complex (one for the compiled
// kernels, whose radix stages run in place; two for the run-time plan's,
// which ping-pong) plus the M twiddles (and, in the z pass, the two FP64
// axis tables of the influence function) within 64 KB.
constexpr int fft_lgb(int M, int real_size, int pass) {
  const int tables = pass == kPassZ ? 2 * 8 * M : 0;
  const int nbuf = fft_compiled(M) ? 1 : 2;
  int B = fft_batch_cap(pass, real_size);
  while (B > 1 &&
         (M * B > 16 * kThreads || (nbuf * M * B + M) * 2 * real_size + tables > 65536))
    B >>= 1;
  int lg = 0;
  while ((1 << lg) < B) ++lg;
  return lg;
}

// Tile counters are spaced one cache line apart: device-wide atomics on the
// same line serialise, on different lines they proceed in parallel.
constexpr int kCountStride = 32;

// Cells per work-group of the two-level scan of the cell counts (taken above
// kScanOneGroupMax cells); the offsets array of a binning holds
// ncells + 1 + scan_chunks(ncells) ints, the chunk sums after the offsets.
constexpr int kScanChunk = 2048;
constexpr int kScanOneGroupMax = 2048;
constexpr int scan_chunks(int ncells) { return (ncells + kScanChunk - 1) / kScanChunk; }

}  // namespace sek
