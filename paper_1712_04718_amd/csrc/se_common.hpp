// Internal declarations shared by the translation units of libsekspace.so.
// Not part of the public ABI (that is include/sekspace.h).
#pragma once

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

struct FftPlan {
  int M;                        // transform length
  int nstages;                  // number of radix stages
  int radix[kMaxRadixStages];   // radices in stage order (2, 3, 4, 5, 8)
};

struct DeviceBuffers {
  void *grid = nullptr;       // M^3 real: spread grid G, later the scaled grid Phi
  void *spec = nullptr;       // M*M*(M/2+1) complex half spectrum
  void *sorted = nullptr;     // n_max SortedParticle<R>
  int2 *meta = nullptr;       // n_max (packed local anchor, original index)
  int2 *key = nullptr;        // n_max (tile, rank within tile)
  int *counts = nullptr;      // ntiles
  int *offsets = nullptr;     // ntiles + 1
  unsigned *done = nullptr;   // 2 arrival counters (binning, energy)
  double *part = nullptr;     // per-block partial sums (q^2 and energy)
  double *qsq = nullptr;      // sum q^2 of the last forward
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
  int zfft_blocks; // blocks of the z-pass (energy partials)
  int fft_batch;   // pencils per FFT work-group

  sek::FftPlan fft;
  sek::DeviceBuffers buf;

  int last_N;      // particles of the last se_forward, -1 before the first

  // optional per-kernel timing (SE_FLAG_TIMING)
  bool timing;
  hipEvent_t ev_begin[SE_NUM_STAGES];
  hipEvent_t ev_end[SE_NUM_STAGES];
  bool ev_used[SE_NUM_STAGES];
};

namespace sek {

// Launch wrappers (one per translation unit); each enqueues on plan.stream
// and returns the launch status.
hipError_t launch_bin(se_plan &plan, int N, const void *x, const void *q);
hipError_t launch_spread(se_plan &plan, int N);
hipError_t launch_fft_forward_scale_inverse(se_plan &plan, double *E_dev);
hipError_t launch_gather(se_plan &plan, int N, const double *gscale, int mode,
                         void *out_pot, void *out_vec);

// Event pair around one kernel launch when the plan records timings.
inline void stage_begin(se_plan &p, int stage) {
  if (p.timing) (void)hipEventRecord(p.ev_begin[stage], p.stream);
}
inline void stage_end(se_plan &p, int stage) {
  if (p.timing) {
    (void)hipEventRecord(p.ev_end[stage], p.stream);
    p.ev_used[stage] = true;
  }
}

// LDS bytes a spreading / gathering work-group needs (tile edge T, support S).
size_t spread_lds_bytes(int real_size, int S, int T);
size_t gather_lds_bytes(int real_size, int window, int S, int T);
constexpr size_t kMaxLds = 160 * 1024;

// gather modes
constexpr int kGatherPotentialForce = 0;  // out_pot = phi, out_vec = F
constexpr int kGatherAdjoint = 1;         // out_pot = gE phi, out_vec = -gE F

constexpr int kThreads = 256;  // work-group size of every kernel but the scan

}  // namespace sek
