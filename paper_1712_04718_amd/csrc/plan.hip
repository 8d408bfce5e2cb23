// Host side of the C ABI declared in include/sekspace.h: argument checks,
// derived parameters (section 4, eq. 5.2), influence-function tables
// (eqs. 4.6 and 6.2), FFT radix plan, workspace, and the call sequence.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "se_common.hpp"

namespace {

thread_local std::string g_last_error;

se_status fail(se_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
se_status fail(se_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

se_status hip_fail(hipError_t e, const char *where) {
  return fail(SE_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

bool only_235(int m) {
  for (int f : {2, 3, 5})
    while (m % f == 0) m /= f;
  return m == 1;
}

double shape_c(const se_params &p) { return p.c > 0.0 ? p.c : 0.95; }

// eta of section 4 / eq. (5.2): eta = P L^2 xi^2 / (c^2 pi M^2).
double eta_of(const se_params &p) {
  const double c = shape_c(p);
  return p.P * p.L * p.L * p.xi * p.xi / (c * c * M_PI * p.M * static_cast<double>(p.M));
}

int real_size(const se_params &p) { return p.dtype == SE_FP64 ? 8 : 4; }

// Tile edge for spreading/gathering: the largest of 16, 12, 8 that still
// leaves at least 512 tiles (enough work-groups for 256 CUs) and whose LDS
// blocks fit; larger tiles have fewer halo points per particle.
int choose_tile(const se_params &p) {
  const int rs = real_size(p), S = p.P;
  const auto fits = [&](int T) {
    return sek::spread_lds_bytes(rs, p.window, S, T) <= sek::kMaxLds &&
           sek::gather_lds_bytes(rs, p.window, S, T) <= sek::kMaxLds;
  };
  for (int T : {16, 12}) {
    const long long nt = (p.M + T - 1) / T;
    if (nt * nt * nt >= 512 && fits(T)) return T;
  }
  return fits(8) ? 8 : 0;  // 0: no tile edge fits (the plan is refused)
}


sek::FftPlan radix_plan(int M) {
  sek::FftPlan pl{};
  pl.M = M;
  int m = M, n = 0;
  while (m % 8 == 0) { pl.radix[n++] = 8; m /= 8; }
  if (m % 4 == 0) { pl.radix[n++] = 4; m /= 4; }
  if (m % 2 == 0) { pl.radix[n++] = 2; m /= 2; }
  while (m % 5 == 0) { pl.radix[n++] = 5; m /= 5; }
  while (m % 3 == 0) { pl.radix[n++] = 3; m /= 3; }
  pl.nstages = n;
  int ns = 1;
  for (int s = 0; s < n; ++s) {
    pl.ns[s] = ns;
    pl.ns_magic[s] = sek::div_magic(ns);
    pl.tstep[s] = M / (ns * pl.radix[s]);
    ns *= pl.radix[s];
  }
  pl.m_magic = sek::div_magic(M);
  return pl;
}

se_status check_params(const se_params *prm, double *eta_out) {
  if (!prm) return fail(SE_ERR_ARG, "params is NULL");
  const se_params &p = *prm;
  if (!(p.L > 0.0) || !std::isfinite(p.L)) return fail(SE_ERR_ARG, "L must be finite and > 0 (got %g)", p.L);
  if (!(p.xi > 0.0) || !std::isfinite(p.xi)) return fail(SE_ERR_ARG, "xi must be finite and > 0 (got %g)", p.xi);
  if (!std::isfinite(p.c)) return fail(SE_ERR_ARG, "c must be finite");
  if (p.window != SE_WINDOW_GAUSSIAN && p.window != SE_WINDOW_BSPLINE)
    return fail(SE_ERR_ARG, "unknown window %d", p.window);
  if (p.dtype != SE_FP32 && p.dtype != SE_FP64) return fail(SE_ERR_ARG, "unknown dtype %d", p.dtype);
  if (p.flags & ~(SE_FLAG_ADD_SELF | SE_FLAG_TIMING | SE_FLAG_IK_FORCE | SE_FLAG_CALLER_WORKSPACE))
    return fail(SE_ERR_ARG, "unknown flags 0x%x", p.flags);
  if (p.M < 8 || p.M > 512 || (p.M & 1) || !only_235(p.M))
    return fail(SE_ERR_GRID, "M=%d must be even, 8..512 and of the form 2^a 3^b 5^c", p.M);
  if (p.P > p.M) return fail(SE_ERR_GRID, "support %d exceeds M=%d", p.P, p.M);
  double eta = 0.0;
  if (p.window == SE_WINDOW_GAUSSIAN) {
    const bool wide = p.dtype == SE_FP64 && p.P >= 18 && p.P <= 24;
    if ((p.P & 1) || p.P < 4 || (p.P > 16 && !wide))
      return fail(SE_ERR_UNSUPPORTED,
                  "Gaussian support P=%d: built for even P in 4..16 (FP32) and 4..24 (FP64)", p.P);
    eta = eta_of(p);
    if (!(eta > 0.0 && eta < 1.0))
      return fail(SE_ERR_ETA, "eta = P L^2 xi^2 / (c^2 pi M^2) = %g is outside (0,1)", eta);
  } else {
    if (p.P < 3 || p.P > 8)
      return fail(SE_ERR_UNSUPPORTED, "B-spline order p=%d: built for 3..8", p.P);
  }
  if ((p.flags & SE_FLAG_IK_FORCE) && p.window == SE_WINDOW_GAUSSIAN && p.P > 16)
    return fail(SE_ERR_UNSUPPORTED, "ik forces are built for the tiled supports (P <= 16)");
  if (eta_out) *eta_out = eta;
  return SE_OK;
}

struct Sizes {
  size_t grid, ghost, cover, cover_count, spec, spec2, field, sorted, meta, key, counts, offsets,
      part, tw, f, k2, total;
};

int stencil_offset(const se_params &p) {
  return p.window == SE_WINDOW_GAUSSIAN ? -(p.P / 2 - 1) : -(p.P - 1);
}

// Tile blocks covering grid index g along one axis: block of tile t starts at
// grid index t*T + off and spans TS = T + S - 1 points (periodically wrapped).
// Counted without allocating (the no-allocation entry point sizes its
// scratch with it).
int cover_count_at(int M, int T, int S, int off, int g) {
  const int ntx = (M + T - 1) / T, TS = T + S - 1;
  int n = 0;
  for (int t = 0; t < ntx; ++t)
    for (int l = 0; l < TS; ++l) {
      int v = (t * T + off + l) % M;
      if (v < 0) v += M;
      n += v == g;
    }
  return n;
}

size_t max_cover(const se_params &p, int T) {
  if (T <= 0) return 0;
  int kc = 0;
  for (int g = 0; g < p.M; ++g)
    kc = std::max(kc, cover_count_at(p.M, T, p.P, stencil_offset(p), g));
  return static_cast<size_t>(kc);
}

Sizes sizes_of(const se_params &p, int n_max, int ntiles, int bin_blocks, int zblocks, int T) {
  const size_t rs = real_size(p), M = p.M, K = M / 2 + 1;
  const size_t n = n_max > 0 ? n_max : 1;
  Sizes s{};
  // every buffer gets at least 256 bytes (the untiled path has no tiles) and
  // starts on a 256-byte boundary of the workspace
  auto al = [](size_t b) { return ((b ? b : 1) + 255) & ~static_cast<size_t>(255); };
  const size_t TS = T + p.P - 1;
  s.grid = al(M * M * M * rs);
  s.ghost = al(T > 0 ? static_cast<size_t>(ntiles) * sek::ghost_stride(static_cast<int>(TS)) * rs : 0);
  s.cover = al(T > 0 ? M * max_cover(p, T) * 4 : 0);
  s.cover_count = al(M * 4);
  s.spec = al(M * M * K * 2 * rs);
  const bool ik = (p.flags & SE_FLAG_IK_FORCE) != 0;
  s.spec2 = al(ik ? M * M * K * 2 * rs : 0);
  s.field = al(ik ? 3 * M * M * M * rs : 0);
  s.sorted = al(n * 4 * rs);
  s.meta = al(n * 8);
  s.key = al(n * 8);
  s.counts = al(static_cast<size_t>(ntiles) * sek::kCountStride * 4);
  s.offsets = al((ntiles + 1 + sek::scan_chunks(ntiles)) * 4);
  s.part = al((bin_blocks + zblocks) * 8);
  s.tw = al(M * 2 * rs);
  s.f = al(M * 8);
  s.k2 = al(M * 8);
  s.total = s.grid + s.ghost + s.cover + s.cover_count + s.spec + s.spec2 + s.field + s.sorted +
            s.meta + s.key +
            s.counts + s.offsets + s.part + s.tw + s.f + s.k2;
  return s;
}

// The plan's buffers as consecutive pieces of one workspace (base 256-byte
// aligned), in the order of Sizes.
sek::DeviceBuffers carve(const Sizes &s, void *base) {
  sek::DeviceBuffers b{};
  char *c = static_cast<char *>(base);
  auto take = [&c](size_t n) {
    void *r = c;
    c += n;
    return r;
  };
  b.grid = take(s.grid);
  b.ghost = take(s.ghost);
  b.cover = static_cast<int *>(take(s.cover));
  b.cover_count = static_cast<int *>(take(s.cover_count));
  b.spec = take(s.spec);
  b.spec2 = take(s.spec2);
  b.field = take(s.field);
  b.sorted = take(s.sorted);
  b.meta = static_cast<int2 *>(take(s.meta));
  b.key = static_cast<int2 *>(take(s.key));
  b.counts = static_cast<int *>(take(s.counts));
  b.offsets = static_cast<int *>(take(s.offsets));
  b.part = static_cast<double *>(take(s.part));
  b.twiddle = take(s.tw);
  b.axis_f = take(s.f);
  b.axis_k2 = take(s.k2);
  b.bytes = s.total;
  return b;
}

// Cardinal B-spline M_p at the integers 0..p (section 6.1 recursion from
// M_2(u) = 1 - |u - 1| on [0, 2]): v[u] = M_p(u).
__device__ void bspline_integers(int p, double (&v)[sek::kMaxSplineOrder + 1]) {
  for (int u = 0; u <= sek::kMaxSplineOrder; ++u) v[u] = (u == 1) ? 1.0 : 0.0;
  for (int n = 3; n <= p; ++n)
    for (int u = n; u >= 1; --u)
      v[u] = (u * v[u] + (n - u) * v[u - 1]) / (n - 1);
}

// Tables of a plan, computed on the device (so that a plan and the
// no-allocation entry point hold the same bits), and the tile counters
// cleared:
//   twiddle[j] = e^{-2 pi i j/M};
//   axis_k2[n] = k_n^2, k_n = 2 pi n~/L with n~ = n or n - M (Nyquist |n~| = M/2);
//   axis_f[n] = e^{-(1-eta) k_n^2/4xi^2} (SE, eq. 4.6) or
//               |b(n)|^2 e^{-k_n^2/4xi^2} (SPME, eq. 6.2) with
//               |b(n)|^2 = 1/|sum_{l=0}^{p-2} M_p(l+1) e^{2 pi i n l/M}|^2,
//               0 where the sum vanishes (odd p at n = M/2);
//   cover[g][k], cover_count[g]: the tile blocks covering grid index g
//               along one axis (tile * 64 + index inside the block).
template <typename R>
__global__ void __launch_bounds__(sek::kThreads)
k_plan_tables(int M, double L, double xi, double eta, int bspline, int P, int T, int off,
              int KC, R *__restrict__ twiddle, double *__restrict__ axis_f,
              double *__restrict__ axis_k2, int *__restrict__ cover, int *__restrict__ cover_count,
              int *__restrict__ counts, int ncounts) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncounts; i += stride) counts[i] = 0;
  for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < M; n += stride) {
    const double ang = 2.0 * M_PI * n / M;
    twiddle[2 * n] = static_cast<R>(cos(ang));
    twiddle[2 * n + 1] = static_cast<R>(-sin(ang));
    const int ns = (2 * n <= M) ? n : n - M;
    const double k = 2.0 * M_PI * ns / L;
    const double k2 = k * k;
    axis_k2[n] = k2;
    if (!bspline) {
      axis_f[n] = exp(-(1.0 - eta) * k2 / (4.0 * xi * xi));
    } else {
      double v[sek::kMaxSplineOrder + 1];
      bspline_integers(P, v);
      double re = 0.0, im = 0.0;
      for (int l = 0; l <= P - 2; ++l) {
        const double a = 2.0 * M_PI * static_cast<double>(n) * l / M;
        re += v[l + 1] * cos(a);
        im += v[l + 1] * sin(a);
      }
      const double d = re * re + im * im;
      axis_f[n] = (d > 1e-10 ? 1.0 / d : 0.0) * exp(-k2 / (4.0 * xi * xi));
    }
    if (T > 0) {
      const int ntx = (M + T - 1) / T, TS = T + P - 1;
      int c = 0;
      for (int t = 0; t < ntx; ++t)
        for (int l = 0; l < TS; ++l) {
          int g = (t * T + off + l) % M;
          if (g < 0) g += M;
          if (g == n && c < KC) cover[n * KC + c++] = t * 64 + l;
        }
      for (int k = c; k < KC; ++k) cover[n * KC + k] = 0;
      cover_count[n] = c;
    }
  }
}

// Point the plan at a workspace of sz.total bytes and enqueue its tables
// and the clearing of its tile counters on the plan's stream.
hipError_t attach(se_plan &pl, const Sizes &sz, void *base) {
  pl.buf = carve(sz, base);
  const int M = pl.prm.M;
  const int KC = pl.T > 0 ? static_cast<int>(max_cover(pl.prm, pl.T)) : 0;
  if (pl.T > 0)
    pl.fold = sek::FoldTables{pl.buf.cover, pl.buf.cover_count, KC, pl.T + pl.prm.P - 1, pl.ntx};
  const int ncounts = pl.ntiles * sek::kCountStride;
  const int blocks = std::max(1, std::min(256, (std::max(M, ncounts) + sek::kThreads - 1) / sek::kThreads));
  const bool bs = pl.prm.window == SE_WINDOW_BSPLINE;
  if (pl.prm.dtype == SE_FP64)
    k_plan_tables<double><<<blocks, sek::kThreads, 0, pl.stream>>>(
        M, pl.prm.L, pl.prm.xi, pl.eta, bs, pl.prm.P, pl.T, stencil_offset(pl.prm), KC,
        static_cast<double *>(pl.buf.twiddle), static_cast<double *>(pl.buf.axis_f),
        static_cast<double *>(pl.buf.axis_k2), pl.buf.cover, pl.buf.cover_count, pl.buf.counts,
        ncounts);
  else
    k_plan_tables<float><<<blocks, sek::kThreads, 0, pl.stream>>>(
        M, pl.prm.L, pl.prm.xi, pl.eta, bs, pl.prm.P, pl.T, stencil_offset(pl.prm), KC,
        static_cast<float *>(pl.buf.twiddle), static_cast<double *>(pl.buf.axis_f),
        static_cast<double *>(pl.buf.axis_k2), pl.buf.cover, pl.buf.cover_count, pl.buf.counts,
        ncounts);
  return hipGetLastError();
}

void derive(se_plan &pl) {
  const se_params &p = pl.prm;
  pl.h = p.L / p.M;
  pl.wscale = 4.0 * M_PI / (p.L * p.L * p.L);
  if (p.window == SE_WINDOW_GAUSSIAN) {
    pl.eta = eta_of(p);
    pl.a = 2.0 * p.xi * p.xi / pl.eta;
    pl.cg = pl.a * pl.h * pl.h;
    pl.beta = pl.h * std::sqrt(pl.a / M_PI);
  } else {
    pl.eta = pl.a = pl.cg = pl.beta = 0.0;
  }
  pl.direct = p.window == SE_WINDOW_GAUSSIAN && p.P > 16;
  pl.T = pl.direct ? 0 : choose_tile(p);
  pl.ntx = pl.T > 0 ? (p.M + pl.T - 1) / pl.T : 0;
  pl.ntiles = pl.ntx * pl.ntx * pl.ntx;
  pl.bin_blocks = (pl.n_max + sek::kThreads - 1) / sek::kThreads;
  if (pl.bin_blocks < 1) pl.bin_blocks = 1;
  for (int pass = 0; pass < 3; ++pass) pl.fft_lgb[pass] = sek::fft_lgb(p.M, real_size(p), pass);
  pl.fft_threads = sek::kThreads;
  const int bz = 1 << pl.fft_lgb[sek::kPassZ];
  pl.zfft_blocks = (p.M * (p.M / 2 + 1) + bz - 1) / bz;
  pl.fft = radix_plan(p.M);
  if (pl.T > 0) {
    const int TS = pl.T + p.P - 1;
    pl.fold_by_tiles = (p.M % pl.T == 0) && (TS <= p.M) && (pl.ntx >= (TS + pl.T - 1) / pl.T);
  }
}

void destroy_events(se_plan &pl) {
  if (!pl.timing) return;
  for (auto &t : pl.timers)
    for (int k = 0; k < sek::kTimingSlots; ++k) {
      if (t.begin[k]) (void)hipEventDestroy(t.begin[k]);
      if (t.end[k]) (void)hipEventDestroy(t.end[k]);
      t.begin[k] = t.end[k] = nullptr;
    }
}

void free_targets(se_plan &pl) {
  void *ptrs[] = {pl.tgt.counts, pl.tgt.offsets, pl.tgt.key, pl.tgt.meta, pl.tgt.sorted,
                  pl.tgt.part, pl.tgt.ones};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  pl.tgt = sek::TargetBuffers{};
}

void free_all(se_plan &pl) {
  destroy_events(pl);
  free_targets(pl);
  if (pl.owned) (void)hipFree(pl.owned);
  pl.owned = nullptr;
  pl.buf = sek::DeviceBuffers{};
}

// Plans the caller creates without a workspace refuse to enqueue until one
// is attached.
se_status need_workspace(const se_plan *plan) {
  if (plan->buf.grid) return SE_OK;
  return fail(SE_ERR_STATE, "no workspace attached (plan created with SE_FLAG_CALLER_WORKSPACE: "
                            "call se_plan_set_workspace first)");
}

se_status forward_impl(se_plan &plan, int N, const void *x, const void *q, double *E_dev) {
  if (N < 0 || N > plan.n_max) return fail(SE_ERR_ARG, "N=%d outside [0, n_max=%d]", N, plan.n_max);
  if (N > 0 && (!x || !q)) return fail(SE_ERR_ARG, "x or q is NULL");
  if (!E_dev) return fail(SE_ERR_ARG, "E_dev is NULL");
  hipError_t e;
  if (plan.direct) {
    if ((e = sek::launch_direct_forward(plan, N, x, q)) != hipSuccess)
      return hip_fail(e, "spreading (untiled)");
  } else {
    if ((e = sek::launch_bin(plan, N, x, q)) != hipSuccess) return hip_fail(e, "binning");
    if ((e = sek::launch_spread(plan)) != hipSuccess) return hip_fail(e, "spreading");
  }
  if ((e = sek::launch_fft_forward_scale_inverse(plan, E_dev)) != hipSuccess)
    return hip_fail(e, "FFT/scaling");
  plan.last_N = N;
  return SE_OK;
}

se_status gather_impl(se_plan &plan, void *phi, void *F) {
  if (plan.last_N < 0) return fail(SE_ERR_STATE, "se_gather before se_forward");
  hipError_t e = sek::launch_gather(plan, plan.last_N, nullptr, sek::kGatherPotentialForce, phi, F);
  return e == hipSuccess ? SE_OK : hip_fail(e, "gathering");
}

// A plan refused because no tile edge fits, or because the staged tile
// blocks would wrap the grid more than the kernels handle: staged blocks
// index the grid in [-(P-1), M + T + P - 3], wrapped without division (holds
// for every M >= 8 with P <= M at the tile edges chosen).
se_status check_tiling(const se_plan &pl) {
  if (pl.T == 0 && !pl.direct)
    return fail(SE_ERR_UNSUPPORTED, "support %d in this precision needs more LDS than a CU has",
                pl.prm.P);
  if (!pl.direct && pl.T + pl.prm.P - 3 >= 2 * pl.prm.M)
    return fail(SE_ERR_GRID, "tile edge %d with support %d needs a larger grid than M=%d", pl.T,
                pl.prm.P, pl.prm.M);
  return SE_OK;
}

// ------------------------------------------------ no-allocation entry point
// se_kspace_noalloc carves the workspace of one evaluation out of this
// file-scope array instead of allocating: each GPU the library runs on holds
// its own copy (its address differs per device) until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxScratchDevices];  // device address of scratch, per device

// Device address of the current device's scratch, resolved once per device
// (with that device current) by hipGetSymbolAddress; host code uses only this
// address, never the array's name.
hipError_t scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

}  // namespace

namespace sek {
// Tile edge a plan with these parameters uses (0: none fits); the runtime
// model of the parameter selection prices the tile blocks with it.
int tile_edge_of(const se_params &p) { return choose_tile(p); }

se_status report(se_status s, const char *msg) {
  g_last_error = msg;
  return s;
}
}  // namespace sek

extern "C" {

const char *se_status_string(se_status s) {
  switch (s) {
    case SE_OK: return "SE_OK";
    case SE_ERR_ARG: return "SE_ERR_ARG: invalid argument";
    case SE_ERR_GRID: return "SE_ERR_GRID: unsupported grid size";
    case SE_ERR_ETA: return "SE_ERR_ETA: Gaussian shape eta outside (0,1)";
    case SE_ERR_UNSUPPORTED: return "SE_ERR_UNSUPPORTED: window/support/precision not built";
    case SE_ERR_WORKSPACE: return "SE_ERR_WORKSPACE: device allocation failed or workspace too small";
    case SE_ERR_HIP: return "SE_ERR_HIP: HIP runtime error";
    case SE_ERR_STATE: return "SE_ERR_STATE: no forward pass (or no workspace) on this plan yet";
  }
  return "unknown se_status";
}

const char *se_last_error(void) { return g_last_error.c_str(); }

se_status se_params_check(const se_params *prm, double *eta) { return check_params(prm, eta); }

se_status se_plan_workspace_size(const se_params *prm, int n_max, size_t *bytes) {
  se_status s = check_params(prm, nullptr);
  if (s != SE_OK) return s;
  if (n_max < 1) return fail(SE_ERR_ARG, "n_max must be >= 1 (got %d)", n_max);
  if (!bytes) return fail(SE_ERR_ARG, "bytes is NULL");
  se_plan tmp{};
  tmp.prm = *prm;
  tmp.n_max = n_max;
  derive(tmp);
  if ((s = check_tiling(tmp)) != SE_OK) return s;
  *bytes = sizes_of(tmp.prm, n_max, tmp.ntiles, tmp.bin_blocks, tmp.zfft_blocks, tmp.T).total;
  return SE_OK;
}

se_status se_plan_create(const se_params *prm, int n_max, void *hip_stream, se_plan **out) {
  if (!out) return fail(SE_ERR_ARG, "out is NULL");
  *out = nullptr;
  se_status s = check_params(prm, nullptr);
  if (s != SE_OK) return s;
  if (n_max < 1) return fail(SE_ERR_ARG, "n_max must be >= 1 (got %d)", n_max);

  se_plan *pl = new (std::nothrow) se_plan{};
  if (!pl) return fail(SE_ERR_WORKSPACE, "host allocation failed");
  pl->prm = *prm;
  if (pl->prm.c <= 0.0) pl->prm.c = 0.95;
  pl->n_max = n_max;
  pl->stream = static_cast<hipStream_t>(hip_stream);
  pl->last_N = -1;
  derive(*pl);
  if ((s = check_tiling(*pl)) != SE_OK) {
    delete pl;
    return s;
  }
  pl->timing = (pl->prm.flags & SE_FLAG_TIMING) != 0;
  const bool caller_ws = (pl->prm.flags & SE_FLAG_CALLER_WORKSPACE) != 0;
  if (caller_ws && !pl->timing) {  // nothing on the device until a workspace is attached
    *out = pl;
    return SE_OK;
  }
  pl->touched = true;
  hipError_t e = hipSuccess;
  for (int i = 0; i < SE_NUM_STAGES && pl->timing && e == hipSuccess; ++i)
    for (int k = 0; k < sek::kTimingSlots && e == hipSuccess; ++k) {
      e = hipEventCreate(&pl->timers[i].begin[k]);
      if (e == hipSuccess) e = hipEventCreate(&pl->timers[i].end[k]);
    }
  if (e == hipSuccess && !caller_ws) {
    const Sizes sz = sizes_of(pl->prm, n_max, pl->ntiles, pl->bin_blocks, pl->zfft_blocks, pl->T);
    e = hipMalloc(&pl->owned, sz.total);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      pl->owned = nullptr;
      free_all(*pl);
      delete pl;
      return fail(SE_ERR_WORKSPACE, "hipMalloc(%zu) failed: %s", sz.total, hipGetErrorString(e));
    }
    e = attach(*pl, sz, pl->owned);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_all(*pl);
    delete pl;
    return hip_fail(e, "plan set-up");
  }
  *out = pl;
  return SE_OK;
}

se_status se_plan_set_workspace(se_plan *plan, void *dev_ptr, size_t bytes) {
  if (!plan) return fail(SE_ERR_ARG, "plan is NULL");
  if (!(plan->prm.flags & SE_FLAG_CALLER_WORKSPACE))
    return fail(SE_ERR_ARG, "the plan owns its workspace (created without SE_FLAG_CALLER_WORKSPACE)");
  if (!dev_ptr) return fail(SE_ERR_ARG, "dev_ptr is NULL");
  const Sizes sz =
      sizes_of(plan->prm, plan->n_max, plan->ntiles, plan->bin_blocks, plan->zfft_blocks, plan->T);
  if (bytes < sz.total)
    return fail(SE_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu the plan needs",
                bytes, sz.total);
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0)
    return fail(SE_ERR_WORKSPACE, "workspace address is not a multiple of 256 bytes");
  plan->touched = true;
  hipError_t e = attach(*plan, sz, dev_ptr);
  if (e != hipSuccess) {
    plan->buf = sek::DeviceBuffers{};
    return hip_fail(e, "workspace tables");
  }
  plan->last_N = -1;  // the stored grid was in the previous workspace
  return SE_OK;
}

se_status se_plan_set_stream(se_plan *plan, void *hip_stream) {
  if (!plan) return fail(SE_ERR_ARG, "plan is NULL");
  plan->stream = static_cast<hipStream_t>(hip_stream);
  return SE_OK;
}

se_status se_plan_eta(const se_plan *plan, double *eta) {
  if (!plan || !eta) return fail(SE_ERR_ARG, "NULL argument");
  *eta = plan->eta;
  return SE_OK;
}

se_status se_plan_stage_times(se_plan *plan, double *ms, int n) {
  if (!plan || (!ms && n > 0) || n < 0) return fail(SE_ERR_ARG, "bad arguments");
  if (!plan->timing) return fail(SE_ERR_STATE, "plan was created without SE_FLAG_TIMING");
  for (int i = 0; i < SE_NUM_STAGES; ++i) {
    sek::StageTimer &t = plan->timers[i];
    while (t.harvested < t.issued) {
      hipError_t e = sek::harvest_oldest(t);
      if (e != hipSuccess) return hip_fail(e, "stage timing");
    }
    if (i < n) ms[i] = t.count > 0 ? t.sum_ms / static_cast<double>(t.count) : -1.0;
    t.sum_ms = 0.0;
    t.count = 0;
  }
  for (int i = SE_NUM_STAGES; i < n; ++i) ms[i] = -1.0;
  return SE_OK;
}

se_status se_plan_destroy(se_plan *plan) {
  if (!plan) return SE_OK;
  hipError_t e = plan->touched ? hipStreamSynchronize(plan->stream) : hipSuccess;
  free_all(*plan);
  delete plan;
  return e == hipSuccess ? SE_OK : hip_fail(e, "hipStreamSynchronize");
}

se_status se_forward(se_plan *plan, int N, const void *x, const void *q, double *E_dev) {
  if (!plan) return fail(SE_ERR_ARG, "plan is NULL");
  se_status s = need_workspace(plan);
  return s != SE_OK ? s : forward_impl(*plan, N, x, q, E_dev);
}

se_status se_gather(se_plan *plan, void *phi, void *F) {
  if (!plan) return fail(SE_ERR_ARG, "plan is NULL");
  return gather_impl(*plan, phi, F);
}

se_status se_kspace(se_plan *plan, int N, const void *x, const void *q, double *E_dev, void *phi,
                    void *F) {
  se_status s = se_forward(plan, N, x, q, E_dev);
  if (s != SE_OK) return s;
  return se_gather(plan, phi, F);
}

se_status se_plan_reserve_targets(se_plan *plan, int nt_max) {
  if (!plan) return fail(SE_ERR_ARG, "plan is NULL");
  if (nt_max < 1) return fail(SE_ERR_ARG, "nt_max must be >= 1 (got %d)", nt_max);
  plan->touched = true;
  hipError_t e = hipStreamSynchronize(plan->stream);  // earlier target work may use the old buffers
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  free_targets(*plan);
  sek::TargetBuffers &t = plan->tgt;
  const size_t rs = plan->prm.dtype == SE_FP64 ? 8 : 4;
  const size_t n = static_cast<size_t>(nt_max);
  struct { void **ptr; size_t bytes; } allocs[] = {
      {reinterpret_cast<void **>(&t.counts), static_cast<size_t>(std::max(plan->ntiles, 1)) * sek::kCountStride * 4},
      {reinterpret_cast<void **>(&t.offsets),
       static_cast<size_t>(plan->ntiles + 1 + sek::scan_chunks(plan->ntiles)) * 4},
      {reinterpret_cast<void **>(&t.key), n * 8},
      {reinterpret_cast<void **>(&t.meta), n * 8},
      {&t.sorted, n * 4 * rs},
      {reinterpret_cast<void **>(&t.part), ((n + sek::kThreads - 1) / sek::kThreads + 1) * 8},
      {&t.ones, n * rs}};
  for (auto &a : allocs) {
    if ((e = hipMalloc(a.ptr, a.bytes)) != hipSuccess) {
      (void)hipGetLastError();
      free_targets(*plan);
      return fail(SE_ERR_WORKSPACE, "hipMalloc of %zu bytes for evaluation points failed", a.bytes);
    }
  }
  std::vector<double> one64;
  std::vector<float> one32;
  const void *src;
  if (rs == 8) {
    one64.assign(n, 1.0);
    src = one64.data();
  } else {
    one32.assign(n, 1.0f);
    src = one32.data();
  }
  e = hipMemcpy(t.ones, src, n * rs, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemset(t.counts, 0, static_cast<size_t>(std::max(plan->ntiles, 1)) * sek::kCountStride * 4);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_targets(*plan);
    return hip_fail(e, "evaluation-point set-up");
  }
  t.cap = nt_max;
  return SE_OK;
}

se_status se_eval_targets(se_plan *plan, int nt, const void *xt, void *phi_t, void *field_t) {
  if (!plan) return fail(SE_ERR_ARG, "plan is NULL");
  if (plan->last_N < 0) return fail(SE_ERR_STATE, "se_eval_targets before se_forward");
  if (nt < 0 || nt > plan->tgt.cap)
    return fail(SE_ERR_ARG, "nt=%d outside [0, reserved %d] (se_plan_reserve_targets)", nt,
                plan->tgt.cap);
  if (nt == 0 || (!phi_t && !field_t)) return SE_OK;
  if (!xt) return fail(SE_ERR_ARG, "xt is NULL");
  sek::BinJob j;
  j.N = nt;
  j.x = xt;
  j.q = plan->tgt.ones;
  j.fp64 = plan->prm.dtype == SE_FP64;
  j.h = plan->h;
  j.M = plan->prm.M;
  j.T = plan->T;
  j.ntx = plan->ntx;
  j.ncells = plan->ntiles;
  j.counts = plan->tgt.counts;
  j.key = plan->tgt.key;
  j.offsets = plan->tgt.offsets;
  j.sorted = plan->tgt.sorted;
  j.meta = plan->tgt.meta;
  j.qsq_part = plan->tgt.part;
  j.stream = plan->stream;
  hipError_t e = plan->direct ? sek::launch_direct_prep(*plan, nt, xt, plan->tgt.ones,
                                                        plan->tgt.sorted, plan->tgt.meta,
                                                        plan->tgt.part, nullptr)
                              : sek::launch_bin_job(j, nullptr);
  if (e != hipSuccess) return hip_fail(e, "binning evaluation points");
  e = sek::launch_gather(*plan, nt, nullptr, sek::kGatherTargets, phi_t, field_t);
  return e == hipSuccess ? SE_OK : hip_fail(e, "gathering at evaluation points");
}

se_status se_backward(se_plan *plan, const double *gE_dev, void *grad_x, void *grad_q) {
  if (!plan) return fail(SE_ERR_ARG, "plan is NULL");
  if (!gE_dev) return fail(SE_ERR_ARG, "gE_dev is NULL");
  if (plan->last_N < 0) return fail(SE_ERR_STATE, "se_backward before se_forward");
  hipError_t e = sek::launch_gather(*plan, plan->last_N, gE_dev, sek::kGatherAdjoint, grad_q, grad_x);
  return e == hipSuccess ? SE_OK : hip_fail(e, "adjoint gathering");
}

}  // extern "C"

extern "C" se_status se_kspace_noalloc(const se_params *prm, int N, const void *x, const void *q,
                                       double *E_dev, void *phi, void *F, void *hip_stream) {
  se_status s = check_params(prm, nullptr);
  if (s != SE_OK) return s;
  if (prm->flags & (SE_FLAG_TIMING | SE_FLAG_CALLER_WORKSPACE))
    return fail(SE_ERR_ARG, "se_kspace_noalloc takes neither SE_FLAG_TIMING nor "
                            "SE_FLAG_CALLER_WORKSPACE");
  if (N < 0) return fail(SE_ERR_ARG, "N=%d is negative", N);
  // a plan on the stack: derived parameters and buffer pointers only
  se_plan pl{};
  pl.prm = *prm;
  if (pl.prm.c <= 0.0) pl.prm.c = 0.95;
  pl.n_max = N > 0 ? N : 1;
  pl.stream = static_cast<hipStream_t>(hip_stream);
  pl.last_N = -1;
  derive(pl);
  if ((s = check_tiling(pl)) != SE_OK) return s;
  const Sizes sz = sizes_of(pl.prm, pl.n_max, pl.ntiles, pl.bin_blocks, pl.zfft_blocks, pl.T);
  if (sz.total > kScratchBytes)
    return fail(SE_ERR_WORKSPACE,
                "this evaluation needs %zu bytes of workspace; the static scratch holds %zu",
                sz.total, kScratchBytes);
  void *base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return hip_fail(e, "address of the static scratch");
  if ((e = attach(pl, sz, base)) != hipSuccess) return hip_fail(e, "scratch tables");
  if ((s = forward_impl(pl, N, x, q, E_dev)) != SE_OK) return s;
  return gather_impl(pl, phi, F);
}
