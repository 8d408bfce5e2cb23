// Throughput of LDS integer atomics on the GPU it runs on, in the access
// pattern of the tile spread (libsekspace's k_spread_lane): 512-thread
// work-groups, each wave holding 8 particle groups of 8 lanes, each lane adding
// 64 values (8 x 8 rows of a 19^3 block at a random anchor) with ds_add_u32.
// It sets the ceiling the spread is measured against: the spread issues one
// LDS atomic lane per grid point it touches (N P^3 per call).
//
//   hipcc --offload-arch=gfx950 -O3 paper_1712_04718_amd/probes/lds_atomic_rate.hip -o lds_atomic_rate
//   ./lds_atomic_rate
//
// Prints, for 512 and 1728 work-groups (two and about seven per CU of a
// 256-CU device), the lane-atomics per second and per clock per CU (at the
// clock given on the command line, default 2.4 GHz), for plain integer values
// and for values converted from float (the spread's fixed-point step), and
// for a conflict-free pattern, then one JSON line with the same figures (its
// "spread_pattern_float_lane_atomics_per_s" is the larger of the two grids'
// float->int rates).  Every LDS index stays inside the block.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kT = 12, kS = 8, kTS = kT + kS - 1, kTS3 = kTS * kTS * kTS;
constexpr int kThreads = 512;
constexpr int kRounds = 25;  // particle rounds per wave (8 particles each)

__device__ unsigned mix(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// kind 0: integer values; 1: float products rounded to the nearest integer
template <int kKind>
__global__ void __launch_bounds__(kThreads) k_spread_pattern(int *sink, float w0) {
  __shared__ int blk[kTS3];
  for (int i = threadIdx.x; i < kTS3; i += kThreads) blk[i] = 0;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = lane / kS, jx = lane % kS;
  float gy[kS];
  for (int j = 0; j < kS; ++j) gy[j] = w0 * (j + 1) * 0.37f;
  for (int r = 0; r < kRounds; ++r) {
    const unsigned h = mix(blockIdx.x * 4096u + wave * 256u + r * 8u + grp);
    const int ax = h % kT, ay = (h / kT) % kT, az = (h / (kT * kT)) % kT;  // anchors in [0, T)
    int *row = blk + (az * kTS + ay) * kTS + ax + jx;  // max index (TS-1)(TS^2+TS+1) = TS^3-1
    const float wq = w0 * (1.0f + (h & 1023));
#pragma unroll
    for (int jz = 0; jz < kS; ++jz) {
      const float wz = wq * gy[jz];
#pragma unroll
      for (int jy = 0; jy < kS; ++jy)
        atomicAdd(row + (jz * kTS + jy) * kTS, kKind == 0 ? jy + jz : __float2int_rn(wz * gy[jy]));
    }
  }
  __syncthreads();
  long long s = 0;
  for (int i = threadIdx.x; i < kTS3; i += kThreads) s += blk[i];
  if (s == 0x7fffffff) sink[blockIdx.x] = 1;  // keeps the block live
}

// conflict-free reference: lane l of a wave adds to word l + 64 k
__global__ void __launch_bounds__(kThreads) k_linear_pattern(int *sink) {
  __shared__ int blk[kTS3];
  for (int i = threadIdx.x; i < kTS3; i += kThreads) blk[i] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = 0; r < kRounds; ++r)
#pragma unroll
    for (int k = 0; k < 64; ++k)
      atomicAdd(&blk[lane + 64 * ((k + wave * 13 + r) % 100)], k);  // < 64 * 100 <= TS^3
  __syncthreads();
  long long s = 0;
  for (int i = threadIdx.x; i < kTS3; i += kThreads) s += blk[i];
  if (s == 0x7fffffff) sink[blockIdx.x] = 1;
}

bool ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return true;
  std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
  return false;
}

}  // namespace

int main(int argc, char **argv) {
  const double ghz = argc > 1 ? std::atof(argv[1]) : 2.4;
  int *sink = nullptr;
  if (!ok(hipMalloc(&sink, 4096 * sizeof(int)), "hipMalloc")) return 1;
  hipDeviceProp_t prop;
  if (!ok(hipGetDeviceProperties(&prop, 0), "device properties")) return 1;
  const int cus = prop.multiProcessorCount;
  hipEvent_t a, b;
  if (!ok(hipEventCreate(&a), "event") || !ok(hipEventCreate(&b), "event")) return 1;
  std::printf("device %s, %d CUs, clock assumed %.2f GHz\n", prop.name, cus, ghz);
  double rate[2][3] = {};
  const int grids[2] = {512, 1728};
  for (int gi = 0; gi < 2; ++gi) {
    const int grid = grids[gi];
    int kind = 0;
    const double lanes = double(grid) * (kThreads / 64) * kRounds * 64 * 64;  // lane-atomics
    const auto run = [&](const char *name, auto launch) {
      for (int w = 0; w < 3; ++w) launch();
      if (!ok(hipDeviceSynchronize(), "warm-up")) std::exit(1);
      const int reps = 20;
      (void)hipEventRecord(a);
      for (int i = 0; i < reps; ++i) launch();
      (void)hipEventRecord(b);
      if (!ok(hipEventSynchronize(b), "timing")) std::exit(1);
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, a, b);
      const double s = ms * 1e-3 / reps;
      std::printf("grid %5d  %-28s %8.2f us  %.3e lane-atomics/s  %5.2f per clock per CU\n", grid,
                  name, s * 1e6, lanes / s, lanes / s / (ghz * 1e9) / cus);
      rate[gi][kind++] = lanes / s;
    };
    run("spread pattern, integer", [&] { k_spread_pattern<0><<<grid, kThreads>>>(sink, 0.5f); });
    run("spread pattern, float->int", [&] { k_spread_pattern<1><<<grid, kThreads>>>(sink, 0.5f); });
    run("conflict-free pattern", [&] { k_linear_pattern<<<grid, kThreads>>>(sink); });
  }
  std::printf("{\"device\": \"%s\", \"cus\": %d, \"clock_ghz_assumed\": %.2f", prop.name, cus, ghz);
  const char *keys[3] = {"integer", "float_to_int", "conflict_free"};
  for (int gi = 0; gi < 2; ++gi)
    for (int k = 0; k < 3; ++k)
      std::printf(", \"grid%d_%s_lane_atomics_per_s\": %.4e", grids[gi], keys[k], rate[gi][k]);
  std::printf(", \"spread_pattern_float_lane_atomics_per_s\": %.4e}\n",
              rate[0][1] > rate[1][1] ? rate[0][1] : rate[1][1]);
  const bool good = ok(hipGetLastError(), "launch");
  (void)hipFree(sink);
  return good ? 0 : 1;
}
