// Steps 3-5 of Algorithm 1: forward 3D FFT of the real grid, multiplication
// by the influence function with the k-space energy, inverse 3D FFT.
//
// Passes over a half spectrum stored as C[z][kx][y], kx = 0..M/2
// (K = M/2 + 1 values), y contiguous, all built on one batched Stockham FFT
// held in LDS.  Where a z plane fits in LDS (compiled M: twice, ping-pong
// stages, FP32 M <= 128 and FP64 M <= 96; once, in-place stages, FP32
// M = 144..192 and FP64 M = 120, 128) the x and y passes of each direction
// run as one plane pass (k_fft_xy_r2c, k_fft_yx_c2r, below), so the sequence
// is xy, z, yx; other sizes run the five passes (for compiled M with one
// LDS buffer of pencils and in-place stages, which leaves room for more
// work-groups per CU; the run-time plan's kernels ping-pong between two):
//   x_r2c : pairs of real rows packed as one complex row, transformed, and
//           split into two half spectra, written as runs along y;
//   y_fwd : FFT of B contiguous y pencils (consecutive (z, kx));
//   z     : FFT along z of B adjacent (kx, ky) pencils, scale by the
//           influence function w(k) (eq. 4.6 for SE, eq. 6.2 for SPME)
//           times 4 pi / L^3, accumulate the energy
//             E = 1/2 sum_k mu(kx) w(k) |G^(k)|^2   (FP64),
//           mu = 1 on kx = 0 and kx = M/2 and 2 elsewhere (Hermitian half),
//           then the inverse FFT along z; one energy partial per block;
//   y_inv : inverse FFT along y; its first work-group adds the energy
//           partials in a fixed order;
//   x_c2r : two half spectra rebuilt into one Hermitian-packed complex row,
//           inverse FFT, real and imaginary parts are the two real rows.
// Forward transforms use e^{-i k.x}, inverse ones e^{+i k.x}, both
// unnormalised; the inverse is conj(FFT(conj(.))).
//
// In LDS a batch of B pencils of length M is stored element-major
// (element k of pencil b at k*PB + b, PB >= B) so that the B threads working
// on the same butterfly index of different pencils touch consecutive
// addresses.
#include "se_common.hpp"

namespace sek {
namespace {

extern __shared__ __align__(16) unsigned char f_smem[];

// Complex elements per thread when a work-group loads its B pencils
// (M * B <= 16 * threads for every plan, see fft_lgb).
constexpr int kMaxPerThread = 16;

// Work-group size of the z pass: 512 threads for compiled M >= 384, whose
// work-groups each hold 1700-3500 values through the twenty-odd in-place
// stages of the pass (measured: 242 -> 209 us at M = 432, 149 -> 129 us at
// M = 384, FP32), else kThreads (at M = 192-288 the wider work-groups were
// no faster or slower).
constexpr int zpass_threads(int MC) { return MC >= 384 ? 512 : kThreads; }

// Work-group size of the five-pass x and y kernels: 512 threads for FP64 at
// compiled M >= 384 (M = 432: inverse y 331 -> 254 us, inverse x 293 -> 258
// us), else kThreads (FP32 lost 5-15% with 512 at M = 384 and 432).
template <typename R> constexpr int xy_threads(int MC) {
  return sizeof(R) == 8 && MC >= 384 ? 512 : kThreads;
}

template <typename C> __device__ inline C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C> __device__ inline C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __device__ inline C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __device__ inline C cconj(C a) { a.y = -a.y; return a; }
// Two adjacent complex values, moved as one 16- or 32-byte access.
template <typename R> struct alignas(4 * sizeof(R)) C2 {
  cplx_t<R> a, b;
};

// multiply by -i
template <typename C> __device__ inline C cmul_mi(C a) { C r; r.x = a.y; r.y = -a.x; return r; }

// Forward DFTs of small prime-power sizes (X_k = sum_n x_n e^{-2 pi i nk/R}).
template <typename R, typename C> __device__ inline void dft2(C *v) {
  const C a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <typename R, typename C> __device__ inline void dft3(C *v) {
  const R s3 = static_cast<R>(0.86602540378443864676);  // sin(2 pi / 3)
  const C t1 = cadd(v[1], v[2]);
  C t2;
  t2.x = v[0].x - R(0.5) * t1.x;
  t2.y = v[0].y - R(0.5) * t1.y;
  const C d = csub(v[1], v[2]);
  C t3;  // -i sin(2pi/3) (v1 - v2)
  t3.x = s3 * d.y;
  t3.y = -s3 * d.x;
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, t3);
  v[2] = csub(t2, t3);
}
template <typename R, typename C> __device__ inline void dft4(C *v) {
  const C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  const C c = cadd(v[1], v[3]), d = cmul_mi(csub(v[1], v[3]));
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}
template <typename R, typename C> __device__ inline void dft5(C *v) {
  const R c1 = static_cast<R>(0.30901699437494742410);   // cos(2 pi/5)
  const R c2 = static_cast<R>(-0.80901699437494742410);  // cos(4 pi/5)
  const R s1 = static_cast<R>(0.95105651629515357212);   // sin(2 pi/5)
  const R s2 = static_cast<R>(0.58778525229247312917);   // sin(4 pi/5)
  const C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  const C t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
  C a1, a2, b1, b2;
  a1.x = v[0].x + c1 * t1.x + c2 * t2.x;  a1.y = v[0].y + c1 * t1.y + c2 * t2.y;
  a2.x = v[0].x + c2 * t1.x + c1 * t2.x;  a2.y = v[0].y + c2 * t1.y + c1 * t2.y;
  b1.x = s1 * t3.x + s2 * t4.x;           b1.y = s1 * t3.y + s2 * t4.y;
  b2.x = s2 * t3.x - s1 * t4.x;           b2.y = s2 * t3.y - s1 * t4.y;
  v[0] = cadd(v[0], cadd(t1, t2));
  const C mb1 = cmul_mi(b1), mb2 = cmul_mi(b2);
  v[1] = cadd(a1, mb1);
  v[4] = csub(a1, mb1);
  v[2] = cadd(a2, mb2);
  v[3] = csub(a2, mb2);
}
template <typename R, typename C> __device__ inline void dft8(C *v) {
  const R r2 = static_cast<R>(0.70710678118654752440);
  // two radix-4 halves on even/odd samples, then combine
  C e[4] = {v[0], v[2], v[4], v[6]};
  C o[4] = {v[1], v[3], v[5], v[7]};
  dft4<R, C>(e);
  dft4<R, C>(o);
  // twiddles e^{-2 pi i k / 8}, k = 0..3
  C w1; w1.x = r2 * (o[1].x + o[1].y); w1.y = r2 * (o[1].y - o[1].x);
  const C w2 = cmul_mi(o[2]);
  C w3; w3.x = r2 * (o[3].y - o[3].x); w3.y = -r2 * (o[3].x + o[3].y);
  v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], w1);   v[5] = csub(e[1], w1);
  v[2] = cadd(e[2], w2);   v[6] = csub(e[2], w2);
  v[3] = cadd(e[3], w3);   v[7] = csub(e[3], w3);
}

// One radix stage of the Stockham autosort FFT on B = 2^lgB pencils:
//   in[(j + r M/R) B + b] -> twiddle by w^{r k}, k = j mod Ns, w = e^{-2pi i/(Ns R)}
//   -> R-point DFT -> out[((j/Ns) Ns R + k + r Ns) B + b].
template <typename R, int RAD>
__device__ inline void stockham_stage(const cplx_t<R> *in, cplx_t<R> *out, int M, int lgB,
                                      int Ns, unsigned ns_magic, int tstep,
                                      const cplx_t<R> *tw) {
  using C = cplx_t<R>;
  const int nb = M / RAD;
  const int total = nb << lgB;
  const int bmask = (1 << lgB) - 1;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int b = t & bmask, j = t >> lgB;
    const int q = (Ns == 1) ? j : fast_div(j, ns_magic);
    const int k = j - q * Ns;
    C v[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) v[r] = in[((j + r * nb) << lgB) + b];
    if (k != 0) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) v[r] = cmul(v[r], tw[r * k * tstep]);
    }
    if constexpr (RAD == 2) dft2<R, C>(v);
    if constexpr (RAD == 3) dft3<R, C>(v);
    if constexpr (RAD == 4) dft4<R, C>(v);
    if constexpr (RAD == 5) dft5<R, C>(v);
    if constexpr (RAD == 8) dft8<R, C>(v);
    const int dst = q * Ns * RAD + k;
#pragma unroll
    for (int r = 0; r < RAD; ++r) out[((dst + r * Ns) << lgB) + b] = v[r];
  }
}

// Forward FFT of B = 2^lgB pencils held in buf0; returns the buffer with the result.
template <typename R>
__device__ cplx_t<R> *fft_batch(cplx_t<R> *buf0, cplx_t<R> *buf1, int lgB, const FftPlan &pl,
                                const cplx_t<R> *tw) {
  cplx_t<R> *in = buf0, *out = buf1;
  for (int s = 0; s < pl.nstages; ++s) {
    const int Ns = pl.ns[s];
    const unsigned mg = pl.ns_magic[s];
    const int ts = pl.tstep[s];
    switch (pl.radix[s]) {
      case 2: stockham_stage<R, 2>(in, out, pl.M, lgB, Ns, mg, ts, tw); break;
      case 3: stockham_stage<R, 3>(in, out, pl.M, lgB, Ns, mg, ts, tw); break;
      case 4: stockham_stage<R, 4>(in, out, pl.M, lgB, Ns, mg, ts, tw); break;
      case 5: stockham_stage<R, 5>(in, out, pl.M, lgB, Ns, mg, ts, tw); break;
      default: stockham_stage<R, 8>(in, out, pl.M, lgB, Ns, mg, ts, tw); break;
    }
    __syncthreads();
    cplx_t<R> *t = in; in = out; out = t;
  }
  return in;
}

// Compile-time variant for a fixed M and batch: every stage's radix, stride
// and twiddle step are constants, so the index arithmetic folds away and
// the butterfly loops unroll.
struct RadixList {
  int n;
  int r[kMaxRadixStages];
};
constexpr RadixList radix_list(int M) {
  RadixList l{0, {}};
  int m = M;
  while (m % 8 == 0) { l.r[l.n++] = 8; m /= 8; }
  if (m % 4 == 0) { l.r[l.n++] = 4; m /= 4; }
  if (m % 2 == 0) { l.r[l.n++] = 2; m /= 2; }
  while (m % 5 == 0) { l.r[l.n++] = 5; m /= 5; }
  while (m % 3 == 0) { l.r[l.n++] = 3; m /= 3; }
  return l;
}

// B pencils (any count), element e of pencil b at e * PB + b (PB >= B: a
// padded row), NT threads; lanes run over b fastest.
template <typename R, int M, int B, int PB, int NT, int RAD, int NS>
__device__ inline void stockham_stage_ct(const cplx_t<R> *in, cplx_t<R> *out,
                                         const cplx_t<R> *tw) {
  using C = cplx_t<R>;
  constexpr int NB = M / RAD, TOTAL = NB * B, TSTEP = M / (NS * RAD);
#pragma unroll
  for (int t0 = 0; t0 < TOTAL; t0 += NT) {
    const int t = t0 + static_cast<int>(threadIdx.x);
    if (TOTAL % NT == 0 || t < TOTAL) {
      const int j = t / B, b = t - j * B;
      const int q = j / NS, k = j - q * NS;
      C v[RAD];
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[r] = in[(j + r * NB) * PB + b];
      if (NS > 1 && k != 0) {
#pragma unroll
        for (int r = 1; r < RAD; ++r) v[r] = cmul(v[r], tw[r * k * TSTEP]);
      }
      if constexpr (RAD == 2) dft2<R, C>(v);
      if constexpr (RAD == 3) dft3<R, C>(v);
      if constexpr (RAD == 4) dft4<R, C>(v);
      if constexpr (RAD == 5) dft5<R, C>(v);
      if constexpr (RAD == 8) dft8<R, C>(v);
      const int dst = q * NS * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) out[(dst + r * NS) * PB + b] = v[r];
    }
  }
}

// All stages, ping-ponging between in and out; returns the buffer holding
// the result.
template <typename R, int M, int B, int PB, int NT, int STAGE, int NS>
__device__ inline cplx_t<R> *fft_batch_ct(cplx_t<R> *in, cplx_t<R> *out, const cplx_t<R> *tw) {
  constexpr RadixList L = radix_list(M);
  if constexpr (STAGE == L.n) {
    return in;
  } else {
    constexpr int RAD = L.r[STAGE];
    stockham_stage_ct<R, M, B, PB, NT, RAD, NS>(in, out, tw);
    __syncthreads();
    return fft_batch_ct<R, M, B, PB, NT, STAGE + 1, NS * RAD>(out, in, tw);
  }
}

// The same stages in one buffer: each thread reads its butterflies into
// registers, the work-group waits, and the results go back to the same LDS
// (the Stockham permutation of the stage), for plane buffers that fit in LDS
// only once.
template <typename R, int M, int B, int PB, int NT, int RAD, int NS>
__device__ inline void stockham_stage_inplace(cplx_t<R> *buf, const cplx_t<R> *tw) {
  using C = cplx_t<R>;
  constexpr int NB = M / RAD, TOTAL = NB * B, TSTEP = M / (NS * RAD);
  constexpr int NIT = (TOTAL + NT - 1) / NT;
  C v[NIT][RAD];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int t = it * NT + static_cast<int>(threadIdx.x);
    if (TOTAL % NT == 0 || t < TOTAL) {
      const int j = t / B, b = t - j * B;
      const int k = j % NS;
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[it][r] = buf[(j + r * NB) * PB + b];
      if (NS > 1 && k != 0) {
#pragma unroll
        for (int r = 1; r < RAD; ++r) v[it][r] = cmul(v[it][r], tw[r * k * TSTEP]);
      }
      if constexpr (RAD == 2) dft2<R, C>(v[it]);
      if constexpr (RAD == 3) dft3<R, C>(v[it]);
      if constexpr (RAD == 4) dft4<R, C>(v[it]);
      if constexpr (RAD == 5) dft5<R, C>(v[it]);
      if constexpr (RAD == 8) dft8<R, C>(v[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int t = it * NT + static_cast<int>(threadIdx.x);
    if (TOTAL % NT == 0 || t < TOTAL) {
      const int j = t / B, b = t - j * B;
      const int q = j / NS, k = j - q * NS;
      const int dst = q * NS * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf[(dst + r * NS) * PB + b] = v[it][r];
    }
  }
  __syncthreads();
}

template <typename R, int M, int B, int PB, int NT, int STAGE, int NS>
__device__ inline void fft_batch_inplace(cplx_t<R> *buf, const cplx_t<R> *tw) {
  constexpr RadixList L = radix_list(M);
  if constexpr (STAGE < L.n) {
    constexpr int RAD = L.r[STAGE];
    stockham_stage_inplace<R, M, B, PB, NT, RAD, NS>(buf, tw);
    fft_batch_inplace<R, M, B, PB, NT, STAGE + 1, NS * RAD>(buf, tw);
  }
}

// Forward FFT of the B pencils in buf0 for the five-pass kernels: compiled
// M in place in buf0 (buf1 is not used), the run-time plan ping-ponging
// between buf0 and buf1; returns the buffer holding the result.
template <typename R, int MC, int LGBC, int NT = kThreads>
__device__ inline cplx_t<R> *fft_pencils(cplx_t<R> *buf0, cplx_t<R> *buf1, int lgB,
                                         const FftPlan &pl, const cplx_t<R> *tw) {
  if constexpr (MC > 0) {
    fft_batch_inplace<R, MC, 1 << LGBC, 1 << LGBC, NT, 0, 1>(buf0, tw);
    return buf0;
  } else {
    return fft_batch<R>(buf0, buf1, lgB, pl, tw);
  }
}

// i / M: a constant divisor when M is known at compile time, else the
// plan's magic multiplier.
template <int MC> __device__ inline int div_M(int i, const FftPlan &pl) {
  if constexpr (MC > 0) return i / MC;
  else return fast_div(i, pl.m_magic);
}

// ---------------------------------------------------------------- x passes

template <typename R, int MC, int LGBC>
__global__ void __launch_bounds__(xy_threads<R>(MC))
k_fft_x_r2c(const R *__restrict__ grid, cplx_t<R> *__restrict__ spec, FftPlan pl, int lgB,
            const cplx_t<R> *__restrict__ tw_g) {
  using C = cplx_t<R>;
  constexpr int NT = xy_threads<R>(MC), NPT = 16 * kThreads / NT;
  constexpr bool CT = MC > 0;
  const int M = CT ? MC : pl.M;
  const int lgb = CT ? LGBC : lgB;
  const int K = M / 2 + 1, B = 1 << lgb;
  C *b0 = reinterpret_cast<C *>(f_smem), *b1 = CT ? b0 : b0 + M * B;  // compiled M: one buffer
  C *twl = b1 + M * B;  // twiddles staged in LDS
  for (int i = threadIdx.x; i < M; i += NT) twl[i] = tw_g[i];
  const long long nrows = static_cast<long long>(M) * M;
  const long long row0 = static_cast<long long>(xcd_local(blockIdx.x, gridDim.x)) * 2 * B;
  // row r of the batch goes to pencil r/2, real part for even r, imag for odd;
  // all loads are issued before the first LDS store
  R v[2 * NPT];
#pragma unroll
  for (int k = 0; k < 2 * NPT; ++k) {
    const int i = threadIdx.x + k * NT;
    const long long gr = row0 + div_M<MC>(i, pl);
    v[k] = (i < 2 * B * M && gr < nrows) ? grid[row0 * M + i] : R(0);
  }
#pragma unroll
  for (int k = 0; k < 2 * NPT; ++k) {
    const int i = threadIdx.x + k * NT;
    if (i < 2 * B * M) {
      const int r = div_M<MC>(i, pl), xk = i - r * M;
      reinterpret_cast<R *>(&b0[xk * B + (r >> 1)])[r & 1] = v[k];
    }
  }
  __syncthreads();
  const C *Z = fft_pencils<R, MC, LGBC, NT>(b0, b1, lgb, pl, twl);
  // Z = FFT(r1 + i r2): R1[k] = (Z[k] + conj Z[M-k]) / 2, R2[k] = (Z[k] - conj Z[M-k]) / 2i.
  // Rows 2b and 2b+1 are (z, y) and (z, y+1) with y even (M is even), so the
  // two half spectra land side by side in C[z][k][y]: one 2-element store.
  for (int i = threadIdx.x; i < B * K; i += NT) {
    const int k = i >> lgb, b = i & (B - 1);
    const long long gr = row0 + 2 * b;
    if (gr >= nrows) continue;
    const C zk = Z[k * B + b];
    const C zm = Z[(k == 0 ? 0 : M - k) * B + b];
    C2<R> r;
    r.a.x = R(0.5) * (zk.x + zm.x);
    r.a.y = R(0.5) * (zk.y - zm.y);
    r.b.x = R(0.5) * (zk.y + zm.y);
    r.b.y = R(-0.5) * (zk.x - zm.x);
    const int z = div_M<MC>(static_cast<int>(gr), pl), y = static_cast<int>(gr) - z * M;
    *reinterpret_cast<C2<R> *>(&spec[(static_cast<long long>(z) * K + k) * M + y]) = r;
  }
}

template <typename R, int MC, int LGBC>
__global__ void __launch_bounds__(xy_threads<R>(MC))
k_fft_x_c2r(const cplx_t<R> *__restrict__ spec, R *__restrict__ grid, FftPlan pl, int lgB,
            const cplx_t<R> *__restrict__ tw_g) {
  using C = cplx_t<R>;
  constexpr int NT = xy_threads<R>(MC), NPT = 16 * kThreads / NT;
  constexpr bool CT = MC > 0;
  const int M = CT ? MC : pl.M;
  const int lgb = CT ? LGBC : lgB;
  const int K = M / 2 + 1, B = 1 << lgb;
  C *b0 = reinterpret_cast<C *>(f_smem), *b1 = CT ? b0 : b0 + M * B;  // compiled M: one buffer
  C *twl = b1 + M * B;  // twiddles staged in LDS
  for (int i = threadIdx.x; i < M; i += NT) twl[i] = tw_g[i];
  const long long nrows = static_cast<long long>(M) * M;
  const long long row0 = static_cast<long long>(xcd_local(blockIdx.x, gridDim.x)) * 2 * B;
  // Z[k] = R1[k] + i R2[k] on 0..M/2 and conj(R1[M-k]) + i conj(R2[M-k]) above;
  // stored conjugated for the inverse transform.
  for (int i = threadIdx.x; i < B * K; i += NT) {
    const int k = i >> lgb, b = i & (B - 1);
    const long long gr = row0 + 2 * b;
    C r1, r2;
    if (gr < nrows) {
      const int z = div_M<MC>(static_cast<int>(gr), pl), y = static_cast<int>(gr) - z * M;
      const C2<R> r =
          *reinterpret_cast<const C2<R> *>(&spec[(static_cast<long long>(z) * K + k) * M + y]);
      r1 = r.a;
      r2 = r.b;
    } else {
      r1.x = r1.y = r2.x = r2.y = R(0);
    }
    C z;
    z.x = r1.x - r2.y;
    z.y = -(r1.y + r2.x);
    b0[k * B + b] = z;
    if (k > 0 && k < M - k) {
      C zc;
      zc.x = r1.x + r2.y;
      zc.y = -(r2.x - r1.y);
      b0[(M - k) * B + b] = zc;
    }
  }
  __syncthreads();
  const C *Z = fft_pencils<R, MC, LGBC, NT>(b0, b1, lgb, pl, twl);
  for (int i = threadIdx.x; i < 2 * B * M; i += NT) {
    const int r = div_M<MC>(i, pl), xk = i - r * M;
    const long long gr = row0 + r;
    if (gr >= nrows) continue;
    const C z = Z[xk * B + (r >> 1)];
    grid[gr * M + xk] = (r & 1) ? -z.y : z.x;  // conj of the forward result
  }
}

// ---------------------------------------------------------------- y passes

// For the inverse pass, work-group (0,0) also adds the energy partials of
// the z pass in a fixed order and writes E (plus the self energy if asked).
struct EnergyOut {
  const double *part;      // energy partials of the z pass
  int nparts;
  const double *qsq_part;  // per-block sums of q^2 from binning
  int nq;
  double self_coef;        // -xi / sqrt(pi) with the self term, else 0
  double *E;
};

// E = sum of the z pass's energy partials (+ self_coef sum q^2), each sum
// taken in a fixed order: per-thread strided sums, then a fixed tree over
// the lanes of a wave and over the waves.  Called by the whole work-group.
template <int NT>
__device__ inline void write_energy(const EnergyOut &eo) {
  __shared__ double wred[2][NT / 64];
  double se = 0.0, sq = 0.0;
  for (int b = threadIdx.x; b < eo.nparts; b += NT) se += eo.part[b];
  if (eo.self_coef != 0.0)
    for (int b = threadIdx.x; b < eo.nq; b += NT) sq += eo.qsq_part[b];
  const auto add = [](double a, double b) { return a + b; };
  se = wave_reduce0(se, add);
  sq = wave_reduce0(sq, add);
  if ((threadIdx.x & 63) == 0) {
    wred[0][threadIdx.x >> 6] = se;
    wred[1][threadIdx.x >> 6] = sq;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double e = 0.0, q = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      e += wred[0][w];
      q += wred[1][w];
    }
    *eo.E = e + eo.self_coef * q;
  }
}

template <typename R, int MC, int LGBC, bool INV>
__global__ void __launch_bounds__(xy_threads<R>(MC))
k_fft_y(cplx_t<R> *__restrict__ spec, FftPlan pl, int lgB, const cplx_t<R> *__restrict__ tw_g,
        EnergyOut eo) {
  using C = cplx_t<R>;
  constexpr int NT = xy_threads<R>(MC), NPT = 16 * kThreads / NT;
  constexpr bool CT = MC > 0;
  const int M = CT ? MC : pl.M;
  const int lgb = CT ? LGBC : lgB;
  const int K = M / 2 + 1, B = 1 << lgb;
  C *b0 = reinterpret_cast<C *>(f_smem), *b1 = CT ? b0 : b0 + M * B;  // compiled M: one buffer
  C *twl = b1 + M * B;  // twiddles staged in LDS
  for (int i = threadIdx.x; i < M; i += NT) twl[i] = tw_g[i];
  // B consecutive (z, kx) pencils, each M contiguous values along y
  const int npen = M * K;
  const int c0 = xcd_local(blockIdx.x, gridDim.x) * B;
  {
    C v[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int i = threadIdx.x + k * NT;
      const int y = i >> lgb, b = i & (B - 1);
      if (i < M * B && c0 + b < npen) {
        v[k] = spec[static_cast<long long>(c0 + b) * M + y];
        if (INV) v[k] = cconj(v[k]);
      } else {
        v[k].x = v[k].y = R(0);
      }
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int i = threadIdx.x + k * NT;
      if (i < M * B) b0[i] = v[k];
    }
  }
  __syncthreads();
  const C *Z = fft_pencils<R, MC, LGBC, NT>(b0, b1, lgb, pl, twl);
  for (int i = threadIdx.x; i < M * B; i += NT) {
    const int y = i >> lgb, b = i & (B - 1);
    if (c0 + b < npen) {
      C v = Z[i];
      if (INV) v = cconj(v);
      spec[static_cast<long long>(c0 + b) * M + y] = v;
    }
  }
  if (INV && blockIdx.x == 0 && eo.E) write_energy<NT>(eo);
}

// ------------------------------------------------- fused x-y plane passes
//
// When an M x (M/2 + 1) complex buffer fits in LDS, work-groups that each
// hold a whole z plane do both in-plane transforms, so that the 3D FFT and
// its inverse take three launches (xy, z with scaling, yx) instead of five:
//   k_fft_xy_r2c: the plane's real rows in pairs as complex rows (x-major),
//     FFT along x, split into the two half spectra, FFT along y of the kx
//     pencils, store C[z][kx][y];
//   k_fft_yx_c2r: the mirror image (conjugated input, inverse along y,
//     Hermitian rebuild, inverse along x, real rows out).
// NS work-groups may share a plane so that more CUs take part: each repeats
// the first transform of the plane (along x forward, along y inverse) and
// does the second for its 1/NS of the pencils (kx pencils forward, row
// pairs inverse).
// Rows in LDS hold PB = (M/2 + 1) | 1 complex values: with an odd row
// length the column walks of the load, split and store phases keep 64-bit
// LDS accesses conflict-free within each half wave.
template <int M, int NS> struct PlaneGeom {
  static constexpr int H = M / 2, K = M / 2 + 1, PB = K | 1, BUF = M * PB;
  static constexpr int KP = (K + NS - 1) / NS;  // kx pencils per work-group (forward)
  static constexpr int HP = H / NS;             // row pairs per work-group (inverse)
};
// work-groups per plane (two beat one in both directions at M = 96, FP32
// and FP64, despite reading each plane twice)
constexpr int kPlaneSplitFwd = 2, kPlaneSplitInv = 2;
template <typename R, int M> constexpr size_t plane_lds_bytes() {
  return sizeof(cplx_t<R>) * (2 * PlaneGeom<M, 1>::BUF + M);
}
// one plane buffer (in-place stages), one work-group per plane
template <typename R, int M> constexpr size_t plane1_lds_bytes() {
  return sizeof(cplx_t<R>) * (PlaneGeom<M, 1>::BUF + M);
}
// threads per plane work-group: about four complex values per thread, 64..1024
constexpr int plane_threads(int M) {
  int nt = 64;
  while (nt < 1024 && 4 * nt < (M / 2) * M) nt *= 2;
  return nt;
}
template <typename R, int M> constexpr bool plane_fits() {
  return plane_lds_bytes<R, M>() <= kMaxLds && M % 4 == 0 && (M / 2) % kPlaneSplitInv == 0;
}
template <typename R, int M> constexpr bool plane1_fits() {
  return plane1_lds_bytes<R, M>() <= kMaxLds && M % 4 == 0;
}

// ONE: a single plane buffer and in-place stages (NS = 1): the x FFT, the
// split into the two half spectra (every thread first reads the values it
// needs, then all write) and the y FFT all work in the one M x PB buffer.
template <typename R, int M, int NT, int NS, bool ONE>
__global__ void __launch_bounds__(NT)
k_fft_xy_r2c(const R *__restrict__ grid, cplx_t<R> *__restrict__ spec,
             const cplx_t<R> *__restrict__ tw_g) {
  using C = cplx_t<R>;
  using G = PlaneGeom<M, NS>;
  constexpr int H = G::H, K = G::K, PB = G::PB, KP = G::KP;
  static_assert(!ONE || NS == 1, "one plane buffer serves one work-group per plane");
  C *b0 = reinterpret_cast<C *>(f_smem), *b1 = b0 + G::BUF;
  C *twl = ONE ? b1 : b1 + G::BUF;
  for (int i = threadIdx.x; i < M; i += NT) twl[i] = tw_g[i];
  const long long z = blockIdx.x / NS;
  const int k0 = static_cast<int>(blockIdx.x % NS) * KP;  // first kx pencil of this work-group
  const R *plane = grid + z * M * M;
  // pencil b = rows 2b (real part) and 2b + 1 (imaginary part); all loads
  // are issued before the first LDS store
  constexpr int NP = H * M, PER = (NP + NT - 1) / NT;
  R re[PER], im[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + k * NT;  // i = b M + x
    if (NP % NT == 0 || i < NP) {
      const int b = i / M, x = i - b * M;
      re[k] = plane[(2 * b) * M + x];
      im[k] = plane[(2 * b + 1) * M + x];
    }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + k * NT;
    if (NP % NT == 0 || i < NP) {
      const int b = i / M, x = i - b * M;
      C v;
      v.x = re[k];
      v.y = im[k];
      b0[x * PB + b] = v;
    }
  }
  __syncthreads();
  C *X, *Y;
  if constexpr (ONE) {
    fft_batch_inplace<R, M, H, PB, NT, 0, 1>(b0, twl);
    X = Y = b0;
  } else {
    X = fft_batch_ct<R, M, H, PB, NT, 0, 1>(b0, b1, twl);
    Y = (X == b0) ? b1 : b0;
  }
  // Z = FFT(r1 + i r2): R1[k] = (Z[k] + conj Z[M-k]) / 2 (row 2b),
  // R2[k] = (Z[k] - conj Z[M-k]) / 2i (row 2b + 1); element y of this
  // work-group's pencil kx = k0 + kk (zero past the last one)
  const auto split = [&](int b, int kk, C &r1, C &r2) {
    const int k = k0 + kk;
    if (k < K) {
      const C zk = X[k * PB + b];
      const C zm = X[(k == 0 ? 0 : M - k) * PB + b];
      r1.x = R(0.5) * (zk.x + zm.x);
      r1.y = R(0.5) * (zk.y - zm.y);
      r2.x = R(0.5) * (zk.y + zm.y);
      r2.y = R(-0.5) * (zk.x - zm.x);
    } else {
      r1.x = r1.y = r2.x = r2.y = R(0);
    }
  };
  const C *S;
  if constexpr (ONE) {
    constexpr int NSP = H * KP, PS = (NSP + NT - 1) / NT;
    C r1v[PS], r2v[PS];
#pragma unroll
    for (int it = 0; it < PS; ++it) {
      const int i = threadIdx.x + it * NT;
      if (NSP % NT == 0 || i < NSP) split(i / KP, i % KP, r1v[it], r2v[it]);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < PS; ++it) {
      const int i = threadIdx.x + it * NT;
      if (NSP % NT == 0 || i < NSP) {
        const int b = i / KP, kk = i - b * KP;
        Y[(2 * b) * PB + kk] = r1v[it];
        Y[(2 * b + 1) * PB + kk] = r2v[it];
      }
    }
    __syncthreads();
    fft_batch_inplace<R, M, KP, PB, NT, 0, 1>(Y, twl);
    S = Y;
  } else {
    for (int i = threadIdx.x; i < H * KP; i += NT) {
      const int b = i / KP, kk = i - b * KP;
      C r1, r2;
      split(b, kk, r1, r2);
      Y[(2 * b) * PB + kk] = r1;
      Y[(2 * b + 1) * PB + kk] = r2;
    }
    __syncthreads();
    S = fft_batch_ct<R, M, KP, PB, NT, 0, 1>(Y, X, twl);
  }
  C *out = spec + (z * K + k0) * M;
  const int nk = min(KP, K - k0);
  for (int i = threadIdx.x; i < nk * M; i += NT) {
    const int kk = i / M, y = i - kk * M;
    out[i] = S[y * PB + kk];
  }
}

template <typename R, int M, int NT, int NS, bool ONE>
__global__ void __launch_bounds__(NT)
k_fft_yx_c2r(const cplx_t<R> *__restrict__ spec, R *__restrict__ grid,
             const cplx_t<R> *__restrict__ tw_g, EnergyOut eo) {
  using C = cplx_t<R>;
  using G = PlaneGeom<M, NS>;
  constexpr int K = G::K, PB = G::PB, HP = G::HP;
  static_assert(!ONE || NS == 1, "one plane buffer serves one work-group per plane");
  C *b0 = reinterpret_cast<C *>(f_smem), *b1 = b0 + G::BUF;
  C *twl = ONE ? b1 : b1 + G::BUF;
  for (int i = threadIdx.x; i < M; i += NT) twl[i] = tw_g[i];
  const long long z = blockIdx.x / NS;
  const int p0 = static_cast<int>(blockIdx.x % NS) * HP;  // first row pair of this work-group
  const C *in = spec + z * K * M;
  // conjugated on the way in: the inverse is conj(FFT(conj(.)))
  constexpr int NSP = K * M, PER = (NSP + NT - 1) / NT;
  C v[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + k * NT;  // i = kx M + y
    if (NSP % NT == 0 || i < NSP) v[k] = in[i];
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int i = threadIdx.x + k * NT;
    if (NSP % NT == 0 || i < NSP) {
      const int kx = i / M, y = i - kx * M;
      b0[y * PB + kx] = cconj(v[k]);
    }
  }
  __syncthreads();
  C *X, *Y;
  if constexpr (ONE) {
    fft_batch_inplace<R, M, K, PB, NT, 0, 1>(b0, twl);  // conj of the inverse along y
    X = Y = b0;
  } else {
    Y = fft_batch_ct<R, M, K, PB, NT, 0, 1>(b0, b1, twl);  // conj of the inverse along y
    X = (Y == b0) ? b1 : b0;
  }
  // row pair b = p0 + bb (rows 2b, 2b + 1) with half spectra R1, R2 (the
  // conjugates of Y's): Z[k] = R1[k] + i R2[k] on 0..M/2 and
  // conj(R1[M-k]) + i conj(R2[M-k]) above, stored conjugated for the
  // inverse along x
  const auto rebuild = [&](int bb, int k, C &zz, C &zc) {
    const int b = p0 + bb;
    const C r1 = cconj(Y[(2 * b) * PB + k]);
    const C r2 = cconj(Y[(2 * b + 1) * PB + k]);
    zz.x = r1.x - r2.y;
    zz.y = -(r1.y + r2.x);
    zc.x = r1.x + r2.y;
    zc.y = -(r2.x - r1.y);
  };
  const C *Zr;
  if constexpr (ONE) {
    constexpr int NRB = HP * K, PS = (NRB + NT - 1) / NT;
    C zzv[PS], zcv[PS];
#pragma unroll
    for (int it = 0; it < PS; ++it) {
      const int i = threadIdx.x + it * NT;
      if (NRB % NT == 0 || i < NRB) rebuild(i / K, i % K, zzv[it], zcv[it]);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < PS; ++it) {
      const int i = threadIdx.x + it * NT;
      if (NRB % NT == 0 || i < NRB) {
        const int bb = i / K, k = i - bb * K;
        X[k * PB + bb] = zzv[it];
        if (k > 0 && k < M - k) X[(M - k) * PB + bb] = zcv[it];
      }
    }
    __syncthreads();
    fft_batch_inplace<R, M, HP, PB, NT, 0, 1>(X, twl);
    Zr = X;
  } else {
    for (int i = threadIdx.x; i < HP * K; i += NT) {
      const int bb = i / K, k = i - bb * K;
      C zz, zc;
      rebuild(bb, k, zz, zc);
      X[k * PB + bb] = zz;
      if (k > 0 && k < M - k) X[(M - k) * PB + bb] = zc;
    }
    __syncthreads();
    Zr = fft_batch_ct<R, M, HP, PB, NT, 0, 1>(X, Y, twl);
  }
  R *out = grid + z * M * M;
  for (int i = threadIdx.x; i < HP * M; i += NT) {
    const int bb = i / M, x = i - bb * M, b = p0 + bb;
    const C zz = Zr[x * PB + bb];
    out[(2 * b) * M + x] = zz.x;       // real part of the conjugate
    out[(2 * b + 1) * M + x] = -zz.y;  // imaginary part of the conjugate
  }
  if (blockIdx.x == 0 && eo.E) write_energy<NT>(eo);
}

// ------------------------------------------ z pass with scaling and energy

// With ik >= 0 the pass writes, instead of w G^, the spectrum of one
// component of the field -grad Phi: -i k_ik w G^ (section 3.1, the ik
// differentiation), into out, with no energy; the Nyquist plane of that axis
// is zero (its derivative is not defined on the grid).  Otherwise out = in
// and the energy partials go to epart.
template <typename R, int MC, int LGBC>
__global__ void __launch_bounds__(zpass_threads(MC))
k_fft_z_scale(const cplx_t<R> *in, cplx_t<R> *out, FftPlan pl, int lgB,
              const cplx_t<R> *__restrict__ tw_g, const double *__restrict__ axis_f,
              const double *__restrict__ axis_k2, double wscale, double *__restrict__ epart,
              int ik, double two_pi_over_L) {
  using C = cplx_t<R>;
  constexpr int ZT = zpass_threads(MC), ZPT = 16 * kThreads / ZT;
  constexpr bool CT = MC > 0;
  const int M = CT ? MC : pl.M;
  const int lgb = CT ? LGBC : lgB;
  const int K = M / 2 + 1, B = 1 << lgb;
  const int npen = M * K;
  C *b0 = reinterpret_cast<C *>(f_smem), *b1 = CT ? b0 : b0 + M * B;  // compiled M: one buffer
  C *twl = b1 + M * B;  // twiddles staged in LDS
  // the per-axis tables of the influence function too, so that the scaling
  // step between the two transforms needs no global memory round trip
  double *af = reinterpret_cast<double *>(twl + M), *ak2 = af + M;
  for (int i = threadIdx.x; i < M; i += ZT) {
    twl[i] = tw_g[i];
    af[i] = axis_f[i];
    ak2[i] = axis_k2[i];
  }
  const int c0 = xcd_local(blockIdx.x, gridDim.x) * B;  // pencils c = kx M + ky, contiguous in a z plane
  const long long zs = static_cast<long long>(M) * K;
  {
    C v[ZPT];
#pragma unroll
    for (int k = 0; k < ZPT; ++k) {
      const int i = threadIdx.x + k * ZT;
      const int z = i >> lgb, b = i & (B - 1);
      if (i < M * B && c0 + b < npen) {
        v[k] = in[z * zs + c0 + b];
      } else {
        v[k].x = v[k].y = R(0);
      }
    }
#pragma unroll
    for (int k = 0; k < ZPT; ++k) {
      const int i = threadIdx.x + k * ZT;
      if (i < M * B) b0[i] = v[k];
    }
  }
  __syncthreads();
  C *Z = fft_pencils<R, MC, LGBC, ZT>(b0, b1, lgb, pl, twl);
  C *other = (Z == b0) ? b1 : b0;  // Z itself for compiled M
  // signed wave number of an axis index (0 on the Nyquist plane)
  const auto signed_k = [&](int n) {
    return 2 * n == M ? 0.0 : two_pi_over_L * static_cast<double>(2 * n < M ? n : n - M);
  };

  double e = 0.0;
  for (int i = threadIdx.x; i < M * B; i += ZT) {
    const int kz = i >> lgb, b = i & (B - 1);
    const int c = c0 + b;
    C v = Z[i];
    if (c < npen) {
      const int kx = div_M<MC>(c, pl), ky = c - kx * M;
      const double k2 = ak2[kx] + ak2[ky] + ak2[kz];
      const double w = (kx == 0 && ky == 0 && kz == 0)
                           ? 0.0
                           : wscale * af[kx] * af[ky] * af[kz] / k2;
      const double mu = (kx == 0 || 2 * kx == M) ? 1.0 : 2.0;
      const double re = static_cast<double>(v.x), im = static_cast<double>(v.y);
      e += 0.5 * mu * w * (re * re + im * im);
      const R wr = static_cast<R>(w);
      v.x = v.x * wr;  // conjugated for the inverse transform
      v.y = -(v.y * wr);
      if (ik >= 0) {
        // conj(-i k w G^) = i k conj(w G^): (a + i b) -> k (-b + i a)
        const R kd = static_cast<R>(signed_k(ik == 0 ? kx : (ik == 1 ? ky : kz)));
        const R a = v.x;
        v.x = -v.y * kd;
        v.y = a * kd;
      }
    } else {
      v.x = v.y = R(0);
    }
    Z[i] = v;  // holds conj(w * G^)
  }
  __syncthreads();
  const C *Y = fft_pencils<R, MC, LGBC, ZT>(Z, other, lgb, pl, twl);
  for (int i = threadIdx.x; i < M * B; i += ZT) {
    const int z = i >> lgb, b = i & (B - 1);
    if (c0 + b < npen) out[z * zs + c0 + b] = cconj(Y[i]);
  }
  if (!epart) return;  // uniform across the work-group

  // energy: one partial per block (a fixed tree over the lanes of each wave,
  // then the waves in order), added in a fixed order by the next pass
  e = wave_reduce0(e, [](double a, double b) { return a + b; });
  __shared__ double wred[ZT / 64];
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < ZT / 64; ++w) s += wred[w];
    epart[blockIdx.x] = s;
  }
}

// The three-launch sequence with the fused plane passes (compile-time M
// whose plane buffers fit in LDS: twice with NSF and NSI work-groups per
// plane, or, ONE, once with one work-group per plane).
template <typename R, int MC, bool ONE>
hipError_t fft_run_planes(se_plan &p, double *E_dev) {
  using C = cplx_t<R>;
  constexpr int LZ = fft_lgb(MC, sizeof(R), kPassZ);
  constexpr int NT = plane_threads(MC);
  constexpr int NSF = ONE ? 1 : kPlaneSplitFwd, NSI = ONE ? 1 : kPlaneSplitInv;
  constexpr size_t lds = ONE ? plane1_lds_bytes<R, MC>() : plane_lds_bytes<R, MC>();
  constexpr unsigned nfwd = MC * NSF, ninv = MC * NSI;
  if (MC != p.prm.M || LZ != p.fft_lgb[kPassZ] || p.fft_threads != kThreads)
    return hipErrorInvalidValue;
  hipError_t e;
  if (lds > 65536) {
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(
                                     &k_fft_xy_r2c<R, MC, NT, NSF, ONE>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 static_cast<int>(lds))) != hipSuccess)
      return e;
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(
                                     &k_fft_yx_c2r<R, MC, NT, NSI, ONE>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 static_cast<int>(lds))) != hipSuccess)
      return e;
  }
  const size_t lds_z = sizeof(C) * (MC * (1 << LZ) + MC) + 2 * sizeof(double) * MC;
  C *spec = static_cast<C *>(p.buf.spec);
  const C *tw = static_cast<const C *>(p.buf.twiddle);
  stage_begin(p, SE_STAGE_FFT_XY);
  launch_on(&p, k_fft_xy_r2c<R, MC, NT, NSF, ONE>, nfwd, NT, lds, p.stream, static_cast<const R *>(p.buf.grid), spec, tw);
  stage_end(p, SE_STAGE_FFT_XY);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const double tpl = 2.0 * M_PI / p.prm.L;
  const EnergyOut none{nullptr, 0, nullptr, 0, 0.0, nullptr};
  if (p.prm.flags & SE_FLAG_IK_FORCE) {
    // the three field components first (they read the forward spectrum,
    // which the potential's z pass then overwrites); not timed
    C *spec2 = static_cast<C *>(p.buf.spec2);
    for (int d = 0; d < 3; ++d) {
      launch_on(&p, k_fft_z_scale<R, MC, LZ>, p.zfft_blocks, zpass_threads(MC), lds_z, p.stream, 
          spec, spec2, p.fft, LZ, tw, static_cast<const double *>(p.buf.axis_f),
          static_cast<const double *>(p.buf.axis_k2), p.wscale, nullptr, d, tpl);
      launch_on(&p, k_fft_yx_c2r<R, MC, NT, NSI, ONE>, ninv, NT, lds, p.stream, 
          spec2, static_cast<R *>(p.buf.field) + static_cast<long long>(d) * MC * MC * MC, tw,
          none);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  stage_begin(p, SE_STAGE_FFT_Z_SCALE);
  launch_on(&p, k_fft_z_scale<R, MC, LZ>, p.zfft_blocks, zpass_threads(MC), lds_z, p.stream, 
      spec, spec, p.fft, LZ, tw, static_cast<const double *>(p.buf.axis_f),
      static_cast<const double *>(p.buf.axis_k2), p.wscale, p.buf.part + p.bin_blocks, -1, tpl);
  stage_end(p, SE_STAGE_FFT_Z_SCALE);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const double self_coef = (p.prm.flags & SE_FLAG_ADD_SELF) ? -p.prm.xi / sqrt(M_PI) : 0.0;
  const EnergyOut eo{p.buf.part + p.bin_blocks, p.zfft_blocks, p.buf.part, p.bin_parts, self_coef,
                     E_dev};
  stage_begin(p, SE_STAGE_IFFT_YX);
  launch_on(&p, k_fft_yx_c2r<R, MC, NT, NSI, ONE>, ninv, NT, lds, p.stream, spec, static_cast<R *>(p.buf.grid), tw, eo);
  stage_end(p, SE_STAGE_IFFT_YX);
  return hipGetLastError();
}

template <typename R, int MC>
hipError_t fft_run(se_plan &p, double *E_dev) {
  static_assert(MC == 0 || fft_compiled(MC), "every compiled grid size is in kCompiledM");
  if constexpr (MC > 0 && plane_fits<R, MC>()) return fft_run_planes<R, MC, false>(p, E_dev);
  if constexpr (MC > 0 && !plane_fits<R, MC>() && plane1_fits<R, MC>())
    return fft_run_planes<R, MC, true>(p, E_dev);
  // compiled pencils per work-group of each pass (ignored for MC = 0)
  constexpr int LX = MC > 0 ? fft_lgb(MC, sizeof(R), kPassX) : 0;
  constexpr int LY = MC > 0 ? fft_lgb(MC, sizeof(R), kPassY) : 0;
  constexpr int LZ = MC > 0 ? fft_lgb(MC, sizeof(R), kPassZ) : 0;
  using C = cplx_t<R>;
  const int M = p.prm.M, K = M / 2 + 1;
  const int lx = p.fft_lgb[kPassX], ly = p.fft_lgb[kPassY], lz = p.fft_lgb[kPassZ];
  // The compiled kernels assume this M and these batches; the grids below
  // are sized from the plan's.
  if (MC > 0 && (MC != M || LX != lx || LY != ly || LZ != lz || p.fft_threads != kThreads))
    return hipErrorInvalidValue;
  // the plan sized the batches for one buffer exactly when M is compiled
  if (MC == 0 && fft_compiled(M)) return hipErrorInvalidValue;
  const int Bx = 1 << lx, By = 1 << ly;
  // pencil buffers: one for compiled M, two for the run-time plan
  const auto lds_of = [M](int lg) { return sizeof(C) * ((MC > 0 ? 1 : 2) * M * (1 << lg) + M); };
  const auto lds_zof = [M, lds_of](int lg) { return lds_of(lg) + 2 * sizeof(double) * M; };
  C *spec = static_cast<C *>(p.buf.spec);
  const C *tw = static_cast<const C *>(p.buf.twiddle);
  const int xblocks = (M * M + 2 * Bx - 1) / (2 * Bx);
  hipError_t e = hipSuccess;
  stage_begin(p, SE_STAGE_FFT_X);
  launch_on(&p, k_fft_x_r2c<R, MC, LX>, xblocks, xy_threads<R>(MC), lds_of(lx), p.stream, 
      static_cast<const R *>(p.buf.grid), spec, p.fft, lx, tw);
  stage_end(p, SE_STAGE_FFT_X);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const unsigned yg = static_cast<unsigned>((M * K + By - 1) / By);
  const EnergyOut none{nullptr, 0, nullptr, 0, 0.0, nullptr};
  stage_begin(p, SE_STAGE_FFT_Y);
  launch_on(&p, k_fft_y<R, MC, LY, false>, yg, xy_threads<R>(MC), lds_of(ly), p.stream, spec, p.fft, ly, tw, none);
  stage_end(p, SE_STAGE_FFT_Y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const double tpl = 2.0 * M_PI / p.prm.L;
  if (p.prm.flags & SE_FLAG_IK_FORCE) {
    // the three field components first (they read the forward spectrum,
    // which the potential's z pass then overwrites); not timed
    C *spec2 = static_cast<C *>(p.buf.spec2);
    for (int d = 0; d < 3; ++d) {
      launch_on(&p, k_fft_z_scale<R, MC, LZ>, p.zfft_blocks, zpass_threads(MC), lds_zof(lz), p.stream, 
          spec, spec2, p.fft, lz, tw, static_cast<const double *>(p.buf.axis_f),
          static_cast<const double *>(p.buf.axis_k2), p.wscale, nullptr, d, tpl);
      launch_on(&p, k_fft_y<R, MC, LY, true>, yg, xy_threads<R>(MC), lds_of(ly), p.stream, spec2, p.fft, ly, tw,
                                                                           none);
      launch_on(&p, k_fft_x_c2r<R, MC, LX>, xblocks, xy_threads<R>(MC), lds_of(lx), p.stream, 
          spec2, static_cast<R *>(p.buf.field) + static_cast<long long>(d) * M * M * M, p.fft, lx,
          tw);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  stage_begin(p, SE_STAGE_FFT_Z_SCALE);
  launch_on(&p, k_fft_z_scale<R, MC, LZ>, p.zfft_blocks, zpass_threads(MC), lds_zof(lz), p.stream, 
      spec, spec, p.fft, lz, tw, static_cast<const double *>(p.buf.axis_f),
      static_cast<const double *>(p.buf.axis_k2), p.wscale, p.buf.part + p.bin_blocks, -1, tpl);
  stage_end(p, SE_STAGE_FFT_Z_SCALE);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const double self_coef = (p.prm.flags & SE_FLAG_ADD_SELF) ? -p.prm.xi / sqrt(M_PI) : 0.0;
  const EnergyOut eo{p.buf.part + p.bin_blocks, p.zfft_blocks, p.buf.part, p.bin_parts, self_coef,
                     E_dev};
  stage_begin(p, SE_STAGE_IFFT_Y);
  launch_on(&p, k_fft_y<R, MC, LY, true>, yg, xy_threads<R>(MC), lds_of(ly), p.stream, spec, p.fft, ly, tw, eo);
  stage_end(p, SE_STAGE_IFFT_Y);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  stage_begin(p, SE_STAGE_IFFT_X);
  launch_on(&p, k_fft_x_c2r<R, MC, LX>, xblocks, xy_threads<R>(MC), lds_of(lx), p.stream, 
      spec, static_cast<R *>(p.buf.grid), p.fft, lx, tw);
  stage_end(p, SE_STAGE_IFFT_X);
  return hipGetLastError();
}

// Grid sizes with a compile-time FFT; any other size runs the generic passes.
template <typename R>
hipError_t fft_impl(se_plan &p, double *E_dev) {
  switch (p.prm.M) {
    case 16: return fft_run<R, 16>(p, E_dev);
    case 24: return fft_run<R, 24>(p, E_dev);
    case 32: return fft_run<R, 32>(p, E_dev);
    case 40: return fft_run<R, 40>(p, E_dev);
    case 48: return fft_run<R, 48>(p, E_dev);
    case 64: return fft_run<R, 64>(p, E_dev);
    case 80: return fft_run<R, 80>(p, E_dev);
    case 96: return fft_run<R, 96>(p, E_dev);
    case 120: return fft_run<R, 120>(p, E_dev);
    case 128: return fft_run<R, 128>(p, E_dev);
    case 144: return fft_run<R, 144>(p, E_dev);
    case 160: return fft_run<R, 160>(p, E_dev);
    case 192: return fft_run<R, 192>(p, E_dev);
    case 216: return fft_run<R, 216>(p, E_dev);
    case 240: return fft_run<R, 240>(p, E_dev);
    case 256: return fft_run<R, 256>(p, E_dev);
    case 288: return fft_run<R, 288>(p, E_dev);
    case 320: return fft_run<R, 320>(p, E_dev);
    case 384: return fft_run<R, 384>(p, E_dev);
    case 432: return fft_run<R, 432>(p, E_dev);
    case 480: return fft_run<R, 480>(p, E_dev);
    case 512: return fft_run<R, 512>(p, E_dev);
    default: return fft_run<R, 0>(p, E_dev);
  }
}

}  // namespace

hipError_t launch_fft_forward_scale_inverse(se_plan &plan, double *E_dev) {
  return plan.prm.dtype == SE_FP64 ? fft_impl<double>(plan, E_dev)
                                   : fft_impl<float>(plan, E_dev);
}

}  // namespace sek
