// Issue-rate microbenchmarks for gfx950: the cost, in cycles of the
// nominal 2.4 GHz clock per wave64 instruction per SIMD, of the three
// instructions every kernel evaluation of the transforms needs at the least
// (an FP32 FMA, the hardware sine / cosine, and one
// v_mfma_f32_32x32x16_bf16 product).  The transforms' issue ceiling is
// derived from these costs, the chip's 1024 SIMDs and the clock.
//
// Each kernel runs independent dependency chains per lane (enough of them,
// with several waves per SIMD, that latency is hidden and issue binds), on
// a grid of `waves_per_simd` waves on every SIMD of the device; the elapsed
// time of the launch over the instructions each SIMD issued gives the cost.
// The only memory access is one store per lane of the chains' result, so
// the compiler keeps the arithmetic.
#include <hip/hip_runtime.h>
#include <math.h>

#include "ash_ubench.h"

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;   // 4 waves per block
constexpr int kChains = 16;     // independent chains per lane

__global__ __launch_bounds__(kThreads) void k_fma(int iters, float* out) {
  float a[kChains];
  const float x = 1.0f + 1e-7f * threadIdx.x;
#pragma unroll
  for (int c = 0; c < kChains; ++c) a[c] = x + c;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = fmaf(a[c], 0.9999999f, 1e-8f);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += a[c];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// alternating sine and cosine (turns), as the transforms issue them
__global__ __launch_bounds__(kThreads) void k_trans(int iters, float* out) {
  float a[kChains];
  const float x = 1e-3f * threadIdx.x;
#pragma unroll
  for (int c = 0; c < kChains; ++c) a[c] = x + 0.01f * c;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; c += 2) {
      a[c] = __builtin_amdgcn_sinf(a[c]);
      a[c + 1] = __builtin_amdgcn_cosf(a[c + 1]);
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += a[c];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

constexpr int kAcc = 2;  // independent accumulators per wave

__global__ __launch_bounds__(kThreads) void k_mfma(int iters, float* out) {
  const unsigned v = 0x3F803F80u + threadIdx.x;  // bf16 pairs near 1
  const u32x4 a = {v, v ^ 1u, v ^ 2u, v ^ 3u};
  const u32x4 b = {v ^ 4u, v ^ 5u, v ^ 6u, v ^ 7u};
  floatx16 acc[kAcc];
#pragma unroll
  for (int k = 0; k < kAcc; ++k)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[k][i] = 0.0f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kAcc; ++k)
      acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
          __builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
          acc[k], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < kAcc; ++k)
#pragma unroll
    for (int i = 0; i < 16; ++i) s += acc[k][i];
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// Shortest of three timed launches after one untimed launch (code load,
// clock ramp).
template <typename K>
hipError_t time_kernel(K kern, int blocks, int iters, float* out,
                       float* ms_out) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best = -1.0f;
  for (int r = 0; r < 4 && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, nullptr);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), 0, nullptr,
                         iters, out);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && r > 0 && (best < 0.0f || ms < best)) best = ms;
  }
  *ms_out = best;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}


// The irreducible instruction mix of one 32 x 32 block of evaluations of
// the transforms, without their loads: G dependent matrix-core products
// give 16 phases per lane, then per phase (range reduction when kReduce)
// a sine and a cosine, and either two FMAs into the lane's accumulators
// (forward and adjoint) or, with kMoments, 8 further products whose B
// operands are built from the sines and cosines (the moment transform).
// One operand word changes every iteration so that nothing is hoisted.
template <int G, bool kReduce, bool kMoments>
__global__ __launch_bounds__(kThreads) void k_mix(int iters, float* out) {
  const unsigned v = 0x3C003C00u + (threadIdx.x & 63);
  u32x4 a[G], b[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    a[g] = u32x4{v, v ^ 1u, v ^ 2u, v ^ 3u};
    b[g] = u32x4{v ^ 4u, v ^ 5u, v ^ 6u, v ^ 7u};
  }
  float er[16], ei[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) er[k] = ei[k] = 0.0f;
  floatx16 macc;
#pragma unroll
  for (int k = 0; k < 16; ++k) macc[k] = 0.0f;
  const float m = 0.5f + 1e-3f * (threadIdx.x & 63);
  for (int i = 0; i < iters; ++i) {
    b[0][0] += 1u;
    floatx16 th;
#pragma unroll
    for (int k = 0; k < 16; ++k) th[k] = 0.0f;
#pragma unroll
    for (int g = 0; g < G; ++g)
      th = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
          __builtin_bit_cast(bf16x8, a[g]), __builtin_bit_cast(bf16x8, b[g]),
          th, 0, 0, 0);
    float c[16], s[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const float r = kReduce ? __builtin_amdgcn_fractf(th[k]) : th[k];
      c[k] = __builtin_amdgcn_cosf(r);
      s[k] = __builtin_amdgcn_sinf(r);
    }
    if (kMoments) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const u32x4 cc = {__float_as_uint(c[8 * q]), __float_as_uint(c[8 * q + 2]),
                          __float_as_uint(c[8 * q + 4]), __float_as_uint(c[8 * q + 6])};
        const u32x4 cl = {__float_as_uint(c[8 * q + 1]), __float_as_uint(c[8 * q + 3]),
                          __float_as_uint(c[8 * q + 5]), __float_as_uint(c[8 * q + 7])};
        const u32x4 sc = {__float_as_uint(s[8 * q]), __float_as_uint(s[8 * q + 2]),
                          __float_as_uint(s[8 * q + 4]), __float_as_uint(s[8 * q + 6])};
        const u32x4 sl = {__float_as_uint(s[8 * q + 1]), __float_as_uint(s[8 * q + 3]),
                          __float_as_uint(s[8 * q + 5]), __float_as_uint(s[8 * q + 7])};
        macc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            __builtin_bit_cast(bf16x8, a[0]), __builtin_bit_cast(bf16x8, cc), macc, 0, 0, 0);
        macc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            __builtin_bit_cast(bf16x8, a[0]), __builtin_bit_cast(bf16x8, cl), macc, 0, 0, 0);
        macc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            __builtin_bit_cast(bf16x8, a[0]), __builtin_bit_cast(bf16x8, sc), macc, 0, 0, 0);
        macc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            __builtin_bit_cast(bf16x8, a[0]), __builtin_bit_cast(bf16x8, sl), macc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        er[k] = fmaf(m, c[k], er[k]);
        ei[k] = fmaf(m, s[k], ei[k]);
      }
    }
  }
  float t = 0.0f;
#pragma unroll
  for (int k = 0; k < 16; ++k) t += er[k] + ei[k] + macc[k];
  out[blockIdx.x * kThreads + threadIdx.x] = t;
}

template <int G, bool kReduce, bool kMoments>
hipError_t mix_launch(int blocks, int iters, float* out, float* ms) {
  return time_kernel(k_mix<G, kReduce, kMoments>, blocks, iters, out, ms);
}

template <bool kReduce, bool kMoments>
hipError_t mix_dispatch(int G, int blocks, int iters, float* out, float* ms) {
  switch (G) {
#define X(n) \
  case n:    \
    return mix_launch<n, kReduce, kMoments>(blocks, iters, out, ms);
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

extern "C" int ash_ubench_issue(int device, int waves_per_simd,
                                ash_issue_rates* out) {
  if (!out || waves_per_simd < 1 || waves_per_simd > 8) return -1;
  hipError_t e = hipSetDevice(device);
  int n_cu = 0;
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount,
                              device);
  if (e != hipSuccess || n_cu <= 0) return -6;
  const int simds = 4 * n_cu;
  const int blocks = simds * waves_per_simd / (kThreads / 64);
  float* buf = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&buf),
                (size_t)blocks * kThreads * sizeof(float)) != hipSuccess)
    return -5;
  // instructions each SIMD issues: waves on it x iterations x instructions
  // per iteration
  const double nominal_hz = 2.4e9;
  const int it_valu = 16384, it_mfma = 8192;
  float ms[3] = {0, 0, 0};
  e = time_kernel(k_fma, blocks, it_valu, buf, &ms[0]);
  if (e == hipSuccess) e = time_kernel(k_trans, blocks, it_valu, buf, &ms[1]);
  if (e == hipSuccess) e = time_kernel(k_mfma, blocks, it_mfma, buf, &ms[2]);
  (void)hipFree(buf);
  if (e != hipSuccess) return -6;
  const double per_simd_valu = (double)waves_per_simd * it_valu * kChains;
  const double per_simd_mfma = (double)waves_per_simd * it_mfma * kAcc;
  out->simds = simds;
  out->nominal_clock_hz = nominal_hz;
  out->fma_cycles = ms[0] * 1e-3 * nominal_hz / per_simd_valu;
  out->trans_cycles = ms[1] * 1e-3 * nominal_hz / per_simd_valu;
  out->mfma_cycles = ms[2] * 1e-3 * nominal_hz / per_simd_mfma;
  out->ms[0] = ms[0];
  out->ms[1] = ms[1];
  out->ms[2] = ms[2];
  return 0;
}

extern "C" int ash_ubench_mix(int device, int groups, int reduce, int moments,
                              int waves_per_simd, double* evals_per_s) {
  if (!evals_per_s || groups < 1 || groups > 12 || waves_per_simd < 1 ||
      waves_per_simd > 8)
    return -1;
  hipError_t e = hipSetDevice(device);
  int n_cu = 0;
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount,
                              device);
  if (e != hipSuccess || n_cu <= 0) return -6;
  const int blocks = 4 * n_cu * waves_per_simd / (kThreads / 64);
  float* buf = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&buf),
                (size_t)blocks * kThreads * sizeof(float)) != hipSuccess)
    return -5;
  const int iters = 2048;
  float ms = 0.0f;
  if (moments)
    e = reduce ? mix_dispatch<true, true>(groups, blocks, iters, buf, &ms)
               : mix_dispatch<false, true>(groups, blocks, iters, buf, &ms);
  else
    e = reduce ? mix_dispatch<true, false>(groups, blocks, iters, buf, &ms)
               : mix_dispatch<false, false>(groups, blocks, iters, buf, &ms);
  (void)hipFree(buf);
  if (e != hipSuccess || !(ms > 0.0f)) return -6;
  // 1024 evaluations per wave per iteration
  *evals_per_s = (double)blocks * (kThreads / 64) * iters * 1024.0 / (ms * 1e-3);
  return 0;
}
