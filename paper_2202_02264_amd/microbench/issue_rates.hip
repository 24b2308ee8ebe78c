// Issue-rate microbenchmark of the VALU instructions that price the pair-row
// kernel's roofline on gfx950: v_fma_f32, v_exp_f32, the two interleaved, and
// the pair loop itself (v_sub_f32, v_fma_f32, v_exp_f32, v_add_f32 on
// independent rows).  Each kernel runs 8 independent dependency chains per
// lane so that latency is hidden; counts are known at compile time.  Prints
// one JSON line with lane-instructions per second (pairs per second for the
// pair loop) and the chip's nominal single-rate VALU issue rate.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

constexpr int kChains = 8;
constexpr int kIters = 2048;
constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_fma(float* out, float a, float b) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 1e-3f + c;
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], a, b);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_exp(float* out, float a) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = -(threadIdx.x & 7) * 0.1f - c * 0.01f;
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);  // stays in [0.5, 1]
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * kBlock + threadIdx.x] = s * a;
}

// one v_exp_f32 and one v_fma_f32 per chain and iteration, independent
__global__ __launch_bounds__(kBlock) void k_exp_fma(float* out, float a, float b) {
  float x[kChains], y[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    x[c] = -(threadIdx.x & 7) * 0.1f - c * 0.01f;
    y[c] = threadIdx.x * 1e-3f + c;
  }
  for (int i = 0; i < kIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      x[c] = __builtin_amdgcn_exp2f(-x[c]);
      y[c] = __builtin_fmaf(y[c], a, b);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c] + y[c];
  out[blockIdx.x * kBlock + threadIdx.x] = s;
}

// The pair loop of the rows kernel at d_x = 1: per (row, column) pair
// d = u - v, s = beta - d^2, acc += 2^s, with u, beta wave-uniform.
__global__ __launch_bounds__(kBlock) void k_pairs(float* out, const float* __restrict__ col) {
  float v[kChains], acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    v[c] = threadIdx.x * 1e-3f + c * 0.1f;
    acc[c] = 0.f;
  }
  for (int i = 0; i < kIters; i += 32) {
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      const float u = col[2 * ((i + j) & 63)], beta = col[2 * ((i + j) & 63) + 1];
#pragma unroll
      for (int c = 0; c < kChains; ++c) {
        const float d = u - v[c];
        acc[c] += __builtin_amdgcn_exp2f(__builtin_fmaf(-d, d, beta));
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c];
  out[blockIdx.x * kBlock + threadIdx.x] = s;
}

// Philox4x64-10 blocks (the leaf kernel's generator) per second: kChains
// independent blocks per lane and iteration, their words folded into an
// accumulator.
__device__ __forceinline__ void philox_block(uint64_t& c0, uint64_t& c1, uint64_t& c2,
                                             uint64_t& c3, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B97F4A7C15ull;
      k1 += 0xBB67AE8584CAA73Bull;
    }
    const uint64_t hi0 = __umul64hi(0xD2E7470EE14C6C93ull, c0), lo0 = 0xD2E7470EE14C6C93ull * c0;
    const uint64_t hi1 = __umul64hi(0xCA5A826395121157ull, c2), lo1 = 0xCA5A826395121157ull * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

constexpr int kPhiloxIters = 64;

__global__ __launch_bounds__(kBlock) void k_philox(uint64_t* out, uint64_t seed) {
  uint64_t acc = 0;
  const uint64_t n = blockIdx.x * kBlock + threadIdx.x;
  for (int i = 0; i < kPhiloxIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      uint64_t c0 = n, c1 = (uint64_t)i, c2 = 2, c3 = (uint64_t)c;
      philox_block(c0, c1, c2, c3, seed, 0x64534D43ull);
      acc ^= c0 ^ c1 ^ c2 ^ c3;
    }
  }
  out[n] = acc;
}

// Box-Muller pairs per second: fp64 (log, sqrt, cos, sin in double, as the
// leaf kernel of fp64 plans) and fp32 (the hardware v_log_f32, v_sqrt_f32 and
// v_cos_f32 / v_sin_f32, which take revolutions).
__global__ __launch_bounds__(kBlock) void k_box_muller64(double* out) {
  double acc = 0.0;
  const uint64_t n = blockIdx.x * kBlock + threadIdx.x;
  for (int i = 0; i < kPhiloxIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      const uint64_t wa = (n * 0x9E3779B97F4A7C15ull) ^ (uint64_t)(i * 8 + c) * 0xBB67AE8584CAA73Bull;
      const uint64_t wb = wa * 0xD2E7470EE14C6C93ull;
      const double ua = (double)((wa >> 11) + 1ull) * 0x1p-53, ub = (double)(wb >> 11) * 0x1p-53;
      const double rad = sqrt(-2.0 * log(ua)), th = 2.0 * 3.141592653589793 * ub;
      acc += rad * cos(th) + rad * sin(th);
    }
  }
  out[n] = acc;
}

__global__ __launch_bounds__(kBlock) void k_box_muller32(double* out) {
  float acc = 0.0f;
  const uint64_t n = blockIdx.x * kBlock + threadIdx.x;
  for (int i = 0; i < kPhiloxIters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      const uint64_t wa = (n * 0x9E3779B97F4A7C15ull) ^ (uint64_t)(i * 8 + c) * 0xBB67AE8584CAA73Bull;
      const uint64_t wb = wa * 0xD2E7470EE14C6C93ull;
      const float ua = (float)((double)((wa >> 11) + 1ull) * 0x1p-53);
      const float ub = (float)((double)(wb >> 11) * 0x1p-53);
      const float rad = __builtin_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(ua));
      acc += rad * __builtin_amdgcn_cosf(ub) + rad * __builtin_amdgcn_sinf(ub);
    }
  }
  out[n] = acc;
}

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                   \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                \
      return 1;                                                               \
    }                                                                         \
  } while (0)

int main(int argc, char** argv) {
  int dev = 0;
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, dev));
  const int cus = prop.multiProcessorCount;
  const int blocks = cus * 16;  // 16 workgroups of 4 waves per CU: 16 waves per SIMD requested
  const size_t threads = (size_t)blocks * kBlock;
  float *out, *col;
  uint64_t* out64;
  CHECK(hipMalloc(&out, threads * sizeof(float)));
  CHECK(hipMalloc(&out64, threads * sizeof(uint64_t)));
  CHECK(hipMalloc(&col, 128 * sizeof(float)));
  float hc[128];
  for (int i = 0; i < 128; ++i) hc[i] = (i & 1) ? -0.5f : 0.01f * i;
  CHECK(hipMemcpy(col, hc, sizeof hc, hipMemcpyHostToDevice));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const int reps = 20;
  auto timeit = [&](auto launch) -> double {
    launch();  // warm-up (code object load)
    CHECK(hipDeviceSynchronize());
    CHECK(hipEventRecord(e0, 0));
    for (int r = 0; r < reps; ++r) launch();
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    return ms * 1e-3 / reps;
  };
  const double per_thread = (double)kIters * kChains;
  const double t_fma = timeit([&] { k_fma<<<blocks, kBlock>>>(out, 0.999f, 1e-3f); });
  const double t_exp = timeit([&] { k_exp<<<blocks, kBlock>>>(out, 1.0f); });
  const double t_mix = timeit([&] { k_exp_fma<<<blocks, kBlock>>>(out, 0.999f, 1e-3f); });
  const double t_pair = timeit([&] { k_pairs<<<blocks, kBlock>>>(out, col); });
  const double t_philox = timeit([&] { k_philox<<<blocks, kBlock>>>(out64, 12345ull); });
  CHECK(hipGetLastError());
  const double philox_rate = threads * (double)kPhiloxIters * kChains / t_philox;
  const double t_bm64 = timeit([&] { k_box_muller64<<<blocks, kBlock>>>((double*)out64); });
  const double t_bm32 = timeit([&] { k_box_muller32<<<blocks, kBlock>>>((double*)out64); });
  CHECK(hipGetLastError());
  const double bm64_rate = threads * (double)kPhiloxIters * kChains / t_bm64;
  const double bm32_rate = threads * (double)kPhiloxIters * kChains / t_bm32;
  const double fma_rate = threads * per_thread / t_fma;
  const double exp_rate = threads * per_thread / t_exp;
  const double mix_rate = threads * 2.0 * per_thread / t_mix;  // lane-instructions/s, both kinds
  const double pair_rate = threads * per_thread / t_pair;
  const double clock_ghz = prop.clockRate * 1e-6;
  const double nominal = (double)cus * 4 * 16 * clock_ghz * 1e9;
  printf("{\"device\": \"%s\", \"cus\": %d, \"clock_ghz\": %.3f, "
         "\"nominal_lane_instr_per_s\": %.4e, \"v_fma_f32_per_s\": %.4e, "
         "\"v_exp_f32_per_s\": %.4e, \"exp_plus_fma_lane_instr_per_s\": %.4e, "
         "\"pair_loop_pairs_per_s\": %.4e, "
         "\"exp_slots_vs_fma\": %.3f, \"mix_time_vs_sum\": %.3f, "
         "\"pair_slots_at_fma_rate\": %.3f, \"philox4x64_10_blocks_per_s\": %.4e, "
         "\"philox_block_slots_at_fma_rate\": %.1f, \"box_muller_f64_pairs_per_s\": %.4e, "
         "\"box_muller_f32_pairs_per_s\": %.4e}\n",
         prop.name, cus, clock_ghz, nominal, fma_rate, exp_rate, mix_rate, pair_rate,
         fma_rate / exp_rate, t_mix / (t_fma + t_exp), fma_rate / pair_rate, philox_rate,
         fma_rate / philox_rate, bm64_rate, bm32_rate);
  return 0;
}
