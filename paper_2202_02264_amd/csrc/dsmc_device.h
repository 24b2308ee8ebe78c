// Device helpers: Philox4x64-10, Box-Muller, model log densities (fp64),
// real-type traits and workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dsmc_internal.h"

namespace dsmc {

// ------------------------------------------------------------------ Philox
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 64x64->128 multiplications with the round constants below and a Weyl key
// schedule between rounds.
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;
constexpr uint64_t kKey1 = 0x64534D43ull;  // second key word of every stream
constexpr uint64_t kPurposeLeaf = 2;
constexpr uint64_t kPurposeCombine = 3;
constexpr uint64_t kPurposeLazyMH = 4;  // Metropolis-Hastings lazy resampling proposals
constexpr uint64_t kPurposeLazyRS = 5;  // rejection lazy resampling proposals

struct Words4 {
  uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                uint64_t c3, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
    const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return {c0, c1, c2, c3};
}

// [0, 1) with 53 random bits
__device__ __forceinline__ double unif53(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }
// (0, 1] with 53 random bits
__device__ __forceinline__ double unif53_open0(uint64_t w) {
  return (double)((w >> 11) + 1ull) * 0x1p-53;
}

// Two standard normals from two words (Box-Muller, fp64).
__device__ __forceinline__ void box_muller(uint64_t wa, uint64_t wb, double& z0, double& z1) {
  const double ua = unif53_open0(wa);
  const double ub = unif53(wb);
  const double rad = sqrt(-2.0 * log(ua));
  const double th = 2.0 * 3.141592653589793 * ub;
  z0 = rad * cos(th);
  z1 = rad * sin(th);
}

// Box-Muller with the three transcendentals written out (used by the fp32
// plans' leaves, whose particles are rounded to fp32): the results agree with
// box_muller to a few fp64 ulps.
//   log u:  u = m 2^e with m in [1/sqrt 2, sqrt 2); log m = 2 atanh s,
//           s = (m - 1) / (m + 1), |s| <= 0.1716, by its odd power series to
//           s^21; e log 2 with log 2 split in a high part exact in e log2_hi.
//   cos 2 pi u, sin 2 pi u:  v = 4u is exact; q = nearest integer to v picks
//           the quarter turn, f = v - q in [-1/2, 1/2] is exact, and
//           theta = f pi / 2 in [-pi/4, pi/4] goes through the Taylor series
//           of cos to theta^18 and of sin to theta^17 (truncation below
//           2^-55 relative on that interval).
__device__ __forceinline__ double log_unit(double u) {
  const uint64_t bits = (uint64_t)__double_as_longlong(u);
  int e = (int)((bits >> 52) & 0x7ff) - 1023;
  double m = __longlong_as_double((long long)((bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
  if (m > 1.4142135623730951) {
    m *= 0.5;
    e += 1;
  }
  const double s = (m - 1.0) / (m + 1.0), s2 = s * s;
  double p = 1.0 / 21.0;
  p = fma(p, s2, 1.0 / 19.0);
  p = fma(p, s2, 1.0 / 17.0);
  p = fma(p, s2, 1.0 / 15.0);
  p = fma(p, s2, 1.0 / 13.0);
  p = fma(p, s2, 1.0 / 11.0);
  p = fma(p, s2, 1.0 / 9.0);
  p = fma(p, s2, 1.0 / 7.0);
  p = fma(p, s2, 1.0 / 5.0);
  p = fma(p, s2, 1.0 / 3.0);
  const double logm = 2.0 * fma(s * s2, p, s);
  const double ln2_hi = 6.93147180369123816490e-01;  // leading 32 bits of log 2
  const double ln2_lo = 1.90821492927058770002e-10;  // log 2 - ln2_hi
  return fma((double)e, ln2_hi, fma((double)e, ln2_lo, logm));
}

__device__ __forceinline__ void sincos_turn(double u, double& c, double& s) {
  const double v = 4.0 * u;
  const double q = rint(v);
  const double th = (v - q) * 1.5707963267948966;
  const double t2 = th * th;
  double pc = 1.0 / 6402373705728000.0;             // 1 / 18!
  pc = fma(pc, -t2, 1.0 / 20922789888000.0);         // 1 / 16!
  pc = fma(pc, -t2, 1.0 / 87178291200.0);            // 1 / 14!
  pc = fma(pc, -t2, 1.0 / 479001600.0);              // 1 / 12!
  pc = fma(pc, -t2, 1.0 / 3628800.0);                // 1 / 10!
  pc = fma(pc, -t2, 1.0 / 40320.0);                  // 1 / 8!
  pc = fma(pc, -t2, 1.0 / 720.0);                    // 1 / 6!
  pc = fma(pc, -t2, 1.0 / 24.0);                     // 1 / 4!
  pc = fma(pc, -t2, 0.5);                            // 1 / 2!
  const double cth = fma(pc, -t2, 1.0);
  double ps = 1.0 / 355687428096000.0;               // 1 / 17!
  ps = fma(ps, -t2, 1.0 / 1307674368000.0);          // 1 / 15!
  ps = fma(ps, -t2, 1.0 / 6227020800.0);             // 1 / 13!
  ps = fma(ps, -t2, 1.0 / 39916800.0);               // 1 / 11!
  ps = fma(ps, -t2, 1.0 / 362880.0);                 // 1 / 9!
  ps = fma(ps, -t2, 1.0 / 5040.0);                   // 1 / 7!
  ps = fma(ps, -t2, 1.0 / 120.0);                    // 1 / 5!
  ps = fma(ps, -t2, 1.0 / 6.0);                      // 1 / 3!
  const double sth = fma(th * t2, -ps, th);
  // 2 pi u = q pi / 2 + th
  switch (((int)q) & 3) {
    case 0: c = cth; s = sth; break;
    case 1: c = -sth; s = cth; break;
    case 2: c = -cth; s = -sth; break;
    default: c = sth; s = -cth; break;
  }
}

__device__ __forceinline__ void box_muller_poly(uint64_t wa, uint64_t wb, double& z0, double& z1) {
  const double rad = sqrt(-2.0 * log_unit(unif53_open0(wa)));
  double c, s;
  sincos_turn(unif53(wb), c, s);
  z0 = rad * c;
  z1 = rad * s;
}

// ------------------------------------------------------------- real traits
template <typename R>
struct Real;

template <>
struct Real<float> {
  static __device__ __forceinline__ float exp2(float x) { return __builtin_amdgcn_exp2f(x); }
  static __device__ __forceinline__ float fma(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
  }
  static constexpr double kTiny = 0x1p-80;  // row sums below this are recomputed shifted
};

template <>
struct Real<double> {
  static __device__ __forceinline__ double exp2(double x) { return ::exp2(x); }
  static __device__ __forceinline__ double fma(double a, double b, double c) {
    return __builtin_fma(a, b, c);
  }
  static constexpr double kTiny = 0x1p-900;
};

// log2 of one pair weight, relative to the node's column maximum:
//   beta_n - || u_n - v_m ||^2
// with whitened, pre-scaled coordinates (so exp2 of it is the natural-scale
// weight).  Written with explicit fma so every call site rounds identically.
template <typename R, int DX>
__device__ __forceinline__ R pair_log2w(const R* u, R beta, const R* v) {
  R s = beta;
#pragma unroll
  for (int d = 0; d < DX; ++d) {
    const R del = u[d] - v[d];
    s = Real<R>::fma(-del, del, s);
  }
  return s;
}

// ------------------------------------------------------------ model terms
// Model fields are uniform across a workgroup (one model per time row or
// combine); readfirstlane tells the compiler so, keeping branches and loop
// bounds on them scalar.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;

// -1/2 || Linv (x - mean) ||^2 with Linv lower triangular [dx][dx].
// For DX >= 8 the row loop is not unrolled (only x stays in registers); the
// summation order is the same either way.
template <int DX>
__device__ __forceinline__ double neg_half_quad(const double* Linv, const double* mean,
                                                const double (&x)[DX], int dx) {
  double q = 0.0;
  if constexpr (DX >= 8) {
    for (int i = 0; i < dx; ++i) {
      double z = 0.0;
#pragma unroll
      for (int j = 0; j < DX; ++j)
        if (j <= i) z += Linv[i * dx + j] * (x[j] - mean[j]);
      q += z * z;
    }
  } else {
#pragma unroll
    for (int i = 0; i < DX; ++i) {
      if (i < dx) {
        double z = 0.0;
#pragma unroll
        for (int j = 0; j <= i; ++j) z += Linv[i * dx + j] * (x[j] - mean[j]);
        q += z * z;
      }
    }
  }
  return -0.5 * q;
}

template <int DX>
__device__ __forceinline__ double log_prior(const DevModel& M, const double (&x)[DX]) {
  return neg_half_quad<DX>(M.P0_inv, M.m0, x, uniform(M.dx)) + M.prior_lognorm;
}

template <int DX>
__device__ __forceinline__ double log_proposal(const DevModel& M, int t, const double (&x)[DX]) {
  const int dx = uniform(M.dx);
  if (uniform(M.prop_kind) == 1) {  // uniform on the box q_mean +- diag(q_chol)
    bool inside = true;
#pragma unroll
    for (int i = 0; i < DX; ++i)
      if (i < dx)
        inside = inside && fabs(x[i] - M.q_mean[(size_t)t * dx + i]) <=
                               M.q_chol[((size_t)t * dx + i) * dx + i];
    return inside ? M.q_lognorm[t] : -INFINITY;
  }
  return neg_half_quad<DX>(M.q_inv + (size_t)t * dx * dx, M.q_mean + (size_t)t * dx, x, dx) +
         M.q_lognorm[t];
}

// log h_t(x).  Linear-Gaussian: H and y are pre-whitened on the host
// (H <- R_inv H, y <- R_inv (y - h)), so the quadratic needs no temporaries.
template <int DX>
__device__ __forceinline__ double log_potential(const DevModel& M, int t, const double (&x)[DX]) {
  if (uniform(M.obs_kind) == 2) {  // indicator of the box y_t = (lo, hi)
    const int dx = uniform(M.dx);
    const double* yt = M.y + (size_t)t * 2 * dx;
    bool inside = true;
#pragma unroll
    for (int i = 0; i < DX; ++i)
      if (i < dx) inside = inside && x[i] >= yt[i] && x[i] <= yt[dx + i];
    return inside ? 0.0 : -INFINITY;
  }
  if (uniform(M.obs_kind) == 1) {  // stochastic volatility: y ~ N(0, exp(x))
    const double y = M.y[t];
    return -0.9189385332046728 - 0.5 * x[0] - 0.5 * y * y * exp(-x[0]);
  }
  const int dx = uniform(M.dx), dy = uniform(M.dy);
  const double* yt = M.y + (size_t)t * dy;
  double q = 0.0;
  for (int i = 0; i < dy; ++i) {
    double r = yt[i];
#pragma unroll
    for (int k = 0; k < DX; ++k)
      if (k < dx) r -= M.H[i * dx + k] * x[k];
    q += r * r;
  }
  return -0.5 * q + M.obs_lognorm;
}

// ------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_or_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}

// Workgroup-wide reductions over blockDim.x threads (a multiple of 64, at most
// 64 kMaxWaves); `red` holds kMaxWaves values (2 kMaxWaves for the paired
// forms).  The combination order is fixed for a given workgroup size, so
// results are deterministic.
__device__ __forceinline__ int num_waves() { return (int)(blockDim.x >> 6); }

__device__ __forceinline__ double block_max(double v, double* red) {
  v = wave_max(v);
  const int w = threadIdx.x >> 6, nw = num_waves();
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < nw; ++i) r = fmax(r, red[i]);
  return r;
}
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = num_waves();
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < nw; ++i) r += red[i];
  return r;
}
__device__ __forceinline__ int block_max_i(int v, int* red) {
  v = wave_max_i(v);
  const int w = threadIdx.x >> 6, nw = num_waves();
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  int r = red[0];
  for (int i = 1; i < nw; ++i) r = max(r, red[i]);
  return r;
}
__device__ __forceinline__ int block_or_i(int v, int* red) {
  v = wave_or_i(v);
  const int w = threadIdx.x >> 6, nw = num_waves();
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  int r = red[0];
  for (int i = 1; i < nw; ++i) r |= red[i];
  return r;
}

// Two reductions for the price of one exchange (max and OR are order-free, so
// the results equal those of the separate calls).  red / redi hold
// 2 kMaxWaves values.
__device__ __forceinline__ void block_max_or(double& v, int& f, double* red, int* redi) {
  v = wave_max(v);
  f = wave_or_i(f);
  const int w = threadIdx.x >> 6, nw = num_waves();
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[w] = v;
    redi[w] = f;
  }
  __syncthreads();
  double r = red[0];
  int o = redi[0];
  for (int i = 1; i < nw; ++i) {
    r = fmax(r, red[i]);
    o |= redi[i];
  }
  v = r;
  f = o;
}
__device__ __forceinline__ void block_max2(double& a, double& b, double* red) {
  a = wave_max(a);
  b = wave_max(b);
  const int w = threadIdx.x >> 6, nw = num_waves();
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[w] = a;
    red[kMaxWaves + w] = b;
  }
  __syncthreads();
  double ra = red[0], rb = red[kMaxWaves];
  for (int i = 1; i < nw; ++i) {
    ra = fmax(ra, red[i]);
    rb = fmax(rb, red[kMaxWaves + i]);
  }
  a = ra;
  b = rb;
}
__device__ __forceinline__ void block_max_i_or(int& a, int& b, int* redi) {
  a = wave_max_i(a);
  b = wave_or_i(b);
  const int w = threadIdx.x >> 6, nw = num_waves();
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    redi[w] = a;
    redi[kMaxWaves + w] = b;
  }
  __syncthreads();
  int ra = redi[0], rb = redi[kMaxWaves];
  for (int i = 1; i < nw; ++i) {
    ra = max(ra, redi[i]);
    rb |= redi[kMaxWaves + i];
  }
  a = ra;
  b = rb;
}

}  // namespace dsmc
